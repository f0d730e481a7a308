// Variant selector: tensor statistics, candidate variants, network inputs,
// the privatisation rule of Section V-D2 as the fallback, and inference.
//
// A candidate is a CSF mode order plus the MTTKRP options for one mode; the
// network predicts log(ns per nonzero) of the whole MTTKRP call for each
// candidate and the smallest prediction wins.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "csf.h"

namespace cpd {
namespace {

constexpr int64_t kSampleMax = 1 << 20;
constexpr double kPrivLdsMax = 64.0 * 1024.0;  // LDS bytes of one private copy
constexpr double kPrivCopies = 1024.0;         // private copies (persistent blocks)
constexpr double kPrivThresh = 0.02;           // privatise iff rows * copies <= 0.02 * nnz

// sum_{k=1}^{I} k^-a: the first 1000 terms exactly, the rest by the midpoint
// integral of x^-a over [1000.5, I + 0.5] (relative error below 1e-7 there)
double zipf_norm(double a, int64_t I) {
    const int64_t K = std::min<int64_t>(I, 1000);
    double h = 0.0;
    for (int64_t k = K; k >= 1; --k) h += std::pow((double)k, -a);
    if (I > K) {
        const double lo = K + 0.5, hi = I + 0.5;
        if (std::fabs(a - 1.0) < 1e-12) h += std::log(hi / lo);
        else h += (std::pow(hi, 1.0 - a) - std::pow(lo, 1.0 - a)) / (1.0 - a);
    }
    return h;
}

void asc_modes(const cpd_stats &st, int32_t *out) {
    for (int m = 0; m < st.nmodes; ++m) out[m] = m;
    std::stable_sort(out, out + st.nmodes, [&](int32_t a, int32_t b) { return st.dims[a] < st.dims[b]; });
}

void make_order(const cpd_stats &st, int kind, int mode, int32_t *order) {
    const int N = st.nmodes;
    int32_t asc[CPD_MAX_MODES];
    asc_modes(st, asc);
    int k = 0;
    switch (kind) {
        case CPD_ORDER_ASC:
            for (int l = 0; l < N; ++l) order[l] = asc[l];
            break;
        case CPD_ORDER_FIRST:
            order[k++] = mode;
            for (int l = 0; l < N; ++l)
                if (asc[l] != mode) order[k++] = asc[l];
            break;
        case CPD_ORDER_LAST:
            for (int l = 0; l < N; ++l)
                if (asc[l] != mode) order[k++] = asc[l];
            order[k++] = mode;
            break;
        case CPD_ORDER_ROOTED: {  // the mode, then the rest by descending length (the CP-ALS trees)
            int32_t desc[CPD_MAX_MODES];
            for (int l = 0; l < N; ++l) desc[l] = l;
            std::stable_sort(desc, desc + N, [&](int32_t a, int32_t b) { return st.dims[a] > st.dims[b]; });
            order[k++] = mode;
            for (int l = 0; l < N; ++l)
                if (desc[l] != mode) order[k++] = desc[l];
            break;
        }
        default:  // descending lengths, ties to the lower mode
            for (int l = 0; l < N; ++l) order[l] = asc[l];
            std::stable_sort(order, order + N, [&](int32_t a, int32_t b) { return st.dims[a] > st.dims[b]; });
    }
}

// the lane-group (ROW) kernels' limits for an output at `depth`: gathered
// (other) levels with ids below 2^24, leaf ids below 2^29 (ranked leaf words)
bool row_kernel_fits(const cpd_stats &st, const int32_t *order, int depth) {
    for (int l = 0; l < st.nmodes; ++l)
        if (l != depth && st.dims[order[l]] >= (1 << 24)) return false;
    return st.dims[order[st.nmodes - 1]] <= (1 << 29);
}

// the paper's privatisation rule (Section V-D2): rows x copies <= 0.02 x nnz
bool priv_rule(const cpd_stats &st, int mode) {
    return (double)st.dims[mode] * kPrivCopies <= kPrivThresh * (double)st.nnz;
}

bool priv_fits(const cpd_stats &st, int mode, int rank) {
    return (double)st.dims[mode] * rank * 4.0 <= kPrivLdsMax;
}

cpd_status check_stats(const cpd_stats *st, int32_t rank, int32_t mode) {
    if (!st) CPD_FAIL(CPD_EINVAL, "null statistics");
    if (st->nmodes < 3 || st->nmodes > 5)
        CPD_FAIL(CPD_EUNSUPPORTED, "the selector handles 3..5 modes, not %d", st->nmodes);
    if (rank < 1 || rank > CPD_MAX_RANK) CPD_FAIL(CPD_EINVAL, "rank %d not in [1, %d]", rank, CPD_MAX_RANK);
    if (mode < 0 || mode >= st->nmodes) CPD_FAIL(CPD_EINVAL, "mode %d not in [0, %d)", mode, st->nmodes);
    if (st->nnz < 1) CPD_FAIL(CPD_EINVAL, "nnz %lld < 1", (long long)st->nnz);
    for (int m = 0; m < st->nmodes; ++m)
        if (st->dims[m] < 1) CPD_FAIL(CPD_EINVAL, "dims[%d] = %lld < 1", m, (long long)st->dims[m]);
    return CPD_OK;
}

cpd_choice base_choice(const cpd_stats &st, int kind, int mode) {
    cpd_choice c{};
    c.order_kind = kind;
    make_order(st, kind, mode, c.order);
    for (int l = 0; l < st.nmodes; ++l)
        if (c.order[l] == mode) c.depth = l;
    c.opts.precision = CPD_FP32;
    return c;
}

inline float lg10(double x) { return (float)std::log10(std::max(x, 1e-30)); }

}  // namespace
}  // namespace cpd

using namespace cpd;

extern "C" {

double cpd_zipf_alpha(double top1, int64_t dim) {
    if (dim <= 1 || !(top1 > 1.0 / (double)dim)) return 0.0;
    if (top1 >= 1.0) return 8.0;
    double lo = 0.0, hi = 8.0;
    if (1.0 / zipf_norm(hi, dim) <= top1) return 8.0;
    for (int it = 0; it < 60; ++it) {  // 1 / H(a) rises with a
        const double mid = 0.5 * (lo + hi);
        if (1.0 / zipf_norm(mid, dim) < top1) lo = mid;
        else hi = mid;
    }
    return 0.5 * (lo + hi);
}

cpd_status cpd_tensor_stats(int32_t nmodes, const int64_t *dims, int64_t nnz, const int32_t *const *inds,
                            void *stream, cpd_stats *out) {
    clear_error();
    if (!out || !dims || !inds) CPD_FAIL(CPD_EINVAL, "null argument");
    if (nmodes < 2 || nmodes > CPD_MAX_MODES) CPD_FAIL(CPD_EINVAL, "nmodes %d not in [2, %d]", nmodes, CPD_MAX_MODES);
    if (nnz < 1 || nnz > INT32_MAX) CPD_FAIL(CPD_EINVAL, "nnz %lld not in [1, 2^31-1]", (long long)nnz);
    for (int m = 0; m < nmodes; ++m) {
        if (dims[m] < 1 || dims[m] > INT32_MAX) CPD_FAIL(CPD_EINVAL, "dims[%d] = %lld out of range", m, (long long)dims[m]);
        if (!inds[m]) CPD_FAIL(CPD_EINVAL, "null index array for mode %d", m);
    }
    hipStream_t s = (hipStream_t)stream;
    DevBuf<int32_t> res;
    CPD_TRY(res.alloc(3 * nmodes, s));
    for (int m = 0; m < nmodes; ++m) CPD_TRY(sample_freq(inds[m], nnz, dims[m], kSampleMax, res.p + 3 * m, s));
    std::vector<int32_t> h(3 * nmodes);
    CPD_HIP(hipMemcpyAsync(h.data(), res.p, sizeof(int32_t) * 3 * nmodes, hipMemcpyDeviceToHost, s));
    CPD_HIP(hipStreamSynchronize(s));
    cpd_stats st{};
    st.nmodes = nmodes;
    st.nnz = nnz;
    st.sample = h[2];
    for (int m = 0; m < nmodes; ++m) {
        const double ns = (double)h[3 * m + 2];
        st.dims[m] = dims[m];
        st.top1[m] = h[3 * m + 1] / ns;
        st.distinct[m] = h[3 * m] / std::min<double>((double)dims[m], ns);
        st.alpha[m] = cpd_zipf_alpha(st.top1[m], dims[m]);
    }
    *out = st;
    return CPD_OK;
}

cpd_status cpd_select_candidates(const cpd_stats *st, int32_t rank, int32_t mode, cpd_choice *out, int32_t *n) {
    clear_error();
    CPD_TRY(check_stats(st, rank, mode));
    if (!out || !n) CPD_FAIL(CPD_EINVAL, "null output");
    const int N = st->nmodes;
    int cnt = 0;
    std::vector<std::vector<int32_t>> seen;
    for (int kind = 0; kind < CPD_ORDER_KINDS; ++kind) {
        cpd_choice b = base_choice(*st, kind, mode);
        std::vector<int32_t> ord(b.order, b.order + N);
        if (std::find(seen.begin(), seen.end(), ord) != seen.end()) continue;
        seen.push_back(ord);
        auto push = [&](int variant, int kernel, int tile) {
            if (cnt >= CPD_SEL_MAX_CAND) return;
            cpd_choice c = b;
            c.opts.variant = variant;
            c.opts.kernel = kernel;
            c.opts.tile_nnz = tile;
            out[cnt++] = c;
        };
        const bool row = row_kernel_fits(*st, b.order, b.depth);
        if (b.depth == 0) {
            if (row) {
                for (int t : {32, 128, 512}) push(CPD_VARIANT_AUTO, CPD_KERNEL_ROW, t);
            } else {
                for (int t : {64, 256, 1024}) push(CPD_VARIANT_ATOMIC, CPD_KERNEL_LANE, t);
            }
        } else if (b.depth < N - 1) {
            if (row) {
                push(CPD_VARIANT_ATOMIC, CPD_KERNEL_ROW, 256);
                push(CPD_VARIANT_PRIVATE, CPD_KERNEL_ROW, 256);
            }
            push(CPD_VARIANT_ATOMIC, CPD_KERNEL_TILED, 0);
            push(CPD_VARIANT_ATOMIC, CPD_KERNEL_LANE, 256);
            if (priv_fits(*st, mode, rank)) push(CPD_VARIANT_PRIVATE, CPD_KERNEL_LANE, 256);
        } else {
            push(CPD_VARIANT_ATOMIC, CPD_KERNEL_TILED, 0);
            for (int t : {64, 256, 1024}) push(CPD_VARIANT_ATOMIC, CPD_KERNEL_ROUND, t);
            push(CPD_VARIANT_ATOMIC, CPD_KERNEL_LANE, 256);
            if (priv_fits(*st, mode, rank)) push(CPD_VARIANT_PRIVATE, CPD_KERNEL_LANE, 256);
        }
    }
    *n = cnt;
    return CPD_OK;
}

cpd_status cpd_select_features(const cpd_stats *st, int32_t rank, int32_t mode, const cpd_choice *cand, int32_t n,
                               float *feat) {
    clear_error();
    CPD_TRY(check_stats(st, rank, mode));
    if (n < 0 || (n > 0 && (!cand || !feat))) CPD_FAIL(CPD_EINVAL, "bad candidate arguments");
    const int N = st->nmodes;
    const double I = (double)st->dims[mode], nnz = (double)st->nnz;
    for (int j = 0; j < n; ++j) {
        const cpd_choice &c = cand[j];
        float *f = feat + (int64_t)j * CPD_SEL_NFEAT;
        std::fill(f, f + CPD_SEL_NFEAT, 0.0f);
        // the tensor and the mode
        f[0] = N / 5.0f;
        f[1] = lg10(nnz) / 8.0f;
        f[2] = (float)(std::log2((double)rank) / 6.0);
        f[3] = lg10(I) / 6.0f;
        f[4] = (float)(st->alpha[mode] / 1.5);
        f[5] = (float)st->top1[mode];
        f[6] = (float)st->distinct[mode];
        f[7] = lg10(nnz / I) / 6.0f;
        // the modes in tree order
        for (int l = 0; l < N; ++l) {
            const int m = c.order[l];
            if (m < 0 || m >= N) CPD_FAIL(CPD_EINVAL, "candidate %d: bad order", j);
            f[8 + l] = lg10((double)st->dims[m]) / 6.0f;
            f[13 + l] = (float)(st->alpha[m] / 1.5);
            f[18 + l] = (float)st->top1[m];
            f[23 + l] = (float)st->distinct[m];
        }
        // the variant
        f[28] = c.depth / 4.0f;
        f[29] = c.depth == 0 ? 1.0f : 0.0f;
        f[30] = c.depth == N - 1 ? 1.0f : 0.0f;
        f[31] = c.opts.variant == CPD_VARIANT_PRIVATE ? 1.0f : 0.0f;
        f[32] = c.opts.kernel == CPD_KERNEL_ROW ? 1.0f : 0.0f;
        f[33] = c.opts.tile_nnz > 0 ? (float)(std::log2((double)c.opts.tile_nnz) / 10.0) : 0.0f;
        if (c.order_kind < 0 || c.order_kind >= CPD_ORDER_KINDS) CPD_FAIL(CPD_EINVAL, "candidate %d: bad order kind", j);
        f[34 + c.order_kind] = 1.0f;
        f[39] = lg10(I * rank * 4.0) / 8.0f;
        f[40] = lg10(I * kPrivCopies / nnz) / 4.0f;
        f[41] = c.opts.kernel == CPD_KERNEL_ROUND ? 1.0f : 0.0f;
        f[42] = c.opts.kernel == CPD_KERNEL_TILED ? 1.0f : 0.0f;
    }
    return CPD_OK;
}

cpd_status cpd_select_heuristic(const cpd_stats *st, int32_t rank, int32_t mode, cpd_choice *out) {
    clear_error();
    CPD_TRY(check_stats(st, rank, mode));
    if (!out) CPD_FAIL(CPD_EINVAL, "null output");
    cpd_choice c = base_choice(*st, CPD_ORDER_ASC, mode);
    const int N = st->nmodes;
    const bool row = row_kernel_fits(*st, c.order, c.depth);
    if (c.depth == 0) {
        c.opts.variant = row ? CPD_VARIANT_AUTO : CPD_VARIANT_ATOMIC;
        c.opts.kernel = row ? CPD_KERNEL_ROW : CPD_KERNEL_LANE;
        c.opts.tile_nnz = row ? 128 : 256;
    } else if (priv_fits(*st, mode, rank) && priv_rule(*st, mode)) {
        // the paper's privatised accumulation
        c.opts.variant = CPD_VARIANT_PRIVATE;
        c.opts.kernel = CPD_KERNEL_LANE;
        c.opts.tile_nnz = 256;
    } else {
        // atomics, with the library's default kernel for the level
        c.opts.variant = CPD_VARIANT_ATOMIC;
        c.opts.kernel = c.depth == N - 1 ? CPD_KERNEL_TILED : row ? CPD_KERNEL_ROW : CPD_KERNEL_LANE;
        c.opts.tile_nnz = c.depth == N - 1 ? 0 : 256;
    }
    *out = c;
    return CPD_OK;
}

cpd_status cpd_select(const cpd_stats *st, int32_t rank, int32_t mode, const float *params, int32_t hidden,
                      cpd_choice *out, float *pred, int32_t *ncand, void *stream) {
    clear_error();
    if (!out) CPD_FAIL(CPD_EINVAL, "null output");
    if (!params) {
        if (ncand) *ncand = 0;
        return cpd_select_heuristic(st, rank, mode, out);
    }
    cpd_choice cand[CPD_SEL_MAX_CAND];
    int32_t n = 0;
    CPD_TRY(cpd_select_candidates(st, rank, mode, cand, &n));
    std::vector<float> feat((size_t)n * CPD_SEL_NFEAT), p(n);
    CPD_TRY(cpd_select_features(st, rank, mode, cand, n, feat.data()));
    hipStream_t s = (hipStream_t)stream;
    DevBuf<float> dx, dp;
    CPD_TRY(dx.alloc(feat.size(), s));
    CPD_TRY(dp.alloc(n, s));
    CPD_HIP(hipMemcpyAsync(dx.p, feat.data(), sizeof(float) * feat.size(), hipMemcpyHostToDevice, s));
    CPD_TRY(cpd_mlp_forward(params, CPD_SEL_NFEAT, hidden, dx.p, n, dp.p, stream));
    CPD_HIP(hipMemcpyAsync(p.data(), dp.p, sizeof(float) * n, hipMemcpyDeviceToHost, s));
    CPD_HIP(hipStreamSynchronize(s));
    int best = 0;
    for (int j = 1; j < n; ++j)
        if (p[j] < p[best]) best = j;
    *out = cand[best];
    if (pred) std::copy(p.begin(), p.end(), pred);
    if (ncand) *ncand = n;
    return CPD_OK;
}

}  // extern "C"
