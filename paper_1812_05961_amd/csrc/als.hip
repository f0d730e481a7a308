// CP-ALS driver (Algorithm 1, Section III) over the GPU steps: CSF build, per
// mode { V, MTTKRP, solve, normalise, Gram refresh }, fit once per sweep.
// All work is ordered on the caller's stream; the host waits only for the
// convergence check (tol > 0) and at the end.
#include <stdarg.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "csf.h"

namespace cpd {

// ------------------------------------------------------------ error state
static thread_local char g_err[512];

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = 0; }

void keep_pool_memory() {
    static std::mutex mu;
    static bool done[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        (void)hipGetLastError();
        return;
    }
    std::lock_guard<std::mutex> g(mu);
    if (done[dev]) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t thr = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    (void)hipGetLastError();
    done[dev] = true;
}

cpd_status mttkrp(cpd_csf_s *c, const void *const *factors, int32_t ld, int32_t R, int32_t mode, float *Y,
                  int32_t ldo, const cpd_mttkrp_opts *opts, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1);
cpd_status gram_internal(const float *A, int64_t rows, int R, int64_t ld, double *G, hipStream_t s);
cpd_status solve_normalize(const double *const *grams, int nmodes, int mode, const float *Y, int64_t rows,
                           int R, int64_t ldy, float *A, int64_t lda, uint16_t *Ab, int64_t ldb,
                           double *lambda, double *G_new, int32_t *used_pinv, hipStream_t s);
cpd_status fit(double normX2, const double *lambda, const float *A, int64_t lda, const float *Y,
               int64_t ldy, int64_t rows, int R, const double *const *grams, int nmodes, double *out,
               hipStream_t s);
cpd_status sumsq(const float *v, int64_t n, double *out, hipStream_t s);
cpd_status mttkrp64(cpd_csf_s *c, const float *const *factors, int32_t ld, int32_t R, int32_t mode, double *Y,
                    int32_t ldo, hipStream_t s);
cpd_status fit64(double normX2, const double *lambda, const float *A, int64_t lda, const double *Y,
                 int64_t ldy, int64_t rows, int R, const double *const *grams, int nmodes, double *out,
                 hipStream_t s);

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// U(0,1) initial factor: element (i, r) of mode m is the top 53 bits of
// SplitMix64(key_m + i*R + r) times 2^-53, key_m = SplitMix64(seed ^ (m+1) * golden).
__global__ void k_init_uniform(float *A, int64_t rows, int R, int64_t ld, uint64_t seed, int m) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * R) return;
    const uint64_t key = mix64(seed ^ ((uint64_t)(m + 1) * 0x9E3779B97F4A7C15ull));
    const uint64_t z = mix64(key + (uint64_t)t);
    A[(t / R) * ld + (t % R)] = (float)((double)(z >> 11) * 0x1.0p-53);
}

__global__ void k_to_bf16(const float *A, int64_t rows, int R, int64_t lda, uint16_t *B, int64_t ldb) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * R) return;
    const int64_t i = t / R, r = t % R;
    B[i * ldb + r] = f32_to_bf16(A[i * lda + r]);
}

__global__ void k_fill_zero_f32(float *p, int64_t n) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0.0f;
}

__global__ void k_fill_zero_u16(uint16_t *p, int64_t n) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0;
}

inline int pad_width(int R, bool bf16) {
    if (R <= 8) return bf16 ? 16 : 8;  // rows of at least two 16-byte chunks
    if (R <= 16) return 16;
    if (R <= 32) return 32;
    if (!bf16 && R <= 36) return 36;
    if (bf16 && R <= 40) return 40;
    return 64;
}

struct Events {
    std::vector<hipEvent_t> ev;
    ~Events() {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
    hipEvent_t make() {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        ev.push_back(e);
        return e;
    }
};

// Trees and buffers of one cpd_als call, all used only on its stream: they
// come from and return to the scratch cache of that stream.
struct Owned {
    hipStream_t s;
    std::vector<cpd_csf_s *> csfs;
    std::vector<std::pair<void *, size_t>> bufs;
    explicit Owned(hipStream_t st) : s(st) {}
    ~Owned() {
        for (auto c : csfs) free_csf_on(c, s);
        for (auto &b : bufs) scratch_put(b.first, b.second, s);
    }
    template <typename T>
    cpd_status alloc(T **p, size_t count) {
        const size_t bytes = sizeof(T) * std::max<size_t>(count, 1);
        void *q = nullptr;
        CPD_TRY(scratch_get(bytes, s, &q));
        *p = static_cast<T *>(q);
        bufs.push_back({q, bytes});
        return CPD_OK;
    }
};

float ms_between(hipEvent_t a, hipEvent_t b) {
    float ms = 0.0f;
    if (a && b && hipEventElapsedTime(&ms, a, b) == hipSuccess) return ms;
    (void)hipGetLastError();
    return -1.0f;
}

}  // namespace

cpd_status als(int nm, const int64_t *dims, int64_t nnz, const int32_t *const *inds, const float *vals, int R,
               int max_iters, double tol, const cpd_als_opts *opts_in, float *const *factors_out,
               double *lambda_out, double *fit_out, int32_t *iters_out, hipStream_t s) {
    if (nm < 2 || nm > 5) CPD_FAIL(CPD_EINVAL, "cpd_als handles 2..5 modes, not %d", nm);
    if (R < 1 || R > CPD_MAX_RANK) CPD_FAIL(CPD_EINVAL, "rank %d not in [1, %d]", R, CPD_MAX_RANK);
    if (max_iters < 1) CPD_FAIL(CPD_EINVAL, "max_iters %d < 1", max_iters);
    if (!(tol >= 0.0)) CPD_FAIL(CPD_EINVAL, "tol must be >= 0");
    if (!factors_out || !lambda_out || !fit_out || !iters_out || !dims) CPD_FAIL(CPD_EINVAL, "null output");
    for (int m = 0; m < nm; ++m)
        if (!factors_out[m]) CPD_FAIL(CPD_EINVAL, "null factor output for mode %d", m);
    cpd_als_opts o{};
    if (opts_in) o = *opts_in;
    const bool bf16 = o.precision == CPD_BF16_GATHER;
    if (o.precision != CPD_FP32 && !bf16) CPD_FAIL(CPD_EINVAL, "unknown precision %d", o.precision);
    if (o.fast_fit != 0 && o.fast_fit != 1) CPD_FAIL(CPD_EINVAL, "fast_fit must be 0 or 1, not %d", o.fast_fit);
    const bool exact_fit = o.fast_fit == 0;

    keep_pool_memory();
    Owned own(s);
    Events evs;
    const bool timing = o.timing_ms != nullptr;
    hipEvent_t t_begin = timing ? evs.make() : nullptr;
    if (timing) CPD_HIP(hipEventRecord(t_begin, s));

    // CSF trees: one rooted at each mode (every MTTKRP at the root), one
    // shared tree, or the trees the selector picks (equal orders shared).
    std::vector<cpd_csf_s *> csf_of(nm, nullptr);
    std::vector<cpd_mttkrp_opts> mo_of(nm, cpd_mttkrp_opts{bf16 ? CPD_BF16_GATHER : CPD_FP32, o.variant, o.kernel,
                                                           o.tile_nnz});
    if (o.select != 0 && o.select != 1 && o.select != 2) CPD_FAIL(CPD_EINVAL, "unknown select mode %d", o.select);
    if (o.select == 1 && !o.selector_params) CPD_FAIL(CPD_EINVAL, "select = 1 needs selector_params");
    if (o.select) {
        cpd_stats st{};
        CPD_TRY(cpd_tensor_stats(nm, dims, nnz, inds, s, &st));
        std::vector<std::vector<int32_t>> built;
        for (int m = 0; m < nm; ++m) {
            cpd_choice ch{};
            CPD_TRY(cpd_select(&st, R, m, o.select == 1 ? o.selector_params : nullptr, o.selector_hidden, &ch,
                               nullptr, nullptr, s));
            std::vector<int32_t> ord(ch.order, ch.order + nm);
            auto it = std::find(built.begin(), built.end(), ord);
            if (it == built.end()) {
                cpd_csf c = nullptr;
                CPD_TRY(cpd_csf_build(nm, dims, nnz, inds, vals, ch.order, s, &c));
                own.csfs.push_back(c);
                built.push_back(ord);
                csf_of[m] = c;
            } else {
                csf_of[m] = own.csfs[it - built.begin()];
            }
            mo_of[m].variant = ch.opts.variant;
            mo_of[m].kernel = ch.opts.kernel;
            mo_of[m].tile_nnz = ch.opts.tile_nnz;
        }
    } else if (o.single_csf) {
        cpd_csf c = nullptr;
        CPD_TRY(cpd_csf_build(nm, dims, nnz, inds, vals, o.order, s, &c));
        own.csfs.push_back(c);
        for (int m = 0; m < nm; ++m) csf_of[m] = c;
    } else {
        // one tree rooted at each mode, the others by descending length: the
        // smallest factor sits at the leaf level, gathered once per nonzero
        // (measured 1-4% faster than ascending on the benchmark shapes)
        cpd_csf trees[CPD_MAX_MODES] = {};
        CPD_TRY(cpd_csf_build_rooted(nm, dims, nnz, inds, vals, s, trees));
        for (int m = 0; m < nm; ++m) {
            own.csfs.push_back(trees[m]);
            csf_of[m] = trees[m];
        }
    }
    hipEvent_t t_csf = timing ? evs.make() : nullptr;
    if (timing) CPD_HIP(hipEventRecord(t_csf, s));

    const int ldf = pad_width(R, false), ldb = pad_width(R, true);
    int64_t maxrows = 0;
    for (int m = 0; m < nm; ++m) maxrows = std::max<int64_t>(maxrows, dims[m]);
    float *A[CPD_MAX_MODES] = {};
    uint16_t *Ab[CPD_MAX_MODES] = {};
    double *G[CPD_MAX_MODES] = {};
    float *Y = nullptr;
    double *Y64 = nullptr;
    double *lambda = nullptr, *d_fit = nullptr, *normX2 = nullptr;
    int32_t *d_pinv = nullptr;
    for (int m = 0; m < nm; ++m) {
        CPD_TRY(own.alloc(&A[m], (size_t)dims[m] * ldf));
        CPD_TRY(own.alloc(&G[m], (size_t)R * R));
        if (bf16) CPD_TRY(own.alloc(&Ab[m], (size_t)dims[m] * ldb));
    }
    CPD_TRY(own.alloc(&Y, (size_t)maxrows * ldf));
    if (exact_fit) CPD_TRY(own.alloc(&Y64, (size_t)dims[nm - 1] * ldf));
    CPD_TRY(own.alloc(&lambda, R));
    CPD_TRY(own.alloc(&d_fit, (size_t)max_iters + 1));
    CPD_TRY(own.alloc(&normX2, 1));
    CPD_TRY(own.alloc(&d_pinv, 1));

    // ||X||^2 of the merged tensor
    CPD_TRY(sumsq(csf_of[0]->vals, csf_of[0]->counts[nm - 1], normX2, s));
    double h_normX2 = 0.0;
    CPD_HIP(hipMemcpyAsync(&h_normX2, normX2, sizeof(double), hipMemcpyDeviceToHost, s));

    // initial factors (padding columns zeroed so vector loads read finite values)
    for (int m = 0; m < nm; ++m) {
        const int64_t tot = dims[m] * ldf;
        hipLaunchKernelGGL(k_fill_zero_f32, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, s, A[m], tot);
        CPD_LAUNCH_CHECK();
        if (o.init) {
            if (!o.init[m]) CPD_FAIL(CPD_EINVAL, "null init factor for mode %d", m);
            CPD_HIP(hipMemcpy2DAsync(A[m], sizeof(float) * ldf, o.init[m], sizeof(float) * R, sizeof(float) * R,
                                     dims[m], hipMemcpyDeviceToDevice, s));
        } else {
            hipLaunchKernelGGL(k_init_uniform, dim3((unsigned)ceil_div(dims[m] * R, 256)), dim3(256), 0, s, A[m],
                               dims[m], R, (int64_t)ldf, o.seed, m);
            CPD_LAUNCH_CHECK();
        }
        if (bf16) {
            const int64_t totb = dims[m] * ldb;
            hipLaunchKernelGGL(k_fill_zero_u16, dim3((unsigned)ceil_div(totb, 256)), dim3(256), 0, s, Ab[m], totb);
            hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)ceil_div(dims[m] * R, 256)), dim3(256), 0, s, A[m],
                               dims[m], R, (int64_t)ldf, Ab[m], (int64_t)ldb);
            CPD_LAUNCH_CHECK();
        }
        if (m > 0) CPD_TRY(gram_internal(A[m], dims[m], R, ldf, G[m], s));
    }
    CPD_HIP(hipStreamSynchronize(s));
    if (!(h_normX2 > 0.0)) CPD_FAIL(CPD_EINVAL, "the tensor has no nonzero value (||X|| = 0)");

    const void *fac_ptrs[CPD_MAX_MODES];
    for (int m = 0; m < nm; ++m) fac_ptrs[m] = bf16 ? (const void *)Ab[m] : (const void *)A[m];
    const int fld = bf16 ? ldb : ldf;
    const double *gptr[CPD_MAX_MODES];
    for (int m = 0; m < nm; ++m) gptr[m] = G[m];

    std::vector<hipEvent_t> ev_it, ev_mt0, ev_mt1;
    hipEvent_t t_loop0 = timing ? evs.make() : nullptr;
    if (timing) CPD_HIP(hipEventRecord(t_loop0, s));
    int it = 0;
    double fit_prev = 0.0, h_fit = 0.0;
    for (it = 1; it <= max_iters; ++it) {
        for (int n = 0; n < nm; ++n) {
            hipEvent_t e0 = timing ? evs.make() : nullptr, e1 = timing ? evs.make() : nullptr;
            CPD_TRY(mttkrp(csf_of[n], fac_ptrs, fld, R, n, Y, ldf, &mo_of[n], s, e0, e1));
            ev_mt0.push_back(e0);
            ev_mt1.push_back(e1);
            CPD_TRY(solve_normalize(gptr, nm, n, Y, dims[n], R, ldf, A[n], ldf, bf16 ? Ab[n] : nullptr, ldb,
                                    lambda, G[n], d_pinv, s));
        }
        CPD_TRY(fit(h_normX2, lambda, A[nm - 1], ldf, Y, ldf, dims[nm - 1], R, gptr, nm, d_fit + it - 1, s));
        hipEvent_t ei = timing ? evs.make() : nullptr;
        if (timing) CPD_HIP(hipEventRecord(ei, s));
        ev_it.push_back(ei);
        if (tol > 0.0) {
            CPD_HIP(hipMemcpyAsync(&h_fit, d_fit + it - 1, sizeof(double), hipMemcpyDeviceToHost, s));
            CPD_HIP(hipStreamSynchronize(s));
            if (it > 1 && fabs(h_fit - fit_prev) < tol) break;
            fit_prev = h_fit;
        }
    }
    const int iters = std::min(it, max_iters);
    hipEvent_t t_loop1 = timing ? evs.make() : nullptr;
    if (timing) CPD_HIP(hipEventRecord(t_loop1, s));
    // The reported fit is that of the returned model, evaluated once more from
    // an MTTKRP of the last mode with the final FP32 factors: by default with
    // FP64 products and sums, so that the residual ||X||^2 - 2<X,K> + ||K||^2
    // keeps its accuracy as the fit nears 1 (the FP32 MTTKRP's relative error,
    // ~1e-6 on rows of millions of terms, would otherwise bound the fit near 1
    // to about sqrt(2e-6) ~ 1e-3); with fast_fit and BF16 gathers, with FP32
    // rows and sums.
    if (exact_fit) {
        const float *f32_ptrs[CPD_MAX_MODES];
        for (int m = 0; m < nm; ++m) f32_ptrs[m] = A[m];
        CPD_TRY(mttkrp64(csf_of[nm - 1], f32_ptrs, ldf, R, nm - 1, Y64, ldf, s));
        CPD_TRY(fit64(h_normX2, lambda, A[nm - 1], ldf, Y64, ldf, dims[nm - 1], R, gptr, nm, d_fit + max_iters, s));
    } else if (bf16) {
        const void *f32_ptrs[CPD_MAX_MODES];
        for (int m = 0; m < nm; ++m) f32_ptrs[m] = A[m];
        cpd_mttkrp_opts mf = mo_of[nm - 1];
        mf.precision = CPD_FP32;
        CPD_TRY(mttkrp(csf_of[nm - 1], f32_ptrs, ldf, R, nm - 1, Y, ldf, &mf, s, nullptr, nullptr));
        CPD_TRY(fit(h_normX2, lambda, A[nm - 1], ldf, Y, ldf, dims[nm - 1], R, gptr, nm, d_fit + max_iters, s));
    }
    hipEvent_t t_end = timing ? evs.make() : nullptr;
    if (timing) CPD_HIP(hipEventRecord(t_end, s));

    for (int m = 0; m < nm; ++m)
        CPD_HIP(hipMemcpy2DAsync(factors_out[m], sizeof(float) * R, A[m], sizeof(float) * ldf, sizeof(float) * R,
                                 dims[m], hipMemcpyDeviceToDevice, s));
    CPD_HIP(hipMemcpyAsync(lambda_out, lambda, sizeof(double) * R, hipMemcpyDeviceToHost, s));
    std::vector<double> fits(max_iters + 1, 0.0);
    CPD_HIP(hipMemcpyAsync(fits.data(), d_fit, sizeof(double) * (max_iters + 1), hipMemcpyDeviceToHost, s));
    CPD_HIP(hipStreamSynchronize(s));
    *iters_out = iters;
    *fit_out = (exact_fit || bf16) ? fits[max_iters] : fits[iters - 1];
    if (o.fit_trace)
        for (int i = 0; i < iters; ++i) o.fit_trace[i] = fits[i];
    if (timing) {
        double *t = o.timing_ms;
        t[0] = ms_between(t_begin, t_csf);
        t[1] = ms_between(t_loop0, t_loop1);
        t[2] = ms_between(t_loop1, t_end);
        t[3] = ms_between(t_begin, t_end);
        hipEvent_t prev = t_loop0;
        for (int i = 0; i < iters; ++i) {
            double *row = t + 4 + (size_t)i * (nm + 1);
            for (int n = 0; n < nm; ++n) row[n] = ms_between(ev_mt0[i * nm + n], ev_mt1[i * nm + n]);
            row[nm] = ms_between(prev, ev_it[i]);
            prev = ev_it[i];
        }
    }
    return CPD_OK;
}

}  // namespace cpd

extern "C" {

const char *cpd_last_error(void) { return cpd::g_err; }

int32_t cpd_abi_version(void) { return 4; }

cpd_status cpd_als(int32_t nmodes, const int64_t *dims, int64_t nnz, const int32_t *const *inds, const float *vals,
                   int32_t rank, int32_t max_iters, double tol, const cpd_als_opts *opts, float *const *factors_out,
                   double *lambda_out, double *fit_out, int32_t *iters_out, void *stream) {
    cpd::clear_error();
    return cpd::als(nmodes, dims, nnz, inds, vals, rank, max_iters, tol, opts, factors_out, lambda_out, fit_out,
                    iters_out, (hipStream_t)stream);
}

}  // extern "C"
