// CP with missing values (tensor completion) by row-wise alternating least
// squares over the observed entries, the decomposition the paper lists next
// to least-squares CP among the CPD library's routines (Section III).  For
// mode n, row i of A_n solves
//     (G_i + reg I) a = y_i,   G_i = sum_{k in O_i} h_k h_k^T,   y_i = sum_{k in O_i} x_k h_k,
// with O_i the observed entries in row i and h_k the Hadamard product of the
// other modes' rows.  y is the MTTKRP of the observed entries (the root-level
// kernel on the tree rooted at mode n); G is new work: a Gram per row,
// accumulated here on the same tree.
//
// Row Gram kernel: one wave per run of T leaves.  Chunks of C leaves are
// staged in LDS as FP64 rows h, the next chunk's gathers in flight while the
// wave walks the current chunk's leaves in order, each lane accumulating 4x4
// blocks of the upper triangle of h h^T in registers; the blocks are added to
// G_i with FP64 atomics when the leaf's root node (row i) ends or the run ends.
// Row solve kernel: one wave per row, Gauss-Jordan on [G_i + reg I | y_i] in
// LDS, one matrix row per lane (the matrix is symmetric positive definite for
// reg > 0, so no pivoting), with the row's loss terms a.y and a^T G a.
#include <algorithm>
#include <cmath>
#include <vector>

#include "csf.h"

namespace cpd {

cpd_status mttkrp(cpd_csf_s *c, const void *const *factors, int32_t ld, int32_t R, int32_t mode, float *Y,
                  int32_t ldo, const cpd_mttkrp_opts *opts, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1);
cpd_status sumsq(const float *v, int64_t n, double *out, hipStream_t s);
cpd_status mttkrp64(cpd_csf_s *c, const float *const *factors, int32_t ld, int32_t R, int32_t mode, double *Y,
                    int32_t ldo, hipStream_t s);

namespace {

constexpr int RG_WAVES = 4;   // waves per block
constexpr int RG_C = 16;      // leaves staged per chunk
constexpr int RG_T = 2048;    // leaves per wave run (measured 5% faster than 512, 8192 slower)

struct TreeRefs {
    const int32_t *ids[CPD_MAX_MODES];  // per-leaf index at level l (uprow for 1..N-2, fids at the leaf)
    const float *fac[CPD_MAX_MODES];    // factor of level l
    const int32_t *root_ids;
    const int32_t *leafw;               // (level << 29) | rank
    int64_t nleaves;
};

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// QB: 4x4 blocks of the upper triangle owned per lane (ceil(blocks / 64)).
// The chunks are software-pipelined: while the wave accumulates chunk c from
// LDS, the gathers of chunk c + 1 (their ids staged a chunk earlier) and the
// leaf ids of chunk c + 2 are in flight in registers.
template <int N, int QB>
__global__ void __launch_bounds__(64 * RG_WAVES)
k_row_gram(TreeRefs tr, int64_t ld, int R, const int32_t *__restrict__ starts, int64_t nruns, double *__restrict__ G) {
    constexpr int RPMAX = CPD_MAX_RANK;
    constexpr int NI = (N * RG_C + 63) / 64;    // staged ids per lane and chunk
    __shared__ double s_h[RG_WAVES][RG_C][RPMAX];
    __shared__ int32_t s_id[RG_WAVES][N][RG_C];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t run = (int64_t)blockIdx.x * RG_WAVES + wave;
    if (run >= nruns) return;  // waves are independent: no block barriers
    const int NB = (R + 3) / 4, RP = NB * 4;
    const int nblk = NB * (NB + 1) / 2;
    // this lane's blocks (bi <= bj), enumerated row by row
    int bi[QB], bj[QB];
    bool own[QB];
#pragma unroll
    for (int q = 0; q < QB; ++q) {
        int p = lane + 64 * q;
        own[q] = p < nblk;
        int i = 0;
        while (own[q] && p >= NB - i) {
            p -= NB - i;
            ++i;
        }
        bi[q] = i;
        bj[q] = i + p;
    }
    double acc[QB][16];
#pragma unroll
    for (int q = 0; q < QB; ++q)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[q][e] = 0.0;
    const int64_t k0 = run * RG_T, k1 = min(k0 + (int64_t)RG_T, tr.nleaves);
    int32_t c0 = starts[run];
    int32_t row = tr.root_ids[c0];
    auto flush = [&]() {
        double *g = G + (int64_t)row * R * R;
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            if (!own[q]) continue;
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = bi[q] * 4 + u, c = bj[q] * 4 + v;
                    if (r < R && c < R && r <= c) atomicAdd(g + r * R + c, acc[q][u * 4 + v]);
                    acc[q][u * 4 + v] = 0.0;
                }
        }
    };
    auto chunk_len = [&](int64_t t) { return (int)max((int64_t)0, min((int64_t)RG_C, k1 - t)); };
    // leaf ids of every level below the root and the leaf words of chunk t:
    // issued into registers, stored to LDS later
    int32_t idr[NI];
    auto load_ids = [&](int64_t t) {
        const int len = chunk_len(t);
#pragma unroll
        for (int j = 0; j < NI; ++j) {
            const int e = lane + 64 * j, l = e / RG_C, b = e % RG_C;
            idr[j] = 0;
            if (e < N * RG_C && b < len)
                idr[j] = l >= 1 ? tr.ids[l][t + b] : (int32_t)((uint32_t)tr.leafw[t + b] >> 29);
        }
    };
    // stores the ids to LDS; returns the chunk's leaves that open a root node
    // (bit b: leaf word level 0), a wave-uniform mask
    auto store_ids = [&]() {
#pragma unroll
        for (int j = 0; j < NI; ++j) {
            const int e = lane + 64 * j, l = e / RG_C, b = e % RG_C;
            if (e < N * RG_C && l >= 1) s_id[wave][l][b] = idr[j];
        }
        return (uint64_t)__ballot(lane < RG_C && idr[0] == 0);
    };
    // the factor entries of chunk t's rows h (ids in s_id), issued into
    // registers: lane r gathers column r of every leaf's rows (one contiguous
    // row per load instruction)
    float fr[N - 1][RG_C];
    auto load_rows = [&](int64_t t) {
        const int len = chunk_len(t);
#pragma unroll
        for (int b = 0; b < RG_C; ++b) {
            const bool in = b < len && lane < R;
#pragma unroll
            for (int l = 1; l < N; ++l) {
                // the row id is wave-uniform: a scalar base, the lane as offset
                const int32_t id = __builtin_amdgcn_readfirstlane(s_id[wave][l][b]);
                const float *rowp = tr.fac[l] + (int64_t)id * ld;
                fr[l - 1][b] = in ? rowp[lane] : 0.0f;
            }
        }
    };
    // h = product of the gathered entries in FP64 (zero past the rank)
    auto store_rows = [&](int64_t t) {
        const int len = chunk_len(t);
        if (lane >= RP) return;
#pragma unroll
        for (int b = 0; b < RG_C; ++b) {
            double h = 0.0;
            if (b < len && lane < R) {
                h = 1.0;
#pragma unroll
                for (int l = 1; l < N; ++l) h *= (double)fr[l - 1][b];
            }
            s_h[wave][b][lane] = h;
        }
    };
    load_ids(k0);
    uint64_t opens = store_ids();
    wave_sync();
    load_rows(k0);
    load_ids(k0 + RG_C);
    for (int64_t t0 = k0; t0 < k1; t0 += RG_C) {
        const int len = chunk_len(t0);
        store_rows(t0);
        const uint64_t opens_next = store_ids();  // the next chunk's ids
        wave_sync();
        if (t0 + RG_C < k1) {
            load_rows(t0 + RG_C);
            load_ids(t0 + 2 * RG_C);
        }
        // segments of leaves in one root node (from the wave-uniform mask of
        // opening leaves, no per-leaf LDS read): a flush between segments, the
        // products of a segment in a loop unrolled by 8, so that the LDS reads
        // of later leaves issue before the products of earlier ones
        for (int b = 0; b < len;) {
            if (((opens >> b) & 1ull) && t0 + b > k0) {  // a new root node (row) starts at this leaf
                flush();
                c0 += 1;
                row = tr.root_ids[c0];
            }
            const uint64_t later = (opens >> b) >> 1;  // opens after leaf b
            const int e = later ? min(len, b + 1 + (int)__builtin_ctzll(later)) : len;
#pragma unroll 8
            for (int bb = b; bb < e; ++bb) {
                const double *h = s_h[wave][bb];
#pragma unroll
                for (int q = 0; q < QB; ++q) {
                    if (!own[q]) continue;
                    double hr[4], hc[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        hr[u] = h[bi[q] * 4 + u];
                        hc[u] = h[bj[q] * 4 + u];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc[q][u * 4 + v] = fma(hr[u], hc[v], acc[q][u * 4 + v]);
                }
            }
            b = e;
        }
        opens = opens_next;
        wave_sync();
    }
    flush();
}

// Row i: solve (G_i + reg I) a = y_i (G_i upper triangle, row-major R x R),
// write a as FP32, and the loss terms a.y and a^T G_i a.  Lane r owns row r
// of [G_i + reg I | y_i] in LDS: at step j the pivot row is copied (one column
// per lane), then every lane updates its own row along the columns, so there
// is no index arithmetic per element.
__global__ void __launch_bounds__(64)
k_row_solve(const double *__restrict__ G, const float *__restrict__ Y, int64_t ldy, int64_t rows, int R,
            double reg, float *__restrict__ A, int64_t lda, double *__restrict__ terms) {
    // M (R rows of stride LDM) and the pivot-row copy in dynamic LDS sized
    // for this rank: at rank 35 a block takes 10.6 KB instead of 33 KB, so
    // about four waves share each SIMD instead of one.
    // LDM: the odd stride >= R + 1, so lane rows start on distinct bank pairs
    extern __shared__ double s_dyn[];
    const int LDM = (R + 1) | 1;
    double *M = s_dyn;
    double *rowj = s_dyn + R * LDM;
    const int64_t i = blockIdx.x;
    const int lane = threadIdx.x;
    if (i >= rows) return;
    const double *g = G + i * R * R;
    const int W = R + 1;  // augmented width
    for (int t = lane; t < R * W; t += 64) {
        const int r = t / W, c = t % W;
        double x;
        if (c == R) x = (double)Y[i * ldy + r];
        else x = g[min(r, c) * R + max(r, c)] + (r == c ? reg : 0.0);
        M[r * LDM + c] = x;
    }
    __syncthreads();
    double *mine = M + lane * LDM;
    for (int j = 0; j < R; ++j) {
        for (int c = j + lane; c < W; c += 64) rowj[c] = M[j * LDM + c];
        __syncthreads();
        const double inv = 1.0 / rowj[j];
        if (lane < R) {
            if (lane == j) {
                for (int c = j; c < W; ++c) mine[c] = rowj[c] * inv;
            } else {
                const double f = mine[j] * inv;
                for (int c = j; c < W; ++c) mine[c] -= f * rowj[c];
            }
        }
        __syncthreads();
    }
    // a = last column; the loss terms with the unregularised Gram
    double cross = 0.0, quad = 0.0;
    for (int r = lane; r < R; r += 64) {
        const double a = M[r * LDM + R];
        A[i * lda + r] = (float)a;
        cross += a * (double)Y[i * ldy + r];
        double s = 0.0;
        for (int c = 0; c < R; ++c) s += g[min(r, c) * R + max(r, c)] * M[c * LDM + R];
        quad += a * s;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        cross += __shfl_xor(cross, o, 64);
        quad += __shfl_xor(quad, o, 64);
    }
    if (lane == 0) {
        terms[2 * i] = cross;
        terms[2 * i + 1] = quad;
    }
}

// Sum the per-row loss terms (one block, fixed order).
// Loss terms of the stored (FP32) rows a_i of A against an FP64 MTTKRP y
// (rows x ldy doubles) and the row Grams G (upper triangles): terms[2i] =
// a_i . y_i, terms[2i+1] = a_i^T G_i a_i, in FP64.  One wave per row, lane r
// holding a_r.
__global__ void __launch_bounds__(256) k_row_terms(const double *__restrict__ G, const double *__restrict__ Y,
                                                   int64_t ldy, int64_t rows, int R, const float *__restrict__ A,
                                                   int64_t lda, double *__restrict__ terms) {
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int r = threadIdx.x & 63;
    if (i >= rows) return;
    const double a = r < R ? (double)A[i * lda + r] : 0.0;
    const double *g = G + i * (int64_t)R * R;
    double t = 0.0;
    for (int c = 0; c < R; ++c) {
        const double ac = __shfl(a, c, 64);
        if (r < R) t += (r <= c ? g[r * R + c] : g[c * R + r]) * ac;
    }
    double cross = r < R ? a * Y[i * ldy + r] : 0.0, quad = a * t;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        cross += __shfl_xor(cross, o, 64);
        quad += __shfl_xor(quad, o, 64);
    }
    if (r == 0) {
        terms[2 * i] = cross;
        terms[2 * i + 1] = quad;
    }
}

__global__ void __launch_bounds__(256) k_sum_terms(const double *__restrict__ terms, int64_t rows,
                                                   double *__restrict__ out) {
    __shared__ double sc[4], sq[4];
    double c = 0.0, q = 0.0;
    for (int64_t i = threadIdx.x; i < rows; i += 256) {
        c += terms[2 * i];
        q += terms[2 * i + 1];
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        c += __shfl_xor(c, o, 64);
        q += __shfl_xor(q, o, 64);
    }
    if (lane == 0) {
        sc[wave] = c;
        sq[wave] = q;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = (sc[0] + sc[1]) + (sc[2] + sc[3]);
        out[1] = (sq[0] + sq[1]) + (sq[2] + sq[3]);
    }
}

__global__ void k_zero_f64(double *p, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0.0;
}

__global__ void k_copy_rows(const float *__restrict__ src, int64_t lds, float *__restrict__ dst, int64_t ldd,
                            int64_t rows, int R) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * R) return;
    dst[(t / R) * ldd + t % R] = src[(t / R) * lds + t % R];
}

inline int pad_rank(int R) { return R <= 8 ? 8 : R <= 16 ? 16 : R <= 32 ? 32 : R <= 36 ? 36 : 64; }

}  // namespace

// Row Grams of the mode at the root of tree c into G (rows x R x R FP64,
// upper triangle, accumulated: the caller zeroes it).
cpd_status row_gram(cpd_csf_s *c, const float *const *factors, int64_t ld, int R, int mode, double *G,
                    hipStream_t s) {
    if (!c || !factors || !G) CPD_FAIL(CPD_EINVAL, "null argument");
    const int N = c->nmodes;
    if (R < 1 || R > CPD_MAX_RANK || ld < R) CPD_FAIL(CPD_EINVAL, "rank %d / ld %lld out of range", R, (long long)ld);
    if (c->order[0] != mode) CPD_FAIL(CPD_EINVAL, "row Grams need the mode at the root of the tree");
    if (!c->leafw) CPD_FAIL(CPD_EUNSUPPORTED, "row Grams need leaf ids below 2^29");
    if (N < 3 || N > 5) CPD_FAIL(CPD_EUNSUPPORTED, "row Grams built for 3..5 modes, not %d", N);
    TreeRefs tr{};
    for (int l = 1; l < N; ++l) {
        tr.ids[l] = (l == N - 1) ? c->fids[N - 1] : c->uprow[l];
        tr.fac[l] = factors[c->order[l]];
        if (!tr.fac[l]) CPD_FAIL(CPD_EINVAL, "null factor for mode %d", c->order[l]);
    }
    tr.root_ids = c->fids[0];
    tr.leafw = c->leafw;
    tr.nleaves = c->counts[N - 1];
    const int32_t *starts;
    int64_t nruns;
    CPD_TRY(csf_tiles(c, RG_T, &starts, &nruns, s));
    const int NB = (R + 3) / 4, nblk = NB * (NB + 1) / 2, QB = (nblk + 63) / 64;
    const dim3 grid((unsigned)ceil_div(nruns, RG_WAVES)), block(64 * RG_WAVES);
#define CPD_RG(n, q) hipLaunchKernelGGL((k_row_gram<n, q>), grid, block, 0, s, tr, ld, R, starts, nruns, G)
#define CPD_RG_N(n)                  \
    if (QB == 1) CPD_RG(n, 1);       \
    else if (QB == 2) CPD_RG(n, 2);  \
    else CPD_RG(n, 3);
    switch (N) {
        case 3: CPD_RG_N(3) break;
        case 4: CPD_RG_N(4) break;
        default: CPD_RG_N(5) break;
    }
#undef CPD_RG_N
#undef CPD_RG
    CPD_LAUNCH_CHECK();
    return CPD_OK;
}

cpd_status row_solve(const double *G, const float *Y, int64_t ldy, int64_t rows, int R, double reg, float *A,
                     int64_t lda, double *terms2, hipStream_t s) {
    if (!G || !Y || !A) CPD_FAIL(CPD_EINVAL, "null argument");
    if (R < 1 || R > CPD_MAX_RANK || ldy < R || lda < R || rows < 0) CPD_FAIL(CPD_EINVAL, "bad row solve sizes");
    if (!(reg > 0.0)) CPD_FAIL(CPD_EINVAL, "row solve needs reg > 0 (got %g)", reg);
    if (rows == 0) return CPD_OK;
    DevBuf<double> terms;
    CPD_TRY(terms.alloc((size_t)rows * 2, s));
    const size_t lds = (size_t)(R * ((R + 1) | 1) + R + 1) * sizeof(double);
    hipLaunchKernelGGL(k_row_solve, dim3((unsigned)rows), dim3(64), lds, s, G, Y, ldy, rows, R, reg, A, lda,
                       terms.p);
    CPD_LAUNCH_CHECK();
    if (terms2) {
        hipLaunchKernelGGL(k_sum_terms, dim3(1), dim3(256), 0, s, (const double *)terms.p, rows, terms2);
        CPD_LAUNCH_CHECK();
    }
    return CPD_OK;
}

}  // namespace cpd

using namespace cpd;

extern "C" {

cpd_status cpd_row_gram(cpd_csf csf, const float *const *factors, int64_t ld, int32_t rank, int32_t mode,
                        double *G, void *stream) {
    clear_error();
    if (!csf) CPD_FAIL(CPD_EINVAL, "null CSF handle");
    if (mode < 0 || mode >= csf->nmodes) CPD_FAIL(CPD_EINVAL, "mode %d out of range", mode);
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = csf->dims[mode] * (int64_t)rank * rank;
    if (G) {
        hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, G, n);
        CPD_LAUNCH_CHECK();
    }
    return row_gram(csf, factors, ld, rank, mode, G, s);
}

cpd_status cpd_row_solve(const double *G, const float *Y, int64_t ldy, int64_t rows, int32_t rank, double reg,
                         float *A, int64_t lda, double *terms, void *stream) {
    clear_error();
    return row_solve(G, Y, ldy, rows, rank, reg, A, lda, terms, (hipStream_t)stream);
}

cpd_status cpd_complete(int32_t nmodes, const int64_t *dims, int64_t nnz, const int32_t *const *inds,
                        const float *vals, int32_t rank, int32_t max_iters, double tol, double reg,
                        float *const *factors, double *rmse, int32_t *iters, void *stream) {
    clear_error();
    hipStream_t s = (hipStream_t)stream;
    if (iters) *iters = 0;
    if (nmodes < 3 || nmodes > 5) CPD_FAIL(CPD_EUNSUPPORTED, "completion built for 3..5 modes, not %d", nmodes);
    if (!dims || !inds || !vals || !factors) CPD_FAIL(CPD_EINVAL, "null argument");
    if (rank < 1 || rank > CPD_MAX_RANK) CPD_FAIL(CPD_EINVAL, "rank %d not in [1, %d]", rank, CPD_MAX_RANK);
    if (max_iters < 1) CPD_FAIL(CPD_EINVAL, "max_iters %d < 1", max_iters);
    if (!(reg > 0.0)) CPD_FAIL(CPD_EINVAL, "completion needs reg > 0 (got %g)", reg);
    for (int m = 0; m < nmodes; ++m)
        if (!factors[m]) CPD_FAIL(CPD_EINVAL, "null factor %d", m);
    keep_pool_memory();
    cpd_csf trees[CPD_MAX_MODES] = {};
    CPD_TRY(cpd_csf_build_rooted(nmodes, dims, nnz, inds, vals, stream, trees));
    std::vector<DevBuf<float>> A(nmodes);
    DevBuf<float> Y;
    DevBuf<double> G, d_terms, d_norm;
    const int ld = pad_rank(rank);
    int64_t maxrows = 0;
    cpd_status st = CPD_OK;
    auto done = [&](cpd_status r) {
        for (int m = 0; m < nmodes; ++m)
            if (trees[m]) free_csf_on(trees[m], s);
        return r;
    };
    for (int m = 0; m < nmodes && st == CPD_OK; ++m) {
        maxrows = std::max<int64_t>(maxrows, dims[m]);
        st = A[m].alloc((size_t)dims[m] * ld, s);
        if (st == CPD_OK && hipMemsetAsync(A[m].p, 0, sizeof(float) * dims[m] * ld, s) != hipSuccess) st = CPD_EHIP;
        if (st == CPD_OK) {
            hipLaunchKernelGGL(k_copy_rows, dim3((unsigned)ceil_div(dims[m] * rank, 256)), dim3(256), 0, s,
                               (const float *)factors[m], (int64_t)rank, A[m].p, (int64_t)ld, (int64_t)dims[m], rank);
            if (hipGetLastError() != hipSuccess) st = CPD_EHIP;
        }
    }
    if (st == CPD_OK) st = Y.alloc((size_t)maxrows * ld, s);
    if (st == CPD_OK) st = G.alloc((size_t)maxrows * rank * rank, s);
    if (st == CPD_OK) st = d_terms.alloc(2, s);
    if (st == CPD_OK) st = d_norm.alloc(1, s);
    // the observed entries are the merged nonzeros of the trees
    const int64_t nobs = trees[0]->counts[nmodes - 1];
    if (st == CPD_OK) st = sumsq(trees[0]->vals, nobs, d_norm.p, s);
    if (st != CPD_OK) return done(st);
    double normX2 = 0.0;
    if (hipMemcpyAsync(&normX2, d_norm.p, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return done(CPD_EHIP);
    const void *fac[CPD_MAX_MODES];
    const float *facf[CPD_MAX_MODES];
    for (int m = 0; m < nmodes; ++m) {
        fac[m] = A[m].p;
        facf[m] = A[m].p;
    }
    cpd_mttkrp_opts mo{CPD_FP32, CPD_VARIANT_AUTO, CPD_KERNEL_AUTO, 0};
    double prev = -1.0;
    int it = 0;
    for (it = 1; it <= max_iters; ++it) {
        for (int n = 0; n < nmodes && st == CPD_OK; ++n) {
            const int64_t rows = dims[n];
            const void *fk[CPD_MAX_MODES];
            for (int m = 0; m < nmodes; ++m) fk[m] = (m == n) ? nullptr : fac[m];
            st = mttkrp(trees[n], fk, ld, rank, n, Y.p, ld, &mo, s, nullptr, nullptr);
            if (st == CPD_OK) {
                const int64_t ng = rows * (int64_t)rank * rank;
                hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)ceil_div(ng, 256)), dim3(256), 0, s, G.p, ng);
                if (hipGetLastError() != hipSuccess) st = CPD_EHIP;
            }
            if (st == CPD_OK) st = row_gram(trees[n], facf, ld, rank, n, G.p, s);
            if (st == CPD_OK)
                st = row_solve(G.p, Y.p, ld, rows, rank, reg, A[n].p, ld, n == nmodes - 1 ? d_terms.p : nullptr, s);
        }
        if (st != CPD_OK) return done(st);
        double t2[2];
        if (hipMemcpyAsync(t2, d_terms.p, sizeof(t2), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return done(CPD_EHIP);
        const double r = std::sqrt(std::max(0.0, normX2 - 2.0 * t2[0] + t2[1]) / (double)std::max<int64_t>(nobs, 1));
        if (rmse) rmse[it - 1] = r;
        if (iters) *iters = it;
        if (tol > 0.0 && prev >= 0.0 && std::fabs(r - prev) < tol) break;
        prev = r;
    }
    // The last RMSE is evaluated once more for the returned (FP32) factors from
    // an MTTKRP of the last mode with FP64 products and sums: the sweep's
    // value takes a.y from its FP32 MTTKRP, whose relative error (~1e-6 on
    // long rows) bounds an RMSE near 0 to about 1e-3 of the data's scale.
    if (rmse && st == CPD_OK) {
        const int nl = nmodes - 1;
        const int64_t rows = dims[nl];
        DevBuf<double> Y64, terms;
        st = Y64.alloc((size_t)rows * ld, s);
        if (st == CPD_OK) st = terms.alloc((size_t)rows * 2, s);
        if (st == CPD_OK) st = mttkrp64(trees[nl], facf, ld, rank, nl, Y64.p, ld, s);
        if (st == CPD_OK && rows > 0) {
            hipLaunchKernelGGL(k_row_terms, dim3((unsigned)ceil_div(rows, 4)), dim3(256), 0, s, (const double *)G.p,
                               (const double *)Y64.p, (int64_t)ld, rows, rank, (const float *)A[nl].p, (int64_t)ld,
                               terms.p);
            hipLaunchKernelGGL(k_sum_terms, dim3(1), dim3(256), 0, s, (const double *)terms.p, rows, d_terms.p);
            if (hipGetLastError() != hipSuccess) st = CPD_EHIP;
        }
        double t2[2] = {0.0, 0.0};
        if (st == CPD_OK && (hipMemcpyAsync(t2, d_terms.p, sizeof(t2), hipMemcpyDeviceToHost, s) != hipSuccess ||
                             hipStreamSynchronize(s) != hipSuccess))
            st = CPD_EHIP;
        if (st != CPD_OK) return done(st);
        rmse[std::min(it, max_iters) - 1] =
            std::sqrt(std::max(0.0, normX2 - 2.0 * t2[0] + t2[1]) / (double)std::max<int64_t>(nobs, 1));
    }
    for (int m = 0; m < nmodes && st == CPD_OK; ++m) {
        hipLaunchKernelGGL(k_copy_rows, dim3((unsigned)ceil_div(dims[m] * rank, 256)), dim3(256), 0, s,
                           (const float *)A[m].p, (int64_t)ld, factors[m], (int64_t)rank, (int64_t)dims[m], rank);
        if (hipGetLastError() != hipSuccess) st = CPD_EHIP;
    }
    if (st == CPD_OK && hipStreamSynchronize(s) != hipSuccess) st = CPD_EHIP;
    return done(st);
}

}  // extern "C"
