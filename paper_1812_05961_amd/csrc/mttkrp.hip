// MTTKRP on a CSF tree (the MTTKRP step of Algorithm 1; Section III):
//     Y(i, r) = sum over nonzeros with i_mode = i of x * prod_{m != mode} A_m(i_m, r)
// for an output mode at any level d of the tree.
//
// Work split: the leaves are cut into streams of T consecutive nonzeros; each
// stream starts from the nodes that hold its first leaf (the tile table) and
// walks its leaves in order, advancing the node cursors of the upper levels
// as fibers end.  Every contribution is x * (leaf row) * H, where H is the
// Hadamard product of the rows of the non-leaf levels other than d; it changes
// only when a fiber ends.
//
// Two kernel families:
//   ROW  (levels d < N-1, in mttkrp_root.hip): groups of G lanes, each lane
//        holding 16-byte chunks of the rows, several leaves per wave step;
//        at the root a contention-free segmented combine, at internal levels
//        one atomic flush per output node.
//   LANE (any level): one stream per group of G lanes, column r on lane r of
//        the group; coalesced row loads and coalesced atomics.  For the leaf
//        level each nonzero adds v*H to its row, either with global atomics or
//        into a block-private copy of Y in LDS (the paper's privatisation,
//        Section IV-B / V-D2) that is flushed once per block.  When Y is too
//        large for LDS, the privatised form gives each of the chip's eight
//        XCDs its own copy of Y in HBM (blocks are dispatched to the XCDs in
//        turn, so block b adds into copy b mod 8), summed into Y afterwards.
#include <type_traits>

#include "csf.h"

namespace cpd {
namespace {

constexpr int XCD_COPIES = 8;  // private HBM copies of Y: one per XCD of the chip

struct CsfView {
    const int32_t *fids[CPD_MAX_MODES];
    const int32_t *fptr[CPD_MAX_MODES];
    const float *vals;
    int64_t nleaves;
    const int32_t *leafw;      // (level << 29) | frequency rank of the leaf index
    const int32_t *hot_perm;   // HOT: index of each frequency rank at the output level
    const int32_t *hot_rank;   // HOT: frequency rank of each index at the output level
};

struct FacView {
    const void *a[CPD_MAX_MODES];  // by level
};

template <typename GT>
__device__ __forceinline__ float load1(const void *base, int64_t off);
template <>
__device__ __forceinline__ float load1<float>(const void *base, int64_t off) {
    return static_cast<const float *>(base)[off];
}
template <>
__device__ __forceinline__ float load1<uint16_t>(const void *base, int64_t off) {
    return bf16_to_f32(static_cast<const uint16_t *>(base)[off]);
}

// ------------------------------------------------------------ LANE family
// PRIV: the whole output privatised in LDS (out_rows x R per block).
// HOT (levels below the root): the `hot` most frequent output rows privatised
// in LDS (rows by frequency rank), the others updated with global atomics;
// Zipf-hot rows would otherwise serialise their atomics in L2.
// CPL: columns per lane (lane j of a group holds columns j, j + G, ...), so
// that ranks above 32 run two groups of 32 lanes per wave rather than one of 64.
// copy_stride: 0, or the element distance between the per-XCD copies of Y
// (block b then adds into copy b mod XCD_COPIES; any mapping is correct, the
// device-scope atomics only contend less when a copy stays on one XCD).
// AT: accumulator and output type (double: FP64 products and sums for the
// exact fit pass, without LDS copies).
template <int N, int G, typename GT, bool PRIV, bool HOT, int CPL, typename AT = float>
__global__ void __launch_bounds__(256)
k_mttkrp_lane(CsfView cv, FacView fv, int64_t ld, int d, const int32_t *__restrict__ starts,
              int64_t nstreams, int32_t T, AT *__restrict__ Y, int64_t ldo, int R,
              int64_t out_rows, int32_t hot, int64_t copy_stride) {
    extern __shared__ float ypriv[];  // PRIV: out_rows x R; HOT: hot x R
    constexpr int NG = 256 / G;       // groups per block
    constexpr bool LOCAL = PRIV || HOT;
    static_assert(std::is_same<AT, float>::value || !LOCAL, "LDS copies accumulate in float");
    const int lig = threadIdx.x % G;
    Y += (int64_t)(blockIdx.x % XCD_COPIES) * copy_stride;
    bool col[CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) col[q] = lig + G * q < R;
    const int64_t nloc = PRIV ? out_rows * R : (HOT ? (int64_t)hot * R : 0);
    if (LOCAL) {
        for (int64_t j = threadIdx.x; j < nloc; j += 256) ypriv[j] = 0.0f;
        __syncthreads();
    }
    // persistent over streams when privatised (one flush per block), else one
    // stream per group
    const int64_t g0 = (int64_t)blockIdx.x * NG + threadIdx.x / G;
    const int64_t gstep = LOCAL ? (int64_t)gridDim.x * NG : nstreams + 1;
    // add acc to output row `row` (column lig + G*q)
    auto add_row = [&](int32_t row, const AT (&acc)[CPL]) {
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
            if (!col[q]) continue;
            const int cq = lig + G * q;
            if constexpr (LOCAL) {
                if (PRIV) atomicAdd(&ypriv[(int64_t)row * R + cq], acc[q]);
                else if (HOT && cv.hot_rank[row] < hot)
                    atomicAdd(&ypriv[(int64_t)cv.hot_rank[row] * R + cq], acc[q]);
                else atomicAdd(Y + (int64_t)row * ldo + cq, acc[q]);
            } else {
                atomicAdd(Y + (int64_t)row * ldo + cq, acc[q]);
            }
        }
    };
    for (int64_t sid = g0; sid < nstreams; sid += gstep) {
        int64_t k = sid * (int64_t)T;
        const int64_t kend = min(k + (int64_t)T, cv.nleaves);
        int32_t c[N - 1], e[N - 1];
#pragma unroll
        for (int l = 0; l < N - 1; ++l) {
            c[l] = starts[(int64_t)l * nstreams + sid];
            e[l] = cv.fptr[l][c[l] + 1];
        }
        AT H[CPL];
        auto make_H = [&]() {
#pragma unroll
            for (int q = 0; q < CPL; ++q) H[q] = 1;
#pragma unroll
            for (int l = 0; l < N - 1; ++l) {
                if (l == d) continue;
                const int64_t base = (int64_t)cv.fids[l][c[l]] * ld + lig;
#pragma unroll
                for (int q = 0; q < CPL; ++q) H[q] *= col[q] ? (AT)load1<GT>(fv.a[l], base + G * q) : (AT)0;
            }
        };
        make_H();
        AT acc[CPL];
#pragma unroll
        for (int q = 0; q < CPL; ++q) acc[q] = 0;
        int32_t out_row = d < N - 1 ? cv.fids[d][c[d]] : 0;
        // without the hot-row table the next leaf's value and index are loaded
        // a leaf ahead (6-14% faster at level 1 on the three benchmark shapes;
        // with the table it measured 0-15% slower, also with the leaf's rank
        // loaded ahead, so those forms load in place)
        float v_n = 0.0f;
        int32_t i_n = 0;
        if (!HOT && k < kend) {
            v_n = cv.vals[k];
            i_n = cv.fids[N - 1][k];
        }
        for (; k < kend; ++k) {
            float v;
            int32_t i;
            if (!HOT) {
                v = v_n;
                i = i_n;
                if (k + 1 < kend) {
                    v_n = cv.vals[k + 1];
                    i_n = cv.fids[N - 1][k + 1];
                }
            }
            if (k == e[N - 2]) {
                int lmin = N - 2;
                c[N - 2] += 1;
                e[N - 2] = cv.fptr[N - 2][c[N - 2] + 1];
                int32_t child = c[N - 2];
#pragma unroll
                for (int l = N - 3; l >= 0; --l) {
                    if (child != e[l]) break;
                    c[l] += 1;
                    e[l] = cv.fptr[l][c[l] + 1];
                    child = c[l];
                    lmin = l;
                }
                if (d < N - 1 && lmin <= d) {
                    add_row(out_row, acc);
#pragma unroll
                    for (int q = 0; q < CPL; ++q) acc[q] = 0;
                    out_row = cv.fids[d][c[d]];
                }
                make_H();
            }
            if (HOT) {
                v = cv.vals[k];
                i = cv.fids[N - 1][k];
            }
            if (d == N - 1) {
                AT t[CPL];
#pragma unroll
                for (int q = 0; q < CPL; ++q) t[q] = (AT)v * H[q];
                if constexpr (HOT) {
                    const int32_t rk = cv.leafw[k] & ((1 << 29) - 1);
#pragma unroll
                    for (int q = 0; q < CPL; ++q) {
                        if (!col[q]) continue;
                        const int cq = lig + G * q;
                        if (rk < hot) atomicAdd(&ypriv[(int64_t)rk * R + cq], t[q]);
                        else atomicAdd(Y + (int64_t)i * ldo + cq, t[q]);
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < CPL; ++q) {
                        if (!col[q]) continue;
                        const int cq = lig + G * q;
                        if constexpr (PRIV) atomicAdd(&ypriv[(int64_t)i * R + cq], t[q]);
                        else atomicAdd(Y + (int64_t)i * ldo + cq, t[q]);
                    }
                }
            } else {
                const int64_t base = (int64_t)i * ld + lig;
#pragma unroll
                for (int q = 0; q < CPL; ++q) {
                    const float a = col[q] ? load1<GT>(fv.a[N - 1], base + G * q) : 0.0f;
                    if constexpr (std::is_same<AT, float>::value) acc[q] = fmaf(v * a, H[q], acc[q]);
                    else acc[q] = fma((double)v * (double)a, H[q], acc[q]);
                }
            }
        }
        if (d < N - 1) add_row(out_row, acc);
    }
    if constexpr (LOCAL) {
        __syncthreads();
        for (int64_t j = threadIdx.x; j < nloc; j += 256) {
            float v = ypriv[j];
            const int64_t row = PRIV ? j / R : (int64_t)cv.hot_perm[j / R];
            if (v != 0.0f) atomicAdd(Y + row * ldo + (j % R), v);
        }
    }
}

// Y(i, r) = sum of the per-XCD copies in copy order (copies: P x rows x R).
__global__ void __launch_bounds__(256)
k_sum_copies(const float *__restrict__ cp, int P, int64_t rows, int R, float *__restrict__ Y, int64_t ldo) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= rows * R) return;
    float v = 0.0f;
    for (int q = 0; q < P; ++q) v += cp[(int64_t)q * rows * R + j];
    Y[(j / R) * ldo + (j % R)] = v;
}

template <typename AT>
__global__ void k_zero_rows(AT *Y, int64_t rows, int64_t ldo, int R) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= rows * R) return;
    Y[(j / R) * ldo + (j % R)] = 0;
}

// ------------------------------------------------------------ dispatch
// Padded row widths with a ROW kernel: fp32 rows load as float4, bf16 rows as
// 8-element chunks.
inline int row_width(int R, bool bf16) {
    if (R <= 8) return bf16 ? 16 : 8;  // rows of at least two 16-byte chunks
    if (R <= 16) return 16;
    if (R <= 32) return 32;
    if (!bf16 && R <= 36) return 36;
    if (bf16 && R <= 40) return 40;
    return 64;
}


template <int N, typename GT>
cpd_status launch_lane(int G, bool priv, int32_t hot, dim3 grid, size_t lds, hipStream_t s, const CsfView &cv,
                       const FacView &fv, int64_t ld, int d, const int32_t *starts, int64_t ns,
                       int32_t T, float *Y, int64_t ldo, int R, int64_t out_rows, int64_t copy_stride) {
#define CPD_LANE_CASE2(gcase, g, cpl)                                                                          \
    case gcase:                                                                                               \
        if (priv)                                                                                             \
            hipLaunchKernelGGL((k_mttkrp_lane<N, g, GT, true, false, cpl>), grid, dim3(256), lds, s, cv, fv, ld, \
                               d, starts, ns, T, Y, ldo, R, out_rows, 0, 0);                                  \
        else if (hot)                                                                                         \
            hipLaunchKernelGGL((k_mttkrp_lane<N, g, GT, false, true, cpl>), grid, dim3(256), lds, s, cv, fv, ld, \
                               d, starts, ns, T, Y, ldo, R, out_rows, hot, copy_stride);                      \
        else                                                                                                  \
            hipLaunchKernelGGL((k_mttkrp_lane<N, g, GT, false, false, cpl>), grid, dim3(256), 0, s, cv, fv, ld, \
                               d, starts, ns, T, Y, ldo, R, out_rows, 0, copy_stride);                        \
        break;
#define CPD_LANE_CASE(g) CPD_LANE_CASE2(g, g, 1)
    switch (G) {
        CPD_LANE_CASE(8)
        CPD_LANE_CASE(16)
        CPD_LANE_CASE(32)
        CPD_LANE_CASE(64)
        CPD_LANE_CASE2(-64, 32, 2)  // two groups of 32 lanes per wave, two columns per lane
        default:
            CPD_FAIL(CPD_EUNSUPPORTED, "no lane kernel for group %d", G);
    }
#undef CPD_LANE_CASE
#undef CPD_LANE_CASE2
    CPD_LAUNCH_CHECK();
    return CPD_OK;
}

constexpr size_t PRIV_LDS_MAX = 64 * 1024;
// LDS per wave of the tiled kernel (its tile's rows + its H table) by
// default: 32 waves per CU resident (measured on the three benchmark shapes:
// NELL-2 rank 35 2.5 ms at 16-24 rows per tile against 4.1 ms at 64 and
// 10 ms at 256 and more; NETFLIX rank 16 and 4-mode rank 32 flat within 10%
// from 16 to 64 rows)
constexpr size_t TILED_LDS = 5 * 1024;
constexpr int32_t TILED_MIN_ROWS = 16;
// AUTO takes TILED at an internal level (single ascending trees, ms TILED
// vs the fastest other kernel: NELL-2 rank 35 level 1 2.08 vs 3.36 (ROW);
// NETFLIX rank 16 level 1 2.22 vs 2.30 (ROW); 4-mode rank 32 level 1 1.50 vs
// 2.07 (ROW), level 2 1.50 vs 4.46 (LANE))
constexpr size_t HOT_LDS = 16 * 1024;   // hot output rows privatised per block
constexpr int64_t HOT_BLOCKS = 16384;   // blocks looping over the streams (measured best of 2,048-65,536)
constexpr double PRIV_THRESH = 0.02;  // privatise iff rows * copies <= 0.02 * nnz

}  // namespace

cpd_status launch_root(int N, bool bf16, int RP, int d, const int32_t *const *fids, const int32_t *const *fptr,
                       const float *vals, const int32_t *leafw, const int32_t *leaf_perm, const int32_t *const *uprow,
                       const int64_t *counts, const int64_t *dims_by_level, const void *const *fac_by_level,
                       int64_t ld, const int32_t *starts, int64_t ntiles, int32_t T, float *Y, int64_t ldo, int R,
                       void *perm_buf, const int32_t *hot_rank, const int32_t *hot_perm, int32_t hot,
                       hipStream_t s);
cpd_status launch_root64(int N, int RP, const int32_t *const *fids, const int32_t *const *fptr, const float *vals,
                         const int32_t *leafw, const int32_t *leaf_perm, const int32_t *const *uprow,
                         const int64_t *counts, const int64_t *dims_by_level, const void *const *fac_by_level,
                         int64_t ld, const int32_t *starts, int64_t ntiles, int32_t T, double *Y, int64_t ldo, int R,
                         hipStream_t s);

cpd_status launch_leaf(int N, bool bf16, const int32_t *const *fids, const float *vals, const int32_t *leafw,
                       const int32_t *const *uprow, const int32_t *hot_perm, int32_t hot, int64_t nleaves,
                       const void *const *fac_by_level, int64_t ld, const int32_t *starts, int64_t ntiles, int32_t T,
                       float *Y, int64_t ldo, int R, hipStream_t s);

int32_t tiled_height(int R, size_t lds_max);
cpd_status launch_tiled(int N, bool bf16, const cpd_csf_s::LeafTiling &lt, int64_t nleaves,
                        const void *const *fac_by_level, int64_t ld, float *Y, int64_t ldo, int R, hipStream_t s);

// Lanes the root kernel gives one leaf for a padded rank RP.
int root_lanes_per_leaf(int RP, bool bf16);

// Internal levels with ROW: the hot-row LDS table (variant AUTO) is used
// when the level's nodes hold fewer than MID_HOT_LEAVES leaves on average.
// Measured on the single ascending trees of the benchmark shapes: at 5.8-11.7
// leaves per node the table made ROW 1.2-1.6x slower (its LDS costs resident
// waves; a row there gets few flushes), at 1.5 leaves per node 3.2x faster.
constexpr int64_t MID_HOT_LEAVES = 4;

// Kernel family for a request (host-only rule, also exported as
// cpd_mttkrp_plan).  The ROW kernels are instantiated for 3..5 modes and
// non-leaf output levels; they load 16-byte row chunks, so the padded row must
// fit in ld and rows must be 16-byte multiples; they address a gathered row
// as a 32-bit byte offset formed by a 24-bit multiply (row id times row
// bytes), so every gathered level needs row ids below 2^24 and
// rows * row bytes <= 2^32; they read the tree's leaf words.  The ROUND
// kernel serves the leaf level, the TILED kernels every level below the root
// (on that level's mode tiling): they read the leaf words and gather rows in
// 4-element chunks, so ld must be a multiple of 4 covering the rank rounded
// up to 4, with 16-byte aligned factors.  AUTO: ROW where it applies, else
// TILED at the leaf level, else LANE.
cpd_status mttkrp_plan(int N, const int64_t *dims_by_level, int d, int64_t ld, int R, bool bf16, int request,
                       bool rows_aligned, bool leaf_words, int *kernel) {
    if (N < 2 || N > 5) CPD_FAIL(CPD_EUNSUPPORTED, "MTTKRP kernels are built for 2..5 modes, not %d", N);
    if (d < 0 || d >= N) CPD_FAIL(CPD_EINVAL, "depth %d not in [0, %d)", d, N);
    if (R < 1 || R > CPD_MAX_RANK) CPD_FAIL(CPD_EINVAL, "rank %d not in [1, %d]", R, CPD_MAX_RANK);
    if (ld < R) CPD_FAIL(CPD_EINVAL, "ld %lld below rank %d", (long long)ld, R);
    if (request != CPD_KERNEL_AUTO && request != CPD_KERNEL_ROW && request != CPD_KERNEL_LANE &&
        request != CPD_KERNEL_ROUND && request != CPD_KERNEL_TILED)
        CPD_FAIL(CPD_EINVAL, "unknown kernel %d", request);
    const int RP = row_width(R, bf16);
    const int64_t rowb = ld * (bf16 ? 2 : 4);
    bool row_ok = N >= 3 && d < N - 1 && ld >= RP && rowb % 16 == 0 && rowb < (1 << 24) && rows_aligned &&
                  leaf_words;
    for (int l = 0; l < N && row_ok; ++l) {
        if (l == d) continue;
        const int64_t rows = dims_by_level[l];
        if (rows >= (1 << 24) || rows * rowb > (int64_t(1) << 32)) row_ok = false;
    }
    if (request == CPD_KERNEL_ROW && !row_ok)
        CPD_FAIL(CPD_EUNSUPPORTED,
                 "row kernel needs 3..5 modes, a non-leaf mode, ld >= %d, 16-byte rows, row ids below 2^24 and "
                 "rows * row bytes <= 2^32 at every gathered level",
                 RP);
    // ROUND (the leaf level) and TILED (every level below the root) gather
    // 4-element chunks
    const bool quad_ok = leaf_words && rows_aligned && ld % 4 == 0 && ld >= ((R + 3) & ~3);
    const bool round_ok = quad_ok && d == N - 1;
    const bool tiled_ok = quad_ok && d >= 1;
    if (request == CPD_KERNEL_ROUND && !round_ok)
        CPD_FAIL(CPD_EUNSUPPORTED,
                 "round kernel needs the leaf level, leaf words, ld a multiple of 4 covering the rank and 16-byte "
                 "aligned factors");
    if (request == CPD_KERNEL_TILED && !tiled_ok)
        CPD_FAIL(CPD_EUNSUPPORTED,
                 "tiled kernel needs a level below the root, leaf words, ld a multiple of 4 covering the rank and "
                 "16-byte aligned factors");
    if (request != CPD_KERNEL_AUTO) *kernel = request;
    else *kernel = row_ok ? CPD_KERNEL_ROW : round_ok ? CPD_KERNEL_TILED : CPD_KERNEL_LANE;
    return CPD_OK;
}

// Tile table for width T: cached in the handle (created on first use), or
// with a workspace the cached one or one computed into the workspace.
static cpd_status tiles_for(cpd_csf_s *c, int32_t T, Workspace *ws, const int32_t **starts, int64_t *ns,
                            hipStream_t s) {
    if (!ws) return csf_tiles(c, T, starts, ns, s);
    const int64_t nt = ceil_div(c->counts[c->nmodes - 1], T);
    const size_t need = sizeof(int32_t) * (size_t)std::max<int64_t>(1, (c->nmodes - 1) * nt);
    void *dst = ws->take(need);
    return csf_tiles_into(c, T, static_cast<int32_t *>(dst), dst ? need : 0, starts, ns, s);
}

// Internal entry (also used by the ALS driver).
cpd_status mttkrp(cpd_csf_s *c, const void *const *factors, int32_t ld, int32_t R, int32_t mode,
                  float *Y, int32_t ldo, const cpd_mttkrp_opts *opts, hipStream_t s, hipEvent_t ev0,
                  hipEvent_t ev1) {
    return mttkrp_ws(c, factors, ld, R, mode, Y, ldo, opts, s, ev0, ev1, nullptr);
}

// ws: null (temporaries from the stream's scratch cache, tables cached in
// the handle on first use), or device memory every temporary is carved from
// (no allocation; missing tables are computed into it, a level without a
// ranking runs without the hot-row table).
cpd_status mttkrp_ws(cpd_csf_s *c, const void *const *factors, int32_t ld, int32_t R, int32_t mode, float *Y,
                     int32_t ldo, const cpd_mttkrp_opts *opts, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1,
                     Workspace *ws) {
    if (!c) CPD_FAIL(CPD_EINVAL, "null CSF handle");
    const int N = c->nmodes;
    if (R < 1 || R > CPD_MAX_RANK) CPD_FAIL(CPD_EINVAL, "rank %d not in [1, %d]", R, CPD_MAX_RANK);
    if (mode < 0 || mode >= N) CPD_FAIL(CPD_EINVAL, "mode %d not in [0, %d)", mode, N);
    if (!factors || !Y) CPD_FAIL(CPD_EINVAL, "null factors or output");
    if (ld < R || ldo < R) CPD_FAIL(CPD_EINVAL, "ld %d / ldo %d below rank %d", ld, ldo, R);
    cpd_mttkrp_opts o = opts ? *opts : cpd_mttkrp_opts{CPD_FP32, CPD_VARIANT_AUTO, CPD_KERNEL_AUTO, 0};
    if (o.precision != CPD_FP32 && o.precision != CPD_BF16_GATHER)
        CPD_FAIL(CPD_EINVAL, "unknown precision %d", o.precision);
    if (o.tile_nnz < 0) CPD_FAIL(CPD_EINVAL, "tile_nnz %d < 0", o.tile_nnz);
    const bool bf16 = o.precision == CPD_BF16_GATHER;
    const int d = c->depth_of(mode);
    CsfView cv{};
    FacView fv{};
    for (int l = 0; l < N; ++l) {
        cv.fids[l] = c->fids[l];
        cv.fptr[l] = c->fptr[l];
        const int m = c->order[l];
        fv.a[l] = factors[m];
        if (m != mode && !factors[m]) CPD_FAIL(CPD_EINVAL, "null factor for mode %d", m);
    }
    cv.vals = c->vals;
    cv.nleaves = c->counts[N - 1];
    cv.leafw = c->leafw;
    const int64_t out_rows = c->dims[mode];

    const int RP = row_width(R, bf16);
    int64_t dims_by_level[CPD_MAX_MODES];
    for (int l = 0; l < N; ++l) dims_by_level[l] = c->dims[c->order[l]];
    bool aligned = true;
    for (int l = 0; l < N; ++l)
        if (c->order[l] != mode && (reinterpret_cast<uintptr_t>(factors[c->order[l]]) & 15)) aligned = false;
    int kernel = CPD_KERNEL_LANE;
    CPD_TRY(mttkrp_plan(N, dims_by_level, d, ld, R, bf16, o.kernel, aligned, c->leafw != nullptr, &kernel));
    // AUTO at an internal level with the variant left to the library: TILED
    // where it applies (it has no privatised variant)
    if (o.kernel == CPD_KERNEL_AUTO && o.variant == CPD_VARIANT_AUTO && d >= 1 && d < N - 1 && c->leafw &&
        aligned && ld % 4 == 0 && ld >= ((R + 3) & ~3))
        kernel = CPD_KERNEL_TILED;

    // zero the output (columns < R)
    {
        int64_t tot = out_rows * R;
        hipLaunchKernelGGL(k_zero_rows<float>, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, s, Y, out_rows,
                           (int64_t)ldo, R);
        CPD_LAUNCH_CHECK();
    }
    auto row_path = [&]() -> cpd_status {
        // default tile: 128 leaves per group run, halved (down to 32) while
        // the tile steps would not give every resident wave two of them
        int32_t T = o.tile_nnz;
        if (!T) {
            const int64_t groups = 64 / root_lanes_per_leaf(RP, bf16), waves = 256 * 16;
            T = 128;
            while (T > 32 && cv.nleaves < groups * T * 2 * waves) T /= 2;
        }

        const int32_t *starts;
        int64_t ns;
        CPD_TRY(tiles_for(c, T, ws, &starts, &ns, s));
        const void *fac_by_level[CPD_MAX_MODES];
        for (int l = 0; l < N; ++l) fac_by_level[l] = fv.a[l];
        void *perm_buf = nullptr;  // the leaf factor in rank order
        if (ws) {
            const size_t need = (size_t)dims_by_level[N - 1] * ld * (bf16 ? 2 : 4);
            perm_buf = ws->take(need);
            if (!perm_buf)
                CPD_FAIL(CPD_EUNSUPPORTED, "the leaf factor copy (%zu bytes) does not fit the %zu-byte workspace",
                         need, ws->bytes);
        }
        // internal levels: the most frequent output rows accumulate in LDS
        // (PRIVATE), or not (ATOMIC); AUTO: when the level's nodes are short
        const int32_t *hot_perm = nullptr, *hot_rank = nullptr;
        int32_t hot = 0;
        const bool use_hot = o.variant == CPD_VARIANT_PRIVATE ||
                             (o.variant == CPD_VARIANT_AUTO && c->counts[d] * MID_HOT_LEAVES > c->counts[N - 1]);
        if (d > 0 && use_hot) {
            if (ws) csf_level_rank_cached(c, d, &hot_perm, &hot_rank);
            else CPD_TRY(csf_level_rank(c, d, &hot_perm, &hot_rank, s));
            if (hot_perm) hot = (int32_t)std::min<int64_t>(out_rows, (int64_t)(HOT_LDS / (sizeof(float) * R)));
        }
        if (ev0) CPD_HIP(hipEventRecord(ev0, s));
        cpd_status st = launch_root(N, bf16, RP, d, cv.fids, cv.fptr, cv.vals, c->leafw, c->leaf_perm, c->uprow,
                                    c->counts, dims_by_level, fac_by_level, ld, starts, ns, T, Y, ldo, R, perm_buf,
                                    hot_rank, hot_perm, hot, s);
        if (st == CPD_OK && ev1) CPD_HIP(hipEventRecord(ev1, s));
        return st;
    };
    if (kernel == CPD_KERNEL_ROW) return row_path();
    // the privatised variant below the root runs LANE (AUTO) or is refused (ROUND, TILED asked for)
    if ((kernel == CPD_KERNEL_ROUND || kernel == CPD_KERNEL_TILED) && o.variant == CPD_VARIANT_PRIVATE) {
        if (o.kernel != CPD_KERNEL_AUTO)
            CPD_FAIL(CPD_EUNSUPPORTED, "the round and tiled kernels have no privatised variant");
        kernel = CPD_KERNEL_LANE;
    }
    if (kernel == CPD_KERNEL_TILED) {
        // the tile height that fits a block's LDS; the tiling is built on first
        // use (with a workspace only a cached one is used, else the leaf level
        // runs ROUND and an internal level the kernel AUTO takes there)
        int dev = 0, lds_max = 64 * 1024;
        if (hipGetDevice(&dev) == hipSuccess) {
            int v = 0;
            if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
                lds_max = v;
        }
        (void)hipGetLastError();
        // tile height: tile_nnz when given (capped by the LDS), else the rows
        // that fit TILED_LDS bytes per wave (several waves resident per SIMD).
        // The leaf level's tiling keeps tree order inside a tile (a fiber's
        // leaves consecutive); an internal level's is ordered by size: the
        // rows of its largest other factor repeat in runs and stay in the L1,
        // the rows gathered per leaf come from smaller factors that stay in
        // the L2 (tree order there gathers a row of the leaf factor per leaf)
        const bool leaf = d == N - 1;
        const int order = leaf ? cpd_csf_s::TILE_TREE : cpd_csf_s::TILE_BY_SIZE;
        const size_t lds_cap = (size_t)std::min(lds_max, 160 * 1024) / 4;
        const int32_t Bmax = tiled_height(R, lds_cap);
        const int32_t Bdef = std::max(tiled_height(R, TILED_LDS), TILED_MIN_ROWS);
        const int32_t B = o.tile_nnz > 0 ? std::min<int32_t>(o.tile_nnz, Bmax) : std::min(Bdef, Bmax);
        cpd_csf_s::LeafTiling lt;
        bool no_room = false;  // AUTO and no device memory for the tiling
        if (B >= 1) {
            const cpd_status st = csf_level_tiling(c, d, B, order, ws != nullptr, &lt, s);
            if (st == CPD_ENOMEM && o.kernel == CPD_KERNEL_AUTO) no_room = true;
            else if (st != CPD_OK) return st;
        }
        if (lt.B > 0) {
            const void *fac_by_level[CPD_MAX_MODES];
            for (int l = 0; l < N; ++l) fac_by_level[l] = fv.a[l];
            if (ev0) CPD_HIP(hipEventRecord(ev0, s));
            cpd_status st = launch_tiled(N, bf16, lt, cv.nleaves, fac_by_level, ld, Y, ldo, R, s);
            if (st == CPD_OK && ev1) CPD_HIP(hipEventRecord(ev1, s));
            return st;
        }
        if (!ws && !no_room) CPD_FAIL(CPD_EUNSUPPORTED, "no mode tiling fits %d bytes of LDS at rank %d", lds_max, R);
        // allocation-free call on a tree without a cached tiling, or AUTO
        // without the device memory to build one: a kernel that needs no tiling
        if (leaf) {
            kernel = CPD_KERNEL_ROUND;
            if (o.tile_nnz == 0) o.tile_nnz = 256;
        } else {
            CPD_TRY(mttkrp_plan(N, dims_by_level, d, ld, R, bf16, CPD_KERNEL_AUTO, aligned, c->leafw != nullptr,
                                &kernel));
            o.tile_nnz = 0;
            if (kernel == CPD_KERNEL_ROW) return row_path();
        }
    }
    if (kernel == CPD_KERNEL_ROUND) {
        // tiles of whole 64-leaf rounds
        const int32_t T = o.tile_nnz ? (int32_t)(ceil_div(o.tile_nnz, 64) * 64) : 256;
        const int32_t *starts;
        int64_t ns;
        CPD_TRY(tiles_for(c, T, ws, &starts, &ns, s));
        const int32_t *hot_perm = nullptr, *hot_rank = nullptr;
        if (ws) csf_level_rank_cached(c, N - 1, &hot_perm, &hot_rank);
        else CPD_TRY(csf_level_rank(c, N - 1, &hot_perm, &hot_rank, s));
        const int32_t hot =
            hot_perm ? (int32_t)std::min<int64_t>(out_rows, (int64_t)(HOT_LDS / (sizeof(float) * R))) : 0;
        const void *fac_by_level[CPD_MAX_MODES];
        for (int l = 0; l < N; ++l) fac_by_level[l] = fv.a[l];
        if (ev0) CPD_HIP(hipEventRecord(ev0, s));
        cpd_status st = launch_leaf(N, bf16, cv.fids, cv.vals, c->leafw, c->uprow, hot_perm, hot, cv.nleaves,
                                    fac_by_level, ld, starts, ns, T, Y, ldo, R, s);
        if (st == CPD_OK && ev1) CPD_HIP(hipEventRecord(ev1, s));
        return st;
    }
    // LANE family
    int G = R <= 8 ? 8 : R <= 16 ? 16 : R <= 32 ? 32 : 64;
    int32_t T = o.tile_nnz ? o.tile_nnz : 256;
    const int32_t *starts;
    int64_t ns;
    CPD_TRY(tiles_for(c, T, ws, &starts, &ns, s));
    const size_t lds = (size_t)out_rows * R * sizeof(float);
    bool priv = false;
    if (d >= 1 && lds <= PRIV_LDS_MAX) {
        const int64_t copies = 1024;  // persistent blocks below
        if (o.variant == CPD_VARIANT_PRIVATE) priv = true;
        else if (o.variant == CPD_VARIANT_AUTO)
            priv = (double)out_rows * copies <= PRIV_THRESH * (double)cv.nleaves;
    }
    // privatised but too large for LDS: one HBM copy of Y per XCD (asked for
    // explicitly; AUTO keeps global atomics there)
    const bool xcd_copies = o.variant == CPD_VARIANT_PRIVATE && !priv;
    if (xcd_copies && d < 1) CPD_FAIL(CPD_EUNSUPPORTED, "private variant needs a non-root mode");
    // levels 2 and deeper with atomics: the most frequent output rows (by the
    // tree's ranking of that level) accumulate in LDS, HOT_LDS bytes per block.
    // A level-1 row gets at most one flush per root index, too few for the
    // table to pay for itself (measured slower on all three benchmark shapes).
    int32_t hot = 0;
    size_t lds_launch = lds;
    if (!priv && d >= 2 && c->leafw) {
        if (ws) csf_level_rank_cached(c, d, &cv.hot_perm, &cv.hot_rank);
        else CPD_TRY(csf_level_rank(c, d, &cv.hot_perm, &cv.hot_rank, s));
        if (cv.hot_perm) {
            hot = (int32_t)std::min<int64_t>(c->dims[mode], (int64_t)(HOT_LDS / (sizeof(float) * R)));
            if (hot < 32) hot = 0;
            lds_launch = (size_t)hot * R * sizeof(float);
        }
    }
    // ranks above 32 below the leaf level: groups of 32 lanes holding two
    // columns each (measured 1.35-1.47x faster than one 64-lane group on the
    // rank-35 NELL-2 tree; at the leaf level the extra atomic instructions of
    // the split made it slower)
    if (G == 64 && d < N - 1) G = -64;
    const int NG = 256 / (G == -64 ? 32 : G);
    dim3 grid = priv ? dim3((unsigned)std::min<int64_t>(1024, ceil_div(ns, NG)))
                     : hot ? dim3((unsigned)std::min<int64_t>(HOT_BLOCKS, ceil_div(ns, NG)))
                           : dim3((unsigned)ceil_div(ns, NG));
    if (N < 2 || N > 5) CPD_FAIL(CPD_EUNSUPPORTED, "MTTKRP kernels are built for 2..5 modes, not %d", N);
    DevBuf<float> copies;
    float *Yk = Y;
    int64_t ldk = ldo, copy_stride = 0;
    if (xcd_copies) {
        copy_stride = out_rows * R;
        float *cp = nullptr;
        if (ws) {
            const size_t need = sizeof(float) * (size_t)XCD_COPIES * copy_stride;
            cp = static_cast<float *>(ws->take(need));
            if (!cp)
                CPD_FAIL(CPD_EUNSUPPORTED, "the per-XCD copies (%zu bytes) do not fit the %zu-byte workspace", need,
                         ws->bytes);
        } else {
            CPD_TRY(copies.alloc((size_t)XCD_COPIES * copy_stride, s));
            cp = copies.p;
        }
        const int64_t tot = XCD_COPIES * copy_stride;
        hipLaunchKernelGGL(k_zero_rows<float>, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, s, cp,
                           (int64_t)XCD_COPIES * out_rows, (int64_t)R, R);
        CPD_LAUNCH_CHECK();
        Yk = cp;
        ldk = R;
    }
    if (ev0) CPD_HIP(hipEventRecord(ev0, s));
    cpd_status st = CPD_OK;
#define CPD_LANE_N(n)                                                                                   \
    case n:                                                                                             \
        st = bf16 ? launch_lane<n, uint16_t>(G, priv, hot, grid, lds_launch, s, cv, fv, ld, d, starts, ns, T, Yk, \
                                             ldk, R, out_rows, copy_stride)                             \
                  : launch_lane<n, float>(G, priv, hot, grid, lds_launch, s, cv, fv, ld, d, starts, ns, T, Yk, \
                                          ldk, R, out_rows, copy_stride);                               \
        break;
    switch (N) {
        CPD_LANE_N(2)
        CPD_LANE_N(3)
        CPD_LANE_N(4)
        CPD_LANE_N(5)
    }
#undef CPD_LANE_N
    if (st == CPD_OK && xcd_copies) {
        // the copies live in the workspace or in `copies`: Yk points at them either way
        hipLaunchKernelGGL(k_sum_copies, dim3((unsigned)ceil_div(copy_stride, 256)), dim3(256), 0, s,
                           (const float *)Yk, XCD_COPIES, out_rows, R, Y, (int64_t)ldo);
        CPD_LAUNCH_CHECK();
    }
    if (st == CPD_OK && ev1) CPD_HIP(hipEventRecord(ev1, s));
    return st;
}

// MTTKRP with float rows and FP64 products and sums into a double output (the
// exact fit pass of the ALS driver): the root kernel when the mode is the
// tree's root and the ROW rule allows it, else the LANE kernel with FP64
// atomics.  Y: dims[mode] x ldo doubles, columns < R overwritten.
cpd_status mttkrp64(cpd_csf_s *c, const float *const *factors, int32_t ld, int32_t R, int32_t mode, double *Y,
                    int32_t ldo, hipStream_t s) {
    if (!c || !factors || !Y) CPD_FAIL(CPD_EINVAL, "null argument");
    const int N = c->nmodes;
    if (R < 1 || R > CPD_MAX_RANK || mode < 0 || mode >= N || ld < R || ldo < R)
        CPD_FAIL(CPD_EINVAL, "bad FP64 MTTKRP arguments");
    const int d = c->depth_of(mode);
    CsfView cv{};
    FacView fv{};
    int64_t dims_by_level[CPD_MAX_MODES];
    bool aligned = true;
    for (int l = 0; l < N; ++l) {
        cv.fids[l] = c->fids[l];
        cv.fptr[l] = c->fptr[l];
        const int m = c->order[l];
        fv.a[l] = factors[m];
        dims_by_level[l] = c->dims[m];
        if (m != mode && !factors[m]) CPD_FAIL(CPD_EINVAL, "null factor for mode %d", m);
        if (m != mode && (reinterpret_cast<uintptr_t>(factors[m]) & 15)) aligned = false;
    }
    cv.vals = c->vals;
    cv.nleaves = c->counts[N - 1];
    cv.leafw = c->leafw;
    const int64_t out_rows = c->dims[mode];
    int kernel = CPD_KERNEL_LANE;
    CPD_TRY(mttkrp_plan(N, dims_by_level, d, ld, R, false, CPD_KERNEL_AUTO, aligned, c->leafw != nullptr, &kernel));
    {
        const int64_t tot = out_rows * R;
        hipLaunchKernelGGL(k_zero_rows<double>, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, s, Y, out_rows,
                           (int64_t)ldo, R);
        CPD_LAUNCH_CHECK();
    }
    if (kernel == CPD_KERNEL_ROW) {
        const int RP = row_width(R, false);
        const int64_t groups = 64 / root_lanes_per_leaf(RP, false), waves = 256 * 16;
        int32_t T = 128;
        while (T > 32 && cv.nleaves < groups * T * 2 * waves) T /= 2;
        const int32_t *starts;
        int64_t ns;
        CPD_TRY(csf_tiles(c, T, &starts, &ns, s));
        const void *fac_by_level[CPD_MAX_MODES];
        for (int l = 0; l < N; ++l) fac_by_level[l] = fv.a[l];
        return launch_root64(N, RP, cv.fids, cv.fptr, cv.vals, c->leafw, c->leaf_perm, c->uprow, c->counts,
                             dims_by_level, fac_by_level, ld, starts, ns, T, Y, ldo, R, s);
    }
    int G = R <= 8 ? 8 : R <= 16 ? 16 : R <= 32 ? 32 : 64;
    const int32_t T = 256;
    const int32_t *starts;
    int64_t ns;
    CPD_TRY(csf_tiles(c, T, &starts, &ns, s));
    if (G == 64 && d < N - 1) G = -64;
    const int NG = 256 / (G == -64 ? 32 : G);
    const dim3 grid((unsigned)ceil_div(ns, NG));
#define CPD_LANE64(n, g, cpl)                                                                                  \
    hipLaunchKernelGGL((k_mttkrp_lane<n, g, float, false, false, cpl, double>), grid, dim3(256), 0, s, cv, fv, \
                       (int64_t)ld, d, starts, ns, T, Y, (int64_t)ldo, R, out_rows, 0, (int64_t)0)
#define CPD_LANE64_G(n)                          \
    switch (G) {                                 \
        case 8: CPD_LANE64(n, 8, 1); break;      \
        case 16: CPD_LANE64(n, 16, 1); break;    \
        case 32: CPD_LANE64(n, 32, 1); break;    \
        case 64: CPD_LANE64(n, 64, 1); break;    \
        default: CPD_LANE64(n, 32, 2); break;    \
    }
    switch (N) {
        case 2: CPD_LANE64_G(2) break;
        case 3: CPD_LANE64_G(3) break;
        case 4: CPD_LANE64_G(4) break;
        case 5: CPD_LANE64_G(5) break;
        default: CPD_FAIL(CPD_EUNSUPPORTED, "MTTKRP kernels are built for 2..5 modes, not %d", N);
    }
#undef CPD_LANE64_G
#undef CPD_LANE64
    CPD_LAUNCH_CHECK();
    return CPD_OK;
}

}  // namespace cpd

extern "C" cpd_status cpd_mttkrp_plan(int32_t nmodes, const int64_t *dims_by_level, int32_t depth, int32_t ld,
                                      int32_t rank, int32_t precision, int32_t kernel, int32_t rows_aligned,
                                      int32_t leaf_words, int32_t *kernel_out) {
    cpd::clear_error();
    if (!dims_by_level || !kernel_out) CPD_FAIL(CPD_EINVAL, "null argument");
    if (precision != CPD_FP32 && precision != CPD_BF16_GATHER) CPD_FAIL(CPD_EINVAL, "unknown precision %d", precision);
    if (nmodes >= 2 && nmodes <= CPD_MAX_MODES)
        for (int l = 0; l < nmodes; ++l)
            if (dims_by_level[l] < 1) CPD_FAIL(CPD_EINVAL, "length %lld at level %d", (long long)dims_by_level[l], l);
    return cpd::mttkrp_plan(nmodes, dims_by_level, depth, ld, rank, precision == CPD_BF16_GATHER, kernel,
                            rows_aligned != 0, leaf_words != 0, kernel_out);
}

extern "C" cpd_status cpd_mttkrp(cpd_csf csf, const void *const *factors, int32_t ld, int32_t rank,
                                 int32_t mode, float *out, int32_t ldo, const cpd_mttkrp_opts *opts,
                                 void *stream) {
    cpd::clear_error();
    return cpd::mttkrp(csf, factors, ld, rank, mode, out, ldo, opts, (hipStream_t)stream, nullptr, nullptr);
}
