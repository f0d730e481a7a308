// Root-level MTTKRP on a CSF tree (the output mode is the tree's root, as in
// every MTTKRP of a CSF rooted at its own mode; Section III, Algorithm 1):
//     Y(i, :) = sum over leaves k below root node i of x_k * A_leaf(j_k, :) * H_k,
// H_k = Hadamard product of the rows of the internal levels above leaf k.
//
// Lane layout: a group of G lanes handles one leaf at a time, lane j of the
// group holding 16-byte chunks j, j+G, ... of the factor rows, so each load
// instruction reads whole rows as contiguous runs (G = padded rank / 4 for
// FP32, / 8 for BF16) and a wave walks 64/G leaves per step.
//
// Work split, aimed at Zipf-skewed root rows whose leaves span thousands of
// work units: every wave owns a contiguous range of leaves and walks it in
// tile steps of (64/G)*T leaves, group g taking the g-th run of T leaves.
// Partial rows are combined without contention:
//   - a row that starts and ends inside one group's run is stored directly;
//   - the partial of the row open at the end of each run is combined across
//     the wave's groups by a segmented scan (rows are sorted, so equal rows
//     are adjacent groups); a row closed inside the wave's range is stored
//     directly, the row still open after the last group is carried to the
//     next tile step in group 0's accumulator;
//   - only rows that cross the wave's range boundary, and the closing part of
//     a row that began in an earlier group, use atomic adds -- a few per row.
// Every leaf carries the row ids of its internal levels (per-leaf arrays built
// with the tree), so the rows of a block of leaves -- leaf rows and internal
// rows alike -- are gathered together with no pointer chasing; only root-row
// boundaries, read from the leaf words (level << 29 | leaf id), change the
// control flow.  Leaf words, values and internal ids are staged through LDS
// with coalesced loads.
#include <type_traits>

#include "csf.h"

namespace cpd {
namespace {

struct CsfView {
    const int32_t *fids[CPD_MAX_MODES];
    const int32_t *fptr[CPD_MAX_MODES];
    const int32_t *uprow[CPD_MAX_MODES];  // per-leaf ids of levels 1..N-2
    const float *vals;
    const int32_t *leafw;  // (level << 29) | leaf id
    int64_t nleaves;
    // internal levels: the `hot` most frequent output rows (by the level's
    // frequency ranking) accumulate in LDS, the others in Y
    const int32_t *hot_rank;  // output row -> frequency rank
    const int32_t *hot_perm;  // frequency rank -> output row
    int32_t hot;
};

struct FacView {
    const void *a[CPD_MAX_MODES];  // by level
};

// One lane's chunk of a factor row: 4 floats (16 bytes), 8 bfloat16 (16
// bytes) or 4 bfloat16 (8 bytes: the lane layout of the float rows at half
// the bytes), widened to float.  Rows are addressed by a 32-bit byte offset
// from a uniform base (row id times row bytes, both below 2^24), which keeps
// address arithmetic at one 24-bit multiply per row.
struct bf16x4;  // tag: 4 bfloat16 per lane

template <typename GT>
struct Chunk;

// Rows stay in registers as loaded (RAW words per lane: floats, or pairs of
// bfloat16) and are widened element by element at use, which keeps the
// bfloat16 forms at half the registers of widened rows.
template <>
struct Chunk<float> {
    static constexpr int W = 4, BYTES = 16, ELEM = 4, RAW = 4;
    using raw_t = float;
    __device__ static __forceinline__ void load(const char *base, uint32_t off, raw_t *r) {
        const float4 x = *reinterpret_cast<const float4 *>(base + off);
        r[0] = x.x;
        r[1] = x.y;
        r[2] = x.z;
        r[3] = x.w;
    }
    __device__ static __forceinline__ float get(const raw_t *r, int e) { return r[e]; }
};

template <>
struct Chunk<uint16_t> {
    static constexpr int W = 8, BYTES = 16, ELEM = 2, RAW = 4;
    using raw_t = uint32_t;
    __device__ static __forceinline__ void load(const char *base, uint32_t off, raw_t *r) {
        const uint4 x = *reinterpret_cast<const uint4 *>(base + off);
        r[0] = x.x;
        r[1] = x.y;
        r[2] = x.z;
        r[3] = x.w;
    }
    __device__ static __forceinline__ float get(const raw_t *r, int e) {
        return (e & 1) ? bf16_hi(r[e >> 1]) : bf16_lo(r[e >> 1]);
    }
};

template <>
struct Chunk<bf16x4> {
    static constexpr int W = 4, BYTES = 8, ELEM = 2, RAW = 2;
    using raw_t = uint32_t;
    __device__ static __forceinline__ void load(const char *base, uint32_t off, raw_t *r) {
        const uint2 x = *reinterpret_cast<const uint2 *>(base + off);
        r[0] = x.x;
        r[1] = x.y;
    }
    __device__ static __forceinline__ float get(const raw_t *r, int e) {
        return (e & 1) ? bf16_hi(r[e >> 1]) : bf16_lo(r[e >> 1]);
    }
};

// Leaves per LDS staging chunk (per group): fewer when a wave has many groups.
// Larger chunks mean fewer waits on the streamed per-leaf words (measured:
// 32 instead of 16 is 2-6% faster on rank 35 and 16 rows; 16 instead of 8 is
// 11-18% faster at 32 groups; 32 at 32 groups is slower, the staging LDS
// then costs resident waves).
template <int NG>
constexpr int root_chunk() {
    return NG >= 32 ? 16 : 32;
}
constexpr int ROOT_C = 32;      // tile widths must be multiples of this
constexpr int BF16_NARROW_MAX = 16;
constexpr int ROOT_WAVES = 4;   // waves per block

// Leaves per block whose rows are gathered together.  Two: measured faster
// than four or eight on every workload (fewer registers, more resident waves
// to cover the gather latency).
template <int N, typename GT>
constexpr int root_unroll() {
    return 2;
}

// Minimum resident waves per SIMD asked of the compiler for 16-byte bfloat16
// chunks: 6 on 3 modes, 5 on 4 modes (measured faster); no constraint
// otherwise.
template <int N, typename GT>
constexpr int root_min_waves() {
    return !std::is_same<GT, uint16_t>::value ? 1 : N == 3 ? 6 : N == 4 ? 5 : 1;
}

__device__ __forceinline__ void wave_sync_lds_root() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Row stride (in words) of a wave's LDS staging of the leaf stream: C leaves
// per run plus one, so that the groups' reads of one position (one run each)
// fall in different banks.
template <int C>
constexpr int stage_stride() {
    return C + 1;
}

typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Stage leaf words, values and internal ids of positions t0..t0+C-1 of the
// NG runs of a tile step (run s starts at leaf base + s*T) into the wave's
// LDS rows: 16-byte loads, four leaves a lane (runs and chunks start at
// multiples of 4 leaves and the tree's arrays are 16-byte aligned), so a
// chunk costs a quarter of the load instructions of one leaf a lane.  The
// four words go to LDS one at a time (the rows' odd stride keeps them in
// distinct banks across the lanes).
template <int NG, int C, int NU>
__device__ __forceinline__ void stage_chunk(const CsfView &cv, int64_t base, int64_t T, int t0, int lane,
                                            int32_t *sw, float *sv, int32_t (*su)[NG * stage_stride<C>()]) {
    constexpr int Q = C / 4, S = stage_stride<C>();
    const int64_t nleaves = cv.nleaves;
    for (int e2 = lane; e2 < NG * Q; e2 += 64) {
        const int s = e2 / Q, j = 4 * (e2 % Q);
        const int64_t k = base + (int64_t)s * T + t0 + j;
        const int at = s * S + j;
        if (k + 4 <= nleaves) {
            const i32x4 w = __builtin_nontemporal_load(reinterpret_cast<const i32x4 *>(cv.leafw + k));
            const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(cv.vals + k));
            i32x4 u[NU > 0 ? NU : 1];
#pragma unroll
            for (int l = 0; l < NU; ++l)
                u[l] = __builtin_nontemporal_load(reinterpret_cast<const i32x4 *>(cv.uprow[l + 1] + k));
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                sw[at + i] = w[i];
                sv[at + i] = v[i];
#pragma unroll
                for (int l = 0; l < NU; ++l) su[l][at + i] = u[l][i];
            }
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const bool in = k + i < nleaves;
                sw[at + i] = in ? stream_load(cv.leafw + k + i) : 0;
                sv[at + i] = in ? stream_load(cv.vals + k + i) : 0.0f;
#pragma unroll
                for (int l = 0; l < NU; ++l) su[l][at + i] = in ? stream_load(cv.uprow[l + 1] + k + i) : 0;
            }
        }
    }
}

// One leaf's contribution x * A_leaf(j, c) * H(c) for element e of a lane's
// chunk, added to the accumulator: FP32 products and sums, or (AT = double,
// float rows only) FP64 products and sums.
template <typename GT, int NU, typename AT, typename raw_t>
__device__ __forceinline__ void leaf_fma(AT &acc, float v, const raw_t *row, const raw_t (*H)[Chunk<GT>::RAW],
                                         int e) {
    if constexpr (std::is_same<AT, float>::value) {
        float h = Chunk<GT>::get(H[0], e);
#pragma unroll
        for (int l = 1; l < NU; ++l) h *= Chunk<GT>::get(H[l], e);
        acc = fmaf(v * Chunk<GT>::get(row, e), h, acc);
    } else {
        double h = (double)Chunk<GT>::get(H[0], e);
#pragma unroll
        for (int l = 1; l < NU; ++l) h *= (double)Chunk<GT>::get(H[l], e);
        acc = fma((double)v * (double)Chunk<GT>::get(row, e), h, acc);
    }
}

// a_leaf: the leaf factor with rows in rank order (row r = factor row
// leaf_perm[r]), so the most used rows share cache lines and pages.
// AT: the accumulator and output type (float; double for the exact fit pass).
template <int N, int G, typename GT, typename AT>
__global__ void __launch_bounds__(64 * ROOT_WAVES, (root_min_waves<N, GT>()))
k_mttkrp_root(CsfView cv, FacView fv, const char *__restrict__ a_leaf, uint32_t rowb,
              const int32_t *__restrict__ starts, int64_t ntiles, int32_t T, int64_t nsteps, int64_t nwaves,
              AT *__restrict__ Y, int64_t ldo, int R) {
    constexpr int NG = 64 / G;  // groups per wave
    constexpr int C = root_chunk<NG>(), U = root_unroll<N, GT>();
    static_assert(C % U == 0 && ROOT_C % C == 0, "staging chunk must hold whole blocks");
    constexpr int W = Chunk<GT>::W;
    constexpr int E = W;        // row elements per lane
    constexpr int NU = N - 2;   // internal levels
    constexpr int SS = NG * stage_stride<C>();
    constexpr int32_t IDMASK = (1 << 29) - 1;
    __shared__ int32_t s_w[ROOT_WAVES][SS];
    __shared__ float s_v[ROOT_WAVES][SS];
    __shared__ int32_t s_u[ROOT_WAVES][NU][SS];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane / G, lig = lane % G;  // g == NG: idle lane
    const int64_t gw = (int64_t)blockIdx.x * ROOT_WAVES + wave;
    if (gw >= nwaves) return;  // waves are independent: no block barriers below
    const int64_t nleaves = cv.nleaves;
    const int64_t s_begin = gw * nsteps / nwaves, s_end = (gw + 1) * nsteps / nwaves;
    const int64_t span = NG * (int64_t)T;
    const int64_t W0 = s_begin * span;  // first leaf of this wave's range
    const int32_t *__restrict__ leafw = cv.leafw;
    const float *__restrict__ vals = cv.vals;
    const int32_t *__restrict__ root_ids = cv.fids[0];
    int32_t *sw = s_w[wave];
    float *sv = s_v[wave];
    const int gs = g < NG ? g : NG - 1;  // staged slot this lane reads (idle lanes never do)
    auto col_of = [&](int e) { return (lig * W) + e; };
    const uint32_t lane_off = (uint32_t)lig * Chunk<GT>::BYTES;  // this lane's chunk within a row
    const char *a_up[NU];
#pragma unroll
    for (int l = 0; l < NU; ++l) a_up[l] = static_cast<const char *>(fv.a[l + 1]);

    AT acc[E];
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = 0;
    int32_t carry_row = -1;  // row carried into group 0 of the next tile step

    for (int64_t st = s_begin; st < s_end; ++st) {
        const int64_t base = st * span;
        const int64_t k0 = base + (int64_t)gs * T;
        const bool active = g < NG && k0 < nleaves;
        const int64_t kend = active ? min(k0 + (int64_t)T, nleaves) : k0;
        const int64_t tile = active ? (base / T + g) : (ntiles - 1);
        int32_t c0 = starts[tile];  // root node of the run's first leaf
        const int32_t w_first = active ? leafw[k0] : 0;
        const int32_t w_next = (active && kend < nleaves) ? leafw[kend] : 0;
        const bool first_here = active && ((uint32_t)w_first >> 29) == 0;  // a root row starts at k0
        bool first_in_range = true;
        if (active && !first_here) {  // first leaf of the current root node
            int64_t fl = c0;
#pragma unroll
            for (int l = 0; l < N - 1; ++l) fl = cv.fptr[l][fl];
            first_in_range = fl >= W0;
        }
        const bool closes_at_end = !active || kend == nleaves || ((uint32_t)w_next >> 29) == 0;
        int32_t cur_row = root_ids[c0];
        bool is_first = true;
        if (g != 0 || carry_row < 0) {
#pragma unroll
            for (int e = 0; e < E; ++e) acc[e] = 0;
        }
        // internal rows of the previous leaf (reused while the ids repeat)
        int32_t last_up[NU];
        using raw_t = typename Chunk<GT>::raw_t;
        constexpr int RW = Chunk<GT>::RAW;
        raw_t Hl[NU][RW];
#pragma unroll
        for (int l = 0; l < NU; ++l) last_up[l] = -1;
        for (int t0 = 0; t0 < T; t0 += C) {
            // stage leaf words, values and internal ids: run s, positions t0..t0+C-1
            stage_chunk<NG, C, NU>(cv, base, T, t0, lane, sw, sv, s_u[wave]);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int len = (int)(kend - k0) - t0;  // leaves of this run left in the chunk
            for (int j0 = 0; j0 < C; j0 += U) {
                if (j0 >= len) break;
                // a block of U leaves: every row of the block is in flight before any use
                int32_t wu[U];
                float vu[U];
                raw_t rowu[U][RW], hu[U][NU][RW];
                bool need[U][NU];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int at = gs * stage_stride<C>() + j0 + u;
                    wu[u] = sw[at];
                    vu[u] = sv[at];
                    Chunk<GT>::load(a_leaf, __umul24((uint32_t)wu[u] & IDMASK, rowb) + lane_off, rowu[u]);
#pragma unroll
                    for (int l = 0; l < NU; ++l) {
                        const int32_t id = s_u[wave][l][at];
                        need[u][l] = id != last_up[l];
                        last_up[l] = id;
                        if (need[u][l]) Chunk<GT>::load(a_up[l], __umul24((uint32_t)id, rowb) + lane_off, hu[u][l]);
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int jr = j0 + u;  // position in the chunk
                    if (jr < len) {
                        if (((uint32_t)wu[u] >> 29) == 0 && (t0 | jr) != 0) {  // a new root row starts here
                            AT *y = Y + (int64_t)cur_row * ldo;
                            if (is_first && !first_here) {
                                // began in an earlier run: add this part now, the
                                // earlier groups' part after the scan
#pragma unroll
                                for (int e = 0; e < E; ++e)
                                    if (col_of(e) < R) atomicAdd(y + col_of(e), acc[e]);
                            } else {
                                // began and ended in this run: exclusive
#pragma unroll
                                for (int e = 0; e < E; ++e)
                                    if (col_of(e) < R) y[col_of(e)] = acc[e];
                            }
#pragma unroll
                            for (int e = 0; e < E; ++e) acc[e] = 0;
                            is_first = false;
                            c0 += 1;
                            cur_row = root_ids[c0];
                        }
#pragma unroll
                        for (int l = 0; l < NU; ++l)
                            if (need[u][l]) {
#pragma unroll
                                for (int q = 0; q < RW; ++q) Hl[l][q] = hu[u][l][q];
                            }
#pragma unroll
                        for (int e = 0; e < E; ++e) leaf_fma<GT, NU>(acc[e], vu[u], rowu[u], Hl, e);
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        // --- end of the run: classify the open row
        const bool head_closed = !is_first && !first_here;  // row that began earlier closed inside
        const bool open_here = !is_first || first_here;     // open row began in this run
        const bool open_in_range = is_first ? first_in_range : true;
        const int32_t key = active ? cur_row : INT32_MAX;
        if (active && closes_at_end && open_here) {
            AT *y = Y + (int64_t)cur_row * ldo;
#pragma unroll
            for (int e = 0; e < E; ++e)
                if (col_of(e) < R) y[col_of(e)] = acc[e];
#pragma unroll
            for (int e = 0; e < E; ++e) acc[e] = 0;
        }
        // segment heads: first group of each run of equal keys (rows are sorted)
        const int32_t key_prev = __shfl_up(key, G, 64);
        const bool seg_head = g == 0 || key_prev != key;
        int head_group = seg_head ? g : 0;
#pragma unroll
        for (int o = 1; o < NG; o <<= 1) {
            const int h = __shfl_up(head_group, o * G, 64);
            if (g >= o) head_group = max(head_group, h);
        }
        const bool seg_in_range =
            __shfl(open_in_range ? 1 : 0, min(head_group, NG - 1) * G + lig, 64) != 0;
        // inclusive segmented scan of the open partials over groups
#pragma unroll
        for (int o = 1; o < NG; o <<= 1) {
            const int32_t ko = __shfl_up(key, o * G, 64);
            const bool take = g >= o && ko == key;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const AT x = __shfl_up(acc[e], o * G, 64);
                if (take) acc[e] += x;
            }
        }
        // a row that began in earlier groups and closed inside this group's run:
        // add the earlier groups' part (group g-1's segment total)
        const bool add_prev = active && head_closed && g > 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const AT x = __shfl_up(acc[e], G, 64);
            if (add_prev && col_of(e) < R) atomicAdd(Y + (int64_t)key_prev * ldo + col_of(e), x);
        }
        // open row closing exactly at the end of this run (not exclusive)
        if (active && closes_at_end && !open_here) {
            AT *y = Y + (int64_t)cur_row * ldo;
            if (seg_in_range) {
#pragma unroll
                for (int e = 0; e < E; ++e)
                    if (col_of(e) < R) y[col_of(e)] = acc[e];
            } else {
#pragma unroll
                for (int e = 0; e < E; ++e)
                    if (col_of(e) < R) atomicAdd(y + col_of(e), acc[e]);
            }
        }
        // carry: the last group's open segment, if it stays open, moves to group 0
        const int src = (NG - 1) * G + lig;
        const bool last_open = __shfl(active && !closes_at_end ? 1 : 0, src, 64) != 0;
        const int32_t last_key = __shfl(key, src, 64);
#pragma unroll
        for (int e = 0; e < E; ++e) acc[e] = __shfl(acc[e], src, 64);
        carry_row = last_open ? last_key : -1;
        if (g != 0 || !last_open) {
#pragma unroll
            for (int e = 0; e < E; ++e) acc[e] = 0;
        }
    }
    // the row still open at the end of the range continues in the next wave
    if (g == 0 && carry_row >= 0) {
        AT *y = Y + (int64_t)carry_row * ldo;
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (col_of(e) < R) atomicAdd(y + col_of(e), acc[e]);
    }
}

// Internal-level MTTKRP (output mode at depth d, 1 <= d <= N-2):
//     Y(i, :) += H_above * sum over leaves k below each level-d node with
//                index i of x_k * A_leaf(j_k, :) * H_below(k),
// H_above the Hadamard product of the node's ancestor rows, H_below that of
// leaf k's rows at the levels between d and the leaf.  Same lane groups,
// wave ranges and LDS staging of the leaf stream as the root kernel; the
// ancestor rows are gathered when a node starts, the rows below d reused
// while their ids repeat.  A level-d index recurs under other ancestors, so
// each node's partial (times H_above) is added to its output row -- batched:
// when a node (or the group's run) ends, the group writes its partial into a
// per-wave LDS list of finished nodes, and when the list is nearly full the
// wave adds the listed rows one row per instruction, the rank spread over
// the lanes (consecutive addresses, no loads in between): the most frequent
// output rows into a block-private LDS table (added to Y once, at the end),
// the others into Y.  A direct add from the lane groups would take E atomic
// instructions per node with addresses a chunk apart; every atomic add into
// Y is a request the memory side completes, the limit at these levels.
template <int N, int G, typename GT>
__global__ void __launch_bounds__(64 * ROOT_WAVES)
k_mttkrp_mid(CsfView cv, FacView fv, const char *__restrict__ a_leaf, uint32_t rowb, int d,
             const int32_t *__restrict__ starts, int32_t T, int64_t nsteps, int64_t nwaves, float *__restrict__ Y,
             int64_t ldo, int R, const int32_t *__restrict__ hot_rank) {
    constexpr int NG = 64 / G;
    constexpr int C = root_chunk<NG>(), U = root_unroll<N, GT>();
    constexpr int W = Chunk<GT>::W;
    constexpr int E = W;
    constexpr int NU = N - 2;  // internal levels 1..N-2
    constexpr int SS = NG * stage_stride<C>();
    constexpr int32_t IDMASK = (1 << 29) - 1;
    constexpr int SR = G * W;            // row stride of the list of finished nodes
    constexpr int CAP = NG * U + NG;  // its length: drained once more than NG entries wait
    using raw_t = typename Chunk<GT>::raw_t;
    constexpr int RW = Chunk<GT>::RAW;
    __shared__ int32_t s_w[ROOT_WAVES][SS];
    __shared__ float s_v[ROOT_WAVES][SS];
    __shared__ int32_t s_u[ROOT_WAVES][NU][SS];
    __shared__ float4 s_y4[ROOT_WAVES][CAP * SR / 4];
    __shared__ int32_t s_yr[ROOT_WAVES][CAP];
    extern __shared__ float mid_hot[];  // cv.hot x R floats
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane / G, lig = lane % G;  // g == NG: idle lane
    const int hot = cv.hot;
    const int64_t nloc = (int64_t)hot * R;
    for (int64_t j = threadIdx.x; j < nloc; j += 64 * ROOT_WAVES) mid_hot[j] = 0.0f;
    __syncthreads();
    const int64_t gw = (int64_t)blockIdx.x * ROOT_WAVES + wave;
    if (gw < nwaves) {  // no early return: the block adds its hot rows to Y at the end
    const int64_t nleaves = cv.nleaves;
    const int64_t s_begin = gw * nsteps / nwaves, s_end = (gw + 1) * nsteps / nwaves;
    const int64_t span = NG * (int64_t)T;
    const int32_t *__restrict__ leafw = cv.leafw;
    const float *__restrict__ vals = cv.vals;
    const int32_t *__restrict__ root_ids = cv.fids[0];
    int32_t *sw = s_w[wave];
    float *sv = s_v[wave];
    float *sy = reinterpret_cast<float *>(s_y4[wave]);
    int32_t *syr = s_yr[wave];
    const int gs = g < NG ? g : NG - 1;
    const uint64_t below = (1ull << (gs * G)) - 1;  // lanes of the groups before this one
    auto col_of = [&](int e) { return (lig * W) + e; };
    const uint32_t lane_off = (uint32_t)lig * Chunk<GT>::BYTES;
    int nst = 0;  // finished nodes in the list (wave-uniform)

    float acc[E];
    int32_t out_row = -1;   // index of the open level-d node
    raw_t Ha[N][RW];        // its ancestor rows (levels 0..d-1)
    // list the open node of every group with `fin` set (the same call on every lane)
    auto finish = [&](bool fin) {
        const uint64_t m = __ballot(fin && lig == 0);
        if (fin) {
            const int slot = nst + __popcll(m & below);
            float *y = sy + slot * SR + lig * W;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                float h = acc[e];
#pragma unroll
                for (int l = 0; l < N - 1; ++l)
                    if (l < d) h *= Chunk<GT>::get(Ha[l], e);
                y[e] = h;
                acc[e] = 0.0f;
            }
            if (lig == 0) syr[slot] = out_row;
        }
        nst += __popcll(m);
    };
    // add the listed rows (to the hot table or Y) when fewer than `room` entries are left
    auto drain = [&](int room) {
        if (nst <= CAP - room) return;
        wave_sync_lds_root();
        for (int q = 0; q < nst; ++q) {
            const int32_t row = __builtin_amdgcn_readfirstlane(syr[q]);
            // a uniform address: a scalar load, which waits on no vector memory
            // operation (the atomics and gathers in flight)
            const int32_t rk = hot > 0 ? hot_rank[row] : INT32_MAX;
            if (lane < R) {
                const float v = sy[q * SR + lane];
                if (rk < hot) atomicAdd(&mid_hot[(int64_t)rk * R + lane], v);
                else atomicAdd(Y + (int64_t)row * ldo + lane, v);
            }
        }
        wave_sync_lds_root();
        nst = 0;
    };

    for (int64_t st = s_begin; st < s_end; ++st) {
        const int64_t base = st * span;
        const int64_t k0 = base + (int64_t)gs * T;
        const bool active = g < NG && k0 < nleaves;
        const int64_t kend = active ? min(k0 + (int64_t)T, nleaves) : k0;
        int32_t c0 = active ? starts[st * NG + g] : 0;  // root node of the run's first leaf
#pragma unroll
        for (int e = 0; e < E; ++e) acc[e] = 0.0f;
        out_row = -1;
        int32_t last_up[NU];    // rows below d, reused while the ids repeat
        raw_t Hl[NU][RW];
#pragma unroll
        for (int l = 0; l < NU; ++l) last_up[l] = -1;
        for (int t0 = 0; t0 < T; t0 += C) {
            stage_chunk<NG, C, NU>(cv, base, T, t0, lane, sw, sv, s_u[wave]);
            wave_sync_lds_root();
            const int len = (int)(kend - k0) - t0;  // this group's leaves left in the chunk
            // every group steps through the whole chunk (the list is filled and
            // drained by the whole wave); positions past a group's run do nothing
            for (int j0 = 0; j0 < C; j0 += U) {
                int32_t wu[U];
                float vu[U];
                raw_t rowu[U][RW], hu[U][NU][RW];
                bool need[U][NU];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int at = gs * stage_stride<C>() + j0 + u;
                    wu[u] = sw[at];
                    vu[u] = sv[at];
                    Chunk<GT>::load(a_leaf, __umul24((uint32_t)wu[u] & IDMASK, rowb) + lane_off, rowu[u]);
#pragma unroll
                    for (int l = 0; l < NU; ++l) {
                        need[u][l] = false;
                        if (l + 1 > d) {  // levels below d
                            const int32_t id = s_u[wave][l][at];
                            need[u][l] = id != last_up[l];
                            last_up[l] = id;
                            if (need[u][l])
                                Chunk<GT>::load(static_cast<const char *>(fv.a[l + 1]),
                                                __umul24((uint32_t)id, rowb) + lane_off, hu[u][l]);
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int jr = j0 + u;
                    const bool live = active && jr < len;
                    const int at = gs * stage_stride<C>() + jr;
                    const int lvl = (int)((uint32_t)wu[u] >> 29);
                    const bool first = (t0 | jr) == 0;
                    const bool opens = live && (first || lvl <= d);  // a level-d node opens here
                    finish(opens && out_row >= 0);
                    if (live) {
                        if (!first && lvl == 0) c0 += 1;
                        if (opens) {
                            out_row = s_u[wave][d - 1][at];
                            Chunk<GT>::load(static_cast<const char *>(fv.a[0]),
                                            __umul24((uint32_t)root_ids[c0], rowb) + lane_off, Ha[0]);
#pragma unroll
                            for (int l = 1; l < N - 1; ++l)
                                if (l < d)
                                    Chunk<GT>::load(static_cast<const char *>(fv.a[l]),
                                                    __umul24((uint32_t)s_u[wave][l - 1][at], rowb) + lane_off, Ha[l]);
                        }
#pragma unroll
                        for (int l = 0; l < NU; ++l)
                            if (need[u][l]) {
#pragma unroll
                                for (int q = 0; q < RW; ++q) Hl[l][q] = hu[u][l][q];
                            }
#pragma unroll
                        for (int e = 0; e < E; ++e) {
                            float h = vu[u] * Chunk<GT>::get(rowu[u], e);
#pragma unroll
                            for (int l = 0; l < NU; ++l)
                                if (l + 1 > d) h *= Chunk<GT>::get(Hl[l], e);
                            acc[e] += h;
                        }
                    }
                }
                drain(NG * U);
            }
            __builtin_amdgcn_wave_barrier();
        }
        // the node open at the end of the run
        finish(active && out_row >= 0);
        drain(NG * U);
    }
    drain(CAP);
    }
    __syncthreads();
    for (int64_t j = threadIdx.x; j < nloc; j += 64 * ROOT_WAVES) {
        const float v = mid_hot[j];
        if (v != 0.0f) atomicAdd(Y + (int64_t)cv.hot_perm[j / R] * ldo + (j % R), v);
    }
}

// Rows of the leaf factor in rank order: dst row r = src row perm[r] (16-byte chunks).
__global__ void k_permute_rows(const uint4 *__restrict__ src, const int32_t *__restrict__ perm, int64_t rows,
                               int chunks, uint4 *__restrict__ dst) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * chunks) return;
    const int64_t r = t / chunks, q = t % chunks;
    dst[t] = src[(int64_t)perm[r] * chunks + q];
}

}  // namespace

// Launch the root kernel (FP32 rows when GT = float, bf16 when uint16_t):
// G lanes per leaf, one 16-byte chunk each, cover the padded row; one wave
// range per resident wave.
template <int N, int G, typename GT>
static cpd_status launch_mid_g(const CsfView &cv, const FacView &fv, const char *a_leaf, uint32_t rowb, int d,
                               const int32_t *starts, int32_t T, float *Y, int64_t ldo, int R, hipStream_t s) {
    constexpr int NG = 64 / G;
    auto kern = k_mttkrp_mid<N, G, GT>;
    const int64_t nsteps = ceil_div(cv.nleaves, NG * (int64_t)T);
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) ncu = v;
    }
    const size_t lds = sizeof(float) * (size_t)cv.hot * R;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * ROOT_WAVES, lds) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    per_cu = std::min(per_cu, 6);
    const int64_t nwaves = std::max<int64_t>(1, std::min<int64_t>(nsteps, (int64_t)ncu * per_cu * ROOT_WAVES));
    hipLaunchKernelGGL(kern, dim3((unsigned)ceil_div(nwaves, ROOT_WAVES)), dim3(64 * ROOT_WAVES), lds, s, cv, fv,
                       a_leaf, rowb, d, starts, T, nsteps, nwaves, Y, ldo, R, cv.hot_rank);
    CPD_LAUNCH_CHECK();
    return CPD_OK;
}

template <int N, int G, typename GT, typename AT>
static cpd_status launch_root_g(const CsfView &cv, const FacView &fv, const char *a_leaf, uint32_t rowb, int d,
                                const int32_t *starts, int64_t ntiles, int32_t T, AT *Y, int64_t ldo, int R,
                                hipStream_t s) {
    if constexpr (std::is_same<AT, float>::value) {
        if (d > 0) return launch_mid_g<N, G, GT>(cv, fv, a_leaf, rowb, d, starts, T, Y, ldo, R, s);
    } else {
        if (d > 0) CPD_FAIL(CPD_EUNSUPPORTED, "FP64 accumulation at the root level only");
    }
    constexpr int NG = 64 / G;
    auto kern = k_mttkrp_root<N, G, GT, AT>;
    const int64_t nsteps = ceil_div(cv.nleaves, NG * (int64_t)T);
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) ncu = v;
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * ROOT_WAVES, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    // at most 6 resident waves per SIMD: more thrash the L1 with gathered rows
    // (measured slower on the 8-byte bfloat16 form, neutral elsewhere)
    per_cu = std::min(per_cu, 6);
    const int64_t nwaves = std::max<int64_t>(1, std::min<int64_t>(nsteps, (int64_t)ncu * per_cu * ROOT_WAVES));
    hipLaunchKernelGGL(kern, dim3((unsigned)ceil_div(nwaves, ROOT_WAVES)), dim3(64 * ROOT_WAVES), 0, s, cv, fv, a_leaf,
                       rowb, starts, ntiles, T, nsteps, nwaves, Y, ldo, R);
    CPD_LAUNCH_CHECK();
    return CPD_OK;
}

template <int N, typename GT, typename AT>
static cpd_status launch_root_n(int RP, const CsfView &cv, const FacView &fv, const char *a_leaf, int64_t ld, int d,
                                const int32_t *starts, int64_t ntiles, int32_t T, AT *Y, int64_t ldo, int R,
                                hipStream_t s) {
    constexpr int W = Chunk<GT>::W;
    const uint32_t rowb = (uint32_t)(ld * (int64_t)Chunk<GT>::ELEM);
    switch (RP / W) {
#define CPD_ROOT_G(g) \
    case g: return launch_root_g<N, g, GT, AT>(cv, fv, a_leaf, rowb, d, starts, ntiles, T, Y, ldo, R, s);
        CPD_ROOT_G(2)
        CPD_ROOT_G(4)
        CPD_ROOT_G(5)
        CPD_ROOT_G(8)
        CPD_ROOT_G(9)
        CPD_ROOT_G(16)
#undef CPD_ROOT_G
        default: CPD_FAIL(CPD_EUNSUPPORTED, "no root kernel for padded rank %d", RP);
    }
}

int root_lanes_per_leaf(int RP, bool bf16) {
    if (!bf16) return RP / Chunk<float>::W;
    return RP <= BF16_NARROW_MAX ? RP / Chunk<bf16x4>::W : RP / Chunk<uint16_t>::W;
}

// Shared body of the float and double launches.  perm_buf: device scratch of
// at least leaf rows * row bytes for the leaf factor in rank order, or null
// to take it from the stream's scratch cache.
template <typename AT>
static cpd_status launch_root_t(int N, bool bf16, int RP, int d, const int32_t *const *fids,
                                const int32_t *const *fptr, const float *vals, const int32_t *leafw,
                                const int32_t *leaf_perm, const int32_t *const *uprow, const int64_t *counts,
                                const int64_t *dims_by_level, const void *const *fac_by_level, int64_t ld,
                                const int32_t *starts, int64_t ntiles, int32_t T, AT *Y, int64_t ldo, int R,
                                void *perm_buf, const int32_t *hot_rank, const int32_t *hot_perm, int32_t hot,
                                hipStream_t s) {
    if (hot > 0 && (d == 0 || !hot_rank || !hot_perm)) CPD_FAIL(CPD_EINVAL, "hot rows need an internal level's ranking");
    if (d < 0 || d > N - 2) CPD_FAIL(CPD_EINVAL, "lane-group kernel for depth %d of %d levels", d, N);
    if (!leafw || !leaf_perm) CPD_FAIL(CPD_EUNSUPPORTED, "root kernel needs leaf ids below 2^29");
    const int64_t rowb = ld * (bf16 ? 2 : 4);
    if (rowb >= (1 << 24) || rowb % 16) CPD_FAIL(CPD_EUNSUPPORTED, "root kernel needs 16-byte rows below 16 MiB");
    // gathered rows are addressed as 32-bit byte offsets (24-bit row id times row bytes)
    for (int l = 0; l < N; ++l)
        if (l != d && (dims_by_level[l] >= (1 << 24) || dims_by_level[l] * rowb > (int64_t(1) << 32)))
            CPD_FAIL(CPD_EUNSUPPORTED, "level %d: %lld rows of %lld bytes exceed 32-bit row offsets", l,
                     (long long)dims_by_level[l], (long long)rowb);
    if (T < ROOT_C || T % ROOT_C)
        CPD_FAIL(CPD_EINVAL, "root kernel tile width %d must be a multiple of %d", T, ROOT_C);
    CsfView cv{};
    FacView fv{};
    for (int l = 0; l < N; ++l) {
        cv.fids[l] = fids[l];
        cv.fptr[l] = fptr[l];
        fv.a[l] = fac_by_level[l];
    }
    cv.vals = vals;
    cv.leafw = leafw;
    cv.nleaves = counts[N - 1];
    cv.hot_rank = hot_rank;
    cv.hot_perm = hot_perm;
    cv.hot = hot;
    for (int l = 1; l < N - 1; ++l) {
        if (!uprow[l]) CPD_FAIL(CPD_EUNSUPPORTED, "root kernel needs the per-leaf internal ids");
        cv.uprow[l] = uprow[l];
    }
    // the leaf factor in rank order (hot rows first)
    const int64_t leaf_rows = dims_by_level[N - 1];
    DevBuf<uint4> perm;
    uint4 *pb = static_cast<uint4 *>(perm_buf);
    if (!pb) {
        CPD_TRY(perm.alloc((size_t)leaf_rows * (rowb / 16), s));
        pb = perm.p;
    }
    {
        const int chunks = (int)(rowb / 16);
        const int64_t tot = leaf_rows * chunks;
        hipLaunchKernelGGL(k_permute_rows, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, s,
                           static_cast<const uint4 *>(fac_by_level[N - 1]), leaf_perm, leaf_rows, chunks, pb);
        CPD_LAUNCH_CHECK();
    }
    const char *a_leaf = reinterpret_cast<const char *>(pb);
    if constexpr (std::is_same<AT, double>::value) {
        if (bf16) CPD_FAIL(CPD_EUNSUPPORTED, "FP64 accumulation takes float rows");
        switch (N) {
            case 3: return launch_root_n<3, float>(RP, cv, fv, a_leaf, ld, d, starts, ntiles, T, Y, ldo, R, s);
            case 4: return launch_root_n<4, float>(RP, cv, fv, a_leaf, ld, d, starts, ntiles, T, Y, ldo, R, s);
            case 5: return launch_root_n<5, float>(RP, cv, fv, a_leaf, ld, d, starts, ntiles, T, Y, ldo, R, s);
            default: CPD_FAIL(CPD_EUNSUPPORTED, "root kernel built for 3..5 modes, not %d", N);
        }
    } else {
        // bfloat16 rows: 8-byte chunks (the float layout at half the bytes) up to
        // a padded rank of BF16_NARROW_MAX, 16-byte chunks above
        const bool narrow = bf16 && RP <= BF16_NARROW_MAX;
#define CPD_ROOT_N(n)                                                                                           \
    case n:                                                                                                     \
        if (narrow) return launch_root_n<n, bf16x4>(RP, cv, fv, a_leaf, ld, d, starts, ntiles, T, Y, ldo, R, s); \
        return bf16 ? launch_root_n<n, uint16_t>(RP, cv, fv, a_leaf, ld, d, starts, ntiles, T, Y, ldo, R, s)    \
                    : launch_root_n<n, float>(RP, cv, fv, a_leaf, ld, d, starts, ntiles, T, Y, ldo, R, s);
        switch (N) {
            CPD_ROOT_N(3)
            CPD_ROOT_N(4)
            CPD_ROOT_N(5)
            default: CPD_FAIL(CPD_EUNSUPPORTED, "root kernel built for 3..5 modes, not %d", N);
        }
#undef CPD_ROOT_N
    }
}

cpd_status launch_root(int N, bool bf16, int RP, int d, const int32_t *const *fids, const int32_t *const *fptr,
                       const float *vals, const int32_t *leafw, const int32_t *leaf_perm, const int32_t *const *uprow,
                       const int64_t *counts, const int64_t *dims_by_level, const void *const *fac_by_level,
                       int64_t ld, const int32_t *starts, int64_t ntiles, int32_t T, float *Y, int64_t ldo, int R,
                       void *perm_buf, const int32_t *hot_rank, const int32_t *hot_perm, int32_t hot,
                       hipStream_t s) {
    return launch_root_t<float>(N, bf16, RP, d, fids, fptr, vals, leafw, leaf_perm, uprow, counts, dims_by_level,
                                fac_by_level, ld, starts, ntiles, T, Y, ldo, R, perm_buf, hot_rank, hot_perm, hot,
                                s);
}

// Root-level MTTKRP with float rows and FP64 products and sums (the exact fit pass).
cpd_status launch_root64(int N, int RP, const int32_t *const *fids, const int32_t *const *fptr, const float *vals,
                         const int32_t *leafw, const int32_t *leaf_perm, const int32_t *const *uprow,
                         const int64_t *counts, const int64_t *dims_by_level, const void *const *fac_by_level,
                         int64_t ld, const int32_t *starts, int64_t ntiles, int32_t T, double *Y, int64_t ldo, int R,
                         hipStream_t s) {
    return launch_root_t<double>(N, false, RP, 0, fids, fptr, vals, leafw, leaf_perm, uprow, counts, dims_by_level,
                                 fac_by_level, ld, starts, ntiles, T, Y, ldo, R, nullptr, nullptr, nullptr, 0, s);
}

}  // namespace cpd
