// Leaf-level MTTKRP on a CSF tree (the output mode sits at the tree's leaf
// level; the MTTKRP step of Algorithm 1, Section III):
//     Y(j_k, :) += x_k * H_f,
// H_f = Hadamard product of the rows of the levels above leaf k, one row per
// fiber f (the leaves that share every index but the last).
//
// Work split: each wave owns a contiguous range of tiles (T leaves each, T a
// multiple of 64) and takes it in rounds of 64 leaves.
//   - Lane j loads leaf j's value, leaf index, leaf word and per-leaf internal
//     ids with coalesced loads.  The leaves that open a root node and those
//     that open a fiber (leaf-word level 0, resp. <= N-2, plus the round's first
//     leaf) form wave-uniform bit masks; popcounts give every leaf its root
//     node and its fiber.
//   - The H rows of the round's fibers are gathered a batch at a time into a
//     per-wave LDS table (G lanes per row, four elements each, so a load
//     instruction fetches 64/G rows).
//   - The wave then walks the batch's leaves one per step, the rank spread over
//     the lanes: value, index and frequency rank read from the leaf's lane, the
//     row of H from LDS, one FP32 atomic add per leaf -- into a block-private
//     LDS copy of the most frequent output rows (Zipf-hot rows would otherwise
//     serialise their atomics in L2), else into Y.
// The walk issues no loads, so its atomics go out back to back; a wave waits
// on memory once per batch of fibers (the gathers), not once per leaf.
#include <type_traits>

#include "csf.h"

namespace cpd {
namespace {

constexpr int LEAF_WAVES = 4;  // waves per block
constexpr int32_t LEAF_IDMASK = (1 << 29) - 1;

struct LeafView {
    const int32_t *root_ids;              // fids[0]
    const int32_t *leaf_ids;              // fids[N-1]
    const float *vals;
    const int32_t *leafw;                 // (level << 29) | frequency rank of the leaf index
    const int32_t *uprow[CPD_MAX_MODES];  // per-leaf ids of levels 1..N-2
    const int32_t *hot_perm;              // output row of each frequency rank
    int64_t nleaves;
};

struct LeafFac {
    const void *a[CPD_MAX_MODES];  // factor of each level (levels 0..N-2 are read)
};

// Four consecutive row elements (float, or bfloat16 widened to float) at
// element offset off (a multiple of 4; rows 16-byte resp. 8-byte aligned).
template <typename GT>
struct Quad;
template <>
struct Quad<float> {
    __device__ static __forceinline__ float4 load(const void *base, int64_t off) {
        return *reinterpret_cast<const float4 *>(static_cast<const float *>(base) + off);
    }
};
template <>
struct Quad<uint16_t> {
    __device__ static __forceinline__ float4 load(const void *base, int64_t off) {
        const uint2 w = *reinterpret_cast<const uint2 *>(static_cast<const uint16_t *>(base) + off);
        return make_float4(bf16_lo(w.x), bf16_hi(w.x), bf16_lo(w.y), bf16_hi(w.y));
    }
};

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// UF: gather instructions per level and batch (a batch holds UF * 64/G fibers).
// Dynamic LDS: LEAF_WAVES x PF x RQ floats (each wave's table of H rows; RQ =
// R rounded up to a multiple of 4, so rows are 16-byte aligned), then hot x R
// floats (the hot output rows).
template <int N, typename GT, int UF>
__global__ void __launch_bounds__(64 * LEAF_WAVES)
k_mttkrp_leaf(LeafView cv, LeafFac fv, int64_t ld, const int32_t *__restrict__ starts, int64_t ntiles, int32_t T,
              int64_t nwaves, float *__restrict__ Y, int64_t ldo, int R, int32_t hot) {
    extern __shared__ float4 lds4[];
    __shared__ int32_t s_fpos[LEAF_WAVES][65];
    float *lds = reinterpret_cast<float *>(lds4);
    const int RQ = (R + 3) & ~3;
    const int G = RQ >> 2;      // lanes per row in the gather
    const int NG = 64 / G;      // rows per gather instruction
    const int PF = NG * UF;     // fibers per batch
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane / G, lig = lane - (lane / G) * G;
    float *Hs = lds + (int64_t)wave * PF * RQ;
    float *ypriv = lds + (int64_t)LEAF_WAVES * PF * RQ;
    int32_t *fpos = s_fpos[wave];
    const int64_t nloc = (int64_t)hot * R;
    for (int64_t j = threadIdx.x; j < nloc; j += 64 * LEAF_WAVES) ypriv[j] = 0.0f;
    __syncthreads();

    const int64_t gw = (int64_t)blockIdx.x * LEAF_WAVES + wave;
    if (gw < nwaves) {  // no early return: the block flushes its hot rows below
        const int64_t t_begin = gw * ntiles / nwaves, t_end = (gw + 1) * ntiles / nwaves;
        const int64_t kb = t_begin * (int64_t)T;
        const int64_t ke = min(t_end * (int64_t)T, cv.nleaves);
        int32_t c_base = starts[t_begin];  // root node holding leaf kb
        bool first = true;
        for (int64_t k0 = kb; k0 < ke; k0 += 64) {
            const int64_t k = k0 + lane;
            const bool in = k < ke;
            // lanes past the range load the range's last leaf (straight-line loads) and drop it
            const int64_t kk = in ? k : ke - 1;
            const int32_t w = stream_load(cv.leafw + kk);
            const float x = stream_load(cv.vals + kk);
            const int32_t oi = stream_load(cv.leaf_ids + kk);
            int32_t up[N > 2 ? N - 2 : 1];
#pragma unroll
            for (int l = 0; l < N - 2; ++l) up[l] = stream_load(cv.uprow[l + 1] + kk);
            const int lvl = (int)((uint32_t)w >> 29);
            const uint64_t nrmask = __ballot(in && lvl == 0);
            const uint64_t fmask = __ballot(in && (lvl <= N - 2 || lane == 0));
            const int nin = (int)min<int64_t>(64, ke - k0);
            // c_base: root node of the leaf before the round (the tile table
            // gives the node holding leaf kb itself)
            if (first && (nrmask & 1ull)) c_base -= 1;
            first = false;
            const uint64_t upto = ~0ull >> (63 - lane);  // bits 0..lane
            // root node of each leaf (lanes past the range: that of the last leaf)
            const int32_t rid = cv.root_ids[c_base + __popcll(nrmask & upto)];
            c_base += __popcll(nrmask);
            const int F = __popcll(fmask);
            if ((fmask >> lane) & 1ull) fpos[__popcll(fmask & upto) - 1] = lane;
            if (lane == 0) fpos[F] = nin;
            wave_sync_lds();
            for (int f0 = 0; f0 < F; f0 += PF) {
                const int f1 = min(F, f0 + PF);
                // gather the H rows of fibers f0..f1-1: every load is issued before any
                // use (lanes without a fiber of the batch load fiber f0's rows again
                // and store nothing)
                int32_t ids[UF][N - 1];
                bool ok[UF];
#pragma unroll
                for (int u = 0; u < UF; ++u) {
                    const int f = f0 + u * NG + g;
                    ok[u] = g < NG && f < f1;
                    const int p = fpos[ok[u] ? f : f0];
                    ids[u][0] = __shfl(rid, p, 64);
#pragma unroll
                    for (int l = 1; l < N - 1; ++l) ids[u][l] = __shfl(up[l - 1], p, 64);
                }
                float4 rows[UF][N - 1];
#pragma unroll
                for (int u = 0; u < UF; ++u)
#pragma unroll
                    for (int l = 0; l < N - 1; ++l)
                        rows[u][l] = Quad<GT>::load(fv.a[l], (int64_t)ids[u][l] * ld + 4 * lig);
#pragma unroll
                for (int u = 0; u < UF; ++u) {
                    float4 h = rows[u][0];
#pragma unroll
                    for (int l = 1; l < N - 1; ++l) {
                        h.x *= rows[u][l].x;
                        h.y *= rows[u][l].y;
                        h.z *= rows[u][l].z;
                        h.w *= rows[u][l].w;
                    }
                    if (ok[u]) *reinterpret_cast<float4 *>(Hs + (int64_t)(u * NG + g) * RQ + 4 * lig) = h;
                }
                wave_sync_lds();
                // the batch's leaves, one per step
                const int jb = __builtin_amdgcn_readfirstlane(fpos[f0]);
                const int je = __builtin_amdgcn_readfirstlane(fpos[f1]);
                for (int j = jb; j < je; ++j) {
                    const int f = __popcll(fmask & (~0ull >> (63 - j))) - 1 - f0;
                    const float xj = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), j));
                    const int32_t oj = __builtin_amdgcn_readlane(oi, j);
                    const int32_t rk = __builtin_amdgcn_readlane(w, j) & LEAF_IDMASK;
                    if (lane < R) {
                        const float t = xj * Hs[f * RQ + lane];
                        if (rk < hot) atomicAdd(&ypriv[(int64_t)rk * R + lane], t);
                        else atomicAdd(Y + (int64_t)oj * ldo + lane, t);
                    }
                }
                wave_sync_lds();
            }
        }
    }
    __syncthreads();
    for (int64_t j = threadIdx.x; j < nloc; j += 64 * LEAF_WAVES) {
        const float v = ypriv[j];
        if (v != 0.0f) atomicAdd(Y + (int64_t)cv.hot_perm[j / R] * ldo + (j % R), v);
    }
}

template <int N, typename GT>
cpd_status launch_leaf_n(const LeafView &cv, const LeafFac &fv, int64_t ld, const int32_t *starts, int64_t ntiles,
                         int32_t T, float *Y, int64_t ldo, int R, int32_t hot, hipStream_t s) {
    const int RQ = (R + 3) & ~3;
    const int NG = 64 / (RQ / 4);
    const int UF = NG >= 7 ? 2 : 4;
    const int PF = NG * UF;
    const size_t lds = sizeof(float) * ((size_t)hot * R + (size_t)LEAF_WAVES * PF * RQ);
    auto kern = UF == 2 ? k_mttkrp_leaf<N, GT, 2> : k_mttkrp_leaf<N, GT, 4>;
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) ncu = v;
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * LEAF_WAVES, lds) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    const int64_t nwaves = std::max<int64_t>(1, std::min<int64_t>(ntiles, (int64_t)ncu * per_cu * LEAF_WAVES));
    hipLaunchKernelGGL(kern, dim3((unsigned)ceil_div(nwaves, LEAF_WAVES)), dim3(64 * LEAF_WAVES), lds, s, cv, fv,
                       ld, starts, ntiles, T, nwaves, Y, ldo, R, hot);
    CPD_LAUNCH_CHECK();
    return CPD_OK;
}

// ------------------------------------------------------------ mode tiling
// Level d >= 1 on the level's mode tiling (the leaves regrouped by tiles of
// B level-d indices):
//     Y(i, :) += x_k * H_k for every leaf k whose level-d index is i,
// H_k = Hadamard product of leaf k's rows at every other level.  A fiber here
// is a run of leaves that agree on every other level's index (at the leaf
// level, in tree order inside a tile, the fibers of the tree; at an internal
// level, ordered by size, leaves that differ only in their level-d index).
// Each wave owns a contiguous range of the regrouped leaves and a private LDS
// table of one tile's B x R output rows: it takes its range tile by tile
// (zero the table, add every leaf of the tile into it, add the table's
// nonzero entries to Y), so every nonzero is a plain LDS read-add-write by
// the one wave that owns the row -- no atomics (the LDS FP32 atomic add
// measured several times slower than a plain read-modify-write here).
// Rounds of 64 leaves as in the ROUND kernel: each lane loads its leaf's
// record (value, local row, the other levels' indices) with one or two
// 16-byte loads (a fiber run starts where any of those indices changes),
// each run's H row is gathered once into the wave's H table, a batch of PF
// runs at a time, then the batch's leaves are walked two per step, the rank
// across the lanes.
typedef int32_t i32x4_t __attribute__((ext_vector_type(4)));

struct TiledView {
    const int32_t *toff;
    const int32_t *rec;  // one record per regrouped leaf: value bits, local row, other levels' indices
    int64_t n;
    int64_t ntiles;
    int32_t B;
};

constexpr int TILED_WAVES = 4;  // waves per block (each on its own range and tables)

// Minimum resident waves per SIMD asked of the compiler: 8 for three modes
// with two gathers per lane group (64 registers, no spills; the record
// prefetch would otherwise take it to 66 and 7 waves), no constraint
// elsewhere (the forms with four gathers, or four and five modes, would
// spill).
template <int N, int UF>
constexpr int tiled_min_waves() {
    return N == 3 && UF == 2 ? 8 : 1;
}

// Leaf k's record of a mode tiling: one 16-byte load for 2..3 modes, two for
// 4..5 (records of 4 or 8 words, 16-byte aligned).
template <int N>
__device__ __forceinline__ void load_record(const int32_t *rec, int64_t k, float &x, int32_t &row, int32_t (&id)[N - 1]) {
    constexpr int RW = N <= 3 ? 4 : 8;
    const i32x4_t a = __builtin_nontemporal_load(reinterpret_cast<const i32x4_t *>(rec + k * RW));
    x = __int_as_float(a.x);
    row = a.y;
    id[0] = a.z;
    if constexpr (N >= 3) id[1] = a.w;
    if constexpr (N >= 4) {
        const i32x4_t b = __builtin_nontemporal_load(reinterpret_cast<const i32x4_t *>(rec + k * RW + 4));
        id[2] = b.x;
        if constexpr (N >= 5) id[3] = b.y;
    }
}

// Dynamic LDS per wave: (PF + 1) x RQ floats (H rows and a spare row), then
// B x R floats (its tile).
template <int N, typename GT, int UF>
__global__ void __launch_bounds__(64 * TILED_WAVES, (tiled_min_waves<N, UF>()))
k_mttkrp_tiled(TiledView tv, LeafFac fv, int64_t ld, int64_t nwaves, float *__restrict__ Y, int64_t ldo, int R) {
    extern __shared__ float4 lds4[];
    __shared__ int32_t s_fpos[TILED_WAVES][65];
    const int RQ = (R + 3) & ~3;
    const int G = RQ >> 2;
    const int NG = 64 / G;
    const int PF = NG * UF;
    // x mod PF for 0 <= x < 64 as x - ((x * pf_inv) >> 16) * PF: exact, as
    // pf_inv * PF - 2^16 < PF and x * PF < 2^16
    const uint32_t pf_inv = (65536u + (uint32_t)PF - 1) / (uint32_t)PF;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane / G, lig = lane - (lane / G) * G;
    const int64_t nloc = (int64_t)tv.B * R;
    // per-wave stride in floats, a multiple of 4 (16-byte aligned H rows)
    const int64_t stride = ((int64_t)(PF + 1) * RQ + nloc + 3) & ~int64_t(3);
    float *Hs = reinterpret_cast<float *>(lds4) + (int64_t)wave * stride;
    float *tab = Hs + (int64_t)(PF + 1) * RQ;
    int32_t *fpos = s_fpos[wave];
    const int64_t gw = (int64_t)blockIdx.x * TILED_WAVES + wave;
    if (gw >= nwaves) return;  // waves are independent: no block barriers
    // this wave's range, whole rounds apart
    const int64_t nr = ceil_div(tv.n, 64);
    const int64_t r0 = gw * nr / nwaves, r1 = (gw + 1) * nr / nwaves;
    const int64_t b1 = min(r1 * 64, tv.n);
    int64_t pos = r0 * 64;
    while (pos < b1) {
        // the tile holding regrouped leaf pos: the largest t with toff[t] <= pos
        int64_t lo = 0, hi = tv.ntiles;
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if ((int64_t)tv.toff[mid] <= pos) lo = mid;
            else hi = mid;
        }
        const int64_t t = lo;
        const int64_t e = min(b1, (int64_t)tv.toff[t + 1]);
        for (int64_t j = lane; j < nloc; j += 64) tab[j] = 0.0f;
        // records of the round (the next round's are loaded during this
        // round's first batch, so a round does not start waiting on them)
        float x;
        int32_t row, hid[N - 1];
        load_record<N>(tv.rec, min(pos + lane, e - 1), x, row, hid);
        for (int64_t k0 = pos; k0 < e; k0 += 64) {
            const int64_t k = k0 + lane;
            const bool in = k < e;
            float nx = 0.0f;
            int32_t nrow = 0, nhid[N - 1] = {};
            bool newf = lane == 0;
#pragma unroll
            for (int l = 0; l < N - 1; ++l) newf |= __shfl_up(hid[l], 1, 64) != hid[l];
            // a fiber is its index tuple: a new run where any level's index changes
            const uint64_t fmask = __ballot(in && newf);
            const int nin = (int)min<int64_t>(64, e - k0);
            const uint64_t upto = ~0ull >> (63 - lane);
            const int F = __popcll(fmask);
            const int fo = __popcll(fmask & upto) - 1;  // fiber of this lane's leaf
            if ((fmask >> lane) & 1ull) fpos[fo] = lane;
            if (lane == 0) fpos[F] = nin;
            // this leaf's LDS byte offsets, packed: its fiber's H row (batches
            // are PF fibers apart) in the low half, its tile row in the high
            // half (a wave's LDS is below 64 KiB)
            const uint32_t fb = (uint32_t)fo - (((uint32_t)fo * pf_inv) >> 16) * (uint32_t)PF;  // fo mod PF
            const uint32_t pk = fb * (uint32_t)(RQ * 4) | ((uint32_t)(row * R * 4) << 16);
            wave_sync_lds();
            // one batch of PF fibers from fiber f0 (the round's last batch, which
            // always exists, also loads the next round's records)
            auto batch = [&](const int f0, auto last) {
                const int f1 = min(F, f0 + PF);
                int32_t ids[UF][N - 1];
                bool ok[UF];
#pragma unroll
                for (int u = 0; u < UF; ++u) {
                    const int ff = f0 + u * NG + g;
                    ok[u] = g < NG && ff < f1;
                    const int p = fpos[ok[u] ? ff : f0];
#pragma unroll
                    for (int l = 0; l < N - 1; ++l) ids[u][l] = __shfl(hid[l], p, 64);
                }
                float4 rows[UF][N - 1];
#pragma unroll
                for (int u = 0; u < UF; ++u)
#pragma unroll
                    for (int l = 0; l < N - 1; ++l)
                        rows[u][l] = Quad<GT>::load(fv.a[l], (int64_t)ids[u][l] * ld + 4 * lig);
                // the next round's records, after the gathers of the round's last
                // batch: the wait for the gathers leaves them in flight during
                // the walk, and no later gather waits behind them (past the
                // tile's end: its last record again)
                if constexpr (decltype(last)::value)
                    load_record<N>(tv.rec, min(k0 + 64 + lane, e - 1), nx, nrow, nhid);
#pragma unroll
                for (int u = 0; u < UF; ++u) {
                    float4 h = rows[u][0];
#pragma unroll
                    for (int l = 1; l < N - 1; ++l) {
                        h.x *= rows[u][l].x;
                        h.y *= rows[u][l].y;
                        h.z *= rows[u][l].z;
                        h.w *= rows[u][l].w;
                    }
                    // unconditional store, so the gathers stay ahead of the
                    // prefetch: a group without a fiber writes its own slot,
                    // which this batch's walk does not read, the idle lanes
                    // the spare row PF (distinct rows: no bank conflicts)
                    *reinterpret_cast<float4 *>(Hs + (int64_t)(g < NG ? u * NG + g : PF) * RQ + 4 * lig) = h;
                }
                wave_sync_lds();
                const int jb = __builtin_amdgcn_readfirstlane(fpos[f0]);
                const int je = __builtin_amdgcn_readfirstlane(fpos[f1]);
                // two leaves per step, both tile rows read before either is
                // written: when they share a row, the second write holds both
                // contributions (every row is this wave's alone)
                // (the lanes past the rank skip the walk; v_readlane reads
                // any lane)
                if (lane < R) {
                    const char *hl = reinterpret_cast<const char *>(Hs + lane);
                    char *tl = reinterpret_cast<char *>(tab + lane);
                    int j = jb;
                    for (; j + 1 < je; j += 2) {
                        const uint32_t pa = __builtin_amdgcn_readlane(pk, j);
                        const uint32_t pb = __builtin_amdgcn_readlane(pk, j + 1);
                        const float xa = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), j));
                        const float xb = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), j + 1));
                        float *ya = reinterpret_cast<float *>(tl + (pa >> 16));
                        float *yb = reinterpret_cast<float *>(tl + (pb >> 16));
                        const float ta = xa * *reinterpret_cast<const float *>(hl + (pa & 0xffffu));
                        const float tb = xb * *reinterpret_cast<const float *>(hl + (pb & 0xffffu));
                        const float va = *ya, vb = *yb;
                        *yb = vb + tb;
                        *ya = va + ta + ((pa >> 16) == (pb >> 16) ? tb : 0.0f);
                    }
                    if (j < je) {
                        const uint32_t pa = __builtin_amdgcn_readlane(pk, j);
                        const float xa = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), j));
                        float *ya = reinterpret_cast<float *>(tl + (pa >> 16));
                        *ya += xa * *reinterpret_cast<const float *>(hl + (pa & 0xffffu));
                    }
                }
                wave_sync_lds();
            };
            int f0 = 0;
            for (; f0 + PF < F; f0 += PF) batch(f0, std::false_type{});
            batch(f0, std::true_type{});
            x = nx;
            row = nrow;
#pragma unroll
            for (int l = 0; l < N - 1; ++l) hid[l] = nhid[l];
        }
        // the tile's rows into Y (nonzero entries)
        const int64_t base = t * (int64_t)tv.B;
        for (int64_t j = lane; j < nloc; j += 64) {
            const float v = tab[j];
            if (v != 0.0f) atomicAdd(Y + (base + j / R) * ldo + (j % R), v);
        }
        wave_sync_lds();
        pos = e;
    }
}

template <int N, typename GT>
cpd_status launch_tiled_n(const TiledView &tv, const LeafFac &fv, int64_t ld, float *Y, int64_t ldo, int R, int UF,
                          size_t lds_wave, hipStream_t s) {
    auto kern = UF == 2 ? k_mttkrp_tiled<N, GT, 2> : k_mttkrp_tiled<N, GT, 4>;
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) ncu = v;
    }
    const size_t lds = lds_wave * TILED_WAVES;
    CPD_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * TILED_WAVES, lds) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    // one range per resident wave
    const int64_t nwaves = std::max<int64_t>(1, std::min<int64_t>(ceil_div(tv.n, 64), (int64_t)ncu * per_cu * TILED_WAVES));
    hipLaunchKernelGGL(kern, dim3((unsigned)ceil_div(nwaves, TILED_WAVES)), dim3(64 * TILED_WAVES), lds, s, tv, fv,
                       ld, nwaves, Y, ldo, R);
    CPD_LAUNCH_CHECK();
    return CPD_OK;
}

}  // namespace

// Leaf-level MTTKRP with the round kernel: Y (out_rows x R floats, stride
// ldo) must be zeroed.  fac_by_level: factors in tree order (levels 0..N-2
// read), row stride ld elements with ld % 4 == 0 and ld >= R rounded up to a
// multiple of 4, bases 16-byte (float) or 8-byte (bfloat16) aligned.
// starts: the level-0 rows of the tile table for width T (a multiple of 64).
// hot_perm / hot: the leaf level's frequency ranking and the number of hot
// rows held in LDS (0: none).
cpd_status launch_leaf(int N, bool bf16, const int32_t *const *fids, const float *vals, const int32_t *leafw,
                       const int32_t *const *uprow, const int32_t *hot_perm, int32_t hot, int64_t nleaves,
                       const void *const *fac_by_level, int64_t ld, const int32_t *starts, int64_t ntiles, int32_t T,
                       float *Y, int64_t ldo, int R, hipStream_t s) {
    if (N < 2 || N > 5) CPD_FAIL(CPD_EUNSUPPORTED, "leaf round kernel built for 2..5 modes, not %d", N);
    if (T < 64 || T % 64) CPD_FAIL(CPD_EINVAL, "leaf round kernel tile width %d must be a multiple of 64", T);
    if (R < 1 || R > 64 || ld % 4 || ld < ((R + 3) & ~3))
        CPD_FAIL(CPD_EUNSUPPORTED, "leaf round kernel needs rank <= 64 and ld a multiple of 4 covering the rank");
    if (!leafw) CPD_FAIL(CPD_EUNSUPPORTED, "leaf round kernel needs the tree's leaf words");
    if (hot > 0 && !hot_perm) CPD_FAIL(CPD_EINVAL, "hot rows without a ranking");
    LeafView cv{};
    LeafFac fv{};
    cv.root_ids = fids[0];
    cv.leaf_ids = fids[N - 1];
    cv.vals = vals;
    cv.leafw = leafw;
    cv.hot_perm = hot_perm;
    cv.nleaves = nleaves;
    for (int l = 1; l < N - 1; ++l) {
        if (!uprow[l]) CPD_FAIL(CPD_EUNSUPPORTED, "leaf round kernel needs the per-leaf internal ids");
        cv.uprow[l] = uprow[l];
    }
    for (int l = 0; l < N - 1; ++l) fv.a[l] = fac_by_level[l];
    if (nleaves == 0) return CPD_OK;
    switch (N) {
#define CPD_LEAF_N(n)                                                                                        \
    case n:                                                                                                  \
        return bf16 ? launch_leaf_n<n, uint16_t>(cv, fv, ld, starts, ntiles, T, Y, ldo, R, hot, s)           \
                    : launch_leaf_n<n, float>(cv, fv, ld, starts, ntiles, T, Y, ldo, R, hot, s);
        CPD_LEAF_N(2)
        CPD_LEAF_N(3)
        CPD_LEAF_N(4)
        CPD_LEAF_N(5)
#undef CPD_LEAF_N
    }
    return CPD_OK;
}


// Tile height of a mode tiling for rank R: one wave's tile of R-float
// rows and its H table within lds_wave bytes of LDS.
int32_t tiled_height(int R, size_t lds_wave) {
    const int RQ = (R + 3) & ~3;
    const int NG = 64 / (RQ / 4);
    const int PF = NG * (NG >= 7 ? 2 : 4);
    const size_t fixed = sizeof(float) * ((size_t)(PF + 1) * RQ + 3) + sizeof(int32_t) * 65;
    if (lds_wave <= fixed) return 0;
    return (int32_t)((lds_wave - fixed) / (sizeof(float) * R));
}

// MTTKRP of level lt.depth (1..N-1) on its mode tiling (Y zeroed by the
// caller; factor rules as for launch_leaf; fac_by_level: every level's factor
// in tree order).
cpd_status launch_tiled(int N, bool bf16, const cpd_csf_s::LeafTiling &lt, int64_t nleaves,
                        const void *const *fac_by_level, int64_t ld, float *Y, int64_t ldo, int R, hipStream_t s) {
    if (N < 2 || N > 5) CPD_FAIL(CPD_EUNSUPPORTED, "tiled kernel built for 2..5 modes, not %d", N);
    if (R < 1 || R > 64 || ld % 4 || ld < ((R + 3) & ~3))
        CPD_FAIL(CPD_EUNSUPPORTED, "tiled kernel needs rank <= 64 and ld a multiple of 4 covering the rank");
    TiledView tv{};
    tv.toff = lt.toff;
    if (lt.rw != (N <= 3 ? 4 : 8)) CPD_FAIL(CPD_EINVAL, "mode tiling records of %d words for %d modes", lt.rw, N);
    if (lt.depth < 1 || lt.depth >= N) CPD_FAIL(CPD_EINVAL, "tiling of level %d of %d", lt.depth, N);
    tv.rec = lt.rec;
    tv.n = nleaves;
    tv.ntiles = lt.ntiles;
    tv.B = lt.B;
    // the factors of the other levels, in the order of the records' indices
    LeafFac fv{};
    for (int l = 0, m = 0; l < N; ++l)
        if (l != lt.depth) fv.a[m++] = fac_by_level[l];
    if (nleaves == 0) return CPD_OK;
    const int RQ = (R + 3) & ~3;
    const int NG = 64 / (RQ / 4);
    const int UF = NG >= 7 ? 2 : 4;
    const size_t lds = sizeof(float) * ((((size_t)NG * UF + 1) * RQ + (size_t)lt.B * R + 3) & ~size_t(3));  // per wave
    switch (N) {
#define CPD_TILED_N(n)                                                                         \
    case n:                                                                                    \
        return bf16 ? launch_tiled_n<n, uint16_t>(tv, fv, ld, Y, ldo, R, UF, lds, s)           \
                    : launch_tiled_n<n, float>(tv, fv, ld, Y, ldo, R, UF, lds, s);
        CPD_TILED_N(2)
        CPD_TILED_N(3)
        CPD_TILED_N(4)
        CPD_TILED_N(5)
#undef CPD_TILED_N
    }
    return CPD_OK;
}

}  // namespace cpd
