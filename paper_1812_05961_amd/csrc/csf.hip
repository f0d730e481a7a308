// CSF construction on the GPU: index check, key packing, stable LSD radix sort,
// duplicate merge and fiber compression (the one-time "Sort" preprocessing of
// Section V-C and the compressed sparse fiber tree of Section III), plus the
// per-tile start nodes that the MTTKRP kernels split their work by.
#include <algorithm>
#include <numeric>

#include "csf.h"
#include "scan.h"

namespace cpd {

namespace {

constexpr int RS_THREADS = 256;            // == radix, one digit per thread in bookkeeping
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;

// Launch a kernel template instantiated for the level count (2..5; check_coo
// rejects other counts before any launch, and the rest are never launched).
constexpr int CSF_MAX_LEVELS = 5;
#define CPD_BY_LEVELS(nl, CALL)      \
    switch (nl) {                    \
        case 2: CALL(2); break;      \
        case 3: CALL(3); break;      \
        case 4: CALL(4); break;      \
        case 5: CALL(5); break;      \
        default: break;              \
    }

// Where each level's index sits in the packed 128-bit key (root most
// significant, leaf least).
struct KeyLayout {
    int nl;
    int shift[CPD_MAX_MODES];
    int bits[CPD_MAX_MODES];
};

struct LevelInds {
    const int32_t *p[CPD_MAX_MODES];
};

__device__ __forceinline__ uint32_t key_field(uint64_t lo, uint64_t hi, int s, int b) {
    if (b == 0) return 0u;
    uint64_t mask = (1ull << b) - 1ull;
    if (s >= 64) return (uint32_t)((hi >> (s - 64)) & mask);
    if (s + b <= 64) return (uint32_t)((lo >> s) & mask);
    return (uint32_t)(((lo >> s) | (hi << (64 - s))) & mask);
}

// Keys of the same nonzeros in another tree order: level l of the new order
// takes the field of level src[l] of the old one.
struct LevelMap {
    int src[CPD_MAX_MODES];
};

// The key of the same nonzero in the other layout (one-word keys).
// Level l of the new key: the field at bit src_shift[l] (mask[l] wide, already
// shifted down) of the old key, moved to bit dst_shift[l] -- resolved on the
// host, so the device reads each level's three numbers at fixed offsets.
struct Repack {
    const uint64_t *a;  // sorted keys in the old layout
    const float *val;   // their values
    int src_shift[CPD_MAX_MODES], dst_shift[CPD_MAX_MODES];
    uint64_t mask[CPD_MAX_MODES];
};

Repack make_repack(const uint64_t *a, const float *val, const KeyLayout &ka, const KeyLayout &kx,
                   const LevelMap &map) {
    Repack r{};
    r.a = a;
    r.val = val;
    for (int l = 0; l < kx.nl; ++l) {
        const int q = map.src[l];
        const bool used = kx.bits[l] > 0;  // a length-1 mode has no field (and may sit at bit 64)
        r.src_shift[l] = used ? ka.shift[q] : 0;
        r.dst_shift[l] = used ? kx.shift[l] : 0;
        r.mask[l] = used ? ((1ull << ka.bits[q]) - 1ull) : 0ull;
    }
    return r;
}

template <int NL>
__device__ __forceinline__ uint64_t repack_key(const Repack &r, uint64_t key) {
    uint64_t out = 0;
#pragma unroll
    for (int l = 0; l < NL; ++l) out |= ((key >> r.src_shift[l]) & r.mask[l]) << r.dst_shift[l];
    return out;
}

// Packed key of nonzero k (root index most significant) and its value as the
// sort payload (bits of the float), with the index check of every level.
template <int NL>
__global__ void k_pack(LevelInds in, KeyLayout kl, const int64_t *dims_by_level, const float *vals, int64_t n,
                       uint64_t *lo, uint64_t *hi, int32_t *pay, int32_t *bad) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    uint64_t a = 0, b = 0;
    bool ok = true;
#pragma unroll
    for (int l = 0; l < NL; ++l) {
        const int32_t v = in.p[l][k];
        ok = ok && v >= 0 && (int64_t)v < dims_by_level[l];
        uint64_t x = (uint64_t)(uint32_t)v;
        int s = kl.shift[l];
        if (kl.bits[l] == 0) continue;
        if (s >= 64) {
            b |= x << (s - 64);
        } else {
            a |= x << s;
            if (s > 0 && s + kl.bits[l] > 64) b |= x >> (64 - s);
        }
    }
    if (!ok) atomicOr(bad, 1);
    lo[k] = a;
    if (hi) hi[k] = b;
    pay[k] = __float_as_int(vals[k]);
}

// The same for four consecutive nonzeros per thread with 16-byte loads and
// stores (index arrays and values 16-byte aligned; the last partial group
// element by element).
template <int NL>
__global__ void k_pack4(LevelInds in, KeyLayout kl, const int64_t *dims_by_level, const float *vals, int64_t n,
                        uint64_t *lo, uint64_t *hi, int32_t *pay, int32_t *bad) {
    const int64_t k0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (k0 >= n) return;
    const bool full = k0 + 4 <= n;
    int32_t v[NL][4];
    float x[4];
    if (full) {
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            const int4 q = *reinterpret_cast<const int4 *>(in.p[l] + k0);
            v[l][0] = q.x;
            v[l][1] = q.y;
            v[l][2] = q.z;
            v[l][3] = q.w;
        }
        const float4 f = *reinterpret_cast<const float4 *>(vals + k0);
        x[0] = f.x;
        x[1] = f.y;
        x[2] = f.z;
        x[3] = f.w;
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const bool in_r = k0 + j < n;
#pragma unroll
            for (int l = 0; l < NL; ++l) v[l][j] = in_r ? in.p[l][k0 + j] : 0;
            x[j] = in_r ? vals[k0 + j] : 0.0f;
        }
    }
    uint64_t a[4], b[4];
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        a[j] = 0;
        b[j] = 0;
        const bool in_r = k0 + j < n;
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            const int32_t w = v[l][j];
            ok = ok && (!in_r || (w >= 0 && (int64_t)w < dims_by_level[l]));
            const uint64_t q = (uint64_t)(uint32_t)w;
            const int sh = kl.shift[l];
            if (kl.bits[l] == 0) continue;
            if (sh >= 64) {
                b[j] |= q << (sh - 64);
            } else {
                a[j] |= q << sh;
                if (sh > 0 && sh + kl.bits[l] > 64) b[j] |= q >> (64 - sh);
            }
        }
    }
    if (!ok) atomicOr(bad, 1);
    if (full) {
        reinterpret_cast<ulonglong2 *>(lo + k0)[0] = make_ulonglong2(a[0], a[1]);
        reinterpret_cast<ulonglong2 *>(lo + k0)[1] = make_ulonglong2(a[2], a[3]);
        if (hi) {
            reinterpret_cast<ulonglong2 *>(hi + k0)[0] = make_ulonglong2(b[0], b[1]);
            reinterpret_cast<ulonglong2 *>(hi + k0)[1] = make_ulonglong2(b[2], b[3]);
        }
        *reinterpret_cast<int4 *>(pay + k0) =
            make_int4(__float_as_int(x[0]), __float_as_int(x[1]), __float_as_int(x[2]), __float_as_int(x[3]));
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (k0 + j < n) {
                lo[k0 + j] = a[j];
                if (hi) hi[k0 + j] = b[j];
                pay[k0 + j] = __float_as_int(x[j]);
            }
    }
}

// ---- radix sort: per-tile digit histogram (digit-major output)
// RPN > 0: the keys are those of rp.a (RPN levels) in layout rp.kx (the
// first pass of a re-sort into another tree order).
template <int RPN>
__global__ void __launch_bounds__(RS_THREADS)
k_radix_hist(const uint64_t *keys, Repack rp, int64_t n, int shift, int32_t *hist, int64_t ntiles) {
    __shared__ int32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    // every load of the tile in flight before the first count
    uint32_t dg[RS_ITEMS];
#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j) {
        const int64_t i = base + (int64_t)j * RS_THREADS + threadIdx.x;
        const uint64_t key = i < n ? (RPN ? repack_key<RPN>(rp, rp.a[i]) : keys[i]) : 0ull;
        dg[j] = i < n ? (uint32_t)(key >> shift) & 255u : 256u;
    }
#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j)
        if (dg[j] < 256u) atomicAdd(&h[dg[j]], 1);
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// ---- radix sort: stable scatter.  Tile items are taken in rounds of 256
// consecutive keys; inside a round, the rank of a key among equal digits is
// (earlier rounds) + (earlier waves of this round) + (earlier lanes of its
// wave), which keeps the input order of equal digits.
__global__ void __launch_bounds__(RS_THREADS)
k_radix_scatter(const uint64_t *klo, const uint64_t *khi, const int32_t *pay, uint64_t *olo,
                uint64_t *ohi, int32_t *opay, const int32_t *offsets, int64_t n, int64_t ntiles,
                int word, int shift) {
    __shared__ int32_t base_d[256];
    __shared__ int32_t wcnt[4][256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    base_d[tid] = offsets[(int64_t)tid * ntiles + blockIdx.x];
    for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    const int64_t tbase = (int64_t)blockIdx.x * RS_TILE;
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    for (int r = 0; r < RS_ITEMS; ++r) {
        int64_t i = tbase + (int64_t)r * RS_THREADS + tid;
        bool valid = i < n;
        uint64_t a = valid ? klo[i] : 0ull;
        uint64_t b = (valid && khi) ? khi[i] : 0ull;
        uint32_t d = (uint32_t)(((word ? b : a) >> shift) & 255u);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            bool set = (d >> bit) & 1u;
            uint64_t m = __ballot(set);
            peers &= set ? m : ~m;
        }
        int rank_w = __popcll(peers & lt);
        if (valid && rank_w == 0) wcnt[wave][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int32_t pos = base_d[d] + rank_w;
            for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
            olo[pos] = a;
            if (ohi) ohi[pos] = b;
            opay[pos] = pay[i];
        }
        __syncthreads();
        base_d[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
        wcnt[0][tid] = wcnt[1][tid] = wcnt[2][tid] = wcnt[3][tid] = 0;
        __syncthreads();
    }
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---- radix sort: stable scatter of one-word keys through LDS.  Each wave
// ranks a contiguous quarter of the tile against its own digit counters (no
// block barrier per round); the per-wave counts then give every wave's start
// for each digit.  The tile is reordered by digit in LDS and written out run
// by run, so consecutive threads store to consecutive addresses: first the
// keys, then the payloads through the same LDS buffer.  Equal digits keep
// their input order (waves in tile order, rounds in wave order, lanes in
// round order).
constexpr int RS_WAVES = RS_THREADS / 64;
constexpr int RS_WAVE_ITEMS = RS_TILE / RS_WAVES;

template <int RPN>
__global__ void __launch_bounds__(RS_THREADS)
k_radix_scatter1(const uint64_t *__restrict__ keys, const int32_t *__restrict__ pay, Repack rp,
                 uint64_t *__restrict__ okeys, int32_t *__restrict__ opay, const int32_t *__restrict__ offsets,
                 int64_t n, int64_t ntiles, int shift) {
    __shared__ uint64_t s_buf[RS_TILE];       // the tile in digit order: keys, then payloads
    __shared__ int32_t s_cnt[RS_WAVES][256];  // per-wave digit counts, then each wave's digit starts
    __shared__ int32_t s_off[256];            // global start minus tile start, per digit
    __shared__ int32_t s_wsum[RS_WAVES];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t tbase = (int64_t)blockIdx.x * RS_TILE;
    const int tn = (int)min<int64_t>(RS_TILE, n - tbase);
    int32_t *wc = s_cnt[wave];
    for (int j = lane; j < 256; j += 64) wc[j] = 0;
    uint64_t k[RS_ITEMS];
    int32_t p[RS_ITEMS], rk[RS_ITEMS];
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
        const int j = wave * RS_WAVE_ITEMS + r * 64 + lane;
        if (RPN) {
            k[r] = j < tn ? repack_key<RPN>(rp, rp.a[tbase + j]) : 0ull;
            p[r] = j < tn ? __float_as_int(rp.val[tbase + j]) : 0;
        } else {
            k[r] = j < tn ? keys[tbase + j] : 0ull;
            p[r] = j < tn ? pay[tbase + j] : 0;
        }
    }
    wave_sync();
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
        const bool valid = wave * RS_WAVE_ITEMS + r * 64 + lane < tn;
        const uint32_t d = (uint32_t)(k[r] >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool set = (d >> bit) & 1u;
            const uint64_t m = __ballot(set);
            peers &= set ? m : ~m;
        }
        const int below = __popcll(peers & lt);
        const int before = valid ? wc[d] : 0;
        rk[r] = before + below;
        wave_sync();
        if (valid && below == 0) wc[d] = before + __popcll(peers);
        wave_sync();
    }
    __syncthreads();
    // thread tid owns digit tid: the tile's count, its exclusive scan over
    // digits, and each wave's start
    int32_t c[RS_WAVES], tot = 0;
#pragma unroll
    for (int w = 0; w < RS_WAVES; ++w) {
        c[w] = s_cnt[w][tid];
        tot += c[w];
    }
    int32_t incl = tot;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) s_wsum[wave] = incl;
    __syncthreads();
    int32_t excl = incl - tot;
    for (int w = 0; w < wave; ++w) excl += s_wsum[w];
    int32_t run = excl;
#pragma unroll
    for (int w = 0; w < RS_WAVES; ++w) {
        s_cnt[w][tid] = run;
        run += c[w];
    }
    s_off[tid] = offsets[(int64_t)tid * ntiles + blockIdx.x] - excl;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
        if (wave * RS_WAVE_ITEMS + r * 64 + lane < tn) {
            rk[r] += wc[(uint32_t)(k[r] >> shift) & 255u];  // position in the digit-ordered tile
            s_buf[rk[r]] = k[r];
        }
    }
    __syncthreads();
    int32_t g[RS_ITEMS];
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        const int e = i * RS_THREADS + tid;
        g[i] = -1;
        if (e < tn) {
            const uint64_t key = s_buf[e];
            const int64_t at = (int64_t)s_off[(key >> shift) & 255u] + e;
            if ((uint64_t)at < (uint64_t)n) {  // always, when the histogram matches the tile
                okeys[at] = key;
                g[i] = (int32_t)at;
            }
        }
    }
    __syncthreads();
    int32_t *s_pay = reinterpret_cast<int32_t *>(s_buf);
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r)
        if (wave * RS_WAVE_ITEMS + r * 64 + lane < tn) s_pay[rk[r]] = p[r];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        const int e = i * RS_THREADS + tid;
        if (e < tn && g[i] >= 0) opay[g[i]] = s_pay[e];
    }
}

struct HistAt {
    const int32_t *h;
    __device__ int32_t operator()(int64_t i) const { return h[i]; }
};

}  // namespace

// Stable LSD radix sort of n keys (one or two 64-bit words) on key bits
// [lo_bit, bits) with an int32 payload, 8 bits per pass, ping-ponging between
// the (k*, p*) and (o*, op*) buffers; on return k*, kp point at the sorted
// data.  With lo_bit > 0 the order of equal sorted bits is the input order.
static cpd_status radix_sort_rp(uint64_t *&klo, uint64_t *&khi, int32_t *&kp, uint64_t *&olo, uint64_t *&ohi,
                                int32_t *&op, int64_t n, int bits, hipStream_t s, int lo_bit, const Repack *rp,
                                int rp_levels = 0) {
    const int64_t ntiles = ceil_div(n, RS_TILE);
    if (ntiles == 0) return CPD_OK;
    DevBuf<int32_t> hist;
    CPD_TRY(hist.alloc((size_t)256 * ntiles, s));
    const int passes = std::max((bits - lo_bit + 7) / 8, rp ? 1 : 0);
    const Repack none{};
    for (int d = 0; d < passes; ++d) {
        int word = (lo_bit + 8 * d) / 64, shift = (lo_bit + 8 * d) % 64;
        const uint64_t *src = word ? khi : klo;
        const bool first = rp && d == 0;
        const Repack &r = first ? *rp : none;
        if (first) {
#define CPD_HIST_RP(L)                                                                                          \
    hipLaunchKernelGGL(k_radix_hist<L>, dim3((unsigned)ntiles), dim3(RS_THREADS), 0, s, src, r, n, shift, hist.p, \
                       ntiles)
            CPD_BY_LEVELS(rp_levels, CPD_HIST_RP)
#undef CPD_HIST_RP
        } else {
            hipLaunchKernelGGL(k_radix_hist<0>, dim3((unsigned)ntiles), dim3(RS_THREADS), 0, s, src, r, n, shift,
                               hist.p, ntiles);
        }
        CPD_LAUNCH_CHECK();
        CPD_TRY(exclusive_scan(HistAt{hist.p}, 256 * ntiles, hist.p, (int32_t *)nullptr, s));
        if (khi)
            hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)ntiles), dim3(RS_THREADS), 0, s, klo, khi, kp, olo,
                               ohi, op, (const int32_t *)hist.p, n, ntiles, word, shift);
        else if (first) {
#define CPD_SCATTER_RP(L)                                                                                       \
    hipLaunchKernelGGL(k_radix_scatter1<L>, dim3((unsigned)ntiles), dim3(RS_THREADS), 0, s, (const uint64_t *)klo, \
                       (const int32_t *)kp, r, olo, op, (const int32_t *)hist.p, n, ntiles, shift)
            CPD_BY_LEVELS(rp_levels, CPD_SCATTER_RP)
#undef CPD_SCATTER_RP
        } else {
            hipLaunchKernelGGL(k_radix_scatter1<0>, dim3((unsigned)ntiles), dim3(RS_THREADS), 0, s,
                               (const uint64_t *)klo, (const int32_t *)kp, r, olo, op, (const int32_t *)hist.p, n,
                               ntiles, shift);
        }
        CPD_LAUNCH_CHECK();
        std::swap(klo, olo);
        std::swap(khi, ohi);
        std::swap(kp, op);
    }
    return CPD_OK;
}

cpd_status radix_sort(uint64_t *&klo, uint64_t *&khi, int32_t *&kp, uint64_t *&olo, uint64_t *&ohi, int32_t *&op,
                      int64_t n, int bits, hipStream_t s, int lo_bit) {
    return radix_sort_rp(klo, khi, kp, olo, ohi, op, n, bits, s, lo_bit, nullptr);
}

namespace {

// ---- leaf ranking: leaf ids ordered by how often a strided sample of the
// leaves holds them (descending, ties by id); only the order of a private
// copy of the leaf factor depends on it, never a result.
__global__ void k_sample_field(const uint64_t *lo, const uint64_t *hi, int shift, int bits, int64_t stride, int64_t ns,
                               uint64_t *key, int32_t *pay) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ns) return;
    key[i] = key_field(lo[i * stride], hi ? hi[i * stride] : 0ull, shift, bits);
    pay[i] = 0;
}

__global__ void k_sample(const int32_t *ids, int64_t stride, int64_t ns, uint64_t *key, int32_t *pay) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ns) return;
    key[i] = (uint64_t)(uint32_t)ids[i * stride];
    pay[i] = 0;
}

struct RunStart {
    const uint64_t *key;
    __device__ int32_t operator()(int64_t i) const { return (i == 0 || key[i] != key[i - 1]) ? 1 : 0; }
};

__global__ void k_run_starts(const uint64_t *key, const int32_t *pos, int64_t ns, int32_t *starts) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ns || !(i == 0 || key[i] != key[i - 1])) return;
    starts[pos[i]] = (int32_t)i;
}

__global__ void k_run_counts(const uint64_t *key, const int32_t *starts, const int32_t *nruns, int64_t ns,
                             int32_t *cnt) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t nr = *nruns;
    if (r >= nr) return;
    const int32_t b = starts[r], e = (r + 1 < nr) ? starts[r + 1] : (int32_t)ns;
    cnt[key[b]] = e - b;
}

__global__ void k_rank_keys(const int32_t *cnt, int64_t nid, int64_t ns, int ibits, uint64_t *key, int32_t *pay) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nid) return;
    key[i] = ((uint64_t)(ns - cnt[i]) << ibits) | (uint64_t)i;
    pay[i] = 0;
}

__global__ void k_rank_scatter(const uint64_t *key, int64_t nid, int ibits, int32_t *perm, int32_t *rank) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nid) return;
    const int32_t id = (int32_t)(key[r] & ((1ull << ibits) - 1ull));
    perm[r] = id;
    rank[id] = (int32_t)r;
}

// First level at which sorted key k differs from key k-1 (0 for k = 0, NL for
// an exact duplicate, which also sets *dup).  Four consecutive keys per
// thread, their four levels stored as one word (dl 4-byte aligned).
template <int NL>
__device__ __forceinline__ int first_diff_level(const KeyLayout &kl, uint64_t xa, uint64_t xb) {
    int l = NL;
#pragma unroll
    for (int q = NL - 1; q >= 0; --q)
        if (key_field(xa, xb, kl.shift[q], kl.bits[q]) != 0u) l = q;
    return l;
}

template <int NL>
__global__ void k_first_diff(const uint64_t *__restrict__ lo, const uint64_t *__restrict__ hi, KeyLayout kl,
                             int64_t n, uint8_t *__restrict__ dl, int32_t *dup) {
    const int64_t k0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (k0 >= n) return;
    uint64_t a[5], b[5];  // keys k0-1 .. k0+3
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        const int64_t k = k0 - 1 + j;
        const bool in = k >= 0 && k < n;
        a[j] = in ? lo[k] : 0ull;
        b[j] = (in && hi) ? hi[k] : 0ull;
    }
    uint32_t w = 0;
    bool seen_dup = false;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t k = k0 + j;
        int l = 0;
        if (k > 0 && k < n) l = first_diff_level<NL>(kl, a[j + 1] ^ a[j], b[j + 1] ^ b[j]);
        seen_dup = seen_dup || (k < n && l == NL);
        w |= (uint32_t)l << (8 * j);
    }
    if (k0 + 4 <= n) {
        *reinterpret_cast<uint32_t *>(dl + k0) = w;
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (k0 + j < n) dl[k0 + j] = (uint8_t)(w >> (8 * j));
    }
    if (seen_dup && dup) atomicOr(dup, 1);
}

struct IsNew {
    const uint8_t *dl;
    int nl;
    __device__ int32_t operator()(int64_t i) const { return dl[i] < nl ? 1 : 0; }
};

// One thread per run of equal keys: the float sum of the run in input order
// (the sort is stable, so the run is in input order).
__global__ void k_merge(const uint64_t *lo, const uint64_t *hi, const int32_t *pay, const uint8_t *dl,
                        const int32_t *pos, int64_t n, int nl, uint64_t *ulo, uint64_t *uhi, float *uval,
                        uint8_t *udl) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n || dl[k] >= nl) return;
    float s = __int_as_float(pay[k]);
    for (int64_t j = k + 1; j < n && dl[j] >= nl; ++j) s += __int_as_float(pay[j]);
    int32_t p = pos[k];
    ulo[p] = lo[k];
    if (uhi) uhi[p] = hi[k];
    uval[p] = s;
    udl[p] = dl[k];
}

__global__ void k_set_last_const(int32_t *fptr, int64_t at, int32_t value) { fptr[at] = value; }

// Node holding the first leaf of each tile, at every level < N-1.
struct FptrSet {
    const int32_t *p[CPD_MAX_MODES];
    int64_t len[CPD_MAX_MODES];  // count[l] (fptr[l] has count[l]+1 entries)
};

__global__ void k_tiles(FptrSet fp, int nl, int64_t nleaves, int32_t tile, int64_t ntiles,
                        int32_t *starts) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    int64_t pos = t * (int64_t)tile;
    if (pos >= nleaves) pos = nleaves - 1;
    for (int l = nl - 2; l >= 0; --l) {
        // largest j in [0, len) with fptr[l][j] <= pos
        const int32_t *p = fp.p[l];
        int64_t lo = 0, hi = fp.len[l] - 1;
        while (lo < hi) {
            int64_t mid = (lo + hi + 1) >> 1;
            if (p[mid] <= pos) lo = mid; else hi = mid - 1;
        }
        starts[(int64_t)l * ntiles + t] = (int32_t)lo;
        pos = lo;
    }
}

inline unsigned grid1(int64_t n, int t = 256) { return (unsigned)ceil_div(n, t); }

__global__ void k_max_run(const int32_t *starts, const int32_t *nruns, int64_t ns, int32_t *out) {
    __shared__ int32_t red[4];
    const int32_t nr = *nruns;
    int32_t mx = 0;
    for (int64_t r = threadIdx.x; r < nr; r += blockDim.x) {
        const int32_t e = (r + 1 < nr) ? starts[r + 1] : (int32_t)ns;
        mx = max(mx, e - starts[r]);
    }
    for (int o = 32; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = nr;
        out[1] = max(max(red[0], red[1]), max(red[2], red[3]));
        out[2] = (int32_t)ns;
    }
}

// Return every array of the tree for reuse on stream s (the slab to the
// scratch cache, lazily built tables to the stream-ordered pool).
void release_arrays(cpd_csf_s *c, hipStream_t s) {
    if (c->slab) scratch_put(c->slab, c->slab_bytes, s);
    for (int l = 0; l < CPD_MAX_MODES; ++l) {
        if (c->lvl_perm[l]) (void)hipFreeAsync(c->lvl_perm[l], s);
        if (c->lvl_rank[l]) (void)hipFreeAsync(c->lvl_rank[l], s);
    }
    for (auto &t : c->tiles) (void)hipFreeAsync(t.starts, s);
    for (auto &t : c->leaf_tilings) (void)hipFreeAsync(t.slab, s);
    (void)hipGetLastError();
}

}  // namespace

void free_csf_on(cpd_csf_s *c, hipStream_t s) {
    if (!c) return;
    release_arrays(c, s);
    delete c;
}

namespace {

void free_csf(cpd_csf_s *c) {
    if (!c) return;
    // work on any stream may still read the arrays: wait for the device, after
    // which the arrays are idle (the build stream may be gone: use the null
    // stream)
    (void)hipDeviceSynchronize();
    release_arrays(c, nullptr);
    delete c;
}

// Device flag words of a build: [0] an index out of range, [1] merged
// nonzeros (and ranking scratch), [2 .. 2+N-2] node counts per level,
// [FLAG_DUP] duplicates present.
constexpr int FLAG_DUP = 2 + CPD_MAX_MODES, FLAG_WORDS = FLAG_DUP + 1;

// Build arguments shared by every entry point.
cpd_status check_coo(int nm, const int64_t *dims, int64_t nnz, const int32_t *const *inds, const float *vals,
                     const void *out) {
    if (nm < 2 || nm > CPD_MAX_MODES) CPD_FAIL(CPD_EINVAL, "nmodes %d not in [2, %d]", nm, CPD_MAX_MODES);
    // the build kernels are instantiated for 2..5 levels (key packing, first
    // differing level, per-level node counts in 16-bit fields of one word)
    if (nm > CSF_MAX_LEVELS)
        CPD_FAIL(CPD_EUNSUPPORTED, "CSF trees are built for 2..%d modes, not %d", CSF_MAX_LEVELS, nm);
    if (!dims || !inds || !vals || !out) CPD_FAIL(CPD_EINVAL, "null argument");
    if (nnz < 1 || nnz > INT32_MAX) CPD_FAIL(CPD_EINVAL, "nnz %lld not in [1, 2^31-1]", (long long)nnz);
    for (int m = 0; m < nm; ++m) {
        if (dims[m] < 1 || dims[m] > INT32_MAX) CPD_FAIL(CPD_EINVAL, "dim %d = %lld out of range", m, (long long)dims[m]);
        if (!inds[m]) CPD_FAIL(CPD_EINVAL, "null index array for mode %d", m);
    }
    return CPD_OK;
}

// Key layout of a tree order: level l's index at bits [shift[l], shift[l] +
// bits[l]), the root most significant; *total: the key's bit count.
KeyLayout key_layout(int nm, const int64_t *dims, const int32_t *order, int *total) {
    KeyLayout kl{};
    kl.nl = nm;
    int t = 0;
    for (int l = nm - 1; l >= 0; --l) {
        const int64_t d = dims[order[l]];
        int b = 0;
        while ((1ll << b) < d) ++b;
        kl.bits[l] = b;
        kl.shift[l] = t;
        t += b;
    }
    *total = t;
    return kl;
}

// ---- fiber compression in two passes over the sorted nonzeros.  Pass 1:
// per tile of CT_TILE nonzeros, the number that open a node at each level
// l < N-1 (first differing level <= l).
constexpr int CT_THREADS = 256, CT_ITEMS = 16, CT_TILE = CT_THREADS * CT_ITEMS;

// CT_ITEMS consecutive first-difference levels from position i (255 past n):
// one 16-byte load when the run is whole (the array is 16-byte aligned).
__device__ __forceinline__ void load_levels(const uint8_t *__restrict__ dl, int64_t n, int64_t i,
                                            uint8_t (&d)[CT_ITEMS]) {
    static_assert(CT_ITEMS == 16, "one 16-byte load per thread");
    if (i + CT_ITEMS <= n) {
        const uint4 q = *reinterpret_cast<const uint4 *>(dl + i);
        const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int j = 0; j < CT_ITEMS; ++j) d[j] = (uint8_t)(w[j >> 2] >> (8 * (j & 3)));
    } else {
#pragma unroll
        for (int j = 0; j < CT_ITEMS; ++j) d[j] = i + j < n ? dl[i + j] : (uint8_t)255;
    }
}

__global__ void __launch_bounds__(CT_THREADS)
k_level_counts(const uint8_t *__restrict__ dl, int64_t n, int nlv, int32_t *__restrict__ partial, int64_t nb) {
    __shared__ int32_t red[CT_THREADS / 64][CPD_MAX_MODES];
    const int64_t base = (int64_t)blockIdx.x * CT_TILE;
    int32_t c[CPD_MAX_MODES] = {};
    uint8_t d[CT_ITEMS];
    load_levels(dl, n, base + (int64_t)threadIdx.x * CT_ITEMS, d);
#pragma unroll
    for (int j = 0; j < CT_ITEMS; ++j)
        for (int l = 0; l < nlv; ++l) c[l] += d[j] <= l;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int l = 0; l < nlv; ++l) {
        int32_t v = c[l];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) red[wave][l] = v;
    }
    __syncthreads();
    if (threadIdx.x < nlv) {
        int32_t t = 0;
        for (int w = 0; w < CT_THREADS / 64; ++w) t += red[w][threadIdx.x];
        partial[(int64_t)threadIdx.x * nb + blockIdx.x] = t;
    }
}

// One block per level: exclusive scan of that level's tile counts in place,
// the level's node count to total[level].
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_levels(int32_t *partial, int64_t nb, int32_t *total) {
    __shared__ int32_t smem[4];
    int32_t *p = partial + (int64_t)blockIdx.x * nb;
    int32_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += SCAN_THREADS) {
        const int64_t i = b0 + threadIdx.x;
        const int32_t v = i < nb ? p[i] : 0;
        int32_t tot;
        const int32_t inc = block_inclusive_scan(v, smem, &tot);
        if (i < nb) p[i] = carry + inc - v;
        carry += tot;
    }
    if (threadIdx.x == 0) total[blockIdx.x] = carry;
}

struct TreeOut {
    int32_t *fids[CPD_MAX_MODES];
    int32_t *fptr[CPD_MAX_MODES];
    int32_t *uprow[CPD_MAX_MODES];  // levels 1..N-2, or null
    int32_t *leafw;                  // or null
    const int32_t *leaf_rank;        // with leafw
    float *vals;
};

// Pass 2: each tile scans its nonzeros' node openings (per level, packed in
// 16-bit fields: a tile holds at most 4096), so every node finds its slot;
// the node's index and first child are stored there.  Each nonzero's leaf
// index, leaf word, internal rows and value are written alongside.
template <int NL, bool TWO>
__global__ void __launch_bounds__(CT_THREADS)
k_compress(const uint64_t *__restrict__ lo, const uint64_t *__restrict__ hi, KeyLayout kl,
           const uint8_t *__restrict__ dl, const float *__restrict__ val, int64_t n,
           const int32_t *__restrict__ partial, int64_t nb, TreeOut t) {
    __shared__ __align__(16) uint8_t s_dl[CT_TILE];
    __shared__ uint64_t s_pre[CT_TILE];  // per nonzero: openings before it in the tile, per level
    __shared__ uint32_t s_w[2][CT_THREADS / 64];
    constexpr int nl = NL, nlv = NL - 1;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t base = (int64_t)blockIdx.x * CT_TILE;
    {
        uint8_t d[CT_ITEMS];
        load_levels(dl, n, base + (int64_t)tid * CT_ITEMS, d);
        uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int j = 0; j < CT_ITEMS; ++j) w[j >> 2] |= (uint32_t)d[j] << (8 * (j & 3));
        *reinterpret_cast<uint4 *>(s_dl + tid * CT_ITEMS) = make_uint4(w[0], w[1], w[2], w[3]);
    }
    __syncthreads();
    // this thread's CT_ITEMS consecutive nonzeros
    uint64_t own = 0;
    for (int j = 0; j < CT_ITEMS; ++j) {
        const int d = s_dl[tid * CT_ITEMS + j];
#pragma unroll
        for (int l = 0; l < nlv; ++l) own += (uint64_t)(d <= l) << (16 * l);
    }
    // exclusive scan over the block; no field exceeds 4096, so the two
    // 32-bit halves scan independently
    uint32_t h[2] = {(uint32_t)own, (uint32_t)(own >> 32)};
    uint32_t ex[2];
    for (int q = 0; q < 2; ++q) {
        uint32_t v = h[q];
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(v, o, 64);
            if (lane >= o) v += y;
        }
        if (lane == 63) s_w[q][wave] = v;
        ex[q] = v - h[q];
    }
    __syncthreads();
    for (int q = 0; q < 2; ++q)
        for (int w = 0; w < wave; ++w) ex[q] += s_w[q][w];
    uint64_t run = (uint64_t)ex[0] | ((uint64_t)ex[1] << 32);
    for (int j = 0; j < CT_ITEMS; ++j) {
        const int e = tid * CT_ITEMS + j;
        s_pre[e] = run;
        const int d = s_dl[e];
#pragma unroll
        for (int l = 0; l < nlv; ++l) run += (uint64_t)(d <= l) << (16 * l);
    }
    int32_t off[CPD_MAX_MODES];
#pragma unroll
    for (int l = 0; l < nlv; ++l) off[l] = partial[(int64_t)l * nb + blockIdx.x];
    __syncthreads();
    // half a tile at a time: its loads first (independent), then its stores
    constexpr int H = CT_ITEMS / 2;
    const int32_t *__restrict__ rank = t.leaf_rank;
    int32_t *__restrict__ fleaf = t.fids[nl - 1];
    int32_t *__restrict__ lw = t.leafw;
    float *__restrict__ vo = t.vals;
    for (int j0 = 0; j0 < CT_ITEMS; j0 += H) {
        uint64_t ka[H], kb[H];
        float v[H];
        int32_t leaf[H], rk[H];
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const int64_t k = base + (j0 + j) * CT_THREADS + tid;
            const bool in = k < n;
            ka[j] = in ? lo[k] : 0ull;
            kb[j] = (TWO && in) ? hi[k] : 0ull;
            v[j] = in ? val[k] : 0.0f;
        }
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const int64_t k = base + (j0 + j) * CT_THREADS + tid;
            leaf[j] = (int32_t)key_field(ka[j], kb[j], kl.shift[nl - 1], kl.bits[nl - 1]);
            rk[j] = (lw && k < n) ? rank[leaf[j]] : 0;
        }
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const int e = (j0 + j) * CT_THREADS + tid;
            const int64_t k = base + e;
            if (k < n) {
                const int d = s_dl[e];
                const uint64_t pre = s_pre[e];
#pragma unroll
                for (int l = 0; l < nlv; ++l) {
                    if (l < d) continue;
                    const int32_t slot = off[l] + (int32_t)((pre >> (16 * l)) & 0xffffu);
                    t.fids[l][slot] = (int32_t)key_field(ka[j], kb[j], kl.shift[l], kl.bits[l]);
                    t.fptr[l][slot] =
                        l + 1 < nlv ? off[l + 1] + (int32_t)((pre >> (16 * (l + 1))) & 0xffffu) : (int32_t)k;
                }
                fleaf[k] = leaf[j];
#pragma unroll
                for (int l = 1; l < nlv; ++l)
                    if (t.uprow[l]) t.uprow[l][k] = (int32_t)key_field(ka[j], kb[j], kl.shift[l], kl.bits[l]);
                if (lw) lw[k] = (int32_t)(((uint32_t)d << 29) | (uint32_t)rk[j]);
                vo[k] = v[j];
            }
        }
    }
}

// The sorted, merged nonzeros of one tree order: keys, values and the level
// at which each key first differs from the previous one.
struct Sorted {
    DevBuf<uint64_t> lo[2], hi[2];
    DevBuf<int32_t> pay[2];
    DevBuf<uint8_t> dl, mdl;
    DevBuf<float> mval;
    const uint64_t *klo = nullptr, *khi = nullptr;
    const float *val = nullptr;
    const uint8_t *udl = nullptr;
    int64_t n = 0;
};

// Index check, key packing, sort and duplicate merge (duplicates summed in
// input order) for one tree order.
cpd_status sort_merge(int nm, const KeyLayout &kl, int total_bits, const int32_t *const *inds, const int32_t *order,
                      const int64_t *dims, const float *vals, int64_t nnz, int32_t *d_flag, hipStream_t s,
                      Sorted &S) {
    const bool two = total_bits > 64;
    LevelInds li{};
    int64_t dims_l[CPD_MAX_MODES];
    for (int l = 0; l < nm; ++l) {
        li.p[l] = inds[order[l]];
        dims_l[l] = dims[order[l]];
    }
    DevBuf<int64_t> d_dims;
    CPD_TRY(d_dims.alloc(nm, s));
    CPD_HIP(hipMemcpyAsync(d_dims.p, dims_l, sizeof(int64_t) * nm, hipMemcpyHostToDevice, s));
    for (int b = 0; b < 2; ++b) {
        CPD_TRY(S.lo[b].alloc(nnz, s));
        if (two) CPD_TRY(S.hi[b].alloc(nnz, s));
        CPD_TRY(S.pay[b].alloc(nnz, s));
    }
    bool aligned = (reinterpret_cast<uintptr_t>(vals) & 15) == 0;
    for (int l = 0; l < nm; ++l) aligned = aligned && (reinterpret_cast<uintptr_t>(li.p[l]) & 15) == 0;
#define CPD_PACK(L)                                                                                          \
    if (aligned)                                                                                             \
        hipLaunchKernelGGL(k_pack4<L>, dim3(grid1(ceil_div(nnz, 4))), dim3(256), 0, s, li, kl,              \
                           (const int64_t *)d_dims.p, vals, nnz, S.lo[0].p, S.hi[0].p, S.pay[0].p, d_flag); \
    else                                                                                                     \
        hipLaunchKernelGGL(k_pack<L>, dim3(grid1(nnz)), dim3(256), 0, s, li, kl, (const int64_t *)d_dims.p,  \
                           vals, nnz, S.lo[0].p, S.hi[0].p, S.pay[0].p, d_flag)
    CPD_BY_LEVELS(nm, CPD_PACK)
#undef CPD_PACK
    CPD_LAUNCH_CHECK();
    uint64_t *klo = S.lo[0].p, *khi = S.hi[0].p, *olo = S.lo[1].p, *ohi = S.hi[1].p;
    int32_t *kp = S.pay[0].p, *op = S.pay[1].p;
    CPD_TRY(radix_sort(klo, khi, kp, olo, ohi, op, nnz, total_bits, s));

    // a4: duplicate merge (the merge positions only when there are duplicates)
    DevBuf<int32_t> pos;
    CPD_TRY(S.dl.alloc(nnz, s));
#define CPD_FIRST_DIFF(L)                                                                                    \
    hipLaunchKernelGGL(k_first_diff<L>, dim3(grid1(ceil_div(nnz, 4))), dim3(256), 0, s, klo, khi, kl, nnz, S.dl.p, \
                       d_flag + FLAG_DUP)
    CPD_BY_LEVELS(nm, CPD_FIRST_DIFF)
#undef CPD_FIRST_DIFF
    CPD_LAUNCH_CHECK();
    int32_t h_flag[FLAG_WORDS];
    CPD_HIP(hipMemcpyAsync(h_flag, d_flag, sizeof(int32_t) * FLAG_WORDS, hipMemcpyDeviceToHost, s));
    CPD_HIP(hipStreamSynchronize(s));
    if (h_flag[0]) CPD_FAIL(CPD_EINVAL, "an index is out of range for its mode");
    S.n = nnz;
    if (h_flag[FLAG_DUP]) {
        CPD_TRY(pos.alloc(nnz, s));
        CPD_TRY(exclusive_scan(IsNew{S.dl.p, nm}, nnz, pos.p, d_flag + 1, s));
        int32_t h_n = 0;
        CPD_HIP(hipMemcpyAsync(&h_n, d_flag + 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        CPD_HIP(hipStreamSynchronize(s));
        S.n = h_n;
    }
    // without duplicates the sorted arrays are the merged ones (the payload
    // carries the values' bits)
    S.klo = klo;
    S.khi = khi;
    S.udl = S.dl.p;
    S.val = reinterpret_cast<const float *>(kp);
    if (S.n != nnz) {
        CPD_TRY(S.mdl.alloc(nnz, s));
        CPD_TRY(S.mval.alloc(nnz, s));
        hipLaunchKernelGGL(k_merge, dim3(grid1(nnz)), dim3(256), 0, s, klo, khi, kp, S.dl.p, pos.p, nnz, nm, olo, ohi,
                           S.mval.p, S.mdl.p);
        CPD_LAUNCH_CHECK();
        S.klo = olo;
        S.khi = ohi;
        S.udl = S.mdl.p;
        S.val = S.mval.p;
    }
    return CPD_OK;
}

// The nonzeros of tree A (one-word keys, sorted and merged) in the order of
// a tree rooted at mode x with the other levels in A's order: A's order is
// the order of every key sharing a root index, so a stable sort on the new
// root field alone finishes it (Section III's sort, one field instead of all).
cpd_status derive(int nm, const int64_t *dims, const int32_t *order_a, const KeyLayout &ka, const Sorted &A, int x,
                  int32_t *order_x, KeyLayout *kx, hipStream_t s, Sorted &S) {
    LevelMap map{};
    order_x[0] = x;
    map.src[0] = -1;
    for (int l = 0, k = 1; l < nm; ++l) {
        if (order_a[l] == x) map.src[0] = l;
        else {
            order_x[k] = order_a[l];
            map.src[k++] = l;
        }
    }
    int total = 0;
    *kx = key_layout(nm, dims, order_x, &total);
    const int64_t n = A.n;
    for (int b = 0; b < 2; ++b) {
        CPD_TRY(S.lo[b].alloc(n, s));
        CPD_TRY(S.pay[b].alloc(n, s));
    }
    // the first sort pass forms the new keys from A's (no separate repack)
    const Repack rp = make_repack(A.klo, A.val, ka, *kx, map);
    uint64_t *klo = S.lo[0].p, *khi = nullptr, *olo = S.lo[1].p, *ohi = nullptr;
    int32_t *kp = S.pay[0].p, *op = S.pay[1].p;
    CPD_TRY(radix_sort_rp(klo, khi, kp, olo, ohi, op, n, total, s, kx->shift[0], &rp, nm));
    CPD_TRY(S.dl.alloc(n, s));
#define CPD_FIRST_DIFF(L)                                                                                 \
    hipLaunchKernelGGL(k_first_diff<L>, dim3(grid1(ceil_div(n, 4))), dim3(256), 0, s, klo, (const uint64_t *)nullptr, \
                       *kx, n, S.dl.p, (int32_t *)nullptr)
    CPD_BY_LEVELS(nm, CPD_FIRST_DIFF)
#undef CPD_FIRST_DIFF
    CPD_LAUNCH_CHECK();
    S.klo = klo;
    S.udl = S.dl.p;
    S.val = reinterpret_cast<const float *>(kp);
    S.n = n;
    return CPD_OK;
}

// a5: fiber compression of sorted, merged nonzeros into a tree, with the
// leaf words, leaf ranking and internal rows the MTTKRP kernels read.
cpd_status compress(int nm, const int64_t *dims, const int32_t *order, const KeyLayout &kl, const Sorted &S,
                    int32_t *d_flag, hipStream_t s, cpd_csf *out) {
    const int64_t n = S.n;
    const int nlv = nm - 1;
    const int64_t nb = ceil_div(n, CT_TILE);
    DevBuf<int32_t> partial;
    CPD_TRY(partial.alloc((size_t)nlv * nb, s));
    hipLaunchKernelGGL(k_level_counts, dim3((unsigned)nb), dim3(CT_THREADS), 0, s, S.udl, n, nlv, partial.p, nb);
    CPD_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_levels, dim3(nlv), dim3(SCAN_THREADS), 0, s, partial.p, nb, d_flag + 2);
    CPD_LAUNCH_CHECK();
    int32_t h_counts[CPD_MAX_MODES] = {};
    CPD_HIP(hipMemcpyAsync(h_counts, d_flag + 2, sizeof(int32_t) * nlv, hipMemcpyDeviceToHost, s));
    CPD_HIP(hipStreamSynchronize(s));

    cpd_csf_s *c = new (std::nothrow) cpd_csf_s();
    if (!c) CPD_FAIL(CPD_ENOMEM, "host allocation failed");
    c->nmodes = nm;
    for (int m = 0; m < nm; ++m) c->dims[m] = dims[m];
    for (int l = 0; l < nm; ++l) {
        c->order[l] = order[l];
        c->counts[l] = (l == nm - 1) ? n : h_counts[l];
    }
    cpd_status st = CPD_OK;
    // the tree's arrays are carved from one stream-ordered pool allocation
    // (256-byte aligned pieces): one allocation and one free per tree, and
    // repeated builds reuse the pool's pages
    const int64_t nid = dims[order[nm - 1]];
    const bool want_leafw = nid <= (1ll << 29);
    std::vector<std::pair<void **, size_t>> pieces;
    for (int l = 0; l < nm; ++l) {
        pieces.push_back({(void **)&c->fids[l], sizeof(int32_t) * c->counts[l]});
        if (l < nm - 1) pieces.push_back({(void **)&c->fptr[l], sizeof(int32_t) * (c->counts[l] + 1)});
    }
    pieces.push_back({(void **)&c->vals, sizeof(float) * n});
    if (want_leafw) {
        pieces.push_back({(void **)&c->leafw, sizeof(int32_t) * n});
        pieces.push_back({(void **)&c->leaf_perm, sizeof(int32_t) * nid});
        pieces.push_back({(void **)&c->leaf_rank, sizeof(int32_t) * nid});
        for (int l = 1; l < nm - 1; ++l) pieces.push_back({(void **)&c->uprow[l], sizeof(int32_t) * n});
    }
    size_t total = 0;
    for (auto &pc : pieces) total += (pc.second + 255) & ~(size_t)255;
    c->slab_bytes = std::max<size_t>(total, 256);
    void *slab = nullptr;
    bool ok = scratch_get(c->slab_bytes, s, &slab) == CPD_OK;
    c->slab = static_cast<char *>(slab);
    if (ok) {
        size_t off = 0;
        for (auto &pc : pieces) {
            *pc.first = c->slab + off;
            off += (pc.second + 255) & ~(size_t)255;
        }
    }
    if (!ok) {
        free_csf(c);
        CPD_FAIL(CPD_ENOMEM, "device allocation for the CSF failed");
    }
    // rank the leaf ids by frequency in a strided sample of the leaves
    if (c->leafw)
        st = rank_key_field(S.klo, S.khi, kl.shift[nm - 1], kl.bits[nm - 1], n, nid, c->leaf_perm, c->leaf_rank,
                            d_flag + 1, s);
    if (st == CPD_OK) {
        TreeOut t{};
        for (int l = 0; l < nm; ++l) {
            t.fids[l] = c->fids[l];
            t.fptr[l] = c->fptr[l];
            t.uprow[l] = c->uprow[l];
        }
        t.leafw = c->leafw;
        t.leaf_rank = c->leaf_rank;
        t.vals = c->vals;
#define CPD_COMPRESS(L)                                                                                         \
    if (S.khi)                                                                                                  \
        hipLaunchKernelGGL((k_compress<L, true>), dim3((unsigned)nb), dim3(CT_THREADS), 0, s, S.klo, S.khi, kl,   \
                           S.udl, S.val, n, (const int32_t *)partial.p, nb, t);                                 \
    else                                                                                                        \
        hipLaunchKernelGGL((k_compress<L, false>), dim3((unsigned)nb), dim3(CT_THREADS), 0, s, S.klo, S.khi, kl,  \
                           S.udl, S.val, n, (const int32_t *)partial.p, nb, t)
        CPD_BY_LEVELS(nm, CPD_COMPRESS)
#undef CPD_COMPRESS
        if (hipGetLastError() != hipSuccess) st = CPD_EHIP;
        for (int l = 0; l < nlv && st == CPD_OK; ++l) {
            hipLaunchKernelGGL(k_set_last_const, dim3(1), dim3(1), 0, s, c->fptr[l], c->counts[l],
                               (int32_t)c->counts[l + 1]);
            if (hipGetLastError() != hipSuccess) st = CPD_EHIP;
        }
    }
    if (st == CPD_OK && hipStreamSynchronize(s) != hipSuccess) st = CPD_EHIP;
    if (st != CPD_OK) {
        free_csf(c);
        CPD_FAIL(st, "CSF compression kernels failed");
    }
    *out = c;
    return CPD_OK;
}

cpd_status build(int nm, const int64_t *dims, int64_t nnz, const int32_t *const *inds,
                 const float *vals, const int32_t *order_in, hipStream_t s, cpd_csf *out) {
    CPD_TRY(check_coo(nm, dims, nnz, inds, vals, out));
    keep_pool_memory();
    int32_t order[CPD_MAX_MODES];
    if (order_in) {
        bool seen[CPD_MAX_MODES] = {};
        for (int l = 0; l < nm; ++l) {
            int m = order_in[l];
            if (m < 0 || m >= nm || seen[m]) CPD_FAIL(CPD_EINVAL, "order is not a permutation of the modes");
            seen[m] = true;
            order[l] = m;
        }
    } else {
        std::iota(order, order + nm, 0);
        std::stable_sort(order, order + nm, [&](int a, int b) { return dims[a] < dims[b]; });
    }
    int total_bits = 0;
    const KeyLayout kl = key_layout(nm, dims, order, &total_bits);
    if (total_bits > 128) CPD_FAIL(CPD_EUNSUPPORTED, "packed key needs %d bits (> 128)", total_bits);
    DevBuf<int32_t> d_flag;
    CPD_TRY(d_flag.alloc(FLAG_WORDS, s));
    CPD_HIP(hipMemsetAsync(d_flag.p, 0, sizeof(int32_t) * FLAG_WORDS, s));
    Sorted S;
    CPD_TRY(sort_merge(nm, kl, total_bits, inds, order, dims, vals, nnz, d_flag.p, s, S));
    return compress(nm, dims, order, kl, S, d_flag.p, s, out);
}

// One tree rooted at each mode, the other modes by descending length (ties
// by mode index).  The tree of the longest mode is built in full; every
// other tree is derived from its sorted nonzeros by a sort on its root field.
cpd_status build_rooted(int nm, const int64_t *dims, int64_t nnz, const int32_t *const *inds, const float *vals,
                        hipStream_t s, cpd_csf *out) {
    CPD_TRY(check_coo(nm, dims, nnz, inds, vals, out));
    for (int m = 0; m < nm; ++m) out[m] = nullptr;
    keep_pool_memory();
    int32_t desc[CPD_MAX_MODES];
    std::iota(desc, desc + nm, 0);
    std::stable_sort(desc, desc + nm, [&](int a, int b) { return dims[a] > dims[b]; });
    int total_bits = 0;
    const KeyLayout ka = key_layout(nm, dims, desc, &total_bits);
    if (total_bits > 128) CPD_FAIL(CPD_EUNSUPPORTED, "packed key needs %d bits (> 128)", total_bits);
    cpd_csf trees[CPD_MAX_MODES] = {};
    auto fail = [&](cpd_status st) {
        for (int m = 0; m < nm; ++m)
            if (trees[m]) free_csf(trees[m]);
        return st;
    };
    if (total_bits > 64) {
        // two-word keys: independent builds
        for (int m = 0; m < nm; ++m) {
            int32_t ord[CPD_MAX_MODES];
            ord[0] = m;
            for (int l = 0, k = 1; l < nm; ++l)
                if (desc[l] != m) ord[k++] = desc[l];
            cpd_status st = build(nm, dims, nnz, inds, vals, ord, s, &trees[m]);
            if (st != CPD_OK) return fail(st);
        }
    } else {
        DevBuf<int32_t> d_flag;
        CPD_TRY(d_flag.alloc(FLAG_WORDS, s));
        CPD_HIP(hipMemsetAsync(d_flag.p, 0, sizeof(int32_t) * FLAG_WORDS, s));
        Sorted A;
        CPD_TRY(sort_merge(nm, ka, total_bits, inds, desc, dims, vals, nnz, d_flag.p, s, A));
        cpd_status st = compress(nm, dims, desc, ka, A, d_flag.p, s, &trees[desc[0]]);
        if (st != CPD_OK) return fail(st);
        for (int i = 1; i < nm; ++i) {
            Sorted S;
            int32_t ord[CPD_MAX_MODES];
            KeyLayout kx{};
            st = derive(nm, dims, desc, ka, A, desc[i], ord, &kx, s, S);
            if (st == CPD_OK) st = compress(nm, dims, ord, kx, S, d_flag.p, s, &trees[desc[i]]);
            if (st != CPD_OK) return fail(st);
        }
    }
    for (int m = 0; m < nm; ++m) out[m] = trees[m];
    return CPD_OK;
}

}  // namespace

// Rank ids 0..nid-1 by their count in a strided sample (stride max(1,
// n / 2^22)) of n ids that `sample` writes as sort keys: most frequent first,
// ties by id.
template <typename Sampler>
static cpd_status rank_sampled(Sampler sample, int64_t n, int64_t nid, int32_t *perm, int32_t *rank, int32_t *nruns,
                               hipStream_t s) {
    const int64_t stride = std::max<int64_t>(1, n / (1 << 22));
    const int64_t ns = ceil_div(n, stride);
    int ibits = 0, cbits = 0;
    while ((1ll << ibits) < nid) ++ibits;
    while ((1ll << cbits) <= ns) ++cbits;
    DevBuf<uint64_t> sk0, sk1;
    DevBuf<int32_t> sp0, sp1, spos, sstart, cnt;
    const int64_t m = std::max(ns, nid);
    CPD_TRY(sk0.alloc(m, s));
    CPD_TRY(sk1.alloc(m, s));
    CPD_TRY(sp0.alloc(m, s));
    CPD_TRY(sp1.alloc(m, s));
    CPD_TRY(spos.alloc(ns, s));
    CPD_TRY(sstart.alloc(ns, s));
    CPD_TRY(cnt.alloc(nid, s));
    CPD_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int32_t) * nid, s));
    uint64_t *a = sk0.p, *ah = nullptr, *b = sk1.p, *bh = nullptr;
    int32_t *ap = sp0.p, *bp = sp1.p;
    CPD_TRY(sample(stride, ns, a, ap));
    CPD_TRY(radix_sort(a, ah, ap, b, bh, bp, ns, std::max(ibits, 1), s));
    CPD_TRY(exclusive_scan(RunStart{a}, ns, spos.p, nruns, s));
    hipLaunchKernelGGL(k_run_starts, dim3(grid1(ns)), dim3(256), 0, s, (const uint64_t *)a, (const int32_t *)spos.p,
                       ns, sstart.p);
    hipLaunchKernelGGL(k_run_counts, dim3(grid1(ns)), dim3(256), 0, s, (const uint64_t *)a,
                       (const int32_t *)sstart.p, (const int32_t *)nruns, ns, cnt.p);
    // key (ns - count, id): ascending = most frequent first, ties by id
    hipLaunchKernelGGL(k_rank_keys, dim3(grid1(nid)), dim3(256), 0, s, (const int32_t *)cnt.p, nid, ns, ibits, a, ap);
    CPD_LAUNCH_CHECK();
    CPD_TRY(radix_sort(a, ah, ap, b, bh, bp, nid, ibits + cbits, s));
    hipLaunchKernelGGL(k_rank_scatter, dim3(grid1(nid)), dim3(256), 0, s, (const uint64_t *)a, nid, ibits, perm,
                       rank);
    CPD_LAUNCH_CHECK();
    return CPD_OK;
}

cpd_status rank_ids(const int32_t *ids, int64_t n, int64_t nid, int32_t *perm, int32_t *rank, int32_t *nruns,
                    hipStream_t s) {
    auto sample = [&](int64_t stride, int64_t ns, uint64_t *key, int32_t *pay) -> cpd_status {
        hipLaunchKernelGGL(k_sample, dim3(grid1(ns)), dim3(256), 0, s, ids, stride, ns, key, pay);
        CPD_LAUNCH_CHECK();
        return CPD_OK;
    };
    return rank_sampled(sample, n, nid, perm, rank, nruns, s);
}

cpd_status rank_key_field(const uint64_t *lo, const uint64_t *hi, int shift, int bits, int64_t n, int64_t nid,
                          int32_t *perm, int32_t *rank, int32_t *nruns, hipStream_t s) {
    auto sample = [&](int64_t stride, int64_t ns, uint64_t *key, int32_t *pay) -> cpd_status {
        hipLaunchKernelGGL(k_sample_field, dim3(grid1(ns)), dim3(256), 0, s, lo, hi, shift, bits, stride, ns, key, pay);
        CPD_LAUNCH_CHECK();
        return CPD_OK;
    };
    return rank_sampled(sample, n, nid, perm, rank, nruns, s);
}

cpd_status csf_level_rank(cpd_csf_s *c, int l, const int32_t **perm, const int32_t **rank, hipStream_t s) {
    *perm = nullptr;
    *rank = nullptr;
    if (l < 1 || l >= c->nmodes) CPD_FAIL(CPD_EINVAL, "level %d has no ranking", l);
    if (!c->leaf_perm) return CPD_OK;
    if (l == c->nmodes - 1) {
        *perm = c->leaf_perm;
        *rank = c->leaf_rank;
        return CPD_OK;
    }
    std::lock_guard<std::mutex> g(c->mu);
    if (!c->lvl_perm[l]) {
        const int64_t nid = c->dims[c->order[l]];
        int32_t *pp = nullptr, *rr = nullptr;
        DevBuf<int32_t> nr;
        CPD_TRY(nr.alloc(1, s));
        if (device_alloc((void **)&pp, sizeof(int32_t) * nid, s) != CPD_OK ||
            device_alloc((void **)&rr, sizeof(int32_t) * nid, s) != CPD_OK) {
            if (pp) (void)hipFreeAsync(pp, s);
            CPD_FAIL(CPD_ENOMEM, "device allocation for a level ranking failed");
        }
        cpd_status st = rank_ids(c->fids[l], c->counts[l], nid, pp, rr, nr.p, s);
        if (st != CPD_OK) {
            (void)hipFreeAsync(pp, s);
            (void)hipFreeAsync(rr, s);
            return st;
        }
        c->lvl_perm[l] = pp;
        c->lvl_rank[l] = rr;
    }
    *perm = c->lvl_perm[l];
    *rank = c->lvl_rank[l];
    return CPD_OK;
}

cpd_status sample_freq(const int32_t *ids, int64_t n, int64_t nid, int64_t max_samples, int32_t *out,
                       hipStream_t s) {
    const int64_t stride = std::max<int64_t>(1, ceil_div(n, max_samples));
    const int64_t ns = ceil_div(n, stride);
    int ibits = 0;
    while ((1ll << ibits) < nid) ++ibits;
    DevBuf<uint64_t> k0, k1;
    DevBuf<int32_t> p0, p1, pos, starts, nr;
    CPD_TRY(k0.alloc(ns, s));
    CPD_TRY(k1.alloc(ns, s));
    CPD_TRY(p0.alloc(ns, s));
    CPD_TRY(p1.alloc(ns, s));
    CPD_TRY(pos.alloc(ns, s));
    CPD_TRY(starts.alloc(ns, s));
    CPD_TRY(nr.alloc(1, s));
    uint64_t *a = k0.p, *ah = nullptr, *b = k1.p, *bh = nullptr;
    int32_t *ap = p0.p, *bp = p1.p;
    hipLaunchKernelGGL(k_sample, dim3(grid1(ns)), dim3(256), 0, s, ids, stride, ns, a, ap);
    CPD_LAUNCH_CHECK();
    CPD_TRY(radix_sort(a, ah, ap, b, bh, bp, ns, std::max(ibits, 1), s));
    CPD_TRY(exclusive_scan(RunStart{a}, ns, pos.p, nr.p, s));
    hipLaunchKernelGGL(k_run_starts, dim3(grid1(ns)), dim3(256), 0, s, (const uint64_t *)a, (const int32_t *)pos.p, ns,
                       starts.p);
    hipLaunchKernelGGL(k_max_run, dim3(1), dim3(256), 0, s, (const int32_t *)starts.p, (const int32_t *)nr.p, ns, out);
    CPD_LAUNCH_CHECK();
    return CPD_OK;
}

// The ranking of level l when it already exists (the leaf ranking is made
// with the tree; internal levels once csf_level_rank has run): no allocation.
void csf_level_rank_cached(cpd_csf_s *c, int l, const int32_t **perm, const int32_t **rank) {
    *perm = nullptr;
    *rank = nullptr;
    if (l < 1 || l >= c->nmodes || !c->leaf_perm) return;
    if (l == c->nmodes - 1) {
        *perm = c->leaf_perm;
        *rank = c->leaf_rank;
        return;
    }
    std::lock_guard<std::mutex> g(c->mu);
    *perm = c->lvl_perm[l];
    *rank = c->lvl_rank[l];
}

// Tile table for a width without allocating: the cached table when it
// exists, else computed into dst (dst_bytes of device memory), not cached.
cpd_status csf_tiles_into(cpd_csf_s *c, int32_t tile, int32_t *dst, size_t dst_bytes, const int32_t **starts,
                          int64_t *ntiles, hipStream_t s) {
    if (tile < 1) CPD_FAIL(CPD_EINVAL, "tile width %d < 1", tile);
    const int nm = c->nmodes;
    const int64_t nl = c->counts[nm - 1];
    const int64_t nt = ceil_div(nl, tile);
    {
        std::lock_guard<std::mutex> g(c->mu);
        for (auto &t : c->tiles)
            if (t.tile == tile) {
                *starts = t.starts;
                *ntiles = t.ntiles;
                return CPD_OK;
            }
    }
    const size_t need = sizeof(int32_t) * (size_t)std::max<int64_t>(1, (nm - 1) * nt);
    if (!dst || need > dst_bytes)
        CPD_FAIL(CPD_EUNSUPPORTED, "tile table of %zu bytes does not fit the %zu-byte workspace", need, dst_bytes);
    FptrSet fp{};
    for (int l = 0; l < nm - 1; ++l) {
        fp.p[l] = c->fptr[l];
        fp.len[l] = c->counts[l];
    }
    hipLaunchKernelGGL(k_tiles, dim3(grid1(nt)), dim3(256), 0, s, fp, nm, nl, tile, nt, dst);
    CPD_LAUNCH_CHECK();
    *starts = dst;
    *ntiles = nt;
    return CPD_OK;
}

cpd_status csf_tiles(cpd_csf_s *c, int32_t tile, const int32_t **starts, int64_t *ntiles,
                     hipStream_t s) {
    if (tile < 1) CPD_FAIL(CPD_EINVAL, "tile width %d < 1", tile);
    std::lock_guard<std::mutex> g(c->mu);
    for (auto &t : c->tiles)
        if (t.tile == tile) {
            *starts = t.starts;
            *ntiles = t.ntiles;
            return CPD_OK;
        }
    const int nm = c->nmodes;
    const int64_t nl = c->counts[nm - 1];
    const int64_t nt = ceil_div(nl, tile);
    int32_t *p = nullptr;
    if (device_alloc((void **)&p, sizeof(int32_t) * (size_t)std::max<int64_t>(1, (nm - 1) * nt), s) != CPD_OK)
        CPD_FAIL(CPD_ENOMEM, "device allocation for the tile table failed");
    FptrSet fp{};
    for (int l = 0; l < nm - 1; ++l) {
        fp.p[l] = c->fptr[l];
        fp.len[l] = c->counts[l];
    }
    hipLaunchKernelGGL(k_tiles, dim3(grid1(nt)), dim3(256), 0, s, fp, nm, nl, tile, nt, p);
    if (hipGetLastError() != hipSuccess) {
        (void)hipFreeAsync(p, s);
        CPD_FAIL(CPD_EHIP, "tile kernel launch failed");
    }
    c->tiles.push_back({tile, nt, p});
    *starts = p;
    *ntiles = nt;
    return CPD_OK;
}

}  // namespace cpd

using namespace cpd;

extern "C" {

cpd_status cpd_csf_build(int32_t nmodes, const int64_t *dims, int64_t nnz, const int32_t *const *inds,
                         const float *vals, const int32_t *order, void *stream, cpd_csf *out) {
    clear_error();
    if (out) *out = nullptr;
    return build(nmodes, dims, nnz, inds, vals, order, (hipStream_t)stream, out);
}

cpd_status cpd_csf_build_rooted(int32_t nmodes, const int64_t *dims, int64_t nnz, const int32_t *const *inds,
                                const float *vals, void *stream, cpd_csf *out) {
    clear_error();
    if (out)
        for (int m = 0; m < std::min<int32_t>(std::max<int32_t>(nmodes, 0), CPD_MAX_MODES); ++m) out[m] = nullptr;
    return build_rooted(nmodes, dims, nnz, inds, vals, (hipStream_t)stream, out);
}

cpd_status cpd_csf_info(cpd_csf c, int32_t *nmodes, int32_t *order, int64_t *counts) {
    clear_error();
    if (!c) CPD_FAIL(CPD_EINVAL, "null CSF handle");
    if (nmodes) *nmodes = c->nmodes;
    for (int l = 0; l < c->nmodes; ++l) {
        if (order) order[l] = c->order[l];
        if (counts) counts[l] = c->counts[l];
    }
    return CPD_OK;
}

cpd_status cpd_csf_export(cpd_csf c, int32_t level, int32_t *fids, int32_t *fptr, float *vals,
                          void *stream) {
    clear_error();
    if (!c) CPD_FAIL(CPD_EINVAL, "null CSF handle");
    if (level < 0 || level >= c->nmodes) CPD_FAIL(CPD_EINVAL, "level %d out of range", level);
    hipStream_t s = (hipStream_t)stream;
    if (fids)
        CPD_HIP(hipMemcpyAsync(fids, c->fids[level], sizeof(int32_t) * c->counts[level],
                               hipMemcpyDeviceToDevice, s));
    if (fptr && level < c->nmodes - 1)
        CPD_HIP(hipMemcpyAsync(fptr, c->fptr[level], sizeof(int32_t) * (c->counts[level] + 1),
                               hipMemcpyDeviceToDevice, s));
    if (vals && level == c->nmodes - 1)
        CPD_HIP(hipMemcpyAsync(vals, c->vals, sizeof(float) * c->counts[level], hipMemcpyDeviceToDevice, s));
    return CPD_OK;
}

cpd_status cpd_csf_tiles(cpd_csf c, int32_t tile_nnz, int32_t *starts, int64_t *ntiles, void *stream) {
    clear_error();
    if (!c || !ntiles) CPD_FAIL(CPD_EINVAL, "null argument");
    const int32_t *p;
    int64_t nt;
    CPD_TRY(csf_tiles(c, tile_nnz, &p, &nt, (hipStream_t)stream));
    *ntiles = nt;
    if (starts && c->nmodes > 1)
        CPD_HIP(hipMemcpyAsync(starts, p, sizeof(int32_t) * (c->nmodes - 1) * nt, hipMemcpyDeviceToDevice,
                               (hipStream_t)stream));
    return CPD_OK;
}

void cpd_csf_free(cpd_csf c) {
    if (!c) return;
    (void)hipDeviceSynchronize();
    free_csf(c);
}

}  // extern "C"
