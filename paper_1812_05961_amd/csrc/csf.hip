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

// Packed key of nonzero k (root index most significant) and its value as the
// sort payload (bits of the float), with the index check of every level.
__global__ void k_pack(LevelInds in, KeyLayout kl, const int64_t *dims_by_level, const float *vals, int64_t n,
                       uint64_t *lo, uint64_t *hi, int32_t *pay, int32_t *bad) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    uint64_t a = 0, b = 0;
    bool ok = true;
    for (int l = 0; l < kl.nl; ++l) {
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

// ---- radix sort: per-tile digit histogram (digit-major output)
__global__ void __launch_bounds__(RS_THREADS)
k_radix_hist(const uint64_t *keys, int64_t n, int shift, int32_t *hist, int64_t ntiles) {
    __shared__ int32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j) {
        int64_t i = base + (int64_t)j * RS_THREADS + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1);
    }
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

// ---- radix sort: stable scatter of one-word keys through LDS.  The tile is
// ranked as above, reordered by digit in LDS, and written out run by run, so
// consecutive threads store to consecutive addresses.
__global__ void __launch_bounds__(RS_THREADS)
k_radix_scatter1(const uint64_t *__restrict__ keys, const int32_t *__restrict__ pay, uint64_t *__restrict__ okeys,
                 int32_t *__restrict__ opay, const int32_t *__restrict__ offsets, int64_t n, int64_t ntiles,
                 int shift) {
    __shared__ uint64_t s_key[RS_TILE];
    __shared__ int32_t s_pay[RS_TILE];
    __shared__ int32_t s_run[256];      // counts of earlier rounds, then the tile's digit starts
    __shared__ int32_t s_off[256];      // global start minus tile start, per digit
    __shared__ int32_t wcnt[2][4][256];  // per-wave digit counts, two rounds in flight
    __shared__ int32_t s_wsum[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    s_run[tid] = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) wcnt[0][w][tid] = wcnt[1][w][tid] = 0;
    const int64_t tbase = (int64_t)blockIdx.x * RS_TILE;
    const int tn = (int)min<int64_t>(RS_TILE, n - tbase);
    uint64_t k[RS_ITEMS];
    int32_t p[RS_ITEMS], rk[RS_ITEMS];
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
        const int j = r * RS_THREADS + tid;
        k[r] = j < tn ? keys[tbase + j] : 0ull;
        p[r] = j < tn ? pay[tbase + j] : 0;
    }
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
        const bool valid = r * RS_THREADS + tid < tn;
        const uint32_t d = (uint32_t)((k[r] >> shift) & 255u);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool set = (d >> bit) & 1u;
            const uint64_t m = __ballot(set);
            peers &= set ? m : ~m;
        }
        const int rank_w = __popcll(peers & lt);
        const int b = r & 1;
        if (valid && rank_w == 0) wcnt[b][wave][d] = __popcll(peers);
        __syncthreads();
        int x = s_run[d] + rank_w;
        for (int w = 0; w < wave; ++w) x += wcnt[b][w][d];
        rk[r] = x;
        __syncthreads();
        s_run[tid] += wcnt[b][0][tid] + wcnt[b][1][tid] + wcnt[b][2][tid] + wcnt[b][3][tid];
        wcnt[b][0][tid] = wcnt[b][1][tid] = wcnt[b][2][tid] = wcnt[b][3][tid] = 0;
    }
    __syncthreads();
    // exclusive scan of the tile's digit counts
    const int c = s_run[tid];
    int incl = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) s_wsum[wave] = incl;
    __syncthreads();
    int excl = incl - c;
    for (int w = 0; w < wave; ++w) excl += s_wsum[w];
    s_run[tid] = excl;
    s_off[tid] = offsets[(int64_t)tid * ntiles + blockIdx.x] - excl;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
        if (r * RS_THREADS + tid < tn) {
            const uint32_t d = (uint32_t)((k[r] >> shift) & 255u);
            const int at = s_run[d] + rk[r];
            s_key[at] = k[r];
            s_pay[at] = p[r];
        }
    }
    __syncthreads();
    for (int e = tid; e < tn; e += RS_THREADS) {
        const uint64_t key = s_key[e];
        const int64_t g = (int64_t)s_off[(key >> shift) & 255u] + e;
        okeys[g] = key;
        opay[g] = s_pay[e];
    }
}

struct HistAt {
    const int32_t *h;
    __device__ int32_t operator()(int64_t i) const { return h[i]; }
};

}  // namespace

// Stable LSD radix sort of n keys (one or two 64-bit words, `bits` significant
// bits) with an int32 payload, 8 bits per pass, ping-ponging between the
// (k*, p*) and (o*, op*) buffers; on return k*, kp point at the sorted data.
cpd_status radix_sort(uint64_t *&klo, uint64_t *&khi, int32_t *&kp, uint64_t *&olo, uint64_t *&ohi, int32_t *&op,
                      int64_t n, int bits, hipStream_t s) {
    const int64_t ntiles = ceil_div(n, RS_TILE);
    if (ntiles == 0) return CPD_OK;
    DevBuf<int32_t> hist;
    CPD_TRY(hist.alloc((size_t)256 * ntiles, s));
    const int passes = (bits + 7) / 8;
    for (int d = 0; d < passes; ++d) {
        int word = (8 * d) / 64, shift = (8 * d) % 64;
        const uint64_t *src = word ? khi : klo;
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)ntiles), dim3(RS_THREADS), 0, s, src, n, shift, hist.p, ntiles);
        CPD_LAUNCH_CHECK();
        CPD_TRY(exclusive_scan(HistAt{hist.p}, 256 * ntiles, hist.p, (int32_t *)nullptr, s));
        if (khi)
            hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)ntiles), dim3(RS_THREADS), 0, s, klo, khi, kp, olo,
                               ohi, op, (const int32_t *)hist.p, n, ntiles, word, shift);
        else
            hipLaunchKernelGGL(k_radix_scatter1, dim3((unsigned)ntiles), dim3(RS_THREADS), 0, s, klo, kp, olo, op,
                               (const int32_t *)hist.p, n, ntiles, shift);
        CPD_LAUNCH_CHECK();
        std::swap(klo, olo);
        std::swap(khi, ohi);
        std::swap(kp, op);
    }
    return CPD_OK;
}

namespace {

// ---- leaf ranking: leaf ids ordered by how often a strided sample of the
// leaves holds them (descending, ties by id); only the order of a private
// copy of the leaf factor depends on it, never a result.
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

__global__ void k_rank_keys(const int32_t *cnt, int64_t nid, uint64_t *key, int32_t *pay) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nid) return;
    key[i] = ((uint64_t)(0x7fffffff - cnt[i]) << 32) | (uint64_t)i;
    pay[i] = 0;
}

__global__ void k_rank_scatter(const uint64_t *key, int64_t nid, int32_t *perm, int32_t *rank) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nid) return;
    const int32_t id = (int32_t)(key[r] & 0xffffffffull);
    perm[r] = id;
    rank[id] = (int32_t)r;
}

// First level at which sorted key k differs from key k-1 (0 for k = 0, nl for
// an exact duplicate).
__global__ void k_first_diff(const uint64_t *lo, const uint64_t *hi, KeyLayout kl, int64_t n,
                             uint8_t *dl) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    if (k == 0) {
        dl[0] = 0;
        return;
    }
    uint64_t a = lo[k], b = hi ? hi[k] : 0ull, pa = lo[k - 1], pb = hi ? hi[k - 1] : 0ull;
    int l = 0;
    for (; l < kl.nl; ++l)
        if (key_field(a, b, kl.shift[l], kl.bits[l]) != key_field(pa, pb, kl.shift[l], kl.bits[l]))
            break;
    dl[k] = (uint8_t)l;
}

struct IsNew {
    const uint8_t *dl;
    int nl;
    __device__ int32_t operator()(int64_t i) const { return dl[i] < nl ? 1 : 0; }
};

struct AtLevel {
    const uint8_t *dl;
    int l;
    __device__ int32_t operator()(int64_t i) const { return dl[i] <= l ? 1 : 0; }
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

__global__ void k_compact(const uint64_t *lo, const uint64_t *hi, KeyLayout kl, const uint8_t *dl,
                          int64_t n, int l, const int32_t *scan_l, const int32_t *scan_next,
                          int32_t *fids, int32_t *fptr) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n || dl[k] > l) return;
    int32_t j = scan_l[k];
    fids[j] = (int32_t)key_field(lo[k], hi ? hi[k] : 0ull, kl.shift[l], kl.bits[l]);
    fptr[j] = scan_next ? scan_next[k] : (int32_t)k;
}

__global__ void k_leaf(const uint64_t *lo, const uint64_t *hi, KeyLayout kl, int64_t n,
                       int32_t *fids) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int l = kl.nl - 1;
    fids[k] = (int32_t)key_field(lo[k], hi ? hi[k] : 0ull, kl.shift[l], kl.bits[l]);
}

__global__ void k_leafw(const uint8_t *dl, const int32_t *fids, const int32_t *rank, int64_t n, int32_t *leafw) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    leafw[k] = (int32_t)(((uint32_t)dl[k] << 29) | (uint32_t)rank[fids[k]]);
}

__global__ void k_uprow(const uint64_t *lo, const uint64_t *hi, KeyLayout kl, int64_t n, int l, int32_t *out) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    out[k] = (int32_t)key_field(lo[k], hi ? hi[k] : 0ull, kl.shift[l], kl.bits[l]);
}

__global__ void k_set_last(int32_t *fptr, int64_t at, const int32_t *value) {
    fptr[at] = *value;
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

cpd_status build(int nm, const int64_t *dims, int64_t nnz, const int32_t *const *inds,
                 const float *vals, const int32_t *order_in, hipStream_t s, cpd_csf *out) {
    if (nm < 2 || nm > CPD_MAX_MODES) CPD_FAIL(CPD_EINVAL, "nmodes %d not in [2, %d]", nm, CPD_MAX_MODES);
    if (!dims || !inds || !vals || !out) CPD_FAIL(CPD_EINVAL, "null argument");
    if (nnz < 1 || nnz > INT32_MAX) CPD_FAIL(CPD_EINVAL, "nnz %lld not in [1, 2^31-1]", (long long)nnz);
    for (int m = 0; m < nm; ++m) {
        if (dims[m] < 1 || dims[m] > INT32_MAX) CPD_FAIL(CPD_EINVAL, "dim %d = %lld out of range", m, (long long)dims[m]);
        if (!inds[m]) CPD_FAIL(CPD_EINVAL, "null index array for mode %d", m);
    }
    keep_pool_memory();
    int order[CPD_MAX_MODES];
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
    KeyLayout kl{};
    kl.nl = nm;
    int total_bits = 0;
    for (int l = nm - 1; l >= 0; --l) {
        int64_t d = dims[order[l]];
        int b = 0;
        while ((1ll << b) < d) ++b;
        kl.bits[l] = b;
        kl.shift[l] = total_bits;
        total_bits += b;
    }
    if (total_bits > 128) CPD_FAIL(CPD_EUNSUPPORTED, "packed key needs %d bits (> 128)", total_bits);
    const bool two = total_bits > 64;
    LevelInds li{};
    int64_t dims_l[CPD_MAX_MODES];
    for (int l = 0; l < nm; ++l) {
        li.p[l] = inds[order[l]];
        dims_l[l] = dims[order[l]];
    }

    // a1: index check
    DevBuf<int64_t> d_dims;
    DevBuf<int32_t> d_flag;
    CPD_TRY(d_dims.alloc(nm, s));
    CPD_TRY(d_flag.alloc(1 + CPD_MAX_MODES, s));
    CPD_HIP(hipMemcpyAsync(d_dims.p, dims_l, sizeof(int64_t) * nm, hipMemcpyHostToDevice, s));
    CPD_HIP(hipMemsetAsync(d_flag.p, 0, sizeof(int32_t) * (1 + CPD_MAX_MODES), s));

    // a3: keys and stable LSD radix sort
    DevBuf<uint64_t> lo0, lo1, hi0, hi1;
    DevBuf<int32_t> p0, p1;
    CPD_TRY(lo0.alloc(nnz, s));
    CPD_TRY(lo1.alloc(nnz, s));
    if (two) {
        CPD_TRY(hi0.alloc(nnz, s));
        CPD_TRY(hi1.alloc(nnz, s));
    }
    CPD_TRY(p0.alloc(nnz, s));
    CPD_TRY(p1.alloc(nnz, s));
    hipLaunchKernelGGL(k_pack, dim3(grid1(nnz)), dim3(256), 0, s, li, kl, (const int64_t *)d_dims.p, vals, nnz,
                       lo0.p, hi0.p, p0.p, d_flag.p);
    CPD_LAUNCH_CHECK();
    uint64_t *klo = lo0.p, *khi = hi0.p, *olo = lo1.p, *ohi = hi1.p;
    int32_t *kp = p0.p, *op = p1.p;
    CPD_TRY(radix_sort(klo, khi, kp, olo, ohi, op, nnz, total_bits, s));

    // a4: duplicate merge
    DevBuf<uint8_t> dl;
    DevBuf<int32_t> pos;
    CPD_TRY(dl.alloc(nnz, s));
    CPD_TRY(pos.alloc(nnz, s));
    hipLaunchKernelGGL(k_first_diff, dim3(grid1(nnz)), dim3(256), 0, s, klo, khi, kl, nnz, dl.p);
    CPD_LAUNCH_CHECK();
    int32_t *d_nuniq = d_flag.p + 1;
    CPD_TRY(exclusive_scan(IsNew{dl.p, nm}, nnz, pos.p, d_nuniq, s));
    int32_t h_flag[2];
    CPD_HIP(hipMemcpyAsync(h_flag, d_flag.p, sizeof(int32_t) * 2, hipMemcpyDeviceToHost, s));
    CPD_HIP(hipStreamSynchronize(s));
    if (h_flag[0]) CPD_FAIL(CPD_EINVAL, "an index is out of range for its mode");
    const int64_t n = h_flag[1];

    // merged keys, levels and values; without duplicates the sorted arrays
    // are the merged ones (the payload carries the values' bits)
    DevBuf<uint8_t> udl_buf;
    DevBuf<float> uval_buf;
    const uint8_t *udl = dl.p;
    const float *uval = reinterpret_cast<const float *>(kp);
    if (n != nnz) {
        CPD_TRY(udl_buf.alloc(nnz, s));
        CPD_TRY(uval_buf.alloc(nnz, s));
        hipLaunchKernelGGL(k_merge, dim3(grid1(nnz)), dim3(256), 0, s, klo, khi, kp, dl.p, pos.p, nnz, nm, olo, ohi,
                           uval_buf.p, udl_buf.p);
        CPD_LAUNCH_CHECK();
        std::swap(klo, olo);
        std::swap(khi, ohi);
        udl = udl_buf.p;
        uval = uval_buf.p;
    }
    pos.release();

    // a5: fiber compression, levels N-2 .. 0
    std::vector<DevBuf<int32_t>> scans(nm - 1);
    for (int l = 0; l < nm - 1; ++l) {
        CPD_TRY(scans[l].alloc(n, s));
        CPD_TRY(exclusive_scan(AtLevel{udl, l}, n, scans[l].p, d_flag.p + 2 + l, s));
    }
    int32_t h_counts[CPD_MAX_MODES] = {};
    if (nm > 1)
        CPD_HIP(hipMemcpyAsync(h_counts, d_flag.p + 2, sizeof(int32_t) * (nm - 1), hipMemcpyDeviceToHost, s));
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
    const bool want_leafw = dims[order[nm - 1]] <= (1ll << 29);
    std::vector<std::pair<void **, size_t>> pieces;
    for (int l = 0; l < nm; ++l) {
        pieces.push_back({(void **)&c->fids[l], sizeof(int32_t) * c->counts[l]});
        if (l < nm - 1) pieces.push_back({(void **)&c->fptr[l], sizeof(int32_t) * (c->counts[l] + 1)});
    }
    pieces.push_back({(void **)&c->vals, sizeof(float) * n});
    if (want_leafw) {
        pieces.push_back({(void **)&c->leafw, sizeof(int32_t) * n});
        pieces.push_back({(void **)&c->leaf_perm, sizeof(int32_t) * dims[order[nm - 1]]});
        pieces.push_back({(void **)&c->leaf_rank, sizeof(int32_t) * dims[order[nm - 1]]});
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
    for (int l = nm - 2; l >= 0 && st == CPD_OK; --l) {
        const int32_t *next = (l == nm - 2) ? nullptr : scans[l + 1].p;
        hipLaunchKernelGGL(k_compact, dim3(grid1(n)), dim3(256), 0, s, klo, khi, kl, udl, n, l,
                           scans[l].p, next, c->fids[l], c->fptr[l]);
        if (hipGetLastError() != hipSuccess) st = CPD_EHIP;
        hipLaunchKernelGGL(k_set_last_const, dim3(1), dim3(1), 0, s, c->fptr[l], c->counts[l],
                           (int32_t)c->counts[l + 1]);
    }
    hipLaunchKernelGGL(k_leaf, dim3(grid1(n)), dim3(256), 0, s, klo, khi, kl, n, c->fids[nm - 1]);
    if (st == CPD_OK && hipGetLastError() != hipSuccess) st = CPD_EHIP;
    if (c->leafw && st == CPD_OK) {
        // rank the leaf ids by frequency in a strided sample of the leaves
        const int64_t nid = dims[order[nm - 1]];
        cpd_status rs = rank_ids(c->fids[nm - 1], n, nid, c->leaf_perm, c->leaf_rank, d_flag.p + 1, s);
        if (rs == CPD_OK) {
            hipLaunchKernelGGL(k_leafw, dim3(grid1(n)), dim3(256), 0, s, udl,
                               (const int32_t *)c->fids[nm - 1], (const int32_t *)c->leaf_rank, n, c->leafw);
            if (hipGetLastError() != hipSuccess) rs = CPD_EHIP;
        }
        if (rs != CPD_OK) st = rs;
        for (int l = 1; l < nm - 1; ++l) {
            hipLaunchKernelGGL(k_uprow, dim3(grid1(n)), dim3(256), 0, s, klo, khi, kl, n, l, c->uprow[l]);
            if (st == CPD_OK && hipGetLastError() != hipSuccess) st = CPD_EHIP;
        }
    }
    if (st == CPD_OK && hipMemcpyAsync(c->vals, uval, sizeof(float) * n, hipMemcpyDeviceToDevice, s) != hipSuccess)
        st = CPD_EHIP;
    if (st == CPD_OK && hipStreamSynchronize(s) != hipSuccess) st = CPD_EHIP;
    if (st != CPD_OK) {
        free_csf(c);
        CPD_FAIL(st, "CSF compression kernels failed");
    }
    *out = c;
    return CPD_OK;
}

}  // namespace

cpd_status rank_ids(const int32_t *ids, int64_t n, int64_t nid, int32_t *perm, int32_t *rank, int32_t *nruns,
                    hipStream_t s) {
    const int64_t stride = std::max<int64_t>(1, n / (1 << 22));
    const int64_t ns = ceil_div(n, stride);
    int ibits = 0;
    while ((1ll << ibits) < nid) ++ibits;
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
    hipLaunchKernelGGL(k_sample, dim3(grid1(ns)), dim3(256), 0, s, ids, stride, ns, a, ap);
    CPD_LAUNCH_CHECK();
    CPD_TRY(radix_sort(a, ah, ap, b, bh, bp, ns, std::max(ibits, 1), s));
    CPD_TRY(exclusive_scan(RunStart{a}, ns, spos.p, nruns, s));
    hipLaunchKernelGGL(k_run_starts, dim3(grid1(ns)), dim3(256), 0, s, (const uint64_t *)a, (const int32_t *)spos.p,
                       ns, sstart.p);
    hipLaunchKernelGGL(k_run_counts, dim3(grid1(ns)), dim3(256), 0, s, (const uint64_t *)a,
                       (const int32_t *)sstart.p, (const int32_t *)nruns, ns, cnt.p);
    hipLaunchKernelGGL(k_rank_keys, dim3(grid1(nid)), dim3(256), 0, s, (const int32_t *)cnt.p, nid, a, ap);
    CPD_LAUNCH_CHECK();
    CPD_TRY(radix_sort(a, ah, ap, b, bh, bp, nid, 64, s));
    hipLaunchKernelGGL(k_rank_scatter, dim3(grid1(nid)), dim3(256), 0, s, (const uint64_t *)a, nid, perm, rank);
    CPD_LAUNCH_CHECK();
    return CPD_OK;
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
        if (hipMallocAsync((void **)&pp, sizeof(int32_t) * nid, s) != hipSuccess ||
            hipMallocAsync((void **)&rr, sizeof(int32_t) * nid, s) != hipSuccess) {
            (void)hipGetLastError();
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
    if (hipMallocAsync((void **)&p, sizeof(int32_t) * (size_t)std::max<int64_t>(1, (nm - 1) * nt), s) != hipSuccess) {
        (void)hipGetLastError();
        CPD_FAIL(CPD_ENOMEM, "device allocation for the tile table failed");
    }
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
