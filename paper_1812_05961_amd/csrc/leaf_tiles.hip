// Leaf-mode tiling of a CSF tree: the leaves regrouped by tiles of B
// consecutive leaf indices, tree order kept inside each tile, so that a
// leaf-level MTTKRP can keep one tile's B output rows in LDS and add every
// nonzero there (SPLATT's mode tiling, which the paper's port leaves out and
// names as further work, Sections V-A and VII).
//
// Per regrouped leaf j (leaf k of the tree): its value, its leaf index minus
// the tile's first index, and the indices at levels 0..N-2 of its fiber (the
// level N-2 node above it, whose rows form the Hadamard product the leaf is
// scaled by).  The fiber's indices are stored per leaf, not per fiber, so
// that the MTTKRP reads them in coalesced runs: looked up per fiber they are
// a random access into arrays of the tree's fiber count, one cache line per
// fiber run of a tile, which misses the L2.  Built with the CSF builder's
// radix sort (key: the tile number, payload: the position) and device-wide
// scans over the leaf words.
#include <algorithm>

#include "csf.h"
#include "scan.h"

namespace cpd {
namespace {

__global__ void k_tile_keys(const int32_t *__restrict__ leaf_ids, int64_t n, int32_t B, uint64_t *__restrict__ key,
                            int32_t *__restrict__ pos) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    key[i] = (uint64_t)(leaf_ids[i] / B);
    pos[i] = (int32_t)i;
}

// toff[t] = the first regrouped position whose tile is >= t, t = 0..ntiles
__global__ void k_tile_offsets(const uint64_t *__restrict__ key, int64_t n, int64_t ntiles, int32_t *__restrict__ toff) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > ntiles) return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (key[mid] < (uint64_t)t) lo = mid + 1;
        else hi = mid;
    }
    toff[t] = (int32_t)lo;
}

// leaf k opens a node at level <= lvl (its leaf word's level field)
struct OpensAt {
    const int32_t *leafw;
    uint32_t lvl;
    __device__ int32_t operator()(int64_t k) const { return ((uint32_t)leafw[k] >> 29) <= lvl ? 1 : 0; }
};

// fiber f (a level N-2 node) opens a root node: its first leaf's level is 0
struct FiberOpensRoot {
    const int32_t *first_leaf;  // fptr[N-2]
    const int32_t *leafw;
    __device__ int32_t operator()(int64_t f) const { return ((uint32_t)leafw[first_leaf[f]] >> 29) == 0 ? 1 : 0; }
};

struct LeafOut {
    float *tv;
    int32_t *tw;
    int32_t *th[CPD_MAX_MODES];
    const int32_t *fh[CPD_MAX_MODES];  // per fiber: its index at levels 0..N-2
};

__global__ void k_tile_gather(const int32_t *__restrict__ pos, const uint64_t *__restrict__ key, int64_t n, int32_t B,
                              const float *__restrict__ vals, const int32_t *__restrict__ leaf_ids,
                              const int32_t *__restrict__ leafw, uint32_t flvl, const int32_t *__restrict__ fexcl,
                              int nl, LeafOut o) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int32_t k = pos[j];
    o.tv[j] = vals[k];
    o.tw[j] = leaf_ids[k] - (int32_t)key[j] * B;
    const int32_t f = fexcl[k] + (((uint32_t)leafw[k] >> 29) <= flvl ? 1 : 0) - 1;
    for (int l = 0; l < nl; ++l) o.th[l][j] = o.fh[l][f];
}

struct FiberIds {
    const int32_t *fids[CPD_MAX_MODES];
    const int32_t *uprow[CPD_MAX_MODES];
    const int32_t *first_leaf;  // fptr[N-2]
    const int32_t *rexcl;       // exclusive scan of FiberOpensRoot
    const int32_t *leafw;
    int32_t *hid[CPD_MAX_MODES];
};

// hid[l][f]: index of fiber f's ancestor at level l (l = N-2: its own index)
__global__ void k_fiber_ids(FiberIds fi, int N, int64_t nf) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    fi.hid[N - 2][f] = fi.fids[N - 2][f];
    if (N >= 3) {
        const int32_t k = fi.first_leaf[f];
        for (int l = 1; l < N - 2; ++l) fi.hid[l][f] = fi.uprow[l][k];
        const int32_t root = fi.rexcl[f] + (((uint32_t)fi.leafw[k] >> 29) == 0 ? 1 : 0) - 1;
        fi.hid[0][f] = fi.fids[0][root];
    }
}

inline unsigned grid_of(int64_t n) { return (unsigned)ceil_div(std::max<int64_t>(n, 1), 256); }

}  // namespace

cpd_status csf_leaf_tiling(cpd_csf_s *c, int32_t B, bool cached_only, cpd_csf_s::LeafTiling *out, hipStream_t s) {
    *out = cpd_csf_s::LeafTiling{};
    if (B < 1) CPD_FAIL(CPD_EINVAL, "tile height %d < 1", B);
    std::lock_guard<std::mutex> g(c->mu);
    for (auto &t : c->leaf_tilings)
        if (t.B == B) {
            *out = t;
            return CPD_OK;
        }
    if (cached_only) return CPD_OK;
    if (!c->leafw) CPD_FAIL(CPD_EUNSUPPORTED, "the leaf-mode tiling needs the tree's leaf words");
    const int N = c->nmodes;
    if (N < 2 || N > 5) CPD_FAIL(CPD_EUNSUPPORTED, "the leaf-mode tiling is built for 2..5 modes, not %d", N);
    const int64_t n = c->counts[N - 1], nf = c->counts[N - 2];
    const int64_t I = c->dims[c->order[N - 1]];
    const int64_t nt = ceil_div(I, B);
    if (n < 1) CPD_FAIL(CPD_EINVAL, "empty tree");

    cpd_csf_s::LeafTiling lt;
    lt.B = B;
    lt.ntiles = nt;
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t b_toff = al(sizeof(int32_t) * (size_t)(nt + 1)), b_leaf = al(sizeof(int32_t) * (size_t)n);
    lt.bytes = b_toff + (size_t)(N + 1) * b_leaf;
    if (hipMallocAsync((void **)&lt.slab, lt.bytes, s) != hipSuccess) {
        (void)hipGetLastError();
        CPD_FAIL(CPD_ENOMEM, "device allocation of %zu bytes for the leaf-mode tiling failed", lt.bytes);
    }
    char *p = lt.slab;
    lt.toff = reinterpret_cast<int32_t *>(p);
    p += b_toff;
    lt.tv = reinterpret_cast<float *>(p);
    p += b_leaf;
    lt.tw = reinterpret_cast<int32_t *>(p);
    p += b_leaf;
    for (int l = 0; l < N - 1; ++l) {
        lt.th[l] = reinterpret_cast<int32_t *>(p);
        p += b_leaf;
    }
    auto fail = [&](cpd_status st) {
        (void)hipFreeAsync(lt.slab, s);
        (void)hipGetLastError();
        return st;
    };

    DevBuf<uint64_t> k1, k2;
    DevBuf<int32_t> p1, p2, fexcl, rexcl, fh;
    cpd_status st = CPD_OK;
    if ((st = k1.alloc(n, s)) || (st = k2.alloc(n, s)) || (st = p1.alloc(n, s)) || (st = p2.alloc(n, s)) ||
        (st = fexcl.alloc(n, s)) || (st = rexcl.alloc(std::max<int64_t>(nf, 1), s)) ||
        (st = fh.alloc((N - 1) * std::max<int64_t>(nf, 1), s)))
        return fail(st);
    const int32_t *leaf_ids = c->fids[N - 1];
    hipLaunchKernelGGL(k_tile_keys, dim3(grid_of(n)), dim3(256), 0, s, leaf_ids, n, B, k1.p, p1.p);
    if (hipGetLastError() != hipSuccess) return fail(CPD_EHIP);
    int bits = 1;
    while (bits < 63 && ((int64_t)1 << bits) < nt) ++bits;
    uint64_t *klo = k1.p, *khi = nullptr, *olo = k2.p, *ohi = nullptr;
    int32_t *kp = p1.p, *op = p2.p;
    if ((st = radix_sort(klo, khi, kp, olo, ohi, op, n, bits, s))) return fail(st);
    hipLaunchKernelGGL(k_tile_offsets, dim3(grid_of(nt + 1)), dim3(256), 0, s, (const uint64_t *)klo, n, nt, lt.toff);
    if (hipGetLastError() != hipSuccess) return fail(CPD_EHIP);
    FiberIds fi{};
    for (int l = 0; l < N; ++l) {
        fi.fids[l] = c->fids[l];
        fi.uprow[l] = c->uprow[l];
        fi.hid[l] = l < N - 1 ? fh.p + (int64_t)l * nf : nullptr;
    }
    fi.first_leaf = N >= 3 ? c->fptr[N - 2] : nullptr;
    fi.leafw = c->leafw;
    if (N >= 3) {
        for (int l = 1; l < N - 2; ++l)
            if (!c->uprow[l]) return fail(CPD_EUNSUPPORTED);
        if ((st = exclusive_scan(FiberOpensRoot{c->fptr[N - 2], c->leafw}, nf, rexcl.p, (int32_t *)nullptr, s)))
            return fail(st);
        fi.rexcl = rexcl.p;
    }
    hipLaunchKernelGGL(k_fiber_ids, dim3(grid_of(nf)), dim3(256), 0, s, fi, N, nf);
    if (hipGetLastError() != hipSuccess) return fail(CPD_EHIP);
    const uint32_t flvl = (uint32_t)(N - 2);
    if ((st = exclusive_scan(OpensAt{c->leafw, flvl}, n, fexcl.p, (int32_t *)nullptr, s))) return fail(st);
    LeafOut o{};
    o.tv = lt.tv;
    o.tw = lt.tw;
    for (int l = 0; l < N - 1; ++l) {
        o.th[l] = lt.th[l];
        o.fh[l] = fi.hid[l];
    }
    hipLaunchKernelGGL(k_tile_gather, dim3(grid_of(n)), dim3(256), 0, s, (const int32_t *)kp, (const uint64_t *)klo, n,
                       B, (const float *)c->vals, leaf_ids, (const int32_t *)c->leafw, flvl, (const int32_t *)fexcl.p,
                       N - 1, o);
    if (hipGetLastError() != hipSuccess) return fail(CPD_EHIP);
    c->leaf_tilings.push_back(lt);
    *out = lt;
    return CPD_OK;
}

}  // namespace cpd
