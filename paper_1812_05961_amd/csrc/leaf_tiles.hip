// Mode tiling of a CSF tree for the MTTKRP of one level d >= 1: the leaves
// regrouped by tiles of B consecutive indices of level d, so that a kernel
// can keep one tile's B output rows in LDS and add every contribution there
// (SPLATT's mode tiling, which the paper's port leaves out and names as
// further work, Sections V-A and VII).  Inside a tile the leaves keep tree
// order (the leaves of each level-d node and of each fiber stay
// consecutive), or are sorted by their indices at the other levels, the
// level of the largest dimension the major key: consecutive leaves then share
// the row of the largest factor in runs, so a kernel gathering every leaf's
// rows finds it in the L1 (the other rows come from smaller factors, which
// stay in the L2).  The sort key holds the tile number and as many of those
// indices, in that order, as fit 64 bits; the order among leaves that agree on
// the key is the tree order (a stable sort).
//
// Per regrouped leaf j (leaf k of the tree) one record: its value, its
// level-d index minus the tile's first index, and its indices at the other
// levels in level order (at the leaf level: the fiber whose rows form the
// Hadamard product the leaf is scaled by; at an internal level: the node's
// ancestors, then the levels below d), padded to 4 or 8 words so that a lane
// reads its leaf's record with one or two 16-byte loads (a load instruction
// costs the vector-memory return path about the same whatever its width).
// The indices are stored per leaf, not looked up per fiber or node: that
// would be a random access into arrays of the tree's node counts, one cache
// line per run of a tile, which misses the L2.  Built with the CSF builder's radix sort (key:
// the tile number, payload: the position) and a device-wide scan over the
// leaf words (the root node of every leaf).
#include <algorithm>

#include "csf.h"
#include "scan.h"

namespace cpd {
namespace {

// Per-leaf index at every level: level 0 through the leaf's root node,
// levels 1..N-2 from the per-leaf internal ids, level N-1 the leaf index.
struct LevelIds {
    const int32_t *root_fids;            // fids[0]
    const int32_t *mid[CPD_MAX_MODES];   // uprow[1..N-2]
    const int32_t *leaf_ids;             // fids[N-1]
    const int32_t *leafw;
    const int32_t *rexcl;                // exclusive scan of "leaf opens a root node"
    int N;
    __device__ int32_t at(int l, int64_t k) const {
        if (l == N - 1) return leaf_ids[k];
        if (l > 0) return mid[l][k];
        return root_fids[rexcl[k] + (((uint32_t)leafw[k] >> 29) == 0 ? 1 : 0) - 1];
    }
};

// leaf k opens a root node (its leaf word's level field is 0)
struct OpensRoot {
    const int32_t *leafw;
    __device__ int32_t operator()(int64_t k) const { return ((uint32_t)leafw[k] >> 29) == 0 ? 1 : 0; }
};

// Sort-key fields below the tile number: level lvl[f] at bit shift[f];
// the tile number starts at bit `tshift`.
struct KeyFields {
    int nf;
    int lvl[CPD_MAX_MODES];
    int shift[CPD_MAX_MODES];
    int tshift;
};

__global__ void k_tile_keys(LevelIds li, int d, int64_t n, int32_t B, KeyFields kf, uint64_t *__restrict__ key,
                            int32_t *__restrict__ pos) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t k = (uint64_t)(li.at(d, i) / B) << kf.tshift;
    for (int f = 0; f < kf.nf; ++f) k |= (uint64_t)(uint32_t)li.at(kf.lvl[f], i) << kf.shift[f];
    key[i] = k;
    pos[i] = (int32_t)i;
}

// toff[t] = the first regrouped position whose tile is >= t, t = 0..ntiles
__global__ void k_tile_offsets(const uint64_t *__restrict__ key, int tshift, int64_t n, int64_t ntiles,
                               int32_t *__restrict__ toff) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > ntiles) return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((key[mid] >> tshift) < (uint64_t)t) lo = mid + 1;
        else hi = mid;
    }
    toff[t] = (int32_t)lo;
}

__global__ void k_tile_gather(const int32_t *__restrict__ pos, const uint64_t *__restrict__ key, int tshift, int64_t n,
                              int32_t B, const float *__restrict__ vals, LevelIds li, int d, int rw,
                              int32_t *__restrict__ rec) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int32_t k = pos[j];
    int32_t *r = rec + j * rw;
    r[0] = __float_as_int(vals[k]);
    r[1] = li.at(d, k) - (int32_t)(key[j] >> tshift) * B;
    int m = 2;
    for (int l = 0; l < li.N; ++l)
        if (l != d) r[m++] = li.at(l, k);
    for (; m < rw; ++m) r[m] = 0;
}

inline unsigned grid_of(int64_t n) { return (unsigned)ceil_div(std::max<int64_t>(n, 1), 256); }

}  // namespace

cpd_status csf_level_tiling(cpd_csf_s *c, int d, int32_t B, int order, bool cached_only,
                            cpd_csf_s::LeafTiling *out, hipStream_t s) {
    *out = cpd_csf_s::LeafTiling{};
    if (B < 1) CPD_FAIL(CPD_EINVAL, "tile height %d < 1", B);
    if (order != cpd_csf_s::TILE_TREE && order != cpd_csf_s::TILE_BY_SIZE)
        CPD_FAIL(CPD_EINVAL, "unknown order %d inside the tiles", order);
    const int N = c->nmodes;
    if (N < 2 || N > 5) CPD_FAIL(CPD_EUNSUPPORTED, "the mode tiling is built for 2..5 modes, not %d", N);
    if (d < 1 || d >= N) CPD_FAIL(CPD_EUNSUPPORTED, "the mode tiling serves levels 1..%d, not %d", N - 1, d);
    std::lock_guard<std::mutex> g(c->mu);
    for (auto &t : c->leaf_tilings)
        if (t.B == B && t.depth == d && t.order == order) {
            *out = t;
            return CPD_OK;
        }
    if (cached_only) return CPD_OK;
    if (!c->leafw) CPD_FAIL(CPD_EUNSUPPORTED, "the mode tiling needs the tree's leaf words");
    for (int l = 1; l < N - 1; ++l)
        if (!c->uprow[l]) CPD_FAIL(CPD_EUNSUPPORTED, "the mode tiling needs the per-leaf internal ids");
    const int64_t n = c->counts[N - 1];
    const int64_t I = c->dims[c->order[d]];
    const int64_t nt = ceil_div(I, B);
    if (n < 1) CPD_FAIL(CPD_EINVAL, "empty tree");

    cpd_csf_s::LeafTiling lt;
    lt.depth = d;
    lt.B = B;
    lt.order = order;
    lt.ntiles = nt;
    auto bits_of = [](int64_t v) {  // bits of the values 0..v-1
        int b = 1;
        while (b < 63 && ((int64_t)1 << b) < v) ++b;
        return b;
    };
    const int tbits = bits_of(nt);
    // the key's fields below the tile number: the other levels by decreasing
    // dimension (ties: upper level first), while they fit
    KeyFields kf{};
    if (order == cpd_csf_s::TILE_BY_SIZE) {
        int lv[CPD_MAX_MODES], nl = 0;
        for (int l = 0; l < N; ++l)
            if (l != d) lv[nl++] = l;
        std::stable_sort(lv, lv + nl, [&](int a, int b) { return c->dims[c->order[a]] > c->dims[c->order[b]]; });
        int used = 0;
        for (int f = 0; f < nl; ++f) {
            const int b = bits_of(c->dims[c->order[lv[f]]]);
            if (tbits + used + b > 64) break;
            kf.lvl[kf.nf++] = lv[f];
            used += b;
        }
        int at = used;
        for (int f = 0; f < kf.nf; ++f) {
            at -= bits_of(c->dims[c->order[kf.lvl[f]]]);
            kf.shift[f] = at;
        }
        kf.tshift = used;
    }
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    lt.rw = N <= 3 ? 4 : 8;  // value, local row, N-1 indices, padding
    const size_t b_toff = al(sizeof(int32_t) * (size_t)(nt + 1));
    lt.bytes = b_toff + al(sizeof(int32_t) * (size_t)lt.rw * (size_t)n);
    if (device_alloc((void **)&lt.slab, lt.bytes, s) != CPD_OK)
        CPD_FAIL(CPD_ENOMEM, "device allocation of %zu bytes for the mode tiling failed", lt.bytes);
    char *p = lt.slab;
    lt.toff = reinterpret_cast<int32_t *>(p);
    p += b_toff;
    lt.rec = reinterpret_cast<int32_t *>(p);
    auto fail = [&](cpd_status st) {
        (void)hipFreeAsync(lt.slab, s);
        (void)hipGetLastError();
        return st;
    };

    DevBuf<uint64_t> k1, k2;
    DevBuf<int32_t> p1, p2, rexcl;
    cpd_status st = CPD_OK;
    if ((st = k1.alloc(n, s)) || (st = k2.alloc(n, s)) || (st = p1.alloc(n, s)) || (st = p2.alloc(n, s)) ||
        (st = rexcl.alloc(n, s)))
        return fail(st);
    LevelIds li{};
    li.root_fids = c->fids[0];
    for (int l = 1; l < N - 1; ++l) li.mid[l] = c->uprow[l];
    li.leaf_ids = c->fids[N - 1];
    li.leafw = c->leafw;
    li.rexcl = rexcl.p;
    li.N = N;
    if ((st = exclusive_scan(OpensRoot{c->leafw}, n, rexcl.p, (int32_t *)nullptr, s))) return fail(st);
    hipLaunchKernelGGL(k_tile_keys, dim3(grid_of(n)), dim3(256), 0, s, li, d, n, B, kf, k1.p, p1.p);
    if (hipGetLastError() != hipSuccess) return fail(CPD_EHIP);
    uint64_t *klo = k1.p, *khi = nullptr, *olo = k2.p, *ohi = nullptr;
    int32_t *kp = p1.p, *op = p2.p;
    if ((st = radix_sort(klo, khi, kp, olo, ohi, op, n, kf.tshift + tbits, s))) return fail(st);
    hipLaunchKernelGGL(k_tile_offsets, dim3(grid_of(nt + 1)), dim3(256), 0, s, (const uint64_t *)klo, kf.tshift, n, nt,
                       lt.toff);
    if (hipGetLastError() != hipSuccess) return fail(CPD_EHIP);
    hipLaunchKernelGGL(k_tile_gather, dim3(grid_of(n)), dim3(256), 0, s, (const int32_t *)kp, (const uint64_t *)klo,
                       kf.tshift, n, B, (const float *)c->vals, li, d, (int)lt.rw, lt.rec);
    if (hipGetLastError() != hipSuccess) return fail(CPD_EHIP);
    c->leaf_tilings.push_back(lt);
    *out = lt;
    return CPD_OK;
}

}  // namespace cpd
