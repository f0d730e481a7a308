// Internal view of a CSF tree (shared by the CSF builder, the MTTKRP kernels
// and the ALS driver).
#pragma once

#include <mutex>
#include <vector>

#include "common.h"

struct cpd_csf_s {
    int nmodes = 0;
    int64_t dims[CPD_MAX_MODES] = {};     // by mode
    int order[CPD_MAX_MODES] = {};        // level -> mode
    int64_t counts[CPD_MAX_MODES] = {};   // nodes per level (counts[N-1] = nnz)
    char *slab = nullptr;                 // one allocation holding the arrays below
    size_t slab_bytes = 0;
    int32_t *fids[CPD_MAX_MODES] = {};    // per level
    int32_t *fptr[CPD_MAX_MODES] = {};    // per level < N-1
    float *vals = nullptr;
    // Leaf words for the MTTKRP kernels: leafw[k] = (lvl << 29) | rank of
    // fids[N-1][k], lvl = the highest level at which leaf k starts a new node
    // (0 = a new root node, N-1 = same fiber as leaf k-1), rank = position of
    // the leaf index when the indices are ordered by how often they occur
    // (leaf_perm[rank] = index).  Null when a leaf index does not fit in 29 bits.
    int32_t *leafw = nullptr;
    int32_t *leaf_perm = nullptr;
    int32_t *leaf_rank = nullptr;         // index -> rank (inverse of leaf_perm)
    // The same ranking for internal levels (index frequency among the level's
    // nodes), built on first use by csf_level_rank.
    int32_t *lvl_perm[CPD_MAX_MODES] = {};
    int32_t *lvl_rank[CPD_MAX_MODES] = {};
    // Per-leaf row ids of the internal levels 1..N-2 (uprow[l][k] = the index
    // i_order[l] of leaf k), so a kernel can gather every leaf's internal rows
    // without walking fiber pointers.  Allocated with leafw.
    int32_t *uprow[CPD_MAX_MODES] = {};

    struct Tiles {
        int32_t tile;
        int64_t ntiles;
        int32_t *starts;                  // (N-1) x ntiles
    };
    std::vector<Tiles> tiles;
    // The leaves regrouped by tiles of B consecutive indices of one level d
    // (1 <= d <= N-1): the mode tiling of that level's MTTKRP (one tile's
    // output rows fit in LDS).  Inside a tile the leaves keep tree order
    // (TILE_TREE), or are sorted by their other levels' indices, the level
    // of the largest dimension first (TILE_BY_SIZE: the rows of the largest
    // factor repeat in runs).  Built on first use for a level, tile height
    // and order, cached.
    enum { TILE_TREE = 0, TILE_BY_SIZE = 1 };
    struct LeafTiling {
        int32_t depth = 0;
        int32_t B = 0;
        int32_t order = TILE_TREE;
        int64_t ntiles = 0;
        int32_t *toff = nullptr;                 // ntiles + 1 offsets into the regrouped leaves
        // one record of rw words per regrouped leaf (rw = 4 for 2..3 modes, 8
        // for 4..5): its value's bits, its level-d index minus the tile's
        // first index, its indices at the other levels in level order, padding
        int32_t *rec = nullptr;
        int32_t rw = 0;
        char *slab = nullptr;
        size_t bytes = 0;
    };
    std::vector<LeafTiling> leaf_tilings;
    std::mutex mu;

    int depth_of(int mode) const {
        for (int l = 0; l < nmodes; ++l)
            if (order[l] == mode) return l;
        return -1;
    }
};

namespace cpd {

// Device-wide exclusive scan of f(i) for i in [0, n) into out (int32), with the
// total written to *total (device).  f is a device functor returning int32.
template <typename F>
cpd_status exclusive_scan(F f, int64_t n, int32_t *out, int32_t *total, hipStream_t s);

// Stable LSD radix sort (see csf.hip) on key bits [lo_bit, bits); buffers
// ping-pong, k*/kp end on the result.
cpd_status radix_sort(uint64_t *&klo, uint64_t *&khi, int32_t *&kp, uint64_t *&olo, uint64_t *&ohi, int32_t *&op,
                      int64_t n, int bits, hipStream_t s, int lo_bit = 0);

// Index frequencies in a strided sample of at most max_samples of the n ids
// (values in [0, nid)): out (device, 3 int32) = distinct ids in the sample,
// largest count, sample size.
cpd_status sample_freq(const int32_t *ids, int64_t n, int64_t nid, int64_t max_samples, int32_t *out,
                       hipStream_t s);

// Frequency ranking of the values ids[0..n) (in [0, nid)) by a strided sample
// of at most 2^22 of them: perm[r] = the index of rank r (descending count,
// ties to the lower index; unsampled indices last), rank[i] its inverse.
// nruns: device scratch for one int32.
cpd_status rank_ids(const int32_t *ids, int64_t n, int64_t nid, int32_t *perm, int32_t *rank, int32_t *nruns,
                    hipStream_t s);

// The same ranking of the index field [shift, shift + bits) of n sorted
// keys (one or two words; hi may be null).
cpd_status rank_key_field(const uint64_t *lo, const uint64_t *hi, int shift, int bits, int64_t n, int64_t nid,
                          int32_t *perm, int32_t *rank, int32_t *nruns, hipStream_t s);

// Ranking of the indices of level l (1 <= l < N) of a tree: the leaf ranking
// for l = N-1, else built on first use and cached in the handle.  Null
// outputs when the tree has no ranking (leaf index above 2^29).
cpd_status csf_level_rank(cpd_csf_s *c, int l, const int32_t **perm, const int32_t **rank, hipStream_t s);

// Device memory that temporaries are carved from (the allocation-free
// MTTKRP entry point): 256-byte aligned bump allocation, null when full.
struct Workspace {
    char *base = nullptr;
    size_t bytes = 0, used = 0;
    void *take(size_t n) {
        const size_t at = (used + 255) & ~size_t(255);
        if (!base || at > bytes || n > bytes - at) return nullptr;
        used = at + n;
        return base + at;
    }
};

// MTTKRP (cpd_mttkrp) with every temporary taken from ws (null: the scratch
// cache of stream s, tables cached in the handle).
cpd_status mttkrp_ws(cpd_csf_s *c, const void *const *factors, int32_t ld, int32_t R, int32_t mode, float *Y,
                     int32_t ldo, const cpd_mttkrp_opts *opts, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1,
                     Workspace *ws);

// Free a tree whose every use was ordered on stream s (no device-wide wait):
// its arrays go back to the stream-ordered pool on s.
void free_csf_on(cpd_csf_s *c, hipStream_t s);

// The ranking of level l if it exists already (no allocation; null otherwise).
void csf_level_rank_cached(cpd_csf_s *c, int l, const int32_t **perm, const int32_t **rank);

// Tile table without allocating: the cached one, else computed into dst
// (dst_bytes of device memory; CPD_EUNSUPPORTED when it does not fit).
cpd_status csf_tiles_into(cpd_csf_s *c, int32_t tile, int32_t *dst, size_t dst_bytes, const int32_t **starts,
                          int64_t *ntiles, hipStream_t s);

// Tile start nodes for a tile width (cached in the handle; created on first use).
cpd_status csf_tiles(cpd_csf_s *c, int32_t tile, const int32_t **starts, int64_t *ntiles,
                     hipStream_t s);

// The mode tiling of level d (1..N-1) of a tree for tile height B and the
// order inside a tile (TILE_TREE or TILE_BY_SIZE; cached in the handle;
// built on first use; needs the tree's leaf words and per-leaf internal ids);
// *out receives a copy of its descriptor.  `cached_only`: the cached one or
// an empty descriptor (B == 0), building nothing.
cpd_status csf_level_tiling(cpd_csf_s *c, int d, int32_t B, int order, bool cached_only,
                            cpd_csf_s::LeafTiling *out, hipStream_t s);

}  // namespace cpd
