"""CSF reference (oracle; test infrastructure only).

Compressed sparse fiber storage (Section III): one tree per tensor whose
levels follow a mode order pi; level l holds one node per distinct prefix
(i_pi0, ..., i_pil) of the sorted nonzeros.  The paper defers the layout to
the original CSF publication, so the layout below is this project's reading
(R9): for every level l < N-1, ``fids[l]`` (int32, n_l entries) is the index
i_pil of each node and ``fptr[l]`` (int32, n_l + 1 entries) the position of the
node's first child at level l+1, with fptr[l][n_l] = n_{l+1}; the leaf level
stores ``fids[N-1]`` (one per nonzero) and the values.  Root ids are always
stored, empty slices are not nodes, indices are 0-based.

Duplicates (R8): equal coordinates become one nonzero whose value is the
float32 sum of the duplicates in input order, added one after another.

Steps: (1) stable lexicographic sort of the index tuples in pi order
(numpy.lexsort; or, when the tuple fits 62 bits, a stable library sort of
the tuple written as one integer, i_pi0 most significant, which is the same
order); (2) duplicate merge; (3) one run scan per level.

Pinned by: brute-force tree construction from Python tuples on tiny inputs;
expanding the CSF reproduces the sorted, merged COO exactly; fptr strictly
increasing and ending at the next level's count.
"""
from __future__ import annotations

import numpy as np


def heuristic_order(dims) -> list:
    """Modes by ascending length, ties to the lower mode index (R10)."""
    return sorted(range(len(dims)), key=lambda m: (int(dims[m]), m))


def sort_perm(dims, inds, order, method="auto"):
    """Stable permutation sorting the nonzeros lexicographically by
    (i_pi0, i_pi1, ...).  "lexsort": numpy.lexsort on the index rows;
    "packed": the tuple as one integer sum_l i_pil * prod_{l' > l} dims[pi_l']
    (mixed radix, i_pi0 most significant, exact below 2^62), stably sorted by
    torch's CPU sort; "auto": packed when it fits."""
    nm = len(dims)
    span = 1
    for m in order:
        span *= int(dims[m])
    if method == "auto":
        method = "packed" if span < (1 << 62) else "lexsort"
    if method == "lexsort":
        keys = [inds[m] for m in order]                   # primary key first
        return np.lexsort(keys[::-1])                     # lexsort: last key is primary
    if span >= (1 << 62):
        raise ValueError("index tuples do not fit 62 bits")
    import torch
    key = np.zeros(inds.shape[1], dtype=np.int64)
    for m in order:
        key = key * int(dims[m]) + inds[m]
    _, perm = torch.sort(torch.from_numpy(key), stable=True)
    return perm.numpy()


def build(dims, inds, vals, order, method="auto"):
    """Return dict(order, counts, fids, fptr, vals) for the mode order `order`
    (method: the sort of step 1, see sort_perm)."""
    dims = [int(d) for d in dims]
    inds = np.asarray(inds, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float32)
    nm = len(dims)
    order = [int(m) for m in order]
    if sorted(order) != list(range(nm)):
        raise ValueError("order must be a permutation of the modes")
    perm = sort_perm(dims, inds, order, method)
    srt = inds[order][:, perm]                            # rows in pi order
    v = vals[perm]
    nnz = srt.shape[1]
    # duplicate merge: a new nonzero starts where any index differs
    if nnz:
        new = np.ones(nnz, dtype=bool)
        new[1:] = (srt[:, 1:] != srt[:, :-1]).any(axis=0)
    else:
        new = np.zeros(0, dtype=bool)
    starts = np.flatnonzero(new)
    merged = v[starts].copy()
    ends = np.append(starts[1:], nnz)
    for j in np.flatnonzero(ends - starts > 1):           # runs of duplicates only
        acc = np.float32(v[starts[j]])
        for k in range(starts[j] + 1, ends[j]):
            acc = np.float32(acc + v[k])
        merged[j] = acc
    srt = srt[:, starts]
    n = srt.shape[1]
    fids, fptr, counts = [], [], []
    node_of = []                                          # per level: node id of every leaf
    for l in range(nm - 1):
        flag = np.ones(n, dtype=bool)
        if n:
            flag[1:] = (srt[: l + 1, 1:] != srt[: l + 1, :-1]).any(axis=0)
        node_of.append(np.cumsum(flag) - 1)
        fids.append(srt[l][flag].astype(np.int32))
        counts.append(int(flag.sum()))
    fids.append(srt[nm - 1].astype(np.int32))
    counts.append(n)
    node_of.append(np.arange(n))
    for l in range(nm - 1):
        first = np.flatnonzero(np.r_[True, np.diff(node_of[l]) != 0]) if n else np.zeros(0, int)
        p = np.empty(counts[l] + 1, dtype=np.int64)
        p[:-1] = node_of[l + 1][first]
        p[-1] = counts[l + 1]
        fptr.append(p.astype(np.int32))
    return dict(order=order, counts=counts, fids=fids, fptr=fptr, vals=merged)


def expand(csf):
    """Inverse of the compression: the sorted, merged COO (rows in pi order)."""
    nm = len(csf["order"])
    n = csf["counts"][-1]
    rows = [None] * nm
    rows[nm - 1] = csf["fids"][nm - 1].astype(np.int64)
    # owner[l][k]: node at level l that owns leaf k
    owner = np.arange(n)
    for l in range(nm - 2, -1, -1):
        # node j at level l owns children fptr[l][j] .. fptr[l][j+1]-1 at level l+1
        child_owner = np.repeat(np.arange(csf["counts"][l]), np.diff(csf["fptr"][l]))
        owner = child_owner[owner]
        rows[l] = csf["fids"][l].astype(np.int64)[owner]
    return np.stack(rows) if n else np.zeros((nm, 0), np.int64), csf["vals"]


def tile_starts(csf, tile_nnz: int):
    """For tiles of tile_nnz leaves, the node holding each tile's first leaf at
    every level l < N-1: array (N-1, ntiles) int32."""
    nm = len(csf["order"])
    n = csf["counts"][-1]
    ntiles = (n + tile_nnz - 1) // tile_nnz
    out = np.zeros((nm - 1, ntiles), dtype=np.int32)
    pos = np.arange(ntiles, dtype=np.int64) * tile_nnz
    for l in range(nm - 2, -1, -1):
        pos = np.searchsorted(csf["fptr"][l], pos, side="right") - 1
        out[l] = pos
    return out
