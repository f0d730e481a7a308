"""Pins of the oracle's leaf-frequency ranking and of the tree split by it
(oracle/csf.py: frequency_rank, build_split)."""
import collections

import numpy as np
import pytest

from oracle import csf as ocsf


def _brute_rank(ids, nid, stride):
    """Counts over every stride-th entry by a plain loop, then indices sorted
    by (-count, index)."""
    cnt = collections.Counter()
    for i in range(0, len(ids), stride):
        cnt[int(ids[i])] += 1
    return sorted(range(nid), key=lambda j: (-cnt[j], j))


@pytest.mark.parametrize("n,nid,max_samples", [(1000, 50, 1 << 22), (1000, 50, 100), (997, 13, 7), (5, 40, 1 << 22)])
def test_frequency_rank_matches_brute_force(n, nid, max_samples):
    rng = np.random.default_rng(n + nid)
    ids = np.minimum(rng.zipf(1.3, n) - 1, nid - 1)
    perm, rank = ocsf.frequency_rank(ids, nid, max_samples)
    stride = max(1, n // max_samples)
    assert list(perm) == _brute_rank(ids, nid, stride)
    assert (rank[perm] == np.arange(nid)).all()


def _tensor(seed, dims=(6, 7, 9), nnz=300, dups=40):
    rng = np.random.default_rng(seed)
    inds = np.stack([rng.integers(0, d, nnz) for d in dims])
    inds = np.concatenate([inds, inds[:, :dups]], axis=1)            # exact duplicates
    vals = rng.random(inds.shape[1]).astype(np.float32)
    return dims, inds, vals


def _same(a, b):
    for k in ("counts",):
        assert list(a[k]) == list(b[k])
    for l in range(len(a["fids"])):
        assert np.array_equal(a["fids"][l], b["fids"][l])
    for l in range(len(a["fptr"])):
        assert np.array_equal(a["fptr"][l], b["fptr"][l])
    assert np.array_equal(a["vals"], b["vals"])


@pytest.mark.parametrize("order", [[0, 1, 2], [2, 0, 1]])
def test_split_extremes_equal_the_plain_tree(order):
    dims, inds, vals = _tensor(1)
    plain = ocsf.build(dims, inds, vals, order)
    all_hot = ocsf.build_split(dims, inds, vals, order, dims[order[-1]])
    assert all_hot["nhot"] == plain["counts"][-1]
    _same(all_hot, plain)
    none_hot = ocsf.build_split(dims, inds, vals, order, 0)
    assert none_hot["nhot"] == 0
    _same(none_hot, plain)


@pytest.mark.parametrize("hot_rows", [1, 3, 5])
def test_split_tree_partitions_the_merged_nonzeros(hot_rows):
    dims, inds, vals = _tensor(2)
    order = [1, 2, 0]
    t = ocsf.build_split(dims, inds, vals, order, hot_rows)
    plain = ocsf.build(dims, inds, vals, order)
    n, nh = t["counts"][-1], t["nhot"]
    assert n == plain["counts"][-1] and 0 < nh < n
    # a valid tree: pointers increase and end at the next level's count
    for l in range(2):
        assert (np.diff(t["fptr"][l]) > 0).all() and t["fptr"][l][-1] == t["counts"][l + 1]
    rows, v = ocsf.expand(t)
    # the first part holds exactly the leaves whose index is among the hot ones
    _, rank = ocsf.frequency_rank(inds[order[-1]], dims[order[-1]])
    assert (rank[rows[2, :nh]] < hot_rows).all() and (rank[rows[2, nh:]] >= hot_rows).all()
    # each part is in lexicographic order
    for lo, hi in ((0, nh), (nh, n)):
        keys = [tuple(rows[:, k]) for k in range(lo, hi)]
        assert keys == sorted(keys)
    # the same merged nonzeros (coordinates and float32 sums) as the plain tree
    prow, pv = ocsf.expand(plain)
    got = {tuple(rows[:, k]): v[k] for k in range(n)}
    ref = {tuple(prow[:, k]): pv[k] for k in range(n)}
    assert got == ref
