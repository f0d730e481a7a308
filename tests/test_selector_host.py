"""Host-side logic of the variant selector (no GPU needed): the Zipf exponent
inversion, candidate enumeration, network inputs and the fallback rule of
Section V-D2 (privatise iff output rows x copies <= 0.02 x nnz)."""
import numpy as np
import pytest

from paper_1812_05961_amd import cpd


def _zipf_top(alpha, n):
    """Largest probability of Zipf(alpha) over n items, by direct summation."""
    k = np.arange(1, n + 1, dtype=np.float64)
    return 1.0 / np.sum(k ** -alpha)


@pytest.mark.parametrize("n", [7, 1000, 30_000, 1_000_000])
@pytest.mark.parametrize("alpha", [0.15, 0.7, 1.0, 1.3, 2.5])
def test_zipf_alpha_inverts_the_top_probability(n, alpha):
    got = cpd.zipf_alpha(_zipf_top(alpha, n), n)
    assert abs(got - alpha) < 1e-4, (n, alpha, got)


def test_zipf_alpha_edges():
    assert cpd.zipf_alpha(1.0 / 500, 500) == 0.0        # uniform
    assert cpd.zipf_alpha(0.0001, 500) == 0.0           # below uniform
    assert cpd.zipf_alpha(0.5, 1) == 0.0                # one item
    assert cpd.zipf_alpha(1.0, 100) == 8.0              # everything on one index
    assert cpd.zipf_alpha(_zipf_top(9.0, 100), 100) == 8.0   # capped


def _stats(dims, nnz, top1=None, distinct=None):
    nm = len(dims)
    top1 = top1 or [1.0 / d for d in dims]
    distinct = distinct or [1.0] * nm
    return cpd.make_stats(dims, nnz, top1, distinct)


def _orders(cands):
    seen = []
    for c in cands:
        o = tuple(c.as_dict(5)["order"])
        if o not in seen:
            seen.append(o)
    return seen


def test_candidates_three_modes():
    st = _stats((100, 2000, 50_000), 1_000_000)
    c1 = [c.as_dict(3) for c in cpd.select_candidates(st, 16, 1)]
    # asc (0,1,2) depth 1; first (1,0,2) root; last (0,2,1) leaf; desc (2,1,0) depth 1;
    # rooted (1,2,0) root (the CP-ALS tree of mode 1)
    kinds = [(c["order_kind"], tuple(c["order"]), c["depth"]) for c in c1]
    assert sorted(set(kinds)) == sorted({("asc", (0, 1, 2), 1), ("first", (1, 0, 2), 0),
                                         ("last", (0, 2, 1), 2), ("desc", (2, 1, 0), 1),
                                         ("rooted", (1, 2, 0), 0)})
    # 2000 x 16 x 4 B > 64 KiB: no privatised LANE
    assert len(c1) == 3 + 3 + 5 + 4 + 4
    for c in c1:
        if c["depth"] == 0:
            assert c["kernel"] == "row" and c["variant"] == "auto" and c["tile_nnz"] in (32, 128, 512)
        elif c["depth"] == 1:
            assert (c["kernel"], c["variant"], c["tile_nnz"]) in {("row", "atomic", 256), ("row", "private", 256),
                                                                  ("tiled", "atomic", 0), ("lane", "atomic", 256)}
        else:
            assert (c["kernel"], c["variant"]) in {("tiled", "atomic"), ("round", "atomic"), ("lane", "atomic")}
            assert c["tile_nnz"] in {"round": (64, 256, 1024), "tiled": (0,), "lane": (256,)}[c["kernel"]]
    # mode 0 is the shortest: "first" equals "asc" and is listed once; 100 x 16 x 4 B fits LDS
    c0 = [c.as_dict(3) for c in cpd.select_candidates(st, 16, 0)]
    assert len(_orders(cpd.select_candidates(st, 16, 0))) == 4
    assert len(c0) == 3 + 6 + 6 + 3
    assert sum(c["variant"] == "private" for c in c0) == 2
    # the CP-ALS layout of every mode (the mode, then the rest by descending
    # length) is a candidate order, at the root with the default tile among others
    dims = (100, 2000, 50_000)
    for mode in range(3):
        want = [mode] + sorted((m for m in range(3) if m != mode), key=lambda m: -dims[m])
        rooted = [c.as_dict(3) for c in cpd.select_candidates(st, 16, mode) if c.as_dict(3)["order"] == want]
        assert rooted and all(c["depth"] == 0 for c in rooted)
        assert {c["tile_nnz"] for c in rooted} == {32, 128, 512}


def test_candidates_ties_and_five_modes():
    st = _stats((500, 500, 500, 20, 20), 10_000_000)
    cands = cpd.select_candidates(st, 64, 2)
    orders = _orders(cands)
    # ascending with ties to the lower mode: (3, 4, 0, 1, 2); descending: (0, 1, 2, 3, 4)
    assert (3, 4, 0, 1, 2) in orders and (0, 1, 2, 3, 4) in orders
    assert (2, 3, 4, 0, 1) in orders          # first
    assert (2, 0, 1, 3, 4) in orders          # rooted: the mode, then descending lengths
    assert len(orders) == 4                   # last == asc here
    assert len(cands) <= cpd.SEL_MAX_CAND
    for c in cands:
        d = c.as_dict(5)
        assert d["order"][d["depth"]] == 2
        assert sorted(d["order"]) == [0, 1, 2, 3, 4]


def test_features_layout():
    st = _stats((100, 2000, 50_000), 1_000_000, top1=[0.3, 0.01, 0.001], distinct=[1.0, 0.5, 0.2])
    cands = cpd.select_candidates(st, 16, 1)
    F = cpd.select_features(st, 16, 1, cands)
    assert F.shape == (len(cands), cpd.SEL_NFEAT) and np.isfinite(F).all()
    for c, f in zip(cands, F):
        d = c.as_dict(3)
        assert f[34 + cpd.ORDER_KINDS.index(d["order_kind"])] == 1.0
        assert f[34:39].sum() == 1.0
        assert f[29] == (d["depth"] == 0) and f[30] == (d["depth"] == 2)
        assert f[31] == (d["variant"] == "private") and f[32] == (d["kernel"] == "row")
        assert f[41] == (d["kernel"] == "round") and f[42] == (d["kernel"] == "tiled")
        assert abs(f[33] - (np.log2(d["tile_nnz"]) / 10 if d["tile_nnz"] else 0.0)) < 1e-6
        # per-level statistics follow the tree order
        for l, m in enumerate(d["order"]):
            assert f[18 + l] == np.float32(st.top1[m])
            assert f[23 + l] == np.float32(st.distinct[m])
        assert (f[11:13] == 0).all() and (f[16:18] == 0).all()   # levels beyond 3 modes
    assert abs(F[0, 5] - 0.01) < 1e-7 and abs(F[0, 1] - 0.75) < 1e-6


def test_heuristic_rule():
    # mode 0 (50 rows) sits at the root of the ascending tree: the ROW kernel
    st = _stats((50, 3000, 40_000), 2_000_000)
    h = cpd.select_heuristic(st, 16, 0).as_dict(3)
    assert h["order_kind"] == "asc" and h["depth"] == 0 and h["kernel"] == "row" and h["tile_nnz"] == 128
    # mode 1 at depth 1: 3000 x 16 x 4 B > 64 KiB -> atomics with ROW
    h = cpd.select_heuristic(st, 16, 1).as_dict(3)
    assert h["depth"] == 1 and h["variant"] == "atomic" and h["kernel"] == "row" and h["tile_nnz"] == 256
    # mode 2 at the leaf: atomics with TILED (its default tile height)
    h = cpd.select_heuristic(st, 16, 2).as_dict(3)
    assert h["depth"] == 2 and h["variant"] == "atomic" and h["kernel"] == "tiled" and h["tile_nnz"] == 0
    # 900 rows x 8 x 4 B fits LDS; 900 x 1024 <= 0.02 x 50M -> privatised LANE
    st = _stats((20, 900, 40_000), 50_000_000)
    h = cpd.select_heuristic(st, 8, 1).as_dict(3)
    assert h["variant"] == "private" and h["kernel"] == "lane"
    # the same with too few nonzeros for the rule -> atomic
    st = _stats((20, 900, 40_000), 40_000_000)
    assert cpd.select_heuristic(st, 8, 1).as_dict(3)["variant"] == "atomic"
    # the heuristic is always one of the candidates
    for stt, R in ((st, 8), (_stats((50, 3000, 40_000), 2_000_000), 16), (_stats((900, 20, 40, 30), 3_000_000), 64)):
        for mode in range(len(stt.dims[:stt.nmodes])):
            h = cpd.select_heuristic(stt, R, mode).as_dict(stt.nmodes)
            assert h in [c.as_dict(stt.nmodes) for c in cpd.select_candidates(stt, R, mode)]



def test_select_without_network_is_the_heuristic():
    st = _stats((50, 3000, 40_000), 2_000_000)
    ch, pred = cpd.select(st, 16, 2, params=None)
    assert pred == []
    assert ch.as_dict(3) == cpd.select_heuristic(st, 16, 2).as_dict(3)


def test_selector_rejects_bad_requests():
    with pytest.raises(cpd.CpdError) as e:
        cpd.select_candidates(_stats((10, 20), 100), 8, 0)
    assert e.value.status == cpd.CPD_EUNSUPPORTED
    st = _stats((10, 20, 30), 100)
    for rank, mode in ((0, 0), (65, 0), (8, 3), (8, -1)):
        with pytest.raises(cpd.CpdError) as e:
            cpd.select_candidates(st, rank, mode)
        assert e.value.status == cpd.CPD_EINVAL


def test_committed_network_matches_the_library_shape():
    import json
    import os

    from paper_1812_05961_amd import selector_train as st
    with open(st.PARAMS_PATH) as f:
        d = json.load(f)
    assert d["n_in"] == cpd.SEL_NFEAT and 1 <= d["hidden"] <= 64
    p = np.asarray(d["params"], dtype=np.float64)
    assert p.size == cpd.mlp_param_count(d["n_in"], d["hidden"]) and np.isfinite(p).all()
    # trained on the first 1600 corpus tensors, evaluated on the other 400
    rep = d["report"]
    assert rep["train_tensors"] >= 1500 and rep["heldout_tensors"] >= 350


def test_committed_corpus_is_consistent():
    import glob
    import gzip
    import json
    import os

    from paper_1812_05961_amd import selector_train as st
    files = sorted(glob.glob(os.path.join(os.path.dirname(st.PARAMS_PATH), "selector_corpus", "*.jsonl.gz")))
    assert files
    with gzip.open(files[0], "rt") as f:
        recs = [json.loads(next(f)) for _ in range(20)]
    for r in recs:
        s = r["stats"]
        stt = cpd.make_stats(s["dims"], s["nnz"], s["top1"], s["distinct"], s["alpha"], s["sample"])
        # the candidates recorded are the ones the library enumerates today
        now = [c.as_dict(s["nmodes"]) for c in cpd.select_candidates(stt, r["rank"], r["mode"])]
        assert now == r["cands"]
        assert now[r["heur"]] == cpd.select_heuristic(stt, r["rank"], r["mode"]).as_dict(s["nmodes"])
        assert len(r["ms"]) == len(now) and min(r["ms"]) > 0
