"""GPU parity: the HIP path through the C ABI against the CPU oracle, element by
element on the same seeded inputs.

Bars: CSF arrays and tile tables bit-exact; FP32 MTTKRP relative Frobenius
error <= 1e-5 and BF16-gather <= 1e-2 against the FP64 oracle on the same
factors; the dense FP64 steps to ~1e-10; CP-ALS final fit within 1e-4.
"""
import numpy as np
import pytest
import torch

from oracle import als as oals
from oracle import coo as ocoo
from oracle import csf as ocsf
from paper_1812_05961_amd import synth

pytestmark = pytest.mark.gpu


def _cpd():
    from paper_1812_05961_amd import cpd
    cpd.lib()
    return cpd


def _dev(t):
    return t.to("cuda")


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)


def _tensor(dims, nnz, alphas, seed, values="lognormal:1.0"):
    return synth.gen_sparse(dims, nnz, alphas, values, seed, device="cpu", topup=True, fp32=True)


def _with_dups(t, ndup, seed):
    """Append ndup repeats of existing coordinates (new values) in shuffled order."""
    g = torch.Generator().manual_seed(seed)
    pick = torch.randint(0, t.nnz, (ndup,), generator=g)
    inds = torch.cat([t.inds, t.inds[:, pick]], 1)
    vals = torch.cat([t.vals, torch.rand(ndup, generator=g, dtype=torch.float32)])
    perm = torch.randperm(inds.shape[1], generator=g)
    return synth.SparseTensor(t.dims, inds[:, perm].contiguous(), vals[perm].contiguous())


def _small3():
    t = synth.make_config("small3")
    return synth.SparseTensor(t.dims, t.inds, t.vals.to(torch.float32))


CASES = {
    "small3": _small3,
    "two2": lambda: _tensor((300, 500), 20_000, (0.8, 0.5), 41),
    "zipf3": lambda: _tensor((900, 700, 1300), 300_000, (1.1, 1.1, 1.1), 5),
    "zipf4": lambda: _tensor((500, 300, 200, 90), 250_000, (1.0, 1.0, 1.0, 1.0), 6),
    "zipf5": lambda: _tensor((60, 50, 40, 30, 20), 150_000, (0.5, 0.8, 0.0, 1.2, 0.3), 7),
    "dups3": lambda: _with_dups(_tensor((50, 40, 30), 5_000, (0.0, 0.0, 0.0), 8), 2_000, 9),
    "one_nnz": lambda: synth.SparseTensor((5, 6, 7), torch.tensor([[4], [0], [6]]),
                                          torch.tensor([2.5], dtype=torch.float32)),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    t = CASES[request.param]()
    return request.param, t


def _orders(nm):
    import itertools
    allp = list(itertools.permutations(range(nm)))
    rng = np.random.default_rng(nm)
    pick = [allp[i] for i in rng.choice(len(allp), size=min(3, len(allp)), replace=False)]
    return [None] + pick


# ----------------------------------------------------------------- CSF build

def test_csf_bit_exact(case):
    cpd = _cpd()
    name, t = case
    inds, vals = t.numpy()
    for order in _orders(t.nmodes):
        c = cpd.csf_build(_dev(t.inds), _dev(t.vals), t.dims, order)
        ref = ocsf.build(t.dims, inds, t.vals.numpy(), order or ocsf.heuristic_order(t.dims))
        assert c.order == ref["order"]
        assert c.counts == ref["counts"]
        for l in range(t.nmodes):
            fids, fptr, v = c.export(l)
            np.testing.assert_array_equal(fids.cpu().numpy(), ref["fids"][l])
            if l < t.nmodes - 1:
                np.testing.assert_array_equal(fptr.cpu().numpy(), ref["fptr"][l])
            else:
                assert v.cpu().numpy().tobytes() == ref["vals"].tobytes()
        for T in (1, 64, 256, 1000):
            np.testing.assert_array_equal(c.tiles(T).cpu().numpy(), ocsf.tile_starts(ref, T))
        c.free()


def _rooted_order(nm, mode, dims):
    rest = sorted((m for m in range(nm) if m != mode), key=lambda m: (-dims[m], m))
    return [mode] + rest


def _same_tree(c, ref, nm):
    assert c.order == ref["order"]
    assert c.counts == ref["counts"]
    for l in range(nm):
        fids, fptr, v = c.export(l)
        np.testing.assert_array_equal(fids.cpu().numpy(), ref["fids"][l])
        if l < nm - 1:
            np.testing.assert_array_equal(fptr.cpu().numpy(), ref["fptr"][l])
        else:
            assert v.cpu().numpy().tobytes() == ref["vals"].tobytes()


ROOTED_EXTRA = {
    # equal lengths: ties go to the lower mode
    "ties": lambda: _with_dups(_tensor((50, 40, 50, 40), 20_000, (0.8, 0.0, 0.8, 0.0), 31), 3_000, 32),
    # 4 x 14 + 10 = 66-bit keys: every tree is built on its own
    "wide5": lambda: _tensor((9000, 9000, 9000, 9000, 600), 30_000, (1.0, 1.0, 1.0, 1.0, 1.0), 33),
}


@pytest.mark.parametrize("name", list(CASES) + list(ROOTED_EXTRA))
def test_csf_build_rooted_bit_exact(name):
    """One tree per mode, derived from the longest mode's sorted nonzeros:
    each equals the oracle's tree for (mode, others by descending length)."""
    cpd = _cpd()
    t = (CASES.get(name) or ROOTED_EXTRA[name])()
    inds, vals = t.numpy()
    trees = cpd.csf_build_rooted(_dev(t.inds), _dev(t.vals), t.dims)
    assert len(trees) == t.nmodes
    for m, c in enumerate(trees):
        ref = ocsf.build(t.dims, inds, t.vals.numpy(), _rooted_order(t.nmodes, m, t.dims))
        _same_tree(c, ref, t.nmodes)
        c.free()


def test_csf_build_from_unaligned_views():
    """Index and value arrays that start 4 bytes into their allocations (the
    element-by-element key packing) give the same tree."""
    cpd = _cpd()
    t = CASES["dups3"]()
    inds = _dev(t.inds)
    vals = _dev(t.vals)
    pad_i = torch.zeros((t.nmodes, 1), dtype=inds.dtype, device="cuda")
    big_i = torch.cat([pad_i, inds], 1).to(torch.int32)
    big_v = torch.cat([torch.zeros(1, device="cuda"), vals])
    views = [big_i[m, 1:] for m in range(t.nmodes)]
    assert all(v.data_ptr() % 16 != 0 for v in views) and big_v[1:].data_ptr() % 16 != 0
    c = cpd.csf_build(views, big_v[1:], t.dims)
    i_np, v_np = t.numpy()
    ref = ocsf.build(t.dims, i_np, t.vals.numpy(), ocsf.heuristic_order(t.dims))
    _same_tree(c, ref, t.nmodes)
    c.free()


def test_csf_build_rooted_rejects_bad_indices():
    cpd = _cpd()
    inds = torch.tensor([[0, 1], [0, 3], [0, 1]], device="cuda")
    with pytest.raises(cpd.CpdError) as e:
        cpd.csf_build_rooted(inds, torch.ones(2, device="cuda"), (2, 3, 2))
    assert e.value.status == cpd.CPD_EINVAL


def test_csf_build_is_deterministic():
    cpd = _cpd()
    t = CASES["zipf4"]()
    outs = []
    for _ in range(2):
        c = cpd.csf_build(_dev(t.inds), _dev(t.vals), t.dims)
        outs.append([x.cpu().numpy().tobytes() for l in range(4) for x in c.export(l) if x is not None])
    assert outs[0] == outs[1]


def test_csf_rejects_bad_input():
    cpd = _cpd()
    inds = torch.tensor([[0, 1], [0, 3], [0, 1]], device="cuda")
    vals = torch.ones(2, device="cuda")
    with pytest.raises(cpd.CpdError) as e:
        cpd.csf_build(inds, vals, (2, 3, 2))
    assert e.value.status == cpd.CPD_EINVAL
    with pytest.raises(cpd.CpdError):
        cpd.csf_build(torch.tensor([[0], [0], [-1]], device="cuda"), vals[:1], (2, 3, 2))


# ----------------------------------------------------------------- MTTKRP

def _factors(dims, R, seed, ld=None, dtype=torch.float32):
    g = torch.Generator().manual_seed(seed)
    out = []
    for d in dims:
        a = torch.rand((d, R), generator=g, dtype=torch.float64) * 2 - 0.5
        if ld is not None and ld > R:
            buf = torch.zeros((d, ld), dtype=torch.float64)
            buf[:, :R] = a
            out.append(buf)
        else:
            out.append(a)
    return out


def _row_ok(R, ld, prec):
    """Whether the row/root kernel takes this rank and row stride: the padded
    width (fp32 8/16/32/36/64, bf16 16/16/32/40/64) must fit in ld and rows must
    be 16-byte multiples."""
    widths = (8, 16, 32, 36, 64) if prec == "fp32" else (16, 16, 32, 40, 64)
    w = next(x for x in widths if x >= R)
    esize = 4 if prec == "fp32" else 2
    return ld >= w and (ld * esize) % 16 == 0


def _round_ok(R, ld):
    """Whether the leaf-level round kernel takes this rank and row stride: ld a
    multiple of 4 covering the rank rounded up to 4."""
    return ld % 4 == 0 and ld >= (R + 3) // 4 * 4


def _run(cpd, c, facs64, mode, R, precision, kernel, variant, tile=0):
    dt = torch.float32 if precision == "fp32" else torch.bfloat16
    dev = [f.to(dt).to("cuda") for f in facs64]
    dims = [f.shape[0] for f in facs64]
    out = torch.full((dims[mode], R + 3), 7.0, device="cuda")
    cpd.mttkrp(c, dev, mode, out=out, rank=R, precision=precision, kernel=kernel, variant=variant,
               tile_nnz=tile)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    assert (o[:, R:] == 7.0).all(), "columns beyond the rank were written"
    return o[:, :R], [f.to(dt).to(torch.float64)[:, :R].numpy() for f in facs64]


@pytest.mark.parametrize("R,ld", [(8, None), (16, None), (35, 36), (32, None), (3, None), (64, None)])
def test_mttkrp_every_level(case, R, ld):
    cpd = _cpd()
    name, t = case
    inds, vals = t.numpy()
    c = cpd.csf_build(_dev(t.inds), _dev(t.vals), t.dims)
    facs = _factors(t.dims, R, 100 + R, ld)
    for mode in range(t.nmodes):
        depth = c.order.index(mode)
        # auto: the library's pick (ROW at the root, TILED below it where it
        # applies)
        kernels = ["auto", "lane"] + (["row"] if 3 <= t.nmodes <= 5 and depth < t.nmodes - 1 and (ld or R) >= 8
                                      and R in (8, 16, 32, 35, 64) else [])
        if depth == t.nmodes - 1 and _round_ok(R, ld or R):
            kernels += ["round", "tiled"]
        elif depth >= 1 and _round_ok(R, ld or R):
            kernels += ["tiled"]  # the internal level's mode tiling
        # private: a copy of Y in LDS per block when it fits 64 KiB, else one
        # HBM copy per XCD summed afterwards
        variants = ["atomic"] + (["private"] if depth >= 1 else [])
        for kernel in kernels:
            # row kernel below the root: without (atomic) and with (private) the
            # LDS table of the level's most frequent output rows
            kvars = variants if kernel == "lane" else (["atomic", "private"] if kernel == "row" and depth >= 1
                                                       else ["auto"])
            for variant in kvars:
                for prec in ("fp32", "bf16"):
                    if kernel == "row" and not _row_ok(R, ld or R, prec):
                        continue
                    y, used = _run(cpd, c, facs, mode, R, prec, kernel, variant)
                    ref = ocoo.mttkrp(t.dims, inds, vals, [f[:, :R].numpy() for f in facs], mode)
                    tol = 1e-5 if prec == "fp32" else 1e-2
                    err = relerr(y, ref)
                    assert err <= tol, (name, mode, kernel, variant, prec, err)
                    if prec == "bf16":
                        # same kernel arithmetic on the rounded rows: tight
                        ref_b = ocoo.mttkrp(t.dims, inds, vals, used, mode)
                        assert relerr(y, ref_b) <= 1e-5, (name, mode, kernel, variant, err)


@pytest.mark.parametrize("tile", [1, 7, 32, 64, 96, 4096])
def test_mttkrp_tile_widths(tile):
    cpd = _cpd()
    t = CASES["zipf3"]()
    inds, vals = t.numpy()
    c = cpd.csf_build(_dev(t.inds), _dev(t.vals), t.dims)
    facs = _factors(t.dims, 16, 5)
    for mode in range(3):
        ref = ocoo.mttkrp(t.dims, inds, vals, [f.numpy() for f in facs], mode)
        depth = c.order.index(mode)
        # the lane-group (row) kernels take tile widths in multiples of 32; the
        # leaf-level round kernel rounds any width up to a multiple of 64; the
        # tiled kernels take it as the tile height in rows (capped by the LDS)
        row_ok = depth < 2 and tile % 32 == 0
        for kernel in ((["lane", "row"] if row_ok else ["lane"]) + (["round", "tiled"] if depth == 2 else [])
                       + (["tiled"] if depth == 1 else [])):
            y, _ = _run(cpd, c, facs, mode, 16, "fp32", kernel, "auto", tile)
            assert relerr(y, ref) <= 1e-5, (mode, kernel, tile)
    if tile % 32:
        with pytest.raises(cpd.CpdError):
            _run(cpd, c, facs, c.order[0], 16, "fp32", "row", "auto", tile)


@pytest.mark.parametrize("dims,alphas,nnz", [((50, 40, 3000), (2.0, 0.0, 0.0), 200_000),
                                             ((3, 500, 400), (0.0, 0.5, 0.5), 150_000),
                                             ((1, 700, 900), (0.0, 1.0, 1.0), 120_000),
                                             ((20, 30, 40, 50), (1.5, 1.0, 0.0, 0.0), 150_000)])
def test_mttkrp_root_hot_rows(dims, alphas, nnz):
    """Root rows spanning many lanes, tile steps and wave ranges (one root row
    holds most nonzeros), checked for every mode rooted at its own tree."""
    cpd = _cpd()
    t = _tensor(dims, nnz, alphas, 21)
    inds, vals = t.numpy()
    facs = _factors(t.dims, 8, 3)
    for mode in range(t.nmodes):
        order = [mode] + [m for m in range(t.nmodes) if m != mode]
        c = cpd.csf_build(_dev(t.inds), _dev(t.vals), t.dims, order)
        ref = ocoo.mttkrp(t.dims, inds, vals, [f.numpy() for f in facs], mode)
        for tile in (32, 64, 256):
            y, _ = _run(cpd, c, facs, mode, 8, "fp32", "row", "auto", tile)
            assert relerr(y, ref) <= 1e-5, (mode, tile)
        c.free()


def test_mttkrp_rejects_bad_arguments():
    cpd = _cpd()
    t = CASES["small3"]()
    c = cpd.csf_build(_dev(t.inds), _dev(t.vals), t.dims)
    facs = [torch.rand((d, 8), device="cuda") for d in t.dims]
    with pytest.raises(ValueError):
        cpd.mttkrp(c, facs, 3)
    with pytest.raises(cpd.CpdError):
        cpd.mttkrp(c, facs, 3, out=torch.empty((10, 8), device="cuda"))
    with pytest.raises(cpd.CpdError):
        cpd.mttkrp(c, facs, 0, rank=65)
    # the row kernel is not available for the leaf level
    leaf = c.order[-1]
    with pytest.raises(cpd.CpdError) as e:
        cpd.mttkrp(c, facs, leaf, kernel="row")
    assert e.value.status == cpd.CPD_EUNSUPPORTED
    # nor privatisation at the root (its rows never collide)
    with pytest.raises(cpd.CpdError) as e:
        cpd.mttkrp(c, facs, c.order[0], kernel="lane", variant="private")
    assert e.value.status == cpd.CPD_EUNSUPPORTED
    # the round kernel serves the leaf level only, the tiled kernels every level
    # below the root, neither with a privatised variant, and both need a row
    # stride that is a multiple of 4
    for kernel, mode, variant in (("round", c.order[0], "auto"), ("round", c.order[1], "auto"),
                                  ("round", leaf, "private"), ("tiled", c.order[0], "auto"),
                                  ("tiled", c.order[1], "private"), ("tiled", leaf, "private")):
        with pytest.raises(cpd.CpdError) as e:
            cpd.mttkrp(c, facs, mode, kernel=kernel, variant=variant)
        assert e.value.status == cpd.CPD_EUNSUPPORTED
    f6 = [torch.rand((d, 6), device="cuda") for d in t.dims]
    for kernel, mode in (("round", leaf), ("tiled", leaf), ("tiled", c.order[1])):
        with pytest.raises(cpd.CpdError) as e:
            cpd.mttkrp(c, f6, mode, rank=5, kernel=kernel)
        assert e.value.status == cpd.CPD_EUNSUPPORTED


@pytest.mark.parametrize("dims,alphas,order", [((2000, 300, 40), (0.5, 1.0, 0.0), (0, 1, 2)),
                                               ((600, 500, 3000), (0.0, 0.3, 2.0), (0, 1, 2)),
                                               ((400, 50, 90, 2500), (0.5, 0.5, 0.5, 1.5), (3, 1, 2, 0)),
                                               ((7, 9, 4000), (0.0, 0.0, 1.0), (0, 1, 2))])
@pytest.mark.parametrize("R", [8, 35])
def test_mttkrp_leaf_round_hot_rows(dims, alphas, order, R):
    """The leaf-level round kernel where every output row fits the block's LDS
    table (a 40-row leaf mode), where one leaf row takes most updates (Zipf
    2.0), on a 4-mode tree, and with long fibers (9 x 7 fibers over 4,000
    leaves each): against the oracle and the LANE kernel, FP32 and BF16."""
    cpd = _cpd()
    t = _tensor(dims, 150_000, alphas, 23)
    inds, vals = t.numpy()
    c = cpd.csf_build(_dev(t.inds), _dev(t.vals), t.dims, list(order))
    leaf = order[-1]
    ld = (R + 3) // 4 * 4
    facs = _factors(t.dims, R, 31, ld)
    ref = ocoo.mttkrp(t.dims, inds, vals, [f[:, :R].numpy() for f in facs], leaf)
    for prec in ("fp32", "bf16"):
        for tile in (0, 64, 1024):
            y, used = _run(cpd, c, facs, leaf, R, prec, "round", "auto", tile)
            lane, _ = _run(cpd, c, facs, leaf, R, prec, "lane", "atomic", tile)
            ref_b = ocoo.mttkrp(t.dims, inds, vals, used, leaf)
            assert relerr(y, ref_b) <= 1e-5, (dims, prec, tile)
            assert relerr(y, lane) <= 1e-5, (dims, prec, tile)
            if prec == "fp32":
                assert relerr(y, ref) <= 1e-5
        # the leaf-mode tiling (one tile or several, by the rank's LDS rows)
        y, used = _run(cpd, c, facs, leaf, R, prec, "tiled", "auto")
        assert relerr(y, ocoo.mttkrp(t.dims, inds, vals, used, leaf)) <= 1e-5, (dims, prec, "tiled")
    c.free()


@pytest.mark.parametrize("R", [8, 35, 64])
def test_mttkrp_internal_tiled_many_tiles(R):
    """The internal-level mode tiling on a 30,000-row internal mode (tens of
    tiles at rank 35 and 64), Zipf-skewed, with long and single-leaf nodes, at
    every internal level of 3-, 4- and 5-mode trees, FP32 and BF16: every row
    against the oracle (BF16 on the rounded rows), a second call on the cached
    tiling, and ragged tile heights."""
    cpd = _cpd()
    for dims, alphas, order in (((300, 30_000, 200), (1.0, 1.1, 0.5), (0, 1, 2)),
                                ((50, 30_000, 7, 4000), (0.3, 1.2, 0.0, 1.5), (2, 1, 0, 3)),
                                ((20, 30, 40, 30_000, 500), (0.5, 0.0, 0.8, 1.0, 0.0), (0, 1, 2, 3, 4))):
        t = _tensor(dims, 300_000, alphas, 37)
        inds, vals = t.numpy()
        c = cpd.csf_build(_dev(t.inds), _dev(t.vals), t.dims, list(order))
        ld = (R + 3) // 4 * 4
        facs = _factors(t.dims, R, 41, ld)
        for depth in range(1, t.nmodes - 1):
            mode = order[depth]
            ref = ocoo.mttkrp(t.dims, inds, vals, [f[:, :R].numpy() for f in facs], mode)
            for tile in (0, 0, 5):
                y, _u = _run(cpd, c, facs, mode, R, "fp32", "tiled", "auto", tile)
                assert relerr(y, ref) <= 1e-5, (dims, depth, R, tile)
            y, used = _run(cpd, c, facs, mode, R, "bf16", "tiled", "auto")
            assert relerr(y, ocoo.mttkrp(t.dims, inds, vals, used, mode)) <= 1e-5, (dims, depth, R, "bf16")
        c.free()


def test_mttkrp_internal_tiled_wide_key():
    """A size-ordered internal tiling whose sort key does not fit 64 bits:
    three 2^23-row modes and a 60-row root, so at depth 1 the tile number
    (17 bits) and the two large other levels (23 bits each) fill the key and
    the root index is left out of it (the order inside a tile then only
    partly by size; any order is correct).  Every internal level and the
    leaf level against the oracle, FP32, rank 8."""
    cpd = _cpd()
    dims = (1 << 23, 1 << 23, 1 << 23, 60)
    # one batch of draws, de-duplicated (top-up needs fewer than 2^62 cells)
    t = synth.gen_sparse(dims, 200_000, (0.5, 0.5, 0.5, 0.0), "lognormal:1.0", 43, device="cpu", topup=False,
                         fp32=True)
    inds, vals = t.numpy()
    order = [3, 0, 1, 2]
    c = cpd.csf_build(_dev(t.inds), _dev(t.vals), t.dims, order)
    R = 8
    facs = _factors(t.dims, R, 47)
    for depth in (1, 2, 3):
        mode = order[depth]
        ref = ocoo.mttkrp(t.dims, inds, vals, [f.numpy() for f in facs], mode)
        y, _u = _run(cpd, c, facs, mode, R, "fp32", "tiled", "auto")
        assert relerr(y, ref) <= 1e-5, (depth, relerr(y, ref))
    c.free()


@pytest.mark.parametrize("R", [8, 35, 64])
def test_mttkrp_leaf_tiled_many_tiles(R):
    """The leaf-mode tiling on a 30,000-row leaf mode (tens of tiles at rank
    35 and 64, a few at rank 8), Zipf-skewed, 3 and 4 modes: every row against
    the oracle, and a second call on the cached tiling."""
    cpd = _cpd()
    for dims, alphas in (((300, 200, 30_000), (1.0, 0.5, 1.1)), ((40, 50, 60, 30_000), (0.3, 0.8, 0.0, 1.2))):
        t = _tensor(dims, 400_000, alphas, 29)
        inds, vals = t.numpy()
        c = cpd.csf_build(_dev(t.inds), _dev(t.vals), t.dims)
        leaf = c.order[-1]
        assert t.dims[leaf] == 30_000
        ld = (R + 3) // 4 * 4
        facs = _factors(t.dims, R, 33, ld)
        ref = ocoo.mttkrp(t.dims, inds, vals, [f[:, :R].numpy() for f in facs], leaf)
        for _ in range(2):
            y, _u = _run(cpd, c, facs, leaf, R, "fp32", "tiled", "auto")
            assert relerr(y, ref) <= 1e-5, (dims, R)
        c.free()


# ----------------------------------------------------------------- dense steps

@pytest.mark.parametrize("rows,R", [(1, 1), (37, 5), (1000, 16), (4097, 35), (20000, 64)])
def test_gram(rows, R):
    cpd = _cpd()
    g = torch.Generator().manual_seed(rows + R)
    A = (torch.rand((rows, R), generator=g) - 0.3).to(torch.float32)
    G = cpd.gram(A.cuda()).cpu().numpy()
    ref = oals.gram(A.numpy().astype(np.float64))
    np.testing.assert_allclose(G, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    assert (G == G.T).all()


@pytest.mark.parametrize("R", [1, 8, 16, 35, 64])
def test_solve_normalize(R):
    cpd = _cpd()
    rng = np.random.default_rng(R)
    dims = (300, 200, 100)
    facs = [rng.uniform(0, 1, (d, R)) for d in dims]
    grams = [oals.gram(f.astype(np.float32).astype(np.float64)) for f in facs]
    Y = rng.standard_normal((dims[1], R)).astype(np.float32)
    out = cpd.solve_normalize([torch.from_numpy(gm).cuda() for gm in grams], 1,
                              torch.from_numpy(Y).cuda(), want_bf16=True)
    torch.cuda.synchronize()
    An, used = oals.normal_solve(oals.hadamard_v(grams, 1), Y.astype(np.float64))
    Aref, lam = oals.normalize_columns(An)
    assert int(out["used_pinv"].item()) == int(used)
    np.testing.assert_allclose(out["lam"].cpu().numpy(), lam, rtol=1e-9)
    assert relerr(out["A"].cpu().numpy(), Aref) <= 1e-6
    assert torch.equal(out["A_bf16"].cpu(), out["A"].cpu().to(torch.bfloat16))
    Gn = oals.gram(out["A"].cpu().numpy().astype(np.float64))
    np.testing.assert_allclose(out["G"].cpu().numpy(), Gn, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("R", [6, 20])  # the 256- and the 1024-thread inverse block
def test_solve_normalize_singular_uses_pinv(R):
    cpd = _cpd()
    rng = np.random.default_rng(3)
    M = rng.standard_normal((3 * R + 20, R))
    M[:, R - 2] = M[:, 2]
    G1 = M.T @ M
    grams = [np.ones((R, R)), G1, np.ones((R, R))]
    Y = rng.standard_normal((25, R)).astype(np.float32)
    out = cpd.solve_normalize([torch.from_numpy(g).cuda() for g in grams], 0, torch.from_numpy(Y).cuda())
    torch.cuda.synchronize()
    An, used = oals.normal_solve(oals.hadamard_v(grams, 0), Y.astype(np.float64))
    assert used and int(out["used_pinv"].item()) == 1
    Aref, lam = oals.normalize_columns(An)
    assert relerr(out["A"].cpu().numpy(), Aref) <= 1e-5
    np.testing.assert_allclose(out["lam"].cpu().numpy(), lam, rtol=1e-6)


def test_solve_normalize_zero_column():
    cpd = _cpd()
    R = 4
    G = np.eye(R)
    Y = np.ones((10, R), dtype=np.float32)
    Y[:, 1] = 0
    out = cpd.solve_normalize([torch.from_numpy(G).cuda()] * 3, 2, torch.from_numpy(Y).cuda())
    A = out["A"].cpu().numpy()
    assert np.isfinite(A).all() and (A[:, 1] == 0).all()
    assert out["lam"].cpu().numpy()[1] == 0.0


def test_fit_matches_oracle():
    cpd = _cpd()
    t = CASES["zipf3"]()
    inds, vals = t.numpy()
    R = 8
    rng = np.random.default_rng(1)
    facs = [rng.uniform(0, 1, (d, R)).astype(np.float32).astype(np.float64) for d in t.dims]
    lam = rng.uniform(0.5, 2, R)
    Y = ocoo.mttkrp(t.dims, inds, vals, facs, 2)
    grams = [oals.gram(f) for f in facs]
    nx = ocoo.sumsq(vals)
    ref = oals.fit_from(nx, lam, facs[2], Y, grams)
    got = cpd.fit(nx, torch.from_numpy(lam).cuda(), torch.from_numpy(facs[2]).float().cuda(),
                  torch.from_numpy(Y).float().cuda(), [torch.from_numpy(g).cuda() for g in grams])
    assert abs(got.item() - ref) < 1e-6
    s = cpd.sumsq(t.vals.cuda()).item()
    assert abs(s - nx) <= 1e-12 * nx


# ----------------------------------------------------------------- CP-ALS

@pytest.mark.parametrize("single_csf", [False, True])
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_als_small3_matches_oracle(single_csf, precision):
    cpd = _cpd()
    t = synth.make_config("small3")          # float64 values, rounded to FP32 for the GPU
    inds, vals64 = t.numpy()
    R, iters = 8, 20
    init = synth.init_factors(t.dims, R, 11)
    ref = oals.cp_als(t.dims, inds, vals64, R, iters, 0.0, [a.numpy() for a in init])
    got = cpd.als(_dev(t.inds), _dev(t.vals.float()), t.dims, R, iters, 0.0,
                  init=[a.float().cuda() for a in init], precision=precision,
                  single_csf=single_csf)
    assert got["iters"] == iters
    tol = 1e-4
    assert abs(got["fit"] - ref["fit"]) <= tol, (got["fit"], ref["fit"])
    if precision == "fp32":
        np.testing.assert_allclose(got["fits"], ref["fits"], atol=1e-5)
        np.testing.assert_allclose(got["lam"], ref["lam"], rtol=1e-3)
        for m in range(3):
            assert relerr(got["factors"][m].cpu().numpy(), ref["factors"][m]) <= 1e-3


@pytest.mark.parametrize("single_csf", [False, True])
def test_als_planted_block_recovers(single_csf):
    """An exactly rank-8 sparse tensor is recovered: the FP64 oracle's fit of
    the model cpd_als returns is 1 to within 1e-4, and the fit cpd_als reports
    (evaluated from an FP64-accumulated MTTKRP of the last mode: the root
    kernel on the per-mode trees, the LANE kernel on the single tree) agrees
    with it to 1e-4 (Algorithm 1's fit step)."""
    cpd = _cpd()
    t, _ = synth.block_planted()
    inds, vals = t.numpy()
    R = 8
    best = -1.0
    for s in range(3):
        init = synth.init_factors(t.dims, R, 100 + s)
        got = cpd.als(_dev(t.inds), _dev(t.vals.float()), t.dims, R, 500, 1e-9,
                      init=[a.float().cuda() for a in init], single_csf=single_csf)
        A = [f.cpu().double().numpy() for f in got["factors"]]
        lam = np.asarray(got["lam"])
        Y = ocoo.mttkrp(t.dims, inds, vals, A, 2)
        fit64 = oals.fit_from(ocoo.sumsq(vals), lam, A[2], Y, [oals.gram(a) for a in A])
        assert abs(got["fit"] - fit64) <= 1e-4, (got["fit"], fit64)
        best = max(best, fit64)
        if best >= 1 - 1e-4:
            break
    assert best >= 1 - 1e-4, best


def test_als_reported_fit_is_the_returned_models_fit():
    """With the FP64 fit pass the reported fit equals the oracle's fit of the
    returned model to 1e-7 (FP32 and BF16 gathers, 4 modes); with fast_fit
    it is the last sweep's fit."""
    cpd = _cpd()
    t = CASES["zipf4"]()
    inds, vals = t.numpy()
    R = 8
    init = synth.init_factors(t.dims, R, 5)
    for prec in ("fp32", "bf16"):
        got = cpd.als(_dev(t.inds), _dev(t.vals), t.dims, R, 4, 0.0, init=[a.float().cuda() for a in init],
                      precision=prec)
        A = [f.cpu().double().numpy() for f in got["factors"]]
        lam = np.asarray(got["lam"])
        Y = ocoo.mttkrp(t.dims, inds, vals, A, 3)
        ref = oals.fit_from(ocoo.sumsq(vals), lam, A[3], Y, [oals.gram(a) for a in A])
        assert abs(got["fit"] - ref) <= 1e-7, (prec, got["fit"], ref)
    fast = cpd.als(_dev(t.inds), _dev(t.vals), t.dims, R, 4, 0.0, init=[a.float().cuda() for a in init],
                   fast_fit=True)
    assert fast["fit"] == fast["fits"][-1]


def test_als_2mode_matches_oracle():
    """Two modes: every MTTKRP runs the LANE kernel at the root of its tree."""
    cpd = _cpd()
    t = CASES["two2"]()
    inds, vals = t.numpy()
    R = 6
    init = synth.init_factors(t.dims, R, 4)
    ref = oals.cp_als(t.dims, inds, vals, R, 8, 0.0, [a.numpy() for a in init])
    for single in (False, True):
        got = cpd.als(_dev(t.inds), _dev(t.vals), t.dims, R, 8, 0.0, init=[a.float().cuda() for a in init],
                      single_csf=single)
        np.testing.assert_allclose(got["fits"], ref["fits"], atol=1e-5)
        assert abs(got["fit"] - ref["fit"]) <= 1e-5


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_als_planted_literal_matches_oracle(precision):
    """The literal planted rank-8 variant of the 200x150x100 tensor (values = the
    sum of 8 outer products sampled at the 20,000 coordinates): 20 sweeps,
    tol 0, shared init; FP32 trajectory within 1e-5, final fit within 1e-4."""
    cpd = _cpd()
    t = synth.planted_literal()
    inds, vals64 = t.numpy()
    R, iters = 8, 20
    init = synth.init_factors(t.dims, R, 11)
    ref = oals.cp_als(t.dims, inds, vals64, R, iters, 0.0, [a.numpy() for a in init])
    got = cpd.als(_dev(t.inds), _dev(t.vals.float()), t.dims, R, iters, 0.0,
                  init=[a.float().cuda() for a in init], precision=precision)
    assert got["iters"] == iters
    assert abs(got["fit"] - ref["fit"]) <= 1e-4, (got["fit"], ref["fit"])
    if precision == "fp32":
        np.testing.assert_allclose(got["fits"], ref["fits"], atol=1e-5)


def test_als_4mode_and_5mode_match_oracle():
    cpd = _cpd()
    for name, R in (("zipf4", 8), ("zipf5", 4)):
        t = CASES[name]()
        inds, vals = t.numpy()
        init = synth.init_factors(t.dims, R, 3)
        ref = oals.cp_als(t.dims, inds, vals, R, 5, 0.0, [a.numpy() for a in init])
        got = cpd.als(_dev(t.inds), _dev(t.vals), t.dims, R, 5, 0.0, init=[a.float().cuda() for a in init])
        np.testing.assert_allclose(got["fits"], ref["fits"], atol=1e-4)


def test_als_convergence_stop_and_seeded_init():
    cpd = _cpd()
    t = synth.make_config("small3")
    got = cpd.als(_dev(t.inds), _dev(t.vals.float()), t.dims, 4, 50, 1.0, seed=5, timing=True)
    assert got["iters"] == 2
    assert got["timing_ms"]["total"] > 0
    again = cpd.als(_dev(t.inds), _dev(t.vals.float()), t.dims, 4, 3, 0.0, seed=5)
    same = cpd.als(_dev(t.inds), _dev(t.vals.float()), t.dims, 4, 3, 0.0, seed=5)
    assert abs(again["fit"] - same["fit"]) < 1e-6
