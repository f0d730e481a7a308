"""Seeded synthetic sparse tensors for the CSF-MTTKRP / CP-ALS workloads.

This module holds none of the decomposition's arithmetic: only random draws,
Zipf sampling over permuted index ranges, de-duplication of coordinates and the
value distributions.  The HIP path's tests and benchmark and the oracle's tests
all take their inputs from here, so the two sides see identical tensors.

Random numbers come from one counter-based generator, SplitMix64 (Steele, Lea
and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014),
applied to ``stream_key + counter``.  Only 64-bit wrapping adds, multiplies,
xors and shifts are used, so a counter gives the same number on the CPU and on
the GPU.

The tensors stand in for the data sets of the paper's Table I (YELP, NELL-2,
NETFLIX, ...), which are not available here; only their shapes are mirrored.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

_M64 = (1 << 64) - 1
_GOLDEN = 0x9E3779B97F4A7C15
_MUL1 = 0xBF58476D1CE4E5B9
_MUL2 = 0x94D049BB133111EB


def _s64(x: int) -> int:
    """Python int in [0, 2^64) -> the int64 with the same bits."""
    x &= _M64
    return x - (1 << 64) if x >= (1 << 63) else x


def _lsr(x: torch.Tensor, s: int) -> torch.Tensor:
    """Logical right shift of int64 bits (torch's >> is arithmetic)."""
    return (x >> s) & ((1 << (64 - s)) - 1)


def splitmix64(x: torch.Tensor) -> torch.Tensor:
    """SplitMix64 finaliser of (x + golden gamma), on int64 tensors (wrapping)."""
    z = x + _s64(_GOLDEN)
    z = (z ^ _lsr(z, 30)) * _s64(_MUL1)
    z = (z ^ _lsr(z, 27)) * _s64(_MUL2)
    return z ^ _lsr(z, 31)


def splitmix64_int(x: int) -> int:
    """Scalar SplitMix64 on Python ints (same bits as :func:`splitmix64`)."""
    z = (x + _GOLDEN) & _M64
    z = ((z ^ (z >> 30)) * _MUL1) & _M64
    z = ((z ^ (z >> 27)) * _MUL2) & _M64
    return z ^ (z >> 31)


def stream_key(seed: int, stream: int) -> int:
    """Key of an independent random stream for (seed, stream)."""
    return splitmix64_int(splitmix64_int(seed & _M64) ^ ((stream * _GOLDEN) & _M64))


def rand_u64(seed: int, stream: int, start: int, count: int, device="cpu") -> torch.Tensor:
    """Raw 64-bit draws (as int64 bits) for counters start .. start+count-1."""
    ctr = torch.arange(start, start + count, dtype=torch.int64, device=device)
    return splitmix64(ctr + _s64(stream_key(seed, stream)))


def rand_uniform(seed: int, stream: int, start: int, count: int, device="cpu") -> torch.Tensor:
    """U[0, 1) doubles: the top 53 bits of each draw times 2^-53 (exact)."""
    return _lsr(rand_u64(seed, stream, start, count, device), 11).to(torch.float64) * (2.0 ** -53)


def random_permutation(n: int, seed: int, stream: int, device="cpu") -> torch.Tensor:
    """A uniformly random permutation of 0..n-1 (argsort of distinct-with-
    overwhelming-probability 64-bit keys; stable, so ties are still defined)."""
    keys = rand_u64(seed, stream, 0, n, device)
    return torch.argsort(keys, stable=True)


def zipf_cdf(n: int, alpha: float) -> np.ndarray:
    """CDF of P(k) proportional to k^-alpha on k = 1..n, in float64."""
    w = np.arange(1, n + 1, dtype=np.float64) ** (-float(alpha))
    c = np.cumsum(w)
    c /= c[-1]
    return c


def zipf_draw(u: torch.Tensor, n: int, alpha: float, perm: torch.Tensor) -> torch.Tensor:
    """Zipf(alpha) over n by inverse CDF, mapped through the permutation perm.

    alpha == 0 is the uniform distribution, drawn as floor(u * n)."""
    if alpha == 0.0:
        rank = torch.clamp((u * n).to(torch.int64), max=n - 1)
    else:
        cdf = torch.from_numpy(zipf_cdf(n, alpha)).to(u.device)
        rank = torch.clamp(torch.searchsorted(cdf, u, right=True), max=n - 1)
    return perm[rank]


@dataclass
class SparseTensor:
    """A COO tensor: inds is (N, nnz) int64, vals (nnz,) float64 or float32."""
    dims: tuple
    inds: torch.Tensor
    vals: torch.Tensor
    meta: dict = field(default_factory=dict)

    @property
    def nmodes(self) -> int:
        return len(self.dims)

    @property
    def nnz(self) -> int:
        return int(self.vals.numel())

    def to(self, device) -> "SparseTensor":
        return SparseTensor(self.dims, self.inds.to(device), self.vals.to(device), dict(self.meta))

    def numpy(self):
        """(inds int64 (N, nnz), vals float64) on the host."""
        return self.inds.cpu().numpy(), self.vals.cpu().to(torch.float64).numpy()


# --------------------------------------------------------------------------
# Coordinates
# --------------------------------------------------------------------------

_ST_COORD = 1          # streams 1 .. 1+N-1: per-mode coordinate draws
_ST_PERM = 64          # streams 64..: per-mode Zipf rank permutations
_ST_SELECT = 128       # selection of exactly nnz distinct coordinates
_ST_VAL = 256          # values (two streams)
_ST_FACTOR = 1024      # initial factors, one stream per mode


def _strides(dims):
    s, out = 1, []
    for d in reversed(dims):
        out.append(s)
        s *= d
    return list(reversed(out)), s


def _draw_coords(dims, alphas, perms, seed, start, count, device):
    cols = []
    for m, (n, a) in enumerate(zip(dims, alphas)):
        u = rand_uniform(seed, _ST_COORD + m, start, count, device)
        cols.append(zipf_draw(u, n, a, perms[m]))
    return torch.stack(cols)


def distinct_coords(dims, alphas, nnz, seed, device="cpu", topup=True):
    """Distinct coordinates under per-mode Zipf(alpha_m) over permuted ranges.

    With topup, draws continue until at least nnz distinct coordinates exist
    and exactly nnz of them are kept, chosen uniformly by the seed; without it,
    one batch of nnz draws is de-duplicated and its distinct count is kept.
    The result is (N, k) int64 in a seeded random order.
    """
    dims = tuple(int(d) for d in dims)
    perms = [random_permutation(n, seed, _ST_PERM + m, device) for m, n in enumerate(dims)]
    strides, total = _strides(dims)
    if topup and nnz > total:
        raise ValueError("nnz exceeds the number of cells")
    one_word = total < (1 << 62)
    salt = _s64(stream_key(seed, _ST_SELECT))
    if one_word:
        st = torch.tensor(strides, dtype=torch.int64, device=device).view(-1, 1)
        keys = torch.empty(0, dtype=torch.int64, device=device)
        counter, draws = 0, (int(nnz * 1.3) + 1024 if topup else nnz)
        while True:
            c = _draw_coords(dims, alphas, perms, seed, counter, draws, device)
            keys = torch.unique(torch.cat([keys, (c * st).sum(0)]))
            del c
            counter += draws
            if not topup or keys.numel() >= nnz:
                break
            draws = max(3 * (nnz - keys.numel()), 1 << 16)
        keep = keys.numel() if not topup else nnz
        order = torch.argsort(splitmix64(keys ^ salt), stable=True)[:keep]
        keys = keys[order]
        out = torch.empty((len(dims), keep), dtype=torch.int64, device=device)
        for m in range(len(dims)):
            out[m] = (keys // strides[m]) % dims[m]
        return out
    # Very large index spaces (five modes of up to 1e6): one batch, rows made
    # unique directly.
    if topup:
        raise ValueError("top-up needs a product of dims below 2^62")
    c = _draw_coords(dims, alphas, perms, seed, 0, nnz, device)
    rows = torch.unique(c.t().contiguous(), dim=0)
    h = torch.zeros(rows.shape[0], dtype=torch.int64, device=device)
    for m in range(len(dims)):
        h = splitmix64(h ^ rows[:, m])
    order = torch.argsort(splitmix64(h ^ salt), stable=True)
    return rows[order].t().contiguous()


# --------------------------------------------------------------------------
# Values
# --------------------------------------------------------------------------

def draw_values(kind: str, count: int, seed: int, device="cpu") -> torch.Tensor:
    """Values per distinct coordinate, float64.

    kind: "uniform" U(0,1); "lognormal:<sigma>" exp(sigma*z) with z standard
    normal by Box-Muller; "int1to5" uniform integers 1..5."""
    u1 = rand_uniform(seed, _ST_VAL, 0, count, device)
    if kind == "uniform":
        return u1
    if kind == "int1to5":
        return torch.floor(u1 * 5.0) + 1.0
    if kind.startswith("lognormal:"):
        sigma = float(kind.split(":")[1])
        u2 = rand_uniform(seed, _ST_VAL + 1, 0, count, device)
        z = torch.sqrt(-2.0 * torch.log1p(-u1)) * torch.cos(2.0 * math.pi * u2)
        return torch.exp(sigma * z)
    raise ValueError(kind)


def gen_sparse(dims, nnz, alphas, value_kind, seed, device="cpu", topup=True,
               fp32=True) -> SparseTensor:
    inds = distinct_coords(dims, alphas, nnz, seed, device, topup)
    vals = draw_values(value_kind, inds.shape[1], seed, device)
    if fp32:
        vals = vals.to(torch.float32)
    meta = dict(seed=seed, alphas=tuple(alphas), value_kind=value_kind, topup=topup)
    return SparseTensor(tuple(int(d) for d in dims), inds, vals, meta)


def init_factors(dims, rank, seed, device="cpu"):
    """U(0,1) initial factors, one (I_m x R) float64 matrix per mode."""
    return [rand_uniform(seed, _ST_FACTOR + m, 0, int(n) * rank, device).view(int(n), rank)
            for m, n in enumerate(dims)]


# --------------------------------------------------------------------------
# The named workloads
# --------------------------------------------------------------------------

CONFIGS = {
    # 200 x 150 x 100, 20,000 distinct uniform coordinates, U(0,1) values
    # kept in float64, rank 8, 20 iterations.
    "small3": dict(dims=(200, 150, 100), nnz=20_000, alphas=(0.0, 0.0, 0.0),
                   values="uniform", seed=1, rank=8, iters=20, fp32=False, init_seed=11),
    # NELL-2-shaped (Table I): 12k x 9k x 29k, 76M nonzeros, Zipf(1.1) per mode,
    # lognormal(0,1) values, rank 35 (the paper's rank), 10 iterations.
    "nell2": dict(dims=(12_000, 9_000, 29_000), nnz=76_000_000, alphas=(1.1, 1.1, 1.1),
                  values="lognormal:1.0", seed=2, rank=35, iters=10, fp32=True, init_seed=21),
    # NETFLIX-shaped (Table I): 480k x 18k x 2k, 100M nonzeros, Zipf (0.9, 1.2, 0),
    # integer ratings 1..5, rank 16, 20 iterations.
    "netflix": dict(dims=(480_000, 18_000, 2_000), nnz=100_000_000, alphas=(0.9, 1.2, 0.0),
                    values="int1to5", seed=3, rank=16, iters=20, fp32=True, init_seed=31),
    # 4-mode 100k x 50k x 10k x 1k, 50M nonzeros, Zipf(1.0), lognormal(0, 0.5),
    # rank 32, 20 iterations.
    "fourmode": dict(dims=(100_000, 50_000, 10_000, 1_000), nnz=50_000_000,
                     alphas=(1.0, 1.0, 1.0, 1.0), values="lognormal:0.5", seed=4, rank=32,
                     iters=20, fp32=True, init_seed=41),
}


def make_config(name: str, device="cpu", nnz: int | None = None) -> SparseTensor:
    """Generate a named workload (optionally with a smaller nnz, same recipe)."""
    c = CONFIGS[name]
    t = gen_sparse(c["dims"], c["nnz"] if nnz is None else nnz, c["alphas"], c["values"],
                   c["seed"], device, topup=True, fp32=c["fp32"])
    t.meta.update(name=name, rank=c["rank"], iters=c["iters"], init_seed=c["init_seed"])
    return t


def planted_literal(device="cpu", rank=8, seed=12) -> SparseTensor:
    """The small3 coordinates with values = sum of `rank` outer products of
    U(0,1) factors sampled there (a parity case, not a low-rank sparse tensor)."""
    base = make_config("small3", device)
    fac = init_factors(base.dims, rank, seed, device)
    prod = torch.ones((base.nnz, rank), dtype=torch.float64, device=device)
    for m in range(base.nmodes):
        prod = prod * fac[m][base.inds[m]]
    return SparseTensor(base.dims, base.inds, prod.sum(1), dict(base.meta, planted=seed))


def block_planted(dims=(200, 150, 100), rank=8, block=(15, 13, 13), seed=13,
                  device="cpu"):
    """Exactly rank-`rank` sparse tensor: component r is an outer product of
    vectors supported on a random block (block[m] rows per mode) with U(0.5,1.5)
    entries; X is their sum on the union of the blocks, so the zeros outside
    are true zeros.  Returns (tensor, planted factors)."""
    nm = len(dims)
    facs = [torch.zeros((d, rank), dtype=torch.float64) for d in dims]
    for m, d in enumerate(dims):
        for r in range(rank):
            rows = random_permutation(d, seed, 4096 + 64 * m + r)[: block[m]]
            facs[m][rows, r] = 0.5 + rand_uniform(seed, 8192 + 64 * m + r, 0, block[m])
    supp = []
    for r in range(rank):
        idx = [torch.nonzero(facs[m][:, r]).flatten() for m in range(nm)]
        grids = torch.meshgrid(*idx, indexing="ij")
        supp.append(torch.stack([g.reshape(-1) for g in grids]))
    coords = torch.unique(torch.cat(supp, 1), dim=1)
    prod = torch.ones((coords.shape[1], rank), dtype=torch.float64)
    for m in range(nm):
        prod = prod * facs[m][coords[m]]
    vals = prod.sum(1)
    order = random_permutation(coords.shape[1], seed, 3)
    t = SparseTensor(tuple(dims), coords[:, order].contiguous(), vals[order].contiguous(),
                     dict(planted_block=seed, rank=rank))
    return t.to(device), [f.to(device) for f in facs]


# --------------------------------------------------------------------------
# Learned-selector corpus: one seeded spec per tensor
# --------------------------------------------------------------------------

def selector_spec(seed: int, max_nnz: float = 5e7) -> dict:
    """Spec of corpus tensor `seed`: N in {3,4,5}; dims round(10^U(3,6));
    nnz target 10^U(5, log10 max_nnz) (one draw, then de-duplicated);
    alpha_m ~ U(0, 1.5); rank in {8,16,32,64}; lognormal(0,1) values."""
    u = rand_uniform(seed, 77, 0, 16).numpy()
    nm = 3 + int(u[0] * 3)
    dims = tuple(int(round(10 ** (3 + 3 * u[1 + m]))) for m in range(nm))
    nnz = int(round(10 ** (5 + (math.log10(max_nnz) - 5) * u[6])))
    alphas = tuple(float(1.5 * u[7 + m]) for m in range(nm))
    rank = (8, 16, 32, 64)[int(u[12] * 4)]
    return dict(dims=dims, nnz=nnz, alphas=alphas, rank=rank, seed=seed)


def selector_tensor(seed: int, device="cpu", max_nnz: float = 5e7) -> SparseTensor:
    s = selector_spec(seed, max_nnz)
    t = gen_sparse(s["dims"], s["nnz"], s["alphas"], "lognormal:1.0", seed, device,
                   topup=False, fp32=True)
    t.meta.update(s)
    return t
