"""Seeded synthetic sparse tensors (input data only).

This module draws coordinates, values and dense matrices.  It holds none of
the F-COO method's arithmetic: no sorting into modes, no flags, no products
with factor matrices beyond the one data recipe that plants a CP model
(``planted_values``), which turns drawn factors into drawn tensor values.
Both the FP64 oracle (through the tests) and the HIP path consume what it
returns; neither side lives here.

Workloads stand in for the paper's FROSTT tensors (Sec. V, Table IV), which
are not available: uniform coordinates for the regular / dense end, Zipf
skew for the very sparse end with long slices and far-apart gathers.

Every stream comes from ``numpy.random.Generator(PCG64(SeedSequence(...)))``
so a given (config, role) always yields the same numbers.
"""
from __future__ import annotations

import dataclasses
import os
import sys
from typing import List, Optional, Sequence

import numpy as np

SEED_BASE = 170509905

# stream roles: one independent child stream each
_ROLES = ("coords", "values", "factors", "planted", "noise", "perm", "shuffle", "init")


def rng(cfg: int, role: str) -> np.random.Generator:
    """Independent, reproducible stream for (config, role)."""
    k = _ROLES.index(role)
    ss = np.random.SeedSequence([SEED_BASE, int(cfg), k])
    return np.random.Generator(np.random.PCG64(ss))


@dataclasses.dataclass
class SparseTensor:
    dims: List[int]
    idx: List[np.ndarray]          # order int32 arrays, 0-based
    vals: np.ndarray               # float64 values as drawn
    name: str = ""

    @property
    def order(self) -> int:
        return len(self.dims)

    @property
    def nnz(self) -> int:
        return int(self.vals.shape[0])

    def vals_f32(self) -> np.ndarray:
        return self.vals.astype(np.float32)

    def coords(self) -> np.ndarray:
        """(nnz, order) int64 coordinate matrix."""
        if self.nnz == 0:
            return np.zeros((0, self.order), dtype=np.int64)
        return np.stack([i.astype(np.int64) for i in self.idx], axis=1)


# ----------------------------------------------------------------------------
# coordinate samplers
# ----------------------------------------------------------------------------

def _strides(dims: Sequence[int]) -> np.ndarray:
    s = np.ones(len(dims), dtype=np.uint64)
    for m in range(1, len(dims)):
        s[m] = s[m - 1] * np.uint64(dims[m - 1])
    return s


def _pack(cols: List[np.ndarray], dims: Sequence[int]) -> np.ndarray:
    total = 1
    for d in dims:
        total *= int(d)
    if total >= 2 ** 63:
        raise ValueError("coordinate space too large for 63-bit packing")
    st = _strides(dims)
    key = np.zeros(cols[0].shape[0], dtype=np.uint64)
    for m, c in enumerate(cols):
        key += c.astype(np.uint64) * st[m]
    return key


def _unpack(keys: np.ndarray, dims: Sequence[int]) -> List[np.ndarray]:
    out = []
    rem = keys.copy()
    for d in dims:
        out.append((rem % np.uint64(d)).astype(np.int32))
        rem //= np.uint64(d)
    return out


class _ZipfMode:
    """Truncated Zipf over ranks 1..I (P(r) proportional to r^-s), ranks
    mapped to indices through a seeded permutation of [0, I)."""

    def __init__(self, I: int, s: float, perm_rng: np.random.Generator):
        w = np.arange(1, I + 1, dtype=np.float64) ** (-s)
        cdf = np.cumsum(w)
        self.cdf = cdf / cdf[-1]
        self.perm = perm_rng.permutation(I).astype(np.int64)

    def draw(self, n: int, g: np.random.Generator) -> np.ndarray:
        u = g.random(n)
        r = np.searchsorted(self.cdf, u, side="right")
        np.minimum(r, self.cdf.shape[0] - 1, out=r)
        return self.perm[r]


def _unique_coords(dims, nnz, draw_batch, g_sel) -> List[np.ndarray]:
    """Draw batches until >= nnz unique coordinates exist, then keep a seeded
    subset of exactly nnz.  Returns columns in ascending packed-key order."""
    total = 1
    for d in dims:
        total *= int(d)
    if nnz > total:
        raise ValueError("more nonzeros requested than cells")
    keys = np.zeros(0, dtype=np.uint64)
    want = nnz
    while keys.shape[0] < nnz:
        batch = max(1024, int(1.15 * (nnz - keys.shape[0])) + 64)
        cols = draw_batch(batch)
        _note("drew", batch, "coordinates")
        keys = np.unique(np.concatenate([keys, _pack(cols, dims)]))
        _note("unique", keys.shape[0], "of", nnz)
        want = nnz
    if keys.shape[0] > want:
        keep = np.sort(g_sel.choice(keys.shape[0], size=want, replace=False))
        keys = keys[keep]
    return _unpack(keys, dims)


def uniform_tensor(dims, nnz, cfg, name="uniform", value_kind="u01") -> SparseTensor:
    """Unique uniform-random coordinates, values U(0,1), nonzeros shuffled."""
    dims = [int(d) for d in dims]
    gc = rng(cfg, "coords")

    def draw(n):
        return [gc.integers(0, d, size=n, dtype=np.int64) for d in dims]

    cols = _unique_coords(dims, nnz, draw, rng(cfg, "perm"))
    return _finish(dims, cols, cfg, name, value_kind)


def zipf_tensor(dims, nnz, cfg, s=1.1, name="zipf", value_kind="u01") -> SparseTensor:
    """Unique coordinates with independent truncated Zipf(s) skew per mode."""
    dims = [int(d) for d in dims]
    gp = rng(cfg, "perm")
    modes = [_ZipfMode(d, s, gp) for d in dims]
    gc = rng(cfg, "coords")

    def draw(n):
        return [zm.draw(n, gc) for zm in modes]

    cols = _unique_coords(dims, nnz, draw, gp)
    return _finish(dims, cols, cfg, name, value_kind)


def _finish(dims, cols, cfg, name, value_kind) -> SparseTensor:
    nnz = cols[0].shape[0] if cols else 0
    gv = rng(cfg, "values")
    if value_kind == "u01":
        vals = gv.random(nnz)
    elif value_kind == "int":
        vals = gv.integers(1, 5, size=nnz).astype(np.float64)
    else:
        raise ValueError(value_kind)
    order = rng(cfg, "shuffle").permutation(nnz)
    idx = [c[order].astype(np.int32) for c in cols]
    return SparseTensor(dims=list(dims), idx=idx, vals=vals[order], name=name)


def factors(dims, R, cfg, role="factors", kind="normal") -> List[np.ndarray]:
    """Dense I_m x R matrices, row-major float64.  kind: 'normal' N(0,1) or
    'int' (integers in [-3, 3], for exact-arithmetic tests)."""
    g = rng(cfg, role)
    out = []
    for d in dims:
        if kind == "normal":
            out.append(g.standard_normal((int(d), int(R))))
        elif kind == "int":
            out.append(g.integers(-3, 4, size=(int(d), int(R))).astype(np.float64))
        else:
            raise ValueError(kind)
    return out


def planted_values(idx: List[np.ndarray], planted: List[np.ndarray], noise_var: float,
                   cfg: int, chunk: int = 1 << 22) -> np.ndarray:
    """Data recipe for a planted CP tensor sampled at given coordinates:
    value = sum_r prod_m P_m[i_m, r] + N(0, noise_var) noise (variance, so
    sigma = sqrt(noise_var))."""
    nnz = idx[0].shape[0]
    out = np.empty(nnz, dtype=np.float64)
    _note("planting values, rank", planted[0].shape[1])
    for s in range(0, nnz, chunk):
        e = min(nnz, s + chunk)
        p = planted[0][idx[0][s:e]].copy()
        for m in range(1, len(planted)):
            p *= planted[m][idx[m][s:e]]
        out[s:e] = p.sum(axis=1)
    if noise_var > 0:
        out += rng(cfg, "noise").normal(0.0, np.sqrt(noise_var), size=nnz)
    return out


# ----------------------------------------------------------------------------
# the five workloads (sizes mirror the paper's regimes; see the design notes)
# ----------------------------------------------------------------------------

CONFIGS = {
    0: dict(name="uniform-200x150x100-10k", dims=[200, 150, 100], nnz=10_000, skew=None, R=[8]),
    1: dict(name="zipf1.1-100kx80kx60k-20M", dims=[100_000, 80_000, 60_000], nnz=20_000_000,
            skew=1.1, R=[16, 32]),
    2: dict(name="zipf1.1-50kx20kx5kx1k-50M", dims=[50_000, 20_000, 5_000, 1_000],
            nnz=50_000_000, skew=1.1, R=[32]),
    3: dict(name="planted16-200kx150kx100k-100M", dims=[200_000, 150_000, 100_000],
            nnz=100_000_000, skew=None, R=[16], planted_rank=16, noise_var=0.01),
    4: dict(name="zipf1.1-planted64-1Mx500kx50k-200M", dims=[1_000_000, 500_000, 50_000],
            nnz=200_000_000, skew=1.1, R=[64], planted_rank=64, noise_var=0.01),
}


def _note(*parts):
    # generation steps of the large workloads take tens of seconds each
    if os.environ.get("FCOO_SYNTH_VERBOSE") == "1":
        print("[synth]", *parts, file=sys.stderr, flush=True)


def config_tensor(cfg: int, nnz: Optional[int] = None) -> SparseTensor:
    """The synthetic tensor of workload `cfg`; `nnz` overrides the count
    (same dims and distribution) for scaled-down runs.  With FCOO_SYNTH_CACHE
    naming a directory, generated tensors are kept there as .npz files and
    read back on later calls (same arrays; generation is deterministic)."""
    cache = os.environ.get("FCOO_SYNTH_CACHE")
    path = None
    if cache:
        path = os.path.join(cache, f"synth_cfg{cfg}_{nnz or 'full'}.npz")
        if os.path.exists(path):
            d = np.load(path)
            _note("read", path)
            return SparseTensor(dims=[int(x) for x in d["dims"]], idx=[d[f"i{m}"] for m in range(len(d["dims"]))],
                                vals=d["vals"], name=str(d["name"]))
    t = _make_config_tensor(cfg, nnz)
    if path:
        os.makedirs(cache, exist_ok=True)
        np.savez(path, dims=np.array(t.dims), vals=t.vals, name=np.array(t.name),
                 **{f"i{m}": t.idx[m] for m in range(len(t.dims))})
        _note("wrote", path)
    return t


def _make_config_tensor(cfg: int, nnz: Optional[int]) -> SparseTensor:
    c = CONFIGS[cfg]
    z = c["nnz"] if nnz is None else int(nnz)
    _note("workload", cfg, c["name"], "nnz", z)
    if c.get("planted_rank"):
        base = (zipf_tensor(c["dims"], z, cfg, s=c["skew"], name=c["name"])
                if c["skew"] else uniform_tensor(c["dims"], z, cfg, name=c["name"]))
        P = factors(c["dims"], c["planted_rank"], cfg, role="planted")
        base.vals = planted_values(base.idx, P, c["noise_var"], cfg)
        return base
    if c["skew"]:
        return zipf_tensor(c["dims"], z, cfg, s=c["skew"], name=c["name"])
    return uniform_tensor(c["dims"], z, cfg, name=c["name"])


def random_small(dims, nnz, seed, value_kind="u01", duplicates=False) -> SparseTensor:
    """Small random tensor for parity tests.  With duplicates=True the
    coordinates are drawn with replacement (repeated cells add)."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE, 99, int(seed)])))
    dims = [int(d) for d in dims]
    if duplicates:
        cols = [g.integers(0, d, size=nnz).astype(np.int32) for d in dims]
        if value_kind == "int":
            vals = g.integers(1, 5, size=nnz).astype(np.float64)
        else:
            vals = g.random(nnz)
        return SparseTensor(dims=dims, idx=cols, vals=vals, name="dup")
    total = 1
    for d in dims:
        total *= d
    nnz = min(nnz, total)
    keys = g.choice(total, size=nnz, replace=False).astype(np.uint64)
    cols = _unpack(keys, dims)
    if value_kind == "int":
        vals = g.integers(1, 5, size=nnz).astype(np.float64)
    else:
        vals = g.random(nnz)
    return SparseTensor(dims=dims, idx=[c.astype(np.int32) for c in cols], vals=vals,
                        name="small")


def small_factors(dims, R, seed, kind="normal") -> List[np.ndarray]:
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE, 98, int(seed)])))
    out = []
    for d in dims:
        if kind == "normal":
            out.append(g.standard_normal((int(d), int(R))))
        else:
            out.append(g.integers(-3, 4, size=(int(d), int(R))).astype(np.float64))
    return out
