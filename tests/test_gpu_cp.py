"""GPU parity of the CP-ALS pieces (MFMA Gram, float64 solve, row solve,
normalisation, fit) and of whole sweeps against the float64 oracle of
Algorithm 1, started from the same initial factors.  Bar: the fit of every
sweep within 1e-3 of the oracle's (float32 and bfloat16 factor storage)."""
import numpy as np
import pytest

import synth
from oracle import ref

from conftest import gpu_available
from gpu_util import f32, bf16, from_dev, rel_fro, tag, to_dev

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _lib():
    import paper_1705_09905_amd as P
    return P


@pytest.mark.parametrize("R", [1, 8, 16, 31, 32, 40, 64, 100])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_gram_matches_numpy(R, dtype):
    P = _lib()
    g = np.random.default_rng(R)
    I = 5000
    A = g.standard_normal((I, R))
    Ad = f32(A) if dtype == "f32" else bf16(A)
    t = P.Tensor([np.zeros(1, np.int32), np.zeros(1, np.int32)], [1.0], [I, 3])
    tag("gram", R, dtype)
    G = from_dev(t.gram(0, to_dev(Ad, dtype)))
    exp = Ad.T @ Ad
    assert rel_fro(G, exp) <= 1e-6
    np.testing.assert_allclose(G, G.T, rtol=0, atol=1e-9 * np.abs(exp).max())


def _run_both(t, R, sweeps, dtype="f32", seed=0, dup_column=False):
    P = _lib()
    init = synth.small_factors(t.dims, R, seed=seed)
    if dup_column:
        for a in init:
            a[:, 1] = a[:, 0]
    init_dev = [f32(a) if dtype == "f32" else bf16(a) for a in init]
    h = P.Tensor(t.idx, t.vals, t.dims)
    tag("cp_als", t.dims, t.nnz, "R", R, dtype, "sweeps", sweeps)
    out = P.cp_als(h, R, sweeps, init_dev, dtype=dtype)
    orc = ref.cp_als(t.dims, t.idx, f32(t.vals), R, [a.astype(np.float64) for a in init_dev], sweeps,
                     storage="f64")
    return out, orc


def test_cp_als_config0_fp32_fits_match_oracle():
    t = synth.config_tensor(0)
    out, orc = _run_both(t, 8, 10)
    diffs = np.abs(np.array(out["fits"]) - np.array(orc["fits"]))
    tag("fits", out["fits"][-1], orc["fits"][-1], "max diff", diffs.max())
    assert diffs.max() <= 1e-3
    assert out["used_pinv"] == [0] * 10


def test_cp_als_bf16_reaches_fp64_fit():
    t = synth.config_tensor(0)
    out, orc = _run_both(t, 8, 10, dtype="bf16")
    orc64 = ref.cp_als(t.dims, t.idx, f32(t.vals), 8,
                       [a for a in synth.small_factors(t.dims, 8, seed=0)], 10, storage="f64")
    tag("bf16 fit", out["fits"][-1], "fp64 oracle", orc64["fits"][-1])
    assert abs(out["fits"][-1] - orc64["fits"][-1]) <= 1e-3


def test_cp_als_factors_and_lambda_first_sweep():
    # after one sweep from the same start the factors themselves agree
    t = synth.random_small([30, 25, 20], 3000, seed=5)
    out, orc = _run_both(t, 4, 1)
    for m in range(3):
        assert rel_fro(from_dev(out["factors"][m]), orc["factors"][m]) <= 1e-4
    assert rel_fro(from_dev(out["lam"]), orc["lam"]) <= 1e-4
    G = from_dev(out["grams"])
    for m in range(3):
        assert rel_fro(G[m], orc["grams"][m]) <= 1e-4


def test_cp_als_exact_low_rank_reaches_fit_one():
    Pf = synth.small_factors([12, 10, 8], 3, seed=4)
    X = ref.cp_full(Pf)
    idx = [c.astype(np.int32) for c in np.nonzero(np.ones_like(X))]
    t = synth.SparseTensor(dims=[12, 10, 8], idx=idx, vals=X[tuple(idx)])
    P = _lib()
    h = P.Tensor(t.idx, t.vals, t.dims)
    out = P.cp_als(h, 3, 200, [f32(a) for a in synth.small_factors(t.dims, 3, seed=5)], tol=1e-9)
    tag("exact rank-3 fit", out["fits"][-1])
    assert out["fits"][-1] > 1 - 1e-3


def test_cp_als_rank1_exact_in_one_sweep():
    g = np.random.default_rng(2)
    X = np.einsum("i,j,k->ijk", g.standard_normal(8), g.standard_normal(7), g.standard_normal(6))
    idx = [c.astype(np.int32) for c in np.nonzero(np.ones_like(X))]
    t = synth.SparseTensor(dims=[8, 7, 6], idx=idx, vals=X[tuple(idx)])
    out, orc = _run_both(t, 1, 1)
    tag("rank-1 fit", out["fits"][0])
    assert out["fits"][0] > 1 - 1e-3


def test_cp_als_pseudo_inverse_on_singular_normal_equations():
    # columns 0 and 1 equal in every factor: every Gram, hence V, has two equal
    # rows, and the update keeps them equal, so each mode needs V^+
    t = synth.random_small([20, 12, 15], 800, seed=6)
    out, orc = _run_both(t, 5, 4, dup_column=True)
    tag("pinv flags", out["used_pinv"], orc["used_pinv"])
    assert all(all(p) for p in orc["used_pinv"])
    assert out["used_pinv"] == [0b111] * 4
    assert np.abs(np.array(out["fits"]) - np.array(orc["fits"])).max() <= 1e-3


def test_cp_als_order4():
    t = synth.random_small([30, 20, 10, 8], 8000, seed=7)
    out, orc = _run_both(t, 6, 6)
    assert np.abs(np.array(out["fits"]) - np.array(orc["fits"])).max() <= 1e-3


@pytest.mark.parametrize("R", [2, 5, 12, 24, 40, 64])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_cp_als_ranks_first_sweep_factors_and_fits(R, dtype):
    # ranks that are not powers of two pad the row-solve tiles (R rounded up
    # to 2..64); the first sweep's factors from the same start agree with
    # the oracle's, and the fits track it
    t = synth.random_small([120, 90, 70], 30000, seed=R)
    out, orc = _run_both(t, R, 3, dtype=dtype, seed=R)
    tol = 1e-4 if dtype == "f32" else 2e-2
    if dtype == "f32":
        out1, orc1 = _run_both(t, R, 1, dtype=dtype, seed=R)
        for m in range(3):
            assert rel_fro(from_dev(out1["factors"][m]), orc1["factors"][m]) <= tol
    diffs = np.abs(np.array(out["fits"]) - np.array(orc["fits"]))
    tag("R", R, dtype, "fits", out["fits"], "max diff", diffs.max())
    assert diffs.max() <= 1e-3


def test_cp_als_leaves_caller_init_unchanged():
    # a contiguous CUDA float32 init is copied, not overwritten by the sweeps,
    # so one init can start a float32 run and then a bfloat16 run
    import torch
    P = _lib()
    t = synth.random_small([40, 30, 20], 4000, seed=11)
    h = P.Tensor(t.idx, t.vals, t.dims)
    init = [to_dev(f32(a)) for a in synth.small_factors(t.dims, 6, seed=11)]
    keep = [a.clone() for a in init]
    tag("cp_als init untouched")
    r32 = P.cp_als(h, 6, 3, init, dtype="f32")
    for a, b in zip(init, keep):
        assert torch.equal(a, b)
    r16 = P.cp_als(h, 6, 3, init, dtype="bf16")
    for a, b in zip(init, keep):
        assert torch.equal(a, b)
    orc = ref.cp_als(t.dims, t.idx, f32(t.vals), 6, [from_dev(a) for a in keep], 3)
    assert np.abs(np.array(r32["fits"]) - np.array(orc["fits"])).max() <= 1e-3
    assert np.abs(np.array(r16["fits"]) - np.array(orc["fits"])).max() <= 1e-3
