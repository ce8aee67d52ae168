"""Pins for the oracle's CP-ALS (Algorithm 1), its solve, fit and precision
forms, and for the gradient-based sparse CP pieces: closed forms (rank-1
exact in one sweep), invariants (ALS never increases the residual), library
routines (LAPACK, torch autograd, torch.optim.Adam, torch's bfloat16 cast)
and finite differences."""
import numpy as np
import pytest
import torch

import synth
from oracle import ref


def _full_tensor(X):
    idx = [c.astype(np.int32) for c in np.nonzero(np.ones_like(X))]
    return idx, X[tuple(idx)]


def test_cholesky_and_solve_vs_lapack():
    g = np.random.default_rng(0)
    for R in (1, 3, 8, 17):
        B = g.standard_normal((R + 5, R))
        V = B.T @ B + 0.1 * np.eye(R)
        np.testing.assert_allclose(ref.cholesky(V), np.linalg.cholesky(V), rtol=1e-12, atol=1e-12)
        M = g.standard_normal((11, R))
        A, p = ref.solve_rows(V, M)
        assert not p
        np.testing.assert_allclose(A, np.linalg.solve(V, M.T).T, rtol=1e-10, atol=1e-12)


def test_singular_v_uses_pseudoinverse_like_lapack():
    g = np.random.default_rng(1)
    B = g.standard_normal((6, 3))
    B = np.concatenate([B, B[:, :1]], axis=1)  # duplicated column -> rank 3 of 4
    V = B.T @ B
    M = g.standard_normal((5, 4))
    A, p = ref.solve_rows(V, M)
    assert p
    np.testing.assert_allclose(A, M @ np.linalg.pinv(V), rtol=1e-8, atol=1e-10)


def test_rank1_tensor_fit_one_after_one_sweep():
    g = np.random.default_rng(2)
    a, b, c = g.standard_normal(4), g.standard_normal(5), g.standard_normal(3)
    X = np.einsum("i,j,k->ijk", a, b, c)
    idx, vals = _full_tensor(X)
    init = synth.small_factors(X.shape, 1, seed=3)
    out = ref.cp_als(list(X.shape), idx, vals, 1, init, sweeps=1)
    # the model is exact after one sweep ...
    Xh = ref.cp_full(out["factors"], out["lam"])
    assert np.linalg.norm(X - Xh) <= 1e-13 * np.linalg.norm(X)
    # ... and the cancelling fit formula loses about half the digits of float64
    assert out["fits"][0] > 1 - 1e-7


def test_exact_rank_r_tensor_reaches_fit_one():
    P = synth.small_factors([12, 10, 8], 3, seed=4)
    X = ref.cp_full(P)
    idx, vals = _full_tensor(X)
    init = synth.small_factors(X.shape, 3, seed=5)
    out = ref.cp_als(list(X.shape), idx, vals, 3, init, sweeps=300, tol=1e-12)
    assert out["fits"][-1] > 1 - 1e-6


def test_fit_formula_equals_direct_residual_and_als_is_monotone():
    t = synth.random_small([6, 5, 4], 60, seed=6)
    X = ref.dense_from_coo(t.dims, t.idx, t.vals)
    init = synth.small_factors(t.dims, 3, seed=7)
    prev = -np.inf
    for s in range(1, 8):
        out = ref.cp_als(t.dims, t.idx, t.vals, 3, init, sweeps=s)
        Xh = ref.cp_full(out["factors"], out["lam"])
        direct = 1 - np.linalg.norm(X - Xh) / np.linalg.norm(X)
        assert abs(direct - out["fits"][-1]) < 1e-10
        assert out["fits"][-1] >= prev - 1e-12
        prev = out["fits"][-1]


def test_mode_update_is_the_least_squares_solution():
    # after updating mode n, A_n diag(lam) minimises ||X_(n) - A (kr A_m)^T||
    t = synth.random_small([5, 4, 6], 50, seed=8)
    X = ref.dense_from_coo(t.dims, t.idx, t.vals)
    init = synth.small_factors(t.dims, 2, seed=9)
    A = [a.copy() for a in init]
    G = [a.T @ a for a in A]
    M = ref.mttkrp_coo(t.dims, t.idx, t.vals, A, 0)
    V = G[1] * G[2]
    An, _ = ref.solve_rows(V, M)
    K = ref.krp_for_mode(A, 0)
    lsq = np.linalg.lstsq(K, ref.unfold(X, 0).T, rcond=None)[0].T
    np.testing.assert_allclose(An, lsq, rtol=1e-9, atol=1e-11)


def test_normalize_zero_column():
    A = np.array([[3.0, 0.0], [4.0, 0.0]])
    B, lam = ref.normalize_columns(A)
    np.testing.assert_array_equal(lam, [5.0, 0.0])
    np.testing.assert_array_equal(B, [[0.6, 0.0], [0.8, 0.0]])


def test_bf16_round_matches_torch_cast():
    g = np.random.default_rng(10)
    x = np.concatenate([g.standard_normal(20000) * 10.0 ** g.integers(-8, 8, 20000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, -3.0e-39]])
    t = torch.tensor(x, dtype=torch.float64).to(torch.float32).to(torch.bfloat16).to(torch.float64)
    np.testing.assert_array_equal(ref.bf16_round(x), t.numpy())


def test_model_at_nonzeros_vs_dense_cp():
    P = synth.small_factors([5, 4, 3], 2, seed=11)
    t = synth.random_small([5, 4, 3], 30, seed=11)
    X = ref.cp_full(P)
    np.testing.assert_allclose(ref.cp_model_at(t.idx, P), X[tuple(t.idx)], rtol=1e-13)


@pytest.mark.parametrize("dims", [[5, 4, 3], [3, 4, 2, 3]])
def test_mse_gradient_vs_finite_differences(dims):
    t = synth.random_small(dims, 25, seed=12)
    F = synth.small_factors(dims, 2, seed=13)
    G = ref.mse_grad(dims, t.idx, t.vals, F)
    h = 1e-6
    for m in range(len(dims)):
        for (i, r) in [(0, 0), (dims[m] - 1, 1), (1, 1)]:
            Fp = [f.copy() for f in F]
            Fm = [f.copy() for f in F]
            Fp[m][i, r] += h
            Fm[m][i, r] -= h
            fd = (ref.mse_loss(t.idx, t.vals, Fp) - ref.mse_loss(t.idx, t.vals, Fm)) / (2 * h)
            assert abs(fd - G[m][i, r]) <= 1e-6 * max(1.0, abs(fd))


def test_mse_gradient_vs_torch_autograd_of_dense_model_on_observed_entries():
    dims = [4, 5, 3]
    t = synth.random_small(dims, 20, seed=14)
    F = synth.small_factors(dims, 3, seed=15)
    T = [torch.tensor(f, dtype=torch.float64, requires_grad=True) for f in F]
    full = torch.einsum("ir,jr,kr->ijk", *T)
    ii = [torch.tensor(i, dtype=torch.long) for i in t.idx]
    r = full[ii[0], ii[1], ii[2]] - torch.tensor(t.vals)
    loss = 0.5 * (r * r).sum() / t.nnz
    loss.backward()
    G = ref.mse_grad(dims, t.idx, t.vals, F)
    assert abs(loss.item() - ref.mse_loss(t.idx, t.vals, F)) < 1e-14
    for m in range(3):
        np.testing.assert_allclose(G[m], T[m].grad.numpy(), rtol=1e-12, atol=1e-14)


def test_mse_gradient_zero_at_noiseless_planted_optimum():
    dims = [6, 5, 4]
    P = synth.small_factors(dims, 2, seed=16)
    t = synth.random_small(dims, 40, seed=17)
    vals = ref.cp_model_at(t.idx, P)
    G = ref.mse_grad(dims, t.idx, vals, P)
    for g in G:
        assert np.abs(g).max() < 1e-14


def test_adam_vs_torch_optim():
    g = np.random.default_rng(18)
    p = [g.standard_normal((4, 3)), g.standard_normal((2, 3))]
    tp = [torch.tensor(x.copy(), requires_grad=True) for x in p]
    opt = torch.optim.Adam(tp, lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    m = [np.zeros_like(x) for x in p]
    v = [np.zeros_like(x) for x in p]
    for step in range(1, 6):
        grads = [g.standard_normal(x.shape) for x in p]
        p, m, v = ref.adam_step(p, grads, m, v, step)
        for t_, gr in zip(tp, grads):
            t_.grad = torch.tensor(gr)
        opt.step()
    for a, b in zip(p, tp):
        np.testing.assert_allclose(a, b.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_observed_fit_hand_worked():
    # the observed-entry fit of a 2 x 3 tensor with three nonzeros, worked by
    # hand (tests/golden/observed_fit_2x3_handworked.json)
    import json
    import os
    from conftest import GOLDEN
    with open(os.path.join(GOLDEN, "observed_fit_2x3_handworked.json")) as f:
        d = json.load(f)
    idx = [np.array(c, np.int32) for c in d["idx"]]
    A = [np.array(d["A0"], np.float64), np.array(d["A1"], np.float64)]
    np.testing.assert_array_equal(ref.cp_model_at(idx, A), d["xhat"])
    assert abs(ref.observed_fit(idx, d["vals"], A) - d["fit"]) <= 1e-10
    # the same with the model from the C loop (the form the full-size tests use)
    from oracle import cpu
    assert abs(ref.observed_fit(idx, d["vals"], A, model=cpu.model_at) - d["fit"]) <= 1e-10
    # an exact model fits 1, a zero model fits 0
    assert ref.observed_fit(idx, d["xhat"], A) == 1.0
    assert abs(ref.observed_fit(idx, d["vals"], [0 * a for a in A])) <= 1e-15


def _one_sweep_by_hand(X, init, rnd):
    """One Gauss-Seidel sweep of Algorithm 1 on a dense tensor, written with
    other primitives than the oracle: MTTKRP as the dense unfolding times
    scipy's Khatri-Rao product (Eq. 5), the R x R system by LAPACK's general
    solver, column 2-norms by numpy, and the stored factor rounded by `rnd`
    (a torch cast).  Returns the stored factors, lambda and the fit from the
    dense residual."""
    from scipy.linalg import khatri_rao
    N = X.ndim
    A = [rnd(a) for a in init]
    for n in range(N):
        Xn = np.reshape(np.moveaxis(X, n, 0), (X.shape[n], -1), order="F")
        others = [m for m in range(N) if m != n]
        K = A[others[-1]]
        for m in reversed(others[:-1]):
            K = khatri_rao(K, A[m])
        M = Xn @ K
        V = np.ones((A[0].shape[1],) * 2)
        for m in others:
            V = V * (A[m].T @ A[m])
        An = np.linalg.solve(V, M.T).T
        lam = np.linalg.norm(An, axis=0)
        A[n] = rnd(An / lam)
    Xh = ref.cp_full(A, lam)
    return A, lam, 1.0 - np.linalg.norm(X - Xh) / np.linalg.norm(X)


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_cp_als_storage_forms_match_one_sweep_by_hand(storage):
    # the reduced-precision forms of the oracle's CP-ALS round each updated
    # factor after normalisation and feed the rounded values to the next
    # mode's product and Gram; pinned against a by-hand sweep that rounds
    # through torch's own casts
    def rnd(a):
        tdt = torch.float32 if storage == "f32" else torch.bfloat16
        return torch.tensor(a, dtype=torch.float64).to(tdt).to(torch.float64).numpy()

    g = np.random.default_rng(21)
    dims = [7, 6, 5]
    X = np.where(g.random(dims) < 0.4, g.random(dims), 0.0)
    idx = [c.astype(np.int32) for c in np.nonzero(X)]
    vals = X[tuple(idx)]
    R = 3
    init = synth.small_factors(dims, R, seed=22)
    out = ref.cp_als(dims, idx, vals, R, init, sweeps=1, storage=storage)
    A, lam, fit = _one_sweep_by_hand(X, init, rnd)
    for m in range(3):
        np.testing.assert_allclose(out["factors"][m], A[m], rtol=1e-9, atol=1e-12)
        # the stored factors are exactly representable in the storage type
        np.testing.assert_array_equal(rnd(out["factors"][m]), out["factors"][m])
        np.testing.assert_array_equal(out["grams"][m], out["factors"][m].T @ out["factors"][m])
    np.testing.assert_allclose(out["lam"], lam, rtol=1e-9)
    assert abs(out["fits"][0] - fit) <= 1e-9
    # rounding changes the result: the float64 form differs from the stored one
    f64 = ref.cp_als(dims, idx, vals, R, init, sweeps=1, storage="f64")
    assert np.abs(f64["factors"][0] - out["factors"][0]).max() > 0
