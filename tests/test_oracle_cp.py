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
