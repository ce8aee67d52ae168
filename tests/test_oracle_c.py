"""Pins for the C oracle: its plain parallel loops against the NumPy oracle's
pinned definitions and against brute force, exactly on integer data."""
import numpy as np
import pytest

import synth
from oracle import cpu, ref


@pytest.mark.parametrize("dims,Z,R", [([7, 6, 5], 100, 3), ([4, 5, 3, 2], 80, 4), ([30, 20], 200, 1),
                                      ([9, 8, 7, 3, 2], 400, 5)])
@pytest.mark.parametrize("threads", [1, 3])
def test_c_mttkrp_equals_bruteforce(dims, Z, R, threads):
    t = synth.random_small(dims, Z, seed=Z)
    F = synth.small_factors(dims, R, seed=R)
    X = ref.dense_from_coo(dims, t.idx, t.vals)
    for n in range(len(dims)):
        np.testing.assert_allclose(cpu.mttkrp(dims, t.idx, t.vals, F, n, nthreads=threads),
                                   ref.mttkrp_dense(X, F, n), rtol=1e-12, atol=1e-12)


def test_c_mttkrp_exact_on_integers_and_duplicates():
    t = synth.random_small([20, 15, 10], 2000, seed=1, value_kind="int", duplicates=True)
    F = synth.small_factors(t.dims, 8, seed=2, kind="int")
    for n in range(3):
        np.testing.assert_array_equal(cpu.mttkrp(t.dims, t.idx, t.vals, F, n, nthreads=4),
                                      ref.mttkrp_coo(t.dims, t.idx, t.vals, F, n))


@pytest.mark.parametrize("dims", [[6, 5, 4], [3, 4, 5, 2]])
def test_c_ttm_equals_dense(dims):
    t = synth.random_small(dims, 60, seed=3)
    X = ref.dense_from_coo(dims, t.idx, t.vals)
    for n in range(len(dims)):
        U = synth.small_factors([dims[n]], 3, seed=n)[0]
        fib, Y = cpu.ttm(dims, t.idx, t.vals, U, n, nthreads=2)
        f2, Y2 = ref.ttm_coo(dims, t.idx, t.vals, U, n)
        np.testing.assert_array_equal(fib, f2)
        np.testing.assert_allclose(Y, ref.ttm_dense_rows(X, U, n, fib), rtol=1e-12, atol=1e-12)


def test_c_model_and_gradient():
    dims = [7, 6, 5]
    t = synth.random_small(dims, 90, seed=4)
    F = synth.small_factors(dims, 4, seed=5)
    np.testing.assert_allclose(cpu.model_at(t.idx, F), ref.cp_model_at(t.idx, F), rtol=1e-13)
    loss, G = cpu.mse_grad(dims, t.idx, t.vals, F)
    assert abs(loss - ref.mse_loss(t.idx, t.vals, F)) < 1e-13
    for a, b in zip(G, ref.mse_grad(dims, t.idx, t.vals, F)):
        np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-14)
