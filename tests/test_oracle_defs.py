"""Pins for the oracle's definitions (Sec. II, Eq. 1-6): each is checked
against something other than itself -- a hand-written example, a library
routine (numpy / scipy / einsum) or a closed form."""
import json
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse

import synth
from oracle import ref

from conftest import GOLDEN


def test_kron_eq1_handworked_and_numpy():
    A = np.array([[1.0, 2.0], [3.0, 4.0]])
    B = np.array([[0.0, 5.0], [6.0, 7.0]])
    expect = np.array([[0, 5, 0, 10], [6, 7, 12, 14], [0, 15, 0, 20], [18, 21, 24, 28]], float)
    np.testing.assert_array_equal(ref.kron(A, B), expect)
    g = np.random.default_rng(1)
    for shp in [((2, 3), (4, 1)), ((1, 1), (3, 2)), ((3, 2), (2, 3))]:
        a, b = g.standard_normal(shp[0]), g.standard_normal(shp[1])
        np.testing.assert_array_equal(ref.kron(a, b), np.kron(a, b))


def test_khatri_rao_eq2_vs_scipy():
    g = np.random.default_rng(2)
    for I, J, R in [(3, 4, 2), (1, 5, 3), (4, 1, 1), (2, 3, 5)]:
        a, b = g.standard_normal((I, R)), g.standard_normal((J, R))
        np.testing.assert_array_equal(ref.khatri_rao(a, b), scipy.linalg.khatri_rao(a, b))


def test_unfold_2x2x2_handworked():
    with open(os.path.join(GOLDEN, "unfold_2x2x2_kolda.json")) as f:
        g = json.load(f)
    X = np.array(g["X"], float)
    for n in range(3):
        np.testing.assert_array_equal(ref.unfold(X, n), np.array(g[f"X{n}"], float))


@pytest.mark.parametrize("dims", [[5, 4, 3], [3, 7, 2], [4, 3, 2, 3], [2, 3, 2, 2, 3], [6, 5]])
@pytest.mark.parametrize("dup", [False, True])
def test_mttkrp_eq5_dense_unfold_krp_equals_eq6_coo(dims, dup):
    t = synth.random_small(dims, 25, seed=len(dims) * 7 + dup, duplicates=dup)
    F = synth.small_factors(dims, 3, seed=len(dims))
    X = ref.dense_from_coo(dims, t.idx, t.vals)
    for n in range(len(dims)):
        dense = ref.mttkrp_dense(X, F, n)
        coo = ref.mttkrp_coo(dims, t.idx, t.vals, F, n)
        np.testing.assert_allclose(coo, dense, rtol=1e-13, atol=1e-13)


def test_mttkrp_3order_vs_einsum():
    t = synth.random_small([6, 5, 4], 60, seed=3)
    A, B, C = synth.small_factors(t.dims, 4, seed=3)
    X = ref.dense_from_coo(t.dims, t.idx, t.vals)
    np.testing.assert_allclose(ref.mttkrp_coo(t.dims, t.idx, t.vals, [A, B, C], 0),
                               np.einsum("ijk,jr,kr->ir", X, B, C), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(ref.mttkrp_coo(t.dims, t.idx, t.vals, [A, B, C], 1),
                               np.einsum("ijk,ir,kr->jr", X, A, C), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(ref.mttkrp_coo(t.dims, t.idx, t.vals, [A, B, C], 2),
                               np.einsum("ijk,ir,jr->kr", X, A, B), rtol=1e-13, atol=1e-13)


def test_mttkrp_order2_is_sparse_matrix_times_dense():
    t = synth.random_small([30, 20], 90, seed=4)
    A0, A1 = synth.small_factors(t.dims, 5, seed=4)
    S = scipy.sparse.coo_matrix((t.vals, (t.idx[0], t.idx[1])), shape=tuple(t.dims)).tocsr()
    np.testing.assert_allclose(ref.mttkrp_coo(t.dims, t.idx, t.vals, [A0, A1], 0), S @ A1,
                               rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(ref.mttkrp_coo(t.dims, t.idx, t.vals, [A0, A1], 1), S.T @ A0,
                               rtol=1e-13, atol=1e-13)


def test_mttkrp_rank1_ones_is_slice_sums():
    t = synth.random_small([9, 8, 7], 100, seed=5)
    ones = [np.ones((d, 1)) for d in t.dims]
    for n in range(3):
        expect = np.bincount(t.idx[n], weights=t.vals, minlength=t.dims[n])
        np.testing.assert_allclose(ref.mttkrp_coo(t.dims, t.idx, t.vals, ones, n)[:, 0], expect,
                                   rtol=1e-14)


def test_mttkrp_single_nonzero_is_scaled_hadamard_row():
    dims = [4, 5, 6]
    idx = [np.array([2]), np.array([3]), np.array([1])]
    vals = np.array([2.5])
    A, B, C = synth.small_factors(dims, 3, seed=6)
    M = ref.mttkrp_coo(dims, idx, vals, [A, B, C], 0)
    expect = np.zeros((4, 3))
    expect[2] = 2.5 * B[3] * C[1]
    np.testing.assert_array_equal(M, expect)


def test_ttm_eq3_vs_dense_tensordot_and_einsum():
    t = synth.random_small([5, 4, 6], 50, seed=7)
    X = ref.dense_from_coo(t.dims, t.idx, t.vals)
    for n in range(3):
        U = synth.small_factors([t.dims[n]], 3, seed=8 + n)[0]
        fib, Y = ref.ttm_coo(t.dims, t.idx, t.vals, U, n)
        np.testing.assert_allclose(Y, ref.ttm_dense_rows(X, U, n, fib), rtol=1e-13, atol=1e-13)
    U = synth.small_factors([6], 2, seed=9)[0]
    fib, Y = ref.ttm_coo(t.dims, t.idx, t.vals, U, 2)
    E = np.einsum("ijk,kr->ijr", X, U)
    np.testing.assert_allclose(Y, E[fib[:, 0], fib[:, 1]], rtol=1e-13, atol=1e-13)


def test_ttm_identity_matrix_gives_dense_fibres_exactly():
    t = synth.random_small([4, 3, 5], 30, seed=10)
    X = ref.dense_from_coo(t.dims, t.idx, t.vals)
    for n in range(3):
        U = np.eye(t.dims[n])
        fib, Y = ref.ttm_coo(t.dims, t.idx, t.vals, U, n)
        for f, y in zip(fib, Y):
            sl = [slice(None)] * 3
            imodes = [m for m in range(3) if m != n]
            for m, c in zip(imodes, f):
                sl[m] = int(c)
            np.testing.assert_array_equal(y, X[tuple(sl)])
        # every structurally non-empty fibre is listed, none more
        present = set(map(tuple, np.stack([t.idx[m] for m in range(3) if m != n], 1).tolist()))
        assert set(map(tuple, fib.tolist())) == present


def test_mode_roles_table1():
    assert ref.mode_roles(3, 2, ref.OP_TTM) == ([0, 1], [2])          # SpTTM mode-3
    assert ref.mode_roles(3, 0, ref.OP_MTTKRP) == ([0], [1, 2])      # SpMTTKRP mode-1
    assert ref.mode_roles(4, 1, ref.OP_MTTKRP) == ([1], [0, 2, 3])
    assert ref.mode_roles(4, 3, ref.OP_TTM) == ([0, 1, 2], [3])
