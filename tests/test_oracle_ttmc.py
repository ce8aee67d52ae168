"""Pins for the oracle's SpTTMc (Eq. 4, Table I third row): the COO loop of
Kronecker rows is checked against the explicit Kronecker product of Eq. (1)
applied to an unfolding, a chain of dense TTMs, a hand-worked example,
identity factors (the result is then the tensor itself), the sparse-matrix
product for order 2, and the diagonal columns that equal SpMTTKRP."""
import numpy as np
import pytest
import scipy.sparse

import synth
from oracle import ref


def _unfold_kron_order(X, n):
    # Y_(n) column order of Eq. (4): the other modes ascending, the last fastest
    return np.moveaxis(X, n, 0).reshape(X.shape[n], -1)


def _kron_chain(factors, n):
    out = None
    for m, U in enumerate(factors):
        if m != n:
            out = U if out is None else ref.kron(out, U)
    return out


def test_ttmc_handworked_2x2x2():
    # X(0,0,1) = 2, X(1,1,0) = 3; U_1 = [[1,2],[3,4]], U_2 = [[5],[6]]
    # mode 0: row 0 = 2 * (U_1[0] kron U_2[1]) = 2 * [6, 12] = [12, 24]
    #         row 1 = 3 * (U_1[1] kron U_2[0]) = 3 * [15, 20] = [45, 60]
    idx = [np.array([0, 1]), np.array([0, 1]), np.array([1, 0])]
    vals = np.array([2.0, 3.0])
    U = [np.zeros((2, 1)), np.array([[1.0, 2.0], [3.0, 4.0]]), np.array([[5.0], [6.0]])]
    Y = ref.ttmc_coo([2, 2, 2], idx, vals, U, 0)
    np.testing.assert_array_equal(Y, [[12.0, 24.0], [45.0, 60.0]])


@pytest.mark.parametrize("dims,ranks", [([5, 4, 3], [2, 3, 2]), ([3, 6, 2, 4], [2, 2, 3, 2]),
                                        ([4, 3], [3, 5]), ([2, 3, 2, 2, 3], [2, 1, 2, 2, 2])])
@pytest.mark.parametrize("dup", [False, True])
def test_ttmc_equals_unfolding_times_explicit_kron_and_dense_chain(dims, ranks, dup):
    t = synth.random_small(dims, 30, seed=len(dims) * 5 + dup, duplicates=dup)
    g = np.random.default_rng(len(dims))
    F = [g.standard_normal((d, r)) for d, r in zip(dims, ranks)]
    X = ref.dense_from_coo(dims, t.idx, t.vals)
    for n in range(len(dims)):
        coo = ref.ttmc_coo(dims, t.idx, t.vals, F, n)
        assert coo.shape == (dims[n], ref.ttmc_width(F, n))
        np.testing.assert_allclose(coo, _unfold_kron_order(X, n) @ _kron_chain(F, n), rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(coo, ref.ttmc_dense(X, F, n), rtol=1e-12, atol=1e-12)


def test_ttmc_identity_factors_reproduce_the_tensor():
    dims = [4, 5, 3]
    t = synth.random_small(dims, 40, seed=2)
    X = ref.dense_from_coo(dims, t.idx, t.vals)
    F = [np.eye(d) for d in dims]
    for n in range(3):
        np.testing.assert_array_equal(ref.ttmc_coo(dims, t.idx, t.vals, F, n), _unfold_kron_order(X, n))


def test_ttmc_order2_is_sparse_matrix_product():
    t = synth.random_small([30, 20], 120, seed=4)
    U1 = np.random.default_rng(4).standard_normal((20, 6))
    S = scipy.sparse.coo_matrix((t.vals, (t.idx[0], t.idx[1])), shape=(30, 20)).tocsr()
    np.testing.assert_allclose(ref.ttmc_coo(t.dims, t.idx, t.vals, [None, U1], 0), S @ U1, rtol=1e-13, atol=1e-13)


def test_ttmc_diagonal_columns_are_mttkrp():
    # with equal ranks, column (r, r, ..., r) of Y_(n) is column r of M (Eq. 6)
    for dims in ([6, 5, 4], [4, 3, 3, 2]):
        t = synth.random_small(dims, 50, seed=len(dims))
        R = 3
        F = synth.small_factors(dims, R, seed=9)
        for n in range(len(dims)):
            Y = ref.ttmc_coo(dims, t.idx, t.vals, F, n)
            M = ref.mttkrp_coo(dims, t.idx, t.vals, F, n)
            k = len(dims) - 1
            diag = [sum(r * R ** (k - 1 - q) for q in range(k)) for r in range(R)]
            np.testing.assert_allclose(Y[:, diag], M, rtol=1e-14, atol=1e-14)


def test_ttmc_integer_data_exact_and_empty():
    dims = [7, 6, 5]
    t = synth.random_small(dims, 80, seed=5, value_kind="int")
    F = synth.small_factors(dims, 3, seed=5, kind="int")
    X = ref.dense_from_coo(dims, t.idx, t.vals)
    for n in range(3):
        np.testing.assert_array_equal(ref.ttmc_coo(dims, t.idx, t.vals, F, n),
                                      _unfold_kron_order(X, n) @ _kron_chain(F, n))
    empty = ref.ttmc_coo(dims, [np.zeros(0, int)] * 3, np.zeros(0), F, 1)
    assert empty.shape == (6, 9) and not empty.any()
