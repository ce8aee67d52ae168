"""GPU parity of SpTTMc (Eq. 4, Table I third row) against the float64
oracle, through the C ABI: Kronecker rows of the product modes summed per
slice of the SpMTTKRP encoding.  Factors may differ in column count; the
vector path needs the last product mode's count to be a multiple of the
vector width (4 float32 / 8 bfloat16), the scalar path takes any; with the
second-to-last count a multiple of 4 (float32) / 2 (bfloat16) a lane also
owns that many column blocks.  The rank shapes below cover all three."""
import numpy as np
import pytest

import synth
from oracle import ref

from conftest import gpu_available
from gpu_util import TOL_F32, bf16, f32, from_dev, rel_fro, tag, to_dev

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _factors(dims, ranks, seed, kind="normal"):
    g = np.random.default_rng(seed)
    if kind == "int":
        return [g.integers(-3, 4, size=(d, r)).astype(np.float64) for d, r in zip(dims, ranks)]
    return [g.standard_normal((d, r)) for d, r in zip(dims, ranks)]


def _check(t, ranks, mode, dtype="f32", L=16, T=4096, seed=0, kind="normal", exact=False, tol=TOL_F32):
    from paper_1705_09905_amd import Tensor
    F = _factors(t.dims, ranks, seed, kind)
    Fd = [f32(f) if dtype == "f32" else bf16(f) for f in F]
    tag("spttmc", t.dims, t.nnz, "ranks", ranks, "mode", mode, "L", L, "T", T, dtype)
    h = Tensor(t.idx, t.vals, t.dims).build(mode, "mttkrp", threadlen=L, tile_nnz=T)
    dev = [None if m == mode else to_dev(f, dtype) for m, f in enumerate(Fd)]
    Y = from_dev(h.spttmc(mode, dev))
    exp = ref.ttmc_coo(t.dims, t.idx, f32(t.vals), Fd, mode)
    assert Y.shape == exp.shape
    if exact:
        np.testing.assert_array_equal(Y, exp)
    else:
        err = rel_fro(Y, exp)
        assert err <= tol, err
    return h, dev, Y


def test_config0_uniform_200x150x100_all_modes_R8():
    t = synth.config_tensor(0)
    for mode in range(3):
        _check(t, [8, 8, 8], mode, seed=mode)


@pytest.mark.parametrize("ranks", [[4, 4, 4], [8, 16, 4], [3, 5, 7], [16, 16, 16], [32, 32, 32],
                                   [1, 2, 1], [12, 20, 8], [2, 64, 64]])
def test_rank_shapes(ranks):
    t = synth.random_small([50, 40, 30], 20000, seed=sum(ranks))
    for mode in range(3):
        _check(t, ranks, mode, seed=mode)


@pytest.mark.parametrize("ranks", [[8, 8, 8], [4, 4, 4], [16, 8, 24]])
def test_bf16_factors(ranks):
    t = synth.random_small([60, 50, 40], 20000, seed=3)
    for mode in range(3):
        _check(t, ranks, mode, dtype="bf16", seed=mode)


@pytest.mark.parametrize("ranks", [[4, 8, 4], [3, 3, 3], [8, 8, 8]])
def test_integer_data_is_exact(ranks):
    t = synth.random_small([40, 30, 20], 15000, seed=7, value_kind="int")
    for mode in range(3):
        _check(t, ranks, mode, seed=mode, kind="int", exact=True)


@pytest.mark.parametrize("L,T", [(8, 256), (32, 1024), (64, 4096), (16, 8192)])
def test_invariant_to_threadlen_and_tile(L, T):
    t = synth.random_small([30, 200, 100], 30000, seed=9, value_kind="int")
    for mode in range(3):
        _check(t, [4, 4, 4], mode, L=L, T=T, seed=1, kind="int", exact=True)


@pytest.mark.parametrize("dims,ranks", [([8, 7, 6, 5], [4, 4, 4, 4]), ([6, 5, 4, 3, 3], [2, 3, 2, 4, 4]),
                                        ([50, 40], [8, 12]), ([9, 8, 7, 6], [3, 2, 5, 3]),
                                        ([6, 5, 4, 3, 3], [4, 4, 4, 4, 4]), ([7, 6, 5, 4], [8, 2, 8, 8])])
def test_orders_2_to_5(dims, ranks):
    t = synth.random_small(dims, 1500, seed=len(dims))
    for mode in range(len(dims)):
        _check(t, ranks, mode, T=256, seed=mode)


def test_edge_sizes_and_single_slice():
    for Z in [1, 5, 255, 257, 4097]:
        t = synth.random_small([40, 50, 60], Z, seed=Z)
        _check(t, [4, 8, 4], 0, T=256 if Z < 1000 else 4096, seed=Z)
    t = synth.random_small([1, 300, 200], 50000, seed=11)
    _check(t, [4, 8, 8], 0, T=256, seed=3)


def test_empty_tensor_and_errors():
    import torch
    from paper_1705_09905_amd import FcooError, Tensor
    tag("spttmc empty tensor and errors")
    h = Tensor([np.zeros(0, np.int32)] * 3, np.zeros(0), [4, 5, 6]).build(0)
    F = [None, to_dev(np.ones((5, 4))), to_dev(np.ones((6, 4)))]
    Y = torch.full((4, 16), 7.0, device="cuda")
    h.spttmc(0, F, out=Y)
    assert from_dev(Y).sum() == 0.0
    t = synth.random_small([10, 9, 8], 100, seed=1)
    h = Tensor(t.idx, t.vals, t.dims).build(0)
    with pytest.raises(FcooError):   # width 200 * 200 above the limit
        h.spttmc(0, [None, to_dev(np.ones((9, 200))), to_dev(np.ones((8, 200)))])
    with pytest.raises(FcooError):   # the TTM encoding of mode 1 is not built
        h.spttmc(1, [to_dev(np.ones((10, 4))), None, to_dev(np.ones((8, 4)))])


def test_diagonal_columns_equal_spmttkrp_bitwise_inputs():
    # with equal ranks, columns (r, r) of SpTTMc hold the same sums as SpMTTKRP
    t = synth.random_small([60, 50, 40], 20000, seed=5, value_kind="int")
    from paper_1705_09905_amd import Tensor
    F = _factors(t.dims, [8, 8, 8], 5, kind="int")
    h = Tensor(t.idx, t.vals, t.dims).build(1)
    dev = [to_dev(f) for f in F]
    Y = from_dev(h.spttmc(1, [dev[0], None, dev[2]]))
    M = from_dev(h.spmttkrp(1, dev))
    np.testing.assert_array_equal(Y[:, [r * 8 + r for r in range(8)]], M)
