"""GPU parity of the F-COO SpMTTKRP and SpTTM kernels against the float64
oracle, called through the C ABI (Python binding).  Inputs are the oracle's
inputs rounded to the precision the device reads; the bar is a relative
Frobenius error of 1e-5 (float32 factors), exact equality on integer data
(where every partial sum is an integer below 2^24, any summation order gives
the same float32 result), and bitwise repeatability."""
import numpy as np
import pytest

import synth
from oracle import cpu, ref

from conftest import gpu_available
from gpu_util import TOL_BF16, TOL_F32, bf16, f32, from_dev, rel_fro, tag, to_dev

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _fcoo():
    from paper_1705_09905_amd import Tensor
    return Tensor


def _check_mttkrp(t, R, mode, L=16, T=4096, dtype="f32", seed=0, kind="normal", tol=TOL_F32,
                  exact=False, lane_cols=0):
    Tensor = _fcoo()
    F = synth.small_factors(t.dims, R, seed=seed, kind=kind)
    Fd = [f32(f) if dtype == "f32" else bf16(f) for f in F]
    tag("mttkrp", t.dims, t.nnz, "R", R, "mode", mode, "L", L, "T", T, dtype, "lane_cols", lane_cols)
    h = Tensor(t.idx, t.vals, t.dims).build(mode, "mttkrp", threadlen=L, tile_nnz=T, lane_cols=lane_cols)
    dev = [to_dev(f, dtype) for f in Fd]
    M = from_dev(h.spmttkrp(mode, dev))
    exp = cpu.mttkrp(t.dims, t.idx, f32(t.vals), Fd, mode)
    if exact:
        np.testing.assert_array_equal(M, exp)
    else:
        assert rel_fro(M, exp) <= tol, rel_fro(M, exp)
    return h, dev, M


def _check_ttm(t, R, mode, L=16, T=4096, dtype="f32", seed=0, kind="normal", tol=TOL_F32, exact=False,
               lane_cols=0):
    Tensor = _fcoo()
    U = synth.small_factors([t.dims[mode]], R, seed=seed, kind=kind)[0]
    Ud = f32(U) if dtype == "f32" else bf16(U)
    tag("ttm", t.dims, t.nnz, "R", R, "mode", mode, "L", L, "T", T, dtype, "lane_cols", lane_cols)
    h = Tensor(t.idx, t.vals, t.dims).build(mode, "ttm", threadlen=L, tile_nnz=T, lane_cols=lane_cols)
    Yt, fibd = h.spttm(mode, to_dev(Ud, dtype), return_fibres=True)
    Y = from_dev(Yt)
    fib, exp = cpu.ttm(t.dims, t.idx, f32(t.vals), Ud, mode)
    np.testing.assert_array_equal(h.export(mode, "ttm")["fibres"], fib)
    np.testing.assert_array_equal(fibd, fib)
    if exact:
        np.testing.assert_array_equal(Y, exp)
    else:
        assert rel_fro(Y, exp) <= tol, rel_fro(Y, exp)
    return Y


def test_config0_uniform_200x150x100_all_modes_R8():
    t = synth.config_tensor(0)
    for mode in range(3):
        _check_mttkrp(t, 8, mode, seed=mode)
        _check_ttm(t, 8, mode, seed=mode)


@pytest.mark.parametrize("R", [1, 3, 4, 8, 12, 16, 32, 48, 64, 100, 128, 256])
def test_ranks(R):
    t = synth.random_small([60, 50, 40], 20000, seed=R)
    _check_mttkrp(t, R, 1, seed=R)
    _check_ttm(t, R, 2, seed=R)


@pytest.mark.parametrize("R", [1, 3, 8, 16, 32, 64, 128])
def test_integer_data_is_exact(R):
    t = synth.random_small([40, 30, 20], 15000, seed=100 + R, value_kind="int")
    for mode in range(3):
        _check_mttkrp(t, R, mode, seed=R, kind="int", exact=True)
        _check_ttm(t, R, mode, seed=R, kind="int", exact=True)


@pytest.mark.parametrize("L,T", [(8, 256), (16, 512), (32, 1024), (64, 4096), (16, 8192)])
def test_invariant_to_threadlen_and_tile(L, T):
    t = synth.random_small([30, 200, 100], 30000, seed=7, value_kind="int")
    for mode in range(3):
        _check_mttkrp(t, 16, mode, L=L, T=T, seed=1, kind="int", exact=True)
        _check_ttm(t, 16, mode, L=L, T=T, seed=1, kind="int", exact=True)


@pytest.mark.parametrize("dims,Z", [([2, 3], 5), ([50, 40], 1500), ([8, 7, 6, 5], 1500),
                                     ([6, 5, 4, 3, 3], 1000), ([4, 3, 3, 3, 2, 2, 2, 2], 1500)])
def test_orders_2_to_8(dims, Z):
    t = synth.random_small(dims, Z, seed=len(dims))
    for mode in range(len(dims)):
        _check_mttkrp(t, 8, mode, T=256, seed=mode)
        _check_ttm(t, 8, mode, T=256, seed=mode)


def test_edge_sizes():
    # Z = 1, Z < threadlen, Z = tile exactly, Z = tile + 1, ragged tails
    for Z in [1, 5, 16, 255, 256, 257, 4095, 4096, 4097, 8191]:
        t = synth.random_small([40, 50, 60], Z, seed=Z)
        _check_mttkrp(t, 8, 0, T=256 if Z < 1000 else 4096, seed=Z)
        _check_ttm(t, 8, 1, T=256 if Z < 1000 else 4096, seed=Z)


def test_empty_tensor_writes_zero_rows():
    Tensor = _fcoo()
    import torch
    tag("empty tensor")
    h = Tensor([np.zeros(0, np.int32)] * 3, np.zeros(0), [4, 5, 6]).build(0)
    F = [to_dev(np.ones((d, 8))) for d in (4, 5, 6)]
    M = torch.full((4, 8), 7.0, device="cuda")
    h.spmttkrp(0, F, out=M)
    assert from_dev(M).sum() == 0.0
    h.build(1, "ttm")
    assert h.spttm(1, F[1]).shape == (0, 8)


def test_single_segment_spanning_every_tile():
    # I_0 = 1: one slice holds every nonzero, so the carry chain crosses all tiles
    t = synth.random_small([1, 300, 200], 50000, seed=11)
    _check_mttkrp(t, 16, 0, T=256, seed=3)
    _check_mttkrp(t, 32, 0, T=4096, seed=3)
    t2 = synth.random_small([1, 1, 70000], 60000, seed=12)
    _check_ttm(t2, 8, 2, T=256, seed=4)


def test_every_nonzero_its_own_segment_and_empty_slices():
    # SpMTTKRP on a mode whose indices are all distinct; dims leave empty slices
    g = np.random.default_rng(5)
    Z = 5000
    i0 = g.choice(20000, Z, replace=False).astype(np.int32)
    t = synth.SparseTensor(dims=[20000, 30, 20], idx=[i0, g.integers(0, 30, Z).astype(np.int32),
                                                      g.integers(0, 20, Z).astype(np.int32)],
                           vals=g.random(Z))
    _check_mttkrp(t, 8, 0, T=256)
    _check_mttkrp(t, 32, 0, T=1024)


def test_duplicates_add():
    t = synth.random_small([10, 9, 8], 6000, seed=13, duplicates=True, value_kind="int")
    for mode in range(3):
        _check_mttkrp(t, 8, mode, seed=mode, kind="int", exact=True)
        _check_ttm(t, 8, mode, seed=mode, kind="int", exact=True)


def test_bf16_factors():
    t = synth.random_small([80, 70, 60], 40000, seed=14)
    for R in (8, 16, 32, 64, 128, 12):
        # kernel error: the oracle on the same bf16-rounded factors
        _check_mttkrp(t, R, 0, dtype="bf16", seed=R, tol=TOL_F32)
        _check_ttm(t, R, 1, dtype="bf16", seed=R, tol=TOL_F32)
    # end-to-end: bf16 kernel result against the oracle on the float32 factors
    Tensor = _fcoo()
    F = synth.small_factors(t.dims, 32, seed=15)
    h = Tensor(t.idx, t.vals, t.dims).build(2)
    M = from_dev(h.spmttkrp(2, [to_dev(f, "bf16") for f in F]))
    exp = cpu.mttkrp(t.dims, t.idx, f32(t.vals), [f32(f) for f in F], 2)
    err = rel_fro(M, exp)
    tag("bf16 end-to-end rel error", err)
    assert err <= TOL_BF16


def test_bf16_lane_chunks_exact():
    # bfloat16 SpMTTKRP takes 4-column lane chunks for two product modes and
    # R <= 64 (R a multiple of 4; 1..16 lanes, ragged last lane group), else
    # 8-column chunks; small integers are exact in bfloat16 and in the sums
    t = synth.random_small([50, 40, 30], 20000, seed=16, value_kind="int")
    for R in (4, 12, 20, 36, 60, 64, 72, 136):
        for mode in range(3):
            _check_mttkrp(t, R, mode, dtype="bf16", seed=R + mode, kind="int", exact=True)
    t4 = synth.random_small([12, 10, 9, 8], 6000, seed=17, value_kind="int")
    for mode in range(4):
        _check_mttkrp(t4, 16, mode, dtype="bf16", seed=mode, kind="int", exact=True)


@pytest.mark.parametrize("dims,Z", [([300, 200], 20000), ([50, 40, 30], 20000), ([14, 12, 10, 9], 9000),
                                    ([9, 8, 7, 6, 5], 6000)])
def test_bf16_lane_cols_every_order_exact(dims, Z):
    # both lane chunks the autotuner chooses between, for SpMTTKRP with 1..4
    # product modes (4 columns runs with up to three; with more, and for R not
    # a multiple of 4 or above 64, the build's choice falls back to 8) and for
    # SpTTM; integer data, so any summation order gives the oracle's result
    t = synth.random_small(dims, Z, seed=Z + len(dims), value_kind="int")
    for lc in (4, 8):
        for R in (4, 28, 64, 6):
            for mode in range(len(dims)):
                _check_mttkrp(t, R, mode, T=1024, dtype="bf16", seed=R + mode, kind="int", exact=True,
                              lane_cols=lc)
                _check_ttm(t, R, mode, T=1024, dtype="bf16", seed=R + mode, kind="int", exact=True,
                           lane_cols=lc)


def test_bitwise_repeatable():
    t = synth.zipf_tensor([5000, 4000, 3000], 300000, cfg=21)
    Tensor = _fcoo()
    F = [to_dev(f) for f in synth.small_factors(t.dims, 32, seed=2)]
    for op in ("mttkrp", "ttm"):
        h = Tensor(t.idx, t.vals, t.dims).build(1, op)
        tag("repeat", op)
        run = (lambda: h.spmttkrp(1, F)) if op == "mttkrp" else (lambda: h.spttm(1, F[1]))
        a = run().cpu().numpy()
        for _ in range(3):
            assert np.array_equal(run().cpu().numpy(), a)


def test_spmttkrp_values_is_adjoint_with_replaced_values():
    t = synth.random_small([50, 40, 30], 20000, seed=16)
    Tensor = _fcoo()
    import torch
    F = synth.small_factors(t.dims, 16, seed=17)
    g = np.random.default_rng(3).standard_normal(t.nnz)
    h = Tensor(t.idx, t.vals, t.dims)
    for mode in range(3):
        tag("values", mode)
        h.build(mode)
        M = from_dev(h.spmttkrp_values(mode, torch.tensor(g, dtype=torch.float32, device="cuda"),
                                       [to_dev(f) for f in F]))
        exp = cpu.mttkrp(t.dims, t.idx, f32(g), [f32(f) for f in F], mode)
        assert rel_fro(M, exp) <= TOL_F32


def test_autotune_keeps_fastest_build_and_stays_correct():
    Tensor = _fcoo()
    t = synth.zipf_tensor([3000, 2000, 1000], 200000, cfg=31)
    F = synth.small_factors(t.dims, 16, seed=1)
    Fd = [to_dev(f) for f in F]
    h = Tensor(t.idx, t.vals, t.dims)
    tag("autotune mttkrp mode 1")
    r = h.autotune(1, "mttkrp", Fd, tiles=[512, 2048, 8192])
    assert r["tile_nnz"] in (512, 2048, 8192) and r["ms"] > 0
    assert h.info(1)["tile_nnz"] == r["tile_nnz"]
    M = from_dev(h.spmttkrp(1, Fd))
    assert rel_fro(M, cpu.mttkrp(t.dims, t.idx, f32(t.vals), [f32(f) for f in F], 1)) <= TOL_F32
    tag("autotune ttm mode 2")
    r = h.autotune(2, "ttm", Fd)
    assert r["tile_nnz"] in (1024, 2048, 4096, 8192, 16384)
    assert h.info(2, "ttm")["tile_nnz"] == r["tile_nnz"]
    _, Y = cpu.ttm(t.dims, t.idx, f32(t.vals), f32(F[2]), 2)
    assert rel_fro(from_dev(h.spttm(2, Fd[2])), Y) <= TOL_F32
    # bfloat16 factors: the lane chunk is searched too, and XCD blocks by each product mode
    Fb = [to_dev(f, "bf16") for f in F]
    for mode in range(3):
        tag("autotune bf16 mttkrp mode", mode)
        r = h.autotune(mode, "mttkrp", Fb, tiles=[2048])
        inf = h.info(mode)
        assert r["lane_cols"] in (4, 8) and inf["lane_cols"] == r["lane_cols"]
        assert inf["xcd_blocks"] == max(1, r["xcd_blocks"])
        if r["xcd_blocks"] > 1:
            assert inf["block_mode"] == r["xcd_mode"] and r["xcd_mode"] != mode
        M = from_dev(h.spmttkrp(mode, Fb))
        assert rel_fro(M, cpu.mttkrp(t.dims, t.idx, f32(t.vals), [bf16(f) for f in F], mode)) <= TOL_F32


def test_device_copy_is_exact():
    import torch
    from paper_1705_09905_amd import _lib as L
    import ctypes as C
    for n in (16, 4096 + 48, (1 << 24) + 16 * 7):
        tag("device copy bytes", n)
        src = torch.randint(0, 255, (n,), dtype=torch.uint8, device="cuda")
        dst = torch.zeros_like(src)
        L.check(L.fcoo_device_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), n,
                                   C.c_void_p(torch.cuda.current_stream().cuda_stream)))
        torch.cuda.synchronize()
        assert torch.equal(src, dst)
