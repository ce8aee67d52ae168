"""SpMTTKRP builds split into per-XCD blocks (fcoo_opts.xcd_blocks = 8):
results against the float64 oracle for every operation that reads a
SpMTTKRP build (plain, bfloat16, integer-exact, several rank tiles, SpTTMc,
value-replaced and fused residual forms, CP-ALS), the GPU build against the
host build bit for bit, and small and empty tensors where blocks hold no
tile."""
import numpy as np
import pytest
import torch

import synth
from oracle import cpu, ref

from conftest import gpu_available
from gpu_util import TOL_F32, bf16, f32, from_dev, rel_fro, tag, to_dev

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _T():
    from paper_1705_09905_amd import Tensor
    return Tensor


@pytest.mark.parametrize("kind,dims,Z", [("uniform", [300, 400, 500], 200000), ("zipf", [3000, 2000, 1000], 200000),
                                         ("uniform", [40, 30, 20, 50], 30000)])
@pytest.mark.parametrize("R", [16, 32, 256])
def test_blocked_spmttkrp_every_mode(kind, dims, Z, R):
    t = (synth.uniform_tensor(dims, Z, cfg=61) if kind == "uniform" else synth.zipf_tensor(dims, Z, cfg=62))
    F = synth.small_factors(t.dims, R, seed=R)
    Fd = [to_dev(f) for f in F]
    for mode in range(len(dims)):
        tag("blocked spmttkrp", kind, dims, "R", R, "mode", mode)
        h = _T()(t.idx, t.vals, t.dims).build(mode, tile_nnz=2048, xcd_blocks=8)
        assert h.info(mode)["xcd_blocks"] == 8
        M = from_dev(h.spmttkrp(mode, Fd))
        assert rel_fro(M, cpu.mttkrp(t.dims, t.idx, f32(t.vals), [f32(f) for f in F], mode)) <= TOL_F32


def test_blocked_integer_exact_bf16_and_device_build():
    t = synth.random_small([60, 500, 400], 60000, seed=3, value_kind="int")
    F = synth.small_factors(t.dims, 16, seed=3, kind="int")
    for mode in range(3):
        tag("blocked exact / device build", mode)
        hh = _T()(t.idx, t.vals, t.dims).build(mode, tile_nnz=1024, xcd_blocks=8)
        hd = _T()(t.idx, t.vals, t.dims).build(mode, tile_nnz=1024, xcd_blocks=8, device=True)
        a, b = hh.export(mode), hd.export(mode)
        for k in ("val", "bf", "sf", "tile_seg0", "perm", "seg_row"):
            np.testing.assert_array_equal(a[k], b[k], err_msg=k)
        exp = cpu.mttkrp(t.dims, t.idx, f32(t.vals), F, mode)
        np.testing.assert_array_equal(from_dev(hh.spmttkrp(mode, [to_dev(f) for f in F])), exp)
        np.testing.assert_array_equal(from_dev(hd.spmttkrp(mode, [to_dev(f) for f in F])), exp)
        Fb = [bf16(f) for f in synth.small_factors(t.dims, 32, seed=4)]
        M = from_dev(hh.spmttkrp(mode, [to_dev(f, "bf16") for f in Fb]))
        assert rel_fro(M, cpu.mttkrp(t.dims, t.idx, f32(t.vals), Fb, mode)) <= TOL_F32


def test_blocked_small_and_empty():
    for Z in (1, 7, 300):
        t = synth.random_small([30, 40, 50], Z, seed=Z)
        F = synth.small_factors(t.dims, 8, seed=Z)
        tag("blocked small", Z)
        h = _T()(t.idx, t.vals, t.dims).build(1, tile_nnz=256, xcd_blocks=8)
        M = from_dev(h.spmttkrp(1, [to_dev(f) for f in F]))
        assert rel_fro(M, cpu.mttkrp(t.dims, t.idx, f32(t.vals), [f32(f) for f in F], 1)) <= TOL_F32
    h = _T()([np.zeros(0, np.int32)] * 3, np.zeros(0), [4, 5, 6]).build(0, xcd_blocks=8)
    M = torch.full((4, 8), 7.0, device="cuda")
    h.spmttkrp(0, [to_dev(np.ones((d, 8))) for d in (4, 5, 6)], out=M)
    assert from_dev(M).sum() == 0.0


def test_blocked_spttmc_values_resid_and_cp_als():
    from paper_1705_09905_amd import cp_als
    t = synth.zipf_tensor([2000, 1500, 1000], 150000, cfg=63)
    F = synth.small_factors(t.dims, 16, seed=5)
    Fd = [to_dev(f) for f in F]
    h = _T()(t.idx, t.vals, t.dims)
    for m in range(3):
        h.build(m, tile_nnz=2048, xcd_blocks=8)
    tag("blocked spttmc")
    Y = from_dev(h.spttmc(0, [None, Fd[1], Fd[2]]))
    assert rel_fro(Y, ref.ttmc_coo(t.dims, t.idx, f32(t.vals), [None, f32(F[1]), f32(F[2])], 0)) <= TOL_F32
    tag("blocked values / resid")
    g = np.random.default_rng(2).standard_normal(t.nnz)
    M = from_dev(h.spmttkrp_values(1, torch.tensor(g, dtype=torch.float32, device="cuda"), Fd))
    assert rel_fro(M, cpu.mttkrp(t.dims, t.idx, f32(g), [f32(f) for f in F], 1)) <= TOL_F32
    loss = torch.zeros((), dtype=torch.float64, device="cuda")
    exp_loss, exp_g = cpu.mse_grad(t.dims, t.idx, f32(t.vals), [f32(f) for f in F])
    for m in range(3):
        G = from_dev(h.resid_spmttkrp(m, Fd, loss=loss))
        assert rel_fro(G, exp_g[m]) <= TOL_F32
    assert abs(loss.item() - exp_loss) <= 1e-5 * exp_loss
    tag("blocked cp-als")
    init = synth.small_factors(t.dims, 8, seed=6)
    out = cp_als(h, 8, 4, [f32(a) for a in init], build=False)
    orc = ref.cp_als(t.dims, t.idx, f32(t.vals), 8, [f32(a) for a in init], 4,
                     mttkrp=lambda d, i, v, Fm, n: cpu.mttkrp(d, i, v, Fm, n))
    assert np.abs(np.array(out["fits"]) - np.array(orc["fits"])).max() <= 1e-3
