"""GPU parity of the single-pass variant (fcoo_opts.single_pass: segments that
cross tiles are finished inside the tile kernel from published boundary
partials, the paper's adjacent synchronization of Sec. IV-D, instead of the
fix-up pass) against the float64 oracle and against the fix-up pass: integer
data (every partial sum an integer below 2^24, so any summation order gives
the oracle's value exactly), chains across every tile, empty slices, repeated
launches at changing ranks (the launch tags and the word buffer's growth),
every operation of the tile kernel (SpMTTKRP, SpTTM, SpTTMc, value-replaced
and fused residual SpMTTKRP) and CP-ALS; no bounded wait may give up."""
import numpy as np
import pytest

import synth
from oracle import cpu, ref

from conftest import gpu_available
from gpu_util import TOL_F32, f32, from_dev, rel_fro, tag, to_dev

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _T():
    from paper_1705_09905_amd import Tensor
    return Tensor


def _both(t, mode, op, T):
    h1 = _T()(t.idx, t.vals, t.dims).build(mode, op, tile_nnz=T, single_pass=True)
    h0 = _T()(t.idx, t.vals, t.dims).build(mode, op, tile_nnz=T)
    assert h1.info(mode, op)["single_pass"] == 1 and h0.info(mode, op)["single_pass"] == 0
    return h1, h0


def _no_give_up(h, mode, op="mttkrp"):
    assert h.info(mode, op)["sp_gave_up"] == 0


@pytest.mark.parametrize("shape", ["zipf", "uniform", "one-slice"])
def test_single_pass_integer_exact(shape):
    if shape == "zipf":
        t = synth.zipf_tensor([3000, 2000, 1000], 200000, cfg=41, value_kind="int")
    elif shape == "uniform":
        t = synth.random_small([200, 150, 100], 150000, seed=42, value_kind="int")
    else:   # one slice of mode 0 holds every nonzero: one chain over all tiles
        t = synth.random_small([1, 300, 200], 50000, seed=43, value_kind="int")
    for T in (256, 4096):
        for R in (1, 8, 32, 100):
            F = [f32(f) for f in synth.small_factors(t.dims, R, seed=R, kind="int")]
            Fd = [to_dev(f) for f in F]
            for mode in range(3):
                tag("single pass", shape, "T", T, "R", R, "mode", mode)
                h1, h0 = _both(t, mode, "mttkrp", T)
                exp = cpu.mttkrp(t.dims, t.idx, f32(t.vals), F, mode)
                np.testing.assert_array_equal(from_dev(h1.spmttkrp(mode, Fd)), exp)
                np.testing.assert_array_equal(from_dev(h0.spmttkrp(mode, Fd)), exp)
                _no_give_up(h1, mode)
                if shape != "one-slice" or mode == 0:
                    g1, _ = _both(t, mode, "ttm", T)
                    fib, Y = cpu.ttm(t.dims, t.idx, f32(t.vals), F[mode], mode)
                    np.testing.assert_array_equal(from_dev(g1.spttm(mode, Fd[mode])), Y)
                    _no_give_up(g1, mode, "ttm")


def test_single_pass_float_edges_and_repeated_launches():
    import torch
    # Z = 1 .. ragged tails, tiny tiles; then repeated launches with changing R
    for Z in (1, 5, 255, 256, 257, 4097):
        t = synth.random_small([40, 50, 60], Z, seed=Z)
        F = synth.small_factors(t.dims, 8, seed=Z)
        h = _T()(t.idx, t.vals, t.dims).build(0, tile_nnz=256, single_pass=True)
        tag("single pass edge Z", Z)
        M = from_dev(h.spmttkrp(0, [to_dev(f) for f in F]))
        assert rel_fro(M, cpu.mttkrp(t.dims, t.idx, f32(t.vals), [f32(f) for f in F], 0)) <= TOL_F32
        _no_give_up(h, 0)
    t = synth.zipf_tensor([5000, 4000, 3000], 300000, cfg=44)
    h = _T()(t.idx, t.vals, t.dims).build(1, tile_nnz=1024, single_pass=True)
    for R in (8, 32, 8, 64, 32):
        F = synth.small_factors(t.dims, R, seed=R)
        Fd = [to_dev(f) for f in F]
        exp = cpu.mttkrp(t.dims, t.idx, f32(t.vals), [f32(f) for f in F], 1)
        for _ in range(3):
            tag("single pass repeated R", R)
            M = torch.full((t.dims[1], R), float("nan"), device="cuda")
            h.spmttkrp(1, Fd, out=M)
            assert rel_fro(from_dev(M), exp) <= TOL_F32
    _no_give_up(h, 1)


def test_single_pass_every_operation_and_cp_als():
    import torch
    from paper_1705_09905_amd import cp_als
    t = synth.zipf_tensor([3000, 2000, 1000], 200000, cfg=45)
    R = 16
    F = synth.small_factors(t.dims, R, seed=3)
    Fh = [f32(f) for f in F]
    Fd = [to_dev(f) for f in F]
    h = _T()(t.idx, t.vals, t.dims)
    for m in range(3):
        h.build(m, tile_nnz=1024, single_pass=True)
    vals = f32(t.vals)
    for m in range(3):
        tag("single pass spttmc / values / resid, mode", m)
        ranks = [4, 4, 4]
        Fk = [to_dev(synth.small_factors([d], 4, seed=9 + k)[0]) for k, d in enumerate(t.dims)]
        Y = from_dev(h.spttmc(m, [None if k == m else Fk[k] for k in range(3)]))
        exp = ref.ttmc_coo(t.dims, t.idx, vals, [from_dev(x) for x in Fk], m)
        assert rel_fro(Y, exp) <= TOL_F32
        g = np.random.default_rng(m).standard_normal(t.nnz)
        Mv = from_dev(h.spmttkrp_values(m, torch.tensor(g, dtype=torch.float32, device="cuda"), Fd))
        assert rel_fro(Mv, cpu.mttkrp(t.dims, t.idx, f32(g), Fh, m)) <= TOL_F32
        G = torch.empty((t.dims[m], R), device="cuda")
        h.resid_spmttkrp(m, Fd, out=G)
        _, exp_g = cpu.mse_grad(t.dims, t.idx, vals, Fh)
        assert rel_fro(from_dev(G), exp_g[m]) <= TOL_F32
        _no_give_up(h, m)
    init = [f32(a) for a in synth.factors(t.dims, R, cfg=45, role="init")]
    tag("single pass cp-als")
    fits = cp_als(h, R, 3, init, build=False)["fits"]
    orc = ref.cp_als(t.dims, t.idx, vals, R, init, 3)["fits"]
    assert max(abs(a - b) for a, b in zip(fits, orc)) <= 1e-4
    for m in range(3):
        _no_give_up(h, m)


def test_single_pass_refuses_xcd_blocks():
    from paper_1705_09905_amd import _lib as L
    t = synth.random_small([50, 40, 30], 2000, seed=46)
    with pytest.raises(L.FcooError) as e:
        _T()(t.idx, t.vals, t.dims).build(0, xcd_blocks=8, single_pass=True)
    assert e.value.code == L.FCOO_EINVAL
