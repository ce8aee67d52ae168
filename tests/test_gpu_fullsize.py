"""Parity at the benchmark's full size and launch configurations: the Zipf(1.1)
100,000 x 80,000 x 60,000 tensor with 20M nonzeros, SpMTTKRP and SpTTM in
every mode at R = 16 and 32 (threadlen 16, each tile size and XCD-block
layout the benchmark's autotuner picks from), against the float64 C oracle computing every output
row; SpTTMc on sampled rows; plus CP-ALS sweeps (float32 and bfloat16
factors) against the oracle's fits on the same tensor."""
import numpy as np
import pytest

import synth
from oracle import cpu, ref

from conftest import gpu_available
from gpu_util import TOL_BF16, TOL_F32, f32, from_dev, rel_fro, tag, to_dev

pytestmark = [pytest.mark.gpu, pytest.mark.slow,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def c2():
    tag("generating the 20M-nonzero Zipf workload")
    return synth.config_tensor(1)


def test_full_size_spmttkrp_spttm_all_modes(c2):
    # every tile size the benchmark's autotuner chooses from (2048, 4096, 8192)
    from paper_1705_09905_amd import Tensor
    t = c2
    h = Tensor(t.idx, t.vals, t.dims)
    vals = f32(t.vals)
    for R in (16, 32):
        F = [f32(f) for f in synth.factors(t.dims, R, 1)]
        Fd = [to_dev(f) for f in F]
        for m in range(3):
            expM = cpu.mttkrp(t.dims, t.idx, vals, F, m)
            fib, expY = cpu.ttm(t.dims, t.idx, vals, F[m], m)
            for T in (2048, 4096, 8192):
                for xcd in (0, 8):
                    tag("full size mttkrp", m, "R", R, "tile", T, "xcd blocks", xcd)
                    h.build(m, "mttkrp", threadlen=16, tile_nnz=T, xcd_blocks=xcd, device=xcd > 0)
                    err = rel_fro(from_dev(h.spmttkrp(m, Fd)), expM)
                    tag("rel err", err)
                    assert err <= TOL_F32
                tag("full size ttm", m, "R", R, "tile", T)
                h.build(m, "ttm", threadlen=16, tile_nnz=T)
                Yd = from_dev(h.spttm(m, Fd[m]))
                assert Yd.shape == expY.shape
                err = rel_fro(Yd, expY)
                tag("rel err", err)
                assert err <= TOL_F32


def test_full_size_cp_als_f32_and_bf16(c2):
    from paper_1705_09905_amd import Tensor, cp_als
    t = c2
    R, sweeps = 16, 4
    init = synth.factors(t.dims, R, 1, role="init")
    orc = ref.cp_als(t.dims, t.idx, f32(t.vals), R, [f32(a) for a in init], sweeps,
                     mttkrp=lambda d, i, v, F, n: cpu.mttkrp(d, i, v, F, n))
    h = Tensor(t.idx, t.vals, t.dims)
    for dtype, tol in (("f32", 1e-3), ("bf16", 1e-3)):
        out = cp_als(h, R, sweeps, [f32(a) for a in init], dtype=dtype)
        d = np.abs(np.array(out["fits"]) - np.array(orc["fits"])).max()
        tag("cp-als", dtype, out["fits"], "oracle", orc["fits"], "max diff", d)
        assert d <= tol


def test_full_size_spttmc_sampled_rows(c2):
    # SpTTMc at R = 16 per mode (256 Kronecker columns) on the full tensor;
    # the oracle computes a sample of output rows: the three longest slices
    # and 40 seeded others (each row only needs its own slice's nonzeros)
    from paper_1705_09905_amd import Tensor
    t = c2
    h = Tensor(t.idx, t.vals, t.dims)
    vals = f32(t.vals)
    F = [f32(f) for f in synth.factors(t.dims, 16, 1)]
    Fd = [to_dev(f) for f in F]
    g = np.random.default_rng(12)
    for m in range(3):
        h.build(m, "mttkrp", threadlen=16, tile_nnz=4096)
        tag("full size spttmc", m)
        Y = from_dev(h.spttmc(m, [None if k == m else Fd[k] for k in range(3)]))
        counts = np.bincount(t.idx[m], minlength=t.dims[m])
        rows = np.unique(np.concatenate([np.argsort(counts)[-3:], g.choice(t.dims[m], 40, replace=False)]))
        sel = np.isin(t.idx[m], rows)
        sub_idx = [i[sel] for i in t.idx]
        exp = ref.ttmc_coo(t.dims, sub_idx, vals[sel], F, m)[rows]
        err = rel_fro(Y[rows], exp)
        tag("rel err", err, "rows", len(rows), "nnz", int(sel.sum()))
        assert err <= TOL_F32
