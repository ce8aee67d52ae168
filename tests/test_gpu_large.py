"""Parity on the three large workloads at full size, against the float64
oracle (its C loops for the sparse products):

* order-4 Zipf(1.1) tensor 50,000 x 20,000 x 5,000 x 1,000 with 50M
  nonzeros: ten CP-ALS sweeps at R = 32, float32 factors, fit per sweep;
* planted rank-16 CP tensor 200,000 x 150,000 x 100,000 sampled at 100M
  uniform coordinates (noise variance 0.01): ten CP-ALS sweeps at R = 16 with
  float32 and with bfloat16 factor storage, fit per sweep against the float64
  oracle;
* gradient-based CP on the 1,000,000 x 500,000 x 50,000 Zipf(1.1) tensor with
  200M nonzeros and planted rank-64 values at R = 64: the gradient of the MSE
  loss at the start (float32 and bfloat16 factors) and the observed fit after
  a few Adam steps.

Generating a workload and running the oracle take minutes each, so these run
only with FCOO_LARGE=1 in the environment.  Builds run on the GPU, in both
layouts (plain and XCD-blocked) where the benchmark may use either."""
import os

import numpy as np
import pytest

import synth
from oracle import cpu, ref

from conftest import gpu_available
from gpu_util import TOL_BF16, TOL_F32, bf16, f32, from_dev, rel_fro, tag, to_dev

pytestmark = [pytest.mark.gpu, pytest.mark.slow,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU"),
              pytest.mark.skipif(os.environ.get("FCOO_LARGE") != "1",
                                 reason="minutes per workload: set FCOO_LARGE=1")]


def _oracle_mttkrp(d, i, v, F, n):
    return cpu.mttkrp(d, i, v, F, n)


def _observed_fit(idx, vals, factors):
    # the oracle's observed-entry fit, with the model evaluated by its C loop
    x = np.asarray(vals, np.float64)
    r = cpu.model_at(idx, factors) - x
    return 1.0 - float(np.linalg.norm(r) / np.linalg.norm(x))


def _cp_case(cfg, R, sweeps, dtypes):
    from paper_1705_09905_amd import Tensor, cp_als
    tag("generating workload", cfg)
    t = synth.config_tensor(cfg)
    init = [f32(a) for a in synth.factors(t.dims, R, cfg, role="init")]
    vals = f32(t.vals)
    tag("oracle CP-ALS", cfg, "R", R, "sweeps", sweeps)
    orc = ref.cp_als(t.dims, t.idx, vals, R, init, sweeps, mttkrp=_oracle_mttkrp)
    tag("oracle fits", orc["fits"])
    h = Tensor(t.idx, t.vals, t.dims)
    for xcd in (0, 8):                           # both layouts the benchmark's autotuner picks from
        for m in range(t.order):
            h.build(m, device=True, xcd_blocks=xcd)
        for dtype in dtypes:
            out = cp_als(h, R, sweeps, init, dtype=dtype, build=False)
            d = np.abs(np.array(out["fits"]) - np.array(orc["fits"]))
            tag("cp-als", cfg, dtype, "xcd blocks", xcd, "fits", out["fits"], "max |fit - oracle|", d.max())
            assert len(out["fits"]) == sweeps
            assert d.max() <= 1e-3


def test_order4_zipf_50M_cp_als_R32_ten_sweeps():
    _cp_case(2, 32, 10, ("f32",))


def test_planted_rank16_100M_cp_als_f32_and_bf16():
    _cp_case(3, 16, 10, ("f32", "bf16"))


def test_gradient_cp_zipf_200M_R64():
    import torch
    from paper_1705_09905_amd import CPMSELoss, Tensor
    cfg, R = 4, 64
    tag("generating workload", cfg)
    t = synth.config_tensor(cfg)
    vals = f32(t.vals)
    init = [f32(a) for a in synth.factors(t.dims, R, cfg, role="init")]
    h = Tensor(t.idx, t.vals, t.dims)
    # gradient at the start: kernel error (oracle on the stored factors) and,
    # for bfloat16, the end-to-end error (oracle on the float32 factors)
    loss32, g32 = cpu.mse_grad(t.dims, t.idx, vals, init)
    for dtype, xcd in (("f32", 0), ("bf16", 0), ("f32", 8)):
        for m in range(t.order):
            h.build(m, device=True, xcd_blocks=xcd)
        stored = init if dtype == "f32" else [bf16(a) for a in init]
        exp_loss, exp_g = (loss32, g32) if dtype == "f32" else cpu.mse_grad(t.dims, t.idx, vals, stored)
        masters = [to_dev(a).requires_grad_() for a in init]
        loss = CPMSELoss.apply(h, dtype, *masters)
        loss.backward()
        tag("loss", dtype, "xcd blocks", xcd, loss.item(), "oracle", exp_loss)
        assert abs(loss.item() - exp_loss) <= 1e-5 * exp_loss
        for m in range(t.order):
            G = from_dev(masters[m].grad)
            err = rel_fro(G, exp_g[m])
            tag("grad", dtype, "mode", m, "kernel rel err", err)
            assert err <= 5 * TOL_F32
            if dtype == "bf16":
                e2e = rel_fro(G, g32[m])
                tag("grad bf16 mode", m, "end-to-end rel err", e2e)
                assert e2e <= TOL_BF16
    # a few Adam steps: observed fit against the float64 oracle's
    steps, lr = 3, 1e-2
    po = [a.astype(np.float64) for a in init]
    mo = [np.zeros_like(a) for a in po]
    vo = [np.zeros_like(a) for a in po]
    for s in range(1, steps + 1):
        _, g = cpu.mse_grad(t.dims, t.idx, vals, po)
        po, mo, vo = ref.adam_step(po, g, mo, vo, s, lr=lr)
    fit_o = _observed_fit(t.idx, vals, po)
    for m in range(t.order):
        h.build(m, device=True)
    for dtype in ("f32", "bf16"):
        masters = [to_dev(a).requires_grad_() for a in init]
        opt = torch.optim.Adam(masters, lr=lr, betas=(0.9, 0.999), eps=1e-8)
        for _ in range(steps):
            opt.zero_grad()
            CPMSELoss.apply(h, dtype, *masters).backward()
            opt.step()
        fit = _observed_fit(t.idx, vals, [from_dev(m) for m in masters])
        tag("adam", dtype, "observed fit", fit, "oracle", fit_o)
        assert abs(fit - fit_o) <= 1e-3
