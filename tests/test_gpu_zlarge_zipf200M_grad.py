"""Full-size parity of gradient-based sparse CP on the 1,000,000 x 500,000 x
50,000 Zipf(1.1) tensor with 200M nonzeros and planted rank-64 values, at
R = 64: the mean-squared-error loss and its gradient (Eq. 6 with residual
values, fused residual SpMTTKRP) at the start, float32 and bfloat16 factors,
plain and XCD-blocked layouts, against the float64 oracle's chain-rule
gradient (relative Frobenius error 1e-5 for the kernels, 2e-2 bfloat16 end
to end); then three Adam steps, compared on the observed-entry fit and on
the CP model at a seeded sample of 1M nonzeros."""
import numpy as np
import pytest

import synth
from oracle import cpu, ref

from conftest import gpu_available
from gpu_util import (TOL_BF16, TOL_F32, bf16, f32, from_dev, model_values, rel_fro, sample_positions,
                      tag, to_dev)

pytestmark = [pytest.mark.gpu, pytest.mark.slow,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

CFG, R = 4, 64
ADAM_STEPS, LR = 3, 1e-2
TOL_MODEL_F32 = 1e-4


@pytest.fixture(scope="module")
def case():
    tag("generating workload", CFG)
    t = synth.config_tensor(CFG)
    vals = f32(t.vals)
    init = [f32(a) for a in synth.factors(t.dims, R, CFG, role="init")]
    tag("oracle gradient at the float32 start")
    loss32, g32 = cpu.mse_grad(t.dims, t.idx, vals, init)
    return dict(t=t, vals=vals, init=init, loss32=loss32, g32=g32)


def _grad_case(case, dtype, xcd):
    from paper_1705_09905_amd import CPMSELoss, Tensor
    t, init = case["t"], case["init"]
    h = Tensor(t.idx, t.vals, t.dims)
    for m in range(t.order):
        h.build(m, device=True, xcd_blocks=xcd)
    if dtype == "f32":
        exp_loss, exp_g = case["loss32"], case["g32"]
    else:
        tag("oracle gradient at the bfloat16-rounded start")
        exp_loss, exp_g = cpu.mse_grad(t.dims, t.idx, case["vals"], [bf16(a) for a in init])
    masters = [to_dev(a).requires_grad_() for a in init]
    tag("gradient", dtype, "xcd blocks", xcd)
    loss = CPMSELoss.apply(h, dtype, *masters)
    loss.backward()
    tag("loss", dtype, "xcd blocks", xcd, loss.item(), "oracle", exp_loss)
    assert abs(loss.item() - exp_loss) <= 1e-5 * exp_loss
    for m in range(t.order):
        G = from_dev(masters[m].grad)
        err = rel_fro(G, exp_g[m])
        tag("grad", dtype, "xcd", xcd, "mode", m, "kernel rel err", err)
        assert err <= TOL_F32
        if dtype == "bf16":
            e2e = rel_fro(G, case["g32"][m])
            tag("grad bf16 mode", m, "end-to-end rel err", e2e)
            assert e2e <= TOL_BF16


@pytest.mark.parametrize("dtype,xcd", [("f32", 0), ("bf16", 0), ("f32", 8)])
def test_zipf200M_gradient_at_start(case, dtype, xcd):
    _grad_case(case, dtype, xcd)


def test_zipf200M_adam_steps_track_oracle(case):
    import torch
    from paper_1705_09905_amd import CPMSELoss, Tensor
    t, vals, init = case["t"], case["vals"], case["init"]
    po = [a.astype(np.float64) for a in init]
    mo = [np.zeros_like(a) for a in po]
    vo = [np.zeros_like(a) for a in po]
    for s in range(1, ADAM_STEPS + 1):
        tag("oracle Adam step", s)
        g = case["g32"] if s == 1 else cpu.mse_grad(t.dims, t.idx, vals, po)[1]
        po, mo, vo = ref.adam_step(po, g, mo, vo, s, lr=LR)
    fit_o = ref.observed_fit(t.idx, vals, po, model=cpu.model_at)
    sel = sample_positions(t.nnz, 1_000_000, seed=CFG)
    ones = np.ones(R)
    want = model_values(t.idx, po, ones, sel)
    h = Tensor(t.idx, t.vals, t.dims)
    for m in range(t.order):
        h.build(m, device=True)
    for dtype in ("f32", "bf16"):
        masters = [to_dev(a).requires_grad_() for a in init]
        opt = torch.optim.Adam(masters, lr=LR, betas=(0.9, 0.999), eps=1e-8)
        tag("adam", dtype, "steps", ADAM_STEPS)
        for _ in range(ADAM_STEPS):
            opt.zero_grad()
            CPMSELoss.apply(h, dtype, *masters).backward()
            opt.step()
        F = [from_dev(m) for m in masters]
        fit = ref.observed_fit(t.idx, vals, F, model=cpu.model_at)
        err = rel_fro(model_values(t.idx, F, ones, sel), want)
        tag("adam", dtype, "observed fit", fit, "oracle", fit_o, "model at 1M nonzeros rel err", err)
        assert abs(fit - fit_o) <= 1e-3
        assert err <= (TOL_MODEL_F32 if dtype == "f32" else TOL_BF16)
