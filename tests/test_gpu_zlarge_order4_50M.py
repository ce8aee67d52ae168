"""Full-size parity of CP-ALS (Algorithm 1) on the order-4 Zipf(1.1) tensor
50,000 x 20,000 x 5,000 x 1,000 with 50M nonzeros at R = 32, ten sweeps,
float32 and bfloat16 factor storage, in both SpMTTKRP layouts (plain and
XCD-blocked) the benchmark's autotuner picks from.

CP factorizations are unique only up to column order, scale and sign, so the
comparison is on what is unique: the fit of every sweep (within 1e-3 of the
float64 oracle's) and the CP model at a seeded sample of 1M nonzeros after
sweeps 1 and 10 (relative Frobenius error, 1e-4 float32 / 2e-2 bfloat16).
The oracle's sparse products are its C loops."""
import numpy as np
import pytest

import synth
from oracle import cpu, ref

from conftest import gpu_available
from gpu_util import TOL_BF16, f32, from_dev, model_values, rel_fro, sample_positions, tag

pytestmark = [pytest.mark.gpu, pytest.mark.slow,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

CFG, R, SWEEPS = 2, 32, 10
TOL_MODEL_F32 = 1e-4


@pytest.fixture(scope="module")
def case():
    tag("generating workload", CFG)
    t = synth.config_tensor(CFG)
    init = [f32(a) for a in synth.factors(t.dims, R, CFG, role="init")]
    vals = f32(t.vals)
    rec = []
    tag("oracle CP-ALS", CFG, "R", R, "sweeps", SWEEPS)
    orc = ref.cp_als(t.dims, t.idx, vals, R, init, SWEEPS, record=rec,
                     mttkrp=lambda d, i, v, F, n: cpu.mttkrp(d, i, v, F, n))
    tag("oracle fits", orc["fits"])
    sel = sample_positions(t.nnz, 1_000_000, seed=CFG)
    want = {s: model_values(t.idx, rec[s - 1][0], rec[s - 1][1], sel) for s in (1, SWEEPS)}
    return dict(t=t, init=init, orc=orc, sel=sel, want=want)


def _gpu_run(case, dtype, xcd):
    from paper_1705_09905_amd import Tensor, cp_als
    t = case["t"]
    h = Tensor(t.idx, t.vals, t.dims)
    for m in range(t.order):
        h.build(m, device=True, xcd_blocks=xcd)
    for s in (1, SWEEPS):
        tag("cp-als", CFG, dtype, "xcd blocks", xcd, "sweeps", s)
        out = cp_als(h, R, s, case["init"], dtype=dtype, build=False)
        got = model_values(t.idx, [from_dev(f) for f in out["factors"]], from_dev(out["lam"]), case["sel"])
        err = rel_fro(got, case["want"][s])
        tag("model at 1M nonzeros after sweep", s, dtype, "xcd", xcd, "rel err", err)
        assert err <= (TOL_MODEL_F32 if dtype == "f32" else TOL_BF16)
    d = np.abs(np.array(out["fits"]) - np.array(case["orc"]["fits"]))
    tag("fits", out["fits"], "max |fit - oracle|", d.max())
    assert len(out["fits"]) == SWEEPS and d.max() <= 1e-3


@pytest.mark.parametrize("xcd", [0, 8])
def test_order4_zipf50M_cp_als_f32(case, xcd):
    _gpu_run(case, "f32", xcd)


@pytest.mark.parametrize("xcd", [0, 8])
def test_order4_zipf50M_cp_als_bf16(case, xcd):
    _gpu_run(case, "bf16", xcd)
