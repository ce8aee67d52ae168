"""Helpers shared by the GPU tests: tolerances, oracle inputs in the precision
the device sees, and a printed tag before each GPU step."""
import os
import sys
import time

import numpy as np

# relative Frobenius tolerances against the float64 oracle
TOL_F32 = 1e-5
TOL_BF16 = 2e-2


# progress file for the tags (FCOO_TEST_PROGRESS; unset: none)
_PROGRESS = os.environ.get("FCOO_TEST_PROGRESS", "")


def tag(*parts):
    """Print what names the GPU step about to run (test case, shape, seed);
    the line also goes to the progress file if one is set, since pytest
    holds captured output back until a test ends."""
    line = " ".join(str(p) for p in ("[gpu]",) + parts)
    print(line, flush=True)
    sys.stdout.flush()
    if not _PROGRESS:
        return
    try:
        os.makedirs(os.path.dirname(_PROGRESS), exist_ok=True)
        with open(_PROGRESS, "a") as f:
            f.write(f"{time.strftime('%H:%M:%S')} {line}\n")
    except OSError:
        pass


def f32(x):
    """Values as the float32 path sees them, promoted exactly to float64."""
    return np.asarray(x, np.float64).astype(np.float32).astype(np.float64)


def bf16(x):
    from oracle import ref
    return ref.bf16_round(x)


def rel_fro(got, exp):
    got = np.asarray(got, np.float64)
    exp = np.asarray(exp, np.float64)
    den = np.linalg.norm(exp)
    num = np.linalg.norm(got - exp)
    return num / den if den > 0 else num


def to_dev(a, dtype="f32"):
    import torch
    t = torch.tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")
    return t.to(torch.bfloat16).contiguous() if dtype == "bf16" else t


def from_dev(t):
    import torch
    return t.detach().to(torch.float64).cpu().numpy()


def sample_positions(Z, n, seed):
    """Sorted distinct positions of a seeded sample of about n of Z nonzeros."""
    g = np.random.default_rng(seed)
    if n >= Z:
        return np.arange(Z)
    return np.unique(g.integers(0, Z, size=n))


def model_values(idx, factors, lam, sel):
    """The CP model sum_r lam_r prod_m A_m[i_m, r] at the nonzeros `sel`,
    evaluated by the float64 oracle's C loop."""
    from oracle import cpu
    F = [np.asarray(a, np.float64) for a in factors]
    F[-1] = F[-1] * np.asarray(lam, np.float64)[None, :]
    return cpu.model_at([np.ascontiguousarray(i[sel]) for i in idx], F)
