"""Helpers shared by the GPU tests: tolerances, oracle inputs in the precision
the device sees, and a printed tag before each GPU step."""
import sys

import numpy as np

# relative Frobenius tolerances against the float64 oracle
TOL_F32 = 1e-5
TOL_BF16 = 2e-2


def tag(*parts):
    print("[gpu]", *parts, flush=True)
    sys.stdout.flush()


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
