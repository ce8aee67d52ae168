"""GPU test of fcoo_spmttkrp_noalloc, the SpMTTKRP entry point that allocates
nothing (its tile carries and XCD-block partial rows live in a fixed device
array), called through the C ABI: two calls in a row, the second on a smaller
input, each checked against fcoo_spmttkrp on the same build (bitwise: the
same kernels, and the kernels are deterministic) and against the float64
oracle (relative Frobenius error 1e-5 for float32 factors, 2e-2 for
bfloat16); an XCD-blocked build whose partial rows fit the array; and the
size check, which refuses a call that needs more scratch than the array
holds before anything is launched."""
import ctypes as C

import numpy as np
import pytest

import synth
from oracle import cpu

from conftest import gpu_available
from gpu_util import TOL_BF16, TOL_F32, bf16, f32, from_dev, rel_fro, tag, to_dev

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _noalloc(h, mode, F, M):
    """fcoo_spmttkrp_noalloc through the C ABI; returns the status code."""
    import torch
    from paper_1705_09905_amd import _lib as L
    fp, R, dt = h._factors(F, skip=mode)
    return L.fcoo_spmttkrp_noalloc(h.handle, int(mode), fp, dt, R, C.c_void_p(M.data_ptr()),
                                   C.c_void_p(torch.cuda.current_stream().cuda_stream))


def _case(dims, nnz, R, T, dtype, seed, xcd=0):
    from paper_1705_09905_amd import Tensor
    t = synth.random_small(dims, nnz, seed=seed)
    F = synth.small_factors(t.dims, R, seed=seed)
    Fh = [f32(f) if dtype == "f32" else bf16(f) for f in F]
    h = Tensor(t.idx, t.vals, t.dims)
    for m in range(t.order):
        h.build(m, "mttkrp", tile_nnz=T, xcd_blocks=xcd)
    return t, h, Fh, [to_dev(f, dtype) for f in Fh]


def test_noalloc_equals_spmttkrp_two_calls_second_smaller():
    import torch
    from paper_1705_09905_amd import _lib as L
    # several tiles with a ragged tail, then a smaller tensor and rank
    cases = [((300, 200, 150), 200_037, 32, 4096, "f32", 1),
             ((60, 50, 40), 5_003, 8, 1024, "f32", 2),
             ((90, 70, 50), 40_011, 48, 2048, "bf16", 3),
             ((40, 30, 20), 3_001, 16, 256, "bf16", 4)]
    for dims, nnz, R, T, dtype, seed in cases:
        t, h, Fh, Fd = _case(dims, nnz, R, T, dtype, seed)
        for mode in range(t.order):
            tag("noalloc", dims, nnz, "R", R, "T", T, dtype, "mode", mode)
            first = torch.full((t.dims[mode], R), float("nan"), dtype=torch.float32, device="cuda")
            L.check(_noalloc(h, mode, Fd, first))
            second = torch.full_like(first, float("nan"))
            L.check(_noalloc(h, mode, Fd, second))
            ref = h.spmttkrp(mode, Fd)
            torch.cuda.synchronize()
            assert torch.equal(first, ref) and torch.equal(second, ref)
            exp = cpu.mttkrp(t.dims, t.idx, f32(t.vals), Fh, mode)
            err = rel_fro(from_dev(first), exp)
            assert err <= (TOL_F32 if dtype == "f32" else TOL_BF16), err


def test_noalloc_xcd_blocked_build():
    import torch
    from paper_1705_09905_amd import _lib as L
    # 8 x 2000 x 32 floats of partial rows: inside the fixed array
    t, h, Fh, Fd = _case((2000, 1500, 1000), 120_001, 32, 1024, "f32", 5, xcd=8)
    for mode in range(t.order):
        assert h.info(mode)["xcd_blocks"] == 8
        tag("noalloc xcd-blocked", t.dims, t.nnz, "mode", mode)
        got = torch.full((t.dims[mode], 32), float("nan"), dtype=torch.float32, device="cuda")
        L.check(_noalloc(h, mode, Fd, got))
        ref = h.spmttkrp(mode, Fd)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
        assert rel_fro(from_dev(got), cpu.mttkrp(t.dims, t.idx, f32(t.vals), Fh, mode)) <= TOL_F32


def test_noalloc_on_a_single_pass_build_keeps_the_fixup_pass():
    # a single-pass build's words are allocated on first use, so the no-alloc
    # entry point runs such a build with the fix-up pass and its fixed scratch
    import torch
    from paper_1705_09905_amd import Tensor, _lib as L
    t = synth.random_small([200, 150, 100], 80_003, seed=7)
    F = synth.small_factors(t.dims, 16, seed=7)
    Fd = [to_dev(f32(f)) for f in F]
    h = Tensor(t.idx, t.vals, t.dims).build(0, "mttkrp", tile_nnz=256, single_pass=True)
    tag("noalloc on a single-pass build", t.dims, t.nnz)
    got = torch.full((t.dims[0], 16), float("nan"), dtype=torch.float32, device="cuda")
    L.check(_noalloc(h, 0, Fd, got))
    ref = h.spmttkrp(0, Fd)
    torch.cuda.synchronize()
    exp = cpu.mttkrp(t.dims, t.idx, f32(t.vals), [f32(f) for f in F], 0)
    assert rel_fro(from_dev(got), exp) <= TOL_F32 and rel_fro(from_dev(ref), exp) <= TOL_F32
    assert h.info(0)["sp_gave_up"] == 0


def test_noalloc_refuses_scratch_beyond_its_array():
    import torch
    from paper_1705_09905_amd import _lib as L
    # an XCD-blocked build of 5000 rows at R = 256 needs 8 x 5000 x 256 x 4 bytes
    # of partial rows (41 MB), above the fixed 16 MiB: refused on the host
    t, h, Fh, Fd = _case((5000, 300, 200), 20_000, 256, 1024, "f32", 6, xcd=8)
    M = torch.zeros((t.dims[0], 256), dtype=torch.float32, device="cuda")
    rc = _noalloc(h, 0, Fd, M)
    assert rc == L.FCOO_ERANGE
    assert b"scratch" in L.lib.fcoo_last_error()
    torch.cuda.synchronize()
    assert float(M.abs().max()) == 0.0
    # the same build still runs through the allocating entry point
    exp = cpu.mttkrp(t.dims, t.idx, f32(t.vals), Fh, 0)
    assert rel_fro(from_dev(h.spmttkrp(0, Fd)), exp) <= TOL_F32
