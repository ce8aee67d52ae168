"""The F-COO build on the GPU (fcoo_opts.device = 1) against the host build:
every exported array bit for bit (which the host build is itself pinned to,
through the oracle's reference encoder), the counts, and bitwise-equal
operation results; plus its refusals."""
import time

import numpy as np
import pytest

import synth
from oracle import ref

from conftest import gpu_available
from gpu_util import from_dev, tag, to_dev

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

ARRAYS = ("val", "bf", "sf", "tile_seg0", "perm")


def _same_build(t, mode, op, L=16, T=4096):
    from paper_1705_09905_amd import Tensor
    hh = Tensor(t.idx, t.vals, t.dims).build(mode, op, threadlen=L, tile_nnz=T, host_only=True)
    hd = Tensor(t.idx, t.vals, t.dims).build(mode, op, threadlen=L, tile_nnz=T, device=True)
    a, b = hh.export(mode, op), hd.export(mode, op)
    for k in ARRAYS:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    for p, q in zip(a["pidx"], b["pidx"]):
        np.testing.assert_array_equal(p, q)
    key = "seg_row" if op == "mttkrp" else "fibres"
    np.testing.assert_array_equal(a[key], b[key])
    ia, ib = hh.info(mode, op), hd.info(mode, op)
    for k in ("nnz", "nseg", "npart", "ntiles", "nfix", "nempty", "bytes_format"):
        assert ia[k] == ib[k], k
    return hd


@pytest.mark.parametrize("dims,Z,dup", [([40, 50, 60], 20000, False), ([10, 9, 8], 6000, True),
                                        ([8, 7, 6, 5], 1500, False), ([50, 40], 1500, False),
                                        ([4, 3, 3, 3, 2, 2, 2, 2], 1500, False), ([1, 300, 200], 5000, False),
                                        ([40, 50, 60], 1, False), ([40, 50, 60], 4097, False)])
def test_device_build_equals_host_build(dims, Z, dup):
    t = synth.random_small(dims, Z, seed=Z + len(dims), duplicates=dup)
    for mode in range(len(dims)):
        for op in ("mttkrp", "ttm"):
            tag("device build", dims, Z, "dup", dup, "mode", mode, op)
            _same_build(t, mode, op, L=8 if Z % 2 else 16, T=256 if Z < 5000 else 4096)


def test_device_build_matches_reference_encoder_and_gives_identical_results():
    t = synth.zipf_tensor([3000, 2000, 1000], 200000, cfg=31)
    from paper_1705_09905_amd import Tensor
    F = [to_dev(f) for f in synth.small_factors(t.dims, 16, seed=4)]
    for mode in range(3):
        tag("device build vs reference encoder", mode)
        hd = Tensor(t.idx, t.vals, t.dims).build(mode, "mttkrp", device=True)
        enc = ref.fcoo_encode(t.dims, t.idx, t.vals, mode, ref.OP_MTTKRP, 16, 4096)
        got = hd.export(mode, "mttkrp")
        np.testing.assert_array_equal(got["bf"], enc["bf"])
        np.testing.assert_array_equal(got["sf"], enc["sf"])
        np.testing.assert_array_equal(got["seg_row"], enc["seg_row"])
        np.testing.assert_array_equal(got["tile_seg0"], enc["tile_seg0"])
        hh = Tensor(t.idx, t.vals, t.dims).build(mode, "mttkrp")
        np.testing.assert_array_equal(from_dev(hd.spmttkrp(mode, F)), from_dev(hh.spmttkrp(mode, F)))
        hd.build(mode, "ttm", device=True)
        hh.build(mode, "ttm")
        np.testing.assert_array_equal(from_dev(hd.spttm(mode, F[mode])), from_dev(hh.spttm(mode, F[mode])))


def test_device_build_refusals():
    from paper_1705_09905_amd import FcooError, Tensor, _lib
    big = 2 ** 31 - 1
    g = np.random.default_rng(0)
    idx = [g.integers(0, big, 100).astype(np.int32) for _ in range(3)]
    h = Tensor(idx, np.ones(100), [big] * 3)
    with pytest.raises(FcooError) as e:          # 93-bit sort key
        h.build(0, device=True)
    assert e.value.code == _lib.FCOO_EUNSUPPORTED
    h0 = Tensor([np.zeros(0, np.int32)] * 3, np.zeros(0), [4, 5, 6])
    with pytest.raises(FcooError) as e:          # nothing to sort: build on the host
        h0.build(0, device=True)
    assert e.value.code == _lib.FCOO_EUNSUPPORTED
    with pytest.raises(FcooError) as e:
        h0.build(0, host_only=True, device=True)
    assert e.value.code == _lib.FCOO_EINVAL


def test_device_build_full_size_zipf_20M():
    from paper_1705_09905_amd import Tensor
    import torch
    t = synth.config_tensor(1)
    for mode in range(3):
        for op in ("mttkrp", "ttm"):
            h = Tensor(t.idx, t.vals, t.dims)
            h.build(0, "mttkrp", device=True)         # first call uploads the coordinates
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h.build(mode, op, device=True)
            dt_dev = time.perf_counter() - t0
            t0 = time.perf_counter()
            hh = Tensor(t.idx, t.vals, t.dims).build(mode, op, host_only=True)
            dt_host = time.perf_counter() - t0
            tag("full-size build", op, mode, "device s", round(dt_dev, 3), "host s", round(dt_host, 3))
            a, b = hh.export(mode, op), h.export(mode, op)
            for k in ARRAYS:
                np.testing.assert_array_equal(a[k], b[k], err_msg=k)
            for p, q in zip(a["pidx"], b["pidx"]):
                np.testing.assert_array_equal(p, q)
