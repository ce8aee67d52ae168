"""Host logic of the library, no GPU needed: the C ABI loads and exports every
symbol include/fcoo.h declares; the host F-COO builder is bit-exact against
the oracle's reference encoder; bad arguments return the documented codes."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth
from oracle import ref

from conftest import ROOT

from paper_1705_09905_amd import FcooError, Tensor, _lib


def _declared_functions():
    with open(os.path.join(ROOT, "include", "fcoo.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fcoo_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = _declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(_lib.lib, n), n
        assert getattr(_lib.lib, n) is not None
    assert _lib.lib.fcoo_version() == 101


def _build_both(t, mode, op, L, T):
    h = Tensor(t.idx, t.vals, t.dims)
    h.build(mode, op, threadlen=L, tile_nnz=T, host_only=True)
    got = h.export(mode, op)
    exp = ref.fcoo_encode(t.dims, t.idx, t.vals.astype(np.float32), mode,
                          ref.OP_MTTKRP if op == "mttkrp" else ref.OP_TTM, L, T)
    return h, got, exp


def _assert_same(got, exp, op):
    assert got["nseg"] == exp["nseg"]
    for a, b in zip(got["pidx"], exp["pidx"]):
        np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(got["val"], exp["val"])
    np.testing.assert_array_equal(got["bf"], exp["bf"])
    np.testing.assert_array_equal(got["sf"], exp["sf"])
    np.testing.assert_array_equal(got["tile_seg0"], exp["tile_seg0"])
    np.testing.assert_array_equal(got["perm"], exp["perm"])
    if op == "mttkrp":
        np.testing.assert_array_equal(got["seg_row"], exp["seg_row"])
    else:
        np.testing.assert_array_equal(got["fibres"], exp["fibres"])


@pytest.mark.parametrize("dims,Z,seed", [([7, 5, 6], 150, 1), ([3, 4, 5, 2], 100, 2), ([50, 3], 120, 3),
                                          ([9, 8, 7, 3, 2], 333, 5), ([1, 6, 5], 25, 6),
                                          ([40, 30, 20], 5000, 7), ([6, 5, 4, 3, 2, 2, 2, 2], 700, 8)])
@pytest.mark.parametrize("op", ["mttkrp", "ttm"])
@pytest.mark.parametrize("L,T", [(8, 256), (16, 512), (64, 256)])
def test_builder_bit_exact_vs_oracle_encoder(dims, Z, seed, op, L, T):
    t = synth.random_small(dims, Z, seed=seed)
    for mode in range(len(dims)):
        _, got, exp = _build_both(t, mode, op, L, T)
        _assert_same(got, exp, op)


def test_builder_duplicates_and_golden():
    t = synth.random_small([6, 5, 4], 400, seed=9, duplicates=True)
    for op in ("mttkrp", "ttm"):
        for mode in range(3):
            _, got, exp = _build_both(t, mode, op, 8, 256)
            _assert_same(got, exp, op)


def test_builder_large_keys_fall_back_to_comparison_sort():
    # 8 modes of 2^9 = 72 key bits > 64: the comparison sort path
    g = np.random.default_rng(3)
    dims = [512] * 8
    Z = 3000
    idx = [g.integers(0, 512, Z).astype(np.int32) for _ in range(8)]
    idx[1][:100] = idx[1][100:200]  # some repeated prefixes
    vals = g.random(Z)
    t = synth.SparseTensor(dims=dims, idx=idx, vals=vals)
    for op in ("mttkrp", "ttm"):
        _, got, exp = _build_both(t, 3, op, 16, 512)
        _assert_same(got, exp, op)


def test_builder_radix_path_large():
    t = synth.zipf_tensor([3000, 2000, 1000], 200_000, cfg=77)
    for op in ("mttkrp", "ttm"):
        _, got, exp = _build_both(t, 1, op, 16, 4096)
        _assert_same(got, exp, op)


def test_info_sizes_match_table2():
    t = synth.random_small([64, 64, 64], 8 * 32 * 16, seed=4)
    h = Tensor(t.idx, t.vals, t.dims)
    for op in ("mttkrp", "ttm"):
        h.build(0, op, threadlen=16, tile_nnz=256, host_only=True)
        inf = h.info(0, op)
        assert inf["bytes_format"] == ref.table2_bytes(t.nnz, 0 if op == "mttkrp" else 1, 16)
        assert inf["on_device"] == 0


def test_empty_tensor_builds():
    h = Tensor([np.zeros(0, np.int32)] * 3, np.zeros(0), [4, 5, 6])
    h.build(1, "mttkrp", host_only=True)
    inf = h.info(1)
    assert inf["nnz"] == 0 and inf["nseg"] == 0 and inf["ntiles"] == 0 and inf["nempty"] == 5
    e = h.export(1)
    assert e["bf"].size == 0 and e["sf"].size == 0


def _code(fn):
    with pytest.raises(FcooError) as ei:
        fn()
    return ei.value.code


def test_error_codes():
    assert _code(lambda: Tensor([np.array([0, 5], np.int32), np.array([0, 0], np.int32)],
                                [1.0, 2.0], [5, 3])) == _lib.FCOO_ERANGE
    assert _code(lambda: Tensor([np.array([-1], np.int32), np.array([0], np.int32)], [1.0],
                                [5, 3])) == _lib.FCOO_ERANGE
    assert _code(lambda: Tensor([np.array([0], np.int32)], [1.0], [5])) == _lib.FCOO_EUNSUPPORTED
    h = Tensor([np.array([0, 1], np.int32), np.array([2, 0], np.int32)], [1.0, 2.0], [3, 3])
    assert _code(lambda: h.info(0)) == _lib.FCOO_ENOTBUILT
    assert _code(lambda: h.build(2, "mttkrp", host_only=True)) == _lib.FCOO_EINVAL
    assert _code(lambda: h.build(0, "mttkrp", threadlen=12, host_only=True)) == _lib.FCOO_EINVAL
    assert _code(lambda: h.build(0, "mttkrp", tile_nnz=100, host_only=True)) == _lib.FCOO_EINVAL
    h.build(0, "mttkrp", host_only=True)
    # a host-only build is not on the device: device operations refuse it
    rc = _lib.fcoo_spmttkrp(h.handle, 0, _lib.ptr_array([1, 1]), 0, 4, C.c_void_p(1), None)
    assert rc == _lib.FCOO_ENOTBUILT
    rc = _lib.fcoo_create(2, None, 0, None, None, C.byref(C.c_void_p()))
    assert rc == _lib.FCOO_EINVAL
    assert b"dims" in _lib.fcoo_last_error()
    assert _code(lambda: h.build(0, "mttkrp", lane_cols=2, host_only=True)) == _lib.FCOO_EINVAL
    h.build(0, "mttkrp", lane_cols=4, host_only=True)
    assert h.info(0)["lane_cols"] == 4
    # the copy kernel's argument checks come before any device work
    assert _lib.fcoo_device_copy(None, None, 0, None) == _lib.FCOO_OK
    assert _lib.fcoo_device_copy(C.c_void_p(16), C.c_void_p(32), 24, None) == _lib.FCOO_EINVAL
    assert _lib.fcoo_device_copy(None, C.c_void_p(32), 16, None) == _lib.FCOO_EINVAL
    assert _lib.fcoo_device_copy(C.c_void_p(8), C.c_void_p(32), 16, None) == _lib.FCOO_EINVAL


def test_mode_and_op_out_of_range_are_einval():
    # every entry point that takes a mode (and an op) refuses one outside
    # [0, order) or an unknown op with FCOO_EINVAL before any device work
    h = Tensor([np.array([0, 1], np.int32), np.array([2, 0], np.int32), np.array([1, 1], np.int32)],
               [1.0, 2.0], [3, 3, 2])
    h.build(0, "mttkrp", host_only=True)
    L = _lib
    fac = L.ptr_array([1, 1, 1])
    out = C.c_void_p(1)
    info = L.fcoo_info_t()
    ranks = (C.c_int * 3)(4, 4, 4)
    for mode in (-1, 3, 7):
        calls = {
            "fcoo_build": lambda: L.fcoo_build(h.handle, mode, 0, None, None),
            "fcoo_info": lambda: L.fcoo_info(h.handle, mode, 0, C.byref(info)),
            "fcoo_export": lambda: L.fcoo_export(h.handle, mode, 0, None, None, None, None, None, None, None),
            "fcoo_spmttkrp": lambda: L.fcoo_spmttkrp(h.handle, mode, fac, 0, 4, out, None),
            "fcoo_spttm": lambda: L.fcoo_spttm(h.handle, mode, out, 0, 4, out, None),
            "fcoo_spttmc": lambda: L.fcoo_spttmc(h.handle, mode, fac, 0, ranks, out, None),
            "fcoo_spmttkrp_values": lambda: L.fcoo_spmttkrp_values(h.handle, mode, out, fac, 0, 4, out, None),
            "fcoo_resid_spmttkrp": lambda: L.fcoo_resid_spmttkrp(h.handle, mode, fac, 0, 4, out, None, None),
            "fcoo_gram": lambda: L.fcoo_gram(h.handle, mode, out, 0, 4, out, None),
            "fcoo_autotune": lambda: L.fcoo_autotune(h.handle, mode, 0, fac, 0, 4, None, 0, 1, None, None,
                                                     None),
        }
        for name, call in calls.items():
            assert call() == L.FCOO_EINVAL, (name, mode)
            assert b"out of range" in L.fcoo_last_error(), (name, mode)
    for op in (-1, 2):
        assert L.fcoo_build(h.handle, 0, op, None, None) == L.FCOO_EINVAL
        assert L.fcoo_info(h.handle, 0, op, C.byref(info)) == L.FCOO_EINVAL
        assert L.fcoo_export(h.handle, 0, op, None, None, None, None, None, None, None) == L.FCOO_EINVAL
        assert b"unknown op" in L.fcoo_last_error()
    # a valid but unbuilt (op, mode) is FCOO_ENOTBUILT, not FCOO_EINVAL
    assert L.fcoo_info(h.handle, 1, 0, C.byref(info)) == L.FCOO_ENOTBUILT
    assert L.fcoo_spttm(h.handle, 2, out, 0, 4, out, None) == L.FCOO_ENOTBUILT
    # null handles
    assert L.fcoo_info(None, 0, 0, C.byref(info)) == L.FCOO_EINVAL
    assert L.fcoo_spmttkrp(None, 0, fac, 0, 4, out, None) == L.FCOO_EINVAL


def _blocks_of(t, bm, nblk=8):
    # the documented split: indices of mode bm in order, block = floor(nonzeros
    # before the index * nblk / Z)
    cnt = np.bincount(np.asarray(t.idx[bm], np.int64), minlength=t.dims[bm])
    before = np.concatenate([[0], np.cumsum(cnt)[:-1]])
    return np.minimum((before * nblk) // t.nnz, nblk - 1)


@pytest.mark.parametrize("dims,Z,mode,xmode", [([40, 300, 200], 20000, 0, -1), ([500, 30, 20], 12000, 1, -1),
                                                ([30, 40, 50, 60], 9000, 2, -1), ([20, 1000], 5000, 0, -1),
                                                ([40, 300, 200], 20000, 0, 2), ([30, 40, 50, 60], 9000, 2, 1)])
def test_xcd_blocks_layout(dims, Z, mode, xmode):
    # the blocked order is the concatenation, block by block, of the reference
    # encoding of each block's nonzeros; segments are (block, row) pairs; the
    # blocks are ranges of the requested product mode, else the largest one
    t = synth.random_small(dims, Z, seed=Z)
    L, T = 16, 512
    h = Tensor(t.idx, t.vals, t.dims).build(mode, "mttkrp", threadlen=L, tile_nnz=T, host_only=True,
                                             xcd_blocks=8, xcd_mode=xmode)
    info = h.info(mode)
    assert info["xcd_blocks"] == 8
    pm = [m for m in range(len(dims)) if m != mode]
    bm = info["block_mode"]
    assert bm == (xmode if xmode >= 0 else max(pm, key=lambda m: (dims[m], -m)))
    blk = _blocks_of(t, bm)[np.asarray(t.idx[bm])]
    perm, heads, rows = [], [], []
    for b in range(8):
        sel = np.nonzero(blk == b)[0]
        if sel.size == 0:
            continue
        enc = ref.fcoo_encode(t.dims, [c[sel] for c in t.idx], t.vals[sel].astype(np.float32), mode,
                              ref.OP_MTTKRP, L, T)
        perm.append(sel[enc["perm"]])
        heads.append(enc["head"])
        rows.append(enc["seg_row"].astype(np.int64) + b * dims[mode])
    perm = np.concatenate(perm)
    head = np.concatenate(heads).astype(bool)
    got = h.export(mode, "mttkrp")
    np.testing.assert_array_equal(got["perm"], perm)
    np.testing.assert_array_equal(got["val"], t.vals[perm].astype(np.float32))
    for q, m in enumerate(pm):
        np.testing.assert_array_equal(got["pidx"][q], np.asarray(t.idx[m])[perm])
    np.testing.assert_array_equal(got["seg_row"], np.concatenate(rows))
    bf = (np.cumsum(head) & 1).astype(np.uint8)
    np.testing.assert_array_equal(got["bf"], np.packbits(bf, bitorder="little"))
    ntiles = -(-Z // T)
    np.testing.assert_array_equal(got["tile_seg0"], np.cumsum(head)[np.arange(ntiles) * T] - 1)
    assert info["nseg"] == head.sum()
    # about Z / 8 nonzeros per block
    sizes = np.bincount(blk, minlength=8)
    assert sizes.max() <= Z / 8 + np.bincount(np.asarray(t.idx[bm])).max() + 1


def test_xcd_blocks_refusals():
    t = synth.random_small([20, 30, 40], 500, seed=1)
    h = Tensor(t.idx, t.vals, t.dims)
    with pytest.raises(FcooError) as e:
        h.build(0, "ttm", host_only=True, xcd_blocks=8)
    assert e.value.code == _lib.FCOO_EINVAL
    with pytest.raises(FcooError) as e:
        h.build(0, "mttkrp", host_only=True, xcd_blocks=4)
    assert e.value.code == _lib.FCOO_EINVAL
    with pytest.raises(FcooError) as e:                           # the index mode is no product mode
        h.build(0, "mttkrp", host_only=True, xcd_blocks=8, xcd_mode=0)
    assert e.value.code == _lib.FCOO_EINVAL


def test_binding_refuses_wrapping_coordinates_and_bad_outputs():
    import torch
    from paper_1705_09905_amd.tensor import _out
    dims = [4, 5, 6]
    ok = [np.array([0, 3]), np.array([1, 4]), np.array([2, 5])]
    Tensor(ok, np.ones(2), dims)                                     # int64 in range: accepted
    with pytest.raises(ValueError):                                  # 2^32 + 1 would wrap to 1
        Tensor([np.array([0, 2 ** 32 + 1]), ok[1], ok[2]], np.ones(2), dims)
    with pytest.raises(ValueError):
        Tensor([np.array([0, 2 ** 31], np.uint32), ok[1], ok[2]], np.ones(2), dims)
    with pytest.raises(TypeError):
        Tensor([np.array([0.0, 1.0]), ok[1], ok[2]], np.ones(2), dims)
    with pytest.raises(FcooError):                                   # negative: the library's check
        Tensor([np.array([0, -1], np.int32), ok[1], ok[2]], np.ones(2), dims)
    with pytest.raises(ValueError):                                  # a host tensor is no output
        _out(torch.empty((4, 8)), (4, 8), torch.float32)


def test_cp_als_refuses_mis_shaped_initial_factors():
    from paper_1705_09905_amd import cp_als
    t = Tensor([np.array([0, 3]), np.array([1, 4]), np.array([2, 5])], np.ones(2), [4, 5, 6])
    init = [np.ones((4, 3)), np.ones((5, 3)), np.ones((6, 2))]
    with pytest.raises(ValueError):
        cp_als(t, 3, 1, init, build=False)
    with pytest.raises(ValueError):
        cp_als(t, 3, 1, init[:2], build=False)
    with pytest.raises(ValueError):
        cp_als(t, 3, 1, [np.ones((4, 3)), np.ones((5, 3)), np.ones((6, 3))], dtype="f16", build=False)
