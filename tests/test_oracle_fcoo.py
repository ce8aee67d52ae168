"""Pins for the oracle's F-COO encoder (Sec. IV-B): a hand-derived fixture,
Table II's closed-form sizes and invariants of the encoding."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import ref

from conftest import GOLDEN


def _golden():
    with open(os.path.join(GOLDEN, "fcoo_3x4x3_handworked.json")) as f:
        return json.load(f)


def _split(g):
    c = np.array(g["coords"], dtype=np.int64)
    return [c[:, m].astype(np.int32) for m in range(c.shape[1])], np.array(g["vals"], float)


def test_golden_mttkrp_mode0_encoding_and_result():
    g = _golden()
    idx, vals = _split(g)
    e = ref.fcoo_encode(g["dims"], idx, vals, 0, ref.OP_MTTKRP, g["threadlen"], g["tile_nnz"])
    x = g["mttkrp_mode0"]
    np.testing.assert_array_equal(e["perm"], x["perm"])
    for q in range(2):
        np.testing.assert_array_equal(e["pidx"][q], x["pidx"][q])
    np.testing.assert_array_equal(e["val"], np.array(x["val"], np.float32))
    np.testing.assert_array_equal(np.nonzero(e["head"])[0], x["heads"])
    np.testing.assert_array_equal(e["bf"], np.array(x["bf"], np.uint8))
    np.testing.assert_array_equal(e["sf"], np.array(x["sf"], np.uint32))
    np.testing.assert_array_equal(e["seg_row"], x["seg_row"])
    np.testing.assert_array_equal(e["tile_seg0"], x["tile_seg0"])
    A = np.zeros((4, 2))
    M = ref.mttkrp_coo(g["dims"], idx, vals, [A, np.array(g["B"], float), np.array(g["C"], float)], 0)
    np.testing.assert_array_equal(M, np.array(x["M_with_B_C"], float))


def test_golden_ttm_mode2_encoding_and_result():
    g = _golden()
    idx, vals = _split(g)
    e = ref.fcoo_encode(g["dims"], idx, vals, 2, ref.OP_TTM, g["threadlen"], g["tile_nnz"])
    x = g["ttm_mode2"]
    np.testing.assert_array_equal(e["perm"], x["perm"])
    np.testing.assert_array_equal(e["pidx"][0], x["pidx"][0])
    np.testing.assert_array_equal(np.nonzero(e["head"])[0], x["heads"])
    np.testing.assert_array_equal(e["bf"], np.array(x["bf"], np.uint8))
    np.testing.assert_array_equal(e["sf"], np.array(x["sf"], np.uint32))
    np.testing.assert_array_equal(e["fibres"], np.array(x["fibres"]))
    np.testing.assert_array_equal(e["tile_seg0"], x["tile_seg0"])
    fib, Y = ref.ttm_coo(g["dims"], idx, vals, np.array(g["C"], float), 2)
    np.testing.assert_array_equal(fib, np.array(x["fibres"]))
    np.testing.assert_array_equal(Y, np.array(x["Y_with_U_eq_C"], float))


@pytest.mark.parametrize("L", [8, 16, 32, 64])
def test_table2_sizes_closed_form(L):
    # Z a multiple of 8 * 32 * L: every array size is exactly Table II's formula
    Z = 8 * 32 * L
    t = synth.random_small([64, 64, 64], Z, seed=L)
    for op in (ref.OP_MTTKRP, ref.OP_TTM):
        e = ref.fcoo_encode(t.dims, t.idx, t.vals, 0, op, L, 4 * L)
        assert ref.fcoo_stream_bytes(e) == ref.table2_bytes(Z, op, L)
        assert e["bf"].nbytes == Z // 8
        assert e["sf"].nbytes == 4 * ((Z // L + 31) // 32)


@pytest.mark.parametrize("dims,Z,seed", [([7, 5, 6], 150, 1), ([3, 4, 5, 2], 100, 2),
                                          ([50, 3], 120, 3), ([2, 2, 2], 8, 4),
                                          ([9, 8, 7, 3, 2], 333, 5), ([1, 6, 5], 25, 6)])
@pytest.mark.parametrize("op", [0, 1])
@pytest.mark.parametrize("L", [8, 64])
def test_encoding_invariants(dims, Z, seed, op, L):
    t = synth.random_small(dims, Z, seed=seed)
    Z = t.nnz
    for mode in range(len(dims)):
        e = ref.fcoo_encode(dims, t.idx, t.vals, mode, op, L, 2 * L)
        imodes, pmodes = ref.mode_roles(len(dims), mode, op)
        head = e["head"]
        tuples = set(zip(*[t.idx[m].tolist() for m in imodes]))
        assert head.sum() == e["nseg"] == len(tuples)
        # bf: starts at 1, toggles exactly at heads, padding bits zero
        bits = np.unpackbits(e["bf"], bitorder="little")
        assert bits[0] == 1
        assert not bits[Z:].any()
        prev = np.concatenate([[0], bits[:Z - 1]])
        np.testing.assert_array_equal((bits[:Z] ^ prev).astype(bool), head)
        # sf: OR of the heads in each partition, sf bit 0 set, padding zero
        sfb = np.unpackbits(e["sf"].view(np.uint8), bitorder="little")
        P = -(-Z // L)
        for p in range(P):
            assert sfb[p] == head[p * L:(p + 1) * L].any()
        assert sfb[0] == 1 and not sfb[P:].any()
        # decoding reproduces the sorted coordinate list
        cols, v = ref.fcoo_decode(e, dims, mode, op)
        srt = sorted(zip(*[t.idx[m].tolist() for m in imodes + pmodes], range(Z)))
        got = list(zip(*[cols[m].tolist() for m in imodes + pmodes]))
        assert got == [s[:-1] for s in srt]
        np.testing.assert_array_equal(e["perm"], [s[-1] for s in srt])
        np.testing.assert_array_equal(v, t.vals[e["perm"]].astype(np.float32))
        if op == ref.OP_MTTKRP:
            assert np.all(np.diff(e["seg_row"]) > 0)
        # tile_seg0: segment ordinal of each tile's first nonzero
        segord = np.cumsum(head) - 1
        np.testing.assert_array_equal(e["tile_seg0"], segord[::2 * L])


def test_encoding_independent_of_input_order_and_stable_for_duplicates():
    t = synth.random_small([6, 5, 4], 80, seed=11, duplicates=True)
    g = np.random.default_rng(0).permutation(t.nnz)
    idx2 = [i[g] for i in t.idx]
    vals2 = t.vals[g]
    for op in (0, 1):
        a = ref.fcoo_encode(t.dims, t.idx, t.vals, 1, op, 8, 16)
        b = ref.fcoo_encode(t.dims, idx2, vals2, 1, op, 8, 16)
        for k in ("bf", "sf", "tile_seg0"):
            np.testing.assert_array_equal(a[k], b[k])
        for q in range(len(a["pidx"])):
            np.testing.assert_array_equal(a["pidx"][q], b["pidx"][q])
        # ties keep input order: perm is increasing inside runs of equal keys
        keys = np.stack([t.idx[m][a["perm"]] for m in range(3)], 1)
        same = np.all(keys[1:] == keys[:-1], axis=1)
        assert np.all(a["perm"][1:][same] > a["perm"][:-1][same])


def test_mttkrp_mode0_and_ttm_mode2_share_order_for_3order():
    t = synth.random_small([5, 6, 7], 90, seed=12)
    a = ref.fcoo_encode(t.dims, t.idx, t.vals, 0, ref.OP_MTTKRP, 8, 16)
    b = ref.fcoo_encode(t.dims, t.idx, t.vals, 2, ref.OP_TTM, 8, 16)
    np.testing.assert_array_equal(a["perm"], b["perm"])
    np.testing.assert_array_equal(a["pidx"][1], b["pidx"][0])
    # every slice start is also a fibre start
    assert np.all(b["head"][a["head"]])


def test_empty_and_single():
    e = ref.fcoo_encode([3, 3, 3], [np.zeros(0, np.int32)] * 3, np.zeros(0), 0, 0, 8, 8)
    assert e["nseg"] == 0 and e["bf"].size == 0 and e["sf"].size == 0 and e["tile_seg0"].size == 0
    e = ref.fcoo_encode([3, 3, 3], [np.array([1], np.int32)] * 3, np.array([2.0]), 1, 0, 8, 8)
    assert e["nseg"] == 1 and list(e["bf"]) == [1] and list(e["sf"]) == [1]
    assert list(e["seg_row"]) == [1] and list(e["tile_seg0"]) == [0]
