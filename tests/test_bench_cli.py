"""bench.py's command-line contract that needs no GPU: more than one GPU is
refused with a message and exit status 2; the algorithmic and compulsory
byte models agree on a tiny case."""
import os
import subprocess
import sys

from conftest import ROOT


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_byte_models_on_a_tiny_case():
    sys.path.insert(0, ROOT)
    import bench
    # order 3, Z = 10, R = 4: every factor row distinct -> compulsory = algorithmic
    Z, N, R, nseg, In, P = 10, 3, 4, 5, 5, 1
    alg = bench.op_bytes("mttkrp", Z, N, R, nseg, In, P)
    comp = bench.compulsory_bytes("mttkrp", Z, N, R, nseg, In, P, [5, 10, 10], 0)
    # bf only (2 bytes): no kernel reads sf, so the model leaves it out
    assert alg == comp == 4 * Z * 2 + 4 * Z + 2 + 4 * nseg + Z * 2 * R * 4 + 4 * In * R
    # SpTTM with a product mode of 3 distinct rows among 10 nonzeros
    assert bench.op_bytes("ttm", Z, N, R, nseg, In, P) - \
        bench.compulsory_bytes("ttm", Z, N, R, nseg, In, P, [3, 10, 10], 0) == (Z - 3) * R * 4
    assert len(bench.kernel_hash()) == 16


def test_rank_tile_follows_the_launch_rule():
    sys.path.insert(0, ROOT)
    import bench
    # 4 columns per lane, lanes per nonzero the next power of two of R / 4 (<= 16);
    # one-column lanes (64 of them) when R is not a multiple of 4
    assert [bench.rank_tile(R) for R in (4, 8, 16, 32, 64, 128, 256)] == [4, 8, 16, 32, 64, 64, 64]
    assert bench.rank_tile(12) == 16 and bench.rank_tile(40) == 64
    assert bench.rank_tile(3) == 64 and bench.rank_tile(100) == 64


def test_op_parity_is_zero_for_the_oracles_own_outputs():
    # the record's full-size check compares outputs with the float64 oracle;
    # fed the oracle's own results (as float32 tensors), the error is rounding only
    import numpy as np
    import torch
    sys.path.insert(0, ROOT)
    import bench
    import synth
    from oracle import cpu
    t = synth.random_small([30, 20, 10], 3000, seed=7)
    old = bench.WORKLOAD_CFG
    outs = {}
    vals = t.vals.astype(np.float32).astype(np.float64)
    for R in (4, 8):
        F = [f.astype(np.float32).astype(np.float64) for f in synth.factors(t.dims, R, old)]
        for m in range(3):
            outs[("mttkrp", m, R)] = torch.tensor(cpu.mttkrp(t.dims, t.idx, vals, F, m).astype(np.float32))
            outs[("ttm", m, R)] = torch.tensor(cpu.ttm(t.dims, t.idx, vals, F[m], m)[1].astype(np.float32))
    err = bench.op_parity(t, (4, 8), outs, 2)
    assert len(err) == 12 and max(err.values()) < 1e-7
    # a wrong row is seen
    outs[("ttm", 1, 8)][3, 2] += 1.0
    assert bench.op_parity(t, (4, 8), outs, 2)[("ttm", 1, 8)] > 1e-4
