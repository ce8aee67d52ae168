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
