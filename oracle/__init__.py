"""FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the HIP path: `ref` is NumPy
written from the paper's definitions, `cpu` wraps the plain C COO loops in
cpu_oracle.c (built into liborc.so by build.py).
"""
from . import ref  # noqa: F401
