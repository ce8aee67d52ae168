"""ctypes binding of libfcoo.so: the C ABI of include/fcoo.h, function for
function, with the same names.  Argument marshalling only; every step of
the computation runs in the library's HIP kernels.

Importing fails loudly when the library has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfcoo.so")

FCOO_OK = 0
FCOO_EINVAL = -1
FCOO_ENOMEM = -2
FCOO_EHIP = -3
FCOO_ENOTBUILT = -4
FCOO_ERANGE = -5
FCOO_EUNSUPPORTED = -6

FCOO_OP_MTTKRP = 0
FCOO_OP_TTM = 1
FCOO_F32 = 0
FCOO_BF16 = 1

ERROR_NAMES = {
    FCOO_EINVAL: "FCOO_EINVAL", FCOO_ENOMEM: "FCOO_ENOMEM", FCOO_EHIP: "FCOO_EHIP",
    FCOO_ENOTBUILT: "FCOO_ENOTBUILT", FCOO_ERANGE: "FCOO_ERANGE",
    FCOO_EUNSUPPORTED: "FCOO_EUNSUPPORTED",
}


class fcoo_opts(C.Structure):
    _fields_ = [("threadlen", C.c_int), ("tile_nnz", C.c_int), ("host_only", C.c_int),
                ("device", C.c_int), ("xcd_blocks", C.c_int), ("xcd_mode", C.c_int),
                ("lane_cols", C.c_int), ("single_pass", C.c_int)]


class fcoo_info_t(C.Structure):
    _fields_ = [("nnz", C.c_int64), ("nseg", C.c_int64), ("npart", C.c_int64),
                ("ntiles", C.c_int64), ("nfix", C.c_int64), ("nempty", C.c_int64),
                ("bytes_format", C.c_int64), ("bytes_device", C.c_int64),
                ("threadlen", C.c_int32), ("tile_nnz", C.c_int32), ("order", C.c_int32),
                ("on_device", C.c_int32), ("xcd_blocks", C.c_int32), ("block_mode", C.c_int32),
                ("lane_cols", C.c_int32), ("single_pass", C.c_int32), ("sp_gave_up", C.c_int32)]


class FcooError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built: run `python -c 'import __graft_entry__ as g; g.build()'` "
                      "or `python paper_1705_09905_amd/build.py`")

try:  # load torch's HIP runtime first so that one runtime serves both (same SONAME)
    import torch  # noqa: F401
except ImportError:  # host-only use without torch
    pass

lib = C.CDLL(LIB_PATH)

_vp = C.c_void_p
_i = C.c_int
_i64 = C.c_int64
_SIGS = {
    "fcoo_version": (_i, []),
    "fcoo_last_error": (C.c_char_p, []),
    "fcoo_create": (_i, [_i, C.POINTER(_i64), _i64, C.POINTER(_vp), _vp, C.POINTER(_vp)]),
    "fcoo_build": (_i, [_vp, _i, _i, C.POINTER(fcoo_opts), _vp]),
    "fcoo_info": (_i, [_vp, _i, _i, C.POINTER(fcoo_info_t)]),
    "fcoo_export": (_i, [_vp, _i, _i, C.POINTER(_vp), _vp, _vp, _vp, _vp, _vp, _vp]),
    "fcoo_spmttkrp": (_i, [_vp, _i, C.POINTER(_vp), _i, _i, _vp, _vp]),
    "fcoo_spmttkrp_noalloc": (_i, [_vp, _i, C.POINTER(_vp), _i, _i, _vp, _vp]),
    "fcoo_spttm": (_i, [_vp, _i, _vp, _i, _i, _vp, _vp]),
    "fcoo_spttmc": (_i, [_vp, _i, C.POINTER(_vp), _i, C.POINTER(_i), _vp, _vp]),
    "fcoo_spmttkrp_values": (_i, [_vp, _i, _vp, C.POINTER(_vp), _i, _i, _vp, _vp]),
    "fcoo_model_at_nnz": (_i, [_vp, C.POINTER(_vp), _i, _i, _vp, _vp]),
    "fcoo_resid_spmttkrp": (_i, [_vp, _i, C.POINTER(_vp), _i, _i, _vp, _vp, _vp]),
    "fcoo_cp_als_iter": (_i, [_vp, C.POINTER(_vp), _i, _i, _vp, _vp, _i, _vp, _vp, _vp]),
    "fcoo_gram": (_i, [_vp, _i, _vp, _i, _i, _vp, _vp]),
    "fcoo_set_tile_events": (_i, [_vp, _vp, _vp]),
    "fcoo_device_copy": (_i, [_vp, _vp, _i64, _vp]),
    "fcoo_autotune": (_i, [_vp, _i, _i, C.POINTER(_vp), _i, _i, _vp, _i, _i, C.POINTER(fcoo_opts),
                           C.POINTER(C.c_float), _vp]),
    "fcoo_destroy": (None, [_vp]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args
    globals()[_name] = _f


def check(rc: int) -> None:
    """Raise FcooError for a negative status, with the library's message."""
    if rc != FCOO_OK:
        raise FcooError(rc, lib.fcoo_last_error().decode(errors="replace"))


def ptr_array(ptrs):
    """Host array of device (or host) pointers, for `const void *const *` arguments."""
    return (C.c_void_p * len(ptrs))(*[p if p else None for p in ptrs])
