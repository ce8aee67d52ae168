"""Python surface over the C ABI: an F-COO tensor handle whose operations take
and return torch tensors on the GPU.  torch provides device memory and the
current stream; the computation is the library's."""
from __future__ import annotations

import ctypes as C
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import _lib as L

OPS = {"mttkrp": L.FCOO_OP_MTTKRP, "ttm": L.FCOO_OP_TTM}


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float32:
        return L.FCOO_F32
    if t.dtype == torch.bfloat16:
        return L.FCOO_BF16
    raise TypeError(f"factor dtype {t.dtype} not supported (float32 or bfloat16)")


def _out(out, shape, dtype):
    """The caller's output tensor, checked (the library writes exactly
    prod(shape) elements there), or a new one."""
    torch = _torch()
    if out is None:
        return torch.empty(shape, dtype=dtype, device="cuda")
    if (not isinstance(out, torch.Tensor) or not out.is_cuda or out.dtype != dtype
            or tuple(out.shape) != tuple(shape) or not out.is_contiguous()):
        raise ValueError(f"out must be a contiguous CUDA {dtype} tensor of shape {tuple(shape)}")
    return out


def _index_column(c) -> np.ndarray:
    """One mode's coordinates as int32, refusing values a cast would wrap."""
    a = np.asarray(c)
    if a.dtype.kind not in "iu":
        raise TypeError(f"coordinates must be integers (got {a.dtype})")
    if a.size and a.dtype.itemsize * 8 - (a.dtype.kind == "i") > 31:
        if int(a.min()) < 0 or int(a.max()) > np.iinfo(np.int32).max:
            raise ValueError("coordinates outside the int32 range")
    return np.ascontiguousarray(a, dtype=np.int32)


class Tensor:
    """A sparse tensor in COO form, with F-COO builds per (op, mode).

    coords: (Z, N) integer array, or a list of N integer arrays of length Z;
    vals: Z values (stored as float32); dims: N mode sizes.
    """

    def __init__(self, coords, vals, dims: Sequence[int]):
        dims = [int(d) for d in dims]
        N = len(dims)
        if isinstance(coords, np.ndarray) and coords.ndim == 2:
            cols = [_index_column(coords[:, m]) for m in range(N)]
        else:
            cols = [_index_column(c) for c in coords]
        if len(cols) != N:
            raise ValueError("coords must give one index array per mode")
        vals = np.ascontiguousarray(np.asarray(vals), dtype=np.float32)
        Z = vals.shape[0]
        for c in cols:
            if c.shape[0] != Z:
                raise ValueError("index arrays and values differ in length")
        self.dims = dims
        self.order = N
        self.nnz = Z
        self._h = C.c_void_p()
        d = (C.c_int64 * N)(*dims)
        L.check(L.fcoo_create(N, d, Z, L.ptr_array([c.ctypes.data for c in cols]),
                              vals.ctypes.data, C.byref(self._h)))
        self._vals = vals

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                L.fcoo_destroy(h)
            except TypeError:  # interpreter shutdown: the binding is already gone
                pass
            self._h = C.c_void_p()

    @property
    def handle(self):
        return self._h

    # ---- build / inspect --------------------------------------------------
    def build(self, mode: int, op: str = "mttkrp", threadlen: int = 0, tile_nnz: int = 0,
              host_only: bool = False, device: bool = False, xcd_blocks: int = 0,
              xcd_mode: int = -1, lane_cols: int = 0, single_pass: bool = False) -> "Tensor":
        """F-COO encoding of (op, mode); device=True sorts and encodes on the GPU;
        xcd_blocks=8 (SpMTTKRP) splits the nonzeros into per-XCD blocks by
        ranges of product mode xcd_mode (-1: the one with the most rows);
        lane_cols (4 or 8, 0: default) sets the bfloat16 row piece per lane;
        single_pass finishes segments that cross tiles inside the tile kernel."""
        o = L.fcoo_opts(threadlen, tile_nnz, 1 if host_only else 0, 1 if device else 0, int(xcd_blocks),
                        int(xcd_mode) + 1, int(lane_cols), 1 if single_pass else 0)
        stream = C.c_void_p(0) if host_only else _stream()
        L.check(L.fcoo_build(self._h, int(mode), OPS[op], C.byref(o), stream))
        return self

    def autotune(self, mode: int, op: str, factors, tiles: Optional[Sequence[int]] = None,
                 reps: int = 3) -> Dict[str, float]:
        """Time each candidate layout for (op, mode) with these factors (op
        'ttm': factors[mode] is U; SpMTTKRP also tries XCD blocks split by each
        product mode; bfloat16 factors also both lane chunks) and keep the
        fastest.  Returns dict(tile_nnz, threadlen, xcd_blocks, xcd_mode,
        lane_cols, ms), xcd_mode -1 when unblocked or by the default mode."""
        if op == "mttkrp":
            fp, R, dt = self._factors(factors, skip=mode)
        else:
            U = factors[mode]
            ptrs = [0] * self.order
            ptrs[mode] = U.data_ptr()
            fp, R, dt = L.ptr_array(ptrs), int(U.shape[1]), _dtype_code(U)
        cand = None if tiles is None else (C.c_int * len(tiles))(*[int(x) for x in tiles])
        best = L.fcoo_opts()
        ms = C.c_float()
        L.check(L.fcoo_autotune(self._h, int(mode), OPS[op], fp, dt, R, cand, 0 if tiles is None else len(tiles),
                                int(reps), C.byref(best), C.byref(ms), _stream()))
        return {"tile_nnz": int(best.tile_nnz), "threadlen": int(best.threadlen),
                "xcd_blocks": int(best.xcd_blocks), "xcd_mode": int(best.xcd_mode) - 1,
                "lane_cols": int(best.lane_cols), "ms": float(ms.value)}

    def info(self, mode: int, op: str = "mttkrp") -> Dict[str, int]:
        i = L.fcoo_info_t()
        L.check(L.fcoo_info(self._h, int(mode), OPS[op], C.byref(i)))
        return {f: int(getattr(i, f)) for f, _ in L.fcoo_info_t._fields_}

    def export(self, mode: int, op: str = "mttkrp") -> Dict[str, np.ndarray]:
        inf = self.info(mode, op)
        Z, nseg = inf["nnz"], inf["nseg"]
        nprod = self.order - 1 if op == "mttkrp" else 1
        pidx = [np.empty(Z, np.int32) for _ in range(nprod)]
        val = np.empty(Z, np.float32)
        bf = np.empty((Z + 7) // 8, np.uint8)
        sf = np.empty((inf["npart"] + 31) // 32, np.uint32)
        seg = np.empty(nseg if op == "mttkrp" else nseg * (self.order - 1), np.int32)
        ts0 = np.empty(inf["ntiles"], np.int32)
        perm = np.empty(Z, np.int32)
        L.check(L.fcoo_export(self._h, int(mode), OPS[op], L.ptr_array([p.ctypes.data for p in pidx]),
                              val.ctypes.data, bf.ctypes.data, sf.ctypes.data, seg.ctypes.data,
                              ts0.ctypes.data, perm.ctypes.data))
        out = dict(pidx=pidx, val=val, bf=bf, sf=sf, tile_seg0=ts0, perm=perm, nseg=nseg)
        if op == "mttkrp":
            out["seg_row"] = seg
        else:
            out["fibres"] = seg.reshape(nseg, self.order - 1)
        return out

    # ---- operations -------------------------------------------------------
    def _factors(self, factors, skip: int = -1):
        torch = _torch()
        if len(factors) != self.order:
            raise ValueError(f"need {self.order} factors (use None for the skipped mode)")
        R, dt, ptrs = None, None, []
        for m, f in enumerate(factors):
            if m == skip and f is None:
                ptrs.append(0)
                continue
            if not isinstance(f, torch.Tensor) or not f.is_cuda:
                raise TypeError(f"factor {m} must be a CUDA torch tensor")
            if f.dim() != 2 or f.shape[0] != self.dims[m] or not f.is_contiguous():
                raise ValueError(f"factor {m} must be a contiguous {self.dims[m]} x R matrix")
            R = f.shape[1] if R is None else R
            if f.shape[1] != R:
                raise ValueError("factors differ in rank")
            code = _dtype_code(f)
            dt = code if dt is None else dt
            if code != dt:
                raise ValueError("factors differ in dtype")
            ptrs.append(f.data_ptr())
        return L.ptr_array(ptrs), int(R), dt

    def spmttkrp(self, mode: int, factors, out=None):
        """M = X_(mode) (Khatri-Rao product of the other factors), float32."""
        torch = _torch()
        fp, R, dt = self._factors(factors, skip=mode)
        out = _out(out, (self.dims[mode], R), torch.float32)
        L.check(L.fcoo_spmttkrp(self._h, int(mode), fp, dt, R, out.data_ptr(), _stream()))
        return out

    def spttm(self, mode: int, U, out=None, return_fibres: bool = False):
        """Y = X x_mode U over the fibres of the other modes (nseg x R, float32).
        With return_fibres, also the fibres' coordinates (nseg x (N-1) int32,
        the other modes in ascending order, lexicographically increasing):
        returns (Y, fibres)."""
        torch = _torch()
        if U.dim() != 2 or U.shape[0] != self.dims[mode] or not U.is_contiguous() or not U.is_cuda:
            raise ValueError("U must be a contiguous CUDA dims[mode] x R matrix")
        nseg = self.info(mode, "ttm")["nseg"]
        R = int(U.shape[1])
        out = _out(out, (nseg, R), torch.float32)
        L.check(L.fcoo_spttm(self._h, int(mode), U.data_ptr(), _dtype_code(U), R, out.data_ptr(),
                             _stream()))
        if return_fibres:
            seg = np.empty((nseg, self.order - 1), np.int32)
            L.check(L.fcoo_export(self._h, int(mode), OPS["ttm"], None, None, None, None, seg.ctypes.data,
                                  None, None))
            return out, seg
        return out

    def spttmc(self, mode: int, factors, out=None):
        """Y_(mode) = X times every other factor (Eq. 4): row i, column
        (p_1, p_2, ..) in Kronecker order (later modes fastest) holds
        sum val * U_m1[i_m1, p_1] * U_m2[i_m2, p_2] * ..  (float32,
        dims[mode] x prod of the other factors' column counts).  Factors may
        differ in column count; they share one dtype.  Uses the SpMTTKRP
        build of the mode."""
        torch = _torch()
        if len(factors) != self.order:
            raise ValueError(f"need {self.order} factors (use None for the skipped mode)")
        ptrs, ranks, dt, W = [], [], None, 1
        for m, f in enumerate(factors):
            if m == mode:
                ptrs.append(0)
                ranks.append(1)
                continue
            if not isinstance(f, torch.Tensor) or not f.is_cuda:
                raise TypeError(f"factor {m} must be a CUDA torch tensor")
            if f.dim() != 2 or f.shape[0] != self.dims[m] or not f.is_contiguous():
                raise ValueError(f"factor {m} must be a contiguous {self.dims[m]} x R_{m} matrix")
            code = _dtype_code(f)
            dt = code if dt is None else dt
            if code != dt:
                raise ValueError("factors differ in dtype")
            ptrs.append(f.data_ptr())
            ranks.append(int(f.shape[1]))
            W *= int(f.shape[1])
        out = _out(out, (self.dims[mode], W), torch.float32)
        rk = (C.c_int * self.order)(*ranks)
        L.check(L.fcoo_spttmc(self._h, int(mode), L.ptr_array(ptrs), dt, rk, out.data_ptr(), _stream()))
        return out

    def spmttkrp_values(self, mode: int, g, factors, out=None):
        """SpMTTKRP with the values replaced by g (float32, input order)."""
        torch = _torch()
        fp, R, dt = self._factors(factors, skip=mode)
        if g.dtype != torch.float32 or not g.is_cuda or g.numel() != self.nnz or not g.is_contiguous():
            raise ValueError("g must be a contiguous CUDA float32 vector of nnz values")
        out = _out(out, (self.dims[mode], R), torch.float32)
        L.check(L.fcoo_spmttkrp_values(self._h, int(mode), g.data_ptr(), fp, dt, R, out.data_ptr(),
                                       _stream()))
        return out

    def model_at_nnz(self, factors, out=None):
        """xhat[e] = sum_r prod_m A_m[i_m(e), r] in input order (float32)."""
        torch = _torch()
        fp, R, dt = self._factors(factors)
        out = _out(out, (self.nnz,), torch.float32)
        L.check(L.fcoo_model_at_nnz(self._h, fp, dt, R, out.data_ptr(), _stream()))
        return out

    def resid_spmttkrp(self, mode: int, factors, out=None, loss=None):
        """Gradient of L = (1/2Z) sum (xhat - x)^2 w.r.t. factor `mode`;
        `loss` (CUDA float64 scalar tensor) receives L when given."""
        torch = _torch()
        fp, R, dt = self._factors(factors)
        out = _out(out, (self.dims[mode], R), torch.float32)
        if loss is not None and (not isinstance(loss, torch.Tensor) or not loss.is_cuda
                                 or loss.dtype != torch.float64 or loss.numel() != 1):
            raise ValueError("loss must be a CUDA float64 tensor of one element")
        lp = loss.data_ptr() if loss is not None else None
        L.check(L.fcoo_resid_spmttkrp(self._h, int(mode), fp, dt, R, out.data_ptr(), lp, _stream()))
        return out

    def gram(self, mode: int, A, out=None):
        torch = _torch()
        if (not isinstance(A, torch.Tensor) or not A.is_cuda or A.dim() != 2
                or A.shape[0] != self.dims[mode] or not A.is_contiguous()):
            raise ValueError(f"A must be a contiguous CUDA {self.dims[mode]} x R matrix")
        R = int(A.shape[1])
        out = _out(out, (R, R), torch.float64)
        L.check(L.fcoo_gram(self._h, int(mode), A.data_ptr(), _dtype_code(A), R, out.data_ptr(),
                            _stream()))
        return out
