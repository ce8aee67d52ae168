"""Benchmark of the F-COO hot path on one MI355X.

Workload (one "step"): the 3-order Zipf(1.1) tensor 100,000 x 80,000 x 60,000
with 20M unique nonzeros (values U(0,1), float32), SpMTTKRP and SpTTM in
every mode at R = 16 and R = 32, float32 factors N(0,1) -- 12 operations.
Inputs and F-COO arrays are resident in HBM before the timed region.

value = algorithmic bytes of the 12 operations / step time (GB/s): per
nonzero the index and value streams, the bf / sf flags, one factor row per
product mode gathered, plus the output rows written (the dense unfolding and
Khatri-Rao product that the method avoids are not counted).  Gathered rows
are often served by the caches, so this rate counts cache traffic too; the
HBM fraction is taken from measured traffic instead (roofline below).

The same JSON line carries CP-ALS (Algorithm 1) on the planted rank-16
tensor 200,000 x 150,000 x 100,000 with 100M uniform nonzeros at R = 16,
ten sweeps with float32 and with bfloat16 factor storage: seconds per sweep,
the fit of every sweep, and (with the CPU leg) the float64 oracle's fits and
the CP model at sampled nonzeros against the oracle's; and CP-ALS on the
order-4 Zipf tensor 50,000 x 20,000 x 5,000 x 1,000 with 50M nonzeros at
R = 32 (seconds per sweep and fits, float32 and bfloat16).

The roofline object describes the dominant kernel (the SpMTTKRP or SpTTM
tile kernel with the largest total time), timed alone with HIP events that
the library records around each tile-kernel launch.
"""
from __future__ import annotations

import argparse
import ctypes as C
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0          # MI355X HBM3E, vendor figure
METRIC = "SpMTTKRP GB/s & GFLOP/s (%HBM peak), CP-ALS s/iter, BF16 vs FP32 at stated fit"
WORKLOAD_CFG = 1
KERNEL_SOURCES = ["fcoo_segscan.h", "fcoo_device.h", "fcoo_seg_dispatch.h", "fcoo_ops.hip"]


def kernel_hash() -> str:
    """Hash of the kernel sources with comments and blank lines removed, so
    stored counters stay tied to the code they were taken from."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1705_09905_amd", "csrc", f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update("\n".join(ln.rstrip() for ln in text.splitlines() if ln.strip()).encode())
    return h.hexdigest()[:16]


def op_bytes(op, Z, N, R, nseg, In, P, sf=4):
    """Algorithmic bytes of one SpMTTKRP / SpTTM on one mode.  Of the flags
    only bf is counted: the kernels derive the heads before each run from bf
    popcounts and read no sf word (P is kept for the record)."""
    flags = (Z + 7) // 8
    if op == "mttkrp":
        return 4 * Z * (N - 1) + 4 * Z + flags + 4 * nseg + Z * (N - 1) * R * sf + 4 * In * R
    return 4 * Z + 4 * Z + flags + Z * R * sf + 4 * nseg * R


def compulsory_bytes(op, Z, N, R, nseg, In, P, distinct, mode, sf=4):
    """Bytes one SpMTTKRP / SpTTM must move at the least: the streams and
    the output as in op_bytes, but each distinct factor row read once."""
    flags = (Z + 7) // 8
    if op == "mttkrp":
        rows = sum(distinct[k] for k in range(N) if k != mode)
        return 4 * Z * (N - 1) + 4 * Z + flags + 4 * nseg + rows * R * sf + 4 * In * R
    return 8 * Z + flags + distinct[mode] * R * sf + 4 * nseg * R


def device_copy(torch, src, dst):
    """The library's own plain copy kernel (fcoo_device_copy) on torch's stream."""
    from paper_1705_09905_amd import _lib
    _lib.check(_lib.fcoo_device_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()),
                                     src.numel() * src.element_size(),
                                     C.c_void_p(torch.cuda.current_stream().cuda_stream)))


def copy_bandwidth(torch, nbytes=1 << 30, reps=10):
    """Device-to-device copy rate (read + write bytes / time) of the library's
    plain copy kernel over 1 GiB, for comparison with the kernels' traffic."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    device_copy(torch, src, dst)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        device_copy(torch, src, dst)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2 * nbytes / (ms / 1e3) / 1e9


def op_flops(op, Z, N, R):
    return Z * R * N if op == "mttkrp" else 2 * Z * R


class HipEvents:
    """hipEvent_t pool through the HIP runtime already loaded by torch."""

    def __init__(self):
        self.hip = C.CDLL("libamdhip64.so.7")
        self.hip.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        self.hip.hipEventDestroy.argtypes = [C.c_void_p]
        self.events = []

    def new(self):
        e = C.c_void_p()
        rc = self.hip.hipEventCreate(C.byref(e))
        if rc != 0:
            raise RuntimeError(f"hipEventCreate failed: {rc}")
        self.events.append(e)
        return e

    def ms(self, a, b):
        out = C.c_float()
        rc = self.hip.hipEventElapsedTime(C.byref(out), a, b)
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed: {rc}")
        return float(out.value)

    def close(self):
        for e in self.events:
            self.hip.hipEventDestroy(e)
        self.events = []


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(t, Rs, sample_nnz, threads, reps=5):
    """The float64 C oracle (plain COO loops, OpenMP) on a bounded sample of
    the same workload: the first `sample_nnz` nonzeros of the shuffled list.
    Per operation one warm-up run, then the median of `reps` timed runs."""
    from oracle import cpu
    import synth
    Zs = min(sample_nnz, t.nnz)
    idx = [np.ascontiguousarray(i[:Zs]) for i in t.idx]
    vals = t.vals[:Zs].astype(np.float32).astype(np.float64)
    N = t.order
    total_bytes, total_s, used = 0, 0.0, 1
    per_op = {}
    groups = [cpu.ttm_group(t.dims, idx, m) for m in range(N)]

    def med(fn):
        fn()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            r = fn()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts)), r

    for R in Rs:
        F = [f.astype(np.float32).astype(np.float64) for f in synth.factors(t.dims, R, WORKLOAD_CFG)]
        for m in range(N):
            dt, (_, used) = med(lambda: cpu.mttkrp(t.dims, idx, vals, F, m, nthreads=threads,
                                                   return_threads=True))
            per_op[("mttkrp", m, R)] = dt
            total_s += dt
            nseg = len(np.unique(idx[m]))
            total_bytes += op_bytes("mttkrp", Zs, N, R, nseg, t.dims[m], -(-Zs // 16))
            dt, (fib, _, _) = med(lambda: cpu.ttm(t.dims, idx, vals, F[m], m, group=groups[m],
                                                  nthreads=threads, return_threads=True))
            per_op[("ttm", m, R)] = dt
            total_s += dt
            total_bytes += op_bytes("ttm", Zs, N, R, fib.shape[0], t.dims[m], -(-Zs // 16))
    return {"value": round(total_bytes / total_s / 1e9, 3), "unit": "GB/s", "cores": int(used),
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"first {Zs} of {t.nnz} nonzeros (seeded shuffle order), SpMTTKRP + SpTTM, "
                      f"every mode, R in {list(Rs)}, float64; per operation 1 warm-up then the "
                      f"median of {reps} runs, {total_s:.2f} s summed (fibre grouping excluded)",
            "_per_op_s": per_op, "_sample_nnz": Zs}


def op_parity(t, Rs, outs, threads):
    """Full-size parity of the step's outputs (the last timed launch of each
    operation, which is bitwise repeatable): relative Frobenius error against
    the float64 C oracle on the whole tensor, from the same float32 inputs."""
    from oracle import cpu
    import synth
    vals = t.vals.astype(np.float32).astype(np.float64)
    N = t.order
    err = {}
    for R in Rs:
        F = [f.astype(np.float32).astype(np.float64) for f in synth.factors(t.dims, R, WORKLOAD_CFG)]
        for m in range(N):
            want = cpu.mttkrp(t.dims, t.idx, vals, F, m, nthreads=threads)
            got = outs[("mttkrp", m, R)].cpu().numpy().astype(np.float64)
            err[("mttkrp", m, R)] = float(np.linalg.norm(got - want) / np.linalg.norm(want))
            _, want = cpu.ttm(t.dims, t.idx, vals, F[m], m, nthreads=threads)
            got = outs[("ttm", m, R)].cpu().numpy().astype(np.float64)
            err[("ttm", m, R)] = (float(np.linalg.norm(got - want) / np.linalg.norm(want))
                                  if got.shape == want.shape else float("inf"))
    return err


def cp_oracle(t, R, sweeps, init, record=None, storage="f64"):
    """The float64 oracle's CP-ALS (Algorithm 1) on the full workload, with
    the C COO loop for its MTTKRPs, from the same initial factors; storage
    'bf16' rounds every stored factor to bfloat16 as the bfloat16 path does."""
    from oracle import cpu, ref
    vals = t.vals.astype(np.float32).astype(np.float64)
    t0 = time.perf_counter()
    out = ref.cp_als(t.dims, t.idx, vals, R, [a.astype(np.float64) for a in init], sweeps, storage=storage,
                     mttkrp=lambda d, i, v, F, n: cpu.mttkrp(d, i, v, F, n), record=record)
    return out["fits"], (time.perf_counter() - t0) / sweeps


def cp_gpu(h, t, R, sweeps, init, dtype, keep_after=()):
    """CP-ALS sweeps on the device; wall time of every sweep (each call ends
    with the 8-byte fit read-back).  Factors and lambda after the sweeps in
    `keep_after` are copied to the host outside the timed calls.  Returns
    fits, seconds and kept factors per sweep; each sweep's pseudo-inverse
    mask (bit n: mode n's normal equations took the pseudo-inverse) is left
    in cp_gpu.used_pinv."""
    import torch
    from paper_1705_09905_amd import _lib
    tdt = torch.float32 if dtype == "f32" else torch.bfloat16
    F = [torch.tensor(a.astype(np.float32), device="cuda").to(tdt).contiguous() for a in init]
    lam = torch.zeros(R, dtype=torch.float64, device="cuda")
    grams = torch.zeros((t.order, R, R), dtype=torch.float64, device="cuda")
    fp = _lib.ptr_array([f.data_ptr() for f in F])
    fit, used = C.c_double(), C.c_int()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    code = _lib.FCOO_F32 if dtype == "f32" else _lib.FCOO_BF16
    fits, secs, kept = [], [], {}
    cp_gpu.used_pinv = []
    torch.cuda.synchronize()
    for s in range(sweeps):
        t0 = time.perf_counter()
        _lib.check(_lib.fcoo_cp_als_iter(h.handle, fp, code, R, lam.data_ptr(), grams.data_ptr(),
                                         1 if s else 0, C.byref(fit), C.byref(used), stream))
        secs.append(time.perf_counter() - t0)
        fits.append(float(fit.value))
        cp_gpu.used_pinv.append(int(used.value))
        if s + 1 in keep_after:
            kept[s + 1] = ([f.to(torch.float64).cpu().numpy() for f in F], lam.cpu().numpy())
    return fits, secs, kept


def model_sample(idx, factors, lam, sel):
    """CP model sum_r lam_r prod_m A_m[i_m, r] at the sampled nonzeros, by the
    float64 oracle's C loop (the CPU leg compares models, which are unique,
    where factors are not)."""
    from oracle import cpu
    F = [np.asarray(a, np.float64) for a in factors]
    F[-1] = F[-1] * np.asarray(lam, np.float64)[None, :]
    return cpu.model_at([np.ascontiguousarray(i[sel]) for i in idx], F)


def cp_planted(args, log, cpu_rec):
    """CP-ALS (Algorithm 1) on the planted rank-16 tensor 200,000 x 150,000 x
    100,000 with 100M uniform nonzeros, R = 16: float32 and bfloat16 factor
    storage from the same start, seconds per sweep (median of sweeps 2..S)
    and the fit of every sweep.  With the CPU leg (cpu_rec not None): the
    float64 oracle's sweeps (its seconds per sweep are the CP-ALS CPU
    baseline), the largest fit difference, and the relative error of the CP
    model at sampled nonzeros after sweep 1 and sweep S.  ALS treats the
    unsampled cells as zeros, so every fit here is tiny (about 7e-6): the
    model at the nonzeros is what separates a right result from a wrong one."""
    import torch
    import synth
    from paper_1705_09905_amd import Tensor
    cfg, R, S = 3, 16, args.cp_sweeps
    t0 = time.time()
    t = synth.config_tensor(cfg)
    log(f"generated {t.name} Z={t.nnz} in {time.time() - t0:.1f}s")
    h = Tensor(t.idx, t.vals, t.dims)
    init = synth.factors(t.dims, R, cfg, role="init")
    t0 = time.time()
    for m in range(t.order):
        h.build(m, "mttkrp", threadlen=args.threadlen, tile_nnz=4096, device=True)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    log(f"planted CP-ALS: built in {build_s:.2f}s")
    keep = (1, S) if cpu_rec is not None else ()
    rec = {"workload": f"{t.name}: CP-ALS, R = {R}, {S} sweeps", "dims": t.dims, "nnz": t.nnz, "R": R,
           "sweeps": S, "layout": {}, "device_build_s": round(build_s, 3)}
    kept = {}
    for dt in ("f32", "bf16"):
        # tile size, XCD layout and lane chunk per mode, chosen by timing
        # SpMTTKRP with this storage type's factors (not timed below)
        Ft = [torch.tensor(a.astype(np.float32), device="cuda").to(
            torch.float32 if dt == "f32" else torch.bfloat16).contiguous() for a in init]
        layout = {}
        for m in range(t.order):
            r = h.autotune(m, "mttkrp", Ft, tiles=[2048, 4096, 8192])
            layout[f"mode{m}"] = {k: r[k] for k in ("tile_nnz", "xcd_blocks", "xcd_mode", "lane_cols")}
        del Ft
        rec["layout"][dt] = layout
        log(f"planted CP-ALS {dt}: layout {layout}")
        fits, secs, kept[dt] = cp_gpu(h, t, R, S, init, dt, keep_after=keep)
        rec[dt] = {"s_per_iter": round(float(np.median(secs[1:] if len(secs) > 1 else secs)), 6),
                   "s_per_iter_min": round(float(np.min(secs)), 6),
                   "s_per_iter_max": round(float(np.max(secs)), 6),
                   "fits": [float(f"{f:.6g}") for f in fits],
                   "used_pinv": list(cp_gpu.used_pinv)}
        log(f"cp-als {dt}: {rec[dt]['s_per_iter'] * 1e3:.3f} ms/sweep")
    rec["bf16_speedup_vs_f32"] = round(rec["f32"]["s_per_iter"] / rec["bf16"]["s_per_iter"], 3)
    del h
    if cpu_rec is not None:
        orec = []
        t0 = time.time()
        fits, s_per = cp_oracle(t, R, S, init, record=orec)
        log(f"oracle CP-ALS in {time.time() - t0:.1f}s")
        cpu_rec["cp_als"] = {"value": round(s_per, 3), "unit": "s/iter",
                             "cores": len(os.sched_getaffinity(0)), "kind": "oracle",
                             "sample": f"the whole planted 100M tensor, {S} sweeps, float64, C MTTKRP loops",
                             "fits": [float(f"{f:.6g}") for f in fits]}
        # the same oracle with its stored factors rounded to bfloat16: the
        # bfloat16 path's kernel error, apart from the end-to-end drift of
        # bfloat16 storage over the sweeps (which depends on summation order)
        orec16 = []
        fits16, _ = cp_oracle(t, R, S, init, record=orec16, storage="bf16")
        log(f"bfloat16-storage oracle CP-ALS in {time.time() - t0:.1f}s")
        sel = np.unique(np.random.default_rng(cfg).integers(0, t.nnz, size=args.cp_model_sample))
        want = {s: model_sample(t.idx, orec[s - 1][0], orec[s - 1][1], sel) for s in keep}
        want16 = {s: model_sample(t.idx, orec16[s - 1][0], orec16[s - 1][1], sel) for s in keep}

        def rel(a, b):
            return float(f"{np.linalg.norm(a - b) / np.linalg.norm(b):.3g}")

        for dt in ("f32", "bf16"):
            rec[dt]["max_abs_fit_diff_vs_oracle"] = float(
                f"{max(abs(a - b) for a, b in zip(rec[dt]['fits'], fits)):.3g}")
            got = {s: model_sample(t.idx, kept[dt][s][0], kept[dt][s][1], sel) for s in keep}
            rec[dt]["model_rel_err_vs_oracle"] = {f"sweep{s}": rel(got[s], want[s]) for s in keep}
            if dt == "bf16":
                rec[dt]["max_abs_fit_diff_vs_bf16_storage_oracle"] = float(
                    f"{max(abs(a - b) for a, b in zip(rec[dt]['fits'], fits16)):.3g}")
                rec[dt]["model_rel_err_vs_bf16_storage_oracle"] = {f"sweep{s}": rel(got[s], want16[s])
                                                                   for s in keep}
        rec["model_sample"] = f"{sel.size} seeded distinct nonzeros"
    return rec


def cp_order4(args, log):
    """CP-ALS (Algorithm 1) on the order-4 Zipf(1.1) tensor 50,000 x 20,000 x
    5,000 x 1,000 with 50M nonzeros, R = 32: float32 and bfloat16 factor
    storage from the same start, layouts autotuned per storage type,
    seconds per sweep (median of sweeps 2..S) and the fit of every sweep.
    Its parity against the oracle (fits and the CP model at sampled
    nonzeros) is the order-4 GPU test; no oracle runs here."""
    import torch
    import synth
    from paper_1705_09905_amd import Tensor
    cfg, R, S = 2, 32, args.cp4_sweeps
    t0 = time.time()
    t = synth.config_tensor(cfg)
    log(f"generated {t.name} Z={t.nnz} in {time.time() - t0:.1f}s")
    h = Tensor(t.idx, t.vals, t.dims)
    init = synth.factors(t.dims, R, cfg, role="init")
    rec = {"workload": f"{t.name}: CP-ALS, R = {R}, {S} sweeps", "dims": t.dims, "nnz": t.nnz, "R": R,
           "sweeps": S, "layout": {}}
    for dt in ("f32", "bf16"):
        Ft = [torch.tensor(a.astype(np.float32), device="cuda").to(
            torch.float32 if dt == "f32" else torch.bfloat16).contiguous() for a in init]
        layout = {}
        for m in range(t.order):
            r = h.autotune(m, "mttkrp", Ft, tiles=[2048, 4096, 8192])
            layout[f"mode{m}"] = {k: r[k] for k in ("tile_nnz", "xcd_blocks", "xcd_mode", "lane_cols")}
        del Ft
        rec["layout"][dt] = layout
        fits, secs, _ = cp_gpu(h, t, R, S, init, dt)
        rec[dt] = {"s_per_iter": round(float(np.median(secs[1:] if len(secs) > 1 else secs)), 6),
                   "s_per_iter_min": round(float(np.min(secs)), 6),
                   "s_per_iter_max": round(float(np.max(secs)), 6),
                   "fits": [float(f"{f:.6g}") for f in fits]}
        log(f"order-4 cp-als {dt}: {rec[dt]['s_per_iter'] * 1e3:.3f} ms/sweep, layout {layout}")
    rec["bf16_speedup_vs_f32"] = round(rec["f32"]["s_per_iter"] / rec["bf16"]["s_per_iter"], 3)
    rec["max_abs_fit_diff_bf16_vs_f32"] = float(
        f"{max(abs(a - b) for a, b in zip(rec['f32']['fits'], rec['bf16']['fits'])):.3g}")
    del h
    return rec


def kernel_symbol(op, R, N):
    """Demangled name of the tile-kernel instantiation that runs (op, R)
    with float32 factors (16-byte lanes: 4 columns per lane)."""
    lanes = (R + 3) // 4
    lpn = 1
    while lpn < lanes:
        lpn *= 2
    lpn = min(lpn, 16)
    np_ = (N - 1) if op == "mttkrp" else 1
    npt = np_ if np_ <= 3 else 0
    return (f"void fcoo::dev::seg_tile_kernel<float, 4, {lpn}, {npt}, false, "
            f"{'true' if op == 'mttkrp' else 'false'}, false, 1>(fcoo::dev::SegArgs)")


def rank_tile(R):
    """Columns one tile-kernel workgroup covers for float32 factors: 4 per
    lane, lanes per nonzero the next power of two of R / 4 (at most 16); 64
    one-column lanes when R is not a multiple of 4."""
    if R % 4:
        return 64
    lanes = R // 4
    lpn = 1
    while lpn < lanes:
        lpn *= 2
    return min(lpn, 16) * 4


def load_traffic(khash):
    p = os.path.join(ROOT, "profiles", "traffic_tile_kernel_zipf20M.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("kernel_hash") != khash:
        return None
    return d


EXTRA_WORKLOADS = {
    # name: (workload index in synth.CONFIGS, rank, kind)
    "cpals-order4-zipf50M": (2, 32, "cpals"),
    "cpals-planted100M": (3, 16, "cpals"),
    "gradcp-zipf200M": (4, 64, "gradcp"),
}


def run_extra(args, log):
    """CP-ALS (ten sweeps, float32 and bfloat16 factors) or gradient-based CP
    (fused residual SpMTTKRP steps with Adam) on one of the large workloads.
    Prints one JSON line; value = float32 seconds per sweep / per step."""
    import torch
    import synth
    from paper_1705_09905_amd import CPMSELoss, Tensor
    cfg, R, kind = EXTRA_WORKLOADS[args.workload]
    t0 = time.time()
    t = synth.config_tensor(cfg)
    log(f"generated {t.name} Z={t.nnz} in {time.time() - t0:.1f}s")
    h = Tensor(t.idx, t.vals, t.dims)
    t0 = time.time()
    for m in range(t.order):
        h.build(m, "mttkrp", threadlen=args.threadlen, tile_nnz=args.tile)
    build_s = time.time() - t0
    N = t.order
    init = synth.factors(t.dims, R, cfg, role="init")
    layout = {}

    def tune(dt):
        # layout per mode (tile size, XCD blocks, lane chunk) chosen by timing
        # SpMTTKRP with this storage type's factors; the fused residual kernel
        # of gradient CP prefers other tile sizes than plain SpMTTKRP, so there
        # only the XCD layout is chosen
        if args.tile:
            return
        Ft = [torch.tensor(a.astype(np.float32), device="cuda").to(
            torch.float32 if dt == "f32" else torch.bfloat16).contiguous() for a in init]
        cand = [2048, 4096, 8192] if kind == "cpals" else [4096]
        lay = {}
        for m in range(N):
            r = h.autotune(m, "mttkrp", Ft, tiles=cand)
            lay[f"mode{m}"] = {k: r[k] for k in ("tile_nnz", "xcd_blocks", "xcd_mode", "lane_cols")}
        layout[dt] = lay
        log(f"autotuned layout {dt}: {lay}")

    if kind != "cpals":
        tune("f32")
    # slices (non-empty rows) per mode: the segments of the plain layout, which
    # the byte model counts whatever layout the autotuner keeps
    nslices = [int(np.count_nonzero(np.bincount(t.idx[m], minlength=t.dims[m]))) for m in range(N)]
    rec = {"metric": METRIC, "n_gpus": 1, "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "data": "synthetic", "build_s": round(build_s, 2),
           "config": {"workload": f"{t.name}: " + ("CP-ALS" if kind == "cpals" else "gradient CP (MSE, Adam)")
                      + f", R = {R}", "dims": t.dims, "nnz": t.nnz, "R": R,
                      "threadlen": args.threadlen, "tile_nnz": layout or args.tile}}

    def mttkrp_bytes(sf, own=False):
        b = 0
        for m in range(N):
            b += op_bytes("mttkrp", t.nnz, N, R, nslices[m], t.dims[m], -(-t.nnz // args.threadlen), sf)
            if own:
                b += t.dims[m] * R * sf
        return b

    if kind == "cpals":
        sweeps = args.cp_sweeps
        rec["sweeps"] = sweeps
        for dt in ("f32", "bf16"):
            tune(dt)
            fits, secs, _ = cp_gpu(h, t, R, sweeps, init, dt)
            s_it = float(np.median(secs[1:] if len(secs) > 1 else secs))
            B = mttkrp_bytes(4 if dt == "f32" else 2)
            rec[dt] = {"s_per_iter": round(s_it, 6), "fits": [round(f, 6) for f in fits],
                       "spmttkrp_bytes_per_sweep": B, "GBps_spmttkrp_bytes": round(B / s_it / 1e9, 1)}
            log(f"cp-als {dt}: {s_it * 1e3:.3f} ms/sweep, fits {rec[dt]['fits']}")
        rec["value"], rec["unit"], rec["dtype"] = rec["f32"]["s_per_iter"], "s/iter", "f32"
        if not args.no_cpu:
            fits, s_per = cp_oracle(t, R, sweeps, init)
            threads = len(os.sched_getaffinity(0))
            rec["cpu_baseline"] = {"value": round(s_per, 3), "unit": "s/iter", "cores": threads,
                                   "kind": "oracle", "fits": [round(f, 6) for f in fits],
                                   "sample": f"full workload, {sweeps} sweeps, float64, C MTTKRP loops"}
            for dt in ("f32", "bf16"):
                rec[dt]["max_abs_fit_diff_vs_oracle"] = round(
                    max(abs(a - b) for a, b in zip(rec[dt]["fits"], fits)), 6)
    else:
        steps, warm = args.steps, args.warmup
        rec["steps"], rec["warmup"] = steps, warm
        for dt in ("f32", "bf16"):
            masters = [torch.tensor(a.astype(np.float32), device="cuda").requires_grad_() for a in init]
            opt = torch.optim.Adam(masters, lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
            losses = []

            def step():
                opt.zero_grad()
                loss = CPMSELoss.apply(h, dt, *masters)
                loss.backward()
                opt.step()
                return loss

            for _ in range(warm):
                losses.append(step())
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(steps):
                losses.append(step())
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / steps
            B = mttkrp_bytes(4 if dt == "f32" else 2, own=True)
            rec[dt] = {"ms_per_step": round(ms, 4), "losses": [round(float(x.detach()), 6) for x in losses],
                       "fused_resid_bytes_per_step": B, "GBps_fused_resid_bytes": round(B / ms / 1e6, 1)}
            log(f"gradient CP {dt}: {ms:.3f} ms/step")
        rec["value"], rec["unit"], rec["dtype"] = rec["f32"]["ms_per_step"] / 1e3, "s/step", "f32"
    print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="zipf20M", choices=["zipf20M"] + list(EXTRA_WORKLOADS),
                    help="zipf20M: the SpMTTKRP/SpTTM bench (default); the others time CP-ALS or "
                         "gradient CP on a large workload")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--ranks", default="16,32")
    ap.add_argument("--nnz", type=int, default=0, help="override the nonzero count (quick runs)")
    ap.add_argument("--threadlen", type=int, default=16)
    ap.add_argument("--tile", type=int, default=0, help="tile_nnz of every build (0: autotune per op and mode)")
    ap.add_argument("--tile-ttm", type=int, default=0, help="with --tile: another tile_nnz for the SpTTM builds")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=10_000_000,
                    help="nonzeros of the Zipf 20M tensor the CPU oracle baseline times")
    ap.add_argument("--detail", action="store_true", help="print per-operation lines to stderr")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a plain 256 MiB device copy first (scales traffic counters)")
    ap.add_argument("--cp4-sweeps", type=int, default=10,
                    help="CP-ALS sweeps on the order-4 Zipf 50M tensor (0: skip that part)")
    ap.add_argument("--cp-sweeps", type=int, default=10,
                    help="CP-ALS sweeps on the planted 100M tensor (0: skip that part)")
    ap.add_argument("--cp-model-sample", type=int, default=1_000_000,
                    help="nonzeros at which the CPU leg compares the CP model with the oracle's")
    ap.add_argument("--ttmc-rank", type=int, default=16, help="SpTTMc rank per mode (0: skip)")
    ap.add_argument("--records", default="",
                    help="also write the per-operation records, one JSON line each, to this file")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path; "
              "--gpus must be 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_1705_09905_amd import Tensor, _lib

    def log(*a):
        print("[bench]", *a, file=sys.stderr, flush=True)

    if args.workload != "zipf20M":
        run_extra(args, log)
        return

    if args.calibrate_copy:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        device_copy(torch, src, dst)
        torch.cuda.synchronize()
        del src, dst
    Rs = [int(r) for r in args.ranks.split(",")]
    t0 = time.time()
    t = synth.config_tensor(WORKLOAD_CFG, nnz=args.nnz or None)
    log(f"generated {t.name} Z={t.nnz} in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    h = Tensor(t.idx, t.vals, t.dims)
    facs = {R: [torch.tensor(f.astype(np.float32), device=dev)
                for f in synth.factors(t.dims, R, WORKLOAD_CFG)] for R in Rs}
    t0 = time.time()
    build_ms = {}
    for m in range(t.order):
        for op in ("mttkrp", "ttm"):
            tile = (args.tile_ttm or args.tile) if op == "ttm" else args.tile
            tb = time.time()
            h.build(m, op, threadlen=args.threadlen, tile_nnz=tile or 4096)
            build_ms[(op, m)] = (time.time() - tb) * 1e3
    build_s = time.time() - t0
    log(f"F-COO built and uploaded (6 builds) in {build_s:.1f}s")
    tiles = {}
    if args.tile == 0:
        # tile size per (op, mode) chosen by timing at the largest rank (not timed below)
        t0 = time.time()
        for m in range(t.order):
            for op in ("mttkrp", "ttm"):
                r = h.autotune(m, op, facs[max(Rs)], tiles=[2048, 4096, 8192])
                tiles[f"{op}{m}"] = (r["tile_nnz"] if r["xcd_blocks"] <= 1
                                     else f"{r['tile_nnz']}/xcd{r['xcd_blocks']}-by-mode{r['xcd_mode']}")
        log(f"autotuned tile sizes {tiles} in {time.time() - t0:.1f}s")
    # the same builds sorted and encoded on the GPU (identical arrays): timed for the record
    torch.cuda.synchronize()
    t0 = time.time()
    for m in range(t.order):
        for op in ("mttkrp", "ttm"):
            inf = h.info(m, op)
            h.build(m, op, threadlen=args.threadlen, tile_nnz=inf["tile_nnz"], device=True,
                    xcd_blocks=inf["xcd_blocks"], xcd_mode=inf["block_mode"], lane_cols=inf["lane_cols"])
    torch.cuda.synchronize()
    dev_build_s = time.time() - t0
    log(f"F-COO built on the GPU (6 builds) in {dev_build_s:.2f}s")
    infos = {(op, m): h.info(m, op) for m in range(t.order) for op in ("mttkrp", "ttm")}
    # segments of the method: slices (non-empty rows) for SpMTTKRP, whatever
    # layout the autotuner kept (an XCD-blocked build splits them), fibres for SpTTM
    nsegs = {(op, m): (int(np.count_nonzero(np.bincount(t.idx[m], minlength=t.dims[m]))) if op == "mttkrp"
                       else infos[(op, m)]["nseg"]) for (op, m) in infos}
    outs = {}
    for R in Rs:
        for m in range(t.order):
            outs[("mttkrp", m, R)] = torch.empty((t.dims[m], R), dtype=torch.float32, device=dev)
            outs[("ttm", m, R)] = torch.empty((infos[("ttm", m)]["nseg"], R), dtype=torch.float32,
                                              device=dev)
    launches = [(op, m, R) for R in Rs for m in range(t.order) for op in ("mttkrp", "ttm")]

    def run(op, m, R):
        if op == "mttkrp":
            h.spmttkrp(m, facs[R], out=outs[(op, m, R)])
        else:
            h.spttm(m, facs[R][m], out=outs[(op, m, R)])

    ev = HipEvents()
    for _ in range(args.warmup):
        for L in launches:
            run(*L)
    torch.cuda.synchronize()

    pairs = []
    # every event is created before the timed region (creation is a host call)
    pool = [(ev.new(), ev.new()) for _ in range(args.steps * len(launches))]
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for si in range(args.steps):
        for li, L in enumerate(launches):
            a, b = pool[si * len(launches) + li]
            _lib.check(_lib.fcoo_set_tile_events(h.handle, a, b))
            run(*L)
            pairs.append((L, a, b))
    end.record()
    torch.cuda.synchronize()
    _lib.check(_lib.fcoo_set_tile_events(h.handle, None, None))
    total_ms = start.elapsed_time(end)
    ms_per_step = total_ms / args.steps

    N = t.order
    per = {}
    for L, a, b in pairs:
        per.setdefault(L, []).append(ev.ms(a, b))
    ev.close()
    step_bytes, step_flops = 0, 0
    classes = {}
    detail = []
    for (op, m, R) in launches:
        inf = infos[(op, m)]
        B = op_bytes(op, t.nnz, N, R, nsegs[(op, m)], t.dims[m], inf["npart"])
        F = op_flops(op, t.nnz, N, R)
        step_bytes += B
        step_flops += F
        d = float(np.mean(per[(op, m, R)]))
        c = classes.setdefault((op, R), {"bytes": 0, "ms": 0.0, "n": 0, "all": []})
        c["bytes"] += B
        c["ms"] += d
        c["n"] += 1
        c["all"] += per[(op, m, R)]
        detail.append({"op": op, "mode": m, "R": R, "tile_ms": round(d, 4),
                       "GBps": round(B / d / 1e6, 1), "nseg": inf["nseg"], "nfix": inf["nfix"]})
    for c in classes.values():
        c["stats"] = {"mean": float(np.mean(c["all"])), "median": float(np.median(c["all"])),
                      "min": float(np.min(c["all"])), "max": float(np.max(c["all"]))}
    if args.detail:
        for d in detail:
            log(json.dumps(d))
    dom = max(classes, key=lambda k: classes[k]["ms"])
    dc = classes[dom]
    avg_ms = dc["ms"] / dc["n"]
    alg_bytes = int(dc["bytes"] / dc["n"])
    khash = kernel_hash()
    tr = load_traffic(khash)
    # the roofline of the dominant kernel: HBM bytes it moved per launch (copy-
    # calibrated counters) over its average launch time, against 8 TB/s; the
    # byte model's rate counts every gathered row, cache hits included, so it
    # is reported beside it and not as an HBM fraction
    roofline = {"bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": None,
                "traffic": None,
                "kernel": f"seg_tile_kernel ({'SpMTTKRP' if dom[0] == 'mttkrp' else 'SpTTM'}, R={dom[1]}, "
                          f"float32, per-mode launch)",
                "symbol": kernel_symbol(dom[0], dom[1], t.order),
                "avg_launch_ms": round(avg_ms, 4),
                "launch_ms": {k: round(v, 4) for k, v in dc["stats"].items()},
                "algorithmic_bytes_per_launch": alg_bytes,
                "achieved_algorithmic_cache_inclusive": round(alg_bytes / avg_ms / 1e6, 1)}
    if tr is None:
        roofline["traffic_note"] = "no counters for this kernel source (hash mismatch or missing)"
    else:
        rec = tr.get("kernels", {}).get(roofline["symbol"])
        # the counters hold for the layout they were taken with (tile size, blocks)
        lay = tr.get("layout", {}).get(dom[0])
        same = lay is not None and all(
            infos[(dom[0], m)]["tile_nnz"] == lay["tile_nnz"] and
            (infos[(dom[0], m)]["xcd_blocks"] > 1) == (lay["xcd_blocks"] > 1) for m in range(t.order))
        if rec is None:
            roofline["traffic_note"] = "no counters for this kernel symbol"
        elif not same:
            roofline["traffic_note"] = f"counters were taken with layout {lay}, this run used another"
        else:
            roofline["traffic"] = rec["bytes_per_launch"]
            roofline["achieved"] = round(rec["bytes_per_launch"] / (avg_ms / 1e3) / 1e9, 1)
            roofline["frac"] = round(roofline["achieved"] / HBM_PEAK_GBPS, 4)
            roofline["traffic_unit"] = "bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
            if rec.get("limiter"):
                roofline["limiter"] = rec["limiter"]
    # the least bytes of the dominant kernel (each distinct factor row once),
    # and a plain device copy's rate on this GPU
    distinct = [int(np.count_nonzero(np.bincount(t.idx[k], minlength=t.dims[k]))) for k in range(t.order)]
    comp = [compulsory_bytes(op, t.nnz, N, R, nsegs[(op, m)], t.dims[m], infos[(op, m)]["npart"],
                             distinct, m) for (op, m, R) in launches if (op, R) == dom]
    roofline["compulsory_bytes_per_launch"] = int(np.mean(comp))
    roofline["compulsory_GBps"] = round(np.mean(comp) / (avg_ms / 1e3) / 1e9, 1)
    cbw = copy_bandwidth(torch)
    roofline["copy_GBps_measured"] = round(cbw, 1)
    roofline["compulsory_frac_of_copy"] = round(roofline["compulsory_GBps"] / cbw, 4)
    if roofline["achieved"] is not None:
        roofline["traffic_frac_of_copy"] = round(roofline["achieved"] / cbw, 4)
    value = step_bytes / (ms_per_step / 1e3) / 1e9
    mt = {R: classes[("mttkrp", R)] for R in Rs}
    tt = {R: classes[("ttm", R)] for R in Rs}
    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{t.name}: SpMTTKRP + SpTTM, every mode, R in {Rs}",
                   "dims": t.dims, "nnz": t.nnz, "ranks": Rs, "threadlen": args.threadlen,
                   "tile_nnz": tiles or ({"mttkrp": args.tile, "ttm": args.tile_ttm} if args.tile_ttm else args.tile)},
        "value_note": "algorithmic bytes (every gathered factor row counted, cache hits included) / step time",
        "gflops": round(step_flops / (ms_per_step / 1e3) / 1e9, 1),
        "pct_hbm_peak": None if roofline["frac"] is None else round(100 * roofline["frac"], 2),
        "pct_hbm_peak_basis": "measured HBM traffic of the dominant kernel / its launch time / 8 TB/s",
        "spmttkrp_GBps_algorithmic": {str(R): round(mt[R]["bytes"] / mt[R]["ms"] / 1e6, 1) for R in Rs},
        "spttm_GBps_algorithmic": {str(R): round(tt[R]["bytes"] / tt[R]["ms"] / 1e6, 1) for R in Rs},
        "spmttkrp_ms_per_mode": {str(R): round(mt[R]["ms"] / mt[R]["n"], 4) for R in Rs},
        "spttm_ms_per_mode": {str(R): round(tt[R]["ms"] / tt[R]["n"], 4) for R in Rs},
        "tile_ms_per_launch": {f"{op} R={R}": {k: round(v, 4) for k, v in c["stats"].items()}
                               for (op, R), c in classes.items()},
        "roofline": roofline,
        "build_s": round(build_s, 2),
        "device_build_s": round(dev_build_s, 3),
        "kernel_hash": khash,
    }
    # SpTTMc (Kronecker rows, Eq. 4) on the same SpMTTKRP builds: R per mode,
    # output dims[m] x R^(N-1); timed apart from the step (not in `value`)
    Rk = args.ttmc_rank
    if Rk > 0:
        Fk = [torch.tensor(f.astype(np.float32), device=dev) for f in synth.factors(t.dims, Rk, WORKLOAD_CFG)]
        W = Rk ** (N - 1)
        yk = {m: torch.empty((t.dims[m], W), dtype=torch.float32, device=dev) for m in range(N)}
        fk = {m: [None if k == m else Fk[k] for k in range(N)] for m in range(N)}
        for m in range(N):
            h.spttmc(m, fk[m], out=yk[m])
        ev = HipEvents()
        kp = []
        for _ in range(max(3, args.steps // 4)):
            for m in range(N):
                a, b = ev.new(), ev.new()
                _lib.check(_lib.fcoo_set_tile_events(h.handle, a, b))
                h.spttmc(m, fk[m], out=yk[m])
                kp.append((m, a, b))
        torch.cuda.synchronize()
        _lib.check(_lib.fcoo_set_tile_events(h.handle, None, None))
        km = {m: float(np.mean([ev.ms(a, b) for mm, a, b in kp if mm == m])) for m in range(N)}
        ev.close()
        kb = {}
        for m in range(N):
            inf = infos[("mttkrp", m)]
            flags = (t.nnz + 7) // 8
            kb[m] = (4 * t.nnz * N + flags + 4 * nsegs[("mttkrp", m)] + t.nnz * (N - 1) * Rk * 4
                     + 4 * t.dims[m] * W)
        out["spttmc"] = {"R_per_mode": Rk, "width": W,
                         "tile_ms_per_mode": [round(km[m], 4) for m in range(N)],
                         "GBps_per_mode": [round(kb[m] / km[m] / 1e6, 1) for m in range(N)],
                         "GFLOPs_per_mode": [round(t.nnz * W * N / km[m] / 1e6, 1) for m in range(N)]}
        log(f"spttmc R={Rk}: {out['spttmc']['tile_ms_per_mode']} ms")
    oracle_s, parity, sample_nnz, threads = {}, {}, None, None
    if not args.no_cpu:
        threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
        os.environ.setdefault("OMP_PROC_BIND", "close")
        t0 = time.time()
        out["cpu_baseline"] = cpu_baseline(t, Rs, args.cpu_sample, threads)
        oracle_s = out["cpu_baseline"].pop("_per_op_s")
        sample_nnz = out["cpu_baseline"].pop("_sample_nnz")
        log(f"cpu baseline in {time.time() - t0:.1f}s")
        t0 = time.time()
        parity = op_parity(t, Rs, outs, threads)
        log(f"full-size parity of the step's outputs in {time.time() - t0:.1f}s: "
            f"max rel err {max(parity.values()):.2e}")
    else:
        out["cpu_baseline"] = None
    # one record per measured operation (op, mode, R)
    records = []
    for (op, m, R) in launches:
        inf = infos[(op, m)]
        ts = per[(op, m, R)]
        B = op_bytes(op, t.nnz, N, R, nsegs[(op, m)], t.dims[m], inf["npart"])
        F = op_flops(op, t.nnz, N, R)
        med = float(np.median(ts))
        trec = None
        if tr is not None:
            lay = tr.get("layout", {}).get(op)
            if lay is not None and inf["tile_nnz"] == lay["tile_nnz"] and \
                    (inf["xcd_blocks"] > 1) == (lay["xcd_blocks"] > 1):
                trec = tr.get("kernels", {}).get(kernel_symbol(op, R, N))
        records.append({
            "config": t.name, "op": op, "mode": m, "R": R, "dtype": "f32", "Z": t.nnz,
            ("nseg" if op == "mttkrp" else "nfib"): int(nsegs[(op, m)]),
            "threadlen": args.threadlen, "tile_nnz": inf["tile_nnz"], "xcd_blocks": inf["xcd_blocks"],
            "lane_cols": inf["lane_cols"], "rank_tile": rank_tile(R),
            "t_gpu_ms": {"median": round(med, 4), "min": round(float(np.min(ts)), 4),
                         "max": round(float(np.max(ts)), 4), "n": len(ts)},
            "B_alg": int(B), "GBps_eff": round(B / med / 1e6, 1),
            "pct_hbm_spec_alg": round(100 * B / med / 1e6 / HBM_PEAK_GBPS, 1),
            "pct_hbm_copy_alg": round(100 * B / med / 1e6 / cbw, 1),
            "GFLOPs": round(F / med / 1e6, 1),
            "B_compulsory": int(compulsory_bytes(op, t.nnz, N, R, nsegs[(op, m)], t.dims[m], inf["npart"],
                                                 distinct, m)),
            "rocprof_fetch_bytes": None if trec is None else trec["fetch_bytes_per_launch"],
            "rocprof_write_bytes": None if trec is None else trec["write_bytes_per_launch"],
            "rocprof_note": None if trec is None else "per launch, mean over the modes of this kernel class",
            "t_build_ms": round(build_ms[(op, m)], 1),
            "t_oracle_ms": None if (op, m, R) not in oracle_s else round(1e3 * oracle_s[(op, m, R)], 1),
            "oracle_sample_nnz": sample_nnz, "oracle_threads": threads,
            "cpu_model": None if args.no_cpu else cpu_model(),
            "rel_fro_err_vs_oracle": None if (op, m, R) not in parity else float(f"{parity[(op, m, R)]:.3g}"),
        })
    out["records"] = records
    if args.records:
        with open(args.records, "w") as f:
            for r in records:
                f.write(json.dumps(r) + "\n")
    del h, facs, outs
    torch.cuda.synchronize()
    if args.cp_sweeps > 0:
        out["cp_als"] = cp_planted(args, log, out["cpu_baseline"])
    torch.cuda.synchronize()
    if args.cp4_sweeps > 0:
        out["cp_als_order4"] = cp_order4(args, log)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
