"""FP64 CPU oracle for the F-COO sparse tensor path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, calls or
links this module; only the tests, the smoke check and the CPU-baseline leg
of the benchmark do.  It shares no code with the HIP path.

Every function is the plain definition from the paper ("A Unified
Optimization Approach for Sparse Tensor Operations on GPUs", Liu, Wen,
Sarwate, Mehri Dehnavi), written slowly and in float64:

* matricization, Kronecker and Khatri-Rao products      -- Sec. II, Eq. (1)-(2)
* TTM / SpTTM                                           -- Sec. II, Eq. (3)
* TTMc / SpTTMc (Kronecker rows)                        -- Sec. II, Eq. (4), Table I
* MTTKRP / SpMTTKRP (dense and COO forms)               -- Sec. II, Eq. (5)-(6)
* mode roles (index / product modes)                    -- Sec. IV-A, Table I
* F-COO encoding (product indices, val, bf, sf)         -- Sec. IV-B, Fig. 2, Table II
* CP-ALS                                                -- Sec. II, Algorithm 1
* CP model at the nonzeros and the MSE gradient (gradient-based sparse CP;
  not in the paper, derived by the chain rule)

Where the paper is silent the reading taken is stated at the function.
Pins (tests that hold this oracle to something other than itself) live in
tests/test_oracle_*.py.  The F-COO encoding has no printed worked example to
pin against (the paper's figures are not available), so it is pinned by a
hand-derived fixture, closed-form sizes (Table II) and invariants.
"""
from __future__ import annotations

import itertools
from typing import Dict, List, Sequence, Tuple

import numpy as np

OP_MTTKRP = 0
OP_TTM = 1


# ----------------------------------------------------------------------------
# Sec. II: matricization, Kronecker (Eq. 1), Khatri-Rao (Eq. 2)
# ----------------------------------------------------------------------------

def dense_from_coo(dims: Sequence[int], idx: Sequence[np.ndarray], vals: np.ndarray) -> np.ndarray:
    """The tensor X = sum_e vals[e] * 1{coordinate e}.  Repeated coordinates
    add (COO semantics)."""
    X = np.zeros(tuple(int(d) for d in dims), dtype=np.float64)
    if len(vals):
        np.add.at(X, tuple(np.asarray(i, dtype=np.int64) for i in idx), np.asarray(vals, np.float64))
    return X


def unfold_column(coord: Sequence[int], dims: Sequence[int], n: int) -> int:
    """Column of X_(n) holding the entry at `coord`: the mode-n fibres become
    columns, the remaining modes ordered with the lowest mode varying fastest
    (0-based, so the column of (j, k) in X_(1) of an I x J x K tensor is
    j + J*k; this is the order that makes Eq. (5) read X_(1)(C kr B))."""
    col, stride = 0, 1
    for m, (c, d) in enumerate(zip(coord, dims)):
        if m == n:
            continue
        col += c * stride
        stride *= d
    return col


def unfold(X: np.ndarray, n: int) -> np.ndarray:
    """Mode-n matricization X_(n), written out entry by entry (tiny tensors)."""
    dims = X.shape
    ncols = 1
    for m, d in enumerate(dims):
        if m != n:
            ncols *= d
    Xn = np.zeros((dims[n], ncols), dtype=np.float64)
    for coord in itertools.product(*[range(d) for d in dims]):
        Xn[coord[n], unfold_column(coord, dims, n)] = X[coord]
    return Xn


def kron(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Eq. (1): block matrix whose (i, j) block is a_ij * B."""
    I, J = A.shape
    K, L = B.shape
    out = np.zeros((I * K, J * L), dtype=np.float64)
    for i in range(I):
        for j in range(J):
            out[i * K:(i + 1) * K, j * L:(j + 1) * L] = A[i, j] * B
    return out


def khatri_rao(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Eq. (2): column r of A (kr) B is a_r (kron) b_r; A is I x R, B is J x R."""
    I, R = A.shape
    J, R2 = B.shape
    assert R == R2
    out = np.zeros((I * J, R), dtype=np.float64)
    for r in range(R):
        out[:, r] = kron(A[:, r:r + 1], B[:, r:r + 1])[:, 0]
    return out


def krp_for_mode(factors: Sequence[np.ndarray], n: int) -> np.ndarray:
    """A_{N-1} kr ... kr A_{n+1} kr A_{n-1} kr ... kr A_0: the Khatri-Rao
    product that X_(n) multiplies in MTTKRP (for a 3-order tensor and n = 0
    this is C kr B, Eq. (5))."""
    mats = [factors[m] for m in range(len(factors) - 1, -1, -1) if m != n]
    out = mats[0]
    for M in mats[1:]:
        out = khatri_rao(out, M)
    return out


# ----------------------------------------------------------------------------
# Sec. II: MTTKRP, Eq. (5) (dense) and Eq. (6) (over the nonzeros)
# ----------------------------------------------------------------------------

def mttkrp_dense(X: np.ndarray, factors: Sequence[np.ndarray], n: int) -> np.ndarray:
    """Eq. (5): M = X_(n) (kr_{m != n} A_m), with the explicit unfolding and
    the explicit Khatri-Rao product (tiny tensors only)."""
    return unfold(X, n) @ krp_for_mode(factors, n)


def mttkrp_coo(dims, idx, vals, factors, n) -> np.ndarray:
    """Eq. (6), generalised to N modes: for every nonzero e,
    M[i_n(e), :] += vals[e] * (Hadamard product over m != n of A_m[i_m(e), :]).
    Rows with no nonzero stay zero."""
    R = factors[0].shape[1]
    M = np.zeros((int(dims[n]), R), dtype=np.float64)
    if len(vals) == 0:
        return M
    h = np.asarray(vals, np.float64)[:, None] * np.ones((1, R))
    for m in range(len(dims)):
        if m != n:
            h = h * np.asarray(factors[m], np.float64)[np.asarray(idx[m], np.int64)]
    np.add.at(M, np.asarray(idx[n], np.int64), h)
    return M


# ----------------------------------------------------------------------------
# Sec. II: TTM, Eq. (3); the output is semi-sparse (one dense row per fibre)
# ----------------------------------------------------------------------------

def ttm_dense(X: np.ndarray, U: np.ndarray, n: int) -> np.ndarray:
    """Eq. (3) with U of shape I_n x R: Y(..., :) = sum_k X(..., k, ...) U(k, :).
    Result axes: the other modes in ascending order, then R."""
    return np.tensordot(X, U, axes=([n], [0]))


def _lex_order(cols: List[np.ndarray]) -> np.ndarray:
    """Stable ascending lexicographic order of the tuples (cols[0], cols[1], ...)."""
    if not cols:
        raise ValueError("need at least one key")
    return np.lexsort(tuple(np.asarray(c, np.int64) for c in reversed(cols)))


def ttm_coo(dims, idx, vals, U, n) -> Tuple[np.ndarray, np.ndarray]:
    """SpTTM on mode n over the nonzeros: the fibres are the distinct tuples of
    the index modes (all modes but n), kept in lexicographic order, structural
    (a fibre whose sum cancels to zero is still listed).  Returns
    (fibres[nfib, N-1] int64, Y[nfib, R])."""
    N = len(dims)
    imodes = [m for m in range(N) if m != n]
    R = U.shape[1]
    Z = len(vals)
    if Z == 0:
        return np.zeros((0, N - 1), dtype=np.int64), np.zeros((0, R))
    tup = np.stack([np.asarray(idx[m], np.int64) for m in imodes], axis=1)
    fibres, g = np.unique(tup, axis=0, return_inverse=True)
    g = np.asarray(g).reshape(-1)
    Y = np.zeros((fibres.shape[0], R), dtype=np.float64)
    np.add.at(Y, g, np.asarray(vals, np.float64)[:, None] * np.asarray(U, np.float64)[np.asarray(idx[n], np.int64)])
    return fibres, Y


def ttm_dense_rows(X: np.ndarray, U: np.ndarray, n: int, fibres: np.ndarray) -> np.ndarray:
    """Rows of the dense TTM result read at the listed fibres."""
    Yd = ttm_dense(X, U, n)
    return np.stack([Yd[tuple(f)] for f in fibres]) if len(fibres) else np.zeros((0, U.shape[1]))


# ----------------------------------------------------------------------------
# Sec. II, Eq. (4) and Table I (third row): SpTTMc, the tensor times a chain
# of matrices on every mode but one (the kernel of Tucker / HOOI)
# ----------------------------------------------------------------------------

def ttmc_width(factors: Sequence[np.ndarray], n: int) -> int:
    """Columns of Y_(n): the product of the ranks of the modes other than n."""
    w = 1
    for m, U in enumerate(factors):
        if m != n:
            w *= int(np.asarray(U).shape[1])
    return w


def ttmc_coo(dims, idx, vals, factors, n, chunk: int = 1 << 16) -> np.ndarray:
    """Eq. (4) generalised to N modes: for every nonzero e,
    Y_(n)[i_n(e), :] += vals[e] * (U_{m_1}[i_{m_1}(e), :] kron U_{m_2}[i_{m_2}(e), :] kron ...)
    with m_1 < m_2 < ... the modes other than n (the product modes of Table I)
    and kron the Kronecker product of Eq. (1) applied to 1 x R_m rows, so the
    column of (p_1, p_2, ...) is (..(p_1 R_{m_2} + p_2) R_{m_3} + ..): the last
    product mode's column runs fastest.  factors[m] is I_m x R_m; factors[n]
    is not read.  Rows with no nonzero stay zero.  Returns I_n x prod R_m."""
    N = len(dims)
    pm = [m for m in range(N) if m != n]
    W = ttmc_width(factors, n)
    Y = np.zeros((int(dims[n]), W), dtype=np.float64)
    vals = np.asarray(vals, np.float64)
    for s0 in range(0, len(vals), chunk):
        s1 = min(len(vals), s0 + chunk)
        h = vals[s0:s1, None]
        for m in pm:
            rows = np.asarray(factors[m], np.float64)[np.asarray(idx[m][s0:s1], np.int64)]
            # row-wise Eq. (1): block p of (h kron u) is h_p * u
            h = (h[:, :, None] * rows[:, None, :]).reshape(s1 - s0, -1)
        np.add.at(Y, np.asarray(idx[n][s0:s1], np.int64), h)
    return Y


def ttmc_dense(X: np.ndarray, factors: Sequence[np.ndarray], n: int) -> np.ndarray:
    """TTMc as a chain of dense TTMs (Eq. 3): contract every mode m != n of X
    with U_m (one mode at a time), then lay the result out as Y_(n) with the
    column order of Eq. (4) (later product modes fastest)."""
    N = X.ndim
    Y = np.asarray(X, np.float64)
    # contract from the highest mode down so the remaining axis numbers stay put
    for m in reversed(range(N)):
        if m != n:
            Y = np.moveaxis(np.tensordot(Y, np.asarray(factors[m], np.float64), axes=([m], [0])), -1, m)
    Y = np.moveaxis(Y, n, 0)
    return Y.reshape(Y.shape[0], -1)


# ----------------------------------------------------------------------------
# Sec. IV-A, Table I: index modes and product modes
# ----------------------------------------------------------------------------

def mode_roles(order: int, mode: int, op: int) -> Tuple[List[int], List[int]]:
    """(index modes, product modes), each ascending.
    SpMTTKRP on mode n: index = (n), product = every other mode.
    SpTTM on mode n:    index = every other mode, product = (n)."""
    others = [m for m in range(order) if m != mode]
    if op == OP_MTTKRP:
        return [mode], others
    if op == OP_TTM:
        return others, [mode]
    raise ValueError(op)


# ----------------------------------------------------------------------------
# Sec. IV-B: F-COO encoding
# ----------------------------------------------------------------------------

def fcoo_encode(dims, idx, vals, mode: int, op: int, threadlen: int, tile_nnz: int) -> Dict[str, np.ndarray]:
    """Reference F-COO encoder for one (operation, mode).

    Readings taken where the paper is silent (each also listed in the design
    notes):
      * nonzeros are ordered by the index-mode tuple, then the product-mode
        tuple, ascending; ties (repeated coordinates) keep input order;
      * only product-mode indices and values are stored per nonzero;
      * bf is a parity bit that starts at 1 and toggles at every new
        segment (slice for SpMTTKRP, fibre for SpTTM): bf[0] = 1 and the
        segment heads are exactly the positions where bf changes.  Packed as
        one LSB-first bit stream (byte s>>3, bit s&7), ceil(Z/8) bytes;
      * the nonzeros are cut into partitions of `threadlen`; sf[p] = 1 iff a
        segment starts anywhere inside partition p (so sf[0] = 1), packed
        LSB-first into uint32 words, ceil(P/32) words;
      * because the index modes are not stored, each segment's index-mode
        coordinates are kept once per segment: `seg_row` (SpMTTKRP: the
        output row) or `fibres` (SpTTM: the output fibre coordinates);
      * tile_seg0[t] = ordinal of the segment holding nonzero t*tile_nnz
        (0-based), for t < ceil(Z / tile_nnz);
      * perm[s] = input position of the nonzero stored at position s.
    """
    N = len(dims)
    if threadlen not in (8, 16, 32, 64):
        raise ValueError("threadlen must be 8, 16, 32 or 64")
    if tile_nnz <= 0 or tile_nnz % threadlen:
        raise ValueError("tile_nnz must be a positive multiple of threadlen")
    imodes, pmodes = mode_roles(N, mode, op)
    Z = len(vals)
    cols = [np.asarray(idx[m], np.int64) for m in range(N)]
    perm = _lex_order([cols[m] for m in imodes] + [cols[m] for m in pmodes]) if Z else np.zeros(0, np.int64)

    out: Dict[str, np.ndarray] = {}
    out["pidx"] = [cols[m][perm].astype(np.int32) for m in pmodes]
    out["val"] = np.asarray(vals, np.float64)[perm].astype(np.float32)

    head = np.zeros(Z, dtype=bool)
    if Z:
        head[0] = True
        for m in imodes:
            c = cols[m][perm]
            head[1:] |= c[1:] != c[:-1]
    bf = (np.cumsum(head) % 2).astype(np.uint8)
    out["bf"] = np.packbits(bf, bitorder="little") if Z else np.zeros(0, np.uint8)

    P = -(-Z // threadlen)
    padded = np.zeros(P * threadlen, dtype=bool)
    padded[:Z] = head
    sfbits = padded.reshape(P, threadlen).any(axis=1).astype(np.uint8)
    nwords = -(-P // 32)
    sfbytes = np.packbits(sfbits, bitorder="little") if P else np.zeros(0, np.uint8)
    sfbytes = np.concatenate([sfbytes, np.zeros(4 * nwords - sfbytes.shape[0], np.uint8)])
    out["sf"] = sfbytes.view("<u4").astype(np.uint32)

    heads = np.nonzero(head)[0]
    if op == OP_MTTKRP:
        out["seg_row"] = cols[mode][perm][heads].astype(np.int32)
    else:
        out["fibres"] = (np.stack([cols[m][perm][heads] for m in imodes], axis=1).astype(np.int32)
                         if Z else np.zeros((0, N - 1), np.int32))
    ntiles = -(-Z // tile_nnz)
    csum = np.cumsum(head)
    out["tile_seg0"] = (csum[np.arange(ntiles, dtype=np.int64) * tile_nnz] - 1).astype(np.int32)
    out["perm"] = perm.astype(np.int32)
    out["nseg"] = int(head.sum())
    out["head"] = head
    out["index_modes"] = imodes
    out["product_modes"] = pmodes
    return out


def fcoo_decode(enc: Dict[str, np.ndarray], dims, mode: int, op: int):
    """Rebuild the sorted coordinate list from an encoding: heads are where
    the bf bit changes (with bit -1 taken as 0), the segment ordinal of a
    nonzero is the number of heads up to it minus one, and the index-mode
    coordinates come from that segment's seg_row / fibres entry."""
    N = len(dims)
    imodes, pmodes = mode_roles(N, mode, op)
    Z = enc["val"].shape[0]
    bits = np.unpackbits(enc["bf"], bitorder="little")[:Z].astype(np.int64)
    prev = np.concatenate([[0], bits[:-1]]) if Z else bits
    head = (bits ^ prev).astype(bool)
    seg = np.cumsum(head) - 1
    cols = [None] * N
    for q, m in enumerate(pmodes):
        cols[m] = enc["pidx"][q].astype(np.int64)
    if op == OP_MTTKRP:
        cols[mode] = enc["seg_row"].astype(np.int64)[seg]
    else:
        for t, m in enumerate(imodes):
            cols[m] = enc["fibres"][:, t].astype(np.int64)[seg]
    return cols, enc["val"].astype(np.float64)


def table2_bytes(nnz: int, op: int, threadlen: int) -> float:
    """Table II: F-COO bytes of a 3-order tensor, int32 indices and float32
    values: SpTTM (8 + 1/8 + 1/(8 threadlen)) nnz, SpMTTKRP
    (12 + 1/8 + 1/(8 threadlen)) nnz; COO is 16 nnz."""
    base = 12.0 if op == OP_MTTKRP else 8.0
    return (base + 1.0 / 8.0 + 1.0 / (8.0 * threadlen)) * nnz


def fcoo_stream_bytes(enc: Dict[str, np.ndarray]) -> int:
    """Bytes actually held by the per-nonzero arrays of an encoding."""
    return (sum(a.nbytes for a in enc["pidx"]) + enc["val"].nbytes + enc["bf"].nbytes
            + enc["sf"].nbytes)


# ----------------------------------------------------------------------------
# Algorithm 1: CP-ALS, generalised to N modes, float64
# ----------------------------------------------------------------------------

def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float64 -> float32 (IEEE round-to-nearest-even) -> bfloat16
    (round-to-nearest-even on the upper 16 bits), returned as float64.
    NaN/Inf are not expected here."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def cholesky(V: np.ndarray, rel_pivot: float = 1e-13):
    """Plain Cholesky V = L L^T.  Returns None when a pivot is <= 0 or below
    rel_pivot * max(diag(V)) (the matrix is then treated as singular)."""
    R = V.shape[0]
    L = np.zeros_like(V, dtype=np.float64)
    dmax = max(float(np.max(np.diag(V))), 0.0) if R else 0.0
    for j in range(R):
        s = V[j, j] - np.dot(L[j, :j], L[j, :j])
        if not (s > 0.0) or s <= rel_pivot * dmax:
            return None
        L[j, j] = np.sqrt(s)
        for i in range(j + 1, R):
            L[i, j] = (V[i, j] - np.dot(L[i, :j], L[j, :j])) / L[j, j]
    return L


def solve_rows(V: np.ndarray, M: np.ndarray):
    """Solve A V = M for A (V symmetric R x R, M I x R).  Cholesky with
    forward / backward substitution; if Cholesky fails, A = M V^+ with the
    pseudo-inverse from a symmetric eigendecomposition, eigenvalues at or
    below R * eps64 * max eigenvalue treated as zero.
    Returns (A, used_pinv)."""
    R = V.shape[0]
    L = cholesky(V)
    if L is not None:
        # V A^T = M^T  ->  L Y = M^T, L^T A^T = Y
        Y = np.zeros((R, M.shape[0]))
        for j in range(R):
            Y[j] = (M[:, j] - L[j, :j] @ Y[:j]) / L[j, j]
        At = np.zeros_like(Y)
        for j in range(R - 1, -1, -1):
            At[j] = (Y[j] - L[j + 1:, j] @ At[j + 1:]) / L[j, j]
        return At.T.copy(), False
    d, Q = np.linalg.eigh(V)
    cut = R * np.finfo(np.float64).eps * (float(np.max(d)) if R else 0.0)
    dinv = np.where(d > cut, 1.0 / np.where(d > cut, d, 1.0), 0.0)
    Vp = (Q * dinv) @ Q.T
    return M @ Vp, True


def normalize_columns(A: np.ndarray):
    """lambda_r = ||A(:, r)||_2; columns with a positive norm are divided by
    it, a zero column stays zero with lambda_r = 0."""
    lam = np.sqrt(np.sum(A * A, axis=0))
    out = A.copy()
    nz = lam > 0
    out[:, nz] = A[:, nz] / lam[nz]
    return out, lam


def cp_fit(normX2: float, lam: np.ndarray, grams: Sequence[np.ndarray], M_last: np.ndarray,
           A_last: np.ndarray) -> float:
    """fit = 1 - ||X - Xhat|| / ||X|| with
    ||Xhat||^2 = lam^T (Hadamard of all Grams) lam,
    <X, Xhat> = sum_r lam_r sum_i M_{N-1}(i, r) A_{N-1}(i, r),
    the residual square clamped at zero."""
    H = np.ones_like(grams[0])
    for G in grams:
        H = H * G
    xhat2 = float(lam @ H @ lam)
    inner = float(np.sum(lam * np.sum(M_last * A_last, axis=0)))
    res2 = max(0.0, normX2 + xhat2 - 2.0 * inner)
    return 1.0 - np.sqrt(res2) / np.sqrt(normX2)


def cp_als(dims, idx, vals, R: int, init: Sequence[np.ndarray], sweeps: int,
           storage: str = "f64", tol: float = 0.0, mttkrp=None, record=None):
    """Algorithm 1 for N modes (Gauss-Seidel order, newest factors used).

    For each sweep and each mode n:
      M <- SpMTTKRP_n (Eq. 6);  V <- Hadamard of the Grams G_m, m != n;
      A_n <- M V^+ (Cholesky, pseudo-inverse fallback);
      normalise the columns of A_n, lambda <- the norms;
      storage 'f32' / 'bf16' rounds the stored A_n (round to nearest even);
      G_n <- A_n^T A_n from the stored values.
    After the last mode the fit is computed (cp_fit).  Stops after `sweeps`
    sweeps, or earlier when tol > 0 and |delta fit| < tol.
    A_0's initial value is never read (line 2 overwrites it first).
    `mttkrp(dims, idx, vals, factors, n)` may replace mttkrp_coo by another
    implementation of the same definition (the C loop, for large tensors).
    `record`, a list or None, receives a copy (factors, lam) after every
    sweep (observation only).
    Returns dict(factors, lam, fits, used_pinv[sweep][mode], grams)."""
    mttkrp = mttkrp_coo if mttkrp is None else mttkrp
    N = len(dims)
    vals = np.asarray(vals, np.float64)
    normX2 = float(np.sum(vals * vals))

    def store(A):
        if storage == "f64":
            return A
        if storage == "f32":
            return A.astype(np.float32).astype(np.float64)
        if storage == "bf16":
            return bf16_round(A)
        raise ValueError(storage)

    A = [store(np.asarray(a, np.float64).copy()) for a in init]
    G = [a.T @ a for a in A]
    fits, pinv_log = [], []
    lam = np.ones(R)
    M = None
    for s in range(sweeps):
        used = []
        for n in range(N):
            M = mttkrp(dims, idx, vals, A, n)
            V = np.ones((R, R))
            for m in range(N):
                if m != n:
                    V = V * G[m]
            An, p = solve_rows(V, M)
            An, lam = normalize_columns(An)
            A[n] = store(An)
            G[n] = A[n].T @ A[n]
            used.append(p)
        fits.append(cp_fit(normX2, lam, G, M, A[N - 1]))
        pinv_log.append(used)
        if record is not None:
            record.append(([a.copy() for a in A], lam.copy()))
        if tol > 0 and s > 0 and abs(fits[-1] - fits[-2]) < tol:
            break
    return dict(factors=A, lam=lam, fits=fits, used_pinv=pinv_log, grams=G)


def cp_full(factors: Sequence[np.ndarray], lam=None) -> np.ndarray:
    """Dense CP model sum_r lam_r a_r^(0) o ... o a_r^(N-1) (tiny only)."""
    R = factors[0].shape[1]
    lam = np.ones(R) if lam is None else lam
    X = None
    for r in range(R):
        t = np.array(lam[r], dtype=np.float64)
        for A in factors:
            t = np.multiply.outer(t, A[:, r])
        X = t if X is None else X + t
    return X


# ----------------------------------------------------------------------------
# Gradient-based sparse CP (not in the paper): model at the nonzeros, MSE
# ----------------------------------------------------------------------------

def cp_model_at(idx, factors) -> np.ndarray:
    """xhat_e = sum_r prod_m A_m[i_m(e), r]."""
    R = factors[0].shape[1]
    p = np.ones((np.asarray(idx[0]).shape[0], R))
    for m, A in enumerate(factors):
        p = p * np.asarray(A, np.float64)[np.asarray(idx[m], np.int64)]
    return p.sum(axis=1)


def mse_loss(idx, vals, factors) -> float:
    """L = (1 / 2Z) sum_e (xhat_e - x_e)^2."""
    Z = len(vals)
    r = cp_model_at(idx, factors) - np.asarray(vals, np.float64)
    return float(0.5 * np.dot(r, r) / Z)


def model_adjoint(dims, idx, g, factors) -> List[np.ndarray]:
    """Gradient of sum_e g_e * xhat_e w.r.t. each factor, by the chain rule:
    d xhat_e / d A_m[i_m(e), r] = prod_{k != m} A_k[i_k(e), r], so
    grad_m[i, r] = sum_{e : i_m(e) = i} g_e prod_{k != m} A_k[i_k(e), r]."""
    N = len(dims)
    R = factors[0].shape[1]
    g = np.asarray(g, np.float64)
    out = []
    for m in range(N):
        Gm = np.zeros((int(dims[m]), R))
        if len(g):
            h = g[:, None] * np.ones((1, R))
            for k in range(N):
                if k != m:
                    h = h * np.asarray(factors[k], np.float64)[np.asarray(idx[k], np.int64)]
            np.add.at(Gm, np.asarray(idx[m], np.int64), h)
        out.append(Gm)
    return out


def mse_grad(dims, idx, vals, factors) -> List[np.ndarray]:
    """dL/dA_m with L the MSE above: the adjoint with g_e = (xhat_e - x_e) / Z."""
    Z = len(vals)
    g = (cp_model_at(idx, factors) - np.asarray(vals, np.float64)) / Z
    return model_adjoint(dims, idx, g, factors)


def observed_fit(idx, vals, factors, model=None) -> float:
    """fit over the observed entries: 1 - ||xhat - x|| / ||x||.
    `model(idx, factors)` may replace cp_model_at by another implementation
    of the same definition (the C loop, for large tensors)."""
    x = np.asarray(vals, np.float64)
    r = (cp_model_at if model is None else model)(idx, factors) - x
    return 1.0 - float(np.linalg.norm(r) / np.linalg.norm(x))


def adam_step(params, grads, m, v, t: int, lr=1e-2, b1=0.9, b2=0.999, eps=1e-8):
    """Kingma & Ba's Adam with bias correction (in place on lists of arrays):
    m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2;
    p <- p - lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)."""
    for k in range(len(params)):
        m[k] = b1 * m[k] + (1 - b1) * grads[k]
        v[k] = b2 * v[k] + (1 - b2) * grads[k] * grads[k]
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
    return params, m, v
