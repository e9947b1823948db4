"""CPU oracle for IDR(s)stab(l) / M(s)stab(l) (FP64).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package; the HIP library and its binding
never do.  The arithmetic lives in ``oracle.c`` (plain sequential C, compiled
without FMA contraction) and, for the learned initial guess, in ``cnn.py``
(NumPy FP64).  Nothing here shares code with the GPU path.

Functions follow the paper (Neuenhofen, arXiv 1604.06043):

* :func:`solve` -- Algorithm 1 (IDR(s)stab(l)) with the recycling protocol of
  Section 4.2 (M(s)stab(l): pass P, U, V of a former solve as inputs) and the
  fetching of U, V at a cycle end (Section 5, preliminaries);
* :func:`bicgstab` -- textbook BiCGStab, which the IDR cycle of Section 2.3
  reproduces for s = l = 1;
* :func:`assemble_convdiff`, :func:`spmv` -- the upwind finite-difference
  matrices of the synthetic workloads and the plain CSR product;
* :func:`cholqr`, :func:`recycle_start` -- orthonormalization of fetched
  U, V (an option of this build) and the projection of a new right-hand side
  onto recycled data (Section 4.2);
* :func:`jacobi_split`, :func:`solve_jacobi` -- the split preconditioned
  system of Section 5.1, L^{-1} A R^{-1} y = L^{-1} b with x = R^{-1} y, for
  the diagonal splitting L = R = |D|^{1/2};
* :func:`multicolour`, :func:`ilu0`, :func:`solve_ilu` -- the same split form
  with the ILU(0) factors that Section 5.1 uses, computed in a greedy
  multicolour order of the matrix.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, NOT_CONVERGED, E_INVALID, E_NOMEM, E_BREAKDOWN, E_NONFINITE = 0, 1, -1, -3, -4, -5
MSTAB, IDRSTAB = 0, 1
FETCH_THRESHOLD, FETCH_AT_LEVEL, FETCH_AT_END, FETCH_ONCE, FETCH_NEVER, FETCH_ESTIMATE = 0, 1, 2, 3, 4, 5


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (plain gcc, no FMA contraction)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp"
        subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                        "-std=c11", "-Wall", "-o", tmp, src, "-lm"], check=True)
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        _lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int, ctypes.c_double
        _lib.orc_convdiff_nnz.restype = i64
        _lib.orc_convdiff_nnz.argtypes = [i32, i64]
        _lib.orc_assemble_convdiff.restype = None
        _lib.orc_assemble_convdiff.argtypes = [i32, i64, P, f64, P, P, P, P]
        _lib.orc_spmv.restype = None
        _lib.orc_spmv.argtypes = [i64, P, P, P, P, P]
        _lib.orc_solve.restype = i32
        _lib.orc_solve.argtypes = [i64, P, P, P, i32, i32, P, f64, i64, i32, i32, f64, i64, i32,
                                   i32, i32, P, P, P, P, P, P, P, P, P, P, i64, P, i64, P, P, P]
        _lib.orc_ilu0.restype = i32
        _lib.orc_ilu0.argtypes = [i64, P, P, P, P]
        for fn in ("orc_ilu_lower", "orc_ilu_upper", "orc_ilu_upper_mul"):
            getattr(_lib, fn).restype = None
            getattr(_lib, fn).argtypes = [i64, P, P, P, P, P]
        _lib.orc_multicolour.restype = i32
        _lib.orc_multicolour.argtypes = [i64, P, P, P, P]
        _lib.orc_estimate_fetch_cycle.restype = i64
        _lib.orc_estimate_fetch_cycle.argtypes = [P, i64]
        _lib.orc_cholqr.restype = i32
        _lib.orc_cholqr.argtypes = [i64, i32, P, P]
        _lib.orc_recycle_start.restype = i32
        _lib.orc_recycle_start.argtypes = [i64, i32, P, P, P, P, P]
        _lib.orc_set_sum_order.restype = None
        _lib.orc_set_sum_order.argtypes = [i32]
        _lib.orc_bicgstab.restype = i32
        _lib.orc_bicgstab.argtypes = [i64, P, P, P, P, P, P, i32]
        _lib.orc_gmres.restype = i32
        _lib.orc_gmres.argtypes = [i64, P, P, P, i32, f64, i64, P, P, P, P, P, P, i64, P, P]
    return _lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class CSR:
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @property
    def n(self) -> int:
        return self.row_ptr.shape[0] - 1

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def dense(self) -> np.ndarray:
        D = np.zeros((self.n, self.n))
        for i in range(self.n):
            for k in range(self.row_ptr[i], self.row_ptr[i + 1]):
                D[i, self.col[k]] += self.val[k]
        return D

    def scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))


def assemble_convdiff(dim: int, n: int, beta, inv_dt: float, kappa=None) -> CSR:
    lib = _load()
    N = n ** dim
    nnz = int(lib.orc_convdiff_nnz(dim, n))
    rp = np.zeros(N + 1, dtype=np.int32)
    ci = np.zeros(nnz, dtype=np.int32)
    va = np.zeros(nnz, dtype=np.float64)
    b3 = np.zeros(3)
    b3[:dim] = np.asarray(beta, dtype=np.float64)[:dim]
    kap = None if kappa is None else np.ascontiguousarray(kappa, dtype=np.float64)
    lib.orc_assemble_convdiff(dim, n, _ptr(b3), float(inv_dt), _ptr(kap), _ptr(rp), _ptr(ci), _ptr(va))
    return CSR(rp, ci, va)


def spmv(A: CSR, x: np.ndarray) -> np.ndarray:
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(A.n)
    lib.orc_spmv(A.n, _ptr(A.row_ptr), _ptr(A.col), _ptr(A.val), _ptr(x), _ptr(y))
    return y


@dataclass
class Recycle:
    """Recycled data of M(s)stab: U, V (n x s, column-major) and their level;
    est: the fetch cycle that FETCH_ESTIMATE took from the last solve (-1: none)."""
    U: np.ndarray
    V: np.ndarray
    level: int = 0
    have: bool = False
    est: int = -1

    @staticmethod
    def empty(n: int, s: int) -> "Recycle":
        return Recycle(np.zeros((n, s), order="F"), np.zeros((n, s), order="F"), 0, False)

    def copy(self) -> "Recycle":
        return Recycle(self.U.copy(order="F"), self.V.copy(order="F"), self.level, self.have, self.est)


@dataclass
class Info:
    status: int
    mv: int
    mv_check: int
    cycles: int
    level: int
    fetched: int
    converged: bool
    recycled: bool
    restarts: int
    replacements: int
    relres_rec: float
    relres_true: float
    hist_mv: np.ndarray = field(repr=False)
    hist_res: np.ndarray = field(repr=False)

    @property
    def mv_total(self) -> int:
        return self.mv + self.mv_check


def solve(A: CSR, b, x0, s: int, ell: int, P: np.ndarray, tol: float = 1e-8,
          max_mv: int = 10 ** 9, method: int = MSTAB, fetch: int = FETCH_THRESHOLD,
          fetch_rel: float | None = None, fetch_level: int = -1, max_repl: int = 3,
          recycle: Recycle | None = None, dump_cycle: int = -1, replace_every: int = 0,
          orthonormalize: bool = False, ilu: np.ndarray | None = None):
    """Run Algorithm 1 on A x = b from x0.  Returns (x, info, recycle, dump).

    ``replace_every`` = k > 0 replaces the recursive residual by b - A x after
    every k-th cycle (Section 5.1's ocean run: k = 1).  ``orthonormalize``
    applies :func:`cholqr` to the U, V a solve fetches.

    ``ilu`` (the ILU(0) factors of A in its pattern, :func:`ilu0`) makes the
    operator L^{-1} A U^{-1}: the split preconditioned system of Section 5.1,
    whose right-hand side and start the caller prepares (:func:`solve_ilu`).

    ``recycle`` is updated in place (fetched data) and also returned.
    ``dump`` (if dump_cycle >= 0) is a dict with the state after the level
    loop of that cycle and after its update.
    """
    lib = _load()
    n = A.n
    P = np.asfortranarray(P, dtype=np.float64)
    if P.shape != (n, s):
        raise ValueError("P must be n x s")
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.array(x0, dtype=np.float64, copy=True)
    if recycle is None:
        recycle = Recycle.empty(n, s)
    if fetch_rel is None:
        fetch_rel = float(np.sqrt(tol))
    lvl = np.array([recycle.level], dtype=np.int64)
    have = np.array([1 if recycle.have else 0], dtype=np.int32)
    oi = np.zeros(9, dtype=np.int64)
    of = np.zeros(2)
    cap = 100000
    hmv = np.zeros(cap, dtype=np.int64)
    hres = np.zeros(cap)
    hl = np.zeros(1, dtype=np.int64)
    est = np.array([recycle.est], dtype=np.int64)
    dump = None
    if dump_cycle >= 0:
        dump = np.zeros(n * (2 + ell + s * (ell + 2)) + ell + n * (2 + 2 * s))
    st = lib.orc_solve(n, _ptr(A.row_ptr), _ptr(A.col), _ptr(A.val), s, ell, _ptr(P),
                       float(tol), int(max_mv), int(method), int(fetch), float(fetch_rel),
                       int(fetch_level), int(max_repl), int(replace_every), int(bool(orthonormalize)),
                       _ptr(b), _ptr(x),
                       _ptr(recycle.U), _ptr(recycle.V), _ptr(lvl), _ptr(have),
                       _ptr(oi), _ptr(of), _ptr(hmv), _ptr(hres), cap, _ptr(hl),
                       int(dump_cycle), _ptr(dump), _ptr(est),
                       None if ilu is None else _ptr(np.ascontiguousarray(ilu, dtype=np.float64)))
    recycle.level = int(lvl[0])
    recycle.est = int(est[0])
    recycle.have = bool(have[0])
    h = int(min(hl[0], cap))
    info = Info(int(st), int(oi[0]), int(oi[1]), int(oi[2]), int(oi[3]), int(oi[4]), bool(oi[5]),
                bool(oi[6]), int(oi[7]), int(oi[8]), float(of[0]), float(of[1]),
                hmv[:h].copy(), hres[:h].copy())
    dd = None
    if dump is not None:
        o = 0
        def take(k):
            nonlocal o
            v = dump[o:o + k]
            o += k
            return v
        x_l = take(n).copy()
        R = take(n * (ell + 1)).reshape(ell + 1, n).copy()
        W = take(n * s * (ell + 2)).reshape(ell + 2, s, n).copy()
        tau = take(ell).copy()
        x_u = take(n).copy()
        r_u = take(n).copy()
        U_u = take(n * s).reshape(s, n).copy()
        V_u = take(n * s).reshape(s, n).copy()
        dd = dict(x=x_l, R=R, W=W, tau=tau, x_after=x_u, r_after=r_u, U_after=U_u, V_after=V_u)
    return x, info, recycle, dd


SUM_FORWARD, SUM_REVERSE, SUM_BLOCKED = 0, 1, 2


class sum_order:
    """Context: every inner product of the oracle uses another summation order.

    ``SUM_REVERSE`` sums from the last index down; ``SUM_BLOCKED`` sums blocks
    of 256 consecutive terms and adds the block sums pairwise.  Same
    definition, other rounding; comparing runs measures the rounding
    sensitivity of the iteration itself.  The order is a property of the
    calling thread (solves in other threads keep theirs)."""

    def __init__(self, order: int):
        self.order = order

    def __enter__(self):
        _load().orc_set_sum_order(self.order)
        return self

    def __exit__(self, *exc):
        _load().orc_set_sum_order(SUM_FORWARD)
        return False


def estimate_fetch_cycle(hist_res) -> int:
    """The fetch point "shortly before the residual drops" (Section 5, how to
    choose the fetching point) from a solve's history of recursive relative
    residuals (initial, then one per cycle): the cycle before the largest
    one-cycle reduction (at least cycle 1); -1 for no cycle."""
    h = np.ascontiguousarray(hist_res, dtype=np.float64)
    return int(_load().orc_estimate_fetch_cycle(_ptr(h), h.shape[0]))


def cholqr(U: np.ndarray, V: np.ndarray | None = None) -> bool:
    """Orthonormalize recycled data in place (n x s, column-major): CholQR in
    FP64, U := U R^{-1}, V := V R^{-1} with U^T U = R^T R.  Returns False,
    leaving both untouched, when U^T U is not numerically positive definite."""
    for M in (U, V):
        if M is not None and not (M.flags.f_contiguous and M.dtype == np.float64):
            raise ValueError("U, V must be Fortran-ordered float64")
    n, s = U.shape
    st = _load().orc_cholqr(n, s, _ptr(U), _ptr(V))
    if st < 0:
        raise ValueError("cholqr: bad arguments")
    return st == 0


def recycle_start(P: np.ndarray, U: np.ndarray, V: np.ndarray, r: np.ndarray, x: np.ndarray):
    """The projection of a right-hand side onto recycled data (Section 4.2):
    gamma with r - V gamma orthogonal to P; returns (r - V gamma, x + U gamma)."""
    n, s = U.shape
    P = np.asfortranarray(P, dtype=np.float64)
    U = np.asfortranarray(U, dtype=np.float64)
    V = np.asfortranarray(V, dtype=np.float64)
    r = np.array(r, dtype=np.float64, copy=True)
    x = np.array(x, dtype=np.float64, copy=True)
    st = _load().orc_recycle_start(n, s, _ptr(P), _ptr(U), _ptr(V), _ptr(r), _ptr(x))
    if st != 0:
        raise RuntimeError("recycle_start: singular P^T V" if st == 1 else "recycle_start failed")
    return r, x


class reversed_sums(sum_order):
    """Context: every inner product of the oracle sums from the last index down."""

    def __init__(self):
        super().__init__(SUM_REVERSE)


def bicgstab(A: CSR, b, x0, rhat, iters: int) -> np.ndarray:
    lib = _load()
    x = np.array(x0, dtype=np.float64, copy=True)
    b = np.ascontiguousarray(b, dtype=np.float64)
    rhat = np.ascontiguousarray(rhat, dtype=np.float64)
    st = lib.orc_bicgstab(A.n, _ptr(A.row_ptr), _ptr(A.col), _ptr(A.val), _ptr(b), _ptr(x),
                          _ptr(rhat), int(iters))
    if st != OK:
        raise RuntimeError("bicgstab failed")
    return x


@dataclass
class GmresInfo:
    status: int
    mv: int
    steps: int
    cycles: int
    converged: bool
    relres_est: float
    relres_true: float
    hist_mv: np.ndarray
    hist_res: np.ndarray


def gmres(A: CSR, b, x0, m: int, tol: float = 1e-8, max_mv: int = 100000, ilu=None):
    """Restarted GMRES(m), a comparison method of Section 5.1 (oracle.c's
    orc_gmres: classical Gram-Schmidt applied twice, Givens rotations, the
    true residual at every restart decides).  ilu: optional factors (in A's
    pattern) for the split operator L^{-1} A U^{-1}.  Returns (x, GmresInfo)."""
    lib = _load()
    x = np.array(x0, dtype=np.float64, copy=True)
    b = np.ascontiguousarray(b, dtype=np.float64)
    oi = np.zeros(4, dtype=np.int64)
    of = np.zeros(2)
    cap = int(min(max_mv, 1 << 20)) + 2
    hm = np.zeros(cap, dtype=np.int64)
    hr = np.zeros(cap)
    hl = ctypes.c_int64()
    st = lib.orc_gmres(A.n, _ptr(A.row_ptr), _ptr(A.col), _ptr(A.val), int(m), float(tol), int(max_mv),
                       _ptr(b), _ptr(x), _ptr(oi), _ptr(of), _ptr(hm), _ptr(hr), cap, ctypes.byref(hl),
                       _ptr(None if ilu is None else np.ascontiguousarray(ilu, dtype=np.float64)))
    if st < 0:
        raise RuntimeError(f"orc_gmres failed with status {st}")
    k = min(hl.value, cap)
    return x, GmresInfo(int(st), int(oi[0]), int(oi[1]), int(oi[2]), bool(oi[3]), float(of[0]),
                        float(of[1]), hm[:k].copy(), hr[:k].copy())


def gmres_ilu(A: CSR, b, x0, m: int, split=None, **kw):
    """:func:`gmres` on the ILU(0) split system of :func:`solve_ilu` (same
    order, factors and transforms); returns (x, GmresInfo)."""
    Ap, lu, perm = split if split is not None else ilu_split(A)
    b = np.asarray(b, dtype=np.float64)
    bh = ilu_apply(Ap, lu, "lower", b[perm])
    y0 = ilu_apply(Ap, lu, "upper_mul", np.asarray(x0, dtype=np.float64)[perm])
    y, info = gmres(Ap, bh, y0, m, ilu=lu, **kw)
    x = np.empty(A.n)
    x[perm] = ilu_apply(Ap, lu, "upper", y)
    return x, info


def jacobi_split(A: CSR):
    """Split diagonal preconditioning (Section 5.1's form with L = R = |D|^{1/2}).

    Returns (Ahat, d, e) with e_i = sqrt(|a_ii|), d_i = 1 / e_i and
    Ahat_ij = (a_ij d_i) d_j, i.e. Ahat = L^{-1} A R^{-1}.  A row without a
    stored, finite, nonzero diagonal entry is an error.
    """
    n = A.n
    rows = np.repeat(np.arange(n), np.diff(A.row_ptr))
    on_diag = A.col == rows
    diag = np.full(n, np.nan)
    diag[rows[on_diag]] = A.val[on_diag]
    if not np.all(np.isfinite(diag)) or np.any(diag == 0.0):
        raise ValueError("jacobi_split: missing, zero or non-finite diagonal entry")
    e = np.sqrt(np.abs(diag))
    d = 1.0 / e
    val = (A.val * d[rows]) * d[A.col]
    return CSR(A.row_ptr.copy(), A.col.copy(), val), d, e


def solve_jacobi(A: CSR, b, x0, s: int, ell: int, P: np.ndarray, split=None, **kw):
    """:func:`solve` on the split system: y0 = R x0, solve Ahat y = L^{-1} b, x = R^{-1} y.

    The tolerance and the residual replacement act on the preconditioned
    residual L^{-1} (b - A R^{-1} y), as in the ocean run of Section 5.1.
    ``split`` may pass a precomputed :func:`jacobi_split` result.  Returns
    (x, info, recycle, dump) as :func:`solve`; recycled U, V live in the
    split system's space.
    """
    Ah, d, e = split if split is not None else jacobi_split(A)
    b = np.asarray(b, dtype=np.float64)
    y0 = np.asarray(x0, dtype=np.float64) * e
    y, info, rec, dd = solve(Ah, b * d, y0, s, ell, P, **kw)
    return y * d, info, rec, dd


def multicolour(A: CSR):
    """Greedy multicolour order of A's symmetrized pattern: (perm, colour_ptr)
    with perm[new] = old, colours in order, index order within a colour."""
    n = A.n
    perm = np.zeros(n, dtype=np.int32)
    cp = np.zeros(n + 1, dtype=np.int32)
    nc = _load().orc_multicolour(n, _ptr(A.row_ptr), _ptr(A.col), _ptr(perm), _ptr(cp))
    if nc < 0:
        raise MemoryError("multicolour")
    return perm, cp[:nc + 1].copy()


def permute(A: CSR, perm: np.ndarray) -> CSR:
    """The symmetrically permuted matrix Pi A Pi^T (row new = row perm[new]),
    columns sorted within each row."""
    import scipy.sparse as sp
    M = A.scipy()[perm][:, perm].tocsr()
    M.sort_indices()
    return CSR(M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float64))


def ilu0(A: CSR) -> np.ndarray:
    """ILU(0) factors in A's pattern (L below the diagonal, U on and above)."""
    lu = np.empty(A.nnz)
    st = _load().orc_ilu0(A.n, _ptr(A.row_ptr), _ptr(A.col), _ptr(A.val), _ptr(lu))
    if st != 0:
        raise ValueError("ilu0: missing or zero pivot")
    return lu


def ilu_apply(A: CSR, lu: np.ndarray, which: str, v: np.ndarray) -> np.ndarray:
    """'lower': L^{-1} v; 'upper': U^{-1} v; 'upper_mul': U v."""
    fn = {"lower": "orc_ilu_lower", "upper": "orc_ilu_upper", "upper_mul": "orc_ilu_upper_mul"}[which]
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.empty(A.n)
    getattr(_load(), fn)(A.n, _ptr(A.row_ptr), _ptr(A.col), _ptr(lu), _ptr(v), _ptr(out))
    return out


def ilu_split(A: CSR):
    """The split ILU(0) preconditioning in a multicolour order: (A', lu,
    perm) with A' = Pi A Pi^T and lu its ILU(0) factors."""
    perm, _ = multicolour(A)
    Ap = permute(A, perm)
    return Ap, ilu0(Ap), perm


def solve_ilu(A: CSR, b, x0, s: int, ell: int, P: np.ndarray, split=None, **kw):
    """:func:`solve` on the split system of Section 5.1 with ILU(0) factors of
    the multicolour-ordered matrix: L^{-1} A' U^{-1} y = L^{-1} b', x' = U^{-1} y,
    with b' = b[perm], y0 = U x0[perm] and x[perm] = x'.  P (n x s) is the
    cut-space basis of the iteration (permuted) space.  The tolerance and the
    residual history refer to the preconditioned residual.  Returns (x, info,
    recycle, dump) as :func:`solve`."""
    Ap, lu, perm = split if split is not None else ilu_split(A)
    b = np.asarray(b, dtype=np.float64)
    bh = ilu_apply(Ap, lu, "lower", b[perm])
    y0 = ilu_apply(Ap, lu, "upper_mul", np.asarray(x0, dtype=np.float64)[perm])
    y, info, rec, dd = solve(Ap, bh, y0, s, ell, P, ilu=lu, **kw)
    x = np.empty(A.n)
    x[perm] = ilu_apply(Ap, lu, "upper", y)
    return x, info, rec, dd


def rhs_step(x: np.ndarray, inv_dt: float, f: np.ndarray) -> np.ndarray:
    """Implicit Euler right-hand side b = x inv_dt + f (multiply, then add)."""
    return x * inv_dt + f


def solve_sequence(A: CSR, f, inv_dt: float, s: int, ell: int, P, systems: int,
                   method: int = MSTAB, tol: float = 1e-8, fetch: int = FETCH_THRESHOLD,
                   jacobi: bool = False, ilu: bool = False, **kw):
    """Time-stepping sequence: b^(k+1) = x^(k) inv_dt + f, x0 = x^(k), x^(0) = 0.

    ``jacobi`` solves every system in the split diagonally preconditioned form,
    ``ilu`` in the split ILU(0) form of a multicolour order."""
    x = np.zeros(A.n)
    rec = Recycle.empty(A.n, s)
    xs, infos = [], []
    split = jacobi_split(A) if jacobi else (ilu_split(A) if ilu else None)
    for _ in range(systems):
        b = rhs_step(x, inv_dt, f)
        if ilu:
            x, info, rec, _ = solve_ilu(A, b, x, s, ell, P, split=split, tol=tol, method=method,
                                        fetch=fetch, recycle=rec, **kw)
        elif jacobi:
            x, info, rec, _ = solve_jacobi(A, b, x, s, ell, P, split=split, tol=tol, method=method,
                                           fetch=fetch, recycle=rec, **kw)
        else:
            x, info, rec, _ = solve(A, b, x, s, ell, P, tol=tol, method=method, fetch=fetch,
                                    recycle=rec, **kw)
        xs.append(x.copy())
        infos.append(info)
    return xs, infos
