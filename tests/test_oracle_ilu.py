"""Pins of the oracle's ILU(0) split preconditioning in a multicolour order
(Section 5.1 solves L^{-1} A R^{-1} y = L^{-1} b with L, R from an incomplete
LU factorization without fill-in).  CPU only.

- The multicolour order is a permutation whose colour classes are
  independent sets (no entry couples two rows of one colour); a 2-D or 3-D
  stencil gets two colours (red-black).
- ILU(0) reproduces A on its own pattern: (L U)_ij = a_ij wherever a_ij is
  stored, with L unit lower and U upper in A's pattern (dense check).
- Where A's pattern admits no fill (a tridiagonal matrix), ILU(0) is the
  exact LU factorization (dense LAPACK LU without pivoting on a diagonally
  dominant matrix).
- The triangular solves and the product with U agree with SciPy's
  triangular solver and with dense products.
- The split preconditioned solve recovers x with ||x - x_LU|| <= 10 kappa tol
  against LAPACK, on the variable-coefficient grid and the random graph.
- Planted mistakes (a skipped update, L applied instead of L^{-1}) fail them.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
from scipy.sparse.linalg import spsolve_triangular

from paper_1604_06043_amd import inputs as I


def dense_factors(A, lu):
    D = np.zeros((A.n, A.n))
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    D[rows, A.col] = lu
    L = np.tril(D, -1) + np.eye(A.n)
    U = np.triu(D)
    return L, U


def small_matrices(orc):
    cd = I.config("c3", seed=2, n=6)
    A3 = orc.assemble_convdiff(cd.dim, cd.n, cd.beta, cd.inv_dt, cd.kappa)
    cd2 = I.config("c1", seed=0, n=9)
    A2 = orc.assemble_convdiff(cd2.dim, cd2.n, cd2.beta, cd2.inv_dt)
    g = I.rgg(300, 3)
    Ag = orc.CSR(g.row_ptr, g.col, g.val)
    return {"c3_6": A3, "c1_9": A2, "rgg_300": Ag}


@pytest.mark.parametrize("name", ["c3_6", "c1_9", "rgg_300"])
def test_multicolour_classes_are_independent(orc, name):
    A = small_matrices(orc)[name]
    perm, cp = orc.multicolour(A)
    assert np.array_equal(np.sort(perm), np.arange(A.n))
    assert cp[0] == 0 and cp[-1] == A.n and np.all(np.diff(cp) > 0)
    colour = np.empty(A.n, dtype=int)
    for c in range(len(cp) - 1):
        colour[perm[cp[c]:cp[c + 1]]] = c
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    off = rows != A.col
    assert not np.any(colour[rows[off]] == colour[A.col[off]])
    if name != "rgg_300":
        assert len(cp) - 1 == 2          # red-black for a stencil
    # index order within a colour
    for c in range(len(cp) - 1):
        assert np.all(np.diff(perm[cp[c]:cp[c + 1]]) > 0)


@pytest.mark.parametrize("name", ["c3_6", "c1_9", "rgg_300"])
def test_ilu0_reproduces_a_on_its_pattern(orc, name):
    A = small_matrices(orc)[name]
    Ap, lu, perm = orc.ilu_split(A)
    L, U = dense_factors(Ap, lu)
    D = Ap.dense()
    LU = L @ U
    mask = D != 0
    scale = np.abs(D).max()
    assert np.max(np.abs(LU[mask] - D[mask])) <= 1e-13 * scale
    # the factors live in A's pattern (no fill)
    assert np.all((np.tril(L, -1) != 0) <= mask) and np.all((U != 0) <= mask)
    # it is not the exact factorization: the dropped fill is where LU and A differ
    assert np.max(np.abs(LU - D)) > 1e-6 * scale


def test_ilu0_is_exact_without_fill(orc):
    n = 30
    rng = np.random.default_rng(4)
    main = 4.0 + rng.random(n)
    lower, upper = -1.0 + 0.5 * rng.random(n - 1), -1.0 + 0.5 * rng.random(n - 1)
    M = sp.diags([lower, main, upper], [-1, 0, 1]).tocsr()
    M.sort_indices()
    A = orc.CSR(M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.copy())
    lu = orc.ilu0(A)
    L, U = dense_factors(A, lu)
    # LAPACK LU without pivoting is available as scipy's lu with permute_l off:
    # on a diagonally dominant matrix partial pivoting does not swap rows
    Pm, L2, U2 = sla.lu(M.toarray())
    assert np.allclose(Pm, np.eye(n))
    assert np.allclose(L, L2, rtol=1e-13, atol=1e-15) and np.allclose(U, U2, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("name", ["c3_6", "rgg_300"])
def test_triangular_solves_against_scipy(orc, name):
    A = small_matrices(orc)[name]
    Ap, lu, _ = orc.ilu_split(A)
    L, U = dense_factors(Ap, lu)
    v = np.random.default_rng(1).standard_normal(A.n)
    y = orc.ilu_apply(Ap, lu, "lower", v)
    assert np.allclose(y, spsolve_triangular(sp.csr_matrix(L), v, lower=True), rtol=1e-12, atol=1e-12)
    x = orc.ilu_apply(Ap, lu, "upper", v)
    assert np.allclose(x, spsolve_triangular(sp.csr_matrix(U), v, lower=False), rtol=1e-12, atol=1e-12)
    assert np.allclose(orc.ilu_apply(Ap, lu, "upper_mul", v), U @ v, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("name,s,ell", [("c3_6", 4, 2), ("c1_9", 2, 1), ("rgg_300", 4, 2), ("c3_6", 8, 4)])
def test_ilu_split_solve_matches_dense_lu(orc, name, s, ell):
    A = small_matrices(orc)[name]
    D = A.dense()
    b = np.random.default_rng(2).standard_normal(A.n)
    P = I.p_dense(3, A.n, s)
    x, info, _, _ = orc.solve_ilu(A, b, np.zeros(A.n), s, ell, P, tol=1e-10)
    assert info.converged
    xd = np.linalg.solve(D, b)
    kappa = np.linalg.cond(D)
    assert np.linalg.norm(x - xd) <= 10 * kappa * 1e-10 * np.linalg.norm(xd)
    # ILU(0) takes no more products than the unpreconditioned solve (at
    # s = 8, l = 4 one cycle already suffices for both on this small grid)
    _, plain, _, _ = orc.solve(A, b, np.zeros(A.n), s, ell, P, tol=1e-10)
    assert info.mv_total <= plain.mv_total
    if s * ell < 32:
        assert info.mv_total < plain.mv_total


def test_ilu_preconditioned_operator_is_l_inverse_a_u_inverse(orc):
    """The operator the iteration sees, checked column by column on a dense
    copy: L^{-1} A' U^{-1} e_j (so a plain product with L, or U instead of
    U^{-1}, fails)."""
    A = small_matrices(orc)["c1_9"]
    Ap, lu, _ = orc.ilu_split(A)
    L, U = dense_factors(Ap, lu)
    ref = np.linalg.solve(L, Ap.dense() @ np.linalg.inv(U))
    P = I.p_dense(0, A.n, 1)
    # one cycle's first product with the dump: r^(1) = Ahat r^(0)
    b = np.random.default_rng(5).standard_normal(A.n)
    _, _, _, dd = orc.solve(Ap, b, np.zeros(A.n), 1, 1, P, ilu=lu, dump_cycle=0, method=orc.IDRSTAB)
    R = dd["R"]
    assert np.allclose(R[1], ref @ R[0], rtol=1e-12, atol=1e-12 * np.abs(R[1]).max())
