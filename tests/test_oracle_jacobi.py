"""Pins of the oracle's split diagonal preconditioning (Section 5.1's split form
L^{-1} A R^{-1} y = L^{-1} b, x = R^{-1} y, with L = R = |D|^{1/2}).

Each check rests on a fact the splitting fixes, not on the oracle's own code:
the split matrix has a unit-magnitude diagonal, keeps a symmetric matrix
symmetric and is similar to |D|^{-1} A; a diagonal matrix is solved in closed
form; a constant diagonal makes the split system a pure rescaling, under which
the Krylov iteration is invariant; and the recovered x solves the original
system (dense LU).
"""
import numpy as np
import pytest
import scipy.linalg as sla

from paper_1604_06043_amd import inputs as I

EPS = np.finfo(np.float64).eps


def csr_from_dense(orc, D):
    n = D.shape[0]
    rp, ci, va = [0], [], []
    for i in range(n):
        nz = np.nonzero(D[i])[0]
        ci.extend(nz.tolist())
        va.extend(D[i, nz].tolist())
        rp.append(len(ci))
    return orc.CSR(np.array(rp, dtype=np.int32), np.array(ci, dtype=np.int32), np.array(va))


def symmetric_test_matrix(n, seed):
    rng = np.random.default_rng(seed)
    M = np.zeros((n, n))
    for _ in range(3 * n):
        i, j = rng.integers(0, n, 2)
        if i != j:
            v = rng.standard_normal()
            M[i, j] = M[j, i] = v
    diag = np.exp(2.0 * rng.standard_normal(n)) * rng.choice([-1.0, 1.0], n)
    np.fill_diagonal(M, diag)
    return M


def test_split_diagonal_and_symmetry(orc):
    D = symmetric_test_matrix(60, 0)
    A = csr_from_dense(orc, D)
    Ah, d, e = orc.jacobi_split(A)
    H = Ah.dense()
    # |D|^{-1/2} A |D|^{-1/2}: diagonal sign(a_ii), symmetric
    np.testing.assert_allclose(np.diag(H), np.sign(np.diag(D)), rtol=4 * EPS, atol=0)
    np.testing.assert_allclose(H, H.T, rtol=4 * EPS, atol=0)
    np.testing.assert_allclose(d * e, 1.0, rtol=2 * EPS)
    np.testing.assert_allclose(e * e, np.abs(np.diag(D)), rtol=4 * EPS)


def test_split_similar_to_diagonally_scaled_matrix(orc):
    """Spectrum of L^{-1} A R^{-1} equals that of |D|^{-1} A (a similarity)."""
    cd = I.config("c3", seed=2, n=6)
    A = orc.assemble_convdiff(cd.dim, cd.n, cd.beta, cd.inv_dt, cd.kappa)
    Ad = A.dense()
    Ah, _, _ = orc.jacobi_split(A)
    ev_h = sla.eigvals(Ah.dense())
    ev_s = sla.eigvals(Ad / np.abs(np.diag(Ad))[:, None])

    def gap(u, v):   # largest distance from a point of u to the nearest of v, both ways
        dist = np.abs(u[:, None] - v[None, :])
        return max(dist.min(axis=1).max(), dist.min(axis=0).max())

    # (clustered eigenvalues of a nonnormal matrix: rounding moves them ~1e-9)
    assert gap(ev_h, ev_s) <= 1e-7 * np.max(np.abs(ev_s))
    # and the spectrum is not that of A itself (the diagonal varies)
    ev_a = sla.eigvals(Ad)
    assert gap(ev_a / np.max(np.abs(ev_a)), ev_s / np.max(np.abs(ev_s))) > 1e-3


def test_diagonal_matrix_closed_form(orc):
    """A = diag(a): the split matrix is diag(sign a) and x = b / a."""
    rng = np.random.default_rng(3)
    n = 200
    a = np.exp(3.0 * rng.standard_normal(n)) * rng.choice([-1.0, 1.0], n)
    A = csr_from_dense(orc, np.diag(a))
    b = rng.standard_normal(n)
    P = I.p_dense(3, n, 2)
    x, info, _, _ = orc.solve_jacobi(A, b, np.zeros(n), 2, 1, P, method=orc.IDRSTAB)
    assert info.converged
    np.testing.assert_allclose(x, b / a, rtol=1e-12)
    # without the splitting the same solve needs many more products
    _, plain, _, _ = orc.solve(A, b, np.zeros(n), 2, 1, P, method=orc.IDRSTAB)
    assert info.mv_total < plain.mv_total


def test_constant_diagonal_is_a_rescaling(orc):
    """Constant coefficients give a constant diagonal c: the split system is
    A y = sqrt(c) b with A/c, y = sqrt(c) x; the iteration is scale-invariant,
    so the solve takes the same products and reaches the same x."""
    cd, = [I.config("c2", seed=1, n=8)]
    A = orc.assemble_convdiff(cd.dim, cd.n, cd.beta, cd.inv_dt)
    Ah, d, _ = orc.jacobi_split(A)
    c = A.dense().diagonal()
    assert np.all(c == c[0])
    np.testing.assert_allclose(Ah.val, A.val / c[0], rtol=4 * EPS)
    P = I.p_dense(1, cd.N, 4)
    xj, ij, _, _ = orc.solve_jacobi(A, cd.f, np.zeros(cd.N), 4, 2, P, method=orc.IDRSTAB)
    xp, ip, _, _ = orc.solve(A, cd.f, np.zeros(cd.N), 4, 2, P, method=orc.IDRSTAB)
    assert ij.mv_total == ip.mv_total
    np.testing.assert_allclose(ij.hist_res, ip.hist_res, rtol=1e-9, atol=1e-15)
    assert np.linalg.norm(xj - xp) <= 1e-10 * np.linalg.norm(xp)


@pytest.mark.parametrize("kind", ["c3", "graph"])
def test_split_solution_matches_dense_lu(orc, kind):
    if kind == "c3":
        cd = I.config("c3", seed=4, n=8)
        A = orc.assemble_convdiff(cd.dim, cd.n, cd.beta, cd.inv_dt, cd.kappa)
        b = cd.f
    else:
        g = I.rgg(300, 5)
        A = orc.CSR(g.row_ptr, g.col, g.val)
        b = np.random.default_rng(5).standard_normal(A.n)
    Ad = A.dense()
    x_lu = np.linalg.solve(Ad, b)
    P = I.p_dense(4, A.n, 4)
    x, info, _, _ = orc.solve_jacobi(A, b, np.zeros(A.n), 4, 2, P, method=orc.IDRSTAB)
    assert info.converged
    Ah, d, _ = orc.jacobi_split(A)
    # the tolerance holds for the preconditioned residual L^{-1}(b - A x)
    assert np.linalg.norm(d * (b - Ad @ x)) <= 1.01e-8 * np.linalg.norm(d * b)
    kappa = np.linalg.cond(Ah.dense())
    assert np.linalg.norm(x - x_lu) <= 10 * kappa * 1e-8 * np.linalg.norm(x_lu)


def test_split_rejects_missing_or_zero_diagonal(orc):
    D = np.diag(np.arange(1.0, 6.0))
    D[2, 2] = 0.0
    D[2, 3] = 1.0
    with pytest.raises(ValueError):
        orc.jacobi_split(csr_from_dense(orc, D))


def test_periodic_replacement_tracks_true_residual(orc):
    """Section 5.1's ocean run replaces the residual by the true one after the
    solution update of every cycle.  With replace_every = 1 each recorded
    residual (but the last, below the tolerance) is the true residual of that
    cycle's x, computed here independently; each replacement costs one check
    product.  The recycled start of this split system has a recursive/true gap
    of ~1e-10 relative without it."""
    cd = I.config("c3", seed=4, n=14)
    A = orc.assemble_convdiff(cd.dim, cd.n, cd.beta, cd.inv_dt, cd.kappa)
    split = orc.jacobi_split(A)
    Ah, d, _ = split
    S = Ah.scipy()
    P = I.p_dense(4, cd.N, 8)
    x1, _, rec, _ = orc.solve_jacobi(A, cd.f, np.zeros(cd.N), 8, 4, P, split=split)
    b1 = orc.rhs_step(x1, cd.inv_dt, cd.f)
    bh = b1 * d
    gaps, ratio = {}, {}
    for every in (0, 1):
        _, info, _, _ = orc.solve_jacobi(A, b1, x1, 8, 4, P, split=split, recycle=rec.copy(),
                                         replace_every=every)
        assert info.converged
        gaps[every], ratio[every] = [], []
        for c in range(info.cycles):
            _, _, _, dd = orc.solve_jacobi(A, b1, x1, 8, 4, P, split=split, recycle=rec.copy(),
                                           replace_every=every, dump_cycle=c)
            true = np.linalg.norm(bh - S @ dd["x_after"]) / np.linalg.norm(bh)
            gaps[every].append(abs(info.hist_res[c + 1] - true) / true)
            ratio[every].append(true / info.hist_res[c + 1])
        if every == 1:
            assert max(gaps[1][:-1]) <= 1e-8, gaps[1]
            # one check product per replaced cycle, plus the final true residual
            assert info.replacements == info.cycles - 1
            assert info.mv_check == info.cycles
    assert max(ratio[0]) > 1e3   # the gap the replacement removes


def test_periodic_replacement_every_second_cycle(orc):
    """replace_every = 2 replaces after cycles 2, 4, ...: on an unpreconditioned
    system that needs several cycles, the count of check products is fixed by
    the number of cycles."""
    cd = I.config("c1", seed=0, n=32)
    A = orc.assemble_convdiff(cd.dim, cd.n, cd.beta, cd.inv_dt)
    P = I.p_dense(0, cd.N, 2)
    _, info, _, _ = orc.solve(A, cd.f, np.zeros(cd.N), 2, 1, P, method=orc.IDRSTAB,
                              replace_every=2)
    assert info.converged and info.cycles >= 5
    # cycles 2, 4, ... below the last replace; the last ends below tol
    periodic = (info.cycles - 1) // 2
    assert info.mv_check == periodic + 1 + (info.replacements - periodic)
    assert info.replacements >= periodic
