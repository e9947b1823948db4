"""Pins of the oracle's restarted GMRES(m), a comparison method of Section 5.1
(Saad and Schultz's minimal-residual method over the Krylov space, restarted
every m steps).  CPU only.

- Within one cycle the estimate |g_{j+1}| after step j equals the smallest
  residual over x0 + K_j(A, r0), computed independently by least squares over
  an explicit Krylov basis; the x a cycle returns attains it.
- GMRES(1) is the minimal-residual iteration x += a r, a = (Ar, r)/(Ar, Ar)
  (closed form, several restarts).
- With m >= n the method terminates: one cycle solves the system to the
  accuracy of dense LU.
- The true residual decides: a converged run has ||b - Ax|| <= tol ||b||; the
  solution agrees with LAPACK within 10 kappa tol on the variable-coefficient
  grid and the random graph, also through the ILU(0) split system.
- A zero right-hand side gives x = 0 with no product; MV counts follow the
  rule of one product per Arnoldi step plus one per true residual.
"""
import numpy as np
import pytest

from paper_1604_06043_amd import inputs as I


def _small(orc, n=6, seed=0):
    cd = I.config("c1", seed=seed, n=n)
    return orc.assemble_convdiff(cd.dim, cd.n, cd.beta, cd.inv_dt), cd


def test_estimates_equal_least_squares_over_krylov_space(orc):
    A, cd = _small(orc, 7, 3)
    D = A.dense()
    rng = np.random.default_rng(1)
    b = rng.standard_normal(A.n)
    x0 = 0.1 * rng.standard_normal(A.n)
    m = 12
    x, info = orc.gmres(A, b, x0, m, tol=0.0, max_mv=1 + m)
    # the initial residual, m steps and the true residual after the cycle
    assert info.steps == m and info.cycles == 1 and info.mv == 2 + m
    r0 = b - D @ x0
    K = np.empty((A.n, m))
    v = r0 / np.linalg.norm(r0)
    for j in range(m):   # an orthonormal basis of K_j built column by column
        K[:, j] = v
        v = D @ v
        v -= K[:, :j + 1] @ (K[:, :j + 1].T @ v)
        v -= K[:, :j + 1] @ (K[:, :j + 1].T @ v)
        v /= np.linalg.norm(v)
    nb = np.linalg.norm(b)
    for j in range(1, m + 1):
        z, *_ = np.linalg.lstsq(D @ K[:, :j], r0, rcond=None)
        best = np.linalg.norm(r0 - D @ K[:, :j] @ z)
        assert abs(info.hist_res[j] * nb - best) <= 1e-9 * np.linalg.norm(r0), (j, info.hist_res[j] * nb, best)
    # the returned x attains the last estimate
    assert abs(np.linalg.norm(b - D @ x) - info.hist_res[m] * nb) <= 1e-9 * np.linalg.norm(r0)


def test_gmres1_is_the_minimal_residual_iteration(orc):
    A, cd = _small(orc, 6, 1)
    D = A.dense()
    b = I.white_noise(2, 0, A.n)
    x = np.zeros(A.n)
    for _ in range(5):
        r = b - D @ x
        Ar = D @ r
        x = x + (Ar @ r) / (Ar @ Ar) * r
    xo, info = orc.gmres(A, b, np.zeros(A.n), 1, tol=0.0, max_mv=1 + 5 * 2)
    # five cycles of one step each, each cycle with its true residual
    assert info.cycles == 5 and info.steps == 5
    assert np.linalg.norm(xo - x) <= 1e-12 * np.linalg.norm(x)


def test_full_cycle_terminates_like_dense_lu(orc):
    rp, ci, va = I.tridiag_231(40)
    A = orc.CSR(rp, ci, va)
    D = A.dense()
    b = I.sin_rhs(40)
    x, info = orc.gmres(A, b, np.zeros(40), 40, tol=1e-13)
    ref = np.linalg.solve(D, b)
    assert info.converged and info.cycles == 1 and info.steps <= 40
    assert np.linalg.norm(x - ref) <= 10 * np.linalg.cond(D) * 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("which", ["c3", "rgg"])
@pytest.mark.parametrize("m", [5, 30])
def test_solution_matches_dense_lu(orc, which, m):
    if which == "c3":
        cd = I.config("c3", seed=2, n=7)
        A = orc.assemble_convdiff(cd.dim, cd.n, cd.beta, cd.inv_dt, cd.kappa)
        b = cd.f
    else:
        g = I.rgg(300, 3)
        A = orc.CSR(g.row_ptr, g.col, g.val)
        b = 0.1 * I.white_noise(3, 0, g.N)
    D = A.dense()
    x, info = orc.gmres(A, b, np.zeros(A.n), m)
    ref = np.linalg.solve(D, b)
    assert info.converged and info.relres_true <= 1e-8
    assert np.linalg.norm(b - D @ x) <= 1e-8 * np.linalg.norm(b) * (1 + 1e-12)
    assert np.linalg.norm(x - ref) <= 10 * np.linalg.cond(D) * 1e-8 * np.linalg.norm(ref)
    # one product per Arnoldi step and per true residual (one per cycle, plus the last)
    assert info.mv == info.steps + info.cycles + 1
    # the estimates never grow within a cycle
    h = info.hist_res
    if info.cycles == 0 or m >= info.steps:
        assert np.all(np.diff(h[1:]) <= 1e-15)


def test_ilu_split_gmres_solves_the_original_system(orc):
    cd = I.config("c3", seed=2, n=7)
    A = orc.assemble_convdiff(cd.dim, cd.n, cd.beta, cd.inv_dt, cd.kappa)
    D = A.dense()
    x, info = orc.gmres_ilu(A, cd.f, np.zeros(A.n), 10)
    _, plain = orc.gmres(A, cd.f, np.zeros(A.n), 10)
    ref = np.linalg.solve(D, cd.f)
    assert info.converged
    assert np.linalg.norm(x - ref) <= 10 * np.linalg.cond(D) * 1e-8 * np.linalg.norm(ref)
    assert info.mv < plain.mv


def test_zero_rhs_and_budget(orc):
    A, cd = _small(orc, 6, 0)
    x, info = orc.gmres(A, np.zeros(A.n), np.ones(A.n), 5)
    assert info.converged and info.mv == 0 and not x.any()
    x, info = orc.gmres(A, cd.f, np.zeros(A.n), 3, tol=1e-30, max_mv=9)
    assert not info.converged and info.status == orc.NOT_CONVERGED and info.mv == 9
