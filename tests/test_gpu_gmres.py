"""Restarted GMRES(m) on the GPU (METHOD_GMRES), one of Section 5.1's
comparison methods, against the oracle's orc_gmres: the same algorithm
(classical Gram-Schmidt applied twice, Givens rotations, the true residual at
every restart decides), so x agrees to the oracle's own summation-order
spread and the MV counts agree wherever that spread leaves them alone."""
import numpy as np
import pytest

from paper_1604_06043_amd import inputs as I
from test_gpu_parity import dev, gpu_assemble, ms, rel, torch_dev, upload_csr  # noqa: F401

pytestmark = pytest.mark.gpu


def oracle_orders(orc, fn):
    """fn() -> (x, GmresInfo) in the forward order, and the largest relative
    distance of the reverse and blocked orders' x from it, and whether their
    MV counts differ."""
    x, info = fn()
    sen, spread = 0.0, 0
    for order in (orc.SUM_REVERSE, orc.SUM_BLOCKED):
        with orc.sum_order(order):
            xa, ia = fn()
        sen = max(sen, rel(xa, x))
        spread = max(spread, abs(ia.mv - info.mv))
    return x, info, sen, spread


def check(ig, io, err, sen, spread, hist_g):
    assert ig["converged"] and io.converged, (ig, io)
    assert ig["relres_true"] <= 1e-8 * (1 + 1e-12)
    assert err <= max(1e-9, 10 * sen), (err, sen)
    assert abs(ig["mv_total"] - io.mv) <= spread + 2, (ig["mv_total"], io.mv, spread)
    if ig["mv_total"] == io.mv:
        assert list(hist_g[0]) == list(io.hist_mv)
        np.testing.assert_allclose(hist_g[1], io.hist_res, rtol=1e-4, atol=1e-12)


def problem(torch, orc, name, n, seed):
    if name == "rgg":
        g = I.rgg(n, seed)
        Ao = orc.CSR(g.row_ptr, g.col, g.val)
        return Ao, upload_csr(torch, ms_mod(), Ao), 0.1 * I.white_noise(seed, 0, g.N)
    cd = I.config(name, seed=seed, n=n)
    Ao = orc.assemble_convdiff(cd.dim, cd.n, cd.beta, cd.inv_dt, cd.kappa)
    return Ao, gpu_assemble(ms_mod(), cd), cd.f


def ms_mod():
    from paper_1604_06043_amd import mstab
    return mstab


@pytest.mark.parametrize("name,n,seed,m", [
    ("c1", 64, 0, 30), ("c1", 64, 1, 10), ("c1", 50, 2, 1), ("c3", 14, 4, 30), ("c3", 16, 1, 5),
    ("c2", 16, 3, 60), ("rgg", 20000, 5, 20)])
def test_gmres_matches_oracle(torch_dev, ms, orc, name, n, seed, m):
    torch = torch_dev
    print(f"[gmres {name} n={n} m={m}]", flush=True)
    Ao, Ag, b = problem(torch, orc, name, n, seed)
    sv = ms.Solver(Ag, 1, 1, method=ms.METHOD_GMRES, gmres_restart=m)
    # two right-hand sides: b from zero, then b + A-scaled noise from the first x
    x0 = np.zeros(Ao.n)
    for k in range(2):
        bk = b if k == 0 else b + 0.05 * I.white_noise(seed + 7, k, Ao.n)
        x = dev(torch, x0)
        ig = sv.solve_next(dev(torch, bk), x)
        xo, io, sen, spread = oracle_orders(orc, lambda: orc.gmres(Ao, bk, x0, m))
        err = rel(x.cpu().numpy(), xo)
        print(f"  system {k}: gpu mv {ig['mv_total']} (steps {ig['cycles']}, restarts {ig['restarts']}) "
              f"oracle {io.mv} (steps {io.steps}, cycles {io.cycles}), err {err:.1e}, sens {sen:.1e}, "
              f"spread {spread}", flush=True)
        check(ig, io, err, sen, spread, sv.residual_history())
        assert ig["cycles"] == io.steps or ig["mv_total"] != io.mv
        x0 = xo
    sv.close()


@pytest.mark.parametrize("name,n,seed,m", [("c3", 16, 1, 20), ("rgg", 20000, 5, 20)])
def test_gmres_ilu_split_matches_oracle(torch_dev, ms, orc, name, n, seed, m):
    """GMRES on the ILU(0) split system of a multicolour order (Section 5.1
    preconditions its GMRES runs the same way)."""
    torch = torch_dev
    Ao, Ag, b = problem(torch, orc, name, n, seed)
    split = orc.ilu_split(Ao)
    sv = ms.Solver(Ag, 1, 1, method=ms.METHOD_GMRES, gmres_restart=m, precond=ms.PRECOND_ILU0)
    x = torch.zeros(Ao.n, dtype=torch.float64, device="cuda")
    ig = sv.solve_next(dev(torch, b), x)
    xo, io, sen, spread = oracle_orders(orc, lambda: orc.gmres_ilu(Ao, b, np.zeros(Ao.n), m, split=split))
    err = rel(x.cpu().numpy(), xo)
    print(f"  gpu mv {ig['mv_total']} oracle {io.mv}, err {err:.1e}, sens {sen:.1e}", flush=True)
    check(ig, io, err, sen, spread, sv.residual_history())
    sv.close()


def test_gmres_edge_cases(torch_dev, ms, orc):
    """Zero right-hand side: x = 0, no product.  A budget too small to
    converge: NOT_CONVERGED with the oracle's count.  Options GMRES refuses."""
    torch = torch_dev
    cd = I.config("c1", seed=0, n=24)
    Ao = orc.assemble_convdiff(cd.dim, cd.n, cd.beta, cd.inv_dt)
    Ag = gpu_assemble(ms, cd)
    sv = ms.Solver(Ag, 1, 1, method=ms.METHOD_GMRES, gmres_restart=5)
    x = torch.ones(cd.N, dtype=torch.float64, device="cuda")
    ig = sv.solve_next(torch.zeros_like(x), x)
    assert ig["converged"] and ig["mv_total"] == 0 and not x.any()
    sv.close()
    sv = ms.Solver(Ag, 1, 1, method=ms.METHOD_GMRES, gmres_restart=3, max_mv=9, tol=1e-30)
    x = torch.zeros(cd.N, dtype=torch.float64, device="cuda")
    ig = sv.solve_next(dev(torch, cd.f), x)
    _, io = orc.gmres(Ao, cd.f, np.zeros(cd.N), 3, tol=1e-30, max_mv=9)
    assert not ig["converged"] and ig["status"] == ms.NOT_CONVERGED and ig["mv_total"] == io.mv == 9
    sv.close()
    for bad in (dict(gmres_restart=0), dict(precision=ms.PREC_F32_MATRIX), dict(engine=1)):
        with pytest.raises(ms.MstabError):
            ms.Solver(Ag, 1, 1, method=ms.METHOD_GMRES, **bad)
