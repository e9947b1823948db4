"""The random-geometric-graph matrix of the unstructured workload, checked on
small instances against a brute-force construction from its definition."""
import math

import numpy as np
import pytest

from paper_1604_06043_amd import inputs as I


def brute_force(N, seed, degree=14.0):
    pts = I.uniform(seed, I.S_RGG, 3 * N).reshape(N, 3)
    r = (3.0 * degree / (4.0 * math.pi * N)) ** (1.0 / 3.0)
    g = I.normal(seed, I.S_DIR, 3)
    beta = g / np.linalg.norm(g)
    A = np.eye(N)
    for a in range(N):
        for b in range(N):
            if a == b:
                continue
            d = pts[b] - pts[a]
            d -= np.round(d)                      # shortest periodic displacement
            if np.sqrt(d @ d) < r:
                A[a, b] = -1.0 + (d @ beta) / (2.0 * r)
                A[a, a] += 1.0
    keys = I.uniform(seed, I.S_RGG, N, offset=3 * N)
    perm = np.argsort(keys, kind="stable")        # new index k holds old row perm[k]
    return A[np.ix_(perm, perm)]


@pytest.mark.parametrize("N,seed", [(300, 0), (500, 7)])
def test_rgg_matches_brute_force(N, seed):
    g = I.rgg(N, seed)
    assert g.row_ptr.dtype == np.int32 and g.col.dtype == np.int32
    dense = np.zeros((N, N))
    for i in range(N):
        cols = g.col[g.row_ptr[i]:g.row_ptr[i + 1]]
        assert np.all(np.diff(cols) > 0)          # sorted, no duplicates
        dense[i, cols] = g.val[g.row_ptr[i]:g.row_ptr[i + 1]]
    np.testing.assert_allclose(dense, brute_force(N, seed), rtol=0, atol=1e-14)


def test_rgg_structure():
    g = I.rgg(20000, 3)
    N = g.N
    rows = np.repeat(np.arange(N), np.diff(g.row_ptr))
    import scipy.sparse as sp
    A = sp.csr_matrix((g.val, g.col, g.row_ptr), shape=(N, N))
    sym = (A + A.T) / 2
    skew = (A - A.T) / 2
    # I + L: unit row sums; S: antisymmetric with zero diagonal and |S_ij| <= 1/2
    assert np.abs(np.asarray(sym.sum(axis=1)).ravel() - 1.0).max() < 1e-12
    assert np.abs(skew.diagonal()).max() == 0.0
    assert np.abs(skew.data).max() <= 0.5
    # expected degree 14 (Poisson-like spread)
    deg = np.diff(g.row_ptr) - 1
    assert abs(deg.mean() - 14.0) < 0.3
    assert rows.shape[0] == g.nnz
