"""The reverse Cuthill-McKee order of the library (host code, no GPU): a
permutation, exact on a relabelled path (bandwidth 1), components kept
contiguous, and on the random geometric graph a band far narrower than the
random labelling's and comparable to SciPy's reverse_cuthill_mckee."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import reverse_cuthill_mckee

from paper_1604_06043_amd import inputs as I
from paper_1604_06043_amd import mstab


def bandwidth(rp, ci, perm):
    iperm = np.empty_like(perm)
    iperm[perm] = np.arange(perm.size, dtype=perm.dtype)
    rows = np.repeat(np.arange(rp.size - 1), np.diff(rp))
    return int(np.max(np.abs(iperm[rows] - iperm[ci])))


def csr(M):
    M = sp.csr_matrix(M)
    M.sort_indices()
    return M.indptr.astype(np.int32), M.indices.astype(np.int32)


def test_relabelled_path_gets_bandwidth_one():
    n = 500
    rng = np.random.default_rng(0)
    lab = rng.permutation(n)
    i = np.arange(n - 1)
    M = sp.coo_matrix((np.ones(2 * (n - 1)), (np.r_[lab[i], lab[i + 1]], np.r_[lab[i + 1], lab[i]])),
                      shape=(n, n)) + sp.identity(n)
    rp, ci = csr(M)
    perm = mstab.mstab_rcm_order(rp, ci)
    assert np.array_equal(np.sort(perm), np.arange(n))
    assert bandwidth(rp, ci, np.arange(n, dtype=np.int32)) > 100
    assert bandwidth(rp, ci, perm) == 1


def test_components_stay_contiguous():
    a = sp.random(300, 300, density=0.02, random_state=1)
    b = sp.random(200, 200, density=0.03, random_state=2)
    M = sp.block_diag([a + a.T + sp.identity(300), b + b.T + sp.identity(200)])
    lab = np.random.default_rng(3).permutation(500)
    M = sp.csr_matrix(M)[lab][:, lab]
    rp, ci = csr(M)
    perm = mstab.mstab_rcm_order(rp, ci)
    assert np.array_equal(np.sort(perm), np.arange(500))
    # connected components of the relabelled matrix: each is one run of the order
    from scipy.sparse.csgraph import connected_components
    _, comp = connected_components(M, directed=False)
    runs = np.count_nonzero(np.diff(comp[perm]) != 0) + 1
    assert runs == comp.max() + 1


def test_random_geometric_graph_band():
    g = I.rgg(20000, 4)
    rp, ci = g.row_ptr, g.col
    perm = mstab.mstab_rcm_order(rp, ci)
    assert np.array_equal(np.sort(perm), np.arange(rp.size - 1))
    ident = np.arange(rp.size - 1, dtype=np.int32)
    M = sp.csr_matrix((np.ones(ci.size), ci, rp))
    ref = reverse_cuthill_mckee(M, symmetric_mode=False).astype(np.int32)
    b_lib, b_ref, b_id = bandwidth(rp, ci, perm), bandwidth(rp, ci, ref), bandwidth(rp, ci, ident)
    print(f"bandwidth: random labels {b_id}, library {b_lib}, scipy {b_ref}")
    assert b_lib < 0.2 * b_id   # a 3-D graph: the band grows like N^(2/3)
    assert b_lib <= 1.5 * b_ref


def test_rcm_rejects_bad_arguments():
    with pytest.raises(mstab.MstabError):
        mstab.mstab_rcm_order(np.array([0, 2, 1], dtype=np.int32), np.array([0, 1], dtype=np.int32))
    with pytest.raises(mstab.MstabError):
        mstab.mstab_rcm_order(np.array([0, 1, 2], dtype=np.int32), np.array([0, 5], dtype=np.int32))
