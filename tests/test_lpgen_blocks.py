"""Row and column blocks of an LP (the share of K and K^T one GPU would own
under a partition) reassemble the LP exactly; the random-structure cases
carry optimal planted pairs."""
import numpy as np
import scipy.sparse as sp

import lpgen


def _csr(lp):
    return sp.csr_matrix((lp.val, lp.col, lp.rowptr), shape=(lp.m, lp.n))


def test_row_blocks_stack_to_k():
    lp = lpgen.config2(5, m=2000, n=4000, kmax=500)
    P = 8
    blocks = [lpgen.row_block(lp, p * lp.m // P, (p + 1) * lp.m // P) for p in range(P)]
    K = sp.vstack([_csr(b) for b in blocks]).tocsr()
    assert (K != _csr(lp)).nnz == 0
    np.testing.assert_array_equal(np.concatenate([b.rhs for b in blocks]), lp.rhs)
    np.testing.assert_array_equal(np.concatenate([b.row_type for b in blocks]), lp.row_type)
    for b in blocks:
        assert b.n == lp.n and b.rowptr[0] == 0 and b.rowptr[-1] == b.val.size
        np.testing.assert_array_equal(b.c, lp.c)


def test_col_blocks_concatenate_to_k():
    lp = lpgen.config2(6, m=2000, n=4000, kmax=500)
    P = 8
    cuts = [p * lp.n // P for p in range(P + 1)]
    blocks = [lpgen.col_block(lp, cuts[p], cuts[p + 1]) for p in range(P)]
    K = sp.hstack([_csr(b) for b in blocks]).tocsr()
    assert (K != _csr(lp)).nnz == 0
    assert sum(b.nnz for b in blocks) == lp.nnz
    np.testing.assert_array_equal(np.concatenate([b.c for b in blocks]), lp.c)
    np.testing.assert_array_equal(np.concatenate([b.u for b in blocks]), lp.u)
    for b in blocks:
        assert b.m == lp.m and np.all(np.diff(b.rowptr) >= 0)
        assert b.col.dtype == np.int32 and (b.col.size == 0 or (b.col.min() >= 0 and b.col.max() < b.n))
    # entries keep their order inside each row
    for p, b in enumerate(blocks):
        for i in range(0, lp.m, 97):
            c = lp.col[lp.rowptr[i]:lp.rowptr[i + 1]]
            v = lp.val[lp.rowptr[i]:lp.rowptr[i + 1]]
            sel = (c >= cuts[p]) & (c < cuts[p + 1])
            np.testing.assert_array_equal(b.col[b.rowptr[i]:b.rowptr[i + 1]], c[sel] - cuts[p])
            np.testing.assert_array_equal(b.val[b.rowptr[i]:b.rowptr[i + 1]], v[sel])


def test_random_cases_plant_optimal_pairs(orc):
    """The planted (x*, y*) of every random-structure case has KKT error 0 to
    rounding under the oracle's KKT function (Section 2.3.2) and is feasible."""
    names = set()
    for seed in range(32):
        lp = lpgen.random_case(seed)
        k = orc.Oracle(lp).kkt(lp.x_star, lp.y_star)
        assert k["rel_kkt"] <= 1e-9, (seed, lp.name, k)
        assert np.all(lp.x_star >= lp.l - 1e-12) and np.all(lp.x_star <= lp.u + 1e-12)
        names.add(lp.name.split("-")[-1] if "-" in lp.name else lp.name[:4])
    assert "emptied" in names and "tiny" in names  # every family occurs
