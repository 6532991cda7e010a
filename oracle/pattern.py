"""Superset sparsity pattern of A_t (oracle side, TEST INFRASTRUCTURE ONLY).

The pattern is fixed for the whole run: it is the set of node pairs that
co-occur in any candidate tetrahedron of the superset (paper Sec. 3.1: the
superset vertices and candidate pool are allocated up front; Sec. 3.4: the
element-assembled operator is a sum over the fixed superset).  Entries whose
every incident candidate is inactive stay in the pattern with value +0.0.

CSR over 3n rows: dof 3i+p is component p of node i.  Row 3i+p holds the
columns 3j+q for every node j paired with i (including j = i), ascending.
"""
import numpy as np


def pattern(n_nodes: int, tets: np.ndarray):
    """(rowptr int32 (3n+1,), colidx int32 (nnz,)) of the superset pattern."""
    t = np.asarray(tets, dtype=np.int64)
    i = np.repeat(t, 4, axis=1).reshape(-1)      # t[:, a] for a, b in 4x4
    j = np.tile(t, (1, 4)).reshape(-1)           # t[:, b]
    keys = np.unique(i * n_nodes + j)            # sorted unique node pairs (i, j)
    pi, pj = keys // n_nodes, keys % n_nodes
    p = np.arange(3)
    rows = (3 * pi[:, None, None] + p[None, :, None]).repeat(3, axis=2).reshape(-1)
    cols = (3 * pj[:, None, None] + p[None, None, :]).repeat(3, axis=1).reshape(-1)
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    counts = np.bincount(rows, minlength=3 * n_nodes)
    rowptr = np.zeros(3 * n_nodes + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return rowptr.astype(np.int32), cols.astype(np.int32)


def csr_to_dense(rowptr, colidx, vals, n_rows):
    """Dense matrix from CSR (absent entries 0.0)."""
    D = np.zeros((n_rows, n_rows))
    r = np.repeat(np.arange(n_rows), np.diff(rowptr))
    D[r, colidx] = vals
    return D
