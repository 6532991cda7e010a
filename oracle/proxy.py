"""Graph-Laplacian proxy operator (oracle side, TEST INFRASTRUCTURE ONLY).

The paper's proxy system (Sec. 3.1): every active tetrahedron contributes its
six undirected edges; the multiplicity c_t(u,v) counts the active tets that
contain edge (u,v) (eq. (1)); an edge is active when that count is positive
(eq. (2)); the Laplacian has -a_t(u,v) off the diagonal and the number of
active edges at u on it (eq. (3)); the solved matrix adds eps on the diagonal
(eq. (4)).

Computed here from the mask alone, nothing incremental: the streaming update
must reach the same integers and the same matrix entries (Sec. 3.3
invariant).  Layout readings shared with the elasticity operator:

* the pattern is fixed: the scalar CSR over n rows holds, for each vertex that
  lies in some candidate tet, its diagonal and one entry per candidate edge
  at it, columns ascending;
* an inactive edge stays in the pattern with value +0.0 (not -0.0, which
  a literal -a_t would give for a_t = 0);
* a diagonal entry is float64(degree) + eps, one rounding.
"""
import numpy as np

PAIRS = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


def edges_of(tets):
    """(m, 6, 2) int64: the six undirected edges of every tet as (min, max)."""
    t = np.asarray(tets, dtype=np.int64)
    e = np.stack([np.stack([t[:, a], t[:, b]], axis=1) for a, b in PAIRS], axis=1)
    return np.sort(e, axis=2)


def proxy_pattern(n_nodes: int, tets):
    """Scalar superset pattern: (rowptr (n+1,), colidx, edges (E, 2) sorted (u<v) pairs)."""
    e = edges_of(tets).reshape(-1, 2)
    keys = np.unique(e[:, 0] * n_nodes + e[:, 1])
    edges = np.stack([keys // n_nodes, keys % n_nodes], axis=1)
    used = np.unique(np.asarray(tets, dtype=np.int64).reshape(-1))
    rows = np.concatenate([used, edges[:, 0], edges[:, 1]])
    cols = np.concatenate([used, edges[:, 1], edges[:, 0]])
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    rowptr = np.zeros(n_nodes + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n_nodes), out=rowptr[1:])
    return rowptr.astype(np.int32), cols.astype(np.int32), edges.astype(np.int32)


def edge_index(n_nodes: int, edges, pairs):
    """Position in the sorted edge list of each (min, max) pair."""
    keys = edges[:, 0].astype(np.int64) * n_nodes + edges[:, 1]
    want = pairs[..., 0].astype(np.int64) * n_nodes + pairs[..., 1]
    k = np.searchsorted(keys, want)
    assert np.all(keys[k] == want)
    return k


def entry_index(n_nodes: int, rowptr, colidx, rows, cols):
    """CSR position of entries (rows, cols) (the CSR is sorted by row, then column)."""
    r = np.repeat(np.arange(n_nodes, dtype=np.int64), np.diff(rowptr))
    keys = r * n_nodes + colidx
    want = np.asarray(rows, dtype=np.int64) * n_nodes + np.asarray(cols, dtype=np.int64)
    k = np.searchsorted(keys, want)
    assert np.all(keys[k] == want)
    return k


def multiplicity(n_nodes: int, tets, mask, edges):
    """c_t per pattern edge (eq. (1)): for each active tet, +1 on each of its six edges."""
    on = np.asarray(mask).astype(bool)
    c = np.zeros(len(edges), dtype=np.int32)
    np.add.at(c, edge_index(n_nodes, edges, edges_of(tets)[on]).reshape(-1), 1)
    return c


def proxy_rebuild(n_nodes: int, tets, mask, eps: float, pat):
    """(values f64 over the pattern, c_t int32 per edge, degree int32 per node) for mask."""
    rowptr, colidx, edges = pat
    c = multiplicity(n_nodes, tets, mask, edges)
    a = (c > 0).astype(np.int32)                                          # eq. (2)
    deg = np.zeros(n_nodes, dtype=np.int32)
    np.add.at(deg, edges[:, 0], a)
    np.add.at(deg, edges[:, 1], a)                                        # eq. (3), diagonal
    vals = np.zeros(len(colidx), dtype=np.float64)
    act = edges[a == 1]
    vals[entry_index(n_nodes, rowptr, colidx, act[:, 0], act[:, 1])] = -1.0   # eq. (3), off-diagonal
    vals[entry_index(n_nodes, rowptr, colidx, act[:, 1], act[:, 0])] = -1.0
    used = np.unique(np.asarray(tets, dtype=np.int64).reshape(-1))
    vals[entry_index(n_nodes, rowptr, colidx, used, used)] = deg[used].astype(np.float64) + eps  # eq. (4)
    return vals, c, deg


def proxy_dense_bruteforce(n_nodes: int, tets, mask, eps: float):
    """Dense A_t by brute force over vertex pairs: (u,v) is active when some active tet
    holds both u and v; degree = active neighbours.  A route independent of the edge
    list, for tiny meshes only."""
    t = [set(map(int, row)) for row, on in zip(np.asarray(tets), np.asarray(mask)) if on]
    used = set(int(u) for u in np.asarray(tets).reshape(-1))
    A = np.zeros((n_nodes, n_nodes))
    for u in range(n_nodes):
        for v in range(n_nodes):
            if u != v and any(u in s and v in s for s in t):
                A[u, v] = -1.0
    for u in used:
        A[u, u] = float(sum(1 for v in range(n_nodes) if A[u, v] == -1.0)) + eps
    return A
