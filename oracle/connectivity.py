"""Connectivity of the active tetrahedra (oracle side, TEST INFRASTRUCTURE ONLY).

The paper tracks tetrahedron connectivity under the edit stream, rebuilt
periodically from the active mask and spot-checked by sampled breadth-first
searches (Sec. 3.6; Alg. 1 keeps it with the mask).  It does not say when two
tetrahedra count as connected.  Reading used here: two active tets are
connected when they share a vertex, i.e. the components are those of the
assembled operator (tets that share a vertex share its degrees of freedom);
this also joins the two sides of a hanging-node interface in the refinement
superset.  A component is labelled by the smallest vertex id it contains, so
labels do not depend on the order in which an algorithm discovers them.
"""
from collections import deque

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components


def components(n_nodes: int, tets, mask):
    """Per-tet label (smallest vertex id of its component; -1 for inactive tets) and the
    number of components, from the vertex graph of the active tets (library routine)."""
    t = np.asarray(tets, dtype=np.int64)
    on = np.asarray(mask).astype(bool)
    act = t[on]
    rows = np.repeat(act[:, 0], 3)
    cols = act[:, 1:].reshape(-1)
    g = sp.coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(n_nodes, n_nodes))
    _, comp = connected_components(g, directed=False)
    smallest = np.full(comp.max() + 1 if n_nodes else 0, np.iinfo(np.int64).max)
    used = np.unique(act.reshape(-1))
    np.minimum.at(smallest, comp[used], used)
    label = np.full(len(t), -1, dtype=np.int64)
    label[on] = smallest[comp[act[:, 0]]]
    return label, int(len(np.unique(label[on])))


def tets_by_node(n_nodes: int, tets, mask):
    """For each vertex, the active tets that contain it."""
    t = np.asarray(tets, dtype=np.int64)
    by_node = [[] for _ in range(n_nodes)]
    for e in np.nonzero(np.asarray(mask).astype(bool))[0]:
        for a in t[e]:
            by_node[a].append(int(e))
    return by_node


def bfs_component(n_nodes: int, tets, mask, start: int, by_node=None):
    """The set of active tets reachable from active tet `start` through shared vertices
    (plain breadth-first search over tets, the paper's spot check)."""
    t = np.asarray(tets, dtype=np.int64)
    if by_node is None:
        by_node = tets_by_node(n_nodes, tets, mask)
    seen = {int(start)}
    q = deque([int(start)])
    while q:
        e = q.popleft()
        for a in t[e]:
            for f in by_node[a]:
                if f not in seen:
                    seen.add(f)
                    q.append(f)
    return seen
