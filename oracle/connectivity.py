"""Connectivity of the active tetrahedra (oracle side, TEST INFRASTRUCTURE ONLY).

The paper tracks tetrahedron connectivity under the edit stream, rebuilt
periodically from the active mask and spot-checked by sampled breadth-first
searches (Sec. 3.6; Alg. 1 keeps it with the mask).  It does not say when two
tetrahedra count as connected, so two adjacencies are provided:

* vertex: two active tets are connected when they share a vertex, i.e. the
  components are those of the assembled operator (tets that share a vertex
  share its degrees of freedom); this also joins the two sides of a
  hanging-node interface in the refinement superset.  A component is labelled
  by the smallest vertex id it contains.
* face: two active tets are connected when they share a face (the same three
  vertices), the usual notion of a fragment in fracture: pieces that touch
  only along an edge or at a vertex are apart.  A component is labelled by
  the smallest tet id it contains.

Labels do not depend on the order in which an algorithm discovers the
components.
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


def face_pairs(tets):
    """All pairs (e, f), e < f, of candidate tets with a common face: the four
    vertex triples of every tet, sorted, grouped by equal triples (a library sort)."""
    t = np.sort(np.asarray(tets, dtype=np.int64), axis=1)
    m = len(t)
    tri = np.concatenate([np.delete(t, a, axis=1) for a in range(4)])  # 4m sorted triples
    owner = np.tile(np.arange(m, dtype=np.int64), 4)
    order = np.lexsort((owner, tri[:, 2], tri[:, 1], tri[:, 0]))
    tri, owner = tri[order], owner[order]
    if len(tri) == 0:
        return np.zeros((0, 2), dtype=np.int64)
    same = np.all(tri[1:] == tri[:-1], axis=1)
    start = np.concatenate([[0], np.nonzero(~same)[0] + 1])
    length = np.diff(np.concatenate([start, [len(tri)]]))
    two = start[length == 2]
    pairs = [np.stack([owner[two], owner[two + 1]], axis=1)]
    for i, k in zip(start[length > 2], length[length > 2]):  # more than two tets on one triple
        g = owner[i:i + k]
        pairs.append(np.array([(g[u], g[v]) for u in range(k) for v in range(u + 1, k)], dtype=np.int64))
    p = np.concatenate(pairs).reshape(-1, 2)
    p = np.sort(p, axis=1)
    return np.unique(p, axis=0)


def face_components(tets, mask, pairs=None):
    """Per-tet label (smallest tet id of its face-connected component; -1 for inactive
    tets) and the number of components (library connected_components on the graph
    whose edges are the face pairs with both tets active)."""
    on = np.asarray(mask).astype(bool)
    m = len(on)
    if pairs is None:
        pairs = face_pairs(tets)
    p = pairs[on[pairs[:, 0]] & on[pairs[:, 1]]] if len(pairs) else pairs
    g = sp.coo_matrix((np.ones(len(p)), (p[:, 0], p[:, 1])), shape=(m, m))
    _, comp = connected_components(g, directed=False)
    ids = np.nonzero(on)[0]
    smallest = np.full(comp.max() + 1 if m else 0, np.iinfo(np.int64).max)
    np.minimum.at(smallest, comp[ids], ids)
    label = np.full(m, -1, dtype=np.int64)
    label[on] = smallest[comp[ids]]
    return label, int(len(np.unique(label[on])))


def bfs_face_component(tets, mask, start: int, by_node=None):
    """The set of active tets reachable from active tet `start` through shared faces:
    breadth-first search where the neighbours across each face of a tet are the tets
    that hold all three of its vertices (intersections of the per-vertex tet lists),
    without the sorted-triple grouping of face_pairs.
    by_node: tets_by_node of the same mask, if already built."""
    t = np.asarray(tets, dtype=np.int64)
    if by_node is None:
        by_node = tets_by_node(int(t.max()) + 1 if len(t) else 0, tets, mask)
    sets = {}

    def around(a):
        if a not in sets:
            sets[a] = set(by_node[a])
        return sets[a]

    seen = {int(start)}
    q = deque([int(start)])
    while q:
        e = q.popleft()
        v = [int(a) for a in t[e]]
        for skip in range(4):  # the tets holding all three vertices of each face of e
            a, b, c = [v[i] for i in range(4) if i != skip]
            for f in around(a) & around(b) & around(c):
                if f not in seen:
                    seen.add(f)
                    q.append(f)
    return seen
