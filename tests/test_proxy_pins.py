"""Pins of the proxy-operator oracle (paper Sec. 3.1 eqs. (1)-(4), Sec. 3.2 eq. (7)).

Each check fixes the oracle against something other than itself: closed forms
for one and two tetrahedra, counts of the Kuhn triangulation, the zero row
sum of a Laplacian, a brute force over vertex pairs, and the incremental
count rule of eq. (7) run as a separate route over an edit stream.
"""
import math

import numpy as np
import pytest

from oracle import proxy as P
from paper_2605_11673_amd import workloads as W

EPS = W.PROXY_EPS


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float64).view(np.uint64)


def dense(n, pat, vals):
    rowptr, colidx, _ = pat
    A = np.zeros((n, n))
    r = np.repeat(np.arange(n), np.diff(rowptr))
    A[r, colidx] = vals
    return A


def test_single_tet_closed_form():
    """One tet: every edge has multiplicity 1, every vertex degree 3: A = 4I - J + eps I."""
    tets = np.array([[0, 1, 2, 3]], np.int32)
    pat = P.proxy_pattern(4, tets)
    vals, c, deg = P.proxy_rebuild(4, tets, np.ones(1, np.uint8), EPS, pat)
    assert list(map(tuple, pat[2])) == [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    assert np.array_equal(c, np.ones(6)) and np.array_equal(deg, [3, 3, 3, 3])
    want = 4.0 * np.eye(4) - np.ones((4, 4))
    want[np.diag_indices(4)] = 3.0 + EPS
    assert np.array_equal(bits(dense(4, pat, vals)), bits(want))


def test_two_tets_sharing_a_face():
    """Tets (0,1,2,3) and (1,2,3,4) share face {1,2,3}: its three edges have multiplicity
    2, the other six 1; 0 and 4 are not adjacent; degrees 3,4,4,4,3.  Deactivating the
    second tet drops 4's edges to zero (kept as +0.0 entries) and the face edges to 1."""
    tets = np.array([[0, 1, 2, 3], [1, 2, 3, 4]], np.int32)
    pat = P.proxy_pattern(5, tets)
    vals, c, deg = P.proxy_rebuild(5, tets, np.ones(2, np.uint8), EPS, pat)
    cm = {tuple(e): k for e, k in zip(map(tuple, pat[2]), c)}
    assert cm == {(0, 1): 1, (0, 2): 1, (0, 3): 1, (1, 2): 2, (1, 3): 2, (2, 3): 2, (1, 4): 1, (2, 4): 1,
                  (3, 4): 1}
    assert np.array_equal(deg, [3, 4, 4, 4, 3])
    A = dense(5, pat, vals)
    assert A[0, 4] == 0.0 and A[4, 0] == 0.0 and A[1, 4] == -1.0 and A[2, 2] == 4.0 + EPS
    vals2, c2, deg2 = P.proxy_rebuild(5, tets, np.array([1, 0], np.uint8), EPS, pat)
    cm2 = {tuple(e): k for e, k in zip(map(tuple, pat[2]), c2)}
    assert cm2[(1, 2)] == 1 and cm2[(1, 4)] == 0 and np.array_equal(deg2, [3, 3, 3, 3, 0])
    A2 = dense(5, pat, vals2)
    assert A2[4, 4] == EPS and np.signbit(A2[1, 4]) == False and A2[1, 4] == 0.0  # noqa: E712


@pytest.mark.parametrize("n", [1, 2, 4, 7])
def test_kuhn_cube_counts(n):
    """Fully active Kuhn cube of n^3 cells: 3n(n+1)^2 axis + 3n^2(n+1) face-diagonal + n^3
    body-diagonal edges; interior vertices have 14 neighbours; sum of multiplicities =
    6 x active tets; sum of degrees = 2 x active edges."""
    x = W.grid_nodes(n)
    tets = W.kuhn_tets(n)
    pat = P.proxy_pattern(len(x), tets)
    vals, c, deg = P.proxy_rebuild(len(x), tets, np.ones(len(tets), np.uint8), EPS, pat)
    n_edges = 3 * n * (n + 1) ** 2 + 3 * n * n * (n + 1) + n ** 3
    assert len(pat[2]) == n_edges and np.all(c > 0)
    assert int(c.sum()) == 6 * len(tets) and int(deg.sum()) == 2 * n_edges
    ijk = np.stack(np.unravel_index(np.arange(len(x)), (n + 1,) * 3), axis=1)
    interior = np.all((ijk > 0) & (ijk < n), axis=1)
    assert interior.sum() == (n - 1) ** 3 and np.all(deg[interior] == 14)


def test_full_size_structural_counts():
    """40^3 cube: 462,520 edges and a scalar pattern of 68,921 + 2 x 462,520 entries."""
    w = W.make_fracture(seed=0)
    pat = P.proxy_pattern(w.n_nodes, w.tets)
    assert len(pat[2]) == 462520 and len(pat[1]) == 68921 + 2 * 462520


@pytest.mark.parametrize("seed", range(12))
def test_bruteforce_and_laplacian_properties(seed):
    """Random tiny meshes and masks: CSR values bitwise equal to the pair brute force
    (absent and inactive entries +0.0), symmetric, rows summing to eps."""
    w = W.random_small_mesh(seed)
    pat = P.proxy_pattern(w.n_nodes, w.tets)
    vals, c, deg = P.proxy_rebuild(w.n_nodes, w.tets, w.mask0, EPS, pat)
    A = dense(w.n_nodes, pat, vals)
    assert np.array_equal(bits(A), bits(P.proxy_dense_bruteforce(w.n_nodes, w.tets, w.mask0, EPS)))
    assert np.array_equal(bits(A), bits(A.T))
    used = np.unique(w.tets)
    for u in used:
        assert abs(math.fsum(A[u]) - EPS) <= 8 * 2.0 ** -52
    assert np.array_equal(deg[used], (A[used] == -1.0).sum(axis=1))


def test_incremental_rule_matches_rebuild():
    """eq. (7) as its own route: counts updated by +1/-1 per edge of each added/deleted tet,
    and entries flipped on 0 <-> >0 transitions, equal the rebuild at every frame of a
    fracture stream and of its reinsertion."""
    w = W.make_fracture(seed=2, n=6, counts=[5, 12, 30, 7])
    pat = P.proxy_pattern(w.n_nodes, w.tets)
    frames = list(w.frames) + W.merge_stream(w.frames)
    mask = w.mask0.copy()
    _, c, deg = P.proxy_rebuild(w.n_nodes, w.tets, mask, EPS, pat)
    c, deg = c.astype(np.int64), deg.astype(np.int64)
    ek = P.edge_index(w.n_nodes, pat[2], P.edges_of(w.tets))
    for ids, st in frames:
        for tid, s in zip(ids, st):
            if mask[tid] == s:
                continue
            mask[tid] = s
            d = 1 if s else -1
            for k in ek[tid]:
                before = c[k]
                c[k] += d
                if (before == 0) != (c[k] == 0):  # transition: both endpoint degrees move
                    u, v = pat[2][k]
                    deg[u] += d
                    deg[v] += d
        _, c_ref, deg_ref = P.proxy_rebuild(w.n_nodes, w.tets, mask, EPS, pat)
        assert np.array_equal(c, c_ref) and np.array_equal(deg, deg_ref)
