"""Pins of the connectivity oracle (paper Sec. 3.6; reading: tets sharing a vertex are
connected, components labelled by their smallest vertex id)."""
import numpy as np
import pytest

from oracle import connectivity as C
from paper_2605_11673_amd import workloads as W


def test_closed_forms():
    one = np.array([[0, 1, 2, 3]], np.int32)
    assert C.components(4, one, [1])[1] == 1
    vertex = np.array([[0, 1, 2, 3], [3, 4, 5, 6]], np.int32)     # share vertex 3 only
    lab, k = C.components(7, vertex, [1, 1])
    assert k == 1 and list(lab) == [0, 0]
    apart = np.array([[4, 1, 2, 3], [5, 6, 7, 8]], np.int32)
    lab, k = C.components(9, apart, [1, 1])
    assert k == 2 and list(lab) == [1, 5]
    lab, k = C.components(9, apart, [0, 1])
    assert k == 1 and list(lab) == [-1, 5]
    c = W.make_cube(0, n=5)
    lab, k = C.components(c.n_nodes, c.tets, c.mask0)
    assert k == 1 and np.all(lab == 0)


def test_disjoint_union_of_cubes():
    """A batch of k meshes, all active: k components labelled by each mesh's first node."""
    ws = W.make_batch(seed=1, count=5, sizes=[2, 3, 1, 4, 2])
    off = np.cumsum([0] + [w.n_nodes for w in ws])
    tets = np.concatenate([w.tets + off[j] for j, w in enumerate(ws)])
    lab, k = C.components(int(off[-1]), tets, np.ones(len(tets), np.uint8))
    assert k == 5
    toff = np.cumsum([0] + [w.n_tets for w in ws])
    for j in range(5):
        assert np.all(lab[toff[j]:toff[j + 1]] == off[j])


@pytest.mark.parametrize("seed", range(10))
def test_bfs_agrees_on_random_meshes(seed):
    w = W.random_small_mesh(seed, max_tets=40)
    g = np.random.default_rng(seed)
    mask = (g.uniform(size=w.n_tets) < 0.5).astype(np.uint8)
    lab, k = C.components(w.n_nodes, w.tets, mask)
    by = C.tets_by_node(w.n_nodes, w.tets, mask)
    classes = set()
    for e in np.nonzero(mask)[0]:
        comp = C.bfs_component(w.n_nodes, w.tets, mask, e, by)
        assert {int(f) for f in np.nonzero(lab == lab[e])[0]} == comp
        assert lab[e] == min(int(a) for f in comp for a in w.tets[f])
        classes.add(frozenset(comp))
    assert len(classes) == k and np.all(lab[mask == 0] == -1)


def test_fracture_separates_voronoi_regions():
    """With every straddling tet deleted, no component holds tets of two different sites
    (a straddler is exactly a tet whose vertices lie in different sites' regions)."""
    w = W.make_fracture(seed=0, n=12)
    sites = W.rng(0, W.STREAM_SITES).uniform(size=(32, 3))
    d = ((w.x[:, None, :] - sites[None, :, :]) ** 2).sum(axis=2)
    node_site = np.argmin(d, axis=1)
    tet_site = node_site[w.tets]
    straddle = np.any(tet_site != tet_site[:, :1], axis=1)
    mask = (~straddle).astype(np.uint8)
    lab, k = C.components(w.n_nodes, w.tets, mask)
    for l in np.unique(lab[mask == 1]):
        assert len(np.unique(tet_site[lab == l, 0])) == 1
    assert k >= len(np.unique(tet_site[mask == 1, 0]))


# Face adjacency: tets sharing a face (three vertices) are connected; labels are the
# smallest tet id of the component.

def test_face_closed_forms():
    face = np.array([[0, 1, 2, 3], [1, 2, 3, 4]], np.int32)      # share face 123
    edge = np.array([[0, 1, 2, 3], [2, 3, 4, 5]], np.int32)      # share edge 23 only
    vert = np.array([[0, 1, 2, 3], [3, 4, 5, 6]], np.int32)      # share vertex 3 only
    assert [list(x) for x in C.face_pairs(face)] == [[0, 1]]
    assert len(C.face_pairs(edge)) == 0 and len(C.face_pairs(vert)) == 0
    lab, k = C.face_components(face, [1, 1])
    assert k == 1 and list(lab) == [0, 0]
    lab, k = C.face_components(edge, [1, 1])
    assert k == 2 and list(lab) == [0, 1]
    assert C.components(6, edge, [1, 1])[1] == 1                  # one operator component
    lab, k = C.face_components(vert, [0, 1])
    assert k == 1 and list(lab) == [-1, 1]
    # three candidates on one triple (a superset may overlap): every pair is a face pair
    three = np.array([[0, 1, 2, 3], [1, 2, 3, 4], [5, 3, 2, 1]], np.int32)
    assert [list(x) for x in C.face_pairs(three)] == [[0, 1], [0, 2], [1, 2]]
    lab, k = C.face_components(three, [1, 0, 1])
    assert k == 1 and list(lab) == [0, -1, 0]


@pytest.mark.parametrize("n", [1, 2, 5])
def test_face_pairs_of_the_kuhn_cube(n):
    """Every interior face of the n^3 x 6 Kuhn cube is shared by exactly two tets and every
    boundary face (2 triangles per boundary square, 6 n^2 squares) by one: 2m - 6n^2 pairs;
    all active, the cube is one face-connected component labelled 0."""
    c = W.make_cube(0, n=n)
    p = C.face_pairs(c.tets)
    assert len(p) == 2 * c.n_tets - 6 * n * n
    lab, k = C.face_components(c.tets, c.mask0, p)
    assert k == 1 and np.all(lab == 0)


@pytest.mark.parametrize("seed", range(10))
def test_face_bfs_and_refines_vertex_components(seed):
    """On random meshes and masks: the library components equal the sets a direct
    breadth-first search reaches (neighbours found by comparing vertex sets), the label is
    the smallest tet id, and every face component lies inside one vertex component."""
    w = W.random_small_mesh(seed, max_tets=40)
    g = np.random.default_rng(100 + seed)
    mask = (g.uniform(size=w.n_tets) < 0.6).astype(np.uint8)
    lab, k = C.face_components(w.tets, mask)
    vlab, vk = C.components(w.n_nodes, w.tets, mask)
    by = C.tets_by_node(w.n_nodes, w.tets, mask)
    classes = set()
    for e in np.nonzero(mask)[0]:
        comp = C.bfs_face_component(w.tets, mask, e, by)
        assert {int(f) for f in np.nonzero(lab == lab[e])[0]} == comp
        assert lab[e] == min(comp)
        assert len({int(vlab[f]) for f in comp}) == 1
        classes.add(frozenset(comp))
    assert len(classes) == k and k >= vk and np.all(lab[mask == 0] == -1)


def test_face_components_split_at_hanging_nodes():
    """Refinement superset, coarse n = 2: with one parent swapped for its 8 red children,
    the children are face-connected among themselves but share no face with the
    neighbouring parents (their faces carry edge midpoints): two face components, one
    vertex component."""
    r = W.make_refinement(seed=0, n=2, frames=1)
    mask = r.mask0.copy()
    p = 5
    mask[p] = 0
    kids = 6 * 2 ** 3 + 8 * p + np.arange(8)
    mask[kids] = 1
    lab, k = C.face_components(r.tets, mask)
    assert k == 2 and len(set(lab[kids])) == 1 and lab[kids[0]] == kids[0]
    assert C.components(r.n_nodes, r.tets, mask)[1] == 1
