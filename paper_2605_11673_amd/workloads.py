"""Seeded synthetic workloads for exact streaming assembly on a superset tet mesh.

This module only produces inputs: superset meshes (node positions, candidate
tetrahedra), per-element Young's moduli, initial active masks, per-frame edit
streams and load vectors.  It holds none of the assembly arithmetic (no
element matrices, no volumes, no reductions), so both the CPU oracle and the
GPU path can draw from it without sharing any of the method's code.

The paper evaluates on scanned tetrahedral models (Bunny, Gargoyle, Hand) that
are not available here.  Structured Kuhn (Freudenthal) cubes of matching scale
stand in for them; the three edit scenarios follow the paper's experimental
setup (Sec. 5.1): fracture deletes candidate elements along precomputed cut
surfaces, refinement swaps parents for preallocated children, merge reinserts.

Random streams: every draw comes from ``numpy.random.SeedSequence([seed,
stream, *extra])`` so each quantity can be regenerated independently.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

STREAM_JITTER = 1
STREAM_LOGE = 2
STREAM_SITES = 3
STREAM_IMPACT = 4
STREAM_EDITS = 5
STREAM_LOADS = 6
STREAM_FD = 7
STREAM_BATCH = 8

NU = 0.3
RHO = 1000.0
DT = 1e-2
E_MEDIAN = 1e5
LOGE_SIGMA = 0.5
# Diagonal shift of the proxy system A_t = L_t + eps I; the paper asks only for a
# small positive value.
PROXY_EPS = 1e-6

# Permutations of the three axes in lexicographic order; tet p of a cell walks
# from the cell origin along axes PERMS[p][0], PERMS[p][1], PERMS[p][2].
PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


def rng(seed: int, stream: int, *extra: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, stream, *extra])))


Frame = Tuple[np.ndarray, np.ndarray]  # (ids int32, new states uint8)


@dataclass
class Workload:
    """A superset mesh, its material, its initial mask and an edit stream."""
    name: str
    x: np.ndarray            # (n, 3) float64 node positions
    tets: np.ndarray         # (m, 4) int32 candidate tetrahedra
    E: np.ndarray            # (m,) float64 Young's modulus per candidate
    mask0: np.ndarray        # (m,) uint8 initial active mask
    frames: List[Frame] = field(default_factory=list)
    nu: float = NU
    rho: float = RHO
    dt: float = DT
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_tets(self) -> int:
        return int(self.tets.shape[0])

    def mask_after(self, t: int) -> np.ndarray:
        """Active mask after applying frames 0..t inclusive (t = -1: initial)."""
        mask = self.mask0.copy()
        for ids, st in self.frames[: t + 1]:
            mask[ids] = st
        return mask


# ----------------------------------------------------------------------------
# Mesh construction
# ----------------------------------------------------------------------------

def grid_nodes(n: int) -> np.ndarray:
    """Integer lattice coordinates of the (n+1)^3 nodes; node (i,j,k) has id (i(n+1)+j)(n+1)+k."""
    idx = np.arange(n + 1)
    I, J, K = np.meshgrid(idx, idx, idx, indexing="ij")
    return np.stack([I, J, K], -1).reshape(-1, 3)


def kuhn_tets(n: int) -> np.ndarray:
    """Kuhn 6-tet split of an n^3 cell grid.

    Cell c = (ci*n + cj)*n + ck owns tets 6c..6c+5; tet 6c+p has vertices
    v0 = cell origin, v1 = v0 + e_{P[0]}, v2 = v1 + e_{P[1]}, v3 = v2 + e_{P[2]}
    with P = PERMS[p].  The split is conforming across cells.
    """
    N = n + 1
    idx = np.arange(n)
    ci, cj, ck = np.meshgrid(idx, idx, idx, indexing="ij")
    origin = np.stack([ci, cj, ck], -1).reshape(-1, 3)
    tets = np.empty((origin.shape[0], 6, 4), dtype=np.int64)
    for p, perm in enumerate(PERMS):
        v = origin.copy()
        tets[:, p, 0] = (v[:, 0] * N + v[:, 1]) * N + v[:, 2]
        for r, axis in enumerate(perm):
            v = v.copy()
            v[:, axis] += 1
            tets[:, p, r + 1] = (v[:, 0] * N + v[:, 1]) * N + v[:, 2]
    return tets.reshape(-1, 4).astype(np.int32)


def jittered_nodes(n: int, jitter: float, g: np.random.Generator | None) -> np.ndarray:
    """Lattice nodes at spacing h = 1/n, each coordinate moved by U(-jitter*h, +jitter*h)."""
    x = grid_nodes(n).astype(np.float64) / n
    if jitter > 0.0:
        h = 1.0 / n
        x = x + g.uniform(-jitter * h, jitter * h, size=x.shape)
    return x


def lognormal_E(count: int, g: np.random.Generator) -> np.ndarray:
    """E = exp(ln(1e5) + 0.5 z), evaluated once on the host and shared as data."""
    logE = np.log(E_MEDIAN) + LOGE_SIGMA * g.standard_normal(count)
    return np.exp(logE)


# ----------------------------------------------------------------------------
# Edit streams
# ----------------------------------------------------------------------------

def fracture_counts(frames: int = 24, peak: int = 12, base: float = 50.0, ratio: float = 40.0) -> List[int]:
    """Per-frame deletion counts n_t = round(50 * 40^(1 - |t - 12| / 12))."""
    return [int(np.round(base * ratio ** (1.0 - abs(t - peak) / peak))) for t in range(frames)]


def voronoi_straddlers(x: np.ndarray, tets: np.ndarray, sites: np.ndarray) -> np.ndarray:
    """Ids of tets whose four vertices are not all nearest to the same site.

    Node label = index of the nearest site (ties go to the lower index).
    """
    d2 = ((x[:, None, :] - sites[None, :, :]) ** 2).sum(-1)
    label = np.argmin(d2, axis=1)
    lt = label[tets]
    straddle = ~((lt[:, 0] == lt[:, 1]) & (lt[:, 0] == lt[:, 2]) & (lt[:, 0] == lt[:, 3]))
    return np.nonzero(straddle)[0]


def fracture_stream(x, tets, seed, counts, extra=()):
    """Delete Voronoi-face straddlers in order of distance from a seeded impact point."""
    sites = rng(seed, STREAM_SITES, *extra).uniform(0.0, 1.0, size=(32, 3))
    impact = rng(seed, STREAM_IMPACT, *extra).uniform(0.0, 1.0, size=3)
    cand = voronoi_straddlers(x, tets, sites)
    centroid = x[tets[cand]].mean(axis=1)
    dist = ((centroid - impact) ** 2).sum(-1)
    order = cand[np.lexsort((cand, dist))]  # by distance, ties by id
    frames: List[Frame] = []
    pos = 0
    for c in counts:
        ids = order[pos: pos + c].astype(np.int32)
        pos += len(ids)
        frames.append((ids, np.zeros(len(ids), dtype=np.uint8)))
    return frames, {"straddlers": int(len(cand)), "sites": sites, "impact": impact}


def merge_stream(fracture: List[Frame]) -> List[Frame]:
    """Reinsert what a fracture stream deleted, frames in reverse order."""
    return [(ids.copy(), np.ones(len(ids), dtype=np.uint8)) for ids, _ in reversed(fracture)]


# ----------------------------------------------------------------------------
# The five workloads
# ----------------------------------------------------------------------------

def make_cube(seed: int = 0, n: int = 4, frames: int = 24) -> Workload:
    """Unjittered n^3 x 6 cube, E = 1e5; each frame deletes 1-8 random active tets."""
    x = jittered_nodes(n, 0.0, None)
    tets = kuhn_tets(n)
    m = tets.shape[0]
    E = np.full(m, E_MEDIAN)
    mask0 = np.ones(m, dtype=np.uint8)
    g = rng(seed, STREAM_EDITS)
    active = mask0.astype(bool).copy()
    out: List[Frame] = []
    for _ in range(frames):
        k = int(g.integers(1, 9))
        pool = np.nonzero(active)[0]
        k = min(k, len(pool))
        ids = np.sort(g.choice(pool, size=k, replace=False)).astype(np.int32)
        active[ids] = False
        out.append((ids, np.zeros(k, dtype=np.uint8)))
    return Workload(f"cube{n}", x, tets, E, mask0, out, meta={"n": n, "seed": seed})


def make_fracture(seed: int = 0, n: int = 40, frames: int = 24, counts=None) -> Workload:
    """Jittered n^3 x 6 cube with lognormal E and a Voronoi fracture stream."""
    x = jittered_nodes(n, 0.2, rng(seed, STREAM_JITTER))
    tets = kuhn_tets(n)
    m = tets.shape[0]
    E = lognormal_E(m, rng(seed, STREAM_LOGE))
    mask0 = np.ones(m, dtype=np.uint8)
    if counts is None:
        counts = fracture_counts(frames)
    fr, info = fracture_stream(x, tets, seed, counts)
    return Workload(f"fracture{n}", x, tets, E, mask0, fr,
                    meta={"n": n, "seed": seed, "counts": list(counts), **info})


def red_children(parent: np.ndarray, mid) -> np.ndarray:
    """Eight red-refinement children of tet (v0,v1,v2,v3); mid(a,b) gives the edge-midpoint node id.

    Four corner tets, and the inner octahedron split on its m02-m13 diagonal.
    """
    v0, v1, v2, v3 = parent
    m01, m02, m03 = mid(v0, v1), mid(v0, v2), mid(v0, v3)
    m12, m13, m23 = mid(v1, v2), mid(v1, v3), mid(v2, v3)
    return np.array([
        (v0, m01, m02, m03), (v1, m01, m12, m13), (v2, m02, m12, m23), (v3, m03, m13, m23),
        (m01, m02, m03, m13), (m01, m02, m12, m13), (m02, m03, m13, m23), (m02, m12, m13, m23),
    ])


def make_refinement(seed: int = 0, n: int = 20, frames: int = 24) -> Workload:
    """Coarse n^3 x 6 parents, each with 8 preallocated red children on the 2n lattice.

    Node ids are those of the (2n+1)^3 fine lattice; coarse corner nodes are
    jittered by U(-0.2H, 0.2H) (H = 1/n) and every edge-midpoint node sits at
    the exact midpoint of its jittered coarse edge.  Ids: parents 0..6n^3-1,
    child c of parent p is 6n^3 + 8p + c.  Parents start active.  The stream
    holds ``frames`` refine frames followed by ``frames`` merge frames.
    """
    Nf = 2 * n + 1
    fine = grid_nodes(2 * n)
    xc = jittered_nodes(n, 0.2, rng(seed, STREAM_JITTER))
    coarse_id = lambda I: (I[..., 0] * (n + 1) + I[..., 1]) * (n + 1) + I[..., 2]
    lo = fine // 2
    hi = (fine + 1) // 2
    x = 0.5 * (xc[coarse_id(lo)] + xc[coarse_id(hi)])
    even = np.all(fine % 2 == 0, axis=1)
    x[even] = xc[coarse_id(lo[even])]  # exact copy for corner nodes

    parents_c = kuhn_tets(n)
    cN = n + 1
    cI = np.stack([parents_c // (cN * cN), (parents_c // cN) % cN, parents_c % cN], -1)  # (P,4,3)
    parents = ((2 * cI[..., 0]) * Nf + 2 * cI[..., 1]) * Nf + 2 * cI[..., 2]
    # midpoint of fine vertices a, b (both on the even sublattice): fine index (a + b) / 2
    fI = np.stack([parents // (Nf * Nf), (parents // Nf) % Nf, parents % Nf], -1)
    P = parents.shape[0]
    pairs = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    mids = {}
    for a, b in pairs:
        mI = (fI[:, a] + fI[:, b]) // 2
        mids[(a, b)] = (mI[:, 0] * Nf + mI[:, 1]) * Nf + mI[:, 2]
    v = [parents[:, k] for k in range(4)]
    m = lambda a, b: mids[(a, b)]
    children = np.stack([
        np.stack([v[0], m(0, 1), m(0, 2), m(0, 3)], -1),
        np.stack([v[1], m(0, 1), m(1, 2), m(1, 3)], -1),
        np.stack([v[2], m(0, 2), m(1, 2), m(2, 3)], -1),
        np.stack([v[3], m(0, 3), m(1, 3), m(2, 3)], -1),
        np.stack([m(0, 1), m(0, 2), m(0, 3), m(1, 3)], -1),
        np.stack([m(0, 1), m(0, 2), m(1, 2), m(1, 3)], -1),
        np.stack([m(0, 2), m(0, 3), m(1, 3), m(2, 3)], -1),
        np.stack([m(0, 2), m(1, 2), m(1, 3), m(2, 3)], -1),
    ], 1).reshape(-1, 4)
    tets = np.concatenate([parents, children]).astype(np.int32)
    Ep = lognormal_E(P, rng(seed, STREAM_LOGE))
    E = np.concatenate([Ep, np.repeat(Ep, 8)])
    mask0 = np.zeros(tets.shape[0], dtype=np.uint8)
    mask0[:P] = 1

    g = rng(seed, STREAM_EDITS)
    refined = np.zeros(P, dtype=bool)
    out: List[Frame] = []
    kinds: List[str] = []
    for phase in ("refine", "merge"):
        for _ in range(frames):
            r = float(np.exp(g.uniform(np.log(1e-3), np.log(2e-2))))
            k = int(np.round(P * r))
            pool = np.nonzero(~refined if phase == "refine" else refined)[0]
            k = min(k, len(pool))
            pick = np.sort(g.choice(pool, size=k, replace=False))
            refined[pick] = phase == "refine"
            kid = (P + 8 * pick[:, None] + np.arange(8)[None, :]).reshape(-1)
            ids = np.concatenate([pick, kid]).astype(np.int32)
            pstate = 0 if phase == "refine" else 1
            st = np.concatenate([np.full(k, pstate), np.full(8 * k, 1 - pstate)]).astype(np.uint8)
            out.append((ids, st))
            kinds.append(phase)
    return Workload(f"refine{n}", x, tets, E, mask0, out,
                    meta={"n": n, "seed": seed, "parents": P, "kinds": kinds})


def loads_for(w: Workload, mask: np.ndarray, seed: int = 0) -> np.ndarray:
    """Load vector for a compliance objective on the active mesh.

    Gravity: node i gets (0, 0, -9.81) * rho * c_i * h^3 / 24 with c_i the
    number of active tets holding node i (h^3/24 is a quarter of the mean
    Kuhn-tet volume).  Surface load: every vertex of a face owned by exactly
    one active tet gets sigma * N(0, I3), sigma = 10 * mean gravity magnitude.
    Nodes with no active tet get zero load.
    """
    n = w.n_nodes
    h = 1.0 / w.meta.get("n", 1)
    act = w.tets[mask.astype(bool)]
    count = np.bincount(act.reshape(-1), minlength=n).astype(np.float64)
    f = np.zeros((n, 3))
    f[:, 2] = -9.81 * w.rho * count * (h ** 3) / 24.0
    faces = np.concatenate([act[:, [1, 2, 3]], act[:, [0, 2, 3]], act[:, [0, 1, 3]], act[:, [0, 1, 2]]])
    faces = np.sort(faces, axis=1)
    uf, cnt = np.unique(faces, axis=0, return_counts=True)
    surf = np.unique(uf[cnt == 1].reshape(-1))
    used = count > 0
    sigma = 10.0 * float(np.abs(f[used, 2]).mean()) if used.any() else 0.0
    g = rng(seed, STREAM_LOADS)
    f[surf] += sigma * g.standard_normal((len(surf), 3))
    return f


def make_gradient_case(seed: int = 0, n: int = 40, frame: int = 12, n_samples: int = 20):
    """Fracture state after frames 0..frame, its load vector and a seeded FD sample."""
    w = make_fracture(seed, n)
    mask = w.mask_after(frame)
    f = loads_for(w, mask, seed)
    g = rng(seed, STREAM_FD)
    active = np.nonzero(mask)[0]
    tet_sample = np.sort(g.choice(active, size=min(n_samples, len(active)), replace=False))
    used = np.unique(w.tets[mask.astype(bool)].reshape(-1))
    node_sample = np.sort(g.choice(used, size=min(n_samples, len(used)), replace=False))
    return w, mask, f, tet_sample.astype(np.int64), node_sample.astype(np.int64)


def batch_sizes(seed: int = 0, count: int = 64, lo: float = 1e3, hi: float = 1.2e5) -> List[int]:
    """Cells per side n_j = round(cbrt(T_j / 6)), T_j log-uniform in [lo, hi]."""
    g = rng(seed, STREAM_BATCH)
    T = np.exp(g.uniform(np.log(lo), np.log(hi), size=count))
    return [max(1, int(np.round(np.cbrt(t / 6.0)))) for t in T]


def make_batch(seed: int = 0, count: int = 64, frames: int = 24, sizes=None) -> List[Workload]:
    """Independent jittered cubes of uneven size, each with its own fracture stream.

    Mesh j draws its jitter, E, sites and impact point from streams extended by
    j, and deletes max(1, round(n_t * m_j / 384000)) straddlers in frame t.
    """
    if sizes is None:
        sizes = batch_sizes(seed, count)
    base = fracture_counts(frames)
    out = []
    for j, nj in enumerate(sizes):
        x = jittered_nodes(nj, 0.2, rng(seed, STREAM_JITTER, j))
        tets = kuhn_tets(nj)
        m = tets.shape[0]
        E = lognormal_E(m, rng(seed, STREAM_LOGE, j))
        counts = [max(1, int(np.round(c * m / 384000.0))) for c in base]
        fr, info = fracture_stream(x, tets, seed, counts, extra=(j,))
        out.append(Workload(f"batch{j}_n{nj}", x, tets, E, np.ones(m, dtype=np.uint8), fr,
                            meta={"n": nj, "seed": seed, "index": j, **info}))
    return out


def random_small_mesh(seed: int, max_tets: int = 12) -> Workload:
    """A tiny random mesh for brute-force checks: a jittered 1^3 or 2^3 Kuhn cube,
    a random subset of its tets (at most ``max_tets``), relabelled nodes in random
    order, random vertex order inside each tet, random E and a random mask."""
    g = rng(seed, 99)
    n = int(g.integers(1, 3))
    x = jittered_nodes(n, 0.15, g)
    tets = kuhn_tets(n)
    k = int(g.integers(1, min(max_tets, len(tets)) + 1))
    tets = tets[np.sort(g.choice(len(tets), size=k, replace=False))]
    perm = g.permutation(x.shape[0])
    inv = np.empty_like(perm)
    inv[perm] = np.arange(len(perm))
    x = x[perm]
    tets = inv[tets]
    tets = np.array([t[g.permutation(4)] for t in tets], dtype=np.int32)
    E = np.exp(np.log(E_MEDIAN) + 0.5 * g.standard_normal(k))
    mask = (g.uniform(size=k) < 0.7).astype(np.uint8)
    return Workload(f"small{seed}", x, tets, E, mask, [], meta={"n": n, "seed": seed})
