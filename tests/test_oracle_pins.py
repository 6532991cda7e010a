"""Pins for the CPU oracle: closed forms, an independent exact formula,
physical invariants and brute force.  Each test names the mistake it catches.

The paper prints no matrix values (its only parity figure is a tolerance,
Sec. 6.1), so every pin comes from mathematics the paper relies on: the
element-assembled operator of Sec. 3.4 eq. (8) with the standard linear
tetrahedron elasticity matrix, the lumped mass of Sec. 6.2 eq. (9), and the
rebuild invariant of Sec. 3.3.
"""
from fractions import Fraction as F
import math

import numpy as np
import pytest

import oracle
from paper_2605_11673_amd import workloads as W
from tests.exact import exact_dense, voigt_element

EPS = np.finfo(np.float64).eps
NU, RHO, DT = 0.3, 1000.0, 1e-2


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float64).view(np.uint64)


# ---------------------------------------------------------------------------
# Element matrix
# ---------------------------------------------------------------------------

def closed_form_reference_tet(E, nu, rho, dt):
    """Textbook closed form for the reference tet (0, e1, e2, e3): V = 1/6,
    g0 = -(1,1,1), g_a = e_a.  Blocks (exact rationals):
      K00 = V[(lam+mu) J + 3 mu I],   Kaa = V[(lam+mu) e_a e_a^T + mu I]
      K0a = -V[lam 1 e_a^T + mu e_a 1^T + mu I]   (and K_a0 = K0a^T)
      Kab = V[lam e_a e_b^T + mu e_b e_a^T]  (a != b >= 1)
    plus rho V / 4 = rho/24 on the diagonal.  nu is the exact binary64 value."""
    E, nu, rho, dt = F(E), F(nu), F(rho), F(dt)
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    V = F(1, 6)
    I = lambda i, j: F(int(i == j))
    e = lambda a, i: F(int(a == i + 1))  # e_a for a = 1..3, component i
    K = [[F(0)] * 12 for _ in range(12)]
    for a in range(4):
        for b in range(4):
            for i in range(3):
                for j in range(3):
                    if a == 0 and b == 0:
                        v = (lam + mu) + 3 * mu * I(i, j)
                    elif a == 0:
                        v = -(lam * e(b, j) + mu * e(b, i) + mu * I(i, j))
                    elif b == 0:
                        v = -(lam * e(a, i) + mu * e(a, j) + mu * I(i, j))
                    elif a == b:
                        v = (lam + mu) * e(a, i) * e(a, j) + mu * I(i, j)
                    else:
                        v = lam * e(a, i) * e(b, j) + mu * e(b, i) * e(a, j)
                    K[3 * a + i][3 * b + j] = V * v
    A = [[dt * dt * K[r][c] + (rho / 24 if r == c else 0) for c in range(12)] for r in range(12)]
    return A


def assert_close_exact(A, Ex, rel):
    Ex_f = np.array([[float(v) for v in row] for row in Ex])
    scale = np.abs(Ex_f).max()
    err = np.abs(A - Ex_f)
    assert err.max() <= rel * scale, (err.max(), scale)


@pytest.mark.parametrize("E", [1e5, 3.7e4])
def test_reference_tet_closed_form(E):
    """Catches: a dropped lambda/mu/mass term, a wrong sign on g0, transposed g_a g_b^T."""
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.float64)
    A = oracle.element_matrix(X, E, NU, RHO, DT)
    Ex = closed_form_reference_tet(E, NU, RHO, DT)
    Ex_f = np.array([[float(v) for v in row] for row in Ex])
    # no cancellation in this tet: every entry is a same-signed sum, so each
    # entry is within a few ulp of its exact value; exact zeros stay zero
    zero = Ex_f == 0.0
    assert np.all(A[zero] == 0.0)
    rel = np.abs(A[~zero] - Ex_f[~zero]) / np.abs(Ex_f[~zero])
    assert rel.max() <= 8 * EPS


def dyadic_tet(g):
    """A random non-degenerate tet with coordinates k / 64 (exact in binary)."""
    while True:
        P = g.integers(-64, 65, size=(4, 3))
        M = (P[1:] - P[0]).T
        if abs(round(np.linalg.det(M))) >= 200:
            return P / 64.0


@pytest.mark.parametrize("seed", range(6))
def test_general_tet_against_voigt(seed):
    """Independent formula: K = V B^T D B (Voigt, engineering shear) in exact rationals.
    Catches any term, sign or index error in the gradient-outer-product form on a
    general tet (including negative orientation, where V must use |det|)."""
    g = np.random.default_rng(100 + seed)
    X = dyadic_tet(g)
    if seed % 2:
        X = X[[0, 2, 1, 3]]  # flip orientation
    E = float(np.exp(np.log(1e5) + 0.5 * g.standard_normal()))
    A = oracle.element_matrix(X, E, NU, RHO, DT)
    Ex = voigt_element([[F(float(v)) for v in row] for row in X], E, NU, RHO, DT)
    assert_close_exact(A, Ex, 1e-13)


def test_element_bitwise_symmetric():
    """The fixed op order makes A_e[r][c] and A_e[c][r] the same bits (IEEE * is commutative)."""
    g = np.random.default_rng(7)
    for _ in range(50):
        X = g.uniform(size=(4, 3))
        A = oracle.element_matrix(X, 1e5 * g.uniform(0.5, 2), NU, RHO, DT)
        assert np.array_equal(bits(A), bits(A.T))


def test_rigid_modes_annihilated():
    """rho = 0, dt = 1 gives A = K; K kills the 3 translations and 3 rotations."""
    g = np.random.default_rng(3)
    for _ in range(20):
        X = g.uniform(size=(4, 3))
        K = oracle.element_matrix(X, 1e5, NU, 0.0, 1.0)
        c = X.mean(0)
        modes = []
        for k in range(3):
            t = np.zeros((4, 3))
            t[:, k] = 1.0
            modes.append(t.reshape(-1))
        for k in range(3):
            w = np.zeros(3)
            w[k] = 1.0
            modes.append(np.cross(w, X - c).reshape(-1))
        for t in modes:
            r = K @ t
            assert np.abs(r).max() <= 1e-12 * np.abs(K).max() * np.abs(t).max()


def test_positive_semidefinite():
    g = np.random.default_rng(4)
    for _ in range(20):
        X = g.uniform(size=(4, 3))
        K = oracle.element_matrix(X, 1e5, NU, 0.0, 1.0)
        ev = np.linalg.eigvalsh(K)
        assert ev.min() >= -1e-12 * ev.max()
        assert np.sum(ev > 1e-9 * ev.max()) == 6  # 12 dofs - 6 rigid modes


def test_lumped_mass_total():
    """E = 0 leaves A = M: diagonal, each dof of each vertex rho V / 4; total = rho * volume.
    V checked against numpy's determinant (an independent routine)."""
    w = W.make_fracture(seed=1, n=3)
    E0 = np.zeros(w.n_tets)
    pat = oracle.pattern(w.n_nodes, w.tets)
    mask = (np.arange(w.n_tets) % 3 != 0).astype(np.uint8)
    vals = oracle.rebuild(w.x, w.tets, E0, NU, RHO, DT, mask, *pat)
    D = oracle.csr_to_dense(pat[0], pat[1], vals, 3 * w.n_nodes)
    assert np.count_nonzero(D - np.diag(np.diag(D))) == 0
    X = w.x[w.tets]
    V = np.abs(np.linalg.det(X[:, 1:] - X[:, :1])) / 6.0
    total = RHO * V[mask.astype(bool)].sum()
    assert abs(np.trace(D) / 3.0 - total) <= 1e-13 * total
    # unjittered unit cube, all active: total mass is exactly rho * 1
    c = W.make_cube(0, n=2)
    pc = oracle.pattern(c.n_nodes, c.tets)
    vc = oracle.rebuild(c.x, c.tets, np.zeros(c.n_tets), NU, RHO, DT, c.mask0, *pc)
    Dc = oracle.csr_to_dense(pc[0], pc[1], vc, 3 * c.n_nodes)
    assert abs(np.trace(Dc) / 3.0 - RHO) <= 1e-13 * RHO


def test_element_derivatives_complex_step_vs_exact_difference():
    """Complex-step derivatives against an exact-rational central difference of the
    Voigt element (A is rational in x, so the difference is accurate to O(h^2))."""
    g = np.random.default_rng(11)
    X = dyadic_tet(g)
    E = 1.3e5
    D = oracle.element_derivs(X, E, NU, RHO, DT)
    # d/dlogE = dt^2 K (the mass does not depend on E)
    K = oracle.element_matrix(X, E, NU, 0.0, DT)
    assert np.abs(D[0] - K).max() <= 1e-13 * np.abs(K).max()
    Xf = [[F(float(v)) for v in row] for row in X]
    h = F(1, 2 ** 24)
    for k in (0, 4, 8, 11):
        a, i = divmod(k, 3)
        Xp = [row[:] for row in Xf]
        Xm = [row[:] for row in Xf]
        Xp[a][i] += h
        Xm[a][i] -= h
        Ap = voigt_element(Xp, E, NU, RHO, DT)
        Am = voigt_element(Xm, E, NU, RHO, DT)
        fd = np.array([[float((Ap[r][c] - Am[r][c]) / (2 * h)) for c in range(12)] for r in range(12)])
        assert np.abs(D[1 + k] - fd).max() <= 1e-9 * np.abs(fd).max()


# ---------------------------------------------------------------------------
# Pattern and assembly
# ---------------------------------------------------------------------------

def brute_pattern(n, tets):
    s = set()
    for t in tets:
        for a in t:
            for b in t:
                for p in range(3):
                    for q in range(3):
                        s.add((3 * int(a) + p, 3 * int(b) + q))
    return s


@pytest.mark.parametrize("seed", range(5))
def test_pattern_brute_force(seed):
    w = W.random_small_mesh(seed)
    rowptr, colidx = oracle.pattern(w.n_nodes, w.tets)
    got = set()
    for r in range(3 * w.n_nodes):
        cols = colidx[rowptr[r]:rowptr[r + 1]]
        assert np.all(np.diff(cols) > 0)
        got |= {(r, int(c)) for c in cols}
    assert got == brute_pattern(w.n_nodes, w.tets)


def test_structural_counts():
    """Superset sizes of the Kuhn cubes (seed-independent)."""
    c = W.make_cube(0)
    rp, ci = oracle.pattern(c.n_nodes, c.tets)
    assert (c.n_nodes, c.n_tets, len(rp) - 1, len(ci)) == (125, 384, 375, 11997)
    f = W.make_fracture(0, n=40)
    rp, ci = oracle.pattern(f.n_nodes, f.tets)
    assert (f.n_nodes, f.n_tets, len(ci)) == (68921, 384000, 8945649)
    # the refinement superset: 48,000 parents + 8 red children each on the 41^3 node lattice;
    # 591,101 node blocks (diagonal + off-diagonal), and corner nodes in 48 candidate tets
    r = W.make_refinement(0, n=20, frames=1)
    rp, ci = oracle.pattern(r.n_nodes, r.tets)
    assert (r.n_nodes, r.n_tets, len(ci)) == (68921, 432000, 10019529)
    t = r.tets.astype(np.int64)
    deg = np.bincount(t.ravel(), minlength=r.n_nodes)
    pairs = {(min(a, b), max(a, b)) for row in t for a, b in
             ((row[0], row[1]), (row[0], row[2]), (row[0], row[3]), (row[1], row[2]), (row[1], row[3]), (row[2], row[3]))}
    assert int(np.sum(deg > 0)) + len(pairs) == 591101
    assert deg.max() == 48


@pytest.mark.parametrize("seed", range(12))
def test_csr_equals_dense_textbook_bitwise(seed):
    """Element-major scatter into CSR gives the same bits as the dense textbook loop of
    eq. (8); absent pattern entries of the dense matrix are exactly zero."""
    w = W.random_small_mesh(seed)
    pat = oracle.pattern(w.n_nodes, w.tets)
    vals = oracle.rebuild(w.x, w.tets, w.E, w.nu, w.rho, w.dt, w.mask0, *pat)
    D = oracle.dense(w.x, w.tets, w.E, w.nu, w.rho, w.dt, w.mask0)
    r = np.repeat(np.arange(3 * w.n_nodes), np.diff(pat[0]))
    assert np.array_equal(bits(D[r, pat[1]]), bits(vals))
    off = np.ones_like(D, dtype=bool)
    off[r, pat[1]] = False
    assert np.all(D[off] == 0.0)
    # bitwise symmetric
    assert np.array_equal(bits(D), bits(D.T))


@pytest.mark.parametrize("seed", range(6))
def test_row_parallel_rebuild_equals_textbook_bitwise(seed):
    """The multi-threaded row-by-row rebuild (the many-core CPU baseline) against the dense
    textbook loop of eq. (8) on random small meshes, and against the element-major scatter
    on a jittered 8^3 cube after a fracture stream: bitwise equal both times (a row walk
    that ignored the mask, picked the wrong local vertex or summed out of id order fails)."""
    w = W.random_small_mesh(seed)
    pat = oracle.pattern(w.n_nodes, w.tets)
    vals, threads = oracle.rebuild_rows(w.x, w.tets, w.E, w.nu, w.rho, w.dt, w.mask0, *pat)
    assert threads >= 1
    D = oracle.dense(w.x, w.tets, w.E, w.nu, w.rho, w.dt, w.mask0)
    r = np.repeat(np.arange(3 * w.n_nodes), np.diff(pat[0]))
    assert np.array_equal(bits(D[r, pat[1]]), bits(vals))
    f = W.make_fracture(seed=seed, n=8)
    pat = oracle.pattern(f.n_nodes, f.tets)
    m = f.mask_after(12)
    a = oracle.rebuild(f.x, f.tets, f.E, f.nu, f.rho, f.dt, m, *pat)
    b, _ = oracle.rebuild_rows(f.x, f.tets, f.E, f.nu, f.rho, f.dt, m, *pat)
    assert np.array_equal(bits(a), bits(b))


def test_two_tets_exact():
    """Two tets sharing the face {e1, e2, e3}: exact-rational assembly of the 15x15."""
    x = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1]], dtype=np.float64)
    tets = np.array([[0, 1, 2, 3], [1, 2, 3, 4]], dtype=np.int32)
    E = np.array([1e5, 2.5e5])
    mask = np.ones(2, dtype=np.uint8)
    pat = oracle.pattern(5, tets)
    vals = oracle.rebuild(x, tets, E, NU, RHO, DT, mask, *pat)
    D = oracle.csr_to_dense(pat[0], pat[1], vals, 15)
    xf = [[F(float(v)) for v in row] for row in x]
    Ex = exact_dense(xf, tets, E, NU, RHO, DT, mask)
    assert_close_exact(D, Ex, 1e-13)
    # the shared-face block gets both tets, the private vertices only one
    assert D[0, 0] != 0 and D[12, 0] == 0.0


def test_dyadic_cube_exact_assembly():
    """Unjittered 2^3 cube (dyadic coordinates), random mask: exact rational assembly."""
    c = W.make_cube(0, n=2)
    g = np.random.default_rng(5)
    mask = (g.uniform(size=c.n_tets) < 0.6).astype(np.uint8)
    pat = oracle.pattern(c.n_nodes, c.tets)
    vals = oracle.rebuild(c.x, c.tets, c.E, NU, RHO, DT, mask, *pat)
    D = oracle.csr_to_dense(pat[0], pat[1], vals, 3 * c.n_nodes)
    xf = [[F(float(v)) for v in row] for row in c.x]
    Ex = exact_dense(xf, c.tets, c.E, NU, RHO, DT, mask)
    assert_close_exact(D, Ex, 1e-13)


def test_signed_zero_rule():
    """Unjittered cube: many terms are exact (+/-)0.  Sums start at +0.0, so no stored
    value is -0.0, and slots with no active incident tet are +0.0."""
    c = W.make_cube(0)
    mask = c.mask_after(23)
    pat = oracle.pattern(c.n_nodes, c.tets)
    vals = oracle.rebuild(c.x, c.tets, c.E, NU, RHO, DT, mask, *pat)
    assert not np.any((vals == 0.0) & np.signbit(vals))
    X = c.x[c.tets[0]]
    A = oracle.element_matrix(X, 1e5, NU, RHO, DT)
    assert np.any((A == 0.0) & np.signbit(A)), "expected -0.0 terms in an axis-aligned tet"
    none = oracle.rebuild(c.x, c.tets, c.E, NU, RHO, DT, np.zeros(c.n_tets, np.uint8), *pat)
    assert np.all(bits(none) == 0)


def test_rebuild_is_pure_function_of_mask():
    """Sec. 3.3 invariant for the oracle itself: the matrix depends only on the mask, so
    deleting then reinserting a set gives the initial bits back."""
    w = W.make_fracture(seed=2, n=4, counts=[5, 9, 3])
    pat = oracle.pattern(w.n_nodes, w.tets)
    v0 = oracle.rebuild_workload(w, w.mask0, pat)
    m = w.mask_after(2)
    v1 = oracle.rebuild_workload(w, m, pat)
    assert not np.array_equal(bits(v0), bits(v1))
    back = m.copy()
    for ids, _ in w.frames:
        back[ids] = 1
    assert np.array_equal(bits(oracle.rebuild_workload(w, back, pat)), bits(v0))


# ---------------------------------------------------------------------------
# Solve and gradient
# ---------------------------------------------------------------------------

def _small_state(seed=0, n=4):
    w = W.make_fracture(seed=seed, n=n, counts=[10, 20, 15])
    mask = w.mask_after(2)
    pat = oracle.pattern(w.n_nodes, w.tets)
    vals = oracle.rebuild_workload(w, mask, pat)
    f = W.loads_for(w, mask, seed)
    return w, mask, pat, vals, f


def test_pcg_matches_direct_solve():
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    w, mask, pat, vals, f = _small_state()
    A = sp.csr_matrix((vals, pat[1], pat[0]), shape=(3 * w.n_nodes,) * 2)
    live = A.diagonal() != 0
    u, it, rr = oracle.pcg(pat[0], pat[1], vals, f.reshape(-1), rtol=1e-13)
    Al = A[live][:, live]
    ud = spla.spsolve(Al.tocsc(), f.reshape(-1)[live])
    assert rr <= 1e-13
    assert np.abs(u[live] - ud).max() <= 1e-10 * np.abs(ud).max()
    assert np.all(u[~live] == 0.0)


def _compliance_grad(w, mask, pat, vals, f):
    u, _, _ = oracle.pcg(pat[0], pat[1], vals, f.reshape(-1), rtol=1e-14)
    r = np.repeat(np.arange(3 * w.n_nodes), np.diff(pat[0]))
    gA = -(u[r] * u[pat[1]])
    gl, gx = oracle.adjoint(w.x, w.tets, w.E, w.nu, w.rho, w.dt, mask, pat[0], pat[1], gA)
    return u, gl, gx


def test_gradient_identities():
    """Compliance L = f^T u, A u = f.  With slot cotangent -u u^T:
    G2 dL/dlogE_e = -dt^2 u_e^T K_e u_e <= 0;  G3 sum_e dL/dlogE_e = u^T M u - L;
    G4 sum_i dL/dx_i = 0 (translation);  G5 sum_i x_i . dL/dx_i = -(dt^2 u^T K u + 3 u^T M u)."""
    w, mask, pat, vals, f = _small_state()
    u, gl, gx = _compliance_grad(w, mask, pat, vals, f)
    L = float(f.reshape(-1) @ u)
    # M and dt^2 K from separate oracle assemblies
    vM = oracle.rebuild(w.x, w.tets, np.zeros(w.n_tets), w.nu, w.rho, w.dt, mask, *pat)
    vK = oracle.rebuild(w.x, w.tets, w.E, w.nu, 0.0, w.dt, mask, *pat)
    uMu = float(u @ oracle.spmv(pat[0], pat[1], vM, u))
    uKu = float(u @ oracle.spmv(pat[0], pat[1], vK, u))
    act = mask.astype(bool)
    assert np.all(gl[act] <= 1e-14 * np.abs(gl).max())
    assert np.all(gl[~act] == 0.0)
    assert abs(gl.sum() - (uMu - L)) <= 1e-9 * abs(L)
    assert np.abs(gx.sum(0)).max() <= 1e-9 * np.abs(gx).max()
    assert abs((w.x * gx).sum() + (uKu + 3 * uMu)) <= 1e-9 * (uKu + 3 * uMu)


def test_gradient_exact_difference_fd():
    """Central difference with h = 1e-6 in exact-difference form:
    L(+h) - L(-h) = -u_+^T (A_+ - A_-) u_-, A_+ - A_- from the perturbed tets only."""
    w, mask, pat, vals, f = _small_state()
    u, gl, gx = _compliance_grad(w, mask, pat, vals, f)
    fv = f.reshape(-1)
    h = 1e-6

    def solve_with(E=None, x=None):
        Ev = w.E if E is None else E
        xv = w.x if x is None else x
        v = oracle.rebuild(xv, w.tets, Ev, w.nu, w.rho, w.dt, mask, *pat)
        return oracle.pcg(pat[0], pat[1], v, fv, rtol=1e-14)[0]

    def local_diff(tets_ids, xp, xm, Ep, Em):
        up = solve_with(Ep, xp)
        um = solve_with(Em, xm)
        acc = 0.0
        for e in tets_ids:
            t = w.tets[e]
            Ap = oracle.element_matrix(xp[t], Ep[e], w.nu, w.rho, w.dt)
            Am = oracle.element_matrix(xm[t], Em[e], w.nu, w.rho, w.dt)
            dof = (3 * t[:, None] + np.arange(3)[None, :]).reshape(-1)
            acc += up[dof] @ (Ap - Am) @ um[dof]
        return -acc / (2 * h)

    act = np.nonzero(mask)[0]
    g = np.random.default_rng(0)
    for e in g.choice(act, 4, replace=False):
        Ep, Em = w.E.copy(), w.E.copy()
        Ep[e] = np.exp(np.log(w.E[e]) + h)
        Em[e] = np.exp(np.log(w.E[e]) - h)
        fd = local_diff([e], w.x, w.x, Ep, Em)
        assert abs(fd - gl[e]) <= 1e-6 * abs(gl[e])
    used = np.unique(w.tets[act])
    for i in g.choice(used, 3, replace=False):
        ring = [e for e in act if i in w.tets[e]]
        for k in range(3):
            xp, xm = w.x.copy(), w.x.copy()
            xp[i, k] += h
            xm[i, k] -= h
            fd = local_diff(ring, xp, xm, w.E, w.E)
            assert abs(fd - gx[i, k]) <= 1e-6 * np.abs(gx[i]).max()


def test_weighted_magnitude_assembly():
    """The error-bound helper: with unit weights on the active tets its diagonal equals the
    rebuild's (diagonal terms are non-negative, same order), every entry bounds the
    rebuild's magnitude, and count_only gives each entry its number of active incident
    tets (counted here from the node pairs directly)."""
    import oracle
    w = W.make_fracture(seed=4, n=5, counts=[20])
    rowptr, colidx = oracle.pattern(w.n_nodes, w.tets)
    mask = w.mask_after(0)
    vals = oracle.rebuild(w.x, w.tets, w.E, w.nu, w.rho, w.dt, mask, rowptr, colidx)
    mag = oracle.rebuild_weighted(w.x, w.tets, w.E, w.nu, w.rho, w.dt, mask.astype(float), rowptr, colidx)
    cnt = oracle.rebuild_weighted(w.x, w.tets, w.E, w.nu, w.rho, w.dt, mask.astype(float), rowptr, colidx,
                                  count_only=True)
    rows = np.repeat(np.arange(3 * w.n_nodes), np.diff(rowptr))
    diag = rows == colidx
    assert np.array_equal(vals[diag].view(np.uint64), mag[diag].view(np.uint64))
    assert np.all(mag >= np.abs(vals))
    pairs = {}
    for t in w.tets[mask.astype(bool)]:
        for a in t:
            for b in t:
                pairs[(int(a), int(b))] = pairs.get((int(a), int(b)), 0) + 1
    want = np.array([pairs.get((int(r) // 3, int(c) // 3), 0) for r, c in zip(rows, colidx)], dtype=float)
    assert np.array_equal(cnt, want)


def test_lumped_mass_pins():
    """M_t equals the diagonal of the rebuild with E = 0 bit for bit (then A = M: the
    stiffness terms vanish and the element diagonal is exactly its mass term, summed in
    the same order); on the unjittered fully active cube the total mass is rho x volume 1
    (to rounding: each tet's volume h^3/6 is rounded once); a node's three dofs agree."""
    import oracle
    w = W.make_fracture(seed=6, n=6, counts=[60])
    mask = w.mask_after(0)
    m = oracle.lumped_mass(w.x, w.tets, w.rho, mask)
    rowptr, colidx = oracle.pattern(w.n_nodes, w.tets)
    vals = oracle.rebuild(w.x, w.tets, np.zeros(w.n_tets), w.nu, w.rho, w.dt, mask, rowptr, colidx)
    rows = np.repeat(np.arange(3 * w.n_nodes), np.diff(rowptr))
    diag = np.zeros(3 * w.n_nodes)
    diag[rows[rows == colidx]] = vals[rows == colidx]
    assert np.array_equal(m.view(np.uint64), diag.view(np.uint64))
    assert np.array_equal(m[0::3], m[1::3]) and np.array_equal(m[0::3], m[2::3])
    c = W.make_cube(0, n=4)
    mc = oracle.lumped_mass(c.x, c.tets, c.rho, c.mask0)
    assert abs(math.fsum(mc[0::3]) - c.rho) <= 1e-12 * c.rho


def test_euler_step_solves_equation():
    """One implicit-Euler step from rest under gravity: the returned u' satisfies
    (M + h^2 K) u' = M (u + h v) + h^2 f to the solver tolerance (checked with scipy's
    direct solve, a different route), and v' = (u' - u) / h."""
    import oracle
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    w = W.make_fracture(seed=7, n=4, counts=[10])
    mask = w.mask_after(0)
    rowptr, colidx = oracle.pattern(w.n_nodes, w.tets)
    vals = oracle.rebuild(w.x, w.tets, w.E, w.nu, w.rho, w.dt, mask, rowptr, colidx)
    m = oracle.lumped_mass(w.x, w.tets, w.rho, mask)
    f = W.loads_for(w, mask).reshape(-1)
    u = np.zeros_like(m)
    v = np.zeros_like(m)
    u1, v1, it, rr = oracle.euler_step(rowptr, colidx, vals, m, u, v, f, w.dt)
    A = sp.csr_matrix((vals, colidx, rowptr), shape=(len(m), len(m)))
    act = A.diagonal() != 0
    b = m * (u + w.dt * v) + w.dt ** 2 * f
    ref = np.zeros_like(m)
    ref[act] = spla.spsolve(A[act][:, act].tocsc(), b[act])
    assert np.linalg.norm(u1 - ref) <= 1e-9 * np.linalg.norm(ref)
    assert np.array_equal(v1, (u1 - u) / w.dt) and rr <= 1e-12
