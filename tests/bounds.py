"""First-order rounding bounds for per-entry comparisons of two floating-point
implementations of the same computation (the GPU path and the oracle).

Both sides evaluate the same exact expression; each deviates from the exact
value by at most the bound computed here (IEEE binary64, unit roundoff
u = 2^-53, a sum of L terms in any order off by at most gamma_L times the sum
of their magnitudes, gamma_L = L u / (1 - L u)), so two results may differ by
at most twice the bound.  Magnitudes come from a plain run of the same
recurrence in float64 (any run differs from the exact one by far less than
the values themselves, so first order suffices); none of these routines
produces a value that is compared, only tolerances.
"""
import numpy as np

U = 2.0 ** -53


def gamma(n):
    n = np.asarray(n, dtype=np.float64)
    return n * U / (1.0 - n * U)


def abs_spmv(rowptr, colidx, vals, v):
    """|A| v for a non-negative v (CSR)."""
    r = np.repeat(np.arange(len(rowptr) - 1), np.diff(rowptr))
    return np.bincount(r, weights=np.abs(vals) * v[colidx], minlength=len(rowptr) - 1)


def pcg_bound(rowptr, colidx, vals, b, k, eb=None):
    """Jacobi-PCG from x = 0, k iterations, on the dofs with a nonzero diagonal (the others
    held at 0): returns (x_k, ex_k) with ex_k the per-dof first-order bound on the distance
    of any implementation's x_k from the exact-arithmetic x_k, given a per-dof bound eb on
    the error of b.  Per iteration: q = A p, alpha = r.z / p.q, x += alpha p, r -= alpha q,
    z = r / diag, beta = r.z (new) / r.z (old), p = z + beta p."""
    n = len(rowptr) - 1
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    d = np.zeros(n)
    on = colidx == rows
    d[rows[on]] = vals[on]
    live = d != 0.0
    dinv = np.where(live, 1.0 / np.where(live, d, 1.0), 0.0)
    kap = np.diff(rowptr).astype(np.float64)
    gn = float(gamma(int(live.sum())))
    A = lambda v: np.bincount(rows, weights=vals * v[colidx], minlength=n)
    b = np.where(live, b, 0.0)
    eb = np.zeros(n) if eb is None else np.where(live, eb, 0.0)
    x, ex = np.zeros(n), np.zeros(n)
    r, er = b.copy(), eb.copy()
    z = r * dinv
    ez = np.abs(dinv) * er + 2 * U * np.abs(z)
    p, ep = z.copy(), ez.copy()
    rz = float(r @ z)
    erz = float(np.abs(r) @ ez + np.abs(z) @ er) + gn * float(np.abs(r) @ np.abs(z))
    for _ in range(k):
        q = np.where(live, A(p), 0.0)
        eq = np.where(live, abs_spmv(rowptr, colidx, vals, ep) + gamma(kap) * abs_spmv(rowptr, colidx, vals,
                                                                                        np.abs(p)), 0.0)
        pq = float(p @ q)
        epq = float(np.abs(p) @ eq + np.abs(q) @ ep) + gn * float(np.abs(p) @ np.abs(q))
        alpha = rz / pq
        ea = abs(alpha) * (erz / abs(rz) + epq / abs(pq) + U)
        x_new = x + alpha * p
        ex = ex + ea * np.abs(p) + abs(alpha) * ep + U * np.abs(alpha * p) + U * np.abs(x_new)
        x = x_new
        r_new = r - alpha * q
        er = er + ea * np.abs(q) + abs(alpha) * eq + U * np.abs(alpha * q) + U * np.abs(r_new)
        r = r_new
        z = r * dinv
        ez = np.abs(dinv) * er + 2 * U * np.abs(z)
        rz_new = float(r @ z)
        erz_new = float(np.abs(r) @ ez + np.abs(z) @ er) + gn * float(np.abs(r) @ np.abs(z))
        beta = rz_new / rz
        eb_ = abs(beta) * (erz_new / abs(rz_new) + erz / abs(rz) + U)
        p_new = z + beta * p
        ep = ez + eb_ * np.abs(p) + abs(beta) * ep + U * np.abs(beta * p) + U * np.abs(p_new)
        p = p_new
        rz, erz = rz_new, erz_new
    return x, ex


def tet_cotangents(rowptr, colidx, tets, gA, ids):
    """The 144 slot cotangents of each tet in ids, as (len(ids), 4, 4, 3, 3): entry
    [a, b, i, j] is gA at row 3 T[a] + i, column 3 T[b] + j."""
    n_rows = len(rowptr) - 1
    rows = np.repeat(np.arange(n_rows, dtype=np.int64), np.diff(rowptr))
    keys = rows * n_rows + colidx.astype(np.int64)
    T = tets[ids].astype(np.int64)
    dof = 3 * T[:, :, None] + np.arange(3)[None, None, :]  # (m, 4, 3)
    r = dof[:, :, None, :, None]
    c = dof[:, None, :, None, :]
    pos = np.searchsorted(keys, (r * n_rows + c).reshape(-1))
    return gA[pos].reshape(len(ids), 4, 4, 3, 3)


def tet_geometry(x, tets, E, nu, rho, dt, ids):
    """Basis gradients g (m, 4, 3), |det| and the scaled moduli lamV, muV and the lumped
    mass per vertex of each tet in ids (numpy; magnitudes for bounds only)."""
    X = x[tets[ids]]
    D = np.transpose(X[:, 1:] - X[:, :1], (0, 2, 1))  # columns x_k - x_0
    G = np.transpose(np.linalg.inv(D), (0, 2, 1))     # g_k = columns of D^-T
    g = np.concatenate([-G.sum(axis=2, keepdims=True), G], axis=2)  # (m, 3, 4)
    g = np.transpose(g, (0, 2, 1))
    det = np.abs(np.linalg.det(D))
    V = det / 6.0
    lam = E[ids] * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E[ids] * 0.5 / (1 + nu)
    return g, det, lam * V * dt * dt, mu * V * dt * dt, rho * V * 0.25


def adjoint_tolerances(w, mask, rowptr, colidx, gA, chunk=40000):
    """Per-entry tolerances for comparing two implementations of the assembly adjoint at
    fixed slot cotangents gA: (tol_logE (m,), tol_x (n, 3)).

    dL/dlogE_e = sum over the tet's 144 entries of gA * (dt^2 K_e).  Each entry of dt^2 K_e
    is lamV g_ai g_bj + muV g_aj g_bi (+ muV g_a.g_b), a few roundings deep, and the sum
    has 144 terms in either route, so each side is within (144 + 16) u S_e of the exact
    value, S_e = sum |gA| (lamV |g_ai||g_bj| + muV |g_aj||g_bi| + [i=j] muV sum_k |g_ak||g_bk|).

    dL/dx: the derivative of an entry with respect to a vertex coordinate is bounded by
    (lamV + 2 muV) G^3 + m G per unit cotangent (G = the tet's largest gradient component),
    and the reverse-mode chain (pair terms, vertex-gradient cotangents, Vbar, Dbar =
    -G Gbar^T G + ..., vertex sums over <= 48 tets) has six stages of at most ~30
    roundings over intermediates within 200 times that scale; each side is therefore
    within 2^13 u X_e per tet with X_e = W_e ((lamV + 2 muV) G_e^3 + m_e G_e), W_e = sum
    |gA| over the tet's entries, and a node within the sum of its active tets' bounds.
    Both tolerances are for the difference of two implementations (twice one side's)."""
    act = np.nonzero(mask)[0]
    tl = np.zeros(w.n_tets)
    tx = np.zeros(w.n_nodes)
    for s in range(0, len(act), chunk):
        ids = act[s:s + chunk]
        Ab = np.abs(tet_cotangents(rowptr, colidx, w.tets, gA, ids))
        g, det, lamV, muV, ml = tet_geometry(w.x, w.tets, w.E, w.nu, w.rho, w.dt, ids)
        ag = np.abs(g)
        outer = ag[:, :, None, :, None] * ag[:, None, :, None, :]  # |g_ai||g_bj|
        S = (lamV[:, None, None, None, None] * outer + muV[:, None, None, None, None]
             * np.transpose(outer, (0, 1, 2, 4, 3)))
        dots = np.einsum("mak,mbk->mab", ag, ag)
        S = (Ab * S).sum(axis=(1, 2, 3, 4)) + muV * np.einsum("mabii,mab->m", Ab, dots)
        tl[ids] = 2 * 160 * U * S
        Gm = ag.max(axis=(1, 2))
        Xe = Ab.sum(axis=(1, 2, 3, 4)) * ((lamV + 2 * muV) * Gm ** 3 + ml * Gm)
        np.add.at(tx, w.tets[ids].reshape(-1), np.repeat(2 * 2.0 ** 13 * U * Xe, 4))
    return tl, np.repeat(tx[:, None], 3, axis=1)


def euler_rhs_bound(m, u, v, f, h, eu, ev):
    """Per-dof bound on b = (m (u + (h v))) + ((h h) f) given bounds eu, ev on u, v."""
    t1 = h * v
    t2 = u + t1
    t3 = m * t2
    t4 = (h * h) * f
    b = t3 + t4
    e2 = eu + h * ev + U * np.abs(t1) + U * np.abs(t2)
    return np.abs(m) * e2 + U * np.abs(t3) + 2 * U * np.abs(t4) + U * np.abs(b)
