"""Exact-rational references used as pins for the oracle (tests only).

These are deliberately a *different* formula from the oracle's: the element
stiffness is built in Voigt form, K = V B^T D B with engineering shear
strains, from an exact inverse of the edge matrix, in ``fractions.Fraction``.
The oracle instead uses the gradient-outer-product form.  Agreement pins the
oracle's formula (no dropped term, wrong sign or transposed operand).
"""
from fractions import Fraction as F


def mat_inv3(M):
    """Exact inverse of a 3x3 Fraction matrix (adjugate / determinant)."""
    a, b, c = M[0]
    d, e, f = M[1]
    g, h, i = M[2]
    det = a * (e * i - f * h) - b * (d * i - f * g) + c * (d * h - e * g)
    adj = [
        [e * i - f * h, c * h - b * i, b * f - c * e],
        [f * g - d * i, a * i - c * g, c * d - a * f],
        [d * h - e * g, b * g - a * h, a * e - b * d],
    ]
    return [[adj[r][s] / det for s in range(3)] for r in range(3)], det


def voigt_element(X, E, nu, rho, dt):
    """Exact 12x12 A_e = dt^2 V B^T D B + lumped mass, all Fractions.

    X: 4 vertices (Fraction triples).  Gradients of the barycentric functions
    come from the inverse of the edge matrix [x1-x0, x2-x0, x3-x0] (columns).
    """
    E, nu, rho, dt = F(E), F(nu), F(rho), F(dt)
    cols = [[X[k][i] - X[0][i] for i in range(3)] for k in (1, 2, 3)]
    M = [[cols[k][i] for k in range(3)] for i in range(3)]  # M[i][k] = (x_k - x_0)_i
    Minv, det = mat_inv3(M)
    # grad lambda_k (k=1..3) is row k-1 of M^{-1}; grad lambda_0 = -sum
    g = [None, Minv[0], Minv[1], Minv[2]]
    g[0] = [-(g[1][i] + g[2][i] + g[3][i]) for i in range(3)]
    V = abs(det) / 6
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    D = [[F(0)] * 6 for _ in range(6)]
    for i in range(3):
        for j in range(3):
            D[i][j] = lam + (2 * mu if i == j else 0)
        D[3 + i][3 + i] = mu
    # B: 6 x 12, strains (xx, yy, zz, 2yz, 2xz, 2xy)
    B = [[F(0)] * 12 for _ in range(6)]
    for a in range(4):
        gx, gy, gz = g[a]
        B[0][3 * a + 0] = gx
        B[1][3 * a + 1] = gy
        B[2][3 * a + 2] = gz
        B[3][3 * a + 1] = gz
        B[3][3 * a + 2] = gy
        B[4][3 * a + 0] = gz
        B[4][3 * a + 2] = gx
        B[5][3 * a + 0] = gy
        B[5][3 * a + 1] = gx
    DB = [[sum(D[r][k] * B[k][c] for k in range(6)) for c in range(12)] for r in range(6)]
    A = [[dt * dt * V * sum(B[k][r] * DB[k][c] for k in range(6)) for c in range(12)] for r in range(12)]
    for r in range(12):
        A[r][r] += rho * V / 4
    return A


def exact_dense(x, tets, E, nu, rho, dt, mask):
    """Exact dense assembly (Fractions) over active tets; x given as Fractions."""
    n = len(x)
    D = [[F(0)] * (3 * n) for _ in range(3 * n)]
    for e, t in enumerate(tets):
        if not mask[e]:
            continue
        A = voigt_element([x[int(v)] for v in t], E[e], nu, rho, dt)
        for r in range(12):
            for c in range(12):
                D[3 * int(t[r // 3]) + r % 3][3 * int(t[c // 3]) + c % 3] += A[r][c]
    return D
