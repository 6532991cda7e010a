/*
 * CPU oracle for exact assembly of A_t = M_t + dt^2 K_t over a superset tet mesh.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference
 * the GPU path is checked against.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product path never does.  It
 * shares no code, header or table with the GPU library.
 *
 * What it computes (paper Sec. 3.4, eq. (8), with eps = 0):
 *     A_t = sum over active tets tau, in ascending id, of P_tau^T A_tau P_tau
 * where A_tau = dt^2 K_tau + M_tau is the 12x12 element matrix of a P1
 * (linear) tetrahedron under isotropic small-strain linear elasticity, and
 * M_tau is the row-sum lumped mass (rho V / 4 on each dof of each vertex),
 * as in the implicit-Euler system of Sec. 6.2 eq. (9).  The paper calls the
 * stiffness "standard" and prints no formula; the one used here is
 *     K_ab = V (lambda g_a g_b^T + mu g_b g_a^T + mu (g_a . g_b) I),
 * g_a the gradient of the barycentric basis function of vertex a, which is
 * the Hessian of mu eps:eps + lambda/2 tr(eps)^2.
 *
 * Exactness (Sec. 3.3: the maintained matrix equals a rebuild from scratch)
 * is taken bitwise, so every floating-point step below is fixed: IEEE-754
 * binary64, round to nearest even, no contraction (build with
 * -ffp-contract=off), evaluated in the parenthesised order written, sums
 * over elements starting from +0.0 in ascending element id.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_ENOSLOT (-1)
#define OR_ENOMEM (-2)

/* ------------------------------------------------------------------------ */
/* Element matrix (real, the definition)                                    */
/* ------------------------------------------------------------------------ */

/* X: the tet's 4 vertices, vertex a at X[3a..3a+2], in the tet's own vertex
 * order.  A: row-major 12x12, dof 3a+i = component i of vertex a. */
void oracle_element(const double *X, double E, double nu, double rho, double dt, double *A)
{
    /* material constants */
    const double cdt = dt * dt;
    const double den = (1.0 + nu) * (1.0 - (2.0 * nu));
    const double clam = nu / den;
    const double cmu = 0.5 / (1.0 + nu);
    const double lam = E * clam;
    const double mu = E * cmu;

    /* edge vectors d_k = x_k - x_0 */
    double d[4][3];
    for (int k = 1; k <= 3; ++k)
        for (int i = 0; i < 3; ++i)
            d[k][i] = X[3 * k + i] - X[i];

    /* cofactor vectors c1 = d2 x d3, c2 = d3 x d1, c3 = d1 x d2 */
    double c[4][3];
    const int nxt[4][2] = {{0, 0}, {2, 3}, {3, 1}, {1, 2}};
    for (int k = 1; k <= 3; ++k) {
        const double *a = d[nxt[k][0]], *b = d[nxt[k][1]];
        c[k][0] = (a[1] * b[2]) - (a[2] * b[1]);
        c[k][1] = (a[2] * b[0]) - (a[0] * b[2]);
        c[k][2] = (a[0] * b[1]) - (a[1] * b[0]);
    }
    const double det = ((d[1][0] * c[1][0]) + (d[1][1] * c[1][1])) + (d[1][2] * c[1][2]);
    const double inv = 1.0 / det;

    /* basis-function gradients: g_k = c_k / det, g_0 = -(g_1 + g_2 + g_3) */
    double g[4][3];
    for (int k = 1; k <= 3; ++k)
        for (int i = 0; i < 3; ++i)
            g[k][i] = c[k][i] * inv;
    for (int i = 0; i < 3; ++i)
        g[0][i] = -((g[1][i] + g[2][i]) + g[3][i]);

    const double V = fabs(det) / 6.0;
    const double lamV = (lam * V) * cdt;
    const double muV = (mu * V) * cdt;
    const double mlump = (rho * V) * 0.25;

    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            const double s = ((g[a][0] * g[b][0]) + (g[a][1] * g[b][1])) + (g[a][2] * g[b][2]);
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    double v = (lamV * (g[a][i] * g[b][j])) + (muV * (g[a][j] * g[b][i]));
                    if (i == j)
                        v = v + (muV * s);
                    if (a == b && i == j)
                        v = v + mlump;
                    A[(3 * a + i) * 12 + (3 * b + j)] = v;
                }
        }
}

/* Signed volume determinant only (for degeneracy checks in tests). */
double oracle_det(const double *X)
{
    double d[4][3];
    for (int k = 1; k <= 3; ++k)
        for (int i = 0; i < 3; ++i)
            d[k][i] = X[3 * k + i] - X[i];
    const double c0 = (d[2][1] * d[3][2]) - (d[2][2] * d[3][1]);
    const double c1 = (d[2][2] * d[3][0]) - (d[2][0] * d[3][2]);
    const double c2 = (d[2][0] * d[3][1]) - (d[2][1] * d[3][0]);
    return ((d[1][0] * c0) + (d[1][1] * c1)) + (d[1][2] * c2);
}

static void gather_X(const double *x, const int32_t *t, double *X)
{
    for (int a = 0; a < 4; ++a)
        for (int i = 0; i < 3; ++i)
            X[3 * a + i] = x[3 * (int64_t)t[a] + i];
}

/* Position of column col in CSR row row, or -1. */
static int64_t find_slot(const int32_t *rowptr, const int32_t *colidx, int64_t row, int64_t col)
{
    int64_t lo = rowptr[row], hi = rowptr[row + 1];
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (colidx[mid] < col)
            lo = mid + 1;
        else
            hi = mid;
    }
    if (lo < rowptr[row + 1] && colidx[lo] == col)
        return lo;
    return -1;
}

/* ------------------------------------------------------------------------ */
/* Assembly from the mask (the rebuild the maintained matrix must equal)    */
/* ------------------------------------------------------------------------ */

/* values[nnz] := sum over active e ascending of A_e scattered through P_e.
 * Every slot starts at +0.0; each active element adds exactly one term to
 * each of the slots it covers, in element order (the textbook loop of
 * eq. (8)).  Returns OR_ENOSLOT if the pattern lacks an entry. */
int oracle_rebuild(int64_t n_nodes, const double *x, int64_t n_tets, const int32_t *tets,
                   const double *E, double nu, double rho, double dt, const uint8_t *mask,
                   const int32_t *rowptr, const int32_t *colidx, int64_t nnz, double *values)
{
    (void)n_nodes;
    for (int64_t s = 0; s < nnz; ++s)
        values[s] = 0.0;
    double X[12], A[144];
    for (int64_t e = 0; e < n_tets; ++e) {
        if (!mask[e])
            continue;
        const int32_t *t = tets + 4 * e;
        gather_X(x, t, X);
        oracle_element(X, E[e], nu, rho, dt, A);
        for (int r = 0; r < 12; ++r)
            for (int c = 0; c < 12; ++c) {
                int64_t row = 3 * (int64_t)t[r / 3] + r % 3;
                int64_t col = 3 * (int64_t)t[c / 3] + c % 3;
                int64_t s = find_slot(rowptr, colidx, row, col);
                if (s < 0)
                    return OR_ENOSLOT;
                values[s] = values[s] + A[r * 12 + c];
            }
    }
    return OR_OK;
}

/* Weighted magnitude assembly, for error bounds (not part of the method):
 * values[s] = sum over candidates e with w[e] != 0 of w[e] * |A_e term| at
 * slot s, or of w[e] alone when count_only (then an entry gets the weighted
 * number of candidates that reach it).  Same scatter as oracle_rebuild. */
int oracle_rebuild_weighted(int64_t n_nodes, const double *x, int64_t n_tets, const int32_t *tets,
                            const double *E, double nu, double rho, double dt, const double *w, int count_only,
                            const int32_t *rowptr, const int32_t *colidx, int64_t nnz, double *values)
{
    (void)n_nodes;
    for (int64_t s = 0; s < nnz; ++s)
        values[s] = 0.0;
    double X[12], A[144];
    for (int64_t e = 0; e < n_tets; ++e) {
        if (w[e] == 0.0)
            continue;
        const int32_t *t = tets + 4 * e;
        if (!count_only) {
            gather_X(x, t, X);
            oracle_element(X, E[e], nu, rho, dt, A);
        }
        for (int r = 0; r < 12; ++r)
            for (int c = 0; c < 12; ++c) {
                int64_t row = 3 * (int64_t)t[r / 3] + r % 3;
                int64_t col = 3 * (int64_t)t[c / 3] + c % 3;
                int64_t s = find_slot(rowptr, colidx, row, col);
                if (s < 0)
                    return OR_ENOSLOT;
                values[s] = values[s] + (count_only ? w[e] : w[e] * fabs(A[r * 12 + c]));
            }
    }
    return OR_OK;
}

/* The same rebuild as oracle_rebuild, row by row on all host threads (a CPU
 * baseline on many cores, not a second definition).  Each slot (row 3i+p,
 * column 3j+q) is written by exactly one thread: +0.0, then, over the active
 * tets that hold node i in ascending id, the term A_e[3a+p][3b+q] of those
 * that also hold node j (a, b: the local vertices of i and j).  These are
 * the same terms in the same order as the element-major scatter, so the
 * values are bitwise those of oracle_rebuild.  Element matrices of the
 * active tets are computed first (one per tet, in parallel) into scratch
 * the routine allocates.  *threads_out (may be NULL) receives the number of
 * threads used.  Returns OR_ENOMEM if scratch cannot be allocated. */
int oracle_rebuild_rows(int64_t n_nodes, const double *x, int64_t n_tets, const int32_t *tets,
                        const double *E, double nu, double rho, double dt, const uint8_t *mask,
                        const int32_t *rowptr, const int32_t *colidx, double *values, int *threads_out)
{
    double *Ae = (double *)malloc(sizeof(double) * 144 * (size_t)(n_tets > 0 ? n_tets : 1));
    int64_t *start = (int64_t *)calloc((size_t)n_nodes + 1, sizeof(int64_t));
    int64_t *inc = (int64_t *)malloc(sizeof(int64_t) * 4 * (size_t)(n_tets > 0 ? n_tets : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n_nodes + 1));
    if (!Ae || !start || !inc || !fill) {
        free(Ae);
        free(start);
        free(inc);
        free(fill);
        return OR_ENOMEM;
    }
    int threads = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            threads = omp_get_num_threads();
#endif
        }
#pragma omp for schedule(static)
        for (int64_t e = 0; e < n_tets; ++e) {
            if (!mask[e])
                continue;
            double X[12];
            gather_X(x, tets + 4 * e, X);
            oracle_element(X, E[e], nu, rho, dt, Ae + 144 * e);
        }
    }
    /* node -> (tet, local vertex) lists in ascending tet id (counting sort) */
    for (int64_t e = 0; e < n_tets; ++e)
        for (int a = 0; a < 4; ++a)
            start[tets[4 * e + a] + 1] += 1;
    for (int64_t i = 0; i < n_nodes; ++i)
        start[i + 1] += start[i];
    memcpy(fill, start, sizeof(int64_t) * (size_t)n_nodes);
    for (int64_t e = 0; e < n_tets; ++e)
        for (int a = 0; a < 4; ++a)
            inc[fill[tets[4 * e + a]]++] = 4 * e + a;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n_nodes; ++i)
        for (int p = 0; p < 3; ++p) {
            const int64_t row = 3 * i + p;
            for (int64_t s = rowptr[row]; s < rowptr[row + 1]; ++s) {
                const int64_t j = colidx[s] / 3, q = colidx[s] % 3;
                double acc = 0.0;
                for (int64_t k = start[i]; k < start[i + 1]; ++k) {
                    const int64_t e = inc[k] / 4;
                    const int a = (int)(inc[k] % 4);
                    if (!mask[e])
                        continue;
                    for (int b = 0; b < 4; ++b)
                        if (tets[4 * e + b] == j)
                            acc = acc + Ae[144 * e + (3 * a + p) * 12 + (3 * b + q)];
                }
                values[s] = acc;
            }
        }
    free(Ae);
    free(start);
    free(inc);
    free(fill);
    if (threads_out)
        *threads_out = threads;
    return OR_OK;
}

/* Lumped mass of the active set (Sec. 6.2: the maintained M_t of eq. (9)):
 * m[3i+k] = sum over active tets e containing node i, in ascending e, from
 * +0.0, of (rho * V_e) * 0.25 with V_e = |det| / 6 (the mass term of the
 * element formula). */
void oracle_lumped_mass(int64_t n_nodes, const double *x, int64_t n_tets, const int32_t *tets, double rho,
                        const uint8_t *mask, double *m)
{
    for (int64_t s = 0; s < 3 * n_nodes; ++s)
        m[s] = 0.0;
    double X[12];
    for (int64_t e = 0; e < n_tets; ++e) {
        if (!mask[e])
            continue;
        const int32_t *t = tets + 4 * e;
        gather_X(x, t, X);
        const double V = fabs(oracle_det(X)) / 6.0;
        const double me = (rho * V) * 0.25;
        for (int a = 0; a < 4; ++a)
            for (int k = 0; k < 3; ++k)
                m[3 * (int64_t)t[a] + k] = m[3 * (int64_t)t[a] + k] + me;
    }
}

/* Dense textbook assembly, eq. (8): D (3n x 3n, row-major) := 0; for each
 * active element in ascending id, D += P^T A_e P.  For tiny meshes only. */
void oracle_dense(int64_t n_nodes, const double *x, int64_t n_tets, const int32_t *tets,
                  const double *E, double nu, double rho, double dt, const uint8_t *mask, double *D)
{
    const int64_t N = 3 * n_nodes;
    for (int64_t s = 0; s < N * N; ++s)
        D[s] = 0.0;
    double X[12], A[144];
    for (int64_t e = 0; e < n_tets; ++e) {
        if (!mask[e])
            continue;
        const int32_t *t = tets + 4 * e;
        gather_X(x, t, X);
        oracle_element(X, E[e], nu, rho, dt, A);
        for (int r = 0; r < 12; ++r)
            for (int c = 0; c < 12; ++c) {
                int64_t row = 3 * (int64_t)t[r / 3] + r % 3;
                int64_t col = 3 * (int64_t)t[c / 3] + c % 3;
                D[row * N + col] = D[row * N + col] + A[r * 12 + c];
            }
    }
}

/* ------------------------------------------------------------------------ */
/* Derivatives by complex step (an independent route for gradient checks)   */
/* ------------------------------------------------------------------------ */

/* The element matrix evaluated in complex arithmetic.  |det| is continued
 * analytically as sign(Re det) * det.  Only the imaginary parts are used,
 * divided by the step, as derivatives; rounding order is irrelevant here. */
static void element_complex(const double complex *X, double complex E, double nu, double rho, double dt,
                            double complex *A)
{
    const double cdt = dt * dt;
    const double den = (1.0 + nu) * (1.0 - (2.0 * nu));
    const double complex lam = E * (nu / den);
    const double complex mu = E * (0.5 / (1.0 + nu));
    double complex d[4][3], c[4][3], g[4][3];
    for (int k = 1; k <= 3; ++k)
        for (int i = 0; i < 3; ++i)
            d[k][i] = X[3 * k + i] - X[i];
    const int nxt[4][2] = {{0, 0}, {2, 3}, {3, 1}, {1, 2}};
    for (int k = 1; k <= 3; ++k) {
        const double complex *a = d[nxt[k][0]], *b = d[nxt[k][1]];
        c[k][0] = a[1] * b[2] - a[2] * b[1];
        c[k][1] = a[2] * b[0] - a[0] * b[2];
        c[k][2] = a[0] * b[1] - a[1] * b[0];
    }
    const double complex det = d[1][0] * c[1][0] + d[1][1] * c[1][1] + d[1][2] * c[1][2];
    for (int k = 1; k <= 3; ++k)
        for (int i = 0; i < 3; ++i)
            g[k][i] = c[k][i] / det;
    for (int i = 0; i < 3; ++i)
        g[0][i] = -(g[1][i] + g[2][i] + g[3][i]);
    const double complex V = (creal(det) < 0.0 ? -det : det) / 6.0;
    const double complex lamV = lam * V * cdt, muV = mu * V * cdt, ml = rho * V * 0.25;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            double complex s = g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    double complex v = lamV * g[a][i] * g[b][j] + muV * g[a][j] * g[b][i];
                    if (i == j)
                        v += muV * s;
                    if (a == b && i == j)
                        v += ml;
                    A[(3 * a + i) * 12 + 3 * b + j] = v;
                }
        }
}

/* dA/dtheta for one element: out[0..143] = dA/dlogE, out[144*(1+k)..] = dA/dX[k]
 * for the 12 vertex coordinates.  Complex step h = 1e-30. */
void oracle_element_derivs(const double *X, double E, double nu, double rho, double dt, double *out)
{
    const double h = 1e-30;
    double complex Xc[12], A[144];
    for (int k = 0; k < 12; ++k)
        Xc[k] = X[k];
    element_complex(Xc, E + I * (E * h), nu, rho, dt, A); /* d/dlogE = E d/dE */
    for (int r = 0; r < 144; ++r)
        out[r] = cimag(A[r]) / h;
    for (int k = 0; k < 12; ++k) {
        Xc[k] = X[k] + I * h;
        element_complex(Xc, E, nu, rho, dt, A);
        for (int r = 0; r < 144; ++r)
            out[144 * (1 + k) + r] = cimag(A[r]) / h;
        Xc[k] = X[k];
    }
}

/* Given gA = dL/dvalues on every pattern slot, accumulate
 *   g_logE[e] = sum_rc gA[slot(r,c)] dA_e[r][c]/dlogE          (active e, else 0)
 *   g_x[3i+k] = sum over active e holding i, ascending, of
 *               sum_rc gA[slot(r,c)] dA_e[r][c]/dx_{i,k}
 * with derivatives by complex step. */
int oracle_adjoint(int64_t n_nodes, const double *x, int64_t n_tets, const int32_t *tets,
                   const double *E, double nu, double rho, double dt, const uint8_t *mask,
                   const int32_t *rowptr, const int32_t *colidx, const double *gA,
                   double *g_logE, double *g_x)
{
    for (int64_t s = 0; s < 3 * n_nodes; ++s)
        g_x[s] = 0.0;
    double X[12], dA[13 * 144], ga[144];
    for (int64_t e = 0; e < n_tets; ++e) {
        g_logE[e] = 0.0;
        if (!mask[e])
            continue;
        const int32_t *t = tets + 4 * e;
        gather_X(x, t, X);
        for (int r = 0; r < 12; ++r)
            for (int c = 0; c < 12; ++c) {
                int64_t s = find_slot(rowptr, colidx, 3 * (int64_t)t[r / 3] + r % 3,
                                      3 * (int64_t)t[c / 3] + c % 3);
                if (s < 0)
                    return OR_ENOSLOT;
                ga[r * 12 + c] = gA[s];
            }
        oracle_element_derivs(X, E[e], nu, rho, dt, dA);
        double acc = 0.0;
        for (int r = 0; r < 144; ++r)
            acc += ga[r] * dA[r];
        g_logE[e] = acc;
        for (int k = 0; k < 12; ++k) {
            double a = 0.0;
            for (int r = 0; r < 144; ++r)
                a += ga[r] * dA[144 * (1 + k) + r];
            g_x[3 * (int64_t)t[k / 3] + k % 3] += a;
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Jacobi-preconditioned conjugate gradients (Sec. 4: CG with diagonal      */
/* preconditioning), on the dofs whose diagonal entry is nonzero; the other */
/* dofs (nodes with no active tet) are held at 0.                           */
/* ------------------------------------------------------------------------ */

void oracle_spmv(int64_t n_rows, const int32_t *rowptr, const int32_t *colidx, const double *vals,
                 const double *v, double *out)
{
    for (int64_t r = 0; r < n_rows; ++r) {
        double acc = 0.0;
        for (int64_t s = rowptr[r]; s < rowptr[r + 1]; ++s)
            acc += vals[s] * v[colidx[s]];
        out[r] = acc;
    }
}

static double dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        s += a[i] * b[i];
    return s;
}

int oracle_pcg(int64_t n_rows, const int32_t *rowptr, const int32_t *colidx, const double *vals,
               const double *b, double *xout, double rtol, int max_iter, int *iters, double *relres)
{
    double *dinv = malloc(sizeof(double) * n_rows), *r = malloc(sizeof(double) * n_rows);
    double *z = malloc(sizeof(double) * n_rows), *p = malloc(sizeof(double) * n_rows);
    double *q = malloc(sizeof(double) * n_rows);
    if (!dinv || !r || !z || !p || !q) {
        free(dinv); free(r); free(z); free(p); free(q);
        return OR_ENOMEM;
    }
    for (int64_t i = 0; i < n_rows; ++i) {
        int64_t s = find_slot(rowptr, colidx, i, i);
        double d = s >= 0 ? vals[s] : 0.0;
        dinv[i] = d != 0.0 ? 1.0 / d : 0.0;
        xout[i] = 0.0;
        r[i] = d != 0.0 ? b[i] : 0.0;
        z[i] = r[i] * dinv[i];
        p[i] = z[i];
    }
    const double bnorm = sqrt(dot(n_rows, r, r));
    double rz = dot(n_rows, r, z), rn = bnorm;
    int it = 0;
    if (bnorm == 0.0) {
        *iters = 0;
        *relres = 0.0;
        free(dinv); free(r); free(z); free(p); free(q);
        return OR_OK;
    }
    while (it < max_iter) {
        oracle_spmv(n_rows, rowptr, colidx, vals, p, q);
        for (int64_t i = 0; i < n_rows; ++i)
            if (dinv[i] == 0.0)
                q[i] = 0.0;
        const double alpha = rz / dot(n_rows, p, q);
        for (int64_t i = 0; i < n_rows; ++i) {
            xout[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        ++it;
        rn = sqrt(dot(n_rows, r, r));
        if (rn <= rtol * bnorm)
            break;
        for (int64_t i = 0; i < n_rows; ++i)
            z[i] = r[i] * dinv[i];
        const double rz_new = dot(n_rows, r, z);
        const double beta = rz_new / rz;
        rz = rz_new;
        for (int64_t i = 0; i < n_rows; ++i)
            p[i] = z[i] + beta * p[i];
    }
    *iters = it;
    *relres = rn / bnorm;
    free(dinv); free(r); free(z); free(p); free(q);
    return OR_OK;
}
