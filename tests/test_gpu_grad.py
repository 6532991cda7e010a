"""GPU adjoint and CG against the oracle, finite differences and exact identities.

The objective is compliance L = f^T u with A u = f (A symmetric, so the
adjoint state is u itself and dL/dvalues = -u u^T on the pattern).  The
GPU adjoint (hand reverse-mode) is compared entry by entry with the
oracle's complex-step route at the same slot cotangents, within per-entry
rounding bounds (tests/bounds.py), with exact-difference central finite
differences, and with the identities G2-G5 that follow from the structure
of A = M + dt^2 K:
  G2 dL/dlogE_e = -dt^2 u_e^T K_e u_e <= 0,   G3 sum_e dL/dlogE_e = u^T M u - L,
  G4 sum_i dL/dx_i = 0,   G5 sum_i x_i . dL/dx_i = -(dt^2 u^T K u + 3 u^T M u).
The CG iterates are compared with the oracle PCG's at fixed iteration
counts, dof by dof, within a first-order bound on each side's rounding.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2605_11673_amd import workloads as W
from tests.bounds import U, adjoint_tolerances, pcg_bound

pytestmark = pytest.mark.gpu


def S():
    from paper_2605_11673_amd import stafem
    return stafem


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float64).view(np.uint64)


def small_case(seed=0):
    w = W.make_fracture(seed=seed, n=5, counts=[20, 40, 30])
    mask = w.mask_after(2)
    f = W.loads_for(w, mask, seed)
    return w, mask, f


def build_at(w, mask):
    asm = S().Assembler(w.x, w.tets, w.E, w.nu, w.rho, w.dt, mask)
    return asm


def within(got, want, tol, what):
    """Entry by entry: |got - want| <= tol."""
    err = np.abs(got - want)
    bad = np.nonzero(err > tol)
    assert bad[0].size == 0, (f"{what}: {bad[0].size} entries beyond their bound, first {tuple(b[0] for b in bad)}: "
                              f"err {err[bad][0]:.3e} tol {tol[bad][0]:.3e} value {want[bad][0]:.3e}")
    live = tol > 0
    return float((err[live] / tol[live]).max()) if np.any(live) else 0.0


def residual_rows(rowptr, colidx, vals, u, b):
    """b - A u per row, accumulated in extended precision."""
    rows = np.repeat(np.arange(len(rowptr) - 1), np.diff(rowptr))
    prod = vals.astype(np.longdouble) * u.astype(np.longdouble)[colidx]
    Au = np.zeros(len(rowptr) - 1, dtype=np.longdouble)
    np.add.at(Au, rows, prod)
    return (b.astype(np.longdouble) - Au).astype(np.float64)


def check_adjoint_at(asm, w, mask, pat, g, what):
    """GPU adjoint vs the oracle's complex-step adjoint at the same cotangents g, entry by
    entry within the derived rounding bounds; inactive tets get exactly 0."""
    gl, gx = asm.adjoint(torch.from_numpy(g).cuda())
    ol, ox = oracle.adjoint(w.x, w.tets, w.E, w.nu, w.rho, w.dt, mask, pat[0], pat[1], g)
    gl, gx = gl.cpu().numpy(), gx.cpu().numpy()
    tl, tx = adjoint_tolerances(w, mask, pat[0], pat[1], g)
    rl = within(gl, ol, tl, f"{what} dL/dlogE")
    rx = within(gx, ox, tx, f"{what} dL/dx")
    assert np.all(gl[mask == 0] == 0.0)
    print(f"[grad] {what}: worst error / bound: logE {rl:.3e}, x {rx:.3e}", flush=True)
    return gl, gx


def test_adjoint_matches_oracle_random_cotangent():
    """Arbitrary (non-symmetric) slot cotangents: GPU reverse mode vs oracle complex step,
    every tet and every node coordinate within its own bound."""
    w, mask, _ = small_case(1)
    asm = build_at(w, mask)
    pat = oracle.pattern(w.n_nodes, w.tets)
    g = np.random.default_rng(5).standard_normal(asm.nnz)
    check_adjoint_at(asm, w, mask, pat, g, "random cotangents")
    asm.close()


def test_cg_matches_direct_solve():
    """Converged GPU solve against a direct solve, dof by dof: both errors are A^-1 times
    their residuals (computed in extended precision), so the two solutions differ by at
    most the sum of those two error vectors (with a 25% margin for evaluating them in
    float64) plus a few ulp of each entry."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    w, mask, f = small_case(2)
    asm = build_at(w, mask)
    pat = oracle.pattern(w.n_nodes, w.tets)
    vals = asm.values().cpu().numpy()
    b = f.reshape(-1)
    u, it, rr = asm.cg_solve(torch.from_numpy(b).cuda(), rtol=1e-13)
    u = u.cpu().numpy()
    A = sp.csr_matrix((vals, pat[1], pat[0]), shape=(asm.n_rows,) * 2)
    live = A.diagonal() != 0
    Al = A[live][:, live].tocsc()
    ud = np.zeros_like(u)
    ud[live] = spla.spsolve(Al, b[live])
    assert rr <= 1e-13 and it > 0
    err_gpu = np.zeros_like(u)
    err_dir = np.zeros_like(u)
    err_gpu[live] = spla.spsolve(Al, residual_rows(pat[0], pat[1], vals, u, b)[live])
    err_dir[live] = spla.spsolve(Al, residual_rows(pat[0], pat[1], vals, ud, b)[live])
    tol = 1.25 * (np.abs(err_gpu) + np.abs(err_dir)) + 4 * U * np.abs(ud)
    within(u[live], ud[live], tol[live], "converged CG vs direct")
    assert np.all(u[~live] == 0.0)
    # reproducible: a second solve gives the same bits
    u2, it2, _ = asm.cg_solve(torch.from_numpy(f.reshape(-1)).cuda(), rtol=1e-13)
    assert it2 == it and np.array_equal(u2.cpu().numpy(), u)
    asm.close()


def test_cg_iteration_limit():
    """max_iter counts iterations exactly: 0 leaves x = 0 with relative residual 1; after k
    iterations the GPU iterate equals the oracle PCG's k-th iterate dof by dof within the
    first-order bound on the rounding of the recurrence (same algorithm, other summation
    orders); the bound stays meaningful up to about eight iterations."""
    w, mask, f = small_case(3)
    asm = build_at(w, mask)
    pat = oracle.pattern(w.n_nodes, w.tets)
    vals = asm.values().cpu().numpy()
    b = f.reshape(-1)
    fd = torch.from_numpy(b).cuda()
    x0, it0, rr0 = asm.cg_solve(fd, rtol=1e-13, max_iter=0)
    assert it0 == 0 and rr0 == 1.0 and not torch.any(x0)
    for k in (1, 2, 3, 4, 6, 8):
        xk, itk, rrk = asm.cg_solve(fd, rtol=1e-13, max_iter=k)
        ok, oit, orr = oracle.pcg(pat[0], pat[1], vals, b, rtol=1e-13, max_iter=k)
        assert itk == k == oit and rrk > 1e-13
        _, ex = pcg_bound(pat[0], pat[1], vals, b, k)
        r = within(xk.cpu().numpy(), ok, 2 * ex * 1.01 + 1e-300, f"iterate {k}")
        print(f"[cg] iteration {k}: worst error / bound {r:.3e}", flush=True)
        assert abs(rrk - orr) <= 1e-6 * orr
    asm.close()


def compliance_gradient(asm, f_dev, rtol=1e-13):
    u, it, rr = asm.cg_solve(f_dev, rtol=rtol)
    gA = asm.slot_outer(u, u, -1.0)
    gl, gx = asm.adjoint(gA)
    return u, gl, gx, it


def test_compliance_gradient_full_size():
    """384k-tet fracture state after frame 12: the GPU solution's residual row by row; the
    GPU gradient against the oracle's complex-step adjoint at the same cotangents, every
    tet and node coordinate within its rounding bound; identities G2-G5; and
    exact-difference central FD (h = 1e-6) on 20 active tets (logE) and 20 nodes (x, 3
    components each).

    FD: L(+h) - L(-h) = -u_+^T (A_+ - A_-) u_- with u_+/- from GPU solves at the
    perturbed parameters.  For logE, A_+ - A_- = ((E_+ - E_-)/E) dt^2 K_e exactly (A is
    linear in E); forming it by subtracting two rounded matrices would leave an error
    of eps/(2h) * |K_e| |u_e|^2, which swamps tets of floating fragments (large rigid
    u_e, tiny strain energy).  Relative error: per tet |fd - g| / |g|; per node the
    largest component error over the largest component of that node's gradient."""
    Sm = S()
    w, mask, f, tet_s, node_s = W.make_gradient_case(0)
    print(f"[grad] n={w.n_nodes} m={w.n_tets} active={int(mask.sum())}", flush=True)
    asm = build_at(w, mask)
    fd = torch.from_numpy(f.reshape(-1)).cuda()
    u, gl, gx, it = compliance_gradient(asm, fd)
    u_h, gl_h, gx_h = u.cpu().numpy(), gl.cpu().numpy(), gx.cpu().numpy()
    L = float(f.reshape(-1) @ u_h)
    print(f"[grad] GPU CG {it} iterations, L = {L:.12g}", flush=True)

    # oracle: its own rebuild (bitwise), the GPU solution's per-row residual, and its
    # complex-step adjoint at the GPU's cotangents (entry by entry within the bounds)
    pat = oracle.pattern(w.n_nodes, w.tets)
    ov = oracle.rebuild(w.x, w.tets, w.E, w.nu, w.rho, w.dt, mask, *pat)
    assert np.array_equal(ov.view(np.uint64), asm.values().cpu().numpy().view(np.uint64))
    rows = np.repeat(np.arange(3 * w.n_nodes), np.diff(pat[0]))
    live = np.zeros(3 * w.n_nodes, bool)
    live[rows[(pat[1] == rows) & (ov != 0.0)]] = True
    b_live = np.where(live, f.reshape(-1), 0.0)
    res = residual_rows(pat[0], pat[1], ov, u_h, b_live)[live]
    # ||b - A u|| <= rtol ||b|| as the solver measured it bounds every row; the rows'
    # exact residuals may exceed the solver's float64 estimate by the rounding of A u
    kap = np.diff(pat[0])[live]
    slack = 2 * kap * U * np.bincount(rows, weights=np.abs(ov) * np.abs(u_h)[pat[1]], minlength=3 * w.n_nodes)[live]
    assert np.all(np.abs(res) <= 1e-13 * np.linalg.norm(b_live) + slack), "a row's residual exceeds the solver's"
    assert np.all(u_h[~live] == 0.0)
    r = np.repeat(np.arange(3 * w.n_nodes), np.diff(pat[0]))
    gA = -(u_h[r] * u_h[pat[1]])
    gl_o, gx_o = check_adjoint_at(asm, w, mask, pat, gA, "compliance cotangents, full size")
    assert np.array_equal(gl_o.view(np.uint64), gl_h.view(np.uint64))  # same kernels, same input
    assert np.array_equal(gx_o.view(np.uint64), gx_h.view(np.uint64))
    print("[grad] oracle agreement ok", flush=True)

    # identities
    act = mask.astype(bool)
    vM = oracle.rebuild(w.x, w.tets, np.zeros(w.n_tets), w.nu, w.rho, w.dt, mask, *pat)
    vK = oracle.rebuild(w.x, w.tets, w.E, w.nu, 0.0, w.dt, mask, *pat)
    uMu = float(u_h @ oracle.spmv(pat[0], pat[1], vM, u_h))
    uKu = float(u_h @ oracle.spmv(pat[0], pat[1], vK, u_h))
    assert np.all(gl_h[act] <= 1e-12 * np.abs(gl_h).max()) and np.all(gl_h[~act] == 0.0)
    assert abs(gl_h.sum() - (uMu - L)) <= 1e-9 * abs(L)
    assert np.abs(gx_h.sum(0)).max() <= 1e-9 * np.abs(gx_h).max() * np.sqrt(w.n_nodes)
    assert abs((w.x * gx_h).sum() + (uKu + 3 * uMu)) <= 1e-8 * (uKu + 3 * uMu)

    # exact-difference central FD: L(+h) - L(-h) = -u_+^T (A_+ - A_-) u_-
    h = 1e-6
    xd = torch.from_numpy(w.x).cuda()
    Ed = torch.from_numpy(w.E).cuda()

    def solve_with(E=None, x=None):
        asm.set_params(xd if x is None else x, Ed if E is None else E)
        asm.full_rebuild()
        return asm.cg_solve(fd, rtol=1e-13)[0].cpu().numpy()

    def local(ring, xp, xm, Ep, Em, up, um):
        acc = 0.0
        for e in ring:
            t = w.tets[e]
            if Ep is Em:  # x perturbed: A_+ - A_- by subtraction
                dA = (oracle.element_matrix(xp[t], w.E[e], w.nu, w.rho, w.dt)
                      - oracle.element_matrix(xm[t], w.E[e], w.nu, w.rho, w.dt))
            else:  # logE perturbed: A is linear in E, A_+ - A_- = (E_+ - E_-)/E dt^2 K_e
                dA = ((Ep[e] - Em[e]) / w.E[e]) * oracle.element_matrix(w.x[t], w.E[e], w.nu, 0.0, w.dt)
            dof = (3 * t[:, None] + np.arange(3)[None, :]).reshape(-1)
            acc += up[dof] @ dA @ um[dof]
        return -acc / (2 * h)

    worst = 0.0
    for e in tet_s:
        Ep, Em = w.E.copy(), w.E.copy()
        Ep[e] = np.exp(np.log(w.E[e]) + h)
        Em[e] = np.exp(np.log(w.E[e]) - h)
        up = solve_with(E=torch.from_numpy(Ep).cuda())
        um = solve_with(E=torch.from_numpy(Em).cuda())
        fdv = local([e], w.x, w.x, Ep, Em, up, um)
        worst = max(worst, abs(fdv - gl_h[e]) / abs(gl_h[e]))
    print(f"[grad] logE FD worst relative error {worst:.3e}", flush=True)
    assert worst < 1e-6
    worst = 0.0
    for i in node_s:
        ring = [e for e in np.nonzero(np.any(w.tets == i, axis=1))[0] if mask[e]]
        for k in range(3):
            xp, xm = w.x.copy(), w.x.copy()
            xp[i, k] += h
            xm[i, k] -= h
            up = solve_with(x=torch.from_numpy(xp).cuda())
            um = solve_with(x=torch.from_numpy(xm).cuda())
            fdv = local(ring, xp, xm, w.E, w.E, up, um)
            worst = max(worst, abs(fdv - gx_h[i, k]) / np.abs(gx_h[i]).max())
    print(f"[grad] x FD worst relative error {worst:.3e}", flush=True)
    assert worst < 1e-6
    asm.close()


def test_autograd_compliance_matches_adjoint():
    """L = f . u through assemble() and solve(): .backward() gives the adjoint-kernel gradient."""
    from paper_2605_11673_amd.autograd import assemble, solve
    w, mask, f = small_case(3)
    asm = build_at(w, mask)
    logE = torch.from_numpy(np.log(w.E)).cuda().requires_grad_(True)
    x = torch.from_numpy(w.x).cuda().requires_grad_(True)
    fd = torch.from_numpy(f.reshape(-1)).cuda()
    vals = assemble(logE, x, asm, torch.from_numpy(w.E).cuda())
    pat = oracle.pattern(w.n_nodes, w.tets)
    want = oracle.rebuild(w.x, w.tets, w.E, w.nu, w.rho, w.dt, mask, *pat)
    assert np.array_equal(vals.detach().cpu().numpy().view(np.uint64), want.view(np.uint64))
    u = solve(vals, fd, asm, 1e-13)
    L = (fd * u).sum()
    L.backward()
    # the same solves and kernels without autograd: the same bits
    u2, gl, gx, _ = compliance_gradient(asm, fd)
    assert np.array_equal(logE.grad.cpu().numpy().view(np.uint64), gl.cpu().numpy().view(np.uint64))
    assert np.array_equal(x.grad.cpu().numpy().view(np.uint64), gx.cpu().numpy().view(np.uint64))
    asm.close()


def test_batch_adjoint_equals_each_mesh_alone():
    """The adjoint of a batched context, whose meshes' tet ranges do not fall on the element
    pass's chunk boundaries (and whose chunks are ordered per mesh), equals each mesh's own
    adjoint bit for bit after a few frames of every mesh's stream."""
    Sm = S()
    ws = W.make_batch(seed=4, count=5, frames=6, sizes=[2, 5, 3, 1, 4])
    b = Sm.Batch.from_workloads(ws)
    off = b.offsets()
    assert any(int(t) % 16 for t in off["tet"][1:-1])
    singles = [Sm.Assembler.from_workload(w) for w in ws]
    for t in range(4):
        gi = np.concatenate([w.frames[t][0].astype(np.int64) + off["tet"][j] for j, w in enumerate(ws)])
        gs = np.concatenate([w.frames[t][1] for w in ws])
        b.apply_edits(*Sm.upload_frame(gi.astype(np.int32), gs.astype(np.uint8)))
        for a, w in zip(singles, ws):
            a.apply_edits(*Sm.upload_frame(*w.frames[t]))
    rng = np.random.default_rng(11)
    g = rng.standard_normal(b.nnz)
    gl, gx = b.adjoint(torch.from_numpy(g).cuda())
    gl, gx = gl.cpu().numpy(), gx.cpu().numpy().reshape(-1)
    for j, a in enumerate(singles):
        sl, sx = a.adjoint(torch.from_numpy(g[off["nnz"][j]:off["nnz"][j + 1]].copy()).cuda())
        assert np.array_equal(bits(gl[off["tet"][j]:off["tet"][j + 1]]), bits(sl.cpu().numpy())), j
        assert np.array_equal(bits(gx[3 * off["node"][j]:3 * off["node"][j + 1]]), bits(sx.cpu().numpy().reshape(-1))), j
        a.close()
    assert b.status_sync() == Sm.STA_OK
    b.close()
