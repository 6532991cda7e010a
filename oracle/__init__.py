"""CPU oracle for exact streaming assembly (TEST INFRASTRUCTURE ONLY).

Plain, slow, obviously-correct reference for what the GPU path computes:
the superset sparsity pattern, the rebuild of A_t = M_t + dt^2 K_t from the
current active mask (paper Sec. 3.3 invariant, Sec. 3.4 eq. (8)), the
gradient of an objective through the assembled values, and a Jacobi-PCG
solve (Sec. 4); and, in ``proxy.py``, the graph-Laplacian proxy operator of
Sec. 3.1 (edge multiplicities, binary edge activity, L_t + eps I).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU
library: the arithmetic lives in ``oracle.c`` (built with gcc, contraction
off), the patterns in ``pattern.py`` and ``proxy.py`` (numpy).

Functions whose parity has no external pin are marked "parity unpinned" in
their docstring; at present every function is pinned by a test in
``tests/test_oracle_*.py`` (closed forms, invariants, brute force).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .pattern import pattern, csr_to_dense  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC", "-shared", "-fopenmp"]


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_i32 = ctypes.POINTER(ctypes.c_int32)
_u8 = ctypes.POINTER(ctypes.c_uint8)
_i64 = ctypes.c_int64


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_SO)
        L.oracle_element.argtypes = [_d, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, _d]
        L.oracle_element.restype = None
        L.oracle_det.argtypes = [_d]
        L.oracle_det.restype = ctypes.c_double
        L.oracle_rebuild.argtypes = [_i64, _d, _i64, _i32, _d, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, _u8, _i32, _i32, _i64, _d]
        L.oracle_rebuild.restype = ctypes.c_int
        L.oracle_rebuild_weighted.argtypes = [_i64, _d, _i64, _i32, _d, ctypes.c_double, ctypes.c_double,
                                              ctypes.c_double, _d, ctypes.c_int, _i32, _i32, _i64, _d]
        L.oracle_rebuild_weighted.restype = ctypes.c_int
        L.oracle_rebuild_rows.argtypes = [_i64, _d, _i64, _i32, _d, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, _u8, _i32, _i32, _d, ctypes.POINTER(ctypes.c_int)]
        L.oracle_rebuild_rows.restype = ctypes.c_int
        L.oracle_lumped_mass.argtypes = [_i64, _d, _i64, _i32, ctypes.c_double, _u8, _d]
        L.oracle_lumped_mass.restype = None
        L.oracle_dense.argtypes = [_i64, _d, _i64, _i32, _d, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, _u8, _d]
        L.oracle_dense.restype = None
        L.oracle_element_derivs.argtypes = [_d, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double, _d]
        L.oracle_element_derivs.restype = None
        L.oracle_adjoint.argtypes = [_i64, _d, _i64, _i32, _d, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, _u8, _i32, _i32, _d, _d, _d]
        L.oracle_adjoint.restype = ctypes.c_int
        L.oracle_spmv.argtypes = [_i64, _i32, _i32, _d, _d, _d]
        L.oracle_spmv.restype = None
        L.oracle_pcg.argtypes = [_i64, _i32, _i32, _d, _d, _d, ctypes.c_double, ctypes.c_int,
                                 ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]
        L.oracle_pcg.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32a(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _u8a(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


def element_matrix(X, E, nu, rho, dt) -> np.ndarray:
    """12x12 element matrix A_e = dt^2 K_e + M_e of one tet; X is (4, 3)."""
    X = _f64(X).reshape(12)
    A = np.empty(144)
    lib().oracle_element(_p(X, _d), float(E), float(nu), float(rho), float(dt), _p(A, _d))
    return A.reshape(12, 12)


def det(X) -> float:
    X = _f64(X).reshape(12)
    return float(lib().oracle_det(_p(X, _d)))


def rebuild(x, tets, E, nu, rho, dt, mask, rowptr, colidx) -> np.ndarray:
    """CSR values of A_t rebuilt from scratch on the active mask (eq. (8), ascending ids)."""
    x, tets, E, mask = _f64(x), _i32a(tets), _f64(E), _u8a(mask)
    rowptr, colidx = _i32a(rowptr), _i32a(colidx)
    nnz = int(rowptr[-1])
    vals = np.empty(nnz)
    rc = lib().oracle_rebuild(x.shape[0], _p(x, _d), tets.shape[0], _p(tets, _i32), _p(E, _d),
                              float(nu), float(rho), float(dt), _p(mask, _u8),
                              _p(rowptr, _i32), _p(colidx, _i32), nnz, _p(vals, _d))
    if rc != 0:
        raise RuntimeError(f"oracle_rebuild failed ({rc}): pattern lacks an entry")
    return vals


def rebuild_rows(x, tets, E, nu, rho, dt, mask, rowptr, colidx):
    """The rebuild of ``rebuild`` computed row by row on all host threads (OpenMP; the
    thread count follows OMP_NUM_THREADS).  Same terms in the same order per slot, so
    the values are bitwise those of ``rebuild``.  Returns (values, threads used)."""
    x, tets, E, mask = _f64(x), _i32a(tets), _f64(E), _u8a(mask)
    rowptr, colidx = _i32a(rowptr), _i32a(colidx)
    vals = np.empty(int(rowptr[-1]))
    th = ctypes.c_int(0)
    rc = lib().oracle_rebuild_rows(x.shape[0], _p(x, _d), tets.shape[0], _p(tets, _i32), _p(E, _d),
                                   float(nu), float(rho), float(dt), _p(mask, _u8),
                                   _p(rowptr, _i32), _p(colidx, _i32), _p(vals, _d), ctypes.byref(th))
    if rc != 0:
        raise RuntimeError(f"oracle_rebuild_rows failed ({rc})")
    return vals, int(th.value)


def rebuild_weighted(x, tets, E, nu, rho, dt, weights, rowptr, colidx, count_only=False) -> np.ndarray:
    """For error bounds: per CSR entry, the sum over candidates e with weights[e] != 0 of
    weights[e] * |A_e term| (or of weights[e] alone with count_only)."""
    x, tets, E, w = _f64(x), _i32a(tets), _f64(E), _f64(weights)
    rowptr, colidx = _i32a(rowptr), _i32a(colidx)
    nnz = int(rowptr[-1])
    vals = np.empty(nnz)
    rc = lib().oracle_rebuild_weighted(x.shape[0], _p(x, _d), tets.shape[0], _p(tets, _i32), _p(E, _d),
                                       float(nu), float(rho), float(dt), _p(w, _d), int(bool(count_only)),
                                       _p(rowptr, _i32), _p(colidx, _i32), nnz, _p(vals, _d))
    if rc != 0:
        raise RuntimeError(f"oracle_rebuild_weighted failed ({rc}): pattern lacks an entry")
    return vals


def dense(x, tets, E, nu, rho, dt, mask) -> np.ndarray:
    """Dense (3n x 3n) textbook assembly of eq. (8); tiny meshes only."""
    x, tets, E, mask = _f64(x), _i32a(tets), _f64(E), _u8a(mask)
    n = x.shape[0]
    D = np.empty((3 * n, 3 * n))
    lib().oracle_dense(n, _p(x, _d), tets.shape[0], _p(tets, _i32), _p(E, _d),
                       float(nu), float(rho), float(dt), _p(mask, _u8), _p(D, _d))
    return D


def element_derivs(X, E, nu, rho, dt) -> np.ndarray:
    """(13, 12, 12): dA_e/dlogE then dA_e/dX_k for the 12 vertex coordinates (complex step)."""
    X = _f64(X).reshape(12)
    out = np.empty(13 * 144)
    lib().oracle_element_derivs(_p(X, _d), float(E), float(nu), float(rho), float(dt), _p(out, _d))
    return out.reshape(13, 12, 12)


def adjoint(x, tets, E, nu, rho, dt, mask, rowptr, colidx, gA):
    """(g_logE (m,), g_x (n, 3)) from slot cotangents gA, by complex-step element derivatives."""
    x, tets, E, mask = _f64(x), _i32a(tets), _f64(E), _u8a(mask)
    rowptr, colidx, gA = _i32a(rowptr), _i32a(colidx), _f64(gA)
    n, m = x.shape[0], tets.shape[0]
    gl = np.empty(m)
    gx = np.empty(3 * n)
    rc = lib().oracle_adjoint(n, _p(x, _d), m, _p(tets, _i32), _p(E, _d), float(nu), float(rho),
                              float(dt), _p(mask, _u8), _p(rowptr, _i32), _p(colidx, _i32),
                              _p(gA, _d), _p(gl, _d), _p(gx, _d))
    if rc != 0:
        raise RuntimeError(f"oracle_adjoint failed ({rc})")
    return gl, gx.reshape(n, 3)


def spmv(rowptr, colidx, vals, v) -> np.ndarray:
    rowptr, colidx, vals, v = _i32a(rowptr), _i32a(colidx), _f64(vals), _f64(v)
    out = np.empty(len(rowptr) - 1)
    lib().oracle_spmv(len(rowptr) - 1, _p(rowptr, _i32), _p(colidx, _i32), _p(vals, _d), _p(v, _d),
                      _p(out, _d))
    return out


def pcg(rowptr, colidx, vals, b, rtol=1e-12, max_iter=20000):
    """Jacobi-PCG on the dofs with a nonzero diagonal; returns (x, iters, relres)."""
    rowptr, colidx, vals, b = _i32a(rowptr), _i32a(colidx), _f64(vals), _f64(b)
    n = len(rowptr) - 1
    x = np.empty(n)
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    rc = lib().oracle_pcg(n, _p(rowptr, _i32), _p(colidx, _i32), _p(vals, _d), _p(b, _d), _p(x, _d),
                          float(rtol), int(max_iter), ctypes.byref(it), ctypes.byref(rr))
    if rc != 0:
        raise RuntimeError(f"oracle_pcg failed ({rc})")
    return x, int(it.value), float(rr.value)


def lumped_mass(x, tets, rho, mask) -> np.ndarray:
    """M_t per dof (3 per node): active tets' rho V / 4, summed in ascending tet id."""
    x, tets, mask = _f64(x), _i32a(tets), _u8a(mask)
    m = np.empty(3 * x.shape[0])
    lib().oracle_lumped_mass(x.shape[0], _p(x, _d), tets.shape[0], _p(tets, _i32), float(rho), _p(mask, _u8),
                             _p(m, _d))
    return m


def euler_step(rowptr, colidx, vals, m, u, v, f, h, rtol=1e-12, max_iter=20000):
    """One implicit-Euler step (Sec. 6.2 eq. (9)): solve (M_t + h^2 K_t) u' = M_t (u + h v) + h^2 f
    with the oracle PCG (vals = the CSR values of M_t + h^2 K_t, m = M_t per dof), then
    v' = (u' - u) / h.  Returns (u', v', iters, relres)."""
    b = m * (u + h * v) + (h * h) * f
    u1, it, rr = pcg(rowptr, colidx, vals, b, rtol=rtol, max_iter=max_iter)
    return u1, (u1 - u) / h, it, rr


def rebuild_workload(w, mask=None, pat=None):
    """Oracle values for a generated workload at a given mask (default: its initial mask)."""
    if pat is None:
        pat = pattern(w.n_nodes, w.tets)
    if mask is None:
        mask = w.mask0
    return rebuild(w.x, w.tets, w.E, w.nu, w.rho, w.dt, mask, pat[0], pat[1])
