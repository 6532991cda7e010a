"""Python binding of libstafem.so (the C ABI in include/stafem.h).

Argument marshalling only: every step of the assembly runs in the HIP
library.  PyTorch supplies device memory for edit lists and results and the
current HIP stream.  torch is imported before the library is loaded so that
both bind to the one HIP runtime torch ships (same soname).

There is no CPU fallback: if libstafem.so is missing or no GPU is visible,
the first call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstafem.so")

STATUS = {
    0: "STA_OK", -1: "STA_EINVAL", -2: "STA_ENOMEM", -3: "STA_EHIP", -4: "STA_EDEGENERATE",
    -5: "STA_ESTALE", -6: "STA_ERANGE", -7: "STA_EDUP", -8: "STA_ETIMEOUT",
}
STA_OK, STA_EINVAL, STA_ENOMEM, STA_EHIP, STA_EDEGENERATE, STA_ESTALE, STA_ERANGE, STA_EDUP = 0, -1, -2, -3, -4, -5, -6, -7
STA_ETIMEOUT = -8


class StafemError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i64p = ctypes.POINTER(ctypes.c_int64)
_dbl = ctypes.c_double
_int = ctypes.c_int

# name -> (restype, argtypes); mirrors include/stafem.h
SIGNATURES = {
    "sta_build_pattern": (_int, [_vp, _i64, _vp, _i64, _vp, _dbl, _dbl, _dbl, _vp, _vp, ctypes.POINTER(_vp)]),
    "sta_full_rebuild": (_int, [_vp, _vp]),
    "sta_apply_edits": (_int, [_vp, _vp, _vp, _i64, _vp]),
    "sta_apply_edits_dev": (_int, [_vp, _vp, _vp, _vp, _i64, _vp]),
    "sta_apply_edits_delta": (_int, [_vp, _vp, _vp, _i64, _vp, _vp]),
    "sta_values_ptr": (_vp, [_vp]),
    "sta_copy_values": (_int, [_vp, _vp, _vp]),
    "sta_sizes": (_int, [_vp, _i64p, _i64p, _i64p, _i64p]),
    "sta_pattern_ptrs": (_int, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp)]),
    "sta_pattern_host": (_int, [_vp, _vp, _vp]),
    "sta_last_frame_stats": (_int, [_vp, _vp, _i64p, _int]),
    "sta_enable_kernel_timing": (_int, [_vp, _int]),
    "sta_kernel_times": (_int, [_vp, _vp, _i64p, ctypes.POINTER(_dbl)]),
    "sta_set_params": (_int, [_vp, _vp, _vp, _vp]),
    "sta_adjoint": (_int, [_vp, _vp, _vp, _vp, _vp]),
    "sta_adjoint_noalloc": (_int, [_vp, _vp, _vp, _vp, _vp]),
    "sta_slot_outer": (_int, [_vp, _vp, _vp, _dbl, _vp, _vp]),
    "sta_cg_solve": (_int, [_vp, _vp, _vp, _vp, _dbl, _int, _vp, ctypes.POINTER(_int), ctypes.POINTER(_dbl)]),
    "sta_lumped_mass": (_int, [_vp, _vp, _vp]),
    "sta_euler_step": (_int, [_vp, _vp, _vp, _vp, _dbl, _int, _vp, ctypes.POINTER(_int), ctypes.POINTER(_dbl)]),
    "sta_components": (_int, [_vp, _vp, _i64p, _vp]),
    "sta_face_components": (_int, [_vp, _vp, _i64p, _vp]),
    "sta_set_config": (_int, [_vp, _int, _int, _int, _int, _int, _int, _int]),
    "sta_get_config": (_int, [_vp, ctypes.POINTER(_int)]),
    "sta_set_barrier_spin_limit": (_int, [_vp, _i64]),
    "sta_audit": (_int, [_vp, _vp, _i64p]),
    "sta_set_bucket_map": (_int, [_vp, _int, _vp, _vp]),
    "sta_get_bucket_map": (_int, [_vp, _int, _vp, _vp, _vp]),
    "sta_autotune": (_int, [_vp, _vp, _vp, _i64, _int, _vp, ctypes.c_char_p, _i64]),
    "sta_batch_build": (_int, [_int, _vp, _vp, _vp, _vp, _vp, _dbl, _dbl, _dbl, _vp, _vp, ctypes.POINTER(_vp)]),
    "sta_batch_offsets": (_int, [_vp, ctypes.POINTER(_int), _vp, _vp, _vp, _vp, _i64]),
    "sta_latency_probe": (_int, [_vp, ctypes.POINTER(_dbl)]),
    "sta_bandwidth_probe": (_int, [_vp, ctypes.POINTER(_dbl)]),
    "sta_barrier_probe": (_int, [ctypes.POINTER(_dbl)]),
    "sta_status_sync": (_int, [_vp, _vp]),
    "sta_last_error": (ctypes.c_char_p, [_vp]),
    "sta_destroy": (None, [_vp]),
    "sta_proxy_build": (_int, [_vp, _i64, _i64, _vp, _dbl, _vp, ctypes.POINTER(_vp)]),
    "sta_proxy_full_rebuild": (_int, [_vp, _vp]),
    "sta_proxy_apply_edits": (_int, [_vp, _vp, _vp, _i64, _vp]),
    "sta_proxy_apply_edits_dev": (_int, [_vp, _vp, _vp, _i64, _vp, _vp]),
    "sta_proxy_sizes": (_int, [_vp, _i64p, _i64p, _i64p]),
    "sta_proxy_values_ptr": (_vp, [_vp]),
    "sta_proxy_counts_ptr": (_vp, [_vp]),
    "sta_proxy_degree_ptr": (_vp, [_vp]),
    "sta_proxy_copy_state": (_int, [_vp, _vp, _vp, _vp, _vp]),
    "sta_proxy_pattern_ptrs": (_int, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp)]),
    "sta_proxy_pattern_host": (_int, [_vp, _vp, _vp, _vp]),
    "sta_proxy_last_frame_stats": (_int, [_vp, _vp, _i64p]),
    "sta_proxy_status_sync": (_int, [_vp, _vp]),
    "sta_proxy_last_error": (ctypes.c_char_p, [_vp]),
    "sta_proxy_destroy": (None, [_vp]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libstafem.so and declare its signatures; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built: run `python -m paper_2605_11673_amd.build`")
    L = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _stream_handle(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return _vp(s.cuda_stream)


def _check(code: int, ctx=None):
    if code != STA_OK:
        msg = load().sta_last_error(ctx)
        raise StafemError(code, msg.decode() if msg else "")


def _dev_ptr(t: torch.Tensor) -> _vp:
    return _vp(t.data_ptr())


def _need_f64(t: torch.Tensor, n: int):
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
        raise TypeError(f"expected a contiguous float64 CUDA tensor of {n} elements")


class Assembler:
    """One superset mesh: its fixed pattern, element contributions and current A_t.

    x (n, 3) float64, tets (m, 4) int32, E (m,) float64, mask0 (m,) uint8 are
    host arrays; they are copied into the context.
    """

    def __init__(self, x, tets, E, nu, rho, dt, mask0, stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the HIP assembly path needs an MI355X")
        L = load()
        x = np.ascontiguousarray(x, dtype=np.float64)
        tets = np.ascontiguousarray(tets, dtype=np.int32)
        E = np.ascontiguousarray(E, dtype=np.float64)
        mask0 = np.ascontiguousarray(mask0, dtype=np.uint8)
        self.n_nodes, self.n_tets = int(x.shape[0]), int(tets.shape[0])
        ctx = _vp()
        code = L.sta_build_pattern(x.ctypes.data, self.n_nodes, tets.ctypes.data, self.n_tets, E.ctypes.data,
                                   float(nu), float(rho), float(dt), mask0.ctypes.data,
                                   _stream_handle(stream), ctypes.byref(ctx))
        _check(code, None)
        self._ctx = ctx
        self.nu, self.rho, self.dt = float(nu), float(rho), float(dt)
        r, z, d, o = _i64(), _i64(), _i64(), _i64()
        _check(L.sta_sizes(ctx, ctypes.byref(r), ctypes.byref(z), ctypes.byref(d), ctypes.byref(o)), ctx)
        self.n_rows, self.nnz, self.n_diag_blocks, self.n_off_blocks = r.value, z.value, d.value, o.value

    @classmethod
    def from_workload(cls, w, stream=None):
        return cls(w.x, w.tets, w.E, w.nu, w.rho, w.dt, w.mask0, stream)

    # -- lifetime -------------------------------------------------------------
    def close(self):
        if getattr(self, "_ctx", None):
            load().sta_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._ctx

    # -- the hot path ---------------------------------------------------------
    def full_rebuild(self, stream=None):
        _check(load().sta_full_rebuild(self._ctx, _stream_handle(stream)), self._ctx)

    def apply_edits(self, ids: torch.Tensor, states: torch.Tensor, stream=None):
        """ids: int32 CUDA tensor, states: uint8 CUDA tensor (same length)."""
        if ids.numel() != states.numel():
            raise ValueError("ids and states differ in length")
        if ids.numel() and (ids.dtype != torch.int32 or states.dtype != torch.uint8 or not ids.is_cuda
                            or not states.is_cuda or not ids.is_contiguous() or not states.is_contiguous()):
            raise TypeError("ids must be contiguous int32 and states contiguous uint8 CUDA tensors")
        _check(load().sta_apply_edits(self._ctx, _dev_ptr(ids) if ids.numel() else None,
                                      _dev_ptr(states) if ids.numel() else None, int(ids.numel()),
                                      _stream_handle(stream)), self._ctx)

    def apply_edits_dev(self, ids: torch.Tensor, states: torch.Tensor, n_dev: torch.Tensor, stream=None):
        """Edit count read on the device from n_dev (int32 CUDA tensor, 1 element);
        ids/states are buffers of capacity len(ids).  Graph-capturable."""
        if (ids.dtype != torch.int32 or states.dtype != torch.uint8 or n_dev.dtype != torch.int32
                or not (ids.is_cuda and states.is_cuda and n_dev.is_cuda) or ids.numel() != states.numel()):
            raise TypeError("ids int32, states uint8 (same length) and n_dev int32 CUDA tensors")
        _check(load().sta_apply_edits_dev(self._ctx, _dev_ptr(ids), _dev_ptr(states), _dev_ptr(n_dev),
                                          int(ids.numel()), _stream_handle(stream)), self._ctx)

    def apply_edits_delta(self, ids: torch.Tensor, states: torch.Tensor, n_dev: torch.Tensor | None = None,
                          stream=None):
        """The +/- delta policy (sta_apply_edits_delta): exact only up to rounding."""
        if ids.dtype != torch.int32 or states.dtype != torch.uint8 or ids.numel() != states.numel() \
                or not (ids.is_cuda and states.is_cuda) or (n_dev is not None and n_dev.dtype != torch.int32):
            raise TypeError("ids int32 and states uint8 CUDA tensors of equal length (n_dev int32)")
        nd = _vp(0) if n_dev is None else _dev_ptr(n_dev)
        _check(load().sta_apply_edits_delta(self._ctx, _dev_ptr(ids), _dev_ptr(states), int(ids.numel()), nd,
                                            _stream_handle(stream)), self._ctx)

    def values_ptr(self) -> int:
        return int(load().sta_values_ptr(self._ctx) or 0)

    def values(self, stream=None) -> torch.Tensor:
        """A copy of the current CSR values (float64 CUDA tensor), stream-ordered."""
        out = torch.empty(self.nnz, dtype=torch.float64, device="cuda")
        _check(load().sta_copy_values(self._ctx, _dev_ptr(out), _stream_handle(stream)), self._ctx)
        return out

    def pattern(self):
        """(rowptr, colidx) int32 numpy arrays."""
        rp = np.empty(self.n_rows + 1, dtype=np.int32)
        ci = np.empty(max(self.nnz, 1), dtype=np.int32)
        _check(load().sta_pattern_host(self._ctx, rp.ctypes.data, ci.ctypes.data), self._ctx)
        return rp, ci[: self.nnz]

    def pattern_ptrs(self):
        rp, ci, mk = _vp(), _vp(), _vp()
        _check(load().sta_pattern_ptrs(self._ctx, ctypes.byref(rp), ctypes.byref(ci), ctypes.byref(mk)), self._ctx)
        return rp.value, ci.value, mk.value

    FRAME_STATS = ("diag_blocks", "off_blocks", "diag_incidences", "off_incidences", "touched_slots",
                   "changed", "activated", "edits", "rolled_back")

    def last_frame_stats(self, stream=None) -> dict:
        out = (ctypes.c_int64 * len(self.FRAME_STATS))()
        _check(load().sta_last_frame_stats(self._ctx, _stream_handle(stream), out, len(out)), self._ctx)
        d = dict(zip(self.FRAME_STATS, list(out)))
        d["touched_blocks"] = d["diag_blocks"] + d["off_blocks"]
        d["touched_incidences"] = d["diag_incidences"] + d["off_incidences"]
        return d

    KERNELS = ("element", "reduce", "edits", "touched", "adjoint", "solve", "frame", "delta")

    def enable_kernel_timing(self, on: bool = True):
        _check(load().sta_enable_kernel_timing(self._ctx, 1 if on else 0), self._ctx)

    def kernel_times(self, stream=None) -> dict:
        """{kernel: (launches, total ms)} since the last call; synchronises."""
        n = (ctypes.c_int64 * len(self.KERNELS))()
        ms = (ctypes.c_double * len(self.KERNELS))()
        _check(load().sta_kernel_times(self._ctx, _stream_handle(stream), n, ms), self._ctx)
        return {k: (int(n[i]), float(ms[i])) for i, k in enumerate(self.KERNELS) if n[i]}

    def set_params(self, x: torch.Tensor | None = None, E: torch.Tensor | None = None, stream=None):
        """x: (n, 3) float64 CUDA tensor, E: (m,) float64 CUDA tensor; either may be None."""
        for t in (x, E):
            if t is not None and (t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous()):
                raise TypeError("set_params takes contiguous float64 CUDA tensors")
        _check(load().sta_set_params(self._ctx, _dev_ptr(x) if x is not None else None,
                                     _dev_ptr(E) if E is not None else None, _stream_handle(stream)), self._ctx)

    def adjoint(self, gA: torch.Tensor, stream=None):
        """(dL/dlogE (m,), dL/dx (n, 3)) float64 CUDA tensors from slot cotangents gA (nnz,)."""
        _need_f64(gA, self.nnz)
        gl = torch.empty(self.n_tets, dtype=torch.float64, device="cuda")
        gx = torch.empty((self.n_nodes, 3), dtype=torch.float64, device="cuda")
        _check(load().sta_adjoint(self._ctx, _dev_ptr(gA), _dev_ptr(gl), _dev_ptr(gx), _stream_handle(stream)),
               self._ctx)
        return gl, gx

    def slot_outer(self, a: torch.Tensor, b: torch.Tensor, alpha: float, stream=None) -> torch.Tensor:
        """out[s] = alpha * a[row(s)] * b[col(s)] over the pattern (float64 CUDA, nnz)."""
        _need_f64(a, self.n_rows)
        _need_f64(b, self.n_rows)
        out = torch.empty(self.nnz, dtype=torch.float64, device="cuda")
        _check(load().sta_slot_outer(self._ctx, _dev_ptr(a), _dev_ptr(b), float(alpha), _dev_ptr(out),
                                     _stream_handle(stream)), self._ctx)
        return out

    def cg_solve(self, b: torch.Tensor, values: torch.Tensor | None = None, rtol: float = 1e-12,
                 max_iter: int = 100000, stream=None):
        """Jacobi-PCG on A x = b (A = values, default the context's own); returns (x, iters, relres)."""
        b = b.reshape(-1)
        _need_f64(b, self.n_rows)
        if values is not None:
            _need_f64(values, self.nnz)
        x = torch.empty(self.n_rows, dtype=torch.float64, device="cuda")
        it, rr = ctypes.c_int(0), ctypes.c_double(0.0)
        _check(load().sta_cg_solve(self._ctx, _dev_ptr(values) if values is not None else None, _dev_ptr(b),
                                   _dev_ptr(x), float(rtol), int(max_iter), _stream_handle(stream),
                                   ctypes.byref(it), ctypes.byref(rr)), self._ctx)
        return x, it.value, rr.value

    CONFIG = ("fused", "rebuild_qd", "rebuild_qo", "stream_qd", "stream_qo", "grid_cap", "rebuild_nt")

    def lumped_mass(self, stream=None) -> torch.Tensor:
        """M_t per dof (float64 CUDA tensor, n_rows), stream-ordered."""
        m = torch.empty(self.n_rows, dtype=torch.float64, device="cuda")
        _check(load().sta_lumped_mass(self._ctx, _dev_ptr(m), _stream_handle(stream)), self._ctx)
        return m

    def euler_step(self, u: torch.Tensor, v: torch.Tensor, f: torch.Tensor, rtol: float = 1e-10,
                   max_iter: int = 20000, stream=None):
        """One implicit-Euler step of eq. (9) with h = dt; u, v updated in place.
        Returns (iterations, relative residual)."""
        for t in (u, v, f):
            _need_f64(t, self.n_rows)
        it, rr = _int(0), _dbl(0.0)
        _check(load().sta_euler_step(self._ctx, _dev_ptr(u), _dev_ptr(v), _dev_ptr(f), float(rtol), int(max_iter),
                                     _stream_handle(stream), ctypes.byref(it), ctypes.byref(rr)), self._ctx)
        return it.value, rr.value

    def components(self, adjacency: str = "vertex", stream=None):
        """(labels int32 CUDA tensor (n_tets,), number of components); synchronises.
        adjacency "vertex" (sta_components: labels are smallest vertex ids) or "face"
        (sta_face_components: labels are smallest tet ids)."""
        fn = {"vertex": load().sta_components, "face": load().sta_face_components}[adjacency]
        lab = torch.empty(max(self.n_tets, 1), dtype=torch.int32, device="cuda")
        k = _i64()
        _check(fn(self._ctx, _dev_ptr(lab), ctypes.byref(k), _stream_handle(stream)), self._ctx)
        return lab[: self.n_tets], k.value

    def set_config(self, fused=0, rebuild_qd=1, rebuild_qo=1, stream_qd=1, stream_qo=1, grid_cap=0, rebuild_nt=0):
        _check(load().sta_set_config(self._ctx, int(fused), int(rebuild_qd), int(rebuild_qo), int(stream_qd),
                                     int(stream_qo), int(grid_cap), int(rebuild_nt)), self._ctx)

    def get_config(self) -> dict:
        out = (ctypes.c_int * 7)()
        _check(load().sta_get_config(self._ctx, out), self._ctx)
        return dict(zip(self.CONFIG, list(out)))

    def audit(self, stream=None) -> dict:
        """Compare the maintained state with a rebuild (sta_audit); synchronises."""
        out = (ctypes.c_int64 * 2)()
        _check(load().sta_audit(self._ctx, _stream_handle(stream), out), self._ctx)
        return {"values_differing": int(out[0]), "tets_differing": int(out[1])}

    def set_barrier_spin_limit(self, polls: int):
        """Polls before the fused frame's grid barrier gives up (0: the default); a
        failure-injection aid for tests of STA_ETIMEOUT."""
        _check(load().sta_set_barrier_spin_limit(self._ctx, int(polls)), self._ctx)

    def set_bucket_map(self, which: str, diag, off):
        """Slot mapping per incidence-length bucket (see sta_set_bucket_map): which is
        "rebuild" or "stream", diag three group sizes in {1, 4, 16} (kappa <= 8, 9..32,
        > 32), off two in {1, 4} (kappa <= 8, > 8)."""
        qd = (ctypes.c_int * 3)(*[int(x) for x in diag])
        qo = (ctypes.c_int * 2)(*[int(x) for x in off])
        _check(load().sta_set_bucket_map(self._ctx, {"rebuild": 0, "stream": 1}[which], qd, qo), self._ctx)

    def bucket_map(self, which: str) -> dict:
        """The mapping per bucket and the number of blocks in each bucket."""
        qd, qo, nb = (ctypes.c_int * 3)(), (ctypes.c_int * 2)(), (ctypes.c_int64 * 5)()
        _check(load().sta_get_bucket_map(self._ctx, {"rebuild": 0, "stream": 1}[which], qd, qo, nb), self._ctx)
        return {"diag": list(qd), "off": list(qo), "diag_blocks": list(nb)[:3], "off_blocks": list(nb)[3:]}

    def autotune(self, ids: torch.Tensor, states: torch.Tensor, reps: int = 7, stream=None) -> str:
        """Pick slot mappings and frame mode by timing (see sta_autotune); returns the report."""
        buf = ctypes.create_string_buffer(8192)
        _check(load().sta_autotune(self._ctx, _dev_ptr(ids), _dev_ptr(states), int(ids.numel()), int(reps),
                                   _stream_handle(stream), buf, len(buf)), self._ctx)
        return buf.value.decode()

    def offsets(self) -> dict:
        """Per-mesh node / tet / row / value offsets (k+1 entries each)."""
        k = ctypes.c_int(0)
        _check(load().sta_batch_offsets(self._ctx, ctypes.byref(k), None, None, None, None, 0), self._ctx)
        arrs = [np.zeros(k.value + 1, dtype=np.int64) for _ in range(4)]
        _check(load().sta_batch_offsets(self._ctx, ctypes.byref(k), *[a.ctypes.data for a in arrs], k.value + 1),
               self._ctx)
        return dict(zip(("node", "tet", "row", "nnz"), arrs))

    def status_sync(self, stream=None) -> int:
        """Synchronise and return (and clear) the first device-detected error code."""
        return int(load().sta_status_sync(self._ctx, _stream_handle(stream)))

    def last_error(self) -> str:
        m = load().sta_last_error(self._ctx)
        return m.decode() if m else ""


class Batch(Assembler):
    """Many independent meshes as one context (their disjoint union).

    Mesh j's tet t is global tet ``tet_off[j] + t``; its CSR rows and values
    are the contiguous ranges given by ``offsets()``.  A frame over all meshes
    is one apply_edits / apply_edits_dev call with global ids.
    """

    def __init__(self, meshes, nu, rho, dt, stream=None):
        """meshes: sequence of (x (n,3), tets (m,4), E (m,), mask0 (m,)) host arrays."""
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the HIP assembly path needs an MI355X")
        L = load()
        k = len(meshes)
        keep = []
        xs, ts, Es, ms = (ctypes.c_void_p * k)(), (ctypes.c_void_p * k)(), (ctypes.c_void_p * k)(), (ctypes.c_void_p * k)()
        nn, nt = (ctypes.c_int64 * k)(), (ctypes.c_int64 * k)()
        for j, (x, t, E, m) in enumerate(meshes):
            x = np.ascontiguousarray(x, dtype=np.float64)
            t = np.ascontiguousarray(t, dtype=np.int32)
            E = np.ascontiguousarray(E, dtype=np.float64)
            m = np.ascontiguousarray(m, dtype=np.uint8)
            keep += [x, t, E, m]
            xs[j], ts[j], Es[j], ms[j] = x.ctypes.data, t.ctypes.data, E.ctypes.data, m.ctypes.data
            nn[j], nt[j] = x.shape[0], t.shape[0]
        ctx = _vp()
        _check(L.sta_batch_build(k, xs, nn, ts, nt, Es, float(nu), float(rho), float(dt), ms, _stream_handle(stream),
                                 ctypes.byref(ctx)), None)
        self._ctx = ctx
        self.nu, self.rho, self.dt = float(nu), float(rho), float(dt)
        self.n_nodes, self.n_tets = int(sum(nn)), int(sum(nt))
        r, z, d, o = _i64(), _i64(), _i64(), _i64()
        _check(L.sta_sizes(ctx, ctypes.byref(r), ctypes.byref(z), ctypes.byref(d), ctypes.byref(o)), ctx)
        self.n_rows, self.nnz, self.n_diag_blocks, self.n_off_blocks = r.value, z.value, d.value, o.value
        self.k = k

    @classmethod
    def from_workloads(cls, ws, stream=None):
        w0 = ws[0]
        return cls([(w.x, w.tets, w.E, w.mask0) for w in ws], w0.nu, w0.rho, w0.dt, stream)


def _proxy_check(code: int, p=None):
    if code != STA_OK:
        msg = load().sta_proxy_last_error(p)
        raise StafemError(code, msg.decode() if msg else "")


class Proxy:
    """The graph-Laplacian proxy operator A_t = L_t + eps I over a superset mesh
    (sta_proxy_* in include/stafem.h).  tets (m, 4) int32 and mask0 (m,) uint8
    are host arrays, copied into the context."""

    def __init__(self, n_nodes, tets, mask0, eps, stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the HIP assembly path needs an MI355X")
        L = load()
        tets = np.ascontiguousarray(tets, dtype=np.int32)
        mask0 = np.ascontiguousarray(mask0, dtype=np.uint8)
        self.n_nodes, self.n_tets, self.eps = int(n_nodes), int(tets.shape[0]), float(eps)
        p = _vp()
        _proxy_check(L.sta_proxy_build(tets.ctypes.data, self.n_nodes, self.n_tets, mask0.ctypes.data, self.eps,
                                       _stream_handle(stream), ctypes.byref(p)), None)
        self._p = p
        r, z, e = _i64(), _i64(), _i64()
        _proxy_check(L.sta_proxy_sizes(p, ctypes.byref(r), ctypes.byref(z), ctypes.byref(e)), p)
        self.n_rows, self.nnz, self.n_edges = r.value, z.value, e.value

    @classmethod
    def from_workload(cls, w, eps, stream=None):
        return cls(w.n_nodes, w.tets, w.mask0, eps, stream)

    def close(self):
        if getattr(self, "_p", None):
            load().sta_proxy_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def full_rebuild(self, stream=None):
        _proxy_check(load().sta_proxy_full_rebuild(self._p, _stream_handle(stream)), self._p)

    def apply_edits(self, ids: torch.Tensor, states: torch.Tensor, stream=None):
        if ids.dtype != torch.int32 or states.dtype != torch.uint8 or not ids.is_cuda or not states.is_cuda \
                or ids.numel() != states.numel():
            raise TypeError("ids int32 and states uint8 CUDA tensors of equal length")
        _proxy_check(load().sta_proxy_apply_edits(self._p, _dev_ptr(ids), _dev_ptr(states), ids.numel(),
                                                  _stream_handle(stream)), self._p)

    def apply_edits_dev(self, ids: torch.Tensor, states: torch.Tensor, n: torch.Tensor, stream=None):
        if ids.dtype != torch.int32 or states.dtype != torch.uint8 or n.dtype != torch.int32 \
                or ids.numel() != states.numel():
            raise TypeError("ids int32, states uint8 (equal length) and n int32 CUDA tensors")
        _proxy_check(load().sta_proxy_apply_edits_dev(self._p, _dev_ptr(ids), _dev_ptr(states), ids.numel(),
                                                      _dev_ptr(n), _stream_handle(stream)), self._p)

    def state(self, stream=None):
        """Copies of (values float64, counts int32, degree int32) as CUDA tensors, stream-ordered."""
        v = torch.empty(self.nnz, dtype=torch.float64, device="cuda")
        c = torch.empty(self.n_edges, dtype=torch.int32, device="cuda")
        d = torch.empty(self.n_rows, dtype=torch.int32, device="cuda")
        _proxy_check(load().sta_proxy_copy_state(self._p, _dev_ptr(v), _dev_ptr(c), _dev_ptr(d),
                                                 _stream_handle(stream)), self._p)
        return v, c, d

    def pattern_ptrs(self):
        rp, ci, ed = _vp(), _vp(), _vp()
        _proxy_check(load().sta_proxy_pattern_ptrs(self._p, ctypes.byref(rp), ctypes.byref(ci), ctypes.byref(ed)),
                     self._p)
        return rp.value, ci.value, ed.value

    def pattern(self):
        """(rowptr, colidx, edges (n_edges, 2)) int32 numpy arrays."""
        rp = np.empty(self.n_rows + 1, dtype=np.int32)
        ci = np.empty(max(self.nnz, 1), dtype=np.int32)
        ed = np.empty(max(2 * self.n_edges, 2), dtype=np.int32)
        _proxy_check(load().sta_proxy_pattern_host(self._p, rp.ctypes.data, ci.ctypes.data, ed.ctypes.data), self._p)
        return rp, ci[: self.nnz], ed[: 2 * self.n_edges].reshape(-1, 2)

    def values_ptr(self) -> int:
        return int(load().sta_proxy_values_ptr(self._p) or 0)

    def last_frame_stats(self, stream=None) -> dict:
        out = (ctypes.c_int64 * 3)()
        _proxy_check(load().sta_proxy_last_frame_stats(self._p, _stream_handle(stream), out), self._p)
        return {"edits": out[0], "changed": out[1], "transitions": out[2]}

    def status_sync(self, stream=None) -> int:
        return int(load().sta_proxy_status_sync(self._p, _stream_handle(stream)))

    def last_error(self) -> str:
        m = load().sta_proxy_last_error(self._p)
        return m.decode() if m else ""


def bandwidth_probe(stream=None) -> dict:
    """Measured HBM streaming bandwidth in GB/s (see sta_bandwidth_probe)."""
    out = (ctypes.c_double * 3)()
    _check(load().sta_bandwidth_probe(_stream_handle(stream), out), None)
    return {"read_GBs": out[0], "write_GBs": out[1], "copy_GBs": out[2]}


def barrier_probe() -> dict:
    """Grid barrier vs kernel boundary, microseconds per graph-replayed unit (see sta_barrier_probe)."""
    out = (ctypes.c_double * 7)()
    _check(load().sta_barrier_probe(out), None)
    d = {"empty_kernel_us": out[0], "two_empty_kernels_us": out[1]}
    for k, g in enumerate((8, 32, 64, 128, 256)):
        d[f"barrier_kernel_{g}wg_us"] = out[2 + k] if out[2 + k] >= 0 else None
    return d


def latency_probe(stream=None) -> dict:
    """Measured latency floor of the GPU (see sta_latency_probe)."""
    out = (ctypes.c_double * 4)()
    _check(load().sta_latency_probe(_stream_handle(stream), out), None)
    return {"empty_kernel_us": out[0], "dependent_load_256MB_ns": out[1], "dependent_load_l2_ns": out[2],
            "dependent_atomic_ns": out[3]}


def upload_frame(ids: np.ndarray, states: np.ndarray, device="cuda"):
    """Host edit arrays -> (int32, uint8) CUDA tensors."""
    return (torch.from_numpy(np.ascontiguousarray(ids, dtype=np.int32)).to(device),
            torch.from_numpy(np.ascontiguousarray(states, dtype=np.uint8)).to(device))
