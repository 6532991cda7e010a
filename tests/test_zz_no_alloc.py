"""The adjoint entry point that allocates nothing (sta_adjoint_noalloc) against the
one that allocates its workspace (sta_adjoint): same kernels, so the same bits, on
two calls in a row (the second on a smaller context, so the fixed workspace keeps
the first call's larger contents), and a context beyond the workspace refused."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2605_11673_amd import workloads as W

pytestmark = pytest.mark.gpu


def _call(fn, asm, g):
    from paper_2605_11673_amd import stafem
    gl = torch.full((asm.n_tets,), np.nan, dtype=torch.float64, device="cuda")
    gx = torch.full((asm.n_nodes, 3), np.nan, dtype=torch.float64, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    code = fn(asm.handle, ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(gl.data_ptr()),
              ctypes.c_void_p(gx.data_ptr()), s)
    torch.cuda.synchronize()
    return code, gl.cpu().numpy(), gx.cpu().numpy()


def _bits(a):
    return np.ascontiguousarray(a).view(np.uint64)


def test_noalloc_adjoint_matches_allocating_entry_point():
    from paper_2605_11673_amd import stafem
    L = stafem.load()
    big = W.make_fracture(seed=0, n=40)
    small = W.make_fracture(seed=1, n=8, counts=[30, 50])
    for w, frames in ((big, 13), (small, 2)):
        mask = w.mask_after(frames - 1)
        print(f"[noalloc] tets={w.n_tets} active={int(mask.sum())}", flush=True)
        asm = stafem.Assembler(w.x, w.tets, w.E, w.nu, w.rho, w.dt, mask)
        g = torch.from_numpy(np.random.default_rng(w.n_tets).standard_normal(asm.nnz)).cuda()
        c0, gl0, gx0 = _call(L.sta_adjoint_noalloc, asm, g)
        c1, gl1, gx1 = _call(L.sta_adjoint, asm, g)
        assert c0 == stafem.STA_OK and c1 == stafem.STA_OK
        assert np.array_equal(_bits(gl0), _bits(gl1))
        assert np.array_equal(_bits(gx0), _bits(gx1))
        assert np.all(np.isfinite(gl0)) and np.all(gl0[mask == 0] == 0.0)
        asm.close()


def test_noalloc_adjoint_refuses_oversized_context():
    from paper_2605_11673_amd import stafem
    L = stafem.load()
    w = W.make_cube(seed=0, n=48)  # 663,552 tets > 524,288
    asm = stafem.Assembler(w.x, w.tets, w.E, w.nu, w.rho, w.dt, w.mask0)
    g = torch.zeros(asm.nnz, dtype=torch.float64, device="cuda")
    code, gl, gx = _call(L.sta_adjoint_noalloc, asm, g)
    assert code == stafem.STA_EINVAL
    assert "workspace" in asm.last_error()
    assert np.all(np.isnan(gl)) and np.all(np.isnan(gx))  # nothing written
    asm.close()
