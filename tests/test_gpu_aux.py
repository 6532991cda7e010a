"""Auxiliary subsystems on the GPU: the audit of the maintained state against a
rebuild (paper Sec. 3.3 invariant), forced allocation failures (STA_ENOMEM, with
nothing leaked), and the grid-barrier probe."""
import ctypes
import os

import numpy as np
import pytest
import torch

from paper_2605_11673_amd import workloads as W

pytestmark = pytest.mark.gpu


def S():
    from paper_2605_11673_amd import stafem
    return stafem


def _hip():
    lib = ctypes.CDLL("libamdhip64.so.7")
    lib.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    lib.hipMemcpy.restype = ctypes.c_int
    return lib


def test_audit_detects_corrupted_values_and_clears_after_rebuild():
    Sm = S()
    w = W.make_fracture(seed=4, n=10, counts=[300, 700, 200])
    asm = Sm.Assembler.from_workload(w)
    assert asm.audit() == {"values_differing": 0, "tets_differing": 0}
    for ids, st in list(w.frames) + W.merge_stream(w.frames)[:2]:
        asm.apply_edits(*Sm.upload_frame(ids, st))
    assert asm.audit() == {"values_differing": 0, "tets_differing": 0}
    # flip one maintained value behind the library's back
    torch.cuda.synchronize()
    k = asm.nnz // 3
    bad = np.array([12345.678], dtype=np.float64)
    assert _hip().hipMemcpy(asm.values_ptr() + 8 * k, bad.ctypes.data, 8, 1) == 0  # host to device
    assert asm.audit() == {"values_differing": 1, "tets_differing": 0}
    asm.full_rebuild()
    assert asm.audit() == {"values_differing": 0, "tets_differing": 0}
    # parameters changed: the audit refuses until a rebuild
    E2 = torch.from_numpy(w.E * 1.5).cuda()
    asm.set_params(E=E2)
    with pytest.raises(Sm.StafemError) as ex:
        asm.audit()
    assert ex.value.code == Sm.STA_ESTALE
    asm.full_rebuild()
    assert asm.audit() == {"values_differing": 0, "tets_differing": 0}
    asm.close()


def test_forced_allocation_failure_reports_enomem_and_leaks_nothing():
    Sm = S()
    w = W.make_fracture(seed=5, n=30)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    try:
        for k in (1, 9, 20):
            os.environ["STA_FAIL_ALLOC_AT"] = str(k)
            with pytest.raises(Sm.StafemError) as ex:
                Sm.Assembler.from_workload(w)
            assert ex.value.code == Sm.STA_ENOMEM, k
            del os.environ["STA_FAIL_ALLOC_AT"]
            asm = Sm.Assembler.from_workload(w)  # and without the injection the build works
            asm.close()
    finally:
        os.environ.pop("STA_FAIL_ALLOC_AT", None)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    # the 30^3 context holds about 350 MB; three failed builds must not have kept theirs
    assert free0 - free1 < 64 << 20, (free0 - free1)


def test_barrier_probe_reports_positive_costs():
    d = S().barrier_probe()
    assert 0 < d["empty_kernel_us"] < d["two_empty_kernels_us"]
    for g in (8, 32):
        assert d[f"barrier_kernel_{g}wg_us"] is not None and d[f"barrier_kernel_{g}wg_us"] > 0
    print("[barrier]", d, flush=True)


def test_trace_writes_one_line_per_call_with_frame_stats(tmp_path):
    """STA_TRACE names a file at build: every rebuild and frame call appends one JSON line;
    STA_TRACE_STATS=1 adds the frame's statistics, equal to what the stats call returns."""
    import json

    Sm = S()
    w = W.make_fracture(seed=6, n=10, counts=[50, 400, 120])
    path = tmp_path / "trace.jsonl"
    os.environ["STA_TRACE"] = str(path)
    os.environ["STA_TRACE_STATS"] = "1"
    try:
        asm = Sm.Assembler.from_workload(w)
    finally:
        os.environ.pop("STA_TRACE")
        os.environ.pop("STA_TRACE_STATS")
    want = []
    for ids, st in w.frames:
        asm.apply_edits(*Sm.upload_frame(ids, st))
        d = asm.last_frame_stats()
        want.append({k: d[k] for k in Sm.Assembler.FRAME_STATS})
    # the device-count entry point (a buffer of capacity 1024) and the +/- delta policy
    (i0, s0), (i1, s1) = W.merge_stream(w.frames)[:2]
    cap = 1024
    bi = torch.zeros(cap, dtype=torch.int32, device="cuda")
    bs = torch.zeros(cap, dtype=torch.uint8, device="cuda")
    bi[:len(i0)].copy_(torch.from_numpy(i0.astype(np.int32)))
    bs[:len(i0)].copy_(torch.from_numpy(s0.astype(np.uint8)))
    asm.apply_edits_dev(bi, bs, torch.tensor([len(i0)], dtype=torch.int32, device="cuda"))
    asm.apply_edits_delta(*Sm.upload_frame(i1, s1))
    asm.full_rebuild()
    asm.close()
    lines = [json.loads(l) for l in path.read_text().splitlines()]
    nf = len(w.frames)
    assert [l["seq"] for l in lines] == list(range(nf + 3))
    assert [l["call"] for l in lines] == ["apply_edits"] * nf + ["apply_edits_dev", "apply_edits_delta", "full_rebuild"]
    for l, (ids, _), s in zip(lines, w.frames, want):
        assert l["edits"] == len(ids) and l["stats"] == s and l["stats"]["edits"] == len(ids)
    assert lines[nf]["capacity"] == cap and lines[nf]["stats"]["edits"] == len(i0)
    assert lines[nf + 1]["edits"] == len(i1) and lines[nf + 1]["stats"]["edits"] == len(i1)
    assert lines[nf + 1]["stats"]["diag_blocks"] == 0  # the delta policy claims no blocks
    assert "stats" not in lines[-1]
    assert all(a["host_us"] <= b["host_us"] for a, b in zip(lines, lines[1:]))
    # a context built without STA_TRACE writes nothing more
    asm = Sm.Assembler.from_workload(w)
    asm.apply_edits(*Sm.upload_frame(*w.frames[0]))
    asm.close()
    assert len(path.read_text().splitlines()) == len(lines)
    # an unopenable trace file fails the build
    os.environ["STA_TRACE"] = str(tmp_path / "no_such_dir" / "t.jsonl")
    try:
        with pytest.raises(Sm.StafemError) as ex:
            Sm.Assembler.from_workload(w)
        assert ex.value.code == Sm.STA_EINVAL
    finally:
        os.environ.pop("STA_TRACE")
