"""The +/- delta policy (sta_apply_edits_delta) against the oracle, within a
rounding bound derived from the arithmetic.

Bound.  An entry's oracle value is the canonical sum of its active terms
a_e; its recursive-summation error is at most kappa * u * S, with kappa the
entry's candidate count, S = sum over candidates of |a_e| and u = 2^-53.
The delta policy starts from the same canonical sum and then adds or
subtracts one term per state change of an incident tet, K changes in all;
every intermediate exact value is a sum of distinct candidate terms, so each
rounding is at most u * S (to first order).  Hence
    |delta - oracle| <= (2 kappa + K + 2) * u * S * 1.01.
The paper reports the same comparison (largest entry difference between
streaming and rebuild) as 8.3e-17 on its elasticity study (Sec. 6.1).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2605_11673_amd import workloads as W

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


def S():
    from paper_2605_11673_amd import stafem
    return stafem


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float64).view(np.uint64)


def host_values(asm):
    v = asm.values()
    torch.cuda.synchronize()
    return v.cpu().numpy()


class Bound:
    def __init__(self, w, pat):
        self.w, self.pat = w, pat
        ones = np.ones(w.n_tets)
        args = (w.x, w.tets, w.E, w.nu, w.rho, w.dt)
        self.S = oracle.rebuild_weighted(*args, ones, *pat)
        self.kappa = oracle.rebuild_weighted(*args, ones, *pat, count_only=True)
        self.changes = np.zeros(w.n_tets)

    def record(self, ids, st, mask_before):
        self.changes[ids[mask_before[ids] != st]] += 1

    def check(self, got, mask, what):
        w = self.w
        K = oracle.rebuild_weighted(w.x, w.tets, w.E, w.nu, w.rho, w.dt, self.changes, *self.pat, count_only=True)
        want = oracle.rebuild(w.x, w.tets, w.E, w.nu, w.rho, w.dt, mask, *self.pat)
        tol = (2 * self.kappa + K + 2) * U * self.S * 1.01
        err = np.abs(got - want)
        bad = np.nonzero(err > tol)[0]
        assert bad.size == 0, f"{what}: {bad.size} entries beyond the bound, first {bad[0]} err {err[bad[0]]:.3e} " \
                              f"tol {tol[bad[0]]:.3e}"
        scale = np.maximum(np.abs(want), 1e-300)
        return float(err.max()), float((err / np.maximum(self.S, 1e-300)).max()), float((err / scale)[want != 0].max()
                                                                                           if np.any(want != 0) else 0)


def run_delta(w, frames, label, check_every=1):
    Sm = S()
    print(f"[delta] {label}: {w.n_tets} tets, {len(frames)} frames", flush=True)
    pat = oracle.pattern(w.n_nodes, w.tets)
    asm = Sm.Assembler.from_workload(w)
    B = Bound(w, pat)
    mask = w.mask0.copy()
    worst = (0.0, 0.0, 0.0)
    for t, (ids, st) in enumerate(frames):
        asm.apply_edits_delta(*Sm.upload_frame(ids, st))
        B.record(ids, st, mask)
        mask[ids] = st
        if t % check_every == 0 or t == len(frames) - 1:
            e = B.check(host_values(asm), mask, f"{label} frame {t}")
            worst = tuple(max(a, b) for a, b in zip(worst, e))
    assert asm.status_sync() == Sm.STA_OK
    print(f"[delta] {label}: max abs diff {worst[0]:.3e}, max diff / sum|terms| {worst[1]:.3e}, "
          f"max rel diff {worst[2]:.3e}", flush=True)
    return asm, mask, pat


def test_cube_stream_within_bound_then_rebuild_exact():
    """Unjittered 4^3 cube: 24 deletion frames and their reinsertion, every frame within
    the bound; a full rebuild afterwards is bitwise the oracle (the delta policy kept
    the mask and the per-element contributions)."""
    w = W.make_cube(0)
    asm, mask, pat = run_delta(w, list(w.frames) + W.merge_stream(w.frames), "cube")
    asm.full_rebuild()
    assert np.array_equal(bits(host_values(asm)), bits(oracle.rebuild_workload(w, mask, pat)))
    asm.close()


def test_fracture_and_refinement_streams():
    """Jittered fracture (10,368 tets) with reinsertion and a refinement superset: every
    frame within the bound."""
    w = W.make_fracture(seed=3, n=12, counts=[40, 200, 600, 150, 20])
    asm, _, _ = run_delta(w, list(w.frames) + W.merge_stream(w.frames), "fracture 12")
    asm.close()
    r = W.make_refinement(seed=2, n=6, frames=8)
    asm, _, _ = run_delta(r, list(r.frames), "refinement 6")
    asm.close()


def test_mixed_policies_share_state():
    """Delta frames, then exact frames, then delta again: the exact policy's touched
    entries are re-summed from the contributions the delta policy maintained, and a
    final rebuild is bitwise the oracle."""
    Sm = S()
    w = W.make_fracture(seed=5, n=8, counts=[30, 120, 60, 10])
    frames = list(w.frames) + W.merge_stream(w.frames)
    pat = oracle.pattern(w.n_nodes, w.tets)
    asm = Sm.Assembler.from_workload(w)
    mask = w.mask0.copy()
    for t, (ids, st) in enumerate(frames):
        if t % 3 == 1:
            asm.apply_edits(*Sm.upload_frame(ids, st))
        else:
            asm.apply_edits_delta(*Sm.upload_frame(ids, st))
        mask[ids] = st
    assert asm.status_sync() == Sm.STA_OK
    asm.full_rebuild()
    assert np.array_equal(bits(host_values(asm)), bits(oracle.rebuild_workload(w, mask, pat)))
    asm.close()


def test_invalid_edits_skipped_and_reported():
    Sm = S()
    w = W.make_cube(2)
    pat = oracle.pattern(w.n_nodes, w.tets)
    asm = Sm.Assembler.from_workload(w)
    B = Bound(w, pat)
    mask = w.mask0.copy()
    ids = np.array([3, 9, 3], np.int32)
    asm.apply_edits_delta(*Sm.upload_frame(ids, np.zeros(3, np.uint8)))
    assert asm.status_sync() == Sm.STA_EDUP
    B.record(np.array([3, 9]), np.zeros(2, np.uint8), mask)
    mask[[3, 9]] = 0
    B.check(host_values(asm), mask, "duplicate skipped")
    asm.apply_edits_delta(*Sm.upload_frame(np.array([5, w.n_tets], np.int32), np.zeros(2, np.uint8)))
    assert asm.status_sync() == Sm.STA_ERANGE
    B.record(np.array([5]), np.zeros(1, np.uint8), mask)
    mask[5] = 0
    B.check(host_values(asm), mask, "out-of-range skipped")
    asm.full_rebuild()
    assert np.array_equal(bits(host_values(asm)), bits(oracle.rebuild_workload(w, mask, pat)))
    asm.close()


def test_full_size_fracture_drift():
    """40^3 fracture + reinsertion (48 frames, 25,572 state changes) under the delta
    policy; checked against the bound at the peak frame and at the end."""
    w = W.make_fracture(seed=0)
    frames = list(w.frames) + W.merge_stream(w.frames)
    asm, _, _ = run_delta(w, frames, "fracture 40", check_every=12)
    asm.close()
