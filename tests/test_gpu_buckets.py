"""Slot mappings chosen per incidence-length bucket (sta_set_bucket_map).

A block's incidence length kappa (the candidate tets in its segment) puts it
in a bucket, and each bucket has its own lanes per value.  Every mapping
adds the same terms in the same order, so every combination must give the
oracle's values bit for bit, in the rebuild and in every streaming frame.
The refinement superset has diagonal blocks in all three buckets (coarse
corner nodes carry 48 candidate tets); the cube has none above 24.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2605_11673_amd import workloads as W

pytestmark = pytest.mark.gpu


def S():
    from paper_2605_11673_amd import stafem
    return stafem


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float64).view(np.uint64)


def host_values(asm):
    v = asm.values()
    torch.cuda.synchronize()
    return v.cpu().numpy()


def check(got, want, what):
    bad = np.nonzero(bits(got) != bits(want))[0]
    assert len(bad) == 0, f"{what}: {len(bad)} values differ, first at {bad[0]}"


def kappa_buckets(w):
    """Blocks per bucket from the oracle's pattern segments (diag <= 8, 9..32, > 32; off <= 8, > 8)."""
    t = w.tets.astype(np.int64)
    dk = np.bincount(t.ravel(), minlength=w.n_nodes)
    dk = dk[dk > 0]
    pairs = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    keys = np.concatenate([np.minimum(t[:, a], t[:, b]) * w.n_nodes + np.maximum(t[:, a], t[:, b]) for a, b in pairs])
    ok = np.unique(keys, return_counts=True)[1]
    return ([int(np.sum(dk <= 8)), int(np.sum((dk > 8) & (dk <= 32))), int(np.sum(dk > 32))],
            [int(np.sum(ok <= 8)), int(np.sum(ok > 8))])


def test_bucket_counts_and_validation():
    Sm = S()
    w = W.make_refinement(seed=1, n=4, frames=4)
    asm = Sm.Assembler.from_workload(w)
    d, o = kappa_buckets(w)
    for which in ("rebuild", "stream"):
        m = asm.bucket_map(which)
        assert m["diag_blocks"] == d and m["off_blocks"] == o
        assert m["diag"] == [1, 1, 1] and m["off"] == [1, 1]
    assert d[2] > 0 and d[1] > 0  # the refinement superset fills the long bucket
    for bad in ([2, 1, 1], [1, 1, 64], [0, 4, 4]):
        with pytest.raises(Sm.StafemError):
            asm.set_bucket_map("rebuild", bad, [1, 1])
    with pytest.raises(Sm.StafemError):
        asm.set_bucket_map("stream", [1, 4, 16], [1, 16])
    asm.set_bucket_map("stream", [1, 4, 16], [4, 1])
    assert asm.bucket_map("stream")["diag"] == [1, 4, 16] and asm.bucket_map("stream")["off"] == [4, 1]
    cfg = asm.get_config()
    assert (cfg["stream_qd"], cfg["stream_qo"]) == (16, 4)  # the allocation: the largest group
    asm.set_config(0, 4, 1, 4, 1, 0, 0)  # one mapping for every bucket again
    assert asm.bucket_map("stream")["diag"] == [4, 4, 4] and asm.bucket_map("rebuild")["off"] == [1, 1]
    asm.close()


MAPS = [([1, 4, 16], [1, 4]), ([16, 1, 4], [4, 1]), ([4, 16, 1], [1, 1]), ([1, 1, 16], [4, 4]),
        ([4, 4, 16], [1, 1]), ([16, 16, 1], [4, 1])]


@pytest.mark.parametrize("k", range(len(MAPS)))
def test_refinement_stream_every_bucket_map(k):
    """Refinement (refine then merge) with mixed bucket maps, checked every frame; the
    rebuild under its own mixed map after the stream."""
    Sm = S()
    w = W.make_refinement(seed=2 + k, n=4, frames=6)
    frames = list(w.frames)
    pat = oracle.pattern(w.n_nodes, w.tets)
    asm = Sm.Assembler.from_workload(w)
    sd, so = MAPS[k]
    rd, ro = MAPS[(k + 1) % len(MAPS)]
    asm.set_bucket_map("stream", sd, so)
    asm.set_bucket_map("rebuild", rd, ro)
    asm.full_rebuild()
    check(host_values(asm), oracle.rebuild_workload(w, w.mask0, pat), f"map {k} rebuild at mask0")
    mask = w.mask0.copy()
    for t, (ids, st) in enumerate(frames):
        asm.apply_edits(*Sm.upload_frame(ids, st))
        mask[ids] = st
        check(host_values(asm), oracle.rebuild_workload(w, mask, pat), f"map {k} frame {t}")
    asm.full_rebuild()
    check(host_values(asm), oracle.rebuild_workload(w, mask, pat), f"map {k} final rebuild")
    assert asm.status_sync() == Sm.STA_OK
    asm.close()


def test_fused_frame_and_graph_with_bucket_map():
    """The one-launch frame and a captured graph under a mixed map."""
    Sm = S()
    w = W.make_refinement(seed=9, n=4, frames=4)
    pat = oracle.pattern(w.n_nodes, w.tets)
    for fused in (1, 0):
        asm = Sm.Assembler.from_workload(w)
        asm.set_config(fused, 4, 1, 16, 4, 0, 0)
        asm.set_bucket_map("stream", [1, 4, 16], [1, 4])
        cap = max(len(ids) for ids, _ in w.frames)
        ids_d = torch.zeros(cap, dtype=torch.int32, device="cuda")
        st_d = torch.zeros(cap, dtype=torch.uint8, device="cuda")
        n_d = torch.zeros(1, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            asm.apply_edits_dev(ids_d, st_d, n_d)
        torch.cuda.synchronize()
        mask = w.mask0.copy()
        for t, (ids, st) in enumerate(w.frames):
            ids_d[:len(ids)].copy_(torch.from_numpy(ids.astype(np.int32)))
            st_d[:len(ids)].copy_(torch.from_numpy(st.astype(np.uint8)))
            n_d.fill_(len(ids))
            g.replay()
            torch.cuda.synchronize()
            mask[ids] = st
            check(host_values(asm), oracle.rebuild_workload(w, mask, pat), f"fused {fused} graph frame {t}")
        assert asm.status_sync() == Sm.STA_OK
        del g
        asm.close()


def test_autotune_reports_buckets(tmp_path, monkeypatch):
    Sm = S()
    monkeypatch.setenv("STA_TUNE_CACHE", str(tmp_path / "tune.txt"))
    w = W.make_refinement(seed=5, n=4, frames=4)
    pat = oracle.pattern(w.n_nodes, w.tets)
    asm = Sm.Assembler.from_workload(w)
    di, ds = Sm.upload_frame(*w.frames[0])
    rep = asm.autotune(di, ds, reps=2)
    assert "bucket d2" in rep and "chosen" in rep, rep
    maps = {k: asm.bucket_map(k) for k in ("rebuild", "stream")}
    cfg = asm.get_config()
    assert cfg["rebuild_qd"] == max(maps["rebuild"]["diag"]) and cfg["stream_qo"] == max(maps["stream"]["off"])
    mask = w.mask0.copy()
    check(host_values(asm), oracle.rebuild_workload(w, mask, pat), "after tuning")
    for t, (ids, st) in enumerate(w.frames):
        asm.apply_edits(*Sm.upload_frame(ids, st))
        mask[ids] = st
        check(host_values(asm), oracle.rebuild_workload(w, mask, pat), f"tuned frame {t}")
    asm.close()
    asm2 = Sm.Assembler.from_workload(w)
    rep2 = asm2.autotune(di, ds)
    assert rep2.startswith("cached")
    assert asm2.get_config() == cfg and {k: asm2.bucket_map(k) for k in ("rebuild", "stream")} == maps
    asm2.close()
