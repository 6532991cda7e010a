"""GPU parity: the HIP path against the CPU oracle, bit for bit.

The paper's invariant (Sec. 3.3) is that the maintained matrix equals a
rebuild from scratch on the current active set after every frame; here
"equals" is bitwise in binary64 (every entry summed in ascending element id
from +0.0), and the rebuild is the oracle's element-major scatter, a
different route from the GPU's block-major gather.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2605_11673_amd import workloads as W

pytestmark = pytest.mark.gpu


def stafem():
    from paper_2605_11673_amd import stafem as S
    return S


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float64).view(np.uint64)


def gpu_values(asm):
    v = asm.values()
    torch.cuda.synchronize()
    return v.cpu().numpy()


def assert_bitwise(got, want, what):
    if not np.array_equal(bits(got), bits(want)):
        bad = np.nonzero(bits(got) != bits(want))[0]
        i = bad[0]
        raise AssertionError(f"{what}: {len(bad)} of {len(want)} values differ; first at {i}: "
                             f"gpu {got[i]!r} oracle {want[i]!r}")


def run_stream(w, check_every=1, pat=None, with_rebuild=False, label=""):
    S = stafem()
    print(f"[parity] {label or w.name}: n={w.n_nodes} m={w.n_tets} frames={len(w.frames)}", flush=True)
    asm = S.Assembler.from_workload(w)
    rp, ci = asm.pattern()
    if pat is None:
        pat = oracle.pattern(w.n_nodes, w.tets)
    assert np.array_equal(rp, pat[0]) and np.array_equal(ci, pat[1]), "pattern differs from the oracle"
    assert_bitwise(gpu_values(asm), oracle.rebuild_workload(w, w.mask0, pat), f"{label} initial")
    mask = w.mask0.copy()
    for t, (ids, st) in enumerate(w.frames):
        mask[ids] = st
        di, ds = S.upload_frame(ids, st)
        asm.apply_edits(di, ds)
        got = gpu_values(asm)
        if t % check_every == 0 or t == len(w.frames) - 1:
            assert_bitwise(got, oracle.rebuild_workload(w, mask, pat), f"{label} frame {t} (stream vs oracle)")
        if with_rebuild:
            asm.full_rebuild()
            assert_bitwise(gpu_values(asm), got, f"{label} frame {t} (stream vs GPU rebuild)")
    assert asm.status_sync() == S.STA_OK
    return asm, mask, pat


@pytest.mark.parametrize("seed", range(50))
def test_cube_stream_every_frame(seed):
    """384-tet cube, 24 frames of 1-8 random deletions, every frame bitwise."""
    w = W.make_cube(seed)
    asm, mask, pat = run_stream(w, with_rebuild=(seed % 10 == 0), label=f"cube seed {seed}")
    asm.close()


@pytest.mark.parametrize("seed", range(8))
def test_random_small_meshes(seed):
    """Random tet subsets, shuffled node ids (unused nodes -> empty rows), random vertex
    order, random masks, random add/delete edits including no-ops."""
    S = stafem()
    w = W.random_small_mesh(seed)
    g = np.random.default_rng(seed)
    frames = []
    for _ in range(6):
        k = int(g.integers(0, w.n_tets + 1))
        ids = g.choice(w.n_tets, size=k, replace=False).astype(np.int32)
        frames.append((ids, g.integers(0, 2, size=k).astype(np.uint8)))
    w.frames = frames
    asm, _, _ = run_stream(w, label=f"small seed {seed}")
    asm.close()


def test_fracture_full_size_every_frame():
    """384,000 tets, 68,921 nodes, 8,945,649 values; 24 Voronoi fracture frames
    (50..2000 deletions), then the 24 reverse frames that reinsert them (merge);
    each of the 48 frames bitwise equal to the oracle and to the GPU rebuild."""
    w = W.make_fracture(0)
    asm, mask, pat = run_stream(w, with_rebuild=True, label="fracture 40^3")
    S = stafem()
    for t, (ids, st) in enumerate(W.merge_stream(w.frames)):
        mask[ids] = st
        asm.apply_edits(*S.upload_frame(ids, st))
        got = gpu_values(asm)
        assert_bitwise(got, oracle.rebuild_workload(w, mask, pat), f"merge frame {t}")
    assert np.all(mask == 1)
    asm.close()


@pytest.mark.parametrize("seed", [1, 2])
def test_fracture_full_size_other_seeds(seed):
    """The full-size fracture+merge stream for two more seeds (other jitter, moduli,
    Voronoi sites and impact point, so other straddler sets and frame contents): every
    frame bitwise equal to the oracle, and the GPU rebuild at the end."""
    S = stafem()
    w = W.make_fracture(seed)
    frames = list(w.frames) + W.merge_stream(w.frames)
    print(f"[parity] fracture 40^3 seed {seed}: {sum(len(f[0]) for f in frames)} edits", flush=True)
    pat = oracle.pattern(w.n_nodes, w.tets)
    asm = S.Assembler.from_workload(w)
    mask = w.mask0.copy()
    for t, (ids, st) in enumerate(frames):
        mask[ids] = st
        asm.apply_edits(*S.upload_frame(ids, st))
        assert_bitwise(gpu_values(asm), oracle.rebuild_workload(w, mask, pat), f"seed {seed} frame {t}")
    got = gpu_values(asm)
    asm.full_rebuild()
    assert_bitwise(gpu_values(asm), got, f"seed {seed} final rebuild")
    assert np.all(mask == 1)
    assert asm.status_sync() == S.STA_OK
    asm.close()


def test_fracture_full_size_tuned_configuration():
    """The configuration the benchmark times: the autotuner's choice on the peak frame
    (as bench.py makes it), then the 48-frame fracture+merge stream, every frame bitwise
    equal to the oracle, and the rebuild under the tuned rebuild mapping at the end."""
    S = stafem()
    w = W.make_fracture(0)
    frames = list(w.frames) + W.merge_stream(w.frames)
    pat = oracle.pattern(w.n_nodes, w.tets)
    asm = S.Assembler.from_workload(w)
    rep = asm.autotune(*S.upload_frame(*frames[12]), reps=3)
    print("[parity] tuned: " + rep.splitlines()[-1], flush=True)
    mask = w.mask0.copy()
    for t, (ids, st) in enumerate(frames):
        mask[ids] = st
        asm.apply_edits(*S.upload_frame(ids, st))
        assert_bitwise(gpu_values(asm), oracle.rebuild_workload(w, mask, pat), f"tuned frame {t}")
    asm.full_rebuild()
    assert_bitwise(gpu_values(asm), oracle.rebuild_workload(w, mask, pat), "tuned rebuild")
    assert asm.status_sync() == S.STA_OK
    asm.close()


def test_refinement_full_size():
    """432,000-tet red-refinement superset: 24 refine frames (1 parent off, 8 children on,
    children's contributions computed at build) then 24 merge frames, every frame bitwise."""
    w = W.make_refinement(0)
    asm, mask, pat = run_stream(w, with_rebuild=True, label="refine 20^3")
    asm.close()


def test_refinement_full_size_second_seed():
    """The refinement superset with another seed (other jitter, moduli and choice of
    refined parents): every frame of the refine and merge stream bitwise equal to the oracle."""
    w = W.make_refinement(1)
    asm, mask, pat = run_stream(w, label="refine 20^3 seed 1")
    asm.close()


def test_edit_semantics_and_rollback():
    S = stafem()
    w = W.make_cube(3)
    pat = oracle.pattern(w.n_nodes, w.tets)
    asm = S.Assembler.from_workload(w)
    v0 = gpu_values(asm)
    # empty edit list
    asm.apply_edits(*S.upload_frame(np.zeros(0, np.int32), np.zeros(0, np.uint8)))
    assert_bitwise(gpu_values(asm), v0, "empty edit list")
    assert asm.last_frame_stats()["edits"] == 0
    # no-op edits (tets already active): nothing is recomputed, nothing changes
    asm.apply_edits(*S.upload_frame(np.array([0, 5, 9], np.int32), np.ones(3, np.uint8)))
    assert asm.last_frame_stats()["touched_blocks"] == 0
    assert_bitwise(gpu_values(asm), v0, "no-op edits")
    # a duplicate id rolls the whole frame back
    asm.apply_edits(*S.upload_frame(np.array([1, 2, 1], np.int32), np.zeros(3, np.uint8)))
    assert asm.status_sync() == S.STA_EDUP
    assert_bitwise(gpu_values(asm), v0, "rolled back duplicate frame")
    # out-of-range id and bad state
    asm.apply_edits(*S.upload_frame(np.array([4, 384], np.int32), np.zeros(2, np.uint8)))
    assert asm.status_sync() == S.STA_ERANGE
    asm.apply_edits(*S.upload_frame(np.array([4, -1], np.int32), np.zeros(2, np.uint8)))
    assert asm.status_sync() == S.STA_ERANGE
    asm.apply_edits(*S.upload_frame(np.array([4], np.int32), np.array([2], np.uint8)))
    assert asm.status_sync() == S.STA_ERANGE
    assert_bitwise(gpu_values(asm), v0, "rolled back range errors")
    assert asm.status_sync() == S.STA_OK  # errors were cleared
    # too many edits is a host error
    with pytest.raises(S.StafemError):
        n = w.n_tets + 1
        asm.apply_edits(*S.upload_frame(np.zeros(n, np.int32), np.zeros(n, np.uint8)))
    # forward then inverse returns the initial bits
    ids = np.array([3, 17, 100, 200, 383], np.int32)
    asm.apply_edits(*S.upload_frame(ids, np.zeros(5, np.uint8)))
    m = w.mask0.copy()
    m[ids] = 0
    assert_bitwise(gpu_values(asm), oracle.rebuild_workload(w, m, pat), "forward")
    st = asm.last_frame_stats()
    assert st["changed"] == 5 and st["activated"] == 0 and st["touched_blocks"] > 0
    asm.apply_edits(*S.upload_frame(ids, np.ones(5, np.uint8)))
    assert_bitwise(gpu_values(asm), v0, "forward then inverse")
    # everything off: every value is +0.0; everything back on: initial bits
    all_ids = np.arange(w.n_tets, dtype=np.int32)
    asm.apply_edits(*S.upload_frame(all_ids, np.zeros(w.n_tets, np.uint8)))
    assert np.all(bits(gpu_values(asm)) == 0)
    asm.apply_edits(*S.upload_frame(all_ids, np.ones(w.n_tets, np.uint8)))
    assert_bitwise(gpu_values(asm), v0, "all off then all on")
    asm.close()


def test_set_params_stale_then_rebuild():
    """New positions / moduli: apply_edits is refused until full_rebuild; afterwards the
    values and later activations (whose contributions predate the change) match the oracle."""
    S = stafem()
    w = W.make_fracture(seed=1, n=6, counts=[30, 40])
    pat = oracle.pattern(w.n_nodes, w.tets)
    asm = S.Assembler.from_workload(w)
    mask = w.mask_after(1)
    for ids, st in w.frames:
        asm.apply_edits(*S.upload_frame(ids, st))
    g = np.random.default_rng(0)
    x2 = w.x + g.uniform(-1e-3, 1e-3, size=w.x.shape)
    E2 = w.E * np.exp(0.1 * g.standard_normal(w.n_tets))
    asm.set_params(torch.from_numpy(x2).cuda(), torch.from_numpy(E2).cuda())
    with pytest.raises(S.StafemError) as ei:
        asm.apply_edits(*S.upload_frame(np.array([0], np.int32), np.zeros(1, np.uint8)))
    assert ei.value.code == S.STA_ESTALE
    asm.full_rebuild()
    ref = lambda mk: oracle.rebuild(x2, w.tets, E2, w.nu, w.rho, w.dt, mk, *pat)
    assert_bitwise(gpu_values(asm), ref(mask), "after set_params + rebuild")
    # reactivate the deleted tets: their contributions must be recomputed
    back = np.concatenate([ids for ids, _ in w.frames]).astype(np.int32)
    asm.apply_edits(*S.upload_frame(back, np.ones(len(back), np.uint8)))
    mask[back] = 1
    assert asm.last_frame_stats()["activated"] == len(back)
    assert_bitwise(gpu_values(asm), ref(mask), "activation after set_params")
    asm.close()


def test_degenerate_tet_rejected():
    S = stafem()
    x = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], dtype=np.float64)  # coplanar
    with pytest.raises(S.StafemError) as ei:
        S.Assembler(x, np.array([[0, 1, 2, 3]], np.int32), np.ones(1), 0.3, 1000.0, 0.01, np.ones(1, np.uint8))
    assert ei.value.code == S.STA_EDEGENERATE


def test_empty_mesh_and_run_twice_determinism():
    S = stafem()
    asm = S.Assembler(np.zeros((3, 3)), np.zeros((0, 4), np.int32), np.zeros(0), 0.3, 1000.0, 0.01,
                      np.zeros(0, np.uint8))
    assert asm.nnz == 0 and asm.n_rows == 9
    asm.full_rebuild()
    for adj in ("vertex", "face"):
        lab, k = asm.components(adj)
        assert k == 0 and lab.numel() == 0
    assert asm.status_sync() == S.STA_OK
    asm.close()
    w = W.make_fracture(seed=4, n=8, counts=[60, 200, 90])
    runs = []
    for _ in range(2):
        a = S.Assembler.from_workload(w)
        for ids, st in w.frames:
            a.apply_edits(*S.upload_frame(ids, st))
        runs.append(gpu_values(a))
        a.close()
    assert_bitwise(runs[0], runs[1], "run twice")


def test_device_count_and_graph_replay():
    """sta_apply_edits_dev reads the edit count on the device, so one captured HIP graph
    serves every frame: new edit lists are copied into the same buffers and the graph is
    replayed.  Eager frames and synchronisations sit between the replays, and every replay
    is checked against the oracle."""
    S = stafem()
    w = W.make_fracture(seed=3, n=8, counts=[40, 80, 20, 60, 5])
    frames = list(w.frames) + W.merge_stream(w.frames)
    pat = oracle.pattern(w.n_nodes, w.tets)
    asm = S.Assembler.from_workload(w)
    cap = 128
    ids = torch.zeros(cap, dtype=torch.int32, device="cuda")
    st = torch.zeros(cap, dtype=torch.uint8, device="cuda")
    n = torch.zeros(1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        asm.apply_edits_dev(ids, st, n)
    torch.cuda.synchronize()
    assert_bitwise(gpu_values(asm), oracle.rebuild_workload(w, w.mask0, pat), "capture must not execute")
    mask = w.mask0.copy()
    for t, (fi, fs) in enumerate(frames):
        k = len(fi)
        if t % 3 == 2:  # an eager frame between replays
            asm.apply_edits(*S.upload_frame(fi, fs))
        else:
            ids[:k].copy_(torch.from_numpy(fi.astype(np.int32)))
            st[:k].copy_(torch.from_numpy(fs.astype(np.uint8)))
            n.fill_(k)
            g.replay()
        torch.cuda.synchronize()
        mask[fi] = fs
        assert_bitwise(gpu_values(asm), oracle.rebuild_workload(w, mask, pat), f"graph frame {t}")
        s = asm.last_frame_stats()
        assert s["edits"] == k and s["changed"] == k and s["rolled_back"] == 0
    assert asm.status_sync() == S.STA_OK
    # a device count above the capacity is an error and the frame is skipped
    v0 = gpu_values(asm)
    n.fill_(cap + 1)
    g.replay()
    assert asm.status_sync() == S.STA_ERANGE
    assert_bitwise(gpu_values(asm), v0, "out-of-range device count")
    asm.close()


def test_maximum_size_frames():
    """Frames as large as the candidate pool: every tet deleted in one frame (the matrix
    becomes all +0.0, no -0.0), every tet re-added in one frame (the initial bits come
    back), then a random half toggled with random states (no-ops included), each frame's
    ids in random order; also through the device-count entry point at full capacity."""
    S = stafem()
    w = W.make_fracture(seed=11, n=12, counts=[10])
    pat = oracle.pattern(w.n_nodes, w.tets)
    asm = S.Assembler.from_workload(w)
    v0 = gpu_values(asm)
    g = np.random.default_rng(11)
    every = g.permutation(w.n_tets).astype(np.int32)
    asm.apply_edits(*S.upload_frame(every, np.zeros(w.n_tets, np.uint8)))
    zero = gpu_values(asm)
    assert_bitwise(zero, oracle.rebuild_workload(w, np.zeros(w.n_tets, np.uint8), pat), "all deleted")
    assert not np.any(np.signbit(zero)) and not np.any(zero)
    assert asm.last_frame_stats()["edits"] == w.n_tets
    asm.apply_edits(*S.upload_frame(every, np.ones(w.n_tets, np.uint8)))
    assert_bitwise(gpu_values(asm), v0, "all re-added")
    half = g.choice(w.n_tets, size=w.n_tets // 2, replace=False).astype(np.int32)
    st = g.integers(0, 2, size=len(half)).astype(np.uint8)
    ids_d = torch.zeros(w.n_tets, dtype=torch.int32, device="cuda")
    st_d = torch.zeros(w.n_tets, dtype=torch.uint8, device="cuda")
    n_d = torch.tensor([len(half)], dtype=torch.int32, device="cuda")
    ids_d[:len(half)].copy_(torch.from_numpy(half))
    st_d[:len(half)].copy_(torch.from_numpy(st))
    asm.apply_edits_dev(ids_d, st_d, n_d)
    mask = np.ones(w.n_tets, np.uint8)
    mask[half] = st
    assert_bitwise(gpu_values(asm), oracle.rebuild_workload(w, mask, pat), "random half, device count")
    assert asm.status_sync() == S.STA_OK
    asm.close()
