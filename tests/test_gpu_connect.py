"""GPU connectivity (sta_components) against the oracle: per-tet component labels
(smallest vertex id of the component) bitwise, the component count, and the
paper's sampled breadth-first spot checks."""
import numpy as np
import pytest
import torch

from oracle import connectivity as C
from paper_2605_11673_amd import workloads as W

pytestmark = pytest.mark.gpu


def S():
    from paper_2605_11673_amd import stafem
    return stafem


def gpu_labels(asm):
    lab, k = asm.components()
    torch.cuda.synchronize()
    return lab.cpu().numpy().astype(np.int64), k


def check(asm, w, mask, what):
    lab, k = gpu_labels(asm)
    ref, rk = C.components(w.n_nodes, w.tets, mask)
    assert np.array_equal(lab, ref), f"{what}: {np.sum(lab != ref)} labels differ"
    assert k == rk, f"{what}: {k} vs {rk} components"
    return lab, k


def test_fracture_stream_every_frame():
    Sm = S()
    w = W.make_fracture(seed=4, n=12, counts=[100, 400, 900, 300, 60])
    frames = list(w.frames) + W.merge_stream(w.frames)
    asm = Sm.Assembler.from_workload(w)
    mask = w.mask0.copy()
    ks = [check(asm, w, mask, "initial")[1]]
    for t, (ids, st) in enumerate(frames):
        asm.apply_edits(*Sm.upload_frame(ids, st))
        mask[ids] = st
        ks.append(check(asm, w, mask, f"frame {t}")[1])
    assert ks[0] == 1 and max(ks) > 1 and ks[-1] == 1  # the cut separates pieces, reinsertion rejoins them
    asm.close()


@pytest.mark.parametrize("seed", range(6))
def test_random_small_meshes(seed):
    Sm = S()
    w = W.random_small_mesh(seed, max_tets=40)
    asm = Sm.Assembler.from_workload(w)
    check(asm, w, w.mask0, f"small{seed}")
    asm.close()


def test_full_size_with_bfs_spot_checks():
    """40^3 fracture stream: labels vs the oracle at frames 0, 12, 23 and at the end of the
    reinsertion; at the peak frame, breadth-first searches from 20 sampled active tets
    each reach exactly the tets that carry their GPU label; two calls agree."""
    Sm = S()
    w = W.make_fracture(seed=0)
    frames = list(w.frames) + W.merge_stream(w.frames)
    asm = Sm.Assembler.from_workload(w)
    mask = w.mask0.copy()
    for t, (ids, st) in enumerate(frames):
        asm.apply_edits(*Sm.upload_frame(ids, st))
        mask[ids] = st
        if t in (0, 12, 23, 47):
            lab, k = check(asm, w, mask, f"frame {t}")
            print(f"[connect] frame {t}: {k} components", flush=True)
        if t == 12:
            by = C.tets_by_node(w.n_nodes, w.tets, mask)
            g = np.random.default_rng(0)
            act = np.nonzero(mask)[0]
            for e in g.choice(act, size=20, replace=False):
                comp = C.bfs_component(w.n_nodes, w.tets, mask, int(e), by)
                assert comp == set(np.nonzero(lab == lab[e])[0].tolist())
            lab2, _ = gpu_labels(asm)
            assert np.array_equal(lab, lab2)
    asm.close()


def test_refinement_and_batch():
    """Refinement superset (hanging nodes join through shared corners) every 6th frame;
    a batch of disjoint meshes has at least one component per mesh."""
    Sm = S()
    r = W.make_refinement(seed=3, n=8, frames=12)
    asm = Sm.Assembler.from_workload(r)
    mask = r.mask0.copy()
    for t, (ids, st) in enumerate(r.frames):
        asm.apply_edits(*Sm.upload_frame(ids, st))
        mask[ids] = st
        if t % 6 == 5:
            check(asm, r, mask, f"refinement frame {t}")
    asm.close()
    ws = W.make_batch(seed=3, count=6, sizes=[2, 4, 3, 1, 5, 2])
    b = Sm.Batch.from_workloads(ws)
    lab, k = gpu_labels(b)
    assert k == 6
    off = b.offsets()
    for j in range(6):
        assert np.all(lab[off["tet"][j]:off["tet"][j + 1]] == off["node"][j])
    b.close()
