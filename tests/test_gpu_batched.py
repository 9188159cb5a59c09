"""GPU tests of batched contexts: many independent scenes (each with its own
grid, time step and material) advanced by one launch per phase per substep,
frames with per-scene substep counts, frames replayed as HIP graphs, and the
chunk-size autotuner.

Bars: every scene of a batch matches the FP64 oracle run on that scene alone
(1e-4 normwise, as the single-scene parity tests), binning per scene is
bit-exact, and the batched, graph and one-at-a-time forms agree."""
import math

import numpy as np
import pytest

from paper_2111_00699_amd import scenes

from .test_gpu_parity import compare_state, gpu_state, normwise, print_case, TOL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a visible GPU")
    return torch


def small_batch(count=6, nmax=6000, seed=3):
    return scenes.batched_scenes(seed=seed, count=count, nmin=700, nmax=nmax)


def make_batch(torch_cuda, batch, **kw):
    from paper_2111_00699_amd import mpm

    descs = [dict(n=b["n"], dt=b["dt"], bc=b["bc"]) for b in batch]
    return mpm.Sim(batch[0]["n"], batch[0]["dt"], scenes=descs, **kw)


def oracle_cfg(b):
    return dict(n=b["n"], dt=b["dt"], bc=b["bc"])


def test_batch_recipe_covers_the_mix():
    batch = scenes.batched_scenes()
    assert len(batch) == 256
    kinds = {(b["kind"], b["n"]) for b in batch}
    assert kinds == {(k, n) for k in ("jelly", "snow", "water") for n in (64, 128)}
    subs = {math.ceil(scenes.FRAME / b["dt"] - 1e-4) for b in batch}
    assert subs == {84, 167, 334}


def test_batched_substep_matches_oracle_per_scene(torch_cuda, oracle):
    batch = small_batch()
    print_case("batched_substep", scenes=len(batch), N=sum(b["x"].shape[1] for b in batch))
    sim = make_batch(torch_cuda, batch)
    states = []
    for k, b in enumerate(batch):
        st = scenes.nontrivial_state(b["x"], seed=20 + k, kind=b["kind"])
        states.append(st)
        sim.add_particles(b["mat"], st["x"], v=st["v"], C=st["C"], F=st.get("F"), s=st.get("s"), scene=k)
    sim.substep(1)
    for k, b in enumerate(batch):
        gs = {key: v.cpu().numpy() for key, v in sim.read_particles(scene=k).items()}
        os_, om, ov, bad = oracle.substep(oracle_cfg(b), b["mat"], states[k])
        assert bad == 0
        compare_state(gs, os_, b["kind"], n=b["n"])
        gm, gv = (t.cpu().numpy() for t in sim.read_grid(scene=k))
        assert normwise(gm, om) <= TOL, k
        assert normwise(gv, ov) <= TOL, k
        assert sim.scene_stats(k)["substeps"] == 1
    sim.close()


def test_batched_binning_is_bit_exact_per_scene(torch_cuda, oracle):
    batch = small_batch(count=5, seed=8)
    sim = make_batch(torch_cuda, batch)
    for k, b in enumerate(batch):
        sim.add_particles(b["mat"], b["x"], scene=k)
    sim.substep(1)
    for k, b in enumerate(batch):
        keys, perm = sim.read_binning(scene=k)
        blocks = sim.read_blocks(scene=k)
        ref = oracle.bin_particles(b["x"], b["n"])
        assert np.array_equal(keys, ref["sorted"]), k
        assert np.array_equal(perm, ref["perm"]), k
        assert np.array_equal(blocks["gcode"], ref["gblock"]), k
        assert np.array_equal(blocks["gstart"], ref["gstart"]), k
        assert np.array_equal(blocks["gcount"], ref["gcount"]), k
        assert np.array_equal(blocks["active"], ref["pblock"]), k
    sim.close()


def test_frame_gives_each_scene_its_own_substep_count(torch_cuda, oracle):
    """A frame of 1 ms: scene s takes ceil(1e-3 / dt_s) substeps (5, 10 or 20
    here), the scenes with larger dt sitting out the later launches."""
    batch = small_batch(count=6, nmax=3000, seed=5)
    frame = 1e-3
    sim = make_batch(torch_cuda, batch)
    for k, b in enumerate(batch):
        sim.add_particles(b["mat"], b["x"], scene=k)
    sim.frame(frame)
    want = [math.ceil(frame / b["dt"] - 1e-4) for b in batch]
    assert len(set(want)) > 1, "the batch should mix time steps"
    for k, b in enumerate(batch):
        assert sim.scene_stats(k)["substeps"] == want[k]
        gs = {key: v.cpu().numpy() for key, v in sim.read_particles(scene=k).items()}
        os_, _, _, bad = oracle.substep(oracle_cfg(b), b["mat"], {"x": b["x"]}, steps=want[k])
        assert bad == 0
        compare_state(gs, os_, b["kind"], n=b["n"])
    sim.close()


def _run_frames(torch_cuda, batch, frames, frame_dt, separate=False, **kw):
    from paper_2111_00699_amd import mpm

    if separate:
        out = []
        for b in batch:
            sim = mpm.Sim(b["n"], b["dt"], bc=b["bc"], **kw)
            sim.add_particles(b["mat"], b["x"])
            for _ in range(frames):
                sim.frame(frame_dt)
            out.append(gpu_state(sim))
            sim.close()
        return out
    sim = make_batch(torch_cuda, batch, **kw)
    for k, b in enumerate(batch):
        sim.add_particles(b["mat"], b["x"], scene=k)
    for _ in range(frames):
        sim.frame(frame_dt)
    out = [{key: v.cpu().numpy() for key, v in sim.read_particles(scene=k).items()} for k in range(len(batch))]
    sim.close()
    return out


def _agree(a, b, n, tol):
    for k, (sa, sb) in enumerate(zip(a, b)):
        assert normwise(sa["x"], sb["x"]) <= tol, k
        # velocities: normwise against the larger of the field and one cell per frame
        scale = max(np.abs(sb["v"]).max(), 1.0 / n[k])
        assert np.abs(sa["v"] - sb["v"]).max() / scale <= 100 * tol, k


def test_batched_equals_one_scene_at_a_time(torch_cuda):
    batch = small_batch(count=6, seed=11)
    frame = 2e-3
    a = _run_frames(torch_cuda, batch, 2, frame)
    b = _run_frames(torch_cuda, batch, 2, frame, separate=True)
    _agree(a, b, [x["n"] for x in batch], 1e-5)


def test_frame_graphs_match_direct_frames(torch_cuda):
    """Graph frames replayed several times (each of the two buffer-parity
    graphs three times), with eager work and synchronisations between the
    replays; every frame is checked against the same frame run directly."""
    from paper_2111_00699_amd import mpm

    batch = small_batch(count=6, seed=12)
    frame = 2e-3
    s = torch_cuda.cuda.Stream()
    with torch_cuda.cuda.stream(s):
        sims = []
        for flags in (mpm.FLAG_FRAME_GRAPHS, 0):
            sim = make_batch(torch_cuda, batch, flags=flags, stream=s)
            for k, b in enumerate(batch):
                sim.add_particles(b["mat"], b["x"], scene=k)
            sims.append(sim)
        n = [x["n"] for x in batch]
        for f in range(7):
            for sim in sims:
                sim.frame(frame)
            got = [[{key: v.cpu().numpy() for key, v in sim.read_particles(scene=k).items()}
                    for k in range(len(batch))] for sim in sims]
            _agree(got[0], got[1], n, 5e-5)  # up to 280 substeps apart in summation order
            assert sims[0].stats()["error"] == 0
        for sim in sims:
            sim.close()


def test_autotune_restores_the_state(torch_cuda):
    batch = small_batch(count=4, seed=13)
    sim = make_batch(torch_cuda, batch)
    for k, b in enumerate(batch):
        sim.add_particles(b["mat"], b["x"], scene=k)
    sim.frame(1e-3)
    before = [{key: v.cpu().numpy() for key, v in sim.read_particles(scene=k).items()} for k in range(len(batch))]
    steps = [sim.scene_stats(k)["substeps"] for k in range(len(batch))]
    chunk = sim.autotune(1e-3, frames=1)
    assert chunk in (128, 256, 512)
    after = [{key: v.cpu().numpy() for key, v in sim.read_particles(scene=k).items()} for k in range(len(batch))]
    for x0, x1 in zip(before, after):
        for key in x0:
            assert np.array_equal(x0[key], x1[key]), key
    assert steps == [sim.scene_stats(k)["substeps"] for k in range(len(batch))]
    sim.frame(1e-3)
    assert sim.stats()["error"] == 0
    sim.close()
