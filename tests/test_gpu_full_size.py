"""GPU parity at the benchmark's full sizes, in the launch configuration
bench.py times, and on degenerate inputs.

* The snow scene: 12 spheres, 1,280,602 particles, 256^3 grid, chunk 256,
  the bench's capacity and flags.  Binning is compared bit for bit and one
  substep from a random non-trivial state element by element (every
  particle, the whole node grid) with the FP64 oracle, which takes about a
  second for it.
* The 256-scene batch (4.3M particles): binning and one substep per scene.
* An empty scene inside a batch, a single particle, and particles pressed
  against every wall under each boundary condition.

Bars as in test_gpu_parity.py: binning bit-exact; FP32 state within 1e-4
normwise of the oracle."""
import numpy as np
import pytest

from paper_2111_00699_amd import scenes

from .test_gpu_parity import TOL, compare_state, gpu_state, make_sim, normwise, print_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a visible GPU")
    return torch


def snow_sim(N):
    """The simulator exactly as bench.py builds it for the snow scene."""
    from paper_2111_00699_amd import mpm

    cfg = scenes.snow_config()
    sim = mpm.Sim(cfg["n"], cfg["dt"], bc=cfg["bc"], bc_cells=cfg["bc_cells"], gravity=cfg["gravity"],
                  capacity=2 * N + 256)
    return sim, cfg


def assert_binning(sim, oracle, x, n, scene=0):
    keys, perm = sim.read_binning(scene=scene)
    blocks = sim.read_blocks(scene=scene)
    ref = oracle.bin_particles(x, n)
    assert ref["bad"] == 0
    assert np.array_equal(keys, ref["sorted"])
    assert np.array_equal(perm, ref["perm"])
    assert np.array_equal(blocks["gcode"], ref["gblock"])
    assert np.array_equal(blocks["gstart"], ref["gstart"])
    assert np.array_equal(blocks["gcount"], ref["gcount"])
    assert np.array_equal(blocks["active"], ref["pblock"])


def test_full_snow_scene_binning_is_bit_exact(torch_cuda, oracle):
    x = scenes.snow_spheres(1)["x"]
    print_case("full_snow_binning", N=x.shape[1])
    sim, cfg = snow_sim(x.shape[1])
    sim.add_particles(scenes.SNOW, x)
    sim.substep(1)
    assert_binning(sim, oracle, x, cfg["n"])
    sim.close()


def test_full_snow_scene_substep_matches_oracle(torch_cuda, oracle):
    x = scenes.snow_spheres(1)["x"]
    st = scenes.nontrivial_state(x, seed=7, kind="snow")
    N = x.shape[1]
    print_case("full_snow_substep", N=N)
    sim, cfg = snow_sim(N)
    sim.add_particles(scenes.SNOW, st["x"], v=st["v"], C=st["C"], F=st["F"], s=st["s"])
    sim.substep(1)
    stats = sim.stats()
    assert stats["p2g_global_particles"] == 0  # every particle took the LDS tile path
    gs = gpu_state(sim)
    gm, gv = (t.cpu().numpy() for t in sim.read_grid())
    sim.close()
    os_, om, ov, bad = oracle.substep(cfg, scenes.SNOW, st)
    assert bad == 0
    compare_state(gs, os_, "snow", n=cfg["n"])
    assert normwise(gm, om) <= TOL
    assert normwise(gv, ov) <= TOL


@pytest.mark.parametrize("boxes,n", [(4, 128), (16, 256)])
def test_full_sand_blocks_substep_matches_oracle(torch_cuda, oracle, boxes, n):
    """The Sand Blocks cases of 46^3-cell boxes the bench runs: 4 boxes
    (3,114,752 particles, n = 128) and 16 boxes (12,459,008 particles,
    n = 256). One substep from a random state, every particle and the whole
    node grid against the oracle."""
    from paper_2111_00699_amd import mpm

    x = scenes.sand_blocks(l=46, boxes=boxes, n=n)["x"]
    st = scenes.nontrivial_state(x, seed=29, kind="sand")
    N = x.shape[1]
    c = scenes.sand_config(n)
    cfg = dict(n=c["n"], dt=c["dt"], bc=c["bc"], bc_cells=c["bc_cells"], gravity=c["gravity"])
    print_case("full_sand_blocks", boxes=boxes, n=n, N=N)
    sim = mpm.Sim(cfg["n"], cfg["dt"], bc=cfg["bc"], bc_cells=cfg["bc_cells"], gravity=cfg["gravity"],
                  capacity=2 * N + 256)
    sim.add_particles(scenes.SAND, st["x"], v=st["v"], C=st["C"], F=st["F"], s=st["s"])
    sim.substep(1)
    gs = gpu_state(sim)
    gm, gv = (t.cpu().numpy() for t in sim.read_grid())
    sim.close()
    del x
    os_, om, ov, bad = oracle.substep(cfg, scenes.SAND, st)
    assert bad == 0
    compare_state(gs, os_, "sand", n=cfg["n"])
    assert normwise(gm, om) <= TOL
    assert normwise(gv, ov) <= TOL


def test_full_batch_substep_matches_oracle_per_scene(torch_cuda, oracle):
    """All 256 scenes of the batched workload (4.3M particles), one substep."""
    from paper_2111_00699_amd import mpm

    batch = scenes.batched_scenes(seed=3)
    N = sum(b["x"].shape[1] for b in batch)
    print_case("full_batch_substep", scenes=len(batch), N=N)
    descs = [dict(n=b["n"], dt=b["dt"], bc=b["bc"]) for b in batch]
    sim = mpm.Sim(64, 1e-4, scenes=descs, capacity=2 * N + 256)
    states = []
    for k, b in enumerate(batch):
        st = scenes.nontrivial_state(b["x"], seed=1000 + k, kind=b["kind"])
        states.append(st)
        sim.add_particles(b["mat"], st["x"], v=st["v"], C=st["C"], F=st["F"], s=st.get("s"), scene=k)
    sim.substep(1)
    for k, b in enumerate(batch):
        assert_binning(sim, oracle, b["x"], b["n"], scene=k)
        gs = {key: v.cpu().numpy() for key, v in sim.read_particles(scene=k).items()}
        os_, _, _, bad = oracle.substep(dict(n=b["n"], dt=b["dt"], bc=b["bc"]), b["mat"], states[k])
        assert bad == 0
        compare_state(gs, os_, b["kind"], n=b["n"])
    sim.close()


# ------------------------------------------------------------- degenerate
def test_empty_scene_inside_a_batch(torch_cuda, oracle):
    """Scene 1 of three holds no particles: it has no blocks, reads back
    empty, and the scenes around it still match the oracle."""
    from paper_2111_00699_amd import mpm

    batch = scenes.batched_scenes(seed=9, count=3, nmin=700, nmax=3000)
    descs = [dict(n=b["n"], dt=b["dt"], bc=b["bc"]) for b in batch]
    sim = mpm.Sim(64, 1e-4, scenes=descs)
    for k in (0, 2):
        sim.add_particles(batch[k]["mat"], batch[k]["x"], scene=k)
    sim.substep(2)
    assert sim.scene_stats(1)["gblocks"] == 0
    assert sim.read_particles(scene=1)["x"].shape == (3, 0)
    for k in (0, 2):
        b = batch[k]
        gs = {key: v.cpu().numpy() for key, v in sim.read_particles(scene=k).items()}
        os_, _, _, bad = oracle.substep(dict(n=b["n"], dt=b["dt"], bc=b["bc"]), b["mat"], {"x": b["x"]}, steps=2)
        assert bad == 0
        compare_state(gs, os_, b["kind"], n=b["n"])
    sim.close()


def test_single_particle(torch_cuda, oracle):
    x = np.array([[0.41], [0.52], [0.47]], dtype=np.float32)
    st = scenes.nontrivial_state(x, seed=3, kind="snow")
    cfg = dict(n=64, dt=1e-4, bc="separate")
    sim = make_sim(torch_cuda, cfg)
    sim.add_particles(scenes.SNOW, st["x"], v=st["v"], C=st["C"], F=st["F"], s=st["s"])
    sim.substep(3)
    gs = gpu_state(sim)
    os_, _, _, bad = oracle.substep(cfg, scenes.SNOW, st, steps=3)
    assert bad == 0
    compare_state(gs, os_, "snow", n=64)
    sim.close()


def test_particle_at_a_cell_edge_keeps_its_tiny_node(torch_cuda, oracle):
    """Lone particles whose fractional offset is one or a few ulps below 1.5
    (and above 0.5): their far nodes receive weights of 1e-12 and less and
    nothing else.  Such contributions bypass the fixed-point tile (which
    would resolve them to a handful of units) and keep those nodes'
    velocities; the grid is compared node by node (max norm)."""
    n = 64
    x = []
    for k, ulps in enumerate((1, 3, 40)):
        t = np.float32(21.5) - np.float32(ulps * 2.0 ** -19)   # x n = 21.5 - ulps * ulp(21.5)
        lo = np.float32(30.5) + np.float32(ulps * 2.0 ** -19)  # x n = 30.5 + ulps * ulp: f just above 0.5
        x.append([t / np.float32(n), np.float32(24.3 + 9 * k) / np.float32(n), lo / np.float32(n)])
    x = np.array(x, dtype=np.float32).T.copy()
    st = scenes.nontrivial_state(x, seed=11, kind="snow")
    cfg = dict(n=n, dt=1e-4, bc="separate")
    print_case("cell_edge", N=x.shape[1])
    sim = make_sim(torch_cuda, cfg)
    sim.add_particles(scenes.SNOW, st["x"], v=st["v"], C=st["C"], F=st["F"], s=st["s"])
    sim.substep(1)
    gs = gpu_state(sim)
    gm, gv = (t.cpu().numpy() for t in sim.read_grid())
    sim.close()
    os_, om, ov, bad = oracle.substep(cfg, scenes.SNOW, st)
    assert bad == 0
    assert om[om > 0].min() < 1e-12 * om.max()  # the case the test is about
    compare_state(gs, os_, "snow", n=n)
    assert normwise(gm, om) <= TOL
    assert normwise(gv, ov) <= TOL


@pytest.mark.parametrize("bc", ["sticky", "slip", "separate"])
def test_particles_against_every_wall(torch_cuda, oracle, bc):
    """Slabs of particles within 0.6-4 cells of each of the six walls, moving
    into them: the boundary band (3 cells) acts on every face."""
    n = 64
    dx = 1.0 / n
    u = scenes.uniform(17, 3 * 6 * 400, 0, 0.0, 1.0).reshape(6, 3, 400)
    slabs, vel = [], []
    for face in range(6):
        a, hi = face // 2, face % 2
        p = 0.3 + 0.4 * u[face]
        d = (0.6 + 3.4 * u[face][a]) * dx
        p[a] = 1.0 - d if hi else d
        slabs.append(p)
        v = np.zeros_like(p)
        v[a] = 2.0 if hi else -2.0
        vel.append(v)
    x = np.concatenate(slabs, axis=1).astype(np.float32)
    v = np.concatenate(vel, axis=1).astype(np.float32)
    st = {"x": x, "v": v}
    cfg = dict(n=n, dt=1e-4, bc=bc, gravity=(0.0, -9.8, 0.0))
    print_case("walls", bc=bc, N=x.shape[1])
    sim = make_sim(torch_cuda, cfg)
    sim.add_particles(scenes.JELLY, x, v=v)
    sim.substep(3)
    gs = gpu_state(sim)
    os_, _, _, bad = oracle.substep(cfg, scenes.JELLY, st, steps=3)
    assert bad == 0
    compare_state(gs, os_, "jelly", n=n)
    sim.close()
