"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bars (the same inputs on both sides, generated from seeded scenes):
  * binning: particle codes, sort permutation, geometric blocks with their
    ranges and physical blocks are bit-exact;
  * one substep from a random non-trivial state: every particle field and
    the grid mass/velocity within 1e-4 normwise relative error
    (max|gpu - oracle| / max|oracle| per field);
  * short multi-step runs (20 substeps of the jelly scene) within the same
    bar, and the analytic free-fall / affine cases within FP32 rounding.
"""
import numpy as np
import pytest

from paper_2111_00699_amd import scenes

pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a visible GPU")
    return torch


def normwise(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    scale = np.abs(b).max()
    return np.abs(a - b).max() / (scale if scale > 0 else 1.0)


def make_sim(torch_cuda, cfg, **kw):
    from paper_2111_00699_amd import mpm

    return mpm.Sim(cfg["n"], cfg["dt"], bc=cfg.get("bc", "sticky"), bc_cells=cfg.get("bc_cells", 3),
                   gravity=cfg.get("gravity", (0.0, -9.8, 0.0)), **kw)


def gpu_state(sim):
    out = sim.read_particles()
    return {k: v.cpu().numpy() for k, v in out.items()}


# FP32 unit roundoff, and the multiple of the FP32 noise in C that C's error
# may reach where C itself is noise (see compare_state).
EPS32 = 2.0 ** -24
K_C = 32.0


def c_noise(v, n):
    """Size of FP32 cancellation noise in C' = (4/dx^2) sum_i w v_i (x_i - x_p)^T:
    for node velocities uniform up to rounding the sum is 0 in exact arithmetic,
    its terms are about |v| dx, and each node velocity carries a few ulps of
    its own, so FP32 leaves about eps |v| 4/dx = eps 4 n |v|."""
    return EPS32 * 4.0 * n * float(np.abs(np.asarray(v, np.float64)).max())


def compare_state(gs, os_, kind, tol=TOL, n=None, label=""):
    """Normwise errors per field, max|gpu - oracle| / max|oracle|, all printed.
    C passes if its normwise error is within tol or, with n given, if its
    largest error is within K_C times the FP32 noise c_noise(v, n): a state
    at rest or in uniform motion has C = 0 in FP64, while FP32 leaves noise of
    a few eps 4 n |v| (measured: up to 7.3 in free fall from rest).  The
    allowance is reported as C_scale = max(max|C|, K_C c_noise / tol)."""
    c_scale = np.abs(os_["C"]).max()
    if n is not None:
        c_scale = max(c_scale, K_C * c_noise(os_["v"], n) / tol)
    dC = np.abs(np.asarray(gs["C"], np.float64) - os_["C"]).max()
    errs = {"x": normwise(gs["x"], os_["x"]), "v": normwise(gs["v"], os_["v"]),
            "C": dC / max(c_scale, 1e-30)}
    if kind != "water":
        errs["F"] = normwise(gs["F"], os_["F"])
    if kind != "jelly":
        errs["s"] = normwise(gs["s"], os_["s"])
    noise = f" C_err/noise={dC / c_noise(os_['v'], n):.2f}" if n is not None and c_noise(os_["v"], n) > 0 else ""
    print(f"[errs] {label or kind} tol={tol:g} C_scale={c_scale:.3e} max|C|={np.abs(os_['C']).max():.3e}{noise} "
          + " ".join(f"{k}={e:.2e}" for k, e in errs.items()), flush=True)
    bad = {k: e for k, e in errs.items() if not e <= tol}
    assert not bad, f"normwise errors above {tol}: {bad} (all: {errs})"
    return errs


def print_case(name, **kw):
    print(f"[case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


# ------------------------------------------------------------------ binning
@pytest.mark.parametrize("n,which", [(64, "jelly"), (128, "cloud"), (256, "spheres")])
def test_binning_is_bit_exact(torch_cuda, oracle, n, which):
    if which == "jelly":
        x = scenes.jelly_cube(0)["x"]
    elif which == "cloud":  # ragged: not a multiple of any tile size
        x = scenes.uniform(41, 3 * 30001, 0, 0.05, 0.95).reshape(3, -1).astype(np.float32)
    else:
        x = scenes.snow_spheres(1, n=n, target=2.0e5, count=6, rmin=0.03, rmax=0.07)["x"]
    print_case("binning", n=n, which=which, N=x.shape[1])
    sim = make_sim(torch_cuda, dict(n=n, dt=1e-5))
    sim.add_particles(scenes.JELLY, x)
    sim.substep(1)
    keys, perm = sim.read_binning()
    blocks = sim.read_blocks()
    ref = oracle.bin_particles(x, n)
    assert ref["bad"] == 0
    assert np.array_equal(keys, ref["sorted"])
    assert np.array_equal(perm, ref["perm"])
    assert np.array_equal(blocks["gcode"], ref["gblock"])
    assert np.array_equal(blocks["gstart"], ref["gstart"])
    assert np.array_equal(blocks["gcount"], ref["gcount"])
    assert np.array_equal(blocks["active"], ref["pblock"])
    sim.close()


def _compact3(v):
    v = np.asarray(v, dtype=np.int64)
    out = np.zeros_like(v)
    for b in range(11):
        out |= ((v >> (3 * b)) & 1) << b
    return out


def dealt_slot(count, r):
    """Storage slot of rank r in a chunk of `count` particles: the ranks are
    dealt over the chunk's 16-lane passes in the pass order 0, 2, 4, ..., 1,
    3, 5, ..., the short last pass dropping out once full (the layout
    include/mpm.h documents)."""
    P = (count + 15) // 16
    last = count - 16 * (P - 1)
    order = list(range(0, P, 2)) + list(range(1, P, 2))
    seq = [p * 16 + q for q in range(16) for p in order if not (p == P - 1 and q >= last)]
    return seq[r]


def dealt_order(keys):
    """Positions of a chunk's particles (keys in sorted order, no rank bits)
    for each storage slot: ranked by the bank pair (x + 12 y + 8 z) mod 16 of
    their cell, then by block and cell, ties in sorted order; rank r is
    stored at dealt_slot(count, r)."""
    keys = np.asarray(keys, dtype=np.int64)
    b, c = keys >> 6, keys & 63
    x = 4 * _compact3(b) + _compact3(c)
    y = 4 * _compact3(b >> 1) + _compact3(c >> 1)
    z = 4 * _compact3(b >> 2) + _compact3(c >> 2)
    k = (((x + 12 * y + 8 * z) & 15) << 8) | (keys & 255)
    ranked = np.argsort(k, kind="stable")
    order = np.empty(keys.size, dtype=np.int64)
    for r, pos in enumerate(ranked):
        order[dealt_slot(keys.size, r)] = pos
    return order


def chunk_runs(gcode, gstart, gcount, chunk=256):
    """Chunks as (start, count): consecutive blocks of one 2x2x1 slab of blocks
    (equal code >> 2) are packed while they fit in `chunk` particles, larger
    blocks are cut into runs of `chunk` (the layout include/mpm.h documents)."""
    runs, g = [], 0
    gcode, gstart, gcount = list(map(int, gcode)), list(map(int, gstart)), list(map(int, gcount))
    while g < len(gcode):
        h = g
        while h < len(gcode) and gcode[h] >> 2 == gcode[g] >> 2:
            h += 1
        run0, runn = None, 0
        for b in range(g, h):
            n = gcount[b]
            if n > chunk:
                if runn:
                    runs.append((run0, runn))
                runn = 0
                runs += [(gstart[b] + i, min(chunk, n - i)) for i in range(0, n, chunk)]
            else:
                if runn and runn + n > chunk:
                    runs.append((run0, runn))
                    runn = 0
                if not runn:
                    run0 = gstart[b]
                runn += n
        if runn:
            runs.append((run0, runn))
        g = h
    return runs


def storage_order(perm, keys, gcode, gstart, gcount, chunk=256):
    """Insertion ids in storage order after a rebuild: each chunk's particles
    dealt over its 16-lane passes by bank pair (dealt_order)."""
    order = np.empty_like(perm)
    for c0, cc in chunk_runs(gcode, gstart, gcount, chunk):
        order[c0:c0 + cc] = perm[c0 + dealt_order(keys[c0:c0 + cc])]
    return order


def test_binning_after_motion_composes(torch_cuda, oracle):
    """A later rebuild stably sorts the CURRENT storage order."""
    sc = scenes.jelly_cube(0)
    st = scenes.nontrivial_state(sc["x"], seed=7)
    st["v"] = st["v"] * 40.0  # move several cells
    cfg = dict(n=64, dt=2e-4, gravity=(0, 0, 0))
    sim = make_sim(torch_cuda, cfg, flags=0x4)
    sim.add_particles(dict(scenes.JELLY, E=0.0), st["x"], v=st["v"])
    sim.substep(10)
    keys0, perm0 = sim.read_binning()
    b0 = sim.read_blocks()
    x_now = gpu_state(sim)["x"].astype(np.float32)
    sim.rebuild()
    sim.substep(1)
    keys1, perm1 = sim.read_binning()
    # oracle: positions in the storage order left by the first rebuild, then a stable sort
    order0 = storage_order(perm0, keys0, b0["gcode"], b0["gstart"], b0["gcount"])
    assert np.array_equal(np.sort(order0), np.arange(order0.size))
    xs = x_now[:, order0]
    k, _, _ = oracle.keys(xs, 64)
    p, srt = oracle.stable_sort(k)
    assert np.array_equal(keys1, srt)
    assert np.array_equal(perm1, order0[p])
    sim.close()


# --------------------------------------------------------- one substep parity
MATS = {"jelly": (scenes.JELLY, "sticky"), "snow": (scenes.SNOW, "separate"), "water": (scenes.WATER, "slip"),
        "sand": (scenes.SAND, "slip")}


@pytest.mark.parametrize("kind", ["jelly", "snow", "water", "sand"])
@pytest.mark.parametrize("mode", ["tile", "global", "every_step", "sorted_lanes", "g2p_global", "chunk128", "chunk512",
                                  "per_block"])
def test_single_substep_matches_oracle(torch_cuda, oracle, kind, mode):
    mat, bc = MATS[kind]
    sc = scenes.jelly_cube(0)
    st = scenes.nontrivial_state(sc["x"], seed=5, kind=kind)
    cfg = dict(n=64, dt=1e-4, bc=bc)
    flags = {"global": 0x2, "every_step": 0x1, "sorted_lanes": 0x8, "g2p_global": 0x10, "per_block": 0x800}.get(mode, 0)
    chunk = {"chunk128": 128, "chunk512": 512}.get(mode, 0)
    print_case("substep1", kind=kind, mode=mode, N=st["x"].shape[1])
    sim = make_sim(torch_cuda, cfg, flags=flags, chunk=chunk)
    sim.add_particles(mat, st["x"], v=st["v"], C=st["C"], F=st.get("F"), s=st.get("s"))
    sim.substep(1)
    gs = gpu_state(sim)
    gm, gv = (t.cpu().numpy() for t in sim.read_grid())
    os_, om, ov, bad = oracle.substep(cfg, mat, st)
    assert bad == 0
    compare_state(gs, os_, kind)
    assert normwise(gm, om) <= TOL
    assert normwise(gv, ov) <= TOL
    stats = sim.stats()
    assert stats["error"] == 0 and stats["rebuilds"] == 1
    sim.close()


def test_empty_context_then_particles(torch_cuda, oracle):
    """A context that holds no particles: substeps and frames are no-ops,
    reads return zero-length arrays and an all-zero grid, and no rebuild
    runs; particles added afterwards take their first substep as in a fresh
    context, within the single-substep bars."""
    mat, bc = MATS["snow"]
    sc = scenes.jelly_cube(0)
    st = scenes.nontrivial_state(sc["x"], seed=9, kind="snow")
    cfg = dict(n=64, dt=1e-4, bc=bc)
    print_case("empty_context", N=0)
    sim = make_sim(torch_cuda, cfg)
    sim.substep(3)
    sim.frame(1.0 / 60.0)
    empty = gpu_state(sim)
    assert all(a.shape[-1] == 0 for a in empty.values())
    gm, gv = (t.cpu().numpy() for t in sim.read_grid())
    assert not gm.any() and not gv.any()
    stats = sim.stats()
    assert stats["error"] == 0 and stats["rebuilds"] == 0
    print_case("empty_context_then_particles", N=st["x"].shape[1])
    sim.add_particles(mat, st["x"], v=st["v"], C=st["C"], F=st["F"], s=st["s"])
    sim.substep(1)
    gs = gpu_state(sim)
    gm, gv = (t.cpu().numpy() for t in sim.read_grid())
    stats = sim.stats()
    sim.close()
    os_, om, ov, bad = oracle.substep(cfg, mat, st)
    assert bad == 0
    compare_state(gs, os_, "snow")
    assert normwise(gm, om) <= TOL
    assert normwise(gv, ov) <= TOL
    assert stats["error"] == 0 and stats["rebuilds"] == 1


def test_ragged_multi_block_substep(torch_cuda, oracle):
    """30001 particles over many blocks at n=128, small chunks: many partial
    chunks and tiles, snow with the return map active."""
    x = scenes.uniform(42, 3 * 30001, 0, 0.1, 0.9).reshape(3, -1).astype(np.float32)
    st = scenes.nontrivial_state(x, seed=9, kind="snow")
    cfg = dict(n=128, dt=5e-5, bc="separate")
    sim = make_sim(torch_cuda, cfg, chunk=64)
    sim.add_particles(scenes.SNOW, st["x"], v=st["v"], C=st["C"], F=st["F"], s=st["s"])
    sim.substep(1)
    gs = gpu_state(sim)
    os_, om, ov, _ = oracle.substep(cfg, scenes.SNOW, st)
    compare_state(gs, os_, "snow")
    sim.close()


def test_sand_return_map_cases_on_gpu(torch_cuda, oracle):
    """Sand gradients spread over expansion (all strain released), the cone
    (plastic flow) and the elastic interior: one substep, and the three cases
    each cover a good share of the particles (classified on the oracle)."""
    sc = scenes.jelly_cube(0)
    st = scenes.nontrivial_state(sc["x"], seed=17, kind="sand")
    st["F"] = (np.eye(3).reshape(9, 1) + 2.0 * (st["F"].astype(np.float64) - np.eye(3).reshape(9, 1))).astype(np.float32)
    cfg = dict(n=64, dt=2e-4, bc="slip")
    print_case("sand_cases", N=st["x"].shape[1])
    sim = make_sim(torch_cuda, cfg)
    sim.add_particles(scenes.SAND, st["x"], v=st["v"], C=st["C"], F=st["F"], s=st["s"])
    sim.substep(1)
    gs = gpu_state(sim)
    sim.close()
    os_, _, _, bad = oracle.substep(cfg, scenes.SAND, st)
    assert bad == 0
    compare_state(gs, os_, "sand", n=64)
    N = st["x"].shape[1]
    Fh = np.einsum("nab,nbc->nac", np.eye(3) + cfg["dt"] * os_["C"].T.reshape(N, 3, 3),
                   st["F"].astype(np.float64).T.reshape(N, 3, 3))
    tr = np.log(np.abs(np.linalg.det(Fh)))
    dq = os_["s"] - st["s"].astype(np.float64)
    tip, cone, inside = tr > 0, (tr <= 0) & (dq > 0), (tr <= 0) & (dq == 0)
    assert min(tip.sum(), cone.sum(), inside.sum()) > N // 10, (tip.sum(), cone.sum(), inside.sum())


def test_sand_inverted_gradients_on_gpu(torch_cuda, oracle):
    """Sand with every fifth gradient inverted (one column negated): inside
    the cone the map keeps the trial gradient, inverted, on both sides; on
    the cone and in expansion both rebuild it from |sig|.  Three substeps, so
    the kept sign feeds the next substep's map."""
    sc = scenes.jelly_cube(0)
    st = scenes.nontrivial_state(sc["x"], seed=31, kind="sand")
    F = st["F"].astype(np.float64)
    F = np.eye(3).reshape(9, 1) + 2.0 * (F - np.eye(3).reshape(9, 1))
    inv = np.arange(F.shape[1]) % 5 == 0
    for k in (2, 5, 8):
        F[k, inv] = -F[k, inv]
    st["F"] = F.astype(np.float32)
    N = F.shape[1]
    assert np.all(np.linalg.det(st["F"].astype(np.float64).T.reshape(N, 3, 3))[inv] < 0)
    cfg = dict(n=64, dt=2e-4, bc="slip")
    print_case("sand_inverted", N=N, inverted=int(inv.sum()))
    sim = make_sim(torch_cuda, cfg)
    sim.add_particles(scenes.SAND, st["x"], v=st["v"], C=st["C"], F=st["F"], s=st["s"])
    sim.substep(3)
    gs = gpu_state(sim)
    sim.close()
    os_, _, _, bad = oracle.substep(cfg, scenes.SAND, st, steps=3)
    assert bad == 0
    compare_state(gs, os_, "sand", n=64)
    det = np.linalg.det(os_["F"].T.reshape(N, 3, 3))
    kept = inv & (det < 0)
    # both branches occur among the inverted particles
    assert kept.sum() > inv.sum() // 10 and (inv & (det > 0)).sum() > inv.sum() // 10, (kept.sum(), inv.sum())
    assert np.all(np.sign(np.linalg.det(gs["F"].astype(np.float64).T.reshape(N, 3, 3))) == np.sign(det))


def test_sand_blocks_substeps(torch_cuda, oracle):
    """The Sand Blocks layout (4 boxes of 12^3 cells, 55,296 particles) at the
    paper's time step, from a non-trivial state, 6 substeps on the slip box."""
    x = scenes.sand_blocks(l=12, boxes=4, n=128)["x"]
    st = scenes.nontrivial_state(x, seed=23, kind="sand")
    cfg = scenes.sand_config()
    cfg = dict(n=cfg["n"], dt=cfg["dt"], bc=cfg["bc"], bc_cells=cfg["bc_cells"], gravity=cfg["gravity"])
    print_case("sand_blocks6", N=x.shape[1])
    sim = make_sim(torch_cuda, cfg)
    sim.add_particles(scenes.SAND, st["x"], v=st["v"], C=st["C"], F=st["F"], s=st["s"])
    sim.substep(6)
    gs = gpu_state(sim)
    assert sim.stats()["error"] == 0
    sim.close()
    os_, _, _, bad = oracle.substep(cfg, scenes.SAND, st, steps=6)
    assert bad == 0
    compare_state(gs, os_, "sand", n=128)


# --------------------------------------------------------- multi-step runs
def test_jelly_twenty_substeps(torch_cuda, oracle):
    sc = scenes.jelly_cube(0)
    cfg = scenes.jelly_config()
    st = scenes.nontrivial_state(sc["x"], seed=5)
    sim = make_sim(torch_cuda, cfg)
    sim.add_particles(scenes.JELLY, st["x"], v=st["v"], C=st["C"], F=st["F"])
    sim.substep(20)
    gs = gpu_state(sim)
    os_, _, _, _ = oracle.substep(cfg, scenes.JELLY, st, steps=20)
    compare_state(gs, os_, "jelly")
    sim.close()


def test_free_fall_on_gpu(torch_cuda):
    sc = scenes.jelly_cube(0)
    cfg = scenes.jelly_config()
    sim = make_sim(torch_cuda, cfg)
    sim.add_particles(scenes.JELLY, sc["x"])
    steps = 20
    sim.substep(steps)
    gs = gpu_state(sim)
    dt, g = cfg["dt"], -9.8
    assert np.allclose(gs["v"][1], steps * dt * g, rtol=2e-5, atol=0)
    assert np.abs(gs["v"][[0, 2]]).max() < 1e-5
    x0 = sc["x"].astype(np.float64)
    assert np.abs(gs["x"][1] - (x0[1] + dt * dt * g * steps * (steps + 1) / 2)).max() < 2e-7
    assert np.abs(gs["C"]).max() < 2e-2  # FP32 cancellation in (4/dx)(M - v f^T)
    sim.close()


def test_affine_field_on_gpu(torch_cuda):
    n, N = 64, 20000
    x = scenes.uniform(8, 3 * N, 0, 0.3, 0.7).reshape(3, N).astype(np.float32)
    a = np.array([0.3, -0.2, 0.1])
    B = scenes.uniform(8, 9, 1, -2, 2).reshape(3, 3)
    v = (a[:, None] + B @ x.astype(np.float64)).astype(np.float32)
    C = np.repeat(B.reshape(9, 1), N, axis=1).astype(np.float32)
    sim = make_sim(torch_cuda, dict(n=n, dt=1e-4, gravity=(0, 0, 0)))
    sim.add_particles(dict(scenes.JELLY, E=0.0), x, v=v, C=C)
    sim.substep(1)
    gs = gpu_state(sim)
    assert normwise(gs["v"], v) < 1e-5
    assert normwise(gs["C"], C) < 1e-3
    sim.close()


@pytest.mark.parametrize("case", ["moving", "falling"])
def test_mass_and_momentum_on_gpu(torch_cuda, oracle, case):
    """Mass and APIC momentum over one substep, away from the walls.
    * P2G scatters the particle mass exactly: sum_i m_i = N m.
    * The affine and stress terms scatter no net momentum (sum_i w (x_i - x_p)
      = 0), so after the grid update sum_i m_i v_i = sum_p m v_p + dt M g.
    * G2P hands it back: sum_p m v'_p = sum_i m_i v_i.
    "moving": random v, C and F, no gravity; "falling": at rest with random
    C (affine momentum only), under gravity.  Tolerance: 1e-5 of
    sum_i m_i |v_i|, the magnitude of the FP32 terms summed."""
    sc = scenes.jelly_cube(0)
    st = scenes.nontrivial_state(sc["x"], seed=5)
    if case == "falling":
        st["v"] = np.zeros_like(st["v"])
        st["F"] = np.repeat(np.eye(3, dtype=np.float32).reshape(9, 1), st["x"].shape[1], axis=1)
        g = (0.0, -9.8, 0.0)
    else:
        g = (0.0, 0.0, 0.0)
    cfg = dict(n=64, dt=1e-4, gravity=g)
    print_case("momentum", case=case)
    sim = make_sim(torch_cuda, cfg)
    sim.add_particles(scenes.JELLY, st["x"], v=st["v"], C=st["C"], F=st["F"])
    sim.substep(1)
    gm, gv = (t.cpu().numpy().astype(np.float64) for t in sim.read_grid())
    gs = gpu_state(sim)
    sim.close()
    N = st["x"].shape[1]
    mp = scenes.JELLY["rho"] / 64 ** 3 / 8
    M = N * mp
    assert abs(gm.sum() - M) <= 1e-6 * M
    expect = mp * st["v"].astype(np.float64).sum(axis=1) + cfg["dt"] * M * np.array(g)
    p_grid = (gm[None, :] * gv).sum(axis=1)
    p_part = mp * gs["v"].astype(np.float64).sum(axis=1)
    scale = (gm[None, :] * np.abs(gv)).sum(axis=1).max()
    print(f"[momentum] expect={expect} grid={p_grid} particles={p_part} scale={scale:.3e}", flush=True)
    assert np.abs(p_grid - expect).max() <= 1e-5 * scale
    assert np.abs(p_part - expect).max() <= 1e-5 * scale
    if case == "falling":  # the gravity term itself is resolved to better than 1%
        assert 1e-5 * scale < 1e-2 * cfg["dt"] * M * 9.8
    # the oracle agrees on the totals
    _, om, ov, bad = oracle.substep(cfg, scenes.JELLY, st)
    assert bad == 0
    assert np.abs((om[None, :] * ov).sum(axis=1) - expect).max() <= 1e-12 * scale


def test_out_of_free_zone_without_rebuild(torch_cuda, oracle):
    """No rebuild for 40 substeps while particles travel ~5 cells: the
    overflow path (global atomics + block activation) keeps results exact."""
    sc = scenes.jelly_cube(0)
    st = scenes.nontrivial_state(sc["x"], seed=11)
    st["v"] = (st["v"] * 0.2 + np.array([[4.0], [2.0], [-3.0]])).astype(np.float32)
    st["C"] = st["C"] * np.float32(0.1)
    mat = dict(scenes.JELLY, E=100.0)  # soft: elastic CFL 0.32 at this dt
    cfg = dict(n=64, dt=5e-4, gravity=(0, -9.8, 0))
    sim = make_sim(torch_cuda, cfg, flags=0x4)
    sim.add_particles(mat, st["x"], v=st["v"], C=st["C"], F=st["F"])
    sim.substep(40)  # about 5 cells along x
    stats = sim.stats()
    assert stats["rebuilds"] == 1
    assert stats["overflow_blocks"] > 0
    gs = gpu_state(sim)
    os_, _, _, bad = oracle.substep(cfg, mat, st, steps=40)
    assert bad == 0
    # a translating cube: C is small against n |v|, the scale of its FP32 cancellation noise
    compare_state(gs, os_, "jelly", tol=2e-4, n=cfg["n"])
    sim.close()


def test_expanding_cloud_overflows_tiles(torch_cuda, oracle):
    """A cube expanding at 50/s with rebuilds switched off: blocks spread to
    twice their width, chunk boxes outgrow the LDS tile and whole chunks fall
    back to global atomics, while the result still matches the oracle."""
    sc = scenes.jelly_cube(0)
    st = scenes.nontrivial_state(sc["x"], seed=13)
    st["v"] = (50.0 * (st["x"] - np.float32(0.5)) + 0.05 * st["v"]).astype(np.float32)
    st["C"] = (np.eye(3, dtype=np.float32).reshape(9, 1) * np.float32(50.0) + 0.01 * st["C"]).astype(np.float32)
    mat = dict(scenes.JELLY, E=1.0)  # nearly free expansion
    cfg = dict(n=64, dt=5e-4, gravity=(0, 0, 0))
    print_case("expanding", N=st["x"].shape[1])
    sim = make_sim(torch_cuda, cfg, flags=0x4)
    sim.add_particles(mat, st["x"], v=st["v"], C=st["C"], F=st["F"])
    sim.substep(30)
    stats = sim.stats()
    assert stats["rebuilds"] == 1
    assert stats["p2g_fallback_chunks"] > 0, stats
    assert stats["p2g_global_particles"] > 0, stats
    gs = gpu_state(sim)
    os_, _, _, bad = oracle.substep(cfg, mat, st, steps=30)
    assert bad == 0
    compare_state(gs, os_, "jelly", tol=2e-4, n=cfg["n"])
    sim.close()


def test_full_registration_lists_fall_back_to_global_atomics(torch_cuda, oracle):
    """About 16 particles per cell and chunks of 64: a block's registration
    list (chunks whose stencils can reach it, at most 256) overflows for the
    central blocks, those chunks scatter with global atomics, and the substep
    still matches the oracle."""
    x = scenes.uniform(23, 3 * 32000, 0, 0.4, 0.6).reshape(3, -1).astype(np.float32)
    st = scenes.nontrivial_state(x, seed=19)
    cfg = dict(n=64, dt=1e-4)
    print_case("dense_registrations", N=x.shape[1])
    sim = make_sim(torch_cuda, cfg, chunk=64)
    sim.add_particles(scenes.JELLY, st["x"], v=st["v"], C=st["C"], F=st["F"])
    sim.substep(2)
    stats = sim.stats()
    assert stats["p2g_fallback_chunks"] > 0, stats
    assert stats["p2g_global_particles"] > 0, stats
    gs = gpu_state(sim)
    os_, _, _, bad = oracle.substep(cfg, scenes.JELLY, st, steps=2)
    assert bad == 0
    compare_state(gs, os_, "jelly", n=cfg["n"])
    sim.close()


def test_free_zone_triggers_rebuild(torch_cuda):
    sc = scenes.jelly_cube(0)
    v = np.zeros_like(sc["x"])
    v[0] = 3.0
    sim = make_sim(torch_cuda, dict(n=64, dt=5e-4, gravity=(0, 0, 0)), lag=1)
    sim.add_particles(dict(scenes.JELLY, E=100.0), sc["x"], v=v)  # elastic CFL 0.32
    sim.substep(60)  # 3 m/s * 30 ms = 0.09 = 5.8 cells
    sim.synchronize()
    stats = sim.stats()
    assert 2 <= stats["rebuilds"] <= 4, stats
    sim.close()


# ------------------------------------------------------- particle sources
def test_emission_between_substeps(torch_cuda, oracle):
    """Fountain-style: particles added between substeps (the deferred
    deformation update of the old particles is landed first)."""
    cfg = dict(n=128, dt=1e-4, bc="separate")
    e0 = scenes.fountain_emission(0)
    e1 = scenes.fountain_emission(1)
    e1["x"] = e1["x"] + np.float32(0.2)
    sim = make_sim(torch_cuda, cfg, capacity=1024)
    sim.add_particles(scenes.WATER, e0["x"], v=e0["v"])
    sim.substep(3)
    sim.add_particles(None, e1["x"], v=e1["v"])
    sim.substep(2)
    gs = gpu_state(sim)
    assert sim.stats()["capacity"] >= 2 * (e0["x"].shape[1] + e1["x"].shape[1])
    s0, _, _, _ = oracle.substep(cfg, scenes.WATER, e0, steps=3)
    both = {k: np.concatenate([s0[k], oracle._state(e1)[k]], axis=-1) for k in ("x", "v", "C", "F", "s")}
    s1, _, _, _ = oracle.substep(cfg, scenes.WATER, both, steps=2)
    compare_state(gs, s1, "water", n=cfg["n"])
    sim.close()


# ------------------------------------------------------------- fault words
def test_invalid_particles_raise_state_error(torch_cuda):
    from paper_2111_00699_amd import mpm

    x = scenes.jelly_cube(0)["x"].copy()
    x[0, 5] = np.nan
    x[1, 7] = 1.5
    sim = make_sim(torch_cuda, dict(n=64, dt=1e-4))
    sim.add_particles(scenes.JELLY, x)
    sim.substep(2)
    with pytest.raises(mpm.MPMError) as e:
        sim.read_particles()
    assert e.value.code == mpm.ESTATE
    st = sim.stats(check=False)
    assert st["error"] & mpm.ERR_NONFINITE and st["error"] & mpm.ERR_DOMAIN
    sim.clear_error()
    assert sim.stats()["error"] == 0
    sim.close()


def test_binding_rejects_bad_arguments(torch_cuda):
    from paper_2111_00699_amd import mpm

    sim = make_sim(torch_cuda, dict(n=64, dt=1e-4))
    x = scenes.jelly_cube(0)["x"]
    with pytest.raises(mpm.MPMError):
        sim.add_particles(None, x)  # first call needs a material
    sim.add_particles(scenes.JELLY, x)
    with pytest.raises(mpm.MPMError):
        sim.add_particles(scenes.SNOW, x)  # one material per context
    with pytest.raises(mpm.MPMError):
        sim.substep(-1)
    sim.close()


def test_profile_counts_launches(torch_cuda):
    """Phases launched per substep: with the fused G2P, a substep's G2P runs
    inside the next substep's P2G, and one G2P launch brings the state up to
    date when it is read; without fusion (node-box gather off) every substep
    launches its own G2P."""
    sc = scenes.jelly_cube(0)
    for flags, g2p_before, g2p_after in ((0, 0, 1), (0x10, 5, 5)):
        sim = make_sim(torch_cuda, scenes.jelly_config(), flags=flags)
        sim.add_particles(scenes.JELLY, sc["x"])
        sim.profile(0xF)
        sim.substep(5)
        prof = sim.profile_read()
        assert prof["p2g"]["launches"] == 5 and prof["grid"]["launches"] == 5
        assert prof["g2p"]["launches"] == g2p_before, flags
        assert prof["rebuild"]["launches"] == 1
        sim.read_particles()
        prof = sim.profile_read()
        assert prof["g2p"]["launches"] == g2p_after, flags
        assert all(prof[k]["ms"] > 0 for k in ("p2g", "grid", "g2p"))
        sim.close()
    # sampled: every 4th launch of each phase is bracketed (launches 0, 4, 8 of 10)
    from paper_2111_00699_amd import mpm

    sim = make_sim(torch_cuda, scenes.jelly_config())
    sim.add_particles(scenes.JELLY, sc["x"])
    sim.profile(mpm.PHASE_P2G | mpm.PHASE_GRID | mpm.PROFILE_EVERY(4))
    sim.substep(10)
    prof = sim.profile_read()
    assert prof["p2g"]["launches"] == 3 and prof["grid"]["launches"] == 3
    assert prof["g2p"]["launches"] == 0 and prof["rebuild"]["launches"] == 0
    assert prof["p2g"]["ms"] > 0
    sim.close()


@pytest.mark.parametrize("kind", ["snow", "sand"])
def test_fused_g2p_matches_separate_g2p_bit_for_bit(torch_cuda, kind):
    """The G2P fused into the next P2G computes the same values in the same
    order as the G2P launch: 40 substeps with reads in the middle, particles
    added between substeps and rebuilds at fixed substeps give identical
    states.  (Rebuilds are requested by hand because the fused form reports a
    free-zone exit one substep later, and every particle stays on the
    deterministic LDS tile path.)"""
    from paper_2111_00699_amd import mpm

    sc = scenes.jelly_cube(0)
    st = scenes.nontrivial_state(sc["x"], seed=29, kind=kind)
    extra = scenes.uniform(31, 3 * 500, 0, 0.1, 0.2).reshape(3, -1).astype(np.float32)
    cfg = dict(n=64, dt=1e-4, bc="separate")
    mat = MATS[kind][0]
    print_case("fused_vs_separate", kind=kind, N=st["x"].shape[1])
    out = {}
    for flags in (mpm.FLAG_FUSED_G2P, mpm.FLAG_SEPARATE_G2P):
        sim = make_sim(torch_cuda, cfg, flags=flags | mpm.FLAG_MANUAL_REBUILD)
        sim.add_particles(mat, st["x"], v=st["v"], C=st["C"], F=st["F"], s=st["s"])
        sim.substep(10)
        sim.rebuild()
        sim.substep(10)
        mid = gpu_state(sim)
        sim.add_particles(None, extra)
        sim.substep(10)
        sim.rebuild()
        sim.substep(10)
        stats = sim.stats()
        out[flags] = (mid, gpu_state(sim), stats["rebuilds"], stats["p2g_global_particles"])
        sim.close()
    a, b = out[mpm.FLAG_FUSED_G2P], out[mpm.FLAG_SEPARATE_G2P]
    assert a[2] == b[2] == 4, (a[2], b[2])
    assert a[3] == b[3] == 0
    for k in ("x", "v", "C", "F", "s"):
        assert np.array_equal(a[0][k], b[0][k]), ("mid", k)
        assert np.array_equal(a[1][k], b[1][k]), ("end", k)
