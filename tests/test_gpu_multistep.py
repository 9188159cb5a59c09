"""Multi-step runs on the GPU against the FP64 oracle.

Over hundreds of substeps the FP32 state and the FP64 state drift apart
particle by particle, and atomics make the GPU's own sums order-dependent, so
whole frames are compared on conserved totals and bounding statistics:
  * mass: the particle count and the grid's total mass (FP32 sum, 1e-6);
  * momentum: before any wall contact its change is exactly M g t (the APIC
    transfer conserves momentum), checked on both sides;
  * the axis-aligned bounding box within 1 dx per face, the centre of mass
    within 0.1 dx and the kinetic energy within 1% of the oracle's, after one
    1/60 s frame.
The oracle runs its multi-threaded form (equal to the serial one up to FP64
rounding, pinned on the CPU).
"""
import os

import numpy as np
import pytest

from paper_2111_00699_amd import scenes

from .test_gpu_parity import gpu_state, make_sim, print_case

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a visible GPU")
    return torch


def totals(st, mp):
    x = np.asarray(st["x"], np.float64)
    v = np.asarray(st["v"], np.float64)
    N = x.shape[1]
    return dict(N=N, M=N * mp, P=mp * v.sum(axis=1), KE=0.5 * mp * (v * v).sum(),
                com=x.mean(axis=1), lo=x.min(axis=1), hi=x.max(axis=1), mv=mp * np.abs(v).sum(axis=1))


def compare_totals(g, o, n, label):
    dx = 1.0 / n
    d = dict(box=max(np.abs(g["lo"] - o["lo"]).max(), np.abs(g["hi"] - o["hi"]).max()) / dx,
             com=np.abs(g["com"] - o["com"]).max() / dx,
             ke=abs(g["KE"] - o["KE"]) / o["KE"])
    print(f"[totals] {label} N={g['N']} box/dx={d['box']:.3f} com/dx={d['com']:.4f} ke_rel={d['ke']:.2e} "
          f"KE gpu={g['KE']:.6e} oracle={o['KE']:.6e}", flush=True)
    assert g["N"] == o["N"]
    assert d["box"] <= 1.0
    assert d["com"] <= 0.1
    assert d["ke"] <= 1e-2
    return d


def test_snow_collision_frame_totals(torch_cuda, oracle):
    """Two pairs of snow spheres thrown together in mid-air (96,437
    particles, 128^3): one 1/60 s frame of 167 substeps in which they collide
    and deform plastically, with no wall contact."""
    sc = scenes.snow_collision()
    ns, dt = scenes.frame_substeps(1e-4)
    n = 128
    cfg = dict(n=n, dt=dt, bc="separate", bc_cells=3, gravity=(0.0, -9.8, 0.0))
    st = {"x": sc["x"], "v": sc["v"]}
    mp = scenes.SNOW["rho"] / n ** 3 / scenes.SNOW["ppc"]
    print_case("snow_collision_frame", N=sc["x"].shape[1], substeps=ns)
    sim = make_sim(torch_cuda, cfg)
    sim.add_particles(scenes.SNOW, sc["x"], v=sc["v"])
    sim.substep(ns)
    gs = gpu_state(sim)
    gm, _ = (t.cpu().numpy().astype(np.float64) for t in sim.read_grid())
    assert sim.stats()["error"] == 0
    sim.close()
    os_, om, _, bad = oracle.substep(cfg, scenes.SNOW, st, steps=ns, threads=THREADS)
    assert bad == 0
    t0 = totals(st, mp)
    g, o = totals(gs, mp), totals(os_, mp)
    # no wall contact: every stencil stays clear of the 3-cell wall layers
    dx = 1.0 / n
    assert o["lo"].min() > 5 * dx and o["hi"].max() < 1 - 5 * dx
    # the collision is plastic: J_P moved for a good share of the particles
    assert np.mean(np.abs(os_["s"] - 1.0) > 1e-3) > 0.1
    M = t0["M"]
    assert abs(gm.sum() - M) <= 1e-6 * M
    assert abs(om.sum() - M) <= 1e-12 * M
    expect = t0["P"] + ns * dt * M * np.array(cfg["gravity"])
    scale = max(t0["mv"].max(), g["mv"].max())
    print(f"[momentum] expect={expect} gpu={g['P']} oracle={o['P']} scale={scale:.3e}", flush=True)
    assert np.abs(o["P"] - expect).max() <= 1e-10 * scale
    assert np.abs(g["P"] - expect).max() <= 1e-5 * scale
    compare_totals(g, o, n, "snow_collision")


def test_fountain_frame_totals(torch_cuda, oracle):
    """The fountain (water, 128^3, separating slip walls) partway through a
    run: a pool on the floor and the jet above the inlet, plus the frame's
    emission at the inlet (143,500 particles in all); one 1/60 s frame of 167
    substeps against the walls and the pool."""
    cfg0 = scenes.fountain_config()
    n, ns, dt = cfg0["n"], cfg0["substeps_per_frame"], cfg0["dt"]
    cfg = dict(n=n, dt=dt, bc=cfg0["bc"], bc_cells=cfg0["bc_cells"], gravity=cfg0["gravity"])
    e = scenes.fountain_emission(30)
    base = scenes.fountain_midrun(limit=143500 - e["x"].shape[1])
    st = {"x": np.concatenate([base["x"], e["x"]], axis=1), "v": np.concatenate([base["v"], e["v"]], axis=1)}
    N = st["x"].shape[1]
    assert N == 143500
    mp = scenes.WATER["rho"] / n ** 3 / scenes.WATER["ppc"]
    print_case("fountain_frame", N=N, substeps=ns)
    sim = make_sim(torch_cuda, cfg)
    sim.add_particles(scenes.WATER, base["x"], v=base["v"])
    sim.add_particles(None, e["x"], v=e["v"])
    sim.substep(ns)
    gs = gpu_state(sim)
    gm, _ = (t.cpu().numpy().astype(np.float64) for t in sim.read_grid())
    assert sim.stats()["error"] == 0
    sim.close()
    os_, om, _, bad = oracle.substep(cfg, scenes.WATER, st, steps=ns, threads=THREADS)
    assert bad == 0
    M = N * mp
    assert abs(gm.sum() - M) <= 1e-6 * M
    g, o = totals(gs, mp), totals(os_, mp)
    # momentum is not conserved against the floor; compare it with the oracle's
    scale = max(o["mv"].max(), g["mv"].max())
    print(f"[momentum] gpu={g['P']} oracle={o['P']} scale={scale:.3e}", flush=True)
    assert np.abs(g["P"] - o["P"]).max() <= 1e-2 * scale
    compare_totals(g, o, n, "fountain")
    # the water volume stays near its rest volume (weakly compressible)
    J = np.asarray(gs["s"], np.float64)
    assert abs(J.mean() - os_["s"].mean()) <= 1e-3
