"""Pins of the oracle's ASFLIP transfer and automatic time step (CPU).

The paper names both (the fountain's integrator and its automatically deduced
steps) without their formulas; the oracle's reading is pinned by what the
transfer must reduce to and conserve:
  * flip = 0 is the APIC substep, bit for bit;
  * flip = 1 without forces keeps every particle's velocity (FLIP does not
    smooth), with positions moved by PIC (beta = 0) or by the particle's own
    velocity (beta = 1);
  * the velocity is linear in flip;
  * any flip conserves momentum: the particles carry the grid's momentum;
  * beta switches on compression: a converging cloud moves with beta_min, a
    diverging one with beta_max;
  * the frame step obeys its CFL bound, tiles the frame, and is the longest
    such step.
"""
import numpy as np
import pytest

from paper_2111_00699_amd import scenes

CFG = dict(n=64, dt=1e-4, bc="separate", gravity=(0.0, 0.0, 0.0))


def cloud(seed=3, N=4000):
    x = scenes.uniform(seed, 3 * N, 0, 0.3, 0.7).reshape(3, N).astype(np.float32)
    st = scenes.nontrivial_state(x, seed=seed, kind="water")
    return st


@pytest.mark.parametrize("kind", ["water", "jelly"])
def test_flip_zero_is_apic(oracle, kind):
    mat = scenes.WATER if kind == "water" else scenes.JELLY
    st = cloud()
    a, am, av, _ = oracle.substep(CFG, mat, st, steps=3)
    b, bm, bv, _ = oracle.substep_asflip(CFG, mat, st, 0.0, 0.0, 1.0, steps=3)
    for k in "xvCFs":
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(av, bv)


def test_flip_one_without_forces_keeps_velocities(oracle):
    st = cloud(5)
    mat = dict(scenes.JELLY, E=0.0)  # no stress, no gravity, no walls reached
    apic, _, _, _ = oracle.substep(CFG, mat, st)
    pic_pos, _, _, _ = oracle.substep_asflip(CFG, mat, st, 1.0, 0.0, 0.0)
    own_pos, _, _, _ = oracle.substep_asflip(CFG, mat, st, 1.0, 1.0, 1.0)
    v0 = st["v"].astype(np.float64)
    assert np.abs(pic_pos["v"] - v0).max() <= 1e-13
    assert np.abs(apic["v"] - v0).max() > 1e-2  # APIC smooths a random field
    assert np.array_equal(pic_pos["x"], apic["x"])
    assert np.abs(own_pos["x"] - (st["x"].astype(np.float64) + CFG["dt"] * v0)).max() <= 1e-15
    assert np.array_equal(pic_pos["C"], apic["C"])


def test_velocity_is_linear_in_flip(oracle):
    st = cloud(7)
    cfg = dict(CFG, gravity=(0.0, -9.8, 0.0))
    v = {a: oracle.substep_asflip(cfg, scenes.WATER, st, a, 0.0, 1.0)[0]["v"] for a in (0.0, 0.3, 1.0)}
    assert np.abs(v[0.3] - (0.7 * v[0.0] + 0.3 * v[1.0])).max() <= 1e-13 * np.abs(v[1.0]).max()


@pytest.mark.parametrize("flip", [0.0, 0.5, 0.95, 1.0])
def test_momentum_is_the_grids(oracle, flip):
    st = cloud(9)
    cfg = dict(CFG, gravity=(0.0, -9.8, 0.0))
    s, gm, gv, bad = oracle.substep_asflip(cfg, scenes.WATER, st, flip, 0.2, 0.9)
    assert bad == 0
    mp = scenes.WATER["rho"] / 64 ** 3 / 8
    p_part = mp * s["v"].sum(axis=1)
    p_grid = (gm[None, :] * gv).sum(axis=1)
    scale = mp * np.abs(s["v"]).sum()
    assert np.abs(p_part - p_grid).max() <= 1e-13 * scale
    # and the grid's is the particles' before, plus gravity (no wall reached)
    p0 = mp * st["v"].astype(np.float64).sum(axis=1) + cfg["dt"] * gm.sum() * np.array(cfg["gravity"])
    assert np.abs(p_grid - p0).max() <= 1e-13 * scale


@pytest.mark.parametrize("sign", [-1.0, 1.0])
def test_beta_follows_compression(oracle, sign):
    """A cloud converging (sign -1) or diverging (+1) affinely, with a random
    velocity on top: every particle's volume shrinks (grows), so positions
    move with beta_min (beta_max)."""
    st = cloud(11)
    x = st["x"].astype(np.float64)
    st["v"] = (sign * 20.0 * (x - 0.5) + 0.05 * st["v"]).astype(np.float32)
    st["C"] = (np.eye(3).reshape(9, 1) * sign * 20.0 + 0 * st["C"]).astype(np.float32)
    st["s"] = np.ones_like(st["s"])
    mat = dict(scenes.WATER, bulk=0.0)
    got = oracle.substep_asflip(CFG, mat, st, 0.8, 0.1, 0.7)[0]
    want_b = 0.1 if sign < 0 else 0.7
    ref = oracle.substep_asflip(CFG, mat, st, 0.8, want_b, want_b)[0]
    other = oracle.substep_asflip(CFG, mat, st, 0.8, 0.7 + 0.1 - want_b, 0.7 + 0.1 - want_b)[0]
    assert np.array_equal(got["x"], ref["x"])
    assert np.abs(got["x"] - other["x"]).max() > 0


def test_frame_step_obeys_the_bound_and_tiles_the_frame(oracle):
    n, frame = 128, 1.0 / 60.0
    for vmax in (0.0, 0.5, 3.0, 7.5, 40.0):
        for mat in (scenes.WATER, scenes.SNOW, scenes.JELLY):
            for dt_max in (1e-3, 2e-4):
                ns, dt = oracle.frame_time_step(mat, n, vmax, (0, -9.8, 0), 0.3, dt_max, frame)
                if mat is scenes.WATER:
                    c = np.sqrt(mat["bulk"] / mat["rho"])
                else:
                    E, nu, rho = mat["E"], mat["nu"], mat["rho"]
                    c = np.sqrt(E * (1 - nu) / ((1 + nu) * (1 - 2 * nu)) / rho)  # lambda + 2 mu = E(1-nu)/((1+nu)(1-2nu))
                bound = min(dt_max, 0.3 / n / (vmax + 9.8 * frame + c))
                assert abs(ns * dt - frame) <= 1e-15
                assert dt <= bound * (1 + 1e-12)
                assert ns == 1 or frame / (ns - 1) > bound  # one substep fewer would exceed it
