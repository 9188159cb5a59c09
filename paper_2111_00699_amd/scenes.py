"""Seeded synthetic inputs shaped like the paper's workloads.

This module only creates inputs (positions, initial velocities and material
states, material constants and run settings); it contains none of the
simulation method's arithmetic, so both the HIP path and the FP64 oracle can be
fed from it.  Random numbers come from a counter-based splitmix64 stream
(Steele, Lea and Flood 2014) so the arrays do not depend on numpy's generator
versions.

Workloads (Results section of the paper; sizes as printed there where given):
  * jelly cube  -- 64^3 grid, a 0.25^3 cube of fixed-corotated jelly, 8 ppc;
  * snow        -- 12 seeded spheres, about 1.33M particles (the size of the
                   paper's "Crawling in Snow" scene), 256^3 grid;
  * fountain    -- water emitted from a 0.05-radius inlet at 3 m/s, growing
                   to about 143.5K particles (the paper's fountain size);
  * sand blocks -- 4 or 16 boxes of l^3 cells at 8 ppc (l = 12, 23, 46).
Particle samples are stratified: one uniform sample in each of the 2x2x2
half-cell sub-cubes of every covered cell (the paper seeds its blocks "in a
stratified random way" at 8 particles per cell).
"""
from __future__ import annotations

import math

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)


def splitmix64(seed: int, count: int, stream: int = 0) -> np.ndarray:
    """`count` consecutive splitmix64 outputs for (seed, stream) as uint64."""
    with np.errstate(over="ignore"):
        base = np.uint64((int(seed) * 0x100000001B3 + int(stream) * 0xD1B54A32D192ED03) & (2**64 - 1))
        z = base + (np.arange(1, count + 1, dtype=np.uint64) * GOLDEN)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, count: int, stream: int = 0, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """Uniform float64 in [lo, hi) from the top 53 bits of splitmix64."""
    u = (splitmix64(seed, count, stream) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return lo + (hi - lo) * u


# ------------------------------------------------------------------ materials
JELLY = dict(kind="jelly", E=1e4, nu=0.2, rho=1.0, ppc=8.0)
SNOW = dict(kind="snow", E=1.4e5, nu=0.2, rho=400.0, ppc=8.0, theta_c=2.5e-2, theta_s=7.5e-3, xi=10.0)
WATER = dict(kind="water", rho=1000.0, ppc=8.0, bulk=1e4)
# Drucker-Prager sand (Klar et al. 2016's hardening constants h0..h3; its Young's
# modulus scaled down tenfold so that the Sand Blocks time step of 1/48 s / 36
# stays below the elastic wave's CFL limit on cells of 1/128)
SAND = dict(kind="sand", E=3.537e4, nu=0.3, rho=2200.0, ppc=8.0, h0=35.0, h1=9.0, h2=0.2, h3=10.0)

FRAME = 1.0 / 60.0


def frame_substeps(dt_nominal: float, frame: float = FRAME) -> tuple[int, float]:
    """Substeps per frame and the effective dt: ceil(frame/dt) steps of frame/steps."""
    ns = int(math.ceil(frame / dt_nominal - 1e-9))
    return ns, frame / ns


# ---------------------------------------------------------------- samplers
def stratified_cells(cells: np.ndarray, n: int, seed: int, stream: int = 0) -> np.ndarray:
    """One uniform sample per half-cell sub-cube of each cell in `cells` (K,3 ints).
    Returns FP32 positions (3, 8K), cell-major in the order given."""
    K = cells.shape[0]
    dx = 1.0 / n
    sub = np.array([[i, j, k] for i in range(2) for j in range(2) for k in range(2)], dtype=np.float64)
    u = uniform(seed, 3 * 8 * K, stream).reshape(K, 8, 3)
    pos = (cells[:, None, :].astype(np.float64) + 0.5 * (sub[None, :, :] + u)) * dx
    return np.ascontiguousarray(pos.reshape(-1, 3).T.astype(np.float32))


def box_cells(lo_cell, hi_cell) -> np.ndarray:
    """All integer cells in [lo, hi) per axis, as (K,3), x fastest."""
    rng = [np.arange(lo_cell[a], hi_cell[a]) for a in range(3)]
    gz, gy, gx = np.meshgrid(rng[2], rng[1], rng[0], indexing="ij")
    return np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)


def jelly_cube(seed: int = 0, n: int = 64, lo: float = 0.375, hi: float = 0.625) -> dict:
    """The 64^3 jelly parity scene: cube [lo,hi]^3 at 8 ppc, at rest."""
    lc = int(round(lo * n))
    hc = int(round(hi * n))
    x = stratified_cells(box_cells((lc,) * 3, (hc,) * 3), n, seed)
    return {"x": x}


def nontrivial_state(x: np.ndarray, seed: int = 5, kind: str = "jelly") -> dict:
    """A random, non-trivial particle state around positions x (3,N):
    v ~ U(-0.5,0.5) m/s, C ~ U(-5,5) 1/s, F = I + U(-0.05,0.05) per entry
    (det F > 0.8 for such perturbations), and J_P ~ U(0.9,1.05) (snow) or
    J ~ U(0.95,1.05) (water), or 1 + q with the hardening state q ~ U(0,0.5)
    (sand)."""
    N = x.shape[1]
    v = uniform(seed, 3 * N, 1, -0.5, 0.5).reshape(3, N)
    C = uniform(seed, 9 * N, 2, -5.0, 5.0).reshape(9, N)
    F = uniform(seed, 9 * N, 3, -0.05, 0.05).reshape(9, N)
    F[[0, 4, 8]] += 1.0
    assert np.all(np.linalg.det(F.T.reshape(N, 3, 3)) > 0.5)
    st = {"x": x, "v": v.astype(np.float32), "C": C.astype(np.float32), "F": F.astype(np.float32)}
    if kind == "snow":
        st["s"] = uniform(seed, N, 4, 0.9, 1.05).astype(np.float32)
    elif kind == "water":
        st["s"] = uniform(seed, N, 4, 0.95, 1.05).astype(np.float32)
    elif kind == "sand":
        st["s"] = uniform(seed, N, 4, 1.0, 1.5).astype(np.float32)
    return st


def snow_spheres(seed: int = 1, n: int = 256, target: float = 1.33e6, count: int = 12,
                 rmin: float = 0.04, rmax: float = 0.1) -> dict:
    """12 non-overlapping spheres; the radius vector is redrawn until the
    volume estimate 8 * sum(4/3 pi r^3) / dx^3 is within 5% of `target`."""
    dx = 1.0 / n
    trial = 0
    while True:
        r = uniform(seed, count, 100 + trial, rmin, rmax)
        est = 8.0 * np.sum(4.0 / 3.0 * np.pi * r ** 3) / dx ** 3
        trial += 1
        if abs(est - target) <= 0.05 * target:
            break
    r = np.sort(r)[::-1]
    lo = np.array([0.15, 0.30, 0.15])
    hi = np.array([0.85, 0.85, 0.85])
    centers = []
    draw = 0
    for i in range(count):
        while True:
            c = lo + (hi - lo) * uniform(seed, 3, 10000 + draw)
            draw += 1
            ok = all(np.linalg.norm(c - cj) >= r[i] + rj + 2 * dx for cj, rj in zip(centers, r[:i]))
            if ok:
                break
        centers.append(c)
    centers = np.array(centers)
    pieces = []
    for i in range(count):
        lc = np.floor((centers[i] - r[i]) / dx).astype(int)
        hc = np.ceil((centers[i] + r[i]) / dx).astype(int)
        x = stratified_cells(box_cells(lc, hc), n, seed, stream=200 + i)
        d = x.astype(np.float64) - centers[i][:, None]
        keep = np.sum(d * d, axis=0) <= r[i] ** 2
        pieces.append(x[:, keep])
    x = np.ascontiguousarray(np.concatenate(pieces, axis=1))
    return {"x": x, "centers": centers, "radii": r}


def free_fall_state(x: np.ndarray, cfg: dict, k: int) -> dict:
    """State of particles released at rest at x after k substeps of free fall
    (no stress, no wall contact): the symplectic-Euler closed form
    v_k = k dt g, x_k = x_0 + dt^2 g k (k + 1) / 2.  Raises if a particle's
    stencil would have reached a wall layer by then."""
    dt = cfg["dt"]
    g = np.asarray(cfg["gravity"], dtype=np.float64)[:, None]
    xk = x.astype(np.float64) + dt * dt * g * (k * (k + 1) / 2.0)
    dx = 1.0 / cfg["n"]
    b = cfg.get("bc_cells", 3)
    if xk.min() < (b + 2) * dx or xk.max() > 1.0 - (b + 2) * dx:
        raise ValueError("free_fall_state: the particles reach a wall layer before substep %d" % k)
    v = np.repeat(k * dt * g, x.shape[1], axis=1)
    return {"x": xk.astype(np.float32), "v": v.astype(np.float32)}


def fountain_emission(frame: int, seed: int = 2, n: int = 128, radius: float = 0.05,
                      center=(0.5, 0.1, 0.5), height: float = 0.05, speed: float = 3.0) -> dict:
    """One frame's emission: stratified 8-ppc samples in the inlet cylinder
    (axis +y, radius 0.05, y in [0.1, 0.15]) moving up at 3 m/s."""
    dx = 1.0 / n
    cx, cy, cz = center
    lc = np.floor(np.array([cx - radius, cy, cz - radius]) / dx).astype(int)
    hc = np.ceil(np.array([cx + radius, cy + height, cz + radius]) / dx).astype(int)
    x = stratified_cells(box_cells(lc, hc), n, seed, stream=1000 + frame)
    xd = x.astype(np.float64)
    keep = ((xd[0] - cx) ** 2 + (xd[2] - cz) ** 2 <= radius ** 2) & (xd[1] >= cy) & (xd[1] < cy + height)
    x = np.ascontiguousarray(x[:, keep])
    v = np.zeros_like(x)
    v[1] = speed
    return {"x": x, "v": v}


def fountain_midrun(seed: int = 2, n: int = 128, limit: int = 143500) -> dict:
    """The fountain partway through a run, built directly (not simulated): a
    pool at rest on the floor (x, z in [0.25, 0.75), from the wall layer up
    three cells) and the jet above the inlet (radius 0.05 around x = z = 0.5,
    y in [0.15, top)) moving up at the ballistic speed sqrt(9 - 2 g (y - 0.1))
    of water leaving the inlet at 3 m/s; 8 ppc stratified.  The inlet
    cylinder itself (y in [0.1, 0.15)) is left free for the next frame's
    emission.  `top` is the highest cell row that keeps the total within
    `limit` particles."""
    dx = 1.0 / n
    b = 3
    lo = int(round(0.25 * n))
    hi = int(round(0.75 * n))
    pool = stratified_cells(box_cells((lo, b, lo), (hi, b + 3, hi)), n, seed, stream=2000)
    r = 0.05
    lc = np.floor(np.array([0.5 - r, 0.15, 0.5 - r]) / dx).astype(int)
    hc = np.ceil(np.array([0.5 + r, 0.5, 0.5 + r]) / dx).astype(int)
    jet = stratified_cells(box_cells(lc, hc), n, seed, stream=2001)
    jd = jet.astype(np.float64)
    jet = jet[:, ((jd[0] - 0.5) ** 2 + (jd[2] - 0.5) ** 2 <= r * r) & (jd[1] >= 0.15)]
    room = limit - pool.shape[1]
    if jet.shape[1] > room:  # drop the highest rows (the cells are y-major in box_cells)
        order = np.argsort(jet[1], kind="stable")
        jet = jet[:, np.sort(order[:room])]
    x = np.ascontiguousarray(np.concatenate([pool, jet], axis=1))
    v = np.zeros_like(x)
    vy = np.sqrt(np.maximum(9.0 - 2.0 * 9.8 * (jet[1].astype(np.float64) - 0.1), 0.0))
    v[1, pool.shape[1]:] = vy.astype(np.float32)
    return {"x": x, "v": v}


def snow_collision(seed: int = 7, n: int = 128, r: float = 0.07, speed: float = 2.0) -> dict:
    """Two pairs of snow spheres (radius r, 8 ppc stratified) thrown at each
    other in mid-air at +-speed along x, 0.02 apart: they meet about 5 ms in
    and are pressed together for the rest of a 1/60 s frame, well away from
    every wall.  Pairs at z = 0.3 and 0.7, all centres at y = 0.6."""
    dx = 1.0 / n
    pieces, vel = [], []
    k = 0
    for zc in (0.3, 0.7):
        for side in (-1.0, 1.0):
            c = np.array([0.5 + side * (r + 0.01), 0.6, zc])
            lc = np.floor((c - r) / dx).astype(int)
            hc = np.ceil((c + r) / dx).astype(int)
            x = stratified_cells(box_cells(lc, hc), n, seed, stream=3000 + k)
            d = x.astype(np.float64) - c[:, None]
            x = x[:, np.sum(d * d, axis=0) <= r * r]
            v = np.zeros_like(x)
            v[0] = -side * speed
            pieces.append(x)
            vel.append(v)
            k += 1
    return {"x": np.ascontiguousarray(np.concatenate(pieces, axis=1)),
            "v": np.ascontiguousarray(np.concatenate(vel, axis=1))}


def sand_blocks(l: int = 12, boxes: int = 4, n: int = 128, seed: int = 6) -> dict:
    """The paper's Sand Blocks layout: `boxes` cubes of l^3 cells at 8 ppc
    (4 x 12^3 x 8 = 55,296 particles), side by side with a two-cell gap."""
    side = int(round(boxes ** (1 / 2)))
    gap = 2
    total = side * l + (side - 1) * gap
    start = (n - total) // 2
    cells = []
    for bz in range(side):
        for bx in range(side):
            lo = (start + bx * (l + gap), n // 8, start + bz * (l + gap))
            cells.append(box_cells(lo, (lo[0] + l, lo[1] + l, lo[2] + l)))
    x = stratified_cells(np.concatenate(cells), n, seed)
    return {"x": x}


# ------------------------------------------------------------- run settings
def snow_config(n: int = 256) -> dict:
    ns, dt = frame_substeps(5e-5)
    return dict(n=n, bc="separate", bc_cells=3, gravity=(0.0, -9.8, 0.0), dt=dt, substeps_per_frame=ns)


def jelly_config(n: int = 64) -> dict:
    return dict(n=n, bc="sticky", bc_cells=3, gravity=(0.0, -9.8, 0.0), dt=1e-4, substeps_per_frame=167)


def sand_config(n: int = 128) -> dict:
    """Sand Blocks: a frictionless (slip) box, 36 substeps per 1/48 s frame on
    cells of 1/128 (the paper's step); finer grids keep the step's CFL number
    (72 substeps on cells of 1/256)."""
    ns = 36 * n // 128
    return dict(n=n, bc="slip", bc_cells=3, gravity=(0.0, -9.8, 0.0), dt=(1.0 / 48.0) / ns, substeps_per_frame=ns,
                frame=1.0 / 48.0)


def fountain_config(n: int = 128) -> dict:
    ns, dt = frame_substeps(1e-4)
    return dict(n=n, bc="separate", bc_cells=3, gravity=(0.0, -9.8, 0.0), dt=dt, substeps_per_frame=ns)


# ------------------------------------------------------------ surrogate inputs
BATCH_MATS = {"jelly": (JELLY, "sticky", 1e-4, 64), "snow": (SNOW, "separate", 5e-5, 256),
              "water": (WATER, "separate", 1e-4, 128)}


def batched_scenes(seed: int = 3, count: int = 256, nmin: int = 2048, nmax: int = 65536,
                   grids=(64, 128)) -> list[dict]:
    """Many small, uneven real-time scenes.  Per scene (seeded splitmix64
    stream k): grid n uniform over `grids`; particle count log-uniform in
    [nmin, nmax], realised as a cube of k^3 cells at 8 ppc (k = round((N/8)^(1/3)),
    so N = 8 k^3) centred in x and z with its bottom at y = 0.4; material
    uniform over jelly / snow / water; dt = dt_ref * n_ref / n with (dt_ref,
    n_ref) = (1e-4, 64) jelly, (5e-5, 256) snow, (1e-4, 128) water, i.e. the
    single-scene time steps scaled to the grid, 84 to 334 substeps per 1/60 s
    frame.  Returns dicts with n, dt, bc, mat, kind, x."""
    out = []
    kinds = ("jelly", "snow", "water")
    for k in range(count):
        u = uniform(seed, 3, stream=k)
        n = int(grids[min(int(u[0] * len(grids)), len(grids) - 1)])
        N = float(np.exp(np.log(nmin) + u[1] * (np.log(nmax) - np.log(nmin))))
        kind = kinds[min(int(u[2] * 3), 2)]
        cells = max(2, int(round((N / 8.0) ** (1.0 / 3.0))))
        cells = min(cells, n // 2 - 6)
        lo = [(n - cells) // 2, int(0.4 * n), (n - cells) // 2]
        x = stratified_cells(box_cells(lo, [lo[0] + cells, lo[1] + cells, lo[2] + cells]), n, seed, stream=1000 + k)
        mat, bc, dt_ref, n_ref = BATCH_MATS[kind]
        out.append(dict(n=n, dt=dt_ref * n_ref / n, bc=bc, mat=mat, kind=kind, x=x))
    return out


MLP_LAYERS = (12, 64, 64, 12)


def mlp_init(seed: int = 4) -> np.ndarray:
    """Seeded initial parameters of the 12-64-64-12 surrogate network as one
    flat FP32 vector [W1 (64x12), b1, W2 (64x64), b2, W3 (12x64), b3]: weights
    uniform in +-sqrt(6/(fan_in + fan_out)) (Glorot), biases zero."""
    parts = []
    for k, (a, b) in enumerate(zip(MLP_LAYERS[:-1], MLP_LAYERS[1:])):
        lim = np.sqrt(6.0 / (a + b))
        parts.append(uniform(seed, a * b, 500 + k, -lim, lim))
        parts.append(np.zeros(b))
    return np.concatenate(parts).astype(np.float32)


def snow_trial_states(seed: int, count: int, spread: float = 0.02) -> dict:
    """Seeded trial states for the snow map in principal space: singular values
    1 + U(-spread, spread) and plastic volumes J_P ~ U(0.85, 1.1).  With the
    default spread about two thirds of the samples lie outside
    [1 - 2.5e-2, 1 + 7.5e-3] on some axis, so the clamp is exercised."""
    s = 1.0 + uniform(seed, 3 * count, 600, -spread, spread).reshape(count, 3)
    jp = uniform(seed, count, 601, 0.85, 1.1)
    return {"sig_hat": s, "Jp": jp}
