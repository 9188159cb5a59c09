"""Benchmark: the snow scene (12 seeded spheres, ~1.28M particles, 256^3 grid).

One benchmark step is one 1/60 s frame: 334 substeps of 4.99e-5 s, each a
full pass of the hot path (rebuild-mapping + radix sort when a particle left
its free zone, P2G with the fused snow return map and stress, grid update
with boundary conditions, G2P with the free-zone test).  Prints ONE JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--workload snow|fountain|batched|surrogate|ablations|sand]

By default K = 60 timed frames after W = 1 warmup frame, so `value` is the
average over 60 frames of the falling, landing and settling snow, as the
paper averages its frame costs.  `value` is particle-substeps per second over
the K timed frames (inputs resident in HBM before timing starts).
`roofline` covers the P2G kernel, timed with HIP events on the library's
stream during the timed frames, against the HBM peak (`frac` from the
algorithmic bytes, `traffic_frac` from the measured HBM bytes);
`roofline_valu` puts them against the VALU issue rate (the kernel's counted
instructions at full issue: a floor under its time), `roofline_lds`
against the LDS 64-bit atomic rate; `cpu_baseline` times the FP64 oracle on
the host on a bounded sample.  The other workloads print their own line: the fountain (ms per
frame against the growing particle count), 256 batched scenes, and the
learned constitutive map.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# P2G launches are timed with HIP events on a sample: every PROFILE_EVERY-th
# launch of the timed frames, about 310 of the 20,040 (each event pair holds
# the stream back a few microseconds; bracketing all launches would cost the
# frame time about 4%).
PROFILE_EVERY = 64
# LDS 64-bit integer atomic throughput of gfx950, measured with a probe of
# ds_add_u64 on distinct addresses: 9.1 lane-operations per clock per compute
# unit, i.e. 9.1 x 256 CUs x 2.4 GHz.  P2G's fixed-point scatter issues 27
# nodes x 4 channels of them per in-zone particle.
LDS_U64_ATOMIC_PEAK = 9.1 * 256 * 2.4e9
P2G_LDS_ATOMICS_PER_PARTICLE = 108
# The surrogate MLP 12-64-64-12 as executed on MFMA (inputs and outputs padded
# to 16): 16x64 + 64x64 + 64x16 = 6,144 multiply-adds per forward pass; a
# training sample adds the weight gradients (6,144) and the activation
# deltas of layers 2 and 3 (4,096 + 1,024).
MLP_FWD_FLOPS = 2 * 6144
MLP_TRAIN_FLOPS = 2 * (6144 + 6144 + 5120)
MFMA_BF16_PEAK_TFLOPS = 2500.0
# Algorithmic bytes per particle and launch (FP32 state, deferred deformation
# update): P2G reads x, v, C, F_E, J_P (100 B) and writes F_E, J_P (40 B);
# G2P reads x (12 B) and writes x, v, C (60 B).
P2G_BYTES = {"jelly": 132, "snow": 140, "water": 68}
# P2G with the previous substep's G2P inside it (the default): reads x, F_E,
# J_P and the block word (56 B), writes x, F_E, J_P (52 B); v and C stay in
# registers.
P2G_FUSED_BYTES = {"snow": 108}
G2P_BYTES = 72
# Algorithmic bytes per particle-substep of the whole substep (P2G + G2P of
# the two-kernel form): what one fused launch is priced at.
SUBSTEP_BYTES = {m: P2G_BYTES[m] + G2P_BYTES for m in P2G_BYTES}

# HBM bytes per P2G launch measured with rocprofv3 counters (FETCH_SIZE x 2.0
# + WRITE_SIZE x 1.0, the factors a plain 1 GiB copy reads back, averaged over
# the 20,040 launches of the 60 timed frames of the default run);
# profiles/substep_snow256_counters.md.  The figure is for the kernel named
# beside it (the fused P2G, the default).
# The figure belongs to the P2G sources whose hash is stored beside it: after
# any change to them the bench reports traffic as null until it is measured
# again (or until the kernel's gfx950 assembly is shown unchanged: host-only
# edits to these files move the hash to the new sources).
P2G_TRAFFIC = {"kernel": "p2g_fused", "sources_sha256_16": "3638342056a9b478", "bytes": 194.65e6,
               # SQ_INSTS_VALU per launch (wave instructions), same runs and sources
               "valu_wave_instructions": 51.13e6}
# VALU issue peak of gfx950: 256 CUs x 4 SIMDs, a wave64 VALU instruction
# every 4 cycles per SIMD, at 2.4 GHz.
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4
P2G_SOURCES = ("paper_2111_00699_amd/csrc/mpm_p2g.hip", "paper_2111_00699_amd/csrc/mpm_internal.h",
               "paper_2111_00699_amd/csrc/mpm_kernels.h", "paper_2111_00699_amd/csrc/mpm_api.hip",
               "paper_2111_00699_amd/build.py")


def p2g_counters_valid(kernel):
    """Whether the stored P2G counter figures belong to these sources and kernel."""
    import hashlib

    h = hashlib.sha256()
    for f in P2G_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16] == P2G_TRAFFIC["sources_sha256_16"] and kernel == P2G_TRAFFIC["kernel"]


def p2g_traffic_bytes(kernel):
    return P2G_TRAFFIC["bytes"] if p2g_counters_valid(kernel) else None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def oracle_threads():
    """Host threads the oracle may use: OMP_NUM_THREADS when set, else the
    CPUs this process may run on."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    return int(env) if env.isdigit() and int(env) > 0 else len(os.sched_getaffinity(0))


def cpu_baseline(sc, cfg, serial_steps=5, threaded_steps=40):
    """The FP64 oracle on the host cores, on bounded samples of the snow
    scene: the serial oracle on one thread and its multi-threaded form on
    every host thread this process may use, each from the frame-0 state (at
    rest) and the frame-10 state.  No sphere comes near the floor before
    frame 13, so the frame-10 state is the free-fall closed form of the
    initial one (scenes.free_fall_state).  `value` is the multi-threaded rate."""
    import oracle
    from paper_2111_00699_amd import scenes

    oracle.build()
    N = sc["x"].shape[1]
    states = {"frame 0": {"x": sc["x"]},
              "frame 10": scenes.free_fall_state(sc["x"], cfg, 10 * cfg["substeps_per_frame"])}
    threads = oracle_threads()
    out = {}
    for label, nthr, steps in (("single_thread", 1, serial_steps), ("all_threads", threads, threaded_steps)):
        per = {}
        total = 0.0
        for name, st in states.items():
            t0 = time.perf_counter()
            _, _, _, bad = oracle.substep(cfg, scenes.SNOW, st, steps=steps, threads=nthr)
            dt = time.perf_counter() - t0
            assert bad == 0
            per[name] = N * steps / dt
            total += dt
        out[label] = {"value": 2 * N * steps / total, "threads": nthr, "seconds": total,
                      "per_state": per, "substeps_per_state": steps}
        log(f"[bench] oracle {label}: {out[label]['value']:.3e} particle-substeps/s ({total:.1f} s)")
    a = out["all_threads"]
    return {"value": a["value"], "unit": "particle-substeps/s", "cores": threads, "kind": "oracle",
            "sample": f"full snow scene ({N} particles, 256^3 dense FP64 grid): {threaded_steps} substeps from the "
                      f"frame-0 and the frame-10 state each on {threads} host threads (OpenMP form of the oracle, "
                      f"{a['seconds']:.1f} s), and {serial_steps} substeps from each on one thread (serial oracle)",
            "single_thread": out["single_thread"], "all_threads": a}


def bench_batched(args):
    """256 small scenes (jelly/snow/water, 64^3 or 128^3, 1.7K-64K particles)
    advanced together, one launch per phase per substep, frames replayed as
    HIP graphs, chunk size from the autotuner; against the same scenes run one
    context at a time through the same library."""
    import math

    import torch

    from paper_2111_00699_amd import mpm, scenes

    torch.cuda.set_device(0)
    batch = scenes.batched_scenes(seed=3)
    frame = scenes.FRAME
    counts = [b["x"].shape[1] for b in batch]
    nsub = [math.ceil(frame / b["dt"] - 1e-4) for b in batch]
    work = sum(c * k for c, k in zip(counts, nsub))  # particle-substeps per frame
    N = sum(counts)
    log(f"[bench] batched: {len(batch)} scenes, N={N}, {work:.3e} particle-substeps per frame")
    stream = torch.cuda.Stream()
    out = {}
    with torch.cuda.stream(stream):
        descs = [dict(n=b["n"], dt=b["dt"], bc=b["bc"]) for b in batch]
        sim = mpm.Sim(64, 1e-4, scenes=descs, flags=mpm.FLAG_FRAME_GRAPHS, stream=stream, capacity=2 * N + 256,
                      chunk=args.chunk)
        for k, b in enumerate(batch):
            sim.add_particles(b["mat"], b["x"], scene=k)
        sim.frame(frame)
        chunk = sim.autotune(frame, frames=1) if not args.chunk else args.chunk
        log(f"[bench] autotuned chunk: {chunk}")
        for _ in range(max(args.warmup, 1)):
            sim.frame(frame)
        sim.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        w0 = time.perf_counter()
        e0.record(stream)
        for f in range(args.steps):
            sim.frame(frame)
        e1.record(stream)
        stream.synchronize()
        wall = time.perf_counter() - w0
        ms = max(e0.elapsed_time(e1), wall * 1e3)
        st = sim.stats()
        sim.close()
        # the same scenes, one context each, one frame after another
        sims = []
        for b in batch:
            s1 = mpm.Sim(b["n"], b["dt"], bc=b["bc"], stream=stream, chunk=chunk)
            s1.add_particles(b["mat"], b["x"])
            s1.frame(frame)
            sims.append(s1)
        stream.synchronize()
        k1 = max(1, min(args.steps, 3))
        w1 = time.perf_counter()
        for _ in range(k1):
            for s1 in sims:
                s1.frame(frame)
        stream.synchronize()
        ms1 = (time.perf_counter() - w1) * 1e3 / k1
        for s1 in sims:
            s1.close()
    ms_frame = ms / args.steps
    # algorithmic bytes per frame: per particle-substep P2G + G2P bytes of its material
    mat_bytes = {"jelly": P2G_BYTES["jelly"], "snow": P2G_BYTES["snow"], "water": P2G_BYTES["water"]}
    frame_bytes = sum((mat_bytes[b["kind"]] + G2P_BYTES) * c * k for b, c, k in zip(batch, counts, nsub))
    achieved = frame_bytes / (ms_frame * 1e-3) / 1e9
    out = {
        "metric": "particle-substeps/s",
        "value": work / (ms_frame * 1e-3),
        "unit": "particle-substeps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_frame, "ms_per_frame": ms_frame,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched: 256 seeded scenes (jelly/snow/water cubes of 1.7K-64K particles on 64^3 or "
                               "128^3 grids, 84-334 substeps per 1/60 s frame), one launch per phase per substep, "
                               "frames as HIP graphs",
                   "scenes": len(batch), "particles": N, "particle_substeps_per_frame": work,
                   "chunk": chunk, "rebuilds": st["rebuilds"]},
        "one_at_a_time": {"ms_per_frame": ms1, "value": work / (ms1 * 1e-3), "frames": k1},
        "speedup_vs_one_at_a_time": ms1 / ms_frame,
        "roofline": {"kernel": "whole frame (P2G + G2P algorithmic bytes)", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None},
    }
    print(json.dumps(out), flush=True)


FOUNTAIN_MAX = 143500
# The fountain's ASFLIP transfer (flip ratio, beta_min, beta_max) and automatic
# step (CFL number, largest step): the paper runs its fountain with ASFLIP
# and automatically deduced steps but gives neither's parameters.
ASFLIP = (0.95, 0.0, 1.0)
AUTO_DT = (0.3, 1e-3)


def bench_fountain(args):
    """The fountain: water emitted from the inlet once per 1/60 s frame until
    143,500 particles, on a 128^3 grid.  Reports ms per frame against the
    particle count: APIC with the fixed step (167 substeps per frame), G2P
    fused into the next P2G (the default) and kept separate; and ASFLIP with
    the automatic step (the paper's fountain integrator)."""
    import torch

    from paper_2111_00699_amd import mpm, scenes

    torch.cuda.set_device(0)
    cfg = scenes.fountain_config()
    nsub = cfg["substeps_per_frame"]
    frames = args.steps
    emissions = []
    total = 0
    for f in range(frames):
        if total >= FOUNTAIN_MAX:
            break
        e = scenes.fountain_emission(f)
        keep = min(e["x"].shape[1], FOUNTAIN_MAX - total)
        emissions.append({"x": np.ascontiguousarray(e["x"][:, :keep]), "v": np.ascontiguousarray(e["v"][:, :keep])})
        total += keep
    log(f"[bench] fountain: {len(emissions)} emitting frames, {total} particles, {frames} frames of {nsub} substeps")
    stream = torch.cuda.current_stream()
    runs = {}
    def setup(sim, name):
        if name == "asflip_auto_dt":  # the paper's fountain integrator and automatic steps
            sim.set_transfer(ASFLIP[0], ASFLIP[1], ASFLIP[2])
            sim.set_auto_dt(AUTO_DT[0], AUTO_DT[1])

    for name, flags in (("default_fused", 0), ("separate_g2p", mpm.FLAG_SEPARATE_G2P), ("asflip_auto_dt", 0)):
        auto = name == "asflip_auto_dt"
        sim = mpm.Sim(cfg["n"], cfg["dt"], bc=cfg["bc"], bc_cells=cfg["bc_cells"], gravity=cfg["gravity"],
                      capacity=2 * total + 256, flags=flags | args.flags, chunk=args.chunk)
        # warmup: one frame of a throwaway emission, then a fresh context
        sim.add_particles(scenes.WATER, emissions[0]["x"], v=emissions[0]["v"])
        setup(sim, name)
        sim.frame(scenes.FRAME)
        sim.synchronize()
        sim.close()
        sim = mpm.Sim(cfg["n"], cfg["dt"], bc=cfg["bc"], bc_cells=cfg["bc_cells"], gravity=cfg["gravity"],
                      capacity=2 * total + 256, flags=flags | args.flags, chunk=args.chunk)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(frames + 1)]
        counts, subs = [], []
        n = 0
        done = 0
        w0 = time.perf_counter()
        ev[0].record(stream)
        for f in range(frames):
            if f < len(emissions):
                sim.add_particles(scenes.WATER if f == 0 else None, emissions[f]["x"], v=emissions[f]["v"])
                n += emissions[f]["x"].shape[1]
                if f == 0:
                    setup(sim, name)
            sim.frame(scenes.FRAME)
            ev[f + 1].record(stream)
            counts.append(n)
            if auto:  # the frame's step count (the automatic step synchronizes every frame anyway)
                k = sim.scene_stats()["substeps"]
                subs.append(k - done)
                done = k
            else:
                subs.append(nsub)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        ms = [ev[f].elapsed_time(ev[f + 1]) for f in range(frames)]
        st = sim.stats()
        sim.close()
        gpu_ms = sum(ms)
        work = sum(c * k for c, k in zip(counts, subs))
        runs[name] = {"ms_total": max(gpu_ms, wall * 1e3), "gpu_event_ms": gpu_ms, "wall_ms": wall * 1e3,
                      "value": work / (max(gpu_ms, wall * 1e3) * 1e-3), "rebuilds": st["rebuilds"],
                      "substeps": sum(subs),
                      "frames": [[f + 1, counts[f], subs[f], round(ms[f], 3)] for f in range(frames)]}
        log(f"[bench] fountain {name}: {runs[name]['ms_total'] / frames:.2f} ms per frame on average")
    r = runs["default_fused"]
    out = {
        "metric": "particle-substeps/s",
        "value": r["value"],
        "unit": "particle-substeps/s",
        "n_gpus": 1, "steps": frames, "warmup": 1,
        "ms_per_step": r["ms_total"] / frames, "ms_per_frame": r["ms_total"] / frames,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "fountain: water (J-based EOS, bulk modulus 1e4) emitted once per frame at 3 m/s "
                               "from a 0.05-radius inlet until 143,500 particles, 128^3 grid, separating walls, "
                               f"{nsub} substeps per 1/60 s frame",
                   "particles_final": total, "emitting_frames": len(emissions), "grid": cfg["n"],
                   "substeps_per_frame": nsub, "fuse_below": 1000000},
        "runs": runs,
        "fused_vs_separate": runs["separate_g2p"]["ms_total"] / r["ms_total"],
        "asflip_auto_dt": {"flip": ASFLIP[0], "beta_min": ASFLIP[1], "beta_max": ASFLIP[2], "cfl": AUTO_DT[0],
                           "dt_max": AUTO_DT[1],
                           "ms_per_frame": runs["asflip_auto_dt"]["ms_total"] / frames,
                           "substeps_per_frame": runs["asflip_auto_dt"]["substeps"] / frames,
                           "speedup_vs_fixed_step": r["ms_total"] / runs["asflip_auto_dt"]["ms_total"]},
    }
    print(json.dumps(out), flush=True)


# (box side in cells, boxes, grid): 55,296 / 389,344 / 3,114,752 / 12,459,008 particles
SAND_CASES = ((12, 4, 128), (23, 4, 128), (46, 4, 128), (46, 16, 256))


def bench_sand(args):
    """Sand Blocks, the paper's main benchmark: 4 boxes of l^3 cells
    (l = 12, 23, 46) of Drucker-Prager sand at 8 ppc dropped into a
    frictionless 128^3 box, frames of 1/48 s in 36 substeps, and 16 boxes of
    46^3 in a 256^3 box (72 substeps, the same CFL number); one warmup frame
    and `steps` timed frames (60, as the paper averages).  Reports ms per
    frame per case; `value` is the largest case's particle-substeps/s."""
    import torch

    from paper_2111_00699_amd import mpm, scenes

    torch.cuda.set_device(0)
    frames = args.steps
    stream = torch.cuda.current_stream()
    runs = {}
    for l, boxes, grid in SAND_CASES:
        cfg = scenes.sand_config(grid)
        nsub = cfg["substeps_per_frame"]
        name = f"{boxes}x{l}^3"
        x = scenes.sand_blocks(l=l, boxes=boxes, n=cfg["n"])["x"]
        N = x.shape[1]
        sim = mpm.Sim(cfg["n"], cfg["dt"], bc=cfg["bc"], bc_cells=cfg["bc_cells"], gravity=cfg["gravity"],
                      capacity=2 * N + 256, flags=args.flags, chunk=args.chunk)
        sim.add_particles(scenes.SAND, x)
        for _ in range(args.warmup):
            sim.substep(nsub)
        sim.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(frames + 1)]
        r0 = sim.stats()["rebuilds"]
        w0 = time.perf_counter()
        ev[0].record(stream)
        for f in range(frames):
            sim.substep(nsub)
            ev[f + 1].record(stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - w0) * 1e3
        ms = [ev[f].elapsed_time(ev[f + 1]) for f in range(frames)]
        st = sim.stats()
        p = sim.read_particles()
        xs = p["x"].cpu().numpy()
        q = p["s"].cpu().numpy() - 1.0
        sim.close()
        if st["error"]:
            raise RuntimeError(f"sand blocks l={l}: device error word {st['error']}")
        total = max(sum(ms), wall)
        runs[name] = {"particles": N, "grid": grid, "substeps_per_frame": nsub,
                      "ms_per_frame": round(total / frames, 3),
                      "gpu_event_ms": round(sum(ms), 2), "wall_ms": round(wall, 2),
                      "value": N * nsub * frames / (total * 1e-3),
                      "rebuilds_per_frame": round((st["rebuilds"] - r0) / frames, 2),
                      "final_y_range": [float(xs[1].min()), float(xs[1].max())],
                      "plastic_fraction": float((q > 0).mean()),
                      "ms_per_frame_min_max": [round(min(ms), 3), round(max(ms), 3)]}
        log(f"[bench] sand blocks {name} N={N}: {total / frames:.3f} ms per frame, "
            f"{runs[name]['rebuilds_per_frame']} rebuilds per frame")
        del x
    l, boxes, grid = SAND_CASES[-1]
    big = runs[f"{boxes}x{l}^3"]
    out = {
        "metric": "particle-substeps/s",
        "value": big["value"],
        "unit": "particle-substeps/s",
        "n_gpus": 1, "steps": frames, "warmup": args.warmup,
        "ms_per_step": big["ms_per_frame"], "ms_per_frame": big["ms_per_frame"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "sand blocks: 4 boxes of l^3 cells (l = 12, 23, 46) of Drucker-Prager sand at 8 ppc "
                               "in a 128^3 slip box (36 substeps per 1/48 s frame) and 16 boxes of 46^3 in a 256^3 "
                               "box (72 substeps); value is the 16-box case (12,459,008 particles)",
                   "frame_s": 1.0 / 48.0},
        "runs": runs,
    }
    print(json.dumps(out), flush=True)


ABLATIONS = (  # (name, library flags, chunk size); the baseline first
    ("baseline", 0, 0),
    ("rebuild_every_step", 0x1, 0),    # no free zone: rebuild and sort before every substep
    ("p2g_global_atomics", 0x2, 0),    # P2G straight to global atomics, no LDS tile
    ("plain_sorted_lanes", 0x8, 0),    # chunks in plain sorted order, not dealt over the LDS passes
    ("g2p_global_gather", 0x10, 0),    # G2P gathers from the dense grid, no LDS node box
    ("g2p_always_fused", 0x40, 0),     # G2P inside the next P2G at any size
    ("g2p_always_separate", 0x80, 0),  # G2P as its own launch at any size
    ("separate_walls", 0x100, 0),      # the wall condition as a launch of its own
    ("separate_clear", 0x200, 0),      # the accumulator clearing as a launch of its own
    ("alloc_exact", 0x400, 0),         # buffers grown to exactly what is needed (the fountain emits)
    ("chunk_per_block", 0x800, 0),     # each chunk holds one block's particles (virtual blocks)
    ("frame_graphs", 0x20, 0),         # frames replayed as HIP graphs
    ("chunk_128", 0, 128),
    ("chunk_512", 0, 512),
)
# Library builds measured as ablations (each in a process of its own):
# IEEE arithmetic instead of fast math, the grouped particle layout instead
# of one array per field, and P2G's stencil weights parked in LDS.
ABLATION_LIBRARIES = ("precise", "aosoa", "lds_weights")


def ablation_cases():
    from paper_2111_00699_amd import scenes

    snow = scenes.snow_config()
    sand = scenes.sand_config()
    fountain = scenes.fountain_config()
    cases = []
    for l, frames in ((12, 10), (23, 10)):
        x = scenes.sand_blocks(l=l, boxes=4, n=128)["x"]
        cases.append((f"sand_blocks_4x{l}^3", {"x": x}, scenes.SAND,
                      dict(n=sand["n"], dt=sand["dt"], bc=sand["bc"], bc_cells=sand["bc_cells"],
                           gravity=sand["gravity"]), frames, sand["frame"]))
    cases.append(("snow", {"x": scenes.snow_spheres(1)["x"]}, scenes.SNOW,
                  dict(n=snow["n"], dt=snow["dt"], bc=snow["bc"], bc_cells=snow["bc_cells"],
                       gravity=snow["gravity"]), 2, scenes.FRAME))
    # the fountain emits every frame: frames 1-24 (emission until 143,500 particles)
    cases.append(("fountain", {"emit": 24}, scenes.WATER,
                  dict(n=fountain["n"], dt=fountain["dt"], bc=fountain["bc"], bc_cells=fountain["bc_cells"],
                       gravity=fountain["gravity"]), 24, scenes.FRAME))
    return cases


def run_ablation_case(case, flags, chunk, stream):
    """ms per frame of one ablation case with the given flags and chunk size."""
    import torch

    from paper_2111_00699_amd import mpm, scenes

    name, data, mat, cfg, frames, frame = case
    emit = data.get("emit", 0)
    N = data["x"].shape[1] if "x" in data else FOUNTAIN_MAX
    sim = mpm.Sim(cfg["n"], cfg["dt"], bc=cfg["bc"], bc_cells=cfg["bc_cells"], gravity=cfg["gravity"],
                  capacity=(2 * N + 256) if not emit else 256, flags=flags, chunk=chunk, stream=stream)
    total = 0
    if emit:  # warm the kernels up on a throwaway context
        e = scenes.fountain_emission(0)
        warm = mpm.Sim(cfg["n"], cfg["dt"], bc=cfg["bc"], bc_cells=cfg["bc_cells"], gravity=cfg["gravity"],
                       flags=flags, chunk=chunk, stream=stream)
        warm.add_particles(mat, e["x"], v=e["v"])
        warm.frame(frame)
        warm.synchronize()
        warm.close()
    else:
        sim.add_particles(mat, data["x"])
        for _ in range(2):  # warmup (a graph context records its frame graphs in the second frame)
            sim.frame(frame)
    sim.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    e0.record(stream)
    for f in range(frames):
        if emit and f < emit and total < FOUNTAIN_MAX:
            e = scenes.fountain_emission(f)
            k = min(e["x"].shape[1], FOUNTAIN_MAX - total)
            sim.add_particles(mat if f == 0 else None, np.ascontiguousarray(e["x"][:, :k]),
                              v=np.ascontiguousarray(e["v"][:, :k]))
            total += k
        sim.frame(frame)
    e1.record(stream)
    stream.synchronize()
    ms = max(e0.elapsed_time(e1), (time.perf_counter() - w0) * 1e3) / frames
    st = sim.stats()
    sim.close()
    return {"ms_per_frame": round(ms, 3), "rebuilds": st["rebuilds"], "particles": N}


def bench_ablation_rows(args):
    """(in a process whose MPM_LIBRARY names a library build) the baseline
    configuration of every ablation case, one JSON line."""
    import torch

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    out = {}
    with torch.cuda.stream(stream):
        for case in ablation_cases():
            out[case[0]] = run_ablation_case(case, 0, 0, stream)
            log(f"[bench] ablation rows {os.environ.get('MPM_LIBRARY')} {case[0]}: {out[case[0]]['ms_per_frame']} ms")
    print(json.dumps(out), flush=True)


def fast_math_stress_error():
    """The paper's fast-math experiment on Sand Blocks (4 boxes of 46^3
    cells, 3,114,752 particles): the fast-math build and the IEEE build, each
    in a process of its own, run ten 1/48 s frames from the same initial state
    (the boxes land in frames 7-8); the Kirchhoff stress of every particle's
    state after them (FP64 Hencky of its deformation gradient, numpy's SVD) is
    compared between the two builds, and the tenth frame is timed."""
    import subprocess
    import tempfile

    from paper_2111_00699_amd import scenes

    d = tempfile.mkdtemp(prefix="mpm_fastmath_")
    res = {}
    for lib in ("fast", "precise"):
        env = dict(os.environ, MPM_LIBRARY=lib)
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--workload", "sand-frame-state",
                            "--out", os.path.join(d, lib + ".npz")], env=env, capture_output=True, text=True,
                           timeout=600)
        if r.returncode != 0:
            raise RuntimeError(f"sand frame with the {lib} build failed: {r.stderr[-2000:]}")
        res[lib] = json.loads(r.stdout.strip().splitlines()[-1])
    taus = {}
    mat = scenes.SAND
    mu = mat["E"] / (2 * (1 + mat["nu"]))
    la = mat["E"] * mat["nu"] / ((1 + mat["nu"]) * (1 - 2 * mat["nu"]))
    for lib in ("fast", "precise"):
        F = np.load(os.path.join(d, lib + ".npz"))["F"].astype(np.float64)
        N = F.shape[1]
        U, sig, _ = np.linalg.svd(F.T.reshape(N, 3, 3))
        eps = np.log(np.maximum(np.abs(sig), 1e-6))
        diag = 2 * mu * eps + la * eps.sum(axis=1, keepdims=True)
        taus[lib] = np.einsum("nik,nk,njk->nij", U, diag, U)
        os.remove(os.path.join(d, lib + ".npz"))
    os.rmdir(d)
    dt = np.abs(taus["fast"] - taus["precise"])
    return {"particles": int(N), "frames": 10, "max_abs_pa": float(dt.max()), "mean_abs_pa": float(dt.mean()),
            "p99_abs_pa": float(np.quantile(dt.max(axis=(1, 2)), 0.99)),
            "max_abs_dyne_per_cm2": float(dt.max() * 10.0), "max_tau_pa": float(np.abs(taus["precise"]).max()),
            "relative_to_max_tau": float(dt.max() / np.abs(taus["precise"]).max()),
            "ms_per_frame": {k: v["ms_per_frame"] for k, v in res.items()}}


def bench_sand_frame_state(args):
    """(child of fast_math_stress_error) ten 1/48 s frames of Sand Blocks
    4 x 46^3 (the boxes land in frames 7-8), the tenth timed; saves F of
    every particle."""
    import torch

    from paper_2111_00699_amd import mpm, scenes

    torch.cuda.set_device(0)
    x = scenes.sand_blocks(l=46, boxes=4, n=128)["x"]
    c = scenes.sand_config()
    N = x.shape[1]
    sim = mpm.Sim(c["n"], c["dt"], bc=c["bc"], bc_cells=c["bc_cells"], gravity=c["gravity"], capacity=2 * N + 256)
    sim.add_particles(scenes.SAND, x)
    for _ in range(9):
        sim.frame(c["frame"])
    sim.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    sim.frame(c["frame"])
    e1.record()
    torch.cuda.synchronize()
    F = sim.read_particles()["F"].cpu().numpy()
    sim.close()
    np.savez(args.out, F=F)
    print(json.dumps({"ms_per_frame": e0.elapsed_time(e1), "library": os.path.basename(mpm.LIB_PATH)}), flush=True)


def bench_ablations(args):
    """The paper's single-GPU ablations, on this library: each design choice
    switched off by a flag, a chunk size or a library build, ms per frame and
    the extra cost against the default.  Scenes: Sand Blocks (4 boxes of
    12^3 and of 23^3 cells at 8 ppc, 55,296 and 389,344 particles,
    Drucker-Prager sand) in a 128^3 grid with slip walls, frames of 1/48 s in
    36 substeps as in the paper, timed from the second frame; the snow scene
    (1.28M particles, 1/60 s frames of 334 substeps); and the fountain's
    first 24 frames (water emitted every frame).  Library builds run in
    processes of their own; the fast-math row also gives the Kirchhoff stress
    difference of the two builds after a Sand Blocks frame (3.1M particles),
    the paper's fast-math error experiment."""
    import subprocess

    import torch

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    cases = ablation_cases()
    table = {c[0]: {"configs": {}} for c in cases}
    with torch.cuda.stream(stream):
        for case in cases:
            for cname, flags, chunk in ABLATIONS:
                r = run_ablation_case(case, flags, chunk, stream)
                table[case[0]]["configs"][cname] = r
                table[case[0]]["particles"] = r["particles"]
                table[case[0]]["frames_timed"] = case[4]
                log(f"[bench] ablation {case[0]} {cname}: {r['ms_per_frame']:.2f} ms per frame")
    for lib in ABLATION_LIBRARIES:
        env = dict(os.environ, MPM_LIBRARY=lib)
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--workload", "ablation-rows"], env=env,
                           capture_output=True, text=True, timeout=900)
        if r.returncode != 0:
            raise RuntimeError(f"ablation rows with the {lib} build failed: {r.stderr[-2000:]}")
        rows = json.loads(r.stdout.strip().splitlines()[-1])
        for name, row in rows.items():
            table[name]["configs"]["library_" + lib] = row
    for t in table.values():
        base = t["configs"]["baseline"]["ms_per_frame"]
        for r in t["configs"].values():
            r["extra_cost"] = round(r["ms_per_frame"] / base - 1.0, 4)
    log("[bench] fast-math stress error (Sand Blocks 4 x 46^3, ten frames)")
    fm = fast_math_stress_error()
    snow = table["snow"]
    snow_base = snow["configs"]["baseline"]["ms_per_frame"]
    from paper_2111_00699_amd import scenes

    nsub = scenes.snow_config()["substeps_per_frame"]
    out = {
        "metric": "particle-substeps/s",
        "value": snow["particles"] * nsub / (snow_base * 1e-3),
        "unit": "particle-substeps/s",
        "n_gpus": 1, "steps": snow["frames_timed"], "warmup": 1,
        "ms_per_step": snow_base, "ms_per_frame": snow_base,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "ablations: each design choice switched off in turn on the Sand Blocks layout "
                               "(4 boxes of 12^3 and 23^3 cells, Drucker-Prager sand, 128^3, 36 substeps per 1/48 s "
                               "frame), the snow scene and the fountain's emitting frames; "
                               "value is the snow baseline over its timed frames 2-3"},
        "ablations": table,
        "fast_math_stress_error": fm,
    }
    print(json.dumps(out), flush=True)


def bench_surrogate(args):
    """The learned snow return map on the snow scene: trained on the GPU from
    exact-path runs of snow scenes with other sphere seeds (4 and 40), then
    the seed-1 scene is advanced with the exact map, the learned map and the
    same eigenvector-free path with the exact clamp (no network); positions
    are compared with the exact run after the timed frames."""
    import torch

    from paper_2111_00699_amd import mpm, scenes

    torch.cuda.set_device(0)
    cfg = scenes.snow_config()
    nsub = cfg["substeps_per_frame"]

    def make(sc):
        sim = mpm.Sim(cfg["n"], cfg["dt"], bc=cfg["bc"], bc_cells=cfg["bc_cells"], gravity=cfg["gravity"],
                      capacity=2 * sc["x"].shape[1] + 256)
        sim.add_particles(scenes.SNOW, sc["x"])
        return sim

    # training pairs: states of two other snow scenes every 1/3 frame after they have landed
    Xs, Ts = [], []
    t0 = time.perf_counter()
    for seed in (4, 40):
        sim = make(scenes.snow_spheres(seed))
        sim.substep(nsub * args.sur_start_frame)
        for k in range(args.train_snapshots):
            sim.substep(nsub // 3)
            X, T = mpm.Surrogate.sample(sim, dt_ref=cfg["dt"])
            Xs.append(X.clone())
            Ts.append(T.clone())
        sim.close()
    X = torch.cat(Xs)
    T = torch.cat(Ts)
    del Xs, Ts
    t_sample = time.perf_counter() - t0
    sur = mpm.Surrogate()
    sur.set(scenes.mlp_init(4))
    sur.fit_norm(X, T)
    t0 = time.perf_counter()
    losses = sur.train(X, T, steps=args.train_steps, batch=16384, lr=1e-3, seed=7)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"[bench] surrogate: {X.shape[0]} pairs in {t_sample:.1f} s, {args.train_steps} Adam steps in {t_train:.1f} s, "
        f"loss {losses[:10].mean():.3e} -> {losses[-10:].mean():.3e}")
    # evaluation: the seed-1 scene advanced to the same frame on the exact path, then each mode from there
    sc = scenes.snow_spheres(1)
    N = sc["x"].shape[1]
    sim = make(sc)
    sim.substep(nsub * args.sur_start_frame)
    start = sim.read_particles()
    sim.close()
    results = {}
    finals = {}
    for name, mode in (("exact", 0), ("surrogate", 1), ("closed_form", 2)):
        sim = mpm.Sim(cfg["n"], cfg["dt"], bc=cfg["bc"], bc_cells=cfg["bc_cells"], gravity=cfg["gravity"],
                      capacity=2 * N + 256)
        sim.add_particles(scenes.SNOW, start["x"], v=start["v"], C=start["C"], F=start["F"], s=start["s"])
        if mode:
            sim.use_surrogate(mode, sur if mode == 1 else None, tol=args.sur_tol, dt_ref=cfg["dt"])
        sim.substep(nsub // 3)  # warm-up
        sim.synchronize()
        sim.profile(mpm.PHASE_P2G | mpm.PHASE_G2P)
        st0 = sim.stats()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            sim.substep(nsub)
        e1.record()
        torch.cuda.synchronize()
        st1 = sim.stats()
        p2g = sim.profile_read()["p2g"]
        p2g_us = 1e3 * p2g["ms"] / max(p2g["launches"], 1)
        finals[name] = sim.read_particles()
        done = st1["surrogate_particles"] - st0["surrogate_particles"]
        fb = st1["surrogate_fallbacks"] - st0["surrogate_fallbacks"]
        results[name] = {"ms_per_frame": e0.elapsed_time(e1) / args.steps, "p2g_avg_launch_us": p2g_us,
                         "fallback_rate": (fb / max(done + fb, 1)) if mode else None}
        if mode == 1:  # network evaluations per P2G launch (both kept and fallen-back particles)
            tflops = MLP_FWD_FLOPS * (done + fb) / max(p2g["launches"], 1) / (p2g_us * 1e-6) / 1e12
            results[name]["p2g_mfma"] = {"achieved": tflops, "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                                         "frac": tflops / MFMA_BF16_PEAK_TFLOPS}
        sim.close()
        log(f"[bench] {name}: {results[name]}")
    dx = 1.0 / cfg["n"]

    def kirchhoff(st):
        """Snow Kirchhoff stress of each particle (FP64): fixed-corotated of F_E with
        Lame parameters scaled by exp(xi (1 - J_P))."""
        m = scenes.SNOW
        F = st["F"].double().cpu().numpy().T.reshape(-1, 3, 3)
        Jp = st["s"].double().cpu().numpy()
        U, sig, Vt = np.linalg.svd(F)
        det = np.linalg.det(F)
        sig[:, 2] *= np.sign(det)
        h = np.exp(m["xi"] * (1.0 - Jp))
        mu0 = m["E"] / (2 * (1 + m["nu"]))
        la0 = m["E"] * m["nu"] / ((1 + m["nu"]) * (1 - 2 * m["nu"]))
        J = np.prod(sig, axis=1)
        d = 2 * (mu0 * h)[:, None] * (sig - 1) * sig + ((la0 * h) * (J - 1) * J)[:, None]
        U[:, :, 2] *= np.sign(det)[:, None]
        return np.einsum("nik,nk,njk->nij", U, d, U)

    tau_exact = kirchhoff(finals["exact"])
    tscale = np.abs(tau_exact).max()
    for name in ("surrogate", "closed_form"):
        d = (finals[name]["x"] - finals["exact"]["x"]).norm(dim=0) / dx
        results[name]["position_error_dx"] = {"mean": float(d.mean()), "max": float(d.max())}
        dt_ = np.abs(kirchhoff(finals[name]) - tau_exact).max(axis=(1, 2))
        results[name]["stress_error"] = {"max_pa": float(dt_.max()), "p99_pa": float(np.quantile(dt_, 0.99)),
                                         "mean_pa": float(dt_.mean()), "max_tau_pa": float(tscale),
                                         "max_rel": float(dt_.max() / tscale)}
    ex = results["exact"]["ms_per_frame"]
    train_tflops = MLP_TRAIN_FLOPS * 16384 * args.train_steps / t_train / 1e12
    out = {
        "metric": "particle-substeps/s", "value": N * nsub / (results["surrogate"]["ms_per_frame"] * 1e-3),
        "unit": "particle-substeps/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": results["surrogate"]["ms_per_frame"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 (MLP bf16 operands, f32 accumulation)", "data": "synthetic",
        "config": {"workload": "snow scene (seed 1, 1.28M particles, 256^3) from the frame after landing, with the "
                               "learned return map; trained on pairs from the exact path on sphere seeds 4 and 40",
                   "frames_timed": args.steps, "start_frame": args.sur_start_frame,
                   "train_pairs": int(X.shape[0]), "train_steps": args.train_steps,
                   "final_loss": float(losses[-10:].mean()), "tol": args.sur_tol},
        "train_mfma": {"seconds": t_train, "achieved": train_tflops, "peak": MFMA_BF16_PEAK_TFLOPS,
                       "unit": "TFLOP/s", "frac": train_tflops / MFMA_BF16_PEAK_TFLOPS},
        "modes": results,
        "speedup_vs_exact": {k: ex / v["ms_per_frame"] for k, v in results.items()},
    }
    sur.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed frames (snow and fountain 60, as the paper averages; batched 10; surrogate 5)")
    ap.add_argument("--warmup", type=int, default=1, help="untimed frames")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--flags", type=int, default=0)
    ap.add_argument("--workload", choices=("snow", "batched", "surrogate", "fountain", "ablations", "sand",
                                           "ablation-rows", "sand-frame-state"),
                    default="snow")
    ap.add_argument("--train-snapshots", type=int, default=4, help="surrogate: training snapshots per scene")
    ap.add_argument("--train-steps", type=int, default=20000, help="surrogate: Adam steps")
    ap.add_argument("--sur-tol", type=float, default=2e-3, help="surrogate: residual tolerance")
    ap.add_argument("--sur-start-frame", type=int, default=24, help="surrogate: frame the comparison starts at")
    ap.add_argument("--out", default="", help="sand-frame-state: where the state goes")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 4 times (HBM counter calibration)")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = {"snow": 60, "fountain": 60, "batched": 10, "surrogate": 5, "ablations": 0,
                      "sand": 60}.get(args.workload, 0)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read_per_launch": src.numel() * 4,
                          "bytes_written_per_launch": dst.numel() * 4, "launches": 4}))
        return

    if args.workload == "batched":
        bench_batched(args)
        return
    if args.workload == "surrogate":
        bench_surrogate(args)
        return
    if args.workload == "fountain":
        bench_fountain(args)
        return
    if args.workload == "ablations":
        bench_ablations(args)
        return
    if args.workload == "ablation-rows":
        bench_ablation_rows(args)
        return
    if args.workload == "sand-frame-state":
        bench_sand_frame_state(args)
        return
    if args.workload == "sand":
        bench_sand(args)
        return

    from paper_2111_00699_amd import mpm, scenes

    torch.cuda.set_device(0)
    sc = scenes.snow_spheres(1)
    cfg = scenes.snow_config()
    N = sc["x"].shape[1]
    nsub = cfg["substeps_per_frame"]
    log(f"[bench] snow scene N={N} n={cfg['n']} substeps/frame={nsub} dt={cfg['dt']:.4e}")
    sim = mpm.Sim(cfg["n"], cfg["dt"], bc=cfg["bc"], bc_cells=cfg["bc_cells"], gravity=cfg["gravity"],
                  capacity=2 * N + 256, chunk=args.chunk, flags=args.flags)
    sim.add_particles(scenes.SNOW, sc["x"])
    torch.cuda.synchronize()
    for f in range(args.warmup):
        sim.substep(nsub)
        log(f"[bench] warmup frame {f + 1}/{args.warmup} enqueued")
    sim.synchronize()
    st0 = sim.stats()
    # every 64th launch: the events cost a few microseconds of stream time each
    sim.profile(mpm.PHASE_P2G | mpm.PHASE_G2P | mpm.PROFILE_EVERY(PROFILE_EVERY))
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record(stream)
    for f in range(args.steps):
        sim.substep(nsub)
        if (f + 1) % 10 == 0:
            log(f"[bench] timed frame {f + 1}/{args.steps} enqueued")
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    gpu_ms = e0.elapsed_time(e1)
    prof = sim.profile_read()
    st1 = sim.stats()
    ms = max(gpu_ms, wall * 1e3)
    substeps = args.steps * nsub
    value = N * substeps / (ms * 1e-3)
    p2g = prof["p2g"]
    p2g_avg_ms = p2g["ms"] / max(p2g["launches"], 1)
    fused = prof["g2p"]["launches"] * 2 < p2g["launches"]  # G2P ran inside P2G (sampled alike)
    # algorithmic bytes of one launch: the per particle-substep state traffic
    # of the substep's two-kernel form (P2G + G2P, 212 B for snow), since the
    # fused launch does one full substep's particle work for every particle
    p2g_bytes = SUBSTEP_BYTES["snow"] if fused else P2G_BYTES["snow"]
    achieved = p2g_bytes * N / (p2g_avg_ms * 1e-3) / 1e9
    kernel_bytes = P2G_FUSED_BYTES["snow"] if fused else P2G_BYTES["snow"]
    rebuilds = st1["rebuilds"] - st0["rebuilds"]
    traffic = p2g_traffic_bytes("p2g_fused" if fused else "p2g")
    out = {
        "metric": "particle-substeps/s",
        "value": value,
        "unit": "particle-substeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "ms_per_frame": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "snow: 12 seeded spheres dropped in a 256^3 grid, snow plasticity with "
                               "hardening, 334 substeps of 4.99e-5 s per 1/60 s frame, "
                               f"frames {args.warmup + 1}-{args.warmup + args.steps} timed",
                   "particles": N, "grid": cfg["n"], "substeps_per_frame": nsub, "frames_timed": args.steps,
                   "rebuilds_in_timed_frames": rebuilds,
                   "substeps_per_rebuild": substeps / max(rebuilds, 1), "chunk": args.chunk or 256},
        "roofline": {"kernel": "p2g_fused" if fused else "p2g", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "traffic_unit": "HBM bytes per launch",
                     "traffic_frac": (traffic / (p2g_avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS) if traffic else None,
                     "traffic_source": ("rocprofv3 --pmc FETCH_SIZE, WRITE_SIZE of the same kernel sources "
                                        "(profiles/substep_snow256_counters.md)") if traffic else
                                       "null: the kernel changed since its counters were taken",
                     "avg_launch_us": p2g_avg_ms * 1e3, "launches_timed": p2g["launches"],
                     "sampled_every": PROFILE_EVERY,
                     "bytes_per_particle": p2g_bytes,
                     "bytes_basis": "per particle-substep state traffic of P2G + G2P (snow: 212 B)",
                     "kernel_bytes_per_particle": kernel_bytes,
                     "kernel_bytes_frac": kernel_bytes * N / (p2g_avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
        # the VALU issue floor: the launch's counted wave instructions at full issue against the
        # live launch time (null once the sources differ from the counted ones)
        "roofline_valu": ({"kernel": "p2g_fused", "bound": "valu_issue",
                           "wave_instructions_per_launch": P2G_TRAFFIC["valu_wave_instructions"],
                           "floor_us": P2G_TRAFFIC["valu_wave_instructions"] / VALU_ISSUE_PEAK * 1e6,
                           "frac": P2G_TRAFFIC["valu_wave_instructions"] / VALU_ISSUE_PEAK / (p2g_avg_ms * 1e-3)}
                          if fused and p2g_counters_valid("p2g_fused") else None),
        # the LDS 64-bit atomics of the same launches against their measured peak rate
        "roofline_lds": {"kernel": "p2g_fused" if fused else "p2g", "bound": "lds_u64_atomics",
                         "achieved": P2G_LDS_ATOMICS_PER_PARTICLE * N / (p2g_avg_ms * 1e-3),
                         "peak": LDS_U64_ATOMIC_PEAK, "unit": "lane-ops/s",
                         "frac": P2G_LDS_ATOMICS_PER_PARTICLE * N / (p2g_avg_ms * 1e-3) / LDS_U64_ATOMIC_PEAK},
        "wall_ms": wall * 1e3,
        "gpu_event_ms": gpu_ms,
    }
    sim.close()
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on the host")
        out["cpu_baseline"] = cpu_baseline(sc, cfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
