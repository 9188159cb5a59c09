"""FP64 CPU oracle for the explicit MLS-MPM substep.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The HIP library never imports, links or
runs anything in this directory, and this package imports nothing from the
library.  The numerical work lives in ``mpm_oracle.c`` (plain C, FP64,
single-threaded); this module is a ctypes shim that marshals numpy arrays.

State dictionaries use structure-of-arrays numpy float64 arrays:
``x (3,N)``, ``v (3,N)``, ``C (9,N)``, ``F (9,N)`` (entry (a,b) at a*3+b),
``s (N,)`` (J_P for snow, 1 + q with q the hardening state for sand, J for
water, ignored for jelly).
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mpm_oracle.c")
_LIB = os.path.join(_HERE, "libmpm_oracle.so")

KIND = {"jelly": 0, "snow": 1, "water": 2, "sand": 3}
BC = {"sticky": 0, "slip": 1, "separate": 2}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no fast-math) into oracle/libmpm_oracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fno-fast-math", "-fopenmp", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Mat(ct.Structure):
    _fields_ = [("kind", ct.c_int)] + [(k, ct.c_double) for k in
                                       ("E", "nu", "rho", "ppc", "theta_c", "theta_s", "xi", "bulk",
                                        "h0", "h1", "h2", "h3")]


class _Cfg(ct.Structure):
    _fields_ = [("n", ct.c_int), ("bc", ct.c_int), ("bc_cells", ct.c_int),
                ("gravity", ct.c_double * 3), ("dt", ct.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ct.CDLL(build())
        D = ct.POINTER(ct.c_double)
        F32 = ct.POINTER(ct.c_float)
        U32 = ct.POINTER(ct.c_uint32)
        I32 = ct.POINTER(ct.c_int32)
        U8 = ct.POINTER(ct.c_uint8)
        L = ct.c_long
        sig = {
            "om_svd3": (None, [D, D, D, D]),
            "om_fixed_corotated": (None, [D, ct.c_double, ct.c_double, D]),
            "om_stress": (None, [ct.POINTER(_Mat), D, ct.c_double, D]),
            "om_snow_project": (None, [ct.POINTER(_Mat), D, ct.c_double, D, D]),
            "om_hencky": (None, [D, ct.c_double, ct.c_double, D]),
            "om_sand_alpha": (ct.c_double, [ct.POINTER(_Mat), ct.c_double]),
            "om_sand_project": (None, [ct.POINTER(_Mat), D, ct.c_double, D, D]),
            "om_weights": (None, [ct.c_double, ct.POINTER(ct.c_int), D]),
            "om_p2g": (L, [ct.POINTER(_Cfg), ct.POINTER(_Mat), L, D, D, D, D, D, D, D]),
            "om_grid_update": (None, [ct.POINTER(_Cfg), D, D]),
            "om_g2p": (L, [ct.POINTER(_Cfg), ct.POINTER(_Mat), L, D, D, D, D, D, D]),
            "om_g2p_trial": (L, [ct.POINTER(_Cfg), ct.POINTER(_Mat), L, D, D, D, D, D, D]),
            "om_substep": (L, [ct.POINTER(_Cfg), ct.POINTER(_Mat), L, D, D, D, D, D, D, D]),
            "om_substep_omp": (L, [ct.POINTER(_Cfg), ct.POINTER(_Mat), L, D, D, D, D, D, D, D, ct.c_int]),
            "om_substep_asflip": (L, [ct.POINTER(_Cfg), ct.POINTER(_Mat), L, D, D, D, D, D, D, D, ct.c_double,
                                      ct.c_double, ct.c_double]),
            "om_keys": (L, [L, F32, ct.c_int, U32, I32]),
            "om_stable_sort": (None, [L, U32, I32, U32]),
            "om_gblocks": (L, [L, U32, U32, I32, I32]),
            "om_pblocks": (L, [ct.c_int, L, U32, I32]),
            "om_free_zone_exit": (L, [L, F32, ct.c_int, I32, U8]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(_lib, name)
            fn.restype = res
            fn.argtypes = args
    return _lib


def _p(a, ctype):
    return a.ctypes.data_as(ct.POINTER(ctype))


def _mat(m: dict) -> _Mat:
    kind = m["kind"] if isinstance(m["kind"], int) else KIND[m["kind"]]
    return _Mat(kind, *(float(m.get(k, 0.0)) for k in
                        ("E", "nu", "rho", "ppc", "theta_c", "theta_s", "xi", "bulk",
                         "h0", "h1", "h2", "h3")))


def _cfg(c: dict) -> _Cfg:
    bc = c.get("bc", "sticky")
    bc = bc if isinstance(bc, int) else BC[bc]
    g = c.get("gravity", (0.0, -9.8, 0.0))
    return _Cfg(int(c["n"]), bc, int(c.get("bc_cells", 3)), (ct.c_double * 3)(*map(float, g)), float(c["dt"]))


def _state(st: dict) -> dict:
    N = st["x"].shape[1]
    out = {
        "x": np.ascontiguousarray(st["x"], dtype=np.float64).copy(),
        "v": np.ascontiguousarray(st.get("v", np.zeros((3, N))), dtype=np.float64).copy(),
        "C": np.ascontiguousarray(st.get("C", np.zeros((9, N))), dtype=np.float64).copy(),
    }
    F = st.get("F")
    if F is None:
        F = np.zeros((9, N))
        F[[0, 4, 8]] = 1.0
    out["F"] = np.ascontiguousarray(F, dtype=np.float64).copy()
    s = st.get("s")
    out["s"] = np.ascontiguousarray(np.ones(N) if s is None else s, dtype=np.float64).copy()
    return out


def num_nodes(n: int) -> int:
    return (n + 1) ** 3


# --------------------------------------------------------------- per-particle
def svd3(F: np.ndarray):
    """One-sided Jacobi SVD of a 3x3 matrix; sigma descending, U,V in SO(3)."""
    F = np.ascontiguousarray(F, dtype=np.float64).reshape(9)
    U, S, V = np.zeros(9), np.zeros(3), np.zeros(9)
    lib().om_svd3(_p(F, ct.c_double), _p(U, ct.c_double), _p(S, ct.c_double), _p(V, ct.c_double))
    return U.reshape(3, 3), S, V.reshape(3, 3)


def fixed_corotated(F: np.ndarray, mu: float, la: float) -> np.ndarray:
    F = np.ascontiguousarray(F, dtype=np.float64).reshape(9)
    tau = np.zeros(9)
    lib().om_fixed_corotated(_p(F, ct.c_double), mu, la, _p(tau, ct.c_double))
    return tau.reshape(3, 3)


def stress(mat: dict, F: np.ndarray, s: float = 1.0) -> np.ndarray:
    F = np.ascontiguousarray(F, dtype=np.float64).reshape(9)
    tau = np.zeros(9)
    m = _mat(mat)
    lib().om_stress(ct.byref(m), _p(F, ct.c_double), float(s), _p(tau, ct.c_double))
    return tau.reshape(3, 3)


def snow_project(mat: dict, Fhat: np.ndarray, Jp: float):
    Fhat = np.ascontiguousarray(Fhat, dtype=np.float64).reshape(9)
    Fe = np.zeros(9)
    jp = ct.c_double(0.0)
    m = _mat(mat)
    lib().om_snow_project(ct.byref(m), _p(Fhat, ct.c_double), float(Jp), _p(Fe, ct.c_double), ct.byref(jp))
    return Fe.reshape(3, 3), jp.value


def hencky(F: np.ndarray, mu: float, la: float) -> np.ndarray:
    """Kirchhoff stress of the sand's log-strain (Hencky) elasticity."""
    F = np.ascontiguousarray(F, dtype=np.float64).reshape(9)
    tau = np.zeros(9)
    lib().om_hencky(_p(F, ct.c_double), mu, la, _p(tau, ct.c_double))
    return tau.reshape(3, 3)


def sand_alpha(mat: dict, q: float) -> float:
    m = _mat(mat)
    return lib().om_sand_alpha(ct.byref(m), float(q))


def sand_project(mat: dict, Fhat: np.ndarray, q: float):
    """Drucker-Prager return map: (elastic gradient, new hardening state q)."""
    Fhat = np.ascontiguousarray(Fhat, dtype=np.float64).reshape(9)
    Fe = np.zeros(9)
    qo = ct.c_double(0.0)
    m = _mat(mat)
    lib().om_sand_project(ct.byref(m), _p(Fhat, ct.c_double), float(q), _p(Fe, ct.c_double), ct.byref(qo))
    return Fe.reshape(3, 3), qo.value


def weights(t: float):
    base = ct.c_int(0)
    w = np.zeros(3)
    lib().om_weights(float(t), ct.byref(base), _p(w, ct.c_double))
    return base.value, w


# ------------------------------------------------------------------ substep
def p2g(cfg: dict, mat: dict, st: dict):
    """Returns (state copy, grid mass (n+1)^3, grid momentum (3,(n+1)^3), #skipped)."""
    s = _state(st)
    n = int(cfg["n"])
    NN = num_nodes(n)
    gm, gp = np.zeros(NN), np.zeros((3, NN))
    c, m = _cfg(cfg), _mat(mat)
    N = s["x"].shape[1]
    bad = lib().om_p2g(ct.byref(c), ct.byref(m), N, *(_p(s[k], ct.c_double) for k in "xvCFs"),
                       _p(gm, ct.c_double), _p(gp, ct.c_double))
    return s, gm, gp, bad


def grid_update(cfg: dict, gm: np.ndarray, gp: np.ndarray) -> np.ndarray:
    gv = np.ascontiguousarray(gp, dtype=np.float64).copy()
    gm = np.ascontiguousarray(gm, dtype=np.float64)
    c = _cfg(cfg)
    lib().om_grid_update(ct.byref(c), _p(gm, ct.c_double), _p(gv, ct.c_double))
    return gv


def g2p(cfg: dict, mat: dict, st: dict, gv: np.ndarray):
    s = _state(st)
    gv = np.ascontiguousarray(gv, dtype=np.float64)
    c, m = _cfg(cfg), _mat(mat)
    N = s["x"].shape[1]
    bad = lib().om_g2p(ct.byref(c), ct.byref(m), N, *(_p(s[k], ct.c_double) for k in "xvCFs"),
                       _p(gv, ct.c_double))
    return s, bad


def substep_asflip(cfg: dict, mat: dict, st: dict, flip: float, beta_min: float, beta_max: float,
                   steps: int = 1):
    """`steps` substeps with the ASFLIP transfer (om_substep_asflip).  Returns
    (state, grid mass, grid velocity of the last substep, skipped count)."""
    s = _state(st)
    n = int(cfg["n"])
    NN = num_nodes(n)
    gm, gv = np.zeros(NN), np.zeros((3, NN))
    c, m = _cfg(cfg), _mat(mat)
    N = s["x"].shape[1]
    bad = 0
    for _ in range(steps):
        bad += lib().om_substep_asflip(ct.byref(c), ct.byref(m), N, *(_p(s[k], ct.c_double) for k in "xvCFs"),
                                       _p(gm, ct.c_double), _p(gv, ct.c_double), float(flip), float(beta_min),
                                       float(beta_max))
    return s, gm, gv, bad


def frame_time_step(mat: dict, n: int, vmax: float, gravity, cfl: float, dt_max: float, frame: float):
    """The automatic step of a frame (a reading of the paper's automatically
    deduced steps): dt = min(dt_max, cfl dx / (vmax + |g| frame + c)) with c
    the pressure-wave speed (sqrt(bulk/rho) for water, sqrt((lambda + 2 mu)/rho)
    otherwise), then the frame cut into the fewest whole substeps no longer
    than that.  Returns (substeps, dt)."""
    import math

    kind = mat["kind"] if isinstance(mat["kind"], str) else {v: k for k, v in KIND.items()}[mat["kind"]]
    if kind == "water":
        c = math.sqrt(mat["bulk"] / mat["rho"])
    else:
        mu = mat["E"] / (2 * (1 + mat["nu"]))
        la = mat["E"] * mat["nu"] / ((1 + mat["nu"]) * (1 - 2 * mat["nu"]))
        c = math.sqrt((la + 2 * mu) / mat["rho"])
    g = math.sqrt(sum(float(a) ** 2 for a in gravity))
    dt = min(dt_max, cfl / n / (vmax + g * frame + c))
    ns = max(1, math.ceil(frame / dt - 1e-9))
    return ns, frame / ns


def g2p_trial(cfg: dict, mat: dict, st: dict, gv: np.ndarray):
    """G2P up to the trial gradient F^ = (I + dt C') F: x, v, C updated, F
    set to F^, s unchanged (no return map)."""
    s = _state(st)
    gv = np.ascontiguousarray(gv, dtype=np.float64)
    c, m = _cfg(cfg), _mat(mat)
    N = s["x"].shape[1]
    bad = lib().om_g2p_trial(ct.byref(c), ct.byref(m), N, *(_p(s[k], ct.c_double) for k in "xvCFs"),
                             _p(gv, ct.c_double))
    return s, bad


def substep(cfg: dict, mat: dict, st: dict, steps: int = 1, threads: int = 1):
    """Advance `steps` substeps.  Returns (state, grid mass, grid velocity of
    the last substep, total skipped-particle count).  threads > 1 (or 0 for
    every core) runs the multi-threaded form, whose sums are ordered
    differently (equal up to FP64 rounding)."""
    s = _state(st)
    n = int(cfg["n"])
    NN = num_nodes(n)
    gm, gv = np.zeros(NN), np.zeros((3, NN))
    c, m = _cfg(cfg), _mat(mat)
    N = s["x"].shape[1]
    bad = 0
    for _ in range(steps):
        args = (ct.byref(c), ct.byref(m), N, *(_p(s[k], ct.c_double) for k in "xvCFs"),
                _p(gm, ct.c_double), _p(gv, ct.c_double))
        if threads == 1:
            bad += lib().om_substep(*args)
        else:
            bad += lib().om_substep_omp(*args, int(threads))
    return s, gm, gv, bad


# ------------------------------------------------------------------ binning
def keys(x32: np.ndarray, n: int):
    """Particle codes of FP32 positions (3,N).  Returns (keys u32, cells (3,N) i32, #out-of-range)."""
    x32 = np.ascontiguousarray(x32, dtype=np.float32)
    N = x32.shape[1]
    k = np.zeros(N, dtype=np.uint32)
    cell = np.zeros((3, N), dtype=np.int32)
    bad = lib().om_keys(N, _p(x32, ct.c_float), int(n), _p(k, ct.c_uint32), _p(cell, ct.c_int32))
    return k, cell, bad


def stable_sort(k: np.ndarray):
    k = np.ascontiguousarray(k, dtype=np.uint32)
    N = k.shape[0]
    perm = np.zeros(N, dtype=np.int32)
    srt = np.zeros(N, dtype=np.uint32)
    lib().om_stable_sort(N, _p(k, ct.c_uint32), _p(perm, ct.c_int32), _p(srt, ct.c_uint32))
    return perm, srt


def gblocks(sorted_keys: np.ndarray):
    sk = np.ascontiguousarray(sorted_keys, dtype=np.uint32)
    N = sk.shape[0]
    code = np.zeros(max(N, 1), dtype=np.uint32)
    start = np.zeros(max(N, 1), dtype=np.int32)
    count = np.zeros(max(N, 1), dtype=np.int32)
    nb = lib().om_gblocks(N, _p(sk, ct.c_uint32), _p(code, ct.c_uint32), _p(start, ct.c_int32),
                          _p(count, ct.c_int32))
    return code[:nb].copy(), start[:nb].copy(), count[:nb].copy()


def pblocks(n: int, gcodes: np.ndarray) -> np.ndarray:
    g = np.ascontiguousarray(gcodes, dtype=np.uint32)
    NB = n // 4 + 2
    out = np.zeros(NB ** 3, dtype=np.int32)
    cnt = lib().om_pblocks(int(n), g.shape[0], _p(g, ct.c_uint32), _p(out, ct.c_int32))
    return out[:cnt].copy()


def free_zone_exit(x32: np.ndarray, n: int, B: np.ndarray) -> np.ndarray:
    x32 = np.ascontiguousarray(x32, dtype=np.float32)
    B = np.ascontiguousarray(B, dtype=np.int32)
    N = x32.shape[1]
    flags = np.zeros(N, dtype=np.uint8)
    lib().om_free_zone_exit(N, _p(x32, ct.c_float), int(n), _p(B, ct.c_int32), _p(flags, ct.c_uint8))
    return flags.astype(bool)


def bin_particles(x32: np.ndarray, n: int) -> dict:
    """Full plain binning: codes, stable order, geometric and physical blocks."""
    k, cell, bad = keys(x32, n)
    perm, srt = stable_sort(k)
    code, start, count = gblocks(srt)
    return {"keys": k, "cell": cell, "bad": bad, "perm": perm, "sorted": srt,
            "gblock": code, "gstart": start, "gcount": count, "pblock": pblocks(n, code)}
