"""ctypes binding of libmpm.so (the C ABI in include/mpm.h).

Argument marshalling only: every step of the simulation runs in the HIP
kernels of the library.  torch supplies device memory and the stream.  If the
library is missing this module raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpm.so")

KIND = {"jelly": 0, "snow": 1, "water": 2}
BC = {"sticky": 0, "slip": 1, "separate": 2}

OK, EINVAL, ENOMEM, EDEVICE, ESTATE = 0, -1, -2, -3, -4
ERR_NONFINITE, ERR_DOMAIN, ERR_CAPACITY = 0x1, 0x2, 0x4
FLAG_REBUILD_EVERY_STEP, FLAG_P2G_GLOBAL_ATOMICS, FLAG_MANUAL_REBUILD, FLAG_P2G_SORTED_LANES = 0x1, 0x2, 0x4, 0x8
FLAG_G2P_GLOBAL_GATHER = 0x10
PHASE_REBUILD, PHASE_P2G, PHASE_GRID, PHASE_G2P = 0x1, 0x2, 0x4, 0x8
PHASES = ("rebuild", "p2g", "grid", "g2p")


class Config(ct.Structure):
    _fields_ = [("n", ct.c_int32), ("bc", ct.c_int32), ("bc_cells", ct.c_int32), ("num_scenes", ct.c_int32),
                ("gravity", ct.c_float * 3), ("dt", ct.c_float), ("capacity", ct.c_int64),
                ("stream", ct.c_uint64), ("flags", ct.c_uint32), ("lag", ct.c_int32), ("chunk", ct.c_int32),
                ("reserved", ct.c_int32)]


class Material(ct.Structure):
    _fields_ = [("kind", ct.c_int32)] + [(k, ct.c_float) for k in
                                         ("E", "nu", "rho", "ppc", "theta_c", "theta_s", "xi", "bulk")]


class Stats(ct.Structure):
    _fields_ = [(k, ct.c_int64) for k in ("num_particles", "capacity", "substeps", "rebuilds", "gblocks",
                                          "active_blocks", "chunks", "overflow_blocks")] + \
               [("error", ct.c_uint32), ("pending_update", ct.c_uint32)] + \
               [("p2g_fallback_chunks", ct.c_int64), ("p2g_global_particles", ct.c_int64)]


class ProfileData(ct.Structure):
    _fields_ = [("launches", ct.c_int64 * 4), ("ms", ct.c_double * 4)]


class MPMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mpm error {code}: {msg}")
        self.code = code


# name -> (restype, argtypes); mirrors include/mpm.h
P = ct.c_void_p
SIGNATURES = {
    "mpm_create": (ct.c_int, [ct.POINTER(Config), ct.POINTER(P)]),
    "mpm_destroy": (ct.c_int, [P]),
    "mpm_add_particles": (ct.c_int, [P, ct.c_int32, ct.POINTER(Material), ct.c_int64, P, P, P, P, P]),
    "mpm_substep": (ct.c_int, [P, ct.c_int32]),
    "mpm_frame": (ct.c_int, [P, ct.c_float]),
    "mpm_rebuild": (ct.c_int, [P]),
    "mpm_synchronize": (ct.c_int, [P]),
    "mpm_read_particles": (ct.c_int, [P, ct.c_int32, ct.c_int64, P, P, P, P, P]),
    "mpm_read_grid": (ct.c_int, [P, ct.c_int32, P, P]),
    "mpm_read_binning": (ct.c_int, [P, ct.c_int32, ct.c_int64, P, P]),
    "mpm_read_blocks": (ct.c_int, [P, ct.c_int32, P, P, P, P]),
    "mpm_get_stats": (ct.c_int, [P, ct.POINTER(Stats)]),
    "mpm_clear_error": (ct.c_int, [P]),
    "mpm_profile": (ct.c_int, [P, ct.c_uint32]),
    "mpm_profile_read": (ct.c_int, [P, ct.POINTER(ProfileData)]),
    "mpm_last_error": (ct.c_char_p, [P]),
}

_lib = None


def load() -> ct.CDLL:
    """Load libmpm.so (built by paper_2111_00699_amd.build); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2111_00699_amd.build`")
        lib = ct.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def material(m: dict) -> Material:
    kind = m["kind"] if isinstance(m["kind"], int) else KIND[m["kind"]]
    return Material(kind, *(float(m.get(k, 0.0)) for k in
                            ("E", "nu", "rho", "ppc", "theta_c", "theta_s", "xi", "bulk")))


def _ptr(t):
    return None if t is None else ct.c_void_p(t.data_ptr())


class Sim:
    """One simulation context on the current CUDA (HIP) device."""

    def __init__(self, n: int, dt: float, bc="sticky", bc_cells: int = 3, gravity=(0.0, -9.8, 0.0),
                 capacity: int = 0, flags: int = 0, lag: int = 0, chunk: int = 0, stream=None):
        import torch

        self.torch = torch
        self.lib = load()
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        cfg = Config(int(n), bc if isinstance(bc, int) else BC[bc], int(bc_cells), 1,
                     (ct.c_float * 3)(*map(float, gravity)), float(dt), int(capacity),
                     int(self.stream.cuda_stream), int(flags), int(lag), int(chunk), 0)
        self.cfg = cfg
        self.n = int(n)
        h = ct.c_void_p()
        r = self.lib.mpm_create(ct.byref(cfg), ct.byref(h))
        if r != OK:
            raise MPMError(r, self.lib.mpm_last_error(None).decode())
        self.h = h
        self.N = 0

    # ------------------------------------------------------------ helpers
    def _check(self, r):
        if r != OK:
            raise MPMError(r, self.lib.mpm_last_error(self.h).decode())

    def _dev(self, a, rows, count):
        if a is None:
            return None
        t = self.torch.as_tensor(np.asarray(a) if not isinstance(a, self.torch.Tensor) else a,
                                 dtype=self.torch.float32)
        t = t.to(self.device).contiguous()
        if t.numel() != rows * count:
            raise ValueError(f"expected {rows}x{count} values, got shape {tuple(t.shape)}")
        return t

    # ------------------------------------------------------------ ABI calls
    def add_particles(self, mat: dict | None, x, v=None, C=None, F=None, s=None, scene: int = 0):
        x = self.torch.as_tensor(x) if not isinstance(x, self.torch.Tensor) else x
        count = int(x.shape[-1]) if x.dim() == 2 else int(x.numel() // 3)
        ts = [self._dev(x, 3, count), self._dev(v, 3, count), self._dev(C, 9, count),
              self._dev(F, 9, count), self._dev(s, 1, count)]
        m = material(mat) if mat is not None else None
        r = self.lib.mpm_add_particles(self.h, scene, ct.byref(m) if m is not None else None, count,
                                       *(_ptr(t) for t in ts))
        self._keep = ts  # the copies must live until the insert kernel has run
        self._check(r)
        self.N += count

    def substep(self, n: int = 1):
        self._check(self.lib.mpm_substep(self.h, int(n)))

    def frame(self, frame_dt: float):
        self._check(self.lib.mpm_frame(self.h, float(frame_dt)))

    def rebuild(self):
        self._check(self.lib.mpm_rebuild(self.h))

    def synchronize(self):
        self._check(self.lib.mpm_synchronize(self.h))

    def read_particles(self, check: bool = True) -> dict:
        N = self.N
        z = lambda r: self.torch.empty((r, N), dtype=self.torch.float32, device=self.device)
        out = {"x": z(3), "v": z(3), "C": z(9), "F": z(9),
               "s": self.torch.empty(N, dtype=self.torch.float32, device=self.device)}
        r = self.lib.mpm_read_particles(self.h, 0, N, *(_ptr(out[k]) for k in ("x", "v", "C", "F", "s")))
        if check:
            self._check(r)
        return out

    def read_grid(self):
        n1 = self.n + 1
        m = self.torch.empty(n1 ** 3, dtype=self.torch.float32, device=self.device)
        v = self.torch.empty((3, n1 ** 3), dtype=self.torch.float32, device=self.device)
        self._check(self.lib.mpm_read_grid(self.h, 0, _ptr(m), _ptr(v)))
        return m, v

    def read_binning(self, count=None):
        count = self.N if count is None else count
        keys = self.torch.empty(count, dtype=self.torch.int32, device=self.device)
        perm = self.torch.empty(count, dtype=self.torch.int32, device=self.device)
        self._check(self.lib.mpm_read_binning(self.h, 0, count, _ptr(keys), _ptr(perm)))
        return keys.cpu().numpy().view(np.uint32), perm.cpu().numpy()

    def read_blocks(self):
        st = self.stats()
        ng, na = st["gblocks"], st["active_blocks"]
        gcode = np.zeros(max(ng, 1), dtype=np.uint32)
        gstart = np.zeros(max(ng, 1), dtype=np.int32)
        gcount = np.zeros(max(ng, 1), dtype=np.int32)
        active = np.zeros(max(na, 1), dtype=np.int32)
        self._check(self.lib.mpm_read_blocks(self.h, 0, gcode.ctypes.data, gstart.ctypes.data,
                                             gcount.ctypes.data, active.ctypes.data))
        return {"gcode": gcode[:ng], "gstart": gstart[:ng], "gcount": gcount[:ng], "active": active[:na]}

    def stats(self, check: bool = True) -> dict:
        s = Stats()
        r = self.lib.mpm_get_stats(self.h, ct.byref(s))
        if check:
            self._check(r)
        return {k: getattr(s, k) for k, _ in Stats._fields_}

    def clear_error(self):
        self._check(self.lib.mpm_clear_error(self.h))

    def profile(self, mask: int):
        self._check(self.lib.mpm_profile(self.h, int(mask)))

    def profile_read(self) -> dict:
        d = ProfileData()
        self._check(self.lib.mpm_profile_read(self.h, ct.byref(d)))
        return {name: {"launches": d.launches[i], "ms": d.ms[i]} for i, name in enumerate(PHASES)}

    def close(self):
        if getattr(self, "h", None):
            self.lib.mpm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
