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
# MPM_LIBRARY selects a build of the library: "fast" (the default, fast-math
# flags) or one of the ablation builds: "precise" (IEEE division, square root
# and denormals), "aosoa" (grouped particle layout), "lds_weights" (P2G
# stencil weights kept in LDS).
LIB_VARIANTS = {"fast": "libmpm.so", "precise": "libmpm_precise.so", "aosoa": "libmpm_aosoa.so",
                "lds_weights": "libmpm_lds_weights.so"}
LIB_PATH = os.path.join(HERE, LIB_VARIANTS[os.environ.get("MPM_LIBRARY", "fast") or "fast"])

KIND = {"jelly": 0, "snow": 1, "water": 2, "sand": 3}
BC = {"sticky": 0, "slip": 1, "separate": 2}

OK, EINVAL, ENOMEM, EDEVICE, ESTATE = 0, -1, -2, -3, -4
ERR_NONFINITE, ERR_DOMAIN, ERR_CAPACITY = 0x1, 0x2, 0x4
FLAG_REBUILD_EVERY_STEP, FLAG_P2G_GLOBAL_ATOMICS, FLAG_MANUAL_REBUILD, FLAG_P2G_SORTED_LANES = 0x1, 0x2, 0x4, 0x8
FLAG_G2P_GLOBAL_GATHER, FLAG_FRAME_GRAPHS, FLAG_FUSED_G2P, FLAG_SEPARATE_G2P = 0x10, 0x20, 0x40, 0x80
FLAG_SEPARATE_WALLS, FLAG_SEPARATE_CLEAR, FLAG_ALLOC_EXACT, FLAG_CHUNK_PER_BLOCK = 0x100, 0x200, 0x400, 0x800
MAX_SCENES = 256
PHASE_REBUILD, PHASE_P2G, PHASE_GRID, PHASE_G2P = 0x1, 0x2, 0x4, 0x8


def PROFILE_EVERY(n: int) -> int:
    """Mask bits that bracket only every n-th launch of a phase."""
    return (int(n) & 0xFFFF) << 16
PHASES = ("rebuild", "p2g", "grid", "g2p")


class SceneDesc(ct.Structure):
    _fields_ = [("n", ct.c_int32), ("bc", ct.c_int32), ("bc_cells", ct.c_int32), ("gravity", ct.c_float * 3),
                ("dt", ct.c_float)]


class Config(ct.Structure):
    _fields_ = [("n", ct.c_int32), ("bc", ct.c_int32), ("bc_cells", ct.c_int32), ("num_scenes", ct.c_int32),
                ("gravity", ct.c_float * 3), ("dt", ct.c_float), ("capacity", ct.c_int64),
                ("stream", ct.c_uint64), ("flags", ct.c_uint32), ("lag", ct.c_int32), ("chunk", ct.c_int32),
                ("reserved", ct.c_int32), ("scenes", ct.POINTER(SceneDesc))]


class SceneStats(ct.Structure):
    _fields_ = [("num_particles", ct.c_int64), ("substeps", ct.c_int64), ("gblocks", ct.c_int64),
                ("active_blocks", ct.c_int64), ("n", ct.c_int32), ("dt", ct.c_float)]


class Material(ct.Structure):
    _fields_ = [("kind", ct.c_int32)] + [(k, ct.c_float) for k in
                                         ("E", "nu", "rho", "ppc", "theta_c", "theta_s", "xi", "bulk",
                                          "h0", "h1", "h2", "h3")]


class Stats(ct.Structure):
    _fields_ = [(k, ct.c_int64) for k in ("num_particles", "capacity", "substeps", "rebuilds", "gblocks",
                                          "active_blocks", "chunks", "overflow_blocks")] + \
               [("error", ct.c_uint32), ("pending_update", ct.c_uint32)] + \
               [("p2g_fallback_chunks", ct.c_int64), ("p2g_global_particles", ct.c_int64),
                ("surrogate_particles", ct.c_int64), ("surrogate_fallbacks", ct.c_int64)]


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
    "mpm_get_scene_stats": (ct.c_int, [P, ct.c_int32, ct.POINTER(SceneStats)]),
    "mpm_autotune": (ct.c_int, [P, ct.c_float, ct.c_int32, ct.POINTER(ct.c_int32)]),
    "mpm_clear_error": (ct.c_int, [P]),
    "mpm_profile": (ct.c_int, [P, ct.c_uint32]),
    "mpm_profile_read": (ct.c_int, [P, ct.POINTER(ProfileData)]),
    "mpm_last_error": (ct.c_char_p, [P]),
    "mpm_surrogate_create": (ct.c_int, [ct.c_uint64, ct.POINTER(P)]),
    "mpm_surrogate_destroy": (ct.c_int, [P]),
    "mpm_surrogate_set": (ct.c_int, [P, P, P]),
    "mpm_surrogate_get": (ct.c_int, [P, P, P]),
    "mpm_surrogate_forward": (ct.c_int, [P, ct.c_int32, ct.c_int64, P, P]),
    "mpm_surrogate_loss_grad": (ct.c_int, [P, ct.c_int32, ct.c_int64, P, P, P, P]),
    "mpm_surrogate_fit_norm": (ct.c_int, [P, ct.c_int64, P, P]),
    "mpm_surrogate_train": (ct.c_int, [P, ct.c_int64, P, P, ct.c_int32, ct.c_int32, ct.c_float, ct.c_uint64, P]),
    "mpm_surrogate_train_noalloc": (ct.c_int, [P, ct.c_int64, P, P, ct.c_int32, ct.c_int32, ct.c_float, ct.c_uint64,
                                               P]),
    "mpm_surrogate_sample": (ct.c_int, [P, ct.c_int32, ct.c_float, ct.c_int64, P, P, ct.POINTER(ct.c_int64)]),
    "mpm_use_surrogate": (ct.c_int, [P, ct.c_int32, P, ct.c_int32, ct.c_float, ct.c_float]),
    "mpm_set_transfer": (ct.c_int, [P, ct.c_int32, ct.c_float, ct.c_float, ct.c_float]),
    "mpm_set_auto_dt": (ct.c_int, [P, ct.c_float, ct.c_float]),
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
                            ("E", "nu", "rho", "ppc", "theta_c", "theta_s", "xi", "bulk",
                             "h0", "h1", "h2", "h3")))


def _ptr(t):
    return None if t is None else ct.c_void_p(t.data_ptr())


class Sim:
    """One simulation context on the current CUDA (HIP) device.

    `scenes` (optional) is a list of per-scene dicts with keys n, dt and
    optionally bc, bc_cells, gravity; without it the context holds
    `num_scenes` copies of the scene given by the other arguments."""

    def __init__(self, n: int, dt: float, bc="sticky", bc_cells: int = 3, gravity=(0.0, -9.8, 0.0),
                 capacity: int = 0, flags: int = 0, lag: int = 0, chunk: int = 0, stream=None,
                 scenes: list | None = None, num_scenes: int = 1):
        import torch

        self.torch = torch
        self.lib = load()
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        bcv = lambda b: b if isinstance(b, int) else BC[b]
        if scenes is not None:
            num_scenes = len(scenes)
            arr = (SceneDesc * num_scenes)()
            for k, d in enumerate(scenes):
                arr[k] = SceneDesc(int(d["n"]), bcv(d.get("bc", bc)), int(d.get("bc_cells", bc_cells)),
                                   (ct.c_float * 3)(*map(float, d.get("gravity", gravity))), float(d["dt"]))
            self._scene_arr = arr
            self.ns = [int(d["n"]) for d in scenes]
        else:
            arr = None
            self.ns = [int(n)] * num_scenes
        cfg = Config(int(n), bcv(bc), int(bc_cells), int(num_scenes), (ct.c_float * 3)(*map(float, gravity)),
                     float(dt), int(capacity), int(self.stream.cuda_stream), int(flags), int(lag), int(chunk), 0,
                     ct.cast(arr, ct.POINTER(SceneDesc)) if arr is not None else None)
        self.cfg = cfg
        self.n = self.ns[0]
        h = ct.c_void_p()
        r = self.lib.mpm_create(ct.byref(cfg), ct.byref(h))
        if r != OK:
            raise MPMError(r, self.lib.mpm_last_error(None).decode())
        self.h = h
        self.counts = [0] * int(num_scenes)

    @property
    def N(self) -> int:
        return self.counts[0] if len(self.counts) == 1 else sum(self.counts)

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
        self.counts[scene] += count

    def substep(self, n: int = 1):
        self._check(self.lib.mpm_substep(self.h, int(n)))

    def frame(self, frame_dt: float):
        self._check(self.lib.mpm_frame(self.h, float(frame_dt)))

    def rebuild(self):
        self._check(self.lib.mpm_rebuild(self.h))

    def synchronize(self):
        self._check(self.lib.mpm_synchronize(self.h))

    def read_particles(self, check: bool = True, scene: int = 0) -> dict:
        N = self.counts[scene]
        z = lambda r: self.torch.empty((r, N), dtype=self.torch.float32, device=self.device)
        out = {"x": z(3), "v": z(3), "C": z(9), "F": z(9),
               "s": self.torch.empty(N, dtype=self.torch.float32, device=self.device)}
        r = self.lib.mpm_read_particles(self.h, scene, N, *(_ptr(out[k]) for k in ("x", "v", "C", "F", "s")))
        if check:
            self._check(r)
        return out

    def read_grid(self, scene: int = 0):
        n1 = self.ns[scene] + 1
        m = self.torch.empty(n1 ** 3, dtype=self.torch.float32, device=self.device)
        v = self.torch.empty((3, n1 ** 3), dtype=self.torch.float32, device=self.device)
        self._check(self.lib.mpm_read_grid(self.h, scene, _ptr(m), _ptr(v)))
        return m, v

    def read_binning(self, count=None, scene: int = 0):
        count = self.counts[scene] if count is None else count
        keys = self.torch.empty(count, dtype=self.torch.int32, device=self.device)
        perm = self.torch.empty(count, dtype=self.torch.int32, device=self.device)
        self._check(self.lib.mpm_read_binning(self.h, scene, count, _ptr(keys), _ptr(perm)))
        return keys.cpu().numpy().view(np.uint32), perm.cpu().numpy()

    def read_blocks(self, scene: int = 0):
        st = self.scene_stats(scene)
        ng, na = st["gblocks"], st["active_blocks"]
        gcode = np.zeros(max(ng, 1), dtype=np.uint32)
        gstart = np.zeros(max(ng, 1), dtype=np.int32)
        gcount = np.zeros(max(ng, 1), dtype=np.int32)
        active = np.zeros(max(na, 1), dtype=np.int32)
        self._check(self.lib.mpm_read_blocks(self.h, scene, gcode.ctypes.data, gstart.ctypes.data,
                                             gcount.ctypes.data, active.ctypes.data))
        return {"gcode": gcode[:ng], "gstart": gstart[:ng], "gcount": gcount[:ng], "active": active[:na]}

    def stats(self, check: bool = True) -> dict:
        s = Stats()
        r = self.lib.mpm_get_stats(self.h, ct.byref(s))
        if check:
            self._check(r)
        return {k: getattr(s, k) for k, _ in Stats._fields_}

    def scene_stats(self, scene: int = 0) -> dict:
        s = SceneStats()
        self._check(self.lib.mpm_get_scene_stats(self.h, scene, ct.byref(s)))
        return {k: getattr(s, k) for k, _ in SceneStats._fields_}

    def autotune(self, frame_dt: float, frames: int = 1) -> int:
        out = ct.c_int32(0)
        self._check(self.lib.mpm_autotune(self.h, float(frame_dt), int(frames), ct.byref(out)))
        return out.value

    def clear_error(self):
        self._check(self.lib.mpm_clear_error(self.h))

    def use_surrogate(self, mode: int, surrogate=None, tol: float = 1e-3, dt_ref: float = 5e-5, scene: int = 0):
        """0 exact return map, 1 learned surrogate, 2 closed form without the network."""
        h = surrogate.h if surrogate is not None else None
        self._sur = surrogate  # keep it alive while the context uses it
        self._check(self.lib.mpm_use_surrogate(self.h, scene, h, int(mode), float(tol), float(dt_ref)))

    def set_transfer(self, flip: float, beta_min: float = 0.0, beta_max: float = 1.0, scene: int = 0):
        """ASFLIP with flip ratio `flip` and position-correction shares (0 restores APIC)."""
        self._check(self.lib.mpm_set_transfer(self.h, scene, float(flip), float(beta_min), float(beta_max)))

    def set_auto_dt(self, cfl: float, dt_max: float):
        """Per-frame automatic time step (0 turns it off)."""
        self._check(self.lib.mpm_set_auto_dt(self.h, float(cfl), float(dt_max)))

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


SUR_IN, SUR_OUT, SUR_PARAMS, SUR_NORM = 12, 12, 5772, 48
# limits of mpm_surrogate_train_noalloc (its fixed scratch array)
SUR_NOALLOC_MAX_BATCH, SUR_NOALLOC_MAX_STEPS = 65536, 4096
SUR_FP32, SUR_BF16 = 0, 1


class Surrogate:
    """The learned snow return map: an MLP 12 -> 64 -> 64 -> 12 trained and
    run by the library's kernels (BF16 MFMA with FP32 accumulation; FP32 for
    gradient checks).  Arrays are torch CUDA tensors or host arrays."""

    def __init__(self, stream=None):
        import torch

        self.torch = torch
        self.lib = load()
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ct.c_void_p()
        r = self.lib.mpm_surrogate_create(int(self.stream.cuda_stream), ct.byref(h))
        if r != OK:
            raise MPMError(r, self.lib.mpm_last_error(None).decode())
        self.h = h

    def _check(self, r):
        if r != OK:
            raise MPMError(r, self.lib.mpm_last_error(None).decode())

    def _t(self, a, n=None):
        t = self.torch.as_tensor(np.asarray(a) if not isinstance(a, self.torch.Tensor) else a,
                                 dtype=self.torch.float32).to(self.device).contiguous()
        if n is not None and t.numel() != n:
            raise ValueError(f"expected {n} values, got {t.numel()}")
        return t

    def set(self, theta=None, norm=None):
        th = None if theta is None else self._t(theta, SUR_PARAMS)
        nm = None if norm is None else self._t(norm, SUR_NORM)
        self._check(self.lib.mpm_surrogate_set(self.h, _ptr(th), _ptr(nm)))
        self.synchronize()

    def get(self):
        th = self.torch.empty(SUR_PARAMS, dtype=self.torch.float32, device=self.device)
        nm = self.torch.empty(SUR_NORM, dtype=self.torch.float32, device=self.device)
        self._check(self.lib.mpm_surrogate_get(self.h, _ptr(th), _ptr(nm)))
        self.synchronize()
        return th, nm

    def synchronize(self):
        self.stream.synchronize()

    def forward(self, X, precision=SUR_BF16):
        X = self._t(X)
        n = X.numel() // SUR_IN
        Y = self.torch.empty((n, SUR_OUT), dtype=self.torch.float32, device=self.device)
        self._check(self.lib.mpm_surrogate_forward(self.h, int(precision), n, _ptr(X), _ptr(Y)))
        self.synchronize()
        return Y

    def loss_grad(self, X, T, precision=SUR_FP32):
        X, T = self._t(X), self._t(T)
        n = X.numel() // SUR_IN
        g = self.torch.empty(SUR_PARAMS, dtype=self.torch.float32, device=self.device)
        l = self.torch.empty(1, dtype=self.torch.float32, device=self.device)
        self._check(self.lib.mpm_surrogate_loss_grad(self.h, int(precision), n, _ptr(X), _ptr(T), _ptr(g), _ptr(l)))
        self.synchronize()
        return float(l.item()), g

    def fit_norm(self, X, T):
        X, T = self._t(X), self._t(T)
        self._check(self.lib.mpm_surrogate_fit_norm(self.h, X.numel() // SUR_IN, _ptr(X), _ptr(T)))
        self.synchronize()

    def train(self, X, T, steps, batch=4096, lr=1e-3, seed=0, noalloc=False):
        """Adam steps on minibatches of (X, T); noalloc selects the entry point
        that keeps its scratch in the library's fixed device array."""
        X, T = self._t(X), self._t(T)
        losses = np.zeros(max(int(steps), 1), dtype=np.float32)
        fn = self.lib.mpm_surrogate_train_noalloc if noalloc else self.lib.mpm_surrogate_train
        self._check(fn(self.h, X.numel() // SUR_IN, _ptr(X), _ptr(T), int(steps), int(batch), float(lr), int(seed),
                       losses.ctypes.data))
        return losses[:int(steps)]

    @staticmethod
    def sample(sim, scene=0, dt_ref=5e-5, max_count=None):
        """Training pairs (X, T) from the current state of a snow scene."""
        torch = sim.torch
        n = sim.counts[scene] if max_count is None else int(max_count)
        X = torch.empty((max(n, 1), SUR_IN), dtype=torch.float32, device=sim.device)
        T = torch.empty((max(n, 1), SUR_OUT), dtype=torch.float32, device=sim.device)
        w = ct.c_int64(0)
        sim._check(sim.lib.mpm_surrogate_sample(sim.h, scene, float(dt_ref), n, _ptr(X), _ptr(T), ct.byref(w)))
        return X[:w.value], T[:w.value]

    def close(self):
        if getattr(self, "h", None):
            self.lib.mpm_surrogate_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
