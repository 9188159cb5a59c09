"""One-substep parity of a library build against the FP64 oracle, run in a
process of its own by tests/test_gpu_ablations.py (the build is chosen by
MPM_LIBRARY before the library loads).  Prints one JSON line of per-case
normwise errors and exits non-zero if a case misses its bar."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2111_00699_amd import mpm, scenes  # noqa: E402


def normwise(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


def main():
    import torch

    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    tol = float(os.environ.get("VARIANT_TOL", "1e-4"))
    mats = {"jelly": (scenes.JELLY, "sticky"), "snow": (scenes.SNOW, "separate"), "water": (scenes.WATER, "slip"),
            "sand": (scenes.SAND, "slip")}
    out, ok = {"library": os.path.basename(mpm.LIB_PATH)}, True
    for kind, (mat, bc) in mats.items():
        st = scenes.nontrivial_state(scenes.jelly_cube(0)["x"], seed=5, kind=kind)
        cfg = dict(n=64, dt=1e-4, bc=bc)
        sim = mpm.Sim(64, 1e-4, bc=bc)
        sim.add_particles(mat, st["x"], v=st["v"], C=st["C"], F=st.get("F"), s=st.get("s"))
        sim.substep(2)
        gs = {k: t.cpu().numpy() for k, t in sim.read_particles().items()}
        sim.close()
        os_, _, _, bad = oracle.substep(cfg, mat, st, steps=2)
        errs = {k: normwise(gs[k], os_[k]) for k in ("x", "v", "C", "F", "s")
                if not (k == "F" and kind == "water") and not (k == "s" and kind == "jelly")}
        out[kind] = errs
        ok = ok and bad == 0 and all(e <= tol for e in errs.values())
    print(json.dumps(out), flush=True)
    sys.exit(0 if ok else 1)


if __name__ == "__main__":
    main()
