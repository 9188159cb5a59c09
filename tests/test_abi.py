"""CPU checks of the C ABI: the library loads, exports every function the
header declares, and the Python binding's structs match the C layout.
No device work is done here."""
import ctypes as ct

import numpy as np
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpm.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(mpm_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2111_00699_amd import build, mpm

    if not os.path.exists(mpm.LIB_PATH):
        build.build()
    return mpm.load()


def test_header_declares_the_core_entry_points():
    names = _declared()
    for n in ("mpm_create", "mpm_destroy", "mpm_add_particles", "mpm_substep", "mpm_read_particles"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2111_00699_amd import mpm

    names = _declared()
    assert names, "no declarations parsed"
    for n in names:
        assert hasattr(lib, n), n
        assert n in mpm.SIGNATURES, f"binding lacks {n}"
    out = subprocess.run(["nm", "-D", "--defined-only", mpm.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (mpm_\w+)", out))
    assert set(names) <= exported
    assert not (exported - set(names)), f"undeclared exports: {exported - set(names)}"


def test_struct_layouts_match_the_header():
    from paper_2111_00699_amd import mpm

    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "mpm.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(mpm_config), sizeof(mpm_material), sizeof(mpm_stats),
         sizeof(mpm_profile_data), sizeof(mpm_scene), sizeof(mpm_scene_stats));
  printf("%zu %zu %zu %zu %zu %zu\n", offsetof(mpm_config, dt), offsetof(mpm_config, capacity),
         offsetof(mpm_config, stream), offsetof(mpm_config, flags), offsetof(mpm_config, chunk),
         offsetof(mpm_config, scenes));
  printf("%zu %zu %zu %zu\n", offsetof(mpm_stats, error), offsetof(mpm_profile_data, ms),
         offsetof(mpm_scene, dt), offsetof(mpm_scene_stats, n));
  return 0;
}'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "t")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        lines = subprocess.check_output([exe], text=True).split("\n")
    sizes = list(map(int, lines[0].split()))
    assert sizes == [ct.sizeof(mpm.Config), ct.sizeof(mpm.Material), ct.sizeof(mpm.Stats),
                     ct.sizeof(mpm.ProfileData), ct.sizeof(mpm.SceneDesc), ct.sizeof(mpm.SceneStats)]
    offs = list(map(int, lines[1].split()))
    assert offs == [mpm.Config.dt.offset, mpm.Config.capacity.offset, mpm.Config.stream.offset,
                    mpm.Config.flags.offset, mpm.Config.chunk.offset, mpm.Config.scenes.offset]
    assert list(map(int, lines[2].split())) == [mpm.Stats.error.offset, mpm.ProfileData.ms.offset,
                                                mpm.SceneDesc.dt.offset, mpm.SceneStats.n.offset]


def test_create_rejects_bad_configs_without_a_device(lib):
    """Argument validation happens before any device call."""
    from paper_2111_00699_amd import mpm

    def cfg(**kw):
        base = dict(n=64, bc=0, bc_cells=3, num_scenes=1, dt=1e-4, capacity=0, stream=0, flags=0, lag=0, chunk=0)
        base.update(kw)
        c = mpm.Config()
        for k, v in base.items():
            setattr(c, k, v)
        return c

    h = ct.c_void_p()
    for bad in (dict(n=48), dict(n=8), dict(n=1024), dict(bc=7), dict(dt=0.0), dict(num_scenes=0),
                dict(num_scenes=257), dict(n=512, num_scenes=64),  # 3*9 + 6 key bits > 32
                dict(lag=100), dict(chunk=100), dict(capacity=-1), dict(flags=0x20)):  # graphs need a stream
        assert lib.mpm_create(ct.byref(cfg(**bad)), ct.byref(h)) == mpm.EINVAL, bad
        assert lib.mpm_last_error(None)
    # a bad per-scene descriptor
    arr = (mpm.SceneDesc * 2)()
    arr[0] = mpm.SceneDesc(64, 0, 3, (ct.c_float * 3)(0, -9.8, 0), 1e-4)
    arr[1] = mpm.SceneDesc(96, 0, 3, (ct.c_float * 3)(0, -9.8, 0), 1e-4)
    c = cfg(num_scenes=2)
    c.scenes = ct.cast(arr, ct.POINTER(mpm.SceneDesc))
    assert lib.mpm_create(ct.byref(c), ct.byref(h)) == mpm.EINVAL
    assert b"power of two" in lib.mpm_last_error(None)
    assert lib.mpm_create(None, ct.byref(h)) == mpm.EINVAL
    assert lib.mpm_destroy(None) == mpm.OK


def test_binding_refuses_to_run_without_the_library(monkeypatch, tmp_path):
    from paper_2111_00699_amd import mpm

    monkeypatch.setattr(mpm, "_lib", None)
    monkeypatch.setattr(mpm, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        mpm.load()


def test_documented_chunk_layout_rule_is_a_permutation():
    """The dealt storage order include/mpm.h documents is a permutation of
    every chunk size; in a dense half block (32 cells of 8 particles, one
    chunk of 256) each 16-lane pass meets 16 different bank pairs and no cell
    twice; and particles of one cell land in different passes."""
    from tests.test_gpu_parity import _compact3, dealt_order, dealt_slot

    for count in list(range(1, 40)) + [63, 64, 65, 127, 200, 255, 256, 257, 400, 511, 512]:
        slots = [dealt_slot(count, r) for r in range(count)]
        assert sorted(slots) == list(range(count)), count
    # the first 32 cells of a block in Morton order (a 4 x 4 x 2 slab), 8 particles each
    keys = np.repeat((5 << 6) + np.arange(32), 8)
    order = dealt_order(keys)
    assert sorted(order.tolist()) == list(range(keys.size))
    cell = keys[order] & 63
    x = 4 * _compact3(5) + _compact3(cell)
    y = 4 * _compact3(5 >> 1) + _compact3(cell >> 1)
    z = 4 * _compact3(5 >> 2) + _compact3(cell >> 2)
    bank = (x + 12 * y + 8 * z) & 15
    for p in range(0, keys.size, 16):
        assert len(set(bank[p:p + 16].tolist())) == 16
        assert len(set(cell[p:p + 16].tolist())) == 16
    # ragged chunks: the particles of one cell spread over the passes
    for size, want in ((32, 2), (48, 3)):
        ragged = np.array([0, 0, 0] + list(range(1, size - 2)))
        o = dealt_order(ragged)
        passes = {int(np.flatnonzero(o == i)[0]) // 16 for i in range(3)}
        assert len(passes) == want, size


def test_noalloc_limits_match_the_header():
    from paper_2111_00699_amd import mpm

    text = open(HEADER).read()
    got = {k: int(v) for k, v in re.findall(r"#define (MPM_SUR_NOALLOC_MAX_\w+) (\d+)", text)}
    assert got == {"MPM_SUR_NOALLOC_MAX_BATCH": mpm.SUR_NOALLOC_MAX_BATCH,
                   "MPM_SUR_NOALLOC_MAX_STEPS": mpm.SUR_NOALLOC_MAX_STEPS}
