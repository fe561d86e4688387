"""Host-side checks of the C ABI (no GPU compute): the library loads, exports every entry
point declared in include/gsr.h, and fails cleanly on bad arguments or a missing device."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gsr.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w]+\s*\*?\s*(gsr_\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    import paper_2507_21981_amd as g
    return g.lib()


def test_header_declares_the_boundary():
    fns = declared_functions()
    for f in ("gsr_create", "gsr_destroy", "gsr_compose_scene", "gsr_render_rgbd", "gsr_saved_render",
              "gsr_render_backward", "gsr_query_status", "gsr_copy_pairs", "gsr_autotune", "gsr_stage_times"):
        assert f in fns, f


def test_library_exports_every_declared_symbol(lib):
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", lib._name], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (gsr_\w+)", out))
    assert set(declared_functions()) <= exported


def test_create_without_device_or_with_bad_arguments_fails_cleanly(lib):
    import torch
    h = ctypes.c_void_p()
    # out == NULL
    assert lib.gsr_create(0, None, None) == -1
    if not torch.cuda.is_available():
        rc = lib.gsr_create(0, None, ctypes.byref(h))
        assert rc == -3 and not h.value
        assert b"no HIP device" in lib.gsr_last_error(None)


def test_null_context_calls_return_invalid(lib):
    import paper_2507_21981_amd as g
    assert lib.gsr_render_rgbd(None, None, 1, None, 16, 16, None, None, None, 0, None) == -1
    assert lib.gsr_render_backward(None, None, 0, None, None, None, None, None, None) == -1
    rid = ctypes.c_uint64()
    assert lib.gsr_saved_render(None, ctypes.byref(rid), None, None, None) == -1
    assert lib.gsr_compose_scene(None, 1, None, None, 1, None, None) == -1
    s = g.StatusInfo()
    assert lib.gsr_query_status(None, ctypes.byref(s)) == -1
    assert lib.gsr_set_tile(None, 16, 16) == -1
    assert lib.gsr_set_stream_groups(None, 2) == -1
    ms = (ctypes.c_float * 10)()
    assert lib.gsr_stage_times(None, ms) == -1
    lib.gsr_destroy(None)  # no-op
    lib.gsr_scene_destroy(None)  # no-op
    assert lib.gsr_scene_gaussians(None, 0) == -1


def test_struct_layouts_match_the_header(tmp_path):
    """ctypes mirrors against sizeof/offsetof of the real header, compiled with gcc."""
    import paper_2507_21981_amd as g
    prog = tmp_path / "layout.c"
    prog.write_text("""
#include <stddef.h>
#include <stdio.h>
#include "gsr.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(gsr_gaussians), sizeof(gsr_gaussian_grads), sizeof(gsr_config),
         sizeof(gsr_status_info), sizeof(gsr_pose), sizeof(gsr_camera));
  printf("%zu %zu %zu %zu %zu\\n", offsetof(gsr_gaussians, sh), offsetof(gsr_config, persistent_grid),
         offsetof(gsr_status_info, visible), offsetof(gsr_status_info, evals), offsetof(gsr_config, stream_groups));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    l1, l2 = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")[:2]
    sizes, offs = [int(v) for v in l1.split()], [int(v) for v in l2.split()]
    assert sizes[:4] == [ctypes.sizeof(g.Gaussians), ctypes.sizeof(g.GaussianGrads), ctypes.sizeof(g.Config),
                         ctypes.sizeof(g.StatusInfo)]
    assert sizes[4] == 12 * 4 and sizes[5] == 20 * 4  # poses and cameras travel as float32 rows
    assert offs == [g.Gaussians.sh.offset, g.Config.persistent_grid.offset, g.StatusInfo.visible.offset,
                    g.StatusInfo.evals.offset, g.Config.stream_groups.offset]


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode == 2 and "one GPU" in r.stderr
