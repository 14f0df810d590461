"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/*.h, its struct layouts match the header, and invalid
descriptors are rejected on the host before any device call."""
import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

from paper_1611_07289_amd import pvr, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        txt = open(os.path.join(ROOT, "include", h)).read()
        names |= set(re.findall(r"^(?:pvr_status|const char|const float|void|int64_t|int32_t|size_t)[\s*]+"
                                r"(pvr_[a-z0-9_]+)\s*\(", txt, re.M))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = pvr.load()
    out = subprocess.run(["nm", "-D", "--defined-only", pvr.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (pvr_[a-z0-9_]+)", out))
    decl = _declared()
    assert decl, "no declarations found"
    missing = [d for d in decl if d not in exported]
    assert not missing, missing
    assert sorted(decl) == sorted(pvr.EXPORTS)
    for d in decl:
        assert hasattr(L, d)
    assert b"gfx950" in L.pvr_version()


def test_struct_layouts_match_header(tmp_path):
    src = tmp_path / "sz.cpp"
    src.write_text('#include "pvr.h"\n#include <stdio.h>\nint main(){printf("%zu %zu %zu %zu %zu %zu %zu",'
                   'sizeof(pvr_grid),sizeof(pvr_stack),sizeof(pvr_patch),sizeof(pvr_plan_sizes),'
                   'sizeof(pvr_em_state),sizeof(pvr_sr_params),sizeof(pvr_reg_params));}\n')
    exe = tmp_path / "sz"
    subprocess.run(["g++", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                    "-I", "/opt/rocm/include", str(src), "-o", str(exe)], check=True)
    sizes = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                            check=True).stdout.split()]
    mine = [ctypes.sizeof(c) for c in (pvr.Grid, pvr.Stack, pvr.Patch, pvr.PlanSizes,
                                       pvr.EMState, pvr.SRParams, pvr.RegParams)]
    assert sizes == mine


def _descs():
    P = synth.tiny_problem()
    return pvr.make_descriptors([P.grid], [P.stacks], [P.patches])


def _create(g, s, p, k=3.0):
    L = pvr.load()
    h = ctypes.c_void_p()
    st = L.pvr_plan_create(ctypes.addressof(g) if g is not None else None, len(g) if g else 0,
                           ctypes.addressof(s) if s is not None else None, len(s) if s else 0,
                           ctypes.addressof(p) if p is not None else None, len(p) if p else 0,
                           k, ctypes.byref(h))
    return st, h, L.pvr_last_error().decode()


def test_invalid_descriptors_rejected_on_host():
    g, s, p = _descs()
    st, h, msg = _create(None, s, p)
    assert st == 1 and "NULL" in msg and not h.value
    st, h, msg = _create(g, s, p, k=-1.0)
    assert st == 1 and "cutoff_k" in msg
    # a patch outside its slice
    bad = (pvr.Patch * len(p)).from_buffer_copy(bytes(p))
    bad[3].x0 = 30
    st, h, msg = _create(g, s, bad)
    assert st == 2 and "patch 3" in msg
    # a patch naming a stack that does not exist
    bad = (pvr.Patch * len(p)).from_buffer_copy(bytes(p))
    bad[0].stack = 9
    st, h, msg = _create(g, s, bad)
    assert st == 1 and "stack 9" in msg
    # non-orthogonal stack axes
    sb = (pvr.Stack * len(s)).from_buffer_copy(bytes(s))
    sb[1].pix2world[1] = 0.3
    st, h, msg = _create(g, sb, p)
    assert st == 2 and "orthogonal" in msg
    # singular grid
    gb = (pvr.Grid * 1).from_buffer_copy(bytes(g))
    gb[0].vox2world[0] = 0.0
    st, h, msg = _create(gb, s, p)
    assert st == 2 and "singular" in msg
    # zero FWHM
    sb = (pvr.Stack * len(s)).from_buffer_copy(bytes(s))
    sb[0].fwhm_mm[2] = 0.0
    st, h, msg = _create(g, sb, p)
    assert st == 1 and "fwhm" in msg


def test_destroy_null_is_noop_and_null_plan_calls_fail():
    L = pvr.load()
    L.pvr_plan_destroy(None)
    assert L.pvr_plan_info(None, None) == 1
    assert L.pvr_simulate(None, None, None, None, None, None) == 1
    assert L.pvr_backproject(None, None, None, None, None, None, None) == 1
    assert L.pvr_sr_update(None, None, None, None, None, None, None) == 1
    assert L.pvr_register_patches(None, None, None, None, None, None, None, None) == 1
    assert L.pvr_robust_weights(None, None, None, None, None, None, None, 0, None) == 1
    assert L.pvr_check(None, None) == 1
    out = ctypes.c_void_p()
    assert L.pvr_sr_graph_create(None, None, None, None, None, None, None, None, None, None,
                                 None, None, 2, None, ctypes.byref(out)) == 1 and not out.value
    assert L.pvr_sr_graph_create(None, None, None, None, None, None, None, None, None, None,
                                 None, None, 2, None, None) == 1
    assert L.pvr_sr_graph_launch(None, None) == 1
    L.pvr_sr_graph_destroy(None)
    assert "NULL" in L.pvr_last_error().decode()


@pytest.mark.parametrize("env,expect", [(None, 0), ("0", 0), ("", 0), ("1", 1), ("yes", 1)])
def test_debug_mode_starts_from_the_environment(env, expect):
    """PVR_DEBUG decides the initial debug mode (read on first use, in a fresh
    process); pvr_set_debug switches it afterwards.  No device call."""
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1611_07289_amd import pvr\n"
            "a = pvr.get_debug(); pvr.set_debug(not a); b = pvr.get_debug()\n"
            "print(int(a), int(b))\n") % ROOT
    envd = {k: v for k, v in os.environ.items() if k != "PVR_DEBUG"}
    if env is not None:
        envd["PVR_DEBUG"] = env
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=envd,
                         check=True, timeout=120).stdout.split()
    assert out == [str(expect), str(1 - expect)]
