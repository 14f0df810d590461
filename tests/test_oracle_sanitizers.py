"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only) runs the tiny case -- simulation, adjoint,
registration, the exact NCC gradient and the sinc PSF -- without a report,
in a child process with the sanitizer runtime preloaded."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROBE = r'''
import sys
sys.path.insert(0, %r)
import oracle
from paper_1611_07289_amd import synth
P = synth.tiny_problem()
ctx = oracle.Ctx(P.grid, P.stacks, P.patches)
y, Z, val = ctx.simulate(P.x_true, P.theta_true)
ctx.backproject(P.theta_true, y)
ctx.backproject(P.theta_true, y, support=True)
ctx.register(P.x_true, y, P.theta_true + 0.01, max_iter=3)
ctx.register(P.x_true, y, P.theta_true + 0.01, max_iter=3, gradient="analytic")
ctx.ncc_grad(P.x_true, y, P.theta_true + 0.01)
s = oracle.Ctx(P.grid, P.stacks, P.patches, psf="sinc")
s.simulate(P.x_true, P.theta_true)
s.backproject(P.theta_true, y)
print("clean")
''' % ROOT


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_runs_clean_under_asan_and_ubsan(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("libasan not available")
    lib = str(tmp_path / "libpvr_oracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-fopenmp",
                           "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE", "-o", lib,
                           os.path.join(ROOT, "oracle", "pvr_oracle.c"), "-lm"])
    env = dict(os.environ, PVR_ORACLE_LIB=lib, LD_PRELOAD=asan, OMP_NUM_THREADS="4",
               ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-c", PROBE], env=env, capture_output=True, text=True,
                       timeout=600, cwd=str(tmp_path))
    assert r.returncode == 0 and "clean" in r.stdout, r.stderr[-3000:]
