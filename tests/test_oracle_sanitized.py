"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
runs two LES steps (eddy viscosity, explicit terms, Crank-Nicolson,
divergence, SRJ solve, projection, diagnostics) on a small grid, in a child
process, without a sanitizer report; CPU only."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

CHILD = r"""
import numpy as np
import oracle
from oracle import schedule as osched
from paper_1511_07800_amd import inputs
nx, ny, nz, lx, ly, lz = 12, 8, 10, 2.0, 1.5, 2.0
nu, dpdx, dt = 1.0 / 180, -1.0, 1e-4
u, v, w = inputs.channel_state(nx, ny, nz, lz, nu, dpdx, noise=0.1, seed=3)
om = osched.srj_schedule(nx, ny, nz, lx, ly, lz)
P = oracle.make_params(nx, ny, nz, lx, ly, lz, nu=nu, dpdx=dpdx, dt=dt, les=1)
s = oracle.Solver(P, u, v, w, omega=om, rtol=1e-10, maxit=50)
for _ in range(2):
    st = s.step()
assert np.isfinite(s.p).all() and np.isfinite(s.u).all()
print("sanitized oracle ok", st["poisson_cycles"], flush=True)
"""


def _runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


def test_oracle_under_asan_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc has no AddressSanitizer runtime")
    lib = str(tmp_path / "libstp_oracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                           "-o", lib, os.path.join(ROOT, "oracle", "stp_oracle.c"), "-lm"])
    env = dict(os.environ, LD_PRELOAD=asan, STP_ORACLE_LIB=lib, PYTHONMALLOC="malloc", OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", CHILD], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    report = r.stdout + r.stderr
    assert r.returncode == 0, report[-4000:]
    assert "runtime error" not in report and "AddressSanitizer" not in report, report[-4000:]
    assert "sanitized oracle ok" in report
