"""Host-side checks of the C ABI: the library loads, exports every entry
point include/stp.h declares, and the configuration arithmetic behaves (no
device work is issued here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_\s\*]*?\b(stp_[a-z_0-9]+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("stp_init", "stp_step", "stp_poisson_solve", "stp_fields", "stp_destroy", "stp_last_error",
                 "stp_workspace_bytes"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1511_07800_amd import load_library
    lib = load_library()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def cfg(**kw):
    from paper_1511_07800_amd import Config
    c = Config()
    c.nx, c.ny, c.nz, c.les = 32, 16, 16, 0
    c.lx, c.ly, c.lz = 6.28, 3.14, 2.0
    c.nu, c.dpdx, c.dt, c.cs, c.vd_a = 0.01, -0.02, 1e-3, 0.1, 25.0
    c.precision, c.warm_start = 0, 0
    c.poisson_rtol, c.poisson_maxit = 1e-10, 100
    c.srj_m, c.srj_omega = 0, None
    c.srj_reduction, c.mixed_inner, c.tblock, c.cn_tol = 1e-3, 1, 1, 1e-13
    c.stream = None
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def test_workspace_bytes_valid_and_invalid():
    from paper_1511_07800_amd import load_library
    lib = load_library()
    n_ok = lib.stp_workspace_bytes(ctypes.byref(cfg()))
    n = 32 * 16 * 16
    assert n_ok >= 25 * 8 * n      # every FP64 work array of the step fits
    assert n_ok % 256 == 0 or n_ok > 0
    big = lib.stp_workspace_bytes(ctypes.byref(cfg(nx=64)))
    assert big > n_ok
    # the extrapolated warm start keeps p^{n-1} (order 1) and p^{n-2} (order 2)
    for order in (1, 2):
        assert lib.stp_workspace_bytes(ctypes.byref(cfg(extrap_order=order))) == n_ok + order * 8 * n
    # the FP16 right-hand side of the mixed passes: nx*ny*nz halves
    mixed = lib.stp_workspace_bytes(ctypes.byref(cfg(precision=1)))
    assert lib.stp_workspace_bytes(ctypes.byref(cfg(precision=1, mixed_rhs16=1))) == mixed + 2 * n
    # FP32 stencils: nu_T and the nine Adams-Bashforth arrays in FP32 instead of
    # FP64, plus FP32 copies of u, v, w and the nz plane means of u (one
    # 256-byte aligned block here)
    nw = 32 * 16 * 17
    assert lib.stp_workspace_bytes(ctypes.byref(cfg(precision=1, stencils32=1))) == mixed - 24 * n - 8 * nw + 256
    # the least-squares guess keeps proj_depth solutions and their right-hand sides
    for depth in (1, 8):
        assert lib.stp_workspace_bytes(ctypes.byref(cfg(proj_depth=depth))) == n_ok + 2 * depth * 8 * n
    for bad in (dict(nz=1), dict(nx=0), dict(nu=0.0), dict(dt=-1.0), dict(lx=float("nan")),
                dict(precision=7), dict(poisson_maxit=0), dict(poisson_rtol=-1.0), dict(srj_reduction=1.5),
                dict(les=2), dict(tblock=-1), dict(tblock=6), dict(cn_tol=2.0), dict(srj_m=4),
                dict(extrap_order=3), dict(extrap_order=1, warm_start=1), dict(proj_depth=-1),
                dict(proj_depth=9), dict(proj_depth=2, warm_start=1), dict(mixed_rhs16=1),
                dict(precision=1, mixed_rhs16=2), dict(stencils32=1), dict(precision=1, stencils32=2)):
        assert lib.stp_workspace_bytes(ctypes.byref(cfg(**bad))) == 0, bad
    assert lib.stp_workspace_bytes(None) == 0


def test_fields_rejects_null_context():
    from paper_1511_07800_amd import load_library, STP_EINVAL
    lib = load_library()
    ptr = ctypes.c_void_p()
    shape, strides = (ctypes.c_int64 * 3)(), (ctypes.c_int64 * 3)()
    off, dt = (ctypes.c_double * 3)(), ctypes.c_int32()
    assert lib.stp_fields(None, 0, ctypes.byref(ptr), shape, strides, ctypes.byref(dt), off) == STP_EINVAL


def test_init_rejects_small_workspace_and_null():
    from paper_1511_07800_amd import load_library, STP_EINVAL, STP_ENOMEM
    lib = load_library()
    h = ctypes.c_void_p()
    c = cfg()
    assert lib.stp_init(None, None, 0, ctypes.byref(h)) == STP_EINVAL
    assert lib.stp_init(ctypes.byref(c), None, 0, ctypes.byref(h)) == STP_ENOMEM
    assert lib.stp_init(ctypes.byref(cfg(nz=1)), None, 0, ctypes.byref(h)) == STP_EINVAL
    assert lib.stp_destroy(None) == 0


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    import paper_1511_07800_amd.binding as b
    monkeypatch.setattr(b, "_lib", None)
    monkeypatch.setattr(b, "_LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(ImportError):
        b.load_library()


def test_ctypes_structs_match_the_c_layout(tmp_path):
    """The binding's ctypes structures have the sizes and field offsets a C
    compiler gives the structs of include/stp.h."""
    import shutil
    import subprocess
    from paper_1511_07800_amd import Config
    from paper_1511_07800_amd.binding import SolveStats, StepStats, State
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"stp_config": Config, "stp_solve_stats": SolveStats, "stp_step_stats": StepStats, "stp_state": State}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "stp.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_noalloc_entry_point_rejects_on_the_host():
    """stp_residual_norm_noalloc checks its arguments before it touches the
    device: null pointers, a bad grid and a plane too large for the static
    scratch's partials are STP_EINVAL with a message for stp_last_error(NULL)."""
    from paper_1511_07800_amd import load_library, STP_EINVAL
    lib = load_library()
    fake = ctypes.c_void_p(256)  # never dereferenced: every call below is rejected first
    assert lib.stp_residual_norm_noalloc(8, 8, 4, 1.0, 1.0, 1.0, None, fake, fake, None) == STP_EINVAL
    assert b"null" in lib.stp_last_error(None)
    assert lib.stp_residual_norm_noalloc(8, 8, 1, 1.0, 1.0, 1.0, fake, fake, fake, None) == STP_EINVAL
    assert lib.stp_residual_norm_noalloc(8, 8, 4, 1.0, -1.0, 1.0, fake, fake, fake, None) == STP_EINVAL
    # 512 x 4096 column tiles of 64 x 4 cells: more partials than the scratch holds
    assert lib.stp_residual_norm_noalloc(32768, 16384, 2, 1.0, 1.0, 1.0, fake, fake, fake, None) == STP_EINVAL
    assert b"too large" in lib.stp_last_error(None)
    # the same plane limit guards every context's reduction partials
    assert lib.stp_workspace_bytes(ctypes.byref(cfg(nx=32768, ny=16384, nz=2))) == 0
