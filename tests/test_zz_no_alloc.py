"""The allocation-free residual norm (stp_residual_norm_noalloc) against the
context's stp_residual_norm, through the C ABI: two calls in a row on one GPU,
the second on a smaller grid (the shared static scratch keeps the first
call's partials, which the second must not read), plus the host-side
rejections."""
import math

import numpy as np
import pytest

from paper_1511_07800_amd import inputs

pytestmark = pytest.mark.gpu


def test_noalloc_residual_norm_matches_context_entry_point(gpu):
    import torch
    from paper_1511_07800_amd import Channel, StpError, STP_EINVAL, residual_norm_noalloc
    grids = [(200, 96, 48, 4.0, 2.0, 2.0), (40, 24, 13, 2.0, 1.2, 1.0)]
    for n, g in enumerate(grids):
        nx, ny, nz, lx, ly, lz = g
        print(f"noalloc call {n + 1}: grid {g[:3]}", flush=True)
        r = inputs.rng(70 + n)
        b = torch.from_numpy(inputs.poisson_rhs(nx, ny, nz, seed=71 + n)).cuda()
        p = torch.from_numpy(r.standard_normal((nz, ny, nx))).cuda()
        out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        residual_norm_noalloc(nx, ny, nz, lx, ly, lz, b, p, out)
        torch.cuda.synchronize()
        ch = Channel(nx, ny, nz, lx, ly, lz, nu=1.0, dpdx=0.0, dt=1.0)
        ref = ch.residual_norm(b, p)
        ch.close()
        got = float(out.item())
        print(f"  noalloc {got:.17e} context {ref:.17e}", flush=True)
        # same kernels and launch shape: the same value, bit for bit
        assert got == ref and math.isfinite(got)
    # rejections happen on the host, before any launch
    b = torch.zeros(8 * 8 * 4, dtype=torch.float64, device="cuda")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(StpError) as e:
        residual_norm_noalloc(8, 8, 1, 1.0, 1.0, 1.0, b[:64], b[:64], out)
    assert e.value.status == STP_EINVAL
