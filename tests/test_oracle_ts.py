"""Linear Tollmien-Schlichting growth in the FP64 oracle against the
Orr-Sommerfeld eigenvalue (Sec. 4.2), centreline Re = 7500, alpha = 1.

At 128 cells across the channel the wall layer (alpha Re)^(-1/3) ~ 0.05 spans
about three cells and the growth rate (a small difference of production and
dissipation) carries a ~10% discretisation error; the frequency is within 1%.
The GPU tests refine the grid and show the error shrinking to within 5%."""
import math

import numpy as np
import pytest

import oracle
from _ts import ts_initial_state, mode_amplitude, fit_growth


@pytest.mark.slow
def test_oracle_ts_growth_rate():
    nx, ny, nz, lx, ly, lz = 32, 1, 128, 2 * math.pi, 0.5, 2.0
    re, alpha, dt, t_end = 7500.0, 1.0, 0.01, 20.0
    u, v, w, lam, g = ts_initial_state(nx, ny, nz, lx, lz, re, alpha, 1e-5)
    P = oracle.make_params(nx, ny, nz, lx, ly, lz, nu=1 / re, dpdx=g, dt=dt)
    s = oracle.Solver(P, u, v, w, rtol=1e-11, maxit=100)
    ts, amps = [], []
    for n in range(int(round(t_end / dt))):
        st = s.step()
        assert st["status"] == 0
        ts.append((n + 1) * dt)
        amps.append(mode_amplitude(s.w, nx, lx, alpha))
    growth, freq = fit_growth(ts, amps, 5.0)
    print(f"oracle TS: growth {growth:.6f} (OS {lam.real:.6f}), freq {freq:.6f} (OS {lam.imag:.6f})")
    assert lam.real > 0                      # supercritical
    assert abs(growth - lam.real) <= 0.12 * lam.real
    assert abs(freq - lam.imag) <= 0.01 * abs(lam.imag)
