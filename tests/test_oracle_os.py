"""Pins of the Orr-Sommerfeld solver used to judge the Tollmien-Schlichting test.

Pinned to values the paper prints (Sec. 4.1, Sec. 4.2 table) and to Orszag's
eigenvalue that the paper cites as its own validation source."""
import math

import numpy as np
import pytest

from oracle import os_solver
from _golden import load


def test_paper_eigenvalue_re500():
    pins = load("paper_pins.txt")
    lam = os_solver.growth_rate_paper(2 * math.pi / 4, 500.0, n=80)
    assert abs(lam.real - pins["os_lambda_real"][0]) < pins["os_lambda_real"][1]
    assert abs(lam.imag - pins["os_lambda_imag"][0]) < pins["os_lambda_imag"][1]
    period = 2 * math.pi / abs(lam.imag)
    assert abs(period - pins["os_period"][0]) < pins["os_period"][1]


def test_resolution_converged():
    a = os_solver.growth_rate_paper(math.pi / 2, 500.0, n=60)
    b = os_solver.growth_rate_paper(math.pi / 2, 500.0, n=100)
    assert abs(a - b) < 1e-5


def test_orszag_eigenvalue():
    pins = load("orszag_1971.txt")
    u, upp = os_solver.poiseuille_centreline(2.0)
    _, c, _, _ = os_solver.least_stable(1.0, 10000.0, u, upp, 0.0, 2.0, n=100)
    assert abs(c.real - pins["c_real"][0]) < pins["c_real"][1]
    assert abs(c.imag - pins["c_imag"][0]) < pins["c_imag"][1]


def test_critical_reynolds():
    pins = load("paper_pins.txt")
    rec, alpha = os_solver.critical_reynolds_paper(n=60)
    assert abs(rec - pins["re_critical"][0]) < pins["re_critical"][1]
    # the same point in half-height / centreline scaling: Re_cl = Re_*^2 / 8
    assert abs(rec**2 / 8 - 5772.2) < 1.0


def test_scalings_agree():
    """The paper's scaling and the centreline scaling describe the same mode:
    lambda_cl = 2 lambda_paper / Re_*, alpha_half = alpha_paper / 2."""
    re_p = 500.0
    lam_p = os_solver.growth_rate_paper(math.pi / 2, re_p, n=80)
    u, upp = os_solver.poiseuille_centreline(2.0)
    lam_c, _, _, _ = os_solver.least_stable(math.pi / 4, re_p**2 / 8, u, upp, 0.0, 2.0, n=80)
    assert abs(lam_c - 2 * lam_p / re_p) < 1e-7


def test_subcritical_decays():
    lam = os_solver.growth_rate_paper(2.04, 150.0, n=60)
    assert lam.real < 0
    lam = os_solver.growth_rate_paper(2.04, 300.0, n=60)
    assert lam.real > 0
