"""Pins of the learned warm-start network oracle (oracle/net.py): one layer
against an independent correlation routine, pooling/upsampling adjoints, and
every parameter gradient against central finite differences."""
import numpy as np
import pytest
import scipy.signal

from oracle import net


def test_single_conv_matches_scipy_correlate():
    """The 3x3x3 layer is a cross-correlation, periodic in y and x and zero
    beyond the walls in z, computed here with scipy on an explicitly padded
    array."""
    r = np.random.Generator(np.random.PCG64(1))
    x = r.standard_normal((6, 5, 7, 3))
    w = r.standard_normal((27, 4, 3))
    b = r.standard_normal(4)
    got = net.conv_fwd(x, w, b)
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)), mode="wrap")
    xp = np.pad(xp, ((1, 1), (0, 0), (0, 0), (0, 0)), mode="constant")
    ref = np.zeros_like(got)
    for co in range(4):
        acc = np.zeros(x.shape[:3])
        for ci in range(3):
            k = w[:, co, ci].reshape(3, 3, 3)  # tap = 9(dz+1) + 3(dy+1) + (dx+1)
            acc += scipy.signal.correlate(xp[..., ci], k, mode="valid")
        ref[..., co] = acc + b[co]
    np.testing.assert_allclose(got, ref, atol=1e-12)


def test_pool_up_adjoints():
    r = np.random.Generator(np.random.PCG64(2))
    a = r.standard_normal((4, 6, 8, 3))
    d = r.standard_normal((2, 3, 4, 3))
    # <pool(a), d> = <a, pool_bwd(d)>,  <up(d), a> = <d, up_bwd(a)>
    assert np.vdot(net.pool(a), d) == pytest.approx(np.vdot(a, net.pool_bwd(d)), rel=1e-12)
    assert np.vdot(net.up(d), a) == pytest.approx(np.vdot(d, net.up_bwd(a)), rel=1e-12)
    np.testing.assert_allclose(net.pool(net.up(d)), d, atol=1e-15)


def test_bf16_rounding():
    vals = np.array([1.0, 1.00390625, 1.005859375, -3.14159, 0.0, 1e-30])
    got = net.bf16(vals)
    # 1.00390625 = 1 + 2^-8 lies halfway between bf16 neighbours 1 and 1 + 2^-7: ties to even -> 1
    assert got[0] == 1.0 and got[1] == 1.0 and got[2] == 1.0078125
    assert abs(got[3] - (-3.140625)) < 1e-12
    assert got[4] == 0.0


def test_gradients_match_finite_differences():
    r = np.random.Generator(np.random.PCG64(3))
    nz, ny, nx = 8, 8, 8
    x = r.standard_normal((nz, ny, nx, 2))
    t = r.standard_normal((nz, ny, nx))
    params = net.init_params(seed=4)
    for k in params:
        if k.endswith(".b"):
            params[k] = 0.05 * r.standard_normal(params[k].shape)
    loss, g, _ = net.loss_and_grads(params, x, t)
    h = 1e-6
    for k in params:
        flat = params[k].ravel()
        idx = r.choice(flat.size, size=min(6, flat.size), replace=False)
        for i in idx:
            p1 = {kk: vv.copy() for kk, vv in params.items()}
            p2 = {kk: vv.copy() for kk, vv in params.items()}
            p1[k].ravel()[i] += h
            p2[k].ravel()[i] -= h
            l1, _, _ = net.loss_and_grads(p1, x, t)
            l2, _, _ = net.loss_and_grads(p2, x, t)
            fd = (l1 - l2) / (2 * h)
            an = g[k].ravel()[i]
            assert abs(fd - an) <= 1e-7 * max(1.0, abs(fd)) + 1e-9, (k, i, fd, an)


def test_adam_first_step_is_sign_times_lr():
    """With bias correction the first Adam step moves every parameter by
    lr * g / (|g| + eps) (Kingma and Ba)."""
    params = {"a.w": np.array([1.0, -2.0, 3.0])}
    grads = {"a.w": np.array([0.5, -0.25, 0.0])}
    out = net.adam_step(params, grads, {}, lr=1e-3)
    np.testing.assert_allclose(out["a.w"], [1.0 - 1e-3 * 0.5 / (0.5 + 1e-8), -2.0 + 1e-3 * 0.25 / (0.25 + 1e-8), 3.0])


def test_normalisation_and_prediction_identity():
    """A zero network (all weights and biases zero) predicts p_prev exactly;
    the residual channel has unit rms."""
    r = np.random.Generator(np.random.PCG64(5))
    b = r.standard_normal((8, 8, 8))
    p = r.standard_normal((8, 8, 8))
    lap = r.standard_normal((8, 8, 8))
    params = {k: np.zeros_like(v) for k, v in net.init_params().items()}
    np.testing.assert_array_equal(net.predict(params, b, p, lap, 3.0), p)
    x, s_r = net.normalise(b, p, lap, 3.0)
    assert abs(np.sqrt(np.mean(x[..., 0] ** 2)) - 1.0) < 1e-12
    assert abs(np.sqrt(np.mean(x[..., 1] ** 2)) - 1.0) < 1e-12
    np.testing.assert_allclose(x[..., 0] * s_r * 3.0, b - lap, atol=1e-12)
