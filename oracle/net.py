"""FP64 oracle of the learned warm-start network (test infrastructure only).

Not part of the paper: the network predicts the pressure increment of a time
step from the Poisson right-hand side and the previous pressure, so the
relaxation of Sec. 3.4 can start from a better guess; the relaxation still
runs to the same residual, so the network never changes the answer, only the
starting point.  Everything here is plain numpy in float64 with hand-written
backpropagation; an optional mode rounds inputs, weights, stored activations
and back-propagated gradients to bfloat16 at the points where the GPU kernels
store bfloat16.

Tensors are channels-last, shape (nz, ny, nx, C).  A convolution is the 3x3x3
cross-correlation
    out[z, y, x, co] = bias[co] + sum_{tap, ci} in[z+dz, y+dy, x+dx, ci] W[tap, co, ci],
tap = 9 (dz+1) + 3 (dy+1) + (dx+1), periodic in x and y, zero outside the
walls in z.  Architecture (3 levels, 16/32/64 channels):
    e1 = relu(conv1(x))                       x: 2 channels, full grid
    e2 = relu(conv2(pool(e1)))                1/2 grid
    e3 = relu(conv3(pool(e2)))                1/4 grid
    d2 = relu(conv4(concat(up(e3), e2)))      1/2 grid, 64 + 32 -> 32
    d1 = relu(conv5(concat(up(d2), e1)))      full grid, 32 + 16 -> 16
    y  = conv6(d1)                            1 channel, linear
pool: mean of 2x2x2 blocks; up: nearest-neighbour copy to 2x2x2 blocks.

Inputs and scaling (from b and p_prev only).  The exact increment is
p_next - p_prev = L^-1 (b - L p_prev), a linear map of the residual
r = b - L p_prev, so the network sees that residual, computed in FP64:
    s_r = rms(r / D) (1 if that is 0),  s_p = rms(p_prev - mean(p_prev)) (1 if 0),
    x = [r / (D s_r), (p_prev - mean(p_prev)) / s_p],
    prediction p_guess = p_prev + s_r y,  training target t = (p_next - p_prev) / s_r,
    loss = mean over cells of (y - t)^2.
"""
import numpy as np

LAYERS = [("conv1", 2, 16), ("conv2", 16, 32), ("conv3", 32, 64), ("conv4", 96, 32), ("conv5", 48, 16),
          ("conv6", 16, 1)]


def bf16(a):
    """Round float64/float32 values to bfloat16 (round to nearest even) and
    return them as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isfinite(f), out, f.astype(np.float64))


def shift(a, dz, dy, dx):
    """s[z, y, x] = a[z+dz, y+dy, x+dx]: periodic in y, x; zero beyond the walls."""
    s = np.roll(a, shift=(-dy, -dx), axis=(1, 2))
    out = np.zeros_like(s)
    nz = a.shape[0]
    if dz == 0:
        out[:] = s
    elif dz > 0:
        out[: nz - dz] = s[dz:]
    else:
        out[-dz:] = s[: nz + dz]
    return out


TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def conv_fwd(x, w, b):
    """x (nz, ny, nx, ci), w (27, co, ci), b (co,)."""
    out = np.zeros(x.shape[:3] + (w.shape[1],))
    for t, (dz, dy, dx) in enumerate(TAPS):
        out += shift(x, dz, dy, dx) @ w[t].T
    return out + b


def conv_bwd(x, w, dout):
    """Gradients of conv_fwd: (dx, dw, db)."""
    dx = np.zeros_like(x)
    dw = np.zeros_like(w)
    for t, (dz, dy, dxx) in enumerate(TAPS):
        sx = shift(x, dz, dy, dxx)
        dw[t] = np.einsum("zyxo,zyxi->oi", dout, sx)
        # adjoint of the shift: out[z] depends on x[z + dz]
        dx += shift(dout @ w[t], -dz, -dy, -dxx)
    db = dout.sum(axis=(0, 1, 2))
    return dx, dw, db


def pool(a):
    nz, ny, nx, c = a.shape
    return a.reshape(nz // 2, 2, ny // 2, 2, nx // 2, 2, c).mean(axis=(1, 3, 5))


def pool_bwd(d):
    return up(d) / 8.0


def up(a):
    return a.repeat(2, axis=0).repeat(2, axis=1).repeat(2, axis=2)


def up_bwd(d):
    nz, ny, nx, c = d.shape
    return d.reshape(nz // 2, 2, ny // 2, 2, nx // 2, 2, c).sum(axis=(1, 3, 5))


def init_params(seed=0):
    """He-style uniform initialisation, zero biases (FP64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    params = {}
    for name, ci, co in LAYERS:
        lim = np.sqrt(6.0 / (27 * ci))
        params[name + ".w"] = rng.uniform(-lim, lim, (27, co, ci))
        params[name + ".b"] = np.zeros(co)
    return params


def normalise(b, p_prev, lap_p_prev, D):
    """Inputs (nz, ny, nx) float64; lap_p_prev = L p_prev.  Returns (x, s_r)."""
    rd = (b - lap_p_prev) / D
    s_r = np.sqrt(np.mean(rd * rd))
    if s_r == 0.0:
        s_r = 1.0
    dp = p_prev - p_prev.mean()
    s_p = np.sqrt(np.mean(dp * dp))
    if s_p == 0.0:
        s_p = 1.0
    x = np.stack([rd / s_r, dp / s_p], axis=-1)
    return x, s_r


def forward(params, x, round_bf16=False):
    """Returns y (nz, ny, nx) and the cache needed by backward."""
    R = bf16 if round_bf16 else (lambda a: a)
    P = {k: (R(v) if k.endswith(".w") else v) for k, v in params.items()}
    c = {"x": R(x)}
    c["e1"] = R(np.maximum(conv_fwd(c["x"], P["conv1.w"], P["conv1.b"]), 0.0))
    c["q1"] = R(pool(c["e1"]))
    c["e2"] = R(np.maximum(conv_fwd(c["q1"], P["conv2.w"], P["conv2.b"]), 0.0))
    c["q2"] = R(pool(c["e2"]))
    c["e3"] = R(np.maximum(conv_fwd(c["q2"], P["conv3.w"], P["conv3.b"]), 0.0))
    c["c2"] = np.concatenate([up(c["e3"]), c["e2"]], axis=-1)
    c["d2"] = R(np.maximum(conv_fwd(c["c2"], P["conv4.w"], P["conv4.b"]), 0.0))
    c["c1"] = np.concatenate([up(c["d2"]), c["e1"]], axis=-1)
    c["d1"] = R(np.maximum(conv_fwd(c["c1"], P["conv5.w"], P["conv5.b"]), 0.0))
    y = conv_fwd(c["d1"], P["conv6.w"], P["conv6.b"])[..., 0]
    c["P"] = P
    return y, c


def loss_and_grads(params, x, target, round_bf16=False):
    """MSE loss of the prediction against target and d loss / d params."""
    R = bf16 if round_bf16 else (lambda a: a)
    y, c = forward(params, x, round_bf16)
    P = c["P"]
    n = y.size
    loss = np.mean((y - target) ** 2)
    g = {}
    # gradients are rounded where the GPU stores them as bfloat16: the dOut
    # operand of every convolution, after the ReLU mask and the adjoints of
    # pooling, upsampling and concatenation are applied
    dy = R((2.0 / n) * (y - target))[..., None]
    dd1, g["conv6.w"], g["conv6.b"] = conv_bwd(c["d1"], P["conv6.w"], dy)
    dd1 = R(dd1 * (c["d1"] > 0))
    dc1, g["conv5.w"], g["conv5.b"] = conv_bwd(c["c1"], P["conv5.w"], dd1)
    dd2 = R(up_bwd(dc1[..., :32]) * (c["d2"] > 0))
    dc2, g["conv4.w"], g["conv4.b"] = conv_bwd(c["c2"], P["conv4.w"], dd2)
    de3 = R(up_bwd(dc2[..., :64]) * (c["e3"] > 0))
    dq2, g["conv3.w"], g["conv3.b"] = conv_bwd(c["q2"], P["conv3.w"], de3)
    de2 = R((dc2[..., 64:] + pool_bwd(dq2)) * (c["e2"] > 0))
    dq1, g["conv2.w"], g["conv2.b"] = conv_bwd(c["q1"], P["conv2.w"], de2)
    de1 = R((dc1[..., 32:] + pool_bwd(dq1)) * (c["e1"] > 0))
    _, g["conv1.w"], g["conv1.b"] = conv_bwd(c["x"], P["conv1.w"], de1)
    return loss, g, y


def adam_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba) with bias correction; state holds m, v, t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    out = {}
    for k, p in params.items():
        m = state.setdefault("m." + k, np.zeros_like(p))
        v = state.setdefault("v." + k, np.zeros_like(p))
        m[...] = beta1 * m + (1 - beta1) * grads[k]
        v[...] = beta2 * v + (1 - beta2) * grads[k] ** 2
        mh = m / (1 - beta1**t)
        vh = v / (1 - beta2**t)
        out[k] = p - lr * mh / (np.sqrt(vh) + eps)
    return out


def predict(params, b, p_prev, lap_p_prev, D, round_bf16=False):
    x, s_r = normalise(b, p_prev, lap_p_prev, D)
    y, _ = forward(params, x, round_bf16)
    return p_prev + s_r * y
