"""Learned depth / rigidness proposal: a small convolutional encoder-decoder over the flow
stack of a window, FP64 (test infrastructure).

The project's extension of the method (its initial depth is random in the paper, sec. III-A):
a network maps the N flows to an initial inverse depth and initial rigidness maps, and GEM
starts from them.  Plain GEM stays the fallback and the reference for the proposal's error.

Architecture (3x3 convolutions, zero padding 1, NHWC; channel counts as stored, the real
ones in brackets):
  c1  16 [2N]  -> 64   stride 1            ReLU          a1   H x W
  c2  64       -> 128  stride 2            ReLU          a2   ceil(H/2) x ceil(W/2)
  c3  128      -> 128  stride 1            ReLU          a3
  c4  128      -> 128  stride 1            ReLU          a4
  c5  128      -> 64   on 2x nearest upsampling of a4, + a1 before the ReLU    a5   H x W
  c6  64       -> 32 [1 + N]  stride 1     linear        o    H x W
Input features: channel 2(t-1) + c = X_t[c] / FLOW_SCALE (non-finite -> 0), padding zero.
Heads: s = softplus(o_0) is the inverse depth times |t_1| (the translation length of frame 1's
initial pose; flows fix depth only up to that scale), rho_init = clip(s / |t_1|, rho_min,
rho_max); q_init,t = sigmoid(o_t), t = 1..N.

Precision as the network is specified: weights and activations in BF16, products summed in
FP32.  This oracle sums in FP64; `bf16` rounds a value to BF16 (round to nearest even) where
a test wants the stored precision.
"""
import numpy as np

FLOW_SCALE = 16.0
C_IN = 16
C_HEAD = 32
# name, c_in, c_out, stride, upsample input, skip source, relu
LAYERS = [
    ("c1", C_IN, 64, 1, False, None, True),
    ("c2", 64, 128, 2, False, None, True),
    ("c3", 128, 128, 1, False, None, True),
    ("c4", 128, 128, 1, False, None, True),
    ("c5", 128, 64, 1, True, "c1", True),
    ("c6", 64, C_HEAD, 1, False, None, False),
]


def bf16(x):
    """Round to the nearest BF16 value (ties to even), returned as float64.  BF16 keeps the
    top 16 bits of an IEEE single: round the float32 bit pattern at bit 16."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


def init_params(seed, n_frames):
    """He-normal weights [c_out][3][3][c_in] on the real channels (padding channels 0), zero
    biases; FP64."""
    rng = np.random.default_rng(seed)
    params = {}
    real_in = {"c1": 2 * n_frames}
    real_out = {"c6": 1 + n_frames}
    for name, ci, co, _, _, _, _ in LAYERS:
        ri, ro = real_in.get(name, ci), real_out.get(name, co)
        w = np.zeros((co, 3, 3, ci))
        w[:ro, :, :, :ri] = rng.normal(scale=np.sqrt(2.0 / (9 * ri)), size=(ro, 3, 3, ri))
        params[name + ".w"] = w
        params[name + ".b"] = np.zeros(co)
    return params


def features(flow):
    """Flow stack [N][H][W][2] -> input features [H][W][16]."""
    N, H, W, _ = flow.shape
    x = np.zeros((H, W, C_IN))
    for t in range(N):
        f = np.asarray(flow[t], dtype=np.float64) / FLOW_SCALE
        x[:, :, 2 * t:2 * t + 2] = np.where(np.isfinite(f), f, 0.0)
    return x


def upsample2(x):
    return x.repeat(2, axis=0).repeat(2, axis=1)


def out_size(n, stride):
    return (n - 1) // stride + 1


def conv3x3(x, w, b, stride=1, up=False):
    """y[oy][ox][co] = b[co] + sum_{ky,kx,ci} w[co][ky][kx][ci] * x'[s oy + ky - 1][s ox + kx - 1][ci]
    with x' = x (or its 2x nearest upsampling) and zeros outside."""
    if up:
        x = upsample2(x)
    H, W, _ = x.shape
    Ho, Wo = out_size(H, stride), out_size(W, stride)
    xp = np.pad(x, ((1, 1), (1, 1), (0, 0)))
    y = np.broadcast_to(b, (Ho, Wo, len(b))).astype(np.float64).copy()
    for ky in range(3):
        for kx in range(3):
            patch = xp[ky:ky + stride * (Ho - 1) + 1:stride, kx:kx + stride * (Wo - 1) + 1:stride, :]
            y += patch @ w[:, ky, kx, :].T
    return y


def conv3x3_backward(x, w, dy, stride=1, up=False):
    """Gradients (dx, dw, db) of conv3x3 for upstream gradient dy; dx has x's shape (the
    upsampling's gradient sums each 2x2 block)."""
    xu = upsample2(x) if up else x
    H, W, _ = xu.shape
    Ho, Wo, _ = dy.shape
    xp = np.pad(xu, ((1, 1), (1, 1), (0, 0)))
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for ky in range(3):
        for kx in range(3):
            sl = (slice(ky, ky + stride * (Ho - 1) + 1, stride), slice(kx, kx + stride * (Wo - 1) + 1, stride))
            dw[:, ky, kx, :] = np.einsum("hwo,hwi->oi", dy, xp[sl])
            dxp[sl] += dy @ w[:, ky, kx, :]
    dx = dxp[1:-1, 1:-1]
    if up:
        dx = dx.reshape(H // 2, 2, W // 2, 2, -1).sum(axis=(1, 3))
    return dx, dw, dy.sum(axis=(0, 1))


def forward(params, x, round_bf16=False):
    """Activations of every layer (post-activation; 'o' = c6's linear output)."""
    rnd = bf16 if round_bf16 else (lambda a: a)
    acts = {"x": rnd(x)}
    src = acts["x"]
    for name, _, _, stride, up, skip, relu in LAYERS:
        y = conv3x3(src, rnd(params[name + ".w"]), params[name + ".b"], stride, up)   # biases stay FP32
        if skip is not None:
            y = y + acts["a" + skip[1:]]
        if relu:
            y = np.maximum(y, 0.0)
        key = "o" if name == "c6" else "a" + name[1:]
        acts[key] = y if key == "o" else rnd(y)
        src = acts[key]
    return acts


def softplus(z):
    return np.logaddexp(0.0, z)


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def heads(o, n_frames, tnorm, rho_min, rho_max):
    """(rho_init [H][W], q_init [N][H][W]) from the linear output o [H][W][32]."""
    rho = np.clip(softplus(o[..., 0]) / tnorm, rho_min, rho_max)
    q = np.moveaxis(sigmoid(o[..., 1:1 + n_frames]), -1, 0)
    return rho, q


def loss(o, rho_t, q_t, tnorm, mask, lam):
    """L = mean_{mask} |softplus(o_0) - rho_t |t_1|| + lam * mean_{px,t} BCE(sigmoid(o_t), q_t)
    and dL/do.  Targets rho_t [H][W], q_t [N][H][W]; mask [H][W] of pixels with a depth
    target."""
    N = q_t.shape[0]
    s = softplus(o[..., 0])
    d = s - rho_t * tnorm
    m = mask.astype(np.float64)
    cnt = max(m.sum(), 1.0)
    L_rho = float((np.abs(d) * m).sum() / cnt)
    z = np.moveaxis(o[..., 1:1 + N], -1, 0)
    # BCE with logits: softplus(z) - q z
    L_q = float((softplus(z) - q_t * z).mean())
    do = np.zeros_like(o)
    do[..., 0] = np.sign(d) * m * sigmoid(o[..., 0]) / cnt
    do[..., 1:1 + N] = lam * np.moveaxis(sigmoid(z) - q_t, 0, -1) / q_t.size
    return L_rho + lam * L_q, do


def backward(params, acts, do):
    """Gradients of every parameter for upstream gradient do of the linear output."""
    grads = {}
    g = do
    dskip = None
    for name, _, _, stride, up, skip, relu in reversed(LAYERS):
        out_key = "o" if name == "c6" else "a" + name[1:]
        if relu:
            g = g * (acts[out_key] > 0)
        if skip is not None:
            dskip = g
        src_key = {"c1": "x", "c2": "a1", "c3": "a2", "c4": "a3", "c5": "a4", "c6": "a5"}[name]
        dx, dw, db = conv3x3_backward(acts[src_key], params[name + ".w"], g, stride, up)
        grads[name + ".w"], grads[name + ".b"] = dw, db
        g = dx
        if name == "c2" and dskip is not None:    # a1 feeds c2 and the skip of c5
            g = g + dskip
    return grads


def adam_step(params, grads, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in place (step counts from 1)."""
    for k in params:
        m[k] = b1 * m[k] + (1 - b1) * grads[k]
        v[k] = b2 * v[k] + (1 - b2) * grads[k] ** 2
        mh = m[k] / (1 - b1 ** step)
        vh = v[k] / (1 - b2 ** step)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
