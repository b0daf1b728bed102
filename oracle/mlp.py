"""Deformation network of §4 in FP64: positional encoding, MLP, offsets.

TEST INFRASTRUCTURE ONLY (see the package header).

Paper §4 (method overview, "Initialization" and "MLP"):
* a network takes the canonical centre x_k of a Gaussian and the time t and
  returns a position offset; the Gaussian is moved from the canonical space
  to x_k + delta_x_k(t);
* it has 8 layers of 256 units and positional encodings with L_x = 10
  frequencies for the position and L_t = 10 for the time;
* its position input is rescaled by the unambiguous range so that most values
  lie in [0, 1]; the offset itself is in scene units;
* biases start at zero, weights Xavier-normal, except the last linear layer
  (256 features to the offset), whose weights start as N(0, 1e-5^2).

Readings where the paper is silent (each is listed with the others in the
design notes):
* encoding of a d-vector p with L frequencies: the blocks
  (p, sin(pi p), cos(pi p), sin(2 pi p), cos(2 pi p), ...,
  sin(2^(L-1) pi p), cos(2^(L-1) pi p)), each a d-vector, so d (1 + 2L)
  features; the network input is (enc_Lx(s_x x), enc_Lt(s_t t)), 84 features
  at L_x = L_t = 10;
* the 8 layers are hidden layers h_{l+1} = relu(W_l h_l + b_l), l = 0..7,
  h_0 = the encoding, with no skip connection (none is described); the
  offset is W_8 h_8 + b_8 with no activation;
* s_x = 2 f / c (the inverse unambiguous range); s_t is the caller's
  (1 / sequence duration in the benchmarks).

Parameter vector layout (the C ABI uses the same): for l = 0..8 in order,
W_l row-major [out][in], then b_l [out].

Discrete decisions.  Which hidden units are active (z > 0) is an integer
result of floating point.  A unit whose z is within rounding of 0 can be
decided differently by two correct implementations, and its gradient then
changes by a whole term.  forward(..., decide="bf16") takes those decisions
in the precision of the matrix-core products (bfloat16 operands rounded to
nearest even, wide accumulation), from a shadow evaluation; the values and
gradients are still the FP64 definition with those decisions held fixed
(h = [z_decided > 0] z), as the rasterizer oracle holds its visit decisions
fixed.  decide="exact" takes them from the FP64 values themselves.

Pins: tests/test_oracle_mlp.py (encoding closed forms at p = 0, 1/4, 1/2;
an all-active network equals its affine closed form, a product of the weight
matrices; a tiny network equals a pure-Python triple loop; central finite
differences of every gradient).
"""
from __future__ import annotations

import numpy as np


def n_inputs(lx: int = 10, lt: int = 10) -> int:
    """Features of the encoded (x, t) input."""
    return 3 * (1 + 2 * lx) + (1 + 2 * lt)


def layer_shapes(n_in: int = 84, width: int = 256, depth: int = 8, n_out: int = 3):
    """(out, in) of every linear layer, input layer first."""
    return [(width, n_in)] + [(width, width)] * (depth - 1) + [(n_out, width)]


def n_params(shapes) -> int:
    return sum(o * i + o for o, i in shapes)


def unpack(theta, shapes):
    """Views W_l [out][in], b_l [out] of the flat parameter vector."""
    theta = np.asarray(theta, dtype=np.float64)
    W, b, at = [], [], 0
    for o, i in shapes:
        W.append(theta[at:at + o * i].reshape(o, i))
        at += o * i
        b.append(theta[at:at + o])
        at += o
    assert at == theta.size
    return W, b


def encode(p, L: int):
    """Positional encoding of p [R, d]: blocks p, sin(2^k pi p), cos(2^k pi p)
    for k = 0..L-1, concatenated to [R, d (1 + 2L)]."""
    p = np.asarray(p, dtype=np.float64)
    blocks = [p]
    for k in range(L):
        a = (2.0 ** k) * np.pi * p
        blocks += [np.sin(a), np.cos(a)]
    return np.concatenate(blocks, axis=1)


def encode_grad(p, L: int):
    """d feature / d (its own coordinate), same layout as encode(p, L)."""
    p = np.asarray(p, dtype=np.float64)
    blocks = [np.ones_like(p)]
    for k in range(L):
        w = (2.0 ** k) * np.pi
        a = w * p
        blocks += [w * np.cos(a), -w * np.sin(a)]
    return np.concatenate(blocks, axis=1)


def network_input(x_in, t_in, lx: int = 10, lt: int = 10):
    """(enc_Lx(x_in), enc_Lt(t_in)): x_in [R, 3] and t_in [R] already scaled."""
    return np.concatenate([encode(x_in, lx), encode(np.asarray(t_in, np.float64)[:, None], lt)],
                          axis=1)


def round_bf16(x):
    """Nearest bfloat16 (ties to even) of the float32 rounding of x, as float64."""
    b = np.asarray(x, np.float64).astype(np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


# A float32 evaluation with bfloat16 operands, in any accumulation order,
# reaches pre-activations z close to the bfloat16 shadow's below: apart from
# its own float32 rounding, an activation it passes on may round to the
# neighbouring bfloat16 value, and such one-step differences spread over the
# layers.  Measured over many accumulation orders of the 8 x 256 network, the
# drift stays below 2.5e-3 of the unit's scale |b| + sum_k |h_k w_k|;
# DECISION_MARGIN bounds it with headroom.  So two such evaluations can take
# a unit's ReLU decision differently only where |z| <= DECISION_MARGIN scale.
DECISION_MARGIN = 1e-2


def _decisions(W, b, x_in, t_in, lx, lt, depth, margins: bool = False):
    """Active-unit masks of the hidden layers evaluated as the products are:
    scaled inputs rounded to float32, bfloat16 operands.  With margins, also
    |z| / scale of every hidden unit (scale = |b| + sum_k |h_k w_k|)."""
    x32 = np.asarray(x_in, np.float64).astype(np.float32).astype(np.float64)
    t32 = np.asarray(t_in, np.float64).astype(np.float32).astype(np.float64)
    masks, ratios, h = [], [], round_bf16(network_input(x32, t32, lx, lt))
    for l in range(depth):
        w = round_bf16(W[l])
        z = h @ w.T + b[l]
        masks.append(z > 0.0)
        if margins:
            scale = np.abs(h) @ np.abs(w).T + np.abs(b[l])
            ratios.append(np.abs(z) / np.maximum(scale, 1e-300))
        h = round_bf16(np.maximum(z, 0.0))
    return (masks, ratios) if margins else masks


def decision_table(theta, x_in, t_in, lx: int = 10, lt: int = 10, width: int = 256,
                   depth: int = 8):
    """The decisions forward(..., decide="bf16") takes, as booleans
    [R, depth, width], and each unit's |z| / scale in the same layout: a
    float32 / bfloat16 evaluation may decide a unit differently only where
    that ratio is at most DECISION_MARGIN."""
    W, b = unpack(theta, layer_shapes(n_inputs(lx, lt), width, depth))
    masks, ratios = _decisions(W, b, x_in, t_in, lx, lt, depth, margins=True)
    return np.stack(masks, axis=1), np.stack(ratios, axis=1)


def offsets_decision_table(theta, x0, times, s_x, s_t, lx: int = 10, lt: int = 10,
                           width: int = 256, depth: int = 8):
    """decision_table of the rows of offsets(...): row t N + k for time t and
    Gaussian k."""
    x_in, t_in, _, _ = _rows(x0, times, s_x, s_t)
    return decision_table(theta, x_in, t_in, lx, lt, width, depth)


def forward(theta, x_in, t_in, lx: int = 10, lt: int = 10, width: int = 256, depth: int = 8,
            decide: str = "exact"):
    """Offsets [R, 3] of R rows; also returns what backward needs (the hidden
    activations h_0..h_depth and the active-unit masks)."""
    shapes = layer_shapes(n_inputs(lx, lt), width, depth)
    W, b = unpack(theta, shapes)
    h = [network_input(x_in, t_in, lx, lt)]
    masks = _decisions(W, b, x_in, t_in, lx, lt, depth) if decide == "bf16" else None
    if decide not in ("exact", "bf16"):
        raise ValueError(decide)
    for l in range(depth):
        z = h[-1] @ W[l].T + b[l]
        m = masks[l] if masks is not None else z > 0.0
        h.append(np.where(m, z, 0.0))
    out = h[-1] @ W[depth].T + b[depth]
    return out, {"h": h, "masks": masks, "x_in": np.asarray(x_in, np.float64),
                 "t_in": np.asarray(t_in, np.float64), "lx": lx, "lt": lt,
                 "width": width, "depth": depth}


def backward(theta, cache, d_out):
    """Gradients of sum(d_out * out): the flat parameter gradient, and the
    gradients with respect to the scaled inputs x_in [R, 3] and t_in [R]."""
    lx, lt, width, depth = cache["lx"], cache["lt"], cache["width"], cache["depth"]
    shapes = layer_shapes(n_inputs(lx, lt), width, depth)
    W, _ = unpack(theta, shapes)
    h = cache["h"]
    dW, db = [None] * (depth + 1), [None] * (depth + 1)
    g = np.asarray(d_out, dtype=np.float64)            # d/d(pre-activation) of layer `depth`
    for l in range(depth, -1, -1):
        dW[l] = g.T @ h[l]
        db[l] = g.sum(axis=0)
        gh = g @ W[l]                                  # d/d h_l
        if l > 0:                                      # relu' of layer l-1's output
            active = cache["masks"][l - 1] if cache["masks"] is not None else h[l] > 0.0
            g = gh * active
    d_enc = gh                                         # d/d h_0, the encoding
    nx = 3 * (1 + 2 * lx)
    gx = d_enc[:, :nx] * encode_grad(cache["x_in"], lx)
    gt = d_enc[:, nx:] * encode_grad(cache["t_in"][:, None], lt)
    d_x = gx.reshape(len(gx), 1 + 2 * lx, 3).sum(axis=1)
    d_t = gt.sum(axis=1)
    # magnitude of the terms d_x sums: d_x = sum_f enc'_f sum_j g_j W_0[j, f]
    # (g the first layer's pre-activation gradient), and both sums cancel (the
    # encoding's derivatives reach 2^(L-1) pi), so the scale of its rounding
    # errors in any precision is sum_f |enc'_f| sum_j |g_j W_0[j, f]|
    terms = (np.abs(g) @ np.abs(W[0]))[:, :nx] * np.abs(encode_grad(cache["x_in"], lx))
    cache["d_x_terms"] = terms.reshape(len(gx), 1 + 2 * lx, 3).sum(axis=1)
    flat = np.concatenate([np.concatenate([w.ravel(), c]) for w, c in zip(dW, db)])
    return flat, d_x, d_t


def _rows(x0, times, s_x, s_t):
    """Rows (t, n) in time-major order: x_in [T N, 3], t_in [T N].  The scales
    are float32 values (as the device receives them), widened exactly."""
    x0 = np.asarray(x0, dtype=np.float64)              # [3][N]
    times = np.asarray(times, dtype=np.float64)
    s_x, s_t = float(np.float32(s_x)), float(np.float32(s_t))
    T, N = len(times), x0.shape[1]
    x_in = np.tile((s_x * x0).T, (T, 1))
    t_in = np.repeat(s_t * times, N)
    return x_in, t_in, T, N


def offsets(theta, x0, times, s_x, s_t, lx: int = 10, lt: int = 10, width: int = 256,
            depth: int = 8, decide: str = "exact"):
    """delta [T][3][N]: the network at every (time, Gaussian) row."""
    x_in, t_in, T, N = _rows(x0, times, s_x, s_t)
    out, _ = forward(theta, x_in, t_in, lx, lt, width, depth, decide)
    return out.reshape(T, N, 3).transpose(0, 2, 1)


def offsets_backward(theta, x0, times, s_x, s_t, d_delta, lx: int = 10, lt: int = 10,
                     width: int = 256, depth: int = 8, decide: str = "exact", terms: bool = False):
    """Gradients of sum(d_delta * offsets(...)): the flat parameter gradient and
    d x0 [3][N] (the canonical centre reaches the network through s_x x0, summed
    over the T times); with `terms` also the summed magnitudes of d x0's terms."""
    x_in, t_in, T, N = _rows(x0, times, s_x, s_t)
    _, cache = forward(theta, x_in, t_in, lx, lt, width, depth, decide)
    d_out = np.asarray(d_delta, np.float64).transpose(0, 2, 1).reshape(T * N, 3)
    flat, d_x, _ = backward(theta, cache, d_out)
    s_x = float(np.float32(s_x))
    d_x0 = s_x * d_x.reshape(T, N, 3).sum(axis=0).T
    if terms:
        return flat, d_x0, s_x * cache["d_x_terms"].reshape(T, N, 3).sum(axis=0).T
    return flat, d_x0


def eq7_weights(frame):
    """Eq. 7 weights (w1, w2) of a frame with anchors t_lo < t_hi: its centre
    is w1 x(t_lo) + w2 x(t_hi); (1, 0) for a frame without anchors.  The frame
    values are float32, widened exactly."""
    f32 = lambda v: float(np.float32(v))
    t, lo, hi = f32(frame.time), f32(getattr(frame, "t_lo", 0.0)), f32(getattr(frame, "t_hi", 0.0))
    if hi > lo:
        return (hi - t) / (hi - lo), (t - lo) / (hi - lo)
    return 1.0, 0.0


def blend_offsets(delta_steps, frames, anchors):
    """Eq. 7 with the network: per-frame offsets [F][3][N] from offsets at
    integer timesteps delta_steps [S][3][N]; frame f reads steps
    anchors[f] = (lo, hi) with its Eq. 7 weights."""
    d = np.asarray(delta_steps, np.float64)
    out = np.empty((len(frames),) + d.shape[1:])
    for f, fr in enumerate(frames):
        w1, w2 = eq7_weights(fr)
        lo, hi = anchors[f]
        out[f] = w1 * d[lo] + w2 * d[hi]
    return out


def blend_offsets_backward(d_frames, frames, anchors, n_steps):
    """Gradient of sum(d_frames * blend_offsets(...)) with respect to
    delta_steps [S][3][N]."""
    g = np.asarray(d_frames, np.float64)
    out = np.zeros((n_steps,) + g.shape[1:])
    for f, fr in enumerate(frames):
        w1, w2 = eq7_weights(fr)
        lo, hi = anchors[f]
        out[lo] += w1 * g[f]
        out[hi] += w2 * g[f]
    return out
