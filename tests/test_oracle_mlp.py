"""Pins of the FP64 deformation-network oracle (paper §4, "MLP") against closed
forms, a pure-Python loop and finite differences."""
import math

import numpy as np
import pytest

import scenes
from oracle import mlp


def test_encoding_closed_forms():
    # p = 0: sin terms 0, cos terms 1; p = 1/4: sin(pi/4), sin(pi/2), sin(pi), ...;
    # p = 1/2: sin(pi/2) = 1, cos(pi) = -1, then sin 0 / cos 1 for k >= 2
    L = 4
    r2 = math.sqrt(0.5)
    exp = {0.0: [0.0, 0, 1, 0, 1, 0, 1, 0, 1],
           0.25: [0.25, r2, r2, 1, 0, 0, -1, 0, 1],
           0.5: [0.5, 1, 0, 0, -1, 0, 1, 0, 1]}
    for p, e in exp.items():
        np.testing.assert_allclose(mlp.encode(np.array([[p]]), L)[0], e, atol=1e-15)
    # block layout for a 3-vector: feature (block k, coordinate c) at k * 3 + c
    x = np.array([[0.0, 0.25, 0.5]])
    enc = mlp.encode(x, L)
    assert enc.shape == (1, 27)
    for c, p in enumerate((0.0, 0.25, 0.5)):
        np.testing.assert_allclose(enc[0, c::3], exp[p], atol=1e-15)
    assert mlp.n_inputs(10, 10) == 84


def test_encoding_derivative_by_differences():
    rng = np.random.default_rng(0)
    p = rng.uniform(0, 1, (4, 3))
    h = 1e-7
    fd = (mlp.encode(p + h, 5) - mlp.encode(p - h, 5)) / (2 * h)
    np.testing.assert_allclose(mlp.encode_grad(p, 5), fd, rtol=1e-6, atol=1e-6)


def _theta(rng, shapes, nonneg=False, b0=None):
    parts = []
    for l, (o, i) in enumerate(shapes):
        w = rng.normal(0, 1.0 / math.sqrt(i), (o, i))
        b = rng.normal(0, 0.1, o)
        if nonneg:
            w, b = np.abs(w), np.abs(b)
        if l == 0 and b0 is not None:
            b = np.full(o, b0)
        parts += [w.ravel(), b]
    return np.concatenate(parts)


def test_all_active_network_is_affine():
    # nonnegative weights and biases and a large first bias keep every unit
    # active, so the network is the affine map x -> M enc + c with
    # M = W_3 W_2 W_1 W_0 and c = sum_l (W_3 ... W_{l+1}) b_l
    rng = np.random.default_rng(1)
    lx, lt, width, depth = 2, 1, 6, 3
    shapes = mlp.layer_shapes(mlp.n_inputs(lx, lt), width, depth)
    theta = _theta(rng, shapes, nonneg=True, b0=100.0)
    W, b = mlp.unpack(theta, shapes)
    x_in, t_in = rng.uniform(0, 1, (7, 3)), rng.uniform(0, 1, 7)
    out, cache = mlp.forward(theta, x_in, t_in, lx, lt, width, depth)
    assert all((h[:, :] > 0).all() for h in cache["h"][1:])
    M = np.linalg.multi_dot(W[::-1])
    c = b[-1] + sum(np.linalg.multi_dot(W[l + 1:][::-1] + [b[l][:, None]])[:, 0]
                    for l in range(depth))
    enc = np.concatenate([mlp.encode(x_in, lx), mlp.encode(t_in[:, None], lt)], axis=1)
    np.testing.assert_allclose(out, enc @ M.T + c, rtol=1e-12)


def test_tiny_network_equals_python_loops():
    rng = np.random.default_rng(2)
    lx, lt, width, depth = 1, 1, 4, 2
    shapes = mlp.layer_shapes(mlp.n_inputs(lx, lt), width, depth)
    theta = _theta(rng, shapes)
    W, b = mlp.unpack(theta, shapes)
    x_in, t_in = rng.uniform(0, 1, (3, 3)), rng.uniform(0, 1, 3)
    out, _ = mlp.forward(theta, x_in, t_in, lx, lt, width, depth)
    for r in range(3):
        x = [float(v) for v in x_in[r]]
        t = float(t_in[r])
        feat = x + [math.sin(math.pi * v) for v in x] + [math.cos(math.pi * v) for v in x]
        feat += [t, math.sin(math.pi * t), math.cos(math.pi * t)]
        h = feat
        for l in range(depth + 1):
            nxt = []
            for o in range(len(b[l])):
                s = float(b[l][o])
                for i in range(len(h)):
                    s += float(W[l][o][i]) * h[i]
                nxt.append(max(0.0, s) if l < depth else s)
            h = nxt
        np.testing.assert_allclose(out[r], h, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("decide", ["exact", "bf16"])
def test_backward_central_differences(decide):
    rng = np.random.default_rng(3)
    lx, lt, width, depth = 3, 2, 8, 3
    shapes = mlp.layer_shapes(mlp.n_inputs(lx, lt), width, depth)
    theta = _theta(rng, shapes)
    x_in, t_in = rng.uniform(0, 1, (5, 3)), rng.uniform(0, 1, 5)
    d_out = rng.normal(size=(5, 3))
    out, cache = mlp.forward(theta, x_in, t_in, lx, lt, width, depth, decide)
    # smooth regime: every pre-activation well away from the relu kink
    W, b = mlp.unpack(theta, shapes)
    z = [cache["h"][l] @ W[l].T + b[l] for l in range(depth)]
    assert min(np.abs(zz).min() for zz in z) > 1e-4
    g_theta, g_x, g_t = mlp.backward(theta, cache, d_out)

    def loss(th=theta, xi=x_in, ti=t_in):
        return float((mlp.forward(th, xi, ti, lx, lt, width, depth, decide)[0] * d_out).sum())

    h = 1e-6
    idx = np.concatenate([rng.choice(len(theta), 40, replace=False),
                          np.cumsum([o * i + o for o, i in shapes]) - 1])   # + every last bias
    for j in idx:
        e = np.zeros_like(theta)
        e[j] = h
        fd = (loss(th=theta + e) - loss(th=theta - e)) / (2 * h)
        assert g_theta[j] == pytest.approx(fd, rel=1e-6, abs=1e-9), j
    for r in range(5):
        for c in range(3):
            e = np.zeros_like(x_in)
            e[r, c] = h
            fd = (loss(xi=x_in + e) - loss(xi=x_in - e)) / (2 * h)
            assert g_x[r, c] == pytest.approx(fd, rel=1e-6, abs=1e-9)
        e = np.zeros_like(t_in)
        e[r] = h
        fd = (loss(ti=t_in + e) - loss(ti=t_in - e)) / (2 * h)
        assert g_t[r] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_offsets_rows_and_centre_gradient():
    rng = np.random.default_rng(4)
    lx, lt, width, depth = 2, 2, 8, 2
    shapes = mlp.layer_shapes(mlp.n_inputs(lx, lt), width, depth)
    theta = _theta(rng, shapes)
    x0 = rng.uniform(-1, 1, (3, 6))
    times = np.array([0.0, 0.1, 0.3])
    sx, st = 0.25, 4.0          # exact in float32, the precision of the scales
    d = mlp.offsets(theta, x0, times, sx, st, lx, lt, width, depth)
    assert d.shape == (3, 3, 6)
    for ti, t in enumerate(times):
        o, _ = mlp.forward(theta, sx * x0.T, np.full(6, st * t), lx, lt, width, depth)
        np.testing.assert_allclose(d[ti], o.T, rtol=1e-14)
    up = rng.normal(size=d.shape)
    _, g_x0 = mlp.offsets_backward(theta, x0, times, sx, st, up, lx, lt, width, depth)
    h = 1e-6
    for c in range(3):
        for n in range(6):
            e = np.zeros_like(x0)
            e[c, n] = h
            fd = ((mlp.offsets(theta, x0 + e, times, sx, st, lx, lt, width, depth) * up).sum()
                  - (mlp.offsets(theta, x0 - e, times, sx, st, lx, lt, width, depth) * up).sum()) / (2 * h)
            assert g_x0[c, n] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_initialisation_statistics():
    # Xavier-normal hidden weights, N(0, 1e-5^2) last layer, zero biases (§4)
    theta = scenes.mlp_params(seed=0).astype(np.float64)
    shapes = mlp.layer_shapes()
    assert theta.size == mlp.n_params(shapes) == 483_075
    W, b = mlp.unpack(theta, shapes)
    for l, (o, i) in enumerate(shapes[:-1]):
        assert W[l].std() == pytest.approx(math.sqrt(2.0 / (o + i)), rel=0.03)
        assert abs(W[l].mean()) < 0.01
        assert not b[l].any()
    assert W[-1].std() == pytest.approx(1e-5, rel=0.1)
    assert not b[-1].any()


def test_bfloat16_rounding():
    # 8 significant bits, ties to even: spacing 2^-7 on [1, 2)
    cases = {1.0: 1.0, 1 + 2 ** -8: 1.0, 1 + 3 * 2 ** -8: 1 + 2 ** -6, 1 + 2 ** -7: 1 + 2 ** -7,
             1 + 2 ** -8 + 2 ** -20: 1 + 2 ** -7, -(1 + 3 * 2 ** -8): -(1 + 2 ** -6),
             3.0: 3.0, 0.0: 0.0, 2.0 ** -130: 2.0 ** -130}
    for x, e in cases.items():
        assert mlp.round_bf16(np.array([x]))[0] == e, x
    # an independent implementation of the same rounding: torch's conversion
    import torch
    x = np.random.default_rng(5).normal(0, 10, 10000).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.round_bf16(x), ref)


def test_bfloat16_decisions_differ_only_near_zero():
    # the kernel-precision decisions equal the exact ones except for units
    # whose pre-activation is within bfloat16 rounding of 0; an all-active
    # network is decided identically
    rng = np.random.default_rng(6)
    lx, lt, width, depth = 10, 10, 64, 4
    shapes = mlp.layer_shapes(mlp.n_inputs(lx, lt), width, depth)
    theta = _theta(rng, shapes)
    x_in, t_in = rng.uniform(0, 1, (400, 3)), rng.uniform(0, 1, 400)
    out_e, ce = mlp.forward(theta, x_in, t_in, lx, lt, width, depth, "exact")
    out_b, cb = mlp.forward(theta, x_in, t_in, lx, lt, width, depth, "bf16")
    W, b = mlp.unpack(theta, shapes)
    for l in range(depth):
        z = cb["h"][l] @ W[l].T + b[l]
        scale = np.abs(cb["h"][l]) @ np.abs(W[l]).T + np.abs(b[l])
        differ = cb["masks"][l] != (z > 0)
        assert differ.mean() < 0.01
        assert np.all(np.abs(z[differ]) <= 2 * 2 ** -8 * scale[differ] + 1e-12)
    theta_p = _theta(rng, shapes, nonneg=True, b0=100.0)
    a, _ = mlp.forward(theta_p, x_in, t_in, lx, lt, width, depth, "exact")
    c, _ = mlp.forward(theta_p, x_in, t_in, lx, lt, width, depth, "bf16")
    np.testing.assert_array_equal(a, c)


def test_eq7_blend_of_offsets():
    # Eq. 7 is exact for motion linear in time: offsets A + B t at the integer
    # timesteps blend to A + B t at every fractional frame time
    import dataclasses
    rng = np.random.default_rng(7)
    A, B = rng.normal(size=(3, 5)), rng.normal(size=(3, 5))
    step_t = [0.0, 0.25, 0.5]
    steps = np.stack([A + B * t for t in step_t])
    base = scenes.Frame()
    frames, anchors = [], []
    for k in range(8):
        i, j = divmod(k, 4)
        t = float(np.float32(0.25 * (i + j / 4)))
        frames.append(dataclasses.replace(base, time=t, t_lo=float(np.float32(0.25 * i)),
                                          t_hi=float(np.float32(0.25 * (i + 1)))))
        anchors.append((i, i + 1))
    out = mlp.blend_offsets(steps, frames, anchors)
    for f, fr in enumerate(frames):
        np.testing.assert_allclose(out[f], A + B * fr.time, rtol=1e-12, atol=1e-12)
    # a frame at its first anchor takes that step's offsets; one without
    # anchors takes its first index unchanged
    assert mlp.eq7_weights(frames[0]) == (1.0, 0.0)
    plain = mlp.blend_offsets(steps, [base], [(2, 0)])
    np.testing.assert_array_equal(plain[0], steps[2])
    # the backward is the adjoint: <blend(x), y> = <x, blend_bwd(y)>
    y = rng.normal(size=out.shape)
    lhs = (out * y).sum()
    rhs = (steps * mlp.blend_offsets_backward(y, frames, anchors, 3)).sum()
    assert lhs == pytest.approx(rhs, rel=1e-12)


def _float32_decisions(theta, x_in, t_in, order, seed):
    # a float32 evaluation with bfloat16 operands, as a matrix-core kernel
    # might run it: the encoding within one float32 ulp (as a sinpi of float32
    # accuracy gives it), then per layer the products accumulated in float32
    # in the given order, ReLU and rounding to bfloat16
    import torch
    lx = lt = 10
    W, b = mlp.unpack(theta, mlp.layer_shapes())
    x32 = np.asarray(x_in, np.float64).astype(np.float32).astype(np.float64)
    t32 = np.asarray(t_in, np.float64).astype(np.float32).astype(np.float64)
    v = mlp.network_input(x32, t32, lx, lt).astype(np.float32)
    rng = np.random.default_rng(seed)
    step = np.where(rng.random(v.shape) < 0.5, np.float32(np.inf), np.float32(-np.inf))
    v[:, 3:63] = np.nextafter(v[:, 3:63], step[:, 3:63])          # sin / cos blocks of x
    v[:, 64:] = np.nextafter(v[:, 64:], step[:, 64:])              # sin / cos blocks of t
    h = torch.from_numpy(mlp.round_bf16(v).astype(np.float32))
    masks = []
    for l in range(8):
        w = torch.from_numpy(mlp.round_bf16(W[l]).astype(np.float32))
        bias = torch.from_numpy(b[l].astype(np.float32))
        K = w.shape[1]
        if order == "matmul, bias last":
            z = h @ w.T + bias
        else:
            chunks = [(k, min(k + 32, K)) for k in range(0, K, 32)]
            if order == "k-steps of 32 descending":
                chunks = chunks[::-1]
            z = bias.expand(h.shape[0], -1).clone()
            if order == "sequential":
                for k in range(K):
                    z = z + h[:, k:k + 1] * w[:, k]
            else:
                for k0, k1 in chunks:
                    z = z + h[:, k0:k1] @ w[:, k0:k1].T
        masks.append((z > 0).numpy())
        h = torch.from_numpy(mlp.round_bf16(np.maximum(z.numpy(), 0.0)).astype(np.float32))
    return np.stack(masks, axis=1)


@pytest.mark.parametrize("order", ["k-steps of 32", "k-steps of 32 descending", "matmul, bias last",
                                   "sequential"])
def test_float32_decisions_differ_only_within_the_margin(order):
    # the ReLU decisions of a float32 / bfloat16 evaluation in any of several
    # accumulation orders equal the shadow's except at units whose |z| is
    # within DECISION_MARGIN of their scale; the drift behind such a flip
    # stays well inside the margin, and flips are rare
    theta = scenes.mlp_params(seed=1, last_std=0.05, bias_std=0.1)
    x0, times = scenes.mlp_rows(200, 3, seed=101)
    sx, st = float(np.float32(2 * 30e6 / 299_792_458.0)), 4.0
    x_in, t_in, _, _ = mlp._rows(x0, times, sx, st)
    masks, ratio = mlp.decision_table(theta, x_in, t_in)
    got = _float32_decisions(theta, x_in, t_in, order, seed=len(order))
    differ = got != masks
    assert differ.mean() < 1e-4
    assert np.all(ratio[differ] <= 2.5e-3), ratio[differ].max()
    assert 2.5e-3 * 4 <= mlp.DECISION_MARGIN
    # the margin is not vacuous: most units sit far outside it
    assert (ratio <= mlp.DECISION_MARGIN).mean() < 0.1
