"""Pins of the guess-network oracle (oracle/cnn_oracle.c) against what holds
independently of it: the library's bfloat16 conversion, scipy's correlation
with explicit boundary modes, closed-form Laplacian eigenvalues, central
finite differences and torch's Adam."""
import numpy as np
import pytest
import scipy.ndimage as ndi

import les_inputs as li
from oracle import cnn

BLOCKS = [(27 * ci * co, 27 * ci, co) for ci, co in zip(cnn.CIN, cnn.COUT)]


def correlate(f, k):
    """scipy correlation of a (nz, ny, nx) field with a 3x3x3 kernel after
    padding x and y by wrap-around and z by the even mirror."""
    g = np.pad(f, ((1, 1), (0, 0), (0, 0)), mode="symmetric")
    g = np.pad(g, ((0, 0), (1, 1), (1, 1)), mode="wrap")
    return ndi.correlate(g, k, mode="constant")[1:-1, 1:-1, 1:-1]


def params(seed=1, bias=0.0):
    p = li.cnn_init(seed, BLOCKS)
    if bias:
        rng = np.random.default_rng(seed)
        for l in range(cnn.LAYERS):
            o = cnn.bias_offset(l)
            p[o:o + cnn.COUT[l]] = bias * rng.standard_normal(cnn.COUT[l])
    return p


def test_layout():
    assert cnn.param_count() == sum(nw + nb for nw, _, nb in BLOCKS) == 14737
    assert cnn.weight_offset(1) == 27 * 16 + 16
    assert cnn.bias_offset(3) == cnn.param_count() - 1


def test_bf16_matches_torch():
    import torch
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(4000) * 10.0 ** rng.integers(-6, 6, 4000),
                        [0.0, -0.0, 1.0, -2.5, 3.0e38]]).astype(np.float32)
    # exact ties: low 16 bits 0x8000, both parities of the kept bit
    bits = (rng.integers(0, 2 ** 31, 500, dtype=np.uint32) & np.uint32(0xFFFF0000)) | np.uint32(0x8000)
    x = np.concatenate([x, bits.view(np.float32)]).astype(np.float32)
    x = x[np.isfinite(x)]
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = cnn.bf16(x.astype(np.float64))
    assert np.array_equal(got, ref)
    assert np.isnan(cnn.bf16(np.array([np.nan]))).all()


def _select(p, l_random, c_in, c_out):
    """Parameters whose network output is channel c_out of layer l_random's
    convolution of input channel c_in: other layers pass a channel through
    their centre tap."""
    q = np.zeros_like(p)
    centre = 13
    for l in range(cnn.LAYERS):
        wo, ci, co = cnn.weight_offset(l), cnn.CIN[l], cnn.COUT[l]
        if l == l_random:
            q[wo:wo + 27 * ci * co] = p[wo:wo + 27 * ci * co]
            q[cnn.bias_offset(l):cnn.bias_offset(l) + co] = p[cnn.bias_offset(l):cnn.bias_offset(l) + co]
            continue
        W = np.zeros((27, co, ci))
        if l < l_random:        # route the input into channel c_in
            if ci == 1:
                W[centre, c_in, 0] = 1.0
            else:
                W[centre, c_in, c_in] = 1.0
        else:                   # route channel c_out to the output
            if co == 1:
                W[centre, 0, c_out] = 1.0
            else:
                W[centre, c_out, c_out] = 1.0
        q[wo:wo + W.size] = W.ravel()
    return q


@pytest.mark.parametrize("l,c_in,c_out", [(0, 0, 0), (0, 0, 15), (1, 3, 7), (2, 15, 0), (3, 5, 0)])
@pytest.mark.parametrize("periodic", [True, False])
def test_single_layer_is_scipy_correlation(l, c_in, c_out, periodic):
    """One layer against scipy.ndimage.correlate with x, y wrapping and the
    z even mirror (numpy's 'symmetric' padding)."""
    p = _select(params(3, bias=0.3), l, c_in, c_out)
    rng = np.random.default_rng(l)
    x = rng.standard_normal((2, 7, 11, 13))
    out, _, _ = cnn.forward(p, x, periodic=periodic, alpha=1.0, bf16=False)
    W = p[cnn.weight_offset(l):cnn.bias_offset(l)].reshape(27, cnn.COUT[l], cnn.CIN[l])
    co = 0 if cnn.COUT[l] == 1 else c_out
    ci = 0 if cnn.CIN[l] == 1 else c_in
    k = W[:, co, ci].reshape(3, 3, 3)
    b = p[cnn.bias_offset(l) + co]
    for s in range(2):
        ref = correlate(x[s], k) + b
        if not periodic:
            ref = ref[:, 4:-4, 4:-4]
        np.testing.assert_allclose(out[s], ref, rtol=0, atol=1e-12)


def test_leaky_relu_between_layers():
    """Layer 0 routed through a leaky ReLU of slope 0.1 to the output."""
    p = _select(params(4, bias=0.5), 0, 0, 2)
    x = np.random.default_rng(1).standard_normal((1, 5, 9, 9))
    out, _, pre = cnn.forward(p, x, periodic=True, alpha=0.1, bf16=False)
    W = p[:27 * 16].reshape(27, 16, 1)[:, 2, 0].reshape(3, 3, 3)
    y = correlate(x[0], W) + p[cnn.bias_offset(0) + 2]
    # layers 0, 1 and 2 each end in a leaky ReLU: slope 0.1^3 for y < 0
    np.testing.assert_allclose(out[0], np.where(y >= 0, y, 1e-3 * y), atol=1e-12)
    assert (y < 0).mean() > 0.1


def test_valid_crop_equals_periodic_field():
    """A crop with a 4-cell halo, cut from a periodic field with wrap-around,
    gives exactly the periodic output on the crop (bf16 rounding on)."""
    p = params(5, bias=0.1)
    rng = np.random.default_rng(2)
    f = rng.standard_normal((1, 6, 14, 12))
    full, _, _ = cnn.forward(p, f, periodic=True)
    j0, i0, cy, cx = 9, 5, 6, 7
    jj = (j0 - 4 + np.arange(cy + 8)) % 14
    ii = (i0 - 4 + np.arange(cx + 8)) % 12
    crop = f[:, :, jj][:, :, :, ii]
    out, _, _ = cnn.forward(p, crop, periodic=False)
    ref = full[:, :, (j0 + np.arange(cy)) % 14][:, :, :, (i0 + np.arange(cx)) % 12]
    assert np.array_equal(out, ref)


def test_bf16_rounding_points():
    """With rounding on, every stored layer input is a bfloat16 value and the
    output differs from the unrounded network by a bfloat16-sized amount."""
    p = params(6, bias=0.1)
    x = np.random.default_rng(3).standard_normal((1, 5, 10, 10))
    out, acts, _ = cnn.forward(p, x, periodic=False)
    out64, _, _ = cnn.forward(p, x, periodic=False, bf16=False)
    for a in acts:
        assert np.array_equal(a, cnn.bf16(a))
    err = np.linalg.norm(out - out64) / np.linalg.norm(out64)
    assert 1e-4 < err < 3e-2


def _zmode(nz, m):
    return np.cos(np.pi * m * (np.arange(nz) + 0.5) / nz)


def test_loss_closed_form():
    """Fourier modes are eigenvectors of the compact Laplacian: an x-mode
    has eigenvalue -(2 - 2 cos theta)/dx^2, a z cosine mode under the even
    mirror -(2 - 2 cos(pi m / nz))/dz^2."""
    dx, dy, dz = 35.0, 35.0, 5.0
    d = 2 / dx**2 + 2 / dy**2 + 2 / dz**2
    nz, ny, nx = 8, 9, 10
    i = np.arange(nx)[None, None, :]
    th = 2 * np.pi * 3 / nx
    e = 0.7 * np.cos(th * i) * np.ones((nz, ny, 1))
    t = np.broadcast_to(_zmode(nz, 2)[:, None, None], (nz, ny, nx)).copy()
    y = t + e
    lam_e = (2 - 2 * np.cos(th)) / dx**2 / d
    lam_t = (2 - 2 * np.cos(np.pi * 2 / nz)) / dz**2 / d
    inner = (slice(None), slice(1, -1), slice(1, -1))
    expect = (lam_e**2 * np.sum(e[inner] ** 2)) / (lam_t**2 * np.sum(t[inner] ** 2))
    got, _ = cnn.loss(y[None], t[None], dx, dy, dz)
    assert got == pytest.approx(expect, rel=1e-12)
    zero, g0 = cnn.loss(t[None], t[None], dx, dy, dz)
    assert zero == 0.0 and not g0.any()


def test_loss_gradient_finite_difference():
    rng = np.random.default_rng(4)
    y = rng.standard_normal((2, 5, 6, 7))
    t = rng.standard_normal((2, 5, 6, 7))
    L0, g = cnn.loss(y, t, 35.0, 30.0, 5.0)
    h = 1e-6
    for idx in [(0, 0, 0, 0), (1, 4, 5, 6), (0, 2, 3, 3), (1, 0, 1, 1), (0, 4, 0, 3)]:
        yp, ym = y.copy(), y.copy()
        yp[idx] += h
        ym[idx] -= h
        fd = (cnn.loss(yp, t, 35.0, 30.0, 5.0)[0] - cnn.loss(ym, t, 35.0, 30.0, 5.0)[0]) / (2 * h)
        assert g[idx] == pytest.approx(fd, rel=1e-6, abs=1e-10)


def test_backward_finite_difference():
    """Gradient of loss(forward(params)) against central differences, FP64
    network (no rounding), leaky slope 0.1, valid crops, two batch items."""
    p = params(7, bias=0.2)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((2, 4, 12, 11))
    t = rng.standard_normal((2, 4, 4, 3))
    dx, dy, dz = 35.0, 35.0, 5.0

    def f(q):
        out, _, _ = cnn.forward(q, x, periodic=False, alpha=0.1, bf16=False)
        return cnn.loss(out, t, dx, dy, dz)[0]

    out, acts, pre = cnn.forward(p, x, periodic=False, alpha=0.1, bf16=False)
    _, gy = cnn.loss(out, t, dx, dy, dz)
    grad = cnn.backward(p, x, acts, pre, gy, periodic=False, alpha=0.1, bf16=False)
    scale = np.abs(grad).max()
    picks = []
    for l in range(cnn.LAYERS):
        wo, bo = cnn.weight_offset(l), cnn.bias_offset(l)
        picks += list(rng.integers(wo, bo, 12)) + [bo, bo + cnn.COUT[l] - 1]
    for q in picks:
        h = 1e-5 * max(1.0, abs(p[q]))
        pp, pm = p.copy(), p.copy()
        pp[q] += h
        pm[q] -= h
        fd = (f(pp) - f(pm)) / (2 * h)
        assert abs(grad[q] - fd) <= 1e-7 * scale + 1e-7 * abs(fd), (q, grad[q], fd)


def test_backward_periodic_matches_crop_sum():
    """Gradients are additive over cells: the periodic gradient equals the
    sum of the gradients of disjoint valid crops that tile the field, for
    an output gradient that is a fixed field (no loss coupling)."""
    p = params(8, bias=0.1)
    rng = np.random.default_rng(6)
    f = rng.standard_normal((1, 4, 8, 8))
    gfull = rng.standard_normal((1, 4, 8, 8))
    out, acts, pre = cnn.forward(p, f, periodic=True, alpha=0.1, bf16=False)
    g_per = cnn.backward(p, f, acts, pre, gfull, periodic=True, alpha=0.1, bf16=False)
    total = np.zeros_like(g_per)
    for j0 in (0, 4):
        for i0 in (0, 4):
            jj = (j0 - 4 + np.arange(12)) % 8
            ii = (i0 - 4 + np.arange(12)) % 8
            crop = f[:, :, jj][:, :, :, ii]
            o, a, pr = cnn.forward(p, crop, periodic=False, alpha=0.1, bf16=False)
            total += cnn.backward(p, crop, a, pr, gfull[:, :, j0:j0 + 4, i0:i0 + 4].copy(),
                                  periodic=False, alpha=0.1, bf16=False)
    np.testing.assert_allclose(total, g_per, rtol=1e-10, atol=1e-10 * np.abs(g_per).max())


def test_adam_matches_torch():
    import torch
    rng = np.random.default_rng(7)
    n = 50
    p0 = rng.standard_normal(n)
    grads = [rng.standard_normal(n) for _ in range(4)]
    w = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.Adam([w], lr=2e-3, betas=(0.9, 0.99), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(n), np.zeros(n)
    for s, g in enumerate(grads, 1):
        w.grad = torch.tensor(g)
        opt.step()
        cnn.adam(p, g.copy(), m, v, s, lr=2e-3, beta1=0.9, beta2=0.99, eps=1e-8)
    np.testing.assert_allclose(p, w.detach().numpy(), rtol=1e-12, atol=1e-14)


# ------------------------------------------- three inputs (p_{n-1}, p_{n-2}, rhs)

BLOCKS3 = [(27 * cnn.cin(l, 3) * co, 27 * cnn.cin(l, 3), co) for l, co in enumerate(cnn.COUT)]


def test_layout_three_inputs():
    assert cnn.cin(0, 3) == 3 and cnn.cin(1, 3) == 16
    assert cnn.param_count(3) == sum(nw + nb for nw, _, nb in BLOCKS3) == 14737 + 27 * 16 * 2
    assert cnn.weight_offset(1, 3) == 27 * 3 * 16 + 16
    assert cnn.bias_offset(0, 3) == 27 * 3 * 16
    assert cnn.bias_offset(3, 3) == cnn.param_count(3) - 1
    assert cnn.param_count(2) == -1


def _three_from_one(p1, rng):
    """Three-input parameters: p1's layers, layer 0 widened with random
    weights for input channels 1 and 2 (W[tap][cout][cin])."""
    W1 = p1[:cnn.bias_offset(0)].reshape(27, 16, 1)
    W3 = np.concatenate([W1, rng.standard_normal((27, 16, 2))], axis=2)
    return np.concatenate([W3.ravel(), p1[cnn.bias_offset(0):]])


@pytest.mark.parametrize("c_out", [0, 9])
def test_three_input_layer_is_sum_of_correlations(c_out):
    """Layer 0 of the three-input network: output channel o is the sum over
    input channels of scipy correlations with W[:, o, c] plus the bias;
    layers 1-3 pass channel o through their centre taps (slope 1)."""
    rng = np.random.default_rng(11)
    p1 = _select(params(9, bias=0.4), 0, 0, c_out)
    p = _three_from_one(p1, rng)
    x = rng.standard_normal((2, 3, 6, 9, 10))
    out, acts, _ = cnn.forward(p, x, periodic=True, alpha=1.0, bf16=False)
    assert acts[0].shape == (2, 3, 6, 9, 10)
    W = p[:cnn.bias_offset(0, 3)].reshape(27, 16, 3)
    for s in range(2):
        ref = sum(correlate(x[s, c], W[:, c_out, c].reshape(3, 3, 3)) for c in range(3))
        ref = ref + p[cnn.bias_offset(0, 3) + c_out]
        np.testing.assert_allclose(out[s], ref, rtol=0, atol=1e-12)


def test_three_inputs_with_zero_extra_weights_equal_one_input():
    """Zero weights on input channels 1 and 2 give the one-input network
    bit for bit, bfloat16 rounding on, whatever those channels hold."""
    rng = np.random.default_rng(12)
    p1 = params(10, bias=0.2)
    p3 = _three_from_one(p1, rng)
    W3 = p3[:cnn.bias_offset(0, 3)].reshape(27, 16, 3)
    W3[:, :, 1:] = 0.0
    p3[:cnn.bias_offset(0, 3)] = W3.ravel()
    x1 = rng.standard_normal((1, 5, 12, 12))
    x3 = np.concatenate([x1[:, None], rng.standard_normal((1, 2, 5, 12, 12))], axis=1)
    o1, _, _ = cnn.forward(p1, x1, periodic=False)
    o3, _, _ = cnn.forward(p3, x3, periodic=False)
    assert np.array_equal(o1, o3)


def test_three_input_backward_finite_difference():
    """Gradient of loss(forward(params)) of the three-input network against
    central differences (FP64 network, valid crops), layer-0 weights of every
    input channel included."""
    rng = np.random.default_rng(13)
    p = li.cnn_init(14, BLOCKS3)
    for l in range(cnn.LAYERS):
        o = cnn.bias_offset(l, 3)
        p[o:o + cnn.COUT[l]] = 0.2 * rng.standard_normal(cnn.COUT[l])
    x = rng.standard_normal((2, 3, 4, 11, 12))
    t = rng.standard_normal((2, 4, 3, 4))
    dx, dy, dz = 35.0, 35.0, 5.0

    def f(q):
        out, _, _ = cnn.forward(q, x, periodic=False, alpha=0.1, bf16=False)
        return cnn.loss(out, t, dx, dy, dz)[0]

    out, acts, pre = cnn.forward(p, x, periodic=False, alpha=0.1, bf16=False)
    _, gy = cnn.loss(out, t, dx, dy, dz)
    grad = cnn.backward(p, x, acts, pre, gy, periodic=False, alpha=0.1, bf16=False)
    scale = np.abs(grad).max()
    W0 = np.arange(cnn.bias_offset(0, 3)).reshape(27, 16, 3)
    picks = [int(W0[t_, o, c]) for t_, o, c in ((0, 0, 0), (13, 5, 1), (26, 15, 2), (4, 8, 2),
                                                 (20, 3, 1))]
    for l in range(1, cnn.LAYERS):
        picks += list(rng.integers(cnn.weight_offset(l, 3), cnn.bias_offset(l, 3), 4))
    picks += [cnn.bias_offset(0, 3), cnn.bias_offset(3, 3)]
    for q in picks:
        # a leaky-ReLU kink lies within 1e-5 of one of these weights: 1e-6 steps
        h = 1e-6 * max(1.0, abs(p[q]))
        pp, pm = p.copy(), p.copy()
        pp[q] += h
        pm[q] -= h
        fd = (f(pp) - f(pm)) / (2 * h)
        assert abs(grad[q] - fd) <= 1e-7 * scale + 1e-7 * abs(fd), (q, grad[q], fd)
