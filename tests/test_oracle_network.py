"""Pins of the learned-correction oracle (oracle/network.py) on the CPU.

Each pin fixes the oracle by something other than itself: shifts of delta
kernels, scipy.ndimage.correlate (a library correlation) in 'wrap' and
'constant' modes, the adjoint identity, central finite differences, the
closed form of the first Adam step, and torch's bfloat16 conversion.
"""
import numpy as np
import pytest
import scipy.ndimage as ndi

from oracle import network as net


def _rng(seed=0):
    return np.random.default_rng(seed)


@pytest.mark.parametrize("periodic", [False, True])
@pytest.mark.parametrize("plane", ["x", "v"])
def test_delta_kernel_is_a_shift(plane, periodic):
    h = _rng(1).standard_normal((4, 5, 3, 6, 1))
    for t in range(9):
        a, b = t // 3 - 1, t % 3 - 1
        W = np.zeros((9, 1, 1))
        W[t, 0, 0] = 1.0
        out = net.conv(h, W, np.zeros(1), plane, periodic)[..., 0]
        ax = (0, 1) if plane == "x" else (2, 3)
        ref = np.zeros_like(h[..., 0])
        n0, n1 = h.shape[ax[0]], h.shape[ax[1]]
        it = np.ndindex(h.shape[:4])
        for idx in it:
            j = list(idx)
            j[ax[0]] += a
            j[ax[1]] += b
            if periodic:
                j[ax[0]] %= n0
                j[ax[1]] %= n1
            elif not (0 <= j[ax[0]] < n0 and 0 <= j[ax[1]] < n1):
                continue
            ref[idx] = h[tuple(j) + (0,)]
        assert np.array_equal(out, ref)


@pytest.mark.parametrize("periodic", [False, True])
def test_single_channel_conv_equals_scipy_correlate(periodic):
    rng = _rng(2)
    h = rng.standard_normal((6, 7, 5, 4, 1))
    W = rng.standard_normal((9, 1, 1))
    k = W[:, 0, 0].reshape(3, 3)
    mode = "wrap" if periodic else "constant"
    out = net.conv(h, W, np.array([0.25]), "x", periodic)[..., 0]
    for v1 in range(5):
        for v2 in range(4):
            ref = ndi.correlate(h[:, :, v1, v2, 0], k, mode=mode, cval=0.0) + 0.25
            assert np.allclose(out[:, :, v1, v2], ref, rtol=0, atol=1e-13)
    out = net.conv(h, W, np.zeros(1), "v", periodic)[..., 0]
    for x1 in range(6):
        for x2 in range(7):
            ref = ndi.correlate(h[x1, x2, :, :, 0], k, mode=mode, cval=0.0)
            assert np.allclose(out[x1, x2], ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("periodic", [False, True])
@pytest.mark.parametrize("plane", ["x", "v"])
def test_conv_adjoint_identity(plane, periodic):
    rng = _rng(3)
    h = rng.standard_normal((4, 3, 5, 4, 3))
    W = rng.standard_normal((9, 2, 3))
    dz = rng.standard_normal((4, 3, 5, 4, 2))
    lhs = np.sum(net.conv(h, W, np.zeros(2), plane, periodic) * dz)
    rhs = np.sum(h * net.conv_adjoint(dz, W, plane, periodic))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # weight gradient: d<conv(h; W), dz>/dW
    gW, gb = net.conv_weight_grad(h, dz, plane, periodic)
    E = rng.standard_normal(W.shape)
    lin = np.sum(net.conv(h, E, np.zeros(2), plane, periodic) * dz)
    assert abs(np.sum(gW * E) - lin) <= 1e-12 * abs(lin)
    assert np.allclose(gb, dz.reshape(-1, 2).sum(0))


def _theta(seed, scale=0.2):
    rng = _rng(seed)
    return rng.standard_normal(net.NCONV * net.CONV_PARAMS) * scale / np.sqrt(9 * net.C)


@pytest.mark.parametrize("xper,vper", [(True, False), (False, False)])
def test_backward_matches_finite_differences(xper, vper):
    rng = _rng(4)
    R = 2
    theta = _theta(5, scale=1.5)
    x = rng.standard_normal((3, 4, 3, 3, R))
    target = rng.standard_normal((3, 4, 3, 3, R))

    def L(th, xx):
        y = net.forward(th, xx, xper, vper)
        return net.loss_and_grad(y, target, R)[0]

    y = net.forward(theta, x, xper, vper)
    _, dy = net.loss_and_grad(y, target, R)
    g, gx = net.backward(theta, x, dy, xper, vper)
    eps = 1e-6
    idx = rng.choice(theta.size, 40, replace=False)
    # include biases and weights of every conv
    idx = np.concatenate([idx, [c * net.CONV_PARAMS + net.TAPS * net.C * net.C + 3 for c in range(net.NCONV)]])
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = eps
        fd = (L(theta + e, x) - L(theta - e, x)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])
    for _ in range(10):
        j = tuple(rng.integers(0, s) for s in x.shape)
        e = np.zeros_like(x)
        e[j] = eps
        fd = (L(theta, x + e) - L(theta, x - e)) / (2 * eps)
        assert abs(fd - gx[j]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9


def test_padding_channels_receive_no_gradient():
    """Input channels >= R and output channels >= R stay exactly zero-gradient."""
    rng = _rng(6)
    R = 1
    theta = _theta(7)
    x = rng.standard_normal((3, 3, 3, 3, R))
    y = net.forward(theta, x, True, False)
    _, dy = net.loss_and_grad(y, rng.standard_normal((3, 3, 3, 3, R)), R)
    g, _ = net.backward(theta, x, dy, True, False)
    p = net.unpack_params(g)
    assert np.all(p[0][0][:, :, R:] == 0.0)       # first conv, padded input channels
    assert np.all(p[7][0][:, R:, :] == 0.0)       # last conv, padded output channels
    assert np.all(p[7][1][R:] == 0.0)


def test_first_adam_step_is_signed_lr():
    rng = _rng(8)
    th = rng.standard_normal(50)
    g = rng.standard_normal(50)
    new, m, v = net.adam_step(th, g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    assert np.allclose(new - th, -1e-3 * np.sign(g), rtol=1e-6, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = _rng(9)
    a = np.concatenate([rng.standard_normal(2000) * 10.0 ** rng.integers(-6, 6, 2000),
                        np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8), 0.0, -0.0, 65504.0])])
    ref = torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(net.bf16(a), ref)
    assert net.bf16(np.array([1.0 + 2 ** -8]))[0] == 1.0          # tie to even
    assert net.bf16(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6


def test_identity_network_reproduces_scaled_residual():
    """A hand-set network computing relu(x) - relu(-x) = x gives z = s * r on every grid."""
    from workloads import config_c5, random_vector
    from oracle.operator import Problem
    P = Problem(config_c5(L=3))
    theta = np.zeros(net.NCONV * net.CONV_PARAMS)
    convs = [[np.zeros((9, net.C, net.C)), np.zeros(net.C)] for _ in range(net.NCONV)]
    centre = 4
    convs[0][0][centre, 0, 0], convs[0][0][centre, 1, 0] = 1.0, -1.0   # x-conv: split signs
    for c in range(1, 6):
        convs[c][0][centre, 0, 0] = convs[c][0][centre, 1, 1] = 1.0    # pass-through
    convs[6][0][centre, 0, 0] = convs[6][0][centre, 1, 1] = 1.0
    convs[7][0][centre, 0, 0], convs[7][0][centre, 0, 1] = 1.0, -1.0   # recombine
    for c in range(net.NCONV):
        theta[c * net.CONV_PARAMS:(c + 1) * net.CONV_PARAMS] = np.concatenate([convs[c][0].ravel(), convs[c][1]])
    r = random_vector(P.ndof, 3)[0]
    G = len(P.upper)
    scales = np.linspace(0.5, 2.0, G)
    z = net.apply_learned(P, [theta] * G, scales, r)
    ref = np.concatenate([s * b.ravel() for s, b in zip(scales, P.split(r))])
    assert np.allclose(z, ref, rtol=1e-14, atol=1e-14)
