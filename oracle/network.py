"""The learned correction of the preconditioner, written out plainly (NumPy).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's preconditioner (Algorithm 1's body, Sect. 4.3) maps the residual
of every upper component grid l to a correction on the same grid: the
residual of the lower grid (lx-1, lv) is the x-restriction of r_l itself, so
the CT correction of grid l depends on r_l alone.  The learned form replaces
that per-grid map by a small network N_l per upper grid of a 4D (d = 2)
problem, trained on pairs (r_l, P_CT r_l) that the CT-preconditioned solver
produces:

    z_l = s_l * rms(r_l) * N_l(r_l / rms(r_l)),   rms(r) = ||r||_2 / sqrt(#entries),

with a per-grid output scale s_l taken from the training pairs.

Network (per grid, C = 32 channels; the R time slices are the input and the
output channels, zero-padded to C):
    4 layers, each a 3x3 convolution over the x-plane (x1, x2) followed by a
    3x3 convolution over the v-plane (v1, v2), each with a bias; ReLU after
    the v-convolution of layers 1-3, none after the last.
    Padding: periodic along a periodic domain's axes, zeros otherwise.
Convolution (correlation form), for the x-plane:
    out[x1, x2, v, co] = b[co] + sum_{a, b in {-1,0,1}} sum_ci
                         W[(a+1)*3 + (b+1), co, ci] * h[x1 + a, x2 + b, v, ci]
and likewise over (v1, v2) for the v-plane.  A grid's tensor is
h[x1, x2, v1, v2, c]; its row-major point order (x1, x2, v1, v2) is the
point order x * n_v + v of the grid's coefficient block.

The accelerator stores activations and weights in bfloat16 and accumulates in
FP32; with bf16=True every function here rounds the same quantities to
bfloat16 (round to nearest, ties to even) at the same places and computes
everything else in FP64, so the two differ only by accumulation order.

Parity: pinned by the tests (delta kernels give shifts; single-channel
convolution equals scipy.ndimage.correlate in 'wrap' and 'constant' modes;
the adjoint identity <conv x, y> = <x, conv^T y>; central finite differences
of the loss; the first Adam step equals -lr * sign(g); bfloat16 rounding
equals torch's conversion).
"""
from __future__ import annotations

import numpy as np

C = 32
NCONV = 8          # 4 layers x (x-plane, v-plane)
TAPS = 9
CONV_PARAMS = TAPS * C * C + C


# ----------------------------------------------------------------- bf16 --
def bf16(a):
    """Round FP32/FP64 values to bfloat16 (round to nearest, ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(f)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


# ---------------------------------------------------------- convolution --
def _shift(h, axes, off, periodic):
    """g[i] = h[i + off] along the two axes; zero outside unless periodic."""
    g = h
    for ax, o in zip(axes, off):
        if o == 0:
            continue
        if periodic:
            g = np.roll(g, -o, axis=ax)
        else:
            out = np.zeros_like(g)
            n = g.shape[ax]
            src = [slice(None)] * g.ndim
            dst = [slice(None)] * g.ndim
            if o > 0:
                src[ax], dst[ax] = slice(o, n), slice(0, n - o)
            else:
                src[ax], dst[ax] = slice(0, n + o), slice(-o, n)
            out[tuple(dst)] = g[tuple(src)]
            g = out
    return g


def _axes(plane):
    return (0, 1) if plane == "x" else (2, 3)


def conv(h, W, b, plane, periodic):
    """h: [X1, X2, V1, V2, Cin]; W: [9, Cout, Cin]; b: [Cout]."""
    axes = _axes(plane)
    out = np.zeros(h.shape[:4] + (W.shape[1],))
    for t in range(TAPS):
        a, bb = t // 3 - 1, t % 3 - 1
        out += _shift(h, axes, (a, bb), periodic) @ W[t].T
    return out + b


def conv_adjoint(dz, W, plane, periodic):
    """Adjoint of conv's linear part in h: dh = sum_t shift_{-t}(dz) W_t (scatter of the gather)."""
    axes = _axes(plane)
    dh = np.zeros(dz.shape[:4] + (W.shape[2],))
    for t in range(TAPS):
        a, bb = t // 3 - 1, t % 3 - 1
        dh += _shift(dz @ W[t], axes, (-a, -bb), periodic)
    return dh


def conv_weight_grad(h, dz, plane, periodic):
    """dL/dW[t, co, ci] = sum_points dz[p, co] h[p + t, ci];  dL/db = sum_points dz."""
    axes = _axes(plane)
    dW = np.zeros((TAPS, dz.shape[-1], h.shape[-1]))
    dzf = dz.reshape(-1, dz.shape[-1])
    for t in range(TAPS):
        a, bb = t // 3 - 1, t % 3 - 1
        hs = _shift(h, axes, (a, bb), periodic).reshape(-1, h.shape[-1])
        dW[t] = dzf.T @ hs
    return dW, dzf.sum(axis=0)


# -------------------------------------------------------------- network --
def unpack_params(theta):
    """Flat parameter vector of one grid -> [(W [9, C, C], b [C])] * 8 (x-plane, v-plane per layer)."""
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.size == NCONV * CONV_PARAMS
    out = []
    for c in range(NCONV):
        blk = theta[c * CONV_PARAMS:(c + 1) * CONV_PARAMS]
        out.append((blk[:TAPS * C * C].reshape(TAPS, C, C), blk[TAPS * C * C:]))
    return out


def forward(theta, x, xper, vper, bf16_path=False, keep=False):
    """x: [X1, X2, V1, V2, R] network input (R <= C).  Returns y [X1, X2, V1, V2, C]
    (and the saved tensors with keep=True)."""
    rnd = bf16 if bf16_path else (lambda a: np.asarray(a, dtype=np.float64))
    params = unpack_params(theta)
    h = np.zeros(x.shape[:4] + (C,))
    h[..., :x.shape[-1]] = x
    h = rnd(h)
    saved = []
    y = None
    for k in range(4):
        Wx, bx = params[2 * k]
        Wv, bv = params[2 * k + 1]
        t = rnd(conv(h, rnd(Wx), bx, "x", xper))
        z = conv(t, rnd(Wv), bv, "v", vper)
        saved.append((h, t))
        if k < 3:
            h = rnd(np.maximum(z, 0.0))
        else:
            y = z
    return (y, saved) if keep else y


def backward(theta, x, dy, xper, vper, bf16_path=False):
    """Gradient of <y, dy> with respect to the flat parameters and to x."""
    rnd = bf16 if bf16_path else (lambda a: np.asarray(a, dtype=np.float64))
    params = unpack_params(theta)
    y, saved = forward(theta, x, xper, vper, bf16_path, keep=True)
    grads = [None] * NCONV
    d = np.asarray(dy, dtype=np.float64)
    for k in range(3, -1, -1):
        Wx, _ = params[2 * k]
        Wv, _ = params[2 * k + 1]
        h, t = saved[k]
        if k < 3:
            hn = saved[k + 1][0]               # this layer's ReLU output
            d = d * (hn > 0)
        dz = rnd(d)
        gWv, gbv = conv_weight_grad(t, dz, "v", vper)
        dt = rnd(conv_adjoint(dz, rnd(Wv), "v", vper))
        gWx, gbx = conv_weight_grad(h, dt, "x", xper)
        d = conv_adjoint(dt, rnd(Wx), "x", xper)
        grads[2 * k] = (gWx, gbx)
        grads[2 * k + 1] = (gWv, gbv)
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return flat, d[..., :x.shape[-1]]


def loss_and_grad(y, target, R):
    """Mean squared error over the first R channels of one (sample, grid):
    l = sum (y - t)^2 / (points * R);  returns l and dl/dy."""
    npts = int(np.prod(y.shape[:4]))
    diff = np.zeros_like(y)
    diff[..., :R] = y[..., :R] - target
    return float((diff ** 2).sum() / (npts * R)), 2.0 * diff / (npts * R)


def adam_step(theta, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1); step counts from 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------ grid <-> tensor --
def grid_dims(w, lx, lv):
    """Nodes per axis of the x- and v-lattices of grid (lx, lv) of a d = 2 workload."""
    mx = 2 ** lx if w.x.periodic else 2 ** lx + 1
    mv = 2 ** lv if w.v.periodic else 2 ** lv + 1
    return mx, mv


def block_to_tensor(block, mx, mv):
    """Coefficient block [R][nx][nv] -> tensor [X1, X2, V1, V2, R]."""
    R = block.shape[0]
    return np.moveaxis(block.reshape(R, mx, mx, mv, mv), 0, -1)


def tensor_to_block(t, R):
    mx, mv = t.shape[0], t.shape[2]
    return np.moveaxis(t[..., :R], -1, 0).reshape(R, mx * mx, mv * mv)


def rms(a):
    a = np.asarray(a, dtype=np.float64)
    return np.sqrt((a * a).sum() / a.size)


def apply_learned(P, thetas, scales, r, bf16_path=False):
    """z = P_learned r on every upper grid of problem P (d = 2)."""
    w = P.w
    out = []
    for (lx, lv), rb, theta, s in zip(P.upper, P.split(r), thetas, scales):
        mx, mv = grid_dims(w, lx, lv)
        nrm = rms(rb)
        if nrm == 0.0:
            out.append(np.zeros(rb.size))
            continue
        x = block_to_tensor(rb / nrm, mx, mv)
        if bf16_path:
            x = bf16(x)
        y = forward(theta, x, w.x.periodic, w.v.periodic, bf16_path)
        out.append((s * nrm * tensor_to_block(y, rb.shape[0])).ravel())
    return np.concatenate(out)
