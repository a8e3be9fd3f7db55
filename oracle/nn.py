"""FP64 reference of the learned warm start / preconditioner network (forward and backward).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper has no learned component; this is the reference for the small 3D convolutional
network that stands beside the multigrid solver. Everything is plain NumPy in FP64, written
from the definitions:

* Tensors are channels-last, shaped (nz, ny, nx, C).
* conv3(x, W, b): 3x3x3 correlation with "same" size, periodic padding in x and y and zero
  padding in z (the solver's boundary kinds): out[v, o] = b[o] + sum_{t, c} W[o, t, c] x[v + d_t, c],
  taps t = (dz+1)*9 + (dy+1)*3 + (dx+1) for dz, dy, dx in {-1, 0, 1}.
* pool2: mean over 2x2x2 children; up2: nearest-neighbour copy to the 2x2x2 children.
* relu, concatenation along channels, a 1x1x1 output head.

Architecture (levels at n, n/2, n/4; channels 16 / 32 / 64):
    e1 = relu(conv(relu(conv(in, 4->16)), 16->16))
    e2 = relu(conv(relu(conv(pool2(e1), 16->32)), 32->32))
    e3 = relu(conv(relu(conv(pool2(e2), 32->64)), 64->64))
    d2 = relu(conv(relu(conv([up2(e3), e2], 96->32)), 32->32))
    d1 = relu(conv(relu(conv([up2(d2), e1], 48->16)), 16->16))
    y  = d1 . w_out + b_out                                     (1x1x1 head, one channel)

Parameters are a flat FP32/FP64 vector: for each of the ten 3x3x3 convolutions in the order
above, W[o, t, c] (c fastest, then t, then o) followed by b[o]; then w_out[16], b_out.
"""
from __future__ import annotations

import numpy as np

# (Cin, Cout) of the ten 3x3x3 convolutions, in parameter order
CONVS = [(4, 16), (16, 16), (16, 32), (32, 32), (32, 64), (64, 64), (96, 32), (32, 32),
         (48, 16), (16, 16)]
HEAD_IN = 16


def num_params() -> int:
    return sum(27 * ci * co + co for ci, co in CONVS) + HEAD_IN + 1


def unpack(theta: np.ndarray):
    """Split the flat parameter vector into [(W (co, 27, ci), b (co,)), ...], w_out, b_out."""
    theta = np.asarray(theta, dtype=np.float64)
    layers = []
    off = 0
    for ci, co in CONVS:
        n = 27 * ci * co
        W = theta[off:off + n].reshape(co, 27, ci)
        off += n
        b = theta[off:off + co]
        off += co
        layers.append((W, b))
    w_out = theta[off:off + HEAD_IN]
    off += HEAD_IN
    b_out = theta[off]
    return layers, w_out, b_out


def pack(layers, w_out, b_out) -> np.ndarray:
    parts = []
    for W, b in layers:
        parts += [np.asarray(W).reshape(-1), np.asarray(b).reshape(-1)]
    parts += [np.asarray(w_out).reshape(-1), np.asarray([b_out]).reshape(-1)]
    return np.concatenate(parts).astype(np.float64)


def init_params(seed: int) -> np.ndarray:
    """He-uniform initialisation (weights U(-a, a), a = sqrt(6 / fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    layers = []
    for ci, co in CONVS:
        a = np.sqrt(6.0 / (27 * ci))
        layers.append((rng.uniform(-a, a, size=(co, 27, ci)), np.zeros(co)))
    a = np.sqrt(6.0 / HEAD_IN)
    return pack(layers, rng.uniform(-a, a, size=HEAD_IN), 0.0)


def taps():
    """(dz, dy, dx) of tap t."""
    return [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def shift(x: np.ndarray, dz: int, dy: int, dx: int) -> np.ndarray:
    """s[k, j, i] = x[k + dz, j + dy, i + dx]: periodic in y, x; zero outside in z."""
    s = np.roll(x, (-dy, -dx), axis=(1, 2))
    out = np.zeros_like(s)
    nz = x.shape[0]
    if dz == 0:
        out[:] = s
    elif dz > 0:
        out[: nz - dz] = s[dz:]
    else:
        out[-dz:] = s[: nz + dz]
    return out


def conv3(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """out[v, o] = b[o] + sum_t sum_c W[o, t, c] x[v + d_t, c]."""
    out = np.zeros(x.shape[:3] + (W.shape[0],))
    for t, (dz, dy, dx) in enumerate(taps()):
        out += shift(x, dz, dy, dx) @ W[:, t, :].T
    return out + b


def conv3_backward(x: np.ndarray, W: np.ndarray, g: np.ndarray):
    """Gradients of sum(g * conv3(x, W, b)) with respect to x, W and b."""
    gx = np.zeros_like(x)
    gW = np.zeros_like(W)
    for t, (dz, dy, dx) in enumerate(taps()):
        xs = shift(x, dz, dy, dx)
        gW[:, t, :] = np.einsum("kjio,kjic->oc", g, xs)
        # adjoint of the shift: out[v] receives x[v + d] -> x[u] receives g[u - d]
        gx += shift(g @ W[:, t, :], -dz, -dy, -dx)
    gb = g.sum(axis=(0, 1, 2))
    return gx, gW, gb


def pool2(x: np.ndarray) -> np.ndarray:
    nz, ny, nx, c = x.shape
    return x.reshape(nz // 2, 2, ny // 2, 2, nx // 2, 2, c).mean(axis=(1, 3, 5))


def pool2_backward(g: np.ndarray) -> np.ndarray:
    return up2(g) / 8.0


def up2(x: np.ndarray) -> np.ndarray:
    return x.repeat(2, axis=0).repeat(2, axis=1).repeat(2, axis=2)


def up2_backward(g: np.ndarray) -> np.ndarray:
    return 8.0 * pool2(g)


def forward(theta: np.ndarray, inp: np.ndarray, keep: bool = False, bf16: bool = False):
    """y (nz, ny, nx) from inp (nz, ny, nx, 4). With keep, also the activations for backward.

    bf16=True rounds to bfloat16 where a bfloat16 pipeline stores values: the input features,
    the convolution weights (not the biases or the head), every convolution output after the
    ReLU and every pooled tensor. The arithmetic itself stays FP64.
    """
    R = bf16_round if bf16 else (lambda a: a)
    layers, w_out, b_out = unpack(theta)
    if bf16:
        layers = [(R(W), b) for W, b in layers]
    acts = {}

    def cr(name, x, li):
        W, b = layers[li]
        pre = conv3(x, W, b)
        out = R(np.maximum(pre, 0.0))
        acts[name] = (x, out)
        return out

    inp = R(inp)
    e1 = cr("c1", cr("c0", inp, 0), 1)
    p1 = R(pool2(e1))
    e2 = cr("c3", cr("c2", p1, 2), 3)
    p2 = R(pool2(e2))
    e3 = cr("c5", cr("c4", p2, 4), 5)
    u3 = np.concatenate([up2(e3), e2], axis=-1)
    d2 = cr("c7", cr("c6", u3, 6), 7)
    u2 = np.concatenate([up2(d2), e1], axis=-1)
    d1 = cr("c9", cr("c8", u2, 8), 9)
    y = d1 @ w_out + b_out
    if keep:
        acts["d1"] = d1
        acts["layers"] = layers
        acts["bf16"] = bf16
        return y, acts
    return y


def backward(theta: np.ndarray, acts, gy: np.ndarray) -> np.ndarray:
    """Gradient of sum(gy * y) with respect to the flat parameters.

    When the forward pass rounded to bfloat16, the masked gradient at each convolution output
    (the operand of both backward convolutions) is rounded too; bias gradients use it unrounded.
    """
    _, w_out, b_out = unpack(theta)
    layers = acts["layers"]
    R = bf16_round if acts["bf16"] else (lambda a: a)
    grads = [None] * len(CONVS)
    d1 = acts["d1"]
    g_wout = np.einsum("kji,kjic->c", gy, d1)
    g_bout = gy.sum()
    g = gy[..., None] * w_out

    def back(name, li, g_out):
        x, out = acts[name]
        pre = g_out * (out > 0)
        gx, gW, _ = conv3_backward(x, layers[li][0], R(pre))
        grads[li] = (gW, pre.sum(axis=(0, 1, 2)))
        return gx

    g = back("c8", 8, back("c9", 9, g))               # -> gradient of u2 (48 ch)
    g_up, g_e1 = g[..., :32], g[..., 32:]
    g = back("c6", 6, back("c7", 7, up2_backward(g_up)))   # -> gradient of u3 (96 ch)
    g_up3, g_e2 = g[..., :64], g[..., 64:]
    g = back("c4", 4, back("c5", 5, up2_backward(g_up3)))  # -> gradient of p2
    g_e2 = g_e2 + pool2_backward(g)
    g = back("c2", 2, back("c3", 3, g_e2))                 # -> gradient of p1
    g_e1 = g_e1 + pool2_backward(g)
    back("c0", 0, back("c1", 1, g_e1))
    return pack(grads, g_wout, g_bout)


def loss_and_grad(theta, inp, target, bf16: bool = False):
    """Mean squared error over voxels and its parameter gradient."""
    y, acts = forward(theta, inp, keep=True, bf16=bf16)
    diff = y - target
    nvox = diff.size
    loss = float(np.sum(diff * diff) / nvox)
    return loss, backward(theta, acts, 2.0 * diff / nvox)


def adam_step(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba) with bias correction; t counts from 1."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mhat = m / (1 - beta1 ** t)
    vhat = v / (1 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def features(b, rho, c2, p_prev):
    """Network input (nz, ny, nx, 4) and the right-hand-side scale s = RMS(b).

    Channels: b / s, log rho, log c2, p_prev / s.
    """
    b = np.asarray(b, dtype=np.float64)
    s = float(np.sqrt(np.mean(b * b)))
    s = s if s > 0 else 1.0
    inp = np.stack([b / s, np.log(rho), np.log(c2), np.asarray(p_prev) / s], axis=-1)
    return inp, s


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round FP64 values to the nearest bfloat16 (ties to even), returned as FP64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
