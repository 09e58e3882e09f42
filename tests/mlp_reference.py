"""FP64 reference of the pair-energy network (tests only): forward pass, mean squared
error of standardised targets and its gradient by back-propagation, written from the
definitions of a dense network with exact-erf GELU.  It reads the library's weights blob
(header of 64 floats: magic, version, sizes; feature mean at [8:24], standard deviation at
[24:40], target mean and standard deviation at [40], [41]; then W_l [dout][din] and b_l per
layer) and applies the same BF16 rounding (nearest even) to the weights."""
import math

import numpy as np
from scipy.special import erf

DIN = (16, 128, 128, 128)
DOUT = (128, 128, 128, 1)
HEADER = 64


def layout():
    offs, o = [], 0
    for din, dout in zip(DIN, DOUT):
        offs.append((o, o + dout * din))
        o += dout * din + dout
    return offs, o


def bf16(w):
    u = np.ascontiguousarray(w, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


def unpack(blob):
    f = np.frombuffer(bytes(blob), dtype=np.float32)
    offs, n = layout()
    p = f[HEADER:HEADER + n].astype(np.float64)
    Ws, bs = [], []
    for (ow, ob), din, dout in zip(offs, DIN, DOUT):
        Ws.append(p[ow:ow + dout * din].reshape(dout, din))
        bs.append(p[ob:ob + dout])
    return dict(mean=f[8:24].astype(np.float64), sd=f[24:40].astype(np.float64),
                ym=float(f[40]), ys=float(f[41]), W=Ws, b=bs, params=p)


def pack(blob, params):
    """The blob with its parameters replaced (FP32)."""
    f = np.frombuffer(bytes(blob), dtype=np.float32).copy()
    f[HEADER:HEADER + len(params)] = np.asarray(params, dtype=np.float32)
    return f.tobytes()


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(net, X, params=None):
    """Pre-activations, activations and the output (standardised scale)."""
    Ws, bs = net["W"], net["b"]
    if params is not None:
        offs, _ = layout()
        Ws = [params[ow:ow + dout * din].reshape(dout, din) for (ow, _), din, dout in zip(offs, DIN, DOUT)]
        bs = [params[ob:ob + dout] for (_, ob), dout in zip(offs, DOUT)]
    a = (np.asarray(X, dtype=np.float64) - net["mean"]) / net["sd"]
    xs, zs, acts = [a], [], []
    for l, (W, b) in enumerate(zip(Ws, bs)):
        z = a @ bf16(W).T + b
        a = gelu(z) if l + 1 < len(Ws) else z
        zs.append(z)
        acts.append(a)
        xs.append(a)
    return xs, zs, a[:, 0]


def predict(blob, X):
    net = unpack(blob)
    return forward(net, X)[2] * net["ys"] + net["ym"]


def loss(blob, X, y, params=None):
    net = unpack(blob)
    ys = (np.asarray(y, dtype=np.float64) - net["ym"]) / net["ys"]
    out = forward(net, X, params)[2]
    return float(np.mean((out - ys) ** 2))


def loss_grad(blob, X, y):
    """Loss and its gradient with respect to the parameters (the gradient of the BF16-rounded
    weights is taken as that of the master weights, as the training kernels do)."""
    net = unpack(blob)
    n = len(y)
    ys = (np.asarray(y, dtype=np.float64) - net["ym"]) / net["ys"]
    xs, zs, out = forward(net, X)
    d = (2.0 * (out - ys) / n)[:, None]
    offs, npar = layout()
    g = np.zeros(npar)
    L = len(DIN)
    for l in range(L - 1, -1, -1):
        (ow, ob), din, dout = offs[l], DIN[l], DOUT[l]
        g[ow:ow + dout * din] = (d.T @ xs[l]).ravel()
        g[ob:ob + dout] = d.sum(axis=0)
        if l == 0:
            break
        da = d @ bf16(net["W"][l])
        d = da * gelu_grad(zs[l - 1])
    return float(np.mean((out - ys) ** 2)), g
