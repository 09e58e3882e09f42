"""The FP64 reference of the pair-energy network pinned by central finite differences
(CPU only): its back-propagated gradient equals the derivative of its own loss."""
import numpy as np

import mlp_reference as ref


def _blob(rng):
    _, npar = ref.layout()
    head = np.zeros(64, dtype=np.float32)
    head[:2] = np.frombuffer(np.array([0x4D4C5031, 1], dtype=np.uint32).tobytes(), dtype=np.float32)
    head[8:24] = rng.standard_normal(16).astype(np.float32)
    head[24:40] = (0.5 + rng.random(16)).astype(np.float32)
    head[40], head[41] = 0.3, 2.0
    # weights exactly representable in BF16 so that the rounding is the identity near them
    w = ref.bf16(rng.standard_normal(npar).astype(np.float32) * 0.2).astype(np.float32)
    return np.concatenate([head, w]).tobytes()


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(7)
    blob = _blob(rng)
    X = rng.standard_normal((9, 16))
    y = rng.standard_normal(9)
    _, g = ref.loss_grad(blob, X, y)
    net = ref.unpack(blob)
    p0 = net["params"]
    offs, npar = ref.layout()
    # biases everywhere, and a sample of weights of every layer (the BF16 rounding is
    # piecewise constant in the weights, so biases and the output layer take the check
    # with the weights' rounding held fixed: perturb the biases, and compare the weights'
    # gradient with the derivative with respect to the rounded value)
    picks = []
    for (ow, ob), din, dout in zip(offs, ref.DIN, ref.DOUT):
        picks += list(range(ob, ob + dout, max(1, dout // 5)))
    h = 1e-6
    for k in picks:
        e = np.zeros(npar)
        e[k] = h
        fd = (ref.loss(blob, X, y, p0 + e) - ref.loss(blob, X, y, p0 - e)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 + 1e-6 * abs(fd), (k, fd, g[k])
    # weights: the loss as a function of the rounded weight value (replace W by W + e in a
    # copy where bf16 is bypassed by construction: the perturbed value itself is the rounding)
    orig = ref.bf16
    try:
        ref.bf16 = lambda w: np.asarray(w, dtype=np.float64)
        for (ow, ob), din, dout in zip(offs, ref.DIN, ref.DOUT):
            for k in range(ow, ow + dout * din, max(1, dout * din // 7)):
                e = np.zeros(npar)
                e[k] = h
                fd = (ref.loss(blob, X, y, p0 + e) - ref.loss(blob, X, y, p0 - e)) / (2 * h)
                assert abs(fd - g[k]) <= 1e-7 + 1e-6 * abs(fd), (k, fd, g[k])
    finally:
        ref.bf16 = orig


def test_bf16_rounding():
    """Round to nearest even on the upper 16 bits: ties go to the even BF16 value."""
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -9, -2.5], dtype=np.float32)
    got = ref.bf16(x)
    assert list(got) == [1.0, 1.0, 1.0 + 2.0 ** -6, 1.0, -2.5]
