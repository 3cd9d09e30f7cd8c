"""Pins of the learned-solver oracle against definitions, a library routine,
finite differences and closed forms (CPU only)."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import learned_oracle as lo


def rnd(seed, *shape):
    return np.random.default_rng(seed).standard_normal(shape)


def test_conv3x3_matches_correlate2d():
    x, w, b = rnd(1, 2, 3, 6, 5), rnd(2, 4, 3, 3, 3), rnd(3, 4)
    out = lo.conv3x3(x, w, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(correlate2d(x[n, c], w[o, c], mode="same") for c in range(3))
            assert np.allclose(out[n, o], ref, rtol=1e-13, atol=1e-13)


def fd(f, v, idx, h=1e-6):
    old = v[idx]
    v[idx] = old + h
    fp = f()
    v[idx] = old - h
    fm = f()
    v[idx] = old
    return (fp - fm) / (2 * h)


def test_conv3x3_backward_by_finite_differences():
    x, w, b = rnd(4, 2, 3, 5, 4), rnd(5, 4, 3, 3, 3), rnd(6, 4)
    gout = rnd(7, 2, 4, 5, 4)
    f = lambda: float(np.sum(gout * lo.conv3x3(x, w, b)))
    gx, gw, gb = lo.conv3x3_backward(x, w, gout)
    for idx in [(0, 0, 0, 0), (1, 2, 4, 3), (0, 1, 2, 1), (1, 0, 0, 3)]:
        assert abs(fd(f, x, idx) - gx[idx]) < 1e-7
    for idx in [(0, 0, 0, 0), (3, 2, 2, 2), (1, 1, 0, 2), (2, 0, 1, 1)]:
        assert abs(fd(f, w, idx) - gw[idx]) < 1e-7
    for o in range(4):
        assert abs(fd(f, b, (o,)) - gb[o]) < 1e-7


def tiny_params(seed, c=2, width=3, depth=5):
    chans = [c] + [width] * (depth - 1) + [c]
    return [(rnd(seed + k, chans[k + 1], chans[k], 3, 3) * 0.5, rnd(seed + 50 + k, chans[k + 1]) * 0.1)
            for k in range(depth)]


def test_cnn_backward_by_finite_differences():
    params = tiny_params(10)
    x = rnd(8, 2, 2, 5, 4)
    gout = rnd(9, 2, 2, 5, 4)
    f = lambda: float(np.sum(gout * lo.cnn_forward(x, params)[0]))
    _, acts = lo.cnn_forward(x, params)
    gx, grads = lo.cnn_backward(acts, params, gout)
    for idx in [(0, 0, 0, 0), (1, 1, 4, 3), (0, 1, 2, 2)]:
        assert abs(fd(f, x, idx) - gx[idx]) < 1e-6
    for k in range(5):
        w, b = params[k]
        for idx in [(0, 0, 0, 0), (w.shape[0] - 1, w.shape[1] - 1, 2, 1), (0, w.shape[1] - 1, 1, 2)]:
            assert abs(fd(f, w, idx) - grads[k][0][idx]) < 1e-6
        assert abs(fd(f, b, (0,)) - grads[k][1][0]) < 1e-6


def tiny_system(seed, shape=(1, 1, 4, 3), cond=5.0):
    """A dense Hermitian positive definite stand-in for A^H A on a tiny
    multi-shot k-space (eigenvalues in [1, cond])."""
    n = int(np.prod(shape))
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    m = (q * np.linspace(1.0, cond, n)) @ q.conj().T
    apply = lambda v: (m @ v.reshape(-1)).reshape(shape)
    b = (rng.standard_normal(n) + 1j * rng.standard_normal(n)).reshape(shape)
    return m, apply, b


def test_dc_solve_matches_dense_solve():
    m, apply, b = tiny_system(20)
    z = b * 0.3 + 0.1
    mu = 0.7
    x = lo.dc_solve(apply, b, z, mu, n_cg=60)
    ref = np.linalg.solve(m + mu * np.eye(m.shape[0]), (b + mu * z).reshape(-1)).reshape(b.shape)
    assert np.allclose(x, ref, rtol=1e-12, atol=1e-12)


def test_zero_network_converges_to_least_squares():
    """With C = 0 the iteration is the proximal point method on ||A x - y||^2,
    whose limit is the least-squares solution (A^H A)^-1 A^H y."""
    m, apply, b = tiny_system(21)
    params = [(np.zeros_like(w), np.zeros_like(bb)) for w, bb in tiny_params(30)]
    x, _ = lo.unrolled_forward(b, apply, params, mu=0.5, n_unroll=120, n_cg=60)
    ref = np.linalg.solve(m, b.reshape(-1)).reshape(b.shape)
    assert np.allclose(x, ref, rtol=1e-10, atol=1e-10)


def test_unrolled_gradients_by_finite_differences():
    """With exact data-consistency solves the backward pass is the exact
    gradient of the loss."""
    m, apply, b = tiny_system(22, shape=(1, 1, 4, 3))
    params = tiny_params(40)
    target = b * 0.8 + 0.05j
    mu, K, n_cg = 0.9, 2, 80
    f = lambda: lo.loss_value(lo.unrolled_forward(b, apply, params, mu, K, n_cg)[0], target)
    loss, grads = lo.unrolled_loss_and_grads(b, apply, params, mu, K, n_cg, target)
    assert abs(loss - f()) < 1e-14
    for k in (0, 2, 4):
        w, bb = params[k]
        for idx in [(0, 0, 1, 1), (w.shape[0] - 1, w.shape[1] - 1, 0, 2)]:
            assert abs(fd(f, w, idx) - grads[k][0][idx]) < 1e-7 * max(1.0, abs(grads[k][0][idx]))
        assert abs(fd(f, bb, (0,)) - grads[k][1][0]) < 1e-7 * max(1.0, abs(grads[k][1][0]))


def test_pack_unpack_round_trip():
    x = rnd(50, 2, 3, 4, 5) + 1j * rnd(51, 2, 3, 4, 5)
    c = lo.pack(x, 2.5)
    assert c.shape == (2, 6, 4, 5)
    assert np.allclose(c[:, 2], x[:, 1].real / 2.5) and np.allclose(c[:, 3], x[:, 1].imag / 2.5)
    assert np.allclose(lo.unpack(c, 2.5), x, rtol=1e-15, atol=0)


def test_zero_data_gives_zero():
    """b = 0: x = 0 solves every data-consistency step exactly, whatever the
    network (its term is scaled by s = 0)."""
    m, apply, b = tiny_system(23)
    params = tiny_params(60)           # nonzero biases: C(0) != 0
    x, _ = lo.unrolled_forward(np.zeros_like(b), apply, params, mu=0.5, n_unroll=3, n_cg=20)
    assert np.all(x == 0)


def test_bf16_rounding_closed_forms():
    # exactly representable values are unchanged
    v = np.array([1.0, -2.5, 0.15625, 3.0 * 2 ** -20, 0.0], dtype=np.float32)
    assert np.array_equal(lo.bf16_round(v), v.astype(np.float64))
    # ties to even at the 8-bit significand: 1 + 2^-8 -> 1, 1 + 3 * 2^-8 -> 1 + 2^-6
    assert lo.bf16_round(np.float32(1 + 2 ** -8)) == 1.0
    assert lo.bf16_round(np.float32(1 + 3 * 2 ** -8)) == 1 + 2 ** -6
    # above a tie rounds up, below rounds down
    assert lo.bf16_round(np.float32(1 + 2 ** -8 + 2 ** -20)) == 1 + 2 ** -7
    assert lo.bf16_round(np.float32(1 + 2 ** -8 - 2 ** -20)) == 1.0
    # relative error at most the unit roundoff of an 8-bit significand, 2^-8
    x = np.random.default_rng(3).standard_normal(10000).astype(np.float32)
    assert np.max(np.abs(lo.bf16_round(x) - x) / np.abs(x)) <= 2.0 ** -8


def bf16_exact_network(seed, c=8, depth=5):
    """A network whose activations and gradients stay short dyadic numbers
    (BF16 values): each output channel reads one input channel (a
    permutation) at one tap with weight +-1, biases in quarters."""
    rng = np.random.default_rng(seed)
    params = []
    for _ in range(depth):
        w = np.zeros((c, c, 3, 3))
        perm = rng.permutation(c)
        for o in range(c):
            a, d = rng.integers(0, 3, size=2)
            w[o, perm[o], a, d] = rng.choice([-1.0, 1.0])
        params.append((w, rng.integers(-2, 3, size=c) * 0.25))
    return params


def test_bf16_network_reduces_to_plain_on_bf16_exact_data():
    """Where every rounded quantity is already a BF16 value the BF16 network
    is the plain network: same output, input gradient and parameter
    gradients, exactly."""
    params = bf16_exact_network(21)
    rng = np.random.default_rng(22)
    x = rng.integers(-4, 5, size=(2, 8, 7, 6)).astype(np.float64)
    gout = rng.integers(-3, 4, size=(2, 8, 7, 6)).astype(np.float64)
    out, acts = lo.cnn_forward(x, params)
    out_b, acts_b = lo.cnn_forward(x, params, act_bf16=True)
    assert np.array_equal(out, out_b)
    gin, grads = lo.cnn_backward(acts, params, gout)
    gin_b, grads_b = lo.cnn_backward(acts_b, params, gout, act_bf16=True)
    assert np.array_equal(gin, gin_b)
    for (gw, gb), (gw2, gb2) in zip(grads, grads_b):
        assert np.array_equal(gw, gw2) and np.array_equal(gb, gb2)


def test_bf16_network_activations_are_bf16_values():
    """On general data every convolution input of the BF16 network is a BF16
    value (its FP32 pattern has zero low 16 bits) and the rounding changes
    the output by the BF16 unit roundoff's order, no more."""
    rng = np.random.default_rng(23)
    params = [(rng.standard_normal((8, 8, 3, 3)) * 0.3, rng.standard_normal(8) * 0.1) for _ in range(5)]
    x = rng.standard_normal((1, 8, 9, 9))
    out, _ = lo.cnn_forward(x, params)
    out_b, acts_b = lo.cnn_forward(x, params, act_bf16=True)
    for a in acts_b:
        f = a.astype(np.float32)
        assert np.array_equal(f.astype(np.float64), a)
        assert np.all((f.view(np.uint32) & 0xFFFF) == 0)
    d = np.linalg.norm(out_b - out) / np.linalg.norm(out)
    assert 1e-4 < d < 2.0 ** -6
