"""Why the kernels compute in FP64: the IRLS iteration amplifies rounding.

The oracle's own solve of the 64 x 64 workload is run with its operators
perturbed the way lower precision would perturb them, and compared with the
unperturbed FP64 solve (the NRMSE target of the GPU path is 1e-5):
  * the normal operator and the weights evaluated in FP32 arithmetic (complex64
    FFTs, coil products and sums, Hankel products, single-precision eigh)
    miss 1e-5; rounding only their results to complex64 (storage in FP32,
    arithmetic exact) already uses most of the budget (~6.5e-6);
  * relative noise delta injected into each normal-operator application gives
    an NRMSE of order 100-300 delta, so FP32 rounding (delta ~ 6e-8) sits at
    the target's edge before any arithmetic error is counted, while FP64
    rounding (delta ~ 1e-16) is far inside it.
The amplification comes from the weights: dW / W ~ dG / (2 eps) with eps
falling to 1e-4 of lambda_max.
"""
import numpy as np
import pytest

from oracle import smsm_oracle as o
from tests.helpers import case_for, oracle_params


@pytest.fixture(scope="module")
def small():
    g, case, _, y = case_for("small", 0)
    y = y.astype(np.complex128)
    ref = o.solve(y, case["coils"], case["masks"], case["shifts"], oracle_params(g))
    return g, case, y, ref


def solve_with(monkeypatch, small, normal=None, weight=None):
    g, case, y, ref = small
    with monkeypatch.context() as m:
        if normal is not None:
            m.setattr(o, "normal_op", normal)
        if weight is not None:
            m.setattr(o, "irls_weight", weight)
        x = o.solve(y, case["coils"], case["masks"], case["shifts"], oracle_params(g))
    return o.nrmse(x, ref)


AX = (-2, -1)


def fft2c32(u):
    return np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(u, axes=AX), norm="ortho"), axes=AX)


def ifft2c32(k):
    return np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(k, axes=AX), norm="ortho"), axes=AX)


def normal_f32(v, coils, masks, theta, W, lam, r):
    """N(v) of the oracle's definition evaluated in complex64 arithmetic
    throughout (FFTs, coil products and sums, Hankel products and sums)."""
    c = np.complex64
    v, S, th = v.astype(c), coils.astype(c), theta.astype(c)
    L, Ns, n2, n1 = v.shape
    out = np.zeros_like(v)
    for i in range(Ns):
        m = masks[i].astype(np.float32)[:, None]
        img = [ifft2c32(v[l, i]) for l in range(L)]
        for cc in range(S.shape[1]):
            k = m * sum(th[l][:, None] * fft2c32(S[l, cc] * img[l]) for l in range(L))
            for l in range(L):
                out[l, i] += fft2c32(np.conj(S[l, cc]) * ifft2c32(np.conj(th[l])[:, None] * k))
    P2, P1 = n2 - r + 1, n1 - r + 1
    for l in range(L):
        if W[l] is None:
            continue
        Z = (o.hankel(v[l], r).astype(c) @ W[l].astype(c)).astype(c)
        for i in range(Ns):
            for b2 in range(r):
                for b1 in range(r):
                    out[l, i, b2:b2 + P2, b1:b1 + P1] += np.float32(0.5 * lam) * \
                        Z[:, (i * r + b2) * r + b1].reshape(P2, P1)
    return out.astype(np.complex128)


def weight_f32(G, eps):
    """The oracle's weight definition with the eigendecomposition in single precision."""
    s, V = np.linalg.eigh(G.astype(np.complex64))
    f = (1.0 / np.sqrt(np.maximum(s, 0.0) + np.float32(eps))).astype(np.float32)
    return ((V * f[None, :]) @ V.conj().T).astype(np.complex128)


def test_fp32_arithmetic_misses_the_target(monkeypatch, small):
    err = solve_with(monkeypatch, small, normal_f32, weight_f32)
    print(f"normal operator and weights in FP32 arithmetic: NRMSE {err:.2e}")
    assert err > 1e-5


def test_complex64_storage_alone_is_near_the_target(monkeypatch, small):
    """Rounding only the operator results and weights to complex64 (exact
    arithmetic otherwise) already costs about 6.5e-6 of the 1e-5 budget."""
    exact_normal, exact_weight = o.normal_op, o.irls_weight
    c64 = lambda a: np.asarray(a).astype(np.complex64).astype(np.complex128)

    def normal(v, coils, masks, theta, W, lam, r):
        Wc = [None if w is None else c64(w) for w in W]
        return c64(exact_normal(c64(v), coils, masks, theta, Wc, lam, r))

    def weight(G, eps):
        return c64(exact_weight(c64(G), eps))

    err = solve_with(monkeypatch, small, normal, weight)
    print(f"complex64 storage of operator results and weights: NRMSE {err:.2e}")
    assert 1e-6 < err < 1e-5


@pytest.mark.parametrize("delta", [1e-7, 1e-6])
def test_operator_noise_is_amplified(monkeypatch, small, delta):
    exact_normal = o.normal_op
    rng = np.random.default_rng(5)

    def normal(v, coils, masks, theta, W, lam, r):
        out = exact_normal(v, coils, masks, theta, W, lam, r)
        xi = rng.standard_normal(out.shape) + 1j * rng.standard_normal(out.shape)
        return out * (1.0 + delta * xi / np.sqrt(2.0))

    err = solve_with(monkeypatch, small, normal)
    print(f"relative operator noise {delta:.0e}: NRMSE {err:.2e} ({err / delta:.0f} x delta)")
    assert 30 * delta < err < 1000 * delta
