"""Plain FP64 CPU oracle of the SMS-MUSSELS IRLS solve.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this module.  The GPU library never
calls it and shares no code with it.

What it computes (Mani et al., "SMS MUSSELS", arXiv 1901.01893):
  * the SMS forward operator A of Fig. 1: inverse 2-D DFT of each slice/shot
    k-space, multiply by the slice's coil sensitivities, forward 2-D DFT,
    blipped-CAIPI phase per slice (Theory, Eq. 1 and its multi-shot form
    Eq. 3) summed over the simultaneously excited slices, and the shot's
    interleaved ky sampling mask (Eq. 2);
  * the block-Hankel lift H_l of each slice (Theory, Eq. 8-9): valid r x r
    patches only, (N1-r+1)(N2-r+1) rows per shot, shots side by side;
  * the objective of Eq. 10, ||A x - y||^2 + lam sum_l ||H_l(x)||_*, minimised
    by iteratively reweighted least squares (IRLS) with a fixed schedule:
    W_l = (H_l^H H_l + eps_l I)^(-1/2) from a dense Hermitian eigensolver, and
    conjugate gradients on the normal equations
        N(x) = A^H A x + (lam/2) sum_l H_l^H(H_l(x_l) W_l) = A^H y.
    The paper solved Eq. 10 with an augmented Lagrangian scheme whose steps it
    does not print; IRLS is the majorise-minimise method for the same
    objective, and the factor lam/2 follows from majorising the concave
    t -> sqrt(t) at the current Gram eigenvalues.

  * the root-sum-of-squares image of each slice over its shots' images (the
    paper compares against single-band images without saying how shots are
    combined; pinned by Parseval, a unit-modulus-phase closed form and a
    k-space delta).

Pins: every operator above, the weights, one CG step, the lam = 0 solve and
the monotone decrease of the smoothed objective are checked against
definitions, closed forms and brute force in tests/test_oracle_pins.py.  The
whole solve is pinned in tests/test_oracle_solve_pins.py: it equals a dense
brute-force IRLS written from the readings (to rounding, 2e-15), its fixed
point at a fixed eps zeroes the smoothed objective's gradient, it recovers
noiseless low-rank data that least squares cannot, and run long it reaches
the minimiser of Eq. 10 that the augmented-Lagrangian oracle certifies by the
subgradient optimality condition; ten planted mistakes each fail one of
these.  At the workload sizes the fixed-count iteration is its own reference
beyond those pins.

Readings taken where the paper is silent (every one listed in the design
notes): centred unitary DFT; CAIPI phase exp(-2 pi i s_l (j2 - N2/2)) on the
global ky index with s_l = l/L; per-slice coil maps; Hankel rows p2-major and
columns (shot, b2, b1) shot-major; eps_l = max(eps_frac eta^-k,
eps_floor_frac) * lambda_max(G_l(x0)); x0 = A^H y; CG warm-started at the
current iterate with exactly n_cg steps after the initial residual.

Arrays: k-space and images are [..., N2 (ky / y), N1 (kx / x)], x is
[L][Ns][N2][N1], y is [Ns][Nc][N2][N1] zero-filled, coil maps [L][Nc][N2][N1].
All arithmetic is complex128 / float64.
"""
from __future__ import annotations

import dataclasses
import numpy as np

_AX = (-2, -1)


# ---------------------------------------------------------------------------
# Fourier transform (Fig. 1 steps (i) and (iii))
# ---------------------------------------------------------------------------
def fft2c(u):
    """Centred unitary 2-D DFT over the last two axes (image -> k-space).

    DC sits at index N/2 in both domains; the paper fixes neither centring nor
    normalisation, unitary keeps A^H the exact adjoint.
    """
    u = np.asarray(u, dtype=np.complex128)
    return np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(u, axes=_AX), norm="ortho"), axes=_AX)


def ifft2c(k):
    """Inverse of fft2c (k-space -> image)."""
    k = np.asarray(k, dtype=np.complex128)
    return np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(k, axes=_AX), norm="ortho"), axes=_AX)


# ---------------------------------------------------------------------------
# Acquisition geometry (Theory: blipped CAIPI, Eq. 1-3)
# ---------------------------------------------------------------------------
def caipi_phase(n2: int, shifts) -> np.ndarray:
    """theta_l[j2] = exp(-2 pi i s_l (j2 - N2/2)), shape [L][N2].

    Eq. 1 modulates phase-encode line n of slice l by exp(-i n dky (l-1) 2pi/L)
    and Eq. 3 applies it on the global line index n' of each shot; read as a
    Fourier shift of slice l by s_l of the FOV with s_l = (l-1)/L, measured
    from the k-space centre so the DC line carries no phase.
    """
    s = np.asarray(shifts, dtype=np.float64)
    j2 = np.arange(n2, dtype=np.float64) - n2 / 2
    return np.exp(-2j * np.pi * s[:, None] * j2[None, :])


def interleaved_masks(n2: int, n_shots: int) -> np.ndarray:
    """M_i[j2] = 1 iff j2 = i (mod Ns): Eq. 2, line n' = (n-1) Ns + i (0-based)."""
    j2 = np.arange(n2)
    return np.stack([(j2 % n_shots) == i for i in range(n_shots)]).astype(np.float64)


# ---------------------------------------------------------------------------
# Forward operator A and its adjoint (Fig. 1; data dimensions below Eq. 10)
# ---------------------------------------------------------------------------
def forward(x, coils, masks, theta):
    """(A x)_{i,c} = M_i * sum_l theta_l * F(S_{l,c} * F^-1(x_{l,i})).

    Fig. 1: (i) inverse DFT, (ii) coil multiply, (iii) DFT, (iv) CAIPI phase and
    sum over slices per channel, (v) shot mask.
    """
    x = np.asarray(x, dtype=np.complex128)
    L, Ns, n2, n1 = x.shape
    Nc = coils.shape[1]
    y = np.zeros((Ns, Nc, n2, n1), dtype=np.complex128)
    for i in range(Ns):
        img = [ifft2c(x[l, i]) for l in range(L)]
        for c in range(Nc):
            acc = np.zeros((n2, n1), dtype=np.complex128)
            for l in range(L):
                acc += theta[l][:, None] * fft2c(coils[l, c] * img[l])
            y[i, c] = masks[i][:, None] * acc
    return y


def adjoint(y, coils, masks, theta):
    """A^H: the steps of Fig. 1 in reverse order with conjugated factors."""
    y = np.asarray(y, dtype=np.complex128)
    Ns, Nc, n2, n1 = y.shape
    L = coils.shape[0]
    x = np.zeros((L, Ns, n2, n1), dtype=np.complex128)
    for i in range(Ns):
        for l in range(L):
            acc = np.zeros((n2, n1), dtype=np.complex128)
            for c in range(Nc):
                k = np.conj(theta[l])[:, None] * masks[i][:, None] * y[i, c]
                acc += np.conj(coils[l, c]) * ifft2c(k)
            x[l, i] = fft2c(acc)
    return x


# ---------------------------------------------------------------------------
# Block-Hankel lift (Theory, Eq. 8-9)
# ---------------------------------------------------------------------------
def hankel(xl, r: int) -> np.ndarray:
    """H_l(x_l): rows = valid patch anchors (p2, p1) in [0,N2-r]x[0,N1-r], p2-major;
    columns = (shot i, b2, b1), shot-major; entry x_{l,i}[p2+b2, p1+b1].

    Eq. 8 gives each shot a (N1-r+1)(N2-r+1) x r^2 Hankel matrix built from
    its N1 x N2 Fourier samples; Eq. 9 places the shots side by side.
    """
    xl = np.asarray(xl, dtype=np.complex128)
    Ns, n2, n1 = xl.shape
    P2, P1 = n2 - r + 1, n1 - r + 1
    H = np.empty((P2 * P1, Ns * r * r), dtype=np.complex128)
    for i in range(Ns):
        for b2 in range(r):
            for b1 in range(r):
                H[:, (i * r + b2) * r + b1] = xl[i, b2:b2 + P2, b1:b1 + P1].reshape(-1)
    return H


def hankel_adjoint(Z, n_shots: int, n2: int, n1: int, r: int) -> np.ndarray:
    """H_l^H(Z): every entry of Z is added back to the k-space sample it came from."""
    P2, P1 = n2 - r + 1, n1 - r + 1
    out = np.zeros((n_shots, n2, n1), dtype=np.complex128)
    for i in range(n_shots):
        for b2 in range(r):
            for b1 in range(r):
                out[i, b2:b2 + P2, b1:b1 + P1] += Z[:, (i * r + b2) * r + b1].reshape(P2, P1)
    return out


def gram(xl, r: int) -> np.ndarray:
    """G_l = H_l^H H_l, Hermitian [Ns r^2][Ns r^2]."""
    H = hankel(xl, r)
    return H.conj().T @ H


def nuclear_norm(xl, r: int) -> float:
    """||H_l(x_l)||_* (the penalty of Eq. 10) from a dense SVD."""
    return float(np.sum(np.linalg.svd(hankel(xl, r), compute_uv=False)))


def irls_weight(G, eps: float) -> np.ndarray:
    """W = V diag((max(s,0) + eps)^(-1/2)) V^H with G = V diag(s) V^H.

    Eigenvalues are clamped at zero because rounding can leave tiny negative
    ones in a Gram matrix; W is a matrix function, so it does not depend on
    the eigenvector phases or on how repeated eigenvalues are resolved.
    eps == 0 is allowed only for a slice with G == 0, where W = 0.
    """
    s, V = np.linalg.eigh(G)
    f = 1.0 / np.sqrt(np.maximum(s, 0.0) + eps)
    return (V * f[None, :]) @ V.conj().T


def lambda_max(G) -> float:
    return float(np.linalg.eigvalsh(G)[-1])


# ---------------------------------------------------------------------------
# Objective, surrogate and normal operator
# ---------------------------------------------------------------------------
def objective(x, y, coils, masks, theta, lam, r) -> float:
    """Eq. 10: ||A x - y||^2 + lam sum_l ||H_l(x_l)||_* (squared norm, no 1/2)."""
    res = forward(x, coils, masks, theta) - y
    reg = sum(nuclear_norm(x[l], r) for l in range(x.shape[0]))
    return float(np.vdot(res, res).real + lam * reg)


def smoothed_objective(x, y, coils, masks, theta, lam, r, eps) -> float:
    """J_eps(x) = ||A x - y||^2 + lam sum_l tr((G_l + eps_l I)^(1/2))."""
    res = forward(x, coils, masks, theta) - y
    val = np.vdot(res, res).real
    for l in range(x.shape[0]):
        s = np.linalg.eigvalsh(gram(x[l], r))
        val += lam * np.sum(np.sqrt(np.maximum(s, 0.0) + eps[l]))
    return float(val)


def regulariser(x, weights, lam, r):
    """(lam/2) sum_l H_l^H(H_l(x_l) W_l), the Hankel term of the normal equations."""
    L, Ns, n2, n1 = x.shape
    out = np.zeros_like(x, dtype=np.complex128)
    for l in range(L):
        if weights[l] is None:
            continue
        Z = hankel(x[l], r) @ weights[l]
        out[l] = 0.5 * lam * hankel_adjoint(Z, Ns, n2, n1, r)
    return out


def normal_op(x, coils, masks, theta, weights, lam, r):
    """N(x) = A^H A x + (lam/2) sum_l H_l^H(H_l(x_l) W_l)."""
    return adjoint(forward(x, coils, masks, theta), coils, masks, theta) + \
        regulariser(x, weights, lam, r)


def vdot(a, b) -> complex:
    """<a, b> = sum conj(a) b in FP64."""
    return complex(np.vdot(np.asarray(a).ravel(), np.asarray(b).ravel()))


# ---------------------------------------------------------------------------
# IRLS solve
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class SolveParams:
    lam: float = 1e-3
    r: int = 5
    n_irls: int = 10
    n_cg: int = 10
    eps_frac: float = 0.1
    eps_decay: float = 1.5
    eps_floor_frac: float = 1e-4


def eps_schedule(sigma, k: int, p: SolveParams):
    """eps_l(k) = max(eps_frac * eta^-k, eps_floor_frac) * sigma_l (non-increasing)."""
    frac = max(p.eps_frac * p.eps_decay ** (-k), p.eps_floor_frac)
    return [frac * s for s in sigma]


def cg(apply_n, b, x, n_iter: int):
    """Conjugate gradients on N(x) = b warm-started at x, exactly n_iter steps
    after r0 = b - N(x) (stops early only if <r,r> is exactly zero)."""
    x = x.copy()
    r = b - apply_n(x)
    p = r.copy()
    rr = vdot(r, r).real
    for _ in range(n_iter):
        if rr == 0.0:
            break
        q = apply_n(p)
        alpha = rr / vdot(p, q).real
        x = x + alpha * p
        r = r - alpha * q
        rr_new = vdot(r, r).real
        beta = rr_new / rr
        p = r + beta * p
        rr = rr_new
    return x


def solve(y, coils, masks, shifts, p: SolveParams, x0=None, history=None):
    """The IRLS solve of Eq. 10 with the fixed schedule described above.

    y [Ns][Nc][N2][N1], coils [L][Nc][N2][N1], masks [Ns][N2] (0/1),
    shifts [L].  Returns x [L][Ns][N2][N1] (complex128).  When `history` is a
    list, one dict per IRLS iteration (iterate, eps, weights) is appended.
    """
    y = np.asarray(y, dtype=np.complex128)
    coils = np.asarray(coils, dtype=np.complex128)
    masks = np.asarray(masks, dtype=np.float64)
    L = coils.shape[0]
    n2 = y.shape[2]
    theta = caipi_phase(n2, shifts)
    b = adjoint(y, coils, masks, theta)
    x = b.copy() if x0 is None else np.asarray(x0, dtype=np.complex128).copy()
    sigma = [lambda_max(gram(x[l], p.r)) for l in range(L)]
    for k in range(p.n_irls):
        eps = eps_schedule(sigma, k, p)
        weights = []
        for l in range(L):
            if sigma[l] <= 0.0:
                weights.append(None)          # all-zero slice: unregularised
            else:
                weights.append(irls_weight(gram(x[l], p.r), eps[l]))
        if history is not None:
            history.append({"x": x.copy(), "eps": list(eps), "weights": weights,
                            "sigma": list(sigma)})
        apply_n = lambda v, w=weights: normal_op(v, coils, masks, theta, w, p.lam, p.r)
        x = cg(apply_n, b, x, p.n_cg)
    return x


def simulate(case: dict, n_slices: int, snr: float):
    """k-space data for one generated case: x_true = F(rho_l phi_{l,i}) and
    y = A x_true + n with n = M * sigma_n * noise and
    sigma_n = RMS(A x_true over acquired samples) / snr.

    Follows the paper's simulation (Methods, "Simulations"): per-slice
    k-space multiplied by the CAIPI phase factors and summed over slices.
    Returns (x_true complex128, y complex128).
    """
    rho = case["rho"].astype(np.float64)
    phase = case["phase"].astype(np.complex128)
    coils = case["coils"].astype(np.complex128)
    masks = case["masks"].astype(np.float64)
    m = rho[:, None, :, :] * phase
    x_true = fft2c(m)
    theta = caipi_phase(x_true.shape[2], case["shifts"])
    clean = forward(x_true, coils, masks, theta)
    acquired = np.broadcast_to(masks[:, None, :, None], clean.shape) > 0
    rms = np.sqrt(np.mean(np.abs(clean[acquired]) ** 2))
    sigma_n = rms / snr
    y = clean + masks[:, None, :, None] * sigma_n * case["noise"].astype(np.complex128)
    return x_true, y


def nrmse(x_hat, x_ref) -> float:
    """||x_hat - x_ref||_2 / ||x_ref||_2 over all entries."""
    d = np.asarray(x_hat, dtype=np.complex128) - np.asarray(x_ref, dtype=np.complex128)
    return float(np.linalg.norm(d.ravel()) / np.linalg.norm(np.asarray(x_ref).ravel()))


def sos_images(x) -> np.ndarray:
    """Root-sum-of-squares over shots of the per-shot images, [L][N2][N1]."""
    return np.sqrt(np.sum(np.abs(ifft2c(x)) ** 2, axis=1))
