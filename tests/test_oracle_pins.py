"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test checks one part of the oracle against a closed form, an identity,
brute force on tiny inputs, or an independent library routine, chosen so that
a plausible mistake (a dropped conjugate, a flipped CAIPI sign, an off-by-one
in the Hankel window, a wrong lam/2 factor) fails at least one of them.
"""
import numpy as np
import pytest
import scipy.linalg

import smsm_inputs as si
from oracle import smsm_oracle as o

RTOL = 1e-12


def crand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


def small_geometry(rng, n=8, L=2, Ns=2, Nc=2):
    coils = crand(rng, L, Nc, n, n)
    masks = o.interleaved_masks(n, Ns)
    shifts = np.arange(L) / L
    return coils, masks, shifts, o.caipi_phase(n, shifts)


# ----------------------------------------------------------------------------
# Centred unitary DFT (convention C1): explicit DFT-matrix brute force
# ----------------------------------------------------------------------------
def dft_matrix(n):
    """D[k, v] = exp(-2 pi i k v / n)/sqrt(n) with centred k, v in [-n/2, n/2)."""
    c = np.arange(n) - n // 2
    return np.exp(-2j * np.pi * np.outer(c, c) / n) / np.sqrt(n)


def test_fft2c_matches_explicit_centred_dft():
    rng = np.random.default_rng(1)
    n = 8
    D = dft_matrix(n)
    u = crand(rng, n, n)
    assert rel(o.fft2c(u), D @ u @ D.T) < RTOL
    assert rel(o.ifft2c(u), D.conj().T @ u @ D.conj()) < RTOL


def test_fft2c_delta_at_centre_is_flat_and_unitary():
    n = 16
    u = np.zeros((n, n))
    u[n // 2, n // 2] = 1.0
    k = o.fft2c(u)
    assert np.allclose(k, 1.0 / n, atol=1e-15)
    rng = np.random.default_rng(2)
    v = crand(rng, n, n)
    assert abs(np.linalg.norm(o.fft2c(v)) - np.linalg.norm(v)) < 1e-12 * np.linalg.norm(v)


# ----------------------------------------------------------------------------
# Forward operator A (Fig. 1) and adjoint (P1, P2)
# ----------------------------------------------------------------------------
def forward_bruteforce(x, coils, masks, shifts):
    """Fig. 1 written with explicit DFT matrices and explicit CAIPI/mask loops."""
    L, Ns, n, _ = x.shape
    Nc = coils.shape[1]
    D = dft_matrix(n)
    Di = D.conj()
    y = np.zeros((Ns, Nc, n, n), complex)
    for i in range(Ns):
        for c in range(Nc):
            for l in range(L):
                img = Di @ x[l, i] @ Di          # (i) inverse DFT (D symmetric)
                kc = D @ (coils[l, c] * img) @ D  # (ii) coil, (iii) DFT
                for j2 in range(n):              # (iv) CAIPI phase per ky line
                    ky = j2 - n // 2
                    y[i, c, j2, :] += np.exp(-2j * np.pi * shifts[l] * ky) * kc[j2, :]
            for j2 in range(n):                  # (v) shot i keeps lines j2 = i mod Ns
                if j2 % Ns != i:
                    y[i, c, j2, :] = 0.0
    return y


def test_forward_matches_bruteforce_tiny():
    rng = np.random.default_rng(3)
    coils, masks, shifts, theta = small_geometry(rng, n=8, L=2, Ns=2, Nc=2)
    x = crand(rng, 2, 2, 8, 8)
    assert rel(o.forward(x, coils, masks, theta), forward_bruteforce(x, coils, masks, shifts)) < RTOL


def test_forward_adjoint_inner_product():
    rng = np.random.default_rng(4)
    coils, masks, shifts, theta = small_geometry(rng, n=16, L=3, Ns=4, Nc=3)
    x = crand(rng, 3, 4, 16, 16)
    y = crand(rng, 4, 3, 16, 16)
    lhs = o.vdot(o.forward(x, coils, masks, theta), y)
    rhs = o.vdot(x, o.adjoint(y, coils, masks, theta))
    assert abs(lhs - rhs) < RTOL * abs(lhs)


def test_forward_dense_adjoint_bruteforce():
    """A^H equals the conjugate transpose of the dense matrix of A (N=4)."""
    rng = np.random.default_rng(5)
    n, L, Ns, Nc = 4, 2, 2, 2
    coils, masks, shifts, theta = small_geometry(rng, n=n, L=L, Ns=Ns, Nc=Nc)
    nx = L * Ns * n * n
    Amat = np.zeros((Ns * Nc * n * n, nx), complex)
    for k in range(nx):
        e = np.zeros(nx, complex)
        e[k] = 1.0
        Amat[:, k] = forward_bruteforce(e.reshape(L, Ns, n, n), coils, masks, shifts).ravel()
    y = crand(rng, Ns, Nc, n, n)
    assert rel(o.adjoint(y, coils, masks, theta).ravel(), Amat.conj().T @ y.ravel()) < RTOL


def test_forward_reduces_to_identity():
    """L = Ns = Nc = 1, unit coil, full mask, no shift: A = I."""
    rng = np.random.default_rng(6)
    x = crand(rng, 1, 1, 16, 16)
    coils = np.ones((1, 1, 16, 16), complex)
    masks = o.interleaved_masks(16, 1)
    theta = o.caipi_phase(16, [0.0])
    y = o.forward(x, coils, masks, theta)
    assert rel(y[:, 0][None], x) < RTOL


def test_sense_normal_operator_is_identity_for_sos_maps():
    """One slice, one shot, maps with unit sum of squares: A^H A = I."""
    rng = np.random.default_rng(7)
    coils = si.coil_maps(16, 1, 6).astype(complex)
    masks = o.interleaved_masks(16, 1)
    theta = o.caipi_phase(16, [0.0])
    x = crand(rng, 1, 1, 16, 16)
    assert rel(o.adjoint(o.forward(x, coils, masks, theta), coils, masks, theta), x) < 1e-12


@pytest.mark.parametrize("L", [2, 4])
def test_caipi_phase_is_fov_shift(L):
    """Integer shifts: F^-1(theta_l F u) = u moved down by s_l N2 rows (FOV/L)."""
    rng = np.random.default_rng(8)
    n = 16
    shifts = np.arange(L) / L
    theta = o.caipi_phase(n, shifts)
    u = crand(rng, n, n)
    for l in range(L):
        moved = o.ifft2c(theta[l][:, None] * o.fft2c(u))
        assert rel(moved, np.roll(u, int(round(shifts[l] * n)), axis=0)) < 1e-12


@pytest.mark.parametrize("Ns", [2, 4])
def test_interleaved_mask_alias_closed_form(Ns):
    """F^-1 M_i F u = (1/Ns) sum_t exp(2 pi i t (N/2 - i)/Ns) roll(u, -t N/Ns)."""
    rng = np.random.default_rng(9)
    n = 16
    masks = o.interleaved_masks(n, Ns)
    u = crand(rng, n, n)
    for i in range(Ns):
        lhs = o.ifft2c(masks[i][:, None] * o.fft2c(u))
        rhs = sum(np.exp(2j * np.pi * t * (n // 2 - i) / Ns) * np.roll(u, -t * n // Ns, axis=0)
                  for t in range(Ns)) / Ns
        assert rel(lhs, rhs) < 1e-12


# ----------------------------------------------------------------------------
# Block-Hankel lift (Eq. 8-9) (P3, P4)
# ----------------------------------------------------------------------------
def test_hankel_shape_and_entries():
    rng = np.random.default_rng(10)
    Ns, n, r = 3, 9, 4
    xl = crand(rng, Ns, n, n)
    H = o.hankel(xl, r)
    assert H.shape == ((n - r + 1) ** 2, Ns * r * r)       # (N1-r+1)(N2-r+1) x Ns r^2
    for _ in range(20):
        p2, p1 = rng.integers(0, n - r + 1, size=2)
        i = rng.integers(Ns)
        b2, b1 = rng.integers(0, r, size=2)
        assert H[p2 * (n - r + 1) + p1, (i * r + b2) * r + b1] == xl[i, p2 + b2, p1 + b1]


def test_hankel_adjoint_inner_product():
    rng = np.random.default_rng(11)
    Ns, n, r = 2, 10, 3
    xl = crand(rng, Ns, n, n)
    Z = crand(rng, (n - r + 1) ** 2, Ns * r * r)
    lhs = np.vdot(o.hankel(xl, r), Z)
    rhs = np.vdot(xl, o.hankel_adjoint(Z, Ns, n, n, r))
    assert abs(lhs - rhs) < RTOL * abs(lhs)


def test_hankel_normal_is_count_weighting():
    """H^H H x = c * x with c[q] = cnt(q2) cnt(q1), cnt(t) = min(t+1, r, N-t, N-r+1);
    tr G = sum_i sum_q c[q] |x_i[q]|^2."""
    rng = np.random.default_rng(12)
    Ns, n, r = 2, 11, 4
    xl = crand(rng, Ns, n, n)
    t = np.arange(n)
    cnt = np.minimum.reduce([t + 1, np.full(n, r), n - t, np.full(n, n - r + 1)])
    c = np.outer(cnt, cnt)
    out = o.hankel_adjoint(o.hankel(xl, r), Ns, n, n, r)
    assert rel(out, c[None] * xl) < RTOL
    G = o.gram(xl, r)
    assert abs(np.trace(G) - np.sum(c[None] * np.abs(xl) ** 2)) < 1e-12 * np.trace(G).real


def test_nuclear_norm_from_gram_eigenvalues():
    rng = np.random.default_rng(13)
    xl = crand(rng, 2, 10, 10)
    s = np.linalg.eigvalsh(o.gram(xl, 3))
    assert abs(o.nuclear_norm(xl, 3) - np.sum(np.sqrt(np.maximum(s, 0)))) < 1e-10 * o.nuclear_norm(xl, 3)


def bandlimited_shots(rng, n, Ns, r0):
    """k-space x_i = F(rho phi_i) with phi_hat_i supported on r0 x r0 around DC."""
    rho = rng.uniform(0.2, 1.0, size=(n, n))
    phat = np.zeros((Ns, n, n), complex)
    c, h = n // 2, (r0 - 1) // 2
    for i in range(Ns):
        phat[i, c - h:c + h + 1, c - h:c + h + 1] = crand(rng, r0, r0)
    phi = o.ifft2c(phat)
    return o.fft2c(rho[None] * phi), phat


@pytest.mark.parametrize("r", [3, 5])
def test_hankel_annihilation_and_rank(r):
    """Eq. 6-9: with m_i = rho phi_i and phi_hat_i of support r0 x r0, the pairwise
    filter matrix of Eq. 9 annihilates H_l, and rank H_l <= (r + r0 - 1)^2,
    with equality for generic data."""
    rng = np.random.default_rng(14 + r)
    n, Ns, r0 = 16, 4, 3
    x, phat = bandlimited_shots(rng, n, Ns, r0)
    H = o.hankel(x, r)
    # Filter of shot n in the Hankel column space: f_n[b] = phat_n[c0 - b]
    # (centred index), so (H(x_i) f_n)[p] is the circular convolution
    # (x_i * phat_n) at k-space index p + c0, which no valid anchor wraps.
    c, h = n // 2, (r0 - 1) // 2
    f = np.zeros((Ns, r, r), complex)
    for i in range(Ns):
        for b2 in range(r0):
            for b1 in range(r0):
                f[i, b2, b1] = phat[i, c + h - b2, c + h - b1]
    cols = []
    for a in range(Ns):
        for b in range(a + 1, Ns):
            v = np.zeros((Ns, r * r), complex)
            v[a] = f[b].ravel()
            v[b] = -f[a].ravel()
            cols.append(v.ravel())
    Phi = np.stack(cols, axis=1)
    assert np.linalg.norm(H @ Phi) < 1e-12 * np.linalg.norm(H) * np.linalg.norm(Phi)
    s = np.linalg.svd(H, compute_uv=False)
    rank = int(np.sum(s > 1e-10 * s[0]))
    bound = min(Ns * r * r, (r + r0 - 1) ** 2)
    assert rank == bound


def test_hankel_rank_single_shared_phase():
    """All shots share one phase up to constants (r0 = 1): rank H_l = r^2."""
    rng = np.random.default_rng(20)
    n, Ns, r = 16, 3, 4
    base = o.fft2c(rng.uniform(0.2, 1, (n, n)) * np.exp(1j * rng.uniform(0, 6, (n, n))))
    x = np.stack([(1.0 + 0.5j * i) * base for i in range(Ns)])
    s = np.linalg.svd(o.hankel(x, r), compute_uv=False)
    assert int(np.sum(s > 1e-10 * s[0])) == r * r


# ----------------------------------------------------------------------------
# IRLS weights (P5)
# ----------------------------------------------------------------------------
def test_irls_weight_is_inverse_square_root():
    rng = np.random.default_rng(21)
    xl = crand(rng, 2, 10, 10)
    G = o.gram(xl, 3)
    eps = 1e-3 * np.linalg.eigvalsh(G)[-1]
    W = o.irls_weight(G, eps)
    A = G + eps * np.eye(G.shape[0])
    assert rel(W @ W @ A, np.eye(G.shape[0])) < 1e-11
    ref = scipy.linalg.fractional_matrix_power(A, -0.5)
    assert rel(W, ref) < 1e-10
    assert rel(W, W.conj().T) < 1e-14


def test_irls_weight_of_rank_deficient_gram():
    """Rank-deficient G: the null space gets weight eps^-1/2 exactly."""
    rng = np.random.default_rng(22)
    B = crand(rng, 30, 4)
    G = B @ B.conj().T                     # rank 4, size 30
    eps = 0.5
    W = o.irls_weight(G, eps)
    Q, _ = np.linalg.qr(crand(rng, 30, 30))
    null = Q[:, :30]
    null = null - B @ np.linalg.lstsq(B, null, rcond=None)[0]   # project out range(B)
    v = null[:, 0] / np.linalg.norm(null[:, 0])
    assert rel(W @ v, v / np.sqrt(eps)) < 1e-10


# ----------------------------------------------------------------------------
# Normal equations and solver (P6, P7, P8)
# ----------------------------------------------------------------------------
def tiny_problem(seed, n=8, L=2, Ns=2, Nc=3, r=3):
    rng = np.random.default_rng(seed)
    coils, masks, shifts, theta = small_geometry(rng, n=n, L=L, Ns=Ns, Nc=Nc)
    xt = crand(rng, L, Ns, n, n)
    y = o.forward(xt, coils, masks, theta) + 0.05 * masks[:, None, :, None] * crand(rng, Ns, Nc, n, n)
    return rng, coils, masks, shifts, theta, y


def test_gradient_of_smoothed_objective_matches_normal_equations():
    """Finite differences of J_eps(x) = ||Ax-y||^2 + lam sum tr((G+eps I)^1/2)
    equal 2 Re<g, v> with g = A^H(Ax-y) + (lam/2) sum H^H(H W): pins lam/2 and W."""
    rng, coils, masks, shifts, theta, y = tiny_problem(30)
    lam, r = 0.7, 3
    x = crand(rng, 2, 2, 8, 8)
    eps = [0.3, 0.2]
    W = [o.irls_weight(o.gram(x[l], r), eps[l]) for l in range(2)]
    g = o.normal_op(x, coils, masks, theta, W, lam, r) - o.adjoint(y, coils, masks, theta)
    for k in range(3):
        v = crand(rng, 2, 2, 8, 8)
        h = 1e-5
        jp = o.smoothed_objective(x + h * v, y, coils, masks, theta, lam, r, eps)
        jm = o.smoothed_objective(x - h * v, y, coils, masks, theta, lam, r, eps)
        fd = (jp - jm) / (2 * h)
        an = 2 * np.real(o.vdot(g, v))
        assert abs(fd - an) < 1e-7 * abs(an)


def test_lambda_zero_solve_is_least_squares():
    """lam = 0 and CG run past the dimension: the IRLS solve is the
    least-squares solution of A x = y (dense lstsq, full column rank)."""
    rng = np.random.default_rng(31)
    n, L, Ns, Nc = 4, 2, 2, 4
    coils, masks, shifts, theta = small_geometry(rng, n=n, L=L, Ns=Ns, Nc=Nc)
    nx = L * Ns * n * n
    Amat = np.stack([forward_bruteforce(np.eye(nx)[k].reshape(L, Ns, n, n), coils, masks, shifts).ravel()
                     for k in range(nx)], axis=1)
    assert np.linalg.matrix_rank(Amat) == nx
    y = crand(rng, Ns, Nc, n, n) * masks[:, None, :, None]
    ref = np.linalg.lstsq(Amat, y.ravel(), rcond=None)[0]
    p = o.SolveParams(lam=0.0, r=3, n_irls=3, n_cg=2 * nx)
    x = o.solve(y, coils, masks, shifts, p)
    assert rel(x.ravel(), ref) < 1e-9


def test_cg_step_matches_dense_solve():
    """One IRLS step with CG run to the dimension equals the dense solution of
    N(x) = A^H y with the same weights."""
    rng, coils, masks, shifts, theta, y = tiny_problem(32, n=4, L=2, Ns=2, Nc=2, r=2)
    lam, r = 0.2, 2
    x0 = o.adjoint(y, coils, masks, theta)
    W = [o.irls_weight(o.gram(x0[l], r), 0.1) for l in range(2)]
    apply_n = lambda v: o.normal_op(v, coils, masks, theta, W, lam, r)
    nx = x0.size
    Nmat = np.stack([apply_n(np.eye(nx)[k].reshape(x0.shape)).ravel() for k in range(nx)], axis=1)
    assert rel(Nmat, Nmat.conj().T) < 1e-13          # Hermitian normal operator
    ref = np.linalg.solve(Nmat, x0.ravel())
    got = o.cg(apply_n, x0, x0, 3 * nx)
    assert rel(got.ravel(), ref) < 1e-9


def test_irls_majorise_minimise_monotone():
    """J_{eps_k}(x_k) never increases along the IRLS iterates, even with
    truncated CG (each CG step lowers the quadratic majoriser; eps only drops)."""
    g = si.Geometry(n=16, n_slices=2, n_shots=4, n_coils=4, filt=3, lam=5e-2,
                    n_irls=6, n_cg=3, phase_order=2, snr=20.0)
    case = si.make_case(g, 3, 77)
    xt, y = o.simulate(case, g.n_slices, g.snr)
    p = o.SolveParams(lam=g.lam, r=g.filt, n_irls=g.n_irls, n_cg=g.n_cg)
    hist = []
    x_final = o.solve(y, case["coils"], case["masks"], case["shifts"], p, history=hist)
    theta = o.caipi_phase(g.n, case["shifts"])
    coils = case["coils"].astype(complex)
    masks = case["masks"].astype(float)
    vals = [o.smoothed_objective(h["x"], y, coils, masks, theta, g.lam, g.filt, h["eps"]) for h in hist]
    vals.append(o.smoothed_objective(x_final, y, coils, masks, theta, g.lam, g.filt, hist[-1]["eps"]))
    for a, b in zip(vals[:-1], vals[1:]):
        assert b <= a * (1 + 1e-12)
    assert vals[-1] < vals[0]


def test_all_zero_slice_is_unregularised():
    """sigma_l = 0 (a slice whose data vanish): W_l = 0, the slice stays zero."""
    rng = np.random.default_rng(33)
    n, L, Ns, Nc = 8, 2, 2, 2
    coils, masks, shifts, theta = small_geometry(rng, n=n, L=L, Ns=Ns, Nc=Nc)
    coils[1] = 0.0                               # slice 1 invisible to every coil
    xt = crand(rng, L, Ns, n, n)
    y = o.forward(xt, coils, masks, theta)
    p = o.SolveParams(lam=1e-2, r=3, n_irls=2, n_cg=3)
    x = o.solve(y, coils, masks, shifts, p)
    assert np.all(x[1] == 0)
    assert np.linalg.norm(x[0]) > 0


def test_lambda_max_closed_form_constant_shots():
    """x_i = c_i everywhere: every Hankel row is v = [c_0 1_{r^2}, ..., c_{Ns-1} 1_{r^2}],
    so G = P v v^H and lambda_max = P r^2 sum_i |c_i|^2."""
    n, r = 12, 3
    c = np.array([1.0 + 2.0j, -0.5 + 0.25j, 3.0 - 1.0j])
    x = c[:, None, None] * np.ones((3, n, n))
    P = (n - r + 1) ** 2
    G = o.gram(x, r)
    assert abs(o.lambda_max(G) - P * r * r * np.sum(np.abs(c) ** 2)) < 1e-10 * o.lambda_max(G)


def test_objective_is_smoothed_objective_at_zero_eps():
    """Eq. 10 equals J_eps at eps = 0 (trace of the Gram square root = nuclear norm)."""
    rng, coils, masks, shifts, theta, y = tiny_problem(34)
    x = crand(rng, 2, 2, 8, 8)
    a = o.objective(x, y, coils, masks, theta, 0.3, 3)
    b = o.smoothed_objective(x, y, coils, masks, theta, 0.3, 3, [0.0, 0.0])
    assert abs(a - b) < 1e-10 * abs(a)


# ----------------------------------------------------------------------------
# Root-sum-of-squares shot combination (the optional image output)
# ----------------------------------------------------------------------------
def test_sos_images_parseval_per_slice():
    # the image transform is unitary: sum over pixels of sos^2 is the k-space energy of the slice's shots
    rng = np.random.default_rng(31)
    x = crand(rng, 2, 3, 16, 8)
    img = o.sos_images(x)
    assert img.shape == (2, 16, 8) and np.all(img >= 0)
    for l in range(2):
        assert abs(np.sum(img[l] ** 2) - np.sum(np.abs(x[l]) ** 2)) <= RTOL * np.sum(np.abs(x[l]) ** 2)


def test_sos_images_unit_modulus_phases_closed_form():
    # shots rho * phi_i with |phi_i| = 1 combine to sqrt(Ns) |rho|, whatever the phases
    rng = np.random.default_rng(32)
    n, Ns = 16, 4
    rho = crand(rng, 2, n, n)
    phi = np.exp(1j * rng.uniform(0, 2 * np.pi, (2, Ns, n, n)))
    img = o.sos_images(np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(rho[:, None] * phi, axes=(-2, -1)),
                                                   norm="ortho"), axes=(-2, -1)))
    assert rel(img, np.sqrt(Ns) * np.abs(rho)) < RTOL


def test_sos_images_single_shot_delta():
    # one shot, a k-space delta at the centre: a flat image of height 1/N
    n = 8
    x = np.zeros((1, 1, n, n), complex)
    x[0, 0, n // 2, n // 2] = 1.0
    assert np.allclose(o.sos_images(x), 1.0 / n, rtol=0, atol=1e-15)
