"""Pins of the oracle's whole IRLS solve and of the augmented-Lagrangian oracle.

The operator-level pins live in test_oracle_pins.py.  Here the solve itself
is checked against things that do not come from its own code:
  * a dense brute-force IRLS written from the readings (dense A from Kronecker
    products of DFT matrices, the Hankel lift as an index matrix, W from
    scipy's fractional matrix power, CG from its recurrences), equal to the
    oracle's solve to rounding;
  * the eigenvalue clamp of the weights on a Hermitian G with a negative part;
  * stationarity (P8): at a fixed eps the IRLS fixed point zeroes the gradient
    of the smoothed objective, checked by finite differences;
  * recovery of noiseless low-rank data (P9), where least squares alone fails;
  * the optimality certificate of Eq. 10 (convexity: subgradient condition)
    met by the augmented-Lagrangian oracle, and the IRLS solve run long
    reaching the same minimiser;
  * planted mistakes in copies of the oracle source each fail one of the
    checks above.
"""
import os
import sys
import types

import numpy as np
import pytest
import scipy.linalg

from oracle import al_oracle as al
from oracle import smsm_oracle as o

ORACLE_SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                          "oracle", "smsm_oracle.py")


def crand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def random_coils(rng, L, Nc, n):
    """Complex i.i.d. maps with unit sum of squares per pixel (well-conditioned encoding)."""
    c = crand(rng, L, Nc, n, n)
    return c / np.sqrt(np.sum(np.abs(c) ** 2, axis=1, keepdims=True))


# ----------------------------------------------------------------------------
# Dense brute force, written from the readings without the oracle's code
# ----------------------------------------------------------------------------
def centred_dft(n):
    c = np.arange(n) - n // 2
    return np.exp(-2j * np.pi * np.outer(c, c) / n) / np.sqrt(n)


def dense_forward_matrix(coils, Ns, shifts):
    """A as a dense matrix: per (shot i, coil c) row block and (slice l, shot i)
    column block, diag(M_i) diag(theta_l) F2 diag(S_lc) F2^H with F2 = D kron D
    acting on row-major [ky][kx] vectors (Fig. 1)."""
    L, Nc, n, _ = coils.shape
    D = centred_dft(n)
    F2 = np.kron(D, D)
    ky = np.repeat(np.arange(n), n)                   # ky index of each row-major entry
    nn = n * n
    A = np.zeros((Ns * Nc * nn, L * Ns * nn), complex)
    for i in range(Ns):
        m = (ky % Ns == i).astype(float)
        for l in range(L):
            th = np.exp(-2j * np.pi * shifts[l] * (ky - n // 2))
            for c in range(Nc):
                blk = (m * th)[:, None] * (F2 @ (coils[l, c].ravel()[:, None] * F2.conj().T))
                A[(i * Nc + c) * nn:(i * Nc + c + 1) * nn, (l * Ns + i) * nn:(l * Ns + i + 1) * nn] = blk
    return A


def hankel_index_matrix(Ns, n, r):
    """0/1 matrix Pi with vec(H_l(x_l)) = Pi vec(x_l) (row-major P x K, K = Ns r^2)."""
    P1 = n - r + 1
    p2, p1, i, b2, b1 = np.indices((P1, P1, Ns, r, r)).reshape(5, -1)
    rows = (p2 * P1 + p1) * (Ns * r * r) + (i * r + b2) * r + b1
    cols = i * n * n + (p2 + b2) * n + (p1 + b1)
    Pi = np.zeros((P1 * P1 * Ns * r * r, Ns * n * n))
    Pi[rows, cols] = 1.0
    return Pi


def dense_irls(A, Pi, K, y, L, lam, n_irls, n_cg, eps_frac, eta, floor):
    """IRLS as the readings state it: x0 = A^H y; sigma_l = lambda_max(G_l(x0));
    eps_l(k) = max(eps_frac eta^-k, floor) sigma_l; W_l = (G_l + eps_l I)^-1/2;
    n_cg CG steps on (A^H A + (lam/2) sum_l Pi^H (I kron W_l^T) Pi) x = A^H y
    from the current x (K = Ns r^2 columns of each Hankel matrix)."""
    nb = Pi.shape[1]                                   # entries per slice
    P = Pi.shape[0] // K                               # valid patch anchors
    AhA = A.conj().T @ A
    b = A.conj().T @ y
    x = b.copy()

    def gram(xl):
        H = (Pi @ xl).reshape(P, K)
        return H.conj().T @ H

    sl = [slice(l * nb, (l + 1) * nb) for l in range(L)]
    sigma = [scipy.linalg.eigvalsh(gram(x[s]))[-1] for s in sl]
    for k in range(n_irls):
        frac = max(eps_frac * eta ** (-k), floor)
        N = AhA.copy()
        for l, s in enumerate(sl):
            W = scipy.linalg.fractional_matrix_power(gram(x[s]) + frac * sigma[l] * np.eye(K), -0.5)
            N[s, s] += 0.5 * lam * (Pi.T @ np.kron(np.eye(P), W.T) @ Pi)
        res = b - N @ x
        p = res.copy()
        rr = np.vdot(res, res).real
        for _ in range(n_cg):
            q = N @ p
            alpha = rr / np.vdot(p, q).real
            x = x + alpha * p
            res = res - alpha * q
            rr_new = np.vdot(res, res).real
            p = res + (rr_new / rr) * p
            rr = rr_new
    return x


DENSE = dict(n=6, L=2, Ns=2, Nc=3, r=2, lam=0.4, n_irls=4, n_cg=2, eps_frac=0.3, eta=3.0, floor=0.02)


def dense_case():
    rng = np.random.default_rng(50)
    g = DENSE
    coils = random_coils(rng, g["L"], g["Nc"], g["n"])
    shifts = np.array([0.0, 0.3])     # a non-half shift: its CAIPI phase is not real
    masks = o.interleaved_masks(g["n"], g["Ns"])
    base = crand(rng, g["L"], 1, g["n"], g["n"])
    xt = base * crand(rng, 1, g["Ns"], 1, 1) + 0.2 * crand(rng, g["L"], g["Ns"], g["n"], g["n"])
    A = dense_forward_matrix(coils, g["Ns"], shifts)
    y = (A @ xt.ravel()).reshape(g["Ns"], g["Nc"], g["n"], g["n"])
    y = y + 0.1 * masks[:, None, :, None] * crand(rng, g["Ns"], g["Nc"], g["n"], g["n"])
    return coils, masks, shifts, A, y


def check_dense_irls(om):
    g = DENSE
    coils, masks, shifts, A, y = dense_case()
    Pi = hankel_index_matrix(g["Ns"], g["n"], g["r"])
    ref = dense_irls(A, Pi, g["Ns"] * g["r"] ** 2, y.ravel(), g["L"], g["lam"], g["n_irls"], g["n_cg"],
                     g["eps_frac"], g["eta"], g["floor"])
    p = om.SolveParams(lam=g["lam"], r=g["r"], n_irls=g["n_irls"], n_cg=g["n_cg"],
                       eps_frac=g["eps_frac"], eps_decay=g["eta"], eps_floor_frac=g["floor"])
    x = om.solve(y, coils, masks, shifts, p)
    err = rel(x.ravel(), ref)
    assert err < 1e-12, err


def check_forward_dense(om):
    g = DENSE
    coils, masks, shifts, A, _ = dense_case()
    rng = np.random.default_rng(51)
    x = crand(rng, g["L"], g["Ns"], g["n"], g["n"])
    got = om.forward(x, coils, masks, om.caipi_phase(g["n"], shifts))
    assert rel(got.ravel(), A @ x.ravel()) < 1e-12


def check_adjoint_dense(om):
    g = DENSE
    coils, masks, shifts, A, _ = dense_case()
    rng = np.random.default_rng(52)
    v = crand(rng, g["Ns"], g["Nc"], g["n"], g["n"])
    got = om.adjoint(v, coils, masks, om.caipi_phase(g["n"], shifts))
    assert rel(got.ravel(), A.conj().T @ v.ravel()) < 1e-12


def check_weight_clamp(om):
    """G = B B^H - delta C C^H with orthogonal ranges: clamping the negative
    eigenvalues at zero leaves W = (B B^H + eps I)^-1/2 exactly."""
    rng = np.random.default_rng(53)
    Q, _ = np.linalg.qr(crand(rng, 12, 12))
    B = Q[:, :4] * np.array([3.0, 2.0, 1.0, 0.5])
    C = Q[:, 4:7]
    G = B @ B.conj().T - 0.3 * C @ C.conj().T
    eps = 0.05
    ref = scipy.linalg.fractional_matrix_power(B @ B.conj().T + eps * np.eye(12), -0.5)
    assert rel(om.irls_weight(G, eps), ref) < 1e-11


# ----------------------------------------------------------------------------
# The checks against the oracle as committed
# ----------------------------------------------------------------------------
def test_dense_forward_matrix_agrees_with_adjoint_identity():
    # the brute-force matrix is itself the Fig. 1 chain: A^H A of one slice, one
    # shot, unit-sum-of-squares maps is the identity (no mask, no shift)
    rng = np.random.default_rng(54)
    coils = random_coils(rng, 1, 3, 4)
    A = dense_forward_matrix(coils, 1, [0.0])
    assert rel(A.conj().T @ A, np.eye(16)) < 1e-12


def test_hankel_index_matrix_entries():
    rng = np.random.default_rng(55)
    Ns, n, r = 2, 6, 3
    xl = crand(rng, Ns, n, n)
    Pi = hankel_index_matrix(Ns, n, r)
    assert rel((Pi @ xl.ravel()).reshape(-1, Ns * r * r), o.hankel(xl, r)) == 0.0


def test_solve_matches_dense_bruteforce_irls():
    """The whole IRLS orchestration (x0, sigma anchored at x0, eps schedule and
    floor, W, warm-started truncated CG) equals the dense brute force."""
    check_dense_irls(o)


def test_forward_and_adjoint_match_dense_matrix():
    check_forward_dense(o)
    check_adjoint_dense(o)


def test_weight_clamps_negative_eigenvalues_at_zero():
    check_weight_clamp(o)


def test_stationarity_of_smoothed_objective_at_fixed_point():
    """P8: with eps held fixed (eps_frac = floor, eta = 1) and every CG solve
    exact, the IRLS iterates converge to a stationary point of
    J_eps(x) = ||Ax-y||^2 + lam sum_l tr((G_l + eps_l I)^1/2).  Its gradient
    A^H(Ax-y) + (lam/2) sum_l H_l^H(H_l W_l(x)) (the form the finite-difference
    pin of test_oracle_pins.py fixes) vanishes relative to its value at x0, and
    central finite differences of J_eps agree to their own precision."""
    rng = np.random.default_rng(56)
    n, L, Ns, Nc, r = 4, 2, 2, 3, 2
    coils = random_coils(rng, L, Nc, n)
    shifts = np.arange(L) / L
    masks = o.interleaved_masks(n, Ns)
    theta = o.caipi_phase(n, shifts)
    y = o.forward(crand(rng, L, Ns, n, n), coils, masks, theta) + \
        0.2 * masks[:, None, :, None] * crand(rng, Ns, Nc, n, n)
    lam, frac = 0.8, 0.05
    dim = L * Ns * n * n
    p = o.SolveParams(lam=lam, r=r, n_irls=40, n_cg=2 * dim, eps_frac=frac, eps_decay=1.0,
                      eps_floor_frac=frac)
    hist = []
    x = o.solve(y, coils, masks, shifts, p, history=hist)
    eps = hist[0]["eps"]
    x0 = hist[0]["x"]
    b = o.adjoint(y, coils, masks, theta)

    def grad(at):
        W = [o.irls_weight(o.gram(at[l], r), eps[l]) for l in range(L)]
        return o.normal_op(at, coils, masks, theta, W, lam, r) - b

    assert np.linalg.norm(grad(x)) < 1e-8 * np.linalg.norm(grad(x0))

    def slope(at, v, h=1e-5):
        jp = o.smoothed_objective(at + h * v, y, coils, masks, theta, lam, r, eps)
        jm = o.smoothed_objective(at - h * v, y, coils, masks, theta, lam, r, eps)
        return (jp - jm) / (2 * h)

    for _ in range(3):
        v = crand(rng, L, Ns, n, n)
        v /= np.linalg.norm(v)
        assert abs(slope(x, v)) < 1e-6 * np.linalg.norm(grad(x0))


def p9_case(Nc):
    """Noiseless data of m_{l,i} = rho_l phi_{l,i} with phi_hat of 3 x 3 support
    (Hankel rank (r + 2)^2 = 49 of Ns r^2 = 100 at r = 5), N = 32, two slices,
    four shots, well-conditioned random coil maps."""
    rng = np.random.default_rng(7)
    import smsm_inputs as si
    n, L, Ns, r0 = 32, 2, 4, 3
    rho = np.stack([si.ellipse_phantom(rng, n) for _ in range(L)])
    phat = np.zeros((L, Ns, n, n), complex)
    c = n // 2
    for l in range(L):
        for i in range(Ns):
            phat[l, i, c - 1:c + 2, c - 1:c + 2] = crand(rng, r0, r0)
            phat[l, i, c, c] += 3.0
    phi = o.ifft2c(phat) * n
    xt = o.fft2c(rho[:, None] * phi)
    coils = random_coils(np.random.default_rng(99), L, Nc, n)
    shifts = np.arange(L) / L
    masks = o.interleaved_masks(n, Ns)
    y = o.forward(xt, coils, masks, o.caipi_phase(n, shifts))
    return xt, y, coils, masks, shifts


@pytest.mark.slow
def test_recovery_of_noiseless_low_rank_data():
    """P9: six coils for two slices and four shots leave every shot's data
    underdetermined (6 coils x 8 of 32 lines against 2 slices x 32 lines of
    unknowns: 3/4), so least squares cannot recover the shots (its CG iterates
    stay in the range of A^H: 0.51 after 20 steps); the Hankel penalty brings
    the error to 1.6% (0.0164 at 30 x 30).  Both bounds were fixed at the
    first run."""
    xt, y, coils, masks, shifts = p9_case(Nc=6)
    x = o.solve(y, coils, masks, shifts, o.SolveParams(lam=1e-3, r=5, n_irls=30, n_cg=30))
    assert o.nrmse(x, xt) < 0.02
    x_ls = o.solve(y, coils, masks, shifts, o.SolveParams(lam=0.0, r=5, n_irls=1, n_cg=20))
    assert o.nrmse(x_ls, xt) > 0.45


# ----------------------------------------------------------------------------
# Eq. 10 minimised: augmented-Lagrangian oracle and its optimality certificate
# ----------------------------------------------------------------------------
def al_case(low_rank: bool):
    rng = np.random.default_rng(40)
    n, L, Ns, Nc = 8, 2, 2, 4
    coils = random_coils(rng, L, Nc, n)
    masks = o.interleaved_masks(n, Ns)
    shifts = np.arange(L) / L
    theta = o.caipi_phase(n, shifts)
    if low_rank:
        xt = crand(rng, L, 1, n, n) * crand(rng, 1, Ns, 1, 1)
        sd = 0.1
    else:
        xt = crand(rng, L, Ns, n, n)
        sd = 0.3
    y = o.forward(xt, coils, masks, theta) + sd * masks[:, None, :, None] * crand(rng, Ns, Nc, n, n)
    return y, coils, masks, shifts, theta


def test_svt_is_the_nuclear_norm_proximal_map():
    """SVT(M, tau) minimises tau ||Z||_* + 1/2 ||Z - M||^2: random perturbations
    never do better, and a diagonal M shrinks entrywise."""
    rng = np.random.default_rng(57)
    M = crand(rng, 9, 5)
    tau = 1.3
    f = lambda Z: tau * np.sum(np.linalg.svd(Z, compute_uv=False)) + 0.5 * np.linalg.norm(Z - M) ** 2
    Z = al.svt(M, tau)
    for _ in range(50):
        assert f(Z) <= f(Z + 1e-3 * crand(rng, 9, 5)) + 1e-12
    d = np.diag([4.0, 2.0, 1.0, 0.5])
    assert rel(al.svt(d, 1.5), np.diag([2.5, 0.5, 0.0, 0.0])) < 1e-14


def test_count_weights_are_hankel_normal_operator():
    rng = np.random.default_rng(58)
    xl = crand(rng, 2, 9, 9)
    out = o.hankel_adjoint(o.hankel(xl, 4), 2, 9, 9, 4)
    assert rel(out, al.count_weights(9, 9, 4)[None] * xl) < 1e-14


@pytest.mark.slow
def test_al_reaches_certified_minimiser_with_rank_cut():
    """The augmented-Lagrangian iteration ends at a point meeting the
    subgradient optimality condition of Eq. 10 (which proves global optimality
    by convexity), here with singular values of a slice thresholded to zero."""
    y, coils, masks, shifts, _ = al_case(low_rank=True)
    lam, beta, r = 3.0, 3.0, 3
    hist = []
    x = al.solve_al(y, coils, masks, shifts, al.ALParams(lam=lam, r=r, beta=beta, n_outer=500, n_cg=20),
                    history=hist)
    Y = [beta * u / lam for u in hist[-1]["U"]]
    k = al.kkt_residuals(x, Y, y, coils, masks, shifts, lam, r)
    assert k["stationarity"] < 1e-9 and k["dual_norm"] < 1 + 1e-9 and k["alignment"] < 1e-9, k
    s = np.linalg.svd(o.hankel(x[1], r), compute_uv=False)
    assert np.sum(s > 1e-8 * s[0]) < s.size          # the minimiser is rank-deficient


def test_irls_converges_to_the_minimiser_of_eq10():
    """The IRLS solve run long with a tiny eps floor reaches the minimiser the
    augmented-Lagrangian iteration certifies (the objective is strictly convex
    here: four coils for two slices and two shots make A injective)."""
    y, coils, masks, shifts, theta = al_case(low_rank=False)
    lam, r = 1.0, 3
    hist = []
    x_al = al.solve_al(y, coils, masks, shifts, al.ALParams(lam=lam, r=r, beta=1.0, n_outer=150, n_cg=20),
                       history=hist)
    k = al.kkt_residuals(x_al, [u / lam for u in hist[-1]["U"]], y, coils, masks, shifts, lam, r)
    assert k["stationarity"] < 1e-6 and k["dual_norm"] < 1 + 1e-9 and k["alignment"] < 1e-9, k
    x = o.solve(y, coils, masks, shifts, o.SolveParams(lam=lam, r=r, n_irls=40, n_cg=60, eps_floor_frac=1e-9))
    j_al = o.objective(x_al, y, coils, masks, theta, lam, r)
    j = o.objective(x, y, coils, masks, theta, lam, r)
    assert j >= j_al * (1 - 1e-12)
    assert (j - j_al) / j_al < 1e-9
    assert rel(x, x_al) < 1e-4


# ----------------------------------------------------------------------------
# Planted mistakes: each copy of the oracle with one mistake fails a check
# ----------------------------------------------------------------------------
MUTATIONS = [
    ("cg restarted from b", "x = cg(apply_n, b, x, p.n_cg)", "x = cg(apply_n, b, b, p.n_cg)", check_dense_irls),
    ("sigma re-anchored every step", "    for k in range(p.n_irls):\n        eps = eps_schedule(sigma, k, p)",
     "    for k in range(p.n_irls):\n        sigma = [lambda_max(gram(x[l], p.r)) for l in range(L)]\n"
     "        eps = eps_schedule(sigma, k, p)", check_dense_irls),
    ("eps floor x10", "max(p.eps_frac * p.eps_decay ** (-k), p.eps_floor_frac)",
     "max(p.eps_frac * p.eps_decay ** (-k), 10 * p.eps_floor_frac)", check_dense_irls),
    ("eps increasing", "p.eps_decay ** (-k)", "p.eps_decay ** (k)", check_dense_irls),
    ("|s| instead of max(s, 0)", "np.sqrt(np.maximum(s, 0.0) + eps)", "np.sqrt(np.abs(s) + eps)", check_weight_clamp),
    ("lam instead of lam/2", "out[l] = 0.5 * lam * hankel_adjoint", "out[l] = lam * hankel_adjoint", check_dense_irls),
    ("CG beta inverted", "beta = rr_new / rr", "beta = rr / rr_new", check_dense_irls),
    ("weights from b", "weights.append(irls_weight(gram(x[l], p.r), eps[l]))",
     "weights.append(irls_weight(gram(b[l], p.r), eps[l]))", check_dense_irls),
    ("CAIPI sign flipped", "np.exp(-2j * np.pi * s[:, None] * j2[None, :])",
     "np.exp(2j * np.pi * s[:, None] * j2[None, :])", check_forward_dense),
    ("coil conjugate dropped in A^H", "acc += np.conj(coils[l, c]) * ifft2c(k)", "acc += coils[l, c] * ifft2c(k)",
     check_adjoint_dense),
]


def mutated_oracle(old: str, new: str):
    with open(ORACLE_SRC) as f:
        src = f.read()
    assert src.count(old) == 1, f"snippet not found once in the oracle: {old!r}"
    mod = types.ModuleType("oracle_mutant")
    sys.modules[mod.__name__] = mod            # dataclasses resolve annotations through it
    try:
        exec(compile(src.replace(old, new), "oracle_mutant", "exec"), mod.__dict__)
    finally:
        del sys.modules[mod.__name__]
    return mod


@pytest.mark.parametrize("name,old,new,check", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_fails_a_check(name, old, new, check):
    check(o)                                   # the committed oracle passes
    with pytest.raises(AssertionError):
        check(mutated_oracle(old, new))
