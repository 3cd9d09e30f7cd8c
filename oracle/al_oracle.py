"""Plain FP64 CPU oracle of the augmented-Lagrangian solve of SMS-MUSSELS.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this module.  The GPU library never
calls it and shares no code with it.

The paper minimises its objective (Theory, "SMS MUSSELS", Eq. 10)

    J(x) = ||A x - y||^2 + lam sum_l ||H_l(x_l)||_*

with an augmented-Lagrangian scheme (same section, the paragraph after
Eq. 10; Methods, "Reconstruction"), whose steps it leaves to a cited paper.
Written here from the method itself: split Z_l = H_l(x_l) and alternate, in
the scaled-dual form of the alternating-direction method of multipliers,

    x  <- argmin ||A x - y||^2 + (beta/2) sum_l ||H_l(x_l) - Z_l + U_l||_F^2
          i.e. (A^H A + (beta/2) sum_l H_l^H H_l) x = A^H y + (beta/2) sum_l H_l^H(Z_l - U_l),
          solved by n_cg conjugate-gradient steps warm-started at the previous x;
    Z_l <- argmin lam ||Z||_* + (beta/2) ||Z - (H_l(x_l) + U_l)||_F^2
          = singular-value soft thresholding of H_l(x_l) + U_l at lam / beta;
    U_l <- U_l + H_l(x_l) - Z_l.

H_l^H H_l is the per-sample count weighting (how many valid patches hold a
k-space sample), so the x-step operator is the SENSE normal operator plus a
diagonal.  Readings (the paper is silent on them): x0 = A^H y, Z_l = H_l(x0),
U_l = 0; fixed counts n_outer and n_cg; beta a fixed scalar.  With `rank`
set, the thresholded singular values beyond the first `rank` are also
dropped (the paper imposes one rank for every slice, Methods,
"Reconstruction"); that variant no longer minimises Eq. 10 and is kept
apart from the pins of the convex form.

Optimality certificate (convex analysis of Eq. 10): x minimises J iff there
are Y_l in the subdifferential of the nuclear norm at H_l(x_l) (spectral
norm <= 1 and Re<Y_l, H_l(x_l)> = ||H_l(x_l)||_*) with
A^H(A x - y) + (lam/2) sum_l H_l^H(Y_l) = 0.  At a fixed point of the
iteration Y_l = beta U_l / lam; `kkt_residuals` measures all three parts.

Uses the operators of the IRLS oracle (forward model, Hankel lift, CG),
which are pinned on their own.
"""
from __future__ import annotations

import dataclasses
import numpy as np

from . import smsm_oracle as so


@dataclasses.dataclass
class ALParams:
    lam: float = 1e-3
    r: int = 5
    beta: float = 1e-2
    n_outer: int = 30
    n_cg: int = 10
    rank: int | None = None


def svt(M, tau: float, rank: int | None = None):
    """argmin_Z tau ||Z||_* + 1/2 ||Z - M||_F^2: singular values of M shrunk by
    tau and clipped at zero (optionally only the first `rank` kept)."""
    U, s, Vh = np.linalg.svd(M, full_matrices=False)
    t = np.maximum(s - tau, 0.0)
    if rank is not None:
        t[rank:] = 0.0
    return (U * t[None, :]) @ Vh


def count_weights(n2: int, n1: int, r: int) -> np.ndarray:
    """c[q2, q1] = number of valid r x r patches holding sample q, so that
    H_l^H H_l x = c * x (each shot alike)."""
    def cnt(n):
        t = np.arange(n)
        return np.minimum.reduce([t + 1, np.full(n, r), n - t, np.full(n, n - r + 1)])
    return np.outer(cnt(n2), cnt(n1)).astype(np.float64)


def solve_al(y, coils, masks, shifts, p: ALParams, x0=None, history=None):
    """Augmented-Lagrangian solve of Eq. 10 (steps in the module docstring).

    Shapes as in smsm_oracle.solve.  Returns x [L][Ns][N2][N1] complex128.
    When `history` is a list, one dict per outer iteration is appended with
    the iterate, the splitting variables Z and the scaled duals U.
    """
    y = np.asarray(y, dtype=np.complex128)
    coils = np.asarray(coils, dtype=np.complex128)
    masks = np.asarray(masks, dtype=np.float64)
    L = coils.shape[0]
    Ns, n2, n1 = y.shape[0], y.shape[2], y.shape[3]
    theta = so.caipi_phase(n2, shifts)
    b = so.adjoint(y, coils, masks, theta)
    x = b.copy() if x0 is None else np.asarray(x0, dtype=np.complex128).copy()
    c = count_weights(n2, n1, p.r)
    Z = [so.hankel(x[l], p.r) for l in range(L)]
    U = [np.zeros_like(Z[l]) for l in range(L)]

    def apply_m(v):
        return so.adjoint(so.forward(v, coils, masks, theta), coils, masks, theta) + \
            0.5 * p.beta * c[None, None] * v

    for _ in range(p.n_outer):
        rhs = b.copy()
        for l in range(L):
            rhs[l] += 0.5 * p.beta * so.hankel_adjoint(Z[l] - U[l], Ns, n2, n1, p.r)
        x = so.cg(apply_m, rhs, x, p.n_cg)
        for l in range(L):
            M = so.hankel(x[l], p.r) + U[l]
            Z[l] = svt(M, p.lam / p.beta, p.rank)
            U[l] = M - Z[l]
        if history is not None:
            history.append({"x": x.copy(), "Z": [z.copy() for z in Z], "U": [u.copy() for u in U]})
    return x


def kkt_residuals(x, Y, y, coils, masks, shifts, lam: float, r: int) -> dict:
    """Parts of the optimality certificate of Eq. 10 at x with multipliers Y_l:
      stationarity  ||A^H(Ax - y) + (lam/2) sum_l H_l^H(Y_l)|| / ||A^H y||
      dual_norm     max_l ||Y_l||_2 (must not exceed 1)
      alignment     max_l |Re<Y_l, H_l x_l> - ||H_l x_l||_*| / ||H_l x_l||_*
    """
    y = np.asarray(y, dtype=np.complex128)
    coils = np.asarray(coils, dtype=np.complex128)
    masks = np.asarray(masks, dtype=np.float64)
    L, Ns, n2, n1 = x.shape
    theta = so.caipi_phase(n2, shifts)
    b = so.adjoint(y, coils, masks, theta)
    g = so.adjoint(so.forward(x, coils, masks, theta), coils, masks, theta) - b
    dual, align = 0.0, 0.0
    for l in range(L):
        g[l] += 0.5 * lam * so.hankel_adjoint(Y[l], Ns, n2, n1, r)
        Hx = so.hankel(x[l], r)
        dual = max(dual, float(np.linalg.norm(Y[l], 2)))
        nn = float(np.sum(np.linalg.svd(Hx, compute_uv=False)))
        align = max(align, abs(float(np.vdot(Y[l], Hx).real) - nn) / nn)
    return {"stationarity": float(np.linalg.norm(g) / np.linalg.norm(b)),
            "dual_norm": dual, "alignment": align}
