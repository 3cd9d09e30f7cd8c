"""Seeded synthetic inputs for SMS-MUSSELS workloads.

This module draws the random ingredients of a simulated SMS multi-shot
diffusion acquisition and nothing else: per-slice magnitude phantoms, per-shot
phase images, per-slice coil sensitivities, the interleaved shot sampling
pattern, the CAIPI shift fractions and unit-variance complex noise.  It holds
none of the reconstruction's arithmetic (no Fourier transform, no forward
operator, no Hankel lift); both the FP64 oracle and the GPU library consume
these arrays and form the k-space data with their own operators.

Everything is returned already rounded to complex64 / float32, the precision
the GPU library takes; the oracle promotes the same rounded values to FP64.

Recipe (stand-in for the paper's in-vivo data, which is not available):
  * magnitude rho_l: 6 ellipses painted in order (later ones overwrite),
    intensity U(0.2, 1), centre U(-0.4, 0.4)^2, semi-axes U(0.15, 0.45),
    angle U(0, pi), background 0, on normalised coordinates in [-1, 1).
  * shot phase phi_{l,i} = exp(i * sum_{p+q<=order} a_pq xb^p yb^q) with
    a_pq ~ N(0, sd=pi/4); order 2 for the small case, 3 for the others.  This
    is the per-shot phase of the signal model m_{l,i} = rho_l phi_{l,i}
    (Theory, "SMS accelerated ms-DWI recovery", Eq. 4-5).
  * coil maps: Gaussian bumps of sd 0.4 FOV (0.8 in normalised units) centred
    on a ring of radius 1 at angle 2 pi c/Nc + 2 pi l/(L Nc), times the
    constant phase exp(2 pi i c/Nc), normalised to unit sum of squares at
    every pixel.  Maps differ per slice because the slices sit at different
    positions (Fig. 1 multiplies each slice by its own sensitivities).
  * shot i acquires the ky lines j2 = i (mod Ns) (Eq. 2: line n' = (n-1)Ns+i).
  * CAIPI shift of slice l is l/L of the FOV (Theory, blipped CAIPI: FOV/L).
  * noise: i.i.d. (N(0,1) + i N(0,1))/sqrt(2), scaled later by the consumer to
    the requested linear SNR.
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = ["Geometry", "WORKLOADS", "make_case", "ellipse_phantom", "coil_maps",
           "shot_phases", "shot_masks", "caipi_shifts"]


@dataclasses.dataclass(frozen=True)
class Geometry:
    """One SMS-MUSSELS problem shape plus solver parameters."""
    n: int            # square matrix size N1 = N2
    n_slices: int     # multiband factor L
    n_shots: int      # interleaved shots Ns
    n_coils: int      # receive channels Nc
    filt: int         # Hankel filter support r (r x r)
    lam: float        # regularisation weight lambda
    n_irls: int       # IRLS outer iterations
    n_cg: int         # CG iterations per IRLS step
    phase_order: int  # order of the random shot-phase polynomial
    snr: float        # linear amplitude SNR of the simulated data


# The two single-slice-group workloads: a small case the oracle solves in
# seconds (64^2, MB=2, 4 shots, 8 coils, 5x5 filter, 10x10 iterations) and the
# realistic case throughput is quoted on (256^2, MB=3, 4 shots, 32 coils,
# 7x7 filter, 15x15 iterations).
WORKLOADS = {
    "small": Geometry(n=64, n_slices=2, n_shots=4, n_coils=8, filt=5, lam=1e-3,
                      n_irls=10, n_cg=10, phase_order=2, snr=30.0),
    "sg256": Geometry(n=256, n_slices=3, n_shots=4, n_coils=32, filt=7, lam=1e-3,
                      n_irls=15, n_cg=15, phase_order=3, snr=20.0),
    # an odd-factor matrix size (224 = 7 x 32) at the same multiband and shot
    # counts, for profiling the odd-length column pass
    "sg224": Geometry(n=224, n_slices=3, n_shots=4, n_coils=32, filt=7, lam=1e-3,
                      n_irls=15, n_cg=15, phase_order=3, snr=20.0),
}
WORKLOAD_IDS = {"small": 1, "sg256": 2, "sg224": 3}


def _coords(n):
    t = (np.arange(n) - n / 2) / (n / 2)
    yb, xb = np.meshgrid(t, t, indexing="ij")     # [n2][n1]
    return xb, yb


def ellipse_phantom(rng: np.random.Generator, n: int, n_ellipses: int = 6) -> np.ndarray:
    """Magnitude image [n][n] (float64) of randomly placed filled ellipses."""
    xb, yb = _coords(n)
    img = np.zeros((n, n))
    for _ in range(n_ellipses):
        inten = rng.uniform(0.2, 1.0)
        cx, cy = rng.uniform(-0.4, 0.4, size=2)
        ax, ay = rng.uniform(0.15, 0.45, size=2)
        ang = rng.uniform(0.0, np.pi)
        ca, sa = np.cos(ang), np.sin(ang)
        u = (xb - cx) * ca + (yb - cy) * sa
        v = -(xb - cx) * sa + (yb - cy) * ca
        img[(u / ax) ** 2 + (v / ay) ** 2 <= 1.0] = inten
    return img


def coil_maps(n: int, n_slices: int, n_coils: int, sd: float = 0.8,
              ring: float = 1.0) -> np.ndarray:
    """Complex sensitivities [L][Nc][n][n], unit sum of squares per pixel."""
    xb, yb = _coords(n)
    out = np.empty((n_slices, n_coils, n, n), dtype=np.complex128)
    for l in range(n_slices):
        for c in range(n_coils):
            a = 2 * np.pi * c / n_coils + 2 * np.pi * l / (n_slices * n_coils)
            cx, cy = ring * np.cos(a), ring * np.sin(a)
            bump = np.exp(-((xb - cx) ** 2 + (yb - cy) ** 2) / (2 * sd * sd))
            out[l, c] = bump * np.exp(2j * np.pi * c / n_coils)
        sos = np.sqrt(np.sum(np.abs(out[l]) ** 2, axis=0))
        out[l] /= sos
    return out


def shot_phases(rng: np.random.Generator, n: int, n_shots: int, order: int,
                sd: float = np.pi / 4) -> np.ndarray:
    """Unit-modulus phase images [Ns][n][n] from random 2-D polynomials."""
    xb, yb = _coords(n)
    out = np.empty((n_shots, n, n), dtype=np.complex128)
    for i in range(n_shots):
        arg = np.zeros((n, n))
        for p in range(order + 1):
            for q in range(order + 1 - p):
                arg += rng.normal(0.0, sd) * xb ** p * yb ** q
        out[i] = np.exp(1j * arg)
    return out


def shot_masks(n2: int, n_shots: int) -> np.ndarray:
    """uint8 [Ns][n2]: shot i samples the ky lines j2 with j2 % Ns == i."""
    j2 = np.arange(n2)
    return np.stack([(j2 % n_shots == i) for i in range(n_shots)]).astype(np.uint8)


def caipi_shifts(n_slices: int) -> np.ndarray:
    """Default slice shifts s_l = l/L (fraction of the FOV), l = 0..L-1."""
    return np.arange(n_slices, dtype=np.float64) / n_slices


def make_case(geom: Geometry, seed: int, workload_id: int = 0, noise: bool = True, coils=None) -> dict:
    """All random ingredients of one slice group, rounded to GPU precision.

    Returns a dict with
      rho    float32   [L][n][n]      magnitude phantoms
      phase  complex64 [L][Ns][n][n]  shot phases (unit modulus)
      coils  complex64 [L][Nc][n][n]  sensitivities
      noise  complex64 [Ns][Nc][n][n] unit-variance complex noise (absent when noise=False,
                                      for a consumer that draws it elsewhere)
      masks  uint8     [Ns][n]        ky sampling per shot
      shifts float64   [L]            CAIPI shift fractions
    `coils`: the geometry's maps when already computed (they depend on the
    geometry only); the phantoms and phases do not depend on either option.
    """
    g = geom
    ss = np.random.SeedSequence([int(workload_id), int(seed)])
    r_ph, r_coil, r_phase, r_noise, r_diff = [np.random.Generator(np.random.PCG64(s))
                                              for s in ss.spawn(5)]
    del r_coil, r_diff  # coil maps are deterministic; diffusion scaling unused here
    rho = np.stack([ellipse_phantom(r_ph, g.n) for _ in range(g.n_slices)])
    phase = np.stack([shot_phases(r_phase, g.n, g.n_shots, g.phase_order)
                      for _ in range(g.n_slices)])
    out = {
        "rho": rho.astype(np.float32),
        "phase": phase.astype(np.complex64),
        "coils": (coil_maps(g.n, g.n_slices, g.n_coils) if coils is None else coils).astype(np.complex64),
        "masks": shot_masks(g.n, g.n_shots),
        "shifts": caipi_shifts(g.n_slices),
    }
    if noise:
        shape = (g.n_shots, g.n_coils, g.n, g.n)
        nz = (r_noise.standard_normal(shape) + 1j * r_noise.standard_normal(shape)) / np.sqrt(2.0)
        out["noise"] = nz.astype(np.complex64)
    return out


def random_complex(seed: int, shape, scale: float = 1.0) -> np.ndarray:
    """Seeded complex64 standard-normal array (for operator-level tests)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([99, int(seed)])))
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return (scale * a / np.sqrt(2.0)).astype(np.complex64)


def cnn_init(seed: int, c_io: int, width: int = 64, depth: int = 5, out_scale: float = 0.1) -> list:
    """Initial weights of the learned prior's network: `depth` 3 x 3 layers
    c_io -> width -> ... -> width -> c_io, weights N(0, 2 / (9 c_in)) (He),
    the last layer's scaled by out_scale, biases zero.  Float32 values, as
    the GPU network stores them.  Returns [(w [co][ci][3][3], b [co]), ...]."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 77]))
    chans = [c_io] + [width] * (depth - 1) + [c_io]
    params = []
    for k in range(depth):
        ci, co = chans[k], chans[k + 1]
        w = rng.standard_normal((co, ci, 3, 3)) * np.sqrt(2.0 / (9.0 * ci))
        if k == depth - 1:
            w *= out_scale
        params.append((w.astype(np.float32), np.zeros(co, dtype=np.float32)))
    return params


def direction_case(geom: Geometry, case: dict, direction: int, workload_id: int = 0, noise: bool = True) -> dict:
    """One diffusion direction of a slice group: the same phantoms, coils,
    masks and shifts, the shot phases reseeded, the magnitude scaled by a
    diffusion attenuation factor drawn from U(0.3, 1), and fresh noise
    (absent when noise=False, for a consumer that draws it elsewhere; the
    phases and attenuation do not depend on it)."""
    g = geom
    ss = np.random.SeedSequence([int(workload_id), 5000 + int(direction)])
    r_phase, r_noise, r_att = [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(3)]
    att = r_att.uniform(0.3, 1.0)
    phase = np.stack([shot_phases(r_phase, g.n, g.n_shots, g.phase_order) for _ in range(g.n_slices)])
    out = dict(case)
    out["rho"] = (case["rho"].astype(np.float64) * att).astype(np.float32)
    out["phase"] = phase.astype(np.complex64)
    out.pop("noise", None)
    if noise:
        shape = (g.n_shots, g.n_coils, g.n, g.n)
        nz = (r_noise.standard_normal(shape) + 1j * r_noise.standard_normal(shape)) / np.sqrt(2.0)
        out["noise"] = nz.astype(np.complex64)
    out["attenuation"] = float(att)
    return out
