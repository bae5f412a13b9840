"""Image finaliser of the oracle -- TEST INFRASTRUCTURE ONLY (the GPU library never imports it).

Algorithm finalizer, one polarisation:

1. inverse 2-D Fourier transform of the UV-grid. Grid cell [row][col] holds (u, v) =
   ((col - N/2) du, (row - N/2) du); image pixel [q][p] holds (l, m) = ((p - N/2), (q - N/2))
   / (N du), i.e. the field of view 1/du sampled N times (eq. convgrid), with
   img(l, m) = sum_cells G e^{+2 pi i (u l + v m)};
2. the real part (each record is gridded once, at its w >= 0 representative of eq. conj; its
   Hermitian partner would add the complex conjugate), divided by the normaliser N_p
   (eq. normalizer) to give Jy/beam;
3. division by the tapering function c(l) c(m) (sec. convgriddingmath), the prolate
   spheroidal psi_0(3 pi, 2 l / FOV), normalised to 1 at the centre;
4. division by sinc(pi l du / beta) sinc(pi m du / beta), the attenuation by the nearest
   oversampled kernel sample (eq. coversampled).

W-stacking (eq. stacking) transforms each w-plane grid, multiplies it by the plane's w-term
correction exp(+2 pi i w_k (sqrt(1 - l^2 - m^2) - 1)) in the image plane (0 where l^2 + m^2
> 1), the factor that the w-projection kernel of plane k carries (eq. C_W), and adds the
planes before step 2.

Polarisations (step 2, "convert to multiple-Stokes image and normalise"): each polarised
grid is transformed and divided by its own normaliser N_p, then the Stokes images are the
real parts of the usual linear combinations (the thesis names the outputs, I, Q, U, V or the
subset the polarisations allow, not the formulas; these are the standard feed relations):
  linear   XX = I + Q, XY = U + iV, YX = U - iV, YY = I - Q;
  circular RR = I + V, RL = Q + iU, LR = Q - iU, LL = I - V;
so two parallel hands give (I, Q) or (I, V), four give (I, Q, U, V), and one polarisation
is imaged as it is, as I. A polarisation whose normaliser is 0 (all flagged) adds 0.

Pixels where the taper is zero (l or m = -FOV/2, the first row and column) are set to 0, and
so is the whole image when the normaliser is 0 (nothing was gridded; the thesis leaves this
case open).
"""
from __future__ import annotations

import numpy as np

from .ktable import plane_w, taper


def axis_correction(geom: dict) -> np.ndarray:
    """c(l)/c(0) * sinc(pi l du / beta) for the N pixels of one axis (steps 3 and 4)."""
    n, beta = geom["n"], geom["beta"]
    # x = 2 l / FOV = 2 (p - N/2) / N, taken exactly (the first pixel sits at x = -1 whatever
    # du is; going through l = (p - N/2) / (N du) would round it to inside the interval)
    x = 2.0 * (np.arange(n) - n // 2) / n
    t = taper(x) / taper(np.zeros(1))[0]
    return t * np.sinc(x / (2.0 * beta))        # l du / beta; numpy sinc(x) = sin(pi x) / (pi x)


def transform(geom: dict, grid: np.ndarray) -> np.ndarray:
    """Step 1: sum_cells G e^{+2 pi i (u l + v m)} at every pixel, complex [N][N]."""
    n = geom["n"]
    g = np.asarray(grid, dtype=np.complex128)
    return np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(g))) * float(n * n)


def w_correction(geom: dict, k: int) -> np.ndarray:
    """exp(+2 pi i w_k (n - 1)), n = sqrt(1 - l^2 - m^2), at every pixel [q (m)][p (l)] for
    w-plane k (0 where l^2 + m^2 > 1)."""
    n, du = geom["n"], geom["du"]
    lm = (np.arange(n) - n // 2) / (n * du)
    rr = 1.0 - lm[None, :] ** 2 - lm[:, None] ** 2
    w = plane_w(k, geom["n_w"], geom["w_max"])
    f = np.exp(2j * np.pi * w * (np.sqrt(np.maximum(rr, 0.0)) - 1.0))
    f[rr < 0.0] = 0.0
    return f


def stacked_transform(geom: dict, grids: np.ndarray) -> np.ndarray:
    """Eq. stacking before step 2: sum over planes k of transform(G_k) * w_correction(k)."""
    out = np.zeros((geom["n"], geom["n"]), dtype=np.complex128)
    for k in range(geom["n_w"]):
        out += transform(geom, grids[k]) * w_correction(geom, k)
    return out


def finalise_stacked(geom: dict, grids: np.ndarray, normaliser: float) -> np.ndarray:
    """Dirty image from the [n_w][N][N] w-plane grids of w-stacking."""
    if normaliser == 0.0:
        return np.zeros((geom["n"], geom["n"]))
    return _steps_2_to_4(geom, stacked_transform(geom, grids), normaliser)


def finalise(geom: dict, grid: np.ndarray, normaliser: float) -> np.ndarray:
    """Dirty image, float64 [N][N] (row m, column l), from a complex [N][N] grid."""
    n = geom["n"]
    if normaliser == 0.0:
        return np.zeros((n, n))
    return _steps_2_to_4(geom, transform(geom, grid), normaliser)


def _steps_2_to_4(geom: dict, img: np.ndarray, normaliser: float) -> np.ndarray:
    n = geom["n"]
    c = axis_correction(geom)
    corr = np.outer(c, c)
    out = np.zeros((n, n))
    nz = corr != 0.0
    out[nz] = img.real[nz] / (normaliser * corr[nz])
    return out


# Stokes images from the polarised images: name, coefficient of each polarisation
STOKES = {
    (1, False): [("I", (1.0,))],
    (1, True): [("I", (1.0,))],
    (2, False): [("I", (0.5, 0.5)), ("Q", (0.5, -0.5))],
    (2, True): [("I", (0.5, 0.5)), ("V", (0.5, -0.5))],
    (4, False): [("I", (0.5, 0, 0, 0.5)), ("Q", (0.5, 0, 0, -0.5)), ("U", (0, 0.5, 0.5, 0)),
                 ("V", (0, -0.5j, 0.5j, 0))],
    (4, True): [("I", (0.5, 0, 0, 0.5)), ("Q", (0, 0.5, 0.5, 0)), ("U", (0, -0.5j, 0.5j, 0)),
                ("V", (0.5, 0, 0, -0.5))],
}


def finalise_stokes(geom: dict, grid: np.ndarray, normalisers, circular: bool = False) -> dict:
    """Dirty Stokes images {name: float64 [N][N]} from a [P][N][N] polarised grid (P = 1, 2
    or 4) and its per-polarisation normalisers."""
    g = np.asarray(grid, dtype=np.complex128)
    if g.ndim == 2:
        g = g[None]
    return _stokes(geom, [transform(geom, g[p]) for p in range(g.shape[0])], normalisers, circular)


def finalise_stokes_stacked(geom: dict, grids: np.ndarray, normalisers, circular: bool = False) -> dict:
    """Stokes images of w-stacking with P polarisations: each product's plane grids
    ([n_w][P][N][N]) stacked as in `stacked_transform`, then the Stokes steps."""
    g = np.asarray(grids, dtype=np.complex128)
    return _stokes(geom, [stacked_transform(geom, g[:, p]) for p in range(g.shape[1])], normalisers, circular)


def _stokes(geom: dict, transforms, normalisers, circular: bool) -> dict:
    npol = len(transforms)
    norms = np.atleast_1d(np.asarray(normalisers, dtype=np.float64))
    pol_img = []
    for p in range(npol):
        pol_img.append(transforms[p] / norms[p] if norms[p] != 0.0 else None)
    c = axis_correction(geom)
    corr = np.outer(c, c)
    nz = corr != 0.0
    out = {}
    for name, coef in STOKES[(npol, bool(circular))]:
        acc = np.zeros((geom["n"], geom["n"]), dtype=np.complex128)
        for p in range(npol):
            if coef[p] != 0 and pol_img[p] is not None:
                acc += coef[p] * pol_img[p]
        img = np.zeros((geom["n"], geom["n"]))
        img[nz] = acc.real[nz] / corr[nz]
        out[name] = img
    return out
