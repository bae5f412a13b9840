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

Pixels where the taper is zero (l or m = -FOV/2, the first row and column) are set to 0, and
so is the whole image when the normaliser is 0 (nothing was gridded; the thesis leaves this
case open).
"""
from __future__ import annotations

import numpy as np

from .ktable import taper


def axis_correction(geom: dict) -> np.ndarray:
    """c(l)/c(0) * sinc(pi l du / beta) for the N pixels of one axis (steps 3 and 4)."""
    n, beta = geom["n"], geom["beta"]
    # x = 2 l / FOV = 2 (p - N/2) / N, taken exactly (the first pixel sits at x = -1 whatever
    # du is; going through l = (p - N/2) / (N du) would round it to inside the interval)
    x = 2.0 * (np.arange(n) - n // 2) / n
    t = taper(x) / taper(np.zeros(1))[0]
    return t * np.sinc(x / (2.0 * beta))        # l du / beta; numpy sinc(x) = sin(pi x) / (pi x)


def finalise(geom: dict, grid: np.ndarray, normaliser: float) -> np.ndarray:
    """Dirty image, float64 [N][N] (row m, column l), from a complex [N][N] grid."""
    n = geom["n"]
    if normaliser == 0.0:
        return np.zeros((n, n))
    g = np.asarray(grid, dtype=np.complex128)
    img = np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(g))) * float(n * n)
    c = axis_correction(geom)
    corr = np.outer(c, c)
    out = np.zeros((n, n))
    nz = corr != 0.0
    out[nz] = img.real[nz] / (normaliser * corr[nz])
    return out
