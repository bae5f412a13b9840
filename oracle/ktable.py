"""Oracle kernel table -- TEST INFRASTRUCTURE ONLY (numpy/scipy, FP64).

Follows the Convolution Function Generator (Algorithm convgen and the text after it):
for every w-plane, sample the image-plane function (taper times the inverse w-screen) on an
M x M grid, zero-pad to beta*M, apply a forward FFT, normalise by the w=0 plane's centre
value, find the support from the 1e-3 magnitude threshold, trim, and reorder into one
S x S matrix per oversample offset pair (the "image of M(w,u,v)" of eq. choose), with the
per-matrix sums of real parts of eq. sum.

Readings (the thesis leaves these open):
  * taper: separable prolate spheroidal psi_0(c, x) with c = 3*pi (6-cell support), on
    x = 2 l / FOV; zero on |x| >= 1, the boundary excluded by rect() in eq. convgrid.
    Evaluated with scipy.special.pro_ang1.
  * image samples l_p = (p - M/2) FOV / M, p in [0, M); FOV = 1/du.
  * image-plane w factor exp(+2 pi i w (sqrt(1-l^2-m^2) - 1)), the inverse of g_w in the
    w-projection treatment (eqs. localconv2, C_W), with plane w_k = w_max (k/(n_w-1))^2
    (sqrt(w) spacing).
  * forward FFT e^{-2 pi i}, centred indices on both sides.
  * support: k_max = largest Chebyshev fine-index distance from the centre with
    |C| > 1e-3, r = max(0, ceil((k_max - beta/2)/beta)), S_nat = 2r+1; the throughput
    configurations pad/trim (normal-mode behaviour) to
    S_k = min(s_hi, max(S_nat, s_lo + 2*floor(((s_hi-s_lo)*k + n_w-1) / (2(n_w-1))))).
  * matrix for offsets (o_u, o_v), o in (-beta/2, beta/2]: element [i][j] is the fine sample
    at ((i-H) beta - o_v, (j-H) beta - o_u), H = (S-1)/2; matrices ordered o_v-major.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.special as sps

TAPER_C = 3.0 * math.pi
SUPPORT_THRESHOLD = 1e-3


def taper(x: np.ndarray) -> np.ndarray:
    """psi_0(c=3 pi, x) on |x| < 1, zero elsewhere (scipy's prolate angular function)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    inside = np.abs(x) < 1.0
    out[inside] = sps.pro_ang1(0, 0, TAPER_C, x[inside])[0]
    return out


def w_bounds(n_w: int, w_max: float) -> np.ndarray:
    """Lower edge of each w-plane (entry 0 unused): nearest plane in sqrt(w)."""
    wb = np.zeros(n_w, dtype=np.float64)
    for j in range(1, n_w):
        q = (j - 0.5) / (n_w - 1)
        wb[j] = w_max * (q * q)
    return wb


def plane_w(k: int, n_w: int, w_max: float) -> float:
    if n_w == 1:
        return 0.0
    q = k / (n_w - 1)
    return w_max * (q * q)


def support_law(k: int, n_w: int, s_lo: int, s_hi: int) -> int:
    if n_w == 1:
        return s_lo
    return s_lo + 2 * (((s_hi - s_lo) * k + (n_w - 1)) // (2 * (n_w - 1)))


def image_plane(geom: dict, k: int) -> np.ndarray:
    """Image-plane samples f[q][p] (rows follow m / v, columns l / u) for plane k."""
    M = geom["m_img"]
    x = 2.0 * (np.arange(M) - M / 2) / M
    lm = x / (2.0 * geom["du"])
    t = taper(x)
    w = plane_w(k, geom["n_w"], geom["w_max"])
    rr = 1.0 - lm[None, :] ** 2 - lm[:, None] ** 2
    nm1 = np.sqrt(np.maximum(rr, 0.0)) - 1.0
    f = (t[:, None] * t[None, :]) * np.exp(2j * math.pi * w * nm1)
    f[rr < 0.0] = 0.0
    return f


def fine_plane(geom: dict, k: int) -> np.ndarray:
    """Un-normalised oversampled kernel, L x L with L = beta*M, index [L/2+fv][L/2+fu]."""
    M, L = geom["m_img"], geom["beta"] * geom["m_img"]
    P = np.zeros((L, L), dtype=np.complex128)
    o = L // 2 - M // 2
    P[o:o + M, o:o + M] = image_plane(geom, k)
    return np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(P)))


def natural_support(C: np.ndarray, beta: int) -> tuple[int, int]:
    L = C.shape[0]
    f = np.arange(L) - L // 2
    cheb = np.maximum(np.abs(f)[:, None], np.abs(f)[None, :])
    above = np.abs(C) > SUPPORT_THRESHOLD
    kmax = int(cheb[above].max()) if above.any() else 0
    r = max(0, math.ceil((kmax - beta / 2) / beta))
    return 2 * r + 1, kmax


def round_bf16(x: np.ndarray) -> np.ndarray:
    """Round-to-nearest-even from FP64 straight to bfloat16 (8 significant bits, FP32
    exponent range, gradual underflow at 2^-133), returned as float64 values."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    fin = np.isfinite(x) & (x != 0.0)
    m, e = np.frexp(x[fin])                 # x = m 2^e, 0.5 <= |m| < 1
    e = e.astype(np.int64)
    # quantum of the result: 2^(e-8) for normal values, 2^-133 below 2^-126
    qexp = np.maximum(e - 8, -133)
    scaled = np.ldexp(x[fin], -qexp)
    r = np.ldexp(np.round(scaled), qexp)    # np.round is half-to-even
    big = np.abs(r) > float(np.ldexp(np.float64(0xFF), 120))   # > max bf16 (0x7F7F)
    r[big] = np.copysign(np.inf, r[big])
    out[fin] = r
    out[~np.isfinite(x)] = x[~np.isfinite(x)]
    return out


def round_to(x: np.ndarray, dtype: str) -> np.ndarray:
    if dtype == "f64":
        return x
    if dtype == "f32":
        return x.astype(np.float32).astype(np.float64)
    if dtype == "f16":
        return x.astype(np.float16).astype(np.float64)
    if dtype == "bf16":
        return round_bf16(x)
    raise ValueError(dtype)


def build(geom: dict, dtype: str = "f64", keep_fine: bool = False) -> dict:
    """Full table for `geom` (keys n, beta, n_w, s_lo, s_hi, m_img, du, w_max).
    Returns support[n_w], offset[n_w+1] (complex elements), wbound[n_w],
    zeta[n_w, beta^2], data (complex128, values rounded to `dtype`), s_nat, kmax, c00."""
    beta, n_w = geom["beta"], geom["n_w"]
    L = beta * geom["m_img"]
    planes, s_nat, kmax = [], [], []
    c00 = None
    for k in range(n_w):
        C = fine_plane(geom, k)
        if k == 0:
            c00 = C[L // 2, L // 2].real
        C = C / c00
        sn, km = natural_support(C, beta)
        planes.append(C)
        s_nat.append(sn)
        kmax.append(km)
    support = np.array([min(geom["s_hi"], max(s_nat[k], support_law(k, n_w, geom["s_lo"], geom["s_hi"])))
                        for k in range(n_w)], dtype=np.int32)
    offset = np.zeros(n_w + 1, dtype=np.int64)
    for k in range(n_w):
        offset[k + 1] = offset[k] + beta * beta * int(support[k]) ** 2
    data = np.zeros(int(offset[-1]), dtype=np.complex128)
    zeta = np.zeros((n_w, beta * beta), dtype=np.float64)
    o = np.arange(-beta // 2 + 1, beta // 2 + 1)
    for k in range(n_w):
        S = int(support[k])
        H = (S - 1) // 2
        d = np.arange(S) - H
        # fv[ov, i] and fu[ou, j]
        fv = d[None, :] * beta - o[:, None]
        fu = d[None, :] * beta - o[:, None]
        C = planes[k]
        K = C[L // 2 + fv[:, None, :, None], L // 2 + fu[None, :, None, :]]   # [ov, ou, i, j]
        K = round_to(K.real, dtype) + 1j * round_to(K.imag, dtype)
        data[offset[k]:offset[k + 1]] = K.reshape(-1)
        zeta[k] = K.real.reshape(beta * beta, S * S).sum(axis=1)
    out = dict(support=support, offset=offset, wbound=w_bounds(n_w, geom["w_max"]), zeta=zeta,
               data=data, s_nat=np.array(s_nat), kmax=np.array(kmax), c00=c00, dtype=dtype)
    if keep_fine:
        out["fine"] = planes
    return out


def requantize(table64: dict, dtype: str) -> dict:
    """The same table with its samples rounded to `dtype` and zeta re-summed (eq. sum)."""
    out = dict(table64)
    d = table64["data"]
    out["data"] = round_to(d.real, dtype) + 1j * round_to(d.imag, dtype)
    beta = int(np.sqrt(table64["zeta"].shape[1]))
    zeta = np.zeros_like(table64["zeta"])
    for k, S in enumerate(table64["support"]):
        seg = out["data"][table64["offset"][k]:table64["offset"][k + 1]].real
        zeta[k] = seg.reshape(beta * beta, int(S) * int(S)).sum(axis=1)
    out["zeta"] = zeta
    out["dtype"] = dtype
    out.pop("fine", None)
    return out
