"""Seeded synthetic interferometer workloads (LOFAR/SKA-shaped).

This module only makes inputs. It holds none of the gridding arithmetic, so both the
GPU path and the CPU oracle can consume its output without sharing any method code.

The thesis measures on LOFAR MeasurementSets (ch.5, table tab:datasets) that are not
available here; these workloads stand in for them with the same structure:

* stations uniform in a disk (flat, latitude 52.9 deg), every pair i<j is a baseline;
* records grouped by baseline and time-ordered (sec. 4.4 requires this order);
* earth-rotation uvw tracks at declination 45 deg (textbook rotation, sec. 1.2);
* channels evenly spaced in frequency, uvw stored in metres with 1/lambda per channel
  (sec. 4.4.2 inputs I-1 and I-2);
* visibilities from the measurement equation (sec. 1.3) for seeded point sources plus
  complex Gaussian noise; natural weights of one and no flags.

Record order is [baseline][channel][time] (time fastest), record r = (b*C + ch)*T + t.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

C_LIGHT = 299792458.0
OMEGA_E = 7.2921159e-5          # earth rotation rate, rad/s
LATITUDE_DEG = 52.9
DEC_DEG = 45.0
IMG_C = 3.0 * math.pi           # spheroidal bandwidth c = pi*m/2 for a 6-cell gridding function
DEFAULT_M_IMG = 256             # image samples per side used to build the kernel table

# Workload recipes. Each entry: array, track, band, sky and imaging geometry.
CONFIGS = {
    # Plain w-projection gridding, FP64 oracle case (small; all pins run on it).
    1: dict(n_st=8, radius=2.0e3, n_t=64, dt=10.0, n_ch=4, f_lo=149.0e6, f_hi=151.0e6,
            n_src=5, n=256, beta=8, n_w=8, s_lo=7, s_hi=7),
    # Plain FP32 gridding (the throughput workload).
    2: dict(n_st=44, radius=50.0e3, n_t=512, dt=2.0, n_ch=16, f_lo=120.0e6, f_hi=180.0e6,
            n_src=200, n=2048, beta=8, n_w=32, s_lo=9, s_hi=63),
    # Compression study: 1 s integration, 64 channels, 4096^2 grid.
    3: dict(n_st=44, radius=50.0e3, n_t=512, dt=1.0, n_ch=64, f_lo=120.0e6, f_hi=180.0e6,
            n_src=200, n=4096, beta=8, n_w=64, s_lo=9, s_hi=63),
    # Precision study sub-problem: config-3 array and kernels, 64 timesteps, 8 channels, 512^2.
    4: dict(n_st=44, radius=50.0e3, n_t=64, dt=1.0, n_ch=8, f_lo=120.0e6, f_hi=180.0e6,
            n_src=200, n=512, beta=8, n_w=64, s_lo=9, s_hi=63),
    # Differentiation: 256 stations within 80 km, 4096^2, supports up to 31.
    5: dict(n_st=256, radius=80.0e3, n_t=256, dt=2.0, n_ch=8, f_lo=120.0e6, f_hi=180.0e6,
            n_src=100, n=4096, beta=8, n_w=32, s_lo=7, s_hi=31),
    # Heavy w-projection (the thesis's batch-5 imaging configuration 2: 4500^2 grid, 16
    # w-planes, oversampling 4, supports up to 349), on records shaped like its first LOFAR
    # data set (one channel, 10 s records) at a seventh of its 6.58 M records: 946
    # baselines x 1024 timesteps, to be used with four polarisation products.
    6: dict(n_st=44, radius=50.0e3, n_t=1024, dt=10.0, n_ch=1, f_lo=150.0e6, f_hi=150.0e6,
            n_src=100, n=4500, beta=4, n_w=16, s_lo=9, s_hi=349, m_img=512),
}


@dataclass
class Workload:
    cfg: int
    uvw: np.ndarray            # float64 [B, T, 3], metres
    inv_lambda: np.ndarray     # float64 [C], 1/m
    vis: np.ndarray            # complex64 [B, C, T], or [B, C, T, P] (polarised)
    weight: np.ndarray         # float32, the shape of vis
    flag: np.ndarray           # uint8, the shape of vis
    geom: dict                 # n, beta, n_w, s_lo, s_hi, m_img, du, w_max
    sources: np.ndarray        # float64 [n_src, 3]: l, m, flux
    params: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.vis.shape

    @property
    def n_records(self):
        return int(np.prod(self.vis.shape))


def station_positions(n_st: int, radius: float, seed: int) -> np.ndarray:
    """Stations uniform in a flat disk, returned as local equatorial XYZ (metres)."""
    rng = np.random.default_rng(seed)
    r = radius * np.sqrt(rng.random(n_st))
    th = 2.0 * math.pi * rng.random(n_st)
    e, nn, up = r * np.cos(th), r * np.sin(th), np.zeros(n_st)
    lat = math.radians(LATITUDE_DEG)
    x = -math.sin(lat) * nn + math.cos(lat) * up
    y = e
    z = math.cos(lat) * nn + math.sin(lat) * up
    return np.stack([x, y, z], axis=1)


def baseline_uvw(xyz: np.ndarray, n_t: int, dt: float, dec_deg: float = DEC_DEG) -> np.ndarray:
    """uvw in metres for every baseline i<j over an earth-rotation track, shape [B, T, 3]."""
    i, j = np.triu_indices(xyz.shape[0], k=1)
    L = xyz[j] - xyz[i]                                     # [B, 3]
    h = OMEGA_E * (np.arange(n_t) - n_t / 2.0) * dt         # hour angle per timestep
    d = math.radians(dec_deg)
    sh, ch = np.sin(h)[None, :], np.cos(h)[None, :]
    lx, ly, lz = L[:, 0:1], L[:, 1:2], L[:, 2:3]
    u = sh * lx + ch * ly
    v = -math.sin(d) * ch * lx + math.sin(d) * sh * ly + math.cos(d) * lz
    w = math.cos(d) * ch * lx - math.cos(d) * sh * ly + math.sin(d) * lz
    return np.ascontiguousarray(np.stack([u, v, w], axis=-1))


def _sources(n_src: int, fov: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    lm = (rng.random((n_src, 2)) * 2.0 - 1.0) * 0.4 * fov
    flux = 0.5 + 4.5 * rng.random(n_src)
    return np.concatenate([lm, flux[:, None]], axis=1)


def point_source_vis(uvw: np.ndarray, inv_lambda: np.ndarray, sources: np.ndarray,
                     noise_sigma: float, seed: int, device=None) -> np.ndarray:
    """Measurement-equation visibilities V = sum_s A_s exp(-2 pi i (u l + v m + w (n-1)))
    plus complex Gaussian noise, complex64 [B, C, T]. Uses torch on `device` when given
    (fast path for large workloads), numpy otherwise."""
    B, T, _ = uvw.shape
    C = inv_lambda.shape[0]
    if device is not None:
        import torch
        dev = torch.device(device)
        uvw_t = torch.as_tensor(uvw, dtype=torch.float64, device=dev)
        il = torch.as_tensor(inv_lambda, dtype=torch.float64, device=dev)
        src = torch.as_tensor(sources, dtype=torch.float64, device=dev)
        n = torch.sqrt(1.0 - src[:, 0] ** 2 - src[:, 1] ** 2) - 1.0
        out = torch.empty((B, C, T), dtype=torch.complex64, device=dev)
        bstep = max(1, int(4_000_000 // max(1, T * sources.shape[0])))
        for b0 in range(0, B, bstep):
            b1 = min(B, b0 + bstep)
            # phase per (b, t, s) in metres, scaled per channel
            ph_m = (uvw_t[b0:b1, :, 0:1] * src[None, None, :, 0] + uvw_t[b0:b1, :, 1:2] * src[None, None, :, 1]
                    + uvw_t[b0:b1, :, 2:3] * n[None, None, :])              # [b, T, S]
            for c in range(C):
                ph = (-2.0 * math.pi * il[c]) * ph_m
                acc = torch.complex(torch.cos(ph), torch.sin(ph)) @ src[:, 2].to(torch.complex128)
                out[b0:b1, c, :] = acc.to(torch.complex64)
        g = torch.Generator(device=dev)
        g.manual_seed(seed)
        nr = torch.randn((B, C, T, 2), generator=g, device=dev, dtype=torch.float32) * noise_sigma
        out += torch.complex(nr[..., 0], nr[..., 1])
        return out.cpu().numpy() if dev.type == "cpu" else out
    n = np.sqrt(1.0 - sources[:, 0] ** 2 - sources[:, 1] ** 2) - 1.0
    out = np.empty((B, C, T), dtype=np.complex64)
    for b in range(B):
        ph_m = uvw[b, :, 0:1] * sources[None, :, 0] + uvw[b, :, 1:2] * sources[None, :, 1] + uvw[b, :, 2:3] * n[None, :]
        for c in range(C):
            out[b, c, :] = (np.exp(-2j * math.pi * inv_lambda[c] * ph_m) @ sources[:, 2]).astype(np.complex64)
    rng = np.random.default_rng(seed)
    nz = rng.standard_normal((B, C, T, 2)).astype(np.float32) * np.float32(noise_sigma)
    out += nz[..., 0] + 1j * nz[..., 1]
    return out


def make(cfg: int, device=None, **overrides) -> Workload:
    """Build workload `cfg` (1..5). `overrides` replace recipe entries (n_st, n_t, n_ch, n,
    n_src, ...) for reduced test sizes. With `device` set, visibilities are computed there
    with torch and returned as a device tensor."""
    p = dict(CONFIGS[cfg])
    p.update(overrides)
    p.setdefault("m_img", DEFAULT_M_IMG)
    xyz = station_positions(p["n_st"], p["radius"], 1000 + cfg)
    uvw = baseline_uvw(xyz, p["n_t"], p["dt"])
    freqs = np.linspace(p["f_lo"], p["f_hi"], p["n_ch"]) if p["n_ch"] > 1 else np.array([p["f_lo"]])
    inv_lambda = freqs / C_LIGHT
    max_uv = max(np.abs(uvw[..., 0]).max(), np.abs(uvw[..., 1]).max()) * inv_lambda.max()
    du = 2.0 * max_uv / (0.9 * p["n"])
    w_max = float(np.abs(uvw[..., 2]).max() * inv_lambda.max())
    sources = _sources(p["n_src"], 1.0 / du, 2000 + cfg)
    vis = point_source_vis(uvw, inv_lambda, sources, 0.1, 3000 + cfg, device=device)
    B, T = uvw.shape[:2]
    C = inv_lambda.shape[0]
    if device is not None and not isinstance(vis, np.ndarray):
        import torch
        weight = torch.ones((B, C, T), dtype=torch.float32, device=vis.device)
        flag = torch.zeros((B, C, T), dtype=torch.uint8, device=vis.device)
    else:
        weight = np.ones((B, C, T), dtype=np.float32)
        flag = np.zeros((B, C, T), dtype=np.uint8)
    geom = dict(n=p["n"], beta=p["beta"], n_w=p["n_w"], s_lo=p["s_lo"], s_hi=p["s_hi"],
                m_img=p["m_img"], du=float(du), w_max=w_max)
    return Workload(cfg, uvw, inv_lambda, vis, weight, flag, geom, sources, p)


def polarised(cfg: int, n_pol: int = 4, circular: bool = False, device=None, flag_frac: float = 0.02,
              **overrides) -> Workload:
    """Workload `cfg` with P = n_pol products per record, [B, C, T, P]. Every source of the
    total-intensity workload gets seeded fractional polarisation (|Q|, |U|, |V| up to 0.3 of
    I); the products follow the feed relations XX = I + Q, XY = U + iV, YX = U - iV,
    YY = I - Q (circular: RR = I + V, RL = Q + iU, LR = Q - iU, LL = I - V), P = 2 keeping
    the parallel hands; each product gets its own noise (sigma 0.1), its own natural weight
    (uniform 0.5..2, as from per-polarisation variances) and `flag_frac` of flags, and one
    record in 200 is flagged in every product."""
    assert n_pol in (2, 4)
    w = make(cfg, device=device, **overrides)
    rng = np.random.default_rng(5000 + cfg)
    S = w.sources.shape[0]
    frac = rng.uniform(-0.3, 0.3, (S, 3))
    stokes = [w.vis]
    for k in range(3):
        src = w.sources.copy()
        src[:, 2] = w.sources[:, 2] * frac[:, k]
        stokes.append(point_source_vis(w.uvw, w.inv_lambda, src, 0.0, 3100 + 10 * cfg + k, device=device))
    if device is not None and not isinstance(w.vis, np.ndarray):
        import torch
        xp_stack, j = torch.stack, 1j
    else:
        xp_stack, j = np.stack, 1j
    I, Q, U, V = stokes
    if circular:
        prods = [I + V, Q + j * U, Q - j * U, I - V]
    else:
        prods = [I + Q, U + j * V, U - j * V, I - Q]
    if n_pol == 2:
        prods = [prods[0], prods[3]]
    B, C, T = w.vis.shape
    shp = (B, C, T, n_pol)
    noise = rng.standard_normal(shp + (2,)).astype(np.float32) * np.float32(0.1)
    wt = rng.uniform(0.5, 2.0, shp).astype(np.float32)
    fl = (rng.uniform(size=shp) < flag_frac).astype(np.uint8)
    fl[rng.uniform(size=(B, C, T)) < 0.005] = 1
    if device is not None and not isinstance(w.vis, np.ndarray):
        import torch
        vis = xp_stack(prods, -1).to(torch.complex64)
        nz = torch.as_tensor(noise, device=vis.device)
        vis = vis + torch.complex(nz[..., 0], nz[..., 1])
        wt, fl = torch.as_tensor(wt, device=vis.device), torch.as_tensor(fl, device=vis.device)
    else:
        vis = (xp_stack(prods, -1) + noise[..., 0] + 1j * noise[..., 1]).astype(np.complex64)
    p = dict(w.params, n_pol=n_pol, circular=circular)
    return Workload(cfg, w.uvw, w.inv_lambda, vis, wt, fl, w.geom, w.sources, p)


def target_image(w: Workload, n_src: int = 100, seed: int = 4000) -> np.ndarray:
    """A seeded model sky for the differentiation workload: n_src point sources of flux
    U[0.5, 5] placed on image pixels inside the central 80 % of an N x N image whose pixel
    size is FOV/N = 1/(N du); float64 [N, N], row = m, column = l, centre at N/2."""
    n = w.geom["n"]
    rng = np.random.default_rng(seed + w.cfg)
    img = np.zeros((n, n))
    lim = int(0.4 * n)
    pix = rng.integers(-lim, lim + 1, size=(n_src, 2))
    flux = 0.5 + 4.5 * rng.random(n_src)
    np.add.at(img, (n // 2 + pix[:, 1], n // 2 + pix[:, 0]), flux)
    return img
