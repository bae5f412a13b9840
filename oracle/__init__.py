"""FP64 CPU oracle for w-projection gridding with compression -- TEST INFRASTRUCTURE ONLY.

Only tests/, the package smoke check and the benchmark's CPU-baseline leg may import this
package. The product path (the HIP library and its Python binding) never imports it and
shares no code with it.

* `ktable.build`            -- Convolution Function Generator (numpy FFT, scipy PSWF).
* `compress`, `index`       -- WImager preparation phase, plain C (wgrid_oracle.c).
* `grid`, `degrid`          -- eq. gridding and its adjoint, plain C.
* `image.finalise`          -- Algorithm finalizer (inverse FFT, normaliser, taper and
                               oversampling corrections), numpy.
* `per_channel`             -- one grid per channel: each channel's records compressed,
                               gridded and normalised on their own.
* `w_stacking`              -- eq. stacking: records partitioned by w-plane, each part
                               gridded with the w = 0 kernel on a grid of its own.
* `image.finalise_stacked`  -- the w-plane grids transformed, corrected for their w-term in
                               the image plane and added, then finalised.

Pins (tests/test_oracle_pins.py), one or more per function:
  ktable.build / taper     -- Nystrom eigen-equation of the prolate spheroidal, the w = 0
                              kernel as the spheroidal itself, a direct DFT of the padded
                              samples, symmetries, the support law
  ktable.round_to / requantize -- nearest-even rounding cases; zeta as an exactly rounded
                              sum of the stored values, equal to a table built in that type
  index                    -- hand-derived tie rows (tests/golden), nearest plane in sqrt(w)
  compress                 -- brute-force run scan in exact rational arithmetic, adversarial
                              runs, the unit-visibility normaliser, compressed = uncompressed
  grid                     -- delta-kernel histogram, sum invariant, Hermitian flip, one-cell
                              translation, gridding + inverse DFT = image-plane sum
  degrid                   -- the adjoint identity
  per_channel              -- channel grids = shared grid with the other channels' weights
                              zeroed; they and the normalisers add up to the shared ones; the
                              runs are the shared runs of that channel
  w_stacking (+ _degrid)   -- image-plane sum, w = 0 reduces to w-projection, unit source,
                              adjoint
  image.finalise (+ stacked, Stokes) -- unit and off-centre sources, edge zeros, polarised
                              sources at and off the centre
Parity unpinned: none.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import ktable  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wgrid_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (no FMA contraction, plain -O2)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-o", _LIB_PATH, _SRC, "-lm"])
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.or_compress.restype = i64
        L.or_compress.argtypes = [i32, i32, i32, f64, P, P, P, P, P, P, P, P, i64, i32, i32, i32, i32,
                                  P, P, P, P, P, P, P, P, P, P]
        L.or_index.restype = None
        L.or_index.argtypes = [i32, i32, i32, f64, P, P, P, P, P, i64, i32, i32, i32, P]
        L.or_grid.restype = None
        L.or_grid.argtypes = [i32, i32, i32, P, P, P, i64, P, P, P, P, P, P, P]
        L.or_degrid.restype = None
        L.or_degrid.argtypes = [i32, i32, i32, P, P, P, i64, P, P, P, P, P, P, P, P, P, P, P, i64, i32, i32, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return None if a is None else np.ascontiguousarray(a, dtype=dt)


def uv_scale(geom: dict) -> float:
    return float(geom["beta"]) / float(geom["du"])


def _npol(a):
    """Polarisations of a record array: [B][C][T] holds one, [B][C][T][P] holds P."""
    return int(np.shape(a)[3]) if a is not None and np.ndim(a) == 4 else 1


def index(geom, table, uvw, inv_lambda, flag=None):
    """Per-record (X, Y, plane, o_u, o_v, psi, griddable) as int32 [N_rec, 7]; `flag` is
    [B][C][T] or per polarisation [B][C][T][P] (griddable needs one unflagged)."""
    uvw = _c(uvw, np.float64)
    inv_lambda = _c(inv_lambda, np.float64)
    nb, nt = uvw.shape[0], uvw.shape[1]
    nc = inv_lambda.shape[0]
    npol = _npol(flag)
    flag = _c(None if flag is None else np.asarray(flag).reshape(-1), np.uint8)
    out = np.zeros((nb * nc * nt, 7), dtype=np.int32)
    lib().or_index(geom["n"], geom["beta"], geom["n_w"], uv_scale(geom), _p(_c(table["wbound"], np.float64)),
                   _p(_c(table["support"], np.int32)), _p(uvw), _p(inv_lambda), _p(flag), nb, nc, nt, npol,
                   _p(out))
    return out


def compress(geom, table, uvw, inv_lambda, vis, weight=None, flag=None, compress=True):
    """Runs and statistics. `vis` (and `weight`, `flag`) are [B][C][T], or [B][C][T][P] for P
    = 2 or 4 polarisations. Returns dict(start, len, x, y, plane, ou, ov, gamma (complex128,
    [runs] or [runs][P]), stats (n_records, n_griddable, n_runs, n_compressed, upd_real,
    upd_saved), normaliser (a float, or [P]), npol)."""
    uvw = _c(uvw, np.float64)
    inv_lambda = _c(inv_lambda, np.float64)
    nb, nt = uvw.shape[0], uvw.shape[1]
    nc = inv_lambda.shape[0]
    nrec = nb * nc * nt
    npol = _npol(vis)
    vis = np.ascontiguousarray(np.asarray(vis, dtype=np.complex64).reshape(-1)).view(np.float32)
    weight = _c(None if weight is None else np.asarray(weight).reshape(-1), np.float32)
    flag = _c(None if flag is None else np.asarray(flag).reshape(-1), np.uint8)
    arr = {k: np.zeros(max(nrec, 1), dtype=np.int32) for k in ("start", "len", "x", "y", "plane", "ou", "ov")}
    gamma = np.zeros(2 * max(nrec, 1) * npol, dtype=np.float64)
    stats = np.zeros(6, dtype=np.int64)
    norm = np.zeros(npol, dtype=np.float64)
    n = lib().or_compress(geom["n"], geom["beta"], geom["n_w"], uv_scale(geom),
                          _p(_c(table["wbound"], np.float64)), _p(_c(table["support"], np.int32)),
                          _p(_c(table["zeta"], np.float64)), _p(uvw), _p(inv_lambda), _p(vis),
                          _p(weight), _p(flag), nb, nc, nt, npol, int(bool(compress)),
                          _p(arr["start"]), _p(arr["len"]), _p(arr["x"]), _p(arr["y"]), _p(arr["plane"]),
                          _p(arr["ou"]), _p(arr["ov"]), _p(gamma), _p(stats), _p(norm))
    out = {k: v[:n].copy() for k, v in arr.items()}
    gam = gamma[:2 * n * npol].view(np.complex128).copy()
    out["gamma"] = gam if npol == 1 else gam.reshape(n, npol)
    out["stats"] = stats
    out["normaliser"] = float(norm[0]) if npol == 1 else norm
    out["n_runs"] = int(n)
    out["npol"] = npol
    return out


def grid(geom, table, runs, grid_in=None):
    """eq. gridding in FP64 over `runs`; returns a complex128 [n, n] grid, [P, n, n] with P
    polarisations (accumulates onto grid_in when given)."""
    n = geom["n"]
    npol = runs.get("npol", 1)
    shape = (n, n) if npol == 1 else (npol, n, n)
    g = np.zeros(shape, dtype=np.complex128) if grid_in is None else np.array(grid_in, dtype=np.complex128)
    data = np.ascontiguousarray(table["data"], dtype=np.complex128)
    gam = np.ascontiguousarray(runs["gamma"], dtype=np.complex128)
    lib().or_grid(n, geom["beta"], npol, _p(_c(table["support"], np.int32)), _p(_c(table["offset"], np.int64)),
                  _p(data), runs["n_runs"], _p(_c(runs["x"], np.int32)), _p(_c(runs["y"], np.int32)),
                  _p(_c(runs["plane"], np.int32)), _p(_c(runs["ou"], np.int32)), _p(_c(runs["ov"], np.int32)),
                  _p(gam), _p(g))
    return g


def degrid(geom, table, runs, grid_arr, uvw, weight, shape, flag=None):
    """Adjoint of gridding (and of the weighting/flip); returns complex128 of `shape`,
    [B, C, T] or [B, C, T, P]."""
    nb, nc, nt = shape[:3]
    npol = 1 if len(shape) == 3 else int(shape[3])
    uvw = _c(uvw, np.float64)
    weight = _c(None if weight is None else np.asarray(weight).reshape(-1), np.float32)
    flag = _c(None if flag is None else np.asarray(flag).reshape(-1), np.uint8)
    out = np.zeros(nb * nc * nt * npol, dtype=np.complex128)
    g = np.ascontiguousarray(grid_arr, dtype=np.complex128)
    data = np.ascontiguousarray(table["data"], dtype=np.complex128)
    lib().or_degrid(geom["n"], geom["beta"], npol, _p(_c(table["support"], np.int32)),
                    _p(_c(table["offset"], np.int64)), _p(data), runs["n_runs"],
                    _p(_c(runs["start"], np.int32)), _p(_c(runs["len"], np.int32)),
                    _p(_c(runs["x"], np.int32)), _p(_c(runs["y"], np.int32)), _p(_c(runs["plane"], np.int32)),
                    _p(_c(runs["ou"], np.int32)), _p(_c(runs["ov"], np.int32)), _p(g), _p(uvw), _p(weight),
                    _p(flag), nb, nc, nt, _p(out))
    return out.reshape(shape)


def per_channel(geom, table, uvw, inv_lambda, vis, weight=None, flag=None, compress_runs=True):
    """Per-channel imaging as the thesis's imaging tool sets it up (one WImager instance per
    channel): the records of channel c are compressed and gridded on a grid of their own, with
    their own normaliser (eq. normalizer over that channel's records). Returns the per-channel
    run lists, the grids complex128 [C][n][n] and the normalisers [C]."""
    nc = len(inv_lambda)
    runs, grids, norms = [], [], []
    for c in range(nc):
        sl = slice(c, c + 1)
        r = compress(geom, table, uvw, inv_lambda[sl], vis[:, sl, :],
                     None if weight is None else weight[:, sl, :], None if flag is None else flag[:, sl, :],
                     compress_runs)
        runs.append(r)
        grids.append(grid(geom, table, r))
        norms.append(r["normaliser"])
    return runs, np.stack(grids), np.array(norms)


def plane0_table(geom, table):
    """The w = 0 plane of `table` as a one-plane table (with geometry dict(geom, n_w=1))."""
    off = np.asarray(table["offset"], dtype=np.int64)
    zeta = np.asarray(table["zeta"], dtype=np.float64).reshape(geom["n_w"], -1)
    return dict(support=np.asarray(table["support"])[:1], offset=off[:2], wbound=np.asarray(table["wbound"])[:1],
                zeta=zeta[:1].copy(), data=np.asarray(table["data"])[: off[1]])


def w_stacking(geom, table, uvw, inv_lambda, vis, weight=None, flag=None, compress_runs=True):
    """W-stacking (eq. stacking): each record belongs to the w-plane that w-projection would
    give it (nearest plane in sqrt(w), after the flip of eq. conj); the records of plane j are
    compressed and gridded with the w = 0 kernel (plane 0 of `table`: its support, slices and
    zeta) on grid j. Returns the per-plane run lists (on the one-plane table), the grids
    complex128 [n_w][n][n] ([n_w][P][n][n] with P polarisations) and the normaliser (eq.
    normalizer with the w = 0 zeta; one per polarisation)."""
    vis = np.asarray(vis)
    rec_shape = vis.shape[:3]
    k = index(geom, table, uvw, inv_lambda, flag)[:, 2].reshape(rec_shape)
    if vis.ndim == 4:
        k = k[..., None]
    g0, t0 = dict(geom, n_w=1), plane0_table(geom, table)
    base = np.zeros(vis.shape, dtype=bool) if flag is None else (np.asarray(flag).reshape(vis.shape) != 0)
    runs, grids, norm = [], [], 0.0
    for j in range(geom["n_w"]):
        fj = (base | (k != j)).astype(np.uint8)
        r = compress(g0, t0, uvw, inv_lambda, vis, weight, fj, compress_runs)
        runs.append(r)
        grids.append(grid(g0, t0, r))
        norm += r["normaliser"]
    return runs, np.stack(grids), norm


def w_stacking_degrid(geom, table, runs, grids, uvw, weight, shape, flag=None):
    """Adjoint of `w_stacking`'s gridding: every record is read back from the grid of its
    plane with the w = 0 kernel (each record is in one plane's runs at most)."""
    g0, t0 = dict(geom, n_w=1), plane0_table(geom, table)
    out = np.zeros(shape, dtype=np.complex128)
    for j, r in enumerate(runs):
        out += degrid(g0, t0, r, grids[j], uvw, weight, shape, flag)
    return out
