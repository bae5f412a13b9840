"""Python binding of libwgrid (the C ABI in include/wgrid.h).

Argument marshalling only: every step of the computation runs in the HIP library. PyTorch
supplies device memory and the current stream. Functions named like the C entry points take
torch tensors and raise `WgError` on a non-zero status. The classes below own the buffers a
call sequence needs (table, runs, statistics) and `GridFn` wraps grid/degrid as a
torch.autograd.Function (forward = compress + grid, backward = degrid, the exact adjoint).

The library must be built in-tree (`python -m paper_1403_4209_amd.build`); importing this
module without it raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwgrid.so")

WG_OK, WG_EINVAL, WG_ECAPACITY, WG_EHIP, WG_EUNSUPPORTED = 0, -1, -3, -4, -5
WG_KF32, WG_KBF16, WG_KF16 = 0, 1, 2
WG_COMPRESS = 1
WG_GRID_PER_CHANNEL = 2
WG_W_STACKING = 4
WG_POL_CIRCULAR = 8
WG_PLAIN_SUMS = 16
DTYPES = {"f32": WG_KF32, "bf16": WG_KBF16, "f16": WG_KF16}
_ELEM_BYTES = {WG_KF32: 8, WG_KBF16: 4, WG_KF16: 4}


class WgError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {wg_status_str(status)} ({status})")
        self.status = status


class WgGeom(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("beta", ctypes.c_int32), ("n_w", ctypes.c_int32),
                ("s_lo", ctypes.c_int32), ("s_hi", ctypes.c_int32), ("m_img", ctypes.c_int32),
                ("du", ctypes.c_double), ("w_max", ctypes.c_double), ("flags", ctypes.c_uint32),
                ("n_pol", ctypes.c_int32)]


class WgKtable(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("n_w", ctypes.c_int32), ("beta", ctypes.c_int32),
                ("s_max", ctypes.c_int32), ("support", ctypes.c_void_p), ("offset", ctypes.c_void_p),
                ("wbound", ctypes.c_void_p), ("zeta", ctypes.c_void_p), ("data", ctypes.c_void_p),
                ("data_cap", ctypes.c_int64)]


class WgRuns(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_int64), ("start", ctypes.c_void_p), ("len", ctypes.c_void_p),
                ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("plane", ctypes.c_void_p),
                ("ou", ctypes.c_void_p), ("ov", ctypes.c_void_p), ("gamma", ctypes.c_void_p),
                ("plan", ctypes.c_void_p), ("plan_elems", ctypes.c_int64), ("work", ctypes.c_void_p),
                ("grid", ctypes.c_void_p), ("norm", ctypes.c_void_p)]


_lib = None


def lib():
    """Load libwgrid.so (after torch, so both use torch's HIP runtime)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1403_4209_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.wg_status_str.restype = ctypes.c_char_p
        L.wg_status_str.argtypes = [ctypes.c_int]
        L.wg_version.restype = ctypes.c_int
        L.wg_ktable_sizes.restype = ctypes.c_int
        L.wg_ktable_sizes.argtypes = [P, P, P]
        L.wg_ktable_build.restype = ctypes.c_int
        L.wg_ktable_build.argtypes = [P, P, P, ctypes.c_size_t, P, P, P]
        L.wg_plan_elems.restype = I64
        L.wg_plan_elems.argtypes = [I64, I64]
        L.wg_compress.restype = ctypes.c_int
        L.wg_compress.argtypes = [P, P, P, P, P, P, P, I64, I32, I32, P, P, P]
        L.wg_grid.restype = ctypes.c_int
        L.wg_grid.argtypes = [P, P, P, P, P, P]
        L.wg_grid_records_ws.restype = ctypes.c_int
        L.wg_grid_records_ws.argtypes = [P, I64, I32, I32, P, P, P]
        L.wg_grid_records.restype = ctypes.c_int
        L.wg_grid_records.argtypes = [P, P, P, P, P, P, P, I64, I32, I32, P, P, P, ctypes.c_size_t, P, P]
        L.wg_grid_records_static.restype = ctypes.c_int
        L.wg_grid_records_static.argtypes = [P, P, P, P, P, P, P, I64, I32, I32, P, P, P, P]
        L.wg_degrid.restype = ctypes.c_int
        L.wg_degrid.argtypes = [P, P, P, P, P, P, P, P, I64, I32, I32, P, P]
        L.wg_finalise_ws_bytes.restype = ctypes.c_int
        L.wg_finalise_ws_bytes.argtypes = [P, P]
        L.wg_finalise.restype = ctypes.c_int
        L.wg_finalise.argtypes = [P, P, P, P, P, ctypes.c_size_t, P]
        L.wg_finalise_stacked.restype = ctypes.c_int
        L.wg_finalise_stacked.argtypes = [P, P, P, P, P, ctypes.c_size_t, P]
        _lib = L
    return _lib


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check(status: int, where: str):
    if status != WG_OK:
        raise WgError(status, where)


# ------------------------------------------------------------------------- C entry points
def wg_status_str(status: int) -> str:
    return lib().wg_status_str(int(status)).decode()


def wg_version() -> int:
    return int(lib().wg_version())


def wg_ktable_sizes(geom: WgGeom) -> tuple[int, int]:
    n = ctypes.c_int64(0)
    ws = ctypes.c_size_t(0)
    _check(lib().wg_ktable_sizes(ctypes.byref(geom), ctypes.byref(n), ctypes.byref(ws)), "wg_ktable_sizes")
    return int(n.value), int(ws.value)


def wg_ktable_build(geom: WgGeom, kt: WgKtable, ws: torch.Tensor, stream=None, host_copies=True):
    """Build the table into kt's device arrays. With host_copies the call waits and returns
    (supports, offsets); without, it only enqueues work (kt.data_cap must hold every plane
    at s_hi) and returns None."""
    if not host_copies:
        _check(lib().wg_ktable_build(ctypes.byref(geom), ctypes.byref(kt), _p(ws), ws.numel() * ws.element_size(),
                                     None, None, _stream(stream)), "wg_ktable_build")
        return None
    sup = (ctypes.c_int32 * geom.n_w)()
    off = (ctypes.c_int64 * (geom.n_w + 1))()
    _check(lib().wg_ktable_build(ctypes.byref(geom), ctypes.byref(kt), _p(ws), ws.numel() * ws.element_size(),
                                 sup, off, _stream(stream)), "wg_ktable_build")
    return list(sup), list(off)


def wg_plan_elems(capacity: int, n_segments: int) -> int:
    return int(lib().wg_plan_elems(int(capacity), int(n_segments)))


def wg_compress(geom, kt, uvw, inv_lambda, vis, weight, flag, nb, nc, nt, runs: WgRuns, stats: torch.Tensor,
                stream=None):
    _check(lib().wg_compress(ctypes.byref(geom), ctypes.byref(kt), _p(uvw), _p(inv_lambda), _p(vis), _p(weight),
                             _p(flag), int(nb), int(nc), int(nt), ctypes.byref(runs), _p(stats), _stream(stream)),
           "wg_compress")


def wg_grid(geom, kt, runs: WgRuns, stats: torch.Tensor, grid: torch.Tensor, stream=None):
    _check(lib().wg_grid(ctypes.byref(geom), ctypes.byref(kt), ctypes.byref(runs), _p(stats), _p(grid),
                         _stream(stream)), "wg_grid")


def wg_grid_records_ws(geom: WgGeom, nb: int, nc: int, nt: int, ws: torch.Tensor | None = None):
    """Without `ws`: the workspace size in bytes. With `ws` (a device byte tensor): the
    WgRuns view of it that wg_grid_records fills."""
    size = ctypes.c_size_t(0 if ws is None else ws.numel() * ws.element_size())
    if ws is None:
        _check(lib().wg_grid_records_ws(ctypes.byref(geom), int(nb), int(nc), int(nt), None, ctypes.byref(size),
                                        None), "wg_grid_records_ws")
        return int(size.value)
    runs = WgRuns()
    _check(lib().wg_grid_records_ws(ctypes.byref(geom), int(nb), int(nc), int(nt), _p(ws), ctypes.byref(size),
                                    ctypes.byref(runs)), "wg_grid_records_ws")
    return runs


def wg_grid_records(geom, kt, uvw, inv_lambda, vis, weight, flag, nb, nc, nt, grid, stats, ws: torch.Tensor,
                    stream=None):
    runs = WgRuns()
    _check(lib().wg_grid_records(ctypes.byref(geom), ctypes.byref(kt), _p(uvw), _p(inv_lambda), _p(vis), _p(weight),
                                 _p(flag), int(nb), int(nc), int(nt), _p(grid), _p(stats), _p(ws),
                                 ws.numel() * ws.element_size(), ctypes.byref(runs), _stream(stream)),
           "wg_grid_records")
    return runs


def wg_grid_records_static(geom, kt, uvw, inv_lambda, vis, weight, flag, nb, nc, nt, grid, stats, stream=None):
    """wg_grid_records with the library's own fixed device array as workspace (allocates
    nothing); returns the WgRuns view of that array on the current device."""
    runs = WgRuns()
    _check(lib().wg_grid_records_static(ctypes.byref(geom), ctypes.byref(kt), _p(uvw), _p(inv_lambda), _p(vis),
                                        _p(weight), _p(flag), int(nb), int(nc), int(nt), _p(grid), _p(stats),
                                        ctypes.byref(runs), _stream(stream)), "wg_grid_records_static")
    return runs


def wg_degrid(geom, kt, runs: WgRuns, stats, grid, uvw, weight, flag, nb, nc, nt, vis_out, stream=None):
    _check(lib().wg_degrid(ctypes.byref(geom), ctypes.byref(kt), ctypes.byref(runs), _p(stats), _p(grid), _p(uvw),
                           _p(weight), _p(flag), int(nb), int(nc), int(nt), _p(vis_out), _stream(stream)),
           "wg_degrid")


def wg_finalise_ws_bytes(geom: WgGeom) -> int:
    ws = ctypes.c_size_t(0)
    _check(lib().wg_finalise_ws_bytes(ctypes.byref(geom), ctypes.byref(ws)), "wg_finalise_ws_bytes")
    return int(ws.value)


def wg_finalise(geom: WgGeom, grid: torch.Tensor, normaliser: torch.Tensor, image: torch.Tensor, ws: torch.Tensor,
                stream=None):
    _check(lib().wg_finalise(ctypes.byref(geom), _p(grid), _p(normaliser), _p(image), _p(ws),
                             ws.numel() * ws.element_size(), _stream(stream)), "wg_finalise")


def wg_finalise_stacked(geom: WgGeom, grids: torch.Tensor, normaliser: torch.Tensor, image: torch.Tensor,
                        ws: torch.Tensor, stream=None):
    npol = max(1, geom.n_pol)
    if grids.numel() != 2 * geom.n_w * npol * geom.n * geom.n or image.numel() != npol * geom.n * geom.n \
            or normaliser.numel() < npol:
        raise ValueError("wg_finalise_stacked: grids must hold n_w x P x n x n complex values, image P x n x n, "
                         "and P normalisers")
    _check(lib().wg_finalise_stacked(ctypes.byref(geom), _p(grids), _p(normaliser), _p(image), _p(ws),
                                     ws.numel() * ws.element_size(), _stream(stream)), "wg_finalise_stacked")


def finalise(geom: WgGeom, grid: torch.Tensor, normaliser: torch.Tensor, out=None, ws=None, stream=None) -> torch.Tensor:
    """Dirty image float32 [n][n] from a complex64 [n][n] grid; with P = geom.n_pol > 1
    polarisations, the Stokes images float32 [P][n][n] from a [P][n][n] grid. `normaliser`
    holds P float64 values on the device (a view of the statistics or of the normalisers in
    the runs)."""
    n = geom.n
    npol = max(1, geom.n_pol)
    if out is None:
        out = torch.empty((n, n) if npol == 1 else (npol, n, n), dtype=torch.float32, device=grid.device)
    if grid.numel() != npol * n * n or out.numel() != npol * n * n or normaliser.numel() < npol:
        raise ValueError(f"finalise: grid {tuple(grid.shape)}, image {tuple(out.shape)} and {normaliser.numel()} "
                         f"normalisers do not fit {npol} polarisation(s) of {n} x {n}")
    if ws is None:
        ws = torch.empty(wg_finalise_ws_bytes(geom), dtype=torch.uint8, device=grid.device)
    wg_finalise(geom, torch.view_as_real(grid.contiguous()), normaliser, out, ws, stream)
    return out


# -------------------------------------------------------------------------- owning helpers
def make_geom(n, beta, n_w, s_lo, s_hi, m_img, du, w_max, compress=True, per_channel=False,
              w_stacking=False, n_pol=1, circular=False, plain_sums=False) -> WgGeom:
    flags = ((WG_COMPRESS if compress else 0) | (WG_GRID_PER_CHANNEL if per_channel else 0)
             | (WG_W_STACKING if w_stacking else 0) | (WG_POL_CIRCULAR if circular else 0)
             | (WG_PLAIN_SUMS if plain_sums else 0))
    return WgGeom(int(n), int(beta), int(n_w), int(s_lo), int(s_hi), int(m_img), float(du), float(w_max), flags,
                  int(n_pol))


def geom_from_dict(d: dict, compress=True, per_channel=False, w_stacking=False, n_pol=1, circular=False,
                   plain_sums=False) -> WgGeom:
    return make_geom(d["n"], d["beta"], d["n_w"], d["s_lo"], d["s_hi"], d["m_img"], d["du"], d["w_max"], compress,
                     per_channel, w_stacking, n_pol, circular, plain_sums)


class KernelTable:
    """Device-resident convolution-function table built by wg_ktable_build."""

    def __init__(self, geom: WgGeom, dtype: str = "f32", device="cuda", stream=None):
        dt = DTYPES[dtype]
        cap, ws_bytes = wg_ktable_sizes(geom)
        dev = torch.device(device)
        self.dtype = dtype
        self.support_d = torch.empty(geom.n_w, dtype=torch.int32, device=dev)
        self.offset_d = torch.empty(geom.n_w + 1, dtype=torch.int64, device=dev)
        self.wbound_d = torch.empty(geom.n_w, dtype=torch.float64, device=dev)
        self.zeta_d = torch.empty(geom.n_w * geom.beta * geom.beta, dtype=torch.float64, device=dev)
        self.data_d = torch.empty(cap * _ELEM_BYTES[dt], dtype=torch.uint8, device=dev)
        self.kt = WgKtable(dt, geom.n_w, geom.beta, 0, _p(self.support_d), _p(self.offset_d), _p(self.wbound_d),
                           _p(self.zeta_d), _p(self.data_d), cap)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
        self.support, self.offset = wg_ktable_build(geom, self.kt, ws, stream)
        del ws

    def data_complex(self) -> torch.Tensor:
        """The table samples as complex64 (upcast from bf16/f16), shape [offset[-1]], in the
        library's layout: per plane beta^2 matrices of S rows of S + 2P samples (P = 1 for
        FP32, 3 for 16-bit tables), matrix column j at row position P + j, positions 0..P-1
        repeating columns S-P..S-1 and positions P+S..P+S+P-1 columns 0..P-1."""
        n = self.offset[-1]
        if self.dtype == "f32":
            return torch.view_as_complex(self.data_d[: 8 * n].view(torch.float32).view(n, 2))
        h = self.data_d[: 4 * n].view(torch.bfloat16 if self.dtype == "bf16" else torch.float16).view(n, 2)
        return torch.view_as_complex(h.float().contiguous())


@dataclass
class Stats:
    n_records: int
    n_griddable: int
    n_runs: int
    n_compressed: int
    upd_real: int
    upd_saved: int
    normaliser: float
    n_items: int


class Runs:
    """Run list + plan + normalisers of one record batch, all views of one device workspace
    laid out by wg_grid_records_ws (the workspace wg_grid_records fills), plus the device
    statistics."""

    def __init__(self, geom: WgGeom, nb: int, nc: int, nt: int, device="cuda"):
        dev = torch.device(device)
        self.n_pol = max(1, geom.n_pol)
        self.ws = torch.empty(wg_grid_records_ws(geom, nb, nc, nt), dtype=torch.uint8, device=dev)
        self.c = wg_grid_records_ws(geom, nb, nc, nt, self.ws)
        self.capacity = int(self.c.capacity)
        self.stats_d = torch.zeros(8, dtype=torch.int64, device=dev)
        base = self.ws.data_ptr()
        cap = self.capacity

        def view(ptr, n, dt):
            if ptr is None:
                return None
            off = int(ptr) - base
            nbytes = n * torch.empty((), dtype=dt).element_size()
            return self.ws[off:off + nbytes].view(dt)

        self.start = view(self.c.start, cap, torch.int32)
        self.len = view(self.c.len, cap, torch.int32)
        self.x = view(self.c.x, cap, torch.int32)
        self.y = view(self.c.y, cap, torch.int32)
        self.plane = view(self.c.plane, cap, torch.int16)
        self.ou = view(self.c.ou, cap, torch.int8)
        self.ov = view(self.c.ov, cap, torch.int8)
        self.gamma = view(self.c.gamma, 2 * cap * self.n_pol, torch.float32)
        self.work = view(self.c.work, 2 * cap * self.n_pol, torch.float32)
        self.plan = view(self.c.plan, int(self.c.plan_elems), torch.int32)
        # per-channel grids and w-stacking: the grid of each run; per-channel grids or several
        # polarisations: the normalisers [grid][polarisation]
        per_channel = bool(geom.flags & WG_GRID_PER_CHANNEL)
        self.grid = view(self.c.grid, cap, torch.int16) if per_channel or geom.flags & WG_W_STACKING else None
        n_norms = nc * self.n_pol if per_channel else self.n_pol if self.n_pol > 1 else 0
        self.norm = view(self.c.norm, n_norms, torch.float64) if n_norms else None

    def normaliser(self, g: int | None = None) -> torch.Tensor:
        """float64 device view of the normaliser(s): P values (of grid g with per-channel
        grids; the one in the statistics when P = 1 and the grid is shared)."""
        if self.norm is None:
            return self.stats_d.view(torch.float64)[6:7]
        g = 0 if g is None else g
        return self.norm[g * self.n_pol:(g + 1) * self.n_pol]

    def _gamma_host(self, n):
        g = torch.view_as_complex(self.gamma[: 2 * n * self.n_pol].view(n * self.n_pol, 2)).cpu().numpy()
        return g if self.n_pol == 1 else g.reshape(n, self.n_pol)

    def stats(self) -> Stats:
        h = self.stats_d.cpu()
        return Stats(*[int(v) for v in h[:6]], float(h[6:7].view(torch.float64)[0]), int(h[7]))

    def host(self) -> dict:
        """Run arrays on the host (first n_runs entries)."""
        n = self.stats().n_runs
        return dict(start=self.start[:n].cpu().numpy(), len=self.len[:n].cpu().numpy(),
                    x=self.x[:n].cpu().numpy(), y=self.y[:n].cpu().numpy(),
                    plane=self.plane[:n].cpu().numpy(), ou=self.ou[:n].cpu().numpy(),
                    ov=self.ov[:n].cpu().numpy(),
                    gamma=self._gamma_host(n), n_runs=n,
                    grid=None if self.grid is None else self.grid[:n].cpu().numpy(),
                    norm=None if self.norm is None else self.norm.cpu().numpy())


def _f32_view(vis: torch.Tensor) -> torch.Tensor:
    return torch.view_as_real(vis) if vis.is_complex() else vis


class Gridder:
    """compress -> grid -> degrid over one record batch with a fixed table."""

    def __init__(self, geom: WgGeom, table: KernelTable, uvw, inv_lambda, weight=None, flag=None):
        self.geom, self.table = geom, table
        self.uvw, self.inv_lambda = uvw.contiguous(), inv_lambda.contiguous()
        self.weight = None if weight is None else weight.contiguous()
        self.flag = None if flag is None else flag.contiguous()
        self.nb, self.nt = int(uvw.shape[0]), int(uvw.shape[1])
        self.nc = int(inv_lambda.shape[0])
        self.n_rec = self.nb * self.nc * self.nt
        self.per_channel = bool(geom.flags & WG_GRID_PER_CHANNEL)
        self.w_stacking = bool(geom.flags & WG_W_STACKING)
        self.n_grids = self.nc if self.per_channel else geom.n_w if self.w_stacking else 1
        self.n_pol = max(1, geom.n_pol)
        for name, arr in (("weight", self.weight), ("flag", self.flag)):
            if arr is not None and arr.numel() != self.n_rec * self.n_pol:
                raise ValueError(f"{name} has {arr.numel()} values, expected {self.n_rec} records x {self.n_pol}")
        self.runs = Runs(geom, self.nb, self.nc, self.nt, device=uvw.device)

    def grid_shape(self):
        n = self.geom.n
        if self.n_pol == 1:
            return (self.n_grids, n, n) if (self.per_channel or self.w_stacking) else (n, n)
        return (self.n_grids, self.n_pol, n, n) if (self.per_channel or self.w_stacking) else (self.n_pol, n, n)

    def vis_shape(self):
        shape = (self.nb, self.nc, self.nt)
        return shape if self.n_pol == 1 else shape + (self.n_pol,)

    def compress(self, vis, stream=None):
        if vis.numel() != self.n_rec * self.n_pol * (1 if vis.is_complex() else 2):
            raise ValueError(f"vis has shape {tuple(vis.shape)}, expected {self.vis_shape()} complex values")
        wg_compress(self.geom, self.table.kt, self.uvw, self.inv_lambda, _f32_view(vis.contiguous()), self.weight,
                    self.flag, self.nb, self.nc, self.nt, self.runs.c, self.runs.stats_d, stream)

    def grid_records(self, vis, out=None, stream=None):
        """compress + grid in one call (wg_grid_records): the batch's runs are left in the
        workspace for degrid. Accumulates into `out` (zeros when not given)."""
        if vis.numel() != self.n_rec * self.n_pol * (1 if vis.is_complex() else 2):
            raise ValueError(f"vis has shape {tuple(vis.shape)}, expected {self.vis_shape()} complex values")
        if out is None:
            out = torch.zeros(self.grid_shape(), dtype=torch.complex64, device=self.uvw.device)
        elif tuple(out.shape) != self.grid_shape():
            raise ValueError(f"grid shape {tuple(out.shape)} != {self.grid_shape()}")
        wg_grid_records(self.geom, self.table.kt, self.uvw, self.inv_lambda, _f32_view(vis.contiguous()), self.weight,
                        self.flag, self.nb, self.nc, self.nt, torch.view_as_real(out), self.runs.stats_d, self.runs.ws,
                        stream)
        return out

    def grid(self, out=None, stream=None):
        """Accumulate the batch into a complex64 grid ([n][n], or [nc][n][n] per channel, or
        [n_w][n][n] with w-stacking; [P][n][n] or [nc][P][n][n] with P polarisations)."""
        if out is None:
            out = torch.zeros(self.grid_shape(), dtype=torch.complex64, device=self.uvw.device)
        elif tuple(out.shape) != self.grid_shape():
            raise ValueError(f"grid shape {tuple(out.shape)} != {self.grid_shape()}")
        wg_grid(self.geom, self.table.kt, self.runs.c, self.runs.stats_d, torch.view_as_real(out), stream)
        return out

    def degrid(self, grid, out=None, stream=None):
        if tuple(grid.shape) != self.grid_shape():
            raise ValueError(f"grid shape {tuple(grid.shape)} != {self.grid_shape()}")
        if out is None:
            out = torch.empty(self.vis_shape(), dtype=torch.complex64, device=self.uvw.device)
        elif tuple(out.shape) != self.vis_shape():
            raise ValueError(f"out shape {tuple(out.shape)} != {self.vis_shape()}")
        wg_degrid(self.geom, self.table.kt, self.runs.c, self.runs.stats_d, torch.view_as_real(grid.contiguous()),
                  self.uvw, self.weight, self.flag, self.nb, self.nc, self.nt, torch.view_as_real(out), stream)
        return out

    def finalise(self, grid, out=None, stream=None):
        """Dirty image(s) of `grid` with this batch's normaliser(s) (wg_finalise): float32
        [n][n], or [nc][n][n] for per-channel grids (each with its channel's normaliser); one
        [n][n] image of the w-plane grids with w-stacking (wg_finalise_stacked). With P > 1
        polarisations each image becomes P Stokes images ([P][n][n], [nc][P][n][n])."""
        if self.w_stacking:
            n = self.geom.n
            if out is None:
                out = torch.empty((n, n) if self.n_pol == 1 else (self.n_pol, n, n), dtype=torch.float32,
                                  device=grid.device)
            ws = torch.empty(wg_finalise_ws_bytes(self.geom), dtype=torch.uint8, device=grid.device)
            wg_finalise_stacked(self.geom, torch.view_as_real(grid.contiguous()), self.runs.normaliser(), out, ws,
                                stream)
            return out
        if not self.per_channel:
            return finalise(self.geom, grid, self.runs.normaliser(), out=out, stream=stream)
        n = self.geom.n
        if out is None:
            shape = (self.nc, n, n) if self.n_pol == 1 else (self.nc, self.n_pol, n, n)
            out = torch.empty(shape, dtype=torch.float32, device=grid.device)
        ws = torch.empty(wg_finalise_ws_bytes(self.geom), dtype=torch.uint8, device=grid.device)
        for c in range(self.nc):
            finalise(self.geom, grid[c], self.runs.normaliser(c), out=out[c], ws=ws, stream=stream)
        return out


class GridFn(torch.autograd.Function):
    """grid = G(vis) with compression (forward: wg_grid_records); backward returns G^H(grad_grid) via wg_degrid, the
    adjoint for the real inner product Re<a, b> (PyTorch's complex-gradient convention)."""

    @staticmethod
    def forward(ctx, vis, gridder: Gridder):
        out = gridder.grid_records(vis)
        ctx.gridder = gridder
        return out

    @staticmethod
    def backward(ctx, grad_grid):
        return ctx.gridder.degrid(grad_grid), None
