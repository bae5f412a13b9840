"""HIP path vs the FP64 oracle, through the C ABI (needs an MI355X).

Bars (stated per result): run boundaries, keys and counters bit-exact; table supports
bit-exact and samples equal to the oracle's FP64 table rounded to the storage type (to one
unit in the last place where the two FP64 computations straddle a rounding boundary); grids
and degridded visibilities within relative L2 1e-5 with FP32 tables and 3e-3 with BF16
tables against the FP64 oracle on its FP64 table. Every such bound holds twice: for the
relative L2 norm of the difference and for the largest element difference over the
reference's largest magnitude (`Err`).
"""
import math
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
from oracle import ktable as okt  # noqa: E402
from paper_1403_4209_amd import wgrid as wg  # noqa: E402

DEV = torch.device("cuda:0")
_TABLES = {}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def otable(geom, dtype):
    key = tuple(sorted(geom.items()))
    if key not in _TABLES:
        _TABLES[key] = {"f64": okt.build(geom, "f64")}
    if dtype not in _TABLES[key]:
        _TABLES[key][dtype] = okt.requantize(_TABLES[key]["f64"], dtype)
    return _TABLES[key][dtype]


class Err(float):
    """An error against a reference, as two figures: the relative L2 norm of the difference
    and the largest element difference over the reference's largest magnitude. Its value is
    the larger of the two, so one bound (`err < tol`) holds both the norm and every element;
    formatting prints both."""

    def __new__(cls, l2, mx):
        e = super().__new__(cls, max(l2, mx))
        e.l2, e.maxabs = float(l2), float(mx)
        return e

    def __format__(self, spec):
        return f"L2 {format(self.l2, spec)} max-abs {format(self.maxabs, spec)}"


def unpad_table(tb, beta):
    """The library's table in the oracle's layout: its matrices have rows of S + 2P values
    (P = 1 with FP32 tables, 3 with 16-bit ones), matrix column j at position P + j,
    positions 0..P-1 repeating columns S-P..S-1 and positions P+S..P+S+P-1 columns 0..P-1
    (so that P + 1 neighbouring columns are one load, forwards or backwards, also where they
    wrap). Checks that layout (offsets from the supports, every repeated value equal bit for
    bit) and returns the S x S matrices back to back, with their offsets."""
    P = 1 if tb.dtype == "f32" else 3
    data = tb.data_complex().cpu().numpy().astype(np.complex128)
    sup = [int(v) for v in tb.support]
    off_pad, off = [0], [0]
    for S in sup:
        off_pad.append(off_pad[-1] + beta * beta * S * (S + 2 * P))
        off.append(off[-1] + beta * beta * S * S)
    assert list(tb.offset) == off_pad
    planes = []
    for k, S in enumerate(sup):
        m = data[off_pad[k]:off_pad[k + 1]].reshape(beta * beta, S, S + 2 * P)
        core = m[:, :, P:P + S]
        for x in range(P):
            assert np.array_equal(m[:, :, x], core[:, :, (x - P) % S])
            assert np.array_equal(m[:, :, P + S + x], core[:, :, x % S])
        planes.append(core.reshape(-1))
    return np.concatenate(planes), off


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    d = np.abs(a - b)
    scale = max(float(np.max(np.abs(b))) if b.size else 0.0, 1e-300)
    return Err(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300), float(np.max(d)) / scale if d.size else 0.0)


def to_dev(w):
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(DEV, dt)  # noqa: E731
    return (t(w["uvw"], torch.float64), t(w["il"], torch.float64), t(w["vis"], torch.complex64),
            None if w.get("wt") is None else t(w["wt"], torch.float32),
            None if w.get("flag") is None else t(w["flag"], torch.uint8))


def run_gpu(geom, data, dtype="f32", compress=True, table=None):
    g = wg.geom_from_dict(geom, compress)
    if table is None:
        table = wg.KernelTable(g, dtype, device=DEV)
    uvw, il, vis, wt, fl = to_dev(data)
    gr = wg.Gridder(g, table, uvw, il, wt, fl)
    gr.compress(vis)
    G = gr.grid()
    torch.cuda.synchronize()
    return table, gr, G


def wl_dict(w):
    return dict(uvw=w.uvw, il=w.inv_lambda, vis=w.vis, wt=w.weight, flag=w.flag)


def cfg1():
    w = workloads.make(1)
    return w.geom, wl_dict(w)


def cfg4_small():
    # config-4 array and kernels (64 planes, supports 9..63), fewer baselines and channels
    w = workloads.make(4, n_st=12, n_t=100, n_ch=3)
    return w.geom, wl_dict(w)


def compare_runs(gr, orc):
    h = gr.runs.host()
    st = gr.runs.stats()
    assert h["n_runs"] == orc["n_runs"]
    for k in ("start", "len", "x", "y", "plane", "ou", "ov"):
        assert np.array_equal(h[k].astype(np.int64), orc[k].astype(np.int64)), k
    assert [st.n_records, st.n_griddable, st.n_runs, st.n_compressed, st.upd_real, st.upd_saved] == \
        [int(v) for v in orc["stats"]]
    if orc["n_runs"]:
        assert rel_l2(h["gamma"], orc["gamma"]) < 1e-6
        on = np.atleast_1d(orc["normaliser"])
        assert abs(st.normaliser - on[0]) <= 1e-6 * abs(on[0])
        if on.size > 1 and h["norm"] is not None and h["norm"].size == on.size:
            assert np.max(np.abs(h["norm"] - on)) <= 1e-6 * np.max(np.abs(on))
    return h, st


# ------------------------------------------------------------------------------ table
@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16"])
@pytest.mark.parametrize("case", ["cfg1", "cfg4"])
def test_table_parity(case, dtype):
    geom = cfg1()[0] if case == "cfg1" else cfg4_small()[0]
    say("table", case, dtype, geom)
    g = wg.geom_from_dict(geom)
    tb = wg.KernelTable(g, dtype, device=DEV)
    ref = otable(geom, dtype)
    ref64 = otable(geom, "f64")
    assert list(tb.support) == [int(s) for s in ref["support"]]
    got, off = unpad_table(tb, geom["beta"])
    assert off == [int(o) for o in ref["offset"]]
    exp = ref["data"]
    ulp = {"f32": 2.0 ** -23, "bf16": 2.0 ** -7, "f16": 2.0 ** -10}[dtype]
    sub = 2.0 ** -24 if dtype == "f16" else 0.0       # f16 subnormal spacing
    for part in (np.real, np.imag):
        d = np.abs(part(got) - part(exp))
        # FP64 round-off of the two FFTs is ~1e-16 of the peak (1.0): samples at that level
        # (e.g. the imaginary part of the w=0 plane) may round differently
        assert np.all(d <= ulp * np.abs(part(exp)) + 1e-13 + sub)
        # a straddle needs |FP64 difference| (~1e-16) to reach half a unit of the value,
        # so samples above 1e-4 of the peak should round identically almost always
        big = np.abs(part(exp)) > 1e-4
        assert np.mean(d[big] > 0) < 1e-3
    # against the unrounded FP64 table: within half a unit of the storage type
    e64 = np.abs(got - ref64["data"])
    assert np.all(e64 <= 0.5 * ulp * np.sqrt(2) * np.abs(ref64["data"]) + 1e-13 + sub)
    zeta = tb.zeta_d.cpu().numpy().reshape(ref["zeta"].shape)
    assert np.max(np.abs(zeta - ref["zeta"])) <= 1e-9 * np.max(np.abs(ref["zeta"]))
    wb = tb.wbound_d.cpu().numpy()
    assert np.array_equal(wb[1:], ref["wbound"][1:])


def test_table_with_200_planes():
    """The thesis's 200-plane table (its table-generation cost study) at a small image size:
    supports and offsets bit-exact, samples within one unit of the oracle's rounded FP32
    values, for every plane."""
    geom = dict(n=512, beta=8, n_w=200, s_lo=9, s_hi=31, m_img=64, du=40.0, w_max=3000.0)
    say("table 200 planes", geom)
    g = wg.geom_from_dict(geom)
    tb = wg.KernelTable(g, "f32", device=DEV)
    ref = otable(geom, "f32")
    assert list(tb.support) == [int(s) for s in ref["support"]]
    got, off = unpad_table(tb, geom["beta"])
    assert off == [int(o) for o in ref["offset"]]
    for part in (np.real, np.imag):
        d = np.abs(part(got) - part(ref["data"]))
        assert np.all(d <= 2.0 ** -23 * np.abs(part(ref["data"])) + 1e-13)


def test_table_async_build_matches_oracle():
    """The build without host copies (supports computed on the device, nothing waits) gives
    the oracle's supports and samples too."""
    geom = cfg4_small()[0]
    g = wg.geom_from_dict(geom)
    tb = wg.KernelTable(g, "f32", device=DEV)
    _, ws_bytes = wg.wg_ktable_sizes(g)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=DEV)
    tb.data_d.zero_()
    tb.support_d.zero_()
    wg.wg_ktable_build(g, tb.kt, ws, host_copies=False)
    torch.cuda.synchronize()
    assert tb.kt.s_max == geom["s_hi"]
    ref = otable(geom, "f32")
    assert np.array_equal(tb.support_d.cpu().numpy(), ref["support"])
    tb.support = [int(v) for v in tb.support_d.cpu().numpy()]
    tb.offset = [int(v) for v in tb.offset_d.cpu().numpy()]
    got, off = unpad_table(tb, geom["beta"])
    assert off == [int(o) for o in ref["offset"]]
    assert np.all(np.abs(got - ref["data"]) <= 2.0 ** -23 * np.abs(ref["data"]) + 1e-13)


# ------------------------------------------------------------------------ compression
@pytest.mark.parametrize("compress", [True, False])
@pytest.mark.parametrize("case", ["cfg1", "cfg4"])
def test_runs_bitexact(case, compress):
    geom, data = cfg1() if case == "cfg1" else cfg4_small()
    say("runs", case, compress)
    _, gr, _ = run_gpu(geom, data, compress=compress)
    orc = oracle.compress(geom, otable(geom, "f32"), data["uvw"], data["il"], data["vis"], data["wt"],
                          data["flag"], compress=compress)
    compare_runs(gr, orc)


# --------------------------------------------------------------------------- gridding
@pytest.mark.parametrize("dtype,tol", [("f32", 1e-5), ("bf16", 3e-3), ("f16", 1e-3)])
@pytest.mark.parametrize("case", ["cfg1", "cfg4"])
def test_grid_parity(case, dtype, tol):
    geom, data = cfg1() if case == "cfg1" else cfg4_small()
    say("grid", case, dtype)
    _, gr, G = run_gpu(geom, data, dtype=dtype)
    t64 = otable(geom, "f64")
    orc = oracle.compress(geom, t64, data["uvw"], data["il"], data["vis"], data["wt"], data["flag"])
    Go = oracle.grid(geom, t64, orc)
    Gg = G.cpu().numpy().astype(np.complex128)
    err = rel_l2(Gg, Go)
    # the share of the error that is table rounding: grid the oracle with the rounded table
    tq = otable(geom, dtype)
    Gq = oracle.grid(geom, tq, oracle.compress(geom, tq, data["uvw"], data["il"], data["vis"], data["wt"]))
    err_acc = rel_l2(Gg, Gq)
    say(f"  rel L2 vs FP64 oracle {err:.3e}; vs oracle with rounded table {err_acc:.3e}")
    assert err < tol
    assert err_acc < 1e-5


@pytest.mark.parametrize("case,npol,dtype", [("cfg1", 1, "f32"), ("cfg4", 1, "f32"), ("cfg4", 1, "bf16"),
                                           ("cfg4", 4, "f32"), ("cfg1", 2, "f16")])
def test_plain_sums_match_oracle(case, npol, dtype):
    """WG_PLAIN_SUMS (plain FP32 sums per owned cell, the thesis's single-precision gridder):
    the grid within the table type's bar of the FP64 oracle (1e-5 FP32, 3e-3 BF16, 1e-3 FP16),
    within 1e-5 of the oracle on the same rounded table, and within 1e-5 of the default
    Kahan-compensated grid of the same runs."""
    if npol == 1:
        geom, data = cfg1() if case == "cfg1" else cfg4_small()
    else:
        geom, data = _pol_case(case, npol, False)
    say("plain sums", case, npol, dtype)
    tol = {"f32": 1e-5, "bf16": 3e-3, "f16": 1e-3}[dtype]
    uvw, il, vis, wt, fl = to_dev(data)
    grids = {}
    for plain in (False, True):
        g = wg.geom_from_dict(geom, n_pol=npol, plain_sums=plain)
        table = wg.KernelTable(g, dtype, device=DEV)
        gr = wg.Gridder(g, table, uvw, il, wt, fl)
        gr.compress(vis)
        grids[plain] = gr.grid().cpu().numpy().astype(np.complex128)
    t64, tq = otable(geom, "f64"), otable(geom, dtype)
    Go = oracle.grid(geom, t64, oracle.compress(geom, t64, data["uvw"], data["il"], data["vis"], data["wt"], data["flag"]))
    Gq = oracle.grid(geom, tq, oracle.compress(geom, tq, data["uvw"], data["il"], data["vis"], data["wt"], data["flag"]))
    err, err_q, err_k = rel_l2(grids[True], Go), rel_l2(grids[True], Gq), rel_l2(grids[True], grids[False])
    say(f"  rel L2 vs FP64 oracle {err:.3e}; vs oracle on the rounded table {err_q:.3e}; vs Kahan {err_k:.3e}")
    assert err < tol
    assert err_q < 1e-5
    assert err_k < 1e-5


@pytest.mark.parametrize("dtype,tol", [("f32", 1e-5), ("bf16", 3e-3)])
def test_large_supports_match_oracle(dtype, tol):
    """Supports of 101 to 349 (beyond 63: the plan's per-support words, the gridder's unit
    table, class groups of more than 32 per footprint row and hundreds of waves per chunk;
    349 is the largest support of the thesis's heavy configuration): config 1's records on
    a 2048^2 grid with oversampling 4, 512 image samples and four w-planes. Runs bit-exact;
    grid and degrid against the FP64 oracle, and against the oracle on the same rounded
    table within 1e-5."""
    w = workloads.make(1, n=1024, beta=4, n_w=4, s_lo=101, s_hi=349, m_img=512)
    geom = dict(w.geom)
    geom["n"] = 2048   # the same cell size on a grid twice as wide: every footprint fits
    data = wl_dict(w)
    say("large supports", dtype)
    table, gr, G = run_gpu(geom, data, dtype=dtype)
    assert list(table.support) == [int(v) for v in otable(geom, "f64")["support"]]
    assert max(table.support) == 349
    tq = otable(geom, dtype)
    orc = oracle.compress(geom, tq, data["uvw"], data["il"], data["vis"], data["wt"], data["flag"])
    compare_runs(gr, orc)
    t64 = otable(geom, "f64")
    o64 = oracle.compress(geom, t64, data["uvw"], data["il"], data["vis"], data["wt"], data["flag"])
    Gg = G.cpu().numpy().astype(np.complex128)
    err = rel_l2(Gg, oracle.grid(geom, t64, o64))
    err_q = rel_l2(Gg, oracle.grid(geom, tq, orc))
    say(f"  grid rel L2 vs FP64 oracle {err:.3e}; vs oracle with the rounded table {err_q:.3e}")
    assert err < tol and err_q < 1e-5
    rng = np.random.default_rng(11)
    n = geom["n"]
    g = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))).astype(np.complex64)
    out = gr.degrid(torch.as_tensor(g).to(DEV)).cpu().numpy().astype(np.complex128)
    ref = oracle.degrid(geom, t64, o64, g.astype(np.complex128), data["uvw"], data["wt"], data["vis"].shape)
    errd = rel_l2(out, ref)
    say(f"  degrid rel L2 vs FP64 oracle {errd:.3e}")
    assert errd < tol


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16"])
@pytest.mark.parametrize("S", [1, 3])
def test_tiny_supports_match_oracle(S, dtype):
    """Supports 1 and 3, where a class group (a pair with FP32 tables, a quad with 16-bit
    ones) is longer than or as long as a footprint row: its samples come from the padding
    columns, partly repeated, and with quads some of its classes do not exist. Config 1's
    records; grid and degrid against the oracle on the same rounded table within 1e-5."""
    w = workloads.make(1, s_lo=S, s_hi=S)
    geom, data = w.geom, wl_dict(w)
    say("tiny support", S, dtype)
    table, gr, G = run_gpu(geom, data, dtype=dtype)
    assert list(table.support) == [S] * geom["n_w"]
    tq = otable(geom, dtype)
    orc = oracle.compress(geom, tq, data["uvw"], data["il"], data["vis"], data["wt"], data["flag"])
    compare_runs(gr, orc)
    err = rel_l2(G.cpu().numpy().astype(np.complex128), oracle.grid(geom, tq, orc))
    rng = np.random.default_rng(13)
    n = geom["n"]
    g = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))).astype(np.complex64)
    out = gr.degrid(torch.as_tensor(g).to(DEV)).cpu().numpy().astype(np.complex128)
    errd = rel_l2(out, oracle.degrid(geom, tq, orc, g.astype(np.complex128), data["uvw"], data["wt"],
                                     data["vis"].shape))
    say(f"  grid {err:.3e}, degrid {errd:.3e} against the oracle on the rounded table")
    assert err < 1e-5 and errd < 1e-5


def test_compressed_grid_matches_uncompressed_gpu():
    geom, data = cfg4_small()
    _, _, Gc = run_gpu(geom, data, compress=True)
    _, _, Gu = run_gpu(geom, data, compress=False)
    assert rel_l2(Gc.cpu().numpy(), Gu.cpu().numpy()) < 1e-5


# -------------------------------------------------------------------------- degridding
@pytest.mark.parametrize("dtype,tol", [("f32", 1e-5), ("bf16", 3e-3), ("f16", 1e-3)])
@pytest.mark.parametrize("case", ["cfg1", "cfg4"])
def test_degrid_parity(case, dtype, tol):
    geom, data = cfg1() if case == "cfg1" else cfg4_small()
    say("degrid", case, dtype)
    _, gr, _ = run_gpu(geom, data, dtype=dtype)
    rng = np.random.default_rng(4)
    n = geom["n"]
    g = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))).astype(np.complex64)
    out = gr.degrid(torch.as_tensor(g).to(DEV))
    torch.cuda.synchronize()
    t64 = otable(geom, "f64")
    orc = oracle.compress(geom, t64, data["uvw"], data["il"], data["vis"], data["wt"], data["flag"])
    ref = oracle.degrid(geom, t64, orc, g.astype(np.complex128), data["uvw"], data["wt"], data["vis"].shape)
    err = rel_l2(out.cpu().numpy().astype(np.complex128), ref)
    say(f"  degrid rel L2 {err:.3e}")
    assert err < tol


def test_adjoint_dot_product_gpu():
    geom, data = cfg4_small()
    _, gr, G = run_gpu(geom, data)
    rng = np.random.default_rng(8)
    n = geom["n"]
    g = torch.as_tensor((rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))).astype(np.complex64)).to(DEV)
    v = torch.as_tensor(data["vis"]).to(DEV)
    lhs = torch.vdot(G.flatten().to(torch.complex128), g.flatten().to(torch.complex128)).real
    ghg = gr.degrid(g)
    rhs = torch.vdot(v.flatten().to(torch.complex128), ghg.flatten().to(torch.complex128)).real
    scale = float(torch.linalg.norm(G.to(torch.complex128)) * torch.linalg.norm(g.to(torch.complex128)))
    assert abs(float(lhs - rhs)) < 1e-5 * scale


def test_autograd_finite_difference():
    """GridFn backward = degrid: central difference of L = ||IFFT(grid) - target||^2 along a
    random direction equals Re<grad, direction> (L is quadratic in vis, so the central
    difference has no truncation error; the loss is evaluated in FP64)."""
    w = workloads.make(1, n_st=6, n_t=40, n_ch=2)
    g = wg.geom_from_dict(w.geom)
    table = wg.KernelTable(g, "f32", device=DEV)
    uvw = torch.as_tensor(w.uvw).to(DEV)
    il = torch.as_tensor(w.inv_lambda).to(DEV)
    gridder = wg.Gridder(g, table, uvw, il)
    v = torch.as_tensor(w.vis).to(DEV).requires_grad_(True)
    rng = np.random.default_rng(1)

    def image(vv):
        return torch.fft.ifft2(wg.GridFn.apply(vv, gridder).to(torch.complex128))

    with torch.no_grad():
        scale = float(image(v).abs().std())
    target = torch.as_tensor(rng.standard_normal((256, 256)) * scale).to(DEV)

    def loss(vv):
        img = image(vv)
        return ((img.real - target) ** 2 + img.imag ** 2).sum()

    L = loss(v)
    L.backward()
    grad = v.grad.detach().to(torch.complex128)
    d = torch.as_tensor(rng.standard_normal(w.vis.shape) + 1j * rng.standard_normal(w.vis.shape)).to(DEV)
    d = d.to(torch.complex64)
    h = 0.5
    with torch.no_grad():
        fd = (loss(v + h * d) - loss(v - h * d)) / (2 * h)
    an = torch.sum(grad.conj() * d.to(torch.complex128)).real
    say(f"  FD {float(fd):.9e} analytic {float(an):.9e}")
    assert abs(float(fd - an)) < 1e-4 * abs(float(an))


# ------------------------------------------------------------------------- edge cases
def _records(nb, nc, nt, geom, seed, spread=0.3):
    rng = np.random.default_rng(seed)
    lim = spread * geom["n"] * geom["du"]
    uvw = np.stack([rng.uniform(-lim, lim, (nb, nt)), rng.uniform(-lim, lim, (nb, nt)),
                    rng.uniform(-geom["w_max"], geom["w_max"], (nb, nt))], -1)
    il = np.linspace(0.99, 1.01, nc)
    vis = (rng.standard_normal((nb, nc, nt)) + 1j * rng.standard_normal((nb, nc, nt))).astype(np.complex64)
    wt = rng.uniform(0.0, 2.0, (nb, nc, nt)).astype(np.float32)
    return dict(uvw=uvw, il=il, vis=vis, wt=wt, flag=np.zeros((nb, nc, nt), np.uint8))


EDGE_GEOM = dict(n=128, beta=8, n_w=6, s_lo=9, s_hi=31, m_img=128, du=20.0, w_max=400.0)


@pytest.mark.parametrize("nt", [1, 63, 64, 65, 130, 257])
def test_ragged_segments(nt):
    say("ragged nt", nt)
    data = _records(3, 2, nt, EDGE_GEOM, seed=nt)
    # slow tracks so that runs form and cross 64-record steps
    data["uvw"] = data["uvw"][:, :1, :] + np.cumsum(np.full((3, nt, 3), 0.05), axis=1) * [[[20.0, 7.0, 3.0]]]
    _, gr, G = run_gpu(EDGE_GEOM, data)
    orc = oracle.compress(EDGE_GEOM, otable(EDGE_GEOM, "f32"), data["uvw"], data["il"], data["vis"], data["wt"])
    compare_runs(gr, orc)
    Go = oracle.grid(EDGE_GEOM, otable(EDGE_GEOM, "f64"), orc)
    assert rel_l2(G.cpu().numpy(), Go) < 1e-5


def test_one_long_run_per_segment():
    nt = 300
    data = _records(2, 2, nt, EDGE_GEOM, seed=5)
    data["uvw"][:] = data["uvw"][:, :1, :]
    _, gr, G = run_gpu(EDGE_GEOM, data)
    orc = oracle.compress(EDGE_GEOM, otable(EDGE_GEOM, "f32"), data["uvw"], data["il"], data["vis"], data["wt"])
    h, st = compare_runs(gr, orc)
    assert st.n_runs == 4 and list(h["len"]) == [nt] * 4
    Go = oracle.grid(EDGE_GEOM, otable(EDGE_GEOM, "f64"), orc)
    assert rel_l2(G.cpu().numpy(), Go) < 1e-5


def test_flags_nan_offgrid_and_edges():
    nt = 90
    data = _records(4, 2, nt, EDGE_GEOM, seed=9, spread=0.55)   # some records off the grid
    data["flag"][0, 0, ::3] = 1
    data["flag"][1, :, :] = 1                                    # a fully flagged baseline
    data["uvw"][2, 5, 0] = np.nan
    data["uvw"][2, 6, 2] = np.inf
    data["uvw"][2, 7, :] = -0.0
    data["wt"][3, 1, :10] = 0.0
    _, gr, G = run_gpu(EDGE_GEOM, data)
    orc = oracle.compress(EDGE_GEOM, otable(EDGE_GEOM, "f32"), data["uvw"], data["il"], data["vis"], data["wt"],
                          data["flag"])
    h, st = compare_runs(gr, orc)
    assert st.n_griddable < st.n_records
    Go = oracle.grid(EDGE_GEOM, otable(EDGE_GEOM, "f64"), orc)
    assert rel_l2(G.cpu().numpy(), Go) < 1e-5
    out = gr.degrid(G)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    assert np.all(o[1] == 0)                       # flagged baseline -> exactly zero


def test_many_local_chunks_per_workgroup():
    """w alternating across a plane edge with different supports: every record is a run and
    every run its own local chunk (> 1024 chunks per 4-segment workgroup exercises the
    emit pass's direct-slot path)."""
    nt = 600
    data = _records(4, 1, nt, EDGE_GEOM, seed=12, spread=0.2)
    wb = okt.w_bounds(EDGE_GEOM["n_w"], EDGE_GEOM["w_max"])
    data["uvw"][:, :, 2] = np.where(np.arange(nt) % 2 == 0, 0.5 * wb[1], 1.5 * wb[1])
    _, gr, G = run_gpu(EDGE_GEOM, data)
    st = gr.runs.stats()
    orc = oracle.compress(EDGE_GEOM, otable(EDGE_GEOM, "f32"), data["uvw"], data["il"], data["vis"], data["wt"])
    compare_runs(gr, orc)
    assert st.n_items == st.n_runs == 4 * nt
    Go = oracle.grid(EDGE_GEOM, otable(EDGE_GEOM, "f64"), orc)
    assert rel_l2(G.cpu().numpy(), Go) < 1e-5
    g = torch.as_tensor(Go.astype(np.complex64)).to(DEV)
    out = gr.degrid(g)
    torch.cuda.synchronize()
    ref = oracle.degrid(EDGE_GEOM, otable(EDGE_GEOM, "f64"), orc, Go, data["uvw"], data["wt"], data["vis"].shape)
    assert rel_l2(out.cpu().numpy().astype(np.complex128), ref) < 1e-5


def test_everything_flagged():
    data = _records(2, 2, 70, EDGE_GEOM, seed=2)
    data["flag"][:] = 1
    _, gr, G = run_gpu(EDGE_GEOM, data)
    st = gr.runs.stats()
    assert st.n_runs == 0 and st.n_griddable == 0 and st.n_items == 0
    assert not torch.any(G != 0)
    out = gr.degrid(G)
    torch.cuda.synchronize()
    assert not torch.any(out != 0)


@pytest.mark.parametrize("npol", [1, 4])
def test_degrid_writes_every_record(npol):
    """The degridder writes every record once, into an output filled with NaN beforehand:
    records in no run (flagged ones before the first run, between runs, at segment ends and
    after the last run) read exactly 0, every other record matches the FP64 oracle's adjoint
    within 1e-5. Many short segments put the gaps at the edges of the finish kernel's
    64-run batches too."""
    if npol == 1:
        data = _records(9, 3, 70, EDGE_GEOM, seed=11)
    else:
        data = _pol_records(9, 3, 70, 4, EDGE_GEOM, seed=11)
    rng = np.random.default_rng(12)
    fl = data["flag"]
    fl[(rng.random(fl.shape) < 0.15)] = 1      # scattered records in no run
    fl[0, 0, :5] = 1                            # the first records
    fl[-1, -1, -5:] = 1                         # the last records
    g = wg.geom_from_dict(EDGE_GEOM, n_pol=npol)
    table = wg.KernelTable(g, "f32", device=DEV)
    uvw, il, vis, wt, flg = to_dev(data)
    gr = wg.Gridder(g, table, uvw, il, wt, flg)
    gr.compress(vis)
    st = gr.runs.stats()
    assert st.n_runs > 128          # more than two of the finish kernel's 64-run batches
    n = EDGE_GEOM["n"]
    shape = (n, n) if npol == 1 else (npol, n, n)
    grid = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)
    out = torch.full(gr.vis_shape(), float("nan"), dtype=torch.complex64, device=DEV)
    gr.degrid(torch.as_tensor(grid).to(DEV), out=out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.complex128)
    assert np.all(np.isfinite(got))
    t64 = otable(EDGE_GEOM, "f64")
    orc = oracle.compress(EDGE_GEOM, t64, data["uvw"], data["il"], data["vis"], data["wt"], data["flag"])
    ref = oracle.degrid(EDGE_GEOM, t64, orc, grid.astype(np.complex128), data["uvw"], data["wt"], data["vis"].shape,
                        flag=data["flag"] if npol > 1 else None)
    in_run = np.zeros(data["vis"].shape[:3], bool).reshape(-1)
    for s0, ln in zip(np.asarray(orc["start"]), np.asarray(orc["len"])):
        in_run[s0:s0 + ln] = True
    in_run = in_run.reshape(data["vis"].shape[:3])
    assert (~in_run).sum() > 0
    assert np.all(got[~in_run] == 0)
    err = rel_l2(got[in_run], ref[in_run])
    say(f"  degrid over {int(in_run.sum())} records in runs, rel L2 {err:.3e}; {int((~in_run).sum())} zero")
    assert err < 1e-5


def test_maximum_support_and_grid_border():
    geom = dict(n=160, beta=8, n_w=2, s_lo=63, s_hi=63, m_img=256, du=10.0, w_max=100.0)
    nt = 8
    # pixels chosen so that footprints touch the first and last rows/columns of the grid
    # a = X + n/2 - H must lie in [0, n - S]: X in [-49, 48]
    pu = np.array([-49, 48, -50, 49, 0, 3, -5, 10])   # columns 0 and n-1 touched; two just beyond
    pv = np.array([0, 1, 2, 3, -49, 48, 7, -2])       # rows 0 and n-1 touched
    uvw = np.zeros((1, nt, 3))
    uvw[0, :, 0] = pu * geom["du"]
    uvw[0, :, 1] = pv * geom["du"]
    uvw[0, :, 2] = np.linspace(5, 90, nt)       # w >= 0: no flip, pixels as listed
    data = dict(uvw=uvw, il=np.array([1.0]), vis=(np.arange(nt) + 1j).astype(np.complex64)[None, None, :],
                wt=None, flag=None)
    _, gr, G = run_gpu(geom, data)
    orc = oracle.compress(geom, otable(geom, "f32"), data["uvw"], data["il"], data["vis"])
    h, st = compare_runs(gr, orc)
    assert st.n_griddable == nt - 2
    Go = oracle.grid(geom, otable(geom, "f64"), orc)
    assert rel_l2(G.cpu().numpy(), Go) < 1e-5


# ------------------------------------------------ hand-derived ties through the library
def _golden_index_rows():
    """tests/golden/index_ties.txt: geometry and (u, v, w, inv_lambda, flag) -> expected
    (X, Y, plane, o_u, o_v, psi, griddable) rows, '*' where a value is not checked."""
    import os
    rows, geom = [], None
    with open(os.path.join(os.path.dirname(__file__), "golden", "index_ties.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("geom"):
                kv = dict(t.split("=") for t in line.split()[1:])
                geom = dict(n=int(kv["n"]), beta=int(kv["beta"]), du=float(kv["du"]), n_w=int(kv["n_w"]),
                            w_max=float(kv["w_max"]), support=[int(v) for v in kv["support"].split(",")])
                continue
            lhs, rhs = line.split("|")
            vals = lhs.split()
            inp = [float.fromhex(v) if v.startswith(("0x", "-0x")) else float(v) for v in vals[:4]] + [int(vals[4])]
            rows.append((inp, rhs.split()))
    return geom, rows


def test_golden_index_ties_through_wg_compress():
    """Every hand-derived row of tests/golden/index_ties.txt (half-sample ties, the largest
    double below -1/2, w on a plane boundary, -0.0, 2.5 against 2.5000001, off-grid
    footprints, flags, NaN) through wg_compress, one record per segment: pixel, w-plane,
    oversample offsets and griddability bit-exact; the flip (psi) read from the run's gamma,
    which is the conjugate of the visibility 1 + 2i when psi = -1. The table carries the
    fixture's supports (3, 5, 7) and the w-plane edges of the nearest plane in sqrt(w)."""
    geom, rows = _golden_index_rows()
    n_w = geom["n_w"]
    sup = torch.tensor(geom["support"], dtype=torch.int32, device=DEV)
    s_max = max(geom["support"])
    off_h = [0]
    for S in geom["support"]:
        off_h.append(off_h[-1] + geom["beta"] ** 2 * S * (S + 2))
    off = torch.tensor(off_h, dtype=torch.int64, device=DEV)
    wb = torch.as_tensor(okt.w_bounds(n_w, geom["w_max"])).to(DEV)
    zeta = torch.zeros(n_w * geom["beta"] ** 2, dtype=torch.float64, device=DEV)
    data = torch.zeros(8 * off_h[-1], dtype=torch.uint8, device=DEV)
    kt = wg.WgKtable(wg.WG_KF32, n_w, geom["beta"], s_max, wg._p(sup), wg._p(off), wg._p(wb), wg._p(zeta),
                     wg._p(data), off_h[-1])
    g = wg.make_geom(geom["n"], geom["beta"], n_w, min(geom["support"]), s_max, 16, geom["du"], geom["w_max"])
    by_il = {}
    for inp, exp in rows:
        by_il.setdefault(inp[3], []).append((inp, exp))
    checked = 0
    for il, group in by_il.items():
        nb = len(group)
        uvw = torch.tensor([[[r[0][0], r[0][1], r[0][2]]] for r in group], dtype=torch.float64, device=DEV)
        flag = torch.tensor([r[0][4] for r in group], dtype=torch.uint8, device=DEV).view(nb, 1, 1)
        vis = torch.full((nb, 1, 1), 1 + 2j, dtype=torch.complex64, device=DEV)
        ilt = torch.tensor([il], dtype=torch.float64, device=DEV)
        runs = wg.Runs(g, nb, 1, 1, device=DEV)
        wg.wg_compress(g, kt, uvw, ilt, torch.view_as_real(vis), None, flag, nb, 1, 1, runs.c, runs.stats_d)
        torch.cuda.synchronize()
        h = runs.host()
        by_start = {int(st): q for q, st in enumerate(h["start"])}
        for b, (inp, exp) in enumerate(group):
            q = by_start.get(b)
            got_ok = 0 if q is None else 1
            assert exp[6] == "*" or got_ok == int(exp[6]), (inp, exp, got_ok)
            if q is None:
                continue
            gam = complex(h["gamma"][q])
            psi = 1 if gam.imag > 0 else -1
            assert gam == (1 + 2j if psi == 1 else 1 - 2j), (inp, gam)
            got = [int(h["x"][q]), int(h["y"][q]), int(h["plane"][q]), int(h["ou"][q]), int(h["ov"][q]), psi]
            for o, e in zip(got, exp[:6]):
                assert e == "*" or o == int(e), (inp, got, exp)
            checked += 1
    say(f"  golden rows through wg_compress: {len(rows)} ({checked} griddable)")
    assert checked == sum(1 for _, exp in rows if exp[6] == "1")


# ---------------------------------------------------------------- one-call gridding
@pytest.mark.parametrize("compress", [True, False])
@pytest.mark.parametrize("case", ["cfg1", "cfg4"])
def test_grid_records_matches_oracle(case, compress):
    """wg_grid_records (compress + grid in one call, runs left in the workspace): runs,
    keys and counters bit-exact with the oracle's; the grid within 1e-5 of the FP64 oracle;
    the workspace's runs serve wg_degrid; and the grid equals wg_compress + wg_grid's."""
    geom, data = cfg1() if case == "cfg1" else cfg4_small()
    say("grid_records", case, compress)
    g = wg.geom_from_dict(geom, compress)
    table = wg.KernelTable(g, "f32", device=DEV)
    uvw, il, vis, wt, fl = to_dev(data)
    gr = wg.Gridder(g, table, uvw, il, wt, fl)
    G = gr.grid_records(vis)
    torch.cuda.synchronize()
    t64 = otable(geom, "f64")
    orc = oracle.compress(geom, otable(geom, "f32"), data["uvw"], data["il"], data["vis"], data["wt"],
                          data["flag"], compress)
    compare_runs(gr, orc)
    Go = oracle.grid(geom, t64, orc)
    err = rel_l2(G.cpu().numpy().astype(np.complex128), Go)
    V = gr.degrid(G)
    torch.cuda.synchronize()
    Vo = oracle.degrid(geom, t64, orc, G.cpu().numpy().astype(np.complex128), data["uvw"], data["wt"],
                       data["vis"].shape)
    err_d = rel_l2(V.cpu().numpy().astype(np.complex128), Vo)
    _, _, G2 = run_gpu(geom, data, compress=compress, table=table)
    err_2 = rel_l2(G.cpu().numpy().astype(np.complex128), G2.cpu().numpy().astype(np.complex128))
    say(f"  grid {err:.3e}, degrid {err_d:.3e}, vs compress + grid {err_2:.3e}")
    assert err < 1e-5 and err_d < 1e-5 and err_2 < 1e-6


# --------------------------------------------------------------------- determinism
def cfg3_small():
    # config-3 array and kernels on the 4096^2 grid (64 planes, supports 9..63; the gridder's
    # counter walk), fewer baselines, channels and timesteps
    w = workloads.make(3, n_st=12, n_t=100, n_ch=3)
    return w.geom, wl_dict(w)


@pytest.mark.parametrize("case", ["cfg4", "cfg3"])
def test_same_batch_twice_is_deterministic_where_it_must_be(case):
    """The same batch compressed, gridded and degridded twice: runs, keys, gammas and
    integer counters bit-identical (the scan has no order-dependent arithmetic); grids and degridded
    visibilities equal up to the order of FP32 atomic commits (within 1e-6 of each other,
    per element relative to the largest magnitude); the FP64 normaliser, a sum of atomically
    added parts, to 1e-12."""
    geom, data = cfg4_small() if case == "cfg4" else cfg3_small()
    table, gr1, G1 = run_gpu(geom, data)
    h1, s1 = gr1.runs.host(), gr1.runs.stats()
    V1 = gr1.degrid(G1)
    # the same runs gridded again (the work counters reset themselves after each launch)
    G1b = gr1.grid()
    V1b = gr1.degrid(G1b)
    _, gr2, G2 = run_gpu(geom, data, table=table)
    h2, s2 = gr2.runs.host(), gr2.runs.stats()
    V2 = gr2.degrid(G2)
    torch.cuda.synchronize()
    for k in ("start", "len", "x", "y", "plane", "ou", "ov"):
        assert np.array_equal(h1[k], h2[k]), k
    assert np.array_equal(h1["gamma"].view(np.float32), h2["gamma"].view(np.float32))
    assert [s1.n_records, s1.n_griddable, s1.n_runs, s1.n_compressed, s1.upd_real, s1.upd_saved, s1.n_items] == \
        [s2.n_records, s2.n_griddable, s2.n_runs, s2.n_compressed, s2.upd_real, s2.upd_saved, s2.n_items]
    # the normaliser is an FP64 sum of per-workgroup parts added atomically: order-dependent
    # in its last bits only
    assert abs(s1.normaliser - s2.normaliser) <= 1e-12 * abs(s1.normaliser)
    eg = rel_l2(G1.cpu().numpy().astype(np.complex128), G2.cpu().numpy().astype(np.complex128))
    ev = rel_l2(V1.cpu().numpy().astype(np.complex128), V2.cpu().numpy().astype(np.complex128))
    egb = rel_l2(G1b.cpu().numpy().astype(np.complex128), G1.cpu().numpy().astype(np.complex128))
    evb = rel_l2(V1b.cpu().numpy().astype(np.complex128), V1.cpu().numpy().astype(np.complex128))
    say(f"  repeat: grid {eg:.3e}, degrid {ev:.3e}; same runs again: grid {egb:.3e}, degrid {evb:.3e}")
    assert eg < 1e-6 and ev < 1e-6 and egb < 1e-6 and evb < 1e-6


# ------------------------------------------------------------ full-size (bench) config
def test_full_config2_runs_grid_and_degrid():
    """Config 2 at full size in the launch configuration the benchmark times: every run
    boundary and key bit-exact over all 7.75 M records; the whole grid against the FP64
    oracle's grid of the same runs on its FP64 table; the degridder on that grid against
    the oracle's adjoint; and the finalised image of the grid."""
    w = workloads.make(2, device=DEV)
    say("cfg2 records", w.n_records, w.geom)
    vis_h = w.vis.cpu().numpy()
    data = dict(uvw=w.uvw, il=w.inv_lambda, vis=vis_h, wt=None, flag=None)
    table, gr, G = run_gpu(w.geom, data)
    orc = oracle.compress(w.geom, otable(w.geom, "f32"), w.uvw, w.inv_lambda, vis_h)
    compare_runs(gr, orc)
    t64 = otable(w.geom, "f64")
    Go = oracle.grid(w.geom, t64, orc)
    Gh = G.cpu().numpy().astype(np.complex128)
    err = rel_l2(Gh, Go)
    say(f"  cfg2 full grid vs FP64 oracle {err:.3e}")
    assert err < 1e-5
    V = gr.degrid(G)
    torch.cuda.synchronize()
    Vo = oracle.degrid(w.geom, t64, orc, Gh, w.uvw, None, vis_h.shape)
    err_d = rel_l2(V.cpu().numpy().astype(np.complex128), Vo)
    say(f"  cfg2 full degrid vs FP64 oracle {err_d:.3e}")
    assert err_d < 1e-5
    del Go, Vo, V
    from oracle import image as oimg
    img = gr.finalise(G)
    torch.cuda.synchronize()
    ref = oimg.finalise(w.geom, Gh, gr.runs.stats().normaliser)
    err_img = _fin_err(img.cpu().numpy().astype(np.float64), ref, w.geom)
    say(f"  cfg2 image (before the taper division) {err_img:.3e}")
    assert err_img < 1e-5


def _rel_l2_dev(a, b):
    a = a.to(torch.complex128)
    b = b.to(torch.complex128)
    return Err(float(torch.linalg.norm(a - b) / torch.linalg.norm(b)),
               float(torch.max(torch.abs(a - b)) / torch.max(torch.abs(b))))


def test_full_config3_compression_and_precision():
    """Config 3 at full size (946 baselines x 64 channels x 512 timesteps = 30,998,528
    records, 4096^2, 64 planes, supports 9..63): every run boundary and key bit-exact;
    compressed and uncompressed GPU grids agree; the whole grid with FP32, BF16 and FP16
    tables against the FP64 oracle's grid of the same runs on its FP64 table."""
    w = workloads.make(3, device=DEV)
    say("cfg3 records", w.n_records, w.geom)
    vis_h = w.vis.cpu().numpy()
    data = dict(uvw=w.uvw, il=w.inv_lambda, vis=vis_h, wt=None, flag=None)
    t32, gr, G32 = run_gpu(w.geom, data)
    orc = oracle.compress(w.geom, otable(w.geom, "f32"), w.uvw, w.inv_lambda, vis_h)
    _, st = compare_runs(gr, orc)
    say(f"  cfg3 compression: records/runs {st.n_griddable / st.n_runs:.3f}, "
        f"updates total/real {(st.upd_real + st.upd_saved) / st.upd_real:.3f}")
    del gr
    _, gu, Gu = run_gpu(w.geom, data, compress=False, table=t32)
    err_u = _rel_l2_dev(Gu, G32)
    say(f"  cfg3 uncompressed vs compressed {err_u:.3e}")
    assert err_u < 1e-5
    del gu, Gu
    Go = oracle.grid(w.geom, otable(w.geom, "f64"), orc)
    del orc
    for dt, tol in (("f32", 1e-5), ("bf16", 3e-3), ("f16", 1e-3)):
        if dt == "f32":
            Gd = G32
        else:
            _, g2, Gd = run_gpu(w.geom, data, dtype=dt)
            del g2
        err = rel_l2(Gd.cpu().numpy().astype(np.complex128), Go)
        say(f"  cfg3 full grid {dt} tables vs FP64 oracle {err:.3e}")
        assert err < tol
        del Gd


@pytest.fixture(scope="module")
def cfg4_full():
    w = workloads.make(4, device=DEV)
    vis_h = w.vis.cpu().numpy()
    data = dict(uvw=w.uvw, il=w.inv_lambda, vis=vis_h, wt=None, flag=None)
    t64 = otable(w.geom, "f64")
    orc = oracle.compress(w.geom, t64, w.uvw, w.inv_lambda, vis_h)
    return w.geom, data, orc, oracle.grid(w.geom, t64, orc)


@pytest.mark.parametrize("dtype,tol", [("f32", 1e-5), ("bf16", 3e-3), ("f16", 1e-3)])
def test_full_config4_precision(cfg4_full, dtype, tol):
    """Config 4 (the 512^2 precision sub-problem: 946 x 8 x 64 records, 64 planes, supports
    9..63) at full size: runs bit-exact, grid and degrid of each table type against the FP64
    oracle on its FP64 table."""
    geom, data, orc, Go = cfg4_full
    _, gr, G = run_gpu(geom, data, dtype=dtype)
    # the normaliser sums the stored (rounded) table values: compare against the same table
    compare_runs(gr, oracle.compress(geom, otable(geom, dtype), data["uvw"], data["il"], data["vis"]))
    err = rel_l2(G.cpu().numpy().astype(np.complex128), Go)
    rng = np.random.default_rng(44)
    n = geom["n"]
    g = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))).astype(np.complex64)
    out = gr.degrid(torch.as_tensor(g).to(DEV))
    torch.cuda.synchronize()
    ref = oracle.degrid(geom, otable(geom, "f64"), orc, g.astype(np.complex128), data["uvw"], None,
                        data["vis"].shape)
    err_d = rel_l2(out.cpu().numpy().astype(np.complex128), ref)
    say(f"  cfg4 {dtype}: grid rel L2 {err:.3e}, degrid rel L2 {err_d:.3e}")
    assert err < tol and err_d < tol


def test_full_config5_adjoint_and_finite_difference():
    """Config 5 at full size (32,640 baselines x 8 channels x 256 timesteps = 66,846,720
    records, 4096^2, supports 7..31) through GridFn: runs bit-exact; the whole grid against
    the FP64 oracle's grid of the same runs on its FP64 table; the dot-product test
    <G v, g> = <v, G^H g> with a random grid g; and central differences of
    L = ||IFFT(grid)/normaliser - target||^2 (target: 100 seeded point sources) along the
    data direction and along the returned gradient (L is quadratic, so the central
    difference has no truncation error; only FP32 rounding of the grid enters)."""
    w = workloads.make(5, device=DEV)
    say("cfg5 records", w.n_records, w.geom)
    geom = wg.geom_from_dict(w.geom)
    table = wg.KernelTable(geom, "f32", device=DEV)
    uvw = torch.as_tensor(w.uvw).to(DEV)
    il = torch.as_tensor(w.inv_lambda).to(DEV)
    gridder = wg.Gridder(geom, table, uvw, il)
    v = w.vis
    with torch.no_grad():
        G = wg.GridFn.apply(v, gridder)
    torch.cuda.synchronize()
    orc = oracle.compress(w.geom, otable(w.geom, "f32"), w.uvw, w.inv_lambda, v.cpu().numpy())
    _, st = compare_runs(gridder, orc)
    Go = oracle.grid(w.geom, otable(w.geom, "f64"), orc)
    err = rel_l2(G.cpu().numpy().astype(np.complex128), Go)
    say(f"  cfg5 full grid vs FP64 oracle {err:.3e}")
    assert err < 1e-5
    del orc, Go
    n = w.geom["n"]
    gen = torch.Generator(device=DEV)
    gen.manual_seed(55)
    g = torch.complex(torch.randn((n, n), generator=gen, device=DEV), torch.randn((n, n), generator=gen, device=DEV))
    lhs = torch.vdot(G.flatten().to(torch.complex128), g.flatten().to(torch.complex128)).real
    ghg = gridder.degrid(g)
    rhs = torch.vdot(v.flatten().to(torch.complex128), ghg.flatten().to(torch.complex128)).real
    scale = float(torch.linalg.norm(G.to(torch.complex128)) * torch.linalg.norm(g.to(torch.complex128)))
    say(f"  cfg5 dot-product test: |lhs - rhs| / (|Gv| |g|) = {abs(float(lhs - rhs)) / scale:.3e}")
    assert abs(float(lhs - rhs)) < 1e-5 * scale
    del g, ghg

    norm = n * n / st.normaliser
    target = torch.as_tensor(workloads.target_image(w)).to(DEV)

    def loss(vv):
        grid = wg.GridFn.apply(vv, gridder).to(torch.complex128)
        img = torch.fft.fftshift(torch.fft.ifft2(torch.fft.ifftshift(grid))) * norm
        return ((img.real - target) ** 2 + img.imag ** 2).sum()

    vr = v.clone().requires_grad_(True)
    L = loss(vr)
    L.backward()
    grad = vr.grad.detach()
    for name, d in (("data", v), ("gradient", grad / torch.linalg.norm(grad) * torch.linalg.norm(v))):
        h = 0.25
        with torch.no_grad():
            fd = (loss(v + h * d) - loss(v - h * d)) / (2 * h)
        an = torch.sum(grad.to(torch.complex128).conj() * d.to(torch.complex128)).real
        say(f"  cfg5 FD along {name}: {float(fd):.9e} analytic {float(an):.9e} (L {float(L):.6e})")
        assert abs(float(fd - an)) < 1e-4 * abs(float(an))


# ----------------------------------------------------------------- image finaliser
def _fin_err(got, ref, geom):
    """Relative L2 of two finalised images before the taper and sinc division, i.e. of what
    the FP32 transforms determine. The division itself is an elementwise FP64 step on both
    sides; its factor reaches 1/c(l)^2 ~ 2e5 at the image corners, where it would magnify
    the transforms' 1e-7 rounding of a grid with a concentrated spectrum far beyond its
    share of the image."""
    from oracle import image as oimg
    c = oimg.axis_correction(geom)
    w = np.outer(c, c)
    return rel_l2(got * w, ref * w)


def _device_stats(normaliser):
    return torch.tensor([normaliser], dtype=torch.float64, device=DEV)


@pytest.mark.parametrize("n", [16, 32, 64, 128, 512, 4096])
def test_finaliser_matches_oracle_on_random_grids(n):
    """wg_finalise against the oracle's finaliser on a random complex grid (every pass
    structure of the row transforms: one radix-16 pass; a radix-2/4/8 pass before radix-16
    passes; two and three radix-16 passes). FP32 FFTs: relative L2 within 1e-5, both over the
    finished image and before the taper division."""
    from oracle import image as oimg
    say("finalise n", n)
    rng = np.random.default_rng(n)
    g = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))).astype(np.complex64)
    geom = dict(n=n, beta=8, n_w=2, s_lo=7, s_hi=7, m_img=16, du=3.0, w_max=10.0)
    img = wg.finalise(wg.geom_from_dict(geom), torch.as_tensor(g).to(DEV), _device_stats(1234.5))
    torch.cuda.synchronize()
    ref = oimg.finalise(geom, g.astype(np.complex128), 1234.5)
    got = img.cpu().numpy().astype(np.float64)
    err, err_w = rel_l2(got, ref), _fin_err(got, ref, geom)
    say(f"  finalise rel L2 {err:.3e}, before the taper division {err_w:.3e}")
    assert err < 1e-5 and err_w < 1e-5
    assert not np.any(got[0, :]) and not np.any(got[:, 0])


def test_finaliser_zero_normaliser_gives_zero_image():
    n = 64
    g = torch.ones((n, n), dtype=torch.complex64, device=DEV)
    geom = dict(n=n, beta=8, n_w=2, s_lo=7, s_hi=7, m_img=16, du=3.0, w_max=10.0)
    img = wg.finalise(wg.geom_from_dict(geom), g, _device_stats(0.0))
    torch.cuda.synchronize()
    assert not torch.any(img != 0)


def test_finaliser_recovers_point_source_end_to_end():
    """compress + grid + finalise on the GPU: a 2.5 Jy source at 0.3 of the field of view seen
    by 40000 records at random sub-cell positions is recovered at its pixel to 5e-4 (the
    same bound as the oracle's own pin), and the GPU image equals the oracle's finaliser of
    the GPU grid to 1e-5 before the taper division."""
    from oracle import image as oimg
    N = 128
    geom = dict(n=N, beta=8, n_w=4, s_lo=31, s_hi=31, m_img=N, du=10.0, w_max=12.0)
    rng = np.random.default_rng(5)
    R = 40000
    lim = 0.3 * N * geom["du"]
    u, v, w = rng.uniform(-lim, lim, R), rng.uniform(-lim, lim, R), rng.uniform(-12.0, 12.0, R)
    p0, q0 = N // 2 + int(0.3 * N), N // 2 - int(0.18 * N)
    l0, m0 = (p0 - N // 2) / (N * geom["du"]), (q0 - N // 2) / (N * geom["du"])
    n0 = math.sqrt(1.0 - l0 * l0 - m0 * m0)
    vis = (2.5 * np.exp(-2j * math.pi * (u * l0 + v * m0 + w * (n0 - 1.0)))).astype(np.complex64)[None, None, :]
    data = dict(uvw=np.stack([u, v, w], -1)[None], il=np.array([1.0]), vis=vis, wt=None, flag=None)
    _, gr, G = run_gpu(geom, data)
    img = gr.finalise(G)
    torch.cuda.synchronize()
    D = img.cpu().numpy().astype(np.float64)
    say(f"  source pixel {D[q0, p0]:.6f} (2.5 Jy)")
    assert abs(D[q0, p0] / 2.5 - 1.0) < 5e-4
    ref = oimg.finalise(geom, G.cpu().numpy().astype(np.complex128), gr.runs.stats().normaliser)
    err = _fin_err(D, ref, geom)
    say(f"  image rel L2 (before the taper division) {err:.3e}")
    assert err < 1e-5


# ------------------------------------------------------------------ per-channel grids
@pytest.mark.parametrize("case", ["cfg1", "cfg4"])
def test_per_channel_grids(case):
    """WG_GRID_PER_CHANNEL: the same runs as one shared grid (bit-exact) with the run's channel
    as its grid; every channel grid, normaliser, degridded channel and finalised channel image
    against the oracle's per-channel imaging (each channel on its own); the channel grids add
    up to the shared grid."""
    from oracle import image as oimg
    geom, data = cfg1() if case == "cfg1" else cfg4_small()
    nb, nc, nt = data["vis"].shape
    say("per-channel", case, nc, "channels")
    g = wg.geom_from_dict(geom, per_channel=True)
    table = wg.KernelTable(g, "f32", device=DEV)
    uvw, il, vis, wt, fl = to_dev(data)
    gr = wg.Gridder(g, table, uvw, il, wt, fl)
    gr.compress(vis)
    G = gr.grid()
    torch.cuda.synchronize()
    assert tuple(G.shape) == (nc, geom["n"], geom["n"])
    orc = oracle.compress(geom, otable(geom, "f32"), data["uvw"], data["il"], data["vis"], data["wt"], data["flag"])
    h, _ = compare_runs(gr, orc)
    assert np.array_equal(h["grid"].astype(np.int64), (h["start"].astype(np.int64) // nt) % nc)
    t64 = otable(geom, "f64")
    oruns, Go, onorm = oracle.per_channel(geom, t64, data["uvw"], data["il"], data["vis"], data["wt"], data["flag"])
    _, _, onorm32 = oracle.per_channel(geom, otable(geom, "f32"), data["uvw"], data["il"], data["vis"], data["wt"],
                                       data["flag"])
    assert np.max(np.abs(h["norm"] - onorm32)) <= 1e-6 * np.max(np.abs(onorm32))
    Gh = G.cpu().numpy().astype(np.complex128)
    for c in range(nc):
        err = rel_l2(Gh[c], Go[c])
        say(f"  channel {c}: grid rel L2 {err:.3e}")
        assert err < 1e-5
    _, single, G1 = run_gpu(geom, data)
    assert rel_l2(Gh.sum(0), G1.cpu().numpy().astype(np.complex128)) < 1e-6
    rng = np.random.default_rng(77)
    gr_in = (rng.standard_normal(Gh.shape) + 1j * rng.standard_normal(Gh.shape)).astype(np.complex64)
    out = gr.degrid(torch.as_tensor(gr_in).to(DEV)).cpu().numpy().astype(np.complex128)
    for c in range(nc):
        ref = oracle.degrid(geom, t64, oruns[c], gr_in[c].astype(np.complex128), data["uvw"], data["wt"][:, c:c + 1, :],
                            (nb, 1, nt))
        assert rel_l2(out[:, c:c + 1, :], ref) < 1e-5
    if geom["n"] & (geom["n"] - 1) == 0:
        imgs = gr.finalise(G).cpu().numpy().astype(np.float64)
        for c in range(nc):
            ref = oimg.finalise(geom, Gh[c], float(h["norm"][c]))
            assert _fin_err(imgs[c], ref, geom) < 1e-5


# ------------------------------------------------------------------------ w-stacking
@pytest.mark.parametrize("case", ["cfg1", "cfg4"])
def test_w_stacking(case):
    """WG_W_STACKING against the oracle's w-stacking (eq. stacking): runs bit-exact (with
    plane 0 as kernel and the record's w-plane as grid id) and the statistics; every w-plane
    grid within relative L2 1e-5; the adjoint within 1e-5; the stacked image
    (wg_finalise_stacked) within 1e-5 before the taper division."""
    from oracle import image as oimg
    geom, data = cfg1() if case == "cfg1" else cfg4_small()
    nb, nc, nt = data["vis"].shape
    n_w = geom["n_w"]
    say("w-stacking", case, n_w, "planes")
    g = wg.geom_from_dict(geom, w_stacking=True)
    table = wg.KernelTable(g, "f32", device=DEV)
    uvw, il, vis, wt, fl = to_dev(data)
    gr = wg.Gridder(g, table, uvw, il, wt, fl)
    gr.compress(vis)
    G = gr.grid()
    torch.cuda.synchronize()
    assert tuple(G.shape) == (n_w, geom["n"], geom["n"])
    h = gr.runs.host()
    st = gr.runs.stats()
    oruns32, _, onorm32 = oracle.w_stacking(geom, otable(geom, "f32"), data["uvw"], data["il"], data["vis"],
                                            data["wt"], data["flag"])
    # the oracle's runs per plane, merged in record order, against the GPU's
    cat = {k: np.concatenate([r[k].astype(np.int64) for r in oruns32]) for k in ("start", "len", "x", "y", "ou", "ov")}
    cat["grid"] = np.concatenate([np.full(r["n_runs"], j, np.int64) for j, r in enumerate(oruns32)])
    gam = np.concatenate([r["gamma"] for r in oruns32])
    order = np.argsort(cat["start"], kind="stable")
    assert h["n_runs"] == len(order)
    for k in ("start", "len", "x", "y", "ou", "ov", "grid"):
        assert np.array_equal(h[k].astype(np.int64), cat[k][order]), k
    assert not np.any(h["plane"])
    assert rel_l2(h["gamma"], gam[order]) < 1e-6
    ost = np.sum([r["stats"] for r in oruns32], axis=0)
    assert [st.n_griddable, st.n_runs, st.n_compressed, st.upd_real, st.upd_saved] == [int(v) for v in ost[1:]]
    assert abs(st.normaliser - onorm32) <= 1e-6 * abs(onorm32)
    t64 = otable(geom, "f64")
    oruns, Go, _ = oracle.w_stacking(geom, t64, data["uvw"], data["il"], data["vis"], data["wt"], data["flag"])
    Gh = G.cpu().numpy().astype(np.complex128)
    for k in range(n_w):
        if not np.any(Go[k]):
            assert not np.any(Gh[k])
            continue
        err = rel_l2(Gh[k], Go[k])
        say(f"  plane {k}: grid rel L2 {err:.3e}")
        assert err < 1e-5
    rng = np.random.default_rng(78)
    gr_in = (rng.standard_normal(Gh.shape) + 1j * rng.standard_normal(Gh.shape)).astype(np.complex64)
    out = gr.degrid(torch.as_tensor(gr_in).to(DEV)).cpu().numpy().astype(np.complex128)
    ref = oracle.w_stacking_degrid(geom, t64, oruns, gr_in.astype(np.complex128), data["uvw"], data["wt"],
                                   (nb, nc, nt))
    assert rel_l2(out, ref) < 1e-5
    img = gr.finalise(G).cpu().numpy().astype(np.float64)
    ref = oimg.finalise_stacked(geom, Gh, st.normaliser)
    err = _fin_err(img, ref, geom)
    say(f"  stacked image rel L2 (before the taper division) {err:.3e}")
    assert err < 1e-5



# --------------------------------------------------------------------- polarisations
def _pol_case(case, npol, circular):
    if case == "cfg1":
        w = workloads.polarised(1, npol, circular)
    else:
        w = workloads.polarised(4, npol, circular, n_st=12, n_t=100, n_ch=3)
    return w.geom, wl_dict(w)


@pytest.mark.parametrize("case,npol,circular,per_channel,dtype", [
    ("cfg1", 4, False, False, "f32"), ("cfg1", 2, True, False, "f32"), ("cfg4", 4, False, False, "f32"),
    ("cfg4", 4, True, True, "f32"), ("cfg4", 4, False, False, "bf16"),
    # 16-bit tables with two products take class quads, with four products class pairs
    ("cfg4", 2, True, False, "f16"), ("cfg1", 4, False, False, "f16")])
def test_polarised_records(case, npol, circular, per_channel, dtype):
    """Records of 2 or 4 polarisation products with per-product weights and flags: runs
    bit-exact (a record is griddable with one unflagged product), gamma per product and the
    per-product normalisers against the oracle; the [P][n][n] grid within relative L2 1e-5;
    the adjoint (flagged products get 0) within 1e-5; every Stokes image within 1e-5 before
    the taper division. Per-channel grids: the same per channel. BF16 tables: grid and degrid
    within 3e-3 of the FP64 oracle and within 1e-5 of the oracle on the same rounded table."""
    from oracle import image as oimg
    geom, data = _pol_case(case, npol, circular)
    nb, nc, nt, _ = data["vis"].shape
    say("polarised", case, npol, "circular" if circular else "linear", "per-channel" if per_channel else "", dtype)
    g = wg.geom_from_dict(geom, per_channel=per_channel, n_pol=npol, circular=circular)
    table = wg.KernelTable(g, dtype, device=DEV)
    tol = 1e-5 if dtype == "f32" else 3e-3
    uvw, il, vis, wt, fl = to_dev(data)
    gr = wg.Gridder(g, table, uvw, il, wt, fl)
    gr.compress(vis)
    G = gr.grid()
    torch.cuda.synchronize()
    h = gr.runs.host()
    t64 = otable(geom, "f64")
    if not per_channel:
        tq = otable(geom, dtype)
        orc = oracle.compress(geom, tq, data["uvw"], data["il"], data["vis"], data["wt"], data["flag"])
        compare_runs(gr, orc)
        assert tuple(G.shape) == (npol, geom["n"], geom["n"])
        o64 = oracle.compress(geom, t64, data["uvw"], data["il"], data["vis"], data["wt"], data["flag"])
        Go = oracle.grid(geom, t64, o64)
        Gh = G.cpu().numpy().astype(np.complex128)
        err = rel_l2(Gh, Go)
        say(f"  grid rel L2 {err:.3e}")
        assert err < tol
        if dtype != "f32":
            assert rel_l2(Gh, oracle.grid(geom, tq, orc)) < 1e-5
        rng = np.random.default_rng(79)
        gin = (rng.standard_normal(Gh.shape) + 1j * rng.standard_normal(Gh.shape)).astype(np.complex64)
        out = gr.degrid(torch.as_tensor(gin).to(DEV)).cpu().numpy().astype(np.complex128)
        ref = oracle.degrid(geom, t64, o64, gin.astype(np.complex128), data["uvw"], data["wt"], data["vis"].shape,
                            data["flag"])
        assert rel_l2(out, ref) < tol
        if dtype != "f32":
            refq = oracle.degrid(geom, tq, orc, gin.astype(np.complex128), data["uvw"], data["wt"], data["vis"].shape,
                                 data["flag"])
            assert rel_l2(out, refq) < 1e-5
        assert not np.any(out[data["flag"] != 0])
        imgs = gr.finalise(G).cpu().numpy().astype(np.float64)
        ref = oimg.finalise_stokes(geom, Gh, h["norm"], circular)
        assert imgs.shape[0] == len(ref)
        for k, (name, r) in enumerate(ref.items()):
            e = _fin_err(imgs[k], r, geom)
            say(f"  Stokes {name}: image rel L2 (before the taper division) {e:.3e}")
            assert e < 1e-5
        return
    # per-channel grids: each channel against the oracle imaging that channel alone
    assert tuple(G.shape) == (nc, npol, geom["n"], geom["n"])
    Gh = G.cpu().numpy().astype(np.complex128)
    norms = h["norm"].reshape(nc, npol)
    imgs = gr.finalise(G).cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(80)
    gin = (rng.standard_normal(Gh.shape) + 1j * rng.standard_normal(Gh.shape)).astype(np.complex64)
    back = gr.degrid(torch.as_tensor(gin).to(DEV)).cpu().numpy().astype(np.complex128)
    for c in range(nc):
        sl = slice(c, c + 1)
        oc32 = oracle.compress(geom, otable(geom, "f32"), data["uvw"], data["il"][sl], data["vis"][:, sl],
                               data["wt"][:, sl], data["flag"][:, sl])
        assert np.max(np.abs(norms[c] - oc32["normaliser"])) <= 1e-6 * np.max(np.abs(oc32["normaliser"]))
        oc = oracle.compress(geom, t64, data["uvw"], data["il"][sl], data["vis"][:, sl], data["wt"][:, sl],
                             data["flag"][:, sl])
        err = rel_l2(Gh[c], oracle.grid(geom, t64, oc))
        say(f"  channel {c}: grid rel L2 {err:.3e}")
        assert err < 1e-5
        refb = oracle.degrid(geom, t64, oc, gin[c].astype(np.complex128), data["uvw"], data["wt"][:, sl],
                             (nb, 1, nt, npol), data["flag"][:, sl])
        assert rel_l2(back[:, sl], refb) < 1e-5
        ref = oimg.finalise_stokes(geom, Gh[c], norms[c], circular)
        for k, (name, r) in enumerate(ref.items()):
            assert _fin_err(imgs[c, k], r, geom) < 1e-5, (c, name)


def test_runs_with_grid_ids_beyond_the_grids_are_skipped():
    """Runs are checked before any grid access: with every run's grid id moved past the last
    channel (or negative), wg_grid leaves the grids untouched and wg_degrid returns zeros."""
    geom, data = cfg1()
    g = wg.geom_from_dict(geom, per_channel=True)
    table = wg.KernelTable(g, "f32", device=DEV)
    uvw, il, vis, wt, fl = to_dev(data)
    gr = wg.Gridder(g, table, uvw, il, wt, fl)
    gr.compress(vis)
    n_runs = gr.runs.stats().n_runs
    assert n_runs > 0
    for bad in (gr.nc, -1):
        gr.runs.grid[:n_runs] = bad
        G = gr.grid()
        out = gr.degrid(torch.ones(gr.grid_shape(), dtype=torch.complex64, device=DEV))
        torch.cuda.synchronize()
        assert not torch.any(G != 0) and not torch.any(out != 0)


def test_failed_runs_interleaved_with_good_ones():
    """Every third run's grid id moved past the last channel: those runs are skipped (they add
    zero) and the others, in the same chunks and batches, still grid as the oracle's runs
    with the skipped runs' gammas set to zero (the channel grids summed)."""
    geom, data = cfg1()
    g = wg.geom_from_dict(geom, per_channel=True)
    table = wg.KernelTable(g, "f32", device=DEV)
    uvw, il, vis, wt, fl = to_dev(data)
    gr = wg.Gridder(g, table, uvw, il, wt, fl)
    gr.compress(vis)
    n_runs = gr.runs.stats().n_runs
    gr.runs.grid[0:n_runs:3] = gr.nc
    G = gr.grid().sum(0).cpu().numpy().astype(np.complex128)
    t64 = otable(geom, "f64")
    orc = oracle.compress(geom, t64, data["uvw"], data["il"], data["vis"], data["wt"], data["flag"])
    assert orc["n_runs"] == n_runs
    orc["gamma"] = np.array(orc["gamma"], copy=True)
    orc["gamma"][0::3] = 0
    Go = oracle.grid(geom, t64, orc)
    err = rel_l2(G, Go)
    say("failed runs interleaved: grid rel L2", err)
    assert err < 1e-5


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16"])
@pytest.mark.parametrize("case", ["cfg1", "cfg4"])
def test_table_is_even_in_each_offset(case, dtype):
    """The kernel is even in u and in v (eq. C_W with an even taper and w-screen): on the
    built table, the matrix of offset -o along an axis equals the matrix of +o reversed along
    that axis (which the gridder and degridder read in its place). With FP32 storage the two
    agree to FP32 rounding of the two transform outputs (1e-6 of the plane's largest sample).
    A 16-bit component is the rounding of two FP64 values that agree to far below 1e-12 of the
    plane's peak, so the two stored values differ by at most one unit in the last place of
    the larger, plus that 1e-12 of the peak (components at rounding-noise level, near zero,
    need the second term)."""
    geom = cfg1()[0] if case == "cfg1" else cfg4_small()[0]
    g = wg.geom_from_dict(geom)
    tb = wg.KernelTable(g, dtype, device=DEV)
    beta, hb = geom["beta"], geom["beta"] // 2
    data, off = unpad_table(tb, beta)
    ulp = {"f32": 0.0, "bf16": 2.0 ** -7, "f16": 2.0 ** -10}[dtype]
    sub = 2.0 ** -24 if dtype == "f16" else 0.0
    worst = worst_ulp = 0.0
    differ = total = 0
    for k in range(geom["n_w"]):
        S = tb.support[k]
        plane = data[off[k]:off[k + 1]].reshape(beta, beta, S, S)   # [ov][ou][i][j]
        peak = np.max(np.abs(plane))
        for ov in range(-hb + 1, hb + 1):
            for ou in range(-hb + 1, hb + 1):
                m = plane[ov + hb - 1, ou + hb - 1]
                src = plane[abs(ov) + hb - 1, abs(ou) + hb - 1]
                if ou < 0:
                    src = src[:, ::-1]
                if ov < 0:
                    src = src[::-1, :]
                worst = max(worst, float(np.max(np.abs(m - src))) / peak)
                if ulp:
                    for a, b in ((m.real, src.real), (m.imag, src.imag)):
                        d = np.abs(a - b)
                        big = np.maximum(np.abs(a), np.abs(b))
                        worst_ulp = max(worst_ulp, float(np.max(d / (ulp * big + sub + 1e-12 * peak))))
                        differ += int(np.count_nonzero(d))
                        total += d.size
    say(f"  {case} {dtype}: largest mirror difference {worst:.2e} of the plane peak"
        + (f", {worst_ulp:.3f} of the bound, {differ} of {total} components differ" if ulp else ""))
    if dtype == "f32":
        assert worst < 1e-6
    else:
        assert worst_ulp <= 1.0 + 1e-9


@pytest.mark.parametrize("case", ["cfg1", "cfg4"])
def test_polarised_w_stacking(case):
    """W-stacking of four-product records against the oracle: runs and grid ids bit-exact,
    every [plane][product] grid within 1e-5, per-product normalisers, the adjoint within 1e-5
    and the stacked Stokes images within 1e-5 before the taper division."""
    from oracle import image as oimg
    geom, data = _pol_case(case, 4, False)
    nb, nc, nt, npol = data["vis"].shape
    n_w = geom["n_w"]
    say("polarised w-stacking", case)
    g = wg.geom_from_dict(geom, w_stacking=True, n_pol=npol)
    table = wg.KernelTable(g, "f32", device=DEV)
    uvw, il, vis, wt, fl = to_dev(data)
    gr = wg.Gridder(g, table, uvw, il, wt, fl)
    gr.compress(vis)
    G = gr.grid()
    torch.cuda.synchronize()
    assert tuple(G.shape) == (n_w, npol, geom["n"], geom["n"])
    h = gr.runs.host()
    o32, _, on32 = oracle.w_stacking(geom, otable(geom, "f32"), data["uvw"], data["il"], data["vis"], data["wt"],
                                     data["flag"])
    cat = {k: np.concatenate([r[k].astype(np.int64) for r in o32]) for k in ("start", "len", "x", "y", "ou", "ov")}
    cat["grid"] = np.concatenate([np.full(r["n_runs"], j, np.int64) for j, r in enumerate(o32)])
    order = np.argsort(cat["start"], kind="stable")
    for k in ("start", "len", "x", "y", "ou", "ov", "grid"):
        assert np.array_equal(h[k].astype(np.int64), cat[k][order]), k
    assert np.max(np.abs(h["norm"] - on32)) <= 1e-6 * np.max(np.abs(on32))
    t64 = otable(geom, "f64")
    oruns, Go, _ = oracle.w_stacking(geom, t64, data["uvw"], data["il"], data["vis"], data["wt"], data["flag"])
    Gh = G.cpu().numpy().astype(np.complex128)
    for k in range(n_w):
        if np.any(Go[k]):
            assert rel_l2(Gh[k], Go[k]) < 1e-5, k
        else:
            assert not np.any(Gh[k])
    rng = np.random.default_rng(81)
    gin = (rng.standard_normal(Gh.shape) + 1j * rng.standard_normal(Gh.shape)).astype(np.complex64)
    out = gr.degrid(torch.as_tensor(gin).to(DEV)).cpu().numpy().astype(np.complex128)
    ref = oracle.w_stacking_degrid(geom, t64, oruns, gin.astype(np.complex128), data["uvw"], data["wt"],
                                   data["vis"].shape, data["flag"])
    assert rel_l2(out, ref) < 1e-5
    imgs = gr.finalise(G).cpu().numpy().astype(np.float64)
    ref = oimg.finalise_stokes_stacked(geom, Gh, h["norm"], False)
    for i, (name, r) in enumerate(ref.items()):
        e = _fin_err(imgs[i], r, geom)
        say(f"  stacked Stokes {name}: rel L2 (before the taper division) {e:.3e}")
        assert e < 1e-5


def _pol_records(nb, nc, nt, npol, geom, seed):
    d = _records(nb, nc, nt, geom, seed)
    rng = np.random.default_rng(seed + 100)
    shp = (nb, nc, nt, npol)
    d["vis"] = (rng.standard_normal(shp) + 1j * rng.standard_normal(shp)).astype(np.complex64)
    d["wt"] = rng.uniform(0.0, 2.0, shp).astype(np.float32)
    d["flag"] = (rng.uniform(size=shp) < 0.3).astype(np.uint8)
    return d


@pytest.mark.parametrize("nt", [1, 65, 130])
def test_polarised_ragged_and_partially_flagged(nt):
    """Four products with 30 % of products flagged (zero weights included), ragged segment
    lengths: runs bit-exact, grid and degrid within 1e-5 of the oracle; a record flagged in
    some products only is still gridded, and its flagged products get 0 back."""
    data = _pol_records(3, 2, nt, 4, EDGE_GEOM, seed=60 + nt)
    data["flag"][0, 0, 0, :3] = 1            # one record keeps a single product
    g = wg.geom_from_dict(EDGE_GEOM, n_pol=4)
    table = wg.KernelTable(g, "f32", device=DEV)
    uvw, il, vis, wt, fl = to_dev(data)
    gr = wg.Gridder(g, table, uvw, il, wt, fl)
    gr.compress(vis)
    G = gr.grid()
    orc = oracle.compress(EDGE_GEOM, otable(EDGE_GEOM, "f32"), data["uvw"], data["il"], data["vis"], data["wt"],
                          data["flag"])
    compare_runs(gr, orc)
    t64 = otable(EDGE_GEOM, "f64")
    o64 = oracle.compress(EDGE_GEOM, t64, data["uvw"], data["il"], data["vis"], data["wt"], data["flag"])
    Go = oracle.grid(EDGE_GEOM, t64, o64)
    assert rel_l2(G.cpu().numpy().astype(np.complex128), Go) < 1e-5
    out = gr.degrid(G).cpu().numpy().astype(np.complex128)
    ref = oracle.degrid(EDGE_GEOM, t64, o64, G.cpu().numpy().astype(np.complex128), data["uvw"], data["wt"],
                        data["vis"].shape, data["flag"])
    assert rel_l2(out, ref) < 1e-5
    assert not np.any(out[data["flag"] != 0])


def test_polarised_everything_flagged():
    """Four products all flagged: no runs, zero grids, zero normalisers, zero Stokes images
    and zero degridded values."""
    data = _pol_records(2, 2, 70, 4, EDGE_GEOM, seed=3)
    data["flag"][:] = 1
    g = wg.geom_from_dict(EDGE_GEOM, n_pol=4)
    table = wg.KernelTable(g, "f32", device=DEV)
    uvw, il, vis, wt, fl = to_dev(data)
    gr = wg.Gridder(g, table, uvw, il, wt, fl)
    gr.compress(vis)
    G = gr.grid()
    st = gr.runs.stats()
    assert st.n_runs == 0 and st.n_griddable == 0
    assert not torch.any(G != 0) and not torch.any(gr.runs.norm != 0)
    imgs = gr.finalise(G)
    out = gr.degrid(G)
    torch.cuda.synchronize()
    assert not torch.any(imgs != 0) and not torch.any(out != 0)


def _shifted(t):
    """The same values one element past an aligned allocation (8 bytes for complex64, 4 for
    float32, 1 for uint8), so that a record's products are not 16-byte aligned."""
    flat = t.reshape(-1)
    buf = torch.empty(flat.numel() + 1, dtype=t.dtype, device=t.device)
    buf[1:] = flat
    return buf[1:].view(t.shape)


@pytest.mark.parametrize("npol", [2, 4])
def test_polarised_unaligned_inputs_match_aligned(npol):
    """Two and four products from unaligned vis, weight and flag pointers (the per-product
    loads) give the same runs and gammas, bit for bit, and the same normalisers as from
    aligned ones (the per-record vector loads), and match the oracle."""
    data = _pol_records(3, 2, 70, npol, EDGE_GEOM, seed=80 + npol)
    data["flag"][0, 0, :5, 0] = 1
    g = wg.geom_from_dict(EDGE_GEOM, n_pol=npol)
    table = wg.KernelTable(g, "f32", device=DEV)
    uvw, il, vis, wt, fl = to_dev(data)
    say("unaligned", npol, vis.data_ptr() % 16, _shifted(vis).data_ptr() % 16)
    assert _shifted(vis).data_ptr() % 16 != 0 and _shifted(fl).data_ptr() % npol != 0
    gr_a = wg.Gridder(g, table, uvw, il, wt, fl)
    gr_a.compress(vis)
    gr_u = wg.Gridder(g, table, uvw, il, _shifted(wt), _shifted(fl))
    gr_u.compress(_shifted(vis))
    ha, hu = gr_a.runs.host(), gr_u.runs.host()
    assert ha["n_runs"] == hu["n_runs"] > 0
    for k in ("start", "len", "x", "y", "plane", "ou", "ov", "gamma"):
        assert np.array_equal(ha[k], hu[k]), k
    # the waves' normaliser sums meet in FP64 atomics, whose order may vary between launches
    assert np.allclose(ha["norm"], hu["norm"], rtol=1e-12, atol=0)
    orc = oracle.compress(EDGE_GEOM, otable(EDGE_GEOM, "f32"), data["uvw"], data["il"], data["vis"], data["wt"],
                          data["flag"])
    compare_runs(gr_u, orc)
