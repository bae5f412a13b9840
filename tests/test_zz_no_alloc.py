"""wg_grid_records_static (the workspace-free entry point) against wg_grid_records, through
the C ABI: two calls in a row on one GPU, the second with a smaller batch; runs, keys and
integer counters bit-exact, normaliser to 1e-12, grid within 1e-6 of the workspace
version's (FP32 atomic commit order) and within 1e-5 of the FP64 oracle; the runs it leaves
in its array serve wg_degrid. Batches beyond the array are refused on the host."""
import ctypes

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


def say(*a):
    print(*a, flush=True)


_HIP = None


def _hip():
    """The HIP runtime torch has loaded (one runtime per process), for raw device copies."""
    global _HIP
    if _HIP is None:
        import os
        _HIP = ctypes.CDLL(os.path.join(os.path.dirname(torch.__file__), "lib", "libamdhip64.so"))
        _HIP.hipMemcpy.restype = ctypes.c_int
        _HIP.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    return _HIP


def _host_runs(runs: wg.WgRuns, n):
    """The first n runs of a wg_runs view (device pointers) copied to the host."""
    torch.cuda.synchronize()
    out = {}
    for name, dt in (("start", np.int32), ("len", np.int32), ("x", np.int32), ("y", np.int32),
                     ("plane", np.int16), ("ou", np.int8), ("ov", np.int8), ("gamma", np.float32)):
        a = np.zeros(2 * n if name == "gamma" else n, dtype=dt)
        assert _hip().hipMemcpy(a.ctypes.data, getattr(runs, name), a.nbytes, 2) == 0  # device to host
        out[name] = a
    return out


def _stats(stats_d):
    h = stats_d.cpu()
    return [int(v) for v in h[:6]] + [float(h[6:7].view(torch.float64)[0]), int(h[7])]


def test_static_workspace_matches_workspace_entry_point_on_two_calls():
    w = workloads.make(4, n_st=20, n_t=100, n_ch=4)
    geom = wg.geom_from_dict(w.geom)
    table = wg.KernelTable(geom, "f32", device=DEV)
    t64 = okt.build(w.geom, "f64")
    t32 = okt.requantize(t64, "f32")
    uvw_all = torch.as_tensor(w.uvw).to(DEV)
    il_all = torch.as_tensor(w.inv_lambda).to(DEV)
    vis_all = torch.as_tensor(w.vis).to(DEV)
    n = geom.n
    for call, (nb, nc) in enumerate([(190, 4), (70, 2)]):
        uvw = uvw_all[:nb].contiguous()
        il = il_all[:nc].contiguous()
        vis = vis_all[:nb, :nc].contiguous()
        nt = vis.shape[2]
        say(f"call {call}: {nb} x {nc} x {nt} records")
        # the workspace entry point
        gr = wg.Gridder(geom, table, uvw, il)
        G_ws = gr.grid_records(vis)
        # the workspace-free one
        G_st = torch.zeros((n, n), dtype=torch.complex64, device=DEV)
        stats_st = torch.zeros(8, dtype=torch.int64, device=DEV)
        runs_st = wg.wg_grid_records_static(geom, table.kt, uvw, il, torch.view_as_real(vis), None, None, nb, nc, nt,
                                            torch.view_as_real(G_st), stats_st)
        torch.cuda.synchronize()
        s_ws, s_st = _stats(gr.runs.stats_d), _stats(stats_st)
        assert s_ws[:6] == s_st[:6] and s_ws[7] == s_st[7], (s_ws, s_st)
        assert abs(s_ws[6] - s_st[6]) <= 1e-12 * abs(s_ws[6])
        nr = s_st[2]
        assert nr > 0
        h_ws = gr.runs.host()
        h_st = _host_runs(runs_st, nr)
        for k in ("start", "len", "x", "y", "plane", "ou", "ov"):
            assert np.array_equal(h_ws[k], h_st[k]), k
        assert np.array_equal(h_ws["gamma"].view(np.float32), h_st["gamma"])
        a, b = G_st.cpu().numpy().astype(np.complex128), G_ws.cpu().numpy().astype(np.complex128)
        e_ws = np.linalg.norm(a - b) / np.linalg.norm(b)
        m_ws = np.max(np.abs(a - b)) / np.max(np.abs(b))
        orc = oracle.compress(w.geom, t32, w.uvw[:nb], w.inv_lambda[:nc], w.vis[:nb, :nc])
        Go = oracle.grid(w.geom, t64, orc)
        e_o = np.linalg.norm(a - Go) / np.linalg.norm(Go)
        m_o = np.max(np.abs(a - Go)) / np.max(np.abs(Go))
        # the runs left in the array serve the adjoint
        V = torch.empty_like(vis)
        wg.wg_degrid(geom, table.kt, runs_st, stats_st, torch.view_as_real(G_st), uvw, None, None, nb, nc, nt,
                     torch.view_as_real(V))
        torch.cuda.synchronize()
        Vo = oracle.degrid(w.geom, t64, orc, a, w.uvw[:nb], None, (nb, nc, nt))
        e_v = np.linalg.norm(V.cpu().numpy() - Vo) / np.linalg.norm(Vo)
        say(f"  runs {nr}: vs workspace L2 {e_ws:.2e} max {m_ws:.2e}; vs oracle L2 {e_o:.2e} max {m_o:.2e}; "
            f"degrid {e_v:.2e}")
        assert e_ws < 1e-6 and m_ws < 1e-6
        assert e_o < 1e-5 and m_o < 1e-5 and e_v < 1e-5


def test_static_workspace_refuses_batches_beyond_its_array():
    w = workloads.make(1)
    geom = wg.geom_from_dict(w.geom)
    table = wg.KernelTable(geom, "f32", device=DEV)
    assert wg.wg_grid_records_ws(geom, 4096, 64, 512) > (64 << 20)
    L = wg.lib()
    by = ctypes.byref
    one = torch.zeros(16, dtype=torch.float64, device=DEV)
    grid = torch.zeros(2 * geom.n * geom.n, dtype=torch.float32, device=DEV)
    stats = torch.zeros(8, dtype=torch.int64, device=DEV)
    st = L.wg_grid_records_static(by(geom), by(table.kt), wg._p(one), wg._p(one), wg._p(grid), None, None,
                                  4096, 64, 512, wg._p(grid), wg._p(stats), None, None)
    assert st == wg.WG_ECAPACITY
