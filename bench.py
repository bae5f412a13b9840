#!/usr/bin/env python3
"""Benchmark: w-projection gridding with compression on one MI355X.

One step = the whole hot path over one batch of records: kernel-table build, index +
compression, gridding and degridding (the adjoint), on the plain FP32 throughput workload
(44 stations / 946 baselines x 16 channels x 512 timesteps = 7,749,632 records, 2048^2
grid, oversampling 8, 32 w-planes, supports 9..63). Inputs are synthetic (seeded earth-
rotation tracks and point-source visibilities) and resident in HBM before timing starts.

Prints ONE JSON line. `value` = grid-point updates per second over the step (the gridder's
updates plus the degridder's, each sum over runs of S^2). Per-phase times, the BF16-table
variant, the uncompressed variant, the w-stacking variant (grid per w-plane + stacked image
against w-projection's grid + image), the polarisation variant (the same records as 2 and 4
products), the image finaliser, the table-generation study, the
gridder's roofline and the CPU oracle baseline are extra fields.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_COUNTERS = os.path.join(ROOT, "profiles", "grid_cfg2_counters.txt")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="skip the table study and the BF16, uncompressed and w-stacking variants")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (to scale HBM counters)")
    return ap.parse_args()


def copy_calibration(nbytes: int):
    """A plain copy kernel of known size: its FETCH_SIZE / WRITE_SIZE readings give the
    factor between the counters and real HBM bytes."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "dispatches": 3}), flush=True)


def gpu_step(wg, geom, kt, ws, gridder, vis, grid, vis_out, ev):
    """One pass of the hot path; records events between phases on the current stream."""
    ev[0].record()
    wg.wg_ktable_build(geom, kt, ws, host_copies=False)
    ev[1].record()
    gridder.compress(vis)
    ev[2].record()
    grid.zero_()
    ev[3].record()
    gridder.grid(out=grid)
    ev[4].record()
    gridder.degrid(grid, out=vis_out)
    ev[5].record()
    return ev


def grid_source_hash() -> str:
    """First 16 hex digits of the SHA-256 of the gridder's sources (grid.hip, then
    wg_common.hpp, whose constants set its slot counts)."""
    import hashlib
    h = hashlib.sha256()
    for name in ("grid.hip", "wg_common.hpp"):
        with open(os.path.join(ROOT, "paper_1403_4209_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_counters(kernel):
    """HBM bytes per launch of `kernel` (k_grid or k_degrid) from the committed rocprofv3
    counter summary, or None when their source has changed since the counters were taken."""
    try:
        with open(PROFILE_COUNTERS) as f:
            kv = dict(line.split(":", 1) for line in f if ":" in line)
        if kv["grid_sources_sha256_16"].split()[0] != grid_source_hash():
            return None
        return float(kv[f"traffic_{kernel}"].strip())
    except Exception:
        return None


def roofline(kernel, alg_bytes, ms, traffic):
    achieved = alg_bytes / (ms * 1e-3) / 1e9
    return {"kernel": kernel, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic}


def cpu_baseline(w, vis_h, u_full):
    """The FP64 oracle (single thread) on every 16th baseline; the per-record phases are
    scaled to the full workload by update count, the table build is counted once."""
    import numpy as np

    import oracle
    oracle.build(force=False)
    t0 = time.perf_counter()
    t64 = oracle.ktable.build(w.geom, "f32")
    t_table = time.perf_counter() - t0
    sub = slice(0, None, 16)
    uvw, vis = w.uvw[sub], vis_h[sub]
    t0 = time.perf_counter()
    runs = oracle.compress(w.geom, t64, uvw, w.inv_lambda, vis)
    t1 = time.perf_counter()
    G = oracle.grid(w.geom, t64, runs)
    t2 = time.perf_counter()
    oracle.degrid(w.geom, t64, runs, G, uvw, None, vis.shape)
    t3 = time.perf_counter()
    u_s = int(runs["stats"][4])
    scale = u_full / max(u_s, 1)
    t_full = t_table + (t3 - t0) * scale
    return {"value": round(2 * u_full / t_full / 1e9, 4), "unit": "Gupd/s", "cores": 1, "kind": "oracle",
            "sample": (f"every 16th baseline ({uvw.shape[0]} of {w.uvw.shape[0]}; {vis.size} records, "
                       f"{u_s} updates); table build {t_table:.2f}s once, compress {t1 - t0:.2f}s, "
                       f"grid {t2 - t1:.2f}s, degrid {t3 - t2:.2f}s scaled x{scale:.2f} to the full step"),
            "seconds_full_step": round(t_full, 2)}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); multi-GPU sharding is a design note",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    import numpy as np
    import torch

    import workloads
    from paper_1403_4209_amd import wgrid as wg

    dev = torch.device("cuda:0")
    w = workloads.make(2, device=dev)
    geom = wg.geom_from_dict(w.geom, compress=True)
    uvw = torch.as_tensor(w.uvw).to(dev)
    il = torch.as_tensor(w.inv_lambda).to(dev)
    vis = w.vis
    weight = w.weight
    nb, nt = w.uvw.shape[:2]
    nc = w.inv_lambda.shape[0]

    # persistent buffers: table (f32), table workspace, grid, degrid output
    table = wg.KernelTable(geom, "f32", device=dev)
    _, ws_bytes = wg.wg_ktable_sizes(geom)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    gridder = wg.Gridder(geom, table, uvw, il, weight)
    grid = torch.zeros((geom.n, geom.n), dtype=torch.complex64, device=dev)
    vis_out = torch.empty_like(vis)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]

    for _ in range(args.warmup):
        gpu_step(wg, geom, table.kt, ws, gridder, vis, grid, vis_out, ev)
    torch.cuda.synchronize()
    phase = np.zeros(5)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        gpu_step(wg, geom, table.kt, ws, gridder, vis, grid, vis_out, ev)
        torch.cuda.synchronize()
        phase += [ev[i].elapsed_time(ev[i + 1]) for i in range(5)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    phase /= args.steps
    ms_step = wall * 1e3 / args.steps
    st = gridder.runs.stats()
    U = st.upd_real
    t_ktable, t_comp, t_zero, t_grid, t_degrid = phase
    value = 2.0 * U / (ms_step * 1e-3) / 1e9

    # rooflines: algorithmic bytes per launch = table samples streamed (8 B each for FP32) +
    # run fields read or partial sums written (20 B per run) + the grid read and written once
    # (gridder, 16 B per cell) or read once (degridder, 8 B per cell). The dominant (slower)
    # kernel of the step is reported as `roofline`, the other as `roofline_other`.
    nn = geom.n * geom.n
    rl_grid = roofline("k_grid (wg_grid)", U * 8 + st.n_runs * 20 + 16 * nn, t_grid, read_counters("k_grid"))
    rl_degrid = roofline("k_degrid (wg_degrid)", U * 8 + st.n_runs * 20 + 8 * nn, t_degrid, read_counters("k_degrid"))
    rl_main, rl_other = (rl_degrid, rl_grid) if t_degrid > t_grid else (rl_grid, rl_degrid)

    out = {
        "metric": "grid-point updates/sec (Gupd/s) + HBM GB/s; BF16-kernel vs FP32 at stated rel err",
        "value": round(value, 3),
        "unit": "Gupd/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded LOFAR-like array, earth-rotation tracks, 200 point sources + noise)",
        "config": {"workload": ("plain FP32 gridding, 44 stations (946 baselines) x 16 channels x 512 timesteps = "
                                "7,749,632 records, grid 2048x2048 complex64, oversampling 8, 32 w-planes, "
                                "supports 9..63, compression on"),
                   "records": int(st.n_records), "runs": int(st.n_runs), "upd_real": int(U),
                   "upd_total": int(U + st.upd_saved)},
        "phases_ms": {"ktable": round(t_ktable, 4), "compress": round(t_comp, 4), "grid_zero": round(t_zero, 4),
                      "grid": round(t_grid, 4), "degrid": round(t_degrid, 4)},
        "grid_gupds_real": round(U / (t_grid * 1e-3) / 1e9, 2),
        "grid_gupds_total": round((U + st.upd_saved) / (t_grid * 1e-3) / 1e9, 2),
        "degrid_gupds": round(U / (t_degrid * 1e-3) / 1e9, 2),
        "compression_ratio_records": round(st.n_griddable / max(st.n_runs, 1), 3),
        "compression_ratio_updates": round((U + st.upd_saved) / max(U, 1), 3),
        "roofline": rl_main,
        "roofline_other": rl_other,
    }

    # image finaliser (inverse FFT + corrections) of the step's grid, timed on its own: it is
    # not part of the gridding step
    g32 = grid.clone()
    fin_ws = torch.empty(wg.wg_finalise_ws_bytes(geom), dtype=torch.uint8, device=dev)
    image = torch.empty((geom.n, geom.n), dtype=torch.float32, device=dev)
    gridder.finalise(g32, out=image)
    torch.cuda.synchronize()
    t_fin = 0.0
    for _ in range(args.steps):
        ev[0].record()
        wg.finalise(geom, g32, gridder.runs.normaliser(), out=image, ws=fin_ws)
        ev[1].record()
        torch.cuda.synchronize()
        t_fin += ev[0].elapsed_time(ev[1])
    out["finalise_ms"] = round(t_fin / args.steps, 4)
    del fin_ws, image

    if not args.no_variants:
        # table-generation study: the FP32 table of this geometry with more w-planes, up to the
        # thesis's 200 (build timed alone, host copies off as in the step)
        study = {}
        for n_w in (32, 64, 128, 200):
            gd = dict(w.geom, n_w=n_w)
            gs = wg.geom_from_dict(gd)
            ts = wg.KernelTable(gs, "f32", device=dev)
            _, wsb = wg.wg_ktable_sizes(gs)
            wss = torch.empty(wsb, dtype=torch.uint8, device=dev)
            wg.wg_ktable_build(gs, ts.kt, wss, host_copies=False)
            torch.cuda.synchronize()
            tt = 0.0
            for _ in range(3):
                ev[0].record()
                wg.wg_ktable_build(gs, ts.kt, wss, host_copies=False)
                ev[1].record()
                torch.cuda.synchronize()
                tt += ev[0].elapsed_time(ev[1])
            study[str(n_w)] = round(tt / 3, 4)
            del ts, wss
        out["ktable_ms_by_planes"] = study

        # BF16 table, same records (grid and degrid only; table build timed once)
        tb16 = wg.KernelTable(geom, "bf16", device=dev)
        g16 = wg.Gridder(geom, tb16, uvw, il, weight)
        g16.compress(vis)
        for _ in range(2):
            grid.zero_()
            g16.grid(out=grid)
            g16.degrid(grid, out=vis_out)
        torch.cuda.synchronize()
        tg = td = 0.0
        for _ in range(args.steps):
            grid.zero_()
            ev[0].record()
            g16.grid(out=grid)
            ev[1].record()
            g16.degrid(grid, out=vis_out)
            ev[2].record()
            torch.cuda.synchronize()
            tg += ev[0].elapsed_time(ev[1])
            td += ev[1].elapsed_time(ev[2])
        tg /= args.steps
        td /= args.steps
        g64, d64 = g32.to(torch.complex128), grid.to(torch.complex128)
        rel_bf16 = float(torch.linalg.norm(d64 - g64) / torch.linalg.norm(g64))
        out["bf16"] = {"grid_ms": round(tg, 4), "degrid_ms": round(td, 4),
                       "grid_gupds_real": round(U / (tg * 1e-3) / 1e9, 2),
                       "speedup_grid_vs_f32": round(t_grid / tg, 3), "speedup_degrid_vs_f32": round(t_degrid / td, 3),
                       "rel_l2_vs_f32_table_grid": float(f"{rel_bf16:.3e}"),
                       "rel_err_bound_vs_fp64_oracle": 3e-3}
        del g64, d64
        del g16, tb16
        # compression off: every griddable record is its own run
        geom_u = wg.geom_from_dict(w.geom, compress=False)
        gu = wg.Gridder(geom_u, table, uvw, il, weight)
        tcu = tgu = 0.0
        for i in range(args.steps + 1):
            grid.zero_()
            ev[0].record()
            gu.compress(vis)
            ev[1].record()
            gu.grid(out=grid)
            ev[2].record()
            torch.cuda.synchronize()
            if i:
                tcu += ev[0].elapsed_time(ev[1])
                tgu += ev[1].elapsed_time(ev[2])
        tcu /= args.steps
        tgu /= args.steps
        out["uncompressed"] = {"compress_ms": round(tcu, 4), "grid_ms": round(tgu, 4),
                               "speedup_of_compression": round((tcu + tgu) / (t_comp + t_grid), 3)}
        del gu

        # w-stacking (eq. stacking) of the same records: every record gridded with the w = 0
        # kernel (support 9) on the grid of its w-plane (32 grids of 2048^2), then the planes
        # transformed, w-corrected and added; against w-projection's grid + finalise
        geom_s = wg.geom_from_dict(w.geom, w_stacking=True)
        gs_ = wg.Gridder(geom_s, table, uvw, il, weight)
        grids = torch.zeros(gs_.grid_shape(), dtype=torch.complex64, device=dev)
        img_s = torch.empty((geom.n, geom.n), dtype=torch.float32, device=dev)
        tcs = tgs = tfs = 0.0
        for i in range(args.steps + 1):
            grids.zero_()
            ev[0].record()
            gs_.compress(vis)
            ev[1].record()
            gs_.grid(out=grids)
            ev[2].record()
            gs_.finalise(grids, out=img_s)
            ev[3].record()
            torch.cuda.synchronize()
            if i:
                tcs += ev[0].elapsed_time(ev[1])
                tgs += ev[1].elapsed_time(ev[2])
                tfs += ev[2].elapsed_time(ev[3])
        tcs, tgs, tfs = tcs / args.steps, tgs / args.steps, tfs / args.steps
        ss = gs_.runs.stats()
        out["w_stacking"] = {"grids": int(geom.n_w), "compress_ms": round(tcs, 4), "grid_ms": round(tgs, 4),
                             "finalise_stacked_ms": round(tfs, 4), "upd_real": int(ss.upd_real),
                             "grid_gupds_real": round(ss.upd_real / (tgs * 1e-3) / 1e9, 2),
                             "image_ms": round(tcs + tgs + tfs, 4),
                             "w_projection_image_ms": round(t_comp + t_grid + out["finalise_ms"], 4)}
        del gs_, grids, img_s

        # polarisations (the thesis's experiment batch 4): the same records as 4 and 2
        # products (seeded polarised sources, per-product weights and flags); grid and degrid
        # times against the single-polarisation step, record rates and product updates per second
        pol = {}
        wp = workloads.polarised(2, 4, device=dev)
        for npol in (4, 2):
            vp = wp.vis if npol == 4 else wp.vis[..., [0, 3]].contiguous()
            wtp = wp.weight if npol == 4 else wp.weight[..., [0, 3]].contiguous()
            flp = wp.flag if npol == 4 else wp.flag[..., [0, 3]].contiguous()
            gp_ = wg.geom_from_dict(w.geom, n_pol=npol)
            gpp = wg.Gridder(gp_, table, uvw, il, wtp, flp)
            gridp = torch.zeros(gpp.grid_shape(), dtype=torch.complex64, device=dev)
            voutp = torch.empty(gpp.vis_shape(), dtype=torch.complex64, device=dev)
            tcp = tgp = tdp = 0.0
            for i in range(args.steps + 1):
                gridp.zero_()
                ev[0].record()
                gpp.compress(vp)
                ev[1].record()
                gpp.grid(out=gridp)
                ev[2].record()
                gpp.degrid(gridp, out=voutp)
                ev[3].record()
                torch.cuda.synchronize()
                if i:
                    tcp += ev[0].elapsed_time(ev[1])
                    tgp += ev[1].elapsed_time(ev[2])
                    tdp += ev[2].elapsed_time(ev[3])
            tcp, tgp, tdp = tcp / args.steps, tgp / args.steps, tdp / args.steps
            sp = gpp.runs.stats()
            pol[str(npol)] = {"compress_ms": round(tcp, 4), "grid_ms": round(tgp, 4), "degrid_ms": round(tdp, 4),
                              "runs": int(sp.n_runs),
                              "grid_gupds_products": round(sp.upd_real * npol / (tgp * 1e-3) / 1e9, 2),
                              "degrid_gupds_products": round(sp.upd_real * npol / (tdp * 1e-3) / 1e9, 2),
                              "grid_record_rate_vs_1pol": round(t_grid / tgp, 3)}
            del gpp, gridp, voutp
        pol["1"] = {"grid_ms": round(t_grid, 4), "degrid_ms": round(t_degrid, 4),
                    "grid_gupds_products": round(U / (t_grid * 1e-3) / 1e9, 2)}
        out["polarisations"] = pol
        del wp

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, vis.cpu().numpy(), U)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
