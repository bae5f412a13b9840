#!/usr/bin/env python3
"""Benchmark: w-projection gridding with compression on one MI355X.

One step = the whole hot path over one batch of records: kernel-table build, index +
compression, gridding and degridding (the adjoint), on the compression workload (44
stations / 946 baselines x 64 channels x 512 timesteps of 1 s = 30,998,528 records, 4096^2
grid, oversampling 8, 64 w-planes, supports 9..63): the largest of the workloads by
grid-point updates. Inputs are synthetic (seeded earth-rotation tracks and point-source
visibilities) and resident in HBM before timing starts.

Prints ONE JSON line. `value` = grid-point updates per second over the step (the gridder's
updates plus the degridder's, each the sum over runs of S^2). Extra fields: per-phase
times; the one-call wg_grid_records; BF16 and FP16 tables and the thesis's plain FP32 sums
per owned cell (times, speedups, and their errors against the FP64 oracle measured in the
CPU-baseline leg); the uncompressed variant;
the other throughput workloads (plain FP32, 2048^2; differentiation, 66.8 M records) as
full steps; the table-generation study; w-stacking and polarisations; the image finaliser;
the dominant kernel's roofline against the FP32 vector peak with its measured HBM traffic,
vector memory issue interval and VALU instruction rate; and the CPU oracle baseline.
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
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2 (packed FP32) x 2.4 GHz
FP32_VECTOR_PEAK_TFLOPS = 157.3
FLOPS_PER_UPDATE = 8             # one complex multiply-add per grid-point update
# CU cycles per 64-lane 16-byte vector load measured by a probe of loads from an L2-resident
# table (60 B per CU-clock): the issue interval of the vector memory path
VMEM_PROBE_CYCLES = 17.1
PROFILE_COUNTERS = os.path.join(ROOT, "profiles", "grid_cfg3_counters.txt")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="time the headline step only (no table study, table types, other workloads or modes)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (to scale HBM counters)")
    ap.add_argument("--profile-workload", type=int, default=0, choices=(0, 2, 3, 5), metavar="CFG",
                    help="only run WARMUP + STEPS full steps of workload CFG (2, 3 or 5) and print their "
                         "phase times, for profiler runs")
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


def grid_source_hash() -> str:
    """First 16 hex digits of the SHA-256 of the gridder's sources (grid.hip, then
    wg_common.hpp, whose constants set its slot counts)."""
    import hashlib
    h = hashlib.sha256()
    for name in ("grid.hip", "wg_common.hpp"):
        with open(os.path.join(ROOT, "paper_1403_4209_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_counters():
    """Per-launch figures of k_grid and k_degrid from the committed rocprofv3 counter
    summary (HBM bytes, VALU instructions per SIMD-cycle, CU cycles per vector memory
    instruction, texture-data unit busy fraction), or {} when the gridder's sources have
    changed since the counters were taken."""
    try:
        with open(PROFILE_COUNTERS) as f:
            kv = {k.strip(): v.strip() for k, v in (line.split(":", 1) for line in f if ":" in line)}
        if kv["grid_sources_sha256_16"].split()[0] != grid_source_hash():
            return {}
        return {k: float(v.split()[0]) for k, v in kv.items()
                if k.startswith(("traffic_", "valu_ipc_", "vmem_cycles_per_inst_", "td_busy_"))}
    except Exception:
        return {}


def roofline(kernel, updates, ms, counters):
    """The kernel against the FP32 vector peak (gridding is a scatter of 8-flop complex
    multiply-adds whose table samples the caches serve), with its measured HBM traffic per
    launch and, from the counter summary, what binds it: the vector memory instruction rate
    (CU cycles per instruction against the about 17 of a probe of 16-byte loads from L2) and
    the VALU instruction rate."""
    tf = FLOPS_PER_UPDATE * updates / (ms * 1e-3) / 1e12
    key = "k_grid" if kernel.startswith("k_grid") else "k_degrid"
    traffic = counters.get(f"traffic_{key}")
    out = {"kernel": kernel, "bound": "alu", "achieved": round(tf, 3), "peak": FP32_VECTOR_PEAK_TFLOPS,
           "unit": "TFLOP/s", "frac": round(tf / FP32_VECTOR_PEAK_TFLOPS, 4), "traffic": traffic}
    if traffic is not None:
        gbs = traffic / (ms * 1e-3) / 1e9
        out["hbm_measured"] = {"achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": round(gbs / HBM_PEAK_GBS, 4)}
    if f"vmem_cycles_per_inst_{key}" in counters:
        c = counters[f"vmem_cycles_per_inst_{key}"]
        out["vmem_issue"] = {"cycles_per_inst": c, "probe_cycles_per_inst": VMEM_PROBE_CYCLES,
                             "frac": round(VMEM_PROBE_CYCLES / c, 4)}
    if f"td_busy_{key}" in counters:
        # the vector memory path: fraction of cycles the texture-data units are busy
        out["vmem_td_busy_frac"] = counters[f"td_busy_{key}"]
    if f"valu_ipc_{key}" in counters:
        # VALU wave-instructions per SIMD-cycle: a SIMD issues at most one a cycle, so this
        # is also the fraction of issue slots the VALU took
        out["valu_insts_per_simd_cycle"] = counters[f"valu_ipc_{key}"]
        out["valu_issue_frac"] = counters[f"valu_ipc_{key}"]
    return out


class Case:
    """Device buffers for one workload and table type: table, table workspace, gridder,
    grid, degrid output."""

    def __init__(self, w, dtype="f32", table=None, **geom_kw):
        import torch

        from paper_1403_4209_amd import wgrid as wg
        self.wg, self.w = wg, w
        self.dev = torch.device("cuda:0")
        self.geom = wg.geom_from_dict(w.geom, **geom_kw)
        self.uvw = torch.as_tensor(w.uvw).to(self.dev)
        self.il = torch.as_tensor(w.inv_lambda).to(self.dev)
        self.vis, self.weight = w.vis, w.weight
        self.table = table if table is not None else wg.KernelTable(self.geom, dtype, device=self.dev)
        _, ws_bytes = wg.wg_ktable_sizes(self.geom)
        self.ws = torch.empty(ws_bytes, dtype=torch.uint8, device=self.dev)
        self.gridder = wg.Gridder(self.geom, self.table, self.uvw, self.il, self.weight)
        self.grid = torch.zeros(self.gridder.grid_shape(), dtype=torch.complex64, device=self.dev)
        self.vis_out = torch.empty(self.gridder.vis_shape(), dtype=torch.complex64, device=self.dev)
        self.ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]

    def step(self):
        """One pass of the hot path; events between phases on the current stream."""
        ev = self.ev
        ev[0].record()
        self.wg.wg_ktable_build(self.geom, self.table.kt, self.ws, host_copies=False)
        ev[1].record()
        self.gridder.compress(self.vis)
        ev[2].record()
        self.grid.zero_()
        ev[3].record()
        self.gridder.grid(out=self.grid)
        ev[4].record()
        self.gridder.degrid(self.grid, out=self.vis_out)
        ev[5].record()

    def time_steps(self, steps, warmup):
        import numpy as np
        import torch
        for _ in range(warmup):
            self.step()
        torch.cuda.synchronize()
        phase = np.zeros(5)
        t0 = time.perf_counter()
        for _ in range(steps):
            self.step()
            torch.cuda.synchronize()
            phase += [self.ev[i].elapsed_time(self.ev[i + 1]) for i in range(5)]
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return wall * 1e3 / steps, phase / steps

    def time_grid_degrid(self, steps):
        """Compress once; then grid (into a zeroed grid) and degrid, each timed on its own."""
        import torch
        self.gridder.compress(self.vis)
        for _ in range(2):
            self.grid.zero_()
            self.gridder.grid(out=self.grid)
            self.gridder.degrid(self.grid, out=self.vis_out)
        torch.cuda.synchronize()
        tg = td = 0.0
        ev = self.ev
        for _ in range(steps):
            self.grid.zero_()
            ev[0].record()
            self.gridder.grid(out=self.grid)
            ev[1].record()
            self.gridder.degrid(self.grid, out=self.vis_out)
            ev[2].record()
            torch.cuda.synchronize()
            tg += ev[0].elapsed_time(ev[1])
            td += ev[1].elapsed_time(ev[2])
        return tg / steps, td / steps


def phases_dict(ph):
    names = ("ktable", "compress", "grid_zero", "grid", "degrid")
    return {k: round(float(v), 4) for k, v in zip(names, ph)}


def rel_err(a, b):
    """Relative L2 error of a against b, and the largest element error over b's largest
    magnitude."""
    import torch
    a = a.to(torch.complex128)
    b = b.to(torch.complex128)
    return {"rel_l2": float(f"{float(torch.linalg.norm(a - b) / torch.linalg.norm(b)):.3e}"),
            "max_abs_rel": float(f"{float(torch.max(torch.abs(a - b)) / torch.max(torch.abs(b))):.3e}")}


def workload_step(cfg, steps, warmup, description):
    """A full step of another throughput workload, reported with its phases and rates."""
    import workloads
    c = Case(workloads.make(cfg, device="cuda:0"))
    ms, ph = c.time_steps(steps, warmup)
    st = c.gridder.runs.stats()
    U = st.upd_real
    out = {"workload": description, "records": int(st.n_records), "runs": int(st.n_runs), "upd_real": int(U),
           "upd_total": int(U + st.upd_saved), "ms_per_step": round(ms, 3),
           "gupds_step": round(2.0 * U / (ms * 1e-3) / 1e9, 2), "phases_ms": phases_dict(ph),
           "grid_gupds_real": round(U / (ph[3] * 1e-3) / 1e9, 2),
           "degrid_gupds": round(U / (ph[4] * 1e-3) / 1e9, 2)}
    return out, c


def cpu_baseline(w, vis_h, u_full, gpu_grid_subset, threads=8):
    """The FP64 oracle on every 16th baseline: its table build once, then compress + grid +
    degrid of the sample on 1 thread and on `threads` threads (baseline shards, each on its
    own grid; the C calls release the interpreter lock), scaled to the full step by update
    count. The single-thread grid of the sample is also the reference against which the GPU
    grids of the same sample with FP32, BF16 and FP16 tables are measured."""
    import concurrent.futures as cf

    import numpy as np

    import oracle
    oracle.build(force=False)
    t0 = time.perf_counter()
    t64 = oracle.ktable.build(w.geom, "f64")
    t_table = time.perf_counter() - t0
    sub = slice(0, None, 16)
    uvw, vis = w.uvw[sub], vis_h[sub]

    def run(u, v):
        r = oracle.compress(w.geom, t64, u, w.inv_lambda, v)
        G = oracle.grid(w.geom, t64, r)
        oracle.degrid(w.geom, t64, r, G, u, None, v.shape)
        return r, G

    t0 = time.perf_counter()
    runs, G1 = run(uvw, vis)
    t1 = time.perf_counter() - t0
    shards = np.array_split(np.arange(uvw.shape[0]), threads)
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        list(ex.map(lambda s: run(uvw[s], vis[s]), shards))
    tn = time.perf_counter() - t0
    u_s = int(runs["stats"][4])
    scale = u_full / max(u_s, 1)
    t_full_1 = t_table + t1 * scale
    t_full_n = t_table + tn * scale
    acc = {}
    if gpu_grid_subset is not None:
        import torch
        ref = torch.as_tensor(G1)
        for dt, G in gpu_grid_subset(uvw, vis).items():
            acc[dt] = rel_err(G.cpu(), ref)
    return {"value": round(2 * u_full / t_full_n / 1e9, 4), "unit": "Gupd/s", "cores": threads, "kind": "oracle",
            "sample": (f"every 16th baseline ({uvw.shape[0]} of {w.uvw.shape[0]}; {vis.size} records, {u_s} "
                       f"updates): FP64 table build {t_table:.2f} s once (numpy, 1 thread); compress + grid + degrid "
                       f"{t1:.2f} s on 1 thread, {tn:.2f} s on {threads} threads (baseline shards), scaled "
                       f"x{scale:.2f} by updates to the full step"),
            "value_1thread": round(2 * u_full / t_full_1 / 1e9, 4),
            "seconds_full_step": round(t_full_n, 2), "seconds_full_step_1thread": round(t_full_1, 2)}, acc


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); multi-GPU sharding is a design note",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    import torch

    import workloads
    from paper_1403_4209_amd import wgrid as wg

    dev = torch.device("cuda:0")
    if args.profile_workload:
        w = workloads.make(args.profile_workload, device=dev)
        c = Case(w)
        ms_step, ph = c.time_steps(args.steps, args.warmup)
        st = c.gridder.runs.stats()
        print(json.dumps({"workload": args.profile_workload, "records": int(st.n_records), "runs": int(st.n_runs),
                          "upd_real": int(st.upd_real), "ms_per_step": round(ms_step, 3),
                          "phases_ms": phases_dict(ph)}), flush=True)
        return
    w = workloads.make(3, device=dev)
    c = Case(w)
    ms_step, ph = c.time_steps(args.steps, args.warmup)
    st = c.gridder.runs.stats()
    U = st.upd_real
    t_ktable, t_comp, t_zero, t_grid, t_degrid = ph
    value = 2.0 * U / (ms_step * 1e-3) / 1e9
    counters = read_counters()
    rl_grid = roofline("k_grid (wg_grid)", U, t_grid, counters)
    rl_degrid = roofline("k_degrid (wg_degrid)", U, t_degrid, counters)
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
        "config": {"workload": ("compression workload: 44 stations (946 baselines) x 64 channels x 512 timesteps "
                                "of 1 s = 30,998,528 records, grid 4096x4096 complex64, oversampling 8, 64 w-planes, "
                                "supports 9..63, FP32 tables, compression on"),
                   "records": int(st.n_records), "runs": int(st.n_runs), "upd_real": int(U),
                   "upd_total": int(U + st.upd_saved)},
        "phases_ms": phases_dict(ph),
        "grid_gupds_real": round(U / (t_grid * 1e-3) / 1e9, 2),
        "grid_gupds_total": round((U + st.upd_saved) / (t_grid * 1e-3) / 1e9, 2),
        "degrid_gupds": round(U / (t_degrid * 1e-3) / 1e9, 2),
        "compression_ratio_records": round(st.n_griddable / max(st.n_runs, 1), 3),
        "compression_ratio_updates": round((U + st.upd_saved) / max(U, 1), 3),
        "roofline": rl_main,
        "roofline_other": rl_other,
    }

    # the one-call entry point (compress + grid, runs left in its workspace)
    ev = c.ev
    tr = 0.0
    for i in range(args.steps + 1):
        c.grid.zero_()
        ev[0].record()
        c.gridder.grid_records(c.vis, out=c.grid)
        ev[1].record()
        torch.cuda.synchronize()
        if i:
            tr += ev[0].elapsed_time(ev[1])
    out["grid_records_ms"] = round(tr / args.steps, 4)
    g32 = c.grid.clone()

    # image finaliser of the step's grid, timed on its own (not part of the gridding step)
    fin_ws = torch.empty(wg.wg_finalise_ws_bytes(c.geom), dtype=torch.uint8, device=dev)
    image = torch.empty((c.geom.n, c.geom.n), dtype=torch.float32, device=dev)
    wg.finalise(c.geom, g32, c.gridder.runs.normaliser(), out=image, ws=fin_ws)
    torch.cuda.synchronize()
    t_fin = 0.0
    for _ in range(args.steps):
        ev[0].record()
        wg.finalise(c.geom, g32, c.gridder.runs.normaliser(), out=image, ws=fin_ws)
        ev[1].record()
        torch.cuda.synchronize()
        t_fin += ev[0].elapsed_time(ev[1])
    out["finalise_ms"] = round(t_fin / args.steps, 4)
    del fin_ws, image

    precision = None
    extra_tables = {}
    if not args.no_variants:
        # BF16 and FP16 tables on the same records: grid and degrid times, and the full grid
        # against the FP32-table grid; their errors against the FP64 oracle come from the
        # CPU-baseline leg
        precision = {"f32": {"grid_ms": round(t_grid, 4), "degrid_ms": round(t_degrid, 4)}}
        for dt in ("bf16", "f16"):
            cd = Case(w, dt)
            tg, td = cd.time_grid_degrid(args.steps)
            # the whole step with this table type: its own table build, the FP32 step's
            # compression and grid clearing (which do not depend on the table type)
            tk = 0.0
            for i in range(args.steps + 1):
                cd.ev[0].record()
                wg.wg_ktable_build(cd.geom, cd.table.kt, cd.ws, host_copies=False)
                cd.ev[1].record()
                torch.cuda.synchronize()
                if i:
                    tk += cd.ev[0].elapsed_time(cd.ev[1])
            tk /= args.steps
            step = tk + t_comp + t_zero + tg + td
            precision[dt] = {"grid_ms": round(tg, 4), "degrid_ms": round(td, 4),
                             "grid_gupds_real": round(U / (tg * 1e-3) / 1e9, 2),
                             "speedup_grid_vs_f32": round(t_grid / tg, 3),
                             "speedup_degrid_vs_f32": round(t_degrid / td, 3),
                             "ktable_ms": round(tk, 4), "step_ms": round(step, 4),
                             "speedup_step_vs_f32": round(ms_step / step, 3),
                             "full_grid_vs_f32_table_grid": rel_err(cd.grid, g32)}
            extra_tables[dt] = cd.table
            del cd
        # the thesis's plain FP32 sums per owned cell (WG_PLAIN_SUMS) with the FP32 table
        cp = Case(w, table=c.table, plain_sums=True)
        tg, td = cp.time_grid_degrid(args.steps)
        precision["f32_plain_sums"] = {"grid_ms": round(tg, 4), "degrid_ms": round(td, 4),
                                       "grid_gupds_real": round(U / (tg * 1e-3) / 1e9, 2),
                                       "speedup_grid_vs_f32": round(t_grid / tg, 3),
                                       "full_grid_vs_f32_table_grid": rel_err(cp.grid, g32)}
        extra_tables["f32_plain_sums"] = c.table
        del cp
        out["precision"] = precision

        # compression off: every griddable record is its own run
        cu = Case(w, table=c.table, compress=False)
        tcu = tgu = 0.0
        for i in range(args.steps + 1):
            cu.grid.zero_()
            ev[0].record()
            cu.gridder.compress(cu.vis)
            ev[1].record()
            cu.gridder.grid(out=cu.grid)
            ev[2].record()
            torch.cuda.synchronize()
            if i:
                tcu += ev[0].elapsed_time(ev[1])
                tgu += ev[1].elapsed_time(ev[2])
        tcu /= args.steps
        tgu /= args.steps
        out["uncompressed"] = {"compress_ms": round(tcu, 4), "grid_ms": round(tgu, 4),
                               "speedup_of_compression": round((tcu + tgu) / (t_comp + t_grid), 3),
                               "grid_vs_compressed_grid": rel_err(cu.grid, g32)}
        del cu

        # table-generation study: the FP32 table of this geometry with more w-planes, up to
        # the thesis's 200 (build timed alone, host copies off as in the step)
        study = {}
        for n_w in (32, 64, 128, 200):
            gs = wg.geom_from_dict(dict(w.geom, n_w=n_w))
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

    vis_h = c.vis.cpu().numpy() if not args.no_cpu_baseline else None
    del c

    if not args.no_variants:
        # the other throughput workloads as full steps
        out["plain_fp32_2048"], c2 = workload_step(
            2, args.steps, args.warmup, "plain FP32 gridding: 946 baselines x 16 channels x 512 timesteps = 7,749,632 "
            "records, 2048x2048, 32 w-planes, supports 9..63")
        w2 = c2.w
        t_grid2 = out["plain_fp32_2048"]["phases_ms"]["grid"]
        # w-stacking (eq. stacking) of those records: every record gridded with the w = 0
        # kernel on the grid of its w-plane (32 grids of 2048^2), then the planes transformed,
        # w-corrected and added; against w-projection's compress + grid + finalise
        cs = Case(w2, table=c2.table, w_stacking=True)
        img_s = torch.empty((cs.geom.n, cs.geom.n), dtype=torch.float32, device=dev)
        tcs = tgs = tfs = 0.0
        for i in range(args.steps + 1):
            cs.grid.zero_()
            ev[0].record()
            cs.gridder.compress(cs.vis)
            ev[1].record()
            cs.gridder.grid(out=cs.grid)
            ev[2].record()
            cs.gridder.finalise(cs.grid, out=img_s)
            ev[3].record()
            torch.cuda.synchronize()
            if i:
                tcs += ev[0].elapsed_time(ev[1])
                tgs += ev[1].elapsed_time(ev[2])
                tfs += ev[2].elapsed_time(ev[3])
        tcs, tgs, tfs = tcs / args.steps, tgs / args.steps, tfs / args.steps
        ss = cs.gridder.runs.stats()
        img_w = torch.empty_like(img_s)
        tfw = 0.0
        for i in range(args.steps + 1):
            ev[0].record()
            c2.gridder.finalise(c2.grid, out=img_w)
            ev[1].record()
            torch.cuda.synchronize()
            if i:
                tfw += ev[0].elapsed_time(ev[1])
        tfw /= args.steps
        ph2 = out["plain_fp32_2048"]["phases_ms"]
        out["w_stacking"] = {"workload": "the plain FP32 workload's records", "grids": int(cs.geom.n_w),
                             "compress_ms": round(tcs, 4), "grid_ms": round(tgs, 4),
                             "finalise_stacked_ms": round(tfs, 4), "upd_real": int(ss.upd_real),
                             "grid_gupds_real": round(ss.upd_real / (tgs * 1e-3) / 1e9, 2),
                             "image_ms": round(tcs + tgs + tfs, 4),
                             "w_projection_image_ms": round(ph2["compress"] + ph2["grid"] + tfw, 4)}
        del cs, img_s, img_w

        # polarisations (the thesis's experiment batch 4): the same records as 4 and 2
        # products (seeded polarised sources, per-product weights and flags)
        pol = {}
        wp = workloads.polarised(2, 4, device=dev)
        for npol in (4, 2):
            vp = wp.vis if npol == 4 else wp.vis[..., [0, 3]].contiguous()
            wtp = wp.weight if npol == 4 else wp.weight[..., [0, 3]].contiguous()
            flp = wp.flag if npol == 4 else wp.flag[..., [0, 3]].contiguous()
            gp_ = wg.geom_from_dict(w2.geom, n_pol=npol)
            gpp = wg.Gridder(gp_, c2.table, c2.uvw, c2.il, wtp, flp)
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
                              "grid_record_rate_vs_1pol": round(t_grid2 / tgp, 3)}
            del gpp, gridp, voutp
        pol["1"] = {"grid_ms": t_grid2, "degrid_ms": ph2["degrid"],
                    "grid_gupds_products": out["plain_fp32_2048"]["grid_gupds_real"]}
        out["polarisations"] = {"workload": "the plain FP32 workload's records", **pol}
        del wp, c2, w2

        # heavy w-projection: the thesis's batch-5 imaging configuration 2 (4500^2, 16
        # w-planes, oversampling 4, supports up to 349) on four-product records
        wh = workloads.polarised(6, 4, device=dev)
        gh = wg.geom_from_dict(wh.geom, n_pol=4)
        ev[0].record()
        th = wg.KernelTable(gh, "f32", device=dev)
        ev[1].record()
        torch.cuda.synchronize()
        t_kt = ev[0].elapsed_time(ev[1])
        grh = wg.Gridder(gh, th, torch.as_tensor(wh.uvw).to(dev), torch.as_tensor(wh.inv_lambda).to(dev),
                         wh.weight, wh.flag)
        gridh = torch.zeros(grh.grid_shape(), dtype=torch.complex64, device=dev)
        vouth = torch.empty(grh.vis_shape(), dtype=torch.complex64, device=dev)
        tch = tgh = tdh = 0.0
        nh = 2
        for i in range(nh + 1):
            gridh.zero_()
            ev[0].record()
            grh.compress(wh.vis)
            ev[1].record()
            grh.grid(out=gridh)
            ev[2].record()
            grh.degrid(gridh, out=vouth)
            ev[3].record()
            torch.cuda.synchronize()
            if i:
                tch += ev[0].elapsed_time(ev[1])
                tgh += ev[1].elapsed_time(ev[2])
                tdh += ev[2].elapsed_time(ev[3])
        tch, tgh, tdh = tch / nh, tgh / nh, tdh / nh
        sh = grh.runs.stats()
        out["heavy_4500"] = {
            "workload": ("heavy w-projection: 44 stations (946 baselines) x 1 channel x 1024 timesteps of 10 s = "
                         f"{int(sh.n_records):,} records x 4 polarisation products, grid 4500x4500 complex64 per "
                         "product, oversampling 4, 16 w-planes, supports 9..349, FP32 tables"),
            "runs": int(sh.n_runs), "supports": [int(v) for v in th.support],
            "upd_real_per_product": int(sh.upd_real),
            "ktable_ms": round(t_kt, 3), "compress_ms": round(tch, 4), "grid_ms": round(tgh, 4),
            "degrid_ms": round(tdh, 4),
            "grid_gupds_products": round(sh.upd_real * 4 / (tgh * 1e-3) / 1e9, 2),
            "degrid_gupds_products": round(sh.upd_real * 4 / (tdh * 1e-3) / 1e9, 2)}
        del wh, th, grh, gridh, vouth
        torch.cuda.empty_cache()

        out["differentiation_4096"], c5 = workload_step(
            5, args.steps, args.warmup, "differentiation workload: 256 stations (32,640 baselines) x 8 channels x "
            "256 timesteps = 66,846,720 records, 4096x4096, 32 w-planes, supports 7..31")
        del c5

    if not args.no_cpu_baseline:
        tables = {"f32": None, **extra_tables}

        def gpu_grid_subset(uvw_s, vis_s):
            """The sample's grid on the GPU with each table type (the full workload's tables)."""
            grids = {}
            base = wg.geom_from_dict(w.geom)
            f32 = wg.KernelTable(base, "f32", device=dev) if tables["f32"] is None else tables["f32"]
            for dt in tables:
                tb = f32 if dt == "f32" else tables[dt]
                g = wg.Gridder(wg.geom_from_dict(w.geom, plain_sums=dt == "f32_plain_sums"), tb,
                               torch.as_tensor(uvw_s).to(dev), torch.as_tensor(w.inv_lambda).to(dev))
                grids[dt] = g.grid_records(torch.as_tensor(vis_s).to(dev))
            torch.cuda.synchronize()
            return grids

        out["cpu_baseline"], acc = cpu_baseline(w, vis_h, U, gpu_grid_subset)
        if precision is not None:
            for dt, e in acc.items():
                precision.setdefault(dt, {})["sample_grid_vs_fp64_oracle"] = e
            precision["sample"] = "every 16th baseline of the workload, gridded by the FP64 oracle on its FP64 table"
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
