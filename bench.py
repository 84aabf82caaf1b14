"""Benchmark of the DEAM hot path on one MI355X.

One step = one DEAM iteration (forward projection + polyenergetic mean with
metal-trace substitution, 4-channel backprojection, FP64 update and the FP64
I-divergence reduction) over the whole synthetic scan, with every input
resident in HBM.  Prints one JSON line.

Default workload: the 2D fan-beam case (512 x 512 at 0.98 mm, 984 views x 816
channels, 90/140 kVp spectra on 1-keV bins from 20 to 140 keV, pelvis-like
phantom with two steel implants, I0 = 2e5).  `--workload helical` runs the
3D helical case (512 x 512 x 64, 16 x 816 detector, 4608 views).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_LANE_OPS = 256 * 64 * 2.4e9     # 256 CUs x 64 lanes x 2.4 GHz, one VALU op per lane-cycle
PEAK_HBM = 8.0e12                     # bytes/s

WORKLOAD_DESC = {
    "fan512": "2D fan-beam 512x512 at 0.98 mm, 984 views x 816 channels (360 deg), sid 570 / sdd 1040 mm, "
              "121 energy bins 20-140 keV, 90/140 kVp, pelvis-like phantom with two steel ellipses, I0=2e5",
    "helical": "3D helical cone-beam 512x512x64 at 0.98x0.98x1 mm, 16 rows x 816 channels, 1152 views/rot x 4 rot, "
               "pitch 0.5, 121 energy bins, spine-like phantom with 4 titanium screws, I0=2e5",
    "fan256": "2D fan-beam 256x256 at 1 mm, 360 views x 512 channels",
    "fan128": "2D fan-beam 128x128 at 1 mm, 180 views x 256 channels",
}


def segment_count(geom, chunk_views=64):
    """Number of non-zero h(x,y) (Siddon segments) over all rays: for each ray,
    1 + the number of grid planes it crosses strictly inside the grid."""
    from workloads.geometry import ray_endpoints
    is3d = geom.kind == 1
    n = np.array([geom.nx, geom.ny, geom.nz if is3d else 1], float)
    dl = np.array([geom.dx, geom.dy, geom.dz])
    org = -0.5 * n * dl
    total = 0
    for v0 in range(0, geom.n_views, chunk_views):
        S, P = ray_endpoints(geom, np.arange(v0, min(v0 + chunk_views, geom.n_views)))
        if not is3d:
            S[:, 2] = 0.0
            P[:, 2] = 0.0
        u0 = (S - org) / dl
        du = (P - S) / dl
        lo = np.zeros(len(S))
        hi = np.ones(len(S))
        for a in range(3 if is3d else 2):
            with np.errstate(divide="ignore", invalid="ignore"):
                t0 = (0.0 - u0[:, a]) / du[:, a]
                t1 = (n[a] - u0[:, a]) / du[:, a]
            par = du[:, a] == 0
            inside = (u0[:, a] >= 0) & (u0[:, a] < n[a])
            lo = np.where(par, np.where(inside, lo, 2.0), np.maximum(lo, np.minimum(t0, t1)))
            hi = np.where(par, np.where(inside, hi, -1.0), np.minimum(hi, np.maximum(t0, t1)))
        hit = hi > lo
        cnt = np.where(hit, 1.0, 0.0)
        for a in range(3 if is3d else 2):
            ua = u0[:, a] + lo * du[:, a]
            ub = u0[:, a] + hi * du[:, a]
            a0, a1 = np.minimum(ua, ub), np.maximum(ua, ub)
            # interior planes i (1..n-1) with a0 < i < a1
            c = np.clip(np.ceil(a1) - 1, 0, n[a] - 1) - np.clip(np.floor(a0) + 1, 1, n[a]) + 1
            cnt += np.where(hit, np.maximum(c, 0), 0)
        total += int(cnt.sum())
    return total


def read_traffic(kernel, workload):
    """HBM bytes per launch from a committed rocprofv3 PMC summary (or None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_pmc.txt")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("traffic_bytes_per_launch:"):
            try:
                return float(line.split(":", 1)[1])
            except ValueError:
                return None
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="fan512", choices=sorted(WORKLOAD_DESC))
    ap.add_argument("--fp64-steps", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=8)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy three times (reference for the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (the DEAM path is measured on one MI355X); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    from workloads import make_inputs
    from paper_2202_00116_amd.plan import Plan

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.calibrate_copy:
        n = 1 << 28                       # 2^28 float32 = 1 GiB read and 1 GiB written
        x = torch.ones(n, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}))
        return
    K, W = args.steps, args.warmup
    t_in = time.perf_counter()
    inp = make_inputs(args.workload)
    g = inp["geom"]
    t_in = time.perf_counter() - t_in
    print(f"[bench] inputs {args.workload}: R={g.n_rays} V={g.n_voxels} ({t_in:.1f} s)", file=sys.stderr, flush=True)

    d = torch.from_numpy(inp["d"]).to(dev)
    M = torch.from_numpy(inp["metal"]).to(dev)
    c0 = torch.from_numpy(inp["c0"]).to(dev)
    Z = inp["Z"]
    plan = Plan(g, inp["I0"], inp["mu"], "mixed")
    mask = plan.metal_trace(M, inp["t"])
    torch.cuda.synchronize()

    # --- mixed precision: whole-step throughput ------------------------------
    c = c0.clone()
    hist = torch.zeros(max(K, 1), dtype=torch.float64, device=dev)
    plan.iterate(c, d, mask, Z, W)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.iterate(c, d, mask, Z, K, hist)
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / K
    print(f"[bench] mixed: {t_step * 1e3:.3f} ms/step", file=sys.stderr, flush=True)

    # --- per-kernel device times (HIP events on the launch stream) -------------
    ck = c0.clone()
    plan.iterate(ck, d, mask, Z, 1)
    kms = plan.iterate_timed(ck, d, mask, Z, K)
    t_fp_poly = kms["fp_poly"] / K
    t_bp = kms["backproject"] / K
    t_upd = kms["update"] / K
    # forward projection alone (2 channels), events on torch's current stream
    cf = c0.to(torch.float32)
    plan.forward(cf)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(K):
        plan.forward(cf)
    e1.record()
    torch.cuda.synchronize()
    t_fp2 = e0.elapsed_time(e1) / K
    grays = g.n_rays / ((t_fp2 + t_bp) * 1e-3) / 1e9

    # --- all-FP64 variant --------------------------------------------------
    K64 = args.fp64_steps if args.fp64_steps is not None else max(2, K // 4)
    plan64 = Plan(g, inp["I0"], inp["mu"], "fp64")
    c64 = c0.clone()
    plan64.iterate(c64, d, mask, Z, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan64.iterate(c64, d, mask, Z, K64)
    torch.cuda.synchronize()
    t_step64 = (time.perf_counter() - t0) / K64
    print(f"[bench] fp64: {t_step64 * 1e3:.3f} ms/step", file=sys.stderr, flush=True)

    # --- roofline of the dominant kernel ----------------------------------------
    S = segment_count(g)
    nE = int((inp["I0"].sum(axis=0) > 0).sum())
    ops = {
        "fp_poly": 8.0 * S + (11.0 * nE + 40.0) * g.n_rays,
        "backproject": 10.0 * S,
    }
    times = {"fp_poly": t_fp_poly, "backproject": t_bp}
    dom = max(times, key=times.get)
    achieved = ops[dom] / (times[dom] * 1e-3)
    traffic = read_traffic(dom, args.workload)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                "unit": "Tops/s", "frac": achieved / PEAK_LANE_OPS, "traffic": traffic,
                "kernel": dom, "ops_per_launch": ops[dom], "segments": S,
                "avg_launch_ms": times[dom]}

    out = {
        "metric": "DEAM iterations/s + Grays/s (fwd+back), FP32 vs FP64 GPU at stated error",
        "value": 1.0 / t_step,
        "unit": "iterations/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOAD_DESC[args.workload]}",
                   "precision": "mixed: f32 projection/energy sums/weights, fixed-point backprojection, "
                                "f64 objective and update",
                   "rays": g.n_rays, "voxels": g.n_voxels, "energy_bins": nE,
                   "metal_rays": int(mask.sum().item())},
        "grays_per_s": grays,
        "kernel_ms": {"fp_poly": t_fp_poly, "backproject": t_bp, "update": t_upd,
                      "forward_2ch": t_fp2},
        "fp64": {"iterations_per_s": 1.0 / t_step64, "ms_per_step": t_step64 * 1e3, "steps": K64},
        "speedup_mixed_vs_fp64": t_step64 / t_step,
        "roofline": roofline,
        "cpu_baseline": None,
    }

    # --- CPU baseline (the FP64 oracle) ---------------------------------------------
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        n_it = args.cpu_iters
        mask_np = mask.cpu().numpy()
        t0 = time.perf_counter()
        c_o, h_o = O.iterate(g, inp["I0"], inp["mu"], inp["d"], mask_np, Z, inp["c0"], n_it)
        t_cpu = time.perf_counter() - t0
        cg = c0.clone()
        hg = torch.zeros(n_it, dtype=torch.float64, device=dev)
        plan.iterate(cg, d, mask, Z, n_it, hg)
        cg = cg.cpu().numpy()
        err = float(np.linalg.norm(cg - c_o) / np.linalg.norm(c_o))
        herr = float(np.abs(hg.cpu().numpy() - h_o).max() / abs(h_o[0]))
        out["cpu_baseline"] = {"value": n_it / t_cpu, "unit": "iterations/s",
                               "cores": O.num_threads(), "kind": "oracle",
                               "sample": f"{n_it} full FP64 oracle DEAM iterations of the {args.workload} "
                                         f"workload from the cold start ({t_cpu:.1f} s)"}
        out["error_vs_oracle"] = {"iterations": n_it, "image_rel_l2": err, "objective_rel": herr}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
