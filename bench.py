"""Benchmark of the DEAM hot path on one MI355X.

One step = one DEAM iteration (forward projection + polyenergetic mean with
metal-trace substitution, 4-channel backprojection, FP64 update and the FP64
I-divergence reduction) over the whole synthetic scan, with every input
resident in HBM.  Prints one JSON line.

Default workload: the 3D helical cone-beam case (512 x 512 x 64 at
0.98 x 0.98 x 1 mm, 16 rows x 816 channels, 1152 views per turn over four
turns at pitch 0.5, 90/140 kVp spectra on 1-keV bins from 20 to 140 keV,
spine-like phantom with four titanium screws, I0 = 2e5).  The 2D fan-beam
case (512 x 512, 984 views x 816 channels) and the unrolled reconstruction
are measured as secondary blocks.  `--workload fan512` makes the fan-beam
case the headline.
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


def iteration_model(g, S, nE):
    """Whole-iteration roofline of the op and byte model: VALU lane-ops
    (forward 8/segment, energy sums 11/bin/ray + 40/ray, backprojection
    10/segment, update 32 per voxel-component) and algorithmic HBM bytes
    (41 B per ray, 96 B per voxel)."""
    ops = 8.0 * S + (11.0 * nE + 40.0) * g.n_rays + 10.0 * S + 64.0 * g.n_voxels
    byt = 41.0 * g.n_rays + 96.0 * g.n_voxels
    return ops, byt


def copy_bandwidth(dev, reps=3):
    """HBM bytes per second of a plain 1 GiB device-to-device copy (read plus
    write), the practical ceiling of a streaming kernel; also the reference of
    the FETCH_SIZE / WRITE_SIZE counter calibration."""
    import torch
    n = 1 << 28                       # 2^28 float32 = 1 GiB read and 1 GiB written
    x = torch.ones(n, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    bw = 2 * 4 * n * reps / (e0.elapsed_time(e1) * 1e-3)
    del x, y
    torch.cuda.empty_cache()
    return bw, reps + 1


def measure(workload, K, W, K64, dev, log, extras=True):
    """Mixed-precision step time, per-kernel times, the all-FP64 step time and
    the roofline figures of one workload (inputs resident in HBM); with
    extras, also the penalised iteration, the MAR initialisation and the model
    variants (which launch the same kernels at other sizes)."""
    import torch
    from workloads import make_inputs, PENALTY
    from paper_2202_00116_amd.plan import Plan

    t_in = time.perf_counter()
    inp = make_inputs(workload)
    g = inp["geom"]
    log(f"inputs {workload}: R={g.n_rays} V={g.n_voxels} ({time.perf_counter() - t_in:.1f} s)")
    d = torch.from_numpy(inp["d"]).to(dev)
    M = torch.from_numpy(inp["metal"]).to(dev)
    c0 = torch.from_numpy(inp["c0"]).to(dev)
    Z = inp["Z"]
    plan = Plan(g, inp["I0"], inp["mu"], "mixed")
    mask = plan.metal_trace(M, inp["t"])
    torch.cuda.synchronize()

    # whole-step throughput
    c = c0.clone()
    hist = torch.zeros(max(K, 1), dtype=torch.float64, device=dev)
    plan.iterate(c, d, mask, Z, W)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.iterate(c, d, mask, Z, K, hist)
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / K
    log(f"mixed: {t_step * 1e3:.3f} ms/step")

    # per-kernel device times (HIP events on the launch stream)
    ck = c0.clone()
    plan.iterate(ck, d, mask, Z, 1)
    kms = plan.iterate_timed(ck, d, mask, Z, K)
    t_fp_poly, t_bp, t_upd = kms["fp_poly"] / K, kms["backproject"] / K, kms["update"] / K
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
    # one channel each way (single-image projectors)
    c1 = cf[:1].contiguous()
    w1 = plan.forward(c1)
    plan.backproject(w1)
    e0.record()
    for _ in range(K):
        plan.forward(c1)
    e1.record()
    torch.cuda.synchronize()
    t_fp1 = e0.elapsed_time(e1) / K
    e0.record()
    for _ in range(K):
        plan.backproject(w1)
    e1.record()
    torch.cuda.synchronize()
    t_bp1 = e0.elapsed_time(e1) / K
    grays1 = g.n_rays / ((t_fp1 + t_bp1) * 1e-3) / 1e9
    del c1, w1

    # all-FP64 variant
    plan64 = Plan(g, inp["I0"], inp["mu"], "fp64")
    c64 = c0.clone()
    plan64.iterate(c64, d, mask, Z, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan64.iterate(c64, d, mask, Z, K64)
    torch.cuda.synchronize()
    t_step64 = (time.perf_counter() - t0) / K64
    log(f"fp64: {t_step64 * 1e3:.3f} ms/step")

    # penalised iteration (Eqs. 6-7) with the workload's (lambda, delta): whole
    # step, and the penalised update kernel alone on realistic backprojections
    penalized = None
    if extras:
        lam, delta = PENALTY[workload]
        cpn = c0.clone()
        plan.iterate_penalized(cpn, d, mask, Z, lam, delta, 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.iterate_penalized(cpn, d, mask, Z, lam, delta, K)
        torch.cuda.synchronize()
        t_pen = (time.perf_counter() - t0) / K
        wb, _, _ = plan.poly_mean(plan.forward(cpn.to(plan.dtype)), d, mask)
        bb = plan.backproject(wb)
        del wb
        plan.update_penalized(cpn, bb, Z, lam, delta)
        e0.record()
        for _ in range(K):
            plan.update_penalized(cpn, bb, Z, lam, delta)
        e1.record()
        torch.cuda.synchronize()
        t_upd_pen = e0.elapsed_time(e1) / K
        del bb
        log(f"penalized: {t_pen * 1e3:.3f} ms/step, update kernel {t_upd_pen:.3f} ms")
        penalized = {"lambda": lam, "delta": delta, "ms_per_step": t_pen * 1e3,
                     "iterations_per_s": 1.0 / t_pen, "steps": K, "update_pen_ms": t_upd_pen,
                     "update_ms": t_upd}

    # MAR initialisation (2D fan-beam full scans): the whole pipeline and one
    # two-channel FBP, events on torch's current stream
    mar = None
    if extras and g.kind == 0:
        from workloads import mar_params
        prm = mar_params(g, inp["I0"])
        plan.mar_init(d, prm)
        pli = torch.zeros((2, g.n_rays), dtype=plan.dtype, device=dev)
        plan.fbp(pli)
        e0.record()
        for _ in range(K):
            plan.mar_init(d, prm)
        e1.record()
        torch.cuda.synchronize()
        t_mar = e0.elapsed_time(e1) / K
        e0.record()
        for _ in range(K):
            plan.fbp(pli)
        e1.record()
        torch.cuda.synchronize()
        t_fbp = e0.elapsed_time(e1) / K
        del pli
        log(f"mar_init: {t_mar:.3f} ms, fbp (2 channels) {t_fbp:.3f} ms")
        mar = {"mar_init_ms": t_mar, "fbp_2ch_ms": t_fbp,
               "pipeline": "line integrals, FBP, metal/prior images, metal trace, prior projection, "
                           "NMAR, FBP, Eq. 4 decomposition"}

    # model variants on this workload: ordered subsets (time per epoch and the
    # objective after 4 epochs against 4 iterations), two scans (each with its
    # own plan and trace), and a bowtie filter
    variants = None
    if extras and g.kind == 0:
        from paper_2202_00116_amd.plan import iterate_dual
        from workloads import bowtie
        n_sub, n_ep = 8, 4
        h_os = torch.zeros(n_ep + 1, dtype=torch.float64, device=dev)
        h_it = torch.zeros(n_ep + 1, dtype=torch.float64, device=dev)
        c_os, c_it = c0.clone(), c0.clone()
        plan.iterate_os(c_os, d, mask, Z, n_sub, n_ep + 1, h_os)
        plan.iterate(c_it, d, mask, Z, n_ep + 1, h_it)
        c_os = c0.clone()
        plan.iterate_os(c_os, d, mask, Z, n_sub, 1)
        e0.record()
        plan.iterate_os(c_os, d, mask, Z, n_sub, K)
        e1.record()
        torch.cuda.synchronize()
        t_ep = e0.elapsed_time(e1) / K
        I0 = inp["I0"]
        lo, hi = np.zeros_like(I0), np.zeros_like(I0)
        lo[0], hi[1] = I0[0], I0[1]
        plo, phi = Plan(g, lo, inp["mu"], "mixed"), Plan(g, hi, inp["mu"], "mixed")
        cd = c0.clone()
        iterate_dual(plo, phi, cd, d, mask, d, mask, Z, 1)
        e0.record()
        iterate_dual(plo, phi, cd, d, mask, d, mask, Z, K)
        e1.record()
        torch.cuda.synchronize()
        t_dual = e0.elapsed_time(e1) / K
        del plo, phi
        plan.set_bowtie(bowtie(g))
        cb = c0.clone()
        plan.iterate(cb, d, mask, Z, 1)
        e0.record()
        plan.iterate(cb, d, mask, Z, K)
        e1.record()
        torch.cuda.synchronize()
        t_bt = e0.elapsed_time(e1) / K
        plan.set_bowtie(None)
        ho, hi_ = h_os.cpu().numpy(), h_it.cpu().numpy()
        log(f"variants: OS-{n_sub} epoch {t_ep:.3f} ms, two scans {t_dual:.3f} ms/it, "
            f"bowtie {t_bt:.3f} ms/it")
        variants = {"ordered_subsets": {"n_sub": n_sub, "ms_per_epoch": t_ep,
                                        "objective_after_4": float(ho[n_ep]),
                                        "objective_after_4_iterations_plain": float(hi_[n_ep]),
                                        "objective_start": float(ho[0])},
                    "two_scans_ms_per_iteration": t_dual,
                    "bowtie_ms_per_iteration": t_bt}

    # roofline of the dominant kernel, and of the whole iteration
    S = segment_count(g)
    nE = int((inp["I0"].sum(axis=0) > 0).sum())
    ops = {"fp_poly": 8.0 * S + (11.0 * nE + 40.0) * g.n_rays, "backproject": 10.0 * S}
    times = {"fp_poly": t_fp_poly, "backproject": t_bp}
    dom = max(times, key=times.get)
    achieved = ops[dom] / (times[dom] * 1e-3)
    traffic = read_traffic(dom, workload)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                "unit": "Tops/s", "frac": achieved / PEAK_LANE_OPS,
                "traffic": traffic, "kernel": dom, "ops_per_launch": ops[dom],
                "segments": S, "avg_launch_ms": times[dom],
                "frac_kind": "algorithmic lane-ops of one launch (forward + energy sums: 8 per "
                             "Siddon segment + 11 per ray and energy bin + 40 per ray; "
                             "backprojection: 10 per segment) / its HIP-event time / the VALU "
                             "lane peak (256 CU x 64 lanes x 2.4 GHz); not issued instructions",
                "traffic_source": None if traffic is None else
                f"profiles/{dom}_{workload}_pmc.txt: rocprofv3 FETCH_SIZE + WRITE_SIZE per "
                f"dispatch scaled by a 1 GiB copy's counts, read from the committed summary",
                "traffic_GBps": None if traffic is None else traffic / (times[dom] * 1e-3) / 1e9}
    it_ops, it_bytes = iteration_model(g, S, nE)
    t_valu, t_hbm = it_ops / PEAK_LANE_OPS, it_bytes / PEAK_HBM
    iteration = {"valu_model_ms": t_valu * 1e3, "hbm_model_ms": t_hbm * 1e3,
                 "binding": "alu" if t_valu >= t_hbm else "hbm",
                 "frac_of_binding_roofline": max(t_valu, t_hbm) / t_step,
                 "hbm_frac": it_bytes / t_step / PEAK_HBM}
    return dict(inp=inp, plan=plan, d=d, mask=mask, c0=c0, t_step=t_step, grays=grays,
                grays_1ch=grays1,
                kernel_ms={"fp_poly": t_fp_poly, "backproject": t_bp, "update": t_upd,
                           "forward_2ch": t_fp2, "forward_1ch": t_fp1, "backproject_1ch": t_bp1},
                fp64={"iterations_per_s": 1.0 / t_step64, "ms_per_step": t_step64 * 1e3,
                      "steps": K64},
                speedup=t_step64 / t_step, roofline=roofline, iteration=iteration,
                penalized=penalized, mar_init=mar, variants=variants)


def measure_unrolled(dev, log, batch=8, n_iter=10, reps=3):
    """Differentiable unrolled DEAM: a batch of seeded phantoms on the 256 x 256
    fan-beam geometry, n_iter iterations forward and the backward pass to an
    L2 loss on the non-metal voxels (gradient w.r.t. the starting image)."""
    import torch
    from workloads import unrolled_inputs
    from paper_2202_00116_amd.plan import Plan
    from paper_2202_00116_amd.autograd import unrolled_deam

    t_in = time.perf_counter()
    cases = [unrolled_inputs(50 + s) for s in range(batch)]
    log(f"inputs unrolled: {batch} cases ({time.perf_counter() - t_in:.1f} s)")
    g = cases[0]["geom"]
    plan = Plan(g, cases[0]["I0"], cases[0]["mu"], "mixed")
    data = []
    for cs in cases:
        d = torch.from_numpy(cs["d"]).to(dev)
        mask = plan.metal_trace(torch.from_numpy(cs["metal"]).to(dev), cs["t"])
        data.append((d, mask, torch.from_numpy(cs["c0"]).to(dev),
                     torch.from_numpy(cs["keep"]).to(dev), torch.from_numpy(cs["c_true"]).to(dev),
                     cs["Z"]))

    def run():
        total = 0.0
        for d, mask, c0, keep, ct, Z in data:
            x = c0.clone().requires_grad_(True)
            cn = unrolled_deam(x, plan, d, mask, Z, n_iter)
            loss = (keep * (cn - ct) ** 2).sum()
            loss.backward()
            total += float(loss.detach())
        return total

    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        run()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    log(f"unrolled: {t * 1e3:.2f} ms per batch (forward + backward)")
    return {"workload": f"batch of {batch} seeded phantoms (water disk, two bone disks, 1-3 Ti/steel rods), "
                        f"fan-beam 256x256 at 1 mm, {g.n_views} views x {g.n_cols} channels, "
                        f"{n_iter} unrolled DEAM iterations forward + backward to an L2 loss on the "
                        f"non-metal voxels",
            "ms_per_batch": t * 1e3, "cases_per_s": batch / t,
            "iterations_per_s": batch * n_iter / t}


def view_block(g, n):
    """The middle n views of a scan as a scan of their own: the same rays
    (the helix is centred on the scan's middle view, so a centred block keeps
    every source position); returns (geometry, first view)."""
    import dataclasses
    v0 = (g.n_views - n) // 2
    if (g.n_views - n) % 2:
        n += 1
    beta0 = g.beta0 + 2.0 * math.pi * v0 / g.views_per_rot
    return dataclasses.replace(g, n_views=n, beta0=beta0), v0


def oracle_sample(g, inp, mask_np, n_views, plan_cls, dev, one_core_views=None):
    """The FP64 oracle on a bounded sample of the workload: one DEAM iteration
    over the middle n_views views (forward, poly-mean and backprojection of
    those rays, update of the whole image) on all host cores, scaled to the
    whole scan by its ray count (the update is timed on its own and counted
    once).  The GPU (mixed precision) runs the same iteration on the same
    inputs, and the two images and objectives are compared over the whole
    volume.  Optionally a smaller sample on one core."""
    import torch
    from oracle import oracle as O
    gs, v0 = view_block(g, n_views)
    per_view = g.n_rows * g.n_cols
    sl = slice(v0 * per_view, (v0 + gs.n_views) * per_view)
    d_s = np.ascontiguousarray(inp["d"][:, sl])
    m_s = np.ascontiguousarray(mask_np[sl])
    Z = inp["Z"]
    t0 = time.perf_counter()
    c_o, h_o, b_o = O.iterate(gs, inp["I0"], inp["mu"], d_s, m_s, Z, inp["c0"], 1, want_b=True)
    t_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.update(b_o, Z, inp["c0"])
    t_u = time.perf_counter() - t0
    scale = g.n_views / gs.n_views
    t_full = scale * max(t_s - t_u, 0.0) + t_u
    # the GPU on the same sample
    plan = plan_cls(gs, inp["I0"], inp["mu"], "mixed")
    c = torch.from_numpy(inp["c0"]).to(dev)
    hist = torch.zeros(1, dtype=torch.float64, device=dev)
    plan.iterate(c, torch.from_numpy(d_s).to(dev), torch.from_numpy(m_s).to(dev), Z, 1, hist)
    c = c.cpu().numpy()
    del plan
    bh = b_o[2:]
    lev = (bh / bh.max(axis=1, keepdims=True)).min(axis=0)   # b^ relative to its maximum
    res = lev >= 1e-6
    e = np.abs(c - c_o)
    cmax = np.abs(c_o).max()
    well = lev >= 1e-4
    err = {"sample": f"one DEAM iteration over views {v0}-{v0 + gs.n_views - 1} of the scan "
                     f"({gs.n_rays} rays, the whole image), mixed precision against the FP64 oracle",
           "resolved": "voxels whose oracle b^ (both components) is at least 1e-6 of its "
                       "maximum; the others are seen by no ray of the sample or only by the "
                       "ends of a few chords",
           "image_rel_l2": float(np.linalg.norm(c[:, res] - c_o[:, res])
                                 / np.linalg.norm(c_o[:, res])),
           "image_max_abs_rel": float(e[:, res].max() / cmax),
           "image_max_abs_rel_b_above_1e-4": float(e[:, well].max() / cmax),
           "image_rel_l2_all_voxels": float(np.linalg.norm(c - c_o) / np.linalg.norm(c_o)),
           "image_max_abs_rel_all_voxels": float(e.max() / cmax),
           "resolved_voxels": int(res.sum()), "voxels": int(res.size),
           "objective_rel": float(abs(hist.item() - h_o[0]) / abs(h_o[0]))}
    base = {"value": 1.0 / t_full, "unit": "iterations/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"1 FP64 oracle DEAM iteration over the middle {gs.n_views} of {g.n_views} views "
                      f"({t_s:.1f} s, of which {t_u:.2f} s the whole-image update), scaled by the "
                      f"ray count to the whole scan: {t_full:.1f} s per iteration"}
    if one_core_views:
        g1, w0 = view_block(g, one_core_views)
        sl1 = slice(w0 * per_view, (w0 + g1.n_views) * per_view)
        n_all = O.num_threads()
        O.set_num_threads(1)
        t0 = time.perf_counter()
        _, _, b1 = O.iterate(g1, inp["I0"], inp["mu"], np.ascontiguousarray(inp["d"][:, sl1]),
                             np.ascontiguousarray(mask_np[sl1]), Z, inp["c0"], 1, want_b=True)
        t1 = time.perf_counter() - t0
        t0 = time.perf_counter()
        O.update(b1, Z, inp["c0"])
        tu1 = time.perf_counter() - t0
        O.set_num_threads(n_all)
        t1_full = g.n_views / g1.n_views * max(t1 - tu1, 0.0) + tu1
        base["one_core"] = {"value": 1.0 / t1_full, "unit": "iterations/s", "cores": 1,
                            "sample": f"1 FP64 oracle iteration over the middle {g1.n_views} views "
                                      f"({t1:.1f} s), scaled: {t1_full:.0f} s per iteration"}
    return base, err


def oracle_full_iterations(g, inp, mask_np, n_it, plan, d, mask, c0, dev):
    """The FP64 oracle over n_it whole iterations on all host cores (a workload
    small enough for that), and the GPU's n_it iterations against it."""
    import torch
    from oracle import oracle as O
    Z = inp["Z"]
    t0 = time.perf_counter()
    c_o, h_o = O.iterate(g, inp["I0"], inp["mu"], inp["d"], mask_np, Z, inp["c0"], n_it)
    t_cpu = time.perf_counter() - t0
    cg = c0.clone()
    hg = torch.zeros(n_it, dtype=torch.float64, device=dev)
    plan.iterate(cg, d, mask, Z, n_it, hg)
    cg = cg.cpu().numpy()
    base = {"value": n_it / t_cpu, "unit": "iterations/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"{n_it} whole FP64 oracle DEAM iterations from the cold start ({t_cpu:.1f} s)"}
    err = {"iterations": n_it,
           "image_rel_l2": float(np.linalg.norm(cg - c_o) / np.linalg.norm(c_o)),
           "image_max_abs_rel": float(np.abs(cg - c_o).max() / np.abs(c_o).max()),
           "objective_rel": float(np.abs(hg.cpu().numpy() - h_o).max() / abs(h_o[0]))}
    return base, err


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="helical", choices=sorted(WORKLOAD_DESC))
    ap.add_argument("--fp64-steps", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=4,
                    help="whole oracle iterations of the fan-beam workload")
    ap.add_argument("--cpu-sample-views", type=int, default=1152,
                    help="views of the helical oracle sample (all host cores; default one rotation)")
    ap.add_argument("--cpu-one-core-views", type=int, default=18,
                    help="views of the helical oracle sample timed on one core")
    ap.add_argument("--no-secondary", action="store_true",
                    help="measure the main iteration only (skip the penalised, MAR and variant "
                         "measurements and the secondary and unrolled-reconstruction workloads)")
    ap.add_argument("--secondary-steps", type=int, default=20)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy three times (reference for the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (the DEAM path is measured on one MI355X); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.calibrate_copy:
        bw, launches = copy_bandwidth(dev)
        print(json.dumps({"copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30,
                          "launches": launches, "copy_GBps": bw / 1e9}))
        return
    K, W = args.steps, args.warmup
    K64 = args.fp64_steps if args.fp64_steps is not None else max(3, K // 4)
    log = lambda msg: print(f"[bench] {msg}", file=sys.stderr, flush=True)  # noqa: E731
    copy_bw, _ = copy_bandwidth(dev)
    log(f"device copy: {copy_bw / 1e9:.0f} GB/s (read + write)")
    m = measure(args.workload, K, W, K64, dev, log, extras=not args.no_secondary)
    g, inp, t_step = m["inp"]["geom"], m["inp"], m["t_step"]
    plan, d, mask, c0, Z = m["plan"], m["d"], m["mask"], m["c0"], inp["Z"]

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
                   "rays": g.n_rays, "voxels": g.n_voxels,
                   "energy_bins": int((inp["I0"].sum(axis=0) > 0).sum()),
                   "metal_rays": int(mask.sum().item())},
        "grays_per_s": m["grays"],
        "grays_per_s_1ch": m["grays_1ch"],
        "kernel_ms": m["kernel_ms"],
        "fp64": m["fp64"],
        "speedup_mixed_vs_fp64": m["speedup"],
        "roofline": m["roofline"],
        "iteration_roofline": m["iteration"],
        "hbm_copy_GBps": copy_bw / 1e9,
        "penalized": m["penalized"],
        "mar_init": m["mar_init"],
        "variants": m["variants"],
        "cpu_baseline": None,
    }

    # --- CPU baseline (the FP64 oracle) and the error against it --------------------
    if not args.no_cpu_baseline:
        mask_np = mask.cpu().numpy()
        if g.kind == 1:
            out["cpu_baseline"], out["error_vs_oracle"] = oracle_sample(
                g, inp, mask_np, args.cpu_sample_views, type(plan), dev,
                one_core_views=args.cpu_one_core_views)
        else:
            out["cpu_baseline"], out["error_vs_oracle"] = oracle_full_iterations(
                g, inp, mask_np, args.cpu_iters, plan, d, mask, c0, dev)
        log(f"cpu baseline: {out['cpu_baseline']['value']:.4f} it/s on "
            f"{out['cpu_baseline']['cores']} cores")

    # --- secondary workloads: the other geometry and the unrolled reconstruction
    if not args.no_secondary:
        other = "fan512" if args.workload == "helical" else "helical"
        del m, plan, d, mask, c0
        torch.cuda.empty_cache()
        K2 = args.secondary_steps
        h = measure(other, K2, 1, max(3, K2 // 4), dev, log)
        blk = {"workload": f"{other}: {WORKLOAD_DESC[other]}",
               "iterations_per_s": 1.0 / h["t_step"], "ms_per_step": h["t_step"] * 1e3,
               "steps": K2, "grays_per_s": h["grays"], "grays_per_s_1ch": h["grays_1ch"],
               "kernel_ms": h["kernel_ms"], "fp64": h["fp64"],
               "speedup_mixed_vs_fp64": h["speedup"], "roofline": h["roofline"],
               "iteration_roofline": h["iteration"], "penalized": h["penalized"],
               "mar_init": h["mar_init"], "variants": h["variants"]}
        if not args.no_cpu_baseline:
            hg, hinp = h["inp"]["geom"], h["inp"]
            hmask = h["mask"].cpu().numpy()
            if hg.kind == 1:
                blk["cpu_baseline"], blk["error_vs_oracle"] = oracle_sample(
                    hg, hinp, hmask, args.cpu_sample_views, type(h["plan"]), dev)
            else:
                blk["cpu_baseline"], blk["error_vs_oracle"] = oracle_full_iterations(
                    hg, hinp, hmask, args.cpu_iters, h["plan"], h["d"], h["mask"], h["c0"], dev)
        out[other] = blk
        del h
        torch.cuda.empty_cache()
    if not args.no_secondary:
        out["unrolled"] = measure_unrolled(dev, log)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
