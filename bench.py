#!/usr/bin/env python3
"""Throughput of the fused Shan-Chen extended-stencil step on one MI355X.

Workload (one "step" = one time step of the whole lattice: pull-stream, moments, psi, the
24-vector wide-stencil force, BGK + Guo collision): D2Q9, 4096 x 4096 periodic sites,
forcing shells {1,2,4,5,8} with seeded free weights satisfying e2 = 1, I40 = I60 = 0,
psi = exp(-1/n), G = 1.2 G_c (reduced temperature 0.2), tau = 1, spinodal start
n ~ U(0.5, 1.5); populations stored in FP32 as shifted deviations g = f - w rho0.

Prints one JSON line. MLUPS = sites x steps / time / 1e6. The roofline object prices the
step kernel against HBM: algorithmic bytes per site-step are 2 Q s (each population read
once and written once, s = bytes per stored value).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS & %HBM roofline, FP32 vs FP64 at stated error; adjoint/forward cost ratio"
HBM_PEAK_GBS = 8000.0
WORKLOAD = "D2Q9 4096x4096 periodic, extended forcing stencil shells {1,2,4,5,8} (24 vectors, seeded weights), spinodal start U(0.5,1.5), 2000-step run"
DIMS = (4096, 4096)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step2d_c2_traffic.json")
KERNEL_SOURCES = ["paper_2505_23647_amd/csrc/step2d.hpp", "paper_2505_23647_amd/csrc/scl_common.hpp"]


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return h.hexdigest()[:16]


def workload_inputs():
    from paper_2505_23647_amd import stencil, synth
    u = synth.knob_draws(2, 2, 0.0, 1.0)
    e4, e8, W = stencil.seeded_family2d(u[0], u[1])
    G = -1.2 * np.e ** 2          # 1.2 x the critical coupling -e^2 of psi = exp(-1/n), e2 = 1
    n0 = synth.uniform(DIMS, 0.5, 1.5, seed=1)
    return e4, e8, W, G, n0


def make_lattice(prec, W, G, n0, stream):
    from paper_2505_23647_amd import Lattice
    lat = Lattice([DIMS], prec, stream=stream)
    lat.set_physics(1.0, G).set_stencil([1, 2, 4, 5, 8], W).init_density(n0)
    return lat


def timed(lat, steps, warmup):
    lat.step(warmup)
    ms = lat.step_timed(steps)
    return ms


def c5_problem(prec, stream=None):
    """Batched droplet workload of the adjoint: 16 D2Q9 domains of 256 x 256, each with its own
    seeded shell weights (shells {1,2,4,5,8}), a droplet of radius 40 at the flat coexistence
    densities relaxed for 20000 steps, then a differentiated window of 2000 steps with
    checkpoints every 45 steps."""
    from paper_2505_23647_amd import stencil, synth, thermo
    from paper_2505_23647_amd.autograd import DropletProblem
    L, R, ndom, steps, every = 256, 40.0, 16, 2000, 45
    G = thermo.coupling_for_reduced_temperature(0.2)
    ng, nl, _ = thermo.coexistence_exp(G)
    W = np.array([stencil.seeded_family2d(*synth.knob_draws(5 + b, 2, 0.0, 1.0))[2] for b in range(ndom)])
    n0 = np.concatenate([synth.droplet((L, L), R, nl, ng, noise=1e-3, seed=100 + b) for b in range(ndom)])
    prob = DropletProblem([(L, L)] * ndom, n0, [(L // 2, L // 2)] * ndom, [1, 2, 4, 5, 8], 1.0, steps, every,
                          prec, stream=stream, equilibrate=20000)
    return prob, W, np.full(ndom, G)


def c5_targets(obs):
    """Seeded targets: sigma* = sigma (1 + 0.05 u), delta* = delta + 0.5 u', u, u' ~ U(-1, 1)."""
    from paper_2505_23647_amd import synth
    ndom = obs.shape[0]
    u = synth.knob_draws(7, 2 * ndom, -1.0, 1.0)
    return obs[:, 3] * (1 + 0.05 * u[:ndom]), obs[:, 5] + 0.5 * u[ndom:]


def c3_workload():
    """Batched Laplace-test workload: 32 radii R_k = 8 * 16^(k/31) (log-spaced 8..128), each
    as a droplet (domain 2k) and a bubble (domain 2k + 1) in a periodic square of side
    round(4 R_k + 32) (64..544; 3,976,466 sites in all). E(8) weights, psi = exp(-1/n),
    G = 1.2 G_c, tau = 1, tanh profile of width 3 between the coexistence densities of
    eq. (SCMaxwell) for the stencil's eps = 10/31, noise U(-1e-3, 1e-3) with seed 100 + domain.
    Returns dims, n0 (concatenated), W, G, centers, is_bubble, radii."""
    from paper_2505_23647_amd import synth, thermo
    W = [4 / 21, 4 / 45, 1 / 60, 2 / 315, 1 / 5040]
    G = thermo.coupling_for_reduced_temperature(0.2)
    ng, nl = thermo.coexistence_exp(G, eps=thermo.epsilon(4 / 7))[:2]
    radii = synth.log_radii(32, 8.0, 128.0)
    dims, n0, centers, bubble = [], [], [], []
    for k, R in enumerate(radii):
        L = int(round(4 * R + 32))
        for b in (0, 1):
            dom = 2 * k + b
            n_in, n_out = (ng, nl) if b else (nl, ng)
            dims.append((L, L))
            n0.append(synth.droplet((L, L), R, n_in, n_out, noise=1e-3, seed=100 + dom))
            centers.append((L // 2, L // 2))
            bubble.append(b)
    return dims, np.concatenate(n0), W, G, np.array(centers), np.array(bubble, dtype=np.int8), radii


def batched_leg(stream, steps=2000):
    """The batched Laplace workload (64 domains, 3,976,466 sites) stepped in one launch per
    step, replayed through HIP graphs of 100 steps: whole-batch MLUPS with launch overheads."""
    from paper_2505_23647_amd import SCL_FP32_SHIFTED, Lattice
    dims, n0, W, G, centers, bubble, radii = c3_workload()
    lat = Lattice(dims, SCL_FP32_SHIFTED, stream=stream).set_physics(1.0, G).set_stencil([1, 2, 4, 5, 8], W)
    lat.init_density(n0)
    lat.set_graph_steps(100)
    lat.step(200)
    ms = lat.step_timed(steps)
    ml = lat.cells * steps / (ms / 1e3) / 1e6
    ach = 2 * 9 * 4 * lat.cells / (ms / 1e3 / steps) / 1e9
    out = {"domains": len(dims), "sites": lat.cells, "steps": steps, "MLUPS": round(ml, 1),
           "achieved_GBs": round(ach, 1), "frac": round(ach / HBM_PEAK_GBS, 4), "tiling": list(lat.get_tiling())}
    # the autotuner's pick for this batch (timed on the lattice itself, outside the timed run)
    lat.tune()
    lat.step(100)
    ms = lat.step_timed(steps)
    out["tuned"] = {"MLUPS": round(lat.cells * steps / (ms / 1e3) / 1e6, 1), "tiling": list(lat.get_tiling())}
    lat.close()
    return out


def adjoint_leg(stream):
    """Wall time of the checkpointed forward (with the observables) and of the backward
    (observables VJP + recompute + reverse steps) on the batched droplet workload, FP32;
    loss = squared error of sigma_s and delta against seeded targets."""
    import torch
    from paper_2505_23647_amd import SCL_FP32_SHIFTED
    prob, W, G = c5_problem(SCL_FP32_SHIFTED, stream)
    prob.run(W, G)  # relaxation, allocations, code objects
    prob.load(W, G)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    obs = prob.forward()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ts, td = c5_targets(obs)
    g = np.zeros_like(obs)
    g[:, 3] = 2 * (obs[:, 3] - ts)
    g[:, 5] = 2 * (obs[:, 5] - td)
    t2 = time.perf_counter()
    gW, gG = prob.vjp(g)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    fwd, bwd = t1 - t0, t3 - t2
    prob.lat.close()
    return {"workload": "16 x D2Q9 256^2 droplets R=40 (relaxed 20000 steps), 2000-step window FP32 shifted storage, checkpoints every 45",
            "forward_s": round(fwd, 4), "backward_s": round(bwd, 4), "ratio": round(bwd / fwd, 3),
            "grad_finite": bool(np.all(np.isfinite(gW)) and np.all(np.isfinite(gG)))}


def d3q19_leg(stream, steps=40):
    """D3Q19 512^3 FP32 with the 92-vector stencil (seeded weights near 3D E(8)), tau = 0.8,
    n0 = 1 + U(-1e-2, 1e-2): MLUPS and algorithmic HBM bandwidth (2 x 19 x 4 bytes/site)."""
    from paper_2505_23647_amd import SCL_FP32, Lattice, stencil, synth
    dims = (512, 512, 512)
    u = synth.knob_draws(3, 3, 0.0, 1.0)
    W = stencil.seeded_family3d(*u)[3]
    G = -1.2 * np.e ** 2
    n0 = synth.around(dims, 1.0, 1e-2, seed=4)
    lat = Lattice([dims], SCL_FP32, stream=stream).set_physics(0.8, G).set_stencil(list(stencil.SHELLS_3D), W)
    lat.init_density(n0)
    del n0
    lat.step(5)
    ms = lat.step_timed(steps)
    cells = 512 ** 3
    ml = cells * steps / (ms / 1e3) / 1e6
    ach = 2 * 19 * 4 * cells / (ms / 1e3 / steps) / 1e9
    lat.close()
    return {"MLUPS": round(ml, 1), "achieved_GBs": round(ach, 1), "frac": round(ach / HBM_PEAK_GBS, 4),
            "steps": steps, "stencil_vectors": 92}


def cpu_baseline(W, G, n0_full, budget_s=12.0):
    """The FP64 oracle on the host cores, on a 1024 x 1024 crop of the same workload."""
    import oracle
    crop = n0_full.reshape(DIMS[1], DIMS[0])[:1024, :1024].copy()
    s = oracle.Sim((1024, 1024), 1.0, G, [1, 2, 4, 5, 8], W).init_density(crop)
    s.run(2)  # first touch
    t0 = time.perf_counter()
    steps = 0
    while time.perf_counter() - t0 < budget_s:
        s.run(5)
        steps += 5
    dt = time.perf_counter() - t0
    return {"value": round(1024 * 1024 * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"FP64 oracle, 1024x1024 crop of the same initial field and stencil, {steps} steps in {dt:.1f} s"}


def load_traffic(bytes_alg):
    if not os.path.exists(TRAFFIC_FILE):
        return None
    t = json.load(open(TRAFFIC_FILE))
    if t.get("kernel_hash") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


def _csv_rows(d, suffix):
    import csv
    import glob
    rows = []
    for f in sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)):
        with open(f, newline="") as fh:
            rows += list(csv.DictReader(fh))
    if not rows:
        raise SystemExit(f"no *{suffix} under {d}")
    return rows


def _counter_median(d, name_has, counter):
    vals = [float(r["Counter_Value"]) for r in _csv_rows(d, "counter_collection.csv")
            if name_has in r["Kernel_Name"] and r["Counter_Name"] == counter]
    if not vals:
        raise SystemExit(f"no {counter} rows for a kernel named *{name_has}* under {d}")
    return float(np.median(vals)), len(vals)


def write_traffic(kt_dir, fetch_dir, write_dir, copy_fetch_dir, copy_write_dir):
    """Traffic of the step kernel per launch from rocprofv3 output directories: the kernel
    trace's average duration, FETCH_SIZE and WRITE_SIZE (KiB per dispatch, median) of the step
    kernel, each scaled by what the same counter reads for the device copy of known size
    (bench.py --mode copy). Writes the file that the bench line's roofline.traffic reads."""
    key = "k_step2d<float, float, 1, 512, 1, true, false>"
    stats = [r for r in _csv_rows(kt_dir, "kernel_stats.csv") if key in r["Name"]]
    if len(stats) != 1:
        raise SystemExit(f"expected one kernel-stats row for {key}, found {len(stats)}")
    avg_ns, calls = float(stats[0]["AverageNs"]), int(stats[0]["Calls"])
    fk, _ = _counter_median(fetch_dir, key, "FETCH_SIZE")
    wk, _ = _counter_median(write_dir, key, "WRITE_SIZE")
    cf, _ = _counter_median(copy_fetch_dir, "copyBuffer", "FETCH_SIZE")
    cw, _ = _counter_median(copy_write_dir, "copyBuffer", "WRITE_SIZE")
    copy_bytes = 4 * (1 << 28)
    fscale, wscale = copy_bytes / (cf * 1024), copy_bytes / (cw * 1024)
    fb, wb = fk * 1024 * fscale, wk * 1024 * wscale
    alg = 2 * 9 * 4 * DIMS[0] * DIMS[1]
    t = {"kernel": "void scl::" + key, "kernel_hash": kernel_hash(), "avg_duration_ns": avg_ns, "calls": calls,
         "fetch_kib_raw_median": fk, "write_kib_raw_median": wk, "copy_fetch_kib_raw": cf, "copy_write_kib_raw": cw,
         "fetch_scale": fscale, "write_scale": wscale, "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
         "bytes_per_launch": fb + wb, "bytes_alg_per_launch": alg, "traffic_over_alg": (fb + wb) / alg,
         "fetch_over_alg_reads": fb / (alg / 2), "achieved_alg_GBs_from_trace": alg / avg_ns,
         "achieved_traffic_GBs_from_trace": (fb + wb) / avg_ns}
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(t, fh, indent=1)
    print(json.dumps(t), flush=True)


def copy_calibration():
    """A plain device copy of known size (for scaling the FETCH_SIZE / WRITE_SIZE counters)."""
    import torch
    n = 1 << 28  # 1 GiB of float32
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 5}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--tune", action="store_true", help="run the autotuner before timing")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-3d", action="store_true")
    ap.add_argument("--mode", default="bench", choices=["bench", "copy", "d3q19", "fp64", "fp16"],
                    help="copy: device copy for counter calibration; d3q19: the 3D leg alone; "
                         "fp64, fp16: the main workload in that storage precision alone")
    ap.add_argument("--write-traffic", nargs=5, metavar=("TRACE", "FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="rocprofv3 output directories (kernel trace, FETCH_SIZE and WRITE_SIZE of the bench, "
                         "the same counters of --mode copy): write the step kernel's measured traffic")
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(*args.write_traffic)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.mode == "copy":
        copy_calibration()
        return
    if args.mode == "d3q19":
        print(json.dumps({"d3q19_512cube_fp32": d3q19_leg(None, steps=args.steps)}), flush=True)
        return
    if args.mode in ("fp64", "fp16"):
        from paper_2505_23647_amd import SCL_FP16S_FP32, SCL_FP64
        prec, s = (SCL_FP64, 8) if args.mode == "fp64" else (SCL_FP16S_FP32, 2)
        e4, e8, W, G, n0 = workload_inputs()
        lv = make_lattice(prec, W, G, n0, None)
        msv = timed(lv, args.steps, args.warmup)
        cells = DIMS[0] * DIMS[1]
        ach = 2 * 9 * s * cells / (msv / 1e3 / args.steps) / 1e9
        print(json.dumps({args.mode: {"MLUPS": round(cells * args.steps / (msv / 1e3) / 1e6, 1),
                                      "achieved_GBs": round(ach, 1), "frac": round(ach / HBM_PEAK_GBS, 4),
                                      "tiling": list(lv.get_tiling())}}), flush=True)
        return

    import torch
    from paper_2505_23647_amd import SCL_FP16S_FP32, SCL_FP32_SHIFTED, SCL_FP64

    torch.cuda.init()
    stream = torch.cuda.current_stream().cuda_stream
    e4, e8, W, G, n0 = workload_inputs()
    cells = DIMS[0] * DIMS[1]

    lat = make_lattice(SCL_FP32_SHIFTED, W, G, n0, stream)
    if args.tune:
        lat.tune()
    torch.cuda.synchronize()
    ms = timed(lat, args.steps, args.warmup)
    torch.cuda.synchronize()
    mlups = cells * args.steps / (ms / 1e3) / 1e6
    bytes_alg = 2 * 9 * 4 * cells
    avg_s = ms / 1e3 / args.steps
    achieved = bytes_alg / avg_s / 1e9
    out = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms / args.steps, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOAD, "sites": cells, "stencil_vectors": 24, "precision": "FP32 shifted",
                   "e4": round(float(e4), 6), "e8": round(float(e8), 6), "G": G, "tau": 1.0,
                   "tiling": list(lat.get_tiling())},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": load_traffic(bytes_alg),
                     "bytes_alg_per_launch": bytes_alg, "kernel": "k_step2d (fused step)"},
    }
    if not args.no_variants:
        var = {}
        n_fp32 = lat.density()
        for name, prec, s in (("fp64", SCL_FP64, 8), ("fp16_storage", SCL_FP16S_FP32, 2)):
            lv = make_lattice(prec, W, G, n0, stream)
            msv = timed(lv, args.steps, args.warmup)
            ml = cells * args.steps / (msv / 1e3) / 1e6
            ach = 2 * 9 * s * cells / (msv / 1e3 / args.steps) / 1e9
            var[name] = {"MLUPS": round(ml, 1), "achieved_GBs": round(ach, 1), "frac": round(ach / HBM_PEAK_GBS, 4)}
            if prec == SCL_FP64:
                n64 = lv.density()
                var["fp32_shifted_vs_fp64_density_rel_err"] = float(np.abs(n_fp32 - n64).max() / np.abs(n64).max())
                # the same FP64 run from n0 perturbed by 1e-15 (relative): how far the spinodal
                # dynamics alone carries a rounding-level difference over the same steps
                lt = make_lattice(SCL_FP64, W, G, n0 * (1.0 + 1e-15), stream)
                lt.step(args.steps + args.warmup)
                nt = lt.density()
                var["fp64_twin_perturbed_1e-15_density_rel_err"] = float(np.abs(nt - n64).max() / np.abs(n64).max())
                lt.close()
            lv.close()
        if not args.no_3d:
            var["d3q19_512cube_fp32"] = d3q19_leg(stream)
        var["batched_64_domains_fp32_shifted"] = batched_leg(stream)
        out["variants"] = var
    if not args.no_adjoint:
        out["adjoint"] = adjoint_leg(stream)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(W, G, n0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
