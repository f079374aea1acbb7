#!/usr/bin/env python3
"""Throughput of the PISCO sensitivity-map path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

One step is one full pass of the hot path on one synthetic scan whose ACS is
already resident in HBM: calibration Gram by FFT correlation, FP64 signal /
null split, G(x) on the low-resolution grid, per-voxel power iteration, phase
reference, sinc interpolation and RSS normalisation (pisco_estimate).  The
value is output voxels (maps on the full grid) per second of the mixed form
(G(x) contraction on FP16 matrix cores with split operands); the plain FP32
form is timed the same way and reported beside it, and with the CPU
baseline both forms' map errors against the FP64 oracle are reported.

Prints one JSON line.  The roofline object describes the kernel that takes
the most time in the timed steps: its launches are bracketed by HIP events on
the library's stream (pisco_trace_enable) during the timed region.  The CPU
baseline times the FP64 oracle on this host's cores after the GPU timing.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mvoxel maps/s end-to-end, mixed/learned vs plain FP32 at fixed map error"

# nullspace block per workload (a multiple of 32 comfortably above the signal rank)
BLOCKS = {"2d_64x64_q8_acs24_r3": 64, "2d_256x256_q32_acs32_r5": 96,
          "3d_96x160x160_q16_acs24_r4": 224}

PEAKS = {  # MI355X datasheet, dense
    "hbm": (8000.0, "GB/s"),
    "fp64": (78.6, "TFLOP/s"),        # vector FP64
    "mfma_fp64": (78.6, "TFLOP/s"),   # FP64 matrix cores
    "fp32": (157.3, "TFLOP/s"),
}


def kernel_model(name: str, w, est, rs: int):
    """(bound, algorithmic work per launch, unit) of a kernel, or None.

    Work per unit (the method's own need, not what the kernel happens to do):
      k_gemm_ax  Gram x block, complex FP64 (matrix cores): 8 n^2 b flops
      k_hetrd    Householder tridiagonalisation, order b, complex:
                 16/3 b^3 flops (4/3 b^3 real multiply-adds, x4 for complex)
      k_chol_inv Cholesky + triangular inverse, order b: 8/3 b^3 + 4/3 b^3 flops
      k_herk     K^s_hat over r_s signal vectors:     8 nK P r_s flops
      k_power    power iteration:                     8 Q^2 (iters + 1) N_lr flops
      k_gather   Gram write:                          8 n^2 bytes
      k_rss      read + write of the output maps:     16 Q N_out bytes
    """
    n, b, Q = est.n, est.block, est.Q
    if name.startswith("k_gemm_ax"):
        return "mfma_fp64", 8.0 * n * n * b, "flop"
    if name.startswith("k_hetrd"):
        return "fp64", 16.0 / 3.0 * b ** 3, "flop"
    if name.startswith("k_chol_inv"):
        return "fp64", 4.0 * b ** 3, "flop"
    if name.startswith("k_herk"):
        nK = 1
        tau = int(w.radius)
        for _ in range(w.D):
            nK *= 4 * tau + 1
        return "fp32", 8.0 * nK * est.P * rs, "flop"
    if name.startswith("k_power"):
        return "fp32", 8.0 * Q * Q * (est.opts.power_iters + 1) * est.Nlr, "flop"
    if name.startswith("k_gather"):
        return "hbm", 8.0 * n * n, "byte"
    if name.startswith("k_rss"):
        return "hbm", 16.0 * Q * est.Nout, "byte"
    return None


KERNEL_SOURCES = {"k_gemm_ax": "nullspace.hip", "k_hetrd": "heev.hip", "k_hetrd_reg": "heev.hip",
                  "k_chol": "nullspace.hip", "k_tri_inv": "nullspace.hip",
                  "k_gemm_tn": "nullspace.hip",
                  "k_gemm_nn": "nullspace.hip", "k_herk": "gx.hip", "k_power": "eig.hip",
                  "k_gather": "gram.hip", "k_rss": "maps.hip"}


def measured_traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summaries,
    or None when there is none or the kernel's source changed since."""
    import glob
    import hashlib
    base = kernel.split("<")[0].strip("()")
    src = KERNEL_SOURCES.get(base)
    if not src:
        return None
    path = os.path.join(ROOT, "paper_2302_13431_amd", "csrc", src)
    digest = hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]
    for f in glob.glob(os.path.join(ROOT, "profiles", "*.md")):
        for line in open(f):
            parts = line.split()
            if len(parts) == 5 and parts[0] == "traffic" and parts[1] == base \
                    and parts[3] == src and parts[4] == digest:
                return float(parts[2])
    return None


def cpu_baseline(w, acs, budget_s: float = 25.0):
    """Oracle (FP64 numpy) on a bounded sample: whole-pipeline runs of the same
    scan until about `budget_s` seconds have been spent (at least one)."""
    import numpy as np
    from oracle import pipeline as opipe
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = len(os.sched_getaffinity(0))
    a = acs.astype(np.complex128)
    runs, spent, ref = 0, 0.0, None
    while runs == 0 or spent < budget_s * 0.5:
        t0 = time.perf_counter()
        ref = opipe.estimate(a, w.radius, w.grid_lr, w.grid)
        spent += time.perf_counter() - t0
        runs += 1
        if spent > budget_s:
            break
    nout = 1
    for g in w.grid:
        nout *= g
    return {"value": runs * nout / spent / 1e6, "unit": "Mvoxel/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{runs} full oracle run(s) of the same scan ({nout} output voxels each), "
                      f"{spent:.1f} s"}, ref


def map_error_defined(w, ref, out):
    """Largest gauge-invariant map error vs the FP64 oracle where the map is
    defined (coil-combined apodized low-res image >= 1e-3 of its maximum,
    eroded by one low-res voxel, carried to the output grid)."""
    import numpy as np
    from scipy.ndimage import binary_erosion
    from oracle import metrics
    m = np.abs(np.sum(np.conj(ref.c_lr) * ref.rho_lr, axis=0))
    mask_lr = binary_erosion(m >= 1e-3 * m.max(), iterations=1)
    idx = [np.round(((np.arange(n) - n // 2) / n) * l + l // 2).astype(int) % l
           for n, l in zip(w.grid, w.grid_lr)]
    mask = mask_lr[np.ix_(*idx)]
    return float(metrics.map_error(ref.maps, out)[mask].max())


def learned_report(w, acs, n_scans: int, tol: float = 1e-4):
    """Train the warm-start network (library kernels) on the method's own
    eigenvectors of `n_scans` seeded scans of this workload's family, then
    on the benchmark scan report the power-iteration steps to reach
    ||G c - lambda c|| <= tol |Lambda| from the plain, neighbour-only and
    learned starts, and the time of that eigen stage (for the learned start
    it includes the coarse-grid field and solve, the neighbour gather and the
    network)."""
    import numpy as np
    import torch
    import paper_2302_13431_amd as P
    from paper_2302_13431_amd.warmstart import LearnedSolver
    from synth import generator
    blk = BLOCKS.get(w.name, 0)
    est = P.Estimator(w.Q, w.acs, w.radius, w.grid_lr, w.grid, block=blk)
    est_c = P.Estimator(w.Q, w.acs, w.radius, P.coarse_grid(w.grid_lr), w.grid, block=blk)
    ws = P.WarmStart(w.Q, seed=7)
    solver = LearnedSolver(est, est_c, ws)
    bound = float(est.nsup)
    tight = P.make_opts(power_iters=4000, tol=1e-6, block=est.block)
    t0 = time.perf_counter()
    data = []
    for s in range(n_scans):
        sc = generator.make_scan(30000 + s, w.grid, w.Q, w.acs, 20, w.snr_db, keep_kspace=False)
        G, Gc = solver.fields(torch.from_numpy(generator.as_device_input(sc.acs)).cuda())
        target, _, _ = est.eig(G, opts=tight)
        data.append((G, solver.neighbour(Gc), target))
        if s % 16 == 15:
            print(f"learned: {s + 1} training scans", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    t0 = time.perf_counter()
    first = last = None
    for ep in range(20):
        tot = 0.0
        for i in np.random.default_rng(ep).permutation(len(data)):
            G, nb, target = data[i]
            tot += float(ws.train_step(G, nb, target, bound, 1e-3).item())
        first = tot / len(data) if first is None else first
        last = tot / len(data)
    t_train = time.perf_counter() - t0
    G, Gc = solver.fields(acs)
    opts = P.make_opts(power_iters=4000, tol=tol, block=est.block)
    _, _, ip = est.eig(G, opts=opts)
    _, _, inb = est.eig_from(G, solver.neighbour(Gc), opts)
    _, _, il = solver.solve(G, Gc, opts)

    def timed(fn, reps=20):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps * 1e3

    def learned_stage():
        Gc_ = est_c.gx(*solver_basis)
        return solver.solve(G, Gc_, opts)

    gram = est.gram(acs)
    _, basis, counts = est.nullspace(gram)
    solver_basis = (basis, counts)
    return {"voxels_trained": int(n_scans * est.Nlr), "train_scans": n_scans, "epochs": 20,
            "loss_first_epoch": first, "loss_last_epoch": last,
            "data_s": round(t_data, 2), "train_s": round(t_train, 2), "tol": tol,
            "iters_mean": {"plain": float(ip.float().mean()), "neighbour": float(inb.float().mean()),
                           "learned": float(il.float().mean())},
            "eig_stage_ms": {"plain": timed(lambda: est.eig(G, opts=opts)),
                             "learned": timed(learned_stage)}}


def batched_report(steps: int):
    """64 seeded 2D slices with uneven grids (128^2, 192^2, 256^2, 256x320),
    Q in {8, 16, 32}, ACS 24-40, radius 3-6, 30 dB: all slices in one graph
    launch (pisco_batch_*, autotuned, fixed nullspace schedules) against the
    same slices as one pisco_estimate call each with the same block sizes
    (adaptive schedules, host reads).  Throughput is output voxels of all
    slices per second."""
    import numpy as np
    import torch
    import paper_2302_13431_amd as P
    from synth import as_device_input, workloads
    slices = workloads.batch_slices()
    acs = [torch.from_numpy(as_device_input(s.scan(keep_kspace=False).acs)).cuda() for s in slices]
    print("batched: slices generated", file=sys.stderr, flush=True)
    nout = sum(int(np.prod(s.grid)) for s in slices)
    specs = [{"Q": s.Q, "acs": s.acs, "radius": s.radius, "grid_lr": s.grid_lr,
              "grid_out": s.grid} for s in slices]
    t = time.perf_counter()
    b = P.Batch(specs, acs)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t
    print(f"batched: planned and captured in {t_plan:.1f} s", file=sys.stderr, flush=True)
    # per-slice launches with the same (tuned) block sizes
    ests = [P.Estimator(s.Q, s.acs, s.radius, s.grid_lr, s.grid, block=b.info(i)[0])
            for i, s in enumerate(slices)]
    outs = [torch.empty((s.Q,) + tuple(s.grid), dtype=torch.complex64, device="cuda")
            for s in slices]
    flags_eager = 0
    for e, a, o in zip(ests, acs, outs):
        e.estimate(a, o)
        flags_eager |= e.status()
    torch.cuda.synchronize()
    t = time.perf_counter()
    reps = max(1, steps // 4)
    for _ in range(reps):
        for e, a, o in zip(ests, acs, outs):
            e.estimate(a, o)
    torch.cuda.synchronize()
    t_eager = (time.perf_counter() - t) / reps
    print("batched: eager timed", file=sys.stderr, flush=True)
    b.launch()
    torch.cuda.synchronize()
    flags_graph = b.status()
    t = time.perf_counter()
    for _ in range(steps):
        b.launch()
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t) / steps
    flags_graph |= b.status()
    err = 0.0
    from oracle.metrics import map_error
    for i in range(len(slices)):
        e = map_error(outs[i].cpu().numpy(), b.outputs[i].cpu().numpy())
        err = max(err, float(np.percentile(e, 99)))
    blocks = sorted({b.info(i)[0] for i in range(len(slices))})
    b.close()
    return {"slices": len(slices), "voxels_out": nout,
            "graph": {"Mvoxel_s": nout / t_graph / 1e6, "ms": t_graph * 1e3,
                      "device_status": flags_graph},
            "per_slice_launches": {"Mvoxel_s": nout / t_eager / 1e6, "ms": t_eager * 1e3,
                                   "device_status": flags_eager},
            "plan_and_tune_s": round(t_plan, 2), "tuned_blocks": blocks,
            "graph_vs_eager_map_error_p99_max": err}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="2d_256x256_q32_acs32_r5")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip training and measuring the learned warm start")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batch of 64 uneven slices in one graph launch")
    ap.add_argument("--learned-scans", type=int, default=64,
                    help="training scans for the learned warm start (64 x 56^2 = 200k voxels)")
    ap.add_argument("--breakdown", action="store_true", help="per-kernel times to stderr")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (HBM counter "
                         "calibration under rocprofv3) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.empty(args.copy_calibration * (1 << 20), dtype=torch.uint8, device="cuda")
        src.fill_(1)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel(), "copies": 5}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the path does not run "
              "across GPUs in this build.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    import paper_2302_13431_amd as P
    from synth import as_device_input, workloads

    w = workloads.ALL[args.workload]
    scan = w.scan(keep_kspace=False)
    acs_np = as_device_input(scan.acs)
    acs = torch.from_numpy(acs_np).cuda()
    nout = int(np.prod(w.grid))

    def run_form(precision, trace_all=False):
        """Warm up, find the dominant kernel, time `steps` steps (that kernel
        bracketed by HIP events).  Returns a dict of results."""
        est = P.Estimator(w.Q, w.acs, w.radius, w.grid_lr, w.grid,
                          block=BLOCKS.get(w.name, 0), precision=precision)
        out = torch.empty((w.Q,) + tuple(w.grid), dtype=torch.complex64, device="cuda")
        lam = torch.empty((est.Nlr,), dtype=torch.float32, device="cuda")
        for _ in range(args.warmup):
            est.estimate(acs, out, lam)
        torch.cuda.synchronize()
        status = est.status()
        P.pisco_trace_enable(est.h, True, None)
        est.estimate(acs, out, lam)
        per = P.pisco_trace_read(est.h)
        P.pisco_trace_enable(est.h, False)
        dom = max(per.items(), key=lambda kv: kv[1][1])[0]
        P.pisco_trace_enable(est.h, True, dom)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            est.estimate(acs, out, lam)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        traced = P.pisco_trace_read(est.h).get(dom, (0, 0.0))
        P.pisco_trace_enable(est.h, False)
        status |= est.status()
        return {"est": est, "out": out.cpu().numpy(), "status": status, "per": per, "dom": dom,
                "traced": traced, "ms": elapsed / args.steps * 1e3,
                "value": args.steps * nout / elapsed / 1e6}

    mixed = run_form(P._lib.PREC_SPLIT_F16)
    plain = run_form(P._lib.PREC_FP32)
    # the mixed form as a one-slice graph (fixed nullspace schedule, no host
    # read-back, one launch)
    g1 = P.Batch([{"Q": w.Q, "acs": w.acs, "radius": w.radius, "grid_lr": w.grid_lr,
                   "grid_out": w.grid, "precision": P._lib.PREC_SPLIT_F16,
                   "block": BLOCKS.get(w.name, 0)}], [acs])
    g1.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g1.launch()
    torch.cuda.synchronize()
    g1_ms = (time.perf_counter() - t0) / args.steps * 1e3
    g1_status = g1.status()
    g1_products = g1.info(0)[1]
    g1.close()
    if args.breakdown:
        for tag, r in (("mixed", mixed), ("plain_fp32", plain)):
            tot = sum(v[1] for v in r["per"].values())
            print(f"[{tag}] {r['ms']:.3f} ms/step", file=sys.stderr)
            for k, (cnt, ms) in sorted(r["per"].items(), key=lambda kv: -kv[1][1]):
                print(f"  {k:28s} {cnt:5d} launches {ms:9.3f} ms {100 * ms / tot:5.1f}%",
                      file=sys.stderr)

    est, dom, traced = mixed["est"], mixed["dom"], mixed["traced"]
    roof = None
    _, _, counts = est.nullspace(est.gram(acs))
    rs = int(counts[0].item())
    model = kernel_model(dom, w, est, rs)
    if model and traced[0] > 0:
        bound, work, unit = model
        avg_s = traced[1] / traced[0] / 1e3
        if bound == "hbm":
            achieved = work / avg_s / 1e9
            peak, punit = PEAKS["hbm"]
        else:
            achieved = work / avg_s / 1e12
            peak, punit = PEAKS[bound]
        roof = {"kernel": dom,
                "bound": "hbm" if bound == "hbm" else ("mfma" if bound.startswith("mfma")
                                                      else "alu"),
                "dtype": {"hbm": None, "mfma_fp64": "fp64"}.get(bound, bound),
                "achieved": achieved, "peak": peak, "unit": punit, "frac": achieved / peak,
                "traffic": measured_traffic(dom), "launches": traced[0], "avg_us": avg_s * 1e6,
                "work_per_launch": work, "work_unit": unit}

    line = {"metric": METRIC, "value": mixed["value"], "unit": "Mvoxel/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": mixed["ms"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": w.name, "grid": list(w.grid), "Q": w.Q, "acs": list(w.acs),
                       "radius": w.radius, "grid_lr": list(w.grid_lr),
                       "precision": "G(x) contraction on FP16 matrix cores with split operands "
                                    "and FP32 accumulation; nullspace FP64; rest FP32",
                       "power_iters": 10, "nullspace_block": est.block, "signal_rank": rs,
                       "device_status": mixed["status"] | plain["status"],
                       "plain_fp32": {"value": plain["value"], "ms_per_step": plain["ms"]},
                       "mixed_graph": {"value": nout / g1_ms / 1e3, "ms_per_step": g1_ms,
                                       "nullspace_products": g1_products,
                                       "device_status": g1_status}},
            "roofline": roof}
    if not args.no_learned:
        line["config"]["learned_warm_start"] = learned_report(w, acs, args.learned_scans)
    if not args.no_batched:
        line["config"]["batched"] = batched_report(args.steps)
    if not args.no_cpu_baseline:
        base, ref = cpu_baseline(w, acs_np)
        line["cpu_baseline"] = base
        line["config"]["map_error_vs_fp64"] = {"mixed": map_error_defined(w, ref, mixed["out"]),
                                               "plain_fp32": map_error_defined(w, ref,
                                                                               plain["out"])}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
