#!/usr/bin/env python3
"""ReLCP time-step throughput on one MI355X.

Workload (compacting suspension, Sec. 5.2 of the paper, at 100,000 bodies):
periodic ellipsoids with semiaxes i.i.d. uniform in [0.5, 1.0] and uniform
random orientations, placed by random sequential addition of their bounding
spheres, compressed (untimed set-up) to volume fraction 0.40; each timed step
then compresses the box isotropically by dphi = 5e-5 and takes one overdamped
ReLCP step (dt = 5e-3, overlap_tol = 1e-3, lcp_tol = 1e-6, previous-step
warm start, FP32 products with FP64 residual and acceptance by default).

Prints one JSON line with steps/s, the roofline of the dominant kernel
(measured with HIP events inside the library on its own stream) and the CPU
oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def phi_of(shape, box):
    return float(np.sum(4.0 / 3.0 * np.pi * shape[:, 0] * shape[:, 1] * shape[:, 2]) / np.prod(box))


def lcp_bytes(kind, m, nb, w):
    """Algorithmic bytes of one launch of an LCP pass over m rows, nb bodies,
    word size w (4 = FP32, 8 = FP64).
    gather:  per row ia, ib (8 B), n, r_a x n, r_b x n (9w), qv, A_aa, gamma,
             g read (4w), gamma, g written (2w); per body the velocity (6w).
    scatter: per row two incidence entries (8 B), n, r_a x n, r_b x n,
             gamma, g, A_aa (12w); per body offset (4 B), K (9w), velocity
             written (6w)."""
    if kind == "lcp_gather":
        return m * (8 + 15 * w) + nb * 6 * w
    return m * (8 + 12 * w) + nb * (4 + 15 * w)


def setup(args):
    from paper_2506_14097_amd import inputs as I
    from paper_2506_14097_amd import relcp as R
    t0 = time.time()
    P = I.ellipsoid_packing(args.seed, args.n, sphere_phi=0.3)
    log("placed %d bodies at phi %.3f in %.1fs" % (args.n, P["phi"], time.time() - t0))
    sim = R.Simulation(P["x"], P["q"], P["kind"], P["shape"], P["rho_xi"], P["box"], precision=args.precision,
                       skin=args.skin, warm_start=R.WS_PREV)
    box = P["box"].copy()
    phi = phi_of(P["shape"], box)
    rate = 0.015
    k = 0
    t0 = time.time()
    while phi < args.phi0 - 1e-12:
        target = min(args.phi0, phi * (1 + rate))
        s = (phi / target) ** (1.0 / 3.0)
        sim.affine_rescale(s)
        res = sim.step(args.dt, args.eps, args.tol, raise_on_error=False)
        if res["status"] != 0:
            sim.affine_rescale(1.0 / s)
            rate *= 0.5
            if rate < 1e-5:
                raise RuntimeError("set-up compression stalled at phi %.4f (status %d)" % (phi, res["status"]))
            continue
        box *= s
        phi = target
        k += 1
        if k % 20 == 0:
            log("set-up compression: step %d phi %.4f contacts %d recursions %d (%.1fs)" %
                (k, phi, res["n_contacts_final"], res["recursions"], time.time() - t0))
    log("set-up done: phi %.4f after %d steps (%.1fs)" % (phi, k, time.time() - t0))
    return sim, P, box, phi


def run_steps(sim, shape, box, phi, nsteps, args, stats=None):
    for _ in range(nsteps):
        target = phi + args.dphi
        s = (phi / target) ** (1.0 / 3.0)
        sim.affine_rescale(s)
        box *= s
        phi = target
        res = sim.step(args.dt, args.eps, args.tol)
        if stats is not None:
            stats.append(res)
    return box, phi


def cpu_baseline(args, bench_pairs, bench_rec):
    """The CPU oracle (FP64, single thread) on a bounded sample of the same
    workload: one step of a periodic packing from the same generator.  The
    oracle's step is an all-pairs candidate search (quadratic in N) plus
    per-pair SNSD at C^k and at every trial; the two parts are timed
    separately and scaled to the benchmark's body count (quadratically) and
    candidate-pair x SNSD-pass count (linearly)."""
    import oracle as O
    from paper_2506_14097_amd import inputs as I
    n = args.cpu_n
    P = I.ellipsoid_packing(args.seed + 1, n, sphere_phi=0.3, compress=0.99)
    t0 = time.time()
    O.broadphase(P["x"], P["kind"], P["shape"], P["box"], args.skin)
    t_bp = time.time() - t0
    t0 = time.time()
    r = O.relcp_step(P["x"], P["q"], P["kind"], P["shape"], P["rho_xi"], P["box"], dt=args.dt, eps=args.eps,
                     tol=args.tol, skin=args.skin, lcp_mode=1)
    t = time.time() - t0
    work_sample = r["n_pairs"] * (1 + r["recursions"])
    work_bench = bench_pairs * (1 + bench_rec)
    t_est = t_bp * (args.n / n) ** 2 + max(t - t_bp, 0.0) * work_bench / max(work_sample, 1)
    return {"value": 1.0 / t_est, "unit": "steps/s", "cores": 1, "kind": "oracle",
            "sample": "one FP64 oracle step (single thread, %.1fs, of which %.1fs all-pairs candidate search) of a "
                      "%d-ellipsoid periodic packing at phi %.3f (%d candidate pairs x %d SNSD passes, %d rows); "
                      "scaled to %d bodies (search, quadratic) and %d pairs x %.2f passes per step (rest, linear)"
                      % (t, t_bp, n, P["phi"], r["n_pairs"], 1 + r["recursions"], r["n_rows"], args.n, bench_pairs,
                         1 + bench_rec)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=100000)
    ap.add_argument("--precision", type=int, default=32, choices=(32, 64))
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--phi0", type=float, default=0.40)
    ap.add_argument("--dphi", type=float, default=5e-5)
    ap.add_argument("--dt", type=float, default=5e-3)
    ap.add_argument("--eps", type=float, default=1e-3)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--skin", type=float, default=0.05)
    ap.add_argument("--roofline-steps", type=int, default=5)
    ap.add_argument("--cpu-n", type=int, default=20000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe-mb", type=float, default=0.0,
                    help="only run a device-to-device copy of this many MB (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2506_14097_amd import relcp as R
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_probe_mb > 0:
        nel = int(args.copy_probe_mb * 1e6 / 4)
        a = torch.ones(nel, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        log("copy probe: 5 copies of %d bytes" % (4 * nel))
        return
    R.lib()

    sim, P, box, phi = setup(args)
    shape = P["shape"]
    box, phi = run_steps(sim, shape, box, phi, args.warmup, args)
    log("warm-up done, timing %d steps" % args.steps)
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    box, phi = run_steps(sim, shape, box, phi, args.steps, args, stats)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    value = args.steps / elapsed
    pgd = [s["lcp_iters_total"] for s in stats]
    citers = sum(int(np.dot(s["n_contacts"], s["lcp_iters"])) for s in stats)
    log("timed: %.3f s, %.2f steps/s, PGD iters/step %.1f" % (elapsed, value, np.mean(pgd)))

    # roofline: kernel durations from HIP events recorded by the library on
    # its stream, over further steps of the same protocol
    sim.set_timing(True)
    sim.get_timing(reset=True)
    rstats = []
    box, phi = run_steps(sim, shape, box, phi, args.roofline_steps, args, rstats)
    tm = sim.get_timing(reset=True)
    sim.set_timing(False)
    w_lo = 4 if args.precision == 32 else 8
    nb = args.n
    tot_bytes = {"lcp_gather": 0.0, "lcp_scatter": 0.0}
    for s in rstats:
        for m, it, it64 in zip(s["n_contacts"], s["lcp_iters"], s["lcp_iters64"]):
            itlo = it - it64
            for cls in tot_bytes:
                if args.precision == 32:
                    tot_bytes[cls] += (itlo + 1) * lcp_bytes(cls, m, nb, 4) + (it64 + 1) * lcp_bytes(cls, m, nb, 8)
                else:
                    tot_bytes[cls] += (it + 1) * lcp_bytes(cls, m, nb, 8)
    dom = max(tm, key=lambda k: tm[k][1])
    cnt, ms = tm[dom]
    if dom in tot_bytes:
        achieved = tot_bytes[dom] / (ms * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None, "launches": cnt, "avg_us": 1e3 * ms / max(cnt, 1),
                "bytes_per_launch": tot_bytes[dom] / max(cnt, 1)}
    else:
        roof = {"kernel": dom, "bound": "alu", "achieved": None, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": None, "traffic": None, "launches": cnt, "avg_us": 1e3 * ms / max(cnt, 1)}
    roof["kernel_ms"] = {k: round(v[1], 3) for k, v in tm.items()}
    roof["kernel_launches"] = {k: v[0] for k, v in tm.items()}

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(args, float(np.mean([s["n_pairs"] for s in stats])),
                           float(np.mean([s["recursions"] for s in stats])))

    out = {
        "metric": "ReLCP steps/s @100k ellipsoids; PGD iters to 1e-6 residual (learned vs plain)",
        "value": value, "unit": "steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64" if args.precision == 32 else "f64", "data": "synthetic",
        "config": {"workload": "compaction of %d periodic ellipsoids (semiaxes U[0.5,1]), phi %.2f -> %.5f at "
                               "dphi %.0e/step, overdamped, dt %.0e, overlap_tol %.0e, lcp_tol %.0e, previous-step "
                               "warm start" % (args.n, args.phi0, phi, args.dphi, args.dt, args.eps, args.tol),
                   "bodies": args.n, "precision": args.precision, "skin": args.skin},
        "pgd_iters_per_step": {"plain": float(np.mean(pgd)), "learned": None},
        "contact_iters_per_s": citers / elapsed,
        "recursions_per_step": float(np.mean([s["recursions"] for s in stats])),
        "contacts_final": int(stats[-1]["n_contacts_final"]),
        "residual_fp64_max": float(max(s["residual_fp64"] for s in stats)),
        "max_overlap": float(max(s["max_overlap"] for s in stats)),
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
