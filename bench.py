#!/usr/bin/env python3
"""ReLCP time-step throughput on one MI355X.

Workload (compacting suspension, Sec. 5.2 of the paper, at 100,000 bodies):
periodic ellipsoids with semiaxes i.i.d. uniform in [0.5, 1.0] and uniform
random orientations, placed by random sequential addition of their bounding
spheres, compressed (untimed set-up) to volume fraction 0.40; each timed step
then compresses the box isotropically by dphi = 5e-5 and takes one overdamped
ReLCP step (dt = 5e-3, overlap_tol = 1e-3, lcp_tol = 1e-6, previous-step
warm start, FP32 products with FP64 residual and acceptance by default).

Prints one JSON line with steps/s over the timed steps and, beside it:
 * roofline: the FP32 LCP iteration pass (the dominant kernel) by the
   method's bytes per iteration, its duration measured with HIP events
   inside the library on its own stream;
 * narrowphase: the SNSD pass's launch time and FP64 issue rate;
 * error_vs_oracle and cpu_baseline: the CPU oracle (FP64, OpenMP) timed on
   one step of the benchmark's own state, and the GPU's FP32 and FP64 steps
   from that state against the oracle's;
 * learned_warm_start: the learned start against the previous-step one at
   volume fractions 0.40, 0.50 and 0.60 (the model is trained on the GPU
   first, untimed);
 * workloads: the FP64 path at 100k, the whole compression 0.40 -> 0.60
   (4,000 steps) in windows, the 10,000-ellipsoid compaction 0.30 -> 0.55 in
   both precisions, 512 packings in one context, and the growing colony at
   4,096 cells (--workload colony: also 65,536 and 131,072).

Other workloads (--workload): packings512, colony, lcp-sweep (the LCP pass
across sizes), two-ellipsoids (the timestep refinement of Sec. 5.1) and
chainmail (interlaced rings under the extensile field of Sec. 6, ReLCP
against LCP-SNSD); each prints its own JSON line.
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

# HBM bytes per iterating launch of the FP32 row-graph pass at this workload,
# from two rocprofv3 --pmc runs (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0, the scales
# a plain copy of known size reads), recorded in
# profiles/lcp_rowgraph_pass_100k_hbm_traffic.md for the kernel source with
# the given sha256 prefix (stale once it changes).
MEASURED_TRAFFIC = {"sha256_prefix": "8f6f3f61ee651537", "lcp_rowgraph": 1.3852e7}


# timing class -> kernel
KERNEL_SYMBOLS = {"lcp_rowgraph": "relcp::k_spmv<float, 1>", "lcp_rowgraph64": "relcp::k_spmv<double, 1>",
                  "lcp_rowgraph_start": "relcp::k_spmv<T, 0> / k_spmv<double, 3>", "lcp_gather": "relcp::k_gather<T, 1>",
                  "lcp_scatter": "relcp::k_scatter<T, 1>"}


# FP64 VALU instructions of the narrowphase per candidate pair at this
# workload (rocprofv3 --pmc SQ_INSTS_VALU_ADD_F64, _MUL_F64, _FMA_F64,
# _TRANS_F64: add + mul + 2 fma + trans, times 64 lanes, over the pairs of
# the launch), for the kernel source with the given sha256 prefix.
SNSD_FP64_OPS = {"sha256_prefix": "558655cd61167acf", "fp64_ops_per_pair": 1276.9,
                 "source": "profiles/snsd_pairs_100k_fp64_counters.md: issued FP64 operations (64 lanes per wave "
                           "instruction) per candidate pair, mean of the pass at C^k and the pass at the trial"}


def geometry_source_sha():
    import hashlib
    with open(os.path.join(ROOT, "paper_2506_14097_amd", "csrc", "geometry.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def kernel_source_sha():
    import hashlib
    with open(os.path.join(ROOT, "paper_2506_14097_amd", "csrc", "lcp.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


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


def method_bytes(m, nb, w):
    """Algorithmic bytes of one projected-gradient iteration of the method
    over m constraint rows and nb bodies, word size w (the matrix-free
    iteration on D^T K D): per row, the row's Jacobian (n, r_a x n, r_b x n)
    read twice (scatter and gather, 18w), its two body indices twice (16 B),
    gamma read and written, g, the constant qv, the previous gamma and g
    (8w): 26w + 16 B (120 B in FP32, 224 B in FP64); per body, K (9w) and
    the velocity written and read back (6w each) less one word: 14w (56 B in
    FP32, 112 B in FP64)."""
    return m * (26 * w + 16) + nb * 14 * w


def rowgraph_bytes(m, e, w, iters):
    """Algorithmic bytes of the row-graph passes of one solve: m rows, e
    stored off-diagonal entries of A (padding excluded), word size w, iters
    iterations.  Every pass reads each entry's column (4 B) and value (w).  The start
    pass reads gamma0, qv, A_rr and writes the row state (gamma, h) and g
    (6w per row); an iteration pass reads the row's previous state (gamma,
    h), g, qv, A_rr and writes the new state and g (8w per row; the
    neighbours' states it gathers are the same array, counted once)."""
    return (iters + 1) * e * (4 + w) + m * w * (6 + 8 * iters)


def learned_comparison(args, state):
    """Learned against previous-step warm start on the same workload.  The
    model is trained on the GPU (library kernels) on rows of A_0 logged from
    a 10,000-ellipsoid compaction (seed 1) at volume fractions 0.40 to 0.60;
    then, at the benchmark's state (0.40) and after compressing it further to
    0.60, two contexts start from the same state, take three previous-step
    warm-up steps and `learned_steps` timed steps each, one per warm start.
    Reported per level: PGD iterations per step, wall ms per step, the
    host-clock LCP time per step (time to the 1e-6 residual, inference
    included) and the summed duration of the warm-start kernels."""
    import torch
    from paper_2506_14097_amd import learned as L
    from paper_2506_14097_amd import relcp as R
    from paper_2506_14097_amd.compaction import Compaction
    t0 = time.time()
    C = Compaction(1, 10000, 0.40, dt=args.dt, eps=args.eps, tol=args.tol, precision=args.precision, skin=args.skin)
    C.sim.enable_contact_log(True)
    rows = L.ContactLog()
    for level in (0.40, 0.45, 0.50, 0.55, 0.60):
        C.compress_to(level)
        C.steps(5, args.dphi)
        C.steps(15, args.dphi, on_step=lambda s, r: rows.record(s))
    C.sim.close()
    feat, gam = rows.tensors()
    norm = L.normalisation(feat, gam)
    tr = L.Trainer(norm, seed=0)
    t1 = time.time()
    hist = tr.fit(feat, gam, epochs=20)
    torch.cuda.synchronize()
    t_train = time.time() - t1
    W = tr.weights()
    log("learned warm start: %d training rows, loss %.2e -> %.2e, %.1fs training (%.1fs with logging)" %
        (feat.shape[0], hist[0], hist[-1], t_train, time.time() - t0))
    out = {"training_rows": int(feat.shape[0]), "epochs": 20, "train_s": t_train,
           "loss_first_epoch": hist[0], "loss_last_epoch": hist[-1], "levels": {}}
    B = Compaction(None, None, None, state=state, dt=args.dt, eps=args.eps, tol=args.tol, precision=args.precision,
                   skin=args.skin)
    for level in (0.40, 0.50, 0.60):
        B.compress_to(max(level, B.phi))
        st0 = B.state()
        res = {"volume_fraction": B.phi}
        for name, mode in (("plain", R.WS_PREV), ("learned", R.WS_LEARNED)):
            D = Compaction(None, None, None, state=st0, dt=args.dt, eps=args.eps, tol=args.tol,
                           precision=args.precision, skin=args.skin)
            D.sim.set_warmstart_model(W, norm)
            D.steps(3, args.dphi)
            D.sim.set_warm_start(mode)
            torch.cuda.synchronize()
            t = time.perf_counter()
            st = D.steps(args.learned_steps, args.dphi)
            torch.cuda.synchronize()
            el = time.perf_counter() - t
            D.sim.set_timing(True)
            D.sim.get_timing(reset=True)
            D.steps(3, args.dphi)
            tm = D.sim.get_timing(reset=True)
            res[name] = {"pgd_iters_per_step": float(np.mean([s["lcp_iters_total"] for s in st])),
                         "ms_per_step": 1e3 * el / args.learned_steps,
                         "lcp_ms_per_step": float(np.mean([s["t_lcp"] for s in st])),
                         "warm_start_kernel_ms_per_step": tm["warm_start"][1] / 3.0,
                         "contacts": int(st[-1]["n_contacts_final"])}
            log("  phi %.3f %s: %s" % (B.phi, name, res[name]))
            D.sim.close()
        out["levels"]["%.2f" % level] = res
    B.sim.close()
    return out


def lcp_sweep(args):
    """The LCP loop alone at many sizes: lattice contact graphs (about 1.3
    rows per body, rows sorted by body), solved on the GPU through the
    stateless entry point in the row-graph mode with one launch per pass, 40
    FP32 iterations then 40 FP64 iterations (tolerance out of reach, so the
    pass count is fixed).  Wall time per solve (second of two runs); the
    per-pass kernel durations come from a rocprofv3 kernel trace of this
    command."""
    import torch
    from paper_2506_14097_amd import inputs as I
    from paper_2506_14097_amd import relcp as R
    dev = torch.device("cuda:0")

    def soa(a):
        return torch.tensor(np.ascontiguousarray(np.asarray(a).T), dtype=torch.float64, device=dev).contiguous()

    out = []
    for mt in [int(v) for v in args.sweep_rows.split(",")]:
        L = I.lattice_lcp(1, mt)
        m = int(L["ia"].size)
        a = (L["n"], torch.tensor(L["ia"], device=dev), torch.tensor(L["ib"], device=dev), soa(L["nrm"]),
             soa(L["ta"]), soa(L["tb"]), torch.tensor(L["qv"], dtype=torch.float64, device=dev),
             torch.tensor(L["kt"], dtype=torch.float64, device=dev),
             torch.tensor(L["Kr6"], dtype=torch.float64, device=dev), 0.05)
        for _ in range(2):
            g = torch.zeros(m, dtype=torch.float64, device=dev)
            torch.cuda.synchronize()
            t = time.perf_counter()
            it, res, rc = R.lcp_solve_device(*a, g, precision=32, mode=4, tol=1e-14, max_iters=40)
            torch.cuda.synchronize()
            el = time.perf_counter() - t
        rec = {"rows": m, "bodies": int(L["n"]), "entries": int(L["E"]), "iterations": int(it),
               "solve_ms": 1e3 * el,
               "bytes_per_pass_fp32": rowgraph_bytes(m, L["E"], 4, 1) - rowgraph_bytes(m, L["E"], 4, 0),
               "bytes_per_pass_fp64": rowgraph_bytes(m, L["E"], 8, 1) - rowgraph_bytes(m, L["E"], 8, 0)}
        log("lcp sweep: %s" % json.dumps(rec))
        out.append(rec)
    print(json.dumps({"metric": "row-graph LCP solve time vs size (lattice contact graphs)", "unit": "ms",
                      "data": "synthetic", "sizes": out}), flush=True)


def two_ellipsoid_study(args):
    """Timestep refinement of the two-ellipsoid sliding collision (Sec. 5.1,
    Table 1): ReLCP and LCP-SNSD (the same step with no recursions, the
    first trial accepted) from t0 = 98 to --t-end at each timestep of --dts,
    FP64, overlap_tol 1e-5, lcp_tol 1e-12.  Error of a run: root mean square
    over unit-time samples of the difference of the upper body's centre (x,
    y) and of the angle of its long axis from the ReLCP run at the finest
    timestep.  Per run: wall ms per step, the steps that needed recursions,
    the largest recursion count and the largest accepted overlap."""
    import torch
    from paper_2506_14097_amd import inputs as I
    from paper_2506_14097_amd import relcp as R
    S = I.glancing_ellipsoids()
    dts = sorted((float(v) for v in args.dts.split(",")), reverse=True)
    t0, t_end = S["t0"], args.t_end

    def long_axis_angle(q):
        s, a, b, c = q
        # third column of the rotation matrix: the body z (long) axis
        return np.arctan2(2 * (b * c - s * a), 2 * (a * c + s * b))

    runs = []
    for dt in dts:
        for method, mr in (("ReLCP", 64), ("LCP-SNSD", 0)):
            if method == "LCP-SNSD" and dt == dts[-1] and len(dts) > 1:
                continue  # the reference timestep: ReLCP only
            sim = R.Simulation(S["x"], S["q"], S["kind"], S["shape"], S["rho_xi"], S["box"], precision=64,
                               skin=0.5, max_recursions=mr, warm_start=R.WS_PREV)
            sim.set_external(S["fext"])
            n = int(round((t_end - t0) / dt))
            every = int(round(1.0 / dt))
            samples, nrec, maxrec, maxov = [], 0, 0, 0.0
            torch.cuda.synchronize()
            tw = time.perf_counter()
            for k in range(1, n + 1):
                res = sim.step(dt, 1e-5, 1e-12)
                nrec += res["recursions"] > 0
                maxrec = max(maxrec, res["recursions"])
                maxov = max(maxov, res["max_overlap"])
                if k % every == 0:
                    x, q, _ = sim.get_state()
                    samples.append((x[1, 0], x[1, 1], long_axis_angle(q[1])))
                if k % 100000 == 0:
                    log("two ellipsoids: %s dt %g step %d of %d" % (method, dt, k, n))
            el = time.perf_counter() - tw
            sim.close()
            runs.append(dict(method=method, dt=dt, steps=n, ms_per_step=1e3 * el / n, steps_with_recursions=int(nrec),
                             max_recursions=int(maxrec), max_overlap=maxov, samples=np.array(samples)))
            log("two ellipsoids: %s dt %g: %d steps, %.3f ms/step, %d with recursions, max overlap %.3g" % (
                method, dt, n, 1e3 * el / n, nrec, maxov))
    ref = runs[-1]["samples"]
    out = []
    for r in runs:
        e = np.sqrt(((r.pop("samples") - ref) ** 2).mean(axis=0))
        r.update(err_x=float(e[0]), err_y=float(e[1]), err_angle=float(e[2]))
        out.append(r)
    print(json.dumps({"metric": "two-ellipsoid timestep refinement: L2 error against the finest ReLCP run",
                      "unit": "length, length, rad", "data": "synthetic", "t0": t0, "t_end": t_end,
                      "xi": float(S["rho_xi"][0]), "runs": out}), flush=True)


def chainmail_study(args):
    """Chainmail of interlaced rings pulled taut by the extensile field (Sec.
    6, Fig. chainmail): ReLCP against LCP-SNSD (no recursions, the first
    trial accepted) at --cm-dt up to --cm-t-end, FP64, overlap_tol 1e-5,
    lcp_tol 1e-12, on a --cm-n x --cm-n lattice of node rings with their
    connectors (tori R = 1, r = 0.1, drag --cm-xi, seeded placement jitter
    --cm-jitter; LCP tolerance --cm-lcp-tol, at most 10^6 iterations; a
    step that fails ends its run, which records it).  The field depends on the
    positions, so each step reads the state back and sets the external
    wrench first.  The violation of a step is the largest overlap of the
    accepted configuration on the true ring surfaces (exact torus SNSD).
    Per method: the largest violation, the steps with recursions, ms per
    step (with the read-back) and the violation per window of 1/20 of the
    run; the extent of the network at the end."""
    import torch
    from paper_2506_14097_amd import inputs as I
    from paper_2506_14097_amd import relcp as R
    S = I.chainmail(args.cm_n, args.cm_n, xi=args.cm_xi, jitter=args.cm_jitter, seed=0)
    dt, n = args.cm_dt, int(round(args.cm_t_end / args.cm_dt))
    win = max(1, n // 20)
    runs = []
    for method, mr in (("ReLCP", 64), ("LCP-SNSD", 0)):
        sim = R.Simulation(S["x"], S["q"], S["kind"], S["shape"], S["rho_xi"], S["box"], precision=64, skin=0.1,
                           max_recursions=mr, warm_start=R.WS_PREV, lcp_max_iters=1000000)
        series, wmax, nrec, maxrec, maxov, cont, failed = [], 0.0, 0, 0, 0.0, 0, None
        torch.cuda.synchronize()
        tw = time.perf_counter()
        for k in range(1, n + 1):
            x, _, _ = sim.get_state()
            sim.set_external(I.extensile_field(x))
            res = sim.step(dt, 1e-5, args.cm_lcp_tol, raise_on_error=False)
            if res["status"] != 0:
                failed = dict(step=k, t=round(k * dt, 6), status=int(res["status"]))
                log("chainmail: %s stopped at t %.3f, status %d" % (method, k * dt, res["status"]))
                break
            nrec += res["recursions"] > 0
            maxrec = max(maxrec, res["recursions"])
            wmax = max(wmax, res["max_overlap"])
            cont = res["n_contacts_final"]
            if k % win == 0:
                series.append([round(k * dt, 6), wmax, int(cont)])
                maxov = max(maxov, wmax)
                wmax = 0.0
                log("chainmail: %s t %.3f max violation %.3g contacts %d" % (method, k * dt, series[-1][1], cont))
        el = time.perf_counter() - tw
        x, _, _ = sim.get_state()
        sim.close()
        done = failed["step"] - 1 if failed else n
        runs.append(dict(method=method, steps=done, failed=failed, ms_per_step=1e3 * el / max(done, 1),
                         steps_with_recursions=int(nrec),
                         max_recursions=int(maxrec), max_violation=max(maxov, wmax),
                         extent_xy=[float(np.ptp(x[:, 0])), float(np.ptp(x[:, 1]))], series=series))
    print(json.dumps({"metric": "chainmail: largest overlap of the accepted configurations (true ring surfaces)",
                      "unit": "length (minor radius 0.1)", "data": "synthetic", "rings": int(len(S["x"])),
                      "dt": dt, "t_end": args.cm_t_end, "overlap_tol": 1e-5, "lcp_tol": args.cm_lcp_tol,
                      "xi": args.cm_xi,
                      "jitter": args.cm_jitter,
                      "extent_xy_start": [float(np.ptp(S["x"][:, 0])), float(np.ptp(S["x"][:, 1]))],
                      "runs": runs}), flush=True)


def packings_workload(args, steps=None, warmup=None):
    """Batched workload: 512 independent periodic packings (body counts
    log-uniform in [200, 5000], target volume fractions uniform in [0.3,
    0.5]) in one context; set-up compresses each packing to its own target,
    then every timed step compresses each packing by dphi and steps all of
    them together, in the LCP configuration the autotuner picks.  Returns
    the result record."""
    import torch
    from paper_2506_14097_amd import inputs as I
    from paper_2506_14097_amd import relcp as R
    t0 = time.time()
    B = I.batch_of_packings(3, args.packings, 200, 5000, 0.3, 0.5, sphere_phi=0.3, rescale=False)
    off = B["batch_off"]
    npk = len(off) - 1
    log("placed %d packings, %d bodies in %.1fs" % (npk, off[-1], time.time() - t0))
    sim = R.Simulation(B["x"], B["q"], B["kind"], B["shape"], B["rho_xi"], B["box"], batch_off=off,
                       precision=args.precision, skin=args.skin, warm_start=R.WS_PREV)
    phi = B["phi"].copy()
    target = B["phi_target"]
    rate = 0.015
    k = 0
    t0 = time.time()
    while np.any(phi < target - 1e-12):
        nxt = np.minimum(target, phi * (1 + rate))
        s = (phi / nxt) ** (1.0 / 3.0)
        sim.affine_rescale_packings(s)
        res = sim.step(args.dt, args.eps, args.tol, raise_on_error=False)
        if res["status"] != 0:
            sim.affine_rescale_packings(1.0 / s)
            rate *= 0.5
            if rate < 1e-5:
                raise RuntimeError("set-up compression stalled (status %d)" % res["status"])
            continue
        phi = nxt
        k += 1
        if k % 10 == 0:
            log("set-up compression: step %d mean phi %.4f contacts %d (%.1fs)" % (k, phi.mean(),
                                                                                 res["n_contacts_final"],
                                                                                 time.time() - t0))
    log("set-up done after %d steps (%.1fs)" % (k, time.time() - t0))

    def advance(nsteps, stats=None):
        nonlocal phi
        for _ in range(nsteps):
            nxt = phi + args.dphi
            sim.affine_rescale_packings((phi / nxt) ** (1.0 / 3.0))
            phi = nxt
            r = sim.step(args.dt, args.eps, args.tol)
            if stats is not None:
                stats.append(r)

    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    advance(1)
    tune = sim.autotune(args.dt, args.tol, reps=2)
    log("autotuned LCP configuration: %s" % tune)
    advance(warmup)
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    advance(steps, stats)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sim.set_timing(True)
    sim.get_timing(reset=True)
    rstats = []
    advance(args.roofline_steps, rstats)
    tm = sim.get_timing(reset=True)
    # the timed launches' rows and iterations (a launch covers every packing)
    rg = [(m, it - i64, e) for r in rstats for m, it, i64, e in zip(r["n_contacts"], r["lcp_iters"], r["lcp_iters64"],
                                                                      r["rowgraph_entries"])]

    out = {"metric": "packing-steps/s, %d independent periodic ellipsoid packings in one context" % npk,
           "value": npk * steps / el, "unit": "packing-steps/s", "steps": steps,
           "ms_per_step": 1e3 * el / steps, "bodies": int(off[-1]), "packings": npk,
           "lcp_pass_hbm_frac": lcp_pass_frac(tm, rg, int(off[-1]), args.precision),
           "dtype": "f32+f64" if args.precision == 32 else "f64",
           "pgd_iters_per_step_max_over_packings": float(np.mean([r["lcp_iters_total"] for r in stats])),
           "contacts_final": int(stats[-1]["n_contacts_final"]),
           "recursions_per_step": float(np.mean([r["recursions"] for r in stats])),
           "max_overlap": float(max(r["max_overlap"] for r in stats)), "autotune": tune,
           "kernel_ms": {k2: round(v[1], 3) for k2, v in tm.items()},
           "kernel_launches": {k2: v[0] for k2, v in tm.items()}}
    sim.close()
    return out


def lcp_pass_frac(tm, rows, nb, precision):
    """Fraction of HBM peak of the FP32 (or FP64) iterating row-graph
    passes by the method's bytes per iteration (method_bytes): rows is a
    list of (rows, low-precision iterations, entries) per solve."""
    cls = "lcp_rowgraph" if precision == 32 else "lcp_rowgraph64"
    cnt, ms = tm.get(cls, (0, 0.0))
    if not cnt or ms <= 0:
        return None
    w = 4 if precision == 32 else 8
    tot = sum(k * method_bytes(m, nb, w) for m, k, _ in rows)
    return tot / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_threads():
    """Threads for the oracle's per-pair loops: the host's CPUs, at most 16
    (the CPU share of one GPU on the benchmark machines)."""
    return max(1, min(16, os.cpu_count() or 1))


def host_state(st, s):
    """A state of a Compaction after one more affine rescale by s (the input
    of the next step)."""
    return dict(st, x=st["x"] * s, box=st["box"] * s)


def contact_sets_match(c, ref):
    """Per recursion, the GPU's rows against the oracle's: 'identical', or
    where they first differ; pairs within 1e-9 of the overlap threshold
    (flagged) stop the comparison."""
    band = np.where(ref["margin"] < 1e-9)[0]
    upto = band[0] if band.size else ref["recursions"]
    for r in range(upto + 1):
        g = sorted(zip(c["ia"][c["rec"] == r].tolist(), c["ib"][c["rec"] == r].tolist()))
        o = sorted(zip(ref["ia"][ref["rec"] == r].tolist(), ref["ib"][ref["rec"] == r].tolist()))
        if g != o:
            return "differ at recursion %d" % r
    return "identical" + (" up to the flagged recursion %d" % upto if band.size else "")


def gpu_step_error(args, S, precision, lcp_tol, ref):
    """One GPU step from host state S in a fresh context (zero start) at the
    given precision and LCP tolerance, against the oracle's step ref from the
    same state: contact sets per recursion, velocities (relative to the
    largest), positions and orientations."""
    from paper_2506_14097_amd import relcp as R
    sim = R.Simulation(S["x"], S["q"], S["kind"], S["shape"], S["rho_xi"], S["box"], precision=precision,
                       skin=args.skin, warm_start=R.WS_COLD)
    res = sim.step(args.dt, args.eps, lcp_tol)
    x, q, U = sim.get_state()
    c = sim.get_contacts(res["n_contacts_final"])
    sim.close()
    sets = contact_sets_match(c, ref)
    out = {"precision": precision, "lcp_tol": lcp_tol, "contact_sets": sets,
           "recursions": [int(res["recursions"]), int(ref["recursions"])],
           "rows": [int(res["n_contacts_final"]), int(ref["n_rows"])],
           "U_rel": float(np.abs(U - ref["U"]).max() / max(np.abs(ref["U"]).max(), 1e-300)),
           "x_abs": float(np.abs(x - ref["x"]).max()), "q_abs": float(np.abs(q - ref["q"]).max()),
           "residual_fp64": float(res["residual_fp64"])}
    log("error against the oracle: %s" % out)
    return out


def cpu_baseline(args, S):
    """The CPU oracle (FP64, OpenMP over pairs) timed on the benchmark's own
    state: one step at the benchmark's parameters (lcp_tol as benchmarked,
    zero start), with the candidate search and the SNSD at C^k also timed on
    their own.  Then the oracle's step at lcp_tol 1e-12 from the same state,
    against which the GPU's FP32 step (at the benchmark's tolerance) and FP64
    step (at 1e-12) are compared.  No extrapolation: the figure is the
    oracle's time for a step of this workload."""
    import oracle as O
    th = O.threads(oracle_threads())
    kw = dict(dt=args.dt, eps=args.eps, skin=args.skin, lcp_mode=1)
    t0 = time.time()
    pa, pb = O.broadphase(S["x"], S["kind"], S["shape"], S["box"], args.skin, cells=True)
    t_search = time.time() - t0
    t0 = time.time()
    O.snsd_pairs(pa, pb, S["x"], S["q"], S["kind"], S["shape"], S["box"])
    t_snsd = time.time() - t0
    t0 = time.time()
    r = O.relcp_step(S["x"], S["q"], S["kind"], S["shape"], S["rho_xi"], S["box"], tol=args.tol, **kw)
    t_step = time.time() - t0
    log("oracle step (%d threads): %.2fs (search %.2fs, SNSD at C^k %.2fs), %d rows, %d recursions" %
        (th, t_step, t_search, t_snsd, r["n_rows"], r["recursions"]))
    ref = O.relcp_step(S["x"], S["q"], S["kind"], S["shape"], S["rho_xi"], S["box"], tol=1e-12, **kw)
    errors = {"fp32_at_lcp_tol_%g" % args.tol: gpu_step_error(args, S, 32, args.tol, ref),
              "fp64_at_lcp_tol_1e-12": gpu_step_error(args, S, 64, 1e-12, ref)}
    cpu = {"value": 1.0 / t_step, "unit": "steps/s", "cores": th, "kind": "oracle", "cpu_model": cpu_model(),
           "sample": "one FP64 oracle step (lcp_tol %g, zero start, %d OpenMP threads) on the benchmark's own "
                     "%d-body state at phi %.4f: %.2f s, of which candidate search (cell grid) %.2f s, SNSD of "
                     "the %d candidate pairs at C^k %.2f s, LCP (%d PGD iterations, %d rows) and trial checks the "
                     "rest; %d recursions" % (args.tol, th, len(S["x"]), S["phi"], t_step, t_search, pa.size, t_snsd,
                                               int(sum(r["lcp_iters"])), r["n_rows"], r["recursions"]),
           "seconds": {"step": t_step, "candidate_search": t_search, "snsd_at_Ck": t_snsd}}
    return cpu, errors


def compaction_range(args, C, phi_end=0.60, windows=10):
    """The whole compression from the current volume fraction (~0.40) to
    phi_end at dphi per step (4,000 steps from 0.40), timed per window:
    steps/s, PGD iterations, recursions and rows per step."""
    import torch
    n_total = int(round((phi_end - C.phi) / args.dphi))
    per = max(1, n_total // windows)
    out, tot_t, tot_n, rec = [], 0.0, 0, 0
    done = 0
    while done < n_total:
        k = min(per, n_total - done)
        phi_a = C.phi
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = C.steps(k, args.dphi)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        done += k
        tot_t += el
        tot_n += k
        rec += sum(s["recursions"] for s in st)
        w = {"phi": [round(phi_a, 5), round(C.phi, 5)], "steps": k, "steps_per_s": k / el,
             "pgd_iters_per_step": float(np.mean([s["lcp_iters_total"] for s in st])),
             "recursions_per_step": float(np.mean([s["recursions"] for s in st])),
             "rows": int(st[-1]["n_contacts_final"]), "max_overlap": float(max(s["max_overlap"] for s in st)),
             "residual_fp64_max": float(max(s["residual_fp64"] for s in st))}
        log("range: %s" % w)
        out.append(w)
    return {"steps": tot_n, "steps_per_s": tot_n / tot_t, "recursions_per_step": rec / max(tot_n, 1),
            "windows": out}


def c1_workload(args, precision):
    """The 10,000-ellipsoid compaction: bounding-sphere placement compressed
    (set-up) to volume fraction 0.30, then compressed to 0.55 over 5,000
    timed steps (dphi 5e-5, dt 5e-3, overlap_tol 1e-3, lcp_tol 1e-6)."""
    import torch
    from paper_2506_14097_amd.compaction import Compaction
    C = Compaction(1, 10000, 0.30, dt=args.dt, eps=args.eps, tol=args.tol, precision=precision, skin=args.skin)
    n = int(round((0.55 - C.phi) / args.dphi))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = C.steps(n, args.dphi)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out = {"bodies": 10000, "precision": precision, "phi": [0.30, round(C.phi, 5)], "steps": n,
           "steps_per_s": n / el, "pgd_iters_per_step": float(np.mean([s["lcp_iters_total"] for s in st])),
           "recursions_per_step": float(np.mean([s["recursions"] for s in st])),
           "rows_final": int(st[-1]["n_contacts_final"]), "max_overlap": float(max(s["max_overlap"] for s in st)),
           "residual_fp64_max": float(max(s["residual_fp64"] for s in st))}
    C.sim.close()
    log("10k compaction: %s" % out)
    return out


def colony_workload(args, sizes=(4096, 65536, 131072)):
    """The growing colony (Sec. 5.3) in a monolayer: one spherocylinder
    (diameter 1, total length 1) growing linearly at 0.01 per unit time,
    every cell dividing at total length 2 into its two halves (jitter
    N(0, 0.01^2) rad), dt 1e-2, overlap_tol 1e-3, lcp_tol 1e-6, skin 0.2.
    The set-up grows the colony to each size ten times faster in a context
    with skin 0.5 and at most 20,000 LCP iterations (untimed; the rate is
    halved whenever the rim would still move more than skin / 2 in a step or
    an LCP does not converge).  At each size the state moves to a
    context with the benchmark's skin, takes 5 untimed steps, and a window
    of --colony-steps steps at the benchmarked rate is timed, just after the
    division that reached the size."""
    import torch
    from paper_2506_14097_amd.colony import Colony
    col = Colony(seed=2, rate=0.01, dt=1e-2, eps=args.eps, tol=args.tol, precision=args.precision, skin=0.5,
                 lcp_max_iters=20000)
    out = []
    t0 = time.time()
    for N in sizes:
        col.grow_to(N, rate=0.1, log=log)
        col.reskin(0.2, lcp_max_iters=0)
        for _ in range(5):
            col.step()
        torch.cuda.synchronize()
        t = time.perf_counter()
        st = [col.step() for _ in range(args.colony_steps)]
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        w = {"cells": int(col.n), "steps": args.colony_steps, "steps_per_s": args.colony_steps / el,
             "cell_length": round(col.l + 2 * col.r, 4), "rows": int(st[-1]["n_contacts_final"]),
             "pgd_iters_per_step": float(np.mean([s_["lcp_iters_total"] for s_ in st])),
             "recursions_per_step": float(np.mean([s_["recursions"] for s_ in st])),
             "max_overlap": float(max(s_["max_overlap"] for s_ in st))}
        log("colony: %s (%.1fs)" % (w, time.time() - t0))
        out.append(w)
        col.reskin(0.5, lcp_max_iters=20000)
    col.sim.close()
    return out


def fp64_line(args, state, steps):
    """The benchmark's steps in the FP64 path (FP64 iterations throughout)
    from the same state: steps/s and PGD iterations."""
    import torch
    from paper_2506_14097_amd.compaction import Compaction
    D = Compaction(None, None, None, state=state, dt=args.dt, eps=args.eps, tol=args.tol, precision=64,
                   skin=args.skin)
    D.steps(args.warmup, args.dphi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = D.steps(steps, args.dphi)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    D.sim.close()
    out = {"steps": steps, "steps_per_s": steps / el, "pgd_iters_per_step": float(np.mean([s["lcp_iters_total"]
                                                                                        for s in st])),
           "recursions_per_step": float(np.mean([s["recursions"] for s in st])),
           "residual_fp64_max": float(max(s["residual_fp64"] for s in st))}
    log("FP64 path: %s" % out)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=100000)
    ap.add_argument("--precision", type=int, default=32, choices=(32, 64))
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--phi0", type=float, default=0.40)
    ap.add_argument("--dphi", type=float, default=5e-5)
    ap.add_argument("--dt", type=float, default=5e-3)
    ap.add_argument("--eps", type=float, default=1e-3)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--skin", type=float, default=0.05)
    ap.add_argument("--lcp-mode", type=int, default=0, choices=(0, 1, 2, 3, 4),
                    help="LCP execution: 0 automatic, 1 grid, 2 resident, 3 row graph (graph-replayed passes), "
                         "4 row graph (one launch per pass)")
    ap.add_argument("--roofline-steps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned warm start comparison")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other workloads (FP64 path, the 0.40 -> 0.60 range, 10k compaction, 512 packings)")
    ap.add_argument("--packing-steps", type=int, default=200, help="timed steps of the 512-packing workload")
    ap.add_argument("--colony-steps", type=int, default=200, help="timed steps per colony size")
    ap.add_argument("--learned-steps", type=int, default=50)
    ap.add_argument("--workload", default="compaction100k",
                    choices=("compaction100k", "packings512", "lcp-sweep", "two-ellipsoids", "chainmail", "colony"))
    ap.add_argument("--dts", default="0.1,0.01,0.001,0.0001", help="two-ellipsoids: the timesteps")
    ap.add_argument("--t-end", type=float, default=200.0, help="two-ellipsoids: end time (contact from t = 100)")
    ap.add_argument("--cm-n", type=int, default=5, help="chainmail: node rings per lattice side")
    ap.add_argument("--cm-dt", type=float, default=1e-3, help="chainmail: timestep")
    ap.add_argument("--cm-t-end", type=float, default=10.0, help="chainmail: end time")
    ap.add_argument("--cm-xi", type=float, default=0.1, help="chainmail: drag coefficient")
    ap.add_argument("--cm-jitter", type=float, default=0.05, help="chainmail: placement jitter (rad)")
    ap.add_argument("--cm-lcp-tol", type=float, default=1e-9, help="chainmail: LCP residual tolerance")
    ap.add_argument("--sweep-rows", default="25000,100000,400000,1600000,6400000",
                    help="lcp-sweep: target row counts of the lattice LCPs")
    ap.add_argument("--packings", type=int, default=512)
    ap.add_argument("--copy-probe-mb", type=float, default=0.0,
                    help="only run a device-to-device copy of this many MB (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU only (no multi-GPU path); use --gpus 1", file=sys.stderr)
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
    if args.workload == "packings512":
        print(json.dumps(packings_workload(args)), flush=True)
        return
    if args.workload == "lcp-sweep":
        lcp_sweep(args)
        return
    if args.workload == "chainmail":
        chainmail_study(args)
        return
    if args.workload == "colony":
        print(json.dumps({"metric": "colony steps/s at each size (Sec. 5.3 growth and division)", "unit": "steps/s",
                          "data": "synthetic", "dtype": "f32+f64" if args.precision == 32 else "f64",
                          "sizes": colony_workload(args)}), flush=True)
        return
    if args.workload == "two-ellipsoids":
        two_ellipsoid_study(args)
        return
    R.lib()

    from paper_2506_14097_amd.compaction import Compaction
    t0 = time.time()
    C = Compaction(args.seed, args.n, args.phi0, dt=args.dt, eps=args.eps, tol=args.tol, precision=args.precision,
                   skin=args.skin, log=log)
    sim = C.sim
    log("set-up done: phi %.4f (%.1fs)" % (C.phi, time.time() - t0))
    if args.lcp_mode:
        sim.set_lcp_config(args.lcp_mode)
    start_state = C.state()
    C.steps(args.warmup, args.dphi)
    log("warm-up done, timing %d steps" % args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = C.steps(args.steps, args.dphi)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    value = args.steps / elapsed
    pgd = [s["lcp_iters_total"] for s in stats]
    citers = sum(int(np.dot(s["n_contacts"], s["lcp_iters"])) for s in stats)
    log("timed: %.3f s, %.2f steps/s, PGD iters/step %.1f, host waits/step %.2f (%.3f ms)" %
        (elapsed, value, np.mean(pgd), np.mean([s["n_waits"] for s in stats]),
         np.mean([s["t_wait"] for s in stats])))

    # roofline: kernel durations from HIP events recorded by the library on
    # its stream, over further steps of the same protocol
    sim.set_timing(True)
    sim.get_timing(reset=True)
    rstats = C.steps(args.roofline_steps, args.dphi)
    tm = sim.get_timing(reset=True)
    sim.set_timing(False)
    nb = args.n
    w_lo = 4 if args.precision == 32 else 8
    cls = "lcp_rowgraph" if args.precision == 32 else "lcp_rowgraph64"
    meth, rgm, busy = 0.0, 0.0, 0  # bytes of the iterating passes; launches that did work
    for s_ in rstats:
        for m, it, it64, e in zip(s_["n_contacts"], s_["lcp_iters"], s_["lcp_iters64"], s_["rowgraph_entries"]):
            k = it - it64 if args.precision == 32 else it
            meth += k * method_bytes(m, nb, w_lo)
            rgm += rowgraph_bytes(m, e, w_lo, k) - rowgraph_bytes(m, e, w_lo, 0)
            busy += int(k)
    dom = max(tm, key=lambda k: tm[k][1])
    cnt, ms = tm[cls]
    avg_us = 1e3 * ms / max(cnt, 1)
    achieved = meth / (ms * 1e-3) / 1e9
    traffic = None
    if kernel_source_sha() == MEASURED_TRAFFIC["sha256_prefix"] and args.n == 100000 and args.precision == 32:
        traffic = MEASURED_TRAFFIC["lcp_rowgraph"]
    roof = {"kernel": cls, "kernel_symbol": KERNEL_SYMBOLS.get(cls), "dominant_class": dom, "bound": "hbm",
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "traffic_source": ("rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE of this kernel source (lcp.hip sha256 %s), "
                               "scaled by a plain copy's counters; a profile figure, not measured in this run"
                               % MEASURED_TRAFFIC["sha256_prefix"]) if traffic else None,
            "bytes_model": "method: %d B per row-iteration + %d B per body (26w + 16 B, 14w)" % (26 * w_lo + 16,
                                                                                             14 * w_lo),
            "launches": int(cnt), "busy_launches": int(busy), "avg_us": avg_us,
            "bytes_per_launch": meth / max(cnt, 1),
            "rowgraph_model": {"bytes_per_launch": rgm / max(cnt, 1),
                               "achieved": rgm / (ms * 1e-3) / 1e9, "frac": rgm / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                               "what": "bytes the row-graph pass itself must move: per stored entry its column "
                                       "(4 B) and value (w), per row its state, g, qv and A_rr"}}
    roof["kernel_ms"] = {k: round(v[1], 3) for k, v in tm.items()}
    roof["kernel_launches"] = {k: v[0] for k, v in tm.items()}
    # the narrowphase: FP64 issue rate from the instructions a counter run
    # recorded per pair, over the launch durations measured here
    sc, sms = tm.get("snsd", (0, 0.0))
    pairs = float(np.mean([s_["n_pairs"] for s_ in rstats]))
    narrow = {"kernel": "relcp::k_snsd_pairs<0>", "launches": int(sc), "avg_us": 1e3 * sms / max(sc, 1),
              "pairs_per_launch": pairs, "bound": "fp64 alu", "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s"}
    if geometry_source_sha() == SNSD_FP64_OPS["sha256_prefix"] and sc:
        ops = SNSD_FP64_OPS["fp64_ops_per_pair"] * pairs
        narrow.update(achieved=ops / (sms / sc * 1e-3) / 1e12, fp64_ops_per_pair=SNSD_FP64_OPS["fp64_ops_per_pair"],
                      source=SNSD_FP64_OPS["source"])
        narrow["frac"] = narrow["achieved"] / FP64_PEAK_TFLOPS

    learned = None
    if not args.no_learned:
        learned = learned_comparison(args, start_state)

    extras = {}
    end_state = C.state()
    cpu, errors = None, None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on the benchmark's state")
        s = (C.phi / (C.phi + args.dphi)) ** (1.0 / 3.0)
        S = host_state(end_state, s)
        S["phi"] = C.phi + args.dphi
        cpu, errors = cpu_baseline(args, S)
    if not args.no_extras:
        extras["fp64_path_100k"] = fp64_line(args, start_state, args.steps)
        log("compressing the 100k packing from %.4f to 0.60" % C.phi)
        extras["range_0.40_to_0.60"] = compaction_range(args, C)
        for prec in (64, 32):
            extras["compaction_10k_fp%d" % prec] = c1_workload(args, prec)
        log("512 packings")
        pk = packings_workload(args, steps=args.packing_steps, warmup=2)
        log("colony")
        extras["colony"] = colony_workload(args, sizes=(4096,))
        extras["packings512"] = {k: pk[k] for k in ("value", "unit", "steps", "ms_per_step", "bodies", "packings",
                                                    "lcp_pass_hbm_frac", "pgd_iters_per_step_max_over_packings",
                                                    "contacts_final", "recursions_per_step", "autotune")}

    out = {
        "metric": "ReLCP steps/s @100k ellipsoids; PGD iters to 1e-6 residual (learned vs plain)",
        "value": value, "unit": "steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64" if args.precision == 32 else "f64", "data": "synthetic",
        "config": {"workload": "compaction of %d periodic ellipsoids (semiaxes U[0.5,1]), phi %.2f -> %.5f at "
                               "dphi %.0e/step, overdamped, dt %.0e, overlap_tol %.0e, lcp_tol %.0e, previous-step "
                               "warm start" % (args.n, args.phi0, args.phi0 + args.steps * args.dphi, args.dphi,
                                               args.dt, args.eps, args.tol),
                   "bodies": args.n, "precision": args.precision, "skin": args.skin, "lcp_mode": args.lcp_mode},
        "pgd_iters_per_step": {"plain": float(np.mean(pgd)),
                               "learned": learned["levels"]["0.40"]["learned"]["pgd_iters_per_step"]
                               if learned else None},
        "error_vs_oracle": errors,
        "learned_warm_start": learned,
        "contact_iters_per_s": citers / elapsed,
        "host_waits_per_step": {"n": float(np.mean([s_["n_waits"] for s_ in stats])),
                                "ms": float(np.mean([s_["t_wait"] for s_ in stats]))},
        "recursions_per_step": float(np.mean([s_["recursions"] for s_ in stats])),
        "contacts_final": int(stats[-1]["n_contacts_final"]),
        "residual_fp64_max": float(max(s_["residual_fp64"] for s_ in stats)),
        "max_overlap": float(max(s_["max_overlap"] for s_ in stats)),
        "roofline": roof,
        "narrowphase": narrow,
        "workloads": extras,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
