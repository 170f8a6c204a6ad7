"""Benchmark: steady gray GSIS on one MI355X.

Workload (default): 256 x 256 cells, 128 ordinates (4 Gauss-Legendre polar x
32 Chebyshev azimuthal), thick square sigma_t = 1e3, c = 0.9999 inside,
sigma_t = 1, c = 0.5 outside, unit source in the thick region, vacuum, FP64,
Barth-Jespersen limiter on. A step is one outer GSIS iteration (transport
residual + sweep + moments, boundary fluxes + HoT + synthetic right-hand side,
CG/multigrid synthetic solve, correction + Err) on resident device data.
``--config block1024 [--precision fp32]`` times the 1024 x 1024 x 128 block
medium instead (the configuration whose intensities do not fit the 256 MB
last-level cache), for profiling.

Prints ONE JSON line. value = cell-ordinate updates per second over the timed
steps (nx*ny*K per step). The roofline object charges the transport step's
algorithmic bytes (one read of I^m and one write of I^{m+1/2} per
cell-ordinate: 16 B in FP64, 8 B in FP32-mixed) to the transport step as a
whole, the residual kernel plus the wavefront recurrence, or the pipelined
kernel where it runs (their durations come from HIP events recorded on the
plan's stream around each launch, in a second pass of the same steps on a
plan that records them; the timed steps themselves run without events), and
lists each kernel with its measured HBM traffic; the synthetic solve and the
whole iteration are reported beside it.
Also reported: time-to-converge (Err < 1e-6) for GSIS and for source
iteration, the three additions against the plain FP64 form, and, in the CPU
leg, the oracle timed on a bounded sample of the same workload and the
oracle's fixed points the GPU results are compared with.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
ALG_BYTES = {"fp64": 16.0, "fp32": 8.0}
# Algorithmic bytes of one synthetic CG iteration per cell of the finest
# level: the CG update reads x, r, p, s, z, w and writes x, r, p, s (80 B);
# the V-cycle's level-0 smoothing and restriction read r and the 5-point
# operator (diag, ax, ay) and write the pre-smoothed iterate and the
# restricted residual (48 B); its prolongation and post-smoothing read the
# pre-smoothed iterate, the operator and r and write z and w = A z (56 B);
# the coarser levels add a third of the finest level's V-cycle traffic.
SYNTH_BYTES_PER_CELL = 80.0 + (48.0 + 56.0) * 4.0 / 3.0
# Relative tolerance of the synthetic CG per outer iteration (the library's
# default): the fastest time to Err < 1e-6 on this workload among 3e-3 ..
# 0.5 (outer iterations / ms to converge / V-cycles per iteration: 3e-3
# 24 / 9.9 / 5.7; 1e-2 32 / 11.9 / 4.6; 3e-2 34 / 11.6 / 4.0; 0.1 28 / 8.7 /
# 3.0; 0.2 30 / 9.2 / 2.9; 0.3 60 / 16.7 / 2.0). The fixed point does not
# depend on it.
SYNTH_RTOL = 0.1

# HBM traffic per launch of the transport kernels, per timed configuration,
# from two rocprofv3 --pmc runs of "bench.py --config <cfg> --precision <p>
# --steps 3 --warmup 1 --no-converge --no-cpu-baseline --no-forms"
# (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), scaled by what the same
# counters read for a 256 MiB device copy (bench.py --copy-calibration: it
# reads 131084.5 KiB of FETCH_SIZE and 262144 KiB of WRITE_SIZE per dispatch,
# so FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0). Valid only for the build whose
# traffic_key() is recorded; any change to it turns the figures back to null.
TRAFFIC = {
    "thick256_fp64": {"sha256": "87b8dd5c5c0bb5a95f7669edeab150399734c57078e5c4d7b3c1cf5eb4da77cf",
                      "k_resid": 244573448,     # 84267.8 KiB x 2.0 + 70305.6 KiB
                      "k_chain": 138782520},    # 34856.4 KiB x 2.0 + 65817.0 KiB
    "block1024_fp64": {"sha256": "87b8dd5c5c0bb5a95f7669edeab150399734c57078e5c4d7b3c1cf5eb4da77cf",
                       "k_pipe": 3179074724},   # 980894.8 KiB x 2.0 + 1142775.5 KiB
    "block1024_fp32": {"sha256": "87b8dd5c5c0bb5a95f7669edeab150399734c57078e5c4d7b3c1cf5eb4da77cf",
                       "k_resid": 2965954644,   # 1153944.9 KiB x 2.0 + 588550.3 KiB
                       "k_chain": 1283219692},  # 347933.3 KiB x 2.0 + 557277.6 KiB
}
KERNELS = {"k_resid": "k_resid (second-order residual of every cell-ordinate, ALSM gradient "
                      "and BJ limiter, written as the recurrence's right-hand side)",
           "k_chain": "k_chain / k_chain_split (first-order-upwind recurrence on the "
                      "anti-diagonal wavefront)",
           "k_pipe": "k_pipe (pipelined transport step: residual waves pass the recurrence's "
                     "right-hand side to recurrence waves through LDS, one launch)"}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def cpu_leg(prob, n_iter, inputs, with_refs):
    """The CPU leg: the FP64 oracle (as it stands) timed for up to n_iter
    GSIS iterations of the same workload on this host's cores, stopping at
    Err < 1e-6 (the same options as the GPU's timed steps, limiter on); its
    converged fields are the reference of the headline solve. With
    with_refs, also the oracle's FP64 fixed point of the block medium at
    256 x 256 x 128 (beta 10, limiter off, Err < 1e-6), the reference of the
    FP32-mixed form."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    r = oracle.solve(prob, method=1, tol=1e-6, max_iter=n_iter)
    dt = time.perf_counter() - t0
    N, K = prob["nx"] * prob["ny"], len(prob["mu"])
    omp = os.environ.get("OMP_NUM_THREADS")
    used = min(cores, int(omp)) if omp and omp.isdigit() else cores
    base = {"value": N * K * r["n_iter"] / dt, "unit": "cell-ordinate updates/s", "cores": used,
            "kind": "oracle",
            "sample": "%d GSIS iterations (Err %.2e) of the full %dx%dx%d workload from I=0 "
                      "(incl. one banded-Cholesky factorisation), %.1f s" % (
                          r["n_iter"], r["final_err"], prob["nx"], prob["ny"], K, dt)}
    refs = {"headline": r}
    if with_refs:
        t0 = time.perf_counter()
        refs["block256"] = oracle.solve(inputs.checkerboard_blocks(256), method=1, tol=1e-6,
                                        max_iter=500, beta=10.0, limiter=0)
        log("oracle block medium 256: %d iterations, %.1f s" % (
            refs["block256"]["n_iter"], time.perf_counter() - t0))
    return base, refs


def measure_controls(ctx, gsis, pd, opts, N, K, args, phases, nprof, achieved, torch, dev,
                     tr_ms):
    """The transport step alone (residual + recurrence) as cell-ordinate
    updates/s, the same steps with the limiter off (the residual's arithmetic
    control), and a measured copy ceiling: a 1 GiB FP64 device copy, bytes
    read + written per second, with the transport step's algorithmic rate as
    a fraction of it."""
    n = max(nprof, 1)
    res = {"transport": {"kernels": "residual + recurrence", "ms": tr_ms,
                         "cell_ordinate_updates_per_s": N * K / (tr_ms / 1e3)}}
    plan = gsis.Plan(ctx, pd, tol=0.0, max_iter=args.steps + args.warmup + 1, profile=1,
                     **dict(opts, limiter=0))
    plan.iterate(args.warmup)
    torch.cuda.synchronize()
    plan.reset()
    plan.phase_times()
    plan.iterate(args.steps)
    torch.cuda.synchronize()
    ph, m = plan.phase_times()
    plan.close()
    m = max(m, 1)
    res["limiter_off"] = {"residual_ms": ph["residual"] / m, "sweep_ms": ph["sweep"] / m,
                          "limiter_on_residual_ms": phases["residual"] / n}
    x = torch.ones(128 << 20, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(10):
        y.copy_(x)
    e1.record(stream)
    torch.cuda.synchronize()
    gbs = 2 * x.numel() * 8 * 10 / (e0.elapsed_time(e1) / 1e3) / 1e9
    del x, y
    res["copy_ceiling"] = {"GB_per_s": gbs, "transport_frac_of_copy": achieved / gbs}
    log("controls: %s" % res)
    return res


def traffic_key():
    """sha256 of what the transport kernels are built from: their source, the
    device header it includes and the compile flags (include paths aside)."""
    from paper_2507_03975_amd import build
    h = hashlib.sha256()
    for name in ("kernels_transport.hip", "wave_ops.h"):
        with open(os.path.join(ROOT, "paper_2507_03975_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    h.update(" ".join(a for a in build.COMMON if not a.startswith("-I")).encode())
    return h.hexdigest()


def kernel_traffic(cfg, kernel):
    """Bytes per launch of a transport kernel from the PMC runs of this
    configuration, if the kernels are built as they were when those runs
    were taken (traffic_key)."""
    t = TRAFFIC.get(cfg)
    if not t or t.get(kernel) is None:
        return None
    if traffic_key() != t["sha256"]:
        return None
    return t[kernel]


def _converge(pl, cap, chunk=16):
    """Iterate a plan or batch until it stops; returns wall seconds."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while True:
        pl.iterate(min(chunk, cap - done))
        done += min(chunk, cap - done)
        st = pl.status()
        if hasattr(pl, "tuning"):
            if st[3] == pl.n or done >= cap:
                break
        elif st[1] != 0 or done >= cap:
            break
    return time.perf_counter() - t0


def _rel(a, b):
    return float((a - b).abs().max() / b.abs().max())


def measure_forms(ctx, gsis, inputs, np, torch, dev):
    """FP32-mixed, batched and adjoint forms against the plain FP64 form."""
    dv = lambda p: {k: (torch.from_numpy(v).to(dev) if isinstance(v, np.ndarray) else v)
                    for k, v in p.items()}
    forms = {}
    # FP32-mixed and FP64 fixed points of the block medium at 256 x 256 x 128,
    # kept for the comparison with the oracle's (CPU leg); the synthetic
    # solves run to 1e-8 like the oracle's direct solve, so that the
    # difference shows the storage precision and not where the outer stop
    # lands
    p256 = dv(inputs.checkerboard_blocks(256))
    fp256 = {}
    for name, prec in (("fp64", gsis.GSIS_FP64), ("fp32_mixed", gsis.GSIS_FP32_MIXED)):
        pl = gsis.Plan(ctx, p256, precision=prec, tol=1e-6, max_iter=500, limiter=0, beta=10.0,
                       synth_rtol=1e-8, synth_max_iter=200)
        _converge(pl, 500)
        f = pl.read()
        fp256[name] = {k: f[k].cpu().numpy() for k in ("phi", "Fx", "Fy")}
        pl.close()
    del p256
    # FP32-mixed: 1024 x 1024 x 128 block medium (local pseudo time beta = 10)
    pc = dv(inputs.checkerboard_blocks(1024))
    res = {}
    for name, prec in (("fp64", gsis.GSIS_FP64), ("fp32_mixed", gsis.GSIS_FP32_MIXED)):
        pl = gsis.Plan(ctx, pc, precision=prec, tol=1e-6, max_iter=1000, limiter=0, beta=10.0)
        sec = _converge(pl, 1000)
        n, conv, err = pl.status()
        res[name] = dict(iterations=int(n), seconds=sec, converged=bool(conv == 1),
                         fields=pl.read())
        pl.close()
        log("block medium %s: %d iterations, %.3f s" % (name, n, sec))
    a, b = res["fp32_mixed"]["fields"], res["fp64"]["fields"]
    forms["fp32_mixed"] = {
        "workload": "1024x1024 cells, 128 ordinates, 7x7 blocks sigma_a logU[1e-2,1e2] "
                    "sigma_s logU[1e-1,1e4] (seed 3), beta 10, limiter off, Err < 1e-6",
        "fp64": {k: v for k, v in res["fp64"].items() if k != "fields"},
        "fp32_mixed": {k: v for k, v in res["fp32_mixed"].items() if k != "fields"},
        "time_ratio_fp32_over_fp64": res["fp32_mixed"]["seconds"] / res["fp64"]["seconds"],
        "error_vs_gpu_fp64": {"phi": _rel(a["phi"], b["phi"]), "Fx": _rel(a["Fx"], b["Fx"]),
                              "Fy": _rel(a["Fy"], b["Fy"])},
        "block256_fields": fp256}
    del res, a, b, pc
    # batched: 64 uneven problems in one batch vs 64 sequential plain FP64 solves
    probs = [dv(p) for p in inputs.batch_problems()]
    co = sum(int(p["nx"]) * int(p["ny"]) * len(p["mu"]) for p in probs)
    kw = dict(tol=1e-6, max_iter=1500, limiter=0, beta=20.0)
    bres = {}
    for name, prec in (("batch_fp64", gsis.GSIS_FP64), ("batch_fp32_mixed", gsis.GSIS_FP32_MIXED)):
        t0 = time.perf_counter()
        bt = gsis.Batch(ctx, probs, precision=prec, **kw)
        setup = time.perf_counter() - t0
        bt.iterate(3)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        bt.iterate(10)
        bt.status()
        it_ms = (time.perf_counter() - t1) * 100.0
        bt.reset()
        sec = _converge(bt, 1500, chunk=20)
        its, conv, err, fin = bt.status()
        bres[name] = dict(seconds=sec, setup_seconds=setup, ms_per_iteration=it_ms,
                          cell_ordinate_updates_per_s=co / (it_ms / 1e3),
                          max_iterations=int(max(its)),
                          converged=int(sum(1 for c in conv if c == 1)), tuning=bt.tuning())
        bt.close()
        log("batch %s: %.3f s, %.2f ms/iteration" % (name, sec, it_ms))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p in probs:
        gsis.gsis_solve(ctx, p, **kw)
    torch.cuda.synchronize()
    seq = time.perf_counter() - t0
    log("sequential plain FP64 solves: %.3f s" % seq)
    forms["batched"] = {
        "workload": "64 problems, nx, ny in {64..512}, 32-128 ordinates, 8x8 blocks sigma_t "
                    "logU[0.1,1e4], c U[0.5,0.9999] (seed 4), beta 20, limiter off, Err < 1e-6",
        "cell_ordinates_per_iteration": co,
        "sequential_plain_fp64_seconds": seq, **bres,
        "speedup_batch_fp64_over_sequential": seq / bres["batch_fp64"]["seconds"]}
    del probs
    # adjoint: 512 x 512 x 128 noisy two-region medium, detector objective
    pa = inputs.noisy_thick_square(512)
    W = torch.from_numpy(inputs.detector_window(512)).to(dev)
    pd = dv(pa)
    V = pa["dx"] * pa["dy"]
    gphi = torch.where(W, V * pd["sigma_a"], torch.zeros_like(pd["sigma_a"]))
    pl = gsis.Plan(ctx, pd, tol=1e-6, max_iter=2000, limiter=0)
    fsec = _converge(pl, 2000)
    n, conv, err = pl.status()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ga, gs, gq, info = pl.adjoint(gphi, tol=1e-6, max_iter=2000)
    torch.cuda.synchronize()
    asec = time.perf_counter() - t0
    pl.close()
    log("adjoint: forward %d its %.3f s, adjoint %d its %.3f s" % (n, fsec, info["n_iter"], asec))
    forms["adjoint"] = {
        "workload": "512x512 cells, 128 ordinates, two-region medium with +-20% noise (seed 5), "
                    "J = sum over the 32x32 detector of V sigma_a phi, limiter off, Err < 1e-6",
        "forward": {"iterations": int(n), "seconds": fsec},
        "adjoint": {"iterations": info["n_iter"], "seconds": asec},
        "adjoint_over_forward_time": asec / fsec}
    # time-dependent form (backward Euler with the material energy equation)
    # on the headline medium: GSIS and SI time steps, each to Err < 1e-6
    ptd = dv(inputs.thick_square(256))
    ntd = int(ptd["nx"]) * int(ptd["ny"]) * int(ptd["mu"].shape[0])
    td = {"workload": "thick square 256x256x128 as the timed steps, with emission and the "
                      "material energy equation: c = 1, a = 1, cv = 1, T0 = 0.1, 3 sub-iterations "
                      "per inner iteration, Err < 1e-6 per step (SI capped at 300 inner "
                      "iterations); one untimed step first, then 5 (GSIS) or 2 (SI) timed steps"}
    for cdt in (0.01, 1.0):
        row = {}
        for name, method, cap, steps in (("gsis", gsis.GSIS_GSIS, 500, 5), ("si", gsis.GSIS_SI, 300, 2)):
            pl = gsis.TDPlan(ctx, ptd, 0.1, c=1.0, a=1.0, dt=cdt, cv=1.0, sub_iter=3, method=method,
                             tol=1e-6, max_iter=cap, limiter=1, synth_rtol=SYNTH_RTOL,
                             synth_max_iter=50)
            pl.advance(1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, its, errs = pl.advance(steps)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            pl.close()
            row[name] = {"status": int(st), "inner_iterations": [int(v) for v in its],
                         "converged": bool(all(e < 1e-6 for e in errs)),
                         "seconds_per_step": sec / steps,
                         "ms_per_inner_iteration": sec / max(sum(its), 1) * 1e3,
                         "cell_ordinate_updates_per_s": ntd * sum(its) / sec}
        row["si_over_gsis_inner_iterations"] = (sum(row["si"]["inner_iterations"]) / 2) / (
            sum(row["gsis"]["inner_iterations"]) / 5)
        td["c_dt_%g" % cdt] = row
        log("time-dependent c dt = %g: GSIS %s, SI %s" % (cdt, row["gsis"]["inner_iterations"],
                                                          row["si"]["inner_iterations"]))
    forms["time_dependent"] = td
    del ptd
    # pseudo-time shift (local tau_p with beta, Eqs. tau_pse, elem_main_shifted)
    # on the block medium, whose 1e5 opacity contrasts make plain GSIS diverge
    pb = dv(inputs.checkerboard_blocks(256))
    pt = {"workload": "block medium 256x256x128 (7x7 blocks sigma_a logU[1e-2,1e2] sigma_s "
                      "logU[1e-1,1e4], seed 3), GSIS, limiter off, Err < 1e-6, at most 500 "
                      "iterations"}
    for beta in (0.0, 10.0):
        pl = gsis.Plan(ctx, pb, tol=1e-6, max_iter=500, limiter=0, beta=beta)
        sec = _converge(pl, 500)
        n, conv, err = pl.status()
        pl.close()
        pt["beta_%g" % beta] = {"iterations": int(n), "seconds": sec, "final_err": float(err),
                                "outcome": {1: "converged", -1: "diverged"}.get(int(conv),
                                                                               "not converged")}
        log("pseudo time beta %g: %d iterations, %s" % (beta, n, pt["beta_%g" % beta]["outcome"]))
    forms["pseudo_time"] = pt
    del pb
    # face-averaged synthetic flux (Eq. Fij_d) by sub-iterations against the
    # compact flux, on the headline workload
    pc = dv(inputs.thick_square(256))
    base = dict(method=gsis.GSIS_GSIS, limiter=1, tol=1e-6, max_iter=500, synth_rtol=SYNTH_RTOL,
                synth_max_iter=50)
    res = {}
    for name, extra in (("compact", {}), ("face_average_sub2", dict(synth_form=1, synth_sub=2)),
                        ("face_average_sub4", dict(synth_form=1, synth_sub=4))):
        pl = gsis.Plan(ctx, pc, **dict(base, **extra))
        sec = _converge(pl, 500)
        n, conv, err = pl.status()
        res[name] = dict(iterations=int(n), seconds=sec, converged=bool(conv == 1),
                         phi=pl.read()["phi"])
        pl.close()
        log("synthetic flux %s: %d iterations, %.4f s" % (name, n, sec))
    ref = res["compact"]["phi"]
    forms["synthetic_flux"] = {
        "workload": "thick square 256x256x128 as the timed steps, GSIS to Err < 1e-6",
        **{k: {**{a: b for a, b in v.items() if a != "phi"},
               "phi_rel_diff_vs_compact": _rel(v["phi"], ref)} for k, v in res.items()}}
    return forms


def paper_2d_table(ctx, gsis, inputs, np, torch, dev):
    """The paper's 2D steady experiment (Sec. 5.2.1, Table table:2d_const):
    uniform pure scatterer, hot bottom wall (1/(4 pi)), other walls
    1e-6/(4 pi), 40x40 and 100x100 cells, Gauss-Legendre 36 x 48 with the
    polar axis along x (1728 ordinates), Err < 1e-6, limiter off. GSIS and SI
    iteration counts and GPU seconds (plan set-up excluded; synthetic CG to
    relative residual 1e-8)."""
    quad = inputs.quad_gl_product_full(36, 48)
    rows = []
    for n in (40, 100):
        for st in (0.2, 1.0, 10.0, 20.0, 50.0, 100.0):
            p = inputs.hot_wall_square(n, st, quad)
            pd = {k: (torch.from_numpy(v).to(dev) if isinstance(v, np.ndarray) else v)
                  for k, v in p.items()}
            row = {"cells": "%dx%d" % (n, n), "sigma_t": st}
            for name, method in (("gsis", gsis.GSIS_GSIS), ("si", gsis.GSIS_SI)):
                pl = gsis.Plan(ctx, pd, method=method, tol=1e-6, max_iter=20000, limiter=0,
                               synth_rtol=1e-8, synth_max_iter=200)
                sec = _converge(pl, 20000, chunk=64)
                it, conv, err = pl.status()
                pl.close()
                row[name] = {"iterations": int(it), "seconds": sec, "converged": bool(conv == 1)}
            rows.append(row)
            log("paper 2D %s sigma_t %g: GSIS %d its %.3f s, SI %d its %.3f s" % (
                row["cells"], st, row["gsis"]["iterations"], row["gsis"]["seconds"],
                row["si"]["iterations"], row["si"]["seconds"]))
    return {"workload": "hot bottom wall, uniform pure scatterer, GL 36x48 (K = 1728), "
                        "Err < 1e-6, limiter off", "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-converge", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=40)
    ap.add_argument("--config", choices=("thick256", "block1024"), default="thick256",
                    help="timed workload: the 256x256x128 thick square (default) or the "
                         "1024x1024x128 block medium (timed steps only)")
    ap.add_argument("--precision", choices=("fp64", "fp32"), default="fp64")
    ap.add_argument("--si-cap", type=int, default=3000)
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the FP32-mixed, batched and adjoint measurements")
    ap.add_argument("--paper-2d", action="store_true",
                    help="only run the paper's 2D hot-wall table (GSIS and SI iteration "
                         "counts and GPU seconds, 40x40 and 100x100, six opacities)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy five times (the known-size "
                         "kernel that scales the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2507_03975_amd import gsis, inputs

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        n = 32 << 20
        x = torch.ones(n, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n, "copies": 5}))
        return
    if args.paper_2d:
        print(json.dumps({"paper_2d": paper_2d_table(gsis.Context(0), gsis, inputs, np, torch,
                                                     dev)}), flush=True)
        return
    block = args.config == "block1024"
    fp32 = args.precision == "fp32"
    if block:
        prob = inputs.checkerboard_blocks(1024)
        opts = dict(method=gsis.GSIS_GSIS, limiter=0, beta=10.0)
        wname = ("GSIS %s, 1024x1024 cells, 128 ordinates (GL4x Chebyshev32), 7x7 blocks "
                 "sigma_a logU[1e-2,1e2] sigma_s logU[1e-1,1e4] (seed 3), unit source, vacuum, "
                 "beta 10, limiter off" % ("FP32-mixed" if fp32 else "FP64"))
    else:
        prob = inputs.thick_square(256)
        opts = dict(method=gsis.GSIS_GSIS, limiter=1)
        wname = ("GSIS %s, 256x256 cells, 128 ordinates (GL4x Chebyshev32), thick square "
                 "sigma_t=1e3 c=0.9999 in sigma_t=1 c=0.5, unit source in the thick region, "
                 "vacuum, BJ limiter" % ("FP32-mixed" if fp32 else "FP64"))
    opts.update(synth_rtol=SYNTH_RTOL, synth_max_iter=50,
                precision=gsis.GSIS_FP32_MIXED if fp32 else gsis.GSIS_FP64)
    N, K = prob["nx"] * prob["ny"], len(prob["mu"])
    pd = {k: (torch.from_numpy(v).to(dev) if isinstance(v, np.ndarray) else v)
          for k, v in prob.items()}
    ctx = gsis.Context(0)

    # ---- timed steps: K outer iterations from the initial state, on a plan
    # that records no events between its launches (the headline rate)
    plan = gsis.Plan(ctx, pd, tol=0.0, max_iter=args.steps + args.warmup + 1, **opts)
    plan.iterate(args.warmup)
    torch.cuda.synchronize()
    plan.reset()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    plan.iterate(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    n_done = plan.status()[0]
    vcycles = plan.synth_vcycles()
    form, bands, parts = plan.transport_form()
    pipelined = form == 3
    assert n_done == args.steps, (n_done, args.steps)
    plan.close()
    # ---- the same K steps on a plan that records HIP events on its stream
    # around every phase's launches: the phase and kernel durations (the
    # events themselves cost a few microseconds each, so they stay out of the
    # headline steps)
    prof = gsis.Plan(ctx, pd, tol=0.0, max_iter=args.steps + args.warmup + 1, profile=1, **opts)
    prof.iterate(args.warmup)
    torch.cuda.synchronize()
    prof.reset()
    prof.phase_times()
    prof.iterate(args.steps)
    torch.cuda.synchronize()
    phases, nprof = prof.phase_times()
    assert prof.status()[0] == args.steps
    prof.close()
    ms_step = ms / args.steps
    value = N * K * args.steps / (ms / 1e3)
    nprof = max(nprof, 1)
    per = {k: v / nprof for k, v in phases.items()}
    alg = ALG_BYTES[args.precision] * N * K           # one read of I^m, one write of I^{m+1/2}
    # the pipelined step is one launch in the sweep phase (the residual
    # phase then holds no kernel, only its two events)
    tr_ms = per["sweep"] if pipelined else per["residual"] + per["sweep"]
    achieved = alg / (tr_ms / 1e3) / 1e9
    cfg_key = "%s_%s" % (args.config, args.precision)
    kern = {}
    launches = ([("transport", "k_pipe", per["sweep"])] if pipelined else
                [("residual", "k_resid", per["residual"]), ("sweep", "k_chain", per["sweep"])])
    for ph, name, ms_k in launches:
        t = kernel_traffic(cfg_key, name)
        kern[ph] = {"kernel": KERNELS[name], "avg_ms": ms_k, "traffic": t,
                    "traffic_over_transport_algorithmic": None if t is None else t / alg}
    traffic = None
    if all(k["traffic"] is not None for k in kern.values()):
        traffic = sum(k["traffic"] for k in kern.values())
    vc_step = vcycles / args.steps
    synth_bytes = SYNTH_BYTES_PER_CELL * N * vc_step
    log("step %.3f ms; phases per step (ms): %s; V-cycles per step %.2f" % (
        ms_step, {k: round(v, 4) for k, v in per.items()}, vc_step))

    out = {
        "metric": "cell-ordinate updates/s; time-to-converge GSIS vs SI at rel resid 1e-6",
        "value": value,
        "unit": "cell-ordinate updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if fp32 else "f64",
        "data": "synthetic",
        "config": {"workload": wname, "nx": prob["nx"], "ny": prob["ny"], "ordinates": K,
                   "method": "GSIS", "step": "one outer iteration"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": ("transport step: k_pipe, residual and recurrence in one "
                                "launch (Eqs. RTE_d_res..elem_mtx; %d bands of 64 rows, %d "
                                "parts)" % (bands, parts)) if pipelined else
                               "transport step: k_resid + recurrence (the two launches of "
                               "Eqs. RTE_d_res..elem_mtx)",
                     "algorithmic_bytes_per_launch": alg,
                     "algorithmic_bytes_per_cell_ordinate": ALG_BYTES[args.precision],
                     "avg_ms": tr_ms, "kernels": kern,
                     "whole_iteration": {"ms": ms_step,
                                         "achieved": alg / (ms_step / 1e3) / 1e9,
                                         "frac": alg / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS},
                     "synthetic": {"ms": per["synth"], "vcycles_per_step": vc_step,
                                   "algorithmic_bytes_per_cell_per_cg_iteration":
                                       SYNTH_BYTES_PER_CELL,
                                   "achieved": synth_bytes / (per["synth"] / 1e3) / 1e9
                                   if per["synth"] > 0 else None,
                                   "frac": synth_bytes / (per["synth"] / 1e3) / 1e9 /
                                   HBM_PEAK_GBS if per["synth"] > 0 else None}},
        "phase_ms_per_step": per,
    }
    if block:
        print(json.dumps(out), flush=True)
        return

    # ---- time to converge (Err < 1e-6), GSIS vs SI on the same GPU
    gsis_phi = None
    if not args.no_converge:
        res = {}
        for name, method, cap in (("gsis", gsis.GSIS_GSIS, 500), ("si", gsis.GSIS_SI, args.si_cap)):
            o2 = dict(opts, method=method)
            pl = gsis.Plan(ctx, pd, tol=1e-6, max_iter=cap, **o2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            done = 0
            while True:
                pl.iterate(min(64, cap - done))
                n, conv, err = pl.status()
                done = n
                if conv != 0 or n >= cap:
                    break
            dt = time.perf_counter() - t0
            r = pl.read()
            pl.close()
            hist = r["err_hist"].cpu().numpy() if hasattr(r["err_hist"], "cpu") else r["err_hist"]
            th = r["tres_hist"].cpu().numpy() if hasattr(r["tres_hist"], "cpu") else r["tres_hist"]
            ent = {"iterations": int(n), "seconds": dt, "final_err": float(err),
                   "converged": bool(conv == 1),
                   "final_transport_residual": float(th[-1]) if len(th) else None}
            if name == "gsis":
                gsis_phi = {k: r[k].cpu().numpy() for k in ("phi", "Fx", "Fy")}
            if conv != 1 and len(hist) > 200:
                tail = hist[-200:]
                rho = float(np.exp(np.mean(np.log(tail[1:] / tail[:-1]))))
                if 0 < rho < 1:
                    more = math.log(1e-6 / hist[-1]) / math.log(rho)
                    ent.update(extrapolated=True, contraction=rho,
                               iterations_extrapolated=int(n + more),
                               seconds_extrapolated=dt * (n + more) / n)
            res[name] = ent
            log("%s: %s" % (name, ent))
        g, s = res["gsis"], res["si"]
        s_sec = s.get("seconds_extrapolated", s["seconds"])
        out["time_to_converge"] = {"tol": 1e-6, "synth_rtol": SYNTH_RTOL, "gsis": g, "si": s,
                                   "si_over_gsis_time": s_sec / g["seconds"]}

    if not args.no_forms:
        out["controls"] = measure_controls(ctx, gsis, pd, opts, N, K, args, phases, nprof,
                                           achieved, torch, dev, tr_ms)
        out["forms"] = measure_forms(ctx, gsis, inputs, np, torch, dev)
    f256 = out.get("forms", {}).get("fp32_mixed", {}).pop("block256_fields", None)

    if not args.no_cpu_baseline:
        log("cpu leg: oracle, up to %d iterations" % args.cpu_iters)
        base, refs = cpu_leg(prob, args.cpu_iters, inputs, f256 is not None)
        out["cpu_baseline"] = base
        relnp = lambda a, b: float(np.abs(a - b).max() / np.abs(b).max())
        o = refs["headline"]
        if gsis_phi is not None and o["final_err"] < 1e-6:
            out["time_to_converge"]["gsis"]["error_vs_oracle"] = {
                "oracle_iterations": int(o["n_iter"]),
                **{k: relnp(gsis_phi[k], o[k]) for k in ("phi", "Fx", "Fy")}}
        if f256 is not None and refs.get("block256", {}).get("status") == 0:
            o = refs["block256"]
            out["forms"]["fp32_mixed"]["error_vs_oracle"] = {
                "workload": "the same block medium at 256x256 cells, 128 ordinates, both "
                            "converged to Err < 1e-6 (oracle %d iterations; GPU synthetic "
                            "solves to 1e-8)" % o["n_iter"],
                **{prec: {k: relnp(f256[prec][k], o[k]) for k in ("phi", "Fx", "Fy")}
                   for prec in ("fp64", "fp32_mixed")}}

    print(json.dumps(out), flush=True)

if __name__ == "__main__":
    main()
