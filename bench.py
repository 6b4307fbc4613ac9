"""Benchmark of the co-evolving-subspace step on one MI355X.

Workload: the 1D Holstein ring of 16 sites (one mode per site, omega 1,
g 1.2, J -1, cutoff 12, k=0 Bloch start, dt 0.01, neighbour order 4,
amplitude threshold 1e-8, complex128), synthetic inputs only.  A "step" is
one full time step of the hot path: select, expand (4 rounds), merge,
transfer, build, Chebyshev propagation and observables.  The run starts
from the initial state; `--warmup` steps grow the subspace untimed, then
exactly `--steps` steps are timed between stream synchronisations.

value = sum over timed steps of |S| / wall time (basis-state updates/s).
roofline: the middle Clenshaw term kernel (the dominant kernel), its
algorithmic bytes per launch |S| (4A + 4D + 8) over its HIP-event
duration on the step's stream, from one middle launch per timed step whose
dispatch records the events.
cpu_baseline: the CPU oracle continued from the GPU state at the start of
the timed window, for a bounded number of steps.
forms: the extra forms against plain FP64 single-realization runs on the
same GPU: complex64 amplitudes on the same window; the order-10 Krylov
propagator and the truncated Taylor series on the same window from the
same state; 64 disorder
realizations of the 6x6 lattice in one sim against realizations run one
after another; the adjoint gradient of the 12-site ring against its plain
forward run (time ratio).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=130)
    ap.add_argument("--config", default="ring16")
    ap.add_argument("--precision", type=int, default=64)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--tune", default="auto", choices=["auto", "none"],
                    help="run the library's launch autotuner on the warmed-up "
                         "state before timing (results do not depend on it)")
    ap.add_argument("--batch-steps", type=int, default=40)
    ap.add_argument("--batch-singles", type=int, default=8)
    ap.add_argument("--adjoint-steps", type=int, default=200)
    ap.add_argument("--krylov-order", type=int, default=10)
    ap.add_argument("--stage-steps", type=int, default=5)
    ap.add_argument("--paper-1d", type=float, default=None, metavar="G",
                    help="instead of the benchmark, run the paper's 1D "
                         "calculation at coupling G (its table of 1D runs: "
                         "N, d_pho, q_nom per g; m_init 10, m 2, dt 0.05, "
                         "t = 50) and print one JSON line with its wall "
                         "time and q_true / q_nom")
    ap.add_argument("--q-nom", type=float, default=None,
                    help="q_nom of --paper-1d (default: the paper's)")
    ap.add_argument("--paper-steps", type=int, default=None,
                    help="steps of --paper-1d / --paper-agg (default: the "
                         "paper's, 1000 / 2000)")
    ap.add_argument("--paper-agg", default=None, metavar="DIMS",
                    help="instead of the benchmark, run the paper's "
                         "aggregate calculation on lattice DIMS (e.g. 64, "
                         "8x8, 2x2x2), H aggregate unless --paper-kind J")
    ap.add_argument("--paper-kind", default="H", choices=["H", "J"])
    ap.add_argument("--paper-krylov", type=int, default=0, metavar="P",
                    help="--paper-1d / --paper-agg with the order-P Krylov "
                         "propagator instead of the series")
    ap.add_argument("--paper-taylor", type=int, default=0, metavar="N",
                    help="--paper-1d / --paper-agg with the truncated Taylor "
                         "propagator: N > 0 a fixed order, -1 the adaptive "
                         "degree and substep choice")
    ap.add_argument("--paper-save", default=None, metavar="FILE",
                    help="save the run's per-step records (.npy, fields as "
                         "in the library's observation record)")
    ap.add_argument("--paper-periodic", action="store_true",
                    help="--paper-agg with periodic boundaries wherever an "
                         "extent is >= 3 (default: open)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one plain device copy of this size first (a "
                         "known-size reference for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library drives one GPU "
              "per process and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2603_07341_amd as P
    import workloads as WL

    torch.cuda.set_device(0)
    if args.paper_1d is not None or args.paper_agg is not None:
        print(json.dumps(paper_run(args)), flush=True)
        return
    if args.calib_copy_mib:
        n = args.calib_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    cfg = dict(WL.CONFIGS[args.config])
    cfg["precision"] = args.precision
    params = WL.model_params(cfg)
    run = WL.run_params(cfg)
    exc, occ, coef = WL.initial_state(cfg)
    model = P.Model(params)
    stream = torch.cuda.current_stream()
    sim = P.Sim(model, run, exc, occ, coef, stream=stream)
    print("warmup %d steps" % args.warmup, file=sys.stderr, flush=True)
    sim.step(args.warmup, stream=stream)
    torch.cuda.synchronize()
    tuning = sim.autotune(steps=2, stream=stream) if args.tune == "auto" else sim.tuning()
    torch.cuda.synchronize()
    nS0 = sim.size(stream)
    forms = not args.no_forms and args.config == "ring16" and args.precision == 64
    cpu_state = None
    if not args.no_cpu or forms:
        cpu_state = sim.state(stream)
    t_start = float(sim.series(sim.num_records() - 1, 1, stream)[0, 0])
    nrec0 = sim.num_records()
    print("timing %d steps from |S| = %d" % (args.steps, nS0), file=sys.stderr,
          flush=True)
    # the timed window times one middle Clenshaw launch per step, by events
    # its own dispatch records (no stage markers on the stream)
    sim.profile(True, kernels_only=True)
    sim.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = sim.profile_get(stream)
    sim.profile(False)
    rec = sim.series(nrec0, args.steps, stream)
    # per-stage breakdown from a few further steps with stage events (not
    # part of the timed window)
    nrec1 = sim.num_records()
    sim.profile(True)
    sim.profile_reset()
    sim.step(args.stage_steps, stream=stream)
    sprof = sim.profile_get(stream)
    sim.profile(False)
    srec = sim.series(nrec1, args.stage_steps, stream)
    elapsed = t1 - t0
    updates = float(rec[:, 7].sum())
    value = updates / elapsed
    A = 16 if args.precision == 64 else 8
    D = model.D
    n_term = prof["launches"]["term"]
    term_ms = prof["ms"]["term"] / max(n_term, 1)
    term_bytes = prof["term_bytes"] / max(n_term, 1)
    achieved = term_bytes / (term_ms * 1e-3) / 1e9 if n_term else 0.0
    stage_ms = {k: round(v / args.stage_steps, 4) for k, v in sprof["ms"].items()}
    row_bytes = 4 * A + 4 * D + (8 if model.V <= 2 else 16)
    traffic = committed_traffic(args.config, args.precision,
                                term_bytes / row_bytes if n_term else 0.0)
    out = {
        "metric": "basis-state updates/s (|S|*steps/s)",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128" if args.precision == 64 else "c64",
        "data": "synthetic",
        "config": {"workload": "%s: %d-site Holstein ring, cutoff %d, g %g, "
                               "J %g, k %d, theta %g, dt %g" % (
                                   args.config, WL.n_sites(cfg), cfg["cutoff"][0],
                                   cfg["g"][0], cfg["J"][0], cfg["k"],
                                   cfg["theta"], cfg["dt"]),
                   "timed_steps": [args.warmup, args.warmup + args.steps],
                   "S_start": int(nS0), "S_end": int(rec[-1, 7]),
                   "S_mean": updates / args.steps},
        "roofline": {"bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_cheb_term (middle Clenshaw term)",
                     "launches": n_term, "avg_ms": term_ms,
                     "sampling": "one middle launch per timed step",
                     "bytes_per_launch": term_bytes,
                     "bytes_per_row": row_bytes},
        "stage_ms_per_step": stage_ms,
        "stage_ms_note": "%d further steps after the timed window, with "
                         "stage events" % args.stage_steps,
        "stages": stage_bandwidth(model, A, sprof, srec,
                                  float(rec[-1, 7]), args.stage_steps,
                                  copy_peak_gbs()),
        "tuning": tuning,
        "terms_per_step": float(rec[:, 9].mean()),
    }
    if forms:
        del sim
        out["forms"] = {
            "fp32": form_fp32(args, rec, elapsed, stream),
            "krylov": form_krylov(args, cpu_state, t_start, rec, elapsed,
                                  stream),
            "taylor": form_taylor(args, cpu_state, t_start, rec, elapsed,
                                  stream),
            "batched": form_batched(args, stream),
            "adjoint": form_adjoint(args, stream),
        }
    if cpu_state is not None and not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(params, run, cpu_state, cfg,
                                           args.cpu_seconds)
    print(json.dumps(out), flush=True)


def paper_run(args):
    """One of the paper's own calculations with its own parameters: a row
    of its table of 1D runs (--paper-1d g: open chain, one exciton at the
    centre, J = omega = 1, m_init 10, m 2, dt 0.05, t = 50) or an aggregate
    (--paper-agg: g 0.71, J +-0.55, d_pho 16, k=0 Bloch start, t = 100),
    both with fixed-size truncation q_nom.  Reports the wall time of the
    steps, updates/s and q_true / q_nom = |S| / |M| once |M| = q_nom."""
    import numpy as np
    import torch
    import paper_2603_07341_amd as P
    import workloads as WL
    if args.paper_1d is not None:
        cfg = WL.paper_1d(args.paper_1d, args.q_nom)
        what = "paper 1D run: g %g, N %d, d_pho %d" % (
            args.paper_1d, WL.n_sites(cfg), cfg["cutoff"][0] + 1)
    else:
        ext = [int(x) for x in args.paper_agg.split("x")]
        cfg = WL.paper_aggregate(ext, args.paper_kind, args.q_nom,
                                 periodic=args.paper_periodic)
        what = "paper %s-aggregate run: %s lattice (periodic %s), d_pho 16" % (
            args.paper_kind, args.paper_agg, cfg["periodic"][:len(ext)])
    steps = args.paper_steps or cfg["steps"]
    q = cfg["q_nom"]
    run = dict(WL.run_params(cfg), cap_hint=int(12.5 * q),
               krylov_order=args.paper_krylov, taylor_order=args.paper_taylor)
    if args.paper_krylov:
        what += ", order-%d Krylov propagator" % args.paper_krylov
    if args.paper_taylor:
        what += ", %s Taylor propagator" % (
            "adaptive" if args.paper_taylor < 0 else
            "order-%d" % args.paper_taylor)
    stream = torch.cuda.current_stream()
    sim = P.Sim(P.Model(WL.model_params(cfg)), run, *WL.initial_state(cfg),
                stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        n = min(50, steps - done)
        sim.step(n, stream=stream)
        done += n
        last = sim.series(done - 1, 1, stream)[0]
        print("%s: step %d, |S| %d, |M| %d, %.1f s" % (
            what, done, last[7], last[8], time.perf_counter() - t0),
            file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    rec = sim.series(0, steps, stream)
    if args.paper_save:
        np.save(args.paper_save, rec)
    sat = rec[:, 8] >= q
    ratio = rec[sat, 7] / rec[sat, 8]
    tail = rec[sat][-100:]  # the last 100 steps with |M| = q_nom
    return {"workload": "%s, q_nom %d, m_init %d, m %d, dt %g, %d steps" % (
                what, q, cfg["k_init"], cfg["k"], cfg["dt"], steps),
            "seconds": el, "updates_per_s": float(rec[:, 7].sum()) / el,
            "S_max": int(rec[:, 7].max()),
            "q_true_over_q_nom_mean": float(ratio.mean()) if len(ratio) else None,
            "q_true_over_q_nom_last100":
                float((tail[:, 7] / tail[:, 8]).mean()) if len(tail) else None,
            "final_norm2": float(rec[-1, 1]),
            "norm_loss": float(1.0 - rec[-1, 1]), "final_t": float(rec[-1, 0]),
            "terms_per_step": float(rec[:, 9].mean())}


def copy_peak_gbs(mib=1024, reps=5):
    """Measured device-copy bandwidth in this run (read + write bytes of a
    plain torch copy of `mib` MiB, best of `reps`), a practical peak beside
    the 8 TB/s specification."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b))
    del src, dst
    return 2.0 * mib * (1 << 20) / (best * 1e-3) / 1e9


def stage_bandwidth(model, A, sprof, srec, n_old0, steps, copy_gbs):
    """Effective bandwidth per stage over the stage-event steps: algorithmic
    bytes (compulsory streams, each once per pass; gathers counted as cache
    hits) from the steps' own counts, over the stage's event time.
      select        n_old (A + 1) + 4 |M|
      expand+build  |S| (8W + D (8 + 8W + 4) + rho (8W + 16)),
                    rho = net growth of S / |S| (a lower bound on new rows)
      transfer      n_old (16W + 8 + 2A)
      propagate     |S| K (4A + 4D + 8)  (Clenshaw)
      observe       |S| 2A"""
    W, D = model.W, model.D
    nS = srec[:, 7]
    nM = srec[:, 8]
    K = srec[:, 9]
    n_old = [n_old0] + list(nS[:-1])
    by = {"select": 0.0, "expand+build": 0.0, "transfer": 0.0,
          "propagate": 0.0, "observe": 0.0}
    for s in range(steps):
        rho = max(0.0, nS[s] - n_old[s]) / max(nS[s], 1.0)
        by["select"] += n_old[s] * (A + 1) + 4 * nM[s]
        by["expand+build"] += nS[s] * (8 * W + D * (8 + 8 * W + 4) + rho * (8 * W + 16))
        by["transfer"] += n_old[s] * (16 * W + 8 + 2 * A)
        by["propagate"] += nS[s] * K[s] * (4 * A + 4 * D + 8)
        by["observe"] += nS[s] * 2 * A
    ms = dict(sprof["ms"])
    ms["expand+build"] = ms["expand"] + ms["build"]
    out = {"copy_peak_gbs": copy_gbs, "unit": "GB/s"}
    tb = tt = 0.0
    for k, b in by.items():
        t = ms[k] * 1e-3
        tb += b
        tt += t
        g = b / t / 1e9 if t > 0 else 0.0
        out[k] = {"bytes_per_step": b / steps, "ms_per_step": ms[k] / steps,
                  "effective": g, "frac_spec": g / HBM_PEAK_GBS,
                  "frac_copy": g / copy_gbs}
    g = tb / tt / 1e9 if tt > 0 else 0.0
    out["total"] = {"effective": g, "frac_spec": g / HBM_PEAK_GBS,
                    "frac_copy": g / copy_gbs}
    return out


def timed(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return r, time.perf_counter() - t0


def form_fp32(args, rec64, el64, stream):
    """The same window with complex64 amplitudes (FP64 scalars and sums);
    errors of a(t) and the norm against the FP64 run."""
    import numpy as np
    import paper_2603_07341_amd as P
    import workloads as WL
    cfg = dict(WL.CONFIGS["ring16"], precision=32)
    m = P.Model(WL.model_params(cfg))
    s = P.Sim(m, WL.run_params(cfg), *WL.initial_state(cfg), stream=stream)
    print("fp32: warmup %d steps" % args.warmup, file=sys.stderr, flush=True)
    s.step(args.warmup, stream=stream)
    n0 = s.num_records()
    _, el = timed(lambda: s.step(args.steps, stream=stream))
    rec = s.series(n0, args.steps, stream)
    a32 = rec[:, 3] + 1j * rec[:, 4]
    a64 = rec64[:, 3] + 1j * rec64[:, 4]
    return {"value": float(rec[:, 7].sum()) / el, "unit": "updates/s",
            "ms_per_step": el * 1e3 / args.steps,
            "speedup_vs_fp64": el64 / el,
            "max_abs_err_autocorr_vs_fp64": float(np.max(np.abs(a32 - a64))),
            "max_rel_err_norm_vs_fp64": float(np.max(np.abs(rec[:, 1] / rec64[:, 1] - 1))),
            "S_mean_fp32_over_fp64": float(rec[:, 7].sum() / rec64[:, 7].sum())}


def form_krylov(args, state, t_start, rec_ref, el_ref, stream):
    """The timed window again with the order-10 Krylov (Lanczos) propagator
    in place of the series, from the same state: throughput against the
    series run, deviation of a(t) from it, and the roofline of the Lanczos
    SpMV (its algorithmic bytes per row 2A + 4D + 8: w_j and H w_j once
    each, the columns and the payload)."""
    import numpy as np
    import paper_2603_07341_amd as P
    import workloads as WL
    order = args.krylov_order
    cfg = dict(WL.CONFIGS["ring16"], precision=64)
    m = P.Model(WL.model_params(cfg))
    run = dict(WL.run_params(cfg), krylov_order=order)
    s = P.Sim(m, run, *WL.initial_state(cfg), stream=stream)
    keys, amps = state
    s.set_state(keys, amps, t_start, stream=stream)
    print("krylov: order %d, %d steps from |S| = %d" % (order, args.steps,
                                                        len(keys)),
          file=sys.stderr, flush=True)
    s.profile(True, kernels_only=True)
    s.profile_reset()
    _, el = timed(lambda: s.step(args.steps, stream=stream))
    prof = s.profile_get(stream)
    s.profile(False)
    rec = s.series(0, args.steps, stream)
    n = prof["launches"]["krylov"]
    ms = prof["ms"]["krylov"] / max(n, 1)
    ach = prof["krylov_bytes"] / max(n, 1) / (ms * 1e-3) / 1e9 if n else 0.0
    a = rec[:, 3] + 1j * rec[:, 4]
    a_ref = rec_ref[:, 3] + 1j * rec_ref[:, 4]
    return {"order": order, "value": float(rec[:, 7].sum()) / el,
            "unit": "updates/s", "ms_per_step": el * 1e3 / args.steps,
            "time_vs_series": el / el_ref,
            "max_abs_err_autocorr_vs_series": float(np.max(np.abs(a - a_ref))),
            "max_rel_err_norm_vs_series": float(np.max(np.abs(rec[:, 1] / rec_ref[:, 1] - 1))),
            "spmv_ms_total": round(prof["ms"]["krylov"], 3),
            "spmv_roofline": {"bound": "hbm", "achieved": ach,
                              "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": ach / HBM_PEAK_GBS, "launches": n,
                              "avg_ms": ms}}


def form_taylor(args, state, t_start, rec_ref, el_ref, stream):
    """The timed window again with the truncated Taylor propagator (degree
    and substeps chosen per step as Al-Mohy & Higham do) in place of the
    Chebyshev series, from the same state: throughput and deviation of a(t)
    against the series run; its term launches have the Clenshaw term's
    streams (4A + 4D + 8 bytes per row), timed one per step."""
    import numpy as np
    import paper_2603_07341_amd as P
    import workloads as WL
    cfg = dict(WL.CONFIGS["ring16"], precision=64)
    m = P.Model(WL.model_params(cfg))
    run = dict(WL.run_params(cfg), taylor_order=-1)
    s = P.Sim(m, run, *WL.initial_state(cfg), stream=stream)
    keys, amps = state
    s.set_state(keys, amps, t_start, stream=stream)
    print("taylor: %d steps from |S| = %d" % (args.steps, len(keys)),
          file=sys.stderr, flush=True)
    s.profile(True, kernels_only=True)
    s.profile_reset()
    _, el = timed(lambda: s.step(args.steps, stream=stream))
    prof = s.profile_get(stream)
    s.profile(False)
    rec = s.series(0, args.steps, stream)
    n = prof["launches"]["term"]
    ms = prof["ms"]["term"] / max(n, 1)
    ach = prof["term_bytes"] / max(n, 1) / (ms * 1e-3) / 1e9 if n else 0.0
    a = rec[:, 3] + 1j * rec[:, 4]
    a_ref = rec_ref[:, 3] + 1j * rec_ref[:, 4]
    return {"value": float(rec[:, 7].sum()) / el, "unit": "updates/s",
            "ms_per_step": el * 1e3 / args.steps,
            "time_vs_series": el / el_ref,
            "products_per_step": float(rec[:, 9].mean()),
            "chebyshev_terms_per_step": float(rec_ref[:, 9].mean()),
            "max_abs_err_autocorr_vs_series": float(np.max(np.abs(a - a_ref))),
            "max_rel_err_norm_vs_series": float(np.max(np.abs(rec[:, 1] / rec_ref[:, 1] - 1))),
            "term_roofline": {"bound": "hbm", "achieved": ach,
                              "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": ach / HBM_PEAK_GBS, "launches": n,
                              "avg_ms": ms}}


def form_batched(args, stream):
    """64 disorder realizations of the 6x6 lattice (complex64) in one sim,
    against single-realization sims of the first few realizations run one
    after another, both from the initial state for the same steps."""
    import paper_2603_07341_amd as P
    import workloads as WL
    cfg = WL.CONFIGS["sq6x6"]
    n = args.batch_steps
    bm = P.Model(WL.batch_params(cfg))
    b = P.Sim(bm, WL.run_params(cfg), *WL.initial_state(cfg), stream=stream)
    print("batched: %d realizations x %d steps" % (bm.R, n), file=sys.stderr,
          flush=True)
    _, el_b = timed(lambda: b.step(n, stream=stream))
    rb = b.series(0, n, stream)
    upd_b = float(rb[:, :, 7].sum())
    del b
    el_s, upd_s = 0.0, 0.0
    for r in range(args.batch_singles):
        m = P.Model(WL.model_params(cfg, r))
        s = P.Sim(m, WL.run_params(cfg), *WL.initial_state(cfg), stream=stream)
        _, el = timed(lambda: s.step(n, stream=stream))
        el_s += el
        upd_s += float(s.series(0, n, stream)[:, 7].sum())
    per_real_single = el_s / args.batch_singles
    return {"realizations": bm.R, "steps": n,
            "value": upd_b / el_b, "unit": "updates/s",
            "ms_per_step": el_b * 1e3 / n,
            "single_value": upd_s / el_s,
            "single_ms_per_step_per_realization": per_real_single * 1e3 / n,
            "speedup_vs_sequential": per_real_single * bm.R / el_b,
            "S_final_total": int(rb[-1, :, 7].sum()),
            "S_final_min_max": [int(rb[-1, :, 7].min()), int(rb[-1, :, 7].max())]}


def form_adjoint(args, stream):
    """Adjoint gradient of L = sum_t |a(t) - tau(t)|^2 on the 12-site ring
    (checkpoint every 50; 200 steps by default, by which |S| passes 9e6 and
    keeps growing): time of the recorded forward and of the backward sweep
    (segment replays included) against a plain forward run of the same
    steps, and a central-difference check of two gradient entries."""
    import numpy as np
    import paper_2603_07341_amd as P
    import workloads as WL
    cfg = WL.CONFIGS["ring12"]
    n, ck = args.adjoint_steps, cfg["ckpt_every"]
    p = WL.model_params(cfg)
    init = WL.initial_state(cfg)
    print("adjoint: %d steps, checkpoint every %d" % (n, ck), file=sys.stderr,
          flush=True)
    s0 = P.Sim(P.Model(p), WL.run_params(cfg), *init, stream=stream)
    _, el_plain = timed(lambda: s0.step(n, stream=stream))
    S_end = int(s0.observe(stream=stream)["n_S"])
    print("adjoint: plain forward %.2f s, |S| %d" % (el_plain, S_end),
          file=sys.stderr, flush=True)
    del s0
    m = P.Model(p)
    s = P.Sim(m, WL.run_params(cfg), *init, stream=stream)
    a, el_fwd = timed(lambda: s.adjoint_forward(n, ck, stream=stream))
    print("adjoint: recorded forward %.2f s" % el_fwd, file=sys.stderr,
          flush=True)
    rng = np.random.default_rng(43)
    tau = a * np.exp(1j * 0.05 * rng.standard_normal(len(a)))
    g, el_bwd = timed(lambda: s.adjoint_backward(a - tau, stream=stream))
    print("adjoint: backward %.2f s" % el_bwd, file=sys.stderr, flush=True)
    # self-check on this run: central differences of the frozen-set replay
    # along J and eps_0 against the adjoint gradient
    loss = lambda aa: float(np.sum(np.abs(aa - tau) ** 2))
    theta = P.theta_of(p)
    fd_err = {}
    for k, name in ((0, "J0"), (len(theta) - m.N, "eps0")):
        h = 1e-4
        lp = loss(s.adjoint_replay(P.Model(P.params_with_theta(
            p, theta + h * (np.arange(len(theta)) == k))), stream=stream))
        lm = loss(s.adjoint_replay(P.Model(P.params_with_theta(
            p, theta - h * (np.arange(len(theta)) == k))), stream=stream))
        fd_err[name] = abs((lp - lm) / (2 * h) - g[k]) / max(abs(g[k]), 1e-300)
    return {"steps": n, "ckpt_every": ck, "S_end": S_end,
            "plain_forward_s": el_plain, "recorded_forward_s": el_fwd,
            "backward_s": el_bwd,
            "adjoint_over_forward": el_bwd / el_plain,
            "forward_plus_backward_over_forward": (el_fwd + el_bwd) / el_plain,
            "grad_inf_norm": float(np.max(np.abs(g))),
            "fd_rel_err": fd_err}


def source_hash():
    """Hash of the step kernels' code, comments and blank lines ignored."""
    import hashlib
    h = hashlib.sha256()
    for f in ["kernels.hip", "device.hpp", "kernels.hpp", "common.hpp"]:
        with open(os.path.join(ROOT, "paper_2603_07341_amd", "csrc", f)) as fh:
            for line in fh:
                code = line.split("//")[0].rstrip()
                if code:
                    h.update((code + "\n").encode())
    return h.hexdigest()[:16]


def committed_traffic(config, precision, rows_per_launch):
    """HBM bytes per middle-term launch from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, calibrated with a plain copy), or None when
    the kernel sources changed since the counters were taken or the
    workload differs."""
    path = os.path.join(ROOT, "profiles", "cheb_term_ring16_traffic.txt")
    if config != "ring16" or precision != 64 or not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if "sha256[:16]" in line:
                vals["sha"] = line.rsplit(":", 1)[1].strip()
            elif line.startswith(("fetch_bytes_per_row:", "write_bytes_per_row:")):
                k, v = line.split(":")
                vals[k] = float(v)
    if vals.get("sha") != source_hash() or len(vals) < 3:
        return None
    return (vals["fetch_bytes_per_row"] + vals["write_bytes_per_row"]) * rows_per_launch


def cpu_baseline(params, run, state, cfg, budget_s):
    """The CPU oracle continued from the GPU state for as many whole steps
    as fit in the budget (at least one)."""
    from oracle import oracle as O
    import workloads as WL
    keys, amps = state
    om = O.Model(params)
    exc, occ, coef = WL.initial_state(cfg)
    s = O.Sim(om, run, exc, occ, coef)
    s.set_state(keys, amps, 0.0)
    t0 = time.perf_counter()
    n = 0
    while True:
        s.step(1)
        n += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    upd = sum(o["n_S"] for o in s.observations())
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": upd / el, "unit": "updates/s", "cores": cores,
            "kind": "oracle",
            "sample": "%d step(s) continued from the GPU state at the start "
                      "of the timed window (|S| %d -> %d), %.1f s" % (
                          n, len(keys), int(s.observations()[-1]["n_S"]), el)}


if __name__ == "__main__":
    main()
