"""Benchmark of the co-evolving-subspace step on one MI355X.

Workload: the 1D Holstein ring of 16 sites (one mode per site, omega 1,
g 1.2, J -1, cutoff 12, k=0 Bloch start, dt 0.01, neighbour order 4,
amplitude threshold 1e-8, complex128), synthetic inputs only.  A "step" is
one full time step of the hot path: select, expand (4 rounds), merge,
transfer, build, Chebyshev propagation and observables.  The run starts
from the initial state and takes untimed steps until |S| reaches --grow-to
(default 1e7, where the set no longer fits the last-level cache), runs the
library's launch autotuner, `--warmup` more untimed steps, then exactly
`--steps` steps timed between stream synchronisations.

value = sum over timed steps of |S| / wall time (basis-state updates/s).
roofline: the middle Clenshaw term kernel (the dominant kernel): achieved
= |S| (5A + 4D + 12) bytes per launch (the per-row, per-term bytes of a
Chebyshev term: three vector streams of a forward recurrence plus an
accumulator read and written, the columns and the diagonal) over its
HIP-event duration on the step's stream, from one middle launch per timed
step whose dispatch records the events; the kernel's own streams (Clenshaw
form, 4A + 4D + 8) are reported beside it.  traffic: HBM bytes per launch
counted on this very window (FETCH_SIZE + WRITE_SIZE) in the committed
summary of rocprofv3 runs of the default command, when it matches the
current kernels and window.
cpu_baseline: the CPU oracle continued from the GPU state at the start of
the timed window on all its threads for a bounded time, and one step on
one thread.
forms: the extra forms against plain FP64 single-realization runs on the
same GPU: complex64 amplitudes on the same window; the order-10 Krylov
propagator and the truncated Taylor series on the same window from the
same state; 64 disorder realizations of the 6x6 lattice in one sim against
realizations run one after another; the adjoint gradient of the 12-site
ring against its plain forward run (time ratio).
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
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--grow-to", type=float, default=1e7,
                    help="untimed steps from the initial state until |S| "
                         "reaches this, before the autotuner, --warmup and "
                         "the timed --steps")
    ap.add_argument("--grow-max", type=int, default=1000)
    ap.add_argument("--config", default="ring16")
    ap.add_argument("--precision", type=int, default=64)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-cpu-single", action="store_true",
                    help="skip the one-thread oracle step of the CPU baseline")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--tune", default="auto", choices=["auto", "none"],
                    help="run the library's launch autotuner on the warmed-up "
                         "state before timing (results do not depend on it)")
    ap.add_argument("--batch-steps", type=int, default=40)
    ap.add_argument("--batch-singles", type=int, default=8)
    ap.add_argument("--singles-only", action="store_true",
                    help=argparse.SUPPRESS)  # the batched form's child runs
    ap.add_argument("--batched-only", action="store_true",
                    help=argparse.SUPPRESS)
    ap.add_argument("--adjoint-steps", type=int, default=200)
    ap.add_argument("--long-steps", type=int, default=500,
                    help="steps of the complex64 vs complex128 long run")
    ap.add_argument("--long-cap", type=float, default=2e6,
                    help="state cap of the long run")
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
    ap.add_argument("--cube4-cap", type=float, default=None, metavar="CAP",
                    help="instead of the benchmark, run the 3D workload "
                         "(4x4x4 periodic cubic lattice, two modes, complex64) "
                         "with a state cap of CAP from its start until the "
                         "cap binds, then --cube4-steps more steps, and print "
                         "one JSON line with the times and counts")
    ap.add_argument("--cube4-steps", type=int, default=10)
    ap.add_argument("--cube4-max", type=int, default=400)
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
    if args.singles_only:
        print(json.dumps(batch_singles(args, torch.cuda.current_stream())),
              flush=True)
        return
    if args.batched_only:
        print(json.dumps(batch_run(args, torch.cuda.current_stream())),
              flush=True)
        return
    if args.paper_1d is not None or args.paper_agg is not None:
        print(json.dumps(paper_run(args)), flush=True)
        return
    if args.cube4_cap is not None:
        print(json.dumps(cube4_run(args)), flush=True)
        return
    cfg = dict(WL.CONFIGS[args.config])
    cfg["precision"] = args.precision
    params = WL.model_params(cfg)
    run = WL.run_params(cfg)
    exc, occ, coef = WL.initial_state(cfg)
    model = P.Model(params)
    stream = torch.cuda.current_stream()
    # a plain 1 GiB device copy between the first two marks: the known-size
    # reference of the hardware byte counters
    P.profile_mark(0, stream)
    copy_once(1024)
    P.profile_mark(1, stream)
    sim = P.Sim(model, run, exc, occ, coef, stream=stream)
    grown = grow_until(sim, args.grow_to, args.grow_max, stream)
    print("grown %d steps to |S| = %d" % (grown, sim.size(stream)),
          file=sys.stderr, flush=True)
    tuning = sim.autotune(steps=2, stream=stream) if args.tune == "auto" else sim.tuning()
    print("warmup %d steps" % args.warmup, file=sys.stderr, flush=True)
    sim.step(args.warmup, stream=stream)
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
    # its own dispatch records (no stage markers on the stream); marks 2
    # and 3 bracket it for kernel traces and counter runs
    sim.profile(True, kernels_only=True)
    sim.profile_reset()
    torch.cuda.synchronize()
    P.profile_mark(2, stream)
    t0 = time.perf_counter()
    sim.step(args.steps, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    P.profile_mark(3, stream)
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
    kern_row = 4 * A + 4 * D + (8 if model.V <= 2 else 16)
    # the launch runs over the set's row range, which after in-place steps
    # may hold holes of dropped states; the algorithmic bytes count the
    # states of the set (one timed launch per step: the window's mean |S|)
    rows_range = prof["term_bytes"] / max(n_term, 1) / kern_row
    rows_per_launch = float(rec[:, 7].mean())
    spec_row = 5 * A + 4 * D + 12
    achieved = spec_row * rows_per_launch / (term_ms * 1e-3) / 1e9 if n_term else 0.0
    achieved_k = kern_row * rows_per_launch / (term_ms * 1e-3) / 1e9 if n_term else 0.0
    stage_ms = {k: round(v / args.stage_steps, 4) for k, v in sprof["ms"].items()}
    window = {"grown_steps": grown, "warmup": args.warmup, "steps": args.steps,
              "S_start": int(nS0), "S_end": int(rec[-1, 7])}
    wprof = committed_window_profile(args, window)
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
                   "grown_steps": grown, "grow_to": args.grow_to,
                   "timed_steps": [grown + args.warmup,
                                   grown + args.warmup + args.steps],
                   "S_start": int(nS0), "S_end": int(rec[-1, 7]),
                   "S_mean": updates / args.steps},
        "roofline": {"bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": wprof["traffic_per_launch"] if wprof else None,
                     "kernel": "k_cheb_term (middle Clenshaw term)",
                     "launches": n_term, "avg_ms": term_ms,
                     "sampling": "one middle launch per timed step",
                     "rows_per_launch": rows_per_launch,
                     "row_range_per_launch": rows_range,
                     "bytes_per_row": spec_row,
                     "bytes_per_row_rule": "5A + 4D + 12 per row and term "
                                           "(forward recurrence with an "
                                           "accumulator)",
                     "kernel_bytes_per_row": kern_row,
                     "achieved_kernel_bytes": achieved_k,
                     "frac_kernel_bytes": achieved_k / HBM_PEAK_GBS,
                     "traffic_source": wprof["source"] if wprof else None},
        "stage_ms_per_step": stage_ms,
        "stage_ms_note": "%d further steps after the timed window, with "
                         "stage events" % args.stage_steps,
        "row_range_over_states": float(sprof["rows_steps"]) /
                                 max(float(srec[:, 7].sum()), 1.0),
        "stages": stage_bandwidth(model, A, sprof, srec,
                                  float(rec[-1, 7]), args.stage_steps,
                                  copy_peak_gbs(), wprof,
                                  bool(tuning.get("warm", 0))),
        "tuning": tuning,
        "terms_per_step": float(rec[:, 9].mean()),
    }
    if forms:
        del sim
        out["forms"] = {
            "fp32": form_fp32(args, grown, rec, elapsed, stream),
            "fp32_long": form_fp32_long(args, stream),
            "krylov": form_krylov(args, cpu_state, t_start, rec, elapsed,
                                  stream),
            "taylor": form_taylor(args, cpu_state, t_start, rec, elapsed,
                                  stream),
            "batched": form_batched(args, stream),
            "adjoint": form_adjoint(args, stream),
        }
    if cpu_state is not None and not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(params, run, cpu_state, cfg,
                                           args.cpu_seconds,
                                           not args.no_cpu_single, t_start)
    print(json.dumps(out), flush=True)


def grow_until(sim, target, max_steps, stream):
    """Untimed steps from the initial state until |S| >= target (at most
    max_steps); returns the number taken."""
    n = 0
    while n < max_steps and sim.size(stream) < target:
        sim.step(1, stream=stream)
        n += 1
    return n


def copy_once(mib):
    """One plain device copy of `mib` MiB (read + write), timed by events;
    returns its bandwidth in GB/s."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    dst.copy_(src)
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b)
    del src, dst
    return 2.0 * mib * (1 << 20) / (ms * 1e-3) / 1e9


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
    # the row range the kernels run over against the states of the set
    # (holes of in-place steps), over two further steps outside the timing
    sim.profile(True, kernels_only=True)
    sim.profile_reset()
    sim.step(2, stream=stream)
    extra = sim.series(steps, 2, stream)
    range_over_live = sim.profile_get(stream)["rows_steps"] / float(extra[:, 7].sum())
    sim.profile(False)
    if args.paper_save:  # every record, the two further steps included
        np.save(args.paper_save, sim.series(0, steps + 2, stream))
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
            "terms_per_step": float(rec[:, 9].mean()),
            "row_range_over_states_after": range_over_live}


def cube4_run(args):
    """The 3D workload under its state cap: untimed steps from the start
    until |S| reaches 90% of the cap (or --cube4-max steps), then
    --cube4-steps steps timed.  Reports updates/s over the timed steps,
    the counts, whether every step kept |S| <= cap, and the device memory
    the sim holds."""
    import numpy as np
    import torch
    import paper_2603_07341_amd as P
    import workloads as WL
    cfg = dict(WL.CONFIGS["cube4"])
    cap = int(args.cube4_cap)
    run = dict(WL.run_params(cfg), max_states=cap)
    stream = torch.cuda.current_stream()
    sim = P.Sim(P.Model(WL.model_params(cfg)), run, *WL.initial_state(cfg),
                stream=stream)
    t0 = time.perf_counter()
    n = 0
    while n < args.cube4_max:
        sim.step(1, stream=stream)
        n += 1
        last = sim.series(n - 1, 1, stream)[0]
        if n % 10 == 0 or last[7] >= 0.9 * cap:
            print("cube4: step %d, |S| %d, |M| %d, %.1f s" % (
                n, last[7], last[8], time.perf_counter() - t0),
                file=sys.stderr, flush=True)
        if last[7] >= 0.9 * cap:
            break
    grow_s = time.perf_counter() - t0
    free0, total = torch.cuda.mem_get_info()
    _, el = timed(lambda: sim.step(args.cube4_steps, stream=stream))
    free1, _ = torch.cuda.mem_get_info()
    rec = sim.series(0, sim.num_records(), stream)
    tail = rec[n:]
    print("cube4: %d timed steps, %.2f s" % (args.cube4_steps, el),
          file=sys.stderr, flush=True)
    return {"workload": "cube4: 4x4x4 periodic cubic Holstein lattice, modes "
                        "(1, 1, c 15) and (0.2, 0.5, c 31), J -0.5, k 2, "
                        "theta 1e-7, dt 0.01, complex64, state cap %d" % cap,
            "grow_steps": n, "grow_s": grow_s,
            "timed_steps": args.cube4_steps, "timed_s": el,
            "ms_per_step": el * 1e3 / args.cube4_steps,
            "updates_per_s": float(tail[:, 7].sum()) / el,
            "S_timed": [int(tail[0, 7]), int(tail[-1, 7])],
            "M_timed": [int(tail[0, 8]), int(tail[-1, 8])],
            "S_max_all_steps": int(rec[:, 7].max()),
            "cap_respected": bool(np.all(rec[:, 7] <= cap)),
            "norm2_end": float(rec[-1, 1]), "mass_total_end": float(rec[-1, 6]),
            "device_gib_in_use": [(total - free0) / 2 ** 30,
                                  (total - free1) / 2 ** 30],
            "device_gib_total": total / 2 ** 30,
            "terms_per_step": float(tail[:, 9].mean())}


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


def stage_bandwidth(model, A, sprof, srec, n_old0, steps, copy_gbs, wprof,
                    in_place=False):
    """Effective bandwidth per stage over the stage-event steps: algorithmic
    bytes (compulsory streams, each once per pass; gathers counted as cache
    hits) from the steps' own counts, over the stage's event time.  With a
    committed counter profile of this window, each stage also gets its
    achieved rate: counted HBM bytes (FETCH_SIZE + WRITE_SIZE, calibrated)
    over kernel time, both per step of the window.
      select        n_old (A + 1) + 4 |M|
      expand+build  |S| (8W + D (8 + 8W + 4) + rho (8W + 16)),
                    rho = net growth of S / |S| (a lower bound on new rows)
      transfer      n_old (16W + 8 + 2A)
      propagate     |S| K (4A + 4D + 8)  (Clenshaw)
      observe       |S| 2A
    Steps that expand in place (from the previous step's graph) turn psi
    into phi and drop rows inside the expansion, so their transfer stage
    has no rate of its own: it is reported with the expansion only."""
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
        if in_place and k == "transfer":
            out[k] = {"bytes_per_step": None, "ms_per_step": ms[k] / steps,
                      "effective": None,
                      "note": "inside the in-place expansion; see "
                              "expand+transfer+build"}
            continue
        g = b / t / 1e9 if t > 0 else 0.0
        out[k] = {"bytes_per_step": b / steps, "ms_per_step": ms[k] / steps,
                  "effective": g, "frac_spec": g / HBM_PEAK_GBS,
                  "frac_copy": g / copy_gbs}
        st = (wprof or {}).get("stages", {}).get(k)
        if st and st["kernel_ms"] > 0:
            ach = st["bytes"] / (st["kernel_ms"] * 1e-3) / 1e9
            out[k].update({"counted_bytes_per_step": st["bytes"],
                           "kernel_ms_per_step": st["kernel_ms"],
                           "achieved": ach,
                           "achieved_frac_spec": ach / HBM_PEAK_GBS})
    # steps that expand in place make phi and the dropped weight inside the
    # expansion: the transfer stage keeps only the fold of the weight, so
    # the two are also given together
    b = by["expand+build"] + by["transfer"]
    t = (ms["expand+build"] + ms["transfer"]) * 1e-3
    g = b / t / 1e9 if t > 0 else 0.0
    out["expand+transfer+build"] = {
        "bytes_per_step": b / steps,
        "ms_per_step": (ms["expand+build"] + ms["transfer"]) / steps,
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


def form_fp32(args, grown, rec64, el64, stream):
    """The same window with complex64 amplitudes (FP64 scalars and sums):
    the same number of growth and warm-up steps from the initial state,
    then the timed steps; errors of a(t) and the norm against the FP64
    run."""
    import numpy as np
    import paper_2603_07341_amd as P
    import workloads as WL
    cfg = dict(WL.CONFIGS["ring16"], precision=32)
    m = P.Model(WL.model_params(cfg))
    s = P.Sim(m, WL.run_params(cfg), *WL.initial_state(cfg), stream=stream)
    print("fp32: %d + %d steps" % (grown, args.warmup), file=sys.stderr,
          flush=True)
    s.step(grown + args.warmup, stream=stream)
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


def form_fp32_long(args, stream):
    """complex64 against complex128 over a long run of the same workload
    under a state cap (the free run passes 1e8 states near step 270, so the
    long run is held at the benchmark's window size): both from the initial
    state in lockstep; the first step whose set differs (count, selection
    or spectral bounds, which depend on the set alone; the sets themselves
    at the end), the weight of the symmetric difference of the two sets
    there, and the largest errors of a(t) and the norm before it."""
    import numpy as np
    import paper_2603_07341_amd as P
    import workloads as WL
    n, cap = args.long_steps, int(args.long_cap)
    sims = {}
    for prec in (64, 32):
        cfg = dict(WL.CONFIGS["ring16"], precision=prec)
        run = dict(WL.run_params(cfg), max_states=cap)
        sims[prec] = P.Sim(P.Model(WL.model_params(cfg)), run,
                           *WL.initial_state(cfg), stream=stream)
    print("fp32 long: %d steps, state cap %d" % (n, cap), file=sys.stderr,
          flush=True)
    first, sym = None, None
    da = dn = 0.0
    t0 = time.perf_counter()
    for i in range(n):
        for prec in (64, 32):
            sims[prec].step(1, stream=stream)
        r64 = sims[64].series(i, 1, stream)[0]
        r32 = sims[32].series(i, 1, stream)[0]
        same = (r64[7] == r32[7] and r64[8] == r32[8] and r64[10] == r32[10]
                and r64[11] == r32[11])
        if first is None and not same:
            first = i + 1
            k64, a64 = sims[64].state(stream)
            k32, a32 = sims[32].state(stream)
            row = np.dtype((np.void, 8 * k64.shape[1]))
            v64 = np.ascontiguousarray(k64).view(row).ravel()
            v32 = np.ascontiguousarray(k32).view(row).ravel()
            only64 = ~np.isin(v64, v32)
            only32 = ~np.isin(v32, v64)
            sym = {"step": first, "S_fp64": int(len(k64)), "S_fp32": int(len(k32)),
                   "rows_only_fp64": int(only64.sum()),
                   "rows_only_fp32": int(only32.sum()),
                   "weight_only_fp64": float(np.sum(np.abs(a64[only64]) ** 2)),
                   "weight_only_fp32": float(np.sum(np.abs(a32[only32]) ** 2))}
        if first is None:
            da = max(da, float(abs((r32[3] + 1j * r32[4]) - (r64[3] + 1j * r64[4]))))
            dn = max(dn, float(abs(r32[1] / r64[1] - 1)))
    el = time.perf_counter() - t0
    k64, _ = sims[64].state(stream)
    k32, _ = sims[32].state(stream)
    s64 = {bytes(r) for r in np.ascontiguousarray(k64)}
    s32 = {bytes(r) for r in np.ascontiguousarray(k32)}
    rec = sims[64].series(0, n, stream)
    return {"steps": n, "state_cap": cap, "seconds_both": el,
            "S_end_fp64": int(len(k64)), "S_end_fp32": int(len(k32)),
            "cap_binds_from_step": int(np.argmax(rec[:, 7] > 0.9 * cap)) + 1
            if np.any(rec[:, 7] > 0.9 * cap) else None,
            "first_divergent_step": first,
            "symmetric_difference_there": sym,
            "sets_equal_at_end": s64 == s32,
            "max_abs_err_autocorr_before_divergence": da,
            "max_rel_err_norm_before_divergence": dn}


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


def batch_singles(args, stream):
    """Single-realization sims of the first batch_singles realizations of
    sq6x6, one after another, batch_steps steps each from the initial state:
    seconds and updates."""
    import paper_2603_07341_amd as P
    import workloads as WL
    cfg = WL.CONFIGS["sq6x6"]
    el_s, upd_s = 0.0, 0.0
    for r in range(args.batch_singles):
        m = P.Model(WL.model_params(cfg, r))
        s = P.Sim(m, WL.run_params(cfg), *WL.initial_state(cfg), stream=stream)
        _, el = timed(lambda: s.step(args.batch_steps, stream=stream))
        el_s += el
        upd_s += float(s.series(0, args.batch_steps, stream)[:, 7].sum())
        del s
    return {"seconds": el_s, "updates": upd_s}


def batch_run(args, stream):
    """The 64 sq6x6 realizations in one sim, batch_steps steps from the
    initial state: seconds, updates, the final sizes, and the batched
    Clenshaw launch's rate over two further steps."""
    import paper_2603_07341_amd as P
    import workloads as WL
    cfg = WL.CONFIGS["sq6x6"]
    n = args.batch_steps
    bm = P.Model(WL.batch_params(cfg))
    b = P.Sim(bm, WL.run_params(cfg), *WL.initial_state(cfg), stream=stream)
    _, el_b = timed(lambda: b.step(n, stream=stream))
    rb = b.series(0, n, stream)
    # the batched Clenshaw launch (all realizations in one grid), timed by
    # its own dispatches over two further steps
    b.profile(True, kernels_only=True)
    b.profile_reset()
    nr = b.num_records()
    b.step(2, stream=stream)
    prof = b.profile_get(stream)
    b.profile(False)
    r2 = b.series(nr, 2, stream)
    nl = prof["launches"]["term"]
    ms = prof["ms"]["term"] / max(nl, 1)
    A = 8 if cfg.get("precision", 64) == 32 else 16
    spec_row = 5 * A + 4 * bm.D + 12
    states = float(r2[:, :, 7].sum()) / 2.0
    term = {"bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "launches": nl, "avg_ms": ms, "states_per_launch": states,
            "bytes_per_state": spec_row,
            "bytes_per_state_rule": "5A + 4D + 12 per state and term",
            "achieved": spec_row * states / (ms * 1e-3) / 1e9 if nl else 0.0,
            "achieved_kernel_bytes":
                prof["term_bytes"] / max(nl, 1) / (ms * 1e-3) / 1e9 if nl else 0.0}
    term["frac"] = term["achieved"] / HBM_PEAK_GBS
    return {"realizations": bm.R, "seconds": el_b,
            "updates": float(rb[:, :, 7].sum()),
            "S_final_total": int(rb[-1, :, 7].sum()),
            "S_final_min_max": [int(rb[-1, :, 7].min()), int(rb[-1, :, 7].max())],
            "term_roofline": term}


def _child(args, flag):
    """One of the batched form's runs in a fresh process (last stdout line
    is its JSON)."""
    import subprocess
    child = subprocess.run(
        [sys.executable, os.path.abspath(__file__), flag,
         "--batch-steps", str(args.batch_steps),
         "--batch-singles", str(args.batch_singles)],
        capture_output=True, text=True, timeout=900)
    if child.returncode != 0:
        raise RuntimeError("%s run failed: %s" % (flag, child.stderr[-2000:]))
    return json.loads(child.stdout.strip().splitlines()[-1])


def form_batched(args, stream):
    """64 disorder realizations of the 6x6 lattice (complex64) in one sim,
    against single-realization sims of the first few realizations run one
    after another, both from the initial state for the same steps.  Each
    side runs in a fresh child process: after sims of 10^7 to 10^8 rows
    have been freed, the device allocations of later sims' growth (inside
    their timed steps) are several times slower, which would charge either
    side for the forms run before it."""
    n = args.batch_steps
    print("batched: 64 realizations x %d steps, singles x %d" % (
        n, args.batch_singles), file=sys.stderr, flush=True)
    single = _child(args, "--singles-only")
    batch = _child(args, "--batched-only")
    el_s, upd_s = single["seconds"], single["updates"]
    per_real_single = el_s / args.batch_singles
    el_b = batch["seconds"]
    R = batch["realizations"]
    return {"realizations": R, "steps": n,
            "value": batch["updates"] / el_b, "unit": "updates/s",
            "ms_per_step": el_b * 1e3 / n,
            "single_value": upd_s / el_s,
            "single_ms_per_step_per_realization": per_real_single * 1e3 / n,
            "speedup_vs_sequential": per_real_single * R / el_b,
            "S_final_total": batch["S_final_total"],
            "S_final_min_max": batch["S_final_min_max"],
            "term_roofline": batch["term_roofline"],
            "processes": "each side in a fresh child process"}


def form_adjoint(args, stream):
    """Adjoint gradient of L = sum_t |a(t) - tau(t)|^2 on the 12-site ring
    (checkpoint every 50; 200 steps by default, by which |S| passes 9e6 and
    keeps growing), tau the a(t) of a free run with perturbed parameters (J
    + 0.05, g - 0.05, omega + 0.02, eps + N(0, 0.02)): time of the recorded
    forward and of the backward sweep (segment replays included) against a
    plain forward run of the same steps, and central differences (h = 1e-6)
    of the frozen-set replay along every parameter against the gradient."""
    import numpy as np
    import paper_2603_07341_amd as P
    import workloads as WL
    cfg = WL.CONFIGS["ring12"]
    n, ck = args.adjoint_steps, cfg["ckpt_every"]
    p = WL.model_params(cfg)
    init = WL.initial_state(cfg)
    print("adjoint: %d steps, checkpoint every %d" % (n, ck), file=sys.stderr,
          flush=True)
    st = P.Sim(P.Model(WL.adjoint_target_params(cfg)), WL.run_params(cfg),
               *init, stream=stream)
    st.step(n, stream=stream)
    rt = st.series(0, n, stream)
    tau = np.concatenate([[1.0 + 0j], rt[:, 3] + 1j * rt[:, 4]])
    del st
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
    g, el_bwd = timed(lambda: s.adjoint_backward(a - tau, stream=stream))
    print("adjoint: backward %.2f s" % el_bwd, file=sys.stderr, flush=True)
    # central differences of the frozen-set replay along every parameter
    loss = lambda aa: float(np.sum(np.abs(aa - tau) ** 2))
    theta = P.theta_of(p)
    h = 1e-6
    fd = np.zeros(len(theta))
    t0 = time.perf_counter()
    for k in range(len(theta)):
        e = h * (np.arange(len(theta)) == k)
        lp = loss(s.adjoint_replay(P.Model(P.params_with_theta(p, theta + e)),
                                   stream=stream))
        lm = loss(s.adjoint_replay(P.Model(P.params_with_theta(p, theta - e)),
                                   stream=stream))
        fd[k] = (lp - lm) / (2 * h)
    el_fd = time.perf_counter() - t0
    scale = np.maximum(np.abs(g), 1e-2 * np.max(np.abs(g)))
    rel = np.abs(fd - g) / scale
    names = (["J%d" % a for a in range(p["ndim"])] +
             ["g%d" % v for v in range(p["n_modes"])] +
             ["omega%d" % v for v in range(p["n_modes"])] +
             ["eps%d" % j for j in range(m.N)])
    return {"steps": n, "ckpt_every": ck, "S_end": S_end,
            "target": "a(t) of a free run with J + 0.05, g - 0.05, "
                      "omega + 0.02, eps + N(0, 0.02) (seed 43)",
            "loss": loss(a),
            "plain_forward_s": el_plain, "recorded_forward_s": el_fwd,
            "backward_s": el_bwd,
            "adjoint_over_forward": el_bwd / el_plain,
            "forward_plus_backward_over_forward": (el_fwd + el_bwd) / el_plain,
            "grad_inf_norm": float(np.max(np.abs(g))),
            "fd_h": h, "fd_seconds": el_fd,
            "fd_rel_err_max": float(np.max(rel)),
            "fd_rel_err_rule": "|fd_p - g_p| / max(|g_p|, 1e-2 max|g|)",
            "fd_rel_err": {nm: float(x) for nm, x in zip(names, rel)}}


def source_hash():
    from paper_2603_07341_amd.profile_summary import source_hash as h
    return h()


WINDOW_PROFILE = os.path.join("profiles", "cheb_term_ring16_window.txt")


def committed_window_profile(args, window):
    """Counter figures of this very window from the committed summary of
    the default command's rocprofv3 runs: the middle Clenshaw term's HBM
    bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated) and counted
    bytes and kernel time per stage.  None unless the summary was taken on
    the current kernel sources (comments ignored) and on the same window
    (growth, warm-up and timed steps, |S| at both ends)."""
    path = os.path.join(ROOT, WINDOW_PROFILE)
    if args.config != "ring16" or args.precision != 64 or not os.path.exists(path):
        return None
    vals, stages = {}, {}
    with open(path) as fh:
        for line in fh:
            if ":" not in line or line.startswith("#"):
                continue
            k, v = line.split(":", 1)
            k, v = k.strip(), v.strip()
            if k.startswith("stage "):
                name, what = k[6:].rsplit(" ", 1)
                stages.setdefault(name, {})[what] = float(v)
            else:
                vals[k] = v
    try:
        ok = (vals.get("kernel_sha") == source_hash() and
              all(int(vals.get("window_" + f, -1)) == window[f]
                  for f in ("grown_steps", "warmup", "steps", "S_start",
                            "S_end")))
        if not ok:
            return None
        return {"traffic_per_launch": float(vals["mid_term_bytes_per_launch"]),
                "stages": {k: {"bytes": v["bytes"], "kernel_ms": v["kernel_ms"]}
                           for k, v in stages.items()
                           if "bytes" in v and "kernel_ms" in v},
                "source": WINDOW_PROFILE}
    except (KeyError, ValueError):
        return None


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(params, run, state, cfg, budget_s, single, t_start):
    """The CPU oracle continued from the GPU state at the start of the timed
    window (the same |S| range): on all the threads the oracle runs with,
    for as many whole steps as fit in the budget (at least one); then, with
    one thread, one step from the same state."""
    from oracle import oracle as O
    import workloads as WL
    keys, amps = state
    om = O.Model(params)
    exc, occ, coef = WL.initial_state(cfg)

    def leg(max_s, max_steps):
        s = O.Sim(om, run, exc, occ, coef)
        s.set_state(keys, amps, t_start)
        t0 = time.perf_counter()
        n = 0
        while True:
            s.step(1)
            n += 1
            if n >= max_steps or time.perf_counter() - t0 >= max_s:
                break
        el = time.perf_counter() - t0
        upd = sum(o["n_S"] for o in s.observations())
        return upd / el, n, el, int(s.observations()[-1]["n_S"])

    cores = O.threads()
    v, n, el, s_end = leg(budget_s, 1 << 30)
    out = {"value": v, "unit": "updates/s", "cores": cores, "kind": "oracle",
           "cpu_model": cpu_model(), "nproc": os.cpu_count(),
           "sample": "%d step(s) continued from the GPU state at the start "
                     "of the timed window (|S| %d -> %d), %.1f s on %d "
                     "threads" % (n, len(keys), s_end, el, cores)}
    if single:
        O.set_threads(1)
        try:
            v1, n1, el1, s1 = leg(0.0, 1)
        finally:
            O.set_threads(cores)
        out["single_thread"] = {
            "value": v1, "unit": "updates/s", "cores": 1,
            "sample": "1 step from the same state (|S| %d -> %d), %.1f s" % (
                len(keys), s1, el1)}
    return out


if __name__ == "__main__":
    main()
