"""GPU vs oracle at the benchmark's sizes, in the launch configuration the
benchmark times.

ring16 (the throughput workload): the GPU grows the set as the benchmark
does (steps until |S| >= 1e7), autotunes, takes the benchmark's 5 warm-up
steps and then its first timed step (|S| 1.16e7, an in-place step from the
previous graph) with the benchmark's profiling level; the oracle takes the
same step from the same state.  The whole result is compared: M and S bit for
bit, amplitudes within 1e-10, the record's observables; then the same for
one order-10 Krylov step (the benchmark's Krylov form).

sq6x6 (the batched form): 64 realizations in one complex64 sim, 40 steps
from the start as the benchmark runs them (|S| 1.6e8); the last step of two
sampled realizations is redone by the oracle from the GPU state of step 39
(sets bit for bit, amplitudes within 1e-5)."""
import numpy as np
import pytest

import paper_2603_07341_amd as P
from oracle import oracle as O
from tests.gpu_helpers import (assert_amps, assert_same_set, check_obs,
                               dropped, sort_rows)
import workloads as WL

pytestmark = pytest.mark.gpu


def oracle_step_from(cfg, params, keys, amps, t, **run_over):
    run = dict(WL.run_params(cfg), **run_over)
    s = O.Sim(O.Model(params), run, *WL.initial_state(cfg))
    s.set_state(keys, amps, t)
    s.step(1)
    return s


def gpu_result(gs):
    """M, S and the state of the sim's last step (with realizations)."""
    out = {}
    for which in (O.SET_M, O.SET_S):
        out[which] = gs.get_set(which, with_real=True)
    out["state"] = gs.state(with_real=True)
    return out


def compare_step(res, gobs, prev_mass_total, os_, tol, prev, realization=0):
    """The GPU result of one realization against the oracle's step from the
    same state prev = (keys, amps).  The oracle sim starts there, so its
    cumulative discarded weight is shifted by the GPU's total before the
    step."""
    for which in (O.SET_M, O.SET_S):
        g, greal = res[which]
        assert_same_set(g[greal == realization], os_.get_set(which),
                        "set %d" % which)
    k, a, real = res["state"]
    sel = real == realization
    gk, ga = sort_rows(k[sel], a[sel])
    ok, oa = os_.state()
    assert np.array_equal(gk, ok)
    assert_amps(ga, oa, tol)
    oo = dict(os_.observations()[-1])
    oo["mass_total"] += prev_mass_total
    check_obs(gobs, oo, tol, width=oo["E_max"] - oo["E_min"],
              drop=dropped(prev[0], prev[1], ok))
    return len(gk)


def test_ring16_bench_window_step_matches_oracle():
    cfg = dict(WL.CONFIGS["ring16"])
    params = WL.model_params(cfg)
    gs = P.Sim(P.Model(params), WL.run_params(cfg), *WL.initial_state(cfg))
    grown = 0
    while gs.size() < 10_000_000 and grown < 400:
        gs.step(1)
        grown += 1
    gs.autotune(steps=2)
    gs.step(5)
    keys, amps = gs.state()
    prev = gs.observations()[-1]
    print("ring16: %d + 5 steps, oracle step from %d rows" % (grown, len(keys)),
          flush=True)
    assert len(keys) > 10_000_000
    gs.profile(True, kernels_only=True)
    gs.step(1)
    gs.profile(False)
    os_ = oracle_step_from(cfg, params, keys, amps, prev["t"])
    n = compare_step(gpu_result(gs), gs.observations()[-1],
                     prev["mass_total"], os_, 1e-10, (keys, amps))
    assert n > 10_000_000
    # the Krylov form: an order-10 step from the same state
    gk = P.Sim(P.Model(params), dict(WL.run_params(cfg), krylov_order=10),
               *WL.initial_state(cfg))
    gk.set_state(keys, amps, prev["t"])
    gk.step(1)
    os_ = oracle_step_from(cfg, params, keys, amps, prev["t"],
                           krylov_order=10)
    compare_step(gpu_result(gk), gk.observations()[-1], 0.0, os_, 1e-10,
                 (keys, amps))


def test_sq6x6_batched_full_width_step_matches_oracle():
    cfg = dict(WL.CONFIGS["sq6x6"])
    steps = 40
    bs = P.Sim(P.Model(WL.batch_params(cfg)), WL.run_params(cfg),
               *WL.initial_state(cfg))
    bs.step(steps - 1)
    keys, amps, real = bs.state(with_real=True)
    rec = bs.series()
    bs.step(1)
    assert bs.size() > 100_000_000
    res = gpu_result(bs)
    for r in (0, 37):
        sel = real == r
        os_ = oracle_step_from(cfg, WL.model_params(cfg, r), keys[sel],
                               amps[sel], rec[-1, r, 0])
        compare_step(res, bs.observations(realization=r)[-1], rec[-1, r, 6],
                     os_, 1e-5, (keys[sel], amps[sel]), realization=r)
