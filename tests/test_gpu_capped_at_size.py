"""The state cap at the batched and 3D workloads' sizes, GPU vs oracle
through the C ABI.

sq6x6 (complex64, D = 6, three key words, cap 1e7 states per realization):
four of its disorder realizations in one sim grow from the start until the
cap binds for each.  The oracle then redoes one capped step of one
realization from the GPU state before it, given the counts of the step
before that (the cap's q rule reads them): M and S bit for bit, amplitudes
within 1e-5 element by element, and the cut was active (M smaller than
the threshold selection).

cube4 (complex64, two modes, D = 10, ten key words) at a cap of 4e6, where
the oracle can redo a step: grown until the cap binds, then the same
comparison.  The state cap at cube4's own 5e8 is measured by the benchmark
(bench.py --cube4-cap), not compared here: one oracle step at that size
does not fit a test."""
import numpy as np
import pytest

import paper_2603_07341_amd as P
from oracle import oracle as O
from tests.gpu_helpers import (assert_amps, assert_same_set, check_obs,
                               dropped, sort_rows)
import workloads as WL

pytestmark = pytest.mark.gpu


def records(sim, first=0, n=None):
    """Records as [n, R, fields] whatever R."""
    rec = sim.series(first, n)
    return rec if rec.ndim == 3 else rec[:, None, :]


def grow_until_capped(sim, R, cap, max_steps, settle=3):
    """Step until every realization's set has reached 90% of the cap, then
    `settle` more steps; returns the records."""
    for step in range(max_steps):
        sim.step(1)
        last = records(sim, sim.num_records() - 1, 1)[0]
        print("step %d: |S| per realization %s" % (step, last[:, 7].astype(np.int64)),
              flush=True)
        if np.all(last[:, 7] >= 0.9 * cap):
            break
    else:
        raise AssertionError("the cap did not bind within %d steps" % max_steps)
    sim.step(settle)
    rec = records(sim)
    assert np.all(rec[:, :, 7] <= cap)
    return rec


def redo_capped_step(sim, params, cfg, run, r, cap):
    """One more GPU step; the oracle redoes it for realization r from the
    GPU state before it.  Returns the oracle sim."""
    keys, amps, real = sim.state(with_real=True)
    rec = records(sim)
    sel = real == r
    k0, a0 = keys[sel], amps[sel]
    sim.step(1)
    print("oracle redoes one step of realization %d from %d rows" % (r, len(k0)),
          flush=True)
    os_ = O.Sim(O.Model(params), run, *WL.initial_state(cfg))
    os_.set_state(k0, a0, rec[-1, r, 0])
    os_.set_prev_counts(rec[-1, r, 7], rec[-1, r, 8])
    os_.step(1)
    for which in (O.SET_M, O.SET_S):
        g, greal = sim.get_set(which, with_real=True)
        assert_same_set(g[greal == r], os_.get_set(which), "set %d" % which)
    k, a, rr = sim.state(with_real=True)
    gk, ga = sort_rows(k[rr == r], a[rr == r])
    ok, oa = os_.state()
    assert np.array_equal(gk, ok)
    assert_amps(ga, oa, 1e-5)
    oo = dict(os_.observations()[-1])
    oo["mass_total"] += rec[-1, r, 6]
    go = sim.observations(realization=r)[-1]
    assert go["n_S"] <= cap
    check_obs(go, oo, 1e-5, width=oo["E_max"] - oo["E_min"],
              drop=dropped(k0, a0, ok))
    # the cut was active: M is smaller than the threshold's selection
    w = a0.real ** 2 + a0.imag ** 2
    n_thr = int(np.count_nonzero(w >= run["theta"] * run["theta"]))
    assert oo["n_M"] < n_thr, (oo["n_M"], n_thr)
    return os_


def test_sq6x6_realizations_at_their_cap():
    cfg = dict(WL.CONFIGS["sq6x6"])
    R, cap = 4, cfg["max_states"]
    run = WL.run_params(cfg)
    sim = P.Sim(P.Model(WL.batch_params(cfg, R)), run, *WL.initial_state(cfg))
    grow_until_capped(sim, R, cap, 150)
    redo_capped_step(sim, WL.model_params(cfg, 1), cfg, run, 1, cap)


def test_cube4_at_an_oracle_sized_cap():
    cfg = dict(WL.CONFIGS["cube4"])
    cap = 4_000_000
    run = dict(WL.run_params(cfg), max_states=cap)
    params = WL.model_params(cfg)
    sim = P.Sim(P.Model(params), run, *WL.initial_state(cfg))
    grow_until_capped(sim, 1, cap, 200)
    redo_capped_step(sim, params, cfg, run, 0, cap)
