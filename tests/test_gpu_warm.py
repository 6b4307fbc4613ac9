"""Steps that expand from the previous step's graph in place (tuning warm
= 1, the default, which lays the set out from scratch again after a tenth
of it went into holes, and warm = 2, in place throughout) against steps
that expand from scratch (warm = 0), through the C ABI.  Both compute B_k(M) and the columns of H_eff on it (Eqs.
(def_neighbor_k), (H_eff)); the rows come in another order, while every
row's arithmetic is the same, so per step: the same set S, the same
selection M and frontiers, every amplitude taken per basis state bit for
bit, counts, K and spectral bounds exact, sums to rounding (the Krylov
propagator's inner products are sums too: its amplitudes and Ritz
interval agree to rounding there).  The cases
cover complex64, several realizations, the 3D two-mode lattice with ten
key words, the Krylov and Taylor propagators, and the state cap and the
fixed-size truncation (whose cut selection repeats a step from the same
graph)."""
import numpy as np
import pytest

import paper_2603_07341_amd as P
from oracle import oracle as O
from tests.gpu_helpers import assert_amps, sort_rows
import workloads as WL

pytestmark = pytest.mark.gpu

EXACT = [0, 7, 8, 9, 10, 11]  # t, n_S, n_M, K, E_min, E_max


def pair(name, R, run_over, cfg_over=None, mode=1):
    cfg = dict(WL.CONFIGS[name])
    cfg.update(cfg_over or {})
    params = WL.batch_params(cfg, R) if R > 1 else WL.model_params(cfg)
    run = dict(WL.run_params(cfg), **run_over)
    init = WL.initial_state(cfg)
    warm = P.Sim(P.Model(params), run, *init)
    cold = P.Sim(P.Model(params), run, *init)
    cold.set_tuning(warm=0)
    assert warm.tuning()["warm"] == 1 and cold.tuning()["warm"] == 0
    if mode != 1:
        warm.set_tuning(warm=mode)
    return warm, cold


def full_state(s):
    k, a, r = s.state(with_real=True)
    full = np.concatenate([r[:, None].astype(np.uint64), k], axis=1)
    return sort_rows(full, a)


def keyed_phi(s):
    k, _, r = s.state(with_real=True)
    full = np.concatenate([r[:, None].astype(np.uint64), k], axis=1)
    return sort_rows(full, s.phi())[1]


def set_rows(s, which, rnd=0):
    k, r = s.get_set(which, rnd, with_real=True)
    full = np.concatenate([r[:, None].astype(np.uint64), k], axis=1)
    return full[np.lexsort(full.T[::-1])]


CASES = [
    ("ring16", 1, 60, {}, None),
    ("ring16", 1, 40, dict(precision=32), None),
    ("sq6x6", 4, 14, {}, None),
    ("cube4", 1, 7, {}, None),
    ("ring12", 1, 30, dict(krylov_order=6), None),
    ("ring12", 1, 30, dict(taylor_order=-1), None),
    ("ring12", 1, 40, dict(q_nom=4000), None),
    ("sq6x6", 3, 12, dict(max_states=30000), None),
]


@pytest.mark.parametrize("mode", [1, 2], ids=["relayout", "in-place"])
@pytest.mark.parametrize("name,R,steps,run_over,cfg_over", CASES,
                         ids=["ring16", "ring16-fp32", "sq6x6-R4", "cube4",
                              "krylov", "taylor", "q_nom", "cap"])
def test_warm_steps_equal_steps_from_scratch(name, R, steps, run_over,
                                             cfg_over, mode):
    """mode 1: the default (in place, from scratch again after a tenth of
    the set went into holes); mode 2: in place throughout."""
    warm, cold = pair(name, R, run_over, cfg_over, mode)
    k = WL.CONFIGS[name]["k"]
    krylov = "krylov_order" in run_over
    exact = EXACT[:4] if krylov else EXACT
    for i in range(steps):
        warm.step(1)
        cold.step(1)
        rw, rc = warm.series(i, 1), cold.series(i, 1)
        assert np.array_equal(rw[..., exact], rc[..., exact]), i
        assert np.allclose(rw, rc, rtol=1e-12, atol=1e-15), i
        if i % 4 == 3 or i == steps - 1:
            kw, aw = full_state(warm)
            kc, ac = full_state(cold)
            assert np.array_equal(kw, kc), i
            if krylov:
                assert_amps(aw, ac, 1e-12, what="step %d" % i)
            else:
                assert np.array_equal(aw, ac), i
            assert np.array_equal(set_rows(warm, O.SET_M),
                                  set_rows(cold, O.SET_M)), i
            for rnd in range(k + 1):
                assert np.array_equal(set_rows(warm, O.SET_FRONTIER, rnd),
                                      set_rows(cold, O.SET_FRONTIER, rnd)), \
                    (i, rnd)
            # phi of the transfer, per basis state
            if krylov:
                assert_amps(keyed_phi(warm), keyed_phi(cold), 1e-12)
            else:
                assert np.array_equal(keyed_phi(warm), keyed_phi(cold)), i


def test_warm_steps_across_a_growth_and_a_state_reload():
    """A capacity growth and a reloaded state both leave no graph: the next
    step expands from scratch, the ones after from the graph again."""
    warm, cold = pair("ring16", 1, {})
    warm.step(30)
    cold.step(30)
    keys, amps = warm.state()
    warm.set_state(keys, amps, 0.3)
    cold.set_state(keys, amps, 0.3)
    for i in range(30):
        warm.step(1)
        cold.step(1)
    kw, aw = full_state(warm)
    kc, ac = full_state(cold)
    assert np.array_equal(kw, kc)
    assert np.array_equal(aw, ac)
    rw, rc = warm.series(), cold.series()
    assert np.array_equal(rw[..., EXACT], rc[..., EXACT])


def test_warm_steps_under_a_state_cap_that_binds_every_step():
    """Under a state cap that cuts nearly every step, an in-place step can
    need more rows than the capacity (the old rows keep their places until
    the commit) where a step from scratch fits: that step repeats from
    scratch instead of growing the row arrays step after step.  The run
    stays equal to the one from scratch throughout."""
    warm, cold = pair("ring16", 1, dict(precision=32, max_states=200000,
                                        cap_hint=250000), mode=2)
    for i in range(300):
        warm.step(1)
        cold.step(1)
        rw, rc = warm.series(i, 1), cold.series(i, 1)
        assert np.array_equal(rw[..., EXACT], rc[..., EXACT]), i
        assert rw[0, 7] <= 200000, i
    kw, aw = full_state(warm)
    kc, ac = full_state(cold)
    assert np.array_equal(kw, kc)
    assert np.array_equal(aw, ac)


def test_in_place_step_repeats_its_propagation_when_the_series_grows():
    """A 6-site chain (cutoff 12, g 1, dt 0.5) grown from one state with
    k_init 1 and then k 6: the spectral interval widens so fast that the
    next steps need more Chebyshev terms than the K + 2 launches the host
    enqueued from the step before.  An in-place step has committed its
    set by then, so only its propagation and observables are repeated with
    more launches.  Every step against the oracle (sets bit for bit,
    amplitudes within 1e-10, observables) and against steps from scratch."""
    from tests.gpu_helpers import (assert_amps, assert_same_set, check_obs,
                                   dropped)
    cfg = dict(WL.CONFIGS["ring12"])
    cfg.update(extent=[6, 1, 1], cutoff=[12], g=[1.0], dt=0.5, k_init=1,
               k=6, theta=1e-7)
    p = WL.model_params(cfg)
    run = WL.run_params(cfg)
    init = WL.initial_state(cfg)
    warm = P.Sim(P.Model(p), run, *init)
    warm.set_tuning(warm=2)
    cold = P.Sim(P.Model(p), run, *init)
    cold.set_tuning(warm=0)
    os_ = O.Sim(O.Model(p), run, *init)
    acc = 0.0
    for step in range(4):
        prev = os_.state()
        warm.step(1)
        cold.step(1)
        os_.step(1)
        rw, rc = warm.series(step, 1), cold.series(step, 1)
        assert np.array_equal(rw[..., EXACT], rc[..., EXACT]), step
        for which in (O.SET_M, O.SET_S):  # both sorted by key
            assert_same_set(set_rows(warm, which)[:, 1:], os_.get_set(which),
                            "step %d set %d" % (step, which))
        kw, aw = full_state(warm)
        ok, oa = os_.state()
        assert np.array_equal(kw[:, 1:], ok), step
        assert_amps(aw, oa, 1e-10, steps=step + 1)
        go, oo = warm.observations()[-1], os_.observations()[-1]
        acc += check_obs(go, oo, 1e-10, width=oo["E_max"] - oo["E_min"],
                         drop=dropped(prev[0], prev[1], ok),
                         steps_before=step, mass_prior=acc)
    K = warm.series()[:, 9].astype(int)
    # steps that needed more than the K + 2 launches enqueued after the
    # step before
    assert np.count_nonzero(K[1:] > K[:-1] + 2) >= 2, K
