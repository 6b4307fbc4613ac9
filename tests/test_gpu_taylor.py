"""Truncated Taylor propagator on the GPU vs the CPU oracle, through the C
ABI (paper: App. "The action of the exponential of a sparse matrix", with
the Al-Mohy & Higham degree and substep choice; App. "An effective Hilbert
space up to neighbor order m = 2 is not equivalent to a second-order Taylor
expansion" for the fixed order).

Key sets bit for bit, amplitudes within 1e-10 (FP64) or 1e-5 (FP32),
observables within tol * (|o| + scale), the number of products m s
exactly; the adaptive series equals the Chebyshev propagator; batched
realizations equal single runs."""
import numpy as np
import pytest

import paper_2603_07341_amd as P
from oracle import oracle as O
from tests.gpu_helpers import (assert_amps, assert_same_set, check_obs,
                               dropped, oracle_state, rel_err,
                               sort_rows)
import workloads as WL

pytestmark = pytest.mark.gpu


def pair(name, order, **over):
    cfg = dict(WL.CONFIGS[name])
    cfg.update(over)
    params = WL.model_params(cfg)
    run = dict(WL.run_params(cfg), taylor_order=order)
    init = WL.initial_state(cfg)
    return cfg, P.Sim(P.Model(params), run, *init), O.Sim(O.Model(params), run, *init)


def check_step(gs, os_, tol, prev=None, steps=1, mass_prior=0.0):
    """prev: the oracle's state the step started from (keys, amps), for
    the rows it dropped; steps: steps since the common state; mass_prior:
    the earlier steps' discarded-weight bounds.  Returns the step's bound."""
    for which in (O.SET_M, O.SET_S):
        assert_same_set(gs.get_set(which), os_.get_set(which), "set %d" % which)
    gk, ga = sort_rows(*gs.state())
    ok, oa = os_.state()
    assert np.array_equal(gk, ok)
    assert_amps(ga, oa, tol, steps=steps)
    go, oo = gs.observations()[-1], os_.observations()[-1]
    drop = dropped(prev[0], prev[1], ok) if prev is not None else None
    b = check_obs(go, oo, tol, width=oo["E_max"] - oo["E_min"], drop=drop,
                  steps_before=steps - 1, mass_prior=mass_prior)
    assert go["K"] == oo["terms"]
    for f in ("E_min", "E_max"):
        assert go[f] == pytest.approx(oo[f], rel=1e-13, abs=1e-13), f
    return b


@pytest.mark.parametrize("name,steps", [("ring16", 12), ("ring12", 10),
                                        ("sq6x6", 4), ("cube4", 3)])
def test_single_step_parity(name, steps):
    keys, amps, t = oracle_state(name, steps)
    cfg, gs, os_ = pair(name, -1, precision=64)
    gs.set_state(keys, amps, t)
    os_.set_state(keys, amps, t)
    gs.step(1)
    os_.step(1)
    check_step(gs, os_, 1e-10, prev=(keys, amps))


@pytest.mark.parametrize("order,dt", [(-1, 0.01), (-1, 1.0), (2, 0.01), (6, 0.05)])
def test_multi_step_runs_match_oracle(order, dt):
    # dt 1.0 makes the chosen plan take several substeps
    cfg, gs, os_ = pair("ring12", order, extent=[6, 1, 1], cutoff=[4],
                        theta=1e-6, dt=dt)
    acc = 0.0
    for i in range(12):
        prev = os_.state()
        gs.step(1)
        os_.step(1)
        acc += check_step(gs, os_, 1e-10, prev=prev, steps=i + 1,
                          mass_prior=acc)
    if order == -1 and dt == 1.0:
        K = gs.observations()[-1]["K"]
        m, s = O.taylor_select(0.5 * (gs.observations()[-1]["E_max"]
                                      - gs.observations()[-1]["E_min"]) * dt)
        assert K == m * s and s > 1


def test_fixed_order_two_gains_norm_without_truncation():
    cfg, gs, os_ = pair("ring12", 2, extent=[6, 1, 1], cutoff=[4], theta=0.0)
    gs.step(8)
    os_.step(8)
    n2 = [o["norm2"] for o in gs.observations()]
    assert all(y > x for x, y in zip(n2, n2[1:])) and n2[0] > 1.0
    check_step(gs, os_, 1e-10, steps=8)


def test_single_step_parity_fp32():
    keys, amps, t = oracle_state("ring16", 12)
    amps = amps.astype(np.complex64).astype(np.complex128)
    cfg, gs, os_ = pair("ring16", -1, precision=32)
    gs.set_state(keys, amps, t)
    os_.set_state(keys, amps, t)
    gs.step(1)
    os_.step(1)
    check_step(gs, os_, 1e-5, prev=(keys, amps))


def test_adaptive_series_equals_chebyshev():
    cfg = dict(WL.CONFIGS["ring16"])
    params = WL.model_params(cfg)
    init = WL.initial_state(cfg)
    a = P.Sim(P.Model(params), dict(WL.run_params(cfg), taylor_order=-1), *init)
    b = P.Sim(P.Model(params), WL.run_params(cfg), *init)
    a.step(20)
    b.step(20)
    ka, pa = sort_rows(*a.state())
    kb, pb = sort_rows(*b.state())
    assert np.array_equal(ka, kb)
    assert np.abs(pa - pb).max() <= 1e-12


def test_batched_realizations_match_single_runs():
    cfg = dict(WL.CONFIGS["sq6x6"])
    cfg.update(precision=64)
    R, steps = 3, 4
    init = WL.initial_state(cfg)
    run = dict(WL.run_params(cfg), taylor_order=-1)
    bs = P.Sim(P.Model(WL.batch_params(cfg, R)), run, *init)
    bs.step(steps)
    brec = bs.series()
    bk, ba, breal = bs.state(with_real=True)
    for r in range(R):
        s = P.Sim(P.Model(WL.model_params(cfg, r)), run, *init)
        s.step(steps)
        sk, sa = sort_rows(*s.state())
        rk, ra = sort_rows(bk[breal == r], ba[breal == r])
        assert np.array_equal(rk, sk), r
        assert_amps(ra, sa, 1e-12, steps=steps, what="realization %d" % r)
        srec = s.series()
        assert np.array_equal(brec[:, r, 7:12], srec[:, 7:12])
        assert np.allclose(brec[:, r, 1:7], srec[:, 1:7], rtol=1e-12, atol=1e-13)


def test_graph_replay_matches_eager():
    outs = []
    for graph in (0, 1):
        cfg, gs, _ = pair("ring16", -1)
        t = gs.tuning()
        gs.set_tuning(graph=graph, table_shift=t["table_shift"],
                      term_rows=t["term_rows"])
        gs.step(12)
        outs.append((sort_rows(*gs.state()), gs.series()))
    (k0, a0), r0 = outs[0]
    (k1, a1), r1 = outs[1]
    assert np.array_equal(k0, k1) and np.array_equal(a0, a1)
    assert np.allclose(r0, r1, rtol=1e-12, atol=1e-14)


def test_product_limit_latches_error_and_adjoint_refuses():
    cfg = dict(WL.CONFIGS["ring12"])
    params = WL.model_params(cfg)
    s = P.Sim(P.Model(params), dict(WL.run_params(cfg), taylor_order=-1),
              *WL.initial_state(cfg), k_max_terms=4)
    with pytest.raises(P.PacesError) as ei:
        s.step(1)
    assert ei.value.status == 5
    s = P.Sim(P.Model(params), dict(WL.run_params(cfg), taylor_order=-1),
              *WL.initial_state(cfg))
    with pytest.raises(P.PacesError) as ei:
        s.adjoint_forward(3)
    assert ei.value.status == 8
