"""GPU path vs CPU oracle, through the C ABI, on identical seeded inputs.

Key sets (M, every frontier, S) must agree bit for bit; phi is a copy and
must agree bit for bit; propagated amplitudes within 1e-10 relative (FP64)
or 1e-5 (FP32), in 2-norm and element by element above a rounding floor;
observables within tol * (|o| + scale), the discarded weight relative to
the rows dropped."""
import numpy as np
import pytest

import paper_2603_07341_amd as P
from oracle import oracle as O
from tests.gpu_helpers import (assert_amps, assert_same_set, check_obs,
                               check_series, dropped, make_pair, oracle_state,
                               sort_rows)
import workloads as WL

pytestmark = pytest.mark.gpu


def step_both(gs, os_, keys, amps, t, k):
    gs.set_state(keys, amps, t)
    os_.set_state(keys, amps, t)
    gs.step(1)
    os_.step(1)
    for which in (O.SET_M, O.SET_S):
        assert_same_set(gs.get_set(which), os_.get_set(which), "set %d" % which)
    for r in range(k + 1):
        assert_same_set(gs.get_set(P.SET_FRONTIER, r),
                        os_.get_set(O.SET_FRONTIER, r), "frontier %d" % r)
    gk, ga = gs.state()
    gphi = gs.phi()
    ok, oa = os_.state()
    ophi = os_.phi()
    gk, ga, gphi = sort_rows(gk, ga, gphi)
    assert np.array_equal(gk, ok)
    # phi is a pure copy of psi entries: bit for bit
    assert np.array_equal(gphi, ophi)
    return ga, oa, dropped(keys, amps, ok)


def test_ring4_full_run_matches_oracle():
    cfg, gm, om, gs, os_ = make_pair("ring4")
    steps = cfg["steps"]
    gs.step(steps)
    os_.step(steps)
    gobs, oobs = gs.observations(), os_.observations()
    assert len(gobs) == len(oobs) == steps
    check_series(gobs, oobs, 1e-10, cfg["theta"], 1)
    for g, o in zip(gobs, oobs):
        assert g["t"] == o["t"]
        assert g["E_min"] == pytest.approx(o["E_min"], rel=1e-13, abs=1e-13)
        assert g["E_max"] == pytest.approx(o["E_max"], rel=1e-13, abs=1e-13)
    gk, ga = gs.state()
    ok, oa = os_.state()
    gk, ga = sort_rows(gk, ga)
    assert np.array_equal(gk, ok)
    assert_amps(ga, oa, 1e-10, steps=steps)
    assert len(gk) == 2500  # the run reaches the whole sector


@pytest.mark.parametrize("name,steps", [("ring16", 12), ("ring12", 10),
                                        ("sq6x6", 4), ("cube4", 3)])
def test_single_step_parity(name, steps):
    keys, amps, t = oracle_state(name, steps)
    cfg, gm, om, gs, os_ = make_pair(name, precision=64)
    ga, oa, drop = step_both(gs, os_, keys, amps, t, cfg["k"])
    assert_amps(ga, oa, 1e-10)
    go, oo = gs.observations()[-1], os_.observations()[-1]
    check_obs(go, oo, 1e-10, width=oo["E_max"] - oo["E_min"], drop=drop)


@pytest.mark.parametrize("name,steps", [("ring16", 12), ("sq6x6", 4),
                                        ("cube4", 3)])
def test_single_step_parity_fp32(name, steps):
    # complex64 amplitudes, FP64 scalars and reductions; inputs chosen
    # representable in FP32 so both sides select from identical weights
    keys, amps, t = oracle_state(name, steps)
    amps = amps.astype(np.complex64).astype(np.complex128)
    cfg, gm, om, gs, os_ = make_pair(name, precision=32)
    ga, oa, drop = step_both(gs, os_, keys, amps, t, cfg["k"])
    assert_amps(ga, oa, 1e-5)
    go, oo = gs.observations()[-1], os_.observations()[-1]
    check_obs(go, oo, 1e-5, width=oo["E_max"] - oo["E_min"], drop=drop)


@pytest.mark.parametrize("theta", [0.0, 1e-6, 1e-3])
@pytest.mark.parametrize("k", [0, 1, 3])
def test_threshold_and_order_edge_cases(theta, k):
    keys, amps, t = oracle_state("ring16", 8)
    cfg, gm, om, gs, os_ = make_pair("ring16", theta=theta, k=k)
    ga, oa, drop = step_both(gs, os_, keys, amps, t, k)
    assert_amps(ga, oa, 1e-10)
    go, oo = gs.observations()[-1], os_.observations()[-1]
    check_obs(go, oo, 1e-10, width=oo["E_max"] - oo["E_min"], drop=drop)
    if theta > 0:
        assert drop[0] > 0 and oo["mass_step"] > 0


def test_everything_truncated():
    # theta above every amplitude: M and S are empty, all weight discarded
    keys, amps, t = oracle_state("ring16", 5)
    cfg, gm, om, gs, os_ = make_pair("ring16", theta=10.0)
    gs.set_state(keys, amps, t)
    os_.set_state(keys, amps, t)
    gs.step(1)
    os_.step(1)
    assert gs.size() == 0 and os_.size() == 0
    go, oo = gs.observations()[-1], os_.observations()[-1]
    assert go["norm2"] == 0.0
    assert go["mass_step"] == pytest.approx(oo["mass_step"], rel=1e-12)


def test_single_state_and_long_run_parity():
    cfg, gm, om, gs, os_ = make_pair("ring16")
    for i in range(4):
        gs.step(10)
        os_.step(10)
        gk, ga = gs.state()
        ok, oa = os_.state()
        gk, ga = sort_rows(gk, ga)
        assert np.array_equal(gk, ok)
        assert_amps(ga, oa, 1e-10, steps=10 * (i + 1))
    check_series(gs.observations(), os_.observations(), 1e-10, cfg["theta"],
                 len(WL.initial_state(cfg)[0]))


def test_two_runs_are_bitwise_identical():
    # Row order may differ between runs (new rows are numbered in the order
    # the table admits them); the set and every amplitude, taken per basis
    # state, must not.
    outs = []
    for _ in range(2):
        cfg, gm, om, gs, os_ = make_pair("ring16")
        gs.step(15)
        k, a = gs.state()
        outs.append(sort_rows(k, a))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


def test_series_limit_latches_error():
    cfg = WL.CONFIGS["ring4"]
    gm = P.Model(WL.model_params(cfg))
    exc, occ, coef = WL.initial_state(cfg)
    gs = P.Sim(gm, WL.run_params(cfg), exc, occ, coef, k_max_terms=2)
    with pytest.raises(P.PacesError) as ei:
        gs.step(1)
    assert ei.value.status == 5
    with pytest.raises(P.PacesError) as ei:
        gs.step(1)
    assert ei.value.status == 7


def test_duplicate_input_rejected():
    cfg = WL.CONFIGS["ring4"]
    gm = P.Model(WL.model_params(cfg))
    with pytest.raises(P.PacesError) as ei:
        P.Sim(gm, WL.run_params(cfg), [0, 0], [0] * 8, [0.6, 0, 0.8, 0])
    assert ei.value.status == 1


def test_piecewise_constant_hamiltonian_matches_oracle():
    cfg = dict(WL.CONFIGS["ring12"])
    cfg.update(extent=[6, 1, 1], cutoff=[4], theta=1e-6)
    pa = WL.model_params(cfg)
    pb = dict(pa, J=[-0.6, 0.0, 0.0], g=[1.3, 0, 0, 0],
              eps=list(np.asarray(pa["eps"]) + 0.05))
    run = WL.run_params(cfg)
    init = WL.initial_state(cfg)
    ga, gb = P.Model(pa), P.Model(pb)
    oa, ob = O.Model(pa), O.Model(pb)
    gs = P.Sim(ga, run, *init)
    os_ = O.Sim(oa, run, *init)
    gs.step(5)
    os_.step(5)
    gs.set_model(gb)
    os_.set_model(ob)
    gs.step(5)
    os_.step(5)
    gk, gv = sort_rows(*gs.state())
    ok, ov = os_.state()
    assert np.array_equal(gk, ok)
    assert_amps(gv, ov, 1e-10, steps=10)
    check_series(gs.observations(), os_.observations(), 1e-10, cfg["theta"],
                 len(init[0]))
    with pytest.raises(P.PacesError):
        gs.set_model(P.Model(WL.model_params(dict(cfg, extent=[7, 1, 1]))))


def test_non_finite_inputs_and_overflow_latch():
    """Non-finite amplitudes are refused at the boundary; a spectrum whose
    width overflows FP64 (site energies +-1e308) latches a non-finite
    norm, after which steps are refused until the state is set again."""
    cfg = dict(WL.CONFIGS["ring4"])
    p = WL.model_params(cfg)
    run = WL.run_params(cfg)
    exc, occ, coef = WL.initial_state(cfg)
    with pytest.raises(P.PacesError) as ei:
        P.Sim(P.Model(p), run, exc, occ, [float("nan"), 0.0])
    assert ei.value.status == 1
    s = P.Sim(P.Model(p), run, exc, occ, coef)
    s.step(2)
    keys, amps = s.state()
    bad = amps.copy()
    bad[0] = complex(float("inf"), 0)
    with pytest.raises(P.PacesError) as ei:
        s.set_state(keys, bad, 0.0)
    assert ei.value.status == 1
    q = dict(p, eps=[1e308, -1e308, 0.0, 0.0])
    s = P.Sim(P.Model(q), run, exc, occ, coef)
    with pytest.raises(P.PacesError) as ei:
        s.step(1)
    assert ei.value.status == 4
    with pytest.raises(P.PacesError) as ei:
        s.step(1)
    assert ei.value.status == 7
    s.set_state(keys, amps, 0.0)  # clears the latch
