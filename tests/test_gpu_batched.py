"""Batched disorder realizations through the C ABI: R states share one set,
one hash table and one launch per stage.

Each realization of a batched sim must reproduce a sim of that realization
alone on the same GPU (key sets bit for bit, amplitudes and observables
within 1e-12, counts, K and spectral bounds exact), and the CPU oracle
within the FP64 / FP32 tolerances of the single-realization parity tests."""
import numpy as np
import pytest

import paper_2603_07341_amd as P
from oracle import oracle as O
from tests.gpu_helpers import assert_amps, check_series, rel_err, sort_rows
import workloads as WL

pytestmark = pytest.mark.gpu


def cfg_of(name, **over):
    cfg = dict(WL.CONFIGS[name])
    cfg.update(over)
    return cfg


def batched_sim(cfg, R, first=0):
    bm = P.Model(WL.batch_params(cfg, R, first))
    exc, occ, coef = WL.initial_state(cfg)
    return bm, P.Sim(bm, WL.run_params(cfg), exc, occ, coef)


def single_sim(cfg, r):
    m = P.Model(WL.model_params(cfg, r))
    exc, occ, coef = WL.initial_state(cfg)
    return m, P.Sim(m, WL.run_params(cfg), exc, occ, coef)


def part(keys, amps, real, r):
    sel = real == r
    return sort_rows(keys[sel], amps[sel])


def compare_to_single(cfg, bs, brec, r, steps, amp_tol):
    bk, ba, breal = bs.state(with_real=True)
    _, s = single_sim(cfg, r)
    s.step(steps)
    sk, sa = sort_rows(*s.state())
    rk, ra = part(bk, ba, breal, r)
    assert np.array_equal(rk, sk), "realization %d: key set" % r
    assert_amps(ra, sa, amp_tol, steps=steps, what="realization %d" % r)
    srec = s.series()
    # time, counts, K and the Gershgorin interval are exact
    assert np.array_equal(brec[:, r, 0], srec[:, 0])
    assert np.array_equal(brec[:, r, 7:12], srec[:, 7:12])
    # sums differ from the single run only in reduction order
    assert np.allclose(brec[:, r, 1:7], srec[:, 1:7], rtol=1e-12, atol=1e-13)
    assert np.allclose(brec[:, r, 12:], srec[:, 12:], rtol=1e-12, atol=1e-13)
    return len(sk)


@pytest.mark.parametrize("name,R,steps,over", [
    ("ring12", 5, 25, {}),
    ("sq6x6", 4, 6, {"precision": 64}),
    ("sq6x6", 4, 6, {}),  # complex64 amplitudes
])
def test_batched_equals_single_realizations(name, R, steps, over):
    cfg = cfg_of(name, **over)
    bm, bs = batched_sim(cfg, R)
    bs.step(steps)
    brec = bs.series()
    assert brec.shape == (steps, R, bm.rec_doubles)
    total = sum(compare_to_single(cfg, bs, brec, r, steps, 1e-12)
                for r in range(R))
    assert total == bs.size()


def test_batched_full_width_sq6x6():
    """64 realizations of the 2D workload in one sim; a few of them checked
    against single-realization runs."""
    cfg = cfg_of("sq6x6")
    bm, bs = batched_sim(cfg, 64)
    steps = 4
    bs.step(steps)
    brec = bs.series()
    sizes = brec[-1, :, 7]
    assert sizes.sum() == bs.size()
    for r in (0, 21, 63):
        compare_to_single(cfg, bs, brec, r, steps, 1e-12)


@pytest.mark.parametrize("name,R,steps,over,tol", [
    ("ring12", 3, 15, {}, 1e-10),
    ("sq6x6", 3, 4, {"precision": 64}, 1e-10),
])
def test_batched_matches_oracle(name, R, steps, over, tol):
    cfg = cfg_of(name, **over)
    bm, bs = batched_sim(cfg, R, first=2)
    bs.step(steps)
    bk, ba, breal = bs.state(with_real=True)
    exc, occ, coef = WL.initial_state(cfg)
    for r in range(R):
        om = O.Model(WL.model_params(cfg, 2 + r))
        os_ = O.Sim(om, WL.run_params(cfg), exc, occ, coef)
        os_.step(steps)
        ok, oa = os_.state()
        rk, ra = part(bk, ba, breal, r)
        assert np.array_equal(rk, ok)
        assert_amps(ra, oa, tol, steps=steps)
        check_series(bs.observations(r), os_.observations(), tol,
                     cfg["theta"], len(exc))


def test_identical_realizations_give_identical_states():
    """Without disorder every realization is the same problem."""
    cfg = cfg_of("ring12", eps_sigma=0.0)
    bm, bs = batched_sim(cfg, 3)
    bs.step(12)
    bk, ba, breal = bs.state(with_real=True)
    k0, a0 = part(bk, ba, breal, 0)
    for r in (1, 2):
        kr, ar = part(bk, ba, breal, r)
        assert np.array_equal(kr, k0)
        assert np.array_equal(ar, a0)
    rec = bs.series()
    assert np.array_equal(rec[:, 0, 7:12], rec[:, 2, 7:12])


def test_batched_sets_and_state_round_trip():
    cfg = cfg_of("ring12")
    R, steps = 3, 6
    bm, bs = batched_sim(cfg, R)
    bs.step(steps)
    for r in range(R):
        _, s = single_sim(cfg, r)
        s.step(steps)
        for which in (P.SET_M, P.SET_S):
            k, real = bs.get_set(which, with_real=True)
            a = sort_rows(k[real == r])[0]
            b = sort_rows(s.get_set(which))[0]
            assert np.array_equal(a, b), (r, which)
        for rnd in range(cfg["k"] + 1):
            k, real = bs.get_set(P.SET_FRONTIER, rnd, with_real=True)
            a = sort_rows(k[real == r])[0]
            b = sort_rows(s.get_set(P.SET_FRONTIER, rnd))[0]
            assert np.array_equal(a, b), (r, rnd)
    keys, amps, real = bs.state(with_real=True)
    t = bs.observations(0)[-1]["t"]
    # restart a second batched sim from the state and step both once more
    _, b2 = batched_sim(cfg, R)
    b2.set_state(keys, amps, t, real=real)
    k2, a2, r2 = b2.state(with_real=True)
    for r in range(R):
        x, y = part(keys, amps, real, r), part(k2, a2, r2, r)
        assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])
    bs.step(1)
    b2.step(1)
    ka, aa, ra_ = bs.state(with_real=True)
    kb, ab, rb_ = b2.state(with_real=True)
    for r in range(R):
        x, y = part(ka, aa, ra_, r), part(kb, ab, rb_, r)
        assert np.array_equal(x[0], y[0])
        assert rel_err(y[1], x[1]) <= 1e-12


def test_batched_set_state_validation():
    cfg = cfg_of("ring12")
    bm, bs = batched_sim(cfg, 2)
    keys, amps, real = bs.state(with_real=True)
    with pytest.raises(P.PacesError) as ei:
        bs.set_state(keys, amps, 0.0, real=np.full(len(keys), 2, np.int32))
    assert ei.value.status == 1
    # the same state twice in one realization is rejected; once in each is
    # fine (the initial state has one row per realization per term)
    dup = np.zeros(len(keys), np.int32)
    with pytest.raises(P.PacesError) as ei:
        bs.set_state(keys, amps, 0.0, real=dup)
    assert ei.value.status == 1
    bs.set_state(keys, amps, 0.0, real=real)
    bs.step(1)
    assert bs.num_records() == 1
