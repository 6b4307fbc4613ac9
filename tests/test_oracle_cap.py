"""Pins of the oracle's state cap (the cube4 workload's |S| budget).

When the ball of M would exceed the cap, M is cut to a prefix of M in the
order (weight descending, splitmix64 hash of the key ascending, key
ascending).  Checked here from the outside: |S| never exceeds the cap,
the kept rows are exactly such a prefix of the threshold selection of the
previous state (with the hash computed here from the published splitmix64
definition), the cut is no larger than the first estimate q0, a cap that
never binds changes nothing, and equal weights on the orbits of a
translation-invariant ring are broken by the hash."""
import numpy as np
import pytest

from oracle import oracle as O
import workloads as WL

MASK = (1 << 64) - 1


def mix(x):
    """splitmix64 output function (Steele, Lea & Flood 2014)."""
    z = (x + 0x9E3779B97F4A7C15) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def key_hash(key):
    h = 0
    for w in key:
        h = mix(h ^ int(w))
    return h


def run_case(cap, steps, **over):
    cfg = dict(WL.CONFIGS["ring12"])
    cfg.update(dict(extent=[6, 1, 1], cutoff=[4], theta=1e-6, k=2, k_init=2))
    cfg.update(over)
    p = WL.model_params(cfg)
    run = WL.run_params(cfg)
    run["max_states"] = cap
    m = O.Model(p)
    s = O.Sim(m, run, *WL.initial_state(cfg))
    D = m.D
    prev = s.state()
    prev_counts = None
    bound_hits = 0
    for step in range(steps):
        th2 = cfg["theta"] ** 2
        s.step(1)
        obs = s.observations()[-1]
        assert obs["n_S"] <= cap
        M = s.get_set(O.SET_M)
        keys, amps = prev
        w = amps.real * amps.real + amps.imag * amps.imag
        full = keys if step == 0 else keys[w >= th2]
        wf = w if step == 0 else w[w >= th2]
        if len(M) < len(full):
            bound_hits += 1
            order = sorted(range(len(full)), key=lambda i: (
                -wf[i], key_hash(full[i]), tuple(int(x) for x in full[i])))
            kept = {tuple(int(x) for x in full[i]) for i in order[:len(M)]}
            assert kept == {tuple(int(x) for x in k) for k in M}, step
            q0 = (cap // (D + 1) if step == 0 or not prev_counts
                  else cap * prev_counts[1] // prev_counts[0])
            assert len(M) <= q0
        else:
            assert len(M) == len(full)
        prev_counts = (int(obs["n_S"]), int(obs["n_M"]))
        prev = s.state()
    return s, bound_hits


def test_cap_bounds_the_set_and_keeps_the_heaviest_prefix():
    s, hits = run_case(400, 12)
    assert hits >= 3  # the cap binds on several steps


def test_cap_on_translation_invariant_ring_breaks_ties_by_hash():
    # Bloch start, no disorder: weights repeat on the orbits of the ring,
    # so the cut falls inside groups of equal weight
    s, hits = run_case(300, 8, init="bloch", eps_sigma=0.0)
    assert hits >= 2
    keys, amps = s.state()
    w = np.round(np.abs(amps) ** 2, 300)
    assert len(np.unique(w)) < len(w)


def test_cap_that_never_binds_changes_nothing():
    a, hits = run_case(10 ** 9, 8)
    assert hits == 0
    cfg = dict(WL.CONFIGS["ring12"])
    cfg.update(dict(extent=[6, 1, 1], cutoff=[4], theta=1e-6, k=2, k_init=2))
    p = WL.model_params(cfg)
    b = O.Sim(O.Model(p), WL.run_params(cfg), *WL.initial_state(cfg))
    b.step(8)
    ka, aa = a.state()
    kb, ab = b.state()
    assert np.array_equal(ka, kb) and np.array_equal(aa, ab)


def test_cap_smaller_than_any_ball_truncates_everything():
    s, _ = run_case(1, 2)
    assert s.observations()[-1]["n_S"] <= 1


@pytest.mark.parametrize("over", [{}, dict(init="bloch", eps_sigma=0.0)])
def test_fixed_size_truncation_keeps_the_heaviest_q(over):
    """q_nom mode (the paper's fixed number of retained amplitudes): after
    the first step M is the q heaviest rows of the previous set, in the
    same order as the cap, whatever the threshold."""
    cfg = dict(WL.CONFIGS["ring12"])
    cfg.update(dict(extent=[6, 1, 1], cutoff=[4], theta=0.5, k=2, k_init=2))
    cfg.update(over)
    run = WL.run_params(cfg)
    q = 60
    run["q_nom"] = q
    s = O.Sim(O.Model(WL.model_params(cfg)), run, *WL.initial_state(cfg))
    s.step(1)
    for step in range(6):
        keys, amps = s.state()
        w = amps.real * amps.real + amps.imag * amps.imag
        s.step(1)
        M = s.get_set(O.SET_M)
        assert len(M) == min(q, len(keys))
        order = sorted(range(len(keys)), key=lambda i: (
            -w[i], key_hash(keys[i]), tuple(int(x) for x in keys[i])))
        kept = {tuple(int(x) for x in keys[i]) for i in order[:len(M)]}
        assert kept == {tuple(int(x) for x in k) for k in M}, step
