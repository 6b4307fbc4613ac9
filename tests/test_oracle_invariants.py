"""Invariants of truncation, detruncation and lattice symmetries that pin
the oracle (Sec. "Truncation & post-adaptation detruncation"; App.
"Invariance of localized-state dynamics")."""
import numpy as np
import pytest

from oracle import oracle as O
from tests.test_oracle_model import make
import workloads as WL


def keyset(keys):
    return {tuple(int(w) for w in k) for k in keys}


def small_ring(theta, J=-1.0, N=6, cut=3, eps=None, init="local"):
    cfg = dict(WL.CONFIGS["ring16"], extent=[N, 1, 1], cutoff=[cut], J=[J],
               g=[1.2], theta=theta)
    p = WL.model_params(cfg)
    if eps is not None:
        p["eps"] = eps
    m = O.Model(p)
    exc, occ, coef = WL.initial_state(cfg, init)
    s = O.Sim(m, dict(WL.run_params(cfg), k=2, k_init=2), exc, occ, coef)
    return cfg, m, s


@pytest.mark.parametrize("theta", [0.0, 1e-6, 1e-4, 1e-3])
def test_truncation_invariants(theta):
    cfg, m, s = small_ring(theta)
    s.step(3)
    for _ in range(15):
        prev_keys, prev_amps = s.state()
        s.step(1)
        o = s.observations()[-1]
        M = keyset(s.get_set(O.SET_M))
        S = keyset(s.get_set(O.SET_S))
        prev = keyset(prev_keys)
        # M is exactly the brute-force threshold predicate |c|^2 >= theta^2
        w = prev_amps.real * prev_amps.real + prev_amps.imag * prev_amps.imag
        want = {tuple(int(x) for x in prev_keys[i])
                for i in range(len(prev_keys)) if w[i] >= theta * theta}
        assert M == want
        assert M <= prev and M <= S
        # frontier 0 is M; frontiers partition S
        fr = [keyset(s.get_set(O.SET_FRONTIER, r)) for r in range(3)]
        assert fr[0] == M
        assert set().union(*fr) == S and sum(len(f) for f in fr) == len(S)
        # discarded mass: weight of prev \ S; phi keeps the rest
        lost = sum(w[i] for i in range(len(prev_keys))
                   if tuple(int(x) for x in prev_keys[i]) not in S)
        assert o["mass_step"] >= 0.0
        assert abs(o["mass_step"] - lost) <= 1e-15
        phi = s.phi()
        assert abs(np.vdot(phi, phi).real - (w.sum() - o["mass_step"])) <= 1e-14
        if theta == 0.0:
            assert o["mass_step"] == 0.0 and M == prev


def test_higher_threshold_selects_subset():
    cfg, m, s = small_ring(1e-5)
    s.step(10)
    keys, amps = s.state()
    sets = []
    for th in [0.0, 1e-8, 1e-5, 1e-3, 1e-1]:
        s2 = O.Sim(m, dict(WL.run_params(cfg), k=2, k_init=2, theta=th),
                   [0], [0] * 6, [1.0, 0.0])
        s2.set_state(keys, amps, 0.1)
        s2.step(1)
        sets.append(keyset(s2.get_set(O.SET_M)))
    for a, b in zip(sets, sets[1:]):
        assert b <= a


@pytest.mark.parametrize("shape", [([6], [1]), ([4, 4], [1, 1]), ([5], [0])])
def test_hopping_sign_flip_is_exact(shape):
    # J -> -J on a bipartite lattice with a localized start: the gauge
    # (-1)^parity(j) maps one run onto the other, so weights and key sets
    # agree bit for bit (App. "Invariance of localized-state dynamics").
    ext, per = shape
    nd = len(ext)
    runs = []
    for sign in (1.0, -1.0):
        cfg = dict(WL.CONFIGS["ring16"], ndim=nd,
                   extent=ext + [1] * (3 - nd), periodic=per + [0] * (3 - nd),
                   cutoff=[3], J=[sign * -0.8] * nd, g=[1.0], theta=1e-6)
        p = WL.model_params(cfg)
        m = O.Model(p)
        N = int(np.prod(ext))
        s = O.Sim(m, dict(WL.run_params(cfg), k=2, k_init=2), [1], [0] * N,
                  [1.0, 0.0])
        s.step(25)
        keys, amps = s.state()
        runs.append((keys, amps, s.observations()))
    (k1, a1, o1), (k2, a2, o2) = runs
    assert np.array_equal(k1, k2)
    w1 = a1.real * a1.real + a1.imag * a1.imag
    w2 = a2.real * a2.real + a2.imag * a2.imag
    assert np.array_equal(w1, w2)
    for x, y in zip(o1, o2):
        assert np.array_equal(x["pop"], y["pop"])
        assert x["norm2"] == y["norm2"] and x["n_S"] == y["n_S"]


def test_translation_invariance_of_bloch_start():
    # uniform eps and the k=0 Bloch start on a ring: S is closed under the
    # lattice translation and weights are equal on translation orbits.
    N = 6
    cfg, m, s = small_ring(1e-7, N=N, cut=3, init="bloch")
    s.step(12)
    keys, amps = s.state()
    e, o = m.unpack(keys)
    w = {}
    for i in range(len(e)):
        w[(int(e[i]), tuple(o[i].tolist()))] = abs(amps[i]) ** 2
    for (j, occ), wt in w.items():
        j2 = (j + 1) % N
        occ2 = occ[-1:] + occ[:-1]
        assert (j2, occ2) in w
        assert abs(w[(j2, occ2)] - wt) <= 1e-13 * max(wt, 1e-300) + 1e-30


def test_duplicate_input_rejected():
    p = WL.model_params(WL.CONFIGS["ring4"])
    m = O.Model(p)
    with pytest.raises(RuntimeError):
        O.Sim(m, WL.run_params(WL.CONFIGS["ring4"]), [0, 0], [0] * 8,
              [0.6, 0, 0.8, 0])


def test_series_term_limit_raises():
    p = WL.model_params(WL.CONFIGS["ring4"])
    m = O.Model(p)
    exc, occ, coef = WL.initial_state(WL.CONFIGS["ring4"])
    s = O.Sim(m, WL.run_params(WL.CONFIGS["ring4"]), exc, occ, coef,
              max_terms=3)
    with pytest.raises(RuntimeError):
        s.step(1)
