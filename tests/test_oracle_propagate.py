"""Pins of the oracle's propagation and observables against dense matrix
exponentials and closed forms."""
import cmath
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import oracle as O
from tests import brute
from tests.test_oracle_model import make
import workloads as WL


def amps_in_brute_order(p, m, keys, amps, dim):
    e, o = m.unpack(keys)
    v = np.zeros(dim, dtype=complex)
    for i in range(len(e)):
        v[brute.state_index(p, int(e[i]), o[i])] = amps[i]
    return v


def test_series_matches_dense_expm_on_random_matrices():
    rng = np.random.default_rng(5)
    for n, scale, dt in [(30, 1.0, 0.01), (50, 40.0, 0.3), (80, 5.0, 1.7)]:
        A = sp.random(n, n, density=0.1, random_state=rng.integers(1 << 30))
        H = (A + A.T).toarray() * scale + np.diag(rng.normal(size=n) * scale)
        Hc = sp.csr_matrix(H)
        Hc.sort_indices()
        # any interval containing the spectrum is valid for the shift
        ev = np.linalg.eigvalsh(H)
        v = rng.normal(size=n) + 1j * rng.normal(size=n)
        out, terms = O.expmv(Hc.indptr, Hc.indices, Hc.data, dt,
                             ev[0] - 0.1, ev[-1] + 0.1, v)
        ref = sla.expm(-1j * dt * H) @ v
        assert np.linalg.norm(out - ref) <= 1e-13 * np.linalg.norm(ref)


def ring4_exact(p, steps, dt):
    H = brute.dense_hamiltonian(p)
    U = sla.expm(-1j * dt * H)
    psi = np.zeros(H.shape[0], dtype=complex)
    psi[brute.state_index(p, 0, [0] * 4)] = 1.0
    out = []
    for _ in range(steps):
        psi = U @ psi
        out.append(psi.copy())
    return H, out


def test_full_space_run_matches_dense_expm():
    # ring4 workload with the first step grown over the whole 2500-state
    # sector and no truncation: the method is then exact.
    cfg = WL.CONFIGS["ring4"]
    p = WL.model_params(cfg)
    m = O.Model(p)
    exc, occ, coef = WL.initial_state(cfg)
    s = O.Sim(m, dict(WL.run_params(cfg), theta=0.0, k=4, k_init=60),
              exc, occ, coef)
    steps = 60
    H, exact = ring4_exact(p, steps, cfg["dt"])
    for i in range(steps):
        s.step(1)
        keys, amps = s.state()
        assert len(keys) == 2500
        v = amps_in_brute_order(p, m, keys, amps, 2500)
        assert np.linalg.norm(v - exact[i]) <= 1e-12
    obs = s.observations()
    # conservation without truncation (norm and energy), T9
    E0 = 0.0  # localized vacuum start with eps = 0
    for o in obs:
        assert abs(o["norm2"] - 1.0) <= 1e-12
        assert abs(o["energy"] - E0) <= 1e-12
        assert o["mass_step"] == 0.0


def test_configured_ring4_run_tracks_dense_expm():
    # ring4 as configured (k = 4, threshold 1e-10): the deviation from the
    # exact evolution stays below the accumulated discarded amplitude plus
    # the restriction error of the first steps (before S covers the space).
    cfg = WL.CONFIGS["ring4"]
    p = WL.model_params(cfg)
    m = O.Model(p)
    exc, occ, coef = WL.initial_state(cfg)
    s = O.Sim(m, WL.run_params(cfg), exc, occ, coef)
    steps = 200
    H, exact = ring4_exact(p, steps, cfg["dt"])
    s.step(steps)
    obs = s.observations()
    keys, amps = s.state()
    v = amps_in_brute_order(p, m, keys, amps, 2500)
    err = np.linalg.norm(v - exact[-1])
    bound = sum(math.sqrt(o["mass_step"]) for o in obs)
    assert err <= bound + 1e-8
    # norm loss equals the discarded weight, step by step
    prev = 1.0
    for o in obs:
        assert abs(prev - o["mass_step"] - o["norm2"]) <= 1e-14
        prev = o["norm2"]


@pytest.mark.parametrize("ndim,ext", [(1, [6]), (2, [4, 3]), (3, [3, 3, 3])])
def test_free_exciton_bloch_closed_form(ndim, ext):
    # g = 0, uniform eps, k = 0 Bloch start on a periodic lattice:
    # a(t) = exp(-i (eps + 2 J ndim) t) and the energy is eps + 2 J ndim.
    eps, J = 0.3, -0.7
    N = int(np.prod(ext))
    p = make(ndim=ndim, extent=ext, periodic=[1] * ndim, cutoff=[2],
             g=(0.0,), J=(J,) * ndim, eps=[eps] * N)
    m = O.Model(p)
    exc, occ, coef = WL.initial_state(dict(WL.CONFIGS["ring4"], extent=ext + [1] * (3 - ndim),
                                           n_modes=1), "bloch")
    s = O.Sim(m, {"dt": 0.05, "k": 2, "k_init": 2, "theta": 0.0}, exc, occ, coef)
    s.step(40)
    for o in s.observations():
        a = complex(o["a_re"], o["a_im"])
        ref = cmath.exp(-1j * (eps + 2 * J * ndim) * o["t"])
        assert abs(a - ref) <= 1e-12
        assert abs(o["energy"] - (eps + 2 * J * ndim)) <= 1e-12


def test_free_exciton_localized_closed_form():
    # ring of N sites, localized start at j0:
    # c_j(t) = N^-1 sum_q exp(i q (j - j0)) exp(-i (eps + 2 J cos q) t)
    N, eps, J, j0 = 7, -0.2, 0.9, 2
    p = make(ndim=1, extent=[N], periodic=[1], cutoff=[1], g=(0.0,), J=(J,),
             eps=[eps] * N)
    m = O.Model(p)
    s = O.Sim(m, {"dt": 0.03, "k": 4, "k_init": 4, "theta": 0.0}, [j0],
              [0] * N, [1.0, 0.0])
    s.step(50)
    t = s.observations()[-1]["t"]
    keys, amps = s.state()
    e, _ = m.unpack(keys)
    qs = 2 * np.pi * np.arange(N) / N
    for j, c in zip(e, amps):
        ref = np.sum(np.exp(1j * qs * (j - j0))
                     * np.exp(-1j * (eps + 2 * J * np.cos(qs)) * t)) / N
        assert abs(c - ref) <= 1e-12
    pop = s.observations()[-1]["pop"]
    assert abs(pop.sum() - 1.0) <= 1e-13


@pytest.mark.parametrize("g,omega,cut,eps", [(1.0, 1.0, 60, 0.37),
                                             (2.5, 1.0, 110, 0.0),
                                             (0.5, 0.2, 60, -1.1)])
def test_independent_boson_closed_form(g, omega, cut, eps):
    # J = 0, one site, vacuum start: a(t) = exp(-i eps t + i S omega t
    # - S (1 - exp(-i omega t))), S = (g/omega)^2, and the mean occupation is
    # 2 S (1 - cos omega t).  (2.5, 1.0) is the displaced oscillator of the
    # paper's Fig. moving_basis_set with S = 6.25.
    p = make(ndim=1, extent=[1], periodic=[0], cutoff=[cut], g=(g,),
             omega=(omega,), J=(0.0,), eps=[eps])
    m = O.Model(p)
    s = O.Sim(m, {"dt": 0.1, "k": 4, "k_init": cut, "theta": 0.0}, [0], [0],
              [1.0, 0.0])
    s.step(40)
    S = (g / omega) ** 2
    for o in s.observations():
        t = o["t"]
        a = complex(o["a_re"], o["a_im"])
        ref = cmath.exp(-1j * eps * t + 1j * S * omega * t
                        - S * (1 - cmath.exp(-1j * omega * t)))
        assert abs(a - ref) <= 1e-11
    keys, amps = s.state()
    _, occ = m.unpack(keys)
    nbar = float(np.sum(np.abs(amps) ** 2 * occ[:, 0]))
    t = s.observations()[-1]["t"]
    assert abs(nbar - 2 * S * (1 - math.cos(omega * t))) <= 1e-10


def test_independent_boson_two_modes_factorize():
    g, om = (1.0, 0.5), (1.0, 0.2)
    p = make(ndim=1, extent=[1], periodic=[0], cutoff=[40, 60], V=2,
             g=g, omega=om, J=(0.0,), eps=[0.1])
    m = O.Model(p)
    s = O.Sim(m, {"dt": 0.1, "k": 4, "k_init": 100, "theta": 0.0}, [0], [0, 0],
              [1.0, 0.0])
    s.step(20)
    for o in s.observations():
        t = o["t"]
        ref = cmath.exp(-1j * 0.1 * t)
        for gg, ww in zip(g, om):
            S = (gg / ww) ** 2
            ref *= cmath.exp(1j * S * ww * t - S * (1 - cmath.exp(-1j * ww * t)))
        assert abs(complex(o["a_re"], o["a_im"]) - ref) <= 1e-11


def test_piecewise_constant_hamiltonian_matches_dense_products():
    """Switching the model between steps (same shape): on a space reached
    whole, psi = exp(-i H_B n2 dt) exp(-i H_A n1 dt) psi0 with the dense
    Kronecker-product Hamiltonians."""
    import scipy.linalg as sla
    from tests import brute
    cfg = dict(WL.CONFIGS["ring12"])
    cfg.update(extent=[3, 1, 1], cutoff=[2], theta=0.0, k=30, k_init=30,
               init="local", eps_sigma=0.3)
    pa = WL.model_params(cfg)
    pb = dict(pa, J=[0.7, 0.0, 0.0], g=[1.4, 0, 0, 0], omega=[0.8, 0, 0, 0],
              eps=[0.1, -0.2, 0.05])
    ma, mb = O.Model(pa), O.Model(pb)
    s = O.Sim(ma, WL.run_params(cfg), *WL.initial_state(cfg))
    s.step(4)
    s.set_model(mb)
    s.step(3)
    keys, amps = s.state()
    n = brute.dense_hamiltonian(pa).shape[0]
    assert len(keys) == n
    psi0 = np.zeros(n, complex)
    psi0[brute.state_index(pa, 0, [0, 0, 0])] = 1
    dt = cfg["dt"]
    ref = sla.expm(-1j * brute.dense_hamiltonian(pb) * 3 * dt) @ (
        sla.expm(-1j * brute.dense_hamiltonian(pa) * 4 * dt) @ psi0)
    # oracle rows are sorted keys; map them to the dense index order
    exc, occ = ma.unpack(keys)
    idx = [brute.state_index(pa, int(j), list(o)) for j, o in zip(exc, occ)]
    assert np.max(np.abs(amps - ref[idx])) <= 1e-12


def _differs(pop, ref, tol):
    return np.max(np.abs(pop - ref)) > tol


def test_populations_match_dense_expm_per_site():
    """P(j) of Eq. (RMSD) (the exciton population of site j) against the
    dense-expm state summed over the phonon configurations of each site.
    Site energies break the ring's reflection symmetry, so a permuted,
    shifted or mirrored binning fails."""
    cfg = WL.CONFIGS["ring4"]
    p = dict(WL.model_params(cfg), eps=[0.0, 0.35, -0.2, 0.15])
    m = O.Model(p)
    exc, occ, coef = WL.initial_state(cfg)
    steps = 40
    H, exact = ring4_exact(p, steps, 0.05)
    s = O.Sim(m, dict(WL.run_params(cfg), dt=0.05, theta=0.0, k=4,
                      k_init=60), exc, occ, coef)
    s.step(steps)
    obs = s.observations()
    N = 4
    for i in (0, 9, 19, 39):
        ref = (np.abs(exact[i]) ** 2).reshape(N, -1).sum(axis=1)
        pop = obs[i]["pop"]
        assert np.max(np.abs(pop - ref)) <= 1e-12, (i, pop, ref)
    # the check separates every other assignment of bins to sites
    ref = (np.abs(exact[-1]) ** 2).reshape(N, -1).sum(axis=1)
    pop = obs[-1]["pop"]
    for perm in [np.roll(np.arange(N), 1), np.roll(np.arange(N), -1),
                 np.array([0, 3, 2, 1]), np.arange(N)[::-1]]:
        assert _differs(pop[perm], ref, 1e-6), perm


def test_populations_match_free_exciton_closed_form():
    """P(j) = |c_j(t)|^2 for g = 0 on a ring, from a start spread over two
    sites with a relative phase (no reflection symmetry):
    c_j(t) = sum_{j0} c_{j0} N^-1 sum_q exp(i q (j - j0)) exp(-i (eps + 2 J
    cos q) t)."""
    N, eps, J = 7, -0.2, 0.9
    starts = [(2, 0.6), (3, 0.8j)]
    p = make(ndim=1, extent=[N], periodic=[1], cutoff=[1], g=(0.0,), J=(J,),
             eps=[eps] * N)
    m = O.Model(p)
    coef = []
    for _, c in starts:
        coef += [c.real, c.imag] if isinstance(c, complex) else [c, 0.0]
    s = O.Sim(m, {"dt": 0.03, "k": 4, "k_init": 4, "theta": 0.0},
              [j for j, _ in starts], [0] * (N * len(starts)), coef)
    s.step(50)
    qs = 2 * np.pi * np.arange(N) / N
    for o in s.observations()[9::10]:
        t = o["t"]
        ref = np.zeros(N)
        for j in range(N):
            c = sum(c0 * np.sum(np.exp(1j * qs * (j - j0)) *
                                np.exp(-1j * (eps + 2 * J * np.cos(qs)) * t)) / N
                    for j0, c0 in starts)
            ref[j] = abs(c) ** 2
        assert np.max(np.abs(o["pop"] - ref)) <= 1e-12, (t, o["pop"], ref)
        for perm in [np.roll(np.arange(N), 1), np.roll(np.arange(N), -1),
                     (5 - np.arange(N)) % N]:
            assert _differs(o["pop"][perm], ref, 1e-4), (t, perm)


def test_gershgorin_bounds_from_dense_restriction():
    """E_min / E_max: Gershgorin discs of the dense Hamiltonian restricted to
    the step's set (rows and columns of the states in S), padded by 1e-12
    (|E_max| + |E_min|)."""
    cfg = WL.CONFIGS["ring4"]
    p = dict(WL.model_params(cfg), eps=[0.0, 0.35, -0.2, 0.15])
    m = O.Model(p)
    exc, occ, coef = WL.initial_state(cfg)
    s = O.Sim(m, WL.run_params(cfg), exc, occ, coef)
    Hd = brute.dense_hamiltonian(p)
    for step in range(6):
        s.step(1)
        keys, _ = s.state()
        e, o = m.unpack(keys)
        idx = [brute.state_index(p, int(e[i]), o[i]) for i in range(len(e))]
        Hs = Hd[np.ix_(idx, idx)]
        rad = np.abs(Hs).sum(axis=1) - np.abs(np.diag(Hs))
        lo = float(np.min(np.diag(Hs) - rad))
        hi = float(np.max(np.diag(Hs) + rad))
        pad = 1e-12 * (abs(hi) + abs(lo))
        ob = s.observations()[-1]
        assert abs(ob["E_min"] - (lo - pad)) <= 1e-13 * (abs(lo) + 1), step
        assert abs(ob["E_max"] - (hi + pad)) <= 1e-13 * (abs(hi) + 1), step
