"""Host post-processing of recorded observables (CPU): the damped Fourier
transform against its closed form for a single eigenstate, the
independent-boson progression against the Poisson weights, the spectrum of
an oracle run, and the exciton spread on rings."""
import math

import numpy as np

from oracle import oracle as O
from paper_2603_07341_amd import spectra
import workloads as WL


def test_single_line_matches_closed_form():
    E, dt, n, g = -1.3, 0.01, 4000, 0.0577
    a = np.exp(-1j * E * dt * np.arange(n + 1))
    w = np.linspace(-3, 1, 81)
    A = spectra.absorption_spectrum(a, dt, w, damping=g)
    T = n * dt
    z = 1j * (w - E) - g
    exact = ((np.exp(z * T) - 1) / z).real / np.pi
    # trapezoid error ~ dt^2 |z|^2 / 12 relative
    assert np.max(np.abs(A - exact)) <= 1e-4 * np.max(np.abs(exact))
    assert abs(w[np.argmax(A)] - E) < 0.06


def test_independent_boson_progression():
    """One site: a(t) = exp(-S (1 - exp(-i w t)) + i S w t); the spectrum is
    a Poisson progression of lines at S-shifted multiples of w."""
    S, wv, dt, n = 0.8, 1.0, 0.02, 6000
    t = dt * np.arange(n + 1)
    a = np.exp(-S * (1 - np.exp(-1j * wv * t)) + 1j * S * wv * t)
    grid = np.linspace(-2, 4, 1201)
    A = spectra.absorption_spectrum(a, dt, grid, damping=0.05)
    for k in range(4):
        pos = -S * wv + k * wv
        i = np.argmin(np.abs(grid - pos))
        peak = A[i] * np.pi * 0.05  # height of a unit Lorentzian line is 1/(pi g)
        weight = np.exp(-S) * S ** k / math.factorial(k)
        assert abs(peak - weight) < 0.03, (k, peak, weight)


def test_spectrum_of_free_exciton_oracle_run():
    """g = 0 ring from the Bloch state: a single line at 2J."""
    cfg = dict(WL.CONFIGS["ring12"], extent=[6, 1, 1], g=[0.0],
               eps_sigma=0.0, cutoff=[2], theta=1e-12, dt=0.05)
    s = O.Sim(O.Model(WL.model_params(cfg)), WL.run_params(cfg),
              *WL.initial_state(cfg))
    s.step(600)
    a = [1.0] + [complex(o["a_re"], o["a_im"]) for o in s.observations()]
    w = np.linspace(-4, 2, 601)
    A = spectra.absorption_spectrum(np.array(a), cfg["dt"], w)
    assert abs(w[np.argmax(A)] - 2 * cfg["J"][0]) < 0.02


def test_rmsd_on_rings():
    ext, per = [8, 1, 1], [1, 0, 0]
    p = np.zeros(8)
    p[0] = 1
    assert spectra.exciton_rmsd(p, ext, per) == 0
    p = np.zeros(8)
    p[1] = p[7] = 0.5  # neighbours on both sides of site 0
    assert abs(spectra.exciton_rmsd(p, ext, per) - 1.0) < 1e-15
    u = np.full(8, 1 / 8)  # uniform: displacements -4..3
    d = np.arange(-4, 4)
    assert abs(spectra.exciton_rmsd(u, ext, per) - np.sqrt(np.mean(d ** 2) - np.mean(d) ** 2)) < 1e-14
    pt = np.stack([p, u])
    assert spectra.exciton_rmsd(pt, ext, per).shape == (2,)


def test_electronic_lines_periodic_ring_has_one_bright_state():
    # the uniform state is the k = 0 eigenstate of a ring: one line at 2J
    E, f = spectra.electronic_lines([12], [0.55], [1])
    assert abs(f.sum() - 1.0) < 1e-13
    k = np.argmax(f)
    assert abs(E[k] - 1.1) < 1e-13 and abs(f[k] - 1.0) < 1e-13
    assert np.allclose(np.sort(E), np.sort(2 * 0.55 * np.cos(2 * np.pi * np.arange(12) / 12)),
                       atol=1e-13)


def open_chain_lines(N, J):
    """Closed form of the open chain: E_n = 2 J cos(n pi / (N+1)) with
    eigenvectors sqrt(2/(N+1)) sin(j n pi / (N+1)), j, n = 1..N."""
    n = np.arange(1, N + 1)
    E = 2 * J * np.cos(n * np.pi / (N + 1))
    j = np.arange(1, N + 1)
    amp = np.sqrt(2.0 / (N + 1)) * np.sin(np.outer(j, n) * np.pi / (N + 1)).sum(axis=0)
    return E, amp ** 2 / N


def test_electronic_lines_open_chain_closed_form():
    N, J = 64, -0.55
    E, f = spectra.electronic_lines([N], [J])
    Ec, fc = open_chain_lines(N, J)
    o = np.argsort(Ec)
    assert np.allclose(E, Ec[o], atol=1e-12)
    assert np.allclose(f, fc[o], atol=1e-12)
    # only odd n are bright; the band-edge line carries
    # 2 cot^2(pi / (2 (N+1))) / (N (N+1)), about 8 / pi^2 for long chains
    assert abs(fc[0] - 2 / np.tan(np.pi / (2 * (N + 1))) ** 2 / (N * (N + 1))) < 1e-12
    assert abs(fc[0] - 8 / np.pi ** 2) < 0.02
    assert np.all(fc[1::2] < 1e-20)


def test_electronic_lines_square_lattice_is_a_product():
    # open L x L: E = E_x + E_y, f = f_x f_y (separable hopping)
    L, Jx, Jy = 5, 0.55, 0.3
    E, f = spectra.electronic_lines([L, L], [Jx, Jy])
    ex, fx = open_chain_lines(L, Jx)
    ey, fy = open_chain_lines(L, Jy)
    Ep = (ex[:, None] + ey[None, :]).ravel()
    fp = (fx[:, None] * fy[None, :]).ravel()
    # compare the bright lines (degenerate eigenvectors mix only among
    # equal energies, so sum strengths per distinct energy)
    def per_energy(E, f):
        out = {}
        for e, w in zip(np.round(E, 9), f):
            out[e] = out.get(e, 0.0) + w
        return out
    a, b = per_energy(E, f), per_energy(Ep, fp)
    assert set(a) == set(b)
    assert all(abs(a[k] - b[k]) < 1e-12 for k in a)


def test_oracle_at_zero_coupling_follows_the_electronic_lines():
    # g = 0 never creates phonons, so a(t) of the method (oracle, exact
    # series) is the electronic signal of the open 3 x 3 aggregate
    cfg = WL.paper_aggregate([3, 3], "J", q_nom=10_000)
    cfg["g"] = [0.0]
    s = O.Sim(O.Model(WL.model_params(cfg)), WL.run_params(cfg),
              *WL.initial_state(cfg))
    s.step(40)
    obs = s.observations()
    a = np.array([o["a_re"] + 1j * o["a_im"] for o in obs])
    t = np.array([o["t"] for o in obs])
    E, f = spectra.electronic_lines([3, 3], cfg["J"])
    assert np.abs(a - spectra.electronic_signal(E, f, t)).max() < 1e-12
    assert obs[-1]["n_S"] == 9
    # and the damped transform of the recorded signal approaches the
    # Lorentzian lines as T grows (here only checked for the line positions)
    bright = E[f > 1e-3]
    assert len(bright) >= 2  # an open 3 x 3 lattice has several bright states
