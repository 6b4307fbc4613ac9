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
