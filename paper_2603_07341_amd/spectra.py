"""Post-processing of the recorded observables on the host (numpy).

The library records, per step, the autocorrelation a(t) = <psi0|psi(t)>
and the exciton populations P(j, t).  From them:

* absorption_spectrum: the linear absorption spectrum of a dipole-excited
  start as the damped half-sided Fourier transform of a(t),
  A(w) = Re int_0^T a(t) exp(i w t) exp(-t / tau) dt / pi, the damping
  standing for the finite line width (paper: Sec. "Application to
  vibronic nanoaggregates", spectra of the aggregates; the damping rate
  used there is 0.0577 omega_0);
* exciton_rmsd: the spread of the exciton position,
  sqrt(sum_x P(x) (x - <x>)^2) with x the minimal-image displacement from
  the initial site on periodic axes (the paper's transport measure, read as
  the standard deviation of the population distribution).
"""
import numpy as np

DEFAULT_DAMPING = 0.0577  # 1/tau in units of the mode frequency


def absorption_spectrum(a, dt, omegas, damping=DEFAULT_DAMPING):
    """A(w) on the frequency grid `omegas` from samples a[s] = a(s dt),
    s = 0..n (a[0] = <psi0|psi0>), by the trapezoidal rule."""
    a = np.asarray(a, dtype=np.complex128)
    t = dt * np.arange(len(a))
    w = np.asarray(omegas, dtype=np.float64)
    damped = a * np.exp(-damping * t)
    phase = np.exp(1j * np.outer(w, t))
    f = phase * damped[None, :]
    integral = dt * (f.sum(axis=1) - 0.5 * (f[:, 0] + f[:, -1]))
    return integral.real / np.pi


def site_coords(extent, site):
    ex = list(extent) + [1] * (3 - len(extent))
    return (site % ex[0], (site // ex[0]) % ex[1], site // (ex[0] * ex[1]))


def exciton_rmsd(pop, extent, periodic, origin=0):
    """Standard deviation of the exciton position for populations pop[j]
    (or pop[t, j]) on a lattice of the given extent; displacements from
    `origin` use the minimal image along periodic axes."""
    pop = np.asarray(pop, dtype=np.float64)
    ex = list(extent) + [1] * (3 - len(extent))
    per = list(periodic) + [0] * (3 - len(periodic))
    N = ex[0] * ex[1] * ex[2]
    o = site_coords(ex, origin)
    disp = np.zeros((N, 3))
    for j in range(N):
        c = site_coords(ex, j)
        for ax in range(3):
            d = c[ax] - o[ax]
            if per[ax] and ex[ax] > 1:
                d = (d + ex[ax] // 2) % ex[ax] - ex[ax] // 2
            disp[j, ax] = d
    p = pop / pop.sum(axis=-1, keepdims=True)
    mean = p @ disp
    sq = p @ (disp ** 2)
    var = (sq - mean ** 2).sum(axis=-1)
    return np.sqrt(np.maximum(var, 0.0))
