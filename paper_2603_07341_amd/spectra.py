"""Post-processing of the recorded observables on the host (numpy).

The library records, per step, the autocorrelation a(t) = <psi0|psi(t)>
and the exciton populations P(j, t).  From them:

* absorption_spectrum: the linear absorption spectrum of a dipole-excited
  start as the damped half-sided Fourier transform of a(t),
  A(w) = Re int_0^T a(t) exp(i w t) exp(-t / tau) dt / pi, the damping
  standing for the finite line width (paper: Sec. "Application to
  vibronic nanoaggregates", spectra of the aggregates; the damping rate
  used there is 0.0577 omega_0);
* electronic_lines / electronic_signal / electronic_spectrum: the purely
  electronic (g = 0) reference of those spectra by exact diagonalization
  of the N-site hopping matrix (the dotted lines of the paper's
  aggregate-spectra figure): eigenvalues E_n, oscillator strengths
  f_n = |<n|mu>|^2 of the dipole-excited start mu|0> = N^-1/2 sum_j |j>
  (Eq. init_state_spec), a(t) = sum_n f_n exp(-i E_n t);
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


def hopping_matrix(extent, J, periodic=(0, 0, 0)):
    """N x N single-exciton Hamiltonian of the lattice: J[axis] between
    nearest neighbours along each axis, sites numbered x + Lx (y + Ly z);
    a periodic axis (extent >= 3) closes with one more bond."""
    ex = list(extent) + [1] * (3 - len(extent))
    per = list(periodic) + [0] * (3 - len(periodic))
    Js = list(J) + [0.0] * (3 - len(J))
    N = ex[0] * ex[1] * ex[2]
    H = np.zeros((N, N))
    for j in range(N):
        c = list(site_coords(ex, j))
        for ax in range(3):
            if ex[ax] == 1:
                continue
            if per[ax] and ex[ax] < 3:
                raise ValueError("a periodic extent must be at least 3")
            nxt = c[ax] + 1
            if nxt == ex[ax]:
                if not per[ax]:
                    continue
                nxt = 0
            d = list(c)
            d[ax] = nxt
            k = d[0] + ex[0] * (d[1] + ex[1] * d[2])
            H[j, k] += Js[ax]
            H[k, j] += Js[ax]
    return H


def electronic_lines(extent, J, periodic=(0, 0, 0)):
    """Eigenvalues E_n (ascending) and oscillator strengths f_n of the g = 0
    aggregate for the dipole-excited start; sum_n f_n = 1."""
    H = hopping_matrix(extent, J, periodic)
    E, U = np.linalg.eigh(H)
    f = U.sum(axis=0) ** 2 / H.shape[0]
    return E, f


def electronic_signal(E, f, t):
    """a(t) = sum_n f_n exp(-i E_n t) at the times t."""
    t = np.asarray(t, dtype=np.float64)
    return np.exp(-1j * np.outer(t, E)) @ np.asarray(f, dtype=np.float64)


def electronic_spectrum(E, f, omegas, damping=DEFAULT_DAMPING):
    """The damped transform of electronic_signal over all t >= 0 (the
    convention of absorption_spectrum with T -> infinity): a Lorentzian of
    half width `damping` and area f_n at each E_n."""
    w = np.asarray(omegas, dtype=np.float64)[:, None]
    return (np.asarray(f) * damping / np.pi /
            ((w - np.asarray(E)[None, :]) ** 2 + damping ** 2)).sum(axis=1)


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
