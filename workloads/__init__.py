"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark: lattice shapes, model parameters, initial states and static
disorder.  This module holds none of the method's arithmetic; both the
GPU library and the CPU oracle receive what it produces as plain inputs.

The five workloads are Holstein lattices shaped like the paper's runs
(Sec. "Benchmarking with a 1D Holstein system" and Sec. "Application to
vibronic nanoaggregates"; parameters in App. "Parameters & runtimes"):

  ring4    1D ring, N=4, one mode, cutoff 4 (full space 4*5^4 = 2500),
           localized start, dt 0.01 x 500, k=4, threshold 1e-10, complex128
  ring16   1D ring, N=16, cutoff 12, k=0 Bloch start, dt 0.01 x 4000, k=4,
           threshold 1e-8, complex128 and complex64
  sq6x6    2D 6x6 periodic, cutoff 15, 64 static-disorder realizations
           eps ~ N(0, 0.2), dt 0.02 x 2000, k=2, threshold 1e-7, complex64
  cube4    3D 4x4x4 periodic, two modes (1, 1, c=15) and (0.2, 0.5, c=31),
           localized start at the corner, dt 0.01 x 3000, k=2,
           threshold 1e-7, state cap 5e8, complex64
  ring12   1D ring, N=12, cutoff 10, eps ~ N(0, 0.1) seed 42, dt 0.01 x
           2000, k=4, threshold 1e-8, complex128 (adjoint workload)

Static disorder: splitmix64 (Steele, Lea & Flood 2014) drives a uniform
u = (x >> 11) * 2^-53 and Box-Muller z = sqrt(-2 ln(1-u1)) cos(2 pi u2).
"""
import math

MASK64 = (1 << 64) - 1


def splitmix64_stream(seed):
    """Yield the splitmix64 output sequence for a 64-bit seed."""
    state = seed & MASK64
    while True:
        state = (state + 0x9E3779B97F4A7C15) & MASK64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        yield z ^ (z >> 31)


def normals(seed, n, sigma=1.0):
    """n draws from N(0, sigma^2), two uniforms per draw."""
    gen = splitmix64_stream(seed)
    out = []
    for _ in range(n):
        u1 = (next(gen) >> 11) * 2.0 ** -53
        u2 = (next(gen) >> 11) * 2.0 ** -53
        out.append(sigma * math.sqrt(-2.0 * math.log(1.0 - u1))
                   * math.cos(2.0 * math.pi * u2))
    return out


def _lattice(ndim, extent, periodic):
    ext = list(extent) + [1] * (3 - len(extent))
    per = list(periodic) + [0] * (3 - len(periodic))
    return {"ndim": ndim, "extent": ext, "periodic": per}


CONFIGS = {
    "ring4": dict(
        _lattice(1, [4], [1]), n_modes=1, cutoff=[4], omega=[1.0], g=[1.0],
        J=[-0.5], eps_sigma=0.0, eps_seed=None, n_real=1,
        dt=0.01, steps=500, k=4, k_init=4, theta=1e-10, precision=64,
        init="local", max_states=0),
    "ring16": dict(
        _lattice(1, [16], [1]), n_modes=1, cutoff=[12], omega=[1.0], g=[1.2],
        J=[-1.0], eps_sigma=0.0, eps_seed=None, n_real=1,
        dt=0.01, steps=4000, k=4, k_init=4, theta=1e-8, precision=64,
        init="bloch", max_states=0),
    "sq6x6": dict(
        _lattice(2, [6, 6], [1, 1]), n_modes=1, cutoff=[15], omega=[1.0],
        g=[1.0], J=[-0.8, -0.8], eps_sigma=0.2, eps_seed=1000, n_real=64,
        dt=0.02, steps=2000, k=2, k_init=2, theta=1e-7, precision=32,
        init="bloch", max_states=10_000_000),
    "cube4": dict(
        _lattice(3, [4, 4, 4], [1, 1, 1]), n_modes=2, cutoff=[15, 31],
        omega=[1.0, 0.2], g=[1.0, 0.5], J=[-0.5, -0.5, -0.5], eps_sigma=0.0,
        eps_seed=None, n_real=1, dt=0.01, steps=3000, k=2, k_init=2,
        theta=1e-7, precision=32, init="local", max_states=500_000_000),
    "ring12": dict(
        _lattice(1, [12], [1]), n_modes=1, cutoff=[10], omega=[1.0], g=[1.0],
        J=[-1.0], eps_sigma=0.1, eps_seed=42, n_real=1,
        dt=0.01, steps=2000, k=4, k_init=4, theta=1e-8, precision=64,
        init="bloch", max_states=0, ckpt_every=50),
}

# The paper's 1D benchmark runs (App. "Parameters & runtimes", table of the
# 1D calculations): open chains, J = omega = 1, m_init = 10, m = 2,
# dt = 0.05 up to t = 50 (1000 steps), fixed-size truncation q_nom, one
# exciton at the centre with the vibrational vacuum.  Per g: (N, d_pho,
# q_nom).
PAPER_1D = {1.0: (75, 16, 25e6), 1.5: (75, 16, 25e6), 2.0: (51, 64, 25e6),
            2.5: (25, 64, 32e6), 3.0: (25, 64, 32e6), 3.5: (25, 64, 32e6),
            4.0: (25, 64, 32e6)}


def paper_aggregate(extent, kind="H", q_nom=None, periodic=False):
    """Workload dict of the paper's aggregate runs (App. "Parameters &
    runtimes": g = 0.71, J = +0.55 (H) or -0.55 (J), d_pho = 16, m = 2,
    dt = 0.05 to t = 100 (2000 steps), q_nom = 16e6; m_init = 10 for the 1D
    and 2D lattices, 6 for the 3D ones), started from the dipole-excited k=0
    Bloch state of <mu(t) mu(0)>.  The paper does not state the boundaries:
    open by default, as its chain Hamiltonian is (the 5x5x5 H-aggregate's
    norm loss of nearly 70% is met with open boundaries, not with periodic
    ones); periodic=True closes every extent of at least 3."""
    ext = list(extent)
    nd = len(ext)
    per = [1 if periodic and e >= 3 else 0 for e in ext]
    J = 0.55 if kind == "H" else -0.55
    return dict(_lattice(nd, ext, per), n_modes=1, cutoff=[15], omega=[1.0],
                g=[0.71], J=[J] * nd, eps_sigma=0.0, eps_seed=None, n_real=1,
                dt=0.05, steps=2000, k=2, k_init=6 if nd == 3 else 10,
                theta=0.0, precision=64, init="bloch", max_states=0,
                q_nom=int(16e6 if q_nom is None else q_nom))


def paper_1d(g, q_nom=None):
    """Workload dict of the paper's 1D run at coupling g (q_nom may be
    overridden); the run uses q_nom, so theta is 0."""
    N, d, q = PAPER_1D[g]
    return dict(_lattice(1, [N], [0]), n_modes=1, cutoff=[d - 1],
                omega=[1.0], g=[g], J=[1.0], eps_sigma=0.0, eps_seed=None,
                n_real=1, dt=0.05, steps=1000, k=2, k_init=10, theta=0.0,
                precision=64, init="local", site=N // 2, max_states=0,
                q_nom=int(q if q_nom is None else q_nom))


def n_sites(cfg):
    e = cfg["extent"]
    return e[0] * e[1] * e[2]


def site_energies(cfg, realization=0):
    """eps_n for one realization (zeros when the workload has no disorder).
    Realization r of a batched workload uses seed eps_seed + r."""
    n = n_sites(cfg)
    if not cfg.get("eps_sigma"):
        return [0.0] * n
    return normals(cfg["eps_seed"] + realization, n, cfg["eps_sigma"])


def model_params(cfg, realization=0, **override):
    """Plain dict of model parameters for one realization."""
    c = dict(cfg)
    c.update(override)
    V = c["n_modes"]
    pad = lambda xs, k, v: list(xs) + [v] * (k - len(xs))
    return {
        "ndim": c["ndim"], "extent": list(c["extent"]),
        "periodic": list(c["periodic"]), "n_modes": V,
        "cutoff": pad(c["cutoff"], 4, 0), "omega": pad(c["omega"], 4, 0.0),
        "g": pad(c["g"], 4, 0.0), "J": pad(c["J"], 3, 0.0),
        "eps": list(c["eps"]) if "eps" in c else site_energies(c, realization),
    }


def batch_params(cfg, n_real=None, first=0, **override):
    """Model parameters of a batched run: realizations first .. first +
    n_real - 1 of the workload's disorder, their site energies concatenated
    realization-major."""
    c = dict(cfg)
    c.update(override)
    R = c["n_real"] if n_real is None else n_real
    p = model_params(c, first)
    eps = []
    for r in range(first, first + R):
        eps += site_energies(c, r)
    p["eps"] = eps
    p["n_real"] = R
    return p


def adjoint_target_params(cfg):
    """Model parameters of the run whose a(t) is the adjoint workload's
    target: J + 0.05 per axis, g - 0.05 and omega + 0.02 per mode, and
    site energies shifted by N(0, 0.02) draws of seed 43."""
    p = model_params(cfg)
    nd, V = cfg["ndim"], cfg["n_modes"]
    p["J"] = [x + 0.05 if a < nd else x for a, x in enumerate(p["J"])]
    p["g"] = [x - 0.05 if nu < V else x for nu, x in enumerate(p["g"])]
    p["omega"] = [x + 0.02 if nu < V else x for nu, x in enumerate(p["omega"])]
    p["eps"] = [e + d for e, d in zip(p["eps"], normals(43, n_sites(cfg), 0.02))]
    return p


def initial_state(cfg, kind=None, site=0):
    """(exc, occ, coef) of the initial state.

    'local': one exciton at `site` with the vibrational vacuum.
    'bloch': the k=0 Bloch state N^-1/2 sum_j |j> x |vac>, the dipole-excited
             state of Eq. (init_state_spec).
    occ is a flat site-major list of N*V occupations per term; coef holds
    interleaved (re, im) pairs."""
    kind = kind or cfg["init"]
    site = cfg.get("site", site)
    n = n_sites(cfg)
    V = cfg["n_modes"]
    if kind == "local":
        return [site], [0] * (n * V), [1.0, 0.0]
    if kind == "bloch":
        amp = 1.0 / math.sqrt(n)
        exc = list(range(n))
        occ = [0] * (n * n * V)
        coef = []
        for _ in range(n):
            coef += [amp, 0.0]
        return exc, occ, coef
    raise ValueError(kind)


def run_params(cfg, **override):
    c = dict(cfg)
    c.update(override)
    return {"dt": c["dt"], "k": c["k"], "k_init": c["k_init"],
            "theta": c["theta"], "precision": c["precision"],
            "max_states": c.get("max_states", 0),
            "q_nom": c.get("q_nom", 0)}


def random_amplitudes(seed, n):
    """Seeded complex amplitudes with a heavy tail: magnitudes spread over
    many decades, as the paper's sorted coefficient distribution shows
    (Fig. coeff_distribution).  Interleaved (re, im), not normalised."""
    gen = splitmix64_stream(seed)
    out = []
    for _ in range(n):
        u1 = (next(gen) >> 11) * 2.0 ** -53
        u2 = (next(gen) >> 11) * 2.0 ** -53
        mag = 10.0 ** (-14.0 * u1)
        ph = 2.0 * math.pi * u2
        out += [mag * math.cos(ph), mag * math.sin(ph)]
    return out


def phonon_ball_state(cfg, n_max, seed=7):
    """Every basis state of a single-mode lattice with at most n_max phonons
    in total (any exciton site), with seeded complex normal amplitudes
    normalised to one: (exc, occ, coef) as for initial_state.  A set that
    is closed under hopping and cut at a total phonon number, of size
    N * C(N + n_max, n_max)."""
    import itertools
    import numpy as np
    N = n_sites(cfg)
    cut = cfg["cutoff"][0]
    vecs = []
    for n in range(n_max + 1):
        for combo in itertools.combinations_with_replacement(range(N), n):
            v = np.bincount(np.asarray(combo, dtype=np.int64), minlength=N)
            if v.max(initial=0) <= cut:
                vecs.append(v)
    occ1 = np.asarray(vecs, dtype=np.uint16)
    exc = np.repeat(np.arange(N, dtype=np.int32), len(occ1))
    occ = np.tile(occ1, (N, 1))
    rng = np.random.default_rng(seed)
    c = rng.standard_normal(len(exc)) + 1j * rng.standard_normal(len(exc))
    c /= np.linalg.norm(c)
    coef = np.ascontiguousarray(c.astype(np.complex128)).view(np.float64)
    return exc, occ, coef
