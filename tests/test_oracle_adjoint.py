"""Pins of the oracle's adjoint gradient (Form (3)) on frozen sets.

The gradient is checked against (1) central finite differences of the
oracle's own frozen-set replay, a different computation than the adjoint
recursion; (2) closed forms: the free exciton (g = 0) from the k = 0 Bloch
state, and the independent boson model (one site, J absent); (3) dense
linear algebra on a space small enough to be reached whole: the dense H of
Kronecker products and scipy's Frechet derivative of expm."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import oracle as O
from tests import brute
import workloads as WL


def with_param(p, name, delta):
    p = dict(p)
    for f in ("J", "g", "omega", "eps"):
        p[f] = list(p[f])
    if name.startswith("omega"):
        p["omega"][int(name[5:])] += delta
    elif name.startswith("eps"):
        p["eps"][int(name[3:])] += delta
    elif name.startswith("J"):
        p["J"][int(name[1:])] += delta
    else:
        p["g"][int(name[1:])] += delta
    return p


def frozen_case(name, steps, **over):
    cfg = dict(WL.CONFIGS[name])
    cfg.update(over)
    p = WL.model_params(cfg)
    exc, occ, coef = WL.initial_state(cfg)
    m = O.Model(p)
    return p, m, O.Frozen(m, WL.run_params(cfg), exc, occ, coef, steps)


def complex_derivative(f, m, s):
    """d a_s / d theta from two real losses: gbar = e_s gives 2 Re, gbar =
    i e_s gives 2 Im."""
    g1 = np.zeros(f.steps + 1, complex)
    g1[s] = 1.0
    g2 = np.zeros(f.steps + 1, complex)
    g2[s] = 1j
    a, d1 = f.grad(m, g1)
    _, d2 = f.grad(m, g2)
    return a, (d1 + 1j * d2) / 2


@pytest.mark.parametrize("name,steps,over", [
    ("ring12", 12, dict(extent=[5, 1, 1], cutoff=[3], theta=1e-6)),
    ("sq6x6", 6, dict(extent=[3, 3, 1], cutoff=[2], theta=1e-5, eps_sigma=0.2)),
    ("cube4", 5, dict(extent=[3, 1, 1], ndim=1, periodic=[1, 0, 0],
                      J=[-0.5], cutoff=[2, 3], theta=1e-5, init="local")),
])
def test_gradient_matches_central_differences(name, steps, over):
    p, m, f = frozen_case(name, steps, **over)
    a = f.eval(m)
    rng = np.random.default_rng(7)
    tau = a + 0.3 * (rng.standard_normal(len(a)) + 1j * rng.standard_normal(len(a)))
    loss = lambda aa: float(np.sum(np.abs(aa - tau) ** 2))
    a2, g = f.grad(m, a - tau)  # gbar = dL/d conj(a) = a - tau
    assert np.array_equal(a, a2)
    # fourth-order central differences, h = 1e-4: truncation ~ h^4 and
    # rounding ~ 1e-16 L / h both stay near 1e-12
    h = 1e-4
    Lp = lambda nm, d: loss(f.eval(O.Model(with_param(p, nm, d))))
    fd = np.array([(-Lp(nm, 2 * h) + 8 * Lp(nm, h) - 8 * Lp(nm, -h)
                    + Lp(nm, -2 * h)) / (12 * h) for nm in O.param_names(p)])
    scale = np.maximum(np.abs(g), 1e-2 * np.max(np.abs(g)))
    assert np.all(np.abs(g - fd) <= 1e-7 * scale), np.abs(g - fd) / scale


@pytest.mark.parametrize("ndim,extent", [(1, [5, 1, 1]), (2, [3, 4, 1])])
def test_free_exciton_bloch_closed_form(ndim, extent):
    """g = 0, uniform eps = 0, k = 0 Bloch start: the start is an
    eigenstate with energy 2 sum_a J_a, so a(t) = exp(-2i t sum J_a),
    da/dJ_a = -2i t a, da/deps_n = -(i t / N) a, da/dg = da/domega = 0."""
    J = [-1.0, -0.7, 0.0][:ndim] + [0.0] * (3 - ndim)
    p, m, f = frozen_case("ring12", 8, ndim=ndim, extent=extent,
                          periodic=[1, 1, 0], J=J, g=[0.0], eps_sigma=0.0,
                          cutoff=[3], theta=1e-9)
    N = extent[0] * extent[1]
    dt = WL.CONFIGS["ring12"]["dt"]
    for s in (1, 5, 8):
        t = s * dt
        a, d = complex_derivative(f, m, s)
        exact = np.exp(-2j * t * sum(J))
        assert abs(a[s] - exact) <= 1e-13
        names = O.param_names(p)
        for k, nm in enumerate(names):
            if nm.startswith("J"):
                ref = -2j * t * exact
            elif nm.startswith("eps"):
                ref = -(1j * t / N) * exact
            else:
                ref = 0.0
            assert abs(d[k] - ref) <= 1e-12, (s, nm, d[k], ref)


def test_independent_boson_closed_form():
    """One site, one mode, J absent: a(t) = exp(F) with
    F = -i eps t + i (g^2/w) t - (g/w)^2 (1 - exp(-i w t)); the cutoff
    (40) puts the Poisson tail far below rounding."""
    eps, g, w = 0.3, 0.8, 1.3
    cfg = dict(WL.CONFIGS["ring12"])
    cfg.update(ndim=1, extent=[1, 1, 1], periodic=[0, 0, 0], J=[0.0],
               cutoff=[40], g=[g], omega=[w], eps=[eps], theta=0.0,
               k=45, k_init=45, init="local", dt=0.05)
    p = WL.model_params(cfg)
    exc, occ, coef = WL.initial_state(cfg)
    m = O.Model(p)
    f = O.Frozen(m, WL.run_params(cfg), exc, occ, coef, 6)
    assert np.all(f.sizes()[1:] == 41)
    names = O.param_names(p)
    for s in (2, 6):
        t = s * cfg["dt"]
        e = np.exp(-1j * w * t)
        F = -1j * eps * t + 1j * (g * g / w) * t - (g / w) ** 2 * (1 - e)
        dF = {"eps0": -1j * t,
              "g0": 2j * g * t / w - (2 * g / w ** 2) * (1 - e),
              "omega0": (-1j * g * g * t / w ** 2 + (2 * g * g / w ** 3) * (1 - e)
                         - (g * g / w ** 2) * 1j * t * e),
              "J0": 0.0}
        a, d = complex_derivative(f, m, s)
        assert abs(a[s] - np.exp(F)) <= 1e-12
        for k, nm in enumerate(names):
            assert abs(d[k] - np.exp(F) * dF[nm]) <= 1e-11, (nm, d[k])


def test_gradient_matches_dense_frechet_derivative():
    """A 3-site ring with cutoff 2 (81 states) reached whole at the first
    step: a_s = psi0^H exp(-i H s dt) psi0 exactly, and its derivative is
    psi0^H L(-i H s dt, -i s dt dH/dtheta) psi0 with scipy's expm_frechet
    and dH/dtheta from the Kronecker-product Hamiltonian."""
    cfg = dict(WL.CONFIGS["ring12"])
    cfg.update(extent=[3, 1, 1], cutoff=[2], theta=0.0, k=30, k_init=30,
               init="local", eps_sigma=0.3)
    p, m, f = frozen_case("ring12", 5, **{k: cfg[k] for k in
                                          ("extent", "cutoff", "theta", "k",
                                           "k_init", "init", "eps_sigma")})
    H = brute.dense_hamiltonian(p)
    n = H.shape[0]
    assert np.all(f.sizes()[1:] == n)
    psi0 = np.zeros(n, complex)
    psi0[brute.state_index(p, 0, [0, 0, 0])] = 1.0
    names = O.param_names(p)
    zero = with_param(p, "J0", -p["J"][0])
    for nm in ("g0", "omega0"):
        zero = with_param(zero, nm, -zero[nm[:-1]][0])
    zero["eps"] = [0.0] * 3
    dHs = [brute.dense_hamiltonian(with_param(zero, nm, 1.0)) for nm in names]
    rng = np.random.default_rng(3)
    gbar = rng.standard_normal(f.steps + 1) + 1j * rng.standard_normal(f.steps + 1)
    a, g = f.grad(m, gbar)
    dt = cfg["dt"]
    ref = np.zeros(len(names))
    for s in range(f.steps + 1):
        A = -1j * H * s * dt
        assert abs(a[s] - psi0.conj() @ sla.expm(A) @ psi0) <= 1e-13
        for k, dH in enumerate(dHs):
            L = sla.expm_frechet(A, -1j * s * dt * dH, compute_expm=False)
            ref[k] += 2 * (np.conj(gbar[s]) * (psi0.conj() @ L @ psi0)).real
    assert np.allclose(g, ref, rtol=1e-10, atol=1e-12 * np.max(np.abs(ref)))


def test_replay_reproduces_the_free_run():
    """At the recording parameters the frozen replay is the free run."""
    cfg = dict(WL.CONFIGS["ring12"])
    cfg.update(extent=[5, 1, 1], cutoff=[3], theta=1e-6)
    p = WL.model_params(cfg)
    exc, occ, coef = WL.initial_state(cfg)
    m = O.Model(p)
    f = O.Frozen(m, WL.run_params(cfg), exc, occ, coef, 10)
    s = O.Sim(m, WL.run_params(cfg), exc, occ, coef)
    s.step(10)
    a = f.eval(m)
    obs = s.observations()
    assert a[0] == pytest.approx(1.0, abs=1e-15)
    for i, o in enumerate(obs):
        assert a[i + 1] == complex(o["a_re"], o["a_im"])
    assert np.array_equal(f.get_set(10), s.state()[0])
