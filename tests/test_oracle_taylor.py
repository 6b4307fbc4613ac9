"""Pins of the oracle's truncated Taylor propagator: the method App. "The
action of the exponential of a sparse matrix" names (the degree and
substep choice of Al-Mohy & Higham, 2011) and the fixed-order series of
App. "An effective Hilbert space up to neighbor order m = 2 is not
equivalent to a second-order Taylor expansion".

Checked against:
  * theta_m recomputed here in exact rational arithmetic from its
    definition (the backward error of the degree-m series at unit roundoff
    2^-53);
  * the (degree, substeps) choice by brute force over those exact values;
  * dense exponentials (scipy) for norms that need one to many substeps;
  * the closed form of the two-term series and its norm growth, which the
    paper's second-order comparison shows;
  * the default series propagator inside H_eff.
"""
from fractions import Fraction as Fr
from math import ceil, factorial

import numpy as np
import pytest
import scipy.linalg

from oracle import oracle as O
import workloads as WL

TOL = 2.0 ** -53


def exact_theta(m, extra=40):
    """theta_m = max{t : sum_{k>m} |c_k| t^(k-1) <= 2^-53}, where
    exp(-x) T_m(x) = exp(sum_k c_k x^k), coefficients as exact fractions."""
    M = m + 1 + extra
    g = []
    for k in range(M + 1):
        g.append(sum(Fr((-1) ** (k - j), factorial(k - j) * factorial(j))
                      for j in range(min(k, m) + 1)))
    assert g[0] == 1 and all(g[k] == 0 for k in range(1, m + 1))
    # h = log g as a power series: h' g = g'
    h = [Fr(0)] * (M + 1)
    for k in range(1, M + 1):
        h[k] = g[k] - sum(j * h[j] * g[k - j] for j in range(1, k)) / k
    c = [abs(float(x)) for x in h]
    f = lambda t: sum(c[k] * t ** (k - 1) for k in range(m + 1, M + 1)) - TOL
    lo, hi = 0.0, 1.0
    while f(hi) < 0:
        hi *= 2
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if f(mid) < 0 else (lo, mid)
    return lo


EXACT = {}


def theta(m):
    if m not in EXACT:
        EXACT[m] = exact_theta(m)
    return EXACT[m]


@pytest.mark.parametrize("m", [1, 2, 3, 5, 8, 13, 21, 34, 55])
def test_theta_matches_exact_rational_definition(m):
    assert O.taylor_theta(m) == pytest.approx(theta(m), rel=1e-9)


def test_theta_out_of_range():
    assert O.taylor_theta(0) < 0 and O.taylor_theta(56) < 0


@pytest.mark.parametrize("norm", [0.0, 1e-9, 0.05, 0.2, 0.9, 3.0, 12.5, 40.0])
def test_degree_and_substeps_minimise_the_products(norm):
    # brute force with thetas computed here; all 55 are needed
    th = {m: O.taylor_theta(m) for m in range(1, 56)}
    for m in (1, 5, 13, 34, 55):
        assert th[m] == pytest.approx(theta(m), rel=1e-9)
    best = None
    for m in range(1, 56):
        s = max(1, ceil(norm / th[m]))
        if best is None or m * s < best[0] * best[1]:
            best = (m, s)
    assert O.taylor_select(norm) == best


def random_sym(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(n, n))
    return A + A.T


def csr_of(H):
    rp, cols, vals = [0], [], []
    for i in range(H.shape[0]):
        for j in range(H.shape[1]):
            if H[i, j] != 0.0:
                cols.append(j)
                vals.append(H[i, j])
        rp.append(len(cols))
    return np.array(rp), np.array(cols), np.array(vals)


def gershgorin(H):
    r = np.abs(H).sum(axis=1) - np.abs(np.diag(H))
    lo, hi = (np.diag(H) - r).min(), (np.diag(H) + r).max()
    pad = 1e-12 * (abs(lo) + abs(hi))
    return lo - pad, hi + pad


@pytest.mark.parametrize("dt", [0.01, 0.1, 0.5, 2.0, 6.0])
def test_adaptive_series_equals_dense_exponential(dt):
    H = random_sym(9, 5)
    rng = np.random.default_rng(6)
    v = rng.normal(size=9) + 1j * rng.normal(size=9)
    lo, hi = gershgorin(H)
    out, mvs = O.taylor(*csr_of(H), dt, lo, hi, -1, v)
    ref = scipy.linalg.expm(-1j * dt * H) @ v
    np.testing.assert_allclose(out, ref, rtol=0, atol=2e-13 * np.abs(v).max())
    m, s = O.taylor_select(0.5 * (hi - lo) * dt)
    assert mvs == m * s
    if dt >= 2.0:
        assert s > 1


def test_fixed_order_two_is_the_two_term_polynomial():
    H = random_sym(7, 8)
    rng = np.random.default_rng(9)
    v = rng.normal(size=7) + 1j * rng.normal(size=7)
    lo, hi = gershgorin(H)
    dt = 0.3
    out, mvs = O.taylor(*csr_of(H), dt, lo, hi, 2, v)
    b = 0.5 * (lo + hi)
    A = -1j * dt * (H - b * np.eye(7))
    ref = np.exp(-1j * b * dt) * (v + A @ v + A @ (A @ v) / 2)
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-14 * np.abs(v).max())
    assert mvs == 2


def test_sim_adaptive_taylor_equals_series_and_order_two_gains_norm():
    cfg = dict(WL.CONFIGS["ring4"])
    m = O.Model(WL.model_params(cfg))
    run = dict(WL.run_params(cfg), theta=0.0)
    a = O.Sim(m, run, *WL.initial_state(cfg))
    b = O.Sim(m, dict(run, taylor_order=-1), *WL.initial_state(cfg))
    c = O.Sim(m, dict(run, taylor_order=2), *WL.initial_state(cfg))
    a.step(10)
    b.step(10)
    c.step(10)
    ka, pa = a.state()
    kb, pb = b.state()
    assert np.array_equal(ka, kb)
    assert np.abs(pa - pb).max() <= 1e-12
    # the two-term series is not unitary: |1 - i x - x^2/2|^2 = 1 + x^4/4,
    # so without truncation the norm grows every step
    n2 = [o["norm2"] for o in c.observations()]
    assert all(y > x for x, y in zip(n2, n2[1:])) and n2[0] > 1.0
    assert c.observations()[-1]["terms"] == 2


def test_taylor_and_krylov_are_exclusive_and_adjoint_refuses():
    cfg = dict(WL.CONFIGS["ring4"])
    m = O.Model(WL.model_params(cfg))
    with pytest.raises(RuntimeError):
        O.Sim(m, dict(WL.run_params(cfg), taylor_order=-1, krylov_order=3),
              *WL.initial_state(cfg))
    with pytest.raises(RuntimeError, match="series"):
        O.Frozen(m, dict(WL.run_params(cfg), taylor_order=-1),
                 *WL.initial_state(cfg), steps=2)
