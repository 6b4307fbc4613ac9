"""Pins of the oracle's Krylov (Lanczos) propagator, App. "Series-based
exponentiation compared to a Lanczos algorithm".

Checked against what the paper and the mathematics fix, not against the
oracle itself:
  * the paper's worked examples: the Lanczos vectors V_4 of the
    tight-binding chain (golden fixture), its counting statements
    (|V_n| has n^2 + 2n non-zero entries; H_eff^(n-1) has 3 + 2(n-1)
    states), and the overlaps of higher Krylov vectors with H_eff^(2);
  * the Krylov projection computed through an independent basis (QR of
    the power vectors) and a library exponential;
  * exactness when the Krylov space is invariant (breakdown), against a
    dense exponential, and against the series propagator inside H_eff;
  * orthonormality of the basis, T = V^dag H V, norm and energy
    conservation, and convergence to the series result as the order grows
    (the trend the paper's Fig. lanczos shows).
"""
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import oracle as O
import workloads as WL

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "lanczos_v4_tb.txt")


def load_v4():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        vals = []
        for cell in line.split("|"):
            a, b = cell.split()
            vals.append(int(a) * np.sqrt(int(b)) / 12.0)
        rows.append(vals)
    return np.array(rows)  # [9 states, 4 vectors]


def chain_cfg(L):
    return dict(WL._lattice(1, [L], [0]), n_modes=1, cutoff=[1], omega=[1.0],
                g=[0.0], J=[1.0], eps_sigma=0.0, eps_seed=None, n_real=1,
                dt=0.01, k=1, k_init=1, theta=0.0, precision=64,
                init="local", max_states=0)


def chain_heff(L, center, k):
    """H_eff^(k) of the tight-binding chain around the three-site state
    (|c-1> + |c> + |c+1>)/sqrt(3): (rowptr, cols, vals, phi, sites)."""
    cfg = chain_cfg(L)
    cfg.update(k=k, k_init=k)
    m = O.Model(WL.model_params(cfg))
    exc = [center - 1, center, center + 1]
    occ = [0] * (3 * L)
    coef = []
    for _ in exc:
        coef += [1 / np.sqrt(3), 0.0]
    s = O.Sim(m, WL.run_params(cfg), exc, occ, coef)
    s.step(1)
    keys, _ = s.state()
    sites, _ = m.unpack(keys)
    rp, cols, vals = s.csr()
    return rp, cols, vals, s.phi(), sites


def dense(rp, cols, vals):
    n = len(rp) - 1
    H = np.zeros((n, n))
    for i in range(n):
        for e in range(rp[i], rp[i + 1]):
            H[i, cols[e]] += vals[e]
    return H


def csr_of(H):
    rp, cols, vals = [0], [], []
    for i in range(H.shape[0]):
        for j in range(H.shape[1]):
            if H[i, j] != 0.0:
                cols.append(j)
                vals.append(H[i, j])
        rp.append(len(cols))
    return np.array(rp), np.array(cols), np.array(vals)


def test_tight_binding_example_matches_the_printed_v4():
    c = 5
    rp, cols, vals, phi, sites = chain_heff(11, c, 3)
    assert len(sites) == 9  # H_eff^(3) of the example: d = 9
    _, B, alpha, beta, _ = O.lanczos(rp, cols, vals, 0.01, 3, phi)
    assert B.shape[0] == 4
    V4 = load_v4()
    got = np.zeros((9, 4), dtype=np.complex128)
    for row, site in enumerate(sites):
        got[site - (c - 4)] = B[:, row]
    assert np.abs(got.imag).max() == 0.0
    np.testing.assert_allclose(got.real, V4, rtol=0, atol=1e-14)
    # 24 of its 36 entries are non-zero
    assert np.count_nonzero(np.abs(V4) > 1e-15) == 24


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 7])
def test_lanczos_vector_counts_follow_the_papers_closed_forms(n):
    # H_eff^(n-1) has 3 + 2(n-1) states, the Hamiltonian there 4n non-zero
    # off-diagonal entries, and V_n has n^2 + 2n non-zero entries
    rp, cols, vals, phi, sites = chain_heff(31, 15, n - 1)
    assert len(sites) == 3 + 2 * (n - 1)
    assert np.count_nonzero(vals) == 4 * n  # the diagonal is zero
    _, B, _, _, _ = O.lanczos(rp, cols, vals, 0.01, n - 1, phi)
    assert B.shape[0] == n
    assert np.count_nonzero(np.abs(B) > 1e-13) == n * n + 2 * n
    for k in range(n):
        assert np.count_nonzero(np.abs(B[k]) > 1e-13) == 2 * k + 3


def test_krylov_example_overlaps_with_heff2():
    # Sec. "Relation to Krylov subspaces": psi = (|n-1> + |n+1>)/sqrt(2) on
    # an (effectively infinite) tight-binding chain.  K^3 is spanned by the
    # three printed vectors; v_4 is proportional to |n-4> + 2/3 (|n-2> - |n>
    # + |n+2>) + |n+4>; the unit vector (|n-2> - |n> + |n+2>)/sqrt(3) of
    # H_eff^(2) = span{|n-3> .. |n+3>} overlaps v_4 by sqrt(2/5); v_5, v_7
    # are orthogonal to H_eff^(2); the largest overlaps of its unit sphere
    # with v_6 and v_8 are sqrt(6/35) and sqrt(2/21)
    L, c, k = 41, 20, 8
    cfg = chain_cfg(L)
    cfg.update(k=k, k_init=k)
    m = O.Model(WL.model_params(cfg))
    coef = [1 / np.sqrt(2), 0.0, 1 / np.sqrt(2), 0.0]
    s = O.Sim(m, WL.run_params(cfg), [c - 1, c + 1], [0] * (2 * L), coef)
    s.step(1)
    keys, _ = s.state()
    sites, _ = m.unpack(keys)
    rp, cols, vals = s.csr()
    _, B, _, _, _ = O.lanczos(rp, cols, vals, 0.01, 8, s.phi())
    assert B.shape[0] == 9
    V = np.zeros((9, L), dtype=np.complex128)  # V[j] = v_{j+1}
    for row, site in enumerate(sites):
        V[:, site] = B[:, row]
    printed = np.zeros((3, L))
    printed[0, [c - 1, c + 1]] = 1
    printed[1, [c - 2, c, c + 2]] = [1, 2, 1]
    printed[2, [c - 3, c - 1, c + 1, c + 3]] = [1, 3, 3, 1]
    Q, _ = np.linalg.qr(printed.T)
    P3 = Q @ Q.T
    for j in range(3):
        np.testing.assert_allclose(P3 @ V[j], V[j], atol=1e-14)
    v4 = np.zeros(L)
    v4[[c - 4, c + 4]] = 1
    v4[[c - 2, c, c + 2]] = [2 / 3, -2 / 3, 2 / 3]
    v4 /= np.linalg.norm(v4)
    assert abs(abs(np.vdot(v4, V[3])) - 1) < 1e-14
    u = np.zeros(L)
    u[[c - 2, c, c + 2]] = np.array([1, -1, 1]) / np.sqrt(3)
    assert abs(np.vdot(u, V[3])) == pytest.approx(np.sqrt(2 / 5), rel=1e-13)
    win = slice(c - 3, c + 4)
    assert np.linalg.norm(V[4][win]) < 1e-14
    assert np.linalg.norm(V[6][win]) < 1e-14
    assert np.linalg.norm(V[5][win]) == pytest.approx(np.sqrt(6 / 35), rel=1e-13)
    assert np.linalg.norm(V[7][win]) == pytest.approx(np.sqrt(2 / 21), rel=1e-13)


def random_sym(n, seed, density=1.0):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(n, n))
    A = A * (rng.random((n, n)) < density)
    H = A + A.T
    return H


@pytest.mark.parametrize("order", [6, 10])
def test_invariant_space_gives_the_exact_exponential(order):
    # 7 x 7 dense H: the Krylov space of any start fills it at dimension 7,
    # so the propagator is exact; order 10 exercises the breakdown stop
    H = random_sym(7, 3)
    rng = np.random.default_rng(4)
    v = rng.normal(size=7) + 1j * rng.normal(size=7)
    dt = 0.3
    out, B, alpha, beta, _ = O.lanczos(*csr_of(H), dt, order, v)
    assert B.shape[0] == 7
    ref = scipy.linalg.expm(-1j * dt * H) @ v
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-12 * np.abs(v).max())


@pytest.mark.parametrize("order", [1, 2, 4])
def test_projection_through_an_independent_krylov_basis(order):
    # the Krylov propagator is V exp(-i V^dag H V dt) V^dag v for ANY
    # orthonormal basis V of span{v, .., H^order v}: build one by QR of the
    # power vectors and compare
    cfg = dict(WL.CONFIGS["ring4"])
    m = O.Model(WL.model_params(cfg))
    s = O.Sim(m, WL.run_params(cfg), *WL.initial_state(cfg))
    s.step(3)
    rp, cols, vals = s.csr()
    H = dense(rp, cols, vals)
    keys, psi = s.state()
    v = psi.copy()
    dt = 0.05
    out, B, alpha, beta, _ = O.lanczos(rp, cols, vals, dt, order, v)
    P = [v / np.linalg.norm(v)]
    for _ in range(order):
        w = H @ P[-1]
        P.append(w / np.linalg.norm(w))
    Q, _ = np.linalg.qr(np.array(P).T)
    Hk = Q.conj().T @ H @ Q
    ref = Q @ (scipy.linalg.expm(-1j * dt * Hk) @ (Q.conj().T @ v))
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-12 * np.abs(v).max())


def test_basis_is_orthonormal_and_tridiagonalises_h():
    H = random_sym(40, 7, density=0.15)
    rng = np.random.default_rng(8)
    v = rng.normal(size=40) + 1j * rng.normal(size=40)
    out, B, alpha, beta, (lo, hi) = O.lanczos(*csr_of(H), 0.1, 8, v)
    n = B.shape[0]
    assert n == 9
    np.testing.assert_allclose(B.conj() @ B.T, np.eye(n), atol=1e-12)
    T = B.conj() @ H @ B.T
    Tref = np.diag(alpha) + np.diag(beta[1:n], 1) + np.diag(beta[1:n], -1)
    np.testing.assert_allclose(T, Tref, atol=1e-11)
    assert beta[0] == pytest.approx(np.linalg.norm(v), rel=1e-14)
    # the propagator is unitary on the Krylov space
    assert np.linalg.norm(out) == pytest.approx(np.linalg.norm(v), rel=1e-13)
    # Gershgorin interval of T, padded
    r = np.abs(Tref).sum(axis=1) - np.abs(alpha)
    assert lo == pytest.approx((alpha - r).min() - 1e-12 * (abs((alpha - r).min()) + abs((alpha + r).max())), rel=1e-14)
    assert hi == pytest.approx((alpha + r).max() + 1e-12 * (abs((alpha - r).min()) + abs((alpha + r).max())), rel=1e-14)


def test_zero_vector_gives_zero():
    H = random_sym(5, 1)
    out, B, alpha, beta, _ = O.lanczos(*csr_of(H), 0.1, 3, np.zeros(5))
    assert B.shape[0] == 0 and np.all(out == 0) and beta[0] == 0.0


def small_cfg():
    cfg = dict(WL.CONFIGS["ring4"])
    cfg.update(extent=[3, 1, 1], cutoff=[1], k=1, k_init=1, theta=1e-10)
    return cfg


def test_sim_with_invariant_krylov_space_equals_the_series():
    # a 3-site ring with cutoff 1 has 3 * 2^3 = 24 states: order 30 spans
    # every H_eff it meets, so the Krylov step is the exact exponential
    cfg = small_cfg()
    m = O.Model(WL.model_params(cfg))
    run = WL.run_params(cfg)
    a = O.Sim(m, run, *WL.initial_state(cfg))
    b = O.Sim(m, dict(run, krylov_order=30), *WL.initial_state(cfg))
    for _ in range(6):
        a.step(1)
        b.step(1)
        ka, pa = a.state()
        kb, pb = b.state()
        assert np.array_equal(ka, kb)
        np.testing.assert_allclose(pb, pa, rtol=0, atol=1e-12)
    # (without re-orthogonalisation the plain recurrence need not stop at
    # the invariant dimension: lost orthogonality keeps beta above the
    # breakdown test, and the extra vectors leave the result exact)
    ob = b.observations()[-1]
    assert 1 <= ob["terms"] <= 31
    assert ob["n_S"] == len(kb)


def test_sim_converges_to_the_series_as_the_order_grows():
    cfg = dict(WL.CONFIGS["ring4"])
    m = O.Model(WL.model_params(cfg))
    # no threshold: the sets then do not depend on the propagator's error
    run = dict(WL.run_params(cfg), dt=0.5, theta=0.0)
    ref = O.Sim(m, run, *WL.initial_state(cfg))
    ref.step(10)
    kr, pr = ref.state()
    errs = []
    for order in (2, 5, 10, 24):
        s = O.Sim(m, dict(run, krylov_order=order), *WL.initial_state(cfg))
        s.step(10)
        k, p = s.state()
        assert np.array_equal(k, kr)
        errs.append(np.abs(p - pr).max())
        o = s.observations()[-1]
        assert o["terms"] == order + 1
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[3] < 1e-12


def test_sim_conserves_norm_and_energy_of_phi():
    cfg = dict(WL.CONFIGS["ring4"])
    m = O.Model(WL.model_params(cfg))
    s = O.Sim(m, dict(WL.run_params(cfg), krylov_order=3),
              *WL.initial_state(cfg))
    for _ in range(5):
        s.step(1)
        phi = s.phi()
        rp, cols, vals = s.csr()
        H = dense(rp, cols, vals)
        o = s.observations()[-1]
        assert o["norm2"] == pytest.approx(np.vdot(phi, phi).real, rel=1e-13)
        e_phi = np.vdot(phi, H @ phi).real
        assert o["energy"] == pytest.approx(e_phi, rel=1e-11, abs=1e-13)


def test_adjoint_rejects_the_krylov_propagator():
    cfg = dict(WL.CONFIGS["ring4"])
    m = O.Model(WL.model_params(cfg))
    with pytest.raises(RuntimeError, match="series"):
        O.Frozen(m, dict(WL.run_params(cfg), krylov_order=3),
                 *WL.initial_state(cfg), steps=2)
