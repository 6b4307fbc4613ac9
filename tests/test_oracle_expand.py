"""Pins of the oracle's neighbour ball (Eqs. (def_neighbor_k), (H_eff))."""
import numpy as np
import pytest

from oracle import oracle as O
from tests import brute
from tests.test_oracle_model import make
import workloads as WL


def keyset(keys):
    return {tuple(int(w) for w in k) for k in keys}


def run_one_step(p, exc, occ, coef, k, theta=0.0):
    m = O.Model(p)
    s = O.Sim(m, {"dt": 0.01, "k": k, "k_init": k, "theta": theta},
              exc, occ, coef)
    s.step(1)
    return m, s


def tb_chain(L=41):
    # tight-binding chain: g = 0 freezes the phonons, eps = 0
    return make(ndim=1, extent=[L], periodic=[0], cutoff=[1], g=(0.0,),
                J=(1.0,))


def test_krylov_example_set_sizes():
    # psi = (|n-1> + |n+1>)/sqrt(2) on a tight-binding chain with eps = 0:
    # |N^(0)| = 2, |N^(1)| = 3, |N^(2)| = 4, union {n-3..n+3} of 7 states
    # (Sec. "Relation to Krylov subspaces").
    p = tb_chain()
    n = 20
    c = 2 ** -0.5
    m, s = run_one_step(p, [n - 1, n + 1], [0] * (2 * 41), [c, 0, c, 0], 2)
    fr = [s.get_set(O.SET_FRONTIER, r) for r in range(3)]
    exc = [sorted(m.unpack(f)[0].tolist()) for f in fr]
    assert exc[0] == [n - 1, n + 1]
    # exact-distance frontiers: N^(1) = {n-2, n, n+2} is found whole in round 1
    assert exc[1] == [n - 2, n, n + 2]
    # N^(2) = {n-3, n-1, n+1, n+3}; its new members are n-3 and n+3
    assert exc[2] == [n - 3, n + 3]
    ball = sorted(m.unpack(s.get_set(O.SET_S))[0].tolist())
    assert ball == list(range(n - 3, n + 4))
    # |N^(k)| as sets: the k-th image of the support under H
    N = [set(exc[0])]
    for _ in range(2):
        N.append({j + d for j in N[-1] for d in (-1, 1)})
    assert [len(x) for x in N] == [2, 3, 4]
    assert set().union(*N) == set(ball)


@pytest.mark.parametrize("order", [1, 2, 3, 5, 8])
def test_lanczos_example_dimension_and_nonzeros(order):
    # From {n-1, n, n+1}: H_eff^(n-1) has dimension 3 + 2(n-1) and 4n
    # off-diagonal nonzeros (App. "Series-based exponentiation compared to a
    # Lanczos algorithm"), here with n - 1 = order.
    p = tb_chain()
    c = 3 ** -0.5
    m, s = run_one_step(p, [19, 20, 21], [0] * (3 * 41), [c, 0, c, 0, c, 0],
                        order)
    nn = order + 1
    rp, cols, vals = s.csr()
    assert s.size() == 3 + 2 * (nn - 1)
    assert len(cols) - s.size() == 4 * nn


@pytest.mark.parametrize("case", [
    dict(ndim=1, extent=[4], periodic=[1], cutoff=[2]),
    dict(ndim=1, extent=[3], periodic=[0], cutoff=[3]),
    dict(ndim=2, extent=[2, 2], periodic=[0, 0], cutoff=[1], J=(-0.5, 0.8)),
    dict(ndim=1, extent=[3], periodic=[1], cutoff=[1, 2], V=2,
         omega=(1.0, 0.2), g=(1.0, 0.5)),
])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_ball_equals_bfs_over_python_sets(case, k):
    p = make(**case)
    H = brute.dense_hamiltonian(p)
    rng = np.random.default_rng(11 + k)
    states = list(brute.all_states(p))
    pick = rng.choice(len(states), size=3, replace=False)
    exc = [states[i][0] for i in pick]
    occ = sum([list(states[i][1]) for i in pick], [])
    coef = sum([[1.0, 0.0]] * 3, [])
    m, s = run_one_step(p, exc, occ, coef, k)
    start = {brute.state_index(p, *states[i]) for i in pick}
    ball, fronts = brute.ball_sets(H, start, k)

    def idx_of(keys):
        e, o = m.unpack(keys)
        return {brute.state_index(p, int(e[i]), o[i]) for i in range(len(e))}

    assert idx_of(s.get_set(O.SET_S)) == ball
    for r in range(k + 1):
        assert idx_of(s.get_set(O.SET_FRONTIER, r)) == fronts[r]


@pytest.mark.parametrize("k", [1, 2, 4])
def test_free_exciton_ball_closed_form(k):
    # g = 0 from a vacuum start: the ball is the lattice ball of radius k
    p = make(ndim=2, extent=[7, 7], periodic=[1, 1], cutoff=[3], g=(0.0,),
             J=(-0.5, -0.5))
    N = 49
    j0 = 3 + 7 * 3
    m, s = run_one_step(p, [j0], [0] * N, [1.0, 0.0], k)
    e, o = m.unpack(s.get_set(O.SET_S))
    assert not o.any()

    def dist(a, b):
        ax, ay, bx, by = a % 7, a // 7, b % 7, b // 7
        dx, dy = abs(ax - bx), abs(ay - by)
        return min(dx, 7 - dx) + min(dy, 7 - dy)

    assert sorted(e.tolist()) == [j for j in range(N) if dist(j, j0) <= k]


@pytest.mark.parametrize("k", [1, 2, 3, 6])
def test_independent_boson_ball_closed_form(k):
    # J = 0: the exciton stays put and only its own modes are excited,
    # B_k = {(j0; n) : sum_nu n_nu <= k, n_nu <= c_nu}
    p = make(ndim=1, extent=[5], periodic=[1], cutoff=[2, 4], V=2,
             omega=(1.0, 0.2), g=(1.0, 0.5), J=(0.0,))
    j0 = 2
    m, s = run_one_step(p, [j0], [0] * 10, [1.0, 0.0], k)
    e, o = m.unpack(s.get_set(O.SET_S))
    assert set(e.tolist()) == {j0}
    got = {tuple(r) for r in o.tolist()}
    want = set()
    for n0 in range(3):
        for n1 in range(5):
            if n0 + n1 <= k:
                occ = [0] * 10
                occ[2 * j0] = n0
                occ[2 * j0 + 1] = n1
                want.add(tuple(occ))
    assert got == want


def test_symmetry_sector_preserved():
    # every state of a long run carries exactly one exciton and occupations
    # within the cutoffs (the key has no room for anything else)
    cfg = WL.CONFIGS["ring4"]
    p = WL.model_params(cfg)
    m = O.Model(p)
    exc, occ, coef = WL.initial_state(cfg)
    s = O.Sim(m, WL.run_params(cfg), exc, occ, coef)
    s.step(20)
    keys, amps = s.state()
    e, o = m.unpack(keys)
    assert ((e >= 0) & (e < 4)).all() and (o <= 4).all()
    assert len(keyset(keys)) == len(keys)
