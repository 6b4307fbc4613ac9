"""Pins of the oracle's Hamiltonian (Eqs. (tb), (holstein)) against a dense
Kronecker-product construction and the paper's nonzero counts."""
import numpy as np
import pytest

from oracle import oracle as O
from tests import brute
import workloads as WL


def make(ndim, extent, periodic, cutoff, omega=(1.0,), g=(1.0,), J=(-0.5,),
         eps=None, V=1):
    cfg = dict(WL.CONFIGS["ring4"], ndim=ndim, extent=list(extent) + [1] * (3 - len(extent)),
               periodic=list(periodic) + [0] * (3 - len(periodic)),
               n_modes=V, cutoff=list(cutoff), omega=list(omega), g=list(g),
               J=list(J))
    p = WL.model_params(cfg)
    if eps is not None:
        p["eps"] = list(eps)
    return p


def full_space_sim(p, k_big=60):
    """Oracle run whose first step grows the ball over the whole connected
    single-exciton sector."""
    m = O.Model(p)
    N = brute.sites(p)
    exc, occ, coef = [0], [0] * (N * p["n_modes"]), [1.0, 0.0]
    run = {"dt": 0.01, "k": k_big, "k_init": k_big, "theta": 0.0}
    s = O.Sim(m, run, exc, occ, coef)
    s.step(1)
    return m, s


def csr_to_dense_in_brute_order(p, m, s):
    keys, _ = s.state()
    exc, occ = m.unpack(keys)
    idx = np.array([brute.state_index(p, int(exc[i]), occ[i])
                    for i in range(len(exc))])
    rp, cols, vals = s.csr()
    n = len(idx)
    dim = n
    Hd = np.zeros((dim, dim))
    for r in range(n):
        for e in range(rp[r], rp[r + 1]):
            Hd[r, cols[e]] = vals[e]
    return idx, Hd, rp, cols


SMALL = [
    ("open chain 3, c=2", dict(ndim=1, extent=[3], periodic=[0], cutoff=[2])),
    ("ring 3, c=2", dict(ndim=1, extent=[3], periodic=[1], cutoff=[2])),
    ("ring 4, c=2, eps", dict(ndim=1, extent=[4], periodic=[1], cutoff=[2],
                             eps=[0.3, -0.1, 0.7, 0.05])),
    ("2D open 2x2, c=2", dict(ndim=2, extent=[2, 2], periodic=[0, 0],
                              cutoff=[2], J=(-0.5, 0.8))),
    ("ring 3, two modes", dict(ndim=1, extent=[3], periodic=[1], cutoff=[1, 2],
                               V=2, omega=(1.0, 0.2), g=(1.0, 0.5))),
]


@pytest.mark.parametrize("name,kw", SMALL, ids=[s[0] for s in SMALL])
def test_csr_equals_dense_kronecker_hamiltonian(name, kw):
    p = make(**kw)
    m, s = full_space_sim(p)
    Hfull = brute.dense_hamiltonian(p)
    idx, Hd, rp, cols = csr_to_dense_in_brute_order(p, m, s)
    # the ball from one state covers the whole sector (J != 0 and g != 0)
    assert len(idx) == Hfull.shape[0]
    ref = Hfull[np.ix_(idx, idx)]
    off = ~np.eye(len(idx), dtype=bool)
    # off-diagonal elements are single products: bitwise equal
    assert np.array_equal(ref[off], Hd[off])
    # the Kronecker sum adds omega*n one mode at a time, the oracle forms
    # omega*T: equal up to the rounding of a few additions
    assert np.allclose(np.diag(ref), np.diag(Hd), rtol=0, atol=1e-14)
    # symmetric, one entry per (row, col), diagonal always present
    assert np.array_equal(Hd, Hd.T)
    for r in range(len(idx)):
        row_cols = cols[rp[r]:rp[r + 1]]
        assert len(set(row_cols.tolist())) == len(row_cols)
        assert r in row_cols


@pytest.mark.parametrize("L,d", [(3, 2), (3, 3), (4, 2), (2, 4)])
def test_open_chain_nonzero_count(L, d):
    # counting every diagonal, the open Holstein chain has
    # d^L [(5L - 2) - 2L/d] structural nonzeros (App. "Sparse matrices and
    # their exponentials")
    p = make(ndim=1, extent=[L], periodic=[0], cutoff=[d - 1])
    m, s = full_space_sim(p)
    rp, cols, vals = s.csr()
    assert len(cols) == d ** L * (5 * L - 2) - 2 * L * d ** (L - 1)


@pytest.mark.parametrize("L,d", [(3, 2), (3, 3), (4, 2)])
def test_ring_nonzero_count(L, d):
    p = make(ndim=1, extent=[L], periodic=[1], cutoff=[d - 1])
    m, s = full_space_sim(p)
    rp, cols, vals = s.csr()
    assert len(cols) == d ** L * 5 * L - 2 * L * d ** (L - 1)


def test_printed_sparsity_claim():
    # L = 9, d = 5: density below 1/(4e6); 587 MiB of 8-byte nonzeros
    # against 2248 TiB for the dense matrix.
    L, d = 9, 5
    nnz = d ** L * ((5 * L - 2) - 2 * L / d)
    dim = L * d ** L
    assert nnz / dim ** 2 < 1 / 4e6
    assert round(nnz * 8 / 2 ** 20) == 587
    assert round(dim ** 2 * 8 / 2 ** 40) == 2248


def test_tight_binding_nonzero_count():
    # g = 0 freezes the phonons: the open chain has 3L - 2 nonzeros
    L = 7
    p = make(ndim=1, extent=[L], periodic=[0], cutoff=[1], g=(0.0,))
    m, s = full_space_sim(p)
    rp, cols, vals = s.csr()
    assert s.size() == L and len(cols) == 3 * L - 2


@pytest.mark.parametrize("name", ["ring16", "sq6x6", "cube4"])
def test_slots_give_distinct_neighbours(name):
    cfg = WL.CONFIGS[name]
    p = WL.model_params(cfg)
    m = O.Model(p)
    rng = np.random.default_rng(3)
    N, V = brute.sites(p), p["n_modes"]
    n = 100
    exc = rng.integers(0, N, n)
    occ = np.stack([rng.integers(0, p["cutoff"][f % V] + 1, n)
                    for f in range(N * V)], axis=1)
    keys = m.pack(exc, occ)
    nb, ex, vals, diag = m.neighbors(keys)
    for i in range(n):
        seen = {tuple(nb[i, q].tolist()) for q in range(m.D) if ex[i, q]}
        assert len(seen) == int(ex[i].sum())
        assert tuple(keys[i].tolist()) not in seen
        # diagonal: eps_j + sum_nu omega_nu * total occupation
        T = [int(occ[i][nu::V].sum()) for nu in range(V)]
        d = p["eps"][exc[i]]
        for nu in range(V):
            d = d + p["omega"][nu] * T[nu]
        assert diag[i] == d
