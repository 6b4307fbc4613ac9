"""Brute-force checkers used to pin the oracle (tests only).

Independent formulations, not the oracle's code: the full single-exciton
Hilbert space as a tensor product, the Hamiltonian of Eq. (holstein) built
from Kronecker products of small matrices, graph balls by breadth-first
search over Python sets, and the key integer as a Python big integer.
"""
import itertools
import math

import numpy as np
import scipy.sparse as sp


def sites(p):
    e = p["extent"]
    return e[0] * e[1] * e[2]


def coords(p, i):
    e = p["extent"]
    return (i % e[0], (i // e[0]) % e[1], i // (e[0] * e[1]))


def site_index(p, c):
    e = p["extent"]
    return c[0] + e[0] * (c[1] + e[1] * c[2])


def bonds(p):
    """Nearest-neighbour bonds (i, i2, J_axis), each bond once."""
    out = []
    for i in range(sites(p)):
        c = list(coords(p, i))
        for a in range(p["ndim"]):
            c2 = list(c)
            c2[a] += 1
            if c2[a] >= p["extent"][a]:
                if not p["periodic"][a]:
                    continue
                c2[a] = 0
            out.append((i, site_index(p, c2), p["J"][a]))
    return out


def dims(p):
    V = p["n_modes"]
    return [p["cutoff"][nu] + 1 for _ in range(sites(p)) for nu in range(V)]


def dense_hamiltonian(p):
    """Dense H of Eq. (holstein) on exciton (x) phonon modes, ordered
    exciton first, then (site 0, mode 0), (site 0, mode 1), ..."""
    N, V = sites(p), p["n_modes"]
    ds = dims(p)
    eye = [sp.identity(d, format="csr") for d in ds]

    def kron_all(mats):
        out = mats[0]
        for m in mats[1:]:
            out = sp.kron(out, m, format="csr")
        return out

    E = np.diag(np.asarray(p["eps"], dtype=float))
    for i, i2, J in bonds(p):
        E[i, i2] += J
        E[i2, i] += J
    H = kron_all([sp.csr_matrix(E)] + eye)
    for f, d in enumerate(ds):
        nu = f % V
        num = sp.diags(np.arange(d, dtype=float))
        a = sp.diags(np.sqrt(np.arange(1, d, dtype=float)), 1)
        mats = [sp.identity(N, format="csr")] + list(eye)
        mats[1 + f] = p["omega"][nu] * num
        H = H + kron_all(mats)
        j = f // V
        proj = sp.csr_matrix(([1.0], ([j], [j])), shape=(N, N))
        mats = [proj] + list(eye)
        mats[1 + f] = p["g"][nu] * (a + a.T)
        H = H + kron_all(mats)
    return H.toarray()


def state_index(p, j, occ):
    idx = j
    for n, d in zip(occ, dims(p)):
        idx = idx * d + int(n)
    return idx


def all_states(p):
    ds = dims(p)
    for j in range(sites(p)):
        for occ in itertools.product(*[range(d) for d in ds]):
            yield j, occ


def key_int(p, j, occ):
    """Key as a Python integer: occupations most significant first, site
    field last, widths ceil(log2(c+1)) and max(1, ceil(log2 N))."""
    V = p["n_modes"]
    bj = max(1, math.ceil(math.log2(sites(p))))
    val, pos = j, bj
    for f in reversed(range(len(occ))):
        b = math.ceil(math.log2(p["cutoff"][f % V] + 1))
        val |= int(occ[f]) << pos
        pos += b
    return val, pos


def int_to_words(val, W):
    return [(val >> (64 * (W - 1 - w))) & ((1 << 64) - 1) for w in range(W)]


def ball_sets(H, start, k):
    """Graph ball of radius k around the index set `start` in the graph of
    nonzero off-diagonal entries of the dense matrix H."""
    adj = [set(np.nonzero(H[i])[0].tolist()) - {i} for i in range(H.shape[0])]
    ball = set(start)
    frontier = set(start)
    fronts = [set(start)]
    for _ in range(k):
        nxt = set()
        for i in frontier:
            nxt |= adj[i]
        nxt -= ball
        ball |= nxt
        frontier = nxt
        fronts.append(set(nxt))
    return ball, fronts
