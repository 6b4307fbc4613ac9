"""Shared helpers of the GPU parity tests (GPU path vs the CPU oracle on
identical inputs)."""
import numpy as np

import paper_2603_07341_amd as P
from oracle import oracle as O
import workloads as WL


def sort_rows(keys, *vals):
    order = np.lexsort(keys.T[::-1]) if len(keys) else np.zeros(0, dtype=int)
    return (keys[order],) + tuple(v[order] for v in vals)


def make_pair(name, realization=0, **over):
    cfg = dict(WL.CONFIGS[name])
    cfg.update(over)
    params = WL.model_params(cfg, realization)
    run = WL.run_params(cfg)
    exc, occ, coef = WL.initial_state(cfg)
    gm, om = P.Model(params), O.Model(params)
    gs = P.Sim(gm, run, exc, occ, coef)
    os_ = O.Sim(om, run, exc, occ, coef)
    return cfg, gm, om, gs, os_


def oracle_state(name, steps, **over):
    """State of an oracle run of the workload after `steps` steps."""
    cfg = dict(WL.CONFIGS[name])
    cfg.update(over)
    params = WL.model_params(cfg)
    om = O.Model(params)
    exc, occ, coef = WL.initial_state(cfg)
    s = O.Sim(om, WL.run_params(cfg), exc, occ, coef)
    s.step(steps)
    keys, amps = s.state()
    return keys, amps, s.observations()[-1]["t"]


def assert_same_set(a, b, what):
    a = sort_rows(a)[0]
    b = sort_rows(b)[0]
    assert a.shape == b.shape, "%s: %s vs %s" % (what, a.shape, b.shape)
    assert np.array_equal(a, b), what


def rel_err(x, ref):
    den = np.linalg.norm(ref)
    return np.linalg.norm(x - ref) / (den if den > 0 else 1.0)


def check_obs(go, oo, tol, width=None, N=None):
    """Observables within tol * (|o| + s_o): s_o = 1 for norm and
    autocorrelation, the spectral width for the energy, 1/N for P(j)."""
    for f in ["norm2", "a_re", "a_im", "mass_step", "mass_total"]:
        assert abs(go[f] - oo[f]) <= tol * (abs(oo[f]) + 1.0), (f, go[f], oo[f])
    if width is not None and np.isfinite(go["energy"]):
        assert abs(go["energy"] - oo["energy"]) <= tol * (abs(oo["energy"]) + width), \
            ("energy", go["energy"], oo["energy"])
    for f in ["n_S", "n_M"]:
        assert go[f] == oo[f], (f, go[f], oo[f])
    sN = 1.0 / len(oo["pop"])
    assert np.all(np.abs(go["pop"] - oo["pop"]) <= tol * (np.abs(oo["pop"]) + sN))
