"""Shared helpers of the GPU parity tests (GPU path vs the CPU oracle on
identical inputs).

Amplitude bound.  Both sides reach the same exp(-i H dt) phi by different
series (Chebyshev with Clenshaw on the GPU, shifted Taylor in the oracle),
so an amplitude differs by rounding only.  Every element is held to
    |psi_gpu - psi_oracle| <= tol |psi_oracle| + f ||psi_oracle||_inf,
f = 128 u s: one step rounds each element at most once per operand of K
series terms of a (D + 1)-entry row (K (D + 1) <= 128 for the workloads
here), relative to the largest amplitude that reaches it, and s steps since
the common state add up.  u = 2^-53 for FP64 amplitudes (tol < 1e-7) and
2^-24 for FP32.  Besides, the relative 2-norm error stays within tol.

Discarded weight.  A dropped row with |c| <= cmax (theta under threshold
truncation) has a weight that differs by at most 2 cmax (tol cmax + f), f
as above with ||psi||_inf <= 1; summed over the dropped rows, plus the
rounding of the sum itself."""
import numpy as np

import paper_2603_07341_amd as P
from oracle import oracle as O
import workloads as WL

ROUND_TERMS = 128


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


def unit_roundoff(tol):
    return 2.0 ** -53 if tol < 1e-7 else 2.0 ** -24


def elem_floor(tol, steps):
    """Absolute floor of the element bound, relative to ||psi||_inf."""
    return ROUND_TERMS * unit_roundoff(tol) * max(1, int(steps))


def assert_amps(x, ref, tol, steps=1, what="amplitudes"):
    """x (GPU, rows in the oracle's order) against ref (oracle): relative
    2-norm within tol and every element within tol |ref_n| + floor."""
    x = np.asarray(x)
    ref = np.asarray(ref)
    assert x.shape == ref.shape, (what, x.shape, ref.shape)
    e2 = rel_err(x, ref)
    assert e2 <= tol, (what, "relative 2-norm error", e2)
    if len(ref) == 0:
        return
    inf = float(np.max(np.abs(ref)))
    bound = tol * np.abs(ref) + elem_floor(tol, steps) * inf
    d = np.abs(x - ref)
    bad = np.nonzero(d > bound)[0]
    if len(bad):
        i = int(bad[np.argmax(d[bad] / bound[bad])])
        raise AssertionError(
            "%s: %d element(s) beyond tol |ref| + floor; worst row %d: gpu %r "
            "oracle %r, |diff| %.3e bound %.3e" % (what, len(bad), i, x[i],
                                                   ref[i], d[i], bound[i]))


def mass_bound(oo, tol, cmax, n_drop, steps_before):
    """Bound on |delta_gpu - delta_oracle| of one step that drops at most
    n_drop rows, each with |c| <= cmax, from an input state that has
    diverged for steps_before steps (0: a common input state)."""
    f = elem_floor(tol, steps_before) if steps_before > 0 else 0.0
    per_row = 2.0 * cmax * (tol * cmax + f)
    u = unit_roundoff(1e-10)
    return per_row * n_drop + 4.0 * u * max(1, n_drop) * abs(oo["mass_step"])


def dropped(prev_keys, prev_amps, new_keys):
    """(number, largest |c|) of the rows of a state that a step dropped."""
    prev_keys = np.ascontiguousarray(prev_keys, dtype=np.uint64)
    new_keys = np.ascontiguousarray(new_keys, dtype=np.uint64)
    if len(prev_keys) == 0:
        return 0, 0.0
    W = prev_keys.shape[1]
    row = np.dtype((np.void, 8 * W))
    gone = ~np.isin(prev_keys.view(row).ravel(), new_keys.view(row).ravel())
    n = int(np.count_nonzero(gone))
    return n, (float(np.max(np.abs(prev_amps[gone]))) if n else 0.0)


def check_obs(go, oo, tol, width=None, N=None, drop=None, steps_before=0,
              mass_total_bound=None, mass_prior=0.0):
    """Observables within tol * (|o| + s_o): s_o = 1 for norm and
    autocorrelation, the spectral width for the energy, 1/N for P(j).
    With drop = (n_drop, cmax) given, the discarded weight of the step (and
    the cumulative one, within mass_total_bound when given) is held to the
    bound of mass_bound instead of tol * (|o| + 1); the cumulative weight
    of a run that has diverged for several steps also carries mass_prior,
    the sum of the earlier steps' bounds.  Returns the step's bound (0
    without drop)."""
    for f in ["norm2", "a_re", "a_im"]:
        assert abs(go[f] - oo[f]) <= tol * (abs(oo[f]) + 1.0), (f, go[f], oo[f])
    if drop is not None:
        b = mass_bound(oo, tol, drop[1], drop[0], steps_before)
        assert abs(go["mass_step"] - oo["mass_step"]) <= b, \
            ("mass_step", go["mass_step"], oo["mass_step"], b)
        bt = b if mass_total_bound is None else mass_total_bound
        bt += mass_prior + 4.0 * unit_roundoff(1e-10) * abs(oo["mass_total"])
        assert abs(go["mass_total"] - oo["mass_total"]) <= bt, \
            ("mass_total", go["mass_total"], oo["mass_total"], bt)
    else:
        for f in ["mass_step", "mass_total"]:
            assert abs(go[f] - oo[f]) <= tol * (abs(oo[f]) + 1.0), (f, go[f], oo[f])
    if width is not None and np.isfinite(go["energy"]):
        assert abs(go["energy"] - oo["energy"]) <= tol * (abs(oo["energy"]) + width), \
            ("energy", go["energy"], oo["energy"])
    for f in ["n_S", "n_M"]:
        assert go[f] == oo[f], (f, go[f], oo[f])
    sN = 1.0 / len(oo["pop"])
    assert np.all(np.abs(go["pop"] - oo["pop"]) <= tol * (np.abs(oo["pop"]) + sN))
    return b if drop is not None else 0.0


def check_series(gobs, oobs, tol, theta, n_first, first_diverged=0):
    """check_obs over consecutive records of two threshold-truncated runs
    that started from a common state of n_first rows: a dropped row has
    |c| < theta, at most the previous set is dropped; the per-step bounds
    are summed for the cumulative weight."""
    assert len(gobs) == len(oobs)
    n_old, tot = n_first, 0.0
    for i, (g, o) in enumerate(zip(gobs, oobs)):
        b = mass_bound(o, tol, theta, n_old, first_diverged + i)
        tot += b
        check_obs(g, o, tol, width=o["E_max"] - o["E_min"],
                  drop=(n_old, theta), steps_before=first_diverged + i,
                  mass_total_bound=tot)
        n_old = int(o["n_S"])
