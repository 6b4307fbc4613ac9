"""The step stage by stage (paces_run_stage) through the C ABI: the six
stages in order give what paces_step gives, out-of-order calls are refused,
and an oracle-supplied set of 1.19e6 states with seeded amplitudes is
propagated on exactly its own set (theta = 0, k = 0) against the oracle."""
import numpy as np
import pytest

import paper_2603_07341_amd as P
from oracle import oracle as O
from tests.gpu_helpers import assert_amps, check_obs, sort_rows
import workloads as WL

pytestmark = pytest.mark.gpu

STAGES = ["select", "expand", "transfer", "build", "propagate", "observe"]


@pytest.mark.parametrize("over", [{}, dict(krylov_order=6), dict(taylor_order=-1),
                                  dict(precision=32)],
                         ids=["series", "krylov", "taylor", "fp32"])
def test_staged_steps_equal_fused_steps(over):
    cfg = dict(WL.CONFIGS["ring16"])
    params = WL.model_params(cfg)
    run = dict(WL.run_params(cfg), **over)
    init = WL.initial_state(cfg)
    a = P.Sim(P.Model(params), run, *init)
    b = P.Sim(P.Model(params), run, *init)
    for step in range(14):
        a.step(1)
        for st in STAGES:
            b.run_stage(st)
        ka, va = sort_rows(*a.state())
        kb, vb = sort_rows(*b.state())
        assert np.array_equal(ka, kb), step
        if "krylov_order" in over:
            assert_amps(vb, va, 1e-12, what="step %d" % step)
        else:
            assert np.array_equal(va, vb), step
    ra, rb = a.series(), b.series()
    assert np.array_equal(ra[:, 7:10], rb[:, 7:10])
    assert np.allclose(ra, rb, rtol=1e-12, atol=1e-15)


def test_stage_order_is_enforced():
    cfg = WL.CONFIGS["ring16"]
    s = P.Sim(P.Model(WL.model_params(cfg)), WL.run_params(cfg),
              *WL.initial_state(cfg))
    with pytest.raises(P.PacesError) as ei:
        s.run_stage("expand")
    assert ei.value.status == 7
    s.run_stage("select")
    with pytest.raises(P.PacesError) as ei:
        s.run_stage("transfer")
    assert ei.value.status == 7
    with pytest.raises(P.PacesError) as ei:
        s.run_stage(6)  # a profiling-only stage index
    assert ei.value.status == 1
    # a full step abandons the staged one; the state is intact
    s.step(1)
    assert s.num_records() == 1
    for st in STAGES:
        s.run_stage(st)
    assert s.num_records() == 2


def test_half_done_in_place_step_must_be_finished():
    """Once the expansion stage of an in-place step (one from the previous
    step's graph) has run, the set is already the new one while the
    amplitudes are still phi: a full step refuses to abandon it, and
    finishing its stages gives what a fused step gives.  A staged step that
    has only selected may be abandoned."""
    cfg = dict(WL.CONFIGS["ring16"])
    params = WL.model_params(cfg)
    run = WL.run_params(cfg)
    init = WL.initial_state(cfg)
    a = P.Sim(P.Model(params), run, *init)
    b = P.Sim(P.Model(params), run, *init)
    a.step(3)
    b.step(3)
    b.run_stage("select")
    b.step(1)  # abandons the selection
    a.step(1)
    b.run_stage("select")
    b.run_stage("expand")
    with pytest.raises(P.PacesError) as ei:
        b.step(1)
    assert ei.value.status == 7
    for st in STAGES[2:]:
        b.run_stage(st)
    a.step(1)
    ka, va = sort_rows(*a.state())
    kb, vb = sort_rows(*b.state())
    assert np.array_equal(ka, kb) and np.array_equal(va, vb)
    assert a.num_records() == b.num_records() == 5


def test_propagate_oracle_set_at_size():
    """S = every ring16 state with at most 6 phonons (1.19e6 states), phi
    seeded; with theta = 0 and k = 0 the step is exp(-i H_S dt) phi on S.
    Sets bit for bit, amplitudes to 1e-10 element by element, observables."""
    cfg = dict(WL.CONFIGS["ring16"])
    params = WL.model_params(cfg)
    exc, occ, coef = WL.phonon_ball_state(cfg, 6)
    run = dict(WL.run_params(cfg), theta=0.0, k=0, k_init=0)
    gm = P.Model(params)
    keys = gm.pack(exc, occ)
    amps = coef.view(np.complex128)
    assert len(keys) == 16 * 74613
    init = WL.initial_state(cfg)
    gs = P.Sim(gm, run, *init)
    gs.set_state(keys, amps, 0.25)
    for st in STAGES:
        gs.run_stage(st)
    os_ = O.Sim(O.Model(params), run, *init)
    os_.set_state(keys, amps, 0.25)
    os_.step(1)
    gk, ga = sort_rows(*gs.state())
    ok, oa = os_.state()
    assert np.array_equal(gk, ok)
    assert_amps(ga, oa, 1e-10)
    go, oo = gs.observations()[-1], os_.observations()[-1]
    assert go["n_S"] == go["n_M"] == len(keys)
    check_obs(go, oo, 1e-10, width=oo["E_max"] - oo["E_min"], drop=(0, 0.0))


def _ball_tensors(n_max):
    import torch
    cfg = dict(WL.CONFIGS["ring16"])
    params = WL.model_params(cfg)
    exc, occ, coef = WL.phonon_ball_state(cfg, n_max)
    gm = P.Model(params)
    keys = gm.pack(exc, occ)
    amps = coef.view(np.complex128)
    kd = torch.from_numpy(keys.view(np.int64).copy()).cuda()
    pd = torch.from_numpy(amps.copy()).cuda()
    return cfg, params, gm, keys, amps, kd, pd


def test_expmv_on_a_given_set_matches_oracle():
    """paces_expmv (no sim) on every ring16 state with at most 4 phonons,
    seeded phi: against the oracle's step with theta = 0 and k = 0 from the
    same state, element by element, and bit for bit against the staged
    PROPAGATE of a sim on the same set."""
    cfg, params, gm, keys, amps, kd, pd = _ball_tensors(4)
    dt = cfg["dt"]
    psi = gm.expmv(kd, pd, dt).cpu().numpy()
    run = dict(WL.run_params(cfg), theta=0.0, k=0, k_init=0)
    init = WL.initial_state(cfg)
    os_ = O.Sim(O.Model(params), run, *init)
    os_.set_state(keys, amps, 0.0)
    os_.step(1)
    ok, oa = os_.state()
    order = np.lexsort(keys.T[::-1])
    assert np.array_equal(keys[order], ok)
    assert_amps(psi[order], oa, 1e-10)
    gs = P.Sim(gm, run, *init)
    gs.set_state(keys, amps, 0.0)
    for st in STAGES:
        gs.run_stage(st)
    sk, sa = sort_rows(*gs.state())
    assert np.array_equal(psi[order], sa)


def test_expmv_refuses_bad_sets():
    import torch
    cfg, params, gm, keys, amps, kd, pd = _ball_tensors(2)
    # a repeated key
    k2 = kd.clone()
    k2[1] = k2[0]
    with pytest.raises(P.PacesError) as ei:
        gm.expmv(k2, pd, 0.01)
    assert ei.value.status == 1
    # bits set above the state's 68 bits (and occupations above the cutoff)
    k3 = kd.clone()
    k3[2, 0] = -1
    with pytest.raises(P.PacesError) as ei:
        gm.expmv(k3, pd, 0.01)
    assert ei.value.status == 1
    # the output may not alias the input; no rows is a no-op
    with pytest.raises(P.PacesError):
        gm.expmv(kd, pd, 0.01, out=pd)
    e = torch.zeros(0, dtype=torch.complex128, device="cuda")
    gm.expmv(torch.zeros((0, gm.W), dtype=torch.int64, device="cuda"), e, 0.01)
