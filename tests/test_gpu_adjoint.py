"""Adjoint gradient (Form (3)) on the GPU through the C ABI.

With the sets of the forward run frozen, the GPU's a(t), replay and
gradient are compared with the oracle's frozen-set replay and its
augmented-matrix gradient (gradient parity <= 1e-8 |g|_inf), and the
gradient with fourth-order central differences of the GPU's own replay.
Checkpoint intervals must not change the result beyond rounding, and the
torch.autograd.Function must hand torch the same gradient."""
import numpy as np
import pytest

import paper_2603_07341_amd as P
from oracle import oracle as O
import workloads as WL

pytestmark = pytest.mark.gpu

CASES = {
    # ragged last segment (24 = 3 * 7 + 3)
    "ring": ("ring12", 24, 7, dict(extent=[6, 1, 1], cutoff=[4], theta=1e-6)),
    "square": ("sq6x6", 8, 3, dict(extent=[3, 3, 1], cutoff=[2], theta=1e-5,
                                   precision=64)),
    "two_modes": ("cube4", 6, 4, dict(extent=[3, 1, 1], ndim=1,
                                      periodic=[1, 0, 0], J=[-0.5],
                                      cutoff=[2, 3], theta=1e-5, init="local",
                                      precision=64)),
    # the adjoint workload itself (12-site ring, cutoff 10), 20 steps
    "ring12": ("ring12", 20, 8, {}),
}


def setup(key):
    name, steps, ckpt, over = CASES[key]
    cfg = dict(WL.CONFIGS[name])
    cfg.update(over)
    p = WL.model_params(cfg)
    run = WL.run_params(cfg)
    init = WL.initial_state(cfg)
    gm = P.Model(p)
    gs = P.Sim(gm, run, *init)
    a = gs.adjoint_forward(steps, ckpt)
    return cfg, p, run, init, gm, gs, a, steps, ckpt


def target(a, seed=11):
    rng = np.random.default_rng(seed)
    return a + 0.3 * (rng.standard_normal(len(a)) + 1j * rng.standard_normal(len(a)))


def with_param(p, name, delta):
    return P.params_with_theta(p, P.theta_of(p) + delta * (
        np.arange(len(P.theta_of(p))) == O.param_names(p).index(name)))


@pytest.mark.parametrize("key", ["ring", "square", "two_modes", "ring12"])
def test_gradient_matches_oracle(key):
    cfg, p, run, init, gm, gs, a, steps, ckpt = setup(key)
    om = O.Model(p)
    f = O.Frozen(om, run, *init, steps)
    assert np.array_equal(gm.n_params, f.n_params)
    oa = f.eval(om)
    assert np.max(np.abs(a - oa)) <= 1e-10
    tau = target(oa)
    g_gpu = gs.adjoint_backward(a - tau)
    _, g_orc = f.grad(om, oa - tau)
    assert np.max(np.abs(g_gpu - g_orc)) <= 1e-8 * np.max(np.abs(g_orc)), \
        np.abs(g_gpu - g_orc) / np.max(np.abs(g_orc))
    # the sim is left as after the forward run: the replay still works
    assert np.max(np.abs(gs.adjoint_replay() - a)) <= 1e-13


def test_replay_with_other_parameters_matches_oracle():
    cfg, p, run, init, gm, gs, a, steps, ckpt = setup("ring")
    om = O.Model(p)
    f = O.Frozen(om, run, *init, steps)
    for name, d in (("J0", 2e-3), ("g0", -3e-3), ("omega0", 1e-3), ("eps2", 5e-3)):
        q = with_param(p, name, d)
        ga = gs.adjoint_replay(P.Model(q))
        oa = f.eval(O.Model(q))
        assert np.max(np.abs(ga - oa)) <= 1e-10, name
        assert np.max(np.abs(ga - a)) > 1e-8, name  # the change is seen


def test_gradient_matches_gpu_finite_differences():
    cfg, p, run, init, gm, gs, a, steps, ckpt = setup("ring")
    tau = target(a)
    loss = lambda aa: float(np.sum(np.abs(aa - tau) ** 2))
    g = gs.adjoint_backward(a - tau)
    names = O.param_names(p)
    h = 1e-4
    Lp = lambda nm, d: loss(gs.adjoint_replay(P.Model(with_param(p, nm, d))))
    scale_all = np.max(np.abs(g))
    for nm in ("J0", "g0", "omega0", "eps0", "eps3"):
        fd = (-Lp(nm, 2 * h) + 8 * Lp(nm, h) - 8 * Lp(nm, -h) + Lp(nm, -2 * h)) / (12 * h)
        k = names.index(nm)
        scale = max(abs(g[k]), 1e-2 * scale_all)
        assert abs(g[k] - fd) <= 1e-7 * scale, (nm, g[k], fd)


def test_checkpoint_interval_does_not_change_gradient():
    name, steps, _, over = CASES["ring"]
    cfg = dict(WL.CONFIGS[name])
    cfg.update(over)
    p = WL.model_params(cfg)
    grads = []
    a0 = None
    for ckpt in (1, 5, steps):
        gm = P.Model(p)
        gs = P.Sim(gm, WL.run_params(cfg), *WL.initial_state(cfg))
        a = gs.adjoint_forward(steps, ckpt)
        if a0 is None:
            a0 = a
            tau = target(a)
        assert np.array_equal(a, a0)
        grads.append(gs.adjoint_backward(a - tau))
    for g in grads[1:]:
        assert np.allclose(g, grads[0], rtol=1e-12, atol=1e-14 * np.max(np.abs(grads[0])))


@pytest.mark.parametrize("device", ["cuda", "cpu"])
def test_autograd_function_gives_the_adjoint_gradient(device):
    """AutocorrFn keeps a(t), the incoming gradient and dL/dtheta on the
    GPU (device-buffer adjoint entry points) and returns the gradient on
    theta's device; against the oracle's gradient."""
    import torch
    name, steps, ckpt, over = CASES["ring"]
    cfg = dict(WL.CONFIGS[name])
    cfg.update(over)
    p = WL.model_params(cfg)
    run = WL.run_params(cfg)
    init = WL.initial_state(cfg)
    theta = torch.tensor(P.theta_of(p), dtype=torch.float64, device=device,
                         requires_grad=True)
    a = P.AutocorrFn.apply(theta, p, run, init, steps, ckpt)
    assert a.dtype == torch.complex128 and a.shape == (steps + 1,)
    assert a.is_cuda
    a_host = a.detach().cpu().numpy()
    tau = torch.from_numpy(target(a_host)).to(a.device)
    loss = ((a - tau).abs() ** 2).sum()
    loss.backward()
    assert theta.grad.device == theta.device
    om = O.Model(p)
    f = O.Frozen(om, run, *init, steps)
    _, g_orc = f.grad(om, a_host - tau.cpu().numpy())
    g = theta.grad.cpu().numpy()
    assert np.max(np.abs(g - g_orc)) <= 1e-8 * np.max(np.abs(g_orc))


def test_device_buffer_adjoint_matches_host_buffers():
    """paces_adjoint_forward_dev / backward_dev against the host-buffer
    entry points on the same recorded run: a bit for bit (no reduction
    feeds it), the gradient to rounding (the per-site sums of the epsilon
    components are LDS atomics, whose order is not fixed)."""
    import torch
    name, steps, ckpt, over = CASES["ring"]
    cfg = dict(WL.CONFIGS[name])
    cfg.update(over)
    p = WL.model_params(cfg)
    init = WL.initial_state(cfg)
    hs = P.Sim(P.Model(p), WL.run_params(cfg), *init)
    a_h = hs.adjoint_forward(steps, ckpt)
    ds = P.Sim(P.Model(p), WL.run_params(cfg), *init)
    a_d = torch.empty(steps + 1, dtype=torch.complex128, device="cuda")
    ds.adjoint_forward_dev(steps, a_d, ckpt)
    assert np.array_equal(a_d.cpu().numpy(), a_h)
    gbar = (a_h - target(a_h))
    g_h = hs.adjoint_backward(gbar)
    g_d = torch.zeros(ds.model.n_params, dtype=torch.float64, device="cuda")
    ds.adjoint_backward_dev(torch.from_numpy(gbar).to("cuda"), g_d)
    g_d = g_d.cpu().numpy()
    assert np.max(np.abs(g_d - g_h)) <= 1e-13 * np.max(np.abs(g_h))
    with pytest.raises(ValueError):
        ds.adjoint_backward_dev(torch.from_numpy(gbar), g_d)


def test_adjoint_rejects_what_it_does_not_support():
    name, steps, ckpt, over = CASES["ring"]
    cfg = dict(WL.CONFIGS[name])
    cfg.update(over)
    init = WL.initial_state(cfg)
    p = WL.model_params(cfg)
    # complex64 amplitudes
    s = P.Sim(P.Model(p), WL.run_params(cfg, precision=32), *init)
    with pytest.raises(P.PacesError) as ei:
        s.adjoint_forward(3, 2)
    assert ei.value.status == 8
    # a parameter at zero (the ELL would miss its edges)
    q = dict(p)
    q["g"] = [0.0] + list(p["g"][1:])
    s = P.Sim(P.Model(q), WL.run_params(cfg), *init)
    with pytest.raises(P.PacesError) as ei:
        s.adjoint_forward(3, 2)
    assert ei.value.status == 8
    # several realizations
    b = WL.batch_params(dict(cfg, eps_sigma=0.1, eps_seed=5), 2)
    s = P.Sim(P.Model(b), WL.run_params(cfg), *init)
    with pytest.raises(P.PacesError) as ei:
        s.adjoint_forward(3, 2)
    assert ei.value.status == 8
    # not a new sim; backward before forward
    s = P.Sim(P.Model(p), WL.run_params(cfg), *init)
    with pytest.raises(P.PacesError) as ei:
        s._adj_steps = 3
        s.adjoint_backward(np.zeros(4, complex))
    assert ei.value.status == 7
    s.step(1)
    with pytest.raises(P.PacesError) as ei:
        s.adjoint_forward(3, 2)
    assert ei.value.status == 7
