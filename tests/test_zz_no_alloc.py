"""paces_expmv_static (exp(-i H_S dt) phi with the library's static work
memory, no allocation) against paces_expmv on the same inputs through the
C ABI: two calls in a row, the second on a smaller set, each bit for bit;
a set beyond the static work memory is refused before any device work."""
import numpy as np
import pytest

import paper_2603_07341_amd as P
import workloads as WL

pytestmark = pytest.mark.gpu


def _tensors(gm, keys, amps):
    import torch
    kd = torch.from_numpy(np.ascontiguousarray(keys).view(np.int64).copy()).cuda()
    pd = torch.from_numpy(np.ascontiguousarray(amps).copy()).cuda()
    return kd, pd


def test_static_expmv_matches_allocating_expmv():
    import torch
    cfg = dict(WL.CONFIGS["ring16"])
    params = WL.model_params(cfg)
    gm = P.Model(params)
    dt = cfg["dt"]
    # the ring16 workload's own set after 12 steps, and a seeded state on it
    gs = P.Sim(gm, WL.run_params(cfg), *WL.initial_state(cfg))
    gs.step(12)
    keys, amps = gs.state()
    n = len(keys)
    assert n > 20000, n
    rng = np.random.default_rng(7)
    amps = amps + 1e-3 * (rng.standard_normal(n) + 1j * rng.standard_normal(n))
    for sub in (n, n // 3):  # the second call on a smaller set
        kd, pd = _tensors(gm, keys[:sub], amps[:sub])
        ref = gm.expmv(kd, pd, dt).cpu().numpy()
        out = torch.full_like(pd, complex(float("nan"), float("nan")))
        gm.expmv_static(kd, pd, dt, out=out)
        got = out.cpu().numpy()
        assert got.shape == ref.shape
        assert np.all(np.isfinite(got))
        assert np.array_equal(got, ref), \
            "max |diff| %g" % float(np.max(np.abs(got - ref)))


def test_static_expmv_refuses_sets_beyond_its_memory():
    import torch
    cfg = dict(WL.CONFIGS["ring16"])
    gm = P.Model(WL.model_params(cfg))
    n = 2_000_000  # ~ 200 MB of work memory, above the static 64 MiB
    kd = torch.zeros((n, gm.W), dtype=torch.int64, device="cuda")
    pd = torch.zeros(n, dtype=torch.complex128, device="cuda")
    with pytest.raises(P.PacesError) as ei:
        gm.expmv_static(kd, pd, 0.01)
    assert ei.value.status == 3  # PACES_E_CAPACITY
