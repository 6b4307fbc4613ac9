"""Boundary features beyond the step: device-side record copies into
torch tensors, and device memory from torch's caching allocator."""
import gc

import numpy as np
import pytest
import torch

import paper_2603_07341_amd as P
from tests.gpu_helpers import sort_rows
import workloads as WL

pytestmark = pytest.mark.gpu


def test_series_field_copies_records_to_device():
    cfg = dict(WL.CONFIGS["ring12"], eps_sigma=0.2)
    R, steps = 3, 7
    m = P.Model(WL.batch_params(cfg, R))
    s = P.Sim(m, WL.run_params(cfg), *WL.initial_state(cfg))
    s.step(steps)
    host = s.series()  # [steps, R, rec]
    for field in ("norm2", "a_re", "n_S", "E_max"):
        out = torch.full((steps * R,), -1.0, dtype=torch.float64, device="cuda")
        s.series_field(field, out)
        torch.cuda.synchronize()
        k = P.OBS_FIELDS.index(field)
        assert np.array_equal(out.cpu().numpy().reshape(steps, R), host[:, :, k])
    out = torch.zeros(2 * R, dtype=torch.float64, device="cuda")
    s.series_field(12 + 5, out, first=3, n=2)  # population of site 5
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().reshape(2, R), host[3:5, :, 17])


def run_ring(steps):
    cfg = WL.CONFIGS["ring16"]
    m = P.Model(WL.model_params(cfg))
    s = P.Sim(m, WL.run_params(cfg), *WL.initial_state(cfg))
    s.step(steps)
    k, a = sort_rows(*s.state())
    return m, s, k, a


def test_torch_caching_allocator_gives_identical_results():
    _, _, k0, a0 = run_ring(12)
    gc.collect()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    P.use_torch_allocator(True)
    try:
        m, s, k1, a1 = run_ring(12)
        assert torch.cuda.memory_allocated() > before + (1 << 20)
        assert np.array_equal(k0, k1) and np.array_equal(a0, a1)
    finally:
        # switching back while the sim lives: its blocks still go back to
        # torch when it is freed
        P.use_torch_allocator(False)
    s.step(2)
    del m, s
    gc.collect()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before


def test_step_log_writes_every_record(tmp_path, monkeypatch):
    path = tmp_path / "log.csv"
    monkeypatch.setenv("PACES_LOG", str(path))
    cfg = dict(WL.CONFIGS["ring12"], eps_sigma=0.2)
    m = P.Model(WL.batch_params(cfg, 2))
    s = P.Sim(m, WL.run_params(cfg), *WL.initial_state(cfg))
    s.step(4)
    monkeypatch.delenv("PACES_LOG")
    s.step(1)
    rows = np.loadtxt(path, delimiter=",")
    rec = s.series()
    assert rows.shape == (8, 2 + m.rec_doubles)
    for line in rows:
        step, r = int(line[0]), int(line[1])
        assert np.array_equal(line[2:], rec[step, r])


@pytest.mark.parametrize("kernels_only", [False, True])
def test_profile_levels_time_the_clenshaw_launches(kernels_only):
    # level 1 times every stage and each Clenshaw launch; level 2 one
    # middle Clenshaw launch per step (events recorded by the dispatch).
    # Middle terms carry their algorithmic bytes; results do not change.
    cfg = dict(WL.CONFIGS["ring16"])
    m = P.Model(WL.model_params(cfg))
    a = P.Sim(m, WL.run_params(cfg), *WL.initial_state(cfg))
    b = P.Sim(m, WL.run_params(cfg), *WL.initial_state(cfg))
    a.step(20)
    b.step(20)
    a.profile(True, kernels_only=kernels_only)
    a.profile_reset()
    a.step(3)
    b.step(3)
    prof = a.profile_get()
    K = a.observations()[-1]["K"]
    assert K >= 4
    # level 1: every middle term; level 2: one sampled middle term per step
    assert prof["launches"]["term"] == (3 if kernels_only else 3 * (K - 3))
    assert prof["term_bytes"] > 0 and prof["ms"]["term"] > 0
    staged = prof["launches"]["expand"] > 0
    assert staged == (not kernels_only)
    ka, aa = a.state()
    kb, bb = b.state()
    assert np.array_equal(sort_rows(ka, aa)[1], sort_rows(kb, bb)[1])


def test_capacity_beyond_the_device_is_cut_to_fit():
    # a row-capacity hint of 2^31 rows (several hundred GB of row arrays)
    # is cut to what the device holds instead of failing with E_OOM; the
    # run is the same as with the automatic capacity
    cfg = WL.CONFIGS["ring16"]
    m = P.Model(WL.model_params(cfg))
    torch.cuda.empty_cache()
    free0 = torch.cuda.mem_get_info()[0]
    big = P.Sim(m, dict(WL.run_params(cfg), cap_hint=2 ** 31),
                *WL.initial_state(cfg))
    assert torch.cuda.mem_get_info()[0] < free0
    big.step(6)
    kb, ab = sort_rows(*big.state())
    big.close()
    ref = P.Sim(m, WL.run_params(cfg), *WL.initial_state(cfg))
    ref.step(6)
    kr, ar = sort_rows(*ref.state())
    ref.close()
    assert np.array_equal(kb, kr)
    assert np.array_equal(ab, ar)
