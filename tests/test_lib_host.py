"""Host-side checks of the GPU library that need no GPU: the shared object
loads, exports every symbol of include/paces.h, and its host codec and
model validation agree with the oracle.  No kernel is launched."""
import os
import re

import numpy as np
import pytest

import paper_2603_07341_amd as P
from oracle import oracle as O
from tests import brute
import workloads as WL

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    src = open(os.path.join(ROOT, "include", "paces.h")).read()
    return sorted(set(re.findall(r"\b(paces_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = P.lib()
    declared = header_symbols()
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(P.EXPORTS) == declared
    assert lib.paces_abi_version() == 12


@pytest.mark.parametrize("name", ["ring4", "ring16", "sq6x6", "cube4", "ring12"])
def test_host_codec_matches_oracle(name):
    cfg = WL.CONFIGS[name]
    p = WL.model_params(cfg)
    gm, om = P.Model(p), O.Model(p)
    assert (gm.N, gm.W, gm.D, gm.B) == (om.N, om.W, om.D, om.B)
    rng = np.random.default_rng(1)
    n, V, N = 300, p["n_modes"], brute.sites(p)
    exc = rng.integers(0, N, n)
    occ = np.stack([rng.integers(0, p["cutoff"][f % V] + 1, n)
                    for f in range(N * V)], axis=1)
    k1, k2 = gm.pack(exc, occ), om.pack(exc, occ)
    assert np.array_equal(k1, k2)
    e, o = gm.unpack(k1)
    assert np.array_equal(e, exc) and np.array_equal(o, occ)


@pytest.mark.parametrize("bad", [
    dict(ndim=0), dict(ndim=1, extent=[2, 1, 1], periodic=[1, 0, 0]),
    dict(n_modes=5), dict(cutoff=[0, 0, 0, 0]), dict(cutoff=[300, 0, 0, 0]),
    dict(n_real=257), dict(n_real=-1),
    # R * (N + 3) above the LDS budget of the batched reductions
    dict(extent=[64, 1, 1], n_real=128),
    # N * cutoff above the 14-bit packed total occupation
    dict(extent=[2048, 1, 1], cutoff=[10, 0, 0, 0]),
    # parameters must be finite
    dict(J=[float("nan"), 0, 0]), dict(g=[float("inf"), 0, 0, 0]),
    dict(eps=[0.0, float("nan"), 0.0, 0.0]),
])
def test_model_validation_rejects(bad):
    p = WL.model_params(WL.CONFIGS["ring4"])
    p.update(bad)
    with pytest.raises(P.PacesError) as ei:
        P.Model(p)
    assert ei.value.status == 1


def test_pack_rejects_out_of_range():
    gm = P.Model(WL.model_params(WL.CONFIGS["ring4"]))
    with pytest.raises(P.PacesError):
        gm.pack([4], [0, 0, 0, 0])
    with pytest.raises(P.PacesError):
        gm.pack([0], [0, 5, 0, 0])


def test_batched_model_accepts_eps_per_realization():
    cfg = WL.CONFIGS["sq6x6"]
    p = WL.batch_params(cfg)
    gm = P.Model(p)
    assert gm.R == 64 and len(p["eps"]) == 64 * 36
    # the realization id lives above the canonical key bits: the canonical
    # layout (and so the host codec) is unchanged by batching
    single = P.Model(WL.model_params(cfg))
    assert (gm.N, gm.W, gm.D, gm.B) == (single.N, single.W, single.D, single.B)


def test_model_key_words_matches_info():
    import ctypes as C
    for name in ("ring4", "sq6x6", "cube4"):
        gm = P.Model(WL.model_params(WL.CONFIGS[name]))
        W = C.c_int32()
        assert P.lib().paces_model_key_words(gm.h, C.byref(W)) == 0
        assert W.value == gm.W


def test_allocator_needs_both_functions():
    import ctypes as C
    f = P._ALLOC_FN(lambda n, s, u: None)
    assert P.lib().paces_set_allocator(f, None, None) == 1


def test_library_abi_matches_header():
    src = open(os.path.join(ROOT, "include", "paces.h")).read()
    want = int(re.search(r"#define PACES_ABI_VERSION (\d+)", src).group(1))
    assert P.lib().paces_abi_version() == want


@pytest.mark.parametrize("order", [-1, 64])
def test_krylov_order_out_of_range_is_rejected_before_device_work(order):
    cfg = dict(WL.CONFIGS["ring4"])
    m = P.Model(WL.model_params(cfg))
    run = dict(WL.run_params(cfg), krylov_order=order)
    with pytest.raises(P.PacesError) as ei:
        P.Sim(m, run, *WL.initial_state(cfg))
    assert ei.value.status == 1


@pytest.mark.parametrize("m", [1, 2, 5, 13, 34, 55])
def test_library_taylor_thresholds_match_exact_definition(m):
    # the library's own computation (host code, no GPU) against the exact
    # rational computation of the oracle pins
    from tests.test_oracle_taylor import theta
    assert P.taylor_theta(m) == pytest.approx(theta(m), rel=1e-9)
    assert P.taylor_theta(0) == -1.0 and P.taylor_theta(56) == -1.0


@pytest.mark.parametrize("over", [dict(taylor_order=-2), dict(taylor_order=61),
                                  dict(taylor_order=-1, krylov_order=3)])
def test_taylor_order_validation(over):
    cfg = dict(WL.CONFIGS["ring4"])
    m = P.Model(WL.model_params(cfg))
    with pytest.raises(P.PacesError) as ei:
        P.Sim(m, dict(WL.run_params(cfg), **over), *WL.initial_state(cfg))
    assert ei.value.status == 1
