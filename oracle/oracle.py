"""ctypes binding of the CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use
this module.  The GPU library never imports it.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

OBS_FIELDS = ["t", "norm2", "energy", "a_re", "a_im", "mass_step",
              "mass_total", "n_S", "n_M", "terms", "E_min", "E_max"]
SET_M, SET_S, SET_FRONTIER = 0, 1, 2


class _Desc(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("extent", C.c_int32 * 3),
                ("periodic", C.c_int32 * 3), ("n_modes", C.c_int32),
                ("cutoff", C.c_int32 * 4), ("omega", C.c_double * 4),
                ("g", C.c_double * 4), ("J", C.c_double * 3),
                ("eps", C.POINTER(C.c_double))]


class _Params(C.Structure):
    _fields_ = [("dt", C.c_double), ("k", C.c_int32), ("k_init", C.c_int32),
                ("theta", C.c_double), ("max_terms", C.c_int32),
                ("max_states", C.c_int64), ("q_nom", C.c_int64),
                ("krylov_order", C.c_int32), ("taylor_order", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from oracle import build as _build
            _build.build()
        _lib = C.CDLL(LIB_PATH)
        _lib.orc_last_error.restype = C.c_char_p
    return _lib


def _check(rc):
    if rc != 0:
        raise RuntimeError("oracle: " + lib().orc_last_error().decode())


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def pack_fields(widths, values, W):
    out = np.zeros(W, dtype=np.uint64)
    w = np.asarray(widths, dtype=np.int32)
    v = np.asarray(values, dtype=np.uint64)
    _check(lib().orc_pack_fields(C.c_int32(len(w)), _p(w, C.c_int32),
                                 _p(v, C.c_uint64), C.c_int32(W),
                                 _p(out, C.c_uint64)))
    return out


class Model:
    def __init__(self, params):
        d = _Desc()
        d.ndim = params["ndim"]
        for a in range(3):
            d.extent[a] = params["extent"][a]
            d.periodic[a] = params["periodic"][a]
            d.J[a] = params["J"][a]
        d.n_modes = params["n_modes"]
        for nu in range(4):
            d.cutoff[nu] = params["cutoff"][nu]
            d.omega[nu] = params["omega"][nu]
            d.g[nu] = params["g"][nu]
        self._eps = np.ascontiguousarray(params["eps"], dtype=np.float64)
        d.eps = _p(self._eps, C.c_double)
        h = C.c_void_p()
        _check(lib().orc_model_create(C.byref(d), C.byref(h)))
        self.h = h
        N, W, D, B = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().orc_model_info(h, C.byref(N), C.byref(W), C.byref(D),
                                    C.byref(B)))
        self.N, self.W, self.D, self.B = N.value, W.value, D.value, B.value
        self.V = params["n_modes"]

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.orc_model_destroy(self.h)
            self.h = None

    def pack(self, exc, occ):
        exc = np.ascontiguousarray(exc, dtype=np.int32)
        occ = np.ascontiguousarray(occ, dtype=np.uint16)
        n = len(exc)
        keys = np.zeros(n * self.W, dtype=np.uint64)
        _check(lib().orc_pack(self.h, C.c_int64(n), _p(exc, C.c_int32),
                              _p(occ, C.c_uint16), _p(keys, C.c_uint64)))
        return keys.reshape(n, self.W)

    def unpack(self, keys):
        keys = np.ascontiguousarray(keys, dtype=np.uint64).reshape(-1)
        n = len(keys) // self.W
        exc = np.zeros(n, dtype=np.int32)
        occ = np.zeros(n * self.N * self.V, dtype=np.uint16)
        _check(lib().orc_unpack(self.h, C.c_int64(n), _p(keys, C.c_uint64),
                                _p(exc, C.c_int32), _p(occ, C.c_uint16)))
        return exc, occ.reshape(n, self.N * self.V)

    def neighbors(self, keys):
        keys = np.ascontiguousarray(keys, dtype=np.uint64).reshape(-1)
        n = len(keys) // self.W
        out = np.zeros(n * self.D * self.W, dtype=np.uint64)
        ex = np.zeros(n * self.D, dtype=np.uint8)
        vals = np.zeros(n * self.D, dtype=np.float64)
        diag = np.zeros(n, dtype=np.float64)
        _check(lib().orc_neighbors(self.h, C.c_int64(n), _p(keys, C.c_uint64),
                                   _p(out, C.c_uint64), _p(ex, C.c_uint8),
                                   _p(vals, C.c_double), _p(diag, C.c_double)))
        return (out.reshape(n, self.D, self.W), ex.reshape(n, self.D).astype(bool),
                vals.reshape(n, self.D), diag)


class Sim:
    def __init__(self, model, run, exc, occ, coef, max_terms=200):
        self.model = model
        p = _Params()
        p.dt = run["dt"]
        p.k = run["k"]
        p.k_init = run["k_init"]
        p.theta = run["theta"]
        p.max_terms = max_terms
        p.max_states = int(run.get("max_states", 0))
        p.q_nom = int(run.get("q_nom", 0))
        p.krylov_order = int(run.get("krylov_order", 0))
        p.taylor_order = int(run.get("taylor_order", 0))
        exc = np.ascontiguousarray(exc, dtype=np.int32)
        occ = np.ascontiguousarray(occ, dtype=np.uint16)
        coef = np.ascontiguousarray(coef, dtype=np.float64)
        h = C.c_void_p()
        _check(lib().orc_sim_create(model.h, C.byref(p), C.c_int64(len(exc)),
                                    _p(exc, C.c_int32), _p(occ, C.c_uint16),
                                    _p(coef, C.c_double), C.byref(h)))
        self.h = h

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.orc_sim_destroy(self.h)
            self.h = None

    def step(self, n=1):
        _check(lib().orc_sim_step(self.h, C.c_int64(n)))

    def set_model(self, model):
        _check(lib().orc_sim_set_model(self.h, model.h))
        self.model = model

    def size(self):
        n = C.c_int64()
        _check(lib().orc_sim_size(self.h, C.byref(n)))
        return n.value

    def state(self):
        """(sorted keys [n, W] uint64, amplitudes [n] complex128)."""
        n = self.size()
        keys = np.zeros(n * self.model.W, dtype=np.uint64)
        amps = np.zeros(2 * n, dtype=np.float64)
        _check(lib().orc_sim_get_state(self.h, _p(keys, C.c_uint64),
                                       _p(amps, C.c_double)))
        return keys.reshape(n, self.model.W), amps.view(np.complex128)

    def phi(self):
        n = self.size()
        amps = np.zeros(2 * n, dtype=np.float64)
        _check(lib().orc_sim_get_phi(self.h, _p(amps, C.c_double)))
        return amps.view(np.complex128)

    def set_state(self, keys, amps, t=0.0):
        keys = np.ascontiguousarray(keys, dtype=np.uint64).reshape(-1)
        amps = np.ascontiguousarray(np.asarray(amps, dtype=np.complex128)).view(np.float64)
        n = len(keys) // self.model.W
        _check(lib().orc_sim_set_state(self.h, C.c_int64(n), _p(keys, C.c_uint64),
                                       _p(amps, C.c_double), C.c_double(t)))

    def set_prev_counts(self, nS, nM):
        """|S| and |M| of the step that led to the loaded state (the state
        cap's q rule)."""
        _check(lib().orc_sim_set_prev_counts(self.h, C.c_int64(int(nS)),
                                             C.c_int64(int(nM))))

    def get_set(self, which, rnd=0):
        n = C.c_int64()
        _check(lib().orc_sim_get_set(self.h, C.c_int32(which), C.c_int32(rnd),
                                     C.byref(n), None))
        keys = np.zeros(n.value * self.model.W, dtype=np.uint64)
        _check(lib().orc_sim_get_set(self.h, C.c_int32(which), C.c_int32(rnd),
                                     C.byref(n), _p(keys, C.c_uint64)))
        return keys.reshape(n.value, self.model.W)

    def observations(self):
        """List of dicts (one per step) with the scalar fields and 'pop'."""
        n = C.c_int64()
        _check(lib().orc_sim_num_obs(self.h, C.byref(n)))
        out = []
        for i in range(n.value):
            f = np.zeros(len(OBS_FIELDS), dtype=np.float64)
            pop = np.zeros(self.model.N, dtype=np.float64)
            _check(lib().orc_sim_obs(self.h, C.c_int64(i), _p(f, C.c_double),
                                     _p(pop, C.c_double)))
            d = dict(zip(OBS_FIELDS, f.tolist()))
            d["pop"] = pop
            out.append(d)
        return out

    def csr(self):
        nrows, nnz = C.c_int64(), C.c_int64()
        _check(lib().orc_sim_csr(self.h, C.byref(nrows), C.byref(nnz), None,
                                 None, None))
        rp = np.zeros(nrows.value + 1, dtype=np.int64)
        cols = np.zeros(nnz.value, dtype=np.int64)
        vals = np.zeros(nnz.value, dtype=np.float64)
        _check(lib().orc_sim_csr(self.h, C.byref(nrows), C.byref(nnz),
                                 _p(rp, C.c_int64), _p(cols, C.c_int64),
                                 _p(vals, C.c_double)))
        return rp, cols, vals


def expmv(rowptr, cols, vals, dt, emin, emax, v, max_terms=200):
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    vals = np.ascontiguousarray(vals, dtype=np.float64)
    vin = np.ascontiguousarray(np.asarray(v, dtype=np.complex128)).view(np.float64)
    n = len(rowptr) - 1
    vout = np.zeros(2 * n, dtype=np.float64)
    terms = C.c_int32()
    _check(lib().orc_expmv(C.c_int64(n), _p(rowptr, C.c_int64), _p(cols, C.c_int64),
                           _p(vals, C.c_double), C.c_double(dt), C.c_double(emin),
                           C.c_double(emax), C.c_int32(max_terms),
                           _p(np.ascontiguousarray(vin), C.c_double),
                           _p(vout, C.c_double), C.byref(terms)))
    return vout.view(np.complex128), terms.value


def lanczos(rowptr, cols, vals, dt, order, v):
    """Krylov propagator of order `order` on a CSR matrix: returns
    (v_out, basis [dim, n], alpha [dim], beta [dim], (e_lo, e_hi))."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    vals = np.ascontiguousarray(vals, dtype=np.float64)
    vin = np.ascontiguousarray(np.asarray(v, dtype=np.complex128)).view(np.float64)
    n = len(rowptr) - 1
    vout = np.zeros(2 * n, dtype=np.float64)
    basis = np.zeros(2 * n * (order + 1), dtype=np.float64)
    alpha = np.zeros(order + 1, dtype=np.float64)
    beta = np.zeros(order + 1, dtype=np.float64)
    dim = C.c_int32()
    er = np.zeros(2, dtype=np.float64)
    _check(lib().orc_lanczos(C.c_int64(n), _p(rowptr, C.c_int64), _p(cols, C.c_int64),
                             _p(vals, C.c_double), C.c_double(dt), C.c_int32(order),
                             _p(vin, C.c_double), _p(vout, C.c_double),
                             _p(basis, C.c_double), _p(alpha, C.c_double),
                             _p(beta, C.c_double), C.byref(dim), _p(er, C.c_double)))
    d = dim.value
    B = basis.view(np.complex128).reshape(order + 1, n)[:d]
    return vout.view(np.complex128), B, alpha[:d], beta[:max(d, 1)], tuple(er)


def set_threads(n):
    """Threads of the oracle's row loops (timing only)."""
    _check(lib().orc_set_threads(C.c_int32(int(n))))


def threads():
    lib().orc_threads.restype = C.c_int32
    return int(lib().orc_threads())


def taylor_theta(m):
    lib().orc_taylor_theta.restype = C.c_double
    return lib().orc_taylor_theta(C.c_int32(m))


def taylor_select(norm):
    m, s = C.c_int32(), C.c_int32()
    _check(lib().orc_taylor_select(C.c_double(norm), C.byref(m), C.byref(s)))
    return m.value, s.value


def taylor(rowptr, cols, vals, dt, emin, emax, order, v):
    """Truncated Taylor propagator (order -1: degree and substeps chosen);
    returns (v_out, matrix-vector products)."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    vals = np.ascontiguousarray(vals, dtype=np.float64)
    vin = np.ascontiguousarray(np.asarray(v, dtype=np.complex128)).view(np.float64)
    n = len(rowptr) - 1
    vout = np.zeros(2 * n, dtype=np.float64)
    mvs = C.c_int32()
    _check(lib().orc_taylor(C.c_int64(n), _p(rowptr, C.c_int64), _p(cols, C.c_int64),
                            _p(vals, C.c_double), C.c_double(dt), C.c_double(emin),
                            C.c_double(emax), C.c_int32(order), _p(vin, C.c_double),
                            _p(vout, C.c_double), C.byref(mvs)))
    return vout.view(np.complex128), mvs.value


def param_names(model_params):
    """Names of the gradient entries: J per axis, g and omega per mode,
    eps per site."""
    nd, V = model_params["ndim"], model_params["n_modes"]
    ext = model_params["extent"]
    N = ext[0] * ext[1] * ext[2]
    return (["J%d" % a for a in range(nd)] + ["g%d" % v for v in range(V)]
            + ["omega%d" % v for v in range(V)] + ["eps%d" % i for i in range(N)])


class Frozen:
    """A recorded run whose sets are held fixed for the adjoint gradient."""

    def __init__(self, model, run, exc, occ, coef, steps, max_terms=200):
        p = _Params()
        p.dt = run["dt"]
        p.k = run["k"]
        p.k_init = run["k_init"]
        p.theta = run["theta"]
        p.max_terms = max_terms
        p.max_states = int(run.get("max_states", 0))
        p.q_nom = int(run.get("q_nom", 0))
        p.krylov_order = int(run.get("krylov_order", 0))
        p.taylor_order = int(run.get("taylor_order", 0))
        exc = np.ascontiguousarray(exc, dtype=np.int32)
        occ = np.ascontiguousarray(occ, dtype=np.uint16)
        coef = np.ascontiguousarray(coef, dtype=np.float64)
        h = C.c_void_p()
        _check(lib().orc_frozen_record(model.h, C.byref(p), C.c_int64(len(exc)),
                                       _p(exc, C.c_int32), _p(occ, C.c_uint16),
                                       _p(coef, C.c_double), C.c_int64(steps),
                                       C.byref(h)))
        self.h = h
        self.model = model
        n, P = C.c_int64(), C.c_int32()
        _check(lib().orc_frozen_info(h, C.byref(n), C.byref(P), None))
        self.steps, self.n_params = n.value, P.value

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.orc_frozen_destroy(self.h)
            self.h = None

    def sizes(self):
        out = np.zeros(self.steps + 1, dtype=np.int64)
        _check(lib().orc_frozen_info(self.h, None, None, _p(out, C.c_int64)))
        return out

    def get_set(self, step):
        n = int(self.sizes()[step])
        keys = np.zeros(n * self.model.W, dtype=np.uint64)
        _check(lib().orc_frozen_get_set(self.h, C.c_int64(step),
                                        _p(keys, C.c_uint64)))
        return keys.reshape(n, self.model.W)

    def eval(self, model):
        """a[s] = <psi0|psi_s>, s = 0..steps, replayed with `model`."""
        a = np.zeros(2 * (self.steps + 1), dtype=np.float64)
        _check(lib().orc_frozen_eval(self.h, model.h, _p(a, C.c_double)))
        return a.view(np.complex128)

    def grad(self, model, gbar):
        """(a, dL/dtheta) for gbar[s] = dL/d conj(a_s)."""
        gb = np.ascontiguousarray(np.asarray(gbar, dtype=np.complex128)).view(np.float64)
        a = np.zeros(2 * (self.steps + 1), dtype=np.float64)
        g = np.zeros(self.n_params, dtype=np.float64)
        _check(lib().orc_frozen_grad(self.h, model.h, _p(gb, C.c_double),
                                     _p(a, C.c_double), _p(g, C.c_double)))
        return a.view(np.complex128), g
