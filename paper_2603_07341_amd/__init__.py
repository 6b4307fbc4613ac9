"""MI355X co-evolving-subspace propagator: Python binding of libpaces.so.

Argument marshalling only.  Every stage of the time step runs in the HIP
kernels of the library; there is no CPU path.  torch is imported first so
that the process uses the HIP runtime torch ships, and torch streams are
passed to the library as plain hipStream_t handles.
"""
import ctypes as C
import os

import numpy as np

try:
    import torch  # noqa: F401  (loads the HIP runtime before the library)
except ImportError:  # pragma: no cover - torch is part of the image
    torch = None

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpaces.so")

OBS_FIELDS = ["t", "norm2", "energy", "a_re", "a_im", "mass_step",
              "mass_total", "n_S", "n_M", "K", "E_min", "E_max"]
SET_M, SET_S, SET_FRONTIER = 0, 1, 2
STAGES = ["select", "expand", "transfer", "build", "propagate", "observe",
          "term", "krylov"]
STATUS = {0: "OK", 1: "E_ARG", 2: "E_OOM", 3: "E_CAPACITY", 4: "E_NONFINITE",
          5: "E_PROPAGATOR", 6: "E_HIP", 7: "E_STATE", 8: "E_UNSUPPORTED"}

# Every symbol include/paces.h declares.
EXPORTS = [
    "paces_last_error", "paces_abi_version", "paces_taylor_theta",
    "paces_record_doubles",
    "paces_load_model", "paces_free_model", "paces_model_info",
    "paces_pack_keys", "paces_unpack_keys", "paces_init_state",
    "paces_free_sim", "paces_step", "paces_observe", "paces_num_records",
    "paces_series", "paces_get_state", "paces_set_state", "paces_get_set",
    "paces_get_phi", "paces_profile_enable", "paces_profile_get",
    "paces_profile_reset", "paces_get_tuning", "paces_set_tuning",
    "paces_autotune", "paces_num_params", "paces_adjoint_forward",
    "paces_adjoint_replay", "paces_adjoint_backward", "paces_set_allocator",
    "paces_model_key_words", "paces_series_field", "paces_set_model",
    "paces_run_stage", "paces_adjoint_forward_dev", "paces_adjoint_backward_dev",
    "paces_profile_mark", "paces_expmv", "paces_expmv_static",
]


class PacesError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class _Desc(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("extent", C.c_int32 * 3),
                ("periodic", C.c_int32 * 3), ("n_modes", C.c_int32),
                ("cutoff", C.c_int32 * 4), ("omega", C.c_double * 4),
                ("g", C.c_double * 4), ("J", C.c_double * 3),
                ("n_real", C.c_int32), ("eps", C.POINTER(C.c_double))]


class _Run(C.Structure):
    _fields_ = [("dt", C.c_double), ("k", C.c_int32), ("k_init", C.c_int32),
                ("theta", C.c_double), ("cap_states", C.c_int64),
                ("precision", C.c_int32), ("tol", C.c_double),
                ("k_max_terms", C.c_int32), ("obs_mask", C.c_uint32),
                ("max_states", C.c_int64), ("q_nom", C.c_int64),
                ("krylov_order", C.c_int32), ("taylor_order", C.c_int32)]


class _Obs(C.Structure):
    _fields_ = [("t", C.c_double), ("norm2", C.c_double),
                ("energy", C.c_double), ("autocorr_re", C.c_double),
                ("autocorr_im", C.c_double), ("mass_step", C.c_double),
                ("mass_total", C.c_double), ("n_S", C.c_int64),
                ("n_M", C.c_int64), ("K", C.c_int32), ("E_min", C.c_double),
                ("E_max", C.c_double), ("pop", C.POINTER(C.c_double))]


class _Profile(C.Structure):
    _fields_ = [("ms", C.c_double * 8), ("launches", C.c_int64 * 8),
                ("term_bytes", C.c_double), ("krylov_bytes", C.c_double),
                ("rows_steps", C.c_double)]


class _Tuning(C.Structure):
    _fields_ = [("graph", C.c_int32), ("table_shift", C.c_int32),
                ("term_rows", C.c_int32), ("warm", C.c_int32)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                "libpaces.so is not built; run "
                "python paper_2603_07341_amd/build.py")
        _lib = C.CDLL(LIB_PATH)
        _lib.paces_last_error.restype = C.c_char_p
        _lib.paces_abi_version.restype = C.c_int32
        _lib.paces_taylor_theta.restype = C.c_double
        _lib.paces_record_doubles.restype = C.c_int32
        _lib.paces_num_params.restype = C.c_int32
    return _lib


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)
_allocator_refs = []  # callbacks stay alive: their blocks may outlive a switch


def use_torch_allocator(on=True):
    """Take later device allocations of the library from torch's caching
    allocator (on=True) or from hipMalloc (on=False); blocks already made
    are returned to the allocator that made them."""
    if not on:
        _check(lib().paces_set_allocator(None, None, None))
        return

    def _alloc(nbytes, stream, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes))
        except Exception:  # out of memory: the library reports E_OOM
            return None

    def _free(ptr, stream, user):
        torch.cuda.caching_allocator_delete(ptr)

    refs = (_ALLOC_FN(_alloc), _FREE_FN(_free))
    _check(lib().paces_set_allocator(refs[0], refs[1], None))
    _allocator_refs.append(refs)


def _check(rc):
    if rc != 0:
        raise PacesError(rc, lib().paces_last_error().decode())


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _stream(stream):
    if stream is None:
        if torch is not None and torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
        return C.c_void_p(0)
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


class Model:
    """A Holstein lattice (parameters as a plain dict, see workloads).

    params["n_real"] (default 1) realizations of the site energies share
    one set; params["eps"] then holds n_real * N energies, realization-major.
    """

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
        self.R = int(params.get("n_real", 1))
        d.n_real = self.R
        self._eps = np.ascontiguousarray(params["eps"], dtype=np.float64).reshape(-1)
        d.eps = _p(self._eps, C.c_double)
        h = C.c_void_p()
        _check(lib().paces_load_model(C.byref(d), C.byref(h)))
        self.h = h
        N, W, D, B = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().paces_model_info(h, C.byref(N), C.byref(W), C.byref(D),
                                      C.byref(B)))
        self.N, self.W, self.D, self.B = N.value, W.value, D.value, B.value
        self.V = params["n_modes"]
        self.rec_doubles = lib().paces_record_doubles(h)
        self.n_params = lib().paces_num_params(h)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.paces_free_model(self.h)
            self.h = None

    def expmv(self, keys, phi, dt, out=None, stream=None):
        """psi = exp(-i H_S dt) phi on the set S of the given canonical
        keys (paces_expmv).  keys: int64 cuda tensor [n, W] holding the
        uint64 words; phi: complex128 cuda tensor [n]; returns psi (a new
        tensor, or `out`)."""
        return self._expmv(lib().paces_expmv, keys, phi, dt, out, stream)

    def expmv_static(self, keys, phi, dt, out=None, stream=None):
        """expmv without allocation (paces_expmv_static): the library's work
        memory is a fixed 64 MiB device array; larger sets raise
        PacesError (PACES_E_CAPACITY).  Pass `out` to allocate nothing on
        this side either."""
        return self._expmv(lib().paces_expmv_static, keys, phi, dt, out, stream)

    def _expmv(self, fn, keys, phi, dt, out, stream):
        n = phi.numel()
        if keys.dtype != torch.int64 or not keys.is_cuda or \
                not keys.is_contiguous() or keys.numel() != n * self.W:
            raise ValueError("keys must be a contiguous int64 cuda tensor of "
                             "n * W words")
        if phi.dtype != torch.complex128 or not phi.is_cuda or \
                not phi.is_contiguous():
            raise ValueError("phi must be a contiguous complex128 cuda tensor")
        if out is None:
            out = torch.empty_like(phi)
        elif out.dtype != torch.complex128 or not out.is_cuda or \
                not out.is_contiguous() or out.numel() != n:
            raise ValueError("out must be a contiguous complex128 cuda tensor "
                             "of n entries")
        _check(fn(self.h, C.c_int64(n), C.c_void_p(keys.data_ptr()),
                  C.c_void_p(phi.data_ptr()), C.c_double(dt),
                  C.c_void_p(out.data_ptr()), _stream(stream)))
        return out

    def pack(self, exc, occ):
        exc = np.ascontiguousarray(exc, dtype=np.int32)
        occ = np.ascontiguousarray(occ, dtype=np.uint16)
        n = len(exc)
        keys = np.zeros(n * self.W, dtype=np.uint64)
        _check(lib().paces_pack_keys(self.h, C.c_int64(n), _p(exc, C.c_int32),
                                     _p(occ, C.c_uint16), _p(keys, C.c_uint64)))
        return keys.reshape(n, self.W)

    def unpack(self, keys):
        keys = np.ascontiguousarray(keys, dtype=np.uint64).reshape(-1)
        n = len(keys) // self.W
        exc = np.zeros(n, dtype=np.int32)
        occ = np.zeros(n * self.N * self.V, dtype=np.uint16)
        _check(lib().paces_unpack_keys(self.h, C.c_int64(n),
                                       _p(keys, C.c_uint64), _p(exc, C.c_int32),
                                       _p(occ, C.c_uint16)))
        return exc, occ.reshape(n, self.N * self.V)


class Sim:
    """Device state of one run on the current HIP device."""

    def __init__(self, model, run, exc, occ, coef, stream=None, obs_mask=0,
                 k_max_terms=0, tol=0.0):
        self.model = model
        r = _Run()
        r.dt = run["dt"]
        r.k = run["k"]
        r.k_init = run["k_init"]
        r.theta = run["theta"]
        r.cap_states = int(run.get("cap_hint", 0))
        r.precision = run.get("precision", 64)
        r.tol = tol
        r.k_max_terms = k_max_terms
        r.obs_mask = obs_mask
        r.max_states = int(run.get("max_states", 0))
        r.q_nom = int(run.get("q_nom", 0))
        r.krylov_order = int(run.get("krylov_order", 0))
        r.taylor_order = int(run.get("taylor_order", 0))
        exc = np.ascontiguousarray(exc, dtype=np.int32)
        occ = np.ascontiguousarray(occ, dtype=np.uint16)
        coef = np.ascontiguousarray(coef, dtype=np.float64)
        h = C.c_void_p()
        _check(lib().paces_init_state(model.h, C.byref(r), C.c_int64(len(exc)),
                                      _p(exc, C.c_int32), _p(occ, C.c_uint16),
                                      _p(coef, C.c_double), _stream(stream),
                                      C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.paces_free_sim(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def set_model(self, model):
        """Later steps use `model` (same shape, other J, g, omega, eps):
        a piecewise-constant Hamiltonian."""
        _check(lib().paces_set_model(self.h, model.h))
        self.model = model

    def step(self, n=1, stream=None):
        _check(lib().paces_step(self.h, C.c_int64(n), _stream(stream)))

    def run_stage(self, stage, stream=None):
        """One stage of a step: a name of STAGES[:6] or its index; the six
        in order make one step."""
        idx = STAGES.index(stage) if isinstance(stage, str) else int(stage)
        _check(lib().paces_run_stage(self.h, C.c_int32(idx), _stream(stream)))

    def observe(self, realization=0, stream=None):
        o = _Obs()
        _check(lib().paces_observe(self.h, C.c_int32(realization), C.byref(o),
                                   _stream(stream)))
        d = {f: getattr(o, f) for f in ["t", "norm2", "energy", "mass_step",
                                        "mass_total", "n_S", "n_M", "K",
                                        "E_min", "E_max"]}
        d["a_re"], d["a_im"] = o.autocorr_re, o.autocorr_im
        d["pop"] = np.ctypeslib.as_array(o.pop, shape=(self.model.N,)).copy()
        return d

    def series_field(self, field, out, first=0, n=None, stream=None):
        """Copy one record field (index into OBS_FIELDS, or 12 + site for a
        population) of steps first..first+n-1 into the float64 CUDA tensor
        `out` ([n * R]), asynchronously on the stream."""
        if n is None:
            n = self.num_records() - first
        if isinstance(field, str):
            field = OBS_FIELDS.index(field)
        if out.numel() < n * self.model.R or out.dtype != torch.float64:
            raise ValueError("out needs n * R float64 entries")
        _check(lib().paces_series_field(self.h, C.c_int32(field),
                                        C.c_void_p(out.data_ptr()),
                                        C.c_int64(first), C.c_int64(n),
                                        _stream(stream)))
        return out

    def num_records(self):
        n = C.c_int64()
        _check(lib().paces_num_records(self.h, C.byref(n)))
        return n.value

    def series(self, first=0, n=None, stream=None):
        """Observation records as an array [n, 12 + N], or [n, R, 12 + N]
        for a batched model."""
        if n is None:
            n = self.num_records() - first
        R = self.model.R
        out = np.zeros(n * R * self.model.rec_doubles, dtype=np.float64)
        _check(lib().paces_series(self.h, C.c_int64(first), C.c_int64(n),
                                  _p(out, C.c_double), _stream(stream)))
        if R == 1:
            return out.reshape(n, self.model.rec_doubles)
        return out.reshape(n, R, self.model.rec_doubles)

    def observations(self, realization=0, stream=None):
        """Per-step observation dicts of one realization, same fields as
        the oracle's."""
        rec = self.series(stream=stream)
        if self.model.R > 1:
            rec = rec[:, realization]
        out = []
        for r in rec:
            d = dict(zip(OBS_FIELDS, r[:12].tolist()))
            d["pop"] = r[12:].copy()
            out.append(d)
        return out

    def size(self, stream=None):
        n = C.c_int64()
        _check(lib().paces_get_state(self.h, C.byref(n), None, None, None,
                                     _stream(stream)))
        return n.value

    def state(self, stream=None, with_real=False):
        """(keys [n, W] uint64 in row order, amplitudes [n] complex128), plus
        the realization of each row [n] int32 when with_real."""
        n = self.size(stream)
        keys = np.zeros(n * self.model.W, dtype=np.uint64)
        amps = np.zeros(2 * n, dtype=np.float64)
        real = np.zeros(n, dtype=np.int32)
        nn = C.c_int64()
        _check(lib().paces_get_state(self.h, C.byref(nn), _p(keys, C.c_uint64),
                                     _p(amps, C.c_double), _p(real, C.c_int32),
                                     _stream(stream)))
        keys = keys.reshape(n, self.model.W)
        if with_real:
            return keys, amps.view(np.complex128), real
        return keys, amps.view(np.complex128)

    def set_state(self, keys, amps, t=0.0, stream=None, real=None):
        keys = np.ascontiguousarray(keys, dtype=np.uint64).reshape(-1)
        amps = np.ascontiguousarray(np.asarray(amps, dtype=np.complex128)).view(np.float64)
        n = len(keys) // self.model.W
        rp = None
        if real is not None:
            real = np.ascontiguousarray(real, dtype=np.int32)
            rp = _p(real, C.c_int32)
        _check(lib().paces_set_state(self.h, C.c_int64(n), _p(keys, C.c_uint64),
                                     _p(amps, C.c_double), rp, C.c_double(t),
                                     _stream(stream)))

    def get_set(self, which, rnd=0, stream=None, with_real=False):
        n = C.c_int64()
        _check(lib().paces_get_set(self.h, C.c_int32(which), C.c_int32(rnd),
                                   C.byref(n), None, None, _stream(stream)))
        keys = np.zeros(n.value * self.model.W, dtype=np.uint64)
        real = np.zeros(n.value, dtype=np.int32)
        _check(lib().paces_get_set(self.h, C.c_int32(which), C.c_int32(rnd),
                                   C.byref(n), _p(keys, C.c_uint64),
                                   _p(real, C.c_int32), _stream(stream)))
        keys = keys.reshape(n.value, self.model.W)
        if with_real:
            return keys, real
        return keys

    def phi(self, stream=None):
        n = self.size(stream)
        amps = np.zeros(2 * n, dtype=np.float64)
        _check(lib().paces_get_phi(self.h, _p(amps, C.c_double), _stream(stream)))
        return amps.view(np.complex128)

    def profile(self, on=True, kernels_only=False):
        """Event timing: every stage and the timed kernels, or (kernels_only)
        just the Clenshaw / Lanczos SpMV launches, timed by their own
        dispatches."""
        level = 0 if not on else (2 if kernels_only else 1)
        _check(lib().paces_profile_enable(self.h, C.c_int32(level)))

    def profile_reset(self):
        _check(lib().paces_profile_reset(self.h))

    def profile_get(self, stream=None):
        p = _Profile()
        _check(lib().paces_profile_get(self.h, C.byref(p), _stream(stream)))
        return {"ms": dict(zip(STAGES, list(p.ms))),
                "launches": dict(zip(STAGES, list(p.launches))),
                "term_bytes": p.term_bytes, "krylov_bytes": p.krylov_bytes,
                "rows_steps": p.rows_steps}

    def tuning(self):
        t = _Tuning()
        _check(lib().paces_get_tuning(self.h, C.byref(t)))
        return {"graph": t.graph, "table_shift": t.table_shift,
                "term_rows": t.term_rows, "warm": t.warm}

    def set_tuning(self, graph=None, table_shift=None, term_rows=None,
                   warm=None, stream=None):
        cur = self.tuning()
        t = _Tuning()
        t.graph = cur["graph"] if graph is None else int(graph)
        t.table_shift = cur["table_shift"] if table_shift is None else table_shift
        t.term_rows = cur["term_rows"] if term_rows is None else term_rows
        t.warm = cur["warm"] if warm is None else int(warm)
        _check(lib().paces_set_tuning(self.h, C.byref(t), _stream(stream)))

    def autotune(self, steps=3, stream=None):
        """Pick the fastest launch tuning on trial steps from the current
        state; the state is left as it was.  Returns the chosen tuning."""
        t = _Tuning()
        _check(lib().paces_autotune(self.h, C.c_int32(steps), C.byref(t),
                                    _stream(stream)))
        return {"graph": t.graph, "table_shift": t.table_shift,
                "term_rows": t.term_rows, "warm": t.warm}

    # ---- adjoint gradient (Form (3)) ----
    def adjoint_forward(self, steps, ckpt_every=50, stream=None):
        """Run `steps` steps from a new sim keeping what the adjoint needs;
        returns a[s] = <psi0|psi_s>, s = 0..steps (complex128)."""
        a = np.zeros(2 * (steps + 1), dtype=np.float64)
        _check(lib().paces_adjoint_forward(self.h, C.c_int64(steps),
                                           C.c_int32(ckpt_every),
                                           _p(a, C.c_double), _stream(stream)))
        self._adj_steps = steps
        return a.view(np.complex128)

    def adjoint_forward_dev(self, steps, out, ckpt_every=50, stream=None):
        """As adjoint_forward, writing a into `out` (a contiguous
        complex128 device tensor of steps + 1 entries)."""
        if out.dtype != torch.complex128 or not out.is_cuda or \
                not out.is_contiguous() or out.numel() != steps + 1:
            raise ValueError("out must be a contiguous complex128 cuda tensor "
                             "of steps + 1 entries")
        _check(lib().paces_adjoint_forward_dev(
            self.h, C.c_int64(steps), C.c_int32(ckpt_every),
            C.c_void_p(out.data_ptr()), _stream(stream)))
        self._adj_steps = steps
        return out

    def adjoint_backward_dev(self, gbar, out, stream=None):
        """As adjoint_backward with gbar (complex128 cuda tensor) and the
        gradient `out` (float64 cuda tensor of n_params entries) on the
        device."""
        if gbar.dtype != torch.complex128 or not gbar.is_cuda or \
                not gbar.is_contiguous() or gbar.numel() != self._adj_steps + 1:
            raise ValueError("gbar must be a contiguous complex128 cuda tensor "
                             "with one entry per recorded a_s")
        if out.dtype != torch.float64 or not out.is_cuda or \
                not out.is_contiguous() or out.numel() != self.model.n_params:
            raise ValueError("out must be a contiguous float64 cuda tensor of "
                             "n_params entries")
        _check(lib().paces_adjoint_backward_dev(
            self.h, C.c_void_p(gbar.data_ptr()), C.c_void_p(out.data_ptr()),
            _stream(stream)))
        return out

    def adjoint_replay(self, model=None, stream=None):
        """a[s] of the recorded run replayed on its frozen sets with
        `model` (default: the sim's own)."""
        a = np.zeros(2 * (self._adj_steps + 1), dtype=np.float64)
        _check(lib().paces_adjoint_replay(self.h, model.h if model else None,
                                          _p(a, C.c_double), _stream(stream)))
        return a.view(np.complex128)

    def adjoint_backward(self, gbar, stream=None):
        """dL/dtheta (theta = J per axis, g and omega per mode, eps per
        site) for gbar[s] = dL/d conj(a_s)."""
        gb = np.ascontiguousarray(np.asarray(gbar, dtype=np.complex128)).view(np.float64)
        if len(gb) != 2 * (self._adj_steps + 1):
            raise ValueError("gbar needs one entry per recorded a_s")
        g = np.zeros(self.model.n_params, dtype=np.float64)
        _check(lib().paces_adjoint_backward(self.h, _p(gb, C.c_double),
                                            _p(g, C.c_double), _stream(stream)))
        return g


def profile_mark(tag=0, stream=None):
    """One empty kernel dispatch (k_mark) on the stream, a marker for
    kernel traces and counter runs."""
    _check(lib().paces_profile_mark(C.c_int32(tag), _stream(stream)))


def taylor_theta(m):
    """Backward-error threshold theta_m of the degree-m Taylor series (the
    Taylor propagator's degree choice); -1 outside 1..55."""
    return lib().paces_taylor_theta(C.c_int32(m))


def theta_of(params):
    """theta = (J per axis, g per mode, omega per mode, eps per site)."""
    nd, V = params["ndim"], params["n_modes"]
    return np.array(list(params["J"][:nd]) + list(params["g"][:V])
                    + list(params["omega"][:V]) + list(params["eps"]),
                    dtype=np.float64)


def params_with_theta(params, theta):
    """Copy of the model parameters with theta substituted."""
    nd, V = params["ndim"], params["n_modes"]
    t = [float(x) for x in theta]
    p = dict(params)
    p["J"] = t[:nd] + list(params["J"][nd:])
    p["g"] = t[nd:nd + V] + list(params["g"][V:])
    p["omega"] = t[nd + V:nd + 2 * V] + list(params["omega"][V:])
    p["eps"] = t[nd + 2 * V:]
    return p


if torch is not None:
    class AutocorrFn(torch.autograd.Function):
        """a = AutocorrFn.apply(theta, params, run, init, steps, ckpt_every):
        the autocorrelation a_s = <psi0|psi_s>, s = 0..steps (complex128 on
        the current GPU), of a run with model parameters theta (float64
        [P]: J per axis, g and omega per mode, eps per site).  Backward is
        the adjoint gradient on the forward run's frozen sets; a, the
        incoming gradient and dL/dtheta stay in device memory (the
        gradient is returned on theta's device).  The model tables are
        built on the host from theta's values."""

        @staticmethod
        def forward(ctx, theta, params, run, init, steps, ckpt_every=50):
            p = params_with_theta(params, theta.detach().cpu().numpy())
            model = Model(p)
            exc, occ, coef = init
            sim = Sim(model, run, exc, occ, coef)
            a = torch.empty(steps + 1, dtype=torch.complex128, device="cuda")
            sim.adjoint_forward_dev(steps, a, ckpt_every)
            ctx.sim, ctx.model, ctx.theta_device = sim, model, theta.device
            return a

        @staticmethod
        def backward(ctx, grad_a):
            # torch passes 2 dL/d conj(a) for a complex output
            gbar = (grad_a.detach().to(device="cuda", dtype=torch.complex128)
                    / 2).contiguous()
            g = torch.empty(ctx.model.n_params, dtype=torch.float64,
                            device="cuda")
            ctx.sim.adjoint_backward_dev(gbar, g)
            return (g.to(ctx.theta_device), None, None, None, None, None)
