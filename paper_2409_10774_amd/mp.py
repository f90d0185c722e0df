"""Python binding of the C ABI in include/mp.h (argument marshalling only).

Every step of the solver runs in the HIP library `_lib/libmp.so`; PyTorch
supplies device memory (the plan's workspace) and the stream.  Importing this
module fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
# PyTorch ships its own HIP runtime; loading it before the library makes the
# library bind to that same runtime, so torch's device pointers and streams
# are valid inside it (two runtimes in one process would not share devices).
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
# MP_LIB selects another build of the same library (e.g. an A/B variant)
LIB_PATH = os.environ.get("MP_LIB") or os.path.join(HERE, "_lib", "libmp.so")

MP_OK, MP_E_INVALID, MP_E_NOMEM, MP_E_DEVICE, MP_E_NOT_CONVERGED, MP_E_DIVERGED, MP_E_STATE = range(7)
STATUS_NAMES = {0: "MP_OK", 1: "MP_E_INVALID", 2: "MP_E_NOMEM", 3: "MP_E_DEVICE",
                4: "MP_E_NOT_CONVERGED", 5: "MP_E_DIVERGED", 6: "MP_E_STATE"}
MP_FP64, MP_MIXED = 0, 1
MP_ERR_LOCAL, MP_ERR_AVERAGE = 0, 1
MP_REF_PHASE_MEAN, MP_REF_VOLUME_MEAN, MP_REF_EXPLICIT, MP_REF_TENSOR_MEAN, MP_REF_TENSOR_PHASE_MEAN, \
    MP_REF_GEOMETRIC_MEAN = range(6)
MP_SCHEME_BASIC, MP_SCHEME_AL = 0, 1
MP_GREEN_COMPUTED, MP_GREEN_STORED = 0, 1
FIELDS = {"e": 0, "g": 1, "t": 2, "m": 3, "p": 4, "q": 5}


class mp_phase(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("lam", "mu", "kappa", "alpha", "beta", "gamma",
                                          "tY", "tH", "mY", "mH", "a1", "b1")]


class mp_aniso(C.Structure):
    _fields_ = [("phase", C.c_int32), ("A", C.c_double * 81), ("B", C.c_double * 81)]


class mp_problem(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("h", C.c_double), ("phase", C.POINTER(C.c_uint8)),
                ("n_phases", C.c_int32), ("phases", C.POINTER(mp_phase)), ("ref_mode", C.c_int32),
                ("ref", mp_phase), ("tol", C.c_double), ("max_iter", C.c_int32),
                ("err_norm", C.c_int32), ("precision", C.c_int32), ("n_aniso", C.c_int32),
                ("aniso", C.POINTER(mp_aniso)), ("scheme", C.c_int32), ("relax", C.c_double),
                ("green_mode", C.c_int32)]


class mp_batch_config(C.Structure):
    _fields_ = [("precision", C.c_int32), ("n_shapes", C.c_int32), ("shapes", (C.c_int32 * 3) * 8),
                ("max_rves", C.c_int32), ("iters_per_launch", C.c_int32), ("autotune", C.c_int32)]


class mp_request(C.Structure):
    _fields_ = [("arrival", C.c_double), ("prob", C.POINTER(mp_problem)), ("n_steps", C.c_int32),
                ("times", C.POINTER(C.c_double)), ("E", C.POINTER(C.c_double)),
                ("Gam", C.POINTER(C.c_double)), ("records", C.POINTER(C.c_double)),
                ("field_mask", C.c_uint32), ("fields", C.c_void_p * 6), ("fields_on_device", C.c_int32)]


MP_RVE_RUNNING, MP_RVE_DONE = 0, 1


class MPError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} is missing "
                          "(run __graft_entry__.build())")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
    sig = {
        "mp_plan_workspace_size": (C.c_int, [C.POINTER(mp_problem), C.POINTER(C.c_size_t)]),
        "mp_plan_create": (C.c_int, [C.POINTER(mp_problem), vp, C.c_size_t, vp, C.POINTER(vp)]),
        "mp_solve_load_path": (C.c_int, [vp, i32, dp, dp, dp, C.POINTER(i32)]),
        "mp_homogenized_response": (C.c_int, [vp, i32, dp]),
        "mp_get_fields": (C.c_int, [vp, C.c_uint32, C.POINTER(vp), i32]),
        "mp_step_error_parts": (C.c_int, [vp, i32, dp]),
        "mp_set_fixed_iterations": (C.c_int, [vp, i32]),
        "mp_set_eigenstress": (C.c_int, [vp, vp]),
        "mp_plan_steps": (C.c_int, [vp, C.POINTER(i32)]),
        "mp_green_apply": (C.c_int, [vp, vp, vp]),
        "mp_green_apply_noalloc": (C.c_int, [C.POINTER(i32), C.c_double, dp, vp, vp, vp]),
        "mp_spectrum_forward": (C.c_int, [vp, vp, vp]),
        "mp_radial_return": (C.c_int, [vp, i64] + [vp] * 13),
        "mp_profile": (C.c_int, [vp, i32]),
        "mp_profile_read": (C.c_int, [vp, i32, dp, C.POINTER(C.c_int64)]),
        "mp_plan_destroy": (None, [vp]),
        "mp_batch_footprint": (C.c_int, [C.POINTER(mp_batch_config), C.POINTER(mp_problem), i32,
                                         C.POINTER(C.c_size_t)]),
        "mp_batch_create": (C.c_int, [C.POINTER(mp_batch_config), vp, C.c_size_t, vp, C.POINTER(vp)]),
        "mp_batch_admit": (C.c_int, [vp, C.POINTER(mp_problem), i32, dp, dp, dp, C.POINTER(i32)]),
        "mp_batch_run": (C.c_int, [vp, C.POINTER(i32)]),
        "mp_batch_drain": (C.c_int, [vp, i32, C.POINTER(i32)]),
        "mp_batch_query": (C.c_int, [vp, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32),
                                     C.POINTER(i64)]),
        "mp_batch_response": (C.c_int, [vp, i32, i32, dp]),
        "mp_batch_get_fields": (C.c_int, [vp, i32, C.c_uint32, C.POINTER(vp), i32]),
        "mp_batch_release": (C.c_int, [vp, i32]),
        "mp_batch_set_fixed_iterations": (C.c_int, [vp, i32, i32]),
        "mp_batch_schedule": (C.c_int, [vp, i32, C.POINTER(i32), C.POINTER(C.c_float)]),
        "mp_batch_stats": (C.c_int, [vp, C.POINTER(i64), C.POINTER(C.c_size_t), C.POINTER(i32)]),
        "mp_batch_destroy": (None, [vp]),
        "mp_serve_batched": (C.c_int, [vp, i32, C.POINTER(mp_request), i32, C.c_double, dp, dp,
                                       C.POINTER(i32), C.POINTER(i64)]),
        "mp_serve_sequential": (C.c_int, [i32, C.POINTER(mp_request), vp, C.c_size_t, vp, C.c_double,
                                          dp, dp, C.POINTER(i32), C.POINTER(i64)]),
        "mp_last_error": (C.c_char_p, []),
        "mp_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def check(status):
    if status != MP_OK:
        raise MPError(status, lib.mp_last_error().decode())
    return status


def _phase_struct(p) -> mp_phase:
    if hasattr(p, "as_tuple"):
        vals = p.as_tuple()
    elif isinstance(p, dict):
        vals = tuple(p[k] for k in ("lam", "mu", "kappa", "alpha", "beta", "gamma",
                                    "tY", "tH", "mY", "mH", "a1", "b1"))
    else:
        vals = tuple(p)
    return mp_phase(*[float(v) for v in vals])


def make_problem(phase_map, phases, h=1.0, tol=1e-8, max_iter=20000, err_norm="local",
                 ref_mode="phase_mean", ref=None, precision="fp64", scheme="basic", relax=1.7,
                 green="computed"):
    """Build an mp_problem (and keep its host arrays alive on the returned object)."""
    pm = np.ascontiguousarray(phase_map, dtype=np.uint8)
    if pm.ndim != 3:
        raise ValueError("phase_map must be (n2, n1, n0)")
    n2, n1, n0 = pm.shape
    arr = (mp_phase * len(phases))(*[_phase_struct(p) for p in phases])
    prob = mp_problem()
    prob.n[0], prob.n[1], prob.n[2] = n0, n1, n2
    prob.h = float(h)
    prob.phase = pm.ctypes.data_as(C.POINTER(C.c_uint8))
    prob.n_phases = len(phases)
    prob.phases = C.cast(arr, C.POINTER(mp_phase))
    prob.ref_mode = {"phase_mean": MP_REF_PHASE_MEAN, "volume_mean": MP_REF_VOLUME_MEAN,
                     "explicit": MP_REF_EXPLICIT, "tensor_mean": MP_REF_TENSOR_MEAN,
                     "tensor_phase_mean": MP_REF_TENSOR_PHASE_MEAN,
                     "geometric_mean": MP_REF_GEOMETRIC_MEAN}[ref_mode]
    if ref is not None:
        prob.ref = mp_phase(*(list(float(v) for v in ref) + [0.0] * (12 - len(ref))))
    prob.tol = float(tol)
    prob.max_iter = int(max_iter)
    prob.err_norm = {"local": MP_ERR_LOCAL, "average": MP_ERR_AVERAGE}[err_norm]
    prob.precision = {"fp64": MP_FP64, "mixed": MP_MIXED}[precision]
    prob.scheme = {"basic": MP_SCHEME_BASIC, "al": MP_SCHEME_AL}[scheme]
    prob.relax = float(relax)
    prob.green_mode = {"computed": MP_GREEN_COMPUTED, "stored": MP_GREEN_STORED}[green]
    # phases carrying general Eq. 5 tensors: A[k, l, m, n] = A_klmn and
    # B[l, k, m, n] = B_lkmn, flattened in that index order
    tens = [(i, p) for i, p in enumerate(phases) if getattr(p, "A", None) is not None]
    recs = (mp_aniso * max(len(tens), 1))()
    for j, (i, p) in enumerate(tens):
        recs[j].phase = i
        recs[j].A[:] = [float(v) for v in np.asarray(p.A, np.float64).reshape(81)]
        recs[j].B[:] = [float(v) for v in np.asarray(p.B, np.float64).reshape(81)]
    prob.n_aniso = len(tens)
    prob.aniso = C.cast(recs, C.POINTER(mp_aniso))
    prob._keep = (pm, arr, recs)
    return prob


def mp_plan_workspace_size(prob) -> int:
    n = C.c_size_t()
    check(lib.mp_plan_workspace_size(C.byref(prob), C.byref(n)))
    return n.value


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class Plan:
    """One solver plan on a GPU: owns a torch workspace, wraps the C plan."""

    def __init__(self, phase_map, phases, device="cuda:0", stream=None, **kw):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.prob = make_problem(phase_map, phases, **kw)
        pm = self.prob._keep[0]
        self.shape = pm.shape
        self.nvox = int(pm.size)
        nbytes = mp_plan_workspace_size(self.prob)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        check(lib.mp_plan_create(C.byref(self.prob), _ptr(self.workspace), nbytes,
                                 C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.handle = h

    # -- Alg. 2 -------------------------------------------------------------
    def solve(self, times, E, G, raise_on_error=True):
        times = np.ascontiguousarray(times, dtype=np.float64)
        S = len(times) - 1
        E = np.ascontiguousarray(np.asarray(E, np.float64).reshape(S, 9))
        G = np.ascontiguousarray(np.asarray(G, np.float64).reshape(S, 9))
        it = (C.c_int32 * max(S, 1))()
        dp = C.POINTER(C.c_double)
        st = lib.mp_solve_load_path(self.handle, S, times.ctypes.data_as(dp), E.ctypes.data_as(dp),
                                    G.ctypes.data_as(dp), it)
        iters = [int(it[i]) for i in range(S)]
        if raise_on_error:
            check(st)
            return iters
        return st, iters

    def steps(self):
        n = C.c_int32()
        check(lib.mp_plan_steps(self.handle, C.byref(n)))
        return n.value

    def response(self, step):
        out = (C.c_double * 42)()
        check(lib.mp_homogenized_response(self.handle, int(step), out))
        return np.array(out[:])

    def error_parts(self, step):
        """(err_e, err_t, err_gamma, err_m, 0) of a committed step."""
        out = (C.c_double * 5)()
        check(lib.mp_step_error_parts(self.handle, int(step), out))
        return np.array(out[:])

    def responses(self):
        n = self.steps()
        return np.array([self.response(s) for s in range(1, n + 1)]).reshape(n, 42)

    def field(self, name):
        return self.fields((name,))[name]

    def fields(self, names=FIELDS, device=False):
        """{name: FP64 array} of the committed state (mp_get_fields): numpy
        arrays, or torch tensors on the plan's device when device=True."""
        return _read_fields(lambda mask, dst, dev: lib.mp_get_fields(self.handle, mask, dst, dev),
                            self.shape, names, device, self.device)

    def set_fixed_iterations(self, n):
        check(lib.mp_set_fixed_iterations(self.handle, int(n)))

    def set_eigenstress(self, tm=None):
        """Eigenstress subtracted in every later polarization (mp_set_eigenstress):
        tm (18, n2, n1, n0) host array, tau_m then mu_m with component 3k + l,
        or None to clear.  The plan holds the device copy."""
        if tm is None:
            check(lib.mp_set_eigenstress(self.handle, None))
            self._eig = None
            return
        dt = self.torch.float64 if self.prob.precision == MP_FP64 else self.torch.float32
        a = np.ascontiguousarray(np.asarray(tm, np.float64).reshape((18,) + self.shape))
        t = self.torch.from_numpy(a).to(device=self.device, dtype=dt)
        self.torch.cuda.synchronize(self.device)
        check(lib.mp_set_eigenstress(self.handle, C.c_void_p(t.data_ptr())))
        self._eig = t

    # -- single steps of the hot path ---------------------------------------
    def green_apply(self, tau_mu):
        """tau_mu: torch float64 (18, n2, n1, n0) on the plan's device."""
        x = tau_mu.contiguous()
        assert x.dtype == self.torch.float64 and x.numel() == 18 * self.nvox and x.device == self.device
        out = self.torch.empty_like(x)
        check(lib.mp_green_apply(self.handle, _ptr(x), _ptr(out)))
        return out

    def spectrum_forward(self, fields):
        x = fields.contiguous()
        assert x.dtype == self.torch.float64 and x.numel() == 18 * self.nvox and x.device == self.device
        n2, n1, n0 = self.shape
        out = self.torch.empty((n2, n1, n0 // 2, 18, 2), dtype=self.torch.float64, device=self.device)
        check(lib.mp_spectrum_forward(self.handle, _ptr(x), _ptr(out)))
        return self.torch.view_as_complex(out)   # [kz][ky][kx][c]

    def radial_return(self, phase, e, g, e_n, g_n, t_n, m_n, p_n, q_n):
        """Alg. 1 on n independent points; tensors on the plan's device, float64
        (9, n) / (n,), phase uint8 (n,).  Returns (t, m, p, q)."""
        T = self.torch
        n = phase.numel()
        ins = [x.contiguous() for x in (e, g, e_n, g_n, t_n, m_n, p_n, q_n)]
        for x in ins:
            assert x.dtype == T.float64 and x.device == self.device
        ph = phase.contiguous()
        assert ph.dtype == T.uint8 and ph.device == self.device
        t = T.empty((9, n), dtype=T.float64, device=self.device)
        m = T.empty_like(t)
        p = T.empty(n, dtype=T.float64, device=self.device)
        q = T.empty_like(p)
        check(lib.mp_radial_return(self.handle, n, _ptr(ph), *[_ptr(x) for x in ins],
                                   _ptr(t), _ptr(m), _ptr(p), _ptr(q)))
        return t, m, p, q

    KERNELS = ("y_fwd", "z_green", "y_inv", "x_pass", "err_reduce")

    def profile(self, enable=True):
        """True / 1: events between all loop kernels; 2: around the x pass
        only; False / 0: off (mp_profile)."""
        mode = 1 if enable is True else 0 if enable is False else int(enable)
        check(lib.mp_profile(self.handle, mode))

    def profile_read(self):
        """{kernel: (total ms, launches)} accumulated since profile(True)."""
        k = len(self.KERNELS)
        ms = (C.c_double * k)()
        n = (C.c_int64 * k)()
        check(lib.mp_profile_read(self.handle, k, ms, n))
        return {k: (ms[i], n[i]) for i, k in enumerate(self.KERNELS)}

    def close(self):
        if getattr(self, "handle", None):
            lib.mp_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _read_fields(call, shape, names, device, dev):
    """Marshal a field read-back through `call(mask, dst, dst_is_device)`."""
    nvox = int(np.prod(shape))
    dst = (C.c_void_p * 6)()
    out, mask = {}, 0
    for name in names:
        f = FIELDS[name]
        full = (9,) + tuple(shape) if name in ("e", "g", "t", "m") else tuple(shape)
        if device:
            import torch
            a = torch.empty(full, dtype=torch.float64, device=dev)
            dst[f] = a.data_ptr()
        else:
            a = np.empty(full, np.float64)
            dst[f] = a.ctypes.data
        out[name] = a
        mask |= 1 << f
    check(call(mask, dst, 1 if device else 0))
    if device:
        import torch
        torch.cuda.current_stream(dev).synchronize()
    return out


def _path(times, E, G):
    times = np.ascontiguousarray(times, dtype=np.float64)
    S = len(times) - 1
    E = np.ascontiguousarray(np.asarray(E, np.float64).reshape(S, 9))
    G = np.ascontiguousarray(np.asarray(G, np.float64).reshape(S, 9))
    return S, times, E, G


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def batch_config(shapes, precision="mixed", max_rves=64, iters_per_launch=8, autotune=True):
    cfg = mp_batch_config()
    cfg.precision = {"fp64": MP_FP64, "mixed": MP_MIXED}[precision]
    cfg.n_shapes = len(shapes)
    for i, s in enumerate(shapes):
        for j in range(3):
            cfg.shapes[i][j] = int(s[j])
    cfg.max_rves = int(max_rves)
    cfg.iters_per_launch = int(iters_per_launch)
    cfg.autotune = 1 if autotune else 0
    return cfg


class Batch:
    """A resident batch of RVEs on one GPU (mp_batch_*): owns a torch arena."""

    def __init__(self, shapes, arena_bytes, precision="mixed", max_rves=64, iters_per_launch=8,
                 autotune=True, device="cuda:0", stream=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.precision = precision
        self.cfg = batch_config(shapes, precision, max_rves, iters_per_launch, autotune)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        check(lib.mp_batch_create(C.byref(self.cfg), _ptr(self.arena), int(arena_bytes),
                                  C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.handle = h
        self._shape = {}

    def footprint(self, phase_map, phases, n_steps, **kw):
        prob = make_problem(phase_map, phases, precision=self.precision, **kw)
        n = C.c_size_t()
        check(lib.mp_batch_footprint(C.byref(self.cfg), C.byref(prob), int(n_steps), C.byref(n)))
        return n.value

    def admit(self, phase_map, phases, times, E, G, raise_on_error=True, **kw):
        """Admit one RVE with its load path; returns its id (or a status when
        raise_on_error is False and admission fails)."""
        prob = make_problem(phase_map, phases, precision=self.precision, **kw)
        S, times, E, G = _path(times, E, G)
        i = C.c_int32()
        st = lib.mp_batch_admit(self.handle, C.byref(prob), S, _dp(times), _dp(E), _dp(G), C.byref(i))
        if st != MP_OK:
            if raise_on_error:
                check(st)
            return None, st
        self._shape[i.value] = prob._keep[0].shape
        return (i.value, MP_OK) if not raise_on_error else i.value

    def run(self):
        a = C.c_int32()
        check(lib.mp_batch_run(self.handle, C.byref(a)))
        return a.value

    def drain(self, max_launches=0):
        n = C.c_int32()
        check(lib.mp_batch_drain(self.handle, int(max_launches), C.byref(n)))
        return n.value

    def query(self, rid):
        """(state, status, steps_done, iterations)"""
        st, sc, sd = C.c_int32(), C.c_int32(), C.c_int32()
        it = C.c_int64()
        check(lib.mp_batch_query(self.handle, int(rid), C.byref(st), C.byref(sc), C.byref(sd),
                                 C.byref(it)))
        return st.value, sc.value, sd.value, it.value

    def record(self, rid, step):
        out = (C.c_double * 48)()
        check(lib.mp_batch_response(self.handle, int(rid), int(step), out))
        return np.array(out[:])

    def responses(self, rid):
        """[steps, 47]: response (42) then error parts and a reserved 0 (5)"""
        n = self.query(rid)[2]
        return np.array([self.record(rid, s)[:47] for s in range(1, n + 1)]).reshape(n, 47)

    def field(self, rid, name):
        return self.fields(rid, (name,))[name]

    def fields(self, rid, names=FIELDS, device=False):
        """{name: FP64 array} of RVE rid's committed state (mp_batch_get_fields)."""
        return _read_fields(lambda mask, dst, dev: lib.mp_batch_get_fields(self.handle, int(rid), mask, dst, dev),
                            self._shape[rid], names, device, self.device)

    def set_fixed_iterations(self, rid, n):
        check(lib.mp_batch_set_fixed_iterations(self.handle, int(rid), int(n)))

    def release(self, rid):
        check(lib.mp_batch_release(self.handle, int(rid)))
        self._shape.pop(rid, None)

    def schedule(self, cls):
        out = (C.c_int32 * 8)()
        ms = (C.c_float * 3)()
        check(lib.mp_batch_schedule(self.handle, int(cls), out, ms))
        o = list(out)
        return {"y_fwd": {"tx": o[0], "grid": o[1], "ms": ms[0]},
                "z_green": {"tx": o[2], "grid": o[3], "ms": ms[1]},
                "y_inv": {"tx": o[4], "grid": o[5], "ms": ms[2]},
                "x_grid": o[6], "x_tiles": o[7]}

    def stats(self):
        g, r = C.c_int64(), C.c_int32()
        u = C.c_size_t()
        check(lib.mp_batch_stats(self.handle, C.byref(g), C.byref(u), C.byref(r)))
        return {"graph_launches": g.value, "arena_used": u.value, "resident": r.value}

    def close(self):
        if getattr(self, "handle", None):
            lib.mp_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Requests:
    """Marshalled request trace: items (arrival, phase_map, phases, times, E, G, kw).

    The replies land in self.records[i] ([n_steps, 48] host array, when
    records=True) and self.fields[i] ({name: array} for the names in
    `fields`; torch tensors on `device` when given, else numpy arrays)."""

    def __init__(self, items, precision="mixed", records=True, fields=(), device=None):
        self.arr = (mp_request * max(1, len(items)))()
        self._keep = []
        self.records, self.fields = [], []
        for i, (arrival, pm, phases, times, E, G, kw) in enumerate(items):
            prob = make_problem(pm, phases, precision=precision, **kw)
            S, times, E, G = _path(times, E, G)
            self._keep.append((prob, times, E, G))
            r = self.arr[i]
            r.arrival = float(arrival)
            r.prob = C.pointer(prob)
            r.n_steps = S
            r.times, r.E, r.Gam = _dp(times), _dp(E), _dp(G)
            rec = np.full((S, 48), np.nan) if records else None
            self.records.append(rec)
            r.records = _dp(rec) if records else C.POINTER(C.c_double)()
            out, mask = {}, 0
            shape = np.asarray(pm).shape
            for name in fields:
                f = FIELDS[name]
                full = (9,) + tuple(shape) if name in ("e", "g", "t", "m") else tuple(shape)
                if device is not None:
                    import torch
                    a = torch.full(full, float("nan"), dtype=torch.float64, device=device)
                    r.fields[f] = a.data_ptr()
                else:
                    a = np.full(full, np.nan)
                    r.fields[f] = a.ctypes.data
                out[name] = a
                mask |= 1 << f
            r.field_mask = mask
            r.fields_on_device = 1 if device is not None else 0
            self.fields.append(out)
        self.n = len(items)


def _serve_out(n):
    return (C.c_double * max(1, n))(), (C.c_double * max(1, n))(), (C.c_int32 * max(1, n))(), \
        (C.c_int64 * max(1, n))()


def serve_batched(batch, reqs, max_bypass=16, progress_s=0.0):
    """Continuous batching of a request trace on an empty Batch; returns per
    request (t_admit, t_done, status, iterations) as numpy arrays."""
    a, d, st, it = _serve_out(reqs.n)
    check(lib.mp_serve_batched(batch.handle, reqs.n, reqs.arr, int(max_bypass), float(progress_s),
                               a, d, st, it))
    n = reqs.n
    return np.array(a[:n]), np.array(d[:n]), np.array(st[:n]), np.array(it[:n])


def serve_sequential(reqs, workspace, stream=None, progress_s=0.0):
    """The trace served one request at a time with FP64 plans on `workspace`
    (a torch uint8 device tensor)."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream(workspace.device)
    a, d, st, it = _serve_out(reqs.n)
    check(lib.mp_serve_sequential(reqs.n, reqs.arr, _ptr(workspace), workspace.numel(),
                                  C.c_void_p(s.cuda_stream), float(progress_s), a, d, st, it))
    n = reqs.n
    return np.array(a[:n]), np.array(d[:n]), np.array(st[:n]), np.array(it[:n])


def green_apply_noalloc(n, h, ref, tau_mu, out=None, stream=None):
    """mp_green_apply_noalloc: the spectral step of one iteration on 18 FP64
    fields without a plan (the library's static scratch, nothing allocated
    by the call).  n = (n0, n1, n2); ref = six Eq. 6 constants of the
    reference medium; tau_mu, out: torch float64 (18, n2, n1, n0) on the
    current device.  Returns `out` (allocated here when not given)."""
    import torch
    x = tau_mu
    assert x.dtype == torch.float64 and x.is_contiguous() and x.numel() == 18 * int(np.prod(n))
    if out is None:
        out = torch.empty_like(x)
    nn = (C.c_int32 * 3)(*[int(v) for v in n])
    rr = (C.c_double * 6)(*[float(v) for v in ref])
    s = stream if stream is not None else torch.cuda.current_stream(x.device)
    check(lib.mp_green_apply_noalloc(nn, float(h), rr, _ptr(x), _ptr(out), C.c_void_p(s.cuda_stream)))
    return out


mp_version = lambda: lib.mp_version().decode()
