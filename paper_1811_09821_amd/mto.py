"""Thin ctypes binding of libmto.so (include/mto.h).

Argument marshalling only: every step of the FEA + sensitivity path runs in
the HIP kernels of the library.  PyTorch supplies device memory and the
current HIP stream.  There is no CPU fallback: if the library is missing the
import of this module fails.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmto.so")

MTO_OK, MTO_EINVAL, MTO_ESINGULAR, MTO_ENOCONV, MTO_EBREAKDOWN, MTO_EHIP, MTO_ENOMEM = 0, -1, -2, -3, -4, -5, -6
MTO_MAX_P, MTO_MAX_D = 4, 8  # as in mto.h
PATH_MFMA, PATH_PLAIN = 0, 1
PRECOND_JACOBI, PRECOND_MG, PRECOND_MG_ASM = 0, 1, 2
ERROR_NAMES = {MTO_EINVAL: "MTO_EINVAL", MTO_ESINGULAR: "MTO_ESINGULAR", MTO_ENOCONV: "MTO_ENOCONV",
               MTO_EBREAKDOWN: "MTO_EBREAKDOWN", MTO_EHIP: "MTO_EHIP", MTO_ENOMEM: "MTO_ENOMEM"}


class MtoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class _Mesh(ctypes.Structure):
    _fields_ = [("nelx", ctypes.c_int32), ("nely", ctypes.c_int32),
                ("p", ctypes.POINTER(ctypes.c_int8)), ("d", ctypes.POINTER(ctypes.c_int8))]


class _Support(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("a", ctypes.c_int32), ("b", ctypes.c_int32),
                ("comp_mask", ctypes.c_int32)]


class _Load(ctypes.Structure):
    _fields_ = [("vx", ctypes.c_int32), ("vy", ctypes.c_int32), ("fx", ctypes.c_double),
                ("fy", ctypes.c_double), ("load_case", ctypes.c_int32)]


class _Params(ctypes.Structure):
    _fields_ = [("E0", ctypes.c_double), ("Emin", ctypes.c_double), ("nu", ctypes.c_double),
                ("q", ctypes.c_double), ("rtol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("kernel_path", ctypes.c_int32), ("iters_per_launch", ctypes.c_int32),
                ("max_restarts", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("mg_omega", ctypes.c_double), ("mg_coarse_max", ctypes.c_int32),
                ("stored_matrices", ctypes.c_int32)]


class _Spring(ctypes.Structure):
    _fields_ = [("vx", ctypes.c_int32), ("vy", ctypes.c_int32), ("comp", ctypes.c_int32), ("k", ctypes.c_double)]


class _DpParams(ctypes.Structure):
    _fields_ = [("frac_a_refine", ctypes.c_double), ("frac_a_coarsen", ctypes.c_double),
                ("frac_d_refine", ctypes.c_double), ("frac_d_coarsen", ctypes.c_double),
                ("p_max", ctypes.c_int32), ("d_max", ctypes.c_int32)]


class _Problem(ctypes.Structure):
    _fields_ = [("mesh", _Mesh), ("supports", ctypes.POINTER(_Support)), ("n_supports", ctypes.c_int32),
                ("loads", ctypes.POINTER(_Load)), ("n_loads", ctypes.c_int32),
                ("n_load_cases", ctypes.c_int32), ("springs", ctypes.POINTER(_Spring)),
                ("n_springs", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_systems", ctypes.c_int32), ("max_iterations", ctypes.c_int32),
                ("restarts", ctypes.c_int32), ("iterations", ctypes.POINTER(ctypes.c_int32)),
                ("true_rel_residual", ctypes.POINTER(ctypes.c_double)), ("solve_ms", ctypes.c_double)]


class _Info(ctypes.Structure):
    _fields_ = [("n_instances", ctypes.c_int32), ("n_systems", ctypes.c_int32), ("n_groups", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("n_cells", ctypes.c_int64), ("n_u", ctypes.c_int64),
                ("n_g", ctypes.c_int64), ("n_free_total", ctypes.c_int64), ("n_elements", ctypes.c_int64),
                ("flops_per_matvec", ctypes.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run paper_1811_09821_amd.build.build()")
    # The library and torch must share one HIP runtime in the process.  torch
    # ships its own libamdhip64 with the same soname as the system one the
    # library links against, plus its own HSA runtime; loading torch first
    # makes the dynamic loader bind the library to torch's HIP runtime.  The
    # other order mixes two HSA runtimes, and the library then finds no device.
    import torch  # noqa: F401

    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64p = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)
    sig = {
        "mto_last_error": ([], ctypes.c_char_p),
        "mto_version": ([], ctypes.c_char_p),
        "mto_plan_create": ([ctypes.POINTER(_Problem), ctypes.POINTER(_Params), ctypes.POINTER(vp)], i32),
        "mto_batch_plan_create": ([ctypes.POINTER(_Problem), i32, ctypes.POINTER(_Params), ctypes.POINTER(vp)],
                                  i32),
        "mto_plan_info": ([vp, ctypes.POINTER(_Info)], i32),
        "mto_instance_info": ([vp, i32, i64p, i64p, i64p, i64p, i64p, i64p, i64p, ctypes.POINTER(i32)], i32),
        "mto_solve": ([vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(_Stats)], i32),
        "mto_batch_capture": ([vp, vp, vp, vp, vp, vp], i32),
        "mto_batch_replay": ([vp, vp, ctypes.POINTER(_Stats)], i32),
        "mto_apply_stiffness": ([vp, vp, vp, vp, vp], i32),
        "mto_apply_stiffness_noalloc": ([vp, vp, vp, vp, vp], i32),
        "mto_sensitivity": ([vp, vp, vp, vp, vp], i32),
        "mto_jacobi_diagonal": ([vp, vp, vp, vp], i32),
        "mto_weighted_sensitivity": ([vp, vp, vp, vp, vp], i32),
        "mto_autotune": ([vp, vp, ctypes.c_char_p, vp, ctypes.c_char_p, i32], i32),
        "mto_set_tile": ([vp, i32, i32, i32, i32], i32),
        "mto_time_contraction": ([vp, vp, i32, i32, vp, ctypes.POINTER(ctypes.c_double)], i32),
        "mto_plan_destroy": ([vp], None),
        "mto_qr_error": ([vp, vp, vp, vp, vp], i32),
        "mto_adjoint_sensitivity": ([vp, vp, vp, vp, vp, vp], i32),
        "mto_kelly_indicator": ([vp, vp, vp, vp], i32),
        "mto_density_indicator": ([vp, vp, i32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, vp, vp], i32),
        "mto_dp_update": ([i32, i32, vp, vp, vp, ctypes.POINTER(_DpParams), vp, vp, vp, vp], i32),
        "mto_qr_update": ([i32, vp, vp, ctypes.c_double, i32, vp], i32),
        "mto_filter_create": ([ctypes.POINTER(_Problem), i32, ctypes.c_double, ctypes.POINTER(vp)], i32),
        "mto_filter_apply": ([vp, vp, vp, vp], i32),
        "mto_filter_grad": ([vp, vp, vp, vp], i32),
        "mto_filter_info": ([vp, i64p, i64p], i32),
        "mto_filter_destroy": ([vp], None),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()
EXPORTED = ("mto_last_error", "mto_version", "mto_plan_create", "mto_batch_plan_create", "mto_plan_info",
            "mto_instance_info", "mto_solve", "mto_batch_capture", "mto_batch_replay", "mto_apply_stiffness",
            "mto_apply_stiffness_noalloc",
            "mto_sensitivity", "mto_jacobi_diagonal", "mto_weighted_sensitivity", "mto_autotune", "mto_set_tile",
            "mto_time_contraction", "mto_plan_destroy", "mto_qr_error", "mto_adjoint_sensitivity", "mto_kelly_indicator",
            "mto_density_indicator", "mto_dp_update", "mto_qr_update", "mto_filter_create", "mto_filter_apply", "mto_filter_grad",
            "mto_filter_info", "mto_filter_destroy")


def lib():
    return _lib


def version():
    return _lib.mto_version().decode()


def _check(rc, allow=()):
    if rc != MTO_OK and rc not in allow:
        raise MtoError(rc, _lib.mto_last_error().decode())
    return rc


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _f64_cuda(t, n, name):
    import torch

    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64, got {t.dtype}")
    if not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous")
    if t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return t


def default_params(**kw):
    prm = dict(E0=1.0, Emin=1e-9, nu=0.3, q=3.0, rtol=1e-11, max_iter=0, kernel_path=PATH_MFMA,
               iters_per_launch=0, max_restarts=3, precond=PRECOND_MG_ASM,
               mg_omega=0.0, mg_coarse_max=0, stored_matrices=0)
    prm.update(kw)
    return prm


def _problem_array(problems):
    """ctypes mto_problem array for `problems` plus the host buffers it
    points into (keep them alive for the call)."""
    keep = []
    arr = (_Problem * len(problems))()
    for k, pr in enumerate(problems):
        p = np.ascontiguousarray(pr.p, dtype=np.int8)
        d = np.ascontiguousarray(pr.d, dtype=np.int8)
        sup = (_Support * max(1, len(pr.supports)))(*[_Support(*map(int, s)) for s in pr.supports])
        lds = (_Load * max(1, len(pr.loads)))(
            *[_Load(int(l[0]), int(l[1]), float(l[2]), float(l[3]), int(l[4])) for l in pr.loads])
        sprs = list(getattr(pr, "springs", ()) or ())
        spr = (_Spring * max(1, len(sprs)))(*[_Spring(int(a), int(b), int(c), float(k)) for a, b, c, k in sprs])
        keep += [p, d, sup, lds, spr]
        arr[k].mesh = _Mesh(int(pr.nelx), int(pr.nely), p.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)),
                            d.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)))
        arr[k].supports = ctypes.cast(sup, ctypes.POINTER(_Support))
        arr[k].n_supports = len(pr.supports)
        arr[k].loads = ctypes.cast(lds, ctypes.POINTER(_Load))
        arr[k].n_loads = len(pr.loads)
        arr[k].n_load_cases = int(pr.n_load_cases)
        arr[k].springs = ctypes.cast(spr, ctypes.POINTER(_Spring))
        arr[k].n_springs = len(sprs)
    return arr, keep


class Plan:
    """A plan for one or several design instances (batch), see mto.h.

    `problems` are objects with attributes nelx, nely, p, d, supports,
    loads, n_load_cases (e.g. ``problems.Problem``)."""

    def __init__(self, problems, **params):
        if not isinstance(problems, (list, tuple)):
            problems = [problems]
        prm = default_params(**params)
        self.params = prm
        arr, self._keep = _problem_array(problems)
        cp = _Params(prm["E0"], prm["Emin"], prm["nu"], prm["q"], prm["rtol"], prm["max_iter"],
                     prm["kernel_path"], prm["iters_per_launch"], prm["max_restarts"], prm["precond"],
                     prm["mg_omega"], prm["mg_coarse_max"], prm["stored_matrices"])
        h = ctypes.c_void_p()
        _check(_lib.mto_batch_plan_create(arr, len(problems), ctypes.byref(cp), ctypes.byref(h)))
        self._keep = []
        self.handle = h
        info = _Info()
        _check(_lib.mto_plan_info(self.handle, ctypes.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in _Info._fields_}
        self.n_instances = info.n_instances
        self.n_systems = info.n_systems
        self.instances = []
        for i in range(info.n_instances):
            v = [ctypes.c_int64() for _ in range(7)]
            nl = ctypes.c_int32()
            _check(_lib.mto_instance_info(self.handle, i, *[ctypes.byref(x) for x in v], ctypes.byref(nl)))
            keys = ("cell_off", "n_cells", "u_off", "n_dof", "g_off", "c_off", "n_free")
            rec = {k: x.value for k, x in zip(keys, v)}
            rec["n_load_cases"] = nl.value
            rec["nel"] = int(problems[i].nelx) * int(problems[i].nely)
            self.instances.append(rec)
        acc = 0
        for rec in self.instances:  # QR-error indicator layout: instance-major, load case, element
            rec["eps_off"] = acc
            acc += rec["n_load_cases"] * rec["nel"]
        self.n_eps = acc
        self.n_c = sum(r["n_load_cases"] for r in self.instances)
        self._bound = None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:  # _lib is None during interpreter shutdown
            _lib.mto_plan_destroy(h)
            self.handle = None

    def close(self):
        self.__del__()

    # -- helpers --
    def _empty(self, n, like):
        import torch

        return torch.empty(n, dtype=torch.float64, device=like.device)

    def _stats(self):
        st = _Stats()
        it = (ctypes.c_int32 * self.n_systems)()
        rr = (ctypes.c_double * self.n_systems)()
        st.iterations = ctypes.cast(it, ctypes.POINTER(ctypes.c_int32))
        st.true_rel_residual = ctypes.cast(rr, ctypes.POINTER(ctypes.c_double))
        return st, it, rr

    @staticmethod
    def _stats_dict(st, it, rr):
        return dict(status=st.status, restarts=st.restarts, max_iterations=st.max_iterations,
                    iterations=list(it), true_rel_residual=list(rr), solve_ms=st.solve_ms)

    # -- operations --
    def solve(self, rho, u0=None, sensitivities=True, stream=None, allow_noconv=False):
        """Returns (u, c, g or None, stats) for densities rho (float64 device)."""
        _f64_cuda(rho, self.info["n_cells"], "rho")
        u = self._empty(self.info["n_u"], rho)
        c = self._empty(self.n_c, rho)
        g = self._empty(self.info["n_g"], rho) if sensitivities else None
        if u0 is not None:
            _f64_cuda(u0, self.info["n_u"], "u0")
        st, it, rr = self._stats()
        rc = _lib.mto_solve(self.handle, _ptr(rho), _ptr(u), _ptr(c), _ptr(g), _ptr(u0), _stream(stream),
                            ctypes.byref(st))
        _check(rc, allow=(MTO_ENOCONV,) if allow_noconv else ())
        return u, c, g, self._stats_dict(st, it, rr)

    def capture(self, rho, sensitivities=True, stream=None):
        """Binds output buffers and captures the solve as HIP graphs."""
        _f64_cuda(rho, self.info["n_cells"], "rho")
        u = self._empty(self.info["n_u"], rho)
        c = self._empty(self.n_c, rho)
        g = self._empty(self.info["n_g"], rho) if sensitivities else None
        _check(_lib.mto_batch_capture(self.handle, _ptr(rho), _ptr(u), _ptr(c), _ptr(g), _stream(stream)))
        self._bound = (rho, u, c, g)
        return u, c, g

    def replay(self, stream=None, allow_noconv=False):
        if self._bound is None:
            raise RuntimeError("capture() first")
        st, it, rr = self._stats()
        rc = _lib.mto_batch_replay(self.handle, _stream(stream), ctypes.byref(st))
        _check(rc, allow=(MTO_ENOCONV,) if allow_noconv else ())
        return self._stats_dict(st, it, rr)

    def apply_stiffness(self, rho, x, stream=None):
        _f64_cuda(rho, self.info["n_cells"], "rho")
        _f64_cuda(x, self.info["n_u"], "x")
        y = self._empty(self.info["n_u"], rho)
        _check(_lib.mto_apply_stiffness(self.handle, _ptr(rho), _ptr(x), _ptr(y), _stream(stream)))
        return y

    def apply_stiffness_noalloc(self, rho, x, y, stream=None):
        """y = K x into the caller's y, with the library's static scratch (no
        device allocation in the library; see mto.h)."""
        _f64_cuda(rho, self.info["n_cells"], "rho")
        _f64_cuda(x, self.info["n_u"], "x")
        _f64_cuda(y, self.info["n_u"], "y")
        _check(_lib.mto_apply_stiffness_noalloc(self.handle, _ptr(rho), _ptr(x), _ptr(y), _stream(stream)))
        return y

    def sensitivity(self, rho, u, stream=None):
        _f64_cuda(rho, self.info["n_cells"], "rho")
        _f64_cuda(u, self.info["n_u"], "u")
        g = self._empty(self.info["n_g"], rho)
        _check(_lib.mto_sensitivity(self.handle, _ptr(rho), _ptr(u), _ptr(g), _stream(stream)))
        return g

    def adjoint_sensitivity(self, rho, u, lam, stream=None):
        """-E'(rho) lam_e^T K_s u_e per system (u, lam in the u layout, g
        layout out); see mto.h."""
        _f64_cuda(rho, self.info["n_cells"], "rho")
        _f64_cuda(u, self.info["n_u"], "u")
        _f64_cuda(lam, self.info["n_u"], "lam")
        g = self._empty(self.info["n_g"], rho)
        _check(_lib.mto_adjoint_sensitivity(self.handle, _ptr(rho), _ptr(u), _ptr(lam), _ptr(g), _stream(stream)))
        return g

    def qr_error(self, rho, u, stream=None):
        """QR-error indicator (Sec. 3.2.3, Eq. (9)) of every element and load
        case for displacements u (u layout) at densities rho; see mto.h."""
        _f64_cuda(rho, self.info["n_cells"], "rho")
        _f64_cuda(u, self.info["n_u"], "u")
        eps = self._empty(self.n_eps, rho)
        _check(_lib.mto_qr_error(self.handle, _ptr(rho), _ptr(u), _ptr(eps), _stream(stream)))
        return eps

    def kelly_indicator(self, u, stream=None):
        """Analysis indicator of Sec. 3.2.1 per (instance, load case, element)
        for displacements u (u layout); see mto.h."""
        _f64_cuda(u, self.info["n_u"], "u")
        gam = self._empty(self.n_eps, u)
        _check(_lib.mto_kelly_indicator(self.handle, _ptr(u), _ptr(gam), _stream(stream)))
        return gam

    def density_indicator(self, rho, cycle, alpha=0.2, beta=0.8, rho_min=0.0, rho_max=1.0, stream=None):
        """Density indicator of Sec. 3.2.2 per element (instances
        concatenated); see mto.h."""
        _f64_cuda(rho, self.info["n_cells"], "rho")
        gam = self._empty(self.info["n_elements"], rho)
        _check(_lib.mto_density_indicator(self.handle, _ptr(rho), int(cycle), float(alpha), float(beta),
                                          float(rho_min), float(rho_max), _ptr(gam), _stream(stream)))
        return gam

    def split_eps(self, eps):
        """Per instance [L, nel] views of the QR-error layout."""
        return [eps[r["eps_off"]:r["eps_off"] + r["n_load_cases"] * r["nel"]].view(r["n_load_cases"], r["nel"])
                for r in self.instances]

    def weighted_sensitivity(self, g, w, stream=None):
        """sum_l w_l dc_l/drho per instance (backward of rho -> c)."""
        _f64_cuda(g, self.info["n_g"], "g")
        _f64_cuda(w, self.n_c, "w")
        out = self._empty(self.info["n_cells"], g)
        _check(_lib.mto_weighted_sensitivity(self.handle, _ptr(g), _ptr(w), _ptr(out), _stream(stream)))
        return out

    def jacobi_diagonal(self, rho, stream=None):
        _f64_cuda(rho, self.info["n_cells"], "rho")
        n = sum(r["n_dof"] for r in self.instances)
        dg = self._empty(n, rho)
        _check(_lib.mto_jacobi_diagonal(self.handle, _ptr(rho), _ptr(dg), _stream(stream)))
        return dg

    def autotune(self, rho, cache=None, stream=None):
        """Tile shape per (p, d) group; `cache` is an optional path of the
        tile-shape cache file (see mto.h).  Returns the text report."""
        _f64_cuda(rho, self.info["n_cells"], "rho")
        buf = ctypes.create_string_buffer(8192)
        path = None if cache is None else os.fsencode(cache)
        _check(_lib.mto_autotune(self.handle, _ptr(rho), path, _stream(stream), buf, len(buf)))
        self._bound = None
        return buf.value.decode()

    def time_contraction(self, rho, reps=50, in_loop=False, stream=None):
        """Average ms of one PCG product K p (all groups), HIP events:
        back-to-back launches, or (in_loop) inside eagerly run PCG iterations."""
        _f64_cuda(rho, self.info["n_cells"], "rho")
        ms = ctypes.c_double()
        _check(_lib.mto_time_contraction(self.handle, _ptr(rho), int(reps), int(bool(in_loop)), _stream(stream),
                                         ctypes.byref(ms)))
        return ms.value

    def set_tile(self, ncol, ks=1, p=0, d=0):
        _check(_lib.mto_set_tile(self.handle, int(p), int(d), int(ncol), int(ks)))
        self._bound = None

    # -- layout helpers --
    def split_u(self, u):
        """Per instance [L, n_dof] views of the u layout."""
        return [u[r["u_off"]:r["u_off"] + r["n_load_cases"] * r["n_dof"]].view(r["n_load_cases"], r["n_dof"])
                for r in self.instances]

    def split_g(self, g):
        return [g[r["g_off"]:r["g_off"] + r["n_load_cases"] * r["n_cells"]].view(r["n_load_cases"], r["n_cells"])
                for r in self.instances]

    def split_c(self, c):
        return [c[r["c_off"]:r["c_off"] + r["n_load_cases"]] for r in self.instances]


class Filter:
    """Density filter of Sec. 2.2 (Eqs. (4)-(5)) over the density cells of
    `problems` (plan layout), radius R in element edge lengths; see mto.h."""

    def __init__(self, problems, R):
        if not isinstance(problems, (list, tuple)):
            problems = [problems]
        arr, keep = _problem_array(problems)
        h = ctypes.c_void_p()
        _check(_lib.mto_filter_create(arr, len(problems), float(R), ctypes.byref(h)))
        del keep
        self.handle = h
        self.R = float(R)
        n, nnz = ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.mto_filter_info(self.handle, ctypes.byref(n), ctypes.byref(nnz)))
        self.n_cells, self.nnz = n.value, nnz.value

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.mto_filter_destroy(h)
            self.handle = None

    def apply(self, rho, stream=None):
        """rho~ = W rho (new device tensor)."""
        import torch

        _f64_cuda(rho, self.n_cells, "rho")
        out = torch.empty_like(rho)
        _check(_lib.mto_filter_apply(self.handle, _ptr(rho), _ptr(out), _stream(stream)))
        return out

    def grad(self, g_tilde, stream=None):
        """dJ/drho = W^T dJ/drho~ (new device tensor)."""
        import torch

        _f64_cuda(g_tilde, self.n_cells, "g_tilde")
        out = torch.empty_like(g_tilde)
        _check(_lib.mto_filter_grad(self.handle, _ptr(g_tilde), _ptr(out), _stream(stream)))
        return out


def dp_update(nelx, nely, p, gamma_a, gamma_d, frac_a_refine=0.10, frac_a_coarsen=0.05, frac_d_refine=1.0,
              frac_d_coarsen=1.0, p_max=MTO_MAX_P, d_max=64):
    """Steps 2-3 of the dp update of Sec. 3.3 (host arrays in, numpy out):
    returns (p_new, theta, design_points, cells_per_element); see mto.h."""
    nel = int(nelx) * int(nely)
    p = np.ascontiguousarray(p, dtype=np.int8)
    ga = np.ascontiguousarray(gamma_a, dtype=np.float64)
    gd = np.ascontiguousarray(gamma_d, dtype=np.float64)
    if p.size != nel or ga.size != nel or gd.size != nel:
        raise ValueError("p, gamma_a and gamma_d need one entry per element")
    prm = _DpParams(frac_a_refine, frac_a_coarsen, frac_d_refine, frac_d_coarsen, int(p_max), int(d_max))
    p_out = np.empty(nel, np.int8)
    th = np.empty(nel, np.int8)
    dp = np.empty(nel, np.int32)
    cells = ctypes.c_int32()
    _check(_lib.mto_dp_update(int(nelx), int(nely), p.ctypes.data, ga.ctypes.data, gd.ctypes.data,
                              ctypes.byref(prm), p_out.ctypes.data, th.ctypes.data, dp.ctypes.data,
                              ctypes.byref(cells)))
    return p_out, th, dp, cells.value


def qr_update(p, eps, alpha_qr=0.9, p_max=MTO_MAX_P):
    """Step 4 of the dp update of Sec. 3.3: p + 1 where eps > alpha_qr."""
    p = np.ascontiguousarray(p, dtype=np.int8)
    e = np.ascontiguousarray(eps, dtype=np.float64)
    if e.size != p.size:
        raise ValueError("one QR error per element")
    out = np.empty(p.size, np.int8)
    _check(_lib.mto_qr_update(int(p.size), p.ctypes.data, e.ctypes.data, float(alpha_qr), int(p_max),
                              out.ctypes.data))
    return out
