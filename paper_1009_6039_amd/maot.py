"""Python binding of libmaot.so (ctypes): argument marshalling only.

Every step of the solver runs in the library's HIP kernels.  Tensors are torch
CUDA (HIP) tensors, float64 for densities and potentials, float32 for the
single-step fields; they are passed to the C ABI as device pointers together with
the current torch stream.  The library must be built (``paper_1009_6039_amd.build``);
importing this module fails loudly if it is not.
"""

import ctypes
import os

import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmaot.so")

OK, ENOCONV, ENONCONVEX, ENAN = 0, 1, 2, 3
EINVAL, ENOMEM, EHIP = -1, -2, -3
INTERP = {"bilinear": 0, "nearest": 1}
OP_MODE = {"full": 0, "no_drift": 1}
DAMPING = {"fixed": 0, "backtrack": 1}
SYMBOL = {"spectral": 0, "fd4": 1}
PRECOND = {"none": 0, "diag": 1}
FORCING = {"fixed": 0, "adaptive": 1}
LINEAR = {"strain_gmres": 0, "fd_bicg": 1}

PROF = {"none": 0, "residual": 1, "row_a": 2, "column": 3, "row_c": 4, "bicg_matvec": 5}

EXPORTED = ("ma_abi_version", "ma_options_default", "ma_strerror", "ma_plan_create",
            "ma_plan_destroy", "ma_plan_set_options", "ma_solve", "ma_solve_batched", "ma_solve_noalloc",
            "ma_plan_profile", "ma_plan_profile_read",
            "ma_plan_autotune", "ma_plan_set_tuning", "ma_plan_get_tuning", "ma_tune_geometry",
            "ma_step_residual", "ma_step_fft2", "ma_step_strain_apply",
            "ma_step_lbar_inverse", "ma_step_gmres", "ma_power_inverse", "ma_step_fd_apply", "ma_step_bicg",
            "ma3_plan_create", "ma3_plan_destroy", "ma3_solve", "ma3_step_residual", "ma3_step_strain_apply",
            "ma3_step_lbar_inverse",
            "ma_cnn_create", "ma_cnn_destroy", "ma_cnn_param_count", "ma_cnn_set_params",
            "ma_cnn_get_params", "ma_cnn_prepare_input", "ma_cnn_target", "ma_cnn_forward",
            "ma_cnn_gradients", "ma_cnn_train_step", "ma_cnn_warm_start")


class Options(ctypes.Structure):
    _fields_ = [("max_newton", ctypes.c_int), ("gmres_m", ctypes.c_int),
                ("gmres_max_restarts", ctypes.c_int), ("gmres_tol", ctypes.c_double),
                ("interp", ctypes.c_int), ("op_mode", ctypes.c_int),
                ("damping_policy", ctypes.c_int), ("max_backtrack", ctypes.c_int),
                ("symbol", ctypes.c_int), ("precond", ctypes.c_int), ("boundary_frac", ctypes.c_double),
                ("forcing", ctypes.c_int), ("wait_limit_s", ctypes.c_double), ("max_active", ctypes.c_int),
                ("linear_solver", ctypes.c_int), ("bicg_max_iters", ctypes.c_int)]


class Tuning(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("npairs", ctypes.c_int), ("variant", ctypes.c_int * 4),
                ("from_cache", ctypes.c_int), ("rejected", ctypes.c_int),
                ("us", ctypes.c_double * 4), ("us_default", ctypes.c_double * 4),
                ("us_variant", (ctypes.c_double * 12) * 4), ("npairs_part", ctypes.c_int),
                ("us_part_variant", (ctypes.c_double * 12) * 4)]

    def as_dict(self):
        return {"n": self.n, "npairs": self.npairs, "variant": list(self.variant),
                "from_cache": bool(self.from_cache), "rejected": self.rejected,
                "us": list(self.us), "us_default": list(self.us_default),
                "us_variant": {name: [round(x, 2) for x in self.us_variant[k]]
                               for k, name in enumerate(TUNE_PASSES)},
                "npairs_part": self.npairs_part,
                "us_part_variant": {name: [round(x, 3) for x in self.us_part_variant[k]]
                                    for k, name in enumerate(TUNE_PASSES)}}


TUNE_PASSES = ("row_a", "column", "row_c", "residual")
TUNE_VARIANTS = 12  # MA_TUNE_VARIANTS: 0..3 block-shared kernels, 4..7 wave-owned transforms
                    # (row pass C: 4, 5 wave-owned; 6, 7 block-shared with early coefficient
                    # loads), 8..11 FFT radix plans


def tune_geometry(kernel_class, n, variant):
    """(canonical variant or -1, rows/columns/tile width per workgroup, threads); host only."""
    u, t = ctypes.c_int(), ctypes.c_int()
    k = TUNE_PASSES.index(kernel_class) if isinstance(kernel_class, str) else int(kernel_class)
    c = load().ma_tune_geometry(k, n, variant, ctypes.byref(u), ctypes.byref(t))
    return c, u.value, t.value


def pass_kernel_name(kernel_class, n, variant):
    """The kernel that `variant` of a transform pass launches at grid size n, as the
    profilers name it ("k_passC<512, 3, false, 0>": size, block geometry, early
    coefficient loads, radix plan; "k_passC_w<512, 1>": a wave-owned kernel), or None."""
    canon, units, _ = tune_geometry(kernel_class, n, variant)
    if canon < 0 or kernel_class not in ("row_a", "column", "row_c"):
        return None
    base = {"row_a": "k_passA", "column": "k_passB", "row_c": "k_passC"}[kernel_class]
    second = 3 if kernel_class == "row_c" else 2
    pf, plan = False, 0
    if canon >= 8:  # radix plan at the default or the second geometry
        plan = (canon - 8) % 2 + 1
        g = tune_geometry(kernel_class, n, 0 if canon < 10 else second)[0]
    elif kernel_class == "row_c" and canon in (6, 7):  # early coefficient loads
        pf = True
        g = tune_geometry(kernel_class, n, 0 if canon == 6 else 3)[0]
    elif canon >= 4:
        return "%s_w<%d, %d>" % (base, n, units)
    else:
        g = canon
    if kernel_class == "row_c":
        return "%s<%d, %d, %s, %d>" % (base, n, g, "true" if pf else "false", plan)
    return "%s<%d, %d, %d>" % (base, n, g, plan)


class Report(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("newton_iters", ctypes.c_int),
                ("gmres_iters", ctypes.c_int), ("backtracks", ctypes.c_int),
                ("res_rms", ctypes.c_double), ("res_max", ctypes.c_double),
                ("res0_rms", ctypes.c_double), ("mass_defect", ctypes.c_double),
                ("min_det", ctypes.c_double), ("w2sq", ctypes.c_double),
                ("tau_final", ctypes.c_double), ("time_ms", ctypes.c_double),
                ("warm_steps", ctypes.c_int), ("pad", ctypes.c_int)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def load():
    """Loads libmaot.so once; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libmaot.so is not built: run python -m paper_1009_6039_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I, D = ctypes.c_int, ctypes.c_double
    lib.ma_abi_version.restype = I
    lib.ma_options_default.argtypes = [ctypes.POINTER(Options)]
    lib.ma_strerror.restype = ctypes.c_char_p
    lib.ma_strerror.argtypes = [I]
    lib.ma_plan_create.argtypes = [I, I, ctypes.POINTER(Options), ctypes.POINTER(P)]
    lib.ma_plan_destroy.argtypes = [P]
    lib.ma_plan_set_options.argtypes = [P, ctypes.POINTER(Options)]
    lib.ma_solve.argtypes = [P, P, P, I, D, D, P, P, P, ctypes.POINTER(Report), P]
    lib.ma_solve_batched.argtypes = [P, I, ctypes.POINTER(I), ctypes.POINTER(P), ctypes.POINTER(P),
                                     ctypes.POINTER(P), D, D, ctypes.POINTER(P), ctypes.POINTER(P),
                                     ctypes.POINTER(Report), P]
    lib.ma_solve_noalloc.argtypes = [ctypes.POINTER(Options), P, P, I, D, D, P, P, P, ctypes.POINTER(Report), P]
    lib.ma_plan_profile.argtypes = [P, I, I]
    lib.ma_plan_profile_read.argtypes = [P, ctypes.POINTER(D), ctypes.POINTER(ctypes.c_longlong),
                                         ctypes.POINTER(D), ctypes.POINTER(ctypes.c_longlong),
                                         ctypes.POINTER(D)]
    lib.ma_plan_autotune.argtypes = [P, I, I, ctypes.c_char_p, ctypes.POINTER(Tuning), P]
    lib.ma_plan_set_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
    lib.ma_plan_get_tuning.argtypes = [P, I, ctypes.POINTER(Tuning)]
    lib.ma_tune_geometry.argtypes = [I, I, I, ctypes.POINTER(I), ctypes.POINTER(I)]
    lib.ma_step_residual.argtypes = [P, I, P, P, P, P, P, ctypes.POINTER(D), P]
    lib.ma_step_fft2.argtypes = [P, I, P, P, P]
    lib.ma_step_strain_apply.argtypes = [P, I, P, P, ctypes.POINTER(D), P, P]
    lib.ma_step_lbar_inverse.argtypes = [P, I, P, ctypes.POINTER(D), P, P]
    lib.ma_step_gmres.argtypes = [P, I, P, P, ctypes.POINTER(D), I, D, I, P, ctypes.POINTER(I), P]
    lib.ma_power_inverse.argtypes = [P, I, P, ctypes.POINTER(D), P, I, D, I, I, ctypes.POINTER(D),
                                     ctypes.POINTER(I), P]
    lib.ma_step_fd_apply.argtypes = [P, I, P, P, P, P, P, P]
    lib.ma_step_bicg.argtypes = [P, I, P, P, D, I, P, ctypes.POINTER(I), P]
    lib.ma3_plan_create.argtypes = [I, ctypes.POINTER(Options), ctypes.POINTER(P)]
    lib.ma3_plan_destroy.argtypes = [P]
    lib.ma3_solve.argtypes = [P, P, P, I, D, D, P, P, ctypes.POINTER(Report), P]
    lib.ma3_step_residual.argtypes = [P, I, P, P, P, P, P, ctypes.POINTER(D), P]
    lib.ma3_step_strain_apply.argtypes = [P, I, P, P, ctypes.POINTER(D), P, P]
    lib.ma3_step_lbar_inverse.argtypes = [P, I, P, ctypes.POINTER(D), P, P]
    F, L = ctypes.c_float, ctypes.c_long
    lib.ma_cnn_create.argtypes = [I, I, I, I, ctypes.POINTER(I), ctypes.POINTER(P)]
    lib.ma_cnn_destroy.argtypes = [P]
    lib.ma_cnn_param_count.argtypes = [P]
    lib.ma_cnn_param_count.restype = L
    lib.ma_cnn_set_params.argtypes = [P, ctypes.POINTER(F), L]
    lib.ma_cnn_get_params.argtypes = [P, ctypes.POINTER(F), L]
    lib.ma_cnn_prepare_input.argtypes = [P, P, P, I, P, P]
    lib.ma_cnn_target.argtypes = [P, P, P, P, I, I, P, P]
    lib.ma_cnn_forward.argtypes = [P, P, I, P, P]
    lib.ma_cnn_gradients.argtypes = [P, P, P, I, P, ctypes.POINTER(F), P]
    lib.ma_cnn_train_step.argtypes = [P, P, P, I, F, ctypes.POINTER(F), P]
    lib.ma_cnn_warm_start.argtypes = [P, I, I, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P), P]
    for name in EXPORTED:
        getattr(lib, name).restype = getattr(lib, name).restype or I
    lib.ma_cnn_destroy.restype = None
    lib.ma_plan_destroy.restype = None
    lib.ma_options_default.restype = None
    _lib = lib
    return lib


def strerror(code):
    return load().ma_strerror(int(code)).decode()


class MAError(RuntimeError):
    def __init__(self, code, what):
        super().__init__("%s: %s (%d)" % (what, strerror(code), code))
        self.code = code


def _check(code, what):
    if code < 0:
        raise MAError(code, what)
    return code


def make_options(**kw):
    o = Options()
    load().ma_options_default(ctypes.byref(o))
    for k, v in kw.items():
        if k == "interp":
            v = INTERP[v] if isinstance(v, str) else v
        elif k == "op_mode":
            v = OP_MODE[v] if isinstance(v, str) else v
        elif k == "damping_policy":
            v = DAMPING[v] if isinstance(v, str) else v
        elif k == "symbol":
            v = SYMBOL[v] if isinstance(v, str) else v
        elif k == "precond":
            v = PRECOND[v] if isinstance(v, str) else v
        elif k == "forcing":
            v = FORCING[v] if isinstance(v, str) else v
        elif k == "linear_solver":
            v = LINEAR[v] if isinstance(v, str) else v
        if not hasattr(o, k):
            raise TypeError("unknown option %r" % k)
        setattr(o, k, v)
    return o


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise TypeError("expected a contiguous %s CUDA tensor" % dtype)
    return t


class Plan:
    """Owns one ma_plan (device workspace, options)."""

    def __init__(self, n_max=512, batch_capacity=1, **opts):
        lib = load()
        self.options = make_options(**opts)
        h = ctypes.c_void_p()
        _check(lib.ma_plan_create(int(n_max), int(batch_capacity), ctypes.byref(self.options),
                                  ctypes.byref(h)), "ma_plan_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().ma_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_options(self, **opts):
        self.options = make_options(**opts)
        _check(load().ma_plan_set_options(self._h, ctypes.byref(self.options)), "ma_plan_set_options")

    # -- timing hook -------------------------------------------------------------
    def profile(self, kernel_class, every=1):
        """Times every `every`-th launch of one kernel class ("residual", "row_a",
        "column", "row_c")."""
        k = PROF[kernel_class] if isinstance(kernel_class, str) else int(kernel_class)
        _check(load().ma_plan_profile(self._h, k, int(every)), "ma_plan_profile")

    def profile_read(self):
        """Timed launches: summed event time, count, algorithmic bytes; all launches of
        the class: count and algorithmic bytes."""
        ms, n, b = ctypes.c_double(), ctypes.c_longlong(), ctypes.c_double()
        na, ba = ctypes.c_longlong(), ctypes.c_double()
        _check(load().ma_plan_profile_read(self._h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b),
                                           ctypes.byref(na), ctypes.byref(ba)), "ma_plan_profile_read")
        return {"ms": ms.value, "launches": n.value, "bytes": b.value, "all_launches": na.value,
                "all_bytes": ba.value}

    # -- autotuner -----------------------------------------------------------------
    def autotune(self, n, npairs, cache=None):
        """Chooses the launch geometry for size n from timed, output-checked variants;
        cache: JSON file path (read if it holds an entry, else written)."""
        t = Tuning()
        _check(load().ma_plan_autotune(self._h, int(n), int(npairs), cache.encode() if cache else None,
                                       ctypes.byref(t), _stream()), "ma_plan_autotune")
        return t.as_dict()

    def set_tuning(self, n, variant):
        t = Tuning()
        t.n = int(n)
        for k in range(4):
            t.variant[k] = int(variant[k])
        _check(load().ma_plan_set_tuning(self._h, ctypes.byref(t)), "ma_plan_set_tuning")

    def get_tuning(self, n):
        t = Tuning()
        _check(load().ma_plan_get_tuning(self._h, int(n), ctypes.byref(t)), "ma_plan_get_tuning")
        return list(t.variant)

    # -- full solves ------------------------------------------------------------
    def solve(self, f, g, damping=1.0, tol=1e-6, psi0=None, want_map=True):
        f = _dev(f, torch.float64)
        g = _dev(g, torch.float64)
        psi0 = _dev(psi0, torch.float64)
        n = f.shape[0]
        psi = torch.empty_like(f)
        mp = torch.empty((2, n, n), dtype=torch.float64, device=f.device) if want_map else None
        rep = Report()
        code = load().ma_solve(self._h, _ptr(f), _ptr(g), n, float(damping), float(tol), _ptr(psi0),
                               _ptr(psi), _ptr(mp), ctypes.byref(rep), _stream())
        _check(code, "ma_solve")
        return psi, mp, rep.as_dict()

    def solve_batched(self, fs, gs, damping=1.0, tol=1e-6, psi0s=None, want_map=False):
        npairs = len(fs)
        ns = (ctypes.c_int * npairs)(*[int(f.shape[0]) for f in fs])
        fs = [_dev(f, torch.float64) for f in fs]
        gs = [_dev(g, torch.float64) for g in gs]
        psis = [torch.empty_like(f) for f in fs]
        maps = [torch.empty((2,) + tuple(f.shape), dtype=torch.float64, device=f.device)
                for f in fs] if want_map else None
        arr = ctypes.c_void_p * npairs
        fa = arr(*[t.data_ptr() for t in fs])
        ga = arr(*[t.data_ptr() for t in gs])
        pa = arr(*[(_dev(t, torch.float64).data_ptr() if t is not None else 0) for t in psi0s]) \
            if psi0s is not None else None
        oa = arr(*[t.data_ptr() for t in psis])
        ma_ = arr(*[t.data_ptr() for t in maps]) if maps is not None else None
        reps = (Report * npairs)()
        code = load().ma_solve_batched(self._h, npairs, ns, fa, ga, pa, float(damping), float(tol),
                                       oa, ma_, reps, _stream())
        _check(code, "ma_solve_batched")
        return psis, maps, [r.as_dict() for r in reps]

    # -- single steps -------------------------------------------------------------
    def step_residual(self, u, f, g):
        u, f, g = (_dev(t, torch.float64) for t in (u, f, g))
        n = u.shape[0]
        r = torch.empty((n, n), dtype=torch.float32, device=u.device)
        coef = torch.empty((5, n, n), dtype=torch.float32, device=u.device)
        sc = (ctypes.c_double * 12)()
        _check(load().ma_step_residual(self._h, n, _ptr(u), _ptr(f), _ptr(g), _ptr(r), _ptr(coef),
                                       sc, _stream()), "ma_step_residual")
        names = ("res_rms", "res_max", "mass_defect", "min_det", "min_trace", "abar11", "abar12",
                 "abar22", "bbar1", "bbar2", "w2", "mean_u")
        return r, coef, dict(zip(names, list(sc)))

    def step_fft2(self, v):
        v = _dev(v, torch.float32)
        n = v.shape[0]
        spec = torch.empty((n, n // 2, 2), dtype=torch.float32, device=v.device)
        _check(load().ma_step_fft2(self._h, n, _ptr(v), _ptr(spec), _stream()), "ma_step_fft2")
        return torch.view_as_complex(spec)

    def step_strain_apply(self, v, coef, abar):
        v = _dev(v, torch.float32)
        coef = _dev(coef, torch.float32)
        n = v.shape[0]
        w = torch.empty_like(v)
        ab = (ctypes.c_double * 5)(*[float(a) for a in abar])
        _check(load().ma_step_strain_apply(self._h, n, _ptr(v), _ptr(coef), ab, _ptr(w), _stream()),
               "ma_step_strain_apply")
        return w

    def step_lbar_inverse(self, sigma, abar):
        sigma = _dev(sigma, torch.float32)
        n = sigma.shape[0]
        theta = torch.empty_like(sigma)
        ab = (ctypes.c_double * 5)(*[float(a) for a in abar])
        _check(load().ma_step_lbar_inverse(self._h, n, _ptr(sigma), ab, _ptr(theta), _stream()),
               "ma_step_lbar_inverse")
        return theta

    def step_gmres(self, h, coef, abar, m=10, tol=1e-4, max_restarts=20):
        h = _dev(h, torch.float32)
        coef = _dev(coef, torch.float32)
        n = h.shape[0]
        theta = torch.empty_like(h)
        ab = (ctypes.c_double * 5)(*[float(a) for a in abar])
        its = ctypes.c_int(0)
        _check(load().ma_step_gmres(self._h, n, _ptr(h), _ptr(coef), ab, int(m), float(tol),
                                    int(max_restarts), _ptr(theta), ctypes.byref(its), _stream()),
               "ma_step_gmres")
        return theta, its.value

    def step_fd_apply(self, p, pt, coef):
        """The finite-difference operator of Section 4.1: (tilde A p, tilde A^T pt), FP64."""
        p = _dev(p, torch.float64)
        pt = _dev(pt, torch.float64)
        coef = _dev(coef, torch.float32)
        n = p.shape[0]
        q = torch.empty_like(p)
        qt = torch.empty_like(p)
        _check(load().ma_step_fd_apply(self._h, n, _ptr(p), _ptr(pt), _ptr(coef), _ptr(q), _ptr(qt), _stream()),
               "ma_step_fd_apply")
        return q, qt

    def step_bicg(self, h, coef, tol=1e-4, max_iters=1000):
        """BiCG on tilde A x = h (Section 4.1): (x FP64, iterations)."""
        h = _dev(h, torch.float32)
        coef = _dev(coef, torch.float32)
        n = h.shape[0]
        x = torch.empty(h.shape, dtype=torch.float64, device=h.device)
        its = ctypes.c_int(0)
        _check(load().ma_step_bicg(self._h, n, _ptr(h), _ptr(coef), float(tol), int(max_iters), _ptr(x),
                                   ctypes.byref(its), _stream()), "ma_step_bicg")
        return x, its.value

    def power_inverse(self, coef, abar, b0, iters=8, gmres_tol=1e-6, m=10, max_restarts=50):
        """Power iteration on the inverse operator (Section 5.1): (rho_k, GMRES iterations per step)."""
        coef = _dev(coef, torch.float32)
        b0 = _dev(b0, torch.float32)
        n = b0.shape[0]
        ab = (ctypes.c_double * 5)(*[float(a) for a in abar])
        rho = (ctypes.c_double * iters)()
        its = (ctypes.c_int * iters)()
        _check(load().ma_power_inverse(self._h, n, _ptr(coef), ab, _ptr(b0), int(iters), float(gmres_tol), int(m),
                                       int(max_restarts), rho, its, _stream()), "ma_power_inverse")
        return list(rho), list(its)


class Plan3:
    """Owns one ma3_plan: the damped Newton solver on N x N x N grids."""

    def __init__(self, n_max=64, **opts):
        lib = load()
        self.options = make_options(**opts)
        h = ctypes.c_void_p()
        _check(lib.ma3_plan_create(int(n_max), ctypes.byref(self.options), ctypes.byref(h)), "ma3_plan_create")
        self._h = h

    def close(self):
        if self._h:
            load().ma3_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, f, g, damping=1.0, tol=1e-6, want_map=True):
        f = _dev(f, torch.float64)
        g = _dev(g, torch.float64)
        n = f.shape[0]
        psi = torch.empty_like(f)
        mp = torch.empty((3,) + tuple(f.shape), dtype=torch.float64, device=f.device) if want_map else None
        rep = Report()
        code = load().ma3_solve(self._h, _ptr(f), _ptr(g), n, float(damping), float(tol), _ptr(psi), _ptr(mp),
                                ctypes.byref(rep), _stream())
        if code < 0:
            raise MAError(code, "ma3_solve")
        return psi, mp, rep.as_dict()

    def step_residual(self, u, f, g):
        u, f, g = (_dev(t, torch.float64) for t in (u, f, g))
        n = u.shape[0]
        r = torch.empty(u.shape, dtype=torch.float32, device=u.device)
        coef = torch.empty((9,) + tuple(u.shape), dtype=torch.float32, device=u.device)
        sc = (ctypes.c_double * 17)()
        _check(load().ma3_step_residual(self._h, n, _ptr(u), _ptr(f), _ptr(g), _ptr(r), _ptr(coef), sc, _stream()),
               "ma3_step_residual")
        return r, coef, list(sc)

    def step_strain_apply(self, v, coef, abar):
        v = _dev(v, torch.float32)
        coef = _dev(coef, torch.float32)
        w = torch.empty_like(v)
        ab = (ctypes.c_double * 9)(*[float(a) for a in abar])
        _check(load().ma3_step_strain_apply(self._h, v.shape[0], _ptr(v), _ptr(coef), ab, _ptr(w), _stream()),
               "ma3_step_strain_apply")
        return w

    def step_lbar_inverse(self, sigma, abar):
        sigma = _dev(sigma, torch.float32)
        th = torch.empty_like(sigma)
        ab = (ctypes.c_double * 9)(*[float(a) for a in abar])
        _check(load().ma3_step_lbar_inverse(self._h, sigma.shape[0], _ptr(sigma), ab, _ptr(th), _stream()),
               "ma3_step_lbar_inverse")
        return th


class WarmStartNet:
    """The warm-start network (ma_cnn): BF16 MFMA convolutions with FP32 masters."""

    def __init__(self, layers=8, channels=32, n_net=256, max_batch=16, dilations=None):
        lib = load()
        h = ctypes.c_void_p()
        dil = None
        if dilations is not None:
            if len(dilations) != layers:
                raise ValueError("one dilation per layer")
            dil = (ctypes.c_int * layers)(*[int(d) for d in dilations])
        _check(lib.ma_cnn_create(layers, channels, n_net, max_batch, dil, ctypes.byref(h)), "ma_cnn_create")
        self._h = h
        self.layers, self.channels, self.n_net, self.max_batch = layers, channels, n_net, max_batch
        self.dilations = list(dilations) if dilations is not None else [1] * layers
        self.count = int(lib.ma_cnn_param_count(h))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().ma_cnn_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, flat):
        import numpy as np
        a = np.ascontiguousarray(flat, dtype=np.float32)
        if a.size != self.count:
            raise ValueError("expected %d parameters" % self.count)
        _check(load().ma_cnn_set_params(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size),
               "ma_cnn_set_params")

    def get_params(self):
        import numpy as np
        a = np.empty(self.count, dtype=np.float32)
        _check(load().ma_cnn_get_params(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size),
               "ma_cnn_get_params")
        return a

    def prepare_input(self, f, g):
        """f, g: CUDA float64 [batch, n_net, n_net] -> BF16 input [batch, n_net, n_net, 8]."""
        f = _dev(f, torch.float64)
        g = _dev(g, torch.float64)
        x = torch.empty(f.shape + (8,), dtype=torch.bfloat16, device=f.device)
        _check(load().ma_cnn_prepare_input(self._h, _ptr(f), _ptr(g), f.shape[0], _ptr(x), _stream()),
               "ma_cnn_prepare_input")
        return x

    def target(self, psi, f=None, g=None):
        """Training target [batch, n, n] FP32: Laplacian of psi minus the log-density ratio
        (the plain Laplacian when f and g are None)."""
        psi = _dev(psi, torch.float64)
        if f is not None:
            f = _dev(f, torch.float64)
            g = _dev(g, torch.float64)
        out = torch.empty(psi.shape, dtype=torch.float32, device=psi.device)
        _check(load().ma_cnn_target(self._h, _ptr(psi), _ptr(f) if f is not None else None,
                                    _ptr(g) if g is not None else None, psi.shape[0], psi.shape[-1], _ptr(out),
                                    _stream()), "ma_cnn_target")
        return out

    def forward(self, x):
        x = _dev(x, torch.bfloat16)
        c = torch.empty(x.shape[:3], dtype=torch.float32, device=x.device)
        _check(load().ma_cnn_forward(self._h, _ptr(x), x.shape[0], _ptr(c), _stream()), "ma_cnn_forward")
        return c

    def gradients(self, x, target):
        x = _dev(x, torch.bfloat16)
        target = _dev(target, torch.float32)
        grads = torch.empty(self.count, dtype=torch.float32, device=x.device)
        loss = ctypes.c_float()
        _check(load().ma_cnn_gradients(self._h, _ptr(x), _ptr(target), x.shape[0], _ptr(grads),
                                       ctypes.byref(loss), _stream()), "ma_cnn_gradients")
        return grads, loss.value

    def train_step(self, x, target, lr, want_loss=False):
        x = _dev(x, torch.bfloat16)
        target = _dev(target, torch.float32)
        loss = ctypes.c_float()
        _check(load().ma_cnn_train_step(self._h, _ptr(x), _ptr(target), x.shape[0], float(lr),
                                        ctypes.byref(loss) if want_loss else None, _stream()),
               "ma_cnn_train_step")
        return loss.value if want_loss else None

    def warm_start(self, fs, gs):
        """Initial potentials for lists of CUDA float64 densities of one size."""
        n = int(fs[0].shape[0])
        npairs = len(fs)
        psis = [torch.empty_like(f) for f in fs]
        arr = ctypes.c_void_p * npairs
        fa = arr(*[_dev(t, torch.float64).data_ptr() for t in fs])
        ga = arr(*[_dev(t, torch.float64).data_ptr() for t in gs])
        pa = arr(*[t.data_ptr() for t in psis])
        _check(load().ma_cnn_warm_start(self._h, npairs, n, fa, ga, pa, _stream()), "ma_cnn_warm_start")
        return psis


def solve_noalloc(f, g, damping=1.0, tol=1e-6, psi0=None, psi=None, map=None, **opts):
    """ma_solve_noalloc: one pair with no device allocation inside the library; the
    outputs psi (and map, if given) are caller-owned CUDA float64 tensors (allocated
    here when None).  Returns (psi, map, report)."""
    f = _dev(f, torch.float64)
    g = _dev(g, torch.float64)
    psi0 = _dev(psi0, torch.float64)
    n = f.shape[0]
    psi = _dev(psi, torch.float64) if psi is not None else torch.empty_like(f)
    mp = _dev(map, torch.float64) if map is not None else None
    o = make_options(**opts)
    rep = Report()
    code = load().ma_solve_noalloc(ctypes.byref(o), _ptr(f), _ptr(g), n, float(damping), float(tol), _ptr(psi0),
                                   _ptr(psi), _ptr(mp), ctypes.byref(rep), _stream())
    _check(code, "ma_solve_noalloc")
    return psi, mp, rep.as_dict()


def solve(f, g, damping=1.0, tol=1e-6, psi0=None, **opts):
    """One-shot solve: returns (psi, map, report) for CUDA float64 tensors f, g."""
    plan = Plan(n_max=f.shape[0], batch_capacity=1, **opts)
    try:
        return plan.solve(f, g, damping=damping, tol=tol, psi0=psi0)
    finally:
        plan.close()
