"""ctypes binding of libgsm (include/gsm.h): argument marshalling only.

Every computation runs in the HIP library; this module converts NumPy/torch
arguments to the C structures, allocates the device workspace as a torch
uint8 tensor and passes torch's current HIP stream.  It raises if the
library has not been built (``python paper_1501_01752_amd/csrc/build.py``).
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("GSM_LIBRARY") or os.path.join(_HERE, "libgsm.so")

GSM_OK, GSM_W_NOT_CONVERGED = 0, 1
GSM_E_ARG, GSM_E_NONFINITE, GSM_E_NOMEM, GSM_E_DEVICE = -1, -2, -3, -4
GSM_E_SINGULAR, GSM_E_WORKSPACE, GSM_E_UNSUPPORTED = -5, -6, -7
GSM_MIXED, GSM_FP64 = 0, 1
GSM_GMRES, GSM_BICGSTAB = 0, 1
GSM_OUT_HOST, GSM_SOLVE_GRAPH, GSM_SOLVE_REORTH = 1, 2, 4
GSM_APPLY_FORWARD, GSM_APPLY_ADJOINT, GSM_APPLY_FORWARD_H = 0, 1, 2
GSM_FORM_E, GSM_FORM_H = 0, 1
GSM_PLAN_AUTOTUNE = 1


class Geometry(C.Structure):
    _fields_ = [("period", C.c_double * 3), ("nvox", C.c_int32 * 3), ("eps", C.POINTER(C.c_double))]


class PlanOpts(C.Structure):
    _fields_ = [("m_max", C.c_int32 * 3), ("device", C.c_int32), ("flags", C.c_int32),
                ("reserved", C.c_int32), ("tune_cache", C.c_char_p)]


class Instance(C.Structure):
    _fields_ = [("wavelength", C.c_double), ("k_inc", C.c_double * 3), ("M", C.c_int32 * 3),
                ("n_drive", C.c_int32), ("pol", (C.c_double * 6) * 3), ("eps_b", C.c_double)]


class SolverOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("inner_tol", C.c_double), ("restart", C.c_int32),
                ("max_iter", C.c_int32), ("max_refine", C.c_int32), ("precision", C.c_int32),
                ("method", C.c_int32), ("flags", C.c_int32), ("x0", C.c_void_p),
                ("group_max", C.c_int32), ("formulation", C.c_int32)]


GSM_SHAPE_SPHERE, GSM_SHAPE_ELLIPSOID, GSM_SHAPE_BOX = 0, 1, 2
_SHAPE_KINDS = {"sphere": GSM_SHAPE_SPHERE, "ellipsoid": GSM_SHAPE_ELLIPSOID, "box": GSM_SHAPE_BOX}


class Shape(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("centre", C.c_double * 3),
                ("size", C.c_double * 3), ("eps", C.c_double)]


class ShapeBody(C.Structure):
    _fields_ = [("period", C.c_double * 3), ("eps_host", C.c_double), ("n_shapes", C.c_int32),
                ("reserved", C.c_int32), ("shapes", C.POINTER(Shape))]


class CoeffBody(C.Structure):
    _fields_ = [("period", C.c_double * 3), ("n_max", C.c_int32 * 3), ("reserved", C.c_int32),
                ("coef", C.POINTER(C.c_double)), ("eps_min", C.c_double), ("eps_max", C.c_double),
                ("coef_inv", C.POINTER(C.c_double))]


GSM_POLE_MAX_NP, GSM_POLE_MAX_ND = 8, 32


class PoleQuery(C.Structure):
    _fields_ = [("wavelength", C.c_double), ("k_hat", C.c_double * 3), ("M", C.c_int32 * 3),
                ("n_poles", C.c_int32), ("n_div", C.c_int32), ("component", C.c_int32),
                ("pol", C.c_double * 6), ("kappa_min", C.c_double), ("kappa_max", C.c_double),
                ("eps_b", C.c_double)]


class PoleResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("n_poles", C.c_int32), ("best", C.c_int32),
                ("iterations", C.c_int32), ("eta", (C.c_double * 2) * GSM_POLE_MAX_NP),
                ("zeta", (C.c_double * 2) * GSM_POLE_MAX_NP), ("n_eff", C.c_double),
                ("eps_b", C.c_double), ("max_rel_residual", C.c_double)]

    def as_dict(self):
        n = self.n_poles
        return {"status": self.status, "n_poles": n, "best": self.best, "iterations": self.iterations,
                "eta": np.array([complex(self.eta[k][0], self.eta[k][1]) for k in range(n)]),
                "zeta": np.array([complex(self.zeta[k][0], self.zeta[k][1]) for k in range(n)]),
                "n_eff": self.n_eff, "eps_b": self.eps_b, "max_rel_residual": self.max_rel_residual}


def make_pole_query(wavelength, k_hat, M, kappa_min, kappa_max, drive=(1.0, 0.0, 0.0), component=0,
                    n_poles=5, n_div=10, eps_b=0.0):
    """One pole search along k_hat with the given drive: xi = E_component,0."""
    q = PoleQuery()
    q.wavelength = float(wavelength)
    for a in range(3):
        q.k_hat[a] = float(k_hat[a])
        q.M[a] = int(M[a])
        z = complex(drive[a])
        q.pol[2 * a], q.pol[2 * a + 1] = z.real, z.imag
    q.n_poles, q.n_div, q.component = int(n_poles), int(n_div), int(component)
    q.kappa_min, q.kappa_max, q.eps_b = float(kappa_min), float(kappa_max), float(eps_b)
    return q


def pole_fit(kappa, xi, n_poles, n_div, stream=None):
    """gsm_pole_fit on device tensors: kappa float64 [n, N_d+N_p], xi
    complex128 [n, N_d+N_p] -> (eta, zeta complex128 [n, N_p], status int32 [n])."""
    import torch
    kappa = kappa.contiguous()
    xi = xi.contiguous()
    n = kappa.shape[0]
    eta = torch.empty((n, n_poles), dtype=torch.complex128, device=kappa.device)
    zeta = torch.empty_like(eta)
    status = torch.empty(n, dtype=torch.int32, device=kappa.device)
    _check(lib().gsm_pole_fit(n, n_poles, n_div, C.c_void_p(kappa.data_ptr()), C.c_void_p(xi.data_ptr()),
                              C.c_void_p(eta.data_ptr()), C.c_void_p(zeta.data_ptr()),
                              C.c_void_p(status.data_ptr()), _stream(stream)))
    return eta, zeta, status


def fresnel_indices(eps, k_hat):
    """The two refractive indices (ascending) of direction k_hat in a medium
    of real symmetric permittivity eps (gsm_fresnel_indices, host)."""
    e = (C.c_double * 9)(*np.asarray(eps, dtype=np.float64).reshape(9))
    k = (C.c_double * 3)(*np.asarray(k_hat, dtype=np.float64).reshape(3))
    out = (C.c_double * 2)()
    _check(lib().gsm_fresnel_indices(e, k, out))
    return np.array([out[0], out[1]])


def fresnel_fit(k_hats, n_pairs, diagonal=False):
    """(eps 3x3, rms) fitted to directions and their two indices each
    (gsm_fresnel_fit, host); diagonal: principal axes along x, y, z."""
    k = np.ascontiguousarray(k_hats, dtype=np.float64).reshape(-1, 3)
    n = np.ascontiguousarray(n_pairs, dtype=np.float64).reshape(-1, 2)
    if k.shape[0] != n.shape[0]:
        raise ValueError("one pair of indices per direction")
    out = (C.c_double * 9)()
    rms = C.c_double()
    _check(lib().gsm_fresnel_fit(k.shape[0], k.ctypes.data_as(C.POINTER(C.c_double)),
                                 n.ctypes.data_as(C.POINTER(C.c_double)), 1 if diagonal else 0, out,
                                 C.byref(rms)))
    return np.array(out[:]).reshape(3, 3), rms.value


class SolveInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("refinements", C.c_int32),
                ("fft_size", C.c_int32), ("reorth", C.c_int32), ("reserved", C.c_int32),
                ("rel_residual", C.c_double), ("eps_b", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class KernelStat(C.Structure):
    _fields_ = [("name", C.c_char * 40), ("launches", C.c_int64), ("ms", C.c_double),
                ("bytes", C.c_double), ("flops", C.c_double), ("bytes_min", C.c_double)]


class GsmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libgsm status {status}: {msg}")
        self.status = status


_lib = None

_SIGS = {
    "gsm_version": (C.c_int, []),
    "gsm_strerror": (C.c_char_p, [C.c_int]),
    "gsm_last_error": (C.c_char_p, []),
    "gsm_solver_opts_default": (None, [C.POINTER(SolverOpts)]),
    "gsm_fft_size": (C.c_int, [C.POINTER(C.c_int32)]),
    "gsm_plan_validate": (C.c_int, [C.POINTER(Geometry), C.POINTER(PlanOpts), C.c_int32,
                                    C.POINTER(Instance)]),
    "gsm_basis_eps": (C.c_int, [C.c_void_p, C.POINTER(Instance), C.POINTER(C.c_double)]),
    "gsm_plan": (C.c_int, [C.POINTER(Geometry), C.POINTER(PlanOpts), C.POINTER(C.c_void_p)]),
    "gsm_plan_destroy": (C.c_int, [C.c_void_p]),
    "gsm_plan_shapes": (C.c_int, [C.POINTER(ShapeBody), C.POINTER(PlanOpts), C.POINTER(C.c_void_p)]),
    "gsm_plan_from_coeffs": (C.c_int, [C.POINTER(CoeffBody), C.POINTER(PlanOpts), C.POINTER(C.c_void_p)]),
    "gsm_plan_coefficients": (C.c_int, [C.c_void_p, C.c_void_p]),
    "gsm_plan_inverse_coefficients": (C.c_int, [C.c_void_p, C.c_void_p]),
    "gsm_plan_graph_stats": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "gsm_plan_tuning": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_int32),
                                  C.POINTER(C.c_int32)]),
    "gsm_plan_contrast_grid": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.c_int32, C.c_void_p]),
    "gsm_workspace_size": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(Instance),
                                     C.POINTER(SolverOpts), C.POINTER(C.c_size_t)]),
    "gsm_solve": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(Instance), C.POINTER(SolverOpts),
                            C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(SolveInfo), C.c_void_p]),
    "gsm_apply": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(Instance), C.c_int32, C.c_int32,
                            C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "gsm_apply_static": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(Instance), C.c_int32, C.c_int32,
                                   C.c_void_p, C.c_void_p, C.c_void_p]),
    "gsm_eff_tensor": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(Instance), C.POINTER(SolverOpts),
                                 C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                 C.POINTER(SolveInfo), C.c_void_p]),
    "gsm_solve_adjoint": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(Instance), C.POINTER(SolverOpts),
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                    C.POINTER(SolveInfo), C.c_void_p]),
    "gsm_eff_tensor_vjp": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(Instance),
                                     C.POINTER(SolverOpts), C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_size_t, C.POINTER(SolveInfo),
                                     C.c_void_p]),
    "gsm_allocation_stats": (C.c_int, [C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "gsm_pole_workspace_size": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(PoleQuery),
                                          C.POINTER(SolverOpts), C.POINTER(C.c_size_t)]),
    "gsm_pole_search": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(PoleQuery), C.POINTER(SolverOpts),
                                  C.c_void_p, C.c_size_t, C.POINTER(PoleResult), C.c_void_p]),
    "gsm_pole_fit": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_void_p, C.c_void_p]),
    "gsm_fresnel_indices": (C.c_int, [C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "gsm_fresnel_fit": (C.c_int, [C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int32,
                                  C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "gsm_profile_begin": (C.c_int, []),
    "gsm_profile_begin_only": (C.c_int, [C.c_char_p]),
    "gsm_profile_begin_sampled": (C.c_int, [C.c_char_p, C.c_int32]),
    "gsm_profile_end": (C.c_int, [C.POINTER(KernelStat), C.c_int32, C.POINTER(C.c_int32)]),
}


def lib():
    """Load libgsm.so (raises if it has not been built).

    PyTorch is imported first: its wheel carries its own HIP runtime
    (libamdhip64.so.7), and the library must bind to that same runtime to
    use torch's device memory and streams.  Loaded before torch, the library
    would pull in the system's copy and torch would then fail to find a
    device."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (see above)
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "python paper_1501_01752_amd/csrc/build.py")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status, allow_warn=True):
    if status < 0 or (status > 0 and not allow_warn):
        raise GsmError(status, lib().gsm_last_error().decode())
    return status


def profile_begin(only=None, every=1):
    """Start per-launch timing of every kernel class, or of the class `only`
    (a name such as "pass_b", both precisions); every > 1 times one launch in
    `every` of each class."""
    if every != 1:
        _check(lib().gsm_profile_begin_sampled(None if only is None else only.encode(), every))
    elif only is None:
        _check(lib().gsm_profile_begin())
    else:
        _check(lib().gsm_profile_begin_only(only.encode()))


def profile_end():
    """Per-kernel-class {launches, ms, bytes, flops, bytes_min} since profile_begin()."""
    out = (KernelStat * 64)()
    n = C.c_int32()
    _check(lib().gsm_profile_end(out, 64, C.byref(n)))
    return {out[i].name.decode(): dict(launches=out[i].launches, ms=out[i].ms, bytes=out[i].bytes,
                                      flops=out[i].flops, bytes_min=out[i].bytes_min)
            for i in range(min(n.value, 64))}


def allocation_stats():
    """(allocations, bytes) the library has made since it was loaded (device
    hipMalloc and pinned host hipHostMalloc)."""
    n, b = C.c_int64(), C.c_int64()
    _check(lib().gsm_allocation_stats(C.byref(n), C.byref(b)))
    return n.value, b.value


def default_opts(**kw):
    o = SolverOpts()
    lib().gsm_solver_opts_default(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def fft_size(M):
    return lib().gsm_fft_size((C.c_int32 * 3)(*M))


def make_instance(wavelength, k_inc, M, drives=((1.0, 0.0, 0.0),), eps_b=0.0):
    """One (omega, k) point; drives are up to three complex 3-vectors."""
    inst = Instance()
    inst.wavelength = float(wavelength)
    for a in range(3):
        inst.k_inc[a] = float(k_inc[a])
        inst.M[a] = int(M[a])
    drives = list(drives)
    inst.n_drive = len(drives)
    for d, vec in enumerate(drives):
        for c in range(3):
            z = complex(vec[c])
            inst.pol[d][2 * c] = z.real
            inst.pol[d][2 * c + 1] = z.imag
    inst.eps_b = float(eps_b)
    return inst


def instances_array(insts):
    arr = (Instance * len(insts))()
    for i, x in enumerate(insts):
        arr[i] = x
    return arr


def system_sizes(insts, three=False):
    out = []
    for x in insts:
        n = 3 * (2 * x.M[0] + 1) * (2 * x.M[1] + 1) * (2 * x.M[2] + 1)
        out += [n] * (3 if three else x.n_drive)
    return out


def _stream(stream):
    import torch
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(stream)


class Plan:
    """Owning handle of a gsm_plan_t built from a voxel body (the default),
    or from an analytic shape body (Plan.from_shapes) or given Fourier
    coefficients (Plan.from_coeffs)."""

    def __init__(self, eps, period=(1.0, 1.0, 1.0), m_max=(15, 15, 15), device=0, autotune=False,
                 tune_cache=None, _body=None):
        o = PlanOpts()
        for a in range(3):
            o.m_max[a] = int(m_max[a])
        o.device = device
        o.flags = GSM_PLAN_AUTOTUNE if autotune else 0
        self._tune_cache = None if tune_cache is None else os.fsencode(tune_cache)
        o.tune_cache = self._tune_cache
        h = C.c_void_p()
        if _body is None:
            self.eps = np.ascontiguousarray(eps, dtype=np.float64)
            vz, vy, vx = self.eps.shape
            g = Geometry()
            for a in range(3):
                g.period[a] = float(period[a])
            g.nvox[0], g.nvox[1], g.nvox[2] = vx, vy, vz
            g.eps = self.eps.ctypes.data_as(C.POINTER(C.c_double))
            _check(lib().gsm_plan(C.byref(g), C.byref(o), C.byref(h)), allow_warn=False)
        else:
            kind, body = _body
            fn = lib().gsm_plan_shapes if kind == "shapes" else lib().gsm_plan_from_coeffs
            _check(fn(C.byref(body), C.byref(o), C.byref(h)), allow_warn=False)
        self.handle = h
        self.m_max = tuple(int(m) for m in m_max)
        self.period = tuple(float(p) for p in period)
        self.device = device
        self._ws = None

    @classmethod
    def from_shapes(cls, period, eps_host, shapes, m_max=(15, 15, 15), device=0, autotune=False,
                    tune_cache=None):
        """Plan of a host eps_host with inclusions: shapes are dicts
        {"kind": "sphere" | "ellipsoid" | "box", "centre": (x, y, z),
        "size": radius | semi-axes | half-sides, "eps": value}."""
        arr = (Shape * max(len(shapes), 1))()
        for i, sh in enumerate(shapes):
            arr[i].kind = _SHAPE_KINDS[sh["kind"]]
            size = np.broadcast_to(np.asarray(sh["size"], dtype=np.float64), (3,))
            for a in range(3):
                arr[i].centre[a] = float(sh["centre"][a])
                arr[i].size[a] = float(size[a])
            arr[i].eps = float(sh["eps"])
        b = ShapeBody()
        for a in range(3):
            b.period[a] = float(period[a])
        b.eps_host = float(eps_host)
        b.n_shapes = len(shapes)
        b.shapes = arr
        return cls(None, period, m_max, device, autotune, tune_cache, _body=("shapes", b))

    @classmethod
    def from_coeffs(cls, period, coef, eps_min, eps_max, m_max=(15, 15, 15), device=0, autotune=False,
                    tune_cache=None, coef_inv=None):
        """Plan from Fourier coefficients c_n, a complex array of shape
        (2Nz+1, 2Ny+1, 2Nx+1) indexed n + N (N_a >= 2 m_max[a]); coef_inv
        (same layout), the coefficients of 1/eps, enables the H system."""
        c = np.ascontiguousarray(coef, dtype=np.complex128)
        ci = None if coef_inv is None else np.ascontiguousarray(coef_inv, dtype=np.complex128)
        b = CoeffBody()
        b.coef_inv = None if ci is None else ci.ctypes.data_as(C.POINTER(C.c_double))
        for a in range(3):
            b.period[a] = float(period[a])
        b.n_max[0], b.n_max[1], b.n_max[2] = ((c.shape[2] - 1) // 2, (c.shape[1] - 1) // 2,
                                              (c.shape[0] - 1) // 2)
        b.coef = c.ctypes.data_as(C.POINTER(C.c_double))
        b.eps_min, b.eps_max = float(eps_min), float(eps_max)
        return cls(None, period, m_max, device, autotune, tune_cache, _body=("coeffs", b))

    def close(self):
        if getattr(self, "handle", None):
            lib().gsm_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tuning(self, M, precision=GSM_MIXED):
        """(families per FFT stage [pass A, pass B rows, pass B columns,
        pass C], tuned?) for the orders M in that precision."""
        fam = (C.c_int32 * 4)()
        tuned = C.c_int32()
        _check(lib().gsm_plan_tuning(self.handle, (C.c_int32 * 3)(*M), precision, fam, C.byref(tuned)))
        return list(fam), bool(tuned.value)

    def graph_stats(self):
        """(launch graphs captured, graph launches) of this plan so far."""
        cap, run = C.c_int64(), C.c_int64()
        _check(lib().gsm_plan_graph_stats(self.handle, C.byref(cap), C.byref(run)))
        return cap.value, run.value

    def coefficients(self):
        n = [4 * m + 1 for m in self.m_max]
        out = np.zeros((n[2], n[1], n[0]), dtype=np.complex128)
        _check(lib().gsm_plan_coefficients(self.handle, out.ctypes.data_as(C.c_void_p)))
        return out

    def inverse_coefficients(self):
        """Coefficients of 1/eps (the H-field system's), layout of coefficients()."""
        n = [4 * m + 1 for m in self.m_max]
        out = np.zeros((n[2], n[1], n[0]), dtype=np.complex128)
        _check(lib().gsm_plan_inverse_coefficients(self.handle, out.ctypes.data_as(C.c_void_p)))
        return out

    def contrast_grid(self, M, P):
        out = np.zeros((P, P, P), dtype=np.float64)
        _check(lib().gsm_plan_contrast_grid(self.handle, (C.c_int32 * 3)(*M), P,
                                            out.ctypes.data_as(C.c_void_p)))
        return out

    def basis_eps(self, inst):
        v = C.c_double()
        _check(lib().gsm_basis_eps(self.handle, C.byref(inst), C.byref(v)))
        return v.value

    def workspace(self, insts, opts):
        import torch
        arr = instances_array(insts)
        nb = C.c_size_t()
        _check(lib().gsm_workspace_size(self.handle, len(insts), arr, C.byref(opts), C.byref(nb)))
        need = int(nb.value)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(max(need, 1), dtype=torch.uint8, device=f"cuda:{self.device}")
        return self._ws

    def solve(self, insts, opts=None, x0=None, stream=None):
        """Solve every (instance, drive); returns (E as a flat complex128 torch
        tensor on the device, list of per-system info dicts, status)."""
        import torch
        opts = opts or default_opts()
        arr = instances_array(insts)
        n = sum(system_sizes(insts))
        E = torch.empty(n, dtype=torch.complex128, device=f"cuda:{self.device}")
        info = (SolveInfo * len(system_sizes(insts)))()
        if x0 is not None:
            x0 = x0.contiguous()
            opts.x0 = x0.data_ptr()
        ws = self.workspace(insts, opts)
        st = lib().gsm_solve(self.handle, len(insts), arr, C.byref(opts), C.c_void_p(ws.data_ptr()),
                             ws.numel(), C.c_void_p(E.data_ptr()), info, _stream(stream))
        _check(st)
        return E, [i.as_dict() for i in info], st

    def apply(self, insts, x, precision=GSM_FP64, mode=GSM_APPLY_FORWARD, stream=None):
        """y = A x (or A^H x) for every (instance, drive) vector in x."""
        import torch
        opts = default_opts(precision=precision)
        arr = instances_array(insts)
        x = x.contiguous()
        want = torch.complex128 if precision == GSM_FP64 else torch.complex64
        if x.dtype != want:
            raise TypeError(f"x must be {want}")
        y = torch.empty_like(x)
        ws = self.workspace(insts, opts)
        _check(lib().gsm_apply(self.handle, len(insts), arr, precision, mode, C.c_void_p(x.data_ptr()),
                               C.c_void_p(y.data_ptr()), C.c_void_p(ws.data_ptr()), ws.numel(),
                               _stream(stream)))
        return y

    def apply_static(self, insts, x, y=None, precision=GSM_FP64, mode=GSM_APPLY_FORWARD, stream=None):
        """y = A x (or A^H x) through gsm_apply_static: no workspace, the
        library's static scratch array instead.  y may be given (preallocated
        by the caller); otherwise it is allocated here, outside the call."""
        import torch
        arr = instances_array(insts)
        x = x.contiguous()
        want = torch.complex128 if precision == GSM_FP64 else torch.complex64
        if x.dtype != want:
            raise TypeError(f"x must be {want}")
        if y is None:
            y = torch.empty_like(x)
        elif y.dtype != want or y.numel() != x.numel() or not y.is_contiguous():
            raise TypeError("y must be a contiguous tensor of x's dtype and size")
        _check(lib().gsm_apply_static(self.handle, len(insts), arr, precision, mode,
                                      C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                      _stream(stream)))
        return y

    def pole_search(self, queries, opts=None, stream=None):
        """Mesh solves and pole fit of every query (gsm_pole_search); returns
        (list of result dicts, status)."""
        import torch
        opts = opts or default_opts()
        arr = (PoleQuery * len(queries))(*queries)
        nb = C.c_size_t()
        _check(lib().gsm_pole_workspace_size(self.handle, len(queries), arr, C.byref(opts), C.byref(nb)))
        ws = torch.empty(max(int(nb.value), 1), dtype=torch.uint8, device=f"cuda:{self.device}")
        out = (PoleResult * len(queries))()
        st = lib().gsm_pole_search(self.handle, len(queries), arr, C.byref(opts), C.c_void_p(ws.data_ptr()),
                                   ws.numel(), out, _stream(stream))
        _check(st)
        return [r.as_dict() for r in out], st

    def fresnel_tensor(self, wavelength, M, n_lo, n_hi, opts=None, n_poles=5, n_div=10, eps_b=0.0,
                       stream=None):
        """The effective tensor from propagation constants, for lattices
        whose principal axes are the lattice axes: pole searches along x, y
        and z with the two transverse drives each (xi = the driven component
        of the zeroth order; one call), the indices of the dominant poles
        with n in [n_lo, n_hi], and the diagonal tensor fitted to the three
        index pairs (gsm_fresnel_fit).  Each principal index is measured
        along two directions; the fit's rms shows how far they differ
        (spatial dispersion at a finite period).  Returns (eps 3x3, rms,
        index pairs [3][2] (along x, y, z; the two drives in axis order),
        the six pole-search results)."""
        k0 = 2 * np.pi / wavelength
        queries = []
        for ax in range(3):
            for other in (a for a in range(3) if a != ax):
                k_hat = [0.0, 0.0, 0.0]
                k_hat[ax] = 1.0
                drive = [0.0, 0.0, 0.0]
                drive[other] = 1.0
                queries.append(make_pole_query(wavelength, k_hat, M, n_lo * k0, n_hi * k0, drive=drive,
                                               component=other, n_poles=n_poles, n_div=n_div, eps_b=eps_b))
        res, st = self.pole_search(queries, opts, stream)
        missing = [i for i, r in enumerate(res) if r["best"] < 0]
        if missing:
            raise GsmError(GSM_E_SINGULAR, f"no pole with n in [{n_lo}, {n_hi}] for queries {missing}")
        pairs = np.array([[res[2 * ax]["n_eff"], res[2 * ax + 1]["n_eff"]] for ax in range(3)])
        eps, rms = fresnel_fit(np.eye(3), pairs, diagonal=True)
        return eps, rms, pairs, res

    def solve_adjoint(self, insts, rhs, opts=None, stream=None):
        """lambda = A^-H rhs for every (instance, drive); rhs complex128 (device)."""
        import torch
        opts = opts or default_opts()
        arr = instances_array(insts)
        rhs = rhs.contiguous()
        lam = torch.empty_like(rhs)
        info = (SolveInfo * len(system_sizes(insts)))()
        ws = self.workspace(insts, opts)
        st = lib().gsm_solve_adjoint(self.handle, len(insts), arr, C.byref(opts), C.c_void_p(rhs.data_ptr()),
                                     C.c_void_p(lam.data_ptr()), C.c_void_p(ws.data_ptr()), ws.numel(), info,
                                     _stream(stream))
        _check(st)
        return lam, [i.as_dict() for i in info], st

    def eff_tensor_vjp(self, insts, E_save, eps_eff, gbar, opts=None, stream=None):
        """dL/d eps_voxel (numpy, shape of the voxel body) for gbar = dL/d conj(eps_eff)."""
        import torch
        opts = opts or default_opts()
        arr = instances_array(insts)
        ee = np.ascontiguousarray(eps_eff, dtype=np.complex128)
        gb = np.ascontiguousarray(gbar, dtype=np.complex128)
        grad = torch.zeros(self.eps.size, dtype=torch.float64, device=f"cuda:{self.device}")
        info = (SolveInfo * (3 * len(insts)))()
        ws = self.workspace(insts, opts)
        st = lib().gsm_eff_tensor_vjp(self.handle, len(insts), arr, C.byref(opts), C.c_void_p(E_save.data_ptr()),
                                      ee.ctypes.data_as(C.c_void_p), gb.ctypes.data_as(C.c_void_p),
                                      C.c_void_p(grad.data_ptr()), C.c_void_p(ws.data_ptr()), ws.numel(), info,
                                      _stream(stream))
        _check(st)
        return grad.reshape(self.eps.shape), [i.as_dict() for i in info], st

    def eff_tensor(self, insts, opts=None, save_fields=False, stream=None):
        """eps_eff = D0 E0^-1 per instance (numpy [n, 3, 3] complex128)."""
        import torch
        opts = opts or default_opts()
        arr = instances_array(insts)
        out = np.zeros((len(insts), 3, 3), dtype=np.complex128)
        info = (SolveInfo * (3 * len(insts)))()
        E = None
        if save_fields:
            E = torch.empty(sum(system_sizes(insts, three=True)), dtype=torch.complex128,
                            device=f"cuda:{self.device}")
        ws = self.workspace(insts, opts)
        st = lib().gsm_eff_tensor(self.handle, len(insts), arr, C.byref(opts),
                                  out.ctypes.data_as(C.c_void_p),
                                  C.c_void_p(E.data_ptr() if E is not None else 0),
                                  C.c_void_p(ws.data_ptr()), ws.numel(), info, _stream(stream))
        _check(st)
        return out, E, [i.as_dict() for i in info], st


def _eff_tensor_function():
    import torch

    class EffTensorFn(torch.autograd.Function):
        """eps_eff (complex128 [n_inst, 3, 3]) of a voxel permittivity tensor.

        forward: builds a plan from eps (real, shape (Vz, Vy, Vx)) and calls
        gsm_eff_tensor; backward: gsm_eff_tensor_vjp (three adjoint solves per
        instance, real-space correlation, exact voxel-box images).  torch
        passes grad = 2 dL/d conj(eps_eff) for a real loss, so gbar = grad / 2.
        The basis permittivity is held fixed between forward and backward.
        """

        @staticmethod
        def forward(ctx, eps, period, m_max, insts, opts):
            e = eps.detach().cpu().numpy()
            plan = Plan(e, period, m_max, device=eps.device.index or 0 if eps.is_cuda else 0)
            fixed = []
            for x in insts:
                y = Instance()
                C.pointer(y)[0] = x
                if y.eps_b <= 0:
                    y.eps_b = plan.basis_eps(y)
                fixed.append(y)
            ee, E, info, st = plan.eff_tensor(fixed, opts, save_fields=True)
            ctx.plan, ctx.insts, ctx.opts, ctx.E, ctx.ee = plan, fixed, opts, E, ee
            ctx.eps_device = eps.device
            return torch.from_numpy(ee).to(eps.device)

        @staticmethod
        def backward(ctx, grad):
            gbar = (grad.detach().cpu().numpy() / 2.0).astype(np.complex128)
            g, _, _ = ctx.plan.eff_tensor_vjp(ctx.insts, ctx.E, ctx.ee, gbar, ctx.opts)
            return g.to(ctx.eps_device), None, None, None, None

    return EffTensorFn


_EFF_FN = None


def eff_tensor_fn():
    """The torch.autograd.Function computing eps_eff from voxel permittivities."""
    global _EFF_FN
    if _EFF_FN is None:
        _EFF_FN = _eff_tensor_function()
    return _EFF_FN
