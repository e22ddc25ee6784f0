"""MI355X boundary-element library for the multiple-domain Helmholtz
transmission problem (PMCHWT, Galerkin P1 triangles).

Thin ctypes binding over the C ABI in ``include/bem.h``; every step of the
computation runs in the HIP library ``libbem_mi355x.so`` (built by
``paper_1910_01011_amd/build.py``).  Importing this package fails loudly if
the library is missing: there is no CPU fallback.

Vectors are complex128 and follow the library's unknown order (per domain:
u_D, then u_N).  A ``Problem`` created with ``device=True`` takes and returns
torch CUDA tensors and runs on the current torch stream; otherwise numpy
arrays on the host.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
# torch ships its own HIP runtime with the same soname as the system one; it
# has to be the one in the process, so torch is loaded before the library.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
# BEM_LIBRARY selects another build of the same library in this directory (the
# host-sanitizer build libbem_mi355x_san.so)
LIB_PATH = os.path.join(_HERE, os.path.basename(os.environ.get("BEM_LIBRARY", "libbem_mi355x.so")))

if not os.path.exists(LIB_PATH):
    raise ImportError(f"paper_1910_01011_amd: HIP library not built ({LIB_PATH}); "
                      "run __graft_entry__.build() or python paper_1910_01011_amd/build.py")

_L = ctypes.CDLL(LIB_PATH)

BEM_OK, BEM_WARN_NOT_CONVERGED = 0, 1
BEM_ERR_INVALID_ARG, BEM_ERR_MESH, BEM_ERR_OOM, BEM_ERR_DEVICE, BEM_ERR_UNSUPPORTED = -1, -2, -3, -4, -5
BEM_OTF, BEM_ASSEMBLED_FP32, BEM_ASSEMBLED_SPLIT_BF16 = 0, 1, 2
BEM_DEVICE_PTRS = 1
BEM_AUTOTUNE = 2
BEM_APPLY_DEFAULT, BEM_APPLY_GEMV, BEM_APPLY_MFMA_FP32, BEM_APPLY_MFMA_SPLIT_BF16 = 0, 1, 2, 3
BEM_APPLY_MFMA_SPLIT_BF16_W4, BEM_APPLY_MFMA_SPLIT_BF16_W8 = 4, 5
BEM_APPLY_HMATRIX = 6
BEM_PLANE_WAVE, BEM_POINT_SOURCES, BEM_PISTON_ARRAY = 0, 1, 2
BEM_PRECOND_NONE, BEM_PRECOND_OSRC, BEM_PRECOND_OSRC_LEFT = 0, 1, 2
BEM_PREC_FP32, BEM_PREC_SPLIT_BF16_FGMRES, BEM_PREC_FP32_MFMA_FGMRES = 0, 1, 2
BEM_PREC_HMATRIX, BEM_PREC_HMATRIX_FGMRES = 3, 4


class bem_complex(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class bem_domain(ctypes.Structure):
    _fields_ = [("vertices", ctypes.POINTER(ctypes.c_double)), ("n_vertices", ctypes.c_int64),
                ("triangles", ctypes.POINTER(ctypes.c_int32)), ("n_triangles", ctypes.c_int64),
                ("k", bem_complex), ("rho", ctypes.c_double)]


class bem_assemble_opts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("far_points", ctypes.c_int), ("ss_order", ctypes.c_int),
                ("device", ctypes.c_int), ("stream", ctypes.c_void_p), ("flags", ctypes.c_uint32)]


class bem_incident(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("n_fields", ctypes.c_int32),
                ("params", ctypes.POINTER(ctypes.c_double)), ("n_params", ctypes.c_int64)]


class bem_solve_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int), ("max_iter", ctypes.c_int),
                ("precond", ctypes.c_int), ("n_pade", ctypes.c_int), ("r_eps", ctypes.c_double),
                ("theta", ctypes.c_double), ("precision", ctypes.c_int), ("inner_tol", ctypes.c_double),
                ("inner_restart", ctypes.c_int), ("inner_max_iter", ctypes.c_int), ("osrc_tol", ctypes.c_double)]


class bem_solve_info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32), ("rel_residual", ctypes.c_double)]


class bem_hmatrix_info(ctypes.Structure):
    _fields_ = [("n_blocks", ctypes.c_int64), ("n_lowrank", ctypes.c_int64), ("n_dense", ctypes.c_int64),
                ("n_admissible", ctypes.c_int64),
                ("bytes", ctypes.c_int64), ("dense_bytes", ctypes.c_int64), ("max_rank", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("build_s", ctypes.c_double)]


_vp = ctypes.c_void_p
_L.bem_assemble.argtypes = [ctypes.POINTER(bem_domain), ctypes.c_int32, bem_complex, ctypes.c_double,
                            ctypes.POINTER(bem_assemble_opts), ctypes.POINTER(_vp)]
_L.bem_apply.argtypes = [_vp, _vp, _vp, ctypes.c_int32]
_L.bem_apply_parts.argtypes = [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_int]
_L.bem_apply_noalloc.argtypes = [_vp, _vp, _vp, ctypes.c_int32]
_L.bem_apply_with.argtypes = [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_int]
_L.bem_apply_single_layer.argtypes = [_vp, _vp, _vp, ctypes.c_int32]
_L.bem_hmatrix_build.argtypes = [_vp, ctypes.c_double, ctypes.c_int32, ctypes.c_double, ctypes.POINTER(bem_hmatrix_info)]
_L.bem_hmatrix_plan.argtypes = [ctypes.POINTER(bem_domain), ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                ctypes.POINTER(ctypes.c_int64)]
_L.bem_rhs.argtypes = [_vp, ctypes.POINTER(bem_incident), _vp]
_L.bem_solve.argtypes = [_vp, ctypes.POINTER(bem_incident), ctypes.POINTER(bem_solve_opts), _vp,
                         ctypes.POINTER(bem_solve_info)]
_L.bem_solve_rhs.argtypes = [_vp, _vp, ctypes.c_int32, ctypes.POINTER(bem_solve_opts), _vp,
                             ctypes.POINTER(bem_solve_info)]
_L.bem_apply_preconditioner.argtypes = [_vp, ctypes.POINTER(bem_solve_opts), _vp, _vp, ctypes.c_int32]
_L.bem_evaluate_field.argtypes = [_vp, _vp, ctypes.POINTER(bem_incident), _vp, ctypes.c_int64, _vp, _vp]
_L.bem_batch_create.argtypes = [ctypes.c_int, ctypes.POINTER(_vp)]
_L.bem_batch_attach.argtypes = [_vp, _vp]
_L.bem_batch_stats.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64)]
_L.bem_batch_set_window.argtypes = [_vp, ctypes.c_double]
_L.bem_batch_destroy.argtypes = [_vp]
_L.bem_batch_destroy.restype = None
_L.bem_num_unknowns.argtypes = [_vp]
_L.bem_num_unknowns.restype = ctypes.c_int64
_L.bem_footprint_bytes.argtypes = [ctypes.POINTER(bem_domain), ctypes.c_int32, ctypes.POINTER(bem_assemble_opts),
                                   ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64)]
_L.bem_last_timings.argtypes = [_vp, ctypes.POINTER(ctypes.c_double)]
_L.bem_pair_launch_shape.argtypes = [_vp, ctypes.POINTER(ctypes.c_int32)]
_L.bem_destroy.argtypes = [_vp]
_L.bem_destroy.restype = None
_L.bem_last_error.restype = ctypes.c_char_p
for _f in ("bem_assemble", "bem_apply", "bem_apply_noalloc", "bem_apply_parts", "bem_apply_with", "bem_apply_single_layer",
           "bem_hmatrix_build", "bem_hmatrix_plan", "bem_rhs", "bem_solve", "bem_solve_rhs",
           "bem_apply_preconditioner", "bem_pair_launch_shape",
           "bem_evaluate_field", "bem_footprint_bytes", "bem_last_timings", "bem_batch_create", "bem_batch_attach",
           "bem_batch_stats", "bem_batch_set_window"):
    getattr(_L, _f).restype = ctypes.c_int

EXPORTED = ["bem_assemble", "bem_apply", "bem_apply_noalloc", "bem_apply_parts", "bem_apply_with", "bem_apply_single_layer",
            "bem_hmatrix_build", "bem_hmatrix_plan", "bem_rhs", "bem_solve", "bem_solve_rhs",
            "bem_apply_preconditioner", "bem_pair_launch_shape",
            "bem_evaluate_field", "bem_num_unknowns", "bem_footprint_bytes", "bem_last_timings",
            "bem_batch_create", "bem_batch_attach", "bem_batch_set_window", "bem_batch_stats", "bem_batch_destroy",
            "bem_destroy", "bem_last_error"]


class BemError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"status {status}: {msg}")
        self.status = status


def _check(status, allow_warn=False):
    if status == BEM_OK or (allow_warn and status == BEM_WARN_NOT_CONVERGED):
        return status
    raise BemError(status, _L.bem_last_error().decode(errors="replace"))


def _domains(domains):
    keep = []
    arr = (bem_domain * len(domains))()
    for i, d in enumerate(domains):
        v = np.ascontiguousarray(d.vertices, dtype=np.float64)
        t = np.ascontiguousarray(d.triangles, dtype=np.int32)
        keep += [v, t]
        arr[i].vertices = v.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        arr[i].n_vertices = v.shape[0]
        arr[i].triangles = t.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        arr[i].n_triangles = t.shape[0]
        k = complex(d.k)
        arr[i].k = bem_complex(k.real, k.imag)
        arr[i].rho = float(d.rho)
    return arr, keep


class Incident:
    """Incident field description (kind + parameter rows, see include/bem.h)."""

    def __init__(self, kind, n_fields, params):
        self.kind = int(kind)
        self.n_fields = int(n_fields)
        self.params = np.ascontiguousarray(params, dtype=np.float64)

    @staticmethod
    def plane_waves(directions, amplitudes=None):
        d = np.atleast_2d(np.asarray(directions, dtype=np.float64))
        a = np.ones(d.shape[0], dtype=np.complex128) if amplitudes is None else np.atleast_1d(amplitudes)
        rows = np.column_stack([d, np.real(a), np.imag(a)])
        return Incident(BEM_PLANE_WAVE, d.shape[0], rows)

    @staticmethod
    def point_sources(positions, amplitudes, fields):
        p = np.atleast_2d(np.asarray(positions, dtype=np.float64))
        a = np.atleast_1d(np.asarray(amplitudes, dtype=np.complex128))
        f = np.atleast_1d(np.asarray(fields))
        rows = np.column_stack([p, a.real, a.imag, f.astype(np.float64)])
        return Incident(BEM_POINT_SOURCES, int(f.max()) + 1, rows)

    @staticmethod
    def pistons(centres, normals, radius, amplitudes, fields):
        c = np.atleast_2d(np.asarray(centres, dtype=np.float64))
        n = np.atleast_2d(np.asarray(normals, dtype=np.float64))
        a = np.broadcast_to(np.asarray(amplitudes, dtype=np.complex128), (c.shape[0],))
        r = np.broadcast_to(np.asarray(radius, dtype=np.float64), (c.shape[0],))
        f = np.atleast_1d(np.asarray(fields))
        rows = np.column_stack([c, n, r, a.real, a.imag, f.astype(np.float64)])
        return Incident(BEM_PISTON_ARRAY, int(f.max()) + 1, rows)

    def _c(self):
        s = bem_incident()
        s.kind = self.kind
        s.n_fields = self.n_fields
        s.params = self.params.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        s.n_params = self.params.shape[0]
        return s


def solve_options(tol=1e-5, restart=100, max_iter=1000, precond=BEM_PRECOND_NONE, n_pade=4, r_eps=0.1,
                  theta=np.pi / 3, precision=BEM_PREC_FP32, inner_tol=1e-3, inner_restart=0, inner_max_iter=0,
                  osrc_tol=0.0):
    return bem_solve_opts(tol, restart, max_iter, precond, n_pade, r_eps, theta, precision, inner_tol,
                          inner_restart, inner_max_iter, osrc_tol)


def footprint_bytes(domains, n_rhs=1, restart=100):
    arr, keep = _domains(domains)
    out = ctypes.c_uint64(0)
    _check(_L.bem_footprint_bytes(arr, len(domains), None, n_rhs, restart, ctypes.byref(out)))
    return int(out.value)


def hmatrix_plan(domains, leaf_vertices=64, eta=1.0):
    """Host-only plan of the hierarchical matrix's trees (``bem_hmatrix_plan``)."""
    arr, keep = _domains(domains)
    out = (ctypes.c_int64 * 4)()
    _check(_L.bem_hmatrix_plan(arr, len(domains), int(leaf_vertices), float(eta), out))
    return {"n_blocks": int(out[0]), "n_admissible": int(out[1]), "n_touching": int(out[2]),
            "n_touching_admissible": int(out[3])}


class Batch:
    """Continuous batching of the operator applies of concurrent solves
    (``bem_batch``): attach problems, then solve them from several threads."""

    def __init__(self, gpu=0):
        self._h = _vp()
        _check(_L.bem_batch_create(int(gpu), ctypes.byref(self._h)))

    def attach(self, problem):
        _check(_L.bem_batch_attach(problem._h, self._h))

    def set_window(self, seconds):
        _check(_L.bem_batch_set_window(self._h, float(seconds)))

    def stats(self):
        out = (ctypes.c_int64 * 6)()
        _check(_L.bem_batch_stats(self._h, out))
        keys = ("dispatches", "applies", "pair_launches", "multi_problem_launches", "max_problems_per_launch",
                "pair_work_items")
        return dict(zip(keys, (int(v) for v in out)))

    def close(self):
        if self._h:
            _L.bem_batch_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Problem:
    """A set-up transmission problem on one GPU (wraps ``bem_problem``)."""

    def __init__(self, domains, k0, rho0=1.0, device=False, ss_order=6, mode=BEM_OTF, stream=None, gpu=0,
                 autotune=False):
        self._h = _vp()
        self.device = bool(device)
        arr, keep = _domains(domains)
        opts = bem_assemble_opts()
        opts.mode = mode
        opts.far_points = 6
        opts.ss_order = ss_order
        opts.device = gpu
        if stream is None and self.device:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        opts.stream = stream or 0
        opts.flags = (BEM_DEVICE_PTRS if self.device else 0) | (BEM_AUTOTUNE if autotune else 0)
        k0 = complex(k0)
        _check(_L.bem_assemble(arr, len(domains), bem_complex(k0.real, k0.imag), float(rho0), ctypes.byref(opts),
                               ctypes.byref(self._h)))
        self.n = int(_L.bem_num_unknowns(self._h))

    @classmethod
    def from_config(cls, problem, **kw):
        return cls(problem.domains, problem.k0, problem.rho0, **kw)

    def close(self):
        if self._h:
            _L.bem_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- vector marshalling -------------------------------------------------
    def _host_in(self, x):
        x = np.ascontiguousarray(x, dtype=np.complex128)
        n_rhs = 1 if x.ndim == 1 else x.shape[0]
        if x.size != n_rhs * self.n:
            raise ValueError(f"expected {self.n} unknowns per right-hand side, got shape {x.shape}")
        return x, n_rhs

    def _dev_in(self, x):
        import torch
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.complex128 and x.is_contiguous()):
            raise TypeError("device problems take contiguous complex128 CUDA tensors")
        n_rhs = 1 if x.dim() == 1 else x.shape[0]
        if x.numel() != n_rhs * self.n:
            raise ValueError(f"expected {self.n} unknowns per right-hand side, got shape {tuple(x.shape)}")
        return x, n_rhs

    def apply(self, x, parts=3, out=None, kernel=BEM_APPLY_DEFAULT):
        """y = A x (Galerkin PMCHWT matrix, weak form); parts: 1 far, 2 singular, 3 both;
        kernel: BEM_APPLY_* choice for assembled problems."""
        if self.device:
            import torch
            x, n_rhs = self._dev_in(x)
            y = torch.empty_like(x) if out is None else out
            xp, yp = x.data_ptr(), y.data_ptr()
        else:
            x, n_rhs = self._host_in(x)
            y = np.empty_like(x)
            xp, yp = x.ctypes.data, y.ctypes.data
        if kernel == BEM_APPLY_DEFAULT:
            _check(_L.bem_apply_parts(self._h, xp, yp, n_rhs, parts))
        else:
            _check(_L.bem_apply_with(self._h, xp, yp, n_rhs, kernel))
        return y

    def apply_noalloc(self, x, out=None):
        """y = A x through ``bem_apply_noalloc`` (device problems on the fly: the
        apply's scratch is the library's file-scope device array, nothing is
        allocated by the call)."""
        if not self.device:
            raise TypeError("bem_apply_noalloc takes device vectors: create the problem with device=True")
        import torch
        x, n_rhs = self._dev_in(x)
        y = torch.empty_like(x) if out is None else out
        _check(_L.bem_apply_noalloc(self._h, x.data_ptr(), y.data_ptr(), n_rhs))
        return y

    def apply_single_layer(self, x, out=None):
        """y = V_k0 x (Galerkin single-layer matrix on the union of all boundaries);
        x has one value per vertex (domain order), rows = right-hand sides."""
        nv = self.n // 2
        if self.device:
            import torch
            if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.complex128 and x.is_contiguous()):
                raise TypeError("device problems take contiguous complex128 CUDA tensors")
            n_rhs = 1 if x.dim() == 1 else x.shape[0]
            if x.numel() != n_rhs * nv:
                raise ValueError(f"expected {nv} vertex values per right-hand side, got shape {tuple(x.shape)}")
            y = torch.empty_like(x) if out is None else out
            _check(_L.bem_apply_single_layer(self._h, x.data_ptr(), y.data_ptr(), n_rhs))
            return y
        x = np.ascontiguousarray(x, dtype=np.complex128)
        n_rhs = 1 if x.ndim == 1 else x.shape[0]
        if x.size != n_rhs * nv:
            raise ValueError(f"expected {nv} vertex values per right-hand side, got shape {x.shape}")
        y = np.empty_like(x)
        _check(_L.bem_apply_single_layer(self._h, x.ctypes.data, y.ctypes.data, n_rhs))
        return y

    def rhs(self, incident):
        inc = incident._c()
        if self.device:
            import torch
            b = torch.empty((incident.n_fields, self.n), dtype=torch.complex128, device="cuda")
            _check(_L.bem_rhs(self._h, ctypes.byref(inc), b.data_ptr()))
            return b
        b = np.empty((incident.n_fields, self.n), dtype=np.complex128)
        _check(_L.bem_rhs(self._h, ctypes.byref(inc), b.ctypes.data))
        return b

    def solve(self, b, options=None):
        """Solve A u = b (rows of b are right-hand sides). Returns (u, infos)."""
        opts = options or solve_options()
        if self.device:
            import torch
            b, n_rhs = self._dev_in(b)
            u = torch.empty_like(b)
            infos = (bem_solve_info * n_rhs)()
            _check(_L.bem_solve_rhs(self._h, b.data_ptr(), n_rhs, ctypes.byref(opts), u.data_ptr(), infos), True)
        else:
            b, n_rhs = self._host_in(b)
            u = np.empty_like(b)
            infos = (bem_solve_info * n_rhs)()
            _check(_L.bem_solve_rhs(self._h, b.ctypes.data, n_rhs, ctypes.byref(opts), u.ctypes.data, infos), True)
        return u, [dict(iterations=i.iterations, converged=bool(i.converged), rel_residual=i.rel_residual)
                   for i in infos]

    def precondition(self, y, options):
        """OSRC preconditioner applied to residual vectors y (rows = vectors)."""
        if self.device:
            import torch
            y, n_rhs = self._dev_in(y)
            out = torch.empty_like(y)
            _check(_L.bem_apply_preconditioner(self._h, ctypes.byref(options), y.data_ptr(), out.data_ptr(), n_rhs))
            return out
        y, n_rhs = self._host_in(y)
        out = np.empty_like(y)
        _check(_L.bem_apply_preconditioner(self._h, ctypes.byref(options), y.ctypes.data, out.ctypes.data, n_rhs))
        return out

    def evaluate_field(self, u, points, incident=None):
        inc = incident._c() if incident is not None else None
        n_fields = incident.n_fields if incident is not None else 1
        if self.device:
            import torch
            pts = points.contiguous().to(dtype=torch.float64)
            npnt = pts.shape[0]
            field = torch.empty((n_fields, npnt), dtype=torch.complex128, device="cuda")
            region = torch.empty(npnt, dtype=torch.int32, device="cuda")
            _check(_L.bem_evaluate_field(self._h, u.data_ptr(), ctypes.byref(inc) if inc else None, pts.data_ptr(),
                                         npnt, field.data_ptr(), region.data_ptr()))
            return field, region
        u = np.ascontiguousarray(u, dtype=np.complex128)
        pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
        field = np.empty((n_fields, pts.shape[0]), dtype=np.complex128)
        region = np.empty(pts.shape[0], dtype=np.int32)
        _check(_L.bem_evaluate_field(self._h, u.ctypes.data, ctypes.byref(inc) if inc else None, pts.ctypes.data,
                                     pts.shape[0], field.ctypes.data, region.ctypes.data))
        return field, region

    def hmatrix_build(self, eps=1e-6, leaf_vertices=64, eta=1.0):
        """Hierarchical-matrix compression (ACA) of the operator; returns its statistics.
        Applied with apply(..., kernel=BEM_APPLY_HMATRIX), solved with precision=BEM_PREC_HMATRIX."""
        info = bem_hmatrix_info()
        _check(_L.bem_hmatrix_build(self._h, float(eps), int(leaf_vertices), float(eta), ctypes.byref(info)))
        return {f: getattr(info, f) for f, _ in bem_hmatrix_info._fields_ if f != "pad"}

    def pair_launch_shape(self):
        """(test points per lane, trial splits) of the pair kernel."""
        out = (ctypes.c_int32 * 2)()
        _check(_L.bem_pair_launch_shape(self._h, out))
        return int(out[0]), int(out[1])

    def timings(self):
        """(apply, pair kernel, scatter + singular pass, gather) in ms of the last apply."""
        out = (ctypes.c_double * 4)()
        _check(_L.bem_last_timings(self._h, out))
        return tuple(out)
