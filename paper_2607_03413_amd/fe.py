"""Thin ctypes binding of libfe.so (include/fe.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Device buffers are torch tensors (``torch`` is used for device
memory and streams); calls run on torch's current stream.  The library must
be built (``paper_2607_03413_amd/build_lib.py``); importing this module
without it raises immediately -- there is no fallback path.
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfe.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libfe.so is not built: run paper_2607_03413_amd/build_lib.py")
_lib = ctypes.CDLL(LIB_PATH)

F64, F32 = 0, 1
GEOM_CARTESIAN, GEOM_DEFORMED = 0, 1
SMOOTH_JACOBI, SMOOTH_CHEB_FDM = 0, 1
STATUS = {0: "FE_OK", -1: "FE_EINVAL", -2: "FE_ENOMEM", -3: "FE_EHIP", -4: "FE_ENOTCONV",
          -5: "FE_EBREAKDOWN", -6: "FE_EUNSUPPORTED"}


class FeError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class _Coef(ctypes.Structure):
    _fields_ = [("n_modes", ctypes.c_int), ("modes", ctypes.POINTER(ctypes.c_int32)),
                ("amp", ctypes.POINTER(ctypes.c_double)), ("phase", ctypes.POINTER(ctypes.c_double))]


class _Desc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("degree", ctypes.c_int), ("n", ctypes.c_int), ("geometry", ctypes.c_int),
                ("deform_amp", ctypes.c_double), ("coef", _Coef), ("bc", ctypes.c_int), ("n_coarse", ctypes.c_int)]


class PcgOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxit", ctypes.c_int), ("nu_pre", ctypes.c_int),
                ("nu_post", ctypes.c_int), ("smoother", ctypes.c_int), ("cheb_degree", ctypes.c_int),
                ("cheb_ratio", ctypes.c_double), ("cheb_lmax", ctypes.c_double), ("omega", ctypes.c_double),
                ("inner", ctypes.c_int), ("factors", ctypes.c_int), ("flexible", ctypes.c_int),
                ("precond", ctypes.c_int), ("stop", ctypes.c_int)]


class PcgReport(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("converged", ctypes.c_int), ("relres", ctypes.c_double),
                ("energy0", ctypes.c_double), ("energy", ctypes.c_double), ("t_setup", ctypes.c_double),
                ("t_solve", ctypes.c_double)]


_vp, _i, _i64, _d = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
_SIGS = {
    "fe_problem_create": (_i, [ctypes.POINTER(_Desc), _vp, ctypes.POINTER(_vp)]),
    "fe_problem_destroy": (None, [_vp]),
    "fe_num_cells": (_i64, [_vp]),
    "fe_cellvec_len": (_i64, [_vp]),
    "fe_num_dofs": (_i64, [_vp]),
    "fe_num_levels": (_i, [_vp]),
    "fe_level_cells_1d": (_i, [_vp, _i]),
    "fe_gather": (_i, [_vp, _vp, _vp, _i, _vp]),
    "fe_assemble": (_i, [_vp, _vp, _vp, _i, _vp]),
    "fe_dss": (_i, [_vp, _i, _vp, _i, _i, _vp]),
    "fe_apply": (_i, [_vp, _vp, _vp, _i, _vp]),
    "fe_apply_level": (_i, [_vp, _i, _vp, _vp, _i, _vp]),
    "patch_fdm_inverse": (_i, [_vp, _vp, _vp, _i, _i, _vp]),
    "patch_fdm_inverse_level": (_i, [_vp, _i, _vp, _vp, _i, _i, _vp]),
    "fe_patch_prepare": (_i, [_vp, _i, _i, _i, _vp]),
    "fe_noalloc_scratch_bytes": (ctypes.c_size_t, []),
    "patch_fdm_inverse_noalloc": (_i, [_vp, _i, _vp, _vp, _i, _i, _vp]),
    "fe_prolongate_add": (_i, [_vp, _i, _vp, _vp, _i, _vp]),
    "fe_restrict_residual": (_i, [_vp, _i, _vp, _vp, _vp, _i, _vp]),
    "fe_jacobi_sweep": (_i, [_vp, _i, _vp, _vp, _vp, _d, _i, _i, _vp]),
    "fe_rhs_manufactured": (_i, [_vp, _vp, _vp]),
    "fe_dot": (_i, [_vp, _vp, _vp, _i, ctypes.POINTER(_d), _vp]),
    "fe_assembled_norm2": (_i, [_vp, _vp, _i, ctypes.POINTER(_d), _vp]),
    "fe_pcg_default_opts": (None, [ctypes.POINTER(PcgOpts)]),
    "pcg_solve": (_i, [_vp, _vp, _vp, ctypes.POINTER(PcgOpts), ctypes.POINTER(PcgReport), _vp]),
    "fe_vcycle": (_i, [_vp, _vp, _vp, ctypes.POINTER(PcgOpts), _i, _vp]),
    "fe_mg_iterate": (_i, [_vp, _vp, _vp, ctypes.POINTER(PcgOpts), _i, _vp, _vp, _vp]),
    "fe_estimate_lmax": (_i, [_vp, _i, _i, _i, _i, ctypes.POINTER(_d), _vp]),
    "fe_mlp_num_params": (_i, []),
    "fe_num_patches": (_i64, [_vp, _i]),
    "fe_patch_features": (_i, [_vp, _i, _vp, _vp]),
    "fe_patch_inner_tensor": (_i, [_vp, _i, _vp, _vp]),
    "fe_patch_fit_targets": (_i, [_vp, _i, _i, _vp, _vp]),
    "fe_mlp_set_params": (_i, [_vp, _vp, _vp]),
    "fe_mlp_get_params": (_i, [_vp, _vp, _vp]),
    "fe_mlp_forward": (_i, [_vp, _vp, _vp, _i, _vp]),
    "fe_mlp_loss_grad": (_i, [_vp, _vp, _vp, _i, _vp, ctypes.POINTER(_d), _vp]),
    "fe_mlp_adam_step": (_i, [_vp, _vp, _d, _vp]),
    "fe_mlp_train": (_i, [_vp, _vp, _vp, _i, _i, _i, _d, ctypes.c_uint64, ctypes.POINTER(_d), _vp]),
    "fe_prof_enable": (None, [_i]),
    "fe_set_graphs": (None, [_i]),
    "fe_prof_reset": (None, []),
    "fe_prof_query": (_i, [ctypes.c_char_p, ctypes.POINTER(_i), ctypes.POINTER(_d)]),
    "fe_last_error": (ctypes.c_char_p, []),
    "fe_adaptive_create": (_i, [_vp, _vp, ctypes.POINTER(_vp)]),
    "fe_adaptive_destroy": (None, [_vp]),
    "fe_adaptive_num_levels": (_i, [_vp]),
    "fe_adaptive_level_cells": (_i64, [_vp, _i]),
    "fe_adaptive_level_offset": (_i64, [_vp, _i]),
    "fe_adaptive_active_cells": (_i64, [_vp]),
    "fe_adaptive_level_info": (_i, [_vp, _i, _vp, _vp]),
    "fe_adaptive_brick_neighbors": (_i, [_vp, _i, _vp, _vp]),
    "fe_adaptive_edge_mask": (_i, [_vp, _i, _vp, _vp]),
    "fe_adaptive_dss": (_i, [_vp, _i, _vp, _i, _vp]),
    "fe_adaptive_dinv": (_i, [_vp, _i, _vp, _vp]),
    "fe_adaptive_apply": (_i, [_vp, _vp, _vp, _vp]),
    "fe_adaptive_prolongate_add": (_i, [_vp, _i, _vp, _vp, _vp]),
    "fe_adaptive_restrict_add": (_i, [_vp, _i, _vp, _vp, _vp, _vp]),
    "fe_adaptive_rhs_manufactured": (_i, [_vp, _vp, _vp]),
    "fe_adaptive_precondition": (_i, [_vp, _vp, _vp, ctypes.POINTER(PcgOpts), _vp]),
    "fe_adaptive_pcg": (_i, [_vp, _vp, _vp, ctypes.POINTER(PcgOpts), ctypes.POINTER(PcgReport), _vp]),
    "fe_set_metric_mode": (_i, [_vp, _i, _vp]),
    "fe_multiblock_create": (_i, [_i, _i, _vp, ctypes.POINTER(_vp)]),
    "fe_multiblock_destroy": (None, [_vp]),
    "fe_multiblock_len": (_i64, [_vp]),
    "fe_multiblock_num_nodes": (_i64, [_vp]),
    "fe_multiblock_counts": (_i, [_vp, _vp]),
    "fe_multiblock_dss": (_i, [_vp, _vp, _i, _i, _vp]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def _check(st):
    if st != 0:
        raise FeError(st, _lib.fe_last_error().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dt(t):
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError("cell-wise tensors must be float64 or float32")


def _ptr(t, n=None, name="tensor"):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("%s must be a contiguous device tensor" % name)
    if n is not None and t.numel() != n:
        raise ValueError("%s has %d entries, expected %d" % (name, t.numel(), n))
    return ctypes.c_void_p(t.data_ptr())


def default_opts(**kw):
    o = PcgOpts()
    _lib.fe_pcg_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


class Problem:
    """Owns an fe_problem handle (see include/fe.h)."""

    def __init__(self, dim, degree, n, geometry=GEOM_CARTESIAN, bc=1, deform_amp=0.0, coef=None, n_coarse=0):
        d = _Desc()
        d.dim, d.degree, d.n, d.geometry = dim, degree, n, geometry
        d.deform_amp, d.bc, d.n_coarse = deform_amp, bc, n_coarse
        self._keep = []
        if coef is not None:
            modes, amps, phases = coef
            m = np.ascontiguousarray(modes, dtype=np.int32)
            a = np.ascontiguousarray(amps, dtype=np.float64)
            ph = np.ascontiguousarray(phases, dtype=np.float64)
            self._keep += [m, a, ph]
            d.coef.n_modes = len(a)
            d.coef.modes = m.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            d.coef.amp = a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            d.coef.phase = ph.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        h = ctypes.c_void_p()
        _check(_lib.fe_problem_create(ctypes.byref(d), _stream(), ctypes.byref(h)))
        self.h = h
        self.dim, self.degree, self.n = dim, degree, n
        self.K = degree + 1
        self.n_cells = _lib.fe_num_cells(h)
        self.len = _lib.fe_cellvec_len(h)
        self.n_dofs = _lib.fe_num_dofs(h)
        self.n_levels = _lib.fe_num_levels(h)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            _lib.fe_problem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # shapes
    def level_n(self, level):
        return _lib.fe_level_cells_1d(self.h, level)

    def level_len(self, level):
        n = self.level_n(level)
        return n ** self.dim * self.K ** self.dim

    def cellvec(self, dtype=torch.float64, level=-1):
        ln = self.len if level == -1 else self.level_len(level)
        return torch.zeros(ln, dtype=dtype, device="cuda")

    # operations
    def gather(self, xg, xc):
        _check(_lib.fe_gather(self.h, _ptr(xg, self.n_dofs, "x_glob"), _ptr(xc, self.len, "x_cell"), _dt(xc),
                              _stream()))

    def assemble(self, yc, yg):
        _check(_lib.fe_assemble(self.h, _ptr(yc, self.len, "y_cell"), _ptr(yg, self.n_dofs, "y_glob"), _dt(yc),
                                _stream()))

    def dss(self, v, averaging=False, level=-1):
        _check(_lib.fe_dss(self.h, level, _ptr(v, name="v"), 1 if averaging else 0, _dt(v), _stream()))

    def apply(self, x, y, level=-1):
        _check(_lib.fe_apply_level(self.h, level, _ptr(x, name="x"), _ptr(y, name="y"), _dt(x), _stream()))

    def patch_inverse(self, r, z, factors=0, level=-1):
        _check(_lib.patch_fdm_inverse_level(self.h, level, _ptr(r, name="r"), _ptr(z, name="z"), _dt(r), factors,
                                            _stream()))

    def set_metric_mode(self, mode):
        """0: the deformed operator streams the stored metric; 1: it forms the metric in the kernel."""
        _check(_lib.fe_set_metric_mode(self.h, int(mode), _stream()))

    def patch_prepare(self, dtype=torch.float64, factors=0, level=-1):
        _check(_lib.fe_patch_prepare(self.h, level, F64 if dtype == torch.float64 else F32, factors, _stream()))

    def prolongate_add(self, fine_level, ec, ef):
        _check(_lib.fe_prolongate_add(self.h, fine_level, _ptr(ec, name="e_coarse"), _ptr(ef, name="e_fine"),
                                      _dt(ef), _stream()))

    def restrict_residual(self, fine_level, bf, vf, bc):
        _check(_lib.fe_restrict_residual(self.h, fine_level, _ptr(bf, name="b_fine"), _ptr(vf, name="v_fine"),
                                         _ptr(bc, name="b_coarse"), _dt(bf), _stream()))

    def jacobi_sweep(self, level, b, u, v, omega, u_is_zero=False):
        _check(_lib.fe_jacobi_sweep(self.h, level, _ptr(b, name="b"), _ptr(u, name="u"), _ptr(v, name="v"),
                                    float(omega), 1 if u_is_zero else 0, _dt(u), _stream()))

    def rhs_manufactured(self, b):
        _check(_lib.fe_rhs_manufactured(self.h, _ptr(b, self.len, "b"), _stream()))

    def dot(self, a, b):
        out = ctypes.c_double()
        _check(_lib.fe_dot(self.h, _ptr(a, self.len, "a"), _ptr(b, self.len, "b"), _dt(a), ctypes.byref(out),
                           _stream()))
        return out.value

    def assembled_norm2(self, r):
        out = ctypes.c_double()
        _check(_lib.fe_assembled_norm2(self.h, _ptr(r, self.len, "r"), _dt(r), ctypes.byref(out), _stream()))
        return out.value

    def vcycle(self, b, e, opts):
        _check(_lib.fe_vcycle(self.h, _ptr(b, self.len, "b"), _ptr(e, self.len, "e"), ctypes.byref(opts), _dt(b),
                              _stream()))

    def mg_iterate(self, b, x, opts, cycles):
        """x <- x + MG(b - A x), `cycles` times; returns (eta, res) per cycle (numpy)."""
        eta = np.zeros(max(cycles, 1))
        res = np.zeros(max(cycles, 1))
        _check(_lib.fe_mg_iterate(self.h, _ptr(b, self.len, "b"), _ptr(x, self.len, "x"), ctypes.byref(opts),
                                  cycles, eta.ctypes.data_as(ctypes.c_void_p), res.ctypes.data_as(ctypes.c_void_p),
                                  _stream()))
        return eta[:cycles], res[:cycles]

    def estimate_lmax(self, level=-1, factors=0, steps=15, smoother=SMOOTH_CHEB_FDM):
        out = ctypes.c_double()
        _check(_lib.fe_estimate_lmax(self.h, level, smoother, factors, steps, ctypes.byref(out), _stream()))
        return out.value

    # learned per-patch factors
    def num_patches(self, level=-1):
        return _lib.fe_num_patches(self.h, level)

    def patch_features(self, level=-1):
        out = torch.empty(max(self.num_patches(level), 1) * 64, dtype=torch.float64, device="cuda")
        _check(_lib.fe_patch_features(self.h, level, _ptr(out), _stream()))
        return out[: self.num_patches(level) * 64].view(-1, 64)

    def patch_inner_tensor(self, level=-1):
        out = torch.empty(max(self.num_patches(level), 1) * 64, dtype=torch.float64, device="cuda")
        _check(_lib.fe_patch_inner_tensor(self.h, level, _ptr(out), _stream()))
        return out[: self.num_patches(level) * 64].view(-1, 64)

    def patch_fit_targets(self, level=-1, sweeps=30):
        out = torch.empty(max(self.num_patches(level), 1) * 12, dtype=torch.float64, device="cuda")
        _check(_lib.fe_patch_fit_targets(self.h, level, sweeps, _ptr(out), _stream()))
        return out[: self.num_patches(level) * 12].view(-1, 12)

    def mlp_set_params(self, params):
        _check(_lib.fe_mlp_set_params(self.h, _ptr(params, MLP_PARAMS, "params"), _stream()))

    def mlp_get_params(self):
        out = torch.empty(MLP_PARAMS, dtype=torch.float32, device="cuda")
        _check(_lib.fe_mlp_get_params(self.h, _ptr(out), _stream()))
        return out

    def mlp_forward(self, X):
        X = X.float().contiguous()
        Y = torch.empty(X.shape[0], 12, dtype=torch.float32, device="cuda")
        _check(_lib.fe_mlp_forward(self.h, _ptr(X), _ptr(Y), X.shape[0], _stream()))
        return Y

    def mlp_loss_grad(self, X, T):
        X, T = X.float().contiguous(), T.float().contiguous()
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device="cuda")
        loss = ctypes.c_double()
        _check(_lib.fe_mlp_loss_grad(self.h, _ptr(X), _ptr(T), X.shape[0], _ptr(g), ctypes.byref(loss), _stream()))
        return loss.value, g

    def mlp_adam_step(self, grad, lr=1e-3):
        _check(_lib.fe_mlp_adam_step(self.h, _ptr(grad, MLP_PARAMS, "grad"), float(lr), _stream()))

    def mlp_train(self, X, T, epochs, batch=256, lr=1e-3, seed=0):
        X, T = X.float().contiguous(), T.float().contiguous()
        loss = ctypes.c_double()
        _check(_lib.fe_mlp_train(self.h, _ptr(X), _ptr(T), X.shape[0], epochs, batch, float(lr), seed,
                                 ctypes.byref(loss), _stream()))
        return loss.value

    def pcg_solve(self, b, x, opts=None, raise_on_error=True):
        if opts is None:
            opts = default_opts()
        rep = PcgReport()
        st = _lib.pcg_solve(self.h, _ptr(b, self.len, "b"), _ptr(x, self.len, "x"), ctypes.byref(opts),
                            ctypes.byref(rep), _stream())
        if st != 0 and raise_on_error:
            _check(st)
        return {"status": STATUS.get(st, st), "iters": rep.iters, "converged": bool(rep.converged),
                "relres": rep.relres, "energy0": rep.energy0, "energy": rep.energy, "t_setup": rep.t_setup,
                "t_solve": rep.t_solve}


FEATURE_SPHERE, FEATURE_POINT = 0, 1


class _AdaptiveDesc(ctypes.Structure):
    _fields_ = [("degree", ctypes.c_int), ("global_refinements", ctypes.c_int),
                ("adaptive_refinements", ctypes.c_int), ("feature", ctypes.c_int),
                ("center", ctypes.c_double * 3), ("radius", ctypes.c_double), ("band", ctypes.c_double)]


class Adaptive:
    """Owns an fe_adaptive handle: the locally refined hierarchy (see include/fe.h).
    Vectors of the active mesh are FP64 device tensors in level layout."""

    def __init__(self, degree, global_refinements, adaptive_refinements, feature=FEATURE_SPHERE,
                 center=(0.5, 0.5, 0.5), radius=0.3125, band=1.0):
        d = _AdaptiveDesc()
        d.degree, d.global_refinements, d.adaptive_refinements = degree, global_refinements, adaptive_refinements
        d.feature, d.radius, d.band = feature, radius, band
        for a in range(3):
            d.center[a] = center[a]
        h = ctypes.c_void_p()
        _check(_lib.fe_adaptive_create(ctypes.cast(ctypes.pointer(d), ctypes.c_void_p), _stream(), ctypes.byref(h)))
        self.h = h
        self.degree, self.K = degree, degree + 1
        self.n_levels = _lib.fe_adaptive_num_levels(h)
        self.offsets = [_lib.fe_adaptive_level_offset(h, l) for l in range(self.n_levels + 1)]
        self.len = self.offsets[-1]
        self.active_cells = _lib.fe_adaptive_active_cells(h)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            _lib.fe_adaptive_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def level_cells(self, level):
        return _lib.fe_adaptive_level_cells(self.h, level)

    def level_info(self, level):
        n = self.level_cells(level)
        coords = np.zeros((n, 3), dtype=np.int32)
        refined = np.zeros(n, dtype=np.uint8)
        _check(_lib.fe_adaptive_level_info(self.h, level, coords.ctypes.data_as(ctypes.c_void_p),
                                           refined.ctypes.data_as(ctypes.c_void_p)))
        return coords, refined.astype(bool)

    def brick_neighbors(self, level):
        nb = self.level_cells(level) // 8
        nbr = np.zeros((nb, 6), dtype=np.int32)
        par = np.zeros(nb, dtype=np.int32)
        _check(_lib.fe_adaptive_brick_neighbors(self.h, level, nbr.ctypes.data_as(ctypes.c_void_p),
                                                par.ctypes.data_as(ctypes.c_void_p)))
        return nbr, par

    def vec(self):
        return torch.zeros(self.len, dtype=torch.float64, device="cuda")

    def level_vec(self, level):
        return torch.zeros(self.offsets[level + 1] - self.offsets[level], dtype=torch.float64, device="cuda")

    def edge_mask(self, level):
        m = self.level_vec(level)
        _check(_lib.fe_adaptive_edge_mask(self.h, level, _ptr(m), _stream()))
        return m

    def dss(self, level, v, averaging=False):
        _check(_lib.fe_adaptive_dss(self.h, level, _ptr(v), 1 if averaging else 0, _stream()))

    def dinv(self, level):
        d = self.level_vec(level)
        _check(_lib.fe_adaptive_dinv(self.h, level, _ptr(d), _stream()))
        return d

    def apply(self, x, y):
        _check(_lib.fe_adaptive_apply(self.h, _ptr(x, self.len, "x"), _ptr(y, self.len, "y"), _stream()))

    def prolongate_add(self, fine_level, ec, ef):
        _check(_lib.fe_adaptive_prolongate_add(self.h, fine_level, _ptr(ec), _ptr(ef), _stream()))

    def restrict_add(self, fine_level, bf, vf, bc):
        _check(_lib.fe_adaptive_restrict_add(self.h, fine_level, _ptr(bf), _ptr(vf), _ptr(bc), _stream()))

    def rhs_manufactured(self, b):
        _check(_lib.fe_adaptive_rhs_manufactured(self.h, _ptr(b, self.len, "b"), _stream()))

    def precondition(self, r, z, opts):
        _check(_lib.fe_adaptive_precondition(self.h, _ptr(r, self.len, "r"), _ptr(z, self.len, "z"),
                                             ctypes.byref(opts), _stream()))

    def pcg(self, b, x, opts, raise_on_error=True):
        rep = PcgReport()
        st = _lib.fe_adaptive_pcg(self.h, _ptr(b, self.len, "b"), _ptr(x, self.len, "x"), ctypes.byref(opts),
                                  ctypes.byref(rep), _stream())
        if st != 0 and raise_on_error:
            _check(st)
        return {"status": STATUS.get(st, st), "iters": rep.iters, "converged": bool(rep.converged),
                "relres": rep.relres, "energy0": rep.energy0, "energy": rep.energy, "t_setup": rep.t_setup,
                "t_solve": rep.t_solve}


class MultiBlock:
    """Owns an fe_multiblock handle: the 7-block atlas and its DSS (see include/fe.h)."""

    def __init__(self, degree, n):
        h = ctypes.c_void_p()
        _check(_lib.fe_multiblock_create(degree, n, _stream(), ctypes.byref(h)))
        self.h = h
        self.degree, self.n = degree, n
        self.len = _lib.fe_multiblock_len(h)
        self.n_nodes = _lib.fe_multiblock_num_nodes(h)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            _lib.fe_multiblock_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def counts(self):
        c = np.zeros(3, dtype=np.int64)
        _check(_lib.fe_multiblock_counts(self.h, c.ctypes.data_as(ctypes.c_void_p)))
        return {"face_pairs": int(c[0]), "line_dofs": int(c[1]), "vertex_dofs": int(c[2])}

    def dss(self, v, averaging=False):
        _check(_lib.fe_multiblock_dss(self.h, _ptr(v, self.len, "v"), 1 if averaging else 0, _dt(v), _stream()))


def set_graphs(on=True):
    """Replay the MG-PCG preconditioner as a HIP graph (default) or keep it eager."""
    _lib.fe_set_graphs(1 if on else 0)


def prof_enable(on=True):
    _lib.fe_prof_enable(1 if on else 0)


def prof_reset():
    _lib.fe_prof_reset()


def prof_query(name):
    c, t = ctypes.c_int(), ctypes.c_double()
    _check(_lib.fe_prof_query(name.encode(), ctypes.byref(c), ctypes.byref(t)))
    return c.value, t.value


def last_error():
    return _lib.fe_last_error().decode()


MLP_PARAMS = _lib.fe_mlp_num_params()
