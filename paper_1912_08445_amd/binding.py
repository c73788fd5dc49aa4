"""ctypes binding of libnlte.so: argument marshalling only.

Host-pointer calls take numpy arrays; *_dev calls take torch CUDA (HIP) tensors and
run on torch's current stream unless one is given.  Every computation happens in the
library's HIP kernels; nothing here falls back to the CPU.  If libnlte.so has not
been built, importing this module raises ImportError.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# NLTE_LIB selects another build of the library (same ABI); default: the in-tree one
LIB_PATH = os.environ.get("NLTE_LIB") or os.path.join(_HERE, "libnlte.so")

NLTE_OK = 0
NLTE_E_INVALID_ARG = -1
NLTE_E_STATE = -2
NLTE_E_OOM = -3
NLTE_E_HIP = -4
NLTE_W_NOT_CONVERGED = 1
NLTE_W_NONPHYSICAL = 2
PREC_FP64 = 0
PREC_FP32_BULK = 1

# every entry point declared in include/nlte.h
EXPORTS = (
    "nlte_default_params", "nlte_create", "nlte_destroy", "nlte_last_error", "nlte_set_species",
    "nlte_set_models", "nlte_set_rays", "nlte_set_quadrature", "nlte_set_params", "nlte_trace",
    "nlte_get_ray", "nlte_get_order", "nlte_get_point_cost", "nlte_trace_stats", "nlte_get_line_width_speed", "nlte_lte", "nlte_lte_dev",
    "nlte_formal_solve", "nlte_formal_solve_dev", "nlte_formal_solve_noalloc_dev", "nlte_stateq", "nlte_stateq_dev",
    "nlte_formal_solve_band", "nlte_stateq_band", "nlte_set_rays_healpix", "nlte_get_rays", "nlte_set_scattering", "nlte_set_scattering_dipole", "nlte_formal_solve_scat",
    "nlte_formal_solve_scat_dev", "nlte_scattering_field",
    "nlte_run_ali", "nlte_run_ali_dev", "nlte_get_model_status", "nlte_autotune", "nlte_get_launch",
    "nlte_kernel_stats", "nlte_reset_kernel_stats", "nlte_executed_steps",
    "nlte_default_train_params", "nlte_mlp_param_count", "nlte_features", "nlte_features_dev",
    "nlte_mlp_init", "nlte_mlp_set_weights", "nlte_mlp_get_weights", "nlte_mlp_set_norm",
    "nlte_mlp_forward", "nlte_mlp_loss_grad", "nlte_mlp_train", "nlte_mlp_train_dev",
    "nlte_mlp_predict", "nlte_mlp_predict_dev", "nlte_mlp_rows_dev", "nlte_run_ali_warm", "nlte_run_ali_warm_dev", "nlte_image", "nlte_image_dev",
)

MLP_INPUTS = 8
MLP_HIDDEN = 128


class Params(C.Structure):
    _fields_ = [("t_cmb", C.c_double), ("f_sub", C.c_double), ("tol", C.c_double),
                ("max_iter", C.c_int), ("use_alo", C.c_int), ("precision", C.c_int),
                ("profile", C.c_int), ("use_graph", C.c_int), ("lines_per_lane", C.c_int),
                ("waves_per_simd", C.c_int), ("persistent", C.c_int), ("ng_every", C.c_int),
                ("alo_band", C.c_int), ("long_segments", C.c_int), ("stage_nodes", C.c_int),
                ("tile_points", C.c_int)]


class AliReport(C.Structure):
    _fields_ = [("iterations", C.c_int), ("converged", C.c_int),
                ("max_change", C.c_double * 1024), ("mean_change", C.c_double * 1024),
                ("n_models_converged", C.c_int64),
                ("n_fallback", C.c_int64), ("n_kept", C.c_int64), ("n_maser", C.c_int64),
                ("ms_total", C.c_double), ("n_ng_steps", C.c_int), ("n_ng_rejected", C.c_int64),
                ("n_band", C.c_int)]


class TrainParams(C.Structure):
    _fields_ = [("steps", C.c_int64), ("batch", C.c_int), ("lr", C.c_double), ("beta1", C.c_double),
                ("beta2", C.c_double), ("eps", C.c_double)]


class NlteError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libnlte error {code}: {msg}")
        self.code = code


def load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "or python paper_1912_08445_amd/build.py")
    # torch's ROCm build carries its own HIP runtime with the same soname as the system's
    # and asks for it by its unversioned name.  Loading torch first makes the library bind
    # to that runtime instance; in the other order a second runtime would be loaded and
    # torch would find no device.  Device tensors and streams are torch's, so there must
    # be one runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.nlte_default_params.argtypes = [C.POINTER(Params)]
    L.nlte_default_params.restype = None
    L.nlte_create.argtypes = [C.POINTER(vp), C.c_int]
    L.nlte_destroy.argtypes = [vp]
    L.nlte_destroy.restype = None
    L.nlte_last_error.argtypes = [vp]
    L.nlte_last_error.restype = C.c_char_p
    L.nlte_set_species.argtypes = [vp, C.c_int, vp, vp, dbl, C.c_int, vp, vp, vp, C.c_int, vp, vp,
                                   C.c_int, vp, vp]
    L.nlte_set_models.argtypes = [vp, C.c_int, vp, vp, vp, vp, vp, vp, vp, C.c_int, vp, vp]
    L.nlte_set_rays.argtypes = [vp, C.c_int, vp]
    L.nlte_set_quadrature.argtypes = [vp, C.c_int, vp, vp]
    L.nlte_set_params.argtypes = [vp, C.POINTER(Params)]
    L.nlte_trace.argtypes = [vp]
    L.nlte_get_ray.argtypes = [vp, i64, C.c_int, vp, C.c_int, C.POINTER(C.c_int)]
    L.nlte_get_order.argtypes = [vp, vp]
    L.nlte_get_point_cost.argtypes = [vp, vp]
    L.nlte_trace_stats.argtypes = [vp, C.POINTER(i64), C.POINTER(C.c_int), C.POINTER(i64)]
    L.nlte_get_line_width_speed.argtypes = [vp, vp]
    L.nlte_lte.argtypes = [vp, vp]
    L.nlte_lte_dev.argtypes = [vp, vp, vp]
    L.nlte_formal_solve.argtypes = [vp, vp, vp, vp, vp]
    L.nlte_formal_solve_dev.argtypes = [vp, vp, vp, vp, vp, vp]
    L.nlte_formal_solve_noalloc_dev.argtypes = [vp, vp, vp, vp, vp, vp]
    L.nlte_stateq.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.nlte_stateq_dev.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    L.nlte_formal_solve_band.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    L.nlte_stateq_band.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, C.POINTER(C.c_int), C.POINTER(C.c_int)]
    L.nlte_set_scattering.argtypes = [vp, vp]
    L.nlte_set_scattering_dipole.argtypes = [vp, vp]
    L.nlte_set_rays_healpix.argtypes = [vp, C.c_int]
    L.nlte_get_rays.argtypes = [vp, C.POINTER(C.c_int), vp]
    L.nlte_formal_solve_scat.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.nlte_formal_solve_scat_dev.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    L.nlte_scattering_field.argtypes = [vp, vp]
    L.nlte_run_ali.argtypes = [vp, vp, vp, C.POINTER(AliReport)]
    L.nlte_run_ali_dev.argtypes = [vp, vp, vp, C.POINTER(AliReport), vp]
    L.nlte_get_model_status.argtypes = [vp, vp, vp, vp]
    L.nlte_autotune.argtypes = [vp, C.c_char_p, C.c_int, C.c_char_p, C.c_int]
    L.nlte_get_launch.argtypes = [vp] + [C.POINTER(C.c_int)] * 6
    L.nlte_kernel_stats.argtypes = [vp, C.c_char_p, C.POINTER(dbl), C.POINTER(i64)]
    L.nlte_reset_kernel_stats.argtypes = [vp]
    L.nlte_executed_steps.argtypes = [vp, C.POINTER(i64)]
    L.nlte_default_train_params.argtypes = [C.POINTER(TrainParams)]
    L.nlte_default_train_params.restype = None
    L.nlte_mlp_param_count.argtypes = [C.c_int]
    L.nlte_features.argtypes = [vp, vp]
    L.nlte_features_dev.argtypes = [vp, vp, vp]
    L.nlte_mlp_init.argtypes = [vp, C.c_int, C.c_uint64]
    L.nlte_mlp_set_weights.argtypes = [vp, C.c_int, vp]
    L.nlte_mlp_get_weights.argtypes = [vp, vp]
    L.nlte_mlp_set_norm.argtypes = [vp, vp, vp]
    L.nlte_mlp_forward.argtypes = [vp, vp, i64, vp]
    L.nlte_mlp_loss_grad.argtypes = [vp, vp, vp, i64, vp, C.POINTER(dbl)]
    L.nlte_mlp_train.argtypes = [vp, vp, vp, i64, C.POINTER(TrainParams), vp]
    L.nlte_mlp_train_dev.argtypes = [vp, vp, vp, i64, C.POINTER(TrainParams), vp, vp]
    L.nlte_mlp_predict.argtypes = [vp, vp, C.POINTER(i64)]
    L.nlte_mlp_predict_dev.argtypes = [vp, vp, C.POINTER(i64), vp]
    L.nlte_mlp_rows_dev.argtypes = [vp, vp, vp, vp, vp]
    L.nlte_image.argtypes = [vp, vp, C.c_int, C.c_int, C.c_int, vp, vp, vp]
    L.nlte_image_dev.argtypes = [vp, vp, C.c_int, C.c_int, C.c_int, vp, vp, vp, vp]
    L.nlte_run_ali_warm.argtypes = [vp, vp, C.POINTER(AliReport), C.POINTER(C.c_int)]
    L.nlte_run_ali_warm_dev.argtypes = [vp, vp, C.POINTER(AliReport), C.POINTER(C.c_int), vp]
    for name in EXPORTS:
        fn = getattr(L, name)   # AttributeError if the library lacks a declared entry point
        if name not in ("nlte_destroy", "nlte_default_params", "nlte_last_error",
                        "nlte_default_train_params"):
            fn.restype = C.c_int
    L.nlte_mlp_param_count.restype = C.c_int64
    return L


_L = None


def lib():
    global _L
    if _L is None:
        _L = load()
    return _L


def _p(a):
    return None if a is None else a.ctypes.data


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _tp(t):
    """Device pointer of a torch tensor (must be contiguous and on the GPU)."""
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("device calls need contiguous GPU tensors")
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream


class Solver:
    """One library context: species, model(s), rays, quadrature, parameters."""

    def __init__(self, device: int = 0):
        self.L = lib()
        h = C.c_void_p()
        rc = self.L.nlte_create(C.byref(h), device)
        if rc != 0:
            raise NlteError(rc, "nlte_create failed (no HIP device?)")
        self.h = h
        self._keep = []
        self.params = Params()
        self.L.nlte_default_params(C.byref(self.params))

    def close(self):
        if getattr(self, "h", None):
            self.L.nlte_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc, warn_ok=False):
        if rc < 0 or (rc > 0 and not warn_ok):
            raise NlteError(rc, self.L.nlte_last_error(self.h).decode())
        return rc

    # ---------------------------------------------------------------- inputs
    def set_species(self, sp):
        E, g = _c(sp.energy, np.float64), _c(sp.weight, np.float64)
        up, lo, A = _c(sp.line_up, np.int32), _c(sp.line_lo, np.int32), _c(sp.line_A, np.float64)
        cu, cl = _c(sp.coll_up, np.int32), _c(sp.coll_lo, np.int32)
        T, K = _c(sp.coll_T, np.float64), _c(sp.coll_K, np.float64)
        self._chk(self.L.nlte_set_species(self.h, sp.n_lev, _p(E), _p(g), float(sp.mass), sp.n_lines,
                                          _p(up), _p(lo), _p(A), int(cu.shape[0]), _p(cu), _p(cl),
                                          int(T.shape[0]), _p(T), _p(K)))
        self.n_lev, self.n_lines = sp.n_lev, sp.n_lines

    def set_models(self, model, offsets=None):
        P = model.n_points
        off = _c([0, P] if offsets is None else offsets, np.int64)
        arrs = [_c(model.pos, np.float64), _c(model.vel, np.float64), _c(model.n_h2, np.float64),
                _c(model.temperature, np.float64), _c(model.v_turb, np.float64),
                _c(model.abundance, np.float64)]
        nbr = _c(model.nbr, np.int32)
        bnd = None if model.boundary is None else _c(model.boundary, np.uint8)
        self._chk(self.L.nlte_set_models(self.h, off.shape[0] - 1, _p(off), *[_p(a) for a in arrs],
                                         int(nbr.shape[1]), _p(nbr), _p(bnd)))
        # (recorded only once the library has taken the models: a rejected set leaves both)
        self.P = P
        self.n_models = off.shape[0] - 1

    def set_rays(self, dirs):
        d = _c(dirs, np.float64)
        self._chk(self.L.nlte_set_rays(self.h, d.shape[0], _p(d)))
        self.n_rays = d.shape[0]

    def set_quadrature(self, x, w):
        x, w = _c(x, np.float64), _c(w, np.float64)
        self._chk(self.L.nlte_set_quadrature(self.h, x.shape[0], _p(x), _p(w)))
        self.n_q = x.shape[0]

    def set_params(self, **kw):
        for k, v in kw.items():
            if k == "precision" and isinstance(v, str):
                v = {"fp64": PREC_FP64, "fp32": PREC_FP32_BULK}[v]
            setattr(self.params, k, v)
        self._chk(self.L.nlte_set_params(self.h, C.byref(self.params)))

    def setup(self, workload, trace=True, **params):
        """Species, model(s), rays, quadrature and parameters of a synthetic workload."""
        self.set_species(workload.species)
        self.set_models(workload.model, workload.offsets)
        self.set_rays(workload.rays)
        self.set_quadrature(workload.quad_x, workload.quad_w)
        kw = dict(t_cmb=workload.t_cmb, f_sub=workload.f_sub, max_iter=workload.max_iter,
                  tol=workload.tol)
        kw.update(params)
        self.set_params(**kw)
        if trace:
            self.trace()
        return self

    # ---------------------------------------------------------------- walk
    def trace(self):
        self._chk(self.L.nlte_trace(self.h))

    def get_ray(self, point, ray):
        n = C.c_int()
        self._chk(self.L.nlte_get_ray(self.h, int(point), int(ray), None, 0, C.byref(n)))
        out = np.zeros(max(n.value, 1), dtype=np.int32)
        self._chk(self.L.nlte_get_ray(self.h, int(point), int(ray), _p(out), n.value, C.byref(n)))
        return out[:n.value].copy()

    def order(self):
        """Morton processing order of the points (global indices)."""
        out = np.zeros(self.P, dtype=np.int64)
        self._chk(self.L.nlte_get_order(self.h, _p(out)))
        return out

    def point_cost(self):
        """Elimination steps per frequency from each origin point over all its rays."""
        out = np.zeros(self.P, dtype=np.int64)
        self._chk(self.L.nlte_get_point_cost(self.h, _p(out)))
        return out

    def trace_stats(self):
        """(total cached cells, longest ray, elimination steps per frequency per sweep)"""
        tot, mx, st = C.c_int64(), C.c_int(), C.c_int64()
        self._chk(self.L.nlte_trace_stats(self.h, C.byref(tot), C.byref(mx), C.byref(st)))
        return tot.value, mx.value, st.value

    def line_width_speed(self):
        out = np.zeros(self.P)
        self._chk(self.L.nlte_get_line_width_speed(self.h, _p(out)))
        return out

    # ---------------------------------------------------------------- host calls
    def lte(self):
        out = np.zeros((self.P, self.n_lev))
        self._chk(self.L.nlte_lte(self.h, _p(out)))
        return out

    def formal_solve(self, pops):
        pops = _c(pops, np.float64)
        J = np.zeros((self.P, self.n_lines))
        Je, Ls = np.zeros_like(J), np.zeros_like(J)
        self._chk(self.L.nlte_formal_solve(self.h, _p(pops), _p(J), _p(Je), _p(Ls)))
        return J, Je, Ls

    def stateq(self, pops_old, J, Jeff, L):
        out = np.zeros((self.P, self.n_lev))
        flags = np.zeros(self.P, dtype=np.uint8)
        args = [_c(a, np.float64) for a in (pops_old, J, Jeff, L)]
        self._chk(self.L.nlte_stateq(self.h, *[_p(a) for a in args], _p(out), _p(flags)))
        return out, flags

    def formal_solve_band(self, pops):
        """(J, Jeff, L*, Jb, Ld, Ln) of the band ALO (nlte_formal_solve_band)."""
        pops = _c(pops, np.float64)
        out = [np.zeros((self.P, self.n_lines)) for _ in range(5)]
        Ln = np.zeros((self.P, self.n_lines, self.n_rays))
        self._chk(self.L.nlte_formal_solve_band(self.h, _p(pops), *[_p(a) for a in out], _p(Ln)))
        return (*out, Ln)

    def stateq_band(self, pops_old, J, Jeff, L, Jb, Ld, Ln):
        """(populations, models that kept the band's populations, solver iterations) of the
        coupled band-ALO solve."""
        args = [_c(a, np.float64) for a in (pops_old, J, Jeff, L, Jb, Ld, Ln)]
        out = np.zeros((self.P, self.n_lev))
        used, its = C.c_int(), C.c_int()
        self._chk(self.L.nlte_stateq_band(self.h, *[_p(a) for a in args], _p(out), C.byref(used), C.byref(its)))
        return out, used.value, its.value

    def set_rays_healpix(self, nside):
        """HEALPix pixel centres as the ray set (invalidates the trace)."""
        self._chk(self.L.nlte_set_rays_healpix(self.h, int(nside)))
        self.n_rays = 12 * int(nside) ** 2

    def get_rays(self):
        n = C.c_int()
        self._chk(self.L.nlte_get_rays(self.h, C.byref(n), None))
        out = np.zeros((n.value, 3))
        self._chk(self.L.nlte_get_rays(self.h, C.byref(n), _p(out)))
        return out

    def set_scattering(self, chi_sca=None):
        """Isotropic coherent scattering opacity [P][n_lines] (cm^-1); None clears it."""
        if chi_sca is None:
            self._chk(self.L.nlte_set_scattering(self.h, None))
            return
        self._scat = _c(chi_sca, np.float64)
        self._chk(self.L.nlte_set_scattering(self.h, _p(self._scat)))

    def set_scattering_dipole(self, chi_dip=None):
        """Odd part of the scattering opacity [P][n_lines][3] (cm^-1): the opacity of
        direction n is chi_sca + chi_dip . n; None removes it."""
        if chi_dip is None:
            self._chk(self.L.nlte_set_scattering_dipole(self.h, None))
            return
        d = _c(chi_dip, np.float64)
        self._chk(self.L.nlte_set_scattering_dipole(self.h, _p(d)))

    def formal_solve_scat(self, pops, jnu_in):
        """(J, Jeff, L*, J_nu out) of one formal solve with scattering."""
        pops, jin = _c(pops, np.float64), _c(jnu_in, np.float64)
        J, Je, Ls = (np.zeros((self.P, self.n_lines)) for _ in range(3))
        jout = np.zeros_like(jin)
        self._chk(self.L.nlte_formal_solve_scat(self.h, _p(pops), _p(jin), _p(J), _p(Je), _p(Ls), _p(jout)))
        return J, Je, Ls, jout

    def formal_solve_scat_dev(self, pops, jnu_in, J, Jeff, L, jnu_out, stream=None):
        self._chk(self.L.nlte_formal_solve_scat_dev(self.h, _tp(pops), _tp(jnu_in), _tp(J), _tp(Jeff), _tp(L),
                                                    _tp(jnu_out), _stream(stream)))

    def scattering_field(self):
        """J_nu [P][n_lines][n_q] after the last ALI with scattering."""
        out = np.zeros((self.P, self.n_lines, self.n_q))
        self._chk(self.L.nlte_scattering_field(self.h, _p(out)))
        return out

    def run_ali(self, pops_init=None):
        out = np.zeros((self.P, self.n_lev))
        rep = AliReport()
        pi = None if pops_init is None else _c(pops_init, np.float64)
        rc = self._chk(self.L.nlte_run_ali(self.h, _p(pi), _p(out), C.byref(rep)), warn_ok=True)
        return out, report_dict(rep, rc)

    # ---------------------------------------------------------------- device calls
    def lte_dev(self, pops, stream=None):
        self._chk(self.L.nlte_lte_dev(self.h, _tp(pops), _stream(stream)))

    def formal_solve_dev(self, pops, J, Jeff, L, stream=None):
        self._chk(self.L.nlte_formal_solve_dev(self.h, _tp(pops), _tp(J), _tp(Jeff), _tp(L),
                                               _stream(stream)))

    def formal_solve_noalloc_dev(self, pops, J, Jeff, L, stream=None):
        """formal_solve_dev with the library's fixed per-GPU scratch (allocates nothing)."""
        self._chk(self.L.nlte_formal_solve_noalloc_dev(self.h, _tp(pops), _tp(J), _tp(Jeff), _tp(L),
                                                       _stream(stream)))

    def stateq_dev(self, pops_old, J, Jeff, L, pops_new, flags=None, stream=None):
        self._chk(self.L.nlte_stateq_dev(self.h, _tp(pops_old), _tp(J), _tp(Jeff), _tp(L),
                                         _tp(pops_new), _tp(flags), _stream(stream)))

    def run_ali_dev(self, pops_init, pops_out, stream=None):
        rep = AliReport()
        rc = self._chk(self.L.nlte_run_ali_dev(self.h, _tp(pops_init), _tp(pops_out), C.byref(rep),
                                               _stream(stream)), warn_ok=True)
        return report_dict(rep, rc)

    def model_status(self):
        """(iterations, converged, last max change) per model after run_ali"""
        it = np.zeros(self.n_models, dtype=np.int32)
        cv = np.zeros(self.n_models, dtype=np.uint8)
        ch = np.zeros(self.n_models)
        self._chk(self.L.nlte_get_model_status(self.h, _p(it), _p(cv), _p(ch)))
        return it, cv.astype(bool), ch

    def launch(self):
        """The formal-solve launch the parameters resolve to: dict of lines_per_lane,
        waves_per_simd, long_segments, stage_nodes, persistent, tile_points."""
        v = [C.c_int() for _ in range(6)]
        self._chk(self.L.nlte_get_launch(self.h, *[C.byref(x) for x in v]))
        return dict(zip(("lines_per_lane", "waves_per_simd", "long_segments", "stage_nodes", "persistent",
                         "tile_points"),
                        (x.value for x in v)))

    def autotune(self, cache_path=None, trials=3):
        """Time the formal-solve launch variants and keep the fastest (see nlte_autotune)."""
        buf = C.create_string_buffer(256)
        self._chk(self.L.nlte_autotune(self.h, cache_path.encode() if cache_path else None, int(trials),
                                       buf, 256))
        choice = buf.value.decode()
        fields = dict(kv.split("=") for kv in choice.split() if "=" in kv)
        self.params.lines_per_lane = int(fields["lpl"])
        self.params.waves_per_simd = int(fields["waves"])
        self.params.long_segments = int(fields["long"])
        self.params.stage_nodes = int(fields["ns"])
        self.params.persistent = int(fields["persistent"])
        self.params.tile_points = int(fields["tile"])
        return choice

    # ---------------------------------------------------------------- imaging
    def image(self, pops, ray, line, v_ch):
        """Emergent intensities I [P][n_ch] along `ray` and image-plane coordinates [P][2]."""
        pops = _c(pops, np.float64)
        v = _c(np.atleast_1d(v_ch), np.float64)
        I = np.zeros((self.P, v.shape[0]))
        xy = np.zeros((self.P, 2))
        self._chk(self.L.nlte_image(self.h, _p(pops), int(ray), int(line), v.shape[0], _p(v), _p(I), _p(xy)))
        return I, xy

    def image_dev(self, pops, ray, line, v_ch, I, xy=None, stream=None):
        v = _c(np.atleast_1d(v_ch), np.float64)
        self._chk(self.L.nlte_image_dev(self.h, _tp(pops), int(ray), int(line), v.shape[0], _p(v), _tp(I),
                                        _tp(xy), _stream(stream)))

    # ---------------------------------------------------------------- warm start
    def features(self):
        out = np.zeros((self.P, MLP_INPUTS))
        self._chk(self.L.nlte_features(self.h, _p(out)))
        return out

    def features_dev(self, F, stream=None):
        self._chk(self.L.nlte_features_dev(self.h, _tp(F), _stream(stream)))

    def mlp_init(self, n_out, seed=0):
        self.n_out = int(n_out)
        self._chk(self.L.nlte_mlp_init(self.h, self.n_out, int(seed)))

    def mlp_set_weights(self, theta, n_out):
        t = _c(theta, np.float32)
        if t.shape != (param_count(n_out),):
            raise ValueError("parameter vector has the wrong length")
        self.n_out = int(n_out)
        self._chk(self.L.nlte_mlp_set_weights(self.h, self.n_out, _p(t)))

    def mlp_get_weights(self):
        out = np.zeros(param_count(self.n_out), dtype=np.float32)
        self._chk(self.L.nlte_mlp_get_weights(self.h, _p(out)))
        return out

    def mlp_set_norm(self, mean, std):
        m, s = _c(mean, np.float64), _c(std, np.float64)
        if m.shape != (MLP_INPUTS,) or s.shape != (MLP_INPUTS,):
            raise ValueError("mean and std need 8 entries")
        self._chk(self.L.nlte_mlp_set_norm(self.h, _p(m), _p(s)))

    def mlp_forward(self, X):
        X = _c(X, np.float32)
        Y = np.zeros((X.shape[0], self.n_out), dtype=np.float32)
        self._chk(self.L.nlte_mlp_forward(self.h, _p(X), X.shape[0], _p(Y)))
        return Y

    def mlp_loss_grad(self, X, T):
        X, T = _c(X, np.float32), _c(T, np.float32)
        g = np.zeros(param_count(self.n_out), dtype=np.float32)
        loss = C.c_double()
        self._chk(self.L.nlte_mlp_loss_grad(self.h, _p(X), _p(T), X.shape[0], _p(g), C.byref(loss)))
        return loss.value, g

    def mlp_train(self, X, T, **kw):
        X, T = _c(X, np.float32), _c(T, np.float32)
        tp = train_params(**kw)
        curve = np.zeros(max(tp.steps, 1), dtype=np.float32)
        self._chk(self.L.nlte_mlp_train(self.h, _p(X), _p(T), X.shape[0], C.byref(tp), _p(curve)))
        return curve[:tp.steps]

    def mlp_train_dev(self, X, T, loss_curve=None, stream=None, **kw):
        tp = train_params(**kw)
        self._chk(self.L.nlte_mlp_train_dev(self.h, _tp(X), _tp(T), X.shape[0], C.byref(tp),
                                            _tp(loss_curve), _stream(stream)))

    def mlp_rows_dev(self, pops, X, T, stream=None):
        """Standardised features X [P][8] and targets T [P][n_lev] (float32 GPU tensors)."""
        self._chk(self.L.nlte_mlp_rows_dev(self.h, _tp(pops), _tp(X), _tp(T), _stream(stream)))

    def mlp_predict(self):
        out = np.zeros((self.P, self.n_lev))
        nb = C.c_int64()
        self._chk(self.L.nlte_mlp_predict(self.h, _p(out), C.byref(nb)))
        return out, nb.value

    def mlp_predict_dev(self, pops, stream=None):
        nb = C.c_int64()
        self._chk(self.L.nlte_mlp_predict_dev(self.h, _tp(pops), C.byref(nb), _stream(stream)))
        return nb.value

    def run_ali_warm(self):
        out = np.zeros((self.P, self.n_lev))
        rep = AliReport()
        used = C.c_int()
        rc = self._chk(self.L.nlte_run_ali_warm(self.h, _p(out), C.byref(rep), C.byref(used)), warn_ok=True)
        d = report_dict(rep, rc)
        d["used_network"] = bool(used.value)
        return out, d

    def run_ali_warm_dev(self, pops_out, stream=None):
        rep = AliReport()
        used = C.c_int()
        rc = self._chk(self.L.nlte_run_ali_warm_dev(self.h, _tp(pops_out), C.byref(rep), C.byref(used),
                                                    _stream(stream)), warn_ok=True)
        d = report_dict(rep, rc)
        d["used_network"] = bool(used.value)
        return d

    # ---------------------------------------------------------------- profiling
    def kernel_stats(self, name):
        ms, n = C.c_double(), C.c_int64()
        self._chk(self.L.nlte_kernel_stats(self.h, name.encode(), C.byref(ms), C.byref(n)))
        return ms.value, n.value


    def executed_steps(self):
        """Node-frequency elimination steps the formal-solve kernels executed while
        profiling, since the last reset (a collapsed far-wing segment counts as one)."""
        n = C.c_int64()
        self._chk(self.L.nlte_executed_steps(self.h, C.byref(n)))
        return n.value
    def reset_kernel_stats(self):
        self._chk(self.L.nlte_reset_kernel_stats(self.h))


def param_count(n_out):
    return int(lib().nlte_mlp_param_count(int(n_out)))


def train_params(**kw):
    tp = TrainParams()
    lib().nlte_default_train_params(C.byref(tp))
    for k, v in kw.items():
        setattr(tp, k, v)
    return tp


def report_dict(rep, rc):
    it = rep.iterations
    return dict(status=rc, iterations=it, converged=bool(rep.converged),
                n_models_converged=rep.n_models_converged,
                max_change=list(rep.max_change[:min(it, 1024)]),
                mean_change=list(rep.mean_change[:min(it, 1024)]),
                n_fallback=rep.n_fallback, n_kept=rep.n_kept, n_maser=rep.n_maser,
                ms_total=rep.ms_total, n_ng_steps=rep.n_ng_steps, n_ng_rejected=rep.n_ng_rejected,
                n_band=rep.n_band)
