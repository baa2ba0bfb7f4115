"""ctypes binding of libsnrt (``include/snrt.h``): argument marshalling only.

Every function here has the name of the C entry point it calls and does nothing but convert
arguments: host arrays become FP64 / int32 pointers, device arrays (torch tensors or raw
integer addresses) become ``void*``, and a non-zero status raises :class:`SnrtError` with
the library's own message.  Nothing here computes any part of the step.

The library is loaded from this package directory; if it is missing the import of any
entry point raises -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsnrt.so")

SNRT_OK = 0
SNRT_E_ARG = -1
SNRT_E_SHAPE = -2
SNRT_E_ALIAS = -3
SNRT_E_UNSUPPORTED = -4
SNRT_E_HIP = -5
SNRT_E_OOM = -6
SNRT_E_NONFINITE = -7

SNRT_FP32 = 0
SNRT_BF16X3 = 1
SNRT_BF16X1 = 2
SNRT_BF16X2 = 3
SNRT_FP16X3 = 4

SNRT_REORDER_HILBERT = 0
SNRT_NO_REORDER = 1
SNRT_BC_DIRICHLET = 0
SNRT_BC_NEUMANN = 1
SNRT_MAX_NQ = 1024

# every symbol include/snrt.h declares
EXPORTS = [
    "snrt_abi_version", "snrt_last_error", "snrt_mesh_create", "snrt_mesh_permutation",
    "snrt_mesh_info", "snrt_mesh_destroy", "snrt_quad_create", "snrt_quad_destroy",
    "snrt_scatter_isotropic", "snrt_scatter_dense", "snrt_scatter_destroy",
    "snrt_workspace_size", "snrt_step", "snrt_step_f64", "snrt_step_adjoint",
    "snrt_step_adjoint_f64", "snrt_scatter_apply", "snrt_mass", "snrt_scalar_flux",
    "snrt_dose_accumulate", "snrt_dose_adjoint", "snrt_dose_density_grad", "snrt_permute",
    "snrt_mesh_set_face_midpoints", "snrt_step2_workspace_size", "snrt_step2", "snrt_step2_f64",
    "snrt_step2_limited", "snrt_step2_limited_f64", "snrt_step_dose",
    "snrt_scatter_moments", "snrt_step_imex", "snrt_step_imex_f64",
    "snrt_pn_operators", "snrt_pn_create", "snrt_pn_destroy", "snrt_pn_info",
    "snrt_pn_state_elems", "snrt_pn_layout", "snrt_pn_step", "snrt_pn_step_f64",
    "snrt_stream_copy", "snrt_step_imex_moments", "snrt_step_imex_moments_f64",
    "snrt_rollout", "snrt_rollout_f64", "snrt_rollout_adjoint", "snrt_rollout_adjoint_f64",
    "snrt_step_dose_noalloc", "snrt_scatter_prepare_implicit", "snrt_step_imex_dense",
    "snrt_step_imex_dense_f64", "snrt_kernel_modes",
]


class SnrtError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn} failed with status {status}: {msg}")
        self.status = status


SNRT_LIMITER_BARTH_JESPERSEN = 0
SNRT_LIMITER_VENKATAKRISHNAN = 1
LIMITERS = {"barth-jespersen": SNRT_LIMITER_BARTH_JESPERSEN,
            "venkatakrishnan": SNRT_LIMITER_VENKATAKRISHNAN}


class Limiter(ctypes.Structure):
    """``snrt_limiter``: the second-order step's slope limiter and Venkatakrishnan's K."""
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32), ("k", ctypes.c_double)]


def limiter(kind="barth-jespersen", k: float = 1.0) -> Limiter:
    if isinstance(kind, str):
        if kind not in LIMITERS:
            raise ValueError(f"unknown limiter {kind!r}; expected one of {sorted(LIMITERS)}")
        kind = LIMITERS[kind]
    return Limiter(int(kind), 0, float(k))


class StepArgs(ctypes.Structure):
    """``snrt_step_args`` / ``snrt_step_args_f64`` (identical layout: pointers + scalars)."""
    _fields_ = [("sigma_t", ctypes.c_void_p), ("sigma_s", ctypes.c_void_p),
                ("inv_rho", ctypes.c_void_p), ("source", ctypes.c_void_p),
                ("inflow", ctypes.c_void_p), ("inflow_scale", ctypes.c_double),
                ("dt", ctypes.c_double), ("alpha_t", ctypes.c_double),
                ("alpha_s", ctypes.c_double), ("boundary", ctypes.c_int32)]


class Schedule(ctypes.Structure):
    """``snrt_schedule``: per-step host arrays (FP64, each may be NULL) of a rollout."""
    _fields_ = [("alpha_t", ctypes.c_void_p), ("alpha_s", ctypes.c_void_p),
                ("inflow_scale", ctypes.c_void_p), ("dose_coeff", ctypes.c_void_p)]


def schedule(alpha_t=None, alpha_s=None, inflow_scale=None, dose_coeff=None):
    """A :class:`Schedule` over FP64 copies of the given sequences; the copies are kept on
    the returned object so they outlive the call that reads them."""
    keep = [None if v is None else np.ascontiguousarray(v, dtype=np.float64)
            for v in (alpha_t, alpha_s, inflow_scale, dose_coeff)]
    sch = Schedule(*[None if k is None else k.ctypes.data for k in keep])
    sch._keep = keep
    return sch


_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_lp = ctypes.POINTER(ctypes.c_int64)
_st = ctypes.c_int

_lib = None


def lib() -> ctypes.CDLL:
    """Load ``libsnrt.so`` (raises ``OSError`` if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OSError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() or "
                      "python -m paper_2205_08417_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "snrt_abi_version": (ctypes.c_int, []),
        "snrt_last_error": (ctypes.c_char_p, []),
        "snrt_mesh_create": (_st, [ctypes.POINTER(_vp), ctypes.c_int64, ctypes.c_int32, _ip, _dp,
                                   _dp, _dp, ctypes.c_int64, ctypes.c_uint32]),
        "snrt_mesh_permutation": (_st, [_vp, _lp]),
        "snrt_mesh_info": (_st, [_vp, _lp, _lp, _ip]),
        "snrt_mesh_destroy": (None, [_vp]),
        "snrt_quad_create": (_st, [ctypes.POINTER(_vp), ctypes.c_int32, _dp, _dp]),
        "snrt_quad_destroy": (None, [_vp]),
        "snrt_scatter_isotropic": (_st, [ctypes.POINTER(_vp), _vp]),
        "snrt_scatter_dense": (_st, [ctypes.POINTER(_vp), _vp, _dp, ctypes.c_int]),
        "snrt_scatter_destroy": (None, [_vp]),
        "snrt_workspace_size": (_st, [_vp, _vp, _vp, ctypes.POINTER(ctypes.c_size_t)]),
        "snrt_step": (_st, [_vp, _vp, _vp, ctypes.POINTER(StepArgs), _vp, _vp, _vp,
                            ctypes.c_size_t, _vp]),
        "snrt_step_f64": (_st, [_vp, _vp, _vp, ctypes.POINTER(StepArgs), _vp, _vp, _vp,
                                ctypes.c_size_t, _vp]),
        "snrt_step_adjoint": (_st, [_vp, _vp, _vp, ctypes.POINTER(StepArgs), _vp, _vp, _vp, _vp,
                                    _vp, _vp, _vp, ctypes.c_size_t, _vp]),
        "snrt_step_adjoint_f64": (_st, [_vp, _vp, _vp, ctypes.POINTER(StepArgs), _vp, _vp, _vp,
                                        _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
        "snrt_scatter_apply": (_st, [_vp, _vp, _vp, _vp, _vp, ctypes.c_int32, _vp,
                                     ctypes.c_size_t, _vp]),
        "snrt_mass": (_st, [_vp, _vp, _vp, _vp, _vp]),
        "snrt_scalar_flux": (_st, [_vp, _vp, _vp, _vp, _vp]),
        "snrt_dose_accumulate": (_st, [_vp, _vp, _vp, _vp, ctypes.c_double, _vp, _vp]),
        "snrt_dose_adjoint": (_st, [_vp, _vp, _vp, ctypes.c_double, _vp, _vp, _vp]),
        "snrt_dose_density_grad": (_st, [_vp, _vp, _vp, _vp, _vp, _vp]),
        "snrt_permute": (_st, [_vp, ctypes.c_int32, _vp, _vp, ctypes.c_int64, _vp]),
        "snrt_stream_copy": (_st, [_vp, _vp, ctypes.c_int64, _vp]),
        "snrt_mesh_set_face_midpoints": (_st, [_vp, _dp]),
        "snrt_step_imex": (_st, [_vp, _vp, _vp, ctypes.POINTER(StepArgs), _vp, _vp, _vp]),
        "snrt_step_imex_f64": (_st, [_vp, _vp, _vp, ctypes.POINTER(StepArgs), _vp, _vp, _vp]),
        "snrt_step_imex_moments": (_st, [_vp, _vp, _vp, ctypes.POINTER(StepArgs), _vp, _vp,
                                         _vp, ctypes.c_size_t, _vp]),
        "snrt_step_imex_moments_f64": (_st, [_vp, _vp, _vp, ctypes.POINTER(StepArgs), _vp, _vp,
                                             _vp, ctypes.c_size_t, _vp]),
        "snrt_scatter_moments": (_st, [ctypes.POINTER(_vp), _vp, ctypes.c_int32, _dp,
                                       ctypes.c_int]),
        "snrt_scatter_prepare_implicit": (_st, [_vp]),
        "snrt_kernel_modes": (_st, [ctypes.c_int32, _dp, _dp, _dp, _dp, _dp]),
        "snrt_step_imex_dense": (_st, [_vp, _vp, _vp, ctypes.POINTER(StepArgs), _vp, _vp,
                                       _vp, ctypes.c_size_t, _vp]),
        "snrt_step_imex_dense_f64": (_st, [_vp, _vp, _vp, ctypes.POINTER(StepArgs), _vp, _vp,
                                           _vp, ctypes.c_size_t, _vp]),
        "snrt_step2_workspace_size": (_st, [_vp, _vp, _vp, ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_size_t)]),
        "snrt_step2": (_st, [_vp, _vp, _vp, ctypes.POINTER(StepArgs), _vp, _vp, _vp,
                             ctypes.c_size_t, _vp]),
        "snrt_step2_f64": (_st, [_vp, _vp, _vp, ctypes.POINTER(StepArgs), _vp, _vp, _vp,
                                 ctypes.c_size_t, _vp]),
        "snrt_step_dose": (_st, [_vp, _vp, _vp, ctypes.POINTER(StepArgs), _vp, _vp,
                                 ctypes.c_double, _vp, _vp, ctypes.c_size_t, _vp]),
        "snrt_step_dose_noalloc": (_st, [_vp, _vp, _vp, ctypes.POINTER(StepArgs), _vp, _vp,
                                         ctypes.c_double, _vp, _vp]),
        "snrt_step2_limited": (_st, [_vp, _vp, _vp, ctypes.POINTER(StepArgs),
                                     ctypes.POINTER(Limiter), _vp, _vp, _vp, ctypes.c_size_t,
                                     _vp]),
        "snrt_step2_limited_f64": (_st, [_vp, _vp, _vp, ctypes.POINTER(StepArgs),
                                         ctypes.POINTER(Limiter), _vp, _vp, _vp,
                                         ctypes.c_size_t, _vp]),
        "snrt_rollout": (_st, [_vp, _vp, _vp, ctypes.POINTER(StepArgs), ctypes.POINTER(Schedule),
                               ctypes.c_int64, _vp, _vp, _vp, ctypes.c_int32, _vp, _vp,
                               ctypes.c_size_t, _vp]),
        "snrt_rollout_f64": (_st, [_vp, _vp, _vp, ctypes.POINTER(StepArgs),
                                   ctypes.POINTER(Schedule), ctypes.c_int64, _vp, _vp, _vp,
                                   ctypes.c_int32, _vp, ctypes.c_size_t, _vp]),
        "snrt_rollout_adjoint": (_st, [_vp, _vp, _vp, ctypes.POINTER(StepArgs),
                                       ctypes.POINTER(Schedule), ctypes.c_int64, _vp,
                                       ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                       _vp, ctypes.c_size_t, _vp]),
        "snrt_rollout_adjoint_f64": (_st, [_vp, _vp, _vp, ctypes.POINTER(StepArgs),
                                           ctypes.POINTER(Schedule), ctypes.c_int64, _vp,
                                           ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                           ctypes.c_size_t, _vp]),
        "snrt_pn_operators": (_st, [ctypes.c_int32, _dp, _dp, _dp, _dp]),
        "snrt_pn_create": (_st, [ctypes.POINTER(_vp), ctypes.c_int32, _dp]),
        "snrt_pn_destroy": (None, [_vp]),
        "snrt_pn_info": (_st, [_vp, _ip, _ip]),
        "snrt_pn_state_elems": (_st, [_vp, _vp, _lp]),
        "snrt_pn_layout": (_st, [_vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp]),
        "snrt_pn_step": (_st, [_vp, _vp, ctypes.POINTER(StepArgs), _vp, _vp, _vp]),
        "snrt_pn_step_f64": (_st, [_vp, _vp, ctypes.POINTER(StepArgs), _vp, _vp, _vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


# ------------------------------------------------------------------------------ marshalling

def _ptr(x) -> Optional[int]:
    """Device address of a torch tensor / raw int / None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _f64(a):
    if a is None:
        return None, None
    arr = np.ascontiguousarray(a, dtype=np.float64)
    return arr, arr.ctypes.data_as(_dp)


def _check(fn: str, st: int):
    if st != SNRT_OK:
        raise SnrtError(fn, st, lib().snrt_last_error().decode(errors="replace"))


def step_args(sigma_t, sigma_s, dt, inv_rho=None, source=None, inflow=None,
              inflow_scale=1.0, alpha_t=1.0, alpha_s=1.0, boundary=SNRT_BC_DIRICHLET):
    return StepArgs(_ptr(sigma_t), _ptr(sigma_s), _ptr(inv_rho), _ptr(source), _ptr(inflow),
                    float(inflow_scale), float(dt), float(alpha_t), float(alpha_s),
                    int(boundary))


# ------------------------------------------------------------------------------ entry points

def snrt_abi_version() -> int:
    return int(lib().snrt_abi_version())


def snrt_last_error() -> str:
    return lib().snrt_last_error().decode(errors="replace")


def snrt_mesh_create(face_nbr, face_normal, area, centroid=None, nbfaces=0,
                     flags=SNRT_REORDER_HILBERT) -> int:
    nbr = np.ascontiguousarray(face_nbr, dtype=np.int32)
    nc, mf = (nbr.shape if nbr.ndim == 2 else (0, 3))
    nrm, pn = _f64(face_normal)
    ar, pa = _f64(area)
    ce, pc = _f64(centroid)
    h = _vp()
    _check("snrt_mesh_create",
           lib().snrt_mesh_create(ctypes.byref(h), int(nc), int(mf), nbr.ctypes.data_as(_ip),
                                  pn, pa, pc, int(nbfaces), int(flags)))
    return h.value


def snrt_mesh_set_face_midpoints(mesh: int, face_mid) -> None:
    arr, p = _f64(face_mid)
    _check("snrt_mesh_set_face_midpoints", lib().snrt_mesh_set_face_midpoints(mesh, p))


def snrt_mesh_permutation(mesh: int) -> np.ndarray:
    nc = ctypes.c_int64()
    _check("snrt_mesh_info", lib().snrt_mesh_info(mesh, ctypes.byref(nc), None, None))
    out = np.empty(nc.value, dtype=np.int64)
    _check("snrt_mesh_permutation", lib().snrt_mesh_permutation(mesh, out.ctypes.data_as(_lp)))
    return out


def snrt_mesh_info(mesh: int):
    nc, nbf, mf = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
    _check("snrt_mesh_info", lib().snrt_mesh_info(mesh, ctypes.byref(nc), ctypes.byref(nbf),
                                                  ctypes.byref(mf)))
    return nc.value, nbf.value, mf.value


def snrt_mesh_destroy(mesh: int) -> None:
    lib().snrt_mesh_destroy(mesh)


def snrt_quad_create(omega, w) -> int:
    om, po = _f64(omega)
    ww, pw = _f64(w)
    h = _vp()
    _check("snrt_quad_create", lib().snrt_quad_create(ctypes.byref(h), int(ww.shape[0]), po, pw))
    return h.value


def snrt_quad_destroy(quad: int) -> None:
    lib().snrt_quad_destroy(quad)


def snrt_scatter_isotropic(quad: int) -> int:
    h = _vp()
    _check("snrt_scatter_isotropic", lib().snrt_scatter_isotropic(ctypes.byref(h), quad))
    return h.value


def snrt_scatter_dense(quad: int, K, precision=SNRT_FP32) -> int:
    k, pk = _f64(K)
    h = _vp()
    _check("snrt_scatter_dense", lib().snrt_scatter_dense(ctypes.byref(h), quad, pk,
                                                          int(precision)))
    return h.value


def snrt_scatter_moments(quad: int, sigma_l, precision=SNRT_FP32) -> int:
    arr, p = _f64(sigma_l)
    h = _vp()
    _check("snrt_scatter_moments",
           lib().snrt_scatter_moments(ctypes.byref(h), quad, int(arr.size - 1), p, int(precision)))
    return h.value


def snrt_scatter_destroy(scatter: int) -> None:
    lib().snrt_scatter_destroy(scatter)


def snrt_step_imex(mesh, quad, scatter, args: StepArgs, psi_in, psi_out, stream=None) -> None:
    _check("snrt_step_imex", lib().snrt_step_imex(mesh, quad, scatter, ctypes.byref(args),
                                                  _ptr(psi_in), _ptr(psi_out), _stream(stream)))


def snrt_step_imex_f64(mesh, quad, scatter, args: StepArgs, psi_in, psi_out,
                       stream=None) -> None:
    _check("snrt_step_imex_f64", lib().snrt_step_imex_f64(mesh, quad, scatter, ctypes.byref(args),
                                                          _ptr(psi_in), _ptr(psi_out),
                                                          _stream(stream)))


def snrt_step_imex_moments(mesh, quad, scatter, args: StepArgs, psi_in, psi_out, ws,
                           ws_bytes: int, stream=None) -> None:
    _check("snrt_step_imex_moments",
           lib().snrt_step_imex_moments(mesh, quad, scatter, ctypes.byref(args), _ptr(psi_in),
                                        _ptr(psi_out), _ptr(ws), int(ws_bytes), _stream(stream)))


def snrt_step_imex_moments_f64(mesh, quad, scatter, args: StepArgs, psi_in, psi_out, ws,
                               ws_bytes: int, stream=None) -> None:
    _check("snrt_step_imex_moments_f64",
           lib().snrt_step_imex_moments_f64(mesh, quad, scatter, ctypes.byref(args),
                                            _ptr(psi_in), _ptr(psi_out), _ptr(ws),
                                            int(ws_bytes), _stream(stream)))


def snrt_scatter_prepare_implicit(scatter: int) -> None:
    _check("snrt_scatter_prepare_implicit", lib().snrt_scatter_prepare_implicit(scatter))


def snrt_step_imex_dense(mesh, quad, scatter, args: StepArgs, psi_in, psi_out, ws,
                         ws_bytes: int, stream=None) -> None:
    _check("snrt_step_imex_dense",
           lib().snrt_step_imex_dense(mesh, quad, scatter, ctypes.byref(args), _ptr(psi_in),
                                      _ptr(psi_out), _ptr(ws), int(ws_bytes), _stream(stream)))


def snrt_step_imex_dense_f64(mesh, quad, scatter, args: StepArgs, psi_in, psi_out, ws,
                             ws_bytes: int, stream=None) -> None:
    _check("snrt_step_imex_dense_f64",
           lib().snrt_step_imex_dense_f64(mesh, quad, scatter, ctypes.byref(args), _ptr(psi_in),
                                          _ptr(psi_out), _ptr(ws), int(ws_bytes),
                                          _stream(stream)))


def snrt_step2_workspace_size(mesh: int, quad: int, scatter: int, fp64: bool = False) -> int:
    n = ctypes.c_size_t()
    _check("snrt_step2_workspace_size",
           lib().snrt_step2_workspace_size(mesh, quad, scatter, int(bool(fp64)), ctypes.byref(n)))
    return n.value


def snrt_step2(mesh, quad, scatter, args: StepArgs, psi_in, psi_out, ws=None, ws_bytes=0,
               stream=None) -> None:
    _check("snrt_step2", lib().snrt_step2(mesh, quad, scatter, ctypes.byref(args), _ptr(psi_in),
                                          _ptr(psi_out), _ptr(ws), int(ws_bytes),
                                          _stream(stream)))


def snrt_step2_f64(mesh, quad, scatter, args: StepArgs, psi_in, psi_out, ws=None, ws_bytes=0,
                   stream=None) -> None:
    _check("snrt_step2_f64", lib().snrt_step2_f64(mesh, quad, scatter, ctypes.byref(args),
                                                  _ptr(psi_in), _ptr(psi_out), _ptr(ws),
                                                  int(ws_bytes), _stream(stream)))


def snrt_step_dose(mesh, quad, scatter, args: StepArgs, psi_in, psi_out, coeff: float, dose,
                   ws=None, ws_bytes=0, stream=None) -> None:
    _check("snrt_step_dose",
           lib().snrt_step_dose(mesh, quad, scatter, ctypes.byref(args), _ptr(psi_in),
                                _ptr(psi_out), float(coeff), _ptr(dose), _ptr(ws), int(ws_bytes),
                                _stream(stream)))


def snrt_step_dose_noalloc(mesh, quad, scatter, args: StepArgs, psi_in, psi_out, coeff: float,
                           dose, stream=None) -> None:
    _check("snrt_step_dose_noalloc",
           lib().snrt_step_dose_noalloc(mesh, quad, scatter, ctypes.byref(args), _ptr(psi_in),
                                        _ptr(psi_out), float(coeff), _ptr(dose),
                                        _stream(stream)))


def snrt_step2_limited(mesh, quad, scatter, args: StepArgs, lim: Optional[Limiter], psi_in,
                       psi_out, ws=None, ws_bytes=0, stream=None) -> None:
    _check("snrt_step2_limited",
           lib().snrt_step2_limited(mesh, quad, scatter, ctypes.byref(args),
                                    None if lim is None else ctypes.byref(lim), _ptr(psi_in),
                                    _ptr(psi_out), _ptr(ws), int(ws_bytes), _stream(stream)))


def snrt_step2_limited_f64(mesh, quad, scatter, args: StepArgs, lim: Optional[Limiter], psi_in,
                           psi_out, ws=None, ws_bytes=0, stream=None) -> None:
    _check("snrt_step2_limited_f64",
           lib().snrt_step2_limited_f64(mesh, quad, scatter, ctypes.byref(args),
                                        None if lim is None else ctypes.byref(lim), _ptr(psi_in),
                                        _ptr(psi_out), _ptr(ws), int(ws_bytes),
                                        _stream(stream)))


def snrt_workspace_size(mesh: int, quad: int, scatter: int) -> int:
    n = ctypes.c_size_t()
    _check("snrt_workspace_size", lib().snrt_workspace_size(mesh, quad, scatter,
                                                            ctypes.byref(n)))
    return n.value


def snrt_step(mesh, quad, scatter, args: StepArgs, psi_in, psi_out, ws=None, ws_bytes=0,
              stream=None) -> None:
    _check("snrt_step", lib().snrt_step(mesh, quad, scatter, ctypes.byref(args), _ptr(psi_in),
                                        _ptr(psi_out), _ptr(ws), int(ws_bytes), _stream(stream)))


def snrt_step_f64(mesh, quad, scatter, args: StepArgs, psi_in, psi_out, ws=None, ws_bytes=0,
                  stream=None) -> None:
    _check("snrt_step_f64", lib().snrt_step_f64(mesh, quad, scatter, ctypes.byref(args),
                                                _ptr(psi_in), _ptr(psi_out), _ptr(ws),
                                                int(ws_bytes), _stream(stream)))


def snrt_step_adjoint(mesh, quad, scatter, args: StepArgs, psi_n, lam_np1, lam_n,
                      g_sigma_t=None, g_sigma_s=None, g_rho=None, ws=None, ws_bytes=0,
                      stream=None) -> None:
    _check("snrt_step_adjoint",
           lib().snrt_step_adjoint(mesh, quad, scatter, ctypes.byref(args), _ptr(psi_n),
                                   _ptr(lam_np1), _ptr(lam_n), _ptr(g_sigma_t),
                                   _ptr(g_sigma_s), _ptr(g_rho), _ptr(ws), int(ws_bytes),
                                   _stream(stream)))


def snrt_step_adjoint_f64(mesh, quad, scatter, args: StepArgs, psi_n, lam_np1, lam_n,
                          g_sigma_t=None, g_sigma_s=None, g_rho=None, ws=None, ws_bytes=0,
                          stream=None) -> None:
    _check("snrt_step_adjoint_f64",
           lib().snrt_step_adjoint_f64(mesh, quad, scatter, ctypes.byref(args), _ptr(psi_n),
                                       _ptr(lam_np1), _ptr(lam_n), _ptr(g_sigma_t),
                                       _ptr(g_sigma_s), _ptr(g_rho), _ptr(ws), int(ws_bytes),
                                       _stream(stream)))


def snrt_scatter_apply(mesh, quad, scatter, psi, S, transpose=0, ws=None, ws_bytes=0,
                       stream=None) -> None:
    _check("snrt_scatter_apply", lib().snrt_scatter_apply(mesh, quad, scatter, _ptr(psi), _ptr(S),
                                                          int(transpose), _ptr(ws),
                                                          int(ws_bytes), _stream(stream)))


def snrt_mass(mesh, quad, psi, out_dev, stream=None) -> None:
    _check("snrt_mass", lib().snrt_mass(mesh, quad, _ptr(psi), _ptr(out_dev), _stream(stream)))


def snrt_scalar_flux(mesh, quad, psi, phi, stream=None) -> None:
    _check("snrt_scalar_flux", lib().snrt_scalar_flux(mesh, quad, _ptr(psi), _ptr(phi),
                                                      _stream(stream)))


def snrt_dose_accumulate(mesh, quad, psi, inv_rho, coeff, dose, stream=None) -> None:
    _check("snrt_dose_accumulate",
           lib().snrt_dose_accumulate(mesh, quad, _ptr(psi), _ptr(inv_rho), float(coeff),
                                      _ptr(dose), _stream(stream)))


def snrt_dose_adjoint(mesh, quad, inv_rho, coeff, g_dose, lam, stream=None) -> None:
    _check("snrt_dose_adjoint", lib().snrt_dose_adjoint(mesh, quad, _ptr(inv_rho), float(coeff),
                                                        _ptr(g_dose), _ptr(lam), _stream(stream)))


def snrt_dose_density_grad(mesh, dose, inv_rho, g_dose, g_rho, stream=None) -> None:
    _check("snrt_dose_density_grad",
           lib().snrt_dose_density_grad(mesh, _ptr(dose), _ptr(inv_rho), _ptr(g_dose), _ptr(g_rho),
                                        _stream(stream)))


def snrt_permute(mesh, to_user: int, src, dst, row_bytes: int, stream=None) -> None:
    _check("snrt_permute", lib().snrt_permute(mesh, int(to_user), _ptr(src), _ptr(dst),
                                              int(row_bytes), _stream(stream)))


def snrt_stream_copy(src, dst, nbytes: int, stream=None) -> None:
    """Measurement helper: nontemporal device copy of ``nbytes`` bytes from ``src`` to ``dst``."""
    _check("snrt_stream_copy", lib().snrt_stream_copy(_ptr(src), _ptr(dst), int(nbytes),
                                                      _stream(stream)))


def snrt_rollout(mesh, quad, scatter, args: StepArgs, sched: Optional[Schedule], nsteps: int,
                 psi, tmp, ckpt=None, ckpt_every: int = 1, dose=None, ws=None, ws_bytes=0,
                 stream=None) -> None:
    _check("snrt_rollout",
           lib().snrt_rollout(mesh, quad, scatter, ctypes.byref(args),
                              None if sched is None else ctypes.byref(sched), int(nsteps),
                              _ptr(psi), _ptr(tmp), _ptr(ckpt), int(ckpt_every), _ptr(dose),
                              _ptr(ws), int(ws_bytes), _stream(stream)))


def snrt_rollout_f64(mesh, quad, scatter, args: StepArgs, sched: Optional[Schedule],
                     nsteps: int, psi, tmp, ckpt=None, ckpt_every: int = 1, ws=None, ws_bytes=0,
                     stream=None) -> None:
    _check("snrt_rollout_f64",
           lib().snrt_rollout_f64(mesh, quad, scatter, ctypes.byref(args),
                                  None if sched is None else ctypes.byref(sched), int(nsteps),
                                  _ptr(psi), _ptr(tmp), _ptr(ckpt), int(ckpt_every), _ptr(ws),
                                  int(ws_bytes), _stream(stream)))


def snrt_rollout_adjoint(mesh, quad, scatter, args: StepArgs, sched: Optional[Schedule],
                         nsteps: int, ckpt, ckpt_every: int, seg, lam, tmp, g_sigma_t=None,
                         g_sigma_s=None, g_rho=None, g_dose=None, dose=None, ws=None,
                         ws_bytes=0, stream=None) -> None:
    _check("snrt_rollout_adjoint",
           lib().snrt_rollout_adjoint(mesh, quad, scatter, ctypes.byref(args),
                                      None if sched is None else ctypes.byref(sched),
                                      int(nsteps), _ptr(ckpt), int(ckpt_every), _ptr(seg),
                                      _ptr(lam), _ptr(tmp), _ptr(g_sigma_t), _ptr(g_sigma_s),
                                      _ptr(g_rho), _ptr(g_dose), _ptr(dose), _ptr(ws),
                                      int(ws_bytes), _stream(stream)))


def snrt_rollout_adjoint_f64(mesh, quad, scatter, args: StepArgs, sched: Optional[Schedule],
                             nsteps: int, ckpt, ckpt_every: int, seg, lam, tmp, g_sigma_t=None,
                             g_sigma_s=None, g_rho=None, ws=None, ws_bytes=0,
                             stream=None) -> None:
    _check("snrt_rollout_adjoint_f64",
           lib().snrt_rollout_adjoint_f64(mesh, quad, scatter, ctypes.byref(args),
                                          None if sched is None else ctypes.byref(sched),
                                          int(nsteps), _ptr(ckpt), int(ckpt_every), _ptr(seg),
                                          _ptr(lam), _ptr(tmp), _ptr(g_sigma_t),
                                          _ptr(g_sigma_s), _ptr(g_rho), _ptr(ws), int(ws_bytes),
                                          _stream(stream)))


# ------------------------------------------------------------------------------ P_N solver

def snrt_kernel_modes(A):
    """Host-only: (lam, x0, x1, resid) of A = K W (see include/snrt.h)."""
    a = np.ascontiguousarray(A, dtype=np.float64)
    n = a.shape[0]
    lam = np.zeros(n)
    x0 = np.zeros((n, n))
    x1 = np.zeros((n, n))
    r = ctypes.c_double()
    _check("snrt_kernel_modes",
           lib().snrt_kernel_modes(int(n), a.ctypes.data_as(_dp), lam.ctypes.data_as(_dp),
                                   x0.ctypes.data_as(_dp), x1.ctypes.data_as(_dp),
                                   ctypes.byref(r)))
    return lam, x0, x1, float(r.value)


def snrt_pn_operators(degree: int):
    """Host-only: (A_x, A_y, |A_x|, |A_y|) of degree ``degree`` as [nm][nm] FP64 arrays."""
    nm = (int(degree) + 1) ** 2
    mats = [np.zeros((nm, nm)) for _ in range(4)]
    _check("snrt_pn_operators",
           lib().snrt_pn_operators(int(degree), *[m.ctypes.data_as(_dp) for m in mats]))
    return tuple(mats)


def snrt_pn_create(degree: int, sigma_l=None) -> int:
    arr, p = _f64(sigma_l)
    if arr is not None and arr.size < int(degree) + 1:
        raise ValueError("sigma_l needs degree + 1 entries")
    h = _vp()
    _check("snrt_pn_create", lib().snrt_pn_create(ctypes.byref(h), int(degree), p))
    return h.value


def snrt_pn_destroy(pn: int) -> None:
    lib().snrt_pn_destroy(pn)


def snrt_pn_info(pn: int):
    d = ctypes.c_int32()
    n = ctypes.c_int32()
    _check("snrt_pn_info", lib().snrt_pn_info(pn, ctypes.byref(d), ctypes.byref(n)))
    return d.value, n.value


def snrt_pn_state_elems(mesh: int, pn: int) -> int:
    n = ctypes.c_int64()
    _check("snrt_pn_state_elems", lib().snrt_pn_state_elems(mesh, pn, ctypes.byref(n)))
    return n.value


def snrt_pn_layout(mesh: int, pn: int, to_user: int, elem_bytes: int, src, dst,
                   stream=None) -> None:
    _check("snrt_pn_layout", lib().snrt_pn_layout(mesh, pn, int(to_user), int(elem_bytes),
                                                  _ptr(src), _ptr(dst), _stream(stream)))


def snrt_pn_step(mesh, pn, args: StepArgs, u_in, u_out, stream=None) -> None:
    _check("snrt_pn_step", lib().snrt_pn_step(mesh, pn, ctypes.byref(args), _ptr(u_in),
                                              _ptr(u_out), _stream(stream)))


def snrt_pn_step_f64(mesh, pn, args: StepArgs, u_in, u_out, stream=None) -> None:
    _check("snrt_pn_step_f64", lib().snrt_pn_step_f64(mesh, pn, ctypes.byref(args), _ptr(u_in),
                                                      _ptr(u_out), _stream(stream)))
