"""ctypes binding of libasn.so (include/asn.h).

Argument marshalling only: every step of the as-S_N path runs in the HIP
library.  torch supplies device memory (the problem workspace) and the HIP
stream.  If libasn.so has not been built this module raises on import.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
# torch ships its own HIP runtime (libamdhip64.so.7).  Loading it before
# libasn.so makes the library bind to that same runtime, so device pointers and
# streams from torch are valid inside the library (one runtime per process).
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libasn.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_1911_08801_amd.build.build() "
                      "(or __graft_entry__.build()); there is no fallback path")

_lib = ctypes.CDLL(LIB_PATH)

ASN_OK = 0
ASN_E_INVALID = -1
ASN_E_OOM = -2
ASN_E_HIP = -3
ASN_E_UNSTABLE = -4
ASN_E_STATE = -5
ASN_E_UNSUPPORTED = -6

ASN_GEMM_F32, ASN_GEMM_BF16, ASN_GEMM_F16 = 0, 1, 2
ASN_NORM_SYM, ASN_NORM_ROW = 0, 1
ASN_SCHEME_EULER, ASN_SCHEME_HEUN, ASN_SCHEME_IMPLICIT = 0, 1, 2
ASN_DT_STREAMING, ASN_DT_STIFF = 0, 1
ASN_SOURCE_TEST_ABSOLUTE, ASN_SOURCE_TEST_RELATIVE = 0, 1
ASN_FORM_AUTO, ASN_FORM_SEPARATE, ASN_FORM_FUSED, ASN_FORM_BANDED = 0, 1, 2, 3
FORMS = {"auto": ASN_FORM_AUTO, "separate": ASN_FORM_SEPARATE, "fused": ASN_FORM_FUSED,
         "banded": ASN_FORM_BANDED}
ASN_BUDGET_LEN = 8

DTYPES = {"f32": ASN_GEMM_F32, "bf16": ASN_GEMM_BF16, "f16": ASN_GEMM_F16}
NORMS = {"sym": ASN_NORM_SYM, "row": ASN_NORM_ROW}
SCHEMES = {"euler": ASN_SCHEME_EULER, "heun": ASN_SCHEME_HEUN, "implicit": ASN_SCHEME_IMPLICIT}
DT_RULES = {"streaming": ASN_DT_STREAMING, "stiff": ASN_DT_STIFF}
SOURCE_TESTS = {"absolute": ASN_SOURCE_TEST_ABSOLUTE, "relative": ASN_SOURCE_TEST_RELATIVE}


class AsnError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.asn_last_error().decode()
        super().__init__(f"{where}: {_lib.asn_status_string(status).decode()} ({status}): {msg}")


class asn_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("x_min", ctypes.c_double),
                ("x_max", ctypes.c_double), ("y_min", ctypes.c_double), ("y_max", ctypes.c_double)]


class asn_quadrature(ctypes.Structure):
    _fields_ = [("n_polar", ctypes.c_int32), ("n_azim", ctypes.c_int32),
                ("q_custom", ctypes.c_int32), ("omega_xyz", ctypes.POINTER(ctypes.c_double)),
                ("weights", ctypes.POINTER(ctypes.c_double)),
                ("icosahedron_order", ctypes.c_int32)]


class asn_options(ctypes.Structure):
    _fields_ = [("gemm_dtype", ctypes.c_int32), ("normalization", ctypes.c_int32),
                ("cfl", ctypes.c_double), ("eps_override", ctypes.c_double),
                ("dt_override", ctypes.c_double), ("scale_block", ctypes.c_int32),
                ("scheme", ctypes.c_int32), ("dt_rule", ctypes.c_int32),
                ("step_form", ctypes.c_int32), ("implicit_tol", ctypes.c_double),
                ("source_tol", ctypes.c_double), ("source_test", ctypes.c_int32)]


_P = ctypes.c_void_p
_F = ctypes.POINTER(ctypes.c_float)
_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)
_SIG = {
    "asn_options_default": [ctypes.POINTER(asn_options)],
    "asn_workspace_size": [ctypes.POINTER(asn_grid), ctypes.POINTER(asn_quadrature),
                           ctypes.POINTER(asn_options), ctypes.POINTER(ctypes.c_size_t)],
    "asn_create": [ctypes.POINTER(asn_grid), ctypes.POINTER(asn_quadrature), _F, _F, _F, _F,
                   ctypes.c_double, ctypes.c_double, ctypes.POINTER(asn_options), _P, _P,
                   ctypes.c_size_t, ctypes.POINTER(_P)],
    "asn_set_state": [_P, _P, ctypes.c_int32],
    "asn_set_state_isotropic": [_P, _P, ctypes.c_int32],
    "asn_get_state": [_P, _P, ctypes.c_int32],
    "asn_step": [_P, ctypes.c_int64],
    "asn_step_batch": [ctypes.POINTER(_P), ctypes.c_int32, ctypes.c_int64],
    "asn_step_batch_noalloc": [ctypes.POINTER(_P), ctypes.c_int32, ctypes.c_int64],
    "asn_step_timed": [_P, ctypes.c_int64, _D],
    "asn_batch_create": [ctypes.POINTER(_P), ctypes.c_int32, ctypes.POINTER(_P)],
    "asn_batch_step": [_P, ctypes.c_int64, _I64],
    "asn_batch_destroy": [_P],
    "asn_scalar_flux": [_P, _D],
    "asn_mass_budget": [_P, _D],
    "asn_info": [_P, _D, _I64, _I64, ctypes.POINTER(ctypes.c_int32)],
    "asn_step_form": [_P, ctypes.POINTER(ctypes.c_int32)],
    "asn_destroy": [_P],
    "asn_contraction_work": [_P, _D, _D],
    "asn_contraction_nonzero": [_P, _D],
    "asn_stability": [_P, _D],
    "asn_iteration_counts": [_P, _I64, _I64],
    "asn_build_quadrature": [ctypes.c_int32, ctypes.c_int32, _D, _D],
    "asn_build_icosahedron": [ctypes.c_int32, _D, _D],
    "asn_build_kernel": [ctypes.c_int32, _D, _D, ctypes.c_double, ctypes.c_int32, _D],
    "asn_build_kernel_lowp": [ctypes.c_int32, _D, ctypes.c_int32,
                              ctypes.POINTER(ctypes.c_uint16), _F],
    "asn_time_step": [ctypes.POINTER(asn_grid), ctypes.c_int32, _D, ctypes.c_double,
                      ctypes.c_double, _D, _I64],
    "asn_band_expand": [ctypes.c_int32, ctypes.c_int32, _D, _F, ctypes.POINTER(ctypes.c_int32)],
}
for _name, _args in _SIG.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = ctypes.c_int
_lib.asn_status_string.argtypes = [ctypes.c_int]
_lib.asn_status_string.restype = ctypes.c_char_p
_lib.asn_last_error.argtypes = []
_lib.asn_last_error.restype = ctypes.c_char_p

EXPORTED = list(_SIG) + ["asn_status_string", "asn_last_error"]


def _check(status: int, where: str) -> None:
    if status != ASN_OK:
        raise AsnError(status, where)


def _fptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_F)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


# ------------------------------------------------------------------ host builders

def asn_build_quadrature(n_polar: int, n_azim: int):
    q = n_polar * n_azim
    om = np.zeros((q, 3))
    w = np.zeros(q)
    _check(_lib.asn_build_quadrature(n_polar, n_azim, _dptr(om), _dptr(w)), "asn_build_quadrature")
    return om, w


def asn_build_icosahedron(order: int):
    q = 10 * (order - 1) ** 2 + 2
    om = np.zeros((q, 3))
    w = np.zeros(q)
    _check(_lib.asn_build_icosahedron(order, _dptr(om), _dptr(w)), "asn_build_icosahedron")
    return om, w


def asn_build_kernel(omega: np.ndarray, w: np.ndarray, eps: float, norm: str = "sym") -> np.ndarray:
    omega = np.ascontiguousarray(omega, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    q = w.size
    K = np.zeros((q, q))
    _check(_lib.asn_build_kernel(q, _dptr(omega), _dptr(w), eps, NORMS[norm], _dptr(K)),
           "asn_build_kernel")
    return K


def asn_band_expand(n_polar: int, n_azim: int, K: np.ndarray):
    """(dense FP32 K rebuilt from the banded form the library builds of fp32(K), reach)."""
    K = np.ascontiguousarray(K, dtype=np.float64)
    q = n_polar * n_azim
    if K.shape != (q, q):
        raise ValueError("K must be Q x Q with Q = n_polar * n_azim")
    out = np.zeros((q, q), dtype=np.float32)
    reach = ctypes.c_int32()
    _check(_lib.asn_band_expand(n_polar, n_azim, _dptr(K), _fptr(out), ctypes.byref(reach)),
           "asn_band_expand")
    return out, reach.value


def asn_build_kernel_lowp(K: np.ndarray, dtype: str):
    """(16-bit patterns of T(fp32(K)), row defects) for dtype "bf16" or "f16"."""
    K = np.ascontiguousarray(K, dtype=np.float64)
    q = K.shape[0]
    bits = np.zeros((q, q), dtype=np.uint16)
    r = np.zeros(q, dtype=np.float32)
    _check(_lib.asn_build_kernel_lowp(q, _dptr(K), DTYPES[dtype],
                                      bits.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)),
                                      _fptr(r)), "asn_build_kernel_lowp")
    return bits, r


def make_grid(nx, ny, x_min, x_max, y_min, y_max) -> asn_grid:
    return asn_grid(nx, ny, x_min, x_max, y_min, y_max)


def make_quadrature(n_polar: int, n_azim: int) -> asn_quadrature:
    """The product set of n_polar Gauss-Legendre nodes times n_azim azimuths."""
    return asn_quadrature(n_polar, n_azim, 0, None, None, 0)


def asn_time_step(grid: asn_grid, omega: np.ndarray, cfl: float, t_final: float):
    omega = np.ascontiguousarray(omega, dtype=np.float64)
    dt = ctypes.c_double()
    n = ctypes.c_int64()
    _check(_lib.asn_time_step(ctypes.byref(grid), omega.shape[0], _dptr(omega), cfl, t_final,
                              ctypes.byref(dt), ctypes.byref(n)), "asn_time_step")
    return dt.value, n.value


def asn_options_default() -> asn_options:
    o = asn_options()
    _check(_lib.asn_options_default(ctypes.byref(o)), "asn_options_default")
    return o


def make_options(dtype: str = "f32", norm: str = "sym", cfl: float = 0.95,
                 eps_override: float = 0.0, dt_override: float = 0.0,
                 scheme: str = "euler", dt_rule: str = "streaming",
                 unfused: Optional[bool] = None, implicit_tol: float = 0.0,
                 source_tol: float = 0.0, source_test: str = "absolute",
                 form: Optional[str] = None, scale_block: int = 256) -> asn_options:
    """Options for asn_create.  Kernel form of forward-Euler steps: form "auto",
    "separate", "fused" or "banded"; or unfused (when form is None): None lets the
    library choose, True asks for separate kernels, False for the fused one.
    scale_block: cells per block of the BF16 / FP16 operand scale."""
    o = asn_options_default()
    o.gemm_dtype = DTYPES[dtype]
    o.normalization = NORMS[norm]
    o.scheme = SCHEMES[scheme]
    o.dt_rule = DT_RULES[dt_rule]
    if form is not None:
        o.step_form = FORMS[form]
    else:
        o.step_form = (ASN_FORM_AUTO if unfused is None else
                       ASN_FORM_SEPARATE if unfused else ASN_FORM_FUSED)
    o.implicit_tol = implicit_tol
    o.source_tol = source_tol
    o.source_test = SOURCE_TESTS[source_test]
    o.cfl = cfl
    o.eps_override = eps_override
    o.dt_override = dt_override
    o.scale_block = scale_block
    return o


# ------------------------------------------------------------------ problems

class AsnProblem:
    """An as-S_N problem resident on the GPU (wraps an asn_problem handle)."""

    def __init__(self, handle, nx, ny, q, workspace, keepalive):
        self.handle = handle
        self.nx, self.ny, self.q = nx, ny, q
        self._workspace = workspace          # torch tensor owning the device memory
        self._keep = keepalive

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def close(self):
        if self.handle is not None:
            h, self.handle = self.handle, None
            _check(_lib.asn_destroy(h), "asn_destroy")
            self._workspace = None


def asn_workspace_size(grid: asn_grid, quad: asn_quadrature, opt: asn_options) -> int:
    n = ctypes.c_size_t()
    _check(_lib.asn_workspace_size(ctypes.byref(grid), ctypes.byref(quad), ctypes.byref(opt),
                                   ctypes.byref(n)), "asn_workspace_size")
    return n.value


def asn_create(grid: asn_grid, n_polar: int = 0, n_azim: int = 0, sigma_s=None, sigma_a=None,
               sigma_as=None, source=None, beta: float = 4.5, t_final: float = 1.0,
               options: Optional[asn_options] = None, omega: Optional[np.ndarray] = None,
               weights: Optional[np.ndarray] = None, device: str = "cuda",
               torch_workspace: bool = True, icosahedron_order: int = 0,
               workspace=None) -> AsnProblem:
    """Create a problem on the current torch device and stream.

    The workspace is a torch uint8 tensor (so torch's allocator accounts for it):
    the caller's `workspace` (contiguous, on the device) if given, else a new one of
    asn_workspace_size bytes; torch_workspace=False lets the library allocate.
    The library enqueues all work on torch's current stream.
    """
    import torch
    opt = options if options is not None else asn_options_default()
    keep = []
    if omega is not None:
        om = np.ascontiguousarray(omega, dtype=np.float64)
        w = np.ascontiguousarray(weights, dtype=np.float64)
        keep += [om, w]
        quad = asn_quadrature(0, 0, w.size, _dptr(om), _dptr(w), 0)
        q = w.size
    elif icosahedron_order:
        quad = asn_quadrature(0, 0, 0, None, None, icosahedron_order)
        q = 10 * (icosahedron_order - 1) ** 2 + 2
    else:
        quad = asn_quadrature(n_polar, n_azim, 0, None, None, 0)
        q = n_polar * n_azim
    fields = [_f32(f) for f in (sigma_s, sigma_a, sigma_as)]
    src = None if source is None else _f32(source)
    keep += fields + ([src] if src is not None else [])
    c = grid.nx * grid.ny
    for f in fields + ([src] if src is not None else []):
        if f.size != c:
            raise ValueError("fields must have nx * ny entries")
    ws = None
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        if workspace.dtype != torch.uint8 or not workspace.is_cuda or not workspace.is_contiguous():
            raise ValueError("workspace must be a contiguous uint8 CUDA tensor")
        ws, ws_bytes = workspace, workspace.numel()
        ws_ptr = ws.data_ptr()
    elif torch_workspace:
        ws_bytes = asn_workspace_size(grid, quad, opt)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device=device)
        ws_ptr = ws.data_ptr()
    stream = torch.cuda.current_stream(device=ws.device if ws is not None else None).cuda_stream
    h = _P()
    _check(_lib.asn_create(ctypes.byref(grid), ctypes.byref(quad), _fptr(fields[0]), _fptr(fields[1]),
                           _fptr(fields[2]), _fptr(src), beta, t_final, ctypes.byref(opt),
                           _P(stream), _P(ws_ptr), ws_bytes, ctypes.byref(h)), "asn_create")
    return AsnProblem(h, grid.nx, grid.ny, q, ws, keep)


def asn_set_state(p: AsnProblem, psi) -> None:
    """psi: numpy float32 [Q, ny, nx] (host) or a contiguous CUDA float32 tensor."""
    if hasattr(psi, "is_cuda") and psi.is_cuda:
        assert psi.dtype.itemsize == 4 and psi.is_contiguous() and psi.numel() == p.q * p.nx * p.ny
        _check(_lib.asn_set_state(p.handle, _P(psi.data_ptr()), 1), "asn_set_state")
        return
    a = _f32(psi)
    if a.size != p.q * p.nx * p.ny:
        raise ValueError("state must have Q * ny * nx entries")
    _check(_lib.asn_set_state(p.handle, a.ctypes.data_as(_P), 0), "asn_set_state")


def asn_set_state_isotropic(p: AsnProblem, psi_cell) -> None:
    a = _f32(psi_cell)
    if a.size != p.nx * p.ny:
        raise ValueError("cell values must have ny * nx entries")
    _check(_lib.asn_set_state_isotropic(p.handle, a.ctypes.data_as(_P), 0), "asn_set_state_isotropic")


def asn_get_state(p: AsnProblem) -> np.ndarray:
    out = np.empty((p.q, p.ny, p.nx), dtype=np.float32)
    _check(_lib.asn_get_state(p.handle, out.ctypes.data_as(_P), 0), "asn_get_state")
    return out


def asn_step(p: AsnProblem, n_steps: int = 1) -> None:
    _check(_lib.asn_step(p.handle, int(n_steps)), "asn_step")


KERNEL_NAMES = ("contraction", "stream_collide", "finalize", "budget", "step")


def asn_step_timed(p: AsnProblem, n_steps: int) -> dict:
    """Steps with HIP events between kernels; average ms per step for each kernel."""
    out = np.zeros(5)
    _check(_lib.asn_step_timed(p.handle, int(n_steps), _dptr(out)), "asn_step_timed")
    return dict(zip(KERNEL_NAMES, out.tolist()))


def asn_step_batch(probs, n_steps: int = 1) -> None:
    arr = (_P * len(probs))(*[p.handle for p in probs])
    _check(_lib.asn_step_batch(arr, len(probs), int(n_steps)), "asn_step_batch")

def asn_step_batch_noalloc(probs, n_steps: int = 1) -> None:
    """asn_step_batch without any device allocation (tables in a static device array)."""
    arr = (_P * len(probs))(*[p.handle for p in probs])
    _check(_lib.asn_step_batch_noalloc(arr, len(probs), int(n_steps)), "asn_step_batch_noalloc")



class AsnBatch:
    """Problems stepped together with fused launches (wraps an asn_batch handle)."""

    def __init__(self, handle, probs):
        self.handle = handle
        self.probs = list(probs)          # keeps the problems alive

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def close(self):
        if self.handle is not None:
            h, self.handle = self.handle, None
            _check(_lib.asn_batch_destroy(h), "asn_batch_destroy")


def asn_batch_create(probs) -> AsnBatch:
    arr = (_P * len(probs))(*[p.handle for p in probs])
    h = _P()
    _check(_lib.asn_batch_create(arr, len(probs), ctypes.byref(h)), "asn_batch_create")
    return AsnBatch(h, probs)


def asn_batch_step(b: AsnBatch, n_steps: int, limits=None) -> None:
    lim = None
    if limits is not None:
        lim_arr = np.ascontiguousarray(limits, dtype=np.int64)
        if lim_arr.size != len(b.probs):
            raise ValueError("one limit per problem")
        lim = lim_arr.ctypes.data_as(_I64)
    _check(_lib.asn_batch_step(b.handle, int(n_steps), lim), "asn_batch_step")


def asn_batch_destroy(b: AsnBatch) -> None:
    b.close()


def asn_scalar_flux(p: AsnProblem) -> np.ndarray:
    out = np.empty((p.ny, p.nx), dtype=np.float64)
    _check(_lib.asn_scalar_flux(p.handle, _dptr(out)), "asn_scalar_flux")
    return out


BUDGET_KEYS = ("mass", "mass0", "absorption", "outflow", "source", "defect", "max_residual",
               "steps")


def asn_mass_budget(p: AsnProblem) -> dict:
    out = np.zeros(ASN_BUDGET_LEN)
    _check(_lib.asn_mass_budget(p.handle, _dptr(out)), "asn_mass_budget")
    return dict(zip(BUDGET_KEYS, out.tolist()))


def asn_info(p: AsnProblem) -> dict:
    dt = ctypes.c_double()
    done = ctypes.c_int64()
    tot = ctypes.c_int64()
    q = ctypes.c_int32()
    _check(_lib.asn_info(p.handle, ctypes.byref(dt), ctypes.byref(done), ctypes.byref(tot),
                         ctypes.byref(q)), "asn_info")
    return {"dt": dt.value, "steps_done": done.value, "steps_to_tfinal": tot.value, "q": q.value}


def asn_step_form(p: AsnProblem) -> str:
    """Kernel form of the problem's steps: "fused", "separate" or "banded"."""
    f = ctypes.c_int32()
    _check(_lib.asn_step_form(p.handle, ctypes.byref(f)), "asn_step_form")
    return {ASN_FORM_FUSED: "fused", ASN_FORM_BANDED: "banded"}.get(f.value, "separate")


def asn_iteration_counts(p: AsnProblem) -> dict:
    """Implicit scheme: transport sweeps and GMRES products since the last set_state."""
    sw = ctypes.c_int64()
    mv = ctypes.c_int64()
    _check(_lib.asn_iteration_counts(p.handle, ctypes.byref(sw), ctypes.byref(mv)),
           "asn_iteration_counts")
    return {"sweeps": sw.value, "matvecs": mv.value}


def asn_stability(p: AsnProblem) -> float:
    """Stability number of the problem's dt (explicit schemes need <= 2)."""
    z = ctypes.c_double()
    _check(_lib.asn_stability(p.handle, ctypes.byref(z)), "asn_stability")
    return z.value


def asn_contraction_work(p: AsnProblem) -> dict:
    d = ctypes.c_double()
    t = ctypes.c_double()
    _check(_lib.asn_contraction_work(p.handle, ctypes.byref(d), ctypes.byref(t)),
           "asn_contraction_work")
    nz = ctypes.c_double()
    _check(_lib.asn_contraction_nonzero(p.handle, ctypes.byref(nz)), "asn_contraction_nonzero")
    return {"dense_flops": d.value, "tile_flops": t.value, "nonzero_flops": nz.value}


def asn_destroy(p: AsnProblem) -> None:
    p.close()


def from_spec(spec, dtype: str = "f32", norm: str = "sym", device: str = "cuda",
              eps_override: float = 0.0, dt_override: float = 0.0,
              set_initial_state: bool = True, scheme: str = "euler",
              dt_rule: str = "streaming", unfused: Optional[bool] = None,
              implicit_tol: float = 0.0, source_tol: float = 0.0,
              source_test: str = "absolute", form: Optional[str] = None,
              scale_block: int = 256) -> AsnProblem:
    """Create a problem from any object with the attributes of a problem description
    (nx, ny, x/y extents, n_polar, n_azim, sigma_*, source, psi0_cell, beta, t_final, cfl)."""
    grid = make_grid(spec.nx, spec.ny, spec.x_min, spec.x_max, spec.y_min, spec.y_max)
    opt = make_options(dtype, norm, spec.cfl, eps_override, dt_override, scheme, dt_rule, unfused,
                       implicit_tol, source_tol, source_test, form, scale_block)
    p = asn_create(grid, spec.n_polar, spec.n_azim, spec.sigma_s, spec.sigma_a, spec.sigma_as,
                   spec.source, spec.beta, spec.t_final, opt, device=device,
                   icosahedron_order=getattr(spec, "ico_order", 0))
    if set_initial_state:
        asn_set_state_isotropic(p, spec.psi0_cell)
    return p
