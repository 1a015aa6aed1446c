"""ctypes binding of libexpint.so: argument marshalling only.

Every computation runs in the library (host FP64 phi_setup, HIP kernels for
everything else).  torch supplies device memory and streams.  There is no
fallback: if the library is missing, importing this module raises.

Tensor layout: a tensor with sizes n_1 x ... x n_d is a C-contiguous torch
tensor of shape (n_d, ..., n_1) (first index fastest in memory).  A small
matrix M (natural indices M[i, j]) lives on the device as the C-contiguous
(n, n) tensor holding M^T, i.e. column-major M.
"""

from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libexpint.so")

# status codes, dtypes, precisions, schemes, nonlinearities (include/expint.h)
OK, EINVAL, ENOMEM, EHIP, ENOTSUP, ENUMERIC, ENONFINITE = 0, -1, -2, -3, -4, -5, -6
F64, C128 = 0, 1
PREC_FP64, PREC_FP32, PREC_BF16X3, PREC_SLICED = 0, 1, 2, 3
ROSENBROCK_EULER = 4  # batched Riccati plans only
SCHEMES = {"lawson_euler": 0, "lawson2b": 1, "exp_euler": 2, "etd2rk": 3}
NONLIN = {"none": 0, "allen_cahn": 1, "u2_1mu": 2, "cubic_nls": 3, "adr_paper": 4}
NOALLOC_SCRATCH_BYTES = 64 << 20  # EXPINT_NOALLOC_SCRATCH_BYTES
PRECISIONS = {"fp64": PREC_FP64, "fp32": PREC_FP32, "bf16x3": PREC_BF16X3, "slice": PREC_SLICED}


class ExpintError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"expint error {code}: {msg}")
        self.code = code


def _load():
    # torch ships its own HIP runtime with the same soname (libamdhip64.so.7) as
    # /opt/rocm's.  Loading torch first makes this library bind to that one
    # runtime, so device pointers and streams from torch are valid here.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2304_02327_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    c_int, c_double, c_void_p, c_size_t = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t
    dp = ctypes.POINTER(c_double)
    lib.phi_setup.argtypes = [c_int, dp, c_int, c_double, c_int, dp, c_int]
    lib.phi_setup_z.argtypes = [c_int, dp, c_int, c_double, c_int, dp, c_int]
    lib.phi_setup_ex.argtypes = [c_int, dp, c_int, c_double, c_int, c_int, c_int, dp, c_int]
    lib.tucker_apply.argtypes = [c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_void_p), c_void_p, c_void_p,
                                 c_double, c_double, c_int, c_int, c_void_p, c_size_t, c_void_p]
    lib.tucker_apply_noalloc.argtypes = [c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_void_p), c_void_p,
                                         c_void_p, c_double, c_double, c_int, c_int, c_void_p]
    lib.tucker_workspace_size.argtypes = [c_int, ctypes.POINTER(c_int), c_int, c_int, ctypes.POINTER(c_size_t)]
    lib.tucker_tune.argtypes = [c_int, ctypes.POINTER(c_int), c_int, c_int, c_void_p]
    lib.expint_plan_describe.argtypes = [c_void_p, ctypes.c_char_p, c_size_t, ctypes.POINTER(c_size_t)]
    lib.tucker_fuses_modes12.argtypes = [c_int, ctypes.POINTER(c_int), c_int, c_int, ctypes.POINTER(c_int)]
    lib.expint_plan_create.argtypes = [ctypes.POINTER(c_void_p), ctypes.c_void_p]
    lib.expint_plan_workspace_size.argtypes = [c_void_p, ctypes.POINTER(c_size_t)]
    lib.expint_plan_set_phi.argtypes = [c_void_p, c_int, c_int, dp]
    lib.expint_step.argtypes = [c_void_p, c_void_p, c_double, c_void_p, c_void_p]
    lib.expint_run.argtypes = [c_void_p, c_void_p, c_double, c_int, c_int, c_void_p, c_void_p]
    lib.expint_plan_is_fused.argtypes = [c_void_p, ctypes.POINTER(c_int)]
    lib.expint_plan_check_finite.argtypes = [c_void_p, c_void_p, c_void_p]
    lib.expint_batch_status.argtypes = [c_void_p, c_void_p, c_void_p]
    lib.expint_plan_destroy.argtypes = [c_void_p]
    lib.expint_plan_destroy.restype = None
    lib.expint_riccati_plan_create.argtypes = [ctypes.POINTER(c_void_p), c_int, ctypes.POINTER(c_int),
                                               ctypes.POINTER(c_int), ctypes.POINTER(dp), ctypes.POINTER(dp),
                                               c_void_p, c_void_p, c_double]
    lib.expint_riccati_plan_create_ex.argtypes = [ctypes.POINTER(c_void_p), c_int, ctypes.POINTER(c_int),
                                                  ctypes.POINTER(c_int), ctypes.POINTER(dp), ctypes.POINTER(dp),
                                                  c_void_p, c_void_p, c_double, c_int]
    lib.expint_batch_state_size.argtypes = [c_void_p, ctypes.POINTER(c_size_t)]
    lib.expint_batch_workspace_size.argtypes = [c_void_p, ctypes.POINTER(c_size_t)]
    lib.expint_batch_step.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]
    lib.expint_batch_run.argtypes = [c_void_p, c_void_p, c_int, c_int, c_void_p, c_void_p]
    lib.expint_batch_tune.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]
    lib.expint_batch_describe.argtypes = [c_void_p, ctypes.c_char_p, c_size_t, ctypes.POINTER(c_size_t)]
    lib.expint_batch_plan_destroy.argtypes = [c_void_p]
    lib.expint_batch_plan_destroy.restype = None
    lib.expint_last_error.restype = ctypes.c_char_p
    lib.expint_version.restype = ctypes.c_char_p
    return lib


lib = _load()

EXPORTED_SYMBOLS = (
    "phi_setup", "phi_setup_z", "phi_setup_ex", "tucker_apply", "tucker_apply_noalloc", "tucker_workspace_size",
    "tucker_fuses_modes12", "tucker_tune",
    "expint_plan_create", "expint_plan_describe", "expint_plan_workspace_size", "expint_plan_set_phi",
    "expint_step", "expint_run", "expint_plan_is_fused", "expint_plan_check_finite", "expint_plan_destroy",
    "expint_last_error",
    "expint_version",
    "expint_riccati_plan_create", "expint_riccati_plan_create_ex", "expint_batch_state_size",
    "expint_batch_workspace_size",
    "expint_batch_step", "expint_batch_run", "expint_batch_status", "expint_batch_tune", "expint_batch_describe",
    "expint_batch_plan_destroy",
)


class _Problem(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int),
        ("n", ctypes.c_int * 4),
        ("A", ctypes.POINTER(ctypes.c_double) * 4),
        ("tau", ctypes.c_double),
        ("scheme", ctypes.c_int),
        ("nonlin", ctypes.c_int),
        ("g_param", ctypes.c_double),
        ("g_param2", ctypes.c_double),
        ("dtype", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("phi_method", ctypes.c_int),
        ("tune", ctypes.c_int),
    ]


def _check(rc: int):
    if rc != OK:
        raise ExpintError(rc, lib.expint_last_error().decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _stream_handle(stream) -> ctypes.c_void_p:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def version() -> str:
    return lib.expint_version().decode()


# ---------------------------------------------------------------------------
# phi_setup (host)
# ---------------------------------------------------------------------------

PHI_METHODS = {"taylor": 0, "quad": 1}


def phi_setup(A: np.ndarray, tau: float, ell_max: int, method: str = "taylor") -> List[np.ndarray]:
    """[phi_0(tau A), ..., phi_{ell_max}(tau A)] computed by the library on the host (FP64).
    method: "taylor" (scaled Taylor series) or "quad" (the paper's quadrature construction)."""
    A = np.asarray(A)
    n = A.shape[0]
    cplx = np.iscomplexobj(A)
    dt = np.complex128 if cplx else np.float64
    Acm = np.asfortranarray(A, dtype=dt)  # column-major
    out = np.zeros((ell_max + 1) * n * n, dtype=dt)
    src = Acm.reshape(-1, order="F").view(np.float64) if cplx else Acm.reshape(-1, order="F")
    src = np.ascontiguousarray(src)
    dst = out.view(np.float64)
    if method == "taylor":
        fn = lib.phi_setup_z if cplx else lib.phi_setup
        _check(fn(n, _dptr(src), n, float(tau), int(ell_max), _dptr(dst), n))
    else:
        _check(lib.phi_setup_ex(n, _dptr(src), n, float(tau), int(ell_max), PHI_METHODS[method],
                                C128 if cplx else F64, _dptr(dst), n))
    return [out[l * n * n:(l + 1) * n * n].reshape((n, n), order="F").copy() for l in range(ell_max + 1)]


# ---------------------------------------------------------------------------
# device helpers
# ---------------------------------------------------------------------------

def matrix_to_device(M: np.ndarray, device="cuda"):
    """Natural-index matrix -> device tensor holding it column-major."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(M).T)).to(device)


def tensor_to_device(U: np.ndarray, device="cuda"):
    """Natural-index tensor (n_1..n_d) -> device tensor in memory order (shape n_d..n_1)."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(U).T)).to(device)


def tensor_from_device(Ut) -> np.ndarray:
    """Inverse of tensor_to_device (returns a natural-index numpy array)."""
    return Ut.detach().cpu().numpy().T


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.complex128:
        return C128
    raise TypeError(f"unsupported dtype {t.dtype} (float64 or complex128)")


def _sizes_of(t) -> List[int]:
    return list(reversed(t.shape))


def _check_device_tensor(t, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


# ---------------------------------------------------------------------------
# tucker_apply
# ---------------------------------------------------------------------------

def _precision_code(precision) -> int:
    return PRECISIONS[precision] if isinstance(precision, str) else int(precision)


def tucker_workspace_size(n: Sequence[int], dtype: int = F64, precision=PREC_FP64) -> int:
    d = len(n)
    arr = (ctypes.c_int * d)(*n)
    out = ctypes.c_size_t(0)
    _check(lib.tucker_workspace_size(d, arr, dtype, _precision_code(precision), ctypes.byref(out)))
    return out.value


def tucker_tune(n: Sequence[int], dtype: int = F64, precision=PREC_FP64, stream=None):
    """Autotune the launch configurations of a tucker_apply of these sizes (synchronous)."""
    d = len(n)
    arr = (ctypes.c_int * d)(*n)
    _check(lib.tucker_tune(d, arr, dtype, _precision_code(precision), _stream_handle(stream)))


def tucker_fuses_modes12(n: Sequence[int], dtype: int = F64, precision=PREC_FP64) -> bool:
    """True if a Tucker operator of these sizes (M_1 and M_2 present) runs modes 1
    and 2 as one launch."""
    d = len(n)
    arr = (ctypes.c_int * d)(*n)
    out = ctypes.c_int(0)
    _check(lib.tucker_fuses_modes12(d, arr, dtype, _precision_code(precision), ctypes.byref(out)))
    return bool(out.value)


def _tucker_args(Ms: Sequence, V, W):
    _check_device_tensor(V, "V")
    _check_device_tensor(W, "W")
    n = _sizes_of(V)
    d = len(n)
    if len(Ms) != d:
        raise ValueError("one matrix (or None) per mode")
    dt = _dtype_code(V)
    ptrs = (ctypes.c_void_p * d)()
    for mu, M in enumerate(Ms):
        if M is None:
            ptrs[mu] = None
        else:
            _check_device_tensor(M, f"M[{mu}]")
            if tuple(M.shape) != (n[mu], n[mu]) or M.dtype != V.dtype:
                raise ValueError(f"M[{mu}] must be {n[mu]}x{n[mu]} of {V.dtype}")
            ptrs[mu] = M.data_ptr()
    return n, d, dt, ptrs


def tucker_apply(Ms: Sequence, V, W, alpha: float = 1.0, beta: float = 0.0,
                 precision=PREC_FP64, ws=None, stream=None):
    """W = alpha * (V x_1 M_1 ... x_d M_d) + beta * W on the device (M_mu = None: identity).
    precision: a PREC_* code or one of "fp64", "fp32", "bf16x3", "slice"."""
    precision = _precision_code(precision)
    import torch
    n, d, dt, ptrs = _tucker_args(Ms, V, W)
    need = tucker_workspace_size(n, dt, precision)
    if ws is None and need > 0:
        ws = torch.empty(need, dtype=torch.uint8, device=V.device)
    ws_ptr = ws.data_ptr() if ws is not None else None
    ws_bytes = ws.numel() * ws.element_size() if ws is not None else 0
    arr = (ctypes.c_int * d)(*n)
    _check(lib.tucker_apply(d, arr, ptrs, V.data_ptr(), W.data_ptr(), float(alpha), float(beta), dt,
                            int(precision), ws_ptr, ws_bytes, _stream_handle(stream)))
    return W


def tucker_apply_noalloc(Ms: Sequence, V, W, alpha: float = 1.0, beta: float = 0.0,
                         precision=PREC_FP64, stream=None):
    """tucker_apply with its intermediates in the library's fixed device scratch array
    (NOALLOC_SCRATCH_BYTES per device): no workspace argument and no allocation.
    Calls that overlap on one device race."""
    precision = _precision_code(precision)
    n, d, dt, ptrs = _tucker_args(Ms, V, W)
    arr = (ctypes.c_int * d)(*n)
    _check(lib.tucker_apply_noalloc(d, arr, ptrs, V.data_ptr(), W.data_ptr(), float(alpha), float(beta), dt,
                                    int(precision), _stream_handle(stream)))
    return W


# ---------------------------------------------------------------------------
# plans
# ---------------------------------------------------------------------------

class Plan:
    """A constant-step integrator for u' = K u + g(u) on one device.

    ``A`` are natural-index host matrices (numpy); ``n`` follows from them.
    """

    def __init__(self, A: Sequence[np.ndarray], tau: float, scheme: str, nonlin: str,
                 g_param: float = 0.0, precision: str = "fp64", device="cuda", g_param2: float = 0.0,
                 phi_method: str = "taylor", tune: bool = True):
        import torch
        A = [np.asarray(a) for a in A]
        cplx = any(np.iscomplexobj(a) for a in A) or nonlin == "cubic_nls"
        self.dtype = C128 if cplx else F64
        self.torch_dtype = torch.complex128 if cplx else torch.float64
        self.n = [a.shape[0] for a in A]
        self.d = len(A)
        self.tau = float(tau)
        self.device = torch.device(device)
        npdt = np.complex128 if cplx else np.float64
        self._host_A = [np.ascontiguousarray(np.asarray(a, dtype=npdt).T) for a in A]  # column-major
        prob = _Problem()
        prob.d = self.d
        for mu in range(4):
            prob.n[mu] = self.n[mu] if mu < self.d else 1
        for mu in range(self.d):
            prob.A[mu] = self._host_A[mu].view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        prob.tau = self.tau
        prob.scheme = SCHEMES[scheme]
        prob.nonlin = NONLIN[nonlin]
        prob.g_param = float(g_param)
        prob.g_param2 = float(g_param2)
        prob.dtype = self.dtype
        prob.precision = PRECISIONS[precision]
        prob.phi_method = PHI_METHODS[phi_method]
        prob.tune = 1 if tune else 0
        self._handle = ctypes.c_void_p(None)
        with torch.cuda.device(self.device):
            _check(lib.expint_plan_create(ctypes.byref(self._handle), ctypes.byref(prob)))
        size = ctypes.c_size_t(0)
        _check(lib.expint_plan_workspace_size(self._handle, ctypes.byref(size)))
        self.workspace_bytes = size.value
        self.ws = torch.empty(max(self.workspace_bytes, 16), dtype=torch.uint8, device=self.device)

    def describe(self) -> str:
        """The launch configuration of each mu-mode product of the plan's steps (tuned or default)."""
        need = ctypes.c_size_t(0)
        _check(lib.expint_plan_describe(self._handle, None, 0, ctypes.byref(need)))
        buf = ctypes.create_string_buffer(need.value)
        _check(lib.expint_plan_describe(self._handle, buf, need.value, None))
        return buf.value.decode()

    @property
    def fused(self) -> bool:
        """True if runs go through the fused small-problem launch (one kernel for all steps)."""
        out = ctypes.c_int(0)
        _check(lib.expint_plan_is_fused(self._handle, ctypes.byref(out)))
        return bool(out.value)

    def set_phi(self, mu: int, ell: int, M: np.ndarray):
        npdt = np.complex128 if self.dtype == C128 else np.float64
        cm = np.ascontiguousarray(np.asarray(M, dtype=npdt).T).view(np.float64)
        _check(lib.expint_plan_set_phi(self._handle, int(mu), int(ell), _dptr(cm)))

    def _check_state(self, U):
        _check_device_tensor(U, "U")
        if _sizes_of(U) != self.n or U.dtype != self.torch_dtype:
            raise ValueError(f"U must have sizes {self.n} (memory order) and dtype {self.torch_dtype}")

    def step(self, U, t: float = 0.0, stream=None):
        self._check_state(U)
        _check(lib.expint_step(self._handle, U.data_ptr(), float(t), self.ws.data_ptr(), _stream_handle(stream)))
        return U

    def run(self, U, nsteps: int, t0: float = 0.0, use_graph: bool = False, stream=None):
        self._check_state(U)
        _check(lib.expint_run(self._handle, U.data_ptr(), float(t0), int(nsteps), 1 if use_graph else 0,
                              self.ws.data_ptr(), _stream_handle(stream)))
        return U

    def check_finite(self, U, stream=None) -> bool:
        """True if every entry of U is finite (waits for the stream)."""
        self._check_state(U)
        rc = lib.expint_plan_check_finite(self._handle, U.data_ptr(), _stream_handle(stream))
        if rc == ENONFINITE:
            return False
        _check(rc)
        return True

    def close(self):
        if getattr(self, "_handle", None) is not None and self._handle.value:
            lib.expint_plan_destroy(self._handle)
            self._handle = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# batched Riccati instances
# ---------------------------------------------------------------------------

def _pack_colmajor(mats):
    """Concatenate matrices in column-major order (natural-index numpy inputs)."""
    return np.concatenate([np.asarray(m, dtype=np.float64).ravel(order="F") for m in mats])


def _unpack_colmajor(flat, shapes):
    out, o = [], 0
    for r, c in shapes:
        out.append(flat[o:o + r * c].reshape((r, c), order="F").copy())
        o += r * c
    return out


class RiccatiBatch:
    """ETD2RK (default) or Rosenbrock-Euler phisplit for many instances of
    U' = A1 U + U A2^T + C + U B U.

    ``instances`` hold natural-index host matrices (A1, A2, B, C, U0).  B and C
    are uploaded once and owned by this object; the state is one packed device
    array (instance i column-major at offset sum_{j<i} n1_j n2_j).
    """

    def __init__(self, instances, tau: float, device="cuda", scheme: str = "etd2rk"):
        import torch
        if scheme not in ("etd2rk", "rosenbrock_euler"):
            raise ValueError("batched Riccati schemes: 'etd2rk' or 'rosenbrock_euler'")
        self.scheme = scheme
        self.n1 = [int(x.n1) for x in instances]
        self.n2 = [int(x.n2) for x in instances]
        self.count = len(instances)
        self.device = torch.device(device)
        self.B = torch.from_numpy(_pack_colmajor([x.B for x in instances])).to(self.device)
        self.C = torch.from_numpy(_pack_colmajor([x.C for x in instances])).to(self.device)
        hostA1 = [np.asfortranarray(x.A1, dtype=np.float64) for x in instances]
        hostA2 = [np.asfortranarray(x.A2, dtype=np.float64) for x in instances]
        a1 = (dp_type() * self.count)(*[m.ctypes.data_as(dp_type()) for m in hostA1])
        a2 = (dp_type() * self.count)(*[m.ctypes.data_as(dp_type()) for m in hostA2])
        n1 = (ctypes.c_int * self.count)(*self.n1)
        n2 = (ctypes.c_int * self.count)(*self.n2)
        self._handle = ctypes.c_void_p(None)
        with torch.cuda.device(self.device):
            _check(lib.expint_riccati_plan_create_ex(ctypes.byref(self._handle), self.count, n1, n2, a1, a2,
                                                     self.B.data_ptr(), self.C.data_ptr(), float(tau),
                                                     SCHEMES[scheme] if scheme == "etd2rk" else ROSENBROCK_EULER))
        size = ctypes.c_size_t(0)
        _check(lib.expint_batch_workspace_size(self._handle, ctypes.byref(size)))
        self.ws = torch.empty(max(size.value, 16), dtype=torch.uint8, device=self.device)
        _check(lib.expint_batch_state_size(self._handle, ctypes.byref(size)))
        self.state_size = size.value

    def state_to_device(self, mats):
        import torch
        return torch.from_numpy(_pack_colmajor(mats)).to(self.device)

    def state_from_device(self, U):
        return _unpack_colmajor(U.detach().cpu().numpy(), list(zip(self.n1, self.n2)))

    def _check_state(self, U):
        import torch
        _check_device_tensor(U, "U")
        if U.dtype != torch.float64 or U.numel() != self.state_size:
            raise ValueError(f"U must be a float64 device tensor of {self.state_size} elements")

    def step(self, U, stream=None):
        self._check_state(U)
        _check(lib.expint_batch_step(self._handle, U.data_ptr(), self.ws.data_ptr(), _stream_handle(stream)))
        return U

    def run(self, U, nsteps: int, use_graph: bool = False, stream=None):
        self._check_state(U)
        _check(lib.expint_batch_run(self._handle, U.data_ptr(), int(nsteps), 1 if use_graph else 0,
                                    self.ws.data_ptr(), _stream_handle(stream)))
        return U

    def tune(self, U, stream=None):
        """Time every grouped tile scheme on every phase (from one step of a copy
        of U; U itself is unchanged) and keep the fastest (expint_batch_tune)."""
        self._check_state(U)
        _check(lib.expint_batch_tune(self._handle, U.data_ptr(), self.ws.data_ptr(), _stream_handle(stream)))

    def describe(self) -> str:
        """The grouped tile scheme of each phase (expint_batch_describe)."""
        need = ctypes.c_size_t(0)
        _check(lib.expint_batch_describe(self._handle, None, 0, ctypes.byref(need)))
        buf = ctypes.create_string_buffer(need.value)
        _check(lib.expint_batch_describe(self._handle, buf, need.value, None))
        return buf.value.decode()

    def status(self, U=None, stream=None) -> int:
        """What the steps since the last call found (waits for the stream): OK,
        ENUMERIC (a phi_1 needed more squarings than the plan has) or ENONFINITE
        (U, if given, or a Jacobian direction holds inf / nan)."""
        if U is not None:
            self._check_state(U)
        rc = lib.expint_batch_status(self._handle, U.data_ptr() if U is not None else None,
                                     _stream_handle(stream))
        if rc not in (OK, ENUMERIC, ENONFINITE):
            _check(rc)
        return rc

    def close(self):
        if getattr(self, "_handle", None) is not None and self._handle.value:
            lib.expint_batch_plan_destroy(self._handle)
            self._handle = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dp_type():
    return ctypes.POINTER(ctypes.c_double)
