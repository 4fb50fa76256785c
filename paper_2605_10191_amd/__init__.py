"""Python binding of the MI355X POLFED library (libpolfed.so).

Argument marshalling only: every computation runs in the HIP library behind
the C ABI of include/polfed.h.  PyTorch provides device memory (tensors whose
data_ptr() is handed to the library) and the stream the library runs on.
The library must be built first (``python -m paper_2605_10191_amd.build``);
importing works without a GPU, calling compute entry points needs one.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpolfed.so")

FP64, FP32 = 0, 1
# solves only: FP32 bulk filtering where its step is clearly faster, else FP64
AUTO = 2
MATRIX_FREE, CSR = 0, 1
TARGET_ABSOLUTE, TARGET_RESCALED, TARGET_NORMALIZED = 0, 1, 2
_TARGETS = {"absolute": 0, "rescaled": 1, "normalized": 2, "maxdos": 3, "offset": 4}

STATUS = {0: "OK", 1: "NOT_CONVERGED", -1: "ERR_INVALID", -2: "ERR_OOM",
          -3: "ERR_HIP", -4: "ERR_BOUNDS", -5: "ERR_BREAKDOWN", -6: "ERR_BUSY",
          -7: "ERR_NODEVICE", -8: "ERR_REJECTED"}


class PolfedError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Plan(ctypes.Structure):
    _fields_ = [("E_c", ctypes.c_double), ("dE", ctypes.c_double),
                ("lambda_t", ctypes.c_double), ("mu_t", ctypes.c_double),
                ("Gamma_t", ctypes.c_double), ("rho", ctypes.c_double),
                ("delta", ctypes.c_double), ("K_approx", ctypes.c_double),
                ("K", ctypes.c_int)]


class Params(ctypes.Structure):
    _fields_ = [("target_kind", ctypes.c_int), ("target", ctypes.c_double),
                ("n_ev", ctypes.c_int), ("precision", ctypes.c_int),
                ("K_override", ctypes.c_int), ("omega", ctypes.c_double),
                ("eta", ctypes.c_double), ("tol_resid", ctypes.c_double),
                ("bound_pad", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("E_min", ctypes.c_double), ("E_max", ctypes.c_double),
                ("graph", ctypes.c_int), ("refine_max", ctypes.c_int),
                ("block_size", ctypes.c_int), ("kpm_moments", ctypes.c_int),
                ("kpm_vectors", ctypes.c_int)]


class Report(ctypes.Structure):
    _fields_ = ([(n, ctypes.c_double) for n in
                 ("E_min", "E_max", "lambda_", "lambda_t", "E_c", "dE", "delta",
                  "rho")] +
                [(n, ctypes.c_int) for n in
                 ("K", "M_alloc", "iters", "n_want", "n_converged", "checks",
                  "restarts", "refine_sweeps")] +
                [(n, ctypes.c_double) for n in
                 ("t_bounds", "t_plan", "t_filter", "t_reorth", "t_check",
                  "t_extract", "t_refine", "t_total", "filter_steps",
                  "filter_bytes", "filter_GBps", "t_queue", "t_latency")] +
                [("fp32_fallback", ctypes.c_int), ("precision", ctypes.c_int),
                 ("mem_peak", ctypes.c_double), ("mem_reserved", ctypes.c_double)])

    def as_dict(self) -> dict:
        d = {n: getattr(self, n) for n, _ in self._fields_}
        d["lambda"] = d.pop("lambda_")
        return d


_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64
_D = ctypes.c_double
_DP = ctypes.POINTER(ctypes.c_double)
_I64P = ctypes.POINTER(ctypes.c_int64)
_I32P = ctypes.POINTER(ctypes.c_int32)

# name -> argtypes; every entry point returns int (polfed_status)
SIGNATURES = {
    "polfed_create": [_I, _P, ctypes.POINTER(_P)],
    "polfed_destroy": [_P],
    "polfed_sync": [_P],
    "polfed_basis_dim": [_I, _I, _I64P],
    "polfed_basis_enumerate": [_P, _I, _I, _P],
    "polfed_basis_rank": [_P, _I, _I, _P, _I64, _P],
    "polfed_basis_unrank": [_P, _I, _I, _P, _I64, _P],
    "polfed_op_xxz": [_P, _I, _I, _D, _D, _DP, _I, ctypes.POINTER(_P)],
    "polfed_op_tv": [_P, _I, _I, _D, _D, _DP, _I, ctypes.POINTER(_P)],
    "polfed_op_qsun": [_P, _I, _I, _DP, _D, _D, _D, _DP, _I32P, _DP,
                       ctypes.POINTER(_P)],
    "polfed_op_csr": [_P, _I64, _I64P, _I32P, _DP, ctypes.POINTER(_P)],
    "polfed_op_qrem": [_P, _I, _DP, _D, ctypes.POINTER(_P)],
    "polfed_op_spin_chain": [_P, _I, _I, _I, _DP, _DP, _DP, _I, ctypes.POINTER(_P)],
    "polfed_op_optimize_mapping": [_P, _P, ctypes.POINTER(_I)],
    "polfed_op_materialize_csr": [_P, _P],
    "polfed_op_set_storage": [_P, _I],
    "polfed_op_set_kernel": [_P, _I, _I, ctypes.POINTER(_I)],
    "polfed_op_set_batch_kernel": [_P, _I, _I, _I, ctypes.POINTER(_I)],
    "polfed_op_dim": [_P, _I64P],
    "polfed_op_nnz": [_P, _I64P],
    "polfed_op_export_csr": [_P, _P, _P, _P, _P, _P],
    "polfed_op_destroy": [_P],
    "polfed_op_apply": [_P, _P, _P, _P],
    "polfed_op_moments": [_P, _P, _DP, _DP],
    "polfed_make_plan": [_I64, _D, _D, _D, _D, _D, _D, _I, _D, _I,
                         ctypes.POINTER(Plan)],
    "polfed_filter_coefficients": [_D, _I, _DP],
    "polfed_filter_value": [_D, _I, _DP, _I64, _DP],
    "polfed_filter_quotient": [_DP, _I, _D, _DP, _DP],
    "polfed_filter_apply": [_P, _P, _D, _D, _DP, _I, _P, _P, _I],
    "polfed_filter_apply_noalloc": [_P, _P, _D, _D, _DP, _I, _P, _P, _I],
    "polfed_clenshaw_step": [_P, _P, _D, _D, _D, _P, _P, _P, _I, _I],
    "polfed_filter_apply_batch": [_P, _I, ctypes.POINTER(_P), _DP, _DP,
                                  ctypes.POINTER(_DP), _I32P, _P, _P, _I],
    "polfed_clenshaw_step_batch": [_P, _I, ctypes.POINTER(_P), _DP, _DP, _DP,
                                   _P, _P, _P, _I, _I],
    "polfed_bounds": [_P, _P, _P, _D, _I, _DP, _DP],
    "polfed_lanczos_step": [_P, _P, _D, _D, _DP, _I, _P, _I, _P, _P, _I],
    "polfed_extract": [_P, _P, _P, _I, _P, _I, _P, _P, _P],
    "polfed_gemm_nn": [_P, _I64, _I, _I, _P, _I64, _P, _I64, _P, _I64, _I],
    "polfed_gemm_tn": [_P, _I64, _I, _I, _P, _I64, _P, _I64, _P, _I64],
    "polfed_kpm_moments": [_P, _P, _D, _D, _I, _I, _P, ctypes.c_uint64, _DP],
    "polfed_kpm_density": [_DP, _I, _DP, _I, _DP],
    "polfed_block_lanczos_step": [_P, _P, _D, _D, _DP, _I, _P, _I, _I, _P, _P, _I],
    "polfed_profile_step": [_P, _P, _I, _I, _DP, _DP],
    "polfed_params_default": [ctypes.POINTER(Params)],
    "polfed_solve": [_P, _P, ctypes.POINTER(Params), _P, _P, _P, _P,
                     ctypes.POINTER(_I), ctypes.POINTER(Report)],
    "polfed_solve_batch": [_P, _I, ctypes.POINTER(_P), ctypes.POINTER(Params),
                           ctypes.POINTER(_P), ctypes.POINTER(_P),
                           ctypes.POINTER(_P), ctypes.POINTER(_P),
                           ctypes.POINTER(_I), ctypes.POINTER(Report)],
    "polfed_serve_start": [_P, ctypes.c_size_t, _I],
    "polfed_submit": [_P, _P, ctypes.POINTER(Params), _P, _P, _P, _P,
                      ctypes.POINTER(_P)],
    "polfed_poll": [_P, ctypes.POINTER(_I)],
    "polfed_wait": [_P, ctypes.POINTER(_I), ctypes.POINTER(Report)],
    "polfed_req_destroy": [_P],
    "polfed_serve_stop": [_P],
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Loads libpolfed.so; raises ImportError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with "
            "`python -m paper_2605_10191_amd.build`")
    # torch first: the library then binds to the HIP runtime torch loaded
    # (same soname), so one runtime serves both in the process
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, args in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.polfed_version.argtypes = []
    lib.polfed_version.restype = ctypes.c_int
    lib.polfed_last_error.argtypes = []
    lib.polfed_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(code: int, ok=(0,)) -> int:
    if code not in ok:
        msg = _lib.polfed_last_error().decode(errors="replace")
        raise PolfedError(code, msg)
    return code


def _dptr(a: np.ndarray, ctype=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


# ------------------------------------------------------------------ host ----

def basis_dim(L: int, N: int) -> int:
    lib = load_library()
    out = ctypes.c_int64()
    _check(lib.polfed_basis_dim(L, N, ctypes.byref(out)))
    return out.value


def make_plan(D, E_min, E_max, pad, lam, tr1, tr2, n_window, omega=0.0,
              K_override=0) -> Plan:
    lib = load_library()
    p = Plan()
    _check(lib.polfed_make_plan(int(D), E_min, E_max, pad, lam, tr1, tr2,
                                int(n_window), omega, int(K_override),
                                ctypes.byref(p)))
    return p


def filter_coefficients(lambda_t: float, K: int) -> np.ndarray:
    lib = load_library()
    a = np.empty(K + 1)
    _check(lib.polfed_filter_coefficients(lambda_t, K, _dptr(a)))
    return a


def filter_value(lambda_t: float, K: int, x) -> np.ndarray:
    lib = load_library()
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty_like(x)
    _check(lib.polfed_filter_value(lambda_t, K, _dptr(x), x.size, _dptr(out)))
    return out


def filter_quotient(a, theta: float):
    """(q, p(theta)): Chebyshev coefficients of (p(x) - p(theta)) / (x - theta)
    for p = sum a_n T_n."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    K = len(a) - 1
    q = np.zeros(max(K, 1))
    p = ctypes.c_double()
    _check(_lib.polfed_filter_quotient(_dptr(a), K, float(theta), _dptr(q), ctypes.byref(p)))
    return q[:K], p.value


def default_params() -> Params:
    lib = load_library()
    p = Params()
    _check(lib.polfed_params_default(ctypes.byref(p)))
    return p


# ---------------------------------------------------------------- device ----

class Context:
    """A library context on one GPU, running on torch's current stream of
    that device (so library work is ordered with torch work)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        lib = load_library()
        self.device = device
        self.torch_device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.torch_device)
        self.stream = stream
        h = ctypes.c_void_p()
        _check(lib.polfed_create(device, ctypes.c_void_p(stream.cuda_stream),
                                 ctypes.byref(h)))
        self.handle = h

    def sync(self):
        _check(_lib.polfed_sync(self.handle))

    def close(self):
        if getattr(self, "handle", None):
            _lib.polfed_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def empty(self, n, dtype=None):
        import torch
        return torch.empty(n, dtype=dtype or torch.float64,
                           device=self.torch_device)

    # --- basis
    def basis_enumerate(self, L: int, N: int):
        import torch
        D = basis_dim(L, N)
        out = torch.empty(D, dtype=torch.int32, device=self.torch_device)
        _check(_lib.polfed_basis_enumerate(self.handle, L, N, _ptr(out)))
        return out

    def basis_rank(self, L: int, N: int, states):
        import torch
        assert states.dtype == torch.int32 and states.is_contiguous()
        out = torch.empty(states.numel(), dtype=torch.int64,
                          device=self.torch_device)
        _check(_lib.polfed_basis_rank(self.handle, L, N, _ptr(states),
                                      states.numel(), _ptr(out)))
        return out

    def basis_unrank(self, L: int, N: int, ranks):
        import torch
        assert ranks.dtype == torch.int64 and ranks.is_contiguous()
        out = torch.empty(ranks.numel(), dtype=torch.int32,
                          device=self.torch_device)
        _check(_lib.polfed_basis_unrank(self.handle, L, N, _ptr(ranks),
                                        ranks.numel(), _ptr(out)))
        return out


class Operator:
    def __init__(self, ctx: Context, handle):
        self.ctx = ctx
        self.handle = handle
        d = ctypes.c_int64()
        _check(_lib.polfed_op_dim(handle, ctypes.byref(d)))
        self.D = d.value

    @classmethod
    def xxz(cls, ctx, L, n_up, J, Delta, h, periodic=True):
        h = np.ascontiguousarray(h, dtype=np.float64)
        out = ctypes.c_void_p()
        _check(_lib.polfed_op_xxz(ctx.handle, L, n_up, J, Delta, _dptr(h),
                                  int(periodic), ctypes.byref(out)))
        return cls(ctx, out)

    @classmethod
    def tv(cls, ctx, L, n_part, t, V, eps, periodic=True):
        eps = np.ascontiguousarray(eps, dtype=np.float64)
        out = ctypes.c_void_p()
        _check(_lib.polfed_op_tv(ctx.handle, L, n_part, t, V, _dptr(eps),
                                 int(periodic), ctypes.byref(out)))
        return cls(ctx, out)

    @classmethod
    def qsun(cls, ctx, N_dot, L, A, gamma, g0, alpha, u, n_of_j, h):
        A = np.ascontiguousarray(A, dtype=np.float64)
        u = np.ascontiguousarray(u, dtype=np.float64)
        n_of_j = np.ascontiguousarray(n_of_j, dtype=np.int32)
        h = np.ascontiguousarray(h, dtype=np.float64)
        out = ctypes.c_void_p()
        _check(_lib.polfed_op_qsun(ctx.handle, N_dot, L, _dptr(A), gamma, g0,
                                   alpha, _dptr(u), _dptr(n_of_j, ctypes.c_int32),
                                   _dptr(h), ctypes.byref(out)))
        return cls(ctx, out)

    @classmethod
    def qrem(cls, ctx, L, E, Gamma):
        """Quantum random energy model on the full 2^L space (E: 2^L
        energies, copied)."""
        E = np.ascontiguousarray(E, dtype=np.float64)
        if E.shape != (1 << L,):
            raise ValueError("E must hold 2^L energies")
        out = ctypes.c_void_p()
        _check(_lib.polfed_op_qrem(ctx.handle, int(L), _dptr(E), float(Gamma),
                                   ctypes.byref(out)))
        return cls(ctx, out)

    @classmethod
    def spin_chain(cls, ctx, L, N, Js, Deltas, h, periodic=True):
        """J1-J2(-J3...) chain: couplings of range 1..len(Js), CSR storage."""
        Js = np.ascontiguousarray(Js, dtype=np.float64)
        Ds = np.ascontiguousarray(Deltas, dtype=np.float64)
        h = np.ascontiguousarray(h, dtype=np.float64)
        if Js.shape != Ds.shape or h.shape != (L,):
            raise ValueError("need len(Js) == len(Deltas) and L fields")
        out = ctypes.c_void_p()
        _check(_lib.polfed_op_spin_chain(ctx.handle, int(L), int(N), len(Js), _dptr(Js),
                                         _dptr(Ds), _dptr(h), int(periodic), ctypes.byref(out)))
        return cls(ctx, out)

    @classmethod
    def csr(cls, ctx, D, rowptr, col, val):
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
        out = ctypes.c_void_p()
        _check(_lib.polfed_op_csr(ctx.handle, int(D),
                                  _dptr(rowptr, ctypes.c_int64),
                                  _dptr(col, ctypes.c_int32), _dptr(val),
                                  ctypes.byref(out)))
        return cls(ctx, out)

    def materialize_csr(self):
        _check(_lib.polfed_op_materialize_csr(self.ctx.handle, self.handle))
        return self

    def optimize_mapping(self) -> int:
        """Value table + one-byte codes for the CSR copy; returns the number
        of distinct off-diagonal values (257: more than 256, unchanged)."""
        n = _I()
        _check(_lib.polfed_op_optimize_mapping(self.ctx.handle, self.handle, ctypes.byref(n)))
        return n.value

    def set_storage(self, storage: int):
        _check(_lib.polfed_op_set_storage(self.handle, storage))
        return self

    def set_kernel(self, precision: int, variant: int) -> int:
        """Step-kernel variant for a chain (-1 autotuned, 0 segment, 3 paired
        rows, 4 half segments, 1/2/5 tile kernels with the largest, middle
        and smallest tile, 6-9 staged-tile kernels), or the tile size in bits
        for QREM (-1 autotuned); returns the variant in use."""
        out = _I()
        _check(_lib.polfed_op_set_kernel(self.handle, precision, variant, ctypes.byref(out)))
        return out.value

    def set_batch_kernel(self, B: int, precision: int, variant: int) -> int:
        """Multi-column step kernel for batches of B realizations of this
        pattern (-1 autotuned, 0/1 column-major with 16/8 columns per launch,
        2/3 interleaved with 2/4 workgroups per CU, 4 each column by its own
        single-column kernel, L >= 22, 5 the LDS-resident whole filter for
        short chains); returns the variant in use (-1 while not tuned)."""
        out = _I()
        _check(_lib.polfed_op_set_batch_kernel(self.handle, int(B), precision, variant,
                                               ctypes.byref(out)))
        return out.value

    @property
    def nnz(self) -> int:
        n = ctypes.c_int64()
        _check(_lib.polfed_op_nnz(self.handle, ctypes.byref(n)))
        return n.value

    def export_csr(self):
        import torch
        dev = self.ctx.torch_device
        nnz = self.nnz
        rowptr = torch.empty(self.D + 1, dtype=torch.int64, device=dev)
        col = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
        val = torch.empty(max(nnz, 1), dtype=torch.float64, device=dev)
        diag = torch.empty(self.D, dtype=torch.float64, device=dev)
        _check(_lib.polfed_op_export_csr(self.ctx.handle, self.handle,
                                         _ptr(rowptr), _ptr(col), _ptr(val),
                                         _ptr(diag)))
        return rowptr, col[:nnz], val[:nnz], diag

    def apply(self, x, y=None):
        if y is None:
            y = self.ctx.empty(self.D)
        _check(_lib.polfed_op_apply(self.ctx.handle, self.handle, _ptr(x),
                                    _ptr(y)))
        return y

    def moments(self):
        t1, t2 = ctypes.c_double(), ctypes.c_double()
        _check(_lib.polfed_op_moments(self.ctx.handle, self.handle,
                                      ctypes.byref(t1), ctypes.byref(t2)))
        return t1.value, t2.value

    def close(self):
        if getattr(self, "handle", None):
            _lib.polfed_op_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def filter_apply(op: Operator, E_c, dE, a, v, precision=FP64, w=None):
    import torch
    a = np.ascontiguousarray(a, dtype=np.float64)
    K = len(a) - 1
    if w is None:
        w = torch.empty_like(v)
    _check(_lib.polfed_filter_apply(op.ctx.handle, op.handle, E_c, dE,
                                    _dptr(a), K, _ptr(v), _ptr(w), precision))
    return w


def filter_apply_noalloc(op: Operator, E_c, dE, a, v, w, precision=FP64):
    """filter_apply into the caller's w with the recurrence buffers in the
    library's static device scratch (no device allocation, asynchronous)."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    _check(_lib.polfed_filter_apply_noalloc(op.ctx.handle, op.handle, E_c, dE, _dptr(a),
                                            len(a) - 1, _ptr(v), _ptr(w), precision))
    return w


def clenshaw_step(op: Operator, E_c, dE, a_i, v, b1, b2, precision=FP64,
                  final=False):
    _check(_lib.polfed_clenshaw_step(op.ctx.handle, op.handle, E_c, dE, a_i,
                                     _ptr(v), _ptr(b1), _ptr(b2), precision,
                                     int(final)))
    return b2


def _op_array(ops):
    ctx = ops[0].ctx
    for o in ops:
        if o.ctx is not ctx:
            raise ValueError("operators belong to different contexts")
    return (_P * len(ops))(*[o.handle for o in ops]), ctx


def filter_apply_batch(ops, E_c, dE, a, v, precision=FP64, w=None):
    """Column c of the (B, D) device block w gets P_c(H~_c) v_c for chain
    operators sharing one off-diagonal pattern; a is a list of B coefficient
    arrays (orders may differ)."""
    import torch
    B = len(ops)
    arr, ctx = _op_array(ops)
    Ec = np.ascontiguousarray(E_c, dtype=np.float64)
    dE_ = np.ascontiguousarray(dE, dtype=np.float64)
    coef = [np.ascontiguousarray(x, dtype=np.float64) for x in a]
    K = np.array([len(x) - 1 for x in coef], dtype=np.int32)
    aptr = (_DP * B)(*[_dptr(x) for x in coef])
    if w is None:
        w = torch.empty_like(v)
    _check(_lib.polfed_filter_apply_batch(ctx.handle, B, arr, _dptr(Ec), _dptr(dE_),
                                          aptr, K.ctypes.data_as(_I32P), _ptr(v),
                                          _ptr(w), precision))
    return w


def clenshaw_step_batch(ops, E_c, dE, a_i, v, b1, b2, precision=FP64, final=False):
    B = len(ops)
    arr, ctx = _op_array(ops)
    Ec = np.ascontiguousarray(E_c, dtype=np.float64)
    dE_ = np.ascontiguousarray(dE, dtype=np.float64)
    ai = np.ascontiguousarray(a_i, dtype=np.float64)
    _check(_lib.polfed_clenshaw_step_batch(ctx.handle, B, arr, _dptr(Ec), _dptr(dE_),
                                           _dptr(ai), _ptr(v), _ptr(b1), _ptr(b2),
                                           precision, int(final)))
    return b2


def bounds(op: Operator, x0, tol=1e-10, max_iter=300):
    lo, hi = ctypes.c_double(), ctypes.c_double()
    _check(_lib.polfed_bounds(op.ctx.handle, op.handle, _ptr(x0), tol,
                              max_iter, ctypes.byref(lo), ctypes.byref(hi)))
    return lo.value, hi.value


def lanczos_step(op: Operator, E_c, dE, a, V, k, alpha, beta, precision=FP64):
    """One filtered Lanczos step on the device basis V (a (k+2, D) tensor,
    rows = basis vectors); alpha and beta are one-element device tensors."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    _check(_lib.polfed_lanczos_step(op.ctx.handle, op.handle, E_c, dE, _dptr(a),
                                    len(a) - 1, _ptr(V), int(k), _ptr(alpha),
                                    _ptr(beta), precision))


def extract(op: Operator, V, T):
    """Ritz vectors u_j = V t_j and Rayleigh-Ritz with H on their span.
    V: (m, D) device tensor (rows = basis vectors), T: (n, m) device tensor
    (rows = the chosen eigenvectors of the Lanczos matrix).  Returns E (n,
    ascending), U2 ((n, D), rows = Ritz vectors) and the residual norms."""
    import torch
    m, n = V.shape[0], T.shape[0]
    E = torch.empty(n, dtype=torch.float64, device=V.device)
    U2 = torch.empty((n, op.D), dtype=torch.float64, device=V.device)
    R = torch.empty(n, dtype=torch.float64, device=V.device)
    _check(_lib.polfed_extract(op.ctx.handle, op.handle, _ptr(V), int(m), _ptr(T), int(n),
                               _ptr(E), _ptr(U2), _ptr(R)))
    return E, U2, R


def gemm_nn(ctx: Context, A, B, C, subtract=False):
    """C = A B (or C -= A B) for column-major matrices held as transposed
    row-major tensors: A (m, D), B (n, m), C (n, D)."""
    m, D = A.shape
    n = B.shape[0]
    _check(_lib.polfed_gemm_nn(ctx.handle, int(D), int(m), int(n), _ptr(A), int(max(D, 1)),
                               _ptr(B), int(max(m, 1)), _ptr(C), int(max(D, 1)),
                               int(bool(subtract))))


def gemm_tn(ctx: Context, A, B, G):
    """G = A^T B for column-major A (D x n1) and B (D x n2) held as (n1, D)
    and (n2, D) tensors; G (n1 x n2 column-major) is an (n2, n1) tensor."""
    n1, D = A.shape
    n2 = B.shape[0]
    _check(_lib.polfed_gemm_tn(ctx.handle, int(D), int(n1), int(n2), _ptr(A), int(max(D, 1)),
                               _ptr(B), int(max(D, 1)), _ptr(G), int(max(n1, 1))))


def block_lanczos_step(op: Operator, E_c, dE, a, V, k, s, A, Bn, precision=FP64):
    """One filtered block Lanczos step on the device basis V (a (k+2s, D)
    tensor, rows = basis vectors); A and Bn are (s, s) device tensors that
    receive A_j and B_{j+1} column-major (so A[c, i] is row i, column c)."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    _check(_lib.polfed_block_lanczos_step(op.ctx.handle, op.handle, E_c, dE, _dptr(a),
                                          len(a) - 1, _ptr(V), int(k), int(s), _ptr(A),
                                          _ptr(Bn), precision))


def kpm_moments(op: Operator, E_c, dE, N, R, vectors=None, seed=0) -> np.ndarray:
    """KPM moments mu_0..mu_{N-1} of H~ = (H - E_c)/dE averaged over R random
    vectors: `vectors` is a (R, D) device tensor (rows = vectors), or None for
    the library's counter-based draws from `seed`."""
    mu = np.zeros(int(N))
    _check(_lib.polfed_kpm_moments(op.ctx.handle, op.handle, float(E_c), float(dE), int(N),
                                   int(R), _ptr(vectors) if vectors is not None else None,
                                   int(seed), _dptr(mu)))
    return mu


def kpm_density(mu, x) -> np.ndarray:
    """Jackson-damped KPM density at the points x (host)."""
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    x = np.ascontiguousarray(np.atleast_1d(x), dtype=np.float64)
    rho = np.zeros_like(x)
    _check(_lib.polfed_kpm_density(_dptr(mu), len(mu), _dptr(x), len(x), _dptr(rho)))
    return rho


def profile_step(op: Operator, precision=FP64, iters=200):
    """(mean, min) milliseconds of the fused Clenshaw step kernel."""
    avg, mn = ctypes.c_double(), ctypes.c_double()
    _check(_lib.polfed_profile_step(op.ctx.handle, op.handle, precision,
                                    int(iters), ctypes.byref(avg),
                                    ctypes.byref(mn)))
    return avg.value, mn.value


def make_params(n_ev, target, target_kind="normalized", precision=FP64,
                **kw) -> Params:
    p = default_params()
    p.n_ev = n_ev
    p.target = target
    p.target_kind = _TARGETS[target_kind] if isinstance(target_kind, str) \
        else int(target_kind)
    p.precision = precision
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def solve(op: Operator, x0, n_ev, target, target_kind="normalized",
          precision=FP64, allow_partial=False, **kw):
    """N_ev eigenpairs of op nearest the target.  Returns
    (evals, evecs (D x n, column-major as a (n, D) tensor transposed), resid,
    report dict, status).  A start vector x0 of shape (D,) runs Lanczos; a
    start block of shape (s, D) (rows = columns of the D x s block) runs block
    Lanczos with block size s."""
    if hasattr(x0, "dim") and x0.dim() == 2:
        if kw.get("block_size", x0.shape[0]) != x0.shape[0]:
            raise ValueError("block_size differs from the rows of the start block")
        kw["block_size"] = int(x0.shape[0])
        if not x0.is_contiguous():
            raise ValueError("the start block must be contiguous")
    elif kw.get("block_size", 1) > 1:
        raise ValueError("block_size > 1 needs a start block of shape (s, D)")
    p = make_params(n_ev, target, target_kind, precision, **kw)
    ctx = op.ctx
    evals = ctx.empty(n_ev)
    evecs = ctx.empty(n_ev * op.D)
    resid = ctx.empty(n_ev)
    nf = ctypes.c_int()
    rep = Report()
    code = _lib.polfed_solve(ctx.handle, op.handle, ctypes.byref(p), _ptr(x0),
                             _ptr(evals), _ptr(evecs), _ptr(resid),
                             ctypes.byref(nf), ctypes.byref(rep))
    _check(code, ok=(0, 1) if allow_partial else (0,))
    n = nf.value
    return (evals[:n], evecs.view(n_ev, op.D)[:n].T, resid[:n], rep.as_dict(),
            STATUS[code])


def solve_batch(ops, x0s, n_ev, target, target_kind="normalized", precision=FP64,
                allow_partial=False, **kw):
    """Batched solve of chain realizations sharing the off-diagonal pattern.
    Returns a list of (evals, evecs, resid, report dict) and the status."""
    B = len(ops)
    arr, ctx = _op_array(ops)
    p = make_params(n_ev, target, target_kind, precision, **kw)
    evals = [ctx.empty(n_ev) for _ in ops]
    evecs = [ctx.empty(n_ev * o.D) for o in ops]
    resid = [ctx.empty(n_ev) for _ in ops]
    nf = (_I * B)()
    reps = (Report * B)()
    ptrs = lambda ts: (_P * B)(*[_ptr(t) for t in ts])
    code = _lib.polfed_solve_batch(ctx.handle, B, arr, ctypes.byref(p), ptrs(x0s),
                                   ptrs(evals), ptrs(evecs), ptrs(resid), nf, reps)
    _check(code, ok=(0, 1) if allow_partial else (0,))
    out = []
    for i, o in enumerate(ops):
        n = nf[i]
        out.append((evals[i][:n], evecs[i].view(n_ev, o.D)[:n].T, resid[i][:n],
                    reps[i].as_dict()))
    return out, STATUS[code]


class Request:
    """A solve queued on a Server; keeps its start vector and output tensors
    alive until the result has been collected."""

    def __init__(self, server, op, x0, n_ev, params):
        self.server, self.op, self.x0, self.n_ev = server, op, x0, n_ev
        ctx = op.ctx
        self.evals = ctx.empty(n_ev)
        self.evecs = ctx.empty(n_ev * op.D)
        self.resid = ctx.empty(n_ev)
        self.params = params
        self.handle = _P()
        _check(_lib.polfed_submit(ctx.handle, op.handle, ctypes.byref(params),
                                  _ptr(x0), _ptr(self.evals), _ptr(self.evecs),
                                  _ptr(self.resid), ctypes.byref(self.handle)))
        self.result = None

    def poll(self) -> bool:
        d = _I()
        _check(_lib.polfed_poll(self.handle, ctypes.byref(d)))
        return bool(d.value)

    def wait(self, allow_partial=False):
        """(evals, evecs (D x n), resid, report dict, status)."""
        if self.result is None:
            nf = _I()
            rep = Report()
            code = _lib.polfed_wait(self.handle, ctypes.byref(nf), ctypes.byref(rep))
            msg = _lib.polfed_last_error().decode(errors="replace") if code < 0 else ""
            _lib.polfed_req_destroy(self.handle)
            self.handle = None
            if code < 0:
                raise PolfedError(code, msg)
            if code == 1 and not allow_partial:
                raise PolfedError(code, "not converged")
            n = nf.value
            self.result = (self.evals[:n], self.evecs.view(self.n_ev, self.op.D)[:n].T,
                           self.resid[:n], rep.as_dict(), STATUS[code])
        return self.result


class Server:
    """Continuous-batching solve server on a context: requests are admitted
    while their Krylov bases fit `hbm_budget_bytes` and fewer than `max_cols`
    solves run; solves of chains sharing one pattern filter together."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int, max_cols: int = 16):
        self.ctx = ctx
        _check(_lib.polfed_serve_start(ctx.handle, ctypes.c_size_t(int(hbm_budget_bytes)),
                                       int(max_cols)))
        self.running = True

    def submit(self, op: Operator, x0, n_ev, target, target_kind="normalized",
               precision=FP64, **kw) -> Request:
        p = make_params(n_ev, target, target_kind, precision, **kw)
        return Request(self, op, x0, n_ev, p)

    def stop(self):
        """Finishes every submitted request, then stops the scheduler."""
        if self.running:
            self.running = False
            _check(_lib.polfed_serve_stop(self.ctx.handle))

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.stop()
