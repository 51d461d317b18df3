"""ctypes binding of librtg.so (C ABI in include/rtg.h).

Argument marshalling only: every step of the solver runs in the HIP library.
PyTorch provides device memory and the current stream.  Tensors use the
device layout of the library: a C-contiguous torch tensor of shape
(J, I2, I1), i.e. column-major X[i1, i2, j] with i1 fastest.

The functions keep the names of the C entry points without the ``rtg_``
prefix: setup_operator, setup_operator_psf, apply_operator, setup_sketch, sketch,
sketch_noalloc, workspace_bytes, gk_workspace_bytes, arnoldi, golub_kahan, workspace_layout,
gk_workspace_layout, solve, solve_batched.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librtg.so")
HEADER = os.path.join(HERE, "..", "include", "rtg.h")

F32, BF16 = 0, 1
F32_BF16 = 2      # basis type: float32 storage, bfloat16 sketch products
FLAG_BREAKDOWN, FLAG_DISCREP_UNREACHABLE, FLAG_MU_INF, FLAG_NONFINITE, FLAG_NOT_CONVERGED = 1, 2, 4, 8, 16
FLAG_FALLBACK = 32
FLAG_TIMEOUT = 64


class RTGError(RuntimeError):
    pass


class Params(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int), ("basis_dtype", ctypes.c_int), ("mu", ctypes.c_double),
                ("delta", ctypes.c_double), ("eta", ctypes.c_double), ("stop_res", ctypes.c_double),
                ("bd_tol", ctypes.c_double), ("mu_rule", ctypes.c_int), ("method", ctypes.c_int),
                ("restarts", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("flags", ctypes.c_int), ("mu", ctypes.c_double),
                ("beta", ctypes.c_double), ("res_proj", ctypes.c_double), ("res_ls", ctypes.c_double)]


class Problem(ctypes.Structure):
    _fields_ = [("op", ctypes.c_void_p), ("sk", ctypes.c_void_p), ("C", ctypes.c_void_p),
                ("X0", ctypes.c_void_p), ("X", ctypes.c_void_p), ("params", Params),
                ("info", ctypes.c_void_p)]


class Tune(ctypes.Structure):
    """Launch shapes of a batch (rtg_tune); -1 = the library default."""
    _fields_ = [("phi_jt", ctypes.c_int), ("phi_slab", ctypes.c_int), ("phi_toeplitz", ctypes.c_int),
                ("tile_rows", ctypes.c_int), ("step_rows", ctypes.c_int), ("step_toeplitz", ctypes.c_int),
                ("gram_pairs", ctypes.c_int), ("persist", ctypes.c_int)]

    FIELDS = ("phi_jt", "phi_slab", "phi_toeplitz", "tile_rows", "step_rows", "step_toeplitz", "gram_pairs",
              "persist")

    def as_dict(self):
        return {f: int(getattr(self, f)) for f in self.FIELDS}


def make_tune(**fields) -> Tune:
    t = Tune()
    for f in Tune.FIELDS:
        setattr(t, f, int(fields.pop(f, -1)))
    if fields:
        raise RTGError(f"unknown tune fields {sorted(fields)}")
    return t


def header_symbols() -> List[str]:
    """Entry points declared in include/rtg.h."""
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(rtg_[a-z_]+)\s*\(", text)))


def load_library():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(python -m paper_2603_00839_amd.build_lib)")
    lib = ctypes.CDLL(LIB_PATH)
    c_int, c_vp, c_sz, c_d = ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_double
    fp = ctypes.POINTER(ctypes.c_float)
    sig = {
        "rtg_setup_operator": (c_int, [c_int, c_int, c_int, fp, c_int, fp, c_int, fp, c_int, ctypes.POINTER(c_vp)]),
        "rtg_apply_operator": (c_int, [c_vp, c_int, c_vp, c_vp, c_vp, c_vp]),
        "rtg_destroy_operator": (c_int, [c_vp]),
        "rtg_setup_sketch": (c_int, [c_int, c_int, c_int, c_int, c_int, c_int, fp, fp, fp, ctypes.POINTER(c_vp)]),
        "rtg_sketch_workspace_bytes": (c_sz, [c_vp]),
        "rtg_sketch": (c_int, [c_vp, c_int, c_vp, c_vp, c_vp, c_sz, c_vp]),
        "rtg_sketch_noalloc": (c_int, [c_vp, c_int, c_vp, c_vp, c_vp]),
        "rtg_destroy_sketch": (c_int, [c_vp]),
        "rtg_workspace_bytes": (c_sz, [c_vp, c_vp, c_int, c_int]),
        "rtg_setup_operator_psf": (c_int, [c_int, c_int, c_int, c_vp, c_int, c_vp, c_int, c_vp]),
        "rtg_gk_workspace_bytes": (c_sz, [c_vp, c_vp, c_int, c_int]),
        "rtg_arnoldi": (c_int, [c_vp, c_vp, c_vp, c_int, c_int, c_d, c_vp, c_sz, c_vp, c_vp, c_vp, c_vp]),
        "rtg_workspace_layout": (c_int, [c_vp, c_vp, c_int, c_int, ctypes.POINTER(c_sz), ctypes.POINTER(c_sz)]),
        "rtg_golub_kahan": (c_int, [c_vp, c_vp, c_vp, c_int, c_int, c_d, c_vp, c_sz, c_vp, c_vp, c_vp, c_vp]),
        "rtg_gk_workspace_layout": (c_int, [c_vp, c_vp, c_int, c_int, ctypes.POINTER(c_sz),
                                            ctypes.POINTER(c_sz)]),
        "rtg_solve": (c_int, [c_vp, c_vp, c_vp, c_vp, ctypes.POINTER(Params), c_vp, c_sz, c_vp, c_vp, c_vp]),
        "rtg_batch_workspace_bytes": (c_sz, [c_int, ctypes.POINTER(Problem)]),
        "rtg_solve_batched": (c_int, [c_int, ctypes.POINTER(Problem), c_vp, c_sz, c_vp]),
        "rtg_fallback_workspace_bytes": (c_sz, [c_int, ctypes.POINTER(Problem), c_int, c_int]),
        "rtg_solve_batched_fallback": (c_int, [c_int, ctypes.POINTER(Problem), c_int, c_int, c_int, c_vp, c_sz,
                                               ctypes.POINTER(c_int), c_vp]),
        "rtg_solve_batched_fallback_begin": (c_int, [c_int, ctypes.POINTER(Problem), c_int, c_int, c_int, c_vp,
                                                     c_sz, c_vp, c_vp]),
        "rtg_solve_batched_fallback_end": (c_int, [c_int, ctypes.POINTER(Problem), c_int, c_int, c_int, c_vp,
                                                   c_sz, c_vp, ctypes.POINTER(c_int), c_vp]),
        "rtg_autotune_batched": (c_int, [c_int, ctypes.POINTER(Problem), c_vp, c_sz, c_int, ctypes.POINTER(Tune),
                                         ctypes.POINTER(c_d), c_vp]),
        "rtg_tune_set": (c_int, [c_int, ctypes.POINTER(Problem), ctypes.POINTER(Tune)]),
        "rtg_tune_get": (c_int, [c_int, ctypes.POINTER(Problem), ctypes.POINTER(Tune)]),
        "rtg_tune_clear": (c_int, []),
        "rtg_set_wait_limit": (c_int, [c_int]),
        "rtg_cnn_state_bytes": (c_sz, []),
        "rtg_cnn_workspace_bytes": (c_sz, [c_int, c_int, c_int]),
        "rtg_cnn_init": (c_int, [c_vp, fp, c_vp]),
        "rtg_cnn_export": (c_int, [c_vp, fp, c_vp]),
        "rtg_cnn_forward": (c_int, [c_vp, c_vp, c_int, c_int, c_int, c_vp, c_vp, c_sz, c_vp]),
        "rtg_cnn_gradients": (c_int, [c_vp, c_vp, c_vp, c_int, c_int, c_int, c_vp, c_sz, c_vp, c_vp]),
        "rtg_cnn_read_gradients": (c_int, [c_vp, fp, c_vp]),
        "rtg_cnn_adam": (c_int, [c_vp, ctypes.c_float, c_int, c_vp]),
        "rtg_event_timing_enable": (c_int, [c_int]),
        "rtg_event_timing_read": (c_int, [ctypes.POINTER(c_d), ctypes.POINTER(ctypes.c_longlong), c_int]),
        "rtg_status_string": (ctypes.c_char_p, [c_int]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


def _check(rc: int, what: str):
    if rc != 0:
        raise RTGError(f"{what}: {lib().rtg_status_string(rc).decode()} ({rc})")


def _fptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.bfloat16:
        return BF16
    raise RTGError(f"unsupported dtype {t.dtype}")


def _check_tensor(t, shape, name):
    if not t.is_cuda or not t.is_contiguous():
        raise RTGError(f"{name} must be a contiguous device tensor")
    if tuple(t.shape) != tuple(shape):
        raise RTGError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


# ---------------------------------------------------------------------------
# operator
# ---------------------------------------------------------------------------
class Operator:
    """Handle of rtg_setup_operator; bands are (I, 2r+1) float32 host arrays."""

    def __init__(self, I1, I2, J, a1_band, a2_band, b_band):
        self.shape = (int(I1), int(I2), int(J))
        a1 = np.ascontiguousarray(a1_band, dtype=np.float32)
        a2 = np.ascontiguousarray(a2_band, dtype=np.float32)
        bb = np.ascontiguousarray(b_band, dtype=np.float32)
        self.r1, self.r2, self.rB = (a1.shape[1] - 1) // 2, (a2.shape[1] - 1) // 2, (bb.shape[1] - 1) // 2
        h = ctypes.c_void_p()
        _check(lib().rtg_setup_operator(I1, I2, J, _fptr(a1), self.r1, _fptr(a2), self.r2, _fptr(bb),
                                        self.rB, ctypes.byref(h)), "rtg_setup_operator")
        self.handle = h

    @property
    def device_shape(self):
        I1, I2, J = self.shape
        return (J, I2, I1)

    def close(self):
        if self.handle:
            lib().rtg_destroy_operator(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def setup_operator(I1, I2, J, a1_band, a2_band, b_band) -> Operator:
    return Operator(I1, I2, J, a1_band, a2_band, b_band)


class PSFOperator(Operator):
    """Handle of rtg_setup_operator_psf: a general (2r+1) x (2r+1) PSF
    (float32 host array, row index along i1) and the band of B."""

    def __init__(self, I1, I2, J, psf, b_band):
        self.shape = (int(I1), int(I2), int(J))
        P = np.ascontiguousarray(psf, dtype=np.float32)
        bb = np.ascontiguousarray(b_band, dtype=np.float32)
        if P.ndim != 2 or P.shape[0] != P.shape[1] or P.shape[0] % 2 != 1:
            raise RTGError("psf must be (2r+1) x (2r+1)")
        r = (P.shape[0] - 1) // 2
        self.r1 = self.r2 = r
        self.rB = (bb.shape[1] - 1) // 2
        h = ctypes.c_void_p()
        _check(lib().rtg_setup_operator_psf(I1, I2, J, _fptr(P), r, _fptr(bb), self.rB, ctypes.byref(h)),
               "rtg_setup_operator_psf")
        self.handle = h


def setup_operator_psf(I1, I2, J, psf, b_band) -> PSFOperator:
    return PSFOperator(I1, I2, J, psf, b_band)


def destroy_operator(op: Operator):
    op.close()


def apply_operator(op: Operator, X, C=None, out=None):
    """Y = Phi(X) or, with C, Y = C - Phi(X) (float32 result)."""
    torch = _torch()
    _check_tensor(X, op.device_shape, "X")
    if C is not None:
        _check_tensor(C, op.device_shape, "C")
    if out is None:
        out = torch.empty(op.device_shape, dtype=torch.float32, device=X.device)
    _check(lib().rtg_apply_operator(op.handle, _dtype_code(X), _ptr(X), _ptr(C), _ptr(out), _stream()),
           "rtg_apply_operator")
    return out


# ---------------------------------------------------------------------------
# sketch
# ---------------------------------------------------------------------------
class Sketch:
    """Handle of rtg_setup_sketch; Om_k are (l_k, I_k) float32 arrays or None.
    With all three None the sketch is the identity: the solver then runs the
    unsketched method (Frobenius inner products of the full tensors)."""

    def __init__(self, I1, I2, J, om1=None, om2=None, om3=None):
        self.shape = (int(I1), int(I2), int(J))
        o = [None if x is None else np.ascontiguousarray(x, dtype=np.float32) for x in (om1, om2, om3)]
        self.l = tuple(d if x is None else x.shape[0] for x, d in zip(o, self.shape))
        self._keep = o
        self.identity = all(x is None for x in o)
        h = ctypes.c_void_p()
        _check(lib().rtg_setup_sketch(I1, I2, J, self.l[0], self.l[1], self.l[2], _fptr(o[0]), _fptr(o[1]),
                                      _fptr(o[2]), ctypes.byref(h)), "rtg_setup_sketch")
        self.handle = h

    @property
    def L(self):
        return self.l[0] * self.l[1] * self.l[2]

    def close(self):
        if self.handle:
            lib().rtg_destroy_sketch(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def setup_sketch(I1, I2, J, om1=None, om2=None, om3=None) -> Sketch:
    return Sketch(I1, I2, J, om1, om2, om3)


def destroy_sketch(sk: Sketch):
    sk.close()


def sketch(sk: Sketch, X, ws=None):
    """S(X) as a float32 device tensor of shape (l3, l2, l1) (column-major
    S[a, b, c] with a fastest, like the tensors)."""
    torch = _torch()
    I1, I2, J = sk.shape
    _check_tensor(X, (J, I2, I1), "X")
    nbytes = lib().rtg_sketch_workspace_bytes(sk.handle)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=X.device)
    out = torch.empty((sk.l[2], sk.l[1], sk.l[0]), dtype=torch.float32, device=X.device)
    _check(lib().rtg_sketch(sk.handle, _dtype_code(X), _ptr(X), _ptr(out), _ptr(ws), ws.numel(), _stream()),
           "rtg_sketch")
    return out


def sketch_noalloc(sk: Sketch, X, out):
    """S(X) into the caller's float32 device tensor out (shape (l3, l2, l1))
    through rtg_sketch_noalloc: no workspace, nothing allocated."""
    I1, I2, J = sk.shape
    _check_tensor(X, (J, I2, I1), "X")
    _check_tensor(out, (sk.l[2], sk.l[1], sk.l[0]), "out")
    _check(lib().rtg_sketch_noalloc(sk.handle, _dtype_code(X), _ptr(X), _ptr(out), _stream()),
           "rtg_sketch_noalloc")
    return out


# ---------------------------------------------------------------------------
# Arnoldi and solve
# ---------------------------------------------------------------------------
def workspace_bytes(op: Operator, sk: Sketch, m: int, basis_dtype: int = F32) -> int:
    n = lib().rtg_workspace_bytes(op.handle, sk.handle, m, basis_dtype)
    if n == 0:
        raise RTGError("rtg_workspace_bytes: invalid sizes")
    return n


def workspace_layout(op: Operator, sk: Sketch, m: int, basis_dtype: int = F32):
    v = ctypes.c_size_t()
    s = ctypes.c_size_t()
    _check(lib().rtg_workspace_layout(op.handle, sk.handle, m, basis_dtype, ctypes.byref(v), ctypes.byref(s)),
           "rtg_workspace_layout")
    return v.value, s.value


def arnoldi(op: Operator, sk: Sketch, R0, m: int, basis_dtype: int = F32, bd_tol: float = 1e-6, ws=None):
    """m steps of the sketched global Arnoldi process.  Returns a dict with H
    ((m+1) x m float64), beta, m_done, and views V ((m+1, J, I2, I1)) and SV
    ((m+1, L)) into the workspace; SV is None for the identity sketch (no
    sketches are kept: S(V) is V itself)."""
    torch = _torch()
    _check_tensor(R0, op.device_shape, "R0")
    nbytes = workspace_bytes(op, sk, m, basis_dtype)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=R0.device)
    H = torch.zeros((m, m + 1), dtype=torch.float64, device=R0.device)   # column-major (m+1) x m
    beta = torch.zeros(1, dtype=torch.float64, device=R0.device)
    m_done = torch.zeros(1, dtype=torch.int32, device=R0.device)
    _check(lib().rtg_arnoldi(op.handle, sk.handle, _ptr(R0), m, basis_dtype, bd_tol, _ptr(ws), ws.numel(),
                             _ptr(H), _ptr(beta), _ptr(m_done), _stream()), "rtg_arnoldi")
    voff, soff = workspace_layout(op, sk, m, basis_dtype)
    esz = 2 if basis_dtype == BF16 else 4
    n = int(np.prod(op.shape))
    vdt = torch.bfloat16 if basis_dtype == BF16 else torch.float32
    V = ws[voff:voff + (m + 1) * n * esz].view(vdt).view((m + 1,) + op.device_shape)
    SV = None if sk.identity else ws[soff:soff + (m + 1) * sk.L * 4].view(torch.float32).view(m + 1, sk.L)
    return {"H": H.t(), "beta": beta, "m_done": m_done, "V": V, "SV": SV, "ws": ws}


MU_DISCREPANCY, MU_GCV = 0, 1
METHOD_GMRES, METHOD_GOLUB_KAHAN = 0, 1


def make_params(m, basis_dtype=F32, mu=-1.0, delta=0.0, eta=1.01, stop_res=0.0, bd_tol=1e-6,
                mu_rule=MU_DISCREPANCY, method=METHOD_GMRES, restarts=0) -> Params:
    return Params(int(m), int(basis_dtype), float(mu), float(delta), float(eta), float(stop_res), float(bd_tol),
                  int(mu_rule), int(method), int(restarts))


def gk_workspace_bytes(op: Operator, sk: Sketch, m: int, basis_dtype: int = F32) -> int:
    n = lib().rtg_gk_workspace_bytes(op.handle, sk.handle, m, basis_dtype)
    if n == 0:
        raise RTGError("rtg_gk_workspace_bytes: invalid sizes")
    return n


def gk_workspace_layout(op: Operator, sk: Sketch, m: int, basis_dtype: int = F32):
    v = ctypes.c_size_t()
    u = ctypes.c_size_t()
    _check(lib().rtg_gk_workspace_layout(op.handle, sk.handle, m, basis_dtype, ctypes.byref(v), ctypes.byref(u)),
           "rtg_gk_workspace_layout")
    return v.value, u.value


def golub_kahan(op: Operator, sk: Sketch, R0, m: int, basis_dtype: int = F32, bd_tol: float = 1e-6, ws=None):
    """m columns of the sketched Block Golub-Kahan bidiagonalisation.
    Returns a dict with B ((m+1) x m float64 lower bidiagonal), beta (beta_1),
    m_done, and views U ((m+1, J, I2, I1)) and V ((m+1, ...); V_1..V_m
    written) into the workspace."""
    torch = _torch()
    _check_tensor(R0, op.device_shape, "R0")
    nbytes = gk_workspace_bytes(op, sk, m, basis_dtype)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=R0.device)
    B = torch.zeros((m, m + 1), dtype=torch.float64, device=R0.device)   # column-major (m+1) x m
    beta = torch.zeros(1, dtype=torch.float64, device=R0.device)
    m_done = torch.zeros(1, dtype=torch.int32, device=R0.device)
    _check(lib().rtg_golub_kahan(op.handle, sk.handle, _ptr(R0), m, basis_dtype, bd_tol, _ptr(ws), ws.numel(),
                                 _ptr(B), _ptr(beta), _ptr(m_done), _stream()), "rtg_golub_kahan")
    voff, uoff = gk_workspace_layout(op, sk, m, basis_dtype)
    esz = 2 if basis_dtype == BF16 else 4
    n = int(np.prod(op.shape))
    vdt = torch.bfloat16 if basis_dtype == BF16 else torch.float32
    V = ws[voff:voff + (m + 1) * n * esz].view(vdt).view((m + 1,) + op.device_shape)
    U = ws[uoff:uoff + (m + 1) * n * esz].view(vdt).view((m + 1,) + op.device_shape)
    return {"B": B.t(), "beta": beta, "m_done": m_done, "U": U, "V": V, "ws": ws}


def read_info(info_buf) -> Info:
    raw = info_buf.cpu().numpy().tobytes()
    return Info.from_buffer_copy(raw[:ctypes.sizeof(Info)])


def info_buffer(device="cuda"):
    torch = _torch()
    return torch.zeros(ctypes.sizeof(Info), dtype=torch.uint8, device=device)


def solve(op: Operator, sk: Sketch, C, X0=None, params: Optional[Params] = None, out=None, ws=None,
          info_buf=None):
    """One RTG-GMRES (or, with params.method, sketched Block Golub-Kahan)
    solve; returns (X, info_buf) with the info left on the device (read it
    with read_info)."""
    torch = _torch()
    _check_tensor(C, op.device_shape, "C")
    if X0 is not None:
        _check_tensor(X0, op.device_shape, "X0")
    if params is None:
        raise RTGError("params required")
    if params.method == METHOD_GOLUB_KAHAN:
        nbytes = gk_workspace_bytes(op, sk, params.m, params.basis_dtype)
    else:
        nbytes = workspace_bytes(op, sk, params.m, params.basis_dtype)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=C.device)
    if out is None:
        out = torch.empty(op.device_shape, dtype=torch.float32, device=C.device)
    if info_buf is None:
        info_buf = info_buffer(C.device)
    _check(lib().rtg_solve(op.handle, sk.handle, _ptr(C), _ptr(X0), ctypes.byref(params), _ptr(ws), ws.numel(),
                           _ptr(out), _ptr(info_buf), _stream()), "rtg_solve")
    return out, info_buf


class BatchPlan:
    """Problems, outputs and workspace of one rtg_solve_batched call, kept so
    the same batch can be re-run (e.g. in a timing loop).  With fallback =
    (m, basis_dtype[, fail_mask]) run() calls rtg_solve_batched_fallback: the
    problems whose flags meet fail_mask (default NOT_CONVERGED | NONFINITE)
    are solved again by the plain solver (X0 = 0, m steps); run() is then
    synchronous and n_fallback holds the number of re-solved problems."""

    def __init__(self, ops: Sequence[Operator], sks: Sequence[Sketch], Cs, X0s, params: Sequence[Params],
                 outs=None, device="cuda", fallback=None):
        torch = _torch()
        self.count = len(ops)
        self.ops, self.sks, self.Cs, self.X0s = list(ops), list(sks), list(Cs), list(X0s)
        self.outs = outs if outs is not None else [torch.empty(o.device_shape, dtype=torch.float32, device=device)
                                                   for o in ops]
        self.info = torch.zeros((self.count, ctypes.sizeof(Info)), dtype=torch.uint8, device=device)
        arr = (Problem * self.count)()
        for p in range(self.count):
            _check_tensor(self.Cs[p], ops[p].device_shape, "C")
            if self.X0s[p] is not None:
                _check_tensor(self.X0s[p], ops[p].device_shape, "X0")
            arr[p].op = ops[p].handle
            arr[p].sk = sks[p].handle
            arr[p].C = _ptr(self.Cs[p])
            arr[p].X0 = _ptr(self.X0s[p])
            arr[p].X = _ptr(self.outs[p])
            arr[p].params = params[p]
            arr[p].info = self.info[p].data_ptr()
        self.arr = arr
        self.fallback = None
        self.n_fallback = 0
        if fallback is not None:
            fb_m, fb_basis = int(fallback[0]), int(fallback[1])
            mask = int(fallback[2]) if len(fallback) > 2 else FLAG_NOT_CONVERGED | FLAG_NONFINITE
            self.fallback = (fb_m, fb_basis, mask)
            nbytes = lib().rtg_fallback_workspace_bytes(self.count, arr, fb_m, fb_basis)
        else:
            nbytes = lib().rtg_batch_workspace_bytes(self.count, arr)
        if nbytes == 0:
            raise RTGError("workspace size query: invalid problem")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)

    def run(self):
        if self.fallback is not None:
            n = ctypes.c_int(0)
            fb_m, fb_basis, mask = self.fallback
            _check(lib().rtg_solve_batched_fallback(self.count, self.arr, fb_m, fb_basis, mask, _ptr(self.ws),
                                                    self.ws.numel(), ctypes.byref(n), _stream()),
                   "rtg_solve_batched_fallback")
            self.n_fallback = n.value
            return self.outs
        _check(lib().rtg_solve_batched(self.count, self.arr, _ptr(self.ws), self.ws.numel(), _stream()),
               "rtg_solve_batched")
        return self.outs

    def begin(self):
        """First half of run() with a fallback (rtg_solve_batched_fallback_begin):
        solves the batch and queues the copy of the flags to a page-locked
        host buffer; returns without waiting, so the stream can take other
        work before end()."""
        if self.fallback is None:
            raise RTGError("begin(): the batch was made without a fallback")
        if getattr(self, "flags_host", None) is None:
            self.flags_host = _torch().zeros(self.count, dtype=_torch().int32, pin_memory=True)
        fb_m, fb_basis, mask = self.fallback
        _check(lib().rtg_solve_batched_fallback_begin(self.count, self.arr, fb_m, fb_basis, mask, _ptr(self.ws),
                                                      self.ws.numel(), self.flags_host.data_ptr(), _stream()),
               "rtg_solve_batched_fallback_begin")

    def end(self):
        """Second half (rtg_solve_batched_fallback_end): waits for the flags,
        queues the re-solves and sets n_fallback; returns the outputs."""
        if self.fallback is None or getattr(self, "flags_host", None) is None:
            raise RTGError("end(): no begin() on this batch")
        n = ctypes.c_int(0)
        fb_m, fb_basis, mask = self.fallback
        _check(lib().rtg_solve_batched_fallback_end(self.count, self.arr, fb_m, fb_basis, mask, _ptr(self.ws),
                                                    self.ws.numel(), self.flags_host.data_ptr(), ctypes.byref(n),
                                                    _stream()),
               "rtg_solve_batched_fallback_end")
        self.n_fallback = n.value
        return self.outs

    def infos(self) -> List[Info]:
        raw = self.info.cpu().numpy()
        return [Info.from_buffer_copy(raw[p].tobytes()) for p in range(self.count)]

    def autotune(self, reps: int = 3):
        """Time candidate launch shapes on this batch (rtg_autotune_batched)
        and record the fastest for every later run of a batch of the same
        shapes; returns (Tune, best_ms).  Synchronous; the outputs are not
        written."""
        t, ms = Tune(), ctypes.c_double()
        _check(lib().rtg_autotune_batched(self.count, self.arr, _ptr(self.ws), self.ws.numel(), int(reps),
                                          ctypes.byref(t), ctypes.byref(ms), _stream()),
               "rtg_autotune_batched")
        return t, ms.value

    def set_tune(self, tune: Tune):
        """Record launch shapes for batches of these shapes (rtg_tune_set)."""
        _check(lib().rtg_tune_set(self.count, self.arr, ctypes.byref(tune)), "rtg_tune_set")

    def tune(self) -> Tune:
        """The launch shapes a run of this batch uses (rtg_tune_get)."""
        t = Tune()
        _check(lib().rtg_tune_get(self.count, self.arr, ctypes.byref(t)), "rtg_tune_get")
        return t


def tune_clear():
    """Forget every recorded launch-shape choice (rtg_tune_clear)."""
    _check(lib().rtg_tune_clear(), "rtg_tune_clear")


def set_wait_limit(polls: int):
    """Bound on the waits between workgroups of the persistent launch
    (rtg_set_wait_limit)."""
    _check(lib().rtg_set_wait_limit(int(polls)), "rtg_set_wait_limit")


def solve_batched(ops, sks, Cs, X0s, params, outs=None) -> BatchPlan:
    plan = BatchPlan(ops, sks, Cs, X0s, params, outs)
    plan.run()
    return plan


# ---------------------------------------------------------------------------
# measurement
# ---------------------------------------------------------------------------
KIND_PHI, KIND_TILE, KIND_GRAM, KIND_SOLVE, KIND_STEP, KIND_PERSIST = 0, 1, 2, 3, 4, 5
N_KINDS = 6


def event_timing_enable(kind_mask: int):
    _check(lib().rtg_event_timing_enable(int(kind_mask)), "rtg_event_timing_enable")


def event_timing_read():
    """{kind: (total_ms, launches)} for the kernel kinds recorded since the
    last read (waits for the recorded events)."""
    ms = (ctypes.c_double * N_KINDS)()
    n = (ctypes.c_longlong * N_KINDS)()
    _check(lib().rtg_event_timing_read(ms, n, N_KINDS), "rtg_event_timing_read")
    return {k: (ms[k], n[k]) for k in range(N_KINDS)}


# ---------------------------------------------------------------------------
# learned warm start (network state lives in one device buffer)
# ---------------------------------------------------------------------------
N_CNN_PARAMS = 38755


class WarmStartNet:
    """Handle of the warm-start network state; parameters use the flat layout
    of the C ABI (per layer w[co][t1][t2][ci] then b[co])."""

    def __init__(self, params: np.ndarray, device="cuda"):
        torch = _torch()
        params = np.ascontiguousarray(params, dtype=np.float32)
        if params.size != N_CNN_PARAMS:
            raise RTGError(f"expected {N_CNN_PARAMS} parameters, got {params.size}")
        self.state = torch.zeros(lib().rtg_cnn_state_bytes(), dtype=torch.uint8, device=device)
        self.step = 0
        self._ws = None
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        _check(lib().rtg_cnn_init(_ptr(self.state), _fptr(params), _stream()), "rtg_cnn_init")

    def _workspace(self, N, I1, I2, device):
        torch = _torch()
        n = lib().rtg_cnn_workspace_bytes(N, I1, I2)
        if self._ws is None or self._ws.numel() < n:
            self._ws = torch.empty(n, dtype=torch.uint8, device=device)
        return self._ws

    def export(self) -> np.ndarray:
        out = np.empty(N_CNN_PARAMS, dtype=np.float32)
        _check(lib().rtg_cnn_export(_ptr(self.state), _fptr(out), _stream()), "rtg_cnn_export")
        return out

    def forward(self, C, out=None):
        """C: device float32 (N, 3, I2, I1) or (3, I2, I1); returns X0 = C + f(C)."""
        torch = _torch()
        Cb = C if C.dim() == 4 else C.unsqueeze(0)
        if not Cb.is_contiguous() or Cb.dtype != torch.float32 or Cb.shape[1] != 3:
            raise RTGError("C must be contiguous float32 (N, 3, I2, I1)")
        N, _, I2, I1 = Cb.shape
        if out is None:
            out = torch.empty_like(Cb)
        ws = self._workspace(N, I1, I2, Cb.device)
        _check(lib().rtg_cnn_forward(_ptr(self.state), _ptr(Cb), N, I1, I2, _ptr(out), _ptr(ws), ws.numel(),
                                     _stream()), "rtg_cnn_forward")
        return out if C.dim() == 4 else out[0]

    infer = forward

    def gradients(self, C, Y):
        """Gradients of the mean squared error kept in the state; returns the
        device tensor holding the sum of squared errors."""
        N, _, I2, I1 = C.shape
        ws = self._workspace(N, I1, I2, C.device)
        _check(lib().rtg_cnn_gradients(_ptr(self.state), _ptr(C), _ptr(Y), N, I1, I2, _ptr(ws), ws.numel(),
                                       _ptr(self.loss), _stream()), "rtg_cnn_gradients")
        return self.loss

    def read_gradients(self) -> np.ndarray:
        out = np.empty(N_CNN_PARAMS, dtype=np.float32)
        _check(lib().rtg_cnn_read_gradients(_ptr(self.state), _fptr(out), _stream()), "rtg_cnn_read_gradients")
        return out

    def adam(self, lr: float):
        self.step += 1
        _check(lib().rtg_cnn_adam(_ptr(self.state), float(lr), self.step, _stream()), "rtg_cnn_adam")

    def train_step(self, C, Y, lr: float):
        loss = self.gradients(C, Y)
        self.adam(lr)
        return loss
