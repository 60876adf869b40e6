"""Python binding of ``libbandred.so``, the gfx950 band-reduction library.

Argument marshalling only: every step of the reductions runs in the HIP
kernels of the shared library.  PyTorch supplies device memory and streams.
There is no CPU fallback: if the library is not built, importing the binding
works but every call raises ``BandredUnavailable``.

Raw entry points carry the C names (``bandred_sy2sb`` ...) and take integers
(device addresses); the helpers ``sy2sb`` / ``ge2gb`` / ``sy2sb_batched``
take torch tensors.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbandred.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "bandred.h")

FP64, FP32_UPDATE, SPLIT32_UPDATE, INT8_SPLIT_UPDATE = 0, 1, 2, 3
PREC_NAMES = {"fp64": FP64, "fp32": FP32_UPDATE, "split32": SPLIT32_UPDATE,
              "int8split": INT8_SPLIT_UPDATE}


class BandredUnavailable(RuntimeError):
    pass


class BandredError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} returned {code}: {msg}")
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("lookahead", ctypes.c_int), ("panel_rows", ctypes.c_int),
                ("panel_method", ctypes.c_int), ("update_chunks", ctypes.c_int),
                ("update_lds_cap", ctypes.c_int), ("reserved", ctypes.c_int * 3)]


_i64 = ctypes.c_int64
_vp = ctypes.c_void_p
_lib = None


def declared_symbols(header: str = HEADER) -> list[str]:
    """Names of the functions ``include/bandred.h`` declares."""
    txt = open(header).read()
    return sorted(set(re.findall(r"BANDRED_API\s+[\w\s\*]*?\b(bandred_\w+)\s*\(", txt)))


def load(path: str = LIB_PATH):
    """Load the shared library (once)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise BandredUnavailable(
            f"{path} is not built; run `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(path)
    lib.bandred_sy2sb.argtypes = [_i64, _i64, _i64, _vp, _i64, _vp]
    lib.bandred_ge2gb.argtypes = [_i64, _i64, _i64, _i64, _vp, _i64, _vp, _vp]
    lib.bandred_sy2sb_ex.argtypes = [_i64, _i64, _i64, _vp, _i64, _vp, ctypes.c_int,
                                     ctypes.POINTER(Opts), _vp]
    lib.bandred_ge2gb_ex.argtypes = [_i64, _i64, _i64, _i64, _vp, _i64, _vp, _vp, ctypes.c_int,
                                     ctypes.POINTER(Opts), _vp]
    lib.bandred_ge2gb_lu.argtypes = [_i64, _i64, _i64, _i64, _vp, _i64, _vp, _vp, ctypes.c_int,
                                     ctypes.POINTER(Opts), _vp]
    lib.bandred_sy2sb_apply_q.argtypes = [ctypes.c_int, _i64, _i64, _i64, _vp, _i64, _vp, _i64,
                                          _vp, _i64, _vp]
    lib.bandred_ge2gb_apply.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _i64, _i64,
                                        _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp]
    lib.bandred_tune.argtypes = [ctypes.c_int, _i64, _i64, _i64, ctypes.c_int, ctypes.c_int,
                                 ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_double),
                                 ctypes.c_int]
    lib.bandred_tune_result.argtypes = [ctypes.c_int, _i64, _i64, _i64, ctypes.c_int,
                                        ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_int)]
    lib.bandred_sb2st.argtypes = [_i64, _i64, _vp, _i64, _vp, _vp, _vp]
    lib.bandred_tridiag_eigvals.argtypes = [_i64, _vp, _vp, _vp, _vp]
    lib.bandred_sy2sb_noalloc.argtypes = [_i64, _i64, _i64, _vp, _i64, _vp, ctypes.c_int, _vp]
    lib.bandred_sy2sb_batched.argtypes = [_i64, ctypes.POINTER(_i64), _i64, _i64,
                                          ctypes.POINTER(_vp), ctypes.POINTER(_i64),
                                          ctypes.POINTER(_vp), ctypes.c_int, _vp]
    lib.bandred_status.argtypes = [_vp]
    lib.bandred_release.argtypes = []
    lib.bandred_set_wait_limit_us.argtypes = [ctypes.c_double]
    lib.bandred_status_string.argtypes = [ctypes.c_int]
    lib.bandred_status_string.restype = ctypes.c_char_p
    lib.bandred_profile_enable.argtypes = [ctypes.c_int]
    lib.bandred_profile_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_int]
    lib.bandred_profile_name.argtypes = [ctypes.c_int]
    lib.bandred_profile_name.restype = ctypes.c_char_p
    for name in ("bandred_sy2sb", "bandred_ge2gb", "bandred_sy2sb_ex", "bandred_ge2gb_ex",
                 "bandred_sy2sb_batched", "bandred_sy2sb_noalloc", "bandred_profile_enable",
                 "bandred_profile_read",
                 "bandred_status", "bandred_set_wait_limit_us", "bandred_release",
                 "bandred_ge2gb_lu", "bandred_sy2sb_apply_q", "bandred_ge2gb_apply",
                 "bandred_tune", "bandred_tune_result", "bandred_sb2st",
                 "bandred_tridiag_eigvals"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def status_string(code: int) -> str:
    return load().bandred_status_string(int(code)).decode()


def _check(fn: str, rc: int) -> int:
    if rc != 0:
        raise BandredError(fn, rc, status_string(rc))
    return rc


# ---- raw entry points (same names as the C ABI) ---------------------------

def bandred_sy2sb(n, w, b, A, lda, tau) -> int:
    return load().bandred_sy2sb(n, w, b, A, lda, tau)


def bandred_ge2gb(m, n, w, b, A, lda, tauq, taup) -> int:
    return load().bandred_ge2gb(m, n, w, b, A, lda, tauq, taup)


def bandred_sy2sb_ex(n, w, b, A, lda, tau, prec=FP64, opts=None, stream=None) -> int:
    return load().bandred_sy2sb_ex(n, w, b, A, lda, tau, prec,
                                   ctypes.byref(opts) if opts is not None else None, stream)


def bandred_ge2gb_ex(m, n, w, b, A, lda, tauq, taup, prec=FP64, opts=None, stream=None) -> int:
    return load().bandred_ge2gb_ex(m, n, w, b, A, lda, tauq, taup, prec,
                                   ctypes.byref(opts) if opts is not None else None, stream)


def bandred_ge2gb_lu(m, n, w, b, A, lda, tauq, taup, prec=FP64, opts=None, stream=None) -> int:
    return load().bandred_ge2gb_lu(m, n, w, b, A, lda, tauq, taup, prec,
                                   ctypes.byref(opts) if opts is not None else None, stream)


def bandred_sy2sb_apply_q(trans, n, w, b, A, lda, tau, k, C, ldc, stream=None) -> int:
    return load().bandred_sy2sb_apply_q(trans, n, w, b, A, lda, tau, k, C, ldc, stream)


def bandred_ge2gb_apply(side, form, trans, m, n, w, b, A, lda, tau, k, C, ldc,
                        stream=None) -> int:
    return load().bandred_ge2gb_apply(side, form, trans, m, n, w, b, A, lda, tau, k, C, ldc,
                                      stream)


def bandred_tune(kind, m, n, w, prec=FP64, force=False):
    """Tuned block size: returns (b, {b: ms} of the candidates measured now)."""
    b = _i64(0)
    buf = (ctypes.c_double * 32)()
    rc = load().bandred_tune(int(kind), m, n, w, int(prec), 1 if force else 0, ctypes.byref(b),
                             buf, 16)
    _check("bandred_tune", rc)
    ms = {int(buf[2 * i]): buf[2 * i + 1] for i in range(16) if buf[2 * i] > 0}
    return int(b.value), ms



def bandred_tune_result(kind, m, n, w, prec=FP64):
    """The cached tuning of a problem: (b, update_chunks, update_lds_cap), or
    None when it has not been tuned."""
    b, ch, cap = _i64(0), ctypes.c_int(0), ctypes.c_int(0)
    rc = load().bandred_tune_result(int(kind), m, n, w, int(prec), ctypes.byref(b),
                                    ctypes.byref(ch), ctypes.byref(cap))
    if rc == 3:  # BANDRED_ERR_UNSUPPORTED: not tuned
        return None
    _check("bandred_tune_result", rc)
    return b.value, ch.value, cap.value

def bandred_sb2st(n, w, A, lda, d, e, stream=None) -> int:
    return load().bandred_sb2st(n, w, A, lda, d, e, stream)


def bandred_tridiag_eigvals(n, d, e, lam, stream=None) -> int:
    return load().bandred_tridiag_eigvals(n, d, e, lam, stream)


def bandred_sy2sb_noalloc(n, w, b, A, lda, tau, prec=FP64, stream=None) -> int:
    return load().bandred_sy2sb_noalloc(n, w, b, A, lda, tau, prec, stream)


def bandred_sy2sb_batched(count, n, w, b, A, lda, tau, prec=FP64, stream=None) -> int:
    arr_n = (_i64 * count)(*[int(x) for x in n])
    arr_a = (_vp * count)(*[int(x) if x else None for x in A])
    arr_l = (_i64 * count)(*[int(x) for x in lda])
    arr_t = (_vp * count)(*[int(x) if x else None for x in tau])
    return load().bandred_sy2sb_batched(count, arr_n, w, b, arr_a, arr_l, arr_t, prec, stream)


def bandred_status_string(code: int) -> str:
    return status_string(code)


def bandred_status(stream=None) -> int:
    return load().bandred_status(stream)


def bandred_release() -> int:
    return load().bandred_release()


def bandred_set_wait_limit_us(us: float) -> int:
    return load().bandred_set_wait_limit_us(float(us))


def bandred_profile_enable(on: bool) -> int:
    return load().bandred_profile_enable(1 if on else 0)


def bandred_profile_read() -> dict:
    lib = load()
    buf = (ctypes.c_double * 96)()
    ncls = lib.bandred_profile_read(buf, 96)
    out = {}
    for c in range(ncls):
        name = lib.bandred_profile_name(c).decode()
        out[name] = {"ms": buf[3 * c], "flops": buf[3 * c + 1], "launches": int(buf[3 * c + 2])}
    return out


def bandred_profile_name(cls: int) -> str:
    return load().bandred_profile_name(cls).decode()


# ---- torch helpers ---------------------------------------------------------

def _colmajor_ld(A, rows: int) -> int:
    import torch

    if A.dtype != torch.float64 or not A.is_cuda:
        raise TypeError("A must be a float64 CUDA tensor")
    if A.dim() != 2:
        raise ValueError("A must be 2-D")
    if A.shape[1] > 1 and A.stride(0) != 1:
        raise ValueError("A must be column-major (stride(0) == 1); use A.T.contiguous().T")
    ld = A.stride(1) if A.shape[1] > 1 else max(rows, 1)
    return max(ld, 1)


def _stream_handle(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check_status(fn: str, handle, check: bool):
    """After an asynchronous call: unless the stream is being captured into
    a graph (or check is False), wait for it and raise on a device-side
    failure (a panel wait that timed out)."""
    import torch

    if not check or torch.cuda.is_current_stream_capturing():
        return
    _check(fn + " (device status)", bandred_status(handle))


def sy2sb(A, w: int, b: int | None = None, prec="fp64", lookahead: bool = True,
          panel_rows: int = 0, panel_method: int = 0, stream=None, tau=None, check: bool = True,
          update_chunks: int = 0, update_lds_cap: int = 0):
    """Reduce the symmetric column-major CUDA tensor ``A`` (lower triangle) to
    band width ``w`` in place; returns tau (device tensor).  With ``check``
    (and outside graph capture) the call waits for the device and raises if
    the reduction reported a runtime failure."""
    import torch

    n = A.shape[0]
    b = w if b is None else b
    lda = _colmajor_ld(A, n)
    if tau is None:
        tau = torch.zeros(max(n - w, 1), dtype=torch.float64, device=A.device)
    p = PREC_NAMES[prec] if isinstance(prec, str) else int(prec)
    o = Opts(1 if lookahead else 0, int(panel_rows), int(panel_method), int(update_chunks),
             int(update_lds_cap))
    h = _stream_handle(stream)
    rc = bandred_sy2sb_ex(n, w, b, A.data_ptr(), lda, tau.data_ptr(), p, o, h)
    _check("bandred_sy2sb_ex", rc)
    _check_status("bandred_sy2sb_ex", h, check)
    return tau[: max(n - w, 0)]


def ge2gb(A, w: int, b: int | None = None, prec="fp64", lookahead: bool = True,
          panel_rows: int = 0, panel_method: int = 0, stream=None, check: bool = True,
          update_chunks: int = 0, update_lds_cap: int = 0):
    """Reduce the column-major CUDA tensor ``A`` (m >= n) to upper
    triangular-band width ``w`` in place; returns (tauq, taup)."""
    import torch

    m, n = A.shape
    b = w if b is None else b
    lda = _colmajor_ld(A, m)
    tauq = torch.zeros(max(n, 1), dtype=torch.float64, device=A.device)
    taup = torch.zeros(max(n, 1), dtype=torch.float64, device=A.device)
    p = PREC_NAMES[prec] if isinstance(prec, str) else int(prec)
    o = Opts(1 if lookahead else 0, int(panel_rows), int(panel_method), int(update_chunks),
             int(update_lds_cap))
    h = _stream_handle(stream)
    rc = bandred_ge2gb_ex(m, n, w, b, A.data_ptr(), lda, tauq.data_ptr(), taup.data_ptr(), p, o, h)
    _check("bandred_ge2gb_ex", rc)
    _check_status("bandred_ge2gb_ex", h, check)
    return tauq[:n], taup[:n]


def ge2gb_lu(A, w: int, b: int | None = None, prec="fp64", lookahead: bool = True,
             panel_rows: int = 0, panel_method: int = 0, stream=None, check: bool = True,
             update_chunks: int = 0, update_lds_cap: int = 0):
    """Reduce the column-major CUDA tensor ``A`` (m >= n) to band form with
    lower and upper bandwidth ``w`` in place; returns (tauq, taup)."""
    import torch

    m, n = A.shape
    b = w if b is None else b
    lda = _colmajor_ld(A, m)
    tauq = torch.zeros(max(n, 1), dtype=torch.float64, device=A.device)
    taup = torch.zeros(max(n, 1), dtype=torch.float64, device=A.device)
    p = PREC_NAMES[prec] if isinstance(prec, str) else int(prec)
    o = Opts(1 if lookahead else 0, int(panel_rows), int(panel_method), int(update_chunks),
             int(update_lds_cap))
    h = _stream_handle(stream)
    rc = bandred_ge2gb_lu(m, n, w, b, A.data_ptr(), lda, tauq.data_ptr(), taup.data_ptr(), p, o, h)
    _check("bandred_ge2gb_lu", rc)
    _check_status("bandred_ge2gb_lu", h, check)
    return tauq[:n], taup[:n]


def sy2sb_apply_q(Aout, tau, w: int, C, trans: bool = False, b: int = 128, stream=None):
    """C := Q C (or Q^T C) in place for the result (Aout, tau) of ``sy2sb``;
    C is a column-major CUDA tensor with n rows.  Returns C."""
    n = Aout.shape[0]
    lda = _colmajor_ld(Aout, n)
    ldc = _colmajor_ld(C, n) if C.dim() == 2 else n
    k = C.shape[1] if C.dim() == 2 else 1
    rc = bandred_sy2sb_apply_q(1 if trans else 0, n, w, b, Aout.data_ptr(), lda,
                               tau.data_ptr() if tau.numel() else None, k, C.data_ptr(), ldc,
                               _stream_handle(stream))
    _check("bandred_sy2sb_apply_q", rc)
    return C


def ge2gb_apply(Aout, tau, w: int, C, side: str = "u", equal_band: bool = False,
                trans: bool = False, b: int = 128, stream=None):
    """C := U C / U^T C (side 'u', tau = tauq) or V C / V^T C (side 'v',
    tau = taup) in place for the result of ``ge2gb`` or ``ge2gb_lu``."""
    m, n = Aout.shape
    lda = _colmajor_ld(Aout, m)
    rows = m if side == "u" else n
    ldc = _colmajor_ld(C, rows) if C.dim() == 2 else rows
    k = C.shape[1] if C.dim() == 2 else 1
    rc = bandred_ge2gb_apply(0 if side == "u" else 1, 1 if equal_band else 0, 1 if trans else 0,
                             m, n, w, b, Aout.data_ptr(), lda,
                             tau.data_ptr() if tau.numel() else None, k, C.data_ptr(), ldc,
                             _stream_handle(stream))
    _check("bandred_ge2gb_apply", rc)
    return C


def sb2st(Aout, w: int, stream=None, check: bool = True):
    """Band (0 <= i-j <= w of the column-major CUDA tensor Aout) to symmetric
    tridiagonal form; returns (d, e) device tensors."""
    import torch

    n = Aout.shape[0]
    lda = _colmajor_ld(Aout, n)
    d = torch.zeros(max(n, 1), dtype=torch.float64, device=Aout.device)
    e = torch.zeros(max(n - 1, 1), dtype=torch.float64, device=Aout.device)
    h = _stream_handle(stream)
    _check("bandred_sb2st", bandred_sb2st(n, w, Aout.data_ptr(), lda, d.data_ptr(), e.data_ptr(), h))
    _check_status("bandred_sb2st", h, check)
    return d[:n], e[: max(n - 1, 0)]


def tridiag_eigvals(d, e, stream=None):
    """Eigenvalues (ascending) of the symmetric tridiagonal matrix (d, e)."""
    import torch

    n = d.shape[0]
    lam = torch.zeros(max(n, 1), dtype=torch.float64, device=d.device)
    ep = e.data_ptr() if e.numel() else None
    _check("bandred_tridiag_eigvals",
           bandred_tridiag_eigvals(n, d.data_ptr(), ep, lam.data_ptr(), _stream_handle(stream)))
    return lam[:n]


def sy2sb_batched(mats, w: int, b: int | None = None, prec="fp64", stream=None,
                  check: bool = True):
    """Reduce a list of symmetric column-major CUDA tensors in one call;
    returns the list of tau tensors."""
    import torch

    b = w if b is None else b
    ns, ptrs, lds, taus = [], [], [], []
    for A in mats:
        n = A.shape[0]
        ns.append(n)
        ptrs.append(A.data_ptr())
        lds.append(_colmajor_ld(A, n))
        t = torch.zeros(max(n - w, 1), dtype=torch.float64, device=A.device)
        taus.append(t)
    p = PREC_NAMES[prec] if isinstance(prec, str) else int(prec)
    h = _stream_handle(stream)
    rc = bandred_sy2sb_batched(len(mats), ns, w, b, ptrs, lds, [t.data_ptr() for t in taus], p, h)
    _check("bandred_sy2sb_batched", rc)
    _check_status("bandred_sy2sb_batched", h, check)
    return [t[: max(n - w, 0)] for t, n in zip(taus, ns)]
