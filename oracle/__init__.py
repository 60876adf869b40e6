"""CPU FP64 oracle for the band reductions: a ctypes wrapper over ``oracle.c``.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  The product
library (``paper_1709_00302_amd``) neither imports nor links it; the two
share no code.

``sy2sb`` follows Sec. 2.1 of the paper (reduction of a symmetric matrix to
symmetric band form, eqs. updateA0..updateA2syr2k at block size 1),
``ge2gb`` follows Sec. 3.1 (reduction of a general matrix to upper
triangular-band form, eqs. updateB..updateD at block size 1), ``ge2gb_lu``
Sec. 3.3 (band form with equal lower and upper bandwidth, eqs.
updateB0..updateCD22 at block size 1), and ``apply_refl`` applies the
stored reflectors of any of them (the back-transformation).  The arithmetic
lives in ``oracle.c``; this module only marshals numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "oracle.c")
LIB = os.path.join(_HERE, "liboracle.so")

_c_i64 = ctypes.c_int64
_c_dp = ctypes.POINTER(ctypes.c_double)


def build(out: str = LIB, mutant: int = 0) -> str:
    """Compile ``oracle.c`` into a shared library (gcc, -O2, no FP contraction).

    ``mutant`` > 0 plants one deliberate mistake (see ``oracle.c``); only the
    tests that check that the pins catch such mistakes ask for it.
    """
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-std=c99", SRC, "-o", out + ".tmp", "-lm"]
    if mutant:
        cmd.insert(1, f"-DORACLE_MUTANT={int(mutant)}")
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


class Oracle:
    """Handle on one compiled oracle library (the normal one or a mutant)."""

    def __init__(self, path: str = LIB):
        if not os.path.exists(path):
            raise FileNotFoundError(f"oracle library not built: {path}")
        lib = ctypes.CDLL(path)
        lib.oracle_sy2sb.argtypes = [_c_i64, _c_i64, _c_i64, _c_dp, _c_i64, _c_dp]
        lib.oracle_sy2sb.restype = ctypes.c_int
        lib.oracle_ge2gb.argtypes = [_c_i64, _c_i64, _c_i64, _c_i64, _c_dp, _c_i64,
                                     _c_dp, _c_dp]
        lib.oracle_ge2gb.restype = ctypes.c_int
        lib.oracle_ge2gb_lu.argtypes = [_c_i64, _c_i64, _c_i64, _c_i64, _c_dp, _c_i64,
                                        _c_dp, _c_dp]
        lib.oracle_ge2gb_lu.restype = ctypes.c_int
        lib.oracle_apply_refl.argtypes = [ctypes.c_int, _c_i64, _c_i64, _c_i64, _c_dp, _c_i64,
                                          _c_dp, ctypes.c_int, _c_i64, _c_dp, _c_i64]
        lib.oracle_apply_refl.restype = ctypes.c_int
        lib.oracle_tridiag_eigvals.argtypes = [_c_i64, _c_dp, _c_dp, _c_dp]
        lib.oracle_tridiag_eigvals.restype = ctypes.c_int
        lib.oracle_house.argtypes = [_c_i64, _c_dp, _c_i64, _c_dp]
        lib.oracle_house.restype = ctypes.c_double
        lib.oracle_threads.argtypes = []
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_threads.restype = None
        self.lib = lib
        self.path = path

    @staticmethod
    def _ptr(a: np.ndarray):
        return a.ctypes.data_as(_c_dp)

    def threads(self) -> int:
        return int(self.lib.oracle_threads())

    def set_threads(self, nthreads: int) -> None:
        self.lib.oracle_set_threads(int(nthreads))

    def house(self, x):
        """Householder vector of ``x``: returns (v, tau, beta) with v[0] = 1."""
        x = np.array(x, dtype=np.float64, copy=True)
        beta = ctypes.c_double(0.0)
        tau = self.lib.oracle_house(x.size, self._ptr(x), 1, ctypes.byref(beta))
        v = x.copy()
        v[0] = 1.0
        return v, float(tau), float(beta.value)

    def sy2sb(self, A, w: int, ncols: int = -1, lda: int | None = None):
        """Reduce symmetric ``A`` (lower triangle read) to band width ``w``.

        Returns (Aout, tau): Aout is a Fortran-ordered copy holding the band
        and the reflectors in the lower triangle (upper triangle of the input
        copied through untouched); tau has max(n - w, 0) entries.
        """
        A = np.asarray(A, dtype=np.float64)
        n = A.shape[0]
        assert A.shape == (n, n)
        Aout = np.array(A, dtype=np.float64, order="F", copy=True)
        tau = np.zeros(max(n - w, 1), dtype=np.float64)
        ld = max(n, 1) if lda is None else lda
        if lda is not None and lda != n:
            buf = np.zeros((lda, n), dtype=np.float64, order="F")
            buf[:n, :] = Aout
            info = self.lib.oracle_sy2sb(n, w, ncols, self._ptr(buf), ld, self._ptr(tau))
            Aout = np.array(buf[:n, :], order="F")
        else:
            info = self.lib.oracle_sy2sb(n, w, ncols, self._ptr(Aout), ld, self._ptr(tau))
        if info != 0:
            raise ValueError(f"oracle_sy2sb returned {info}")
        return Aout, tau[: max(n - w, 0)]

    def ge2gb(self, A, w: int, ncols: int = -1):
        """Reduce general ``A`` (m >= n) to upper triangular-band width ``w``.

        Returns (Aout, tauq, taup), each tau of length n.
        """
        A = np.asarray(A, dtype=np.float64)
        m, n = A.shape
        Aout = np.array(A, dtype=np.float64, order="F", copy=True)
        tauq = np.zeros(max(n, 1), dtype=np.float64)
        taup = np.zeros(max(n, 1), dtype=np.float64)
        info = self.lib.oracle_ge2gb(m, n, w, ncols, self._ptr(Aout), max(m, 1),
                                     self._ptr(tauq), self._ptr(taup))
        if info != 0:
            raise ValueError(f"oracle_ge2gb returned {info}")
        return Aout, tauq[:n], taup[:n]

    def ge2gb_lu(self, A, w: int, ncols: int = -1):
        """Reduce general ``A`` (m >= n) to band form with lower and upper
        bandwidth ``w`` (Sec. 3.3).  Returns (Aout, tauq, taup), each tau of
        length n."""
        A = np.asarray(A, dtype=np.float64)
        m, n = A.shape
        Aout = np.array(A, dtype=np.float64, order="F", copy=True)
        tauq = np.zeros(max(n, 1), dtype=np.float64)
        taup = np.zeros(max(n, 1), dtype=np.float64)
        info = self.lib.oracle_ge2gb_lu(m, n, w, ncols, self._ptr(Aout), max(m, 1),
                                        self._ptr(tauq), self._ptr(taup))
        if info != 0:
            raise ValueError(f"oracle_ge2gb_lu returned {info}")
        return Aout, tauq[:n], taup[:n]

    def apply_refl(self, Aout, tau, rowstore: bool, off: int, nrefl: int, C,
                   trans: bool = False):
        """Q C (or Q^T C) for the stored reflectors of a reduction (see
        oracle.h: which rowstore / off / nrefl each factor uses)."""
        Aout = np.asarray(Aout, dtype=np.float64, order="F")
        tau = np.ascontiguousarray(tau, dtype=np.float64)
        C = np.array(C, dtype=np.float64, order="F", copy=True)
        if C.ndim == 1:
            C = C[:, None]
        length, k = C.shape
        tbuf = np.zeros(max(nrefl, 1), dtype=np.float64)
        tbuf[:nrefl] = tau[:nrefl]
        info = self.lib.oracle_apply_refl(1 if rowstore else 0, off, nrefl, length,
                                          self._ptr(Aout), max(Aout.shape[0], 1),
                                          self._ptr(tbuf), 1 if trans else 0, k, self._ptr(C),
                                          max(length, 1))
        if info != 0:
            raise ValueError(f"oracle_apply_refl returned {info}")
        return C

    def tridiag_eigvals(self, d, e):
        """Eigenvalues (ascending) of the symmetric tridiagonal matrix with
        diagonal d and off-diagonal e, by bisection on Sturm counts."""
        d = np.ascontiguousarray(d, dtype=np.float64)
        n = d.size
        e = np.ascontiguousarray(e, dtype=np.float64)
        ebuf = np.zeros(max(n, 1), dtype=np.float64)
        ebuf[: max(n - 1, 0)] = e[: max(n - 1, 0)]
        lam = np.zeros(max(n, 1), dtype=np.float64)
        info = self.lib.oracle_tridiag_eigvals(n, self._ptr(d), self._ptr(ebuf), self._ptr(lam))
        if info != 0:
            raise ValueError(f"oracle_tridiag_eigvals returned {info}")
        return lam[:n]

    def band_eigvals(self, Aout, w: int):
        """Eigenvalues of the symmetric band matrix held in the band (0 <= i-j
        <= w) of a reduced matrix: its Householder tridiagonalisation (the
        oracle's reduction at w = 1, an orthogonal similarity), then
        bisection.  Any tridiagonalisation Z^T B Z with Z e_0 = e_0 has the
        same eigenvalues; its entries are not unique to rounding."""
        Aout = np.asarray(Aout, dtype=np.float64)
        n = Aout.shape[0]
        i = np.arange(n)
        dd = i[:, None] - i[None, :]
        B = np.where((dd >= 0) & (dd <= w), Aout, 0.0)
        B = B + np.tril(B, -1).T
        T, _ = self.sy2sb(B, 1)
        return self.tridiag_eigvals(np.diag(T).copy(), np.diag(T, -1).copy())

    def sy2sb_q(self, Aout, tau, w: int, C, trans: bool = False):
        """Q C or Q^T C for the result of ``sy2sb``."""
        n = Aout.shape[0]
        return self.apply_refl(Aout, tau, False, w, max(n - w, 0), C, trans)

    def ge2gb_u(self, Aout, tauq, w: int, C, trans: bool = False, equal_band: bool = False):
        """U C or U^T C for the result of ``ge2gb`` (or ``ge2gb_lu``)."""
        m, n = Aout.shape
        if equal_band:
            return self.apply_refl(Aout, tauq, False, w, min(n, max(m - w, 0)), C, trans)
        return self.apply_refl(Aout, tauq, False, 0, n, C, trans)

    def ge2gb_v(self, Aout, taup, w: int, C, trans: bool = False):
        """V C or V^T C for the result of ``ge2gb`` or ``ge2gb_lu`` (both
        store the right reflectors the same way)."""
        m, n = Aout.shape
        return self.apply_refl(Aout, taup, True, w, max(n - w, 0), C, trans)

    # raw entry points with explicit sizes, for argument-check tests
    def raw_sy2sb(self, n, w, ncols, A, lda, tau):
        return int(self.lib.oracle_sy2sb(n, w, ncols, A, lda, tau))

    def raw_ge2gb(self, m, n, w, ncols, A, lda, tauq, taup):
        return int(self.lib.oracle_ge2gb(m, n, w, ncols, A, lda, tauq, taup))


_default: Oracle | None = None


def get() -> Oracle:
    """The oracle built from the unmodified source (compiled on first use)."""
    global _default
    if _default is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _default = Oracle(LIB)
    return _default


def sy2sb(A, w, ncols=-1):
    return get().sy2sb(A, w, ncols)


def ge2gb(A, w, ncols=-1):
    return get().ge2gb(A, w, ncols)
