"""Pins of the oracle's eigenvalue step for the two-stage pipeline (band ->
tridiagonal -> eigenvalues): bisection on Sturm counts for a symmetric
tridiagonal matrix, and the band matrix's eigenvalues through the oracle's
own tridiagonalisation.  Independent facts:

  * LAPACK's dsterf (QL/QR, Pal-Walker-Kahan) and dstebz (its own bisection);
  * closed forms: tridiag(-1, 2, -1) has 2 - 2 cos(k pi / (n+1)); the
    symmetric Kac (Clement) matrix, zero diagonal and e_i = sqrt(i (n-i)),
    has the integers -(n-1), -(n-3), ..., n-1; 2 x 2 matrices; a diagonal
    matrix has its sorted diagonal;
  * a band matrix of known spectrum (stage 1 on Q diag(lambda) Q^T) and
    LAPACK's banded eigensolver;
  * a planted mistake in the Sturm recurrence is caught.
"""
import numpy as np
import pytest
from scipy.linalg import eigvals_banded, lapack

import oracle
from paper_1709_00302_amd import inputs

EPS = np.finfo(np.float64).eps


def _tnorm(d, e):
    r = np.abs(d).copy()
    r[:-1] += np.abs(e)
    r[1:] += np.abs(e)
    return r.max()


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (7, 2), (100, 3), (700, 4)])
def test_tridiag_eigvals_vs_lapack(orc, n, seed):
    g = np.random.default_rng(seed)
    d = g.standard_normal(n)
    e = g.standard_normal(max(n - 1, 0))
    got = orc.tridiag_eigvals(d, e)
    if n == 1:
        assert abs(got[0] - d[0]) <= 2 * EPS * abs(d[0])
        return
    ref1, info = lapack.dsterf(d.copy(), e.copy())
    assert info == 0
    m, w, iblock, isplit, info = lapack.dstebz(d, e, 0, 0.0, 0.0, 0, 0, 0.0, b"E")
    assert info == 0 and m == n
    tol = 4 * n * EPS * _tnorm(d, e)
    assert np.abs(got - np.sort(ref1)).max() <= tol
    assert np.abs(got - np.sort(w[:m])).max() <= tol


@pytest.mark.parametrize("n", [1, 2, 50, 400])
def test_tridiag_eigvals_closed_forms(orc, n):
    k = np.arange(1, n + 1)
    got = orc.tridiag_eigvals(2.0 * np.ones(n), -np.ones(max(n - 1, 0)))
    assert np.abs(got - np.sort(2 - 2 * np.cos(k * np.pi / (n + 1)))).max() <= 8 * EPS * 4
    if n > 1:
        i = np.arange(1, n)
        kac = orc.tridiag_eigvals(np.zeros(n), np.sqrt(i * (n - i)))
        assert np.abs(kac - np.arange(-(n - 1), n, 2)).max() <= 8 * n * EPS * n


def test_tridiag_eigvals_2x2_and_diagonal(orc):
    a, b, c = 0.3, -1.7, 2.2
    got = orc.tridiag_eigvals([a, c], [b])
    m, r = 0.5 * (a + c), np.hypot(0.5 * (a - c), b)
    assert np.abs(got - [m - r, m + r]).max() <= 4 * EPS * 3
    d = np.array([3.0, -1.0, 0.5, 2.0, -7.25])
    got = orc.tridiag_eigvals(d, np.zeros(4))
    assert np.abs(got - np.sort(d)).max() <= 2 * EPS * 7.25


def test_band_eigvals_known_spectrum(orc):
    g = inputs.rng(20)
    n, w = 300, 12
    lam = inputs.uniform_lambda(n, g)
    A = inputs.sym_known(n, lam, g)
    Aout, tau = orc.sy2sb(A, w)
    got = orc.band_eigvals(Aout, w)
    assert np.abs(got - np.sort(lam)).max() <= 1e-14 * n
    band = np.zeros((w + 1, n))
    for k in range(w + 1):
        band[k, : n - k] = np.diagonal(Aout, -k)
    assert np.abs(got - np.sort(eigvals_banded(band, lower=True))).max() <= 1e-14 * n


def test_tridiag_argument_errors(orc):
    assert orc.lib.oracle_tridiag_eigvals(-1, None, None, None) == -1


def test_planted_sturm_mistake_is_caught(tmp_path):
    path = str(tmp_path / "liboracle_m10.so")
    oracle.build(out=path, mutant=10)
    o = oracle.Oracle(path)
    n = 60
    k = np.arange(1, n + 1)
    got = o.tridiag_eigvals(2.0 * np.ones(n), -np.ones(n - 1))
    assert np.abs(got - np.sort(2 - 2 * np.cos(k * np.pi / (n + 1)))).max() > 1e-6
