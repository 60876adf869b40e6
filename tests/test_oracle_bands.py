"""Pins of the oracle's equal-bandwidth reduction (Sec. 3.3) and of its
back-transformation (the stored reflectors applied to a matrix).

Each pin checks the oracle against an independent fact:

  * a symmetric input reduced to the equal-bandwidth form is the symmetric
    band reduction of Sec. 2.1 (the left and right reflectors of one step
    coincide), and at w = 1 LAPACK's dsytrd (an independent implementation
    with the same reflector convention);
  * singular values are preserved (self-written one-sided Jacobi for small
    sizes, a known sigma for larger ones);
  * an input that already has the band structure is returned bit-for-bit
    with every tau = 0; the prefix property;
  * the products of stored reflectors equal LAPACK's dormqr on the same
    storage (reflectors stored as the columns of a QR factorisation, shifted
    by the band offset, or transposed for the right reflectors), in both
    directions; Q^T A Q reproduces the band the reduction returned;
  * planted mistakes (rows c+1..c+w-1 skipped by the right update, in-band
    columns skipped by the left update, Q C applied in the order of Q^T C)
    are each caught.
"""
import numpy as np
import pytest
from scipy.linalg import lapack

import oracle
from paper_1709_00302_amd import inputs, metrics
from tests.test_oracle import hestenes_singvals

EPS = np.finfo(np.float64).eps


def lu_band_of(Aout, w):
    """Dense band B (-w <= j-i <= w) of an equal-bandwidth result."""
    m, n = Aout.shape
    i = np.arange(m)[:, None]
    j = np.arange(n)[None, :]
    return np.where(np.abs(j - i) <= w, Aout, 0.0)


def dormqr(Aq, tau, C, trans):
    """LAPACK: Q C or Q^T C for reflectors stored as a QR factorisation
    (column c: v[0] = 1 at row c, v[1:] below)."""
    lw = max(1, C.shape[1]) * 64
    cq, work, info = lapack.dormqr(b"L", b"T" if trans else b"N", np.asfortranarray(Aq),
                                   np.ascontiguousarray(tau), np.asfortranarray(C.copy()), lw)
    assert info == 0
    return cq


# ----------------------------------------------------------------------------
# ge2gb_lu (equal lower and upper bandwidth)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("n,w", [(40, 1), (60, 3), (61, 8), (30, 29)])
def test_ge2gb_lu_symmetric_input_is_sy2sb(orc, n, w):
    A = inputs.sym_normal(n, n + w)
    a1, t1 = orc.sy2sb(A, w)
    a2, tq, tp = orc.ge2gb_lu(A, w)
    tol = 1e-14 * n * np.abs(A).max() * np.sqrt(n)
    assert np.abs(np.tril(a1) - np.tril(a2)).max() <= tol
    k = max(n - w, 0)
    assert np.abs(t1 - tq[:k]).max(initial=0.0) <= 1e-14 * n
    assert np.all(tq[k:] == 0.0) and np.all(tp[k:] == 0.0)
    # the right reflectors are the left ones (mirrored storage)
    assert np.abs(tq - tp).max() <= 1e-14 * n
    assert np.abs(np.triu(a2, 1) - np.tril(a2, -1).T).max() <= tol


def test_ge2gb_lu_w1_symmetric_equals_lapack_dsytrd(orc):
    n = 30
    A = inputs.sym_normal(n, 4)
    a, tq, tp = orc.ge2gb_lu(A, 1)
    c, d, e, tl, info = lapack.dsytrd(A, lower=1)
    assert info == 0
    assert np.abs(np.diag(a) - d).max() <= 1e-13 and np.abs(np.diag(a, -1) - e).max() <= 1e-13
    assert np.abs(tq[: n - 1] - tl).max() <= 1e-13


@pytest.mark.parametrize("m,n,w", [(8, 6, 1), (12, 12, 2), (16, 10, 3), (16, 16, 6), (15, 9, 9)])
def test_ge2gb_lu_singular_values_vs_jacobi(orc, m, n, w):
    A = inputs.ge_normal(m, n, 3 * m * n + w)
    Aout, tq, tp = orc.ge2gb_lu(A, w)
    B = lu_band_of(Aout, w)
    assert np.abs(hestenes_singvals(A) - hestenes_singvals(B)).max() \
        <= 100 * m * EPS * np.linalg.norm(A)


def test_ge2gb_lu_known_sigma(orc):
    g = inputs.rng(13)
    m, n, w = 150, 100, 7
    sig = inputs.logu_sigma(n, g)
    A = inputs.ge_known(m, n, sig, g)
    Aout, tq, tp = orc.ge2gb_lu(A, w)
    err = metrics.ge2gb_errors(A, Aout, tq, tp, w, sigma=sig, lower=w)
    assert err["backward"] <= 1e-14 * m, err
    assert err["orth"] <= 1e-14 * m, err
    assert err["band_trunc"] <= 1e-14 * m, err
    assert err["sv_err"] <= 1e-14 * m, err


def test_ge2gb_lu_tau_layout(orc):
    m, n, w = 50, 40, 6
    A = inputs.ge_normal(m, n, 9)
    Aout, tq, tp = orc.ge2gb_lu(A, w)
    # left reflectors of length >= 2: c <= m-w-2; right: c <= n-w-2
    assert np.all(tq[: m - w - 1] != 0.0) and np.all(tq[m - w - 1:] == 0.0)
    assert np.all(tp[: n - w - 1] != 0.0) and np.all(tp[n - w - 1:] == 0.0)


def test_ge2gb_lu_banded_input_bit_exact(orc):
    m, n, w = 50, 40, 6
    A = inputs.ge_normal(m, n, 10)
    i = np.arange(m)[:, None]
    j = np.arange(n)[None, :]
    A[np.abs(j - i) > w] = 0.0
    Aout, tq, tp = orc.ge2gb_lu(A, w)
    assert np.array_equal(Aout, A)
    assert np.all(tq == 0.0) and np.all(tp == 0.0)


def test_ge2gb_lu_prefix_property(orc):
    A = inputs.ge_normal(60, 50, 11)
    w, k = 5, 7
    full, tqf, tpf = orc.ge2gb_lu(A, w)
    part, tqp, tpp = orc.ge2gb_lu(A, w, ncols=k)
    # columns < k (from row w on) and rows < k are final after k steps
    assert np.array_equal(part[:, :k], full[:, :k])
    assert np.array_equal(part[:k, :], full[:k, :])
    assert np.array_equal(tqp[:k], tqf[:k]) and np.array_equal(tpp[:k], tpf[:k])


def test_ge2gb_lu_argument_errors(orc):
    A = np.zeros((4, 5))
    t = np.zeros(5)
    p = orc._ptr
    lib = orc.lib
    assert lib.oracle_ge2gb_lu(4, 5, 1, -1, p(np.asfortranarray(A)), 4, p(t), p(t)) == -1
    B = np.zeros((5, 4), order="F")
    assert lib.oracle_ge2gb_lu(5, 4, 0, -1, p(B), 5, p(t), p(t)) == -3
    assert lib.oracle_ge2gb_lu(5, 4, 1, -1, p(B), 4, p(t), p(t)) == -6


# ----------------------------------------------------------------------------
# back-transformation
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("trans", [False, True])
def test_sy2sb_q_equals_lapack_dormqr(orc, trans):
    n, w, k = 70, 6, 9
    A = inputs.sym_normal(n, 21)
    Aout, tau = orc.sy2sb(A, w)
    C = inputs.ge_normal(n, k, 22)
    got = orc.sy2sb_q(Aout, tau, w, C, trans)
    # Q is the identity on the first w indices and, below, the Q of a QR
    # factorisation whose column c is stored in Aout(w:, c)
    ref = C.copy()
    ref[w:] = dormqr(Aout[w:, : n - w], tau, C[w:], trans)
    assert np.abs(got - ref).max() <= 1e-14 * n


@pytest.mark.parametrize("trans", [False, True])
def test_ge2gb_factors_equal_lapack_dormqr(orc, trans):
    m, n, w, k = 60, 45, 5, 7
    A = inputs.ge_normal(m, n, 23)
    Aout, tq, tp = orc.ge2gb(A, w)
    C = inputs.ge_normal(m, k, 24)
    got = orc.ge2gb_u(Aout, tq, w, C, trans)
    assert np.abs(got - dormqr(Aout, tq, C, trans)).max() <= 1e-14 * m
    C = inputs.ge_normal(n, k, 25)
    got = orc.ge2gb_v(Aout, tp, w, C, trans)
    ref = C.copy()
    ref[w:] = dormqr(Aout[: n - w, w:].T, tp[: n - w], C[w:], trans)
    assert np.abs(got - ref).max() <= 1e-14 * n


@pytest.mark.parametrize("trans", [False, True])
def test_ge2gb_lu_factors_equal_lapack_dormqr(orc, trans):
    m, n, w, k = 64, 50, 6, 5
    A = inputs.ge_normal(m, n, 26)
    Aout, tq, tp = orc.ge2gb_lu(A, w)
    C = inputs.ge_normal(m, k, 27)
    got = orc.ge2gb_u(Aout, tq, w, C, trans, equal_band=True)
    ref = C.copy()
    nl = min(n, m - w)
    ref[w:] = dormqr(Aout[w:, :nl], tq[:nl], C[w:], trans)
    assert np.abs(got - ref).max() <= 1e-14 * m
    C = inputs.ge_normal(n, k, 28)
    got = orc.ge2gb_v(Aout, tp, w, C, trans)
    ref = C.copy()
    ref[w:] = dormqr(Aout[: n - w, w:].T, tp[: n - w], C[w:], trans)
    assert np.abs(got - ref).max() <= 1e-14 * n


def test_back_transformation_reproduces_the_band(orc):
    """Q^T A Q (SY2SB) and U^T A V (both GE2GB forms) built with the applied
    factors equal the band the reductions returned, zeros outside it."""
    n, w = 80, 7
    A = inputs.sym_normal(n, 29)
    Aout, tau = orc.sy2sb(A, w)
    QtAQ = orc.sy2sb_q(Aout, tau, w, orc.sy2sb_q(Aout, tau, w, A, True).T, True).T
    B = np.tril(Aout)
    i = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    band = np.abs(i - j) <= w
    Bf = np.where(band & (i >= j), B, 0.0)
    Bf = Bf + np.tril(Bf, -1).T
    assert np.abs(QtAQ - Bf).max() <= 1e-14 * n * np.linalg.norm(A)
    m, n = 90, 70
    G = inputs.ge_normal(m, n, 30)
    for lu in (False, True):
        Ao, tq, tp = (orc.ge2gb_lu if lu else orc.ge2gb)(G, w)
        UtA = orc.ge2gb_u(Ao, tq, w, G, True, equal_band=lu)
        UtAV = orc.ge2gb_v(Ao, tp, w, UtA.T, True).T
        ii = np.arange(m)[:, None]
        jj = np.arange(n)[None, :]
        keep = (np.abs(jj - ii) <= w) if lu else ((jj - ii >= 0) & (jj - ii <= w))
        assert np.abs(UtAV - np.where(keep, Ao, 0.0)).max() <= 1e-14 * m * np.linalg.norm(G)


def test_apply_then_transpose_is_identity(orc):
    n, w = 50, 4
    A = inputs.sym_normal(n, 31)
    Aout, tau = orc.sy2sb(A, w)
    C = inputs.ge_normal(n, 6, 32)
    back = orc.sy2sb_q(Aout, tau, w, orc.sy2sb_q(Aout, tau, w, C, False), True)
    assert np.abs(back - C).max() <= 1e-14 * n


# ----------------------------------------------------------------------------
# planted mistakes
# ----------------------------------------------------------------------------

def _pins_fail_lu(o):
    A = inputs.ge_normal(50, 40, 33)
    Aout, tq, tp = o.ge2gb_lu(A, 5)
    err = metrics.ge2gb_errors(A, Aout, tq, tp, 5, svd=False, lower=5)
    if not (err["backward"] <= 1e-14 * 50):
        return True
    S = inputs.sym_normal(30, 34)
    a1, t1 = o.sy2sb(S, 4)
    a2, q2, p2 = o.ge2gb_lu(S, 4)
    return np.abs(np.tril(a1) - np.tril(a2)).max() > 1e-11


def _pins_fail_apply(o):
    n, w = 40, 3
    A = inputs.sym_normal(n, 35)
    Aout, tau = o.sy2sb(A, w)
    C = inputs.ge_normal(n, 4, 36)
    for trans in (False, True):
        ref = C.copy()
        ref[w:] = dormqr(Aout[w:, : n - w], tau, C[w:], trans)
        if np.abs(o.sy2sb_q(Aout, tau, w, C, trans) - ref).max() > 1e-12:
            return True
    return False


@pytest.mark.parametrize("mutant,kind", [(7, "lu"), (8, "lu"), (9, "apply")])
def test_planted_mistakes_are_caught(tmp_path, mutant, kind):
    path = str(tmp_path / f"liboracle_m{mutant}.so")
    oracle.build(out=path, mutant=mutant)
    o = oracle.Oracle(path)
    assert (_pins_fail_lu(o) if kind == "lu" else _pins_fail_apply(o))


def test_unmodified_oracle_passes_the_same_pins(orc):
    assert not _pins_fail_lu(orc)
    assert not _pins_fail_apply(orc)
