"""GPU parity of the back-transformation (the stored reflectors of a
reduction applied to a matrix, through the C ABI) against the oracle's
one-reflector-at-a-time product, element by element, for the factors of
SY2SB (Q), GE2GB (U, V) and the equal-bandwidth GE2GB (U, V), both
directions, several block sizes and ragged column counts.  Each entry of
Q C is a sum of n products of O(1) terms: tolerance 1e-14 n max|C|."""
import numpy as np
import pytest
import torch

from paper_1709_00302_amd import inputs
from tests.gpu_util import to_device_colmajor

pytestmark = pytest.mark.gpu


def _colmajor(X, lda=None):
    t, _ = to_device_colmajor(X, lda)
    return t


@pytest.mark.parametrize("trans", [False, True])
@pytest.mark.parametrize("n,w,b,k", [(700, 32, 32, 50), (1000, 64, 128, 257), (513, 16, 7, 1),
                                     (300, 128, 64, 300)])
def test_sy2sb_apply_q_matches_oracle(bandred, orc, n, w, b, k, trans):
    print(f"case apply_q n={n} w={w} b={b} k={k} trans={trans}", flush=True)
    A = inputs.sym_normal(n, 51)
    Ao, to = orc.sy2sb(A, w)
    C = inputs.ge_normal(n, k, 52)
    ref = orc.sy2sb_q(Ao, to, w, C, trans)
    Ad = _colmajor(Ao)
    td = torch.from_numpy(np.ascontiguousarray(to)).cuda()
    Cd = _colmajor(C, n + 5)  # padded ldc
    bandred.sy2sb_apply_q(Ad, td, w, Cd, trans=trans, b=b)
    torch.cuda.synchronize()
    got = Cd.cpu().numpy()[:n]
    assert np.abs(got - ref).max() <= 1e-14 * n * np.abs(C).max()
    assert np.isnan(Cd.cpu().numpy()[n:]).all()  # padding rows untouched


@pytest.mark.parametrize("equal_band", [False, True])
@pytest.mark.parametrize("side", ["u", "v"])
@pytest.mark.parametrize("trans", [False, True])
def test_ge2gb_apply_matches_oracle(bandred, orc, equal_band, side, trans):
    m, n, w, b, k = 900, 700, 48, 32, 130
    print(f"case ge2gb_apply side={side} equal={equal_band} trans={trans}", flush=True)
    A = inputs.ge_normal(m, n, 53)
    Ao, tq, tp = (orc.ge2gb_lu if equal_band else orc.ge2gb)(A, w)
    rows = m if side == "u" else n
    C = inputs.ge_normal(rows, k, 54)
    if side == "u":
        ref = orc.ge2gb_u(Ao, tq, w, C, trans, equal_band=equal_band)
        tau = tq
    else:
        ref = orc.ge2gb_v(Ao, tp, w, C, trans)
        tau = tp
    Ad = _colmajor(Ao)
    td = torch.from_numpy(np.ascontiguousarray(tau)).cuda()
    Cd = _colmajor(C)
    bandred.ge2gb_apply(Ad, td, w, Cd, side=side, equal_band=equal_band, trans=trans, b=b)
    torch.cuda.synchronize()
    assert np.abs(Cd.cpu().numpy() - ref).max() <= 1e-14 * rows * np.abs(C).max()


def test_gpu_reduction_then_back_transformation(bandred, orc):
    """The whole pipeline on the GPU: reduce, then Q^T A Q from the GPU's own
    reflectors reproduces its band (zeros elsewhere), and Q is orthogonal."""
    n, w = 1200, 64
    A = inputs.sym_normal(n, 55)
    Ad = _colmajor(A)
    tau = bandred.sy2sb(Ad, w, w)
    Af = torch.from_numpy(A).cuda()
    # Q^T A Q = (Q^T (Q^T A)^T)^T with A symmetric
    X = Af.clone().T.contiguous().T
    bandred.sy2sb_apply_q(Ad, tau, w, X, trans=True)
    Y = X.contiguous().T  # (Q^T A)^T, column-major
    bandred.sy2sb_apply_q(Ad, tau, w, Y, trans=True)
    torch.cuda.synchronize()
    B = Y.cpu().numpy()
    Ag = np.tril(Ad.cpu().numpy())
    i = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    band = (i - j >= 0) & (i - j <= w)
    Bl = np.where(band, Ag, 0.0)
    Bf = Bl + np.tril(Bl, -1).T
    nA = np.linalg.norm(A)
    assert np.linalg.norm(B - Bf) <= 1e-14 * n * nA
    Q = torch.eye(n, dtype=torch.float64, device="cuda").T  # column-major
    bandred.sy2sb_apply_q(Ad, tau, w, Q)
    torch.cuda.synchronize()
    Qh = Q.cpu().numpy()
    assert np.linalg.norm(Qh.T @ Qh - np.eye(n)) <= 1e-14 * n


def test_apply_argument_errors(bandred):
    A = torch.zeros((10, 10), dtype=torch.float64, device="cuda")
    t = torch.zeros(10, dtype=torch.float64, device="cuda")
    f = bandred.bandred_sy2sb_apply_q
    p = A.data_ptr()
    assert f(2, 10, 2, 2, p, 10, t.data_ptr(), 3, p, 10) == -1
    assert f(0, 10, 0, 2, p, 10, t.data_ptr(), 3, p, 10) == -3
    assert f(0, 10, 2, 129, p, 10, t.data_ptr(), 3, p, 10) == -4
    assert f(0, 10, 2, 2, p, 10, t.data_ptr(), 3, p, 9) == -10
    g = bandred.bandred_ge2gb_apply
    assert g(2, 0, 0, 10, 10, 2, 2, p, 10, t.data_ptr(), 3, p, 10) == -1
    assert g(0, 0, 0, 9, 10, 2, 2, p, 10, t.data_ptr(), 3, p, 10) == -4
    assert g(1, 1, 0, 10, 10, 2, 2, p, 10, t.data_ptr(), 3, p, 9) == -13
