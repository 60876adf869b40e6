"""GPU tests of the eigenvalue pipeline after the band reduction (through the
C ABI): band -> tridiagonal by bulge chasing (bandred_sb2st) and the
tridiagonal matrix's eigenvalues (bandred_tridiag_eigvals).

The tridiagonal form is unique only up to signs and rounding (two stable
tridiagonalisations of one band differ far above 1e-14 n entry by entry), so
what is compared is the spectrum: the GPU's eigenvalues against the oracle's
(its own Householder tridiagonalisation and bisection) and against the known
spectrum, within 1e-14 n of the matrix scale; the tridiagonal form is checked
for what must hold (orthogonal similarity: same Frobenius norm and trace).
A band that is already tridiagonal comes back bit for bit."""
import numpy as np
import pytest
import torch

from paper_1709_00302_amd import inputs
from tests.gpu_util import to_device_colmajor

pytestmark = pytest.mark.gpu


def _band_dense(Ao, w):
    n = Ao.shape[0]
    i = np.arange(n)
    dd = i[:, None] - i[None, :]
    B = np.where((dd >= 0) & (dd <= w), Ao, 0.0)
    return B + np.tril(B, -1).T


@pytest.mark.parametrize("n,w,seed", [(300, 16, 0), (513, 32, 1), (1000, 64, 2), (700, 128, 3),
                                      (257, 5, 4), (130, 127, 5), (90, 200, 6), (3, 2, 7),
                                      (2, 1, 8), (1, 1, 9), (1500, 48, 10)])
def test_sb2st_spectrum_matches_oracle(bandred, orc, n, w, seed):
    print(f"case sb2st n={n} w={w} seed={seed}", flush=True)
    A = inputs.sym_normal(n, 800 + seed)
    Ao, _ = orc.sy2sb(A, w)  # an oracle band
    Ad, _ = to_device_colmajor(Ao, n)
    d, e = bandred.sb2st(Ad, w)
    torch.cuda.synchronize()
    dh, eh = d.cpu().numpy(), e.cpu().numpy()
    B = _band_dense(Ao, min(w, max(n - 1, 0)))
    nB = np.linalg.norm(B)
    # orthogonal similarity: Frobenius norm and trace
    fro = np.sqrt(np.sum(dh ** 2) + 2 * np.sum(eh ** 2))
    assert abs(fro - nB) <= 1e-14 * n * nB
    assert abs(dh.sum() - np.trace(B)) <= 1e-14 * n * nB
    lam_gpu_T = orc.tridiag_eigvals(dh, eh)
    lam_ref = orc.band_eigvals(Ao, min(w, max(n - 1, 0)))
    assert np.abs(lam_gpu_T - lam_ref).max() <= 1e-14 * n * nB, np.abs(lam_gpu_T - lam_ref).max()
    # the band itself is not modified
    assert torch.equal(Ad, to_device_colmajor(Ao, n)[0])


def test_sb2st_tridiagonal_input_is_exact(bandred):
    n = 400
    g = np.random.default_rng(3)
    T = np.diag(g.standard_normal(n)) + np.diag(g.standard_normal(n - 1), -1)
    Td, _ = to_device_colmajor(T, n)
    d, e = bandred.sb2st(Td, 1)
    torch.cuda.synchronize()
    assert np.array_equal(d.cpu().numpy(), np.diag(T)) and np.array_equal(e.cpu().numpy(),
                                                                          np.diag(T, -1))


@pytest.mark.parametrize("kind,n", [("random", 1), ("random", 2), ("random", 600), ("random", 2049),
                                    ("random", 4096), ("toeplitz", 500), ("kac", 300),
                                    ("diagonal", 100)])
def test_tridiag_eigvals_matches_oracle(bandred, orc, kind, n):
    print(f"case tridiag eig {kind} n={n}", flush=True)
    g = np.random.default_rng(n)
    if kind == "random":
        d, e = g.standard_normal(n), g.standard_normal(max(n - 1, 0))
    elif kind == "toeplitz":
        d, e = 2.0 * np.ones(n), -np.ones(n - 1)
    elif kind == "kac":
        i = np.arange(1, n)
        d, e = np.zeros(n), np.sqrt(i * (n - i))
    else:
        d, e = g.standard_normal(n), np.zeros(n - 1)
    dd = torch.from_numpy(d).cuda()
    ed = torch.from_numpy(np.ascontiguousarray(e)).cuda() if n > 1 else torch.zeros(1, dtype=torch.float64, device="cuda")
    lam = bandred.tridiag_eigvals(dd, ed)
    torch.cuda.synchronize()
    got = lam.cpu().numpy()
    ref = orc.tridiag_eigvals(d, e)
    scale = np.abs(d).max() + 2 * (np.abs(e).max() if n > 1 else 0.0)
    assert np.all(np.diff(got) >= 0)
    assert np.abs(got - ref).max() <= 1e-14 * max(n, 4) * scale, np.abs(got - ref).max()
    if kind == "toeplitz":
        k = np.arange(1, n + 1)
        assert np.abs(got - np.sort(2 - 2 * np.cos(k * np.pi / (n + 1)))).max() <= 1e-14 * n * 4
    if kind == "kac":
        assert np.abs(got - np.arange(-(n - 1), n, 2)).max() <= 1e-14 * n * n


@pytest.mark.parametrize("n", [2048, 4096, 8192, 16384])
def test_tridiag_eigvals_closed_forms_large(bandred, n):
    """The section narrows as n grows (64, 32, 16 and 8 lanes per eigenvalue
    at these orders): the second-difference matrix (eigenvalues 2 - 2 cos(k pi /
    (n + 1))) and the Kac matrix (eigenvalues -(n-1), -(n-3), .., n-1)."""
    print(f"case tridiag eig closed forms n={n}", flush=True)
    k = np.arange(1, n + 1)
    d, e = 2.0 * np.ones(n), -np.ones(n - 1)
    lam = bandred.tridiag_eigvals(torch.from_numpy(d).cuda(), torch.from_numpy(e).cuda())
    i = np.arange(1, n)
    lam2 = bandred.tridiag_eigvals(torch.zeros(n, dtype=torch.float64, device="cuda"),
                                   torch.from_numpy(np.sqrt(i * (n - i))).cuda())
    torch.cuda.synchronize()
    got, got2 = lam.cpu().numpy(), lam2.cpu().numpy()
    assert np.all(np.diff(got) >= 0) and np.all(np.diff(got2) >= 0)
    assert np.abs(got - np.sort(2 - 2 * np.cos(k * np.pi / (n + 1)))).max() <= 1e-14 * n * 4
    assert np.abs(got2 - np.arange(-(n - 1), n, 2)).max() <= 1e-14 * n * n


def test_pipeline_known_spectrum(bandred):
    """Stage 1, stage 2 and the eigenvalues, all on the GPU, for A = Q
    diag(lambda) Q^T: every eigenvalue within 1e-14 n of the known one."""
    n, w = 2000, 64
    g = inputs.rng(11)
    lam = inputs.uniform_lambda(n, g)
    A = inputs.sym_known(n, lam, g)
    Ad, _ = to_device_colmajor(A, n)
    print(f"case pipeline n={n} w={w}", flush=True)
    bandred.sy2sb(Ad, w, w)
    d, e = bandred.sb2st(Ad, w)
    ev = bandred.tridiag_eigvals(d, e)
    torch.cuda.synchronize()
    err = np.abs(ev.cpu().numpy() - np.sort(lam)).max()
    print(f"  max |lambda_gpu - lambda| = {err:.3e}", flush=True)
    assert err <= 1e-14 * n * np.abs(lam).max()


def test_stage2_argument_errors(bandred):
    A = torch.zeros((4, 4), dtype=torch.float64, device="cuda")
    p = A.data_ptr()
    assert bandred.bandred_sb2st(-1, 1, p, 4, p, p) == -1
    assert bandred.bandred_sb2st(4, 0, p, 4, p, p) == -2
    assert bandred.bandred_sb2st(4, 1, p, 3, p, p) == -4
    assert bandred.bandred_tridiag_eigvals(-1, p, p, p) == -1
    assert bandred.bandred_tridiag_eigvals(4, p, None, p) == -3


def test_sb2st_timeout_is_reported(bandred):
    """The bulge chasing's inter-workgroup waits (before a step, and before a
    step loads its block below) bounded to one microsecond from the host: the
    first sweep that waits longer gives up and raises the abort flag, every
    other workgroup returns at its next wait, and the call reports
    BANDRED_ERR_TIMEOUT.  Nothing faults or hangs.  With the default bound the
    same call succeeds and preserves the band's Frobenius norm."""
    n, w = 2000, 32
    A = inputs.sym_normal(n, 812)  # only the band 0 <= i - j <= w is read
    Ad, _ = to_device_colmajor(A, n)
    print(f"case sb2st timeout n={n} w={w}", flush=True)
    assert bandred.bandred_set_wait_limit_us(1.0) == 0
    try:
        with pytest.raises(bandred.BandredError) as ei:
            bandred.sb2st(Ad, w)
        assert ei.value.code == 4  # BANDRED_ERR_TIMEOUT
    finally:
        assert bandred.bandred_set_wait_limit_us(0.0) == 0
    d, e = bandred.sb2st(Ad, w)
    torch.cuda.synchronize()
    assert bandred.bandred_status(None) == 0
    B = _band_dense(A, w)
    dh, eh = d.cpu().numpy(), e.cpu().numpy()
    fro = np.sqrt(np.sum(dh ** 2) + 2 * np.sum(eh ** 2))
    assert abs(fro - np.linalg.norm(B)) <= 1e-14 * n * np.linalg.norm(B)
