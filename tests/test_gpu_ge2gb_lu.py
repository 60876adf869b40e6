"""GPU parity of the equal-bandwidth GE2GB (Sec. 3.3, through the C ABI)
against the CPU oracle, element by element: band entries (-w <= j-i <= w),
the left reflectors below the lower band, the right reflectors right of the
upper band, tauq and taup.  Tolerances as for the other reductions: 1e-14
max(m, n) for v and tau (|v_i| <= 1, tau in [1, 2]), the same scaled by the
largest band entry for band entries."""
import numpy as np
import pytest
import torch

from paper_1709_00302_amd import inputs, metrics
from tests.gpu_util import ge_band_max, to_device_colmajor

pytestmark = pytest.mark.gpu

# (m, n, w, b, seed): Variant V2 (2b > w) and V1 (2b <= w), several panels with
# a ragged last one, m > n (left panels outlast the right ones), b < w, w = 1
CASES = [
    (300, 200, 16, 16, 0),
    (256, 256, 32, 32, 1),
    (513, 300, 24, 8, 2),
    (600, 450, 64, 32, 3),
    (1000, 700, 128, 128, 4),
    (50, 50, 1, 1, 5),
    (130, 129, 40, 40, 6),
    (700, 520, 96, 64, 7),
    (2050, 1100, 128, 128, 8),
]


def lu_compare(Ag, tqg, tpg, Ao, tqo, tpo, w):
    m, n = Ao.shape
    i = np.arange(m)[:, None]
    j = np.arange(n)[None, :]
    band = np.abs(j - i) <= w
    left = i - j > w
    right = j - i > w
    f = lambda msk: float(np.max(np.abs(Ag[msk] - Ao[msk]))) if msk.any() else 0.0
    return (f(band), f(left), f(right), float(np.max(np.abs(tqg - tqo), initial=0.0)),
            float(np.max(np.abs(tpg - tpo), initial=0.0)))


def _run(br, A, w, b, prec="fp64", method=0, lookahead=True):
    Ad, _ = to_device_colmajor(A)
    tq, tp = br.ge2gb_lu(Ad, w, b, prec=prec, panel_method=method, lookahead=lookahead)
    torch.cuda.synchronize()
    return Ad.cpu().numpy(), tq.cpu().numpy(), tp.cpu().numpy()


@pytest.mark.parametrize("method", [0, 1], ids=["cholqr2", "percolumn"])
@pytest.mark.parametrize("m,n,w,b,seed", CASES)
def test_ge2gb_lu_matches_oracle(bandred, orc, m, n, w, b, seed, method):
    print(f"case ge2gb_lu m={m} n={n} w={w} b={b} seed={seed} method={method}", flush=True)
    A = inputs.ge_normal(m, n, 300 + seed)
    Ag, tqg, tpg = _run(bandred, A, w, b, method=method)
    Ao, tqo, tpo = orc.ge2gb_lu(A, w)
    db, dl, dr, dq, dp = lu_compare(Ag, tqg, tpg, Ao, tqo, tpo, w)
    tol = 1e-14 * max(m, n)
    assert db <= tol * ge_band_max(Ao, w, lower=w), (db, tol)
    assert max(dl, dr, dq, dp) <= tol, (dl, dr, dq, dp)
    if m <= 1100:
        err = metrics.ge2gb_errors(A, Ag, tqg, tpg, w, svd=False, lower=w)
        assert err["backward"] <= tol, err


def test_ge2gb_lu_symmetric_input_gives_sy2sb(bandred, orc):
    """A symmetric input: the equal-bandwidth reduction is the symmetric band
    reduction (the GPU result against the oracle's SY2SB)."""
    n, w = 900, 64
    A = inputs.sym_normal(n, 41)
    Ag, tqg, tpg = _run(bandred, A, w, w)
    Ao, to = orc.sy2sb(A, w)
    tol = 1e-14 * n
    k = n - w
    assert np.abs(np.tril(Ag) - np.tril(Ao)).max() <= tol * ge_band_max(Ao, w, lower=w)
    assert np.abs(tqg[:k] - to).max() <= tol and np.abs(tpg[:k] - to).max() <= tol


def test_ge2gb_lu_banded_input_is_exact(bandred):
    m, n, w = 300, 200, 10
    A = inputs.ge_normal(m, n, 42)
    i = np.arange(m)[:, None]
    j = np.arange(n)[None, :]
    A[np.abs(j - i) > w] = 0.0
    Ag, tqg, tpg = _run(bandred, A, w, w)
    assert np.all(tqg == 0.0) and np.all(tpg == 0.0)
    assert np.array_equal(Ag, A)


def test_ge2gb_lu_known_sigma(bandred):
    g = inputs.rng(43)
    m, n, w = 1500, 1200, 64
    sig = inputs.logu_sigma(n, g)
    A = inputs.ge_known(m, n, sig, g)
    Ag, tqg, tpg = _run(bandred, A, w, w)
    err = metrics.ge2gb_errors(A, Ag, tqg, tpg, w, sigma=sig, lower=w)
    print(f"  ge2gb_lu known sigma: {err}", flush=True)
    tol = 1e-14 * m
    assert err["backward"] <= tol and err["orth"] <= tol and err["band_trunc"] <= tol, err
    assert err["sv_err"] <= tol, err


@pytest.mark.parametrize("m,n,w,b", [(1200, 900, 64, 64), (1000, 1000, 128, 64),
                                     (1400, 1300, 128, 128)])
def test_ge2gb_lu_lookahead_is_bit_identical_to_serial(bandred, m, n, w, b):
    print(f"case ge2gb_lu lookahead m={m} n={n} w={w} b={b}", flush=True)
    A = inputs.ge_normal(m, n, 600 + w + b)
    la = _run(bandred, A, w, b, lookahead=True)
    se = _run(bandred, A, w, b, lookahead=False)
    for x, y in zip(la, se):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("prec", ["fp32", "split32"])
def test_ge2gb_lu_precision_forms(bandred, orc, prec):
    """Reduced-precision trailing updates: backward error within the form's
    bound (1e-5 max(m, n) for both; the split form is far inside it), every
    reflector orthogonal to FP64 accuracy, tau = 0 exactly where the oracle
    has it."""
    m, n, w = 1200, 1000, 64
    A = inputs.ge_normal(m, n, 44)
    Ag, tqg, tpg = _run(bandred, A, w, w, prec=prec)
    Ao, tqo, tpo = orc.ge2gb_lu(A, w)
    err = metrics.ge2gb_errors(A, Ag, tqg, tpg, w, svd=False, lower=w)
    print(f"  ge2gb_lu {prec}: {err}", flush=True)
    assert err["backward"] <= 1e-5 * m, err
    assert err["orth"] <= 1e-14 * m, err
    assert np.array_equal(tqg == 0.0, tqo == 0.0) and np.array_equal(tpg == 0.0, tpo == 0.0)


def test_ge2gb_lu_graph_replay_matches_eager(bandred):
    m, n, w = 1000, 900, 64
    A = inputs.ge_normal(m, n, 45)
    A0, _ = to_device_colmajor(A)
    Ad = A0.clone()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        tq_e, tp_e = bandred.ge2gb_lu(Ad, w, w, stream=s)
    torch.cuda.synchronize()
    ref, rq, rp = Ad.clone(), tq_e.clone(), tp_e.clone()
    Ad.copy_(A0)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            tq_g, tp_g = bandred.ge2gb_lu(Ad, w, w, stream=s)
    torch.cuda.synchronize()
    print("case ge2gb_lu graph replays", flush=True)
    for rep in range(3):
        Ad.copy_(A0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()
        assert torch.equal(Ad, ref) and torch.equal(tq_g, rq) and torch.equal(tp_g, rp), rep


def test_ge2gb_lu_argument_errors(bandred):
    A = torch.zeros((10, 8), dtype=torch.float64, device="cuda").T.contiguous().T
    t = torch.zeros(8, dtype=torch.float64, device="cuda")
    f = bandred.bandred_ge2gb_lu
    assert f(8, 10, 2, 2, A.data_ptr(), 8, t.data_ptr(), t.data_ptr()) == -1  # m < n
    assert f(10, 8, 0, 1, A.data_ptr(), 10, t.data_ptr(), t.data_ptr()) == -3
    assert f(10, 8, 2, 3, A.data_ptr(), 10, t.data_ptr(), t.data_ptr()) == -4
    assert f(10, 8, 2, 2, A.data_ptr(), 9, t.data_ptr(), t.data_ptr()) == -6
    assert f(10, 8, 2, 2, A.data_ptr(), 10, t.data_ptr(), t.data_ptr(), 7) == -9
