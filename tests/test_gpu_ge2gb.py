"""GPU parity of GE2GB (through the C ABI) against the CPU oracle.
Tolerances as for SY2SB (1e-14 * n scaled by the largest band entry for band
entries)."""
import numpy as np
import pytest
import torch

from paper_1709_00302_amd import inputs, metrics
from tests.gpu_util import ge_band_max, ge_compare, to_device_colmajor

pytestmark = pytest.mark.gpu

CASES = [
    (300, 200, 16, 16, 0),
    (256, 256, 32, 32, 1),
    (513, 300, 24, 8, 2),
    (400, 390, 64, 64, 3),
    (1000, 700, 128, 128, 4),
    (50, 50, 1, 1, 5),
    (130, 129, 40, 40, 6),
]


def _run(br, A, w, b, prec="fp64", method=0):
    m, n = A.shape
    Ad, lda = to_device_colmajor(A)
    tq, tp = br.ge2gb(Ad, w, b, prec=prec, panel_method=method)
    torch.cuda.synchronize()
    return Ad.cpu().numpy(), tq.cpu().numpy(), tp.cpu().numpy()


@pytest.mark.parametrize("method", [0, 1], ids=["cholqr2", "percolumn"])
@pytest.mark.parametrize("m,n,w,b,seed", CASES)
def test_ge2gb_matches_oracle(bandred, orc, m, n, w, b, seed, method):
    print(f"case ge2gb m={m} n={n} w={w} b={b} seed={seed} method={method}", flush=True)
    A = inputs.ge_normal(m, n, 200 + seed)
    Ag, tqg, tpg = _run(bandred, A, w, b, method=method)
    Ao, tqo, tpo = orc.ge2gb(A, w)
    bmax = ge_band_max(Ao, w)
    db, dl, dr, dq, dp = ge_compare(Ag, tqg, tpg, Ao, tqo, tpo, w)
    tol = 1e-14 * max(m, n)
    assert db <= tol * bmax, (db, tol * bmax)
    assert max(dl, dr, dq, dp) <= tol, (dl, dr, dq, dp)
    err = metrics.ge2gb_errors(A, Ag, tqg, tpg, w, svd=False)
    assert err["backward"] <= tol, err


def test_ge2gb_banded_input_is_exact(bandred):
    m, n, w = 300, 200, 10
    A = inputs.ge_normal(m, n, 77)
    i = np.arange(m)[:, None]
    j = np.arange(n)[None, :]
    A[~((j - i >= 0) & (j - i <= w))] = 0.0
    Ag, tqg, tpg = _run(bandred, A, w, w)
    assert np.all(tqg == 0.0) and np.all(tpg == 0.0)
    assert np.array_equal(Ag, A)


@pytest.mark.parametrize("lookahead", [True, False], ids=["lookahead", "serial"])
def test_ge2gb_reduced_later_panels_fall_back(bandred, orc, lookahead):
    """A = [[A1, 0], [0, D]], D diagonal: the left panels from column s and
    the right panels from row s - w have no nonzero off their band, are
    flagged and take the gated per-column path (tau = 0 as in the oracle)."""
    m, n, w, s = 700, 500, 32, 256
    A = np.zeros((m, n))
    A[:s, :s] = inputs.ge_normal(s, s, 91)
    k = np.arange(n - s)
    A[s + k, s + k] = inputs.ge_normal(n - s, 1, 92)[:, 0]
    print(f"case ge2gb reduced later panels m={m} n={n} w={w} s={s} lookahead={lookahead}",
          flush=True)
    Ad, _ = to_device_colmajor(A)
    tq, tp = bandred.ge2gb(Ad, w, w, lookahead=lookahead)
    torch.cuda.synchronize()
    Ag, tqg, tpg = Ad.cpu().numpy(), tq.cpu().numpy(), tp.cpu().numpy()
    Ao, tqo, tpo = orc.ge2gb(A, w)
    assert np.all(tqo[s:] == 0.0) and np.all(tpo[s - w:] == 0.0)
    assert np.all(tqg[s:] == 0.0) and np.all(tpg[s - w:] == 0.0)
    db, dl, dr, dq, dp = ge_compare(Ag, tqg, tpg, Ao, tqo, tpo, w)
    tol = 1e-14 * m
    assert db <= tol * ge_band_max(Ao, w), db
    assert max(dl, dr, dq, dp) <= tol, (dl, dr, dq, dp)


@pytest.mark.parametrize("m,n,w", [(1200, 900, 64), (700, 700, 32), (1000, 1000, 128)])
def test_ge2gb_lookahead_is_bit_identical_to_serial(bandred, m, n, w):
    """The look-ahead only reorders independent launches (panels on the
    second stream, updates split by rows or columns with the same k order)."""
    print(f"case ge2gb lookahead m={m} n={n} w={w}", flush=True)
    A = inputs.ge_normal(m, n, 500 + w)
    outs = []
    for la in (True, False):
        Ad, _ = to_device_colmajor(A)
        tq, tp = bandred.ge2gb(Ad, w, w, lookahead=la)
        torch.cuda.synchronize()
        outs.append((Ad.cpu().numpy(), tq.cpu().numpy(), tp.cpu().numpy()))
    for x, y in zip(*outs):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("m,n,w", [(1200, 900, 64), (1000, 1000, 128)])
def test_ge2gb_graph_replay_matches_eager(bandred, m, n, w):
    """GE2GB captured in a HIP graph after one eager call and replayed three
    times with eager work in between: each replay equals the eager result."""
    print(f"case ge2gb graph m={m} n={n} w={w}", flush=True)
    A = inputs.ge_normal(m, n, 700 + w)
    A0, _ = to_device_colmajor(A)
    Ad = A0.clone()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        tq_e, tp_e = bandred.ge2gb(Ad, w, w, stream=s)
    torch.cuda.synchronize()
    ref, rq, rp = Ad.clone(), tq_e.clone(), tp_e.clone()
    Ad.copy_(A0)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            tq_g, tp_g = bandred.ge2gb(Ad, w, w, stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        Ad.copy_(A0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()
        assert torch.equal(Ad, ref) and torch.equal(tq_g, rq) and torch.equal(tp_g, rp), rep
