"""GPU parity of the batched SY2SB call (one persistent launch) against the
CPU oracle, matrix by matrix.

Tolerances as for the single-matrix path: band entries within 1e-14 * n *
max|B|, reflector entries and tau within 1e-14 * n, FP64 backward error
<= 1e-14 * n; the FP32-update form is held to a backward error <= 1e-5 * n.
The X = A2 Wt accumulation of the batched kernel adds block contributions of
different waves in arrival order, so two runs agree to rounding, not bit for
bit: repeated runs are compared within the same tolerance.
"""
import numpy as np
import pytest
import torch

from paper_1709_00302_amd import inputs, metrics
from tests.gpu_util import sy_band_max, sy_compare, to_device_colmajor

pytestmark = pytest.mark.gpu


def _batch(sizes, seed, poison=True):
    mats = []
    for k, n in enumerate(sizes):
        A = inputs.sym_normal(n, 1000 * seed + k) if n > 0 else np.zeros((0, 0))
        mats.append(A)
    return mats


def _upload(mats, pads=None, poison=True):
    dev = []
    for k, A in enumerate(mats):
        n = A.shape[0]
        Ain = A.copy()
        if poison and n > 1:
            Ain[np.triu_indices(n, 1)] = np.nan
        pad = 0 if pads is None else pads[k % len(pads)]
        if n == 0:
            dev.append((torch.zeros(1, 1, dtype=torch.float64, device="cuda"), 1))
            continue
        Ad, lda = to_device_colmajor(Ain, n + pad)
        dev.append((Ad, lda))
    return dev


def _run_batched(bandred, dev, ns, w, b, prec=0, stream=None):
    taus = [torch.zeros(max(n - w, 1), dtype=torch.float64, device="cuda") for n in ns]
    rc = bandred.bandred_sy2sb_batched(
        len(ns), ns, w, b, [A.data_ptr() for A, _ in dev], [lda for _, lda in dev],
        [t.data_ptr() for t in taus], prec,
        torch.cuda.current_stream().cuda_stream if stream is None else stream)
    assert rc == 0, bandred.status_string(rc)
    return taus


def _check_against_oracle(orc, mats, dev, taus, w, pads=None, tol_scale=1e-14):
    for k, A in enumerate(mats):
        n = A.shape[0]
        if n == 0:
            continue
        full = dev[k][0].cpu().numpy()
        Ag = full[:n, :]
        tg = taus[k].cpu().numpy()
        assert np.isnan(Ag[np.triu_indices(n, 1)]).all(), f"matrix {k}: upper triangle was written"
        if full.shape[0] > n:
            assert np.isnan(full[n:, :]).all(), f"matrix {k}: rows beyond n were written"
        Ao, to = orc.sy2sb(A, w)
        if n <= w + 1:
            assert np.array_equal(np.tril(Ag), np.tril(A)), k
            assert np.all(tg[: max(n - w, 0)] == 0.0), k
            continue
        db, dr, dt = sy_compare(np.tril(Ag), tg, np.tril(Ao), to, w)
        tol = tol_scale * n
        bmax = sy_band_max(np.tril(Ao), w)
        assert db <= tol * bmax and dr <= tol and dt <= tol, (k, n, db, dr, dt, tol)


@pytest.mark.parametrize("w,b", [(16, 16), (24, 8), (20, 16), (16, 5)])
def test_batched_matches_oracle(bandred, orc, w, b):
    sizes = [33, 160, 17, 1, 0, w, w + 1, w + 2, 97, 300, 64, 250, 129, 511, 18, 75]
    print(f"case batched w={w} b={b} sizes={sizes}", flush=True)
    mats = _batch(sizes, 1)
    pads = [0, 3, 0, 7]
    dev = _upload(mats, pads)
    taus = _run_batched(bandred, dev, sizes, w, b)
    torch.cuda.synchronize()
    _check_against_oracle(orc, mats, dev, taus, w, pads)


def test_batched_largest_order(bandred, orc):
    """n - w = 1024, the largest trailing order the persistent kernel holds,
    next to small matrices; plus n - w = 1025, which goes through the
    single-matrix path inside the same call."""
    w = 16
    sizes = [w + 1024, 40, w + 1025, 200]
    print(f"case batched largest sizes={sizes}", flush=True)
    mats = _batch(sizes, 2)
    dev = _upload(mats)
    taus = _run_batched(bandred, dev, sizes, w, w)
    torch.cuda.synchronize()
    _check_against_oracle(orc, mats, dev, taus, w)
    for k in (0, 2):
        n = sizes[k]
        Ag = dev[k][0].cpu().numpy()
        err = metrics.sy2sb_errors(mats[k], np.tril(Ag), taus[k].cpu().numpy(), w, eig=False)
        assert err["backward"] <= 1e-14 * n and err["orth"] <= 1e-14 * n, err


def test_batched_wide_block_uses_single_path(bandred, orc):
    """b = 32 exceeds the batched kernel's panel width: every matrix is reduced
    by the single-matrix path, with the same result contract."""
    w = b = 32
    sizes = [100, 300, 70]
    mats = _batch(sizes, 3)
    dev = _upload(mats)
    taus = _run_batched(bandred, dev, sizes, w, b)
    torch.cuda.synchronize()
    _check_against_oracle(orc, mats, dev, taus, w)


def test_batched_fp32_update(bandred, orc):
    w = b = 16
    sizes = [64, 96, 500, 1024, 200, 31]
    print(f"case batched fp32 sizes={sizes}", flush=True)
    mats = _batch(sizes, 4)
    dev = _upload(mats)
    taus = _run_batched(bandred, dev, sizes, w, b, prec=1)
    torch.cuda.synchronize()
    for k, A in enumerate(mats):
        n = A.shape[0]
        Ag = dev[k][0].cpu().numpy()[:n, :]
        err = metrics.sy2sb_errors(A, np.tril(Ag), taus[k].cpu().numpy(), w, eig=False)
        assert err["backward"] <= 1e-5 * n, (n, err)
        assert err["orth"] <= 1e-14 * n, (n, err)
        assert err["backward"] > 1e-12, "FP32 form should differ from FP64 beyond rounding"


def test_batched_repeated_and_changed_tables(bandred, orc):
    """Same batch twice (table kept on the device), then a different batch
    (table uploaded again), then the first again."""
    w = 16
    s1, s2 = [90, 40, 260], [300, 21, 77, 150]
    m1, m2 = _batch(s1, 5), _batch(s2, 6)
    for mats, sizes in ((m1, s1), (m1, s1), (m2, s2), (m1, s1)):
        dev = _upload(mats)
        taus = _run_batched(bandred, dev, sizes, w, w)
        torch.cuda.synchronize()
        _check_against_oracle(orc, mats, dev, taus, w)


def test_batched_on_side_stream(bandred, orc):
    w = 16
    sizes = [128, 45, 333]
    mats = _batch(sizes, 7)
    dev = _upload(mats)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        taus = _run_batched(bandred, dev, sizes, w, w, stream=s.cuda_stream)
    s.synchronize()
    _check_against_oracle(orc, mats, dev, taus, w)


def test_batched_graph_replay(bandred, orc):
    """The call captured in a HIP graph (after one eager call with the same
    table) and replayed several times with eager work in between; every replay
    is checked against the oracle."""
    w = 16
    sizes = [200, 64, 96, 31, 400]
    mats = _batch(sizes, 8)
    dev = _upload(mats, poison=False)
    pristine = [A.clone() for A, _ in dev]
    taus = [torch.zeros(max(n - w, 1), dtype=torch.float64, device="cuda") for n in sizes]
    ptrs = [A.data_ptr() for A, _ in dev]
    ldas = [lda for _, lda in dev]

    def call(stream):
        rc = bandred.bandred_sy2sb_batched(len(sizes), sizes, w, w, ptrs, ldas,
                                           [t.data_ptr() for t in taus], 0, stream)
        assert rc == 0, bandred.status_string(rc)

    call(torch.cuda.current_stream().cuda_stream)  # eager: uploads the table
    torch.cuda.synchronize()
    for (A, _), P in zip(dev, pristine):
        A.copy_(P)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            call(s.cuda_stream)
    torch.cuda.synchronize()
    for rep in range(3):
        for (A, _), P in zip(dev, pristine):
            A.copy_(P)
        for t in taus:
            t.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()  # eager work between replays
        for k, A in enumerate(mats):
            n = A.shape[0]
            Ag = dev[k][0].cpu().numpy()[:n, :]
            Ao, to = orc.sy2sb(A, w)
            db, dr, dt = sy_compare(np.tril(Ag), taus[k].cpu().numpy(), np.tril(Ao), to, w)
            tol = 1e-14 * n
            bmax = sy_band_max(np.tril(Ao), w)
            assert db <= tol * bmax and dr <= tol and dt <= tol, (rep, k, db, dr, dt)


def test_batched_banded_input_is_exact(bandred):
    w = 16
    mats = []
    for k, n in enumerate([100, 257, 40]):
        A = inputs.sym_normal(n, 90 + k)
        i = np.arange(n)
        A[np.abs(i[:, None] - i[None, :]) > w] = 0.0
        mats.append(A)
    dev = _upload(mats, poison=False)
    taus = _run_batched(bandred, dev, [A.shape[0] for A in mats], w, w)
    torch.cuda.synchronize()
    for k, A in enumerate(mats):
        n = A.shape[0]
        Ag = dev[k][0].cpu().numpy()[:n, :]
        assert np.all(taus[k].cpu().numpy() == 0.0)
        assert np.array_equal(np.tril(Ag), np.tril(A))
