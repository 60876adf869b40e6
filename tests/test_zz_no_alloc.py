"""GPU tests of bandred_sy2sb_noalloc, the SY2SB entry point whose workspace is
a fixed device array (no allocation): it must give what bandred_sy2sb_ex
gives on the same input, call after call, also when a later call is smaller
(the array keeps the previous call's contents), and refuse problems that do
not fit the array before doing any work."""
import numpy as np
import pytest
import torch

from paper_1709_00302_amd import inputs
from tests.gpu_util import sy_compare, sy_band_max, to_device_colmajor

pytestmark = pytest.mark.gpu

UNSUPPORTED = 3  # BANDRED_ERR_UNSUPPORTED


def _run_noalloc(br, Ad, lda, n, w, b, prec=0):
    s = torch.cuda.current_stream()
    tau = torch.full((n - w,), np.nan, dtype=torch.float64, device="cuda")
    rc = br.bandred_sy2sb_noalloc(n, w, b, Ad.data_ptr(), lda, tau.data_ptr(), prec, s.cuda_stream)
    assert rc == 0, br.status_string(rc)
    torch.cuda.synchronize()
    assert br.bandred_status(s.cuda_stream) == 0
    return tau


def _run_ex(br, Ad, lda, n, w, b, lookahead, prec=0):
    s = torch.cuda.current_stream()
    tau = torch.full((n - w,), np.nan, dtype=torch.float64, device="cuda")
    o = br.Opts(1 if lookahead else 0, 0, 0)
    rc = br.bandred_sy2sb_ex(n, w, b, Ad.data_ptr(), lda, tau.data_ptr(), prec, o, s.cuda_stream)
    assert rc == 0, br.status_string(rc)
    torch.cuda.synchronize()
    assert br.bandred_status(s.cuda_stream) == 0
    return tau


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_matches_ex_twice_second_smaller(bandred, orc, prec):
    # the first call spans several 128-wide panels and a ragged last one; the
    # second is smaller with another w and b, so the array holds stale data
    # from the first call wherever the second does not write
    cases = [(2050, 128, 128, 81), (700, 48, 32, 82)]
    for n, w, b, seed in cases:
        print(f"case noalloc n={n} w={w} b={b} prec={prec}", flush=True)
        A = inputs.sym_normal(n, seed)
        A0, lda = to_device_colmajor(A, n + 3)  # padded lda, NaN padding
        An = A0.clone()
        tn = _run_noalloc(bandred, An, lda, n, w, b, prec)
        for la in (0, 1):
            Ae = A0.clone()
            te = _run_ex(bandred, Ae, lda, n, w, b, la, prec)
            # same kernels in the same order (look-ahead keeps the serial order
            # of every product), hence the same bits
            assert torch.equal(torch.tril(An[:n]), torch.tril(Ae[:n])), (n, la)
            assert torch.equal(tn, te), (n, la)
        if prec == 0:
            Ao, to = orc.sy2sb(A, w)
            db, dr, dt = sy_compare(np.tril(An[:n].cpu().numpy()), tn.cpu().numpy(), np.tril(Ao),
                                    to, w)
            tol = 1e-14 * n
            assert db <= tol * sy_band_max(Ao, w) and dr <= tol and dt <= tol, (db, dr, dt)
        # the strict upper triangle and the lda padding are never touched
        up = torch.triu(An[:n], 1)
        assert torch.equal(up, torch.triu(A0[:n], 1))
        assert torch.isnan(An[n:]).all()


def test_noalloc_int8split_matches_ex(bandred):
    """The exact int8 split through the fixed array (its digit planes and the
    row maxima the SYR2K records live there too): the same bits as the
    allocating call, twice, the second call smaller; a problem whose planes
    do not fit is refused."""
    for n, w, b, seed in [(1000, 64, 64, 91), (600, 48, 32, 92)]:
        print(f"case noalloc int8split n={n} w={w} b={b}", flush=True)
        A = inputs.sym_normal(n, seed)
        A0, lda = to_device_colmajor(A, n)
        An = A0.clone()
        tn = _run_noalloc(bandred, An, lda, n, w, b, 3)
        for la in (0, 1):
            Ae = A0.clone()
            te = _run_ex(bandred, Ae, lda, n, w, b, la, 3)
            assert torch.equal(torch.tril(An), torch.tril(Ae)), (n, la)
            assert torch.equal(tn, te), (n, la)
    n, w = 2050, 128
    A0, lda = to_device_colmajor(inputs.sym_normal(n, 93), n)
    tau = torch.zeros(n - w, dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream()
    rc = bandred.bandred_sy2sb_noalloc(n, w, w, A0.data_ptr(), lda, tau.data_ptr(), 3,
                                       s.cuda_stream)
    assert rc == UNSUPPORTED  # fits in FP64 (see above), not with the digit planes

def test_noalloc_rejects_what_does_not_fit(bandred):
    n, w = 4000, 128  # needs about 69 MiB of the 64 MiB array
    A = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    tau = torch.zeros(n - w, dtype=torch.float64, device="cuda")
    rc = bandred.bandred_sy2sb_noalloc(n, w, w, A.data_ptr(), n, tau.data_ptr(), 0,
                                       torch.cuda.current_stream().cuda_stream)
    assert rc == UNSUPPORTED
    torch.cuda.synchronize()
    assert not A.any() and not tau.any()
    # argument errors as in bandred_sy2sb_ex
    assert bandred.bandred_sy2sb_noalloc(n, w, w + 1, A.data_ptr(), n, tau.data_ptr(), 0,
                                         None) == -3
    assert bandred.bandred_sy2sb_noalloc(n, w, w, A.data_ptr(), n, tau.data_ptr(), 5, None) == -7


def test_noalloc_under_capture_without_eager_call(bandred, orc):
    """Recorded into a HIP graph with no earlier eager call (nothing reserved:
    the library's memory is released first); every replay equals the eager
    no-allocation result, with eager work between the replays."""
    n, w = 900, 64
    A = inputs.sym_normal(n, 83)
    A0, lda = to_device_colmajor(A, n)
    Ae = A0.clone()
    te = _run_noalloc(bandred, Ae, lda, n, w, w)
    assert bandred.bandred_release() == 0
    Ad = A0.clone()
    tau = torch.zeros(n - w, dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            rc = bandred.bandred_sy2sb_noalloc(n, w, w, Ad.data_ptr(), lda, tau.data_ptr(), 0,
                                               s.cuda_stream)
    assert rc == 0
    print("case noalloc graph replays", flush=True)
    B = inputs.sym_normal(300, 84)
    for rep in range(3):
        Ad.copy_(A0)
        tau.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(torch.tril(Ad), torch.tril(Ae)), rep
        assert torch.equal(tau, te), rep
        # eager work on the same array between replays
        Bd, _ = to_device_colmajor(B, 300)
        _run_noalloc(bandred, Bd, 300, 300, 16, 16)
