"""GPU tests of the runtime around the reductions: device-side status
reporting of the asynchronous entry points, and the lifetime of the memory
that a captured HIP graph refers to.

The timeout test forces the error path from the host: it shortens the bound
of the panel kernel's own inter-workgroup wait to one microsecond, so that
the first workgroup to wait gives up, raises the abort flag and every other
kernel of the call exits normally.  Nothing faults or hangs.
"""
import numpy as np
import pytest
import torch

from paper_1709_00302_amd import inputs
from tests.gpu_util import sy_compare, to_device_colmajor

pytestmark = pytest.mark.gpu

TIMEOUT = 4  # BANDRED_ERR_TIMEOUT


def test_timeout_is_reported_by_status(bandred, orc):
    n, w = 3000, 32
    A = inputs.sym_normal(n, 61)
    Ad, lda = to_device_colmajor(A, n)
    print("case timeout: per-column panels with a 1 us wait bound", flush=True)
    assert bandred.bandred_set_wait_limit_us(1.0) == 0
    try:
        # the per-column panel kernel spreads the 2968-row panel over 24
        # workgroups and meets at one grid barrier per column
        with pytest.raises(bandred.BandredError) as ei:
            bandred.sy2sb(Ad, w, w, panel_method=1)
        assert ei.value.code == TIMEOUT
        # the raw status query reports the same word
        assert bandred.bandred_status(torch.cuda.current_stream().cuda_stream) == TIMEOUT
    finally:
        assert bandred.bandred_set_wait_limit_us(0.0) == 0
    # with the default bound the same call succeeds and clears the status
    Ad, lda = to_device_colmajor(A, n)
    tau = bandred.sy2sb(Ad, w, w, panel_method=1)
    torch.cuda.synchronize()
    assert bandred.bandred_status(None) == 0
    Ao, to = orc.sy2sb(A, w)
    db, dr, dt = sy_compare(np.tril(Ad.cpu().numpy()), tau.cpu().numpy(), np.tril(Ao), to, w)
    assert max(dr, dt) <= 1e-14 * n and db <= 1e-14 * n * np.abs(np.tril(Ao)).max()


def test_ge2gb_timeout_is_reported(bandred):
    """The same error path through the GE2GB driver (row panels too)."""
    m, n, w = 2500, 600, 32
    A = inputs.ge_normal(m, n, 62)
    Ad, lda = to_device_colmajor(A, m)
    assert bandred.bandred_set_wait_limit_us(1.0) == 0
    try:
        tq, tp = bandred.ge2gb(Ad, w, w, panel_method=1, check=False)
        assert bandred.bandred_status(torch.cuda.current_stream().cuda_stream) == TIMEOUT
    finally:
        assert bandred.bandred_set_wait_limit_us(0.0) == 0
    Ad, lda = to_device_colmajor(A, m)
    bandred.ge2gb(Ad, w, w, panel_method=1)  # raises unless the status is clear
    assert bandred.bandred_status(None) == 0


def test_graph_replay_after_workspace_growth(bandred, orc):
    """A graph captured with a small workspace stays valid after a later eager
    call needs a larger one (the old workspace is kept, not freed)."""
    n, w = 300, 16
    A = inputs.sym_normal(n, 63)
    A0, _ = to_device_colmajor(A, n)
    Ad = A0.clone()
    assert bandred.bandred_release() == 0
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        tau_e = bandred.sy2sb(Ad, w, w, stream=s)  # eager: reserves a small workspace
    torch.cuda.synchronize()
    ref, tref = Ad.clone(), tau_e.clone()
    Ad.copy_(A0)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            tau_g = bandred.sy2sb(Ad, w, w, stream=s)
    torch.cuda.synchronize()
    # a larger eager call grows the workspace
    B = inputs.sym_normal(1500, 64)
    Bd, _ = to_device_colmajor(B, 1500)
    bandred.sy2sb(Bd, 64, 64)
    torch.cuda.synchronize()
    print("case graph replay after workspace growth", flush=True)
    for rep in range(2):
        Ad.copy_(A0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(Ad, ref), rep
        assert torch.equal(tau_g, tref), rep
    Ao, to = orc.sy2sb(A, w)
    db, dr, dt = sy_compare(np.tril(Ad.cpu().numpy()), tau_g.cpu().numpy(), np.tril(Ao), to, w)
    assert max(dr, dt) <= 1e-14 * n and db <= 1e-14 * n * np.abs(np.tril(Ao)).max()


def test_batched_graph_survives_other_tables(bandred, orc):
    """A captured batched call keeps its own device table: eager calls with
    other tables (and a larger scratch) afterwards do not change what the
    graph reduces."""
    w = b = 16
    sizes_a = [80, 150, 33, 200]
    sizes_b = [40 + k for k in range(260)]  # more matrices: a larger scratch too
    mats_a = [inputs.sym_normal(n, 700 + k) for k, n in enumerate(sizes_a)]
    dev0 = [to_device_colmajor(M, M.shape[0])[0] for M in mats_a]
    dev = [d.clone() for d in dev0]
    taus = [torch.zeros(n - w, dtype=torch.float64, device="cuda") for n in sizes_a]
    assert bandred.bandred_release() == 0
    s = torch.cuda.Stream()

    def call(stream):
        rc = bandred.bandred_sy2sb_batched(len(sizes_a), sizes_a, w, b, [d.data_ptr() for d in dev],
                                           sizes_a, [t.data_ptr() for t in taus], 0,
                                           stream.cuda_stream)
        assert rc == 0, bandred.status_string(rc)

    with torch.cuda.stream(s):
        call(s)  # eager: uploads table A
    torch.cuda.synchronize()
    for d, d0 in zip(dev, dev0):
        d.copy_(d0)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            call(s)
    torch.cuda.synchronize()
    # eager calls with a different table
    mats_b = [inputs.sym_normal(n, 900 + k) for k, n in enumerate(sizes_b)]
    devb = [to_device_colmajor(M, M.shape[0])[0] for M in mats_b]
    bandred.sy2sb_batched(devb, w, b)
    torch.cuda.synchronize()
    for d, d0 in zip(dev, dev0):
        d.copy_(d0)
    for t in taus:
        t.zero_()
    torch.cuda.synchronize()
    print("case batched graph replay after another table", flush=True)
    g.replay()
    torch.cuda.synchronize()
    for k, (M, n) in enumerate(zip(mats_a, sizes_a)):
        Ao, to = orc.sy2sb(M, w)
        db, dr, dt = sy_compare(np.tril(dev[k].cpu().numpy()), taus[k].cpu().numpy(), np.tril(Ao),
                                to, w)
        tol = 1e-14 * n
        assert db <= tol * np.abs(np.tril(Ao)).max() and dr <= tol and dt <= tol, (k, db, dr, dt)
