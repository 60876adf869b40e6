"""GPU tests of the autotuner (bandred_tune and b = 0 in the _ex calls): it
measures every candidate b (multiples of 16 up to min(w, 128)), picks the
fastest, then at that b the split between the look-ahead panel and the update
beside it (update_chunks, update_lds_cap); it caches the choice in memory and
in the JSONL file named by BANDRED_TUNE_CACHE, and a reduction called with
b = 0 is the reduction with the tuned b, bit for bit.  The split knobs change
no result bit (every element is computed by one tile in the same k order):
checked at sizes where the update beside the panel is really cut into
several launches."""
import json
import os

import numpy as np
import pytest
import torch

from paper_1709_00302_amd import inputs
from tests.gpu_util import to_device_colmajor

pytestmark = pytest.mark.gpu

UNSUPPORTED = 3


def test_tune_measures_candidates_and_caches(bandred, tmp_path):
    path = str(tmp_path / "tune.jsonl")
    os.environ["BANDRED_TUNE_CACHE"] = path
    try:
        n, w = 1500, 64
        print(f"case tune sy2sb n={n} w={w}", flush=True)
        b, ms = bandred.bandred_tune(0, n, n, w, force=True)
        assert sorted(ms) == [16, 32, 48, 64] and all(t > 0 for t in ms.values()), ms
        assert b == min(ms, key=ms.get)
        b2, ms2 = bandred.bandred_tune(0, n, n, w)  # cached: nothing measured
        assert b2 == b and ms2 == {}
        lines = [json.loads(x) for x in open(path).read().splitlines()]
        assert lines[-1]["kind"] == "sy2sb" and lines[-1]["n"] == n and lines[-1]["b"] == b
        assert sorted(int(k) for k in lines[-1]["ms"]) == [16, 32, 48, 64]
        # the split phase: 4 launch counts x LDS cap on / off, timed at the tuned b
        assert sorted(int(k) for k in lines[-1]["split_ms"]) == [11, 12, 21, 22, 31, 32, 41, 42]
        res = bandred.bandred_tune_result(0, n, n, w)
        assert res == (b, lines[-1]["chunks"], lines[-1]["cap"]), res
        assert 0 <= res[1] <= 4 and 0 <= res[2] <= 2
        if res[1]:  # a kept setting beat the default by more than 1%
            best = min(lines[-1]["split_ms"].values())
            assert lines[-1]["split_ms"][str(10 * res[1] + res[2])] == best
        assert bandred.bandred_tune_result(0, 777, 777, 64) is None  # never tuned
        # the other kinds, and w below 16 (b = w, nothing to measure)
        bg, msg = bandred.bandred_tune(1, 1200, 900, 48, force=True)
        assert bg in (16, 32, 48) and len(msg) == 3
        bl, msl = bandred.bandred_tune(2, 1200, 900, 32, force=True)
        assert bl in (16, 32) and len(msl) == 2
        bs, mss = bandred.bandred_tune(0, 500, 500, 8, force=True)
        assert bs == 8 and mss == {}
    finally:
        del os.environ["BANDRED_TUNE_CACHE"]


def test_b0_is_the_tuned_b(bandred, orc):
    n, w = 1300, 96
    A = inputs.sym_normal(n, 71)
    print(f"case b=0 sy2sb n={n} w={w}", flush=True)
    Ad, _ = to_device_colmajor(A, n)
    tau0 = bandred.sy2sb(Ad, w, 0)  # tunes on first use
    torch.cuda.synchronize()
    b, ms = bandred.bandred_tune(0, n, n, w)
    assert ms == {} and b in (16, 32, 48, 64, 80, 96)
    Ae, _ = to_device_colmajor(A, n)
    taue = bandred.sy2sb(Ae, w, b)
    torch.cuda.synchronize()
    assert torch.equal(torch.tril(Ad), torch.tril(Ae)) and torch.equal(tau0, taue)
    Ao, to = orc.sy2sb(A, w)
    assert np.abs(tau0.cpu().numpy() - to).max() <= 1e-14 * n
    # GE2GB forms
    G = inputs.ge_normal(1100, 800, 72)
    for fn in (bandred.ge2gb, bandred.ge2gb_lu):
        Gd, _ = to_device_colmajor(G)
        tq, tp = fn(Gd, 32, 0)
        torch.cuda.synchronize()
        kind = 1 if fn is bandred.ge2gb else 2
        bt, _ = bandred.bandred_tune(kind, 1100, 800, 32)
        Ge, _ = to_device_colmajor(G)
        tq2, tp2 = fn(Ge, 32, bt)
        torch.cuda.synchronize()
        assert torch.equal(Gd, Ge) and torch.equal(tq, tq2) and torch.equal(tp, tp2)


# the refused call enqueues nothing, so torch warns that the first graph is empty
@pytest.mark.filterwarnings("ignore:The CUDA Graph is empty")
def test_b0_under_capture_needs_a_cached_choice(bandred):
    n, w = 700, 48
    A = inputs.sym_normal(n, 73)
    Ad, lda = to_device_colmajor(A, n)
    tau = torch.zeros(n - w, dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    # untuned shape: refused under capture, nothing enqueued
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            rc = bandred.bandred_sy2sb_ex(n, w, 0, Ad.data_ptr(), lda, tau.data_ptr(), 0, None,
                                          s.cuda_stream)
    assert rc == UNSUPPORTED
    # once tuned (and the workspace reserved by an eager call), it captures
    b, _ = bandred.bandred_tune(0, n, n, w)
    bandred.sy2sb(Ad.clone(), w, b)
    torch.cuda.synchronize()
    g2 = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g2, stream=s):
            rc = bandred.bandred_sy2sb_ex(n, w, 0, Ad.data_ptr(), lda, tau.data_ptr(), 0, None,
                                          s.cuda_stream)
    assert rc == 0
    A0 = Ad.clone()
    g2.replay()
    torch.cuda.synchronize()
    Ae = A0.clone()
    te = bandred.sy2sb(Ae, w, b)
    torch.cuda.synchronize()
    assert torch.equal(torch.tril(Ad), torch.tril(Ae)) and torch.equal(tau, te)


def test_tune_argument_errors(bandred):
    lib = bandred.load()
    import ctypes
    b = ctypes.c_int64(0)
    assert lib.bandred_tune(3, 10, 10, 2, 0, 0, ctypes.byref(b), None, 0) == -1
    assert lib.bandred_tune(1, 10, 11, 2, 0, 0, ctypes.byref(b), None, 0) == -3
    assert lib.bandred_tune(0, 10, 10, 0, 0, 0, ctypes.byref(b), None, 0) == -4
    assert lib.bandred_tune(0, 10, 10, 2, 0, 0, None, None, 0) == -7


@pytest.mark.parametrize("kind,m,n,w", [
    ("sy2sb", 8192, 8192, 64),
    ("ge2gb", 8192, 8192, 64),
    ("ge2gb_lu", 6144, 6144, 64),
])
def test_split_knobs_change_no_bit(bandred, kind, m, n, w):
    """Every update launch count and LDS-cap setting gives the default
    call's result bit for bit (updates beside the panel are cut into up to 4
    launches at these sizes)."""
    print(f"case split knobs {kind} {m}x{n} w={w}", flush=True)
    g = torch.Generator(device="cuda")
    g.manual_seed(91)
    A0 = torch.randn(n, m, dtype=torch.float64, device="cuda", generator=g).T  # column-major
    if kind == "sy2sb":
        A0 = (A0 + A0.T).T.contiguous().T  # symmetric, column-major
    fn = {"sy2sb": bandred.sy2sb, "ge2gb": bandred.ge2gb, "ge2gb_lu": bandred.ge2gb_lu}[kind]

    def run(ch, cap):
        A = A0.clone(memory_format=torch.preserve_format)
        out = fn(A, w, w, update_chunks=ch, update_lds_cap=cap)
        torch.cuda.synchronize()
        return A, out

    Aref, ref = run(0, 0)
    for ch, cap in ((1, 2), (4, 1), (2, 2), (3, 1)):
        A, out = run(ch, cap)
        if kind == "sy2sb":
            same = torch.equal(torch.tril(A), torch.tril(Aref)) and torch.equal(out, ref)
        else:
            same = torch.equal(A, Aref) and all(torch.equal(x, y) for x, y in zip(out, ref))
        assert same, (kind, ch, cap)
