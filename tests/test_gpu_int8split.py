"""GPU checks of the exact-split form of the trailing update
(BANDRED_INT8_SPLIT_UPDATE), through the C ABI, against the FP64 oracle.

Every trailing-update product takes its operands as per-row (op(A)) and
per-column (op(B)) power-of-two scales times 7 signed base-256 int8 digits,
multiplies the 28 digit pairs of order <= 8 on the int8 matrix cores with
exact int32 sums and combines them in FP64; rank-2k updates scale their two
halves apart.  Per term of the inner dimension the error is below 2^-49 of the
product of the row's and the column's largest entries, under the worst-case
bound of an FP64 dot product; the panels are FP64.  So this form is held to
the FP64 bars of the FP64 parity tests: band entries against the oracle at
1e-14 n max|B|, v and tau at 1e-14 n, backward error 1e-14 n -- and
at full size to the near-FP64 bound 1e-12 n that the FP32-split form misses.
"""
import numpy as np
import pytest
import torch

from paper_1709_00302_amd import inputs, metrics
from tests.gpu_util import ge_band_max, ge_compare, sy_band_max, sy_compare, to_device_colmajor
from tests.test_gpu_ge2gb_lu import lu_compare

pytestmark = pytest.mark.gpu

SY_CASES = [
    # (n, w, b, lda_pad, seed): several 64-tiles, ragged tails, V1 and V2
    # partitions, split-k SYMM (n - w near 2000), symmetric slices over
    # diagonal, lower and mirrored blocks
    (512, 32, 32, 0, 0),
    (257, 20, 8, 3, 2),
    (700, 96, 64, 0, 3),
    (1000, 128, 128, 5, 5),
    (97, 7, 3, 0, 8),
    (2050, 64, 64, 0, 9),
]


@pytest.mark.parametrize("n,w,b,pad,seed", SY_CASES)
def test_sy2sb_int8split_matches_oracle(bandred, orc, n, w, b, pad, seed):
    print(f"case sy2sb int8split n={n} w={w} b={b} pad={pad} seed={seed}", flush=True)
    A = inputs.sym_normal(n, 100 + seed)
    Ain = A.copy()
    Ain[np.triu_indices(n, 1)] = np.nan  # the upper triangle is never read
    Ad, _ = to_device_colmajor(Ain, n + pad)
    tau = bandred.sy2sb(Ad[:n] if pad else Ad, w, b, prec="int8split")
    torch.cuda.synchronize()
    full = Ad.cpu().numpy()
    Ag, tg = full[:n, :], tau.cpu().numpy()
    assert np.isnan(Ag[np.triu_indices(n, 1)]).all(), "upper triangle was written"
    Ao, to = orc.sy2sb(A, w)
    bmax = sy_band_max(np.tril(Ao), w)
    db, dr, dt = sy_compare(np.tril(Ag), tg, np.tril(Ao), to, w)
    tol = 1e-14 * n
    print(f"  band {db / bmax:.2e}  v {dr:.2e}  tau {dt:.2e}  (bar {tol:.1e})", flush=True)
    assert db <= tol * bmax, (db, tol * bmax)
    assert dr <= tol, dr
    assert dt <= tol, dt
    err = metrics.sy2sb_errors(A, np.tril(Ag), tg, w, eig=False)
    assert err["backward"] <= 1e-14 * n, err


def test_sy2sb_int8split_scaled_rows(bandred, orc):
    """Rows and columns of very different magnitudes (a diagonal similarity
    D A D with D from 2^-20 to 2^20): the per-row scales keep the small rows'
    digits, so the result still matches the oracle's."""
    n, w, b = 600, 32, 32
    print(f"case sy2sb int8split scaled n={n} w={w}", flush=True)
    A = inputs.sym_normal(n, 321)
    d = 2.0 ** np.linspace(-20, 20, n)
    A = A * d[:, None] * d[None, :]
    Ad, _ = to_device_colmajor(A, n)
    tau = bandred.sy2sb(Ad, w, b, prec="int8split")
    torch.cuda.synchronize()
    Ag, tg = Ad.cpu().numpy(), tau.cpu().numpy()
    Ao, to = orc.sy2sb(A, w)
    err = metrics.sy2sb_errors(A, np.tril(Ag), tg, w, eig=False)
    erro = metrics.sy2sb_errors(A, np.tril(Ao), to, w, eig=False)
    print(f"  backward {err['backward']:.2e} (oracle {erro['backward']:.2e})", flush=True)
    assert err["backward"] <= 1e-14 * n, err
    assert err["reflector_orth"] <= 1e-14 * n, err


GE_CASES = [
    # (m, n, w, seed)
    (700, 500, 32, 11),
    (1300, 1100, 64, 12),
]


@pytest.mark.parametrize("m,n,w,seed", GE_CASES)
@pytest.mark.parametrize("form", ["ge2gb", "ge2gb_lu"])
def test_ge2gb_int8split_matches_oracle(bandred, orc, m, n, w, seed, form):
    print(f"case {form} int8split {m}x{n} w={w} seed={seed}", flush=True)
    A = inputs.ge_normal(m, n, 300 + seed)
    Ad, _ = to_device_colmajor(A, m)
    fn = bandred.ge2gb if form == "ge2gb" else bandred.ge2gb_lu
    tq, tp = fn(Ad, w, w, prec="int8split")
    torch.cuda.synchronize()
    Ag, tqg, tpg = Ad.cpu().numpy(), tq.cpu().numpy(), tp.cpu().numpy()
    if form == "ge2gb":
        Ao, tqo, tpo = orc.ge2gb(A, w)
        lower = 0
        db, dl, dr, dq, dp = ge_compare(Ag, tqg, tpg, Ao, tqo, tpo, w)
    else:
        Ao, tqo, tpo = orc.ge2gb_lu(A, w)
        lower = w
        db, dl, dr, dq, dp = lu_compare(Ag, tqg, tpg, Ao, tqo, tpo, w)
    tol = 1e-14 * max(m, n)
    bmax = ge_band_max(Ao, w, lower=lower)
    print(f"  band {db / bmax:.2e}  v {max(dl, dr):.2e}  tau {max(dq, dp):.2e}  "
          f"(bar {tol:.1e})", flush=True)
    assert db <= tol * bmax, (db, tol * bmax)
    assert max(dl, dr, dq, dp) <= tol, (dl, dr, dq, dp)
    err = metrics.ge2gb_errors(A, Ag, tqg, tpg, w, svd=False, lower=lower)
    assert err["backward"] <= tol, err


@pytest.mark.parametrize("form", ["ge2gb", "ge2gb_lu"])
def test_ge2gb_int8split_scaled(bandred, orc, form):
    """Graded rows and columns (D1 G D2, D from 2^-20 to 2^20): the rank-2b
    update [X | Vl] [Vr | ZL]^T of the equal-bandwidth form has halves of very
    different scale, each with scales of its own; the backward error stays at
    the FP64 level."""
    m, n, w = 700, 520, 32
    print(f"case {form} int8split scaled {m}x{n} w={w}", flush=True)
    A = inputs.ge_normal(m, n, 322)
    A = A * (2.0 ** np.linspace(-20, 20, m))[:, None] * (2.0 ** np.linspace(20, -20, n))[None, :]
    Ad, _ = to_device_colmajor(A, m)
    fn = bandred.ge2gb if form == "ge2gb" else bandred.ge2gb_lu
    tq, tp = fn(Ad, w, w, prec="int8split")
    torch.cuda.synchronize()
    lower = 0 if form == "ge2gb" else w
    err = metrics.ge2gb_errors(A, Ad.cpu().numpy(), tq.cpu().numpy(), tp.cpu().numpy(), w,
                               svd=False, lower=lower)
    print(f"  backward {err['backward']:.2e}", flush=True)
    assert err["backward"] <= 1e-14 * m, err


@pytest.mark.parametrize("bad", [np.nan, np.inf])
@pytest.mark.parametrize("form", ["sy2sb", "ge2gb"])
def test_int8split_nonfinite_input_propagates(bandred, form, bad):
    """One NaN or Inf in the trailing matrix reaches every result it takes part
    in, as in FP64 arithmetic: a product operand's row or column holding a
    non-finite entry gets no digits but a marker exponent, and every sum it
    meets is NaN.  (Without the marker the entry would turn into finite digits
    and the result would look valid.)  A NaN spreads the same way through
    both forms' products and panels, so the NaN entries of the result sit
    where the FP64 form puts them; an Inf turns into NaN here where FP64 may
    keep an Inf, or a zero after a division by it, so that case checks only
    that the result reports it.  The first panel stays finite."""
    n, w = 300, 32
    m = n if form == "sy2sb" else n + 40
    print(f"case int8split non-finite {form} {m}x{n} w={w} value={bad}", flush=True)
    A = inputs.sym_normal(n, 77) if form == "sy2sb" else inputs.ge_normal(m, n, 78)
    A[n - 2, n - 40] = bad  # lower triangle, beyond the first panel
    masks = {}
    for prec in ("fp64", "int8split"):
        Ad, _ = to_device_colmajor(A, m)
        if form == "sy2sb":
            out = (bandred.sy2sb(Ad, w, w, prec=prec),)
        else:
            out = bandred.ge2gb(Ad, w, w, prec=prec)
        torch.cuda.synchronize()
        Ag = Ad.cpu().numpy()
        if form == "sy2sb":
            Ag = np.tril(Ag)
        masks[prec] = [~np.isfinite(Ag)] + [~np.isfinite(t.cpu().numpy()) for t in out]
    for k, (a, b) in enumerate(zip(masks["fp64"], masks["int8split"])):
        print(f"  output {k}: non-finite fp64 {a.sum()}  int8split {b.sum()}", flush=True)
        if np.isnan(bad):
            assert np.array_equal(a, b), k
    assert masks["fp64"][0].any()
    assert masks["int8split"][0].any()
    assert not masks["int8split"][0][:, :w].any()


@pytest.mark.parametrize("form", ["sy2sb", "ge2gb_lu"])
def test_int8split_graph_replay_matches_eager(bandred, form):
    """The exact-split reduction captured in a HIP graph (after one eager
    call of the same size reserved its digit planes) and replayed three
    times with eager work in between: every replay equals the eager result
    bit for bit (fill kernels, no memset nodes; the row maxima the SYR2K
    records are cleared by a kernel in the graph)."""
    n, w, b = 700, 96, 64
    print(f"case int8split graph {form} n={n} w={w} b={b}", flush=True)
    A = inputs.sym_normal(n, 42) if form == "sy2sb" else inputs.ge_normal(n, n, 43)
    A0, _ = to_device_colmajor(A, n)
    Ad = A0.clone()
    fn = bandred.sy2sb if form == "sy2sb" else bandred.ge2gb_lu
    wb = (w, b) if form == "sy2sb" else (w, w)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        out_e = fn(Ad, *wb, prec="int8split", stream=s)
    torch.cuda.synchronize()
    ref = Ad.clone()
    tref = [x.clone() for x in (out_e if isinstance(out_e, tuple) else (out_e,))]
    Ad.copy_(A0)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            out_g = fn(Ad, *wb, prec="int8split", stream=s)
    torch.cuda.synchronize()
    tg = out_g if isinstance(out_g, tuple) else (out_g,)
    for rep in range(3):
        Ad.copy_(A0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()  # eager work between replays
        assert torch.equal(Ad, ref), rep
        assert all(torch.equal(x, y) for x, y in zip(tg, tref)), rep


def test_sy2sb_int8split_full_size(bandred):
    """The n = 16384, w = b = 128 graded-spectrum workload in the exact-split
    form as the bench times it (look-ahead, eager calls): backward error by
    random probes within the near-FP64 bound 1e-12 n, every reflector
    orthogonal, every tau nonzero."""
    name = "sy2sb_n16384_w128"
    print(f"case {name} int8split: building the input on the GPU", flush=True)
    p = inputs.make_on_device(name, device="cuda")
    A0, n, w, b = p["A"], p["n"], p["w"], p["b"]
    A = A0.clone(memory_format=torch.preserve_format)
    tau = bandred.sy2sb(A, w, b, prec="int8split")
    torch.cuda.synchronize()
    err = metrics.sy2sb_errors(A0, torch.tril(A), tau, w, eig=False)
    print(f"case {name} int8split: {err}", flush=True)
    assert err["backward"] <= 1e-12 * n, err
    assert err["reflector_orth"] <= 1e-14 * n, err
    assert bool(torch.all(tau[: n - w - 1] != 0.0))
