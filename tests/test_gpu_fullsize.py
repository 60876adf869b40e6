"""GPU parity at the full sizes the bench times, in the bench's launch
configuration (look-ahead, the whole reduction replayed from a HIP graph), on
sampled outputs the oracle can compute: the reflector columns of the first
panels, from an oracle run over only those columns (the first k columns of
the result are final after k steps, since later reflectors act on rows and
columns beyond them).  The sampled columns depend on the trailing updates of
the first iterations, which at these sizes run as chunked launches beside the
look-ahead panel.  Properties that hold at any size (backward error,
orthogonality, by random probes) are checked on the whole result.

Tolerances as in the small parity tests: 1e-14 * n * max|B| for band entries
(max|B| the largest band entry of the sampled part), 1e-14 * n for v and
tau; backward error and orthogonality 1e-14 * n."""
import numpy as np
import pytest
import torch

from paper_1709_00302_amd import inputs, metrics

pytestmark = pytest.mark.gpu


def _graph(run, restore):
    """Eager call (reserves the workspace), then the call captured in a HIP
    graph on a side stream and replayed once on the restored input, as the
    bench times it; returns the replay's output (and the graph, kept alive)."""
    restore()
    run({})  # eager: reserves the workspace
    torch.cuda.synchronize()
    restore()
    torch.cuda.synchronize()
    out = {}
    g = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cs):
        with torch.cuda.graph(g, stream=cs):
            run(out)
    torch.cuda.synchronize()
    restore()
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    return out, g


# the headline workload, the n = 8192, w = b = 64 one, and the Variant V1
# workload (w = 256, b = 128: the next panel lies in A1 and is factored beside
# the whole trailing update)
@pytest.mark.parametrize("name", ["sy2sb_n16384_w128", "sy2sb_n8192_w64", "sy2sb_n16384_w256"])
def test_sy2sb_full_size_graph_replay(bandred, orc, name):
    print(f"case {name}: building the input on the GPU", flush=True)
    p = inputs.make_on_device(name, device="cuda")
    A0, n, w, b = p["A"], p["n"], p["w"], p["b"]
    A = torch.empty_like(A0)
    A.copy_(A0)

    def restore():
        A.copy_(A0)

    def run(out):
        out["tau"] = bandred.sy2sb(A, w, b)

    print(f"case {name}: graph replay", flush=True)
    out, _g = _graph(run, restore)
    tau = out["tau"].clone()
    err = metrics.sy2sb_errors(A0, torch.tril(A), tau, w, eig=False)
    print(f"case {name}: backward {err['backward']:.3e} orth {err.get('orth')}", flush=True)
    assert err["backward"] <= 1e-14 * n, err
    if err.get("orth") is not None:
        assert err["orth"] <= 1e-14 * n, err

    k = 3 * b + 16  # the first three panels and part of the fourth
    print(f"case {name}: oracle on the first {k} reflector columns", flush=True)
    Ah = A0.cpu().numpy()
    Ao, to = orc.sy2sb(Ah, w, ncols=k)
    G = A[:, :k].cpu().numpy()
    O = Ao[:, :k]
    tg = tau[:k].cpu().numpy()
    i = np.arange(n)[:, None]
    j = np.arange(k)[None, :]
    band = (i - j >= 0) & (i - j <= w)
    refl = i - j > w
    bmax = np.abs(O[band]).max()  # largest band entry of the sampled columns
    db = np.abs(G - O)[band].max()
    dv = np.abs(G - O)[refl].max()
    dt = np.abs(tg - to[:k]).max()
    print(f"case {name}: band {db:.3e} v {dv:.3e} tau {dt:.3e}", flush=True)
    tol = 1e-14 * n
    assert db <= tol * bmax and dv <= tol and dt <= tol, (db, dv, dt)


@pytest.mark.parametrize("name", ["ge2gb_24576x12288_w128", "ge2gb_8192_w64"])
def test_ge2gb_full_size_graph_replay(bandred, orc, name):
    print(f"case {name}: building the input on the GPU", flush=True)
    p = inputs.make_on_device(name, device="cuda")
    A0, m, n, w, b = p["A"], p["m"], p["n"], p["w"], p["b"]
    A = torch.empty_like(A0)
    A.copy_(A0)

    def restore():
        A.copy_(A0)

    def run(out):
        out["tau"] = bandred.ge2gb(A, w, b)

    print(f"case {name}: graph replay", flush=True)
    out, _g = _graph(run, restore)
    tq, tp = (t.clone() for t in out["tau"])
    err = metrics.ge2gb_errors(A0, A, tq, tp, w, svd=False)
    print(f"case {name}: backward {err['backward']:.3e}", flush=True)
    assert err["backward"] <= 1e-14 * m, err

    k = 2 * b + 8  # the first two steps' panels and part of the third
    print(f"case {name}: oracle on the first {k} steps", flush=True)
    Ah = A0.cpu().numpy()
    Ao, tqo, tpo = orc.ge2gb(Ah, w, ncols=k)
    tol = 1e-14 * m
    # columns 0..k-1 and rows 0..k-1 are final after k steps
    Gc, Oc = A[:, :k].cpu().numpy(), Ao[:, :k]
    Gr, Or = A[:k, :].cpu().numpy(), Ao[:k, :]
    ic = np.arange(m)[:, None]
    jc = np.arange(k)[None, :]
    band_c = (jc - ic >= 0) & (jc - ic <= w)
    ir = np.arange(k)[:, None]
    jr = np.arange(n)[None, :]
    band_r = (jr - ir >= 0) & (jr - ir <= w)
    db = max(np.abs(Gc - Oc)[band_c].max(), np.abs(Gr - Or)[band_r].max())
    bmax = max(np.abs(Oc[band_c]).max(), np.abs(Or[band_r]).max())
    dl = np.abs(Gc - Oc)[ic > jc].max()          # left reflectors below the diagonal
    dr = np.abs(Gr - Or)[jr - ir > w].max()      # right reflectors right of the band
    dq = np.abs(tq[:k].cpu().numpy() - tqo[:k]).max()
    dp = np.abs(tp[:k].cpu().numpy() - tpo[:k]).max()
    print(f"case {name}: band {db:.3e} left {dl:.3e} right {dr:.3e} tauq {dq:.3e} taup {dp:.3e}",
          flush=True)
    assert db <= tol * bmax, db
    assert max(dl, dr, dq, dp) <= tol, (dl, dr, dq, dp)


def test_batched_full_size_graph_replay(bandred, orc):
    """The batched workload as the bench times it (2048 matrices of orders
    64 .. 1024, w = b = 16, one persistent launch replayed from a HIP graph);
    eight matrices spread over the size range, the smallest and the largest
    among them, compared with the oracle element by element."""
    name = "batched_2048_w16"
    print(f"case {name}: building the input on the GPU", flush=True)
    p = inputs.make_on_device(name, device="cuda")
    w, b = p["w"], p["b"]
    sizes = [int(x) for x in p["sizes"]]
    offs = [int(x) for x in p["offsets"]]
    flat0 = p["flat"]
    flat = flat0.clone()
    count = len(sizes)
    ptrs = [flat.data_ptr() + 8 * o for o in offs]
    tl = [max(n - w, 1) for n in sizes]
    taus = torch.zeros(sum(tl), dtype=torch.float64, device="cuda")
    toffs = np.concatenate([[0], np.cumsum(tl)])[:-1]
    tptrs = [taus.data_ptr() + 8 * int(o) for o in toffs]

    def call(s):
        rc = bandred.bandred_sy2sb_batched(count, sizes, w, b, ptrs, sizes, tptrs, 0, s)
        assert rc == 0, bandred.status_string(rc)

    stream = torch.cuda.current_stream()
    call(stream.cuda_stream)  # eager: uploads the matrix table
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    cs.wait_stream(stream)
    with torch.cuda.stream(cs):
        with torch.cuda.graph(g, stream=cs):
            call(cs.cuda_stream)
    torch.cuda.synchronize()
    flat.copy_(flat0)
    taus.zero_()
    torch.cuda.synchronize()
    print(f"case {name}: graph replay", flush=True)
    g.replay()
    torch.cuda.synchronize()
    order = np.argsort(sizes)
    pick = sorted(set(int(order[i]) for i in np.linspace(0, count - 1, 8).round().astype(int)))
    for k in pick:
        n, o = sizes[k], offs[k]
        A = flat0[o:o + n * n].view(n, n).T.cpu().numpy()  # column-major view
        Ag = flat[o:o + n * n].view(n, n).T.cpu().numpy()
        tg = taus[int(toffs[k]):int(toffs[k]) + max(n - w, 0)].cpu().numpy()
        Ao, to = orc.sy2sb(A, w)
        i = np.arange(n)[:, None]
        j = np.arange(n)[None, :]
        band = (i - j >= 0) & (i - j <= w)
        refl = i - j > w
        db = np.abs(Ag - Ao)[band].max()
        dv = np.abs(Ag - Ao)[refl].max() if n > w + 1 else 0.0
        dt = np.abs(tg - to).max() if n > w else 0.0
        print(f"case {name}: matrix {k} n={n}: band {db:.3e} v {dv:.3e} tau {dt:.3e}", flush=True)
        tol = 1e-14 * n
        bmax = np.abs(Ao[band]).max()
        assert db <= tol * bmax and dv <= tol and dt <= tol, (k, n, db, dv, dt)


@pytest.mark.parametrize("kind,m,n,w", [("sy", 9000, 9000, 128), ("ge", 6144, 6144, 128)])
def test_lookahead_bit_identical_with_chunked_updates(bandred, kind, m, n, w):
    """At these sizes the updates beside the look-ahead panel run as two
    column-chunk launches in the first iterations (and below order 8192 with
    the one-workgroup-per-CU reservation); the serial order runs each update
    as one launch.  Every element is computed by one tile in the same k order
    either way, so the two results are identical bit for bit."""
    print(f"case lookahead chunked {kind} m={m} n={n} w={w}", flush=True)
    g = torch.Generator(device="cuda")
    g.manual_seed(77)
    Z = torch.randn(n, m, generator=g, device="cuda", dtype=torch.float64).T  # column-major m x n
    outs = []
    for la in (True, False):
        A = Z.clone(memory_format=torch.preserve_format)
        if kind == "sy":
            tau = bandred.sy2sb(A, w, w, lookahead=la)
            res = (torch.tril(A).cpu(), tau.cpu())
        else:
            tq, tp = bandred.ge2gb(A, w, w, lookahead=la)
            res = (A.cpu(), tq.cpu(), tp.cpu())
        torch.cuda.synchronize()
        outs.append(res)
    for x, y in zip(*outs):
        assert torch.equal(x, y)
