"""Seeded synthetic inputs shaped like the paper's workloads.

This module is shared by the tests, the benchmark and the smoke check.  It
holds no arithmetic of the band reductions themselves: it only draws random
matrices (numpy PCG64 on the host, or torch's generator on a GPU for the
large known-spectrum cases) and builds them from library primitives
(random normals, a QR factorisation used to draw Haar-distributed orthogonal
factors, matrix products).

The paper's own experiments use random matrices with uniform(0,1) entries,
n up to 10000 and bandwidths 32..256 (Sec. 4).  The workloads here keep those
shapes and add matrices of known spectrum so that eigen/singular values can be
checked:

  ``sym_normal``      symmetric, i.i.d. N(0,1) upper triangle (with the
                      diagonal) mirrored into the lower one.
  ``sym_known``       A = Q diag(lam) Q^T with Haar Q, exactly symmetrised.
  ``ge_normal``       general, i.i.d. N(0,1).
  ``ge_known``        A = U diag(sigma) V^T with Haar U (thin) and Haar V.
  ``uniform_lambda``  lam_i ~ U[-1, 1].
  ``graded_lambda``   lam_i = s_i 10^(-6 i / n), s_i = +-1 with p = 1/2.
  ``logu_sigma``      sigma_i = 10^U(-8, 0), unsorted.
  ``batch_sizes``     sizes drawn uniformly from {64, 96, ..., 1024}.
"""
from __future__ import annotations

import numpy as np

#: Named workloads: (kind, parameters, seed).
WORKLOADS = {
    "sy2sb_n512_w32": dict(kind="sym_known", n=512, w=32, b=32, spectrum="uniform", seed=0),
    "sy2sb_n8192_w64": dict(kind="sym_normal", n=8192, w=64, b=64, seed=1),
    "ge2gb_8192_w64": dict(kind="ge_normal", m=8192, n=8192, w=64, b=64, seed=2),
    "sy2sb_n16384_w128": dict(kind="sym_known", n=16384, w=128, b=128, spectrum="graded", seed=3),
    "ge2gb_24576x12288_w128": dict(kind="ge_known", m=24576, n=12288, w=128, b=128, seed=4),
    "batched_2048_w16": dict(kind="batch", count=2048, w=16, b=16, seed=5),
    # the equal-bandwidth form (Sec. 3.3) of the rectangular workload: lower and
    # upper bandwidth 64, a band as wide as the triangular one of w = 128
    "ge2gb_lu_24576x12288_w64": dict(kind="ge_known", form="lu", m=24576, n=12288, w=64, b=64,
                                     seed=4),
    # look-ahead Variant V1 (2b <= w: the next panel lies in A1, Sec. 2.2)
    "sy2sb_n16384_w256": dict(kind="sym_normal", n=16384, w=256, b=128, seed=6),
}


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_lambda(n: int, g: np.random.Generator) -> np.ndarray:
    return g.uniform(-1.0, 1.0, size=n)


def graded_lambda(n: int, g: np.random.Generator) -> np.ndarray:
    s = np.where(g.random(n) < 0.5, -1.0, 1.0)
    return s * 10.0 ** (-6.0 * np.arange(n) / n)


def logu_sigma(n: int, g: np.random.Generator) -> np.ndarray:
    return 10.0 ** g.uniform(-8.0, 0.0, size=n)


def haar(m: int, n: int, g: np.random.Generator) -> np.ndarray:
    """m x n matrix with orthonormal columns, Haar distributed (QR of a normal
    matrix with the signs of diag(R) folded into Q)."""
    Z = g.standard_normal((m, n))
    Q, R = np.linalg.qr(Z)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d


def sym_normal(n: int, seed: int) -> np.ndarray:
    g = rng(seed)
    Z = g.standard_normal((n, n))
    U = np.triu(Z)
    A = U + np.triu(U, 1).T
    return np.asfortranarray(A)


def sym_known(n: int, lam: np.ndarray, g: np.random.Generator) -> np.ndarray:
    Q = haar(n, n, g)
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    return np.asfortranarray(A)


def ge_normal(m: int, n: int, seed: int) -> np.ndarray:
    return np.asfortranarray(rng(seed).standard_normal((m, n)))


def ge_known(m: int, n: int, sigma: np.ndarray, g: np.random.Generator) -> np.ndarray:
    U = haar(m, n, g)
    V = haar(n, n, g)
    return np.asfortranarray((U * sigma) @ V.T)


def batch_sizes(count: int, seed: int) -> np.ndarray:
    g = rng(seed)
    choices = np.arange(64, 1025, 32)
    return g.choice(choices, size=count)


def batch_matrices(sizes, seed: int):
    """One symmetric N(0,1) matrix per size, all from one seeded stream."""
    g = rng(seed + 1000)
    out = []
    for n in sizes:
        Z = g.standard_normal((int(n), int(n)))
        U = np.triu(Z)
        out.append(np.asfortranarray(U + np.triu(U, 1).T))
    return out


def make(name: str):
    """Build a named workload on the host.  Returns a dict with the matrix
    (or list of matrices) and its known spectrum when there is one."""
    p = dict(WORKLOADS[name])
    kind = p["kind"]
    g = rng(p["seed"])
    if kind == "sym_normal":
        p["A"] = sym_normal(p["n"], p["seed"])
    elif kind == "sym_known":
        lam = uniform_lambda(p["n"], g) if p["spectrum"] == "uniform" else graded_lambda(p["n"], g)
        p["lam"] = lam
        p["A"] = sym_known(p["n"], lam, g)
    elif kind == "ge_normal":
        p["A"] = ge_normal(p["m"], p["n"], p["seed"])
    elif kind == "ge_known":
        sig = logu_sigma(p["n"], g)
        p["sigma"] = sig
        p["A"] = ge_known(p["m"], p["n"], sig, g)
    elif kind == "batch":
        sizes = batch_sizes(p["count"], p["seed"])
        p["sizes"] = sizes
        p["A"] = batch_matrices(sizes, p["seed"])
    return p


def make_on_device(name: str, device="cuda"):
    """Large workloads built directly on a GPU with torch (same recipe as
    ``make``, torch's generator seeded with the workload seed).  Returns a
    dict with a device tensor ``A`` (column-major storage: the tensor is the
    transpose view of a row-major buffer) and the known spectrum if any."""
    import torch

    p = dict(WORKLOADS[name])
    kind = p["kind"]
    gen = torch.Generator(device=device)
    gen.manual_seed(int(p["seed"]))
    f64 = torch.float64

    def haar_t(m, n):
        Z = torch.randn(m, n, generator=gen, device=device, dtype=f64)
        Q, R = torch.linalg.qr(Z)
        d = torch.sign(torch.diagonal(R))
        d[d == 0] = 1.0
        return Q * d

    if kind == "sym_normal":
        n = p["n"]
        Z = torch.randn(n, n, generator=gen, device=device, dtype=f64)
        U = torch.triu(Z)
        A = U + torch.triu(U, 1).T
    elif kind == "sym_known":
        n = p["n"]
        if p["spectrum"] == "uniform":
            lam = torch.rand(n, generator=gen, device=device, dtype=f64) * 2.0 - 1.0
        else:
            s = torch.where(torch.rand(n, generator=gen, device=device, dtype=f64) < 0.5, -1.0, 1.0)
            lam = s * 10.0 ** (-6.0 * torch.arange(n, device=device, dtype=f64) / n)
        Q = haar_t(n, n)
        A = (Q * lam) @ Q.T
        A = 0.5 * (A + A.T)
        p["lam"] = lam.cpu().numpy()
    elif kind == "ge_normal":
        A = torch.randn(p["m"], p["n"], generator=gen, device=device, dtype=f64)
    elif kind == "ge_known":
        m, n = p["m"], p["n"]
        sig = 10.0 ** (torch.rand(n, generator=gen, device=device, dtype=f64) * 8.0 - 8.0)
        U = haar_t(m, n)
        V = haar_t(n, n)
        A = (U * sig) @ V.T
        p["sigma"] = sig.cpu().numpy()
    elif kind == "batch":
        # one flat buffer; matrix k is the column-major n_k x n_k block at
        # offsets[k] (lda = n_k).  Entries i.i.d. N(0,1); the reduction reads
        # the lower triangle only, so the symmetric matrix is its lower
        # triangle mirrored.
        sizes = batch_sizes(p["count"], p["seed"])
        offs = np.concatenate([[0], np.cumsum(sizes.astype(np.int64) ** 2)])
        p["sizes"] = sizes
        p["offsets"] = offs[:-1]
        p["flat"] = torch.randn(int(offs[-1]), generator=gen, device=device, dtype=f64)
        return p
    else:
        raise ValueError(kind)
    # column-major storage: keep a row-major buffer of A^T
    p["A"] = A.T.contiguous().T
    return p
