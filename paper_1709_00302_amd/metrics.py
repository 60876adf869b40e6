"""Accuracy metrics for a finished band reduction (torch, any device, FP64).

These measure a result; they are not part of the reduction.  Given the
input A and the in-place output (band + stored Householder vectors + tau),
they rebuild the orthogonal factors one reflector at a time (H = I - tau v v^T,
v[0] = 1) and report

  backward   ||A - Q B Q^T||_F / ||A||_F          (sy2sb)
             ||A - U B V^T||_F / ||A||_F          (ge2gb)
  orth       ||Q^T Q - I||_F (explicit, small n) or
             max_c |tau_c (v_c^T v_c) / 2 - 1| over non-trivial reflectors
             (each H_c is orthogonal exactly when tau_c = 2 / v_c^T v_c)
  band_trunc ||offband(Q^T A Q)||_F / ||A||_F  (small n only)
  eig_err    max_i |lambda_i(B) - lambda_i| / max |lambda|   (known spectrum)

Above ``explicit_max`` rows the Frobenius norm of E = A - Q B Q^T is
estimated from k Gaussian probes: E[||E X||_F^2] = k ||E||_F^2.
"""
from __future__ import annotations

import math

import torch

f64 = torch.float64


def _t(x, device=None):
    if isinstance(x, torch.Tensor):
        return x.to(dtype=f64, device=device if device is not None else x.device)
    return torch.as_tensor(x, dtype=f64, device=device)


# --------------------------------------------------------------------------
# symmetric band
# --------------------------------------------------------------------------

def sym_band_dense(Aout: torch.Tensor, w: int) -> torch.Tensor:
    """Dense symmetric B from the lower band (0 <= i-j <= w) of Aout."""
    n = Aout.shape[0]
    i = torch.arange(n, device=Aout.device)
    d = i[:, None] - i[None, :]
    L = torch.where((d >= 0) & (d <= w), Aout, torch.zeros((), dtype=f64, device=Aout.device))
    return L + torch.tril(L, -1).T


def sym_band_matvec(Aout: torch.Tensor, w: int, X: torch.Tensor) -> torch.Tensor:
    """B @ X using only the lower band diagonals of Aout."""
    n = Aout.shape[0]
    Y = torch.zeros_like(X)
    for d in range(0, min(w, n - 1) + 1):
        diag = torch.diagonal(Aout, offset=-d)  # B[i+d, i]
        if d == 0:
            Y += diag[:, None] * X
        else:
            Y[d:] += diag[:, None] * X[: n - d]
            Y[: n - d] += diag[:, None] * X[d:]
    return Y


def apply_q_sy(Aout: torch.Tensor, tau: torch.Tensor, w: int, X: torch.Tensor,
               transpose: bool = False) -> torch.Tensor:
    """Q X (or Q^T X) with Q = H_0 H_1 ... H_{n-w-1}; reflector c acts on rows
    c+w .. n-1 with v = [1; Aout[c+w+1:, c]]."""
    X = X.clone()
    nref = tau.shape[0]
    order = range(nref) if transpose else range(nref - 1, -1, -1)
    taus = tau.tolist()
    for c in order:
        t = taus[c]
        if t == 0.0:
            continue
        r = c + w
        v = Aout[r:, c].clone()
        v[0] = 1.0
        X[r:] -= t * torch.outer(v, v @ X[r:])
    return X


def reflector_orth_sy(Aout, tau, w) -> float:
    worst = 0.0
    taus = tau.tolist()
    for c, t in enumerate(taus):
        if t == 0.0:
            continue
        r = c + w
        vv = 1.0 + float(torch.dot(Aout[r + 1:, c], Aout[r + 1:, c]))
        worst = max(worst, abs(t * vv / 2.0 - 1.0))
    return worst


def sy2sb_errors(A, Aout, tau, w: int, lam=None, explicit_max: int = 2048,
                 probes: int = 8, seed: int = 1234, eig: bool = True) -> dict:
    A = _t(A)
    Aout = _t(Aout, A.device)
    tau = _t(tau, A.device)
    n = A.shape[0]
    Afull = torch.tril(A) + torch.tril(A, -1).T
    nA = float(torch.linalg.norm(Afull))
    out = {}
    if n <= explicit_max:
        Q = apply_q_sy(Aout, tau, w, torch.eye(n, dtype=f64, device=A.device))
        B = sym_band_dense(Aout, w)
        out["backward"] = float(torch.linalg.norm(Afull - Q @ B @ Q.T)) / nA
        out["orth"] = float(torch.linalg.norm(Q.T @ Q - torch.eye(n, dtype=f64, device=A.device)))
        C = Q.T @ Afull @ Q
        i = torch.arange(n, device=A.device)
        off = (i[:, None] - i[None, :]).abs() > w
        out["band_trunc"] = float(torch.linalg.norm(C[off])) / nA
        if eig:
            ev = torch.linalg.eigvalsh(B)
    else:
        g = torch.Generator(device=A.device)
        g.manual_seed(seed)
        X = torch.randn(n, probes, generator=g, dtype=f64, device=A.device)
        Y = apply_q_sy(Aout, tau, w, X, transpose=True)
        Y = sym_band_matvec(Aout, w, Y)
        Y = apply_q_sy(Aout, tau, w, Y)
        E = Afull @ X - Y
        out["backward"] = float(torch.linalg.norm(E)) / math.sqrt(probes) / nA
        out["orth"] = None
        out["band_trunc"] = None
        ev = None
        if eig and lam is not None:
            try:
                import numpy as np
                from scipy.linalg import eigvals_banded

                Ah = Aout.cpu().numpy()
                band = np.zeros((w + 1, n))
                for d in range(w + 1):
                    band[d, : n - d] = np.diagonal(Ah, -d)
                ev = torch.as_tensor(np.sort(eigvals_banded(band, lower=True)), dtype=f64)
            except Exception:  # pragma: no cover - scipy missing
                ev = None
    out["reflector_orth"] = reflector_orth_sy(Aout, tau, w)
    # ||B||_F from the band diagonals must equal ||A||_F (orthogonal similarity)
    nb2 = float(torch.sum(torch.diagonal(Aout) ** 2))
    for d in range(1, min(w, n - 1) + 1):
        nb2 += 2.0 * float(torch.sum(torch.diagonal(Aout, -d) ** 2))
    out["fro_rel"] = abs(math.sqrt(nb2) - nA) / nA
    if lam is not None and ev is not None:
        lam_t = torch.sort(_t(lam, ev.device)).values
        ev = torch.sort(ev.to(f64)).values
        out["eig_err"] = float((ev - lam_t).abs().max()) / float(lam_t.abs().max())
    return out


# --------------------------------------------------------------------------
# general -> upper triangular-band
# --------------------------------------------------------------------------

def ge_band_dense(Aout: torch.Tensor, w: int, lower: int = 0) -> torch.Tensor:
    """Dense band B (-lower <= j-i <= w) of Aout: lower = 0 for the upper
    triangular-band form, lower = w for the equal-bandwidth form."""
    m, n = Aout.shape
    i = torch.arange(m, device=Aout.device)[:, None]
    j = torch.arange(n, device=Aout.device)[None, :]
    keep = (j - i >= -lower) & (j - i <= w)
    return torch.where(keep, Aout, torch.zeros((), dtype=f64, device=Aout.device))


def ge_band_matvec(Aout: torch.Tensor, w: int, X: torch.Tensor, lower: int = 0) -> torch.Tensor:
    """B @ X for the m x n band B (-lower <= j-i <= w) stored in Aout."""
    m, n = Aout.shape
    Y = torch.zeros(m, X.shape[1], dtype=f64, device=X.device)
    for d in range(-min(lower, m - 1), min(w, n - 1) + 1):
        diag = torch.diagonal(Aout, offset=d)  # B[i, i+d]
        k = diag.shape[0]
        if d >= 0:
            Y[:k] += diag[:, None] * X[d:d + k]
        else:
            Y[-d:-d + k] += diag[:, None] * X[:k]
    return Y


def ge_band_rmatvec(Aout: torch.Tensor, w: int, X: torch.Tensor, lower: int = 0) -> torch.Tensor:
    """B^T @ X (X has m rows)."""
    m, n = Aout.shape
    Y = torch.zeros(n, X.shape[1], dtype=f64, device=X.device)
    for d in range(-min(lower, m - 1), min(w, n - 1) + 1):
        diag = torch.diagonal(Aout, offset=d)
        k = diag.shape[0]
        if d >= 0:
            Y[d:d + k] += diag[:, None] * X[:k]
        else:
            Y[:k] += diag[:, None] * X[-d:-d + k]
    return Y


def apply_u(Aout, tauq, X, transpose=False, off: int = 0):
    """U X (or U^T X), U = H_0 ... H_{n-1}; left reflector c acts on rows
    c+off .. m-1 with v = [1; Aout[c+off+1:, c]] (off = 0 for the upper
    triangular-band form, off = w for the equal-bandwidth form)."""
    X = X.clone()
    m = Aout.shape[0]
    n = tauq.shape[0]
    taus = tauq.tolist()
    order = range(n) if transpose else range(n - 1, -1, -1)
    for c in order:
        t = taus[c]
        if t == 0.0 or c + off >= m:
            continue
        v = Aout[c + off:, c].clone()
        v[0] = 1.0
        X[c + off:] -= t * torch.outer(v, v @ X[c + off:])
    return X


def apply_v(Aout, taup, w, X, transpose=False):
    """V X (or V^T X), V = G_0 ... G_{n-w-2}; right reflector c acts on
    indices c+w .. n-1 with u = [1; Aout[c, c+w+1:]]."""
    X = X.clone()
    n = taup.shape[0]
    taus = taup.tolist()
    order = range(n) if transpose else range(n - 1, -1, -1)
    for c in order:
        t = taus[c]
        if t == 0.0:
            continue
        c0 = c + w
        u = Aout[c, c0:].clone()
        u[0] = 1.0
        X[c0:] -= t * torch.outer(u, u @ X[c0:])
    return X


def ge2gb_errors(A, Aout, tauq, taup, w: int, sigma=None, explicit_max: int = 2048,
                 probes: int = 8, seed: int = 1234, svd: bool = True, lower: int = 0) -> dict:
    """Errors of an upper triangular-band result (lower = 0) or of an
    equal-bandwidth one (lower = w: left reflectors start w rows down)."""
    A = _t(A)
    Aout = _t(Aout, A.device)
    tauq = _t(tauq, A.device)
    taup = _t(taup, A.device)
    m, n = A.shape
    nA = float(torch.linalg.norm(A))
    out = {}
    sv = None
    if m <= explicit_max:
        U = apply_u(Aout, tauq, torch.eye(m, dtype=f64, device=A.device), off=lower)
        V = apply_v(Aout, taup, w, torch.eye(n, dtype=f64, device=A.device))
        B = ge_band_dense(Aout, w, lower)
        out["backward"] = float(torch.linalg.norm(A - U @ B @ V.T)) / nA
        out["orth"] = max(float(torch.linalg.norm(U.T @ U - torch.eye(m, dtype=f64, device=A.device))),
                          float(torch.linalg.norm(V.T @ V - torch.eye(n, dtype=f64, device=A.device))))
        C = U.T @ A @ V
        i = torch.arange(m, device=A.device)[:, None]
        j = torch.arange(n, device=A.device)[None, :]
        off = ~((j - i >= -lower) & (j - i <= w))
        out["band_trunc"] = float(torch.linalg.norm(C[off])) / nA
        if svd:
            sv = torch.linalg.svdvals(B)
    else:
        g = torch.Generator(device=A.device)
        g.manual_seed(seed)
        X = torch.randn(n, probes, generator=g, dtype=f64, device=A.device)
        Y = apply_v(Aout, taup, w, X, transpose=True)
        Y = ge_band_matvec(Aout, w, Y, lower)
        Y = apply_u(Aout, tauq, Y, off=lower)
        E = A @ X - Y
        out["backward"] = float(torch.linalg.norm(E)) / math.sqrt(probes) / nA
        out["orth"] = None
        out["band_trunc"] = None
    if sigma is not None and sv is not None:
        s_ref = torch.sort(_t(sigma, sv.device), descending=True).values
        sv = torch.sort(sv, descending=True).values
        out["sv_err"] = float((sv - s_ref).abs().max()) / float(s_ref.abs().max())
    return out
