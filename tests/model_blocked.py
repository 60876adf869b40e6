"""Numpy model of the blocked drivers run by the GPU library.

Test infrastructure: it replays, on the CPU and in the same order, the steps
the HIP drivers take (panel QR in the one-reduction-per-column form used by
the panel kernel, S = V^T V and T by the LAPACK-style recurrence, the A1 left
update, P = A2 V, X = P T, M = T^T V^T X, W = X - V M / 2, SYR2K split into
the next panel's columns and the rest; GE2GB left/right GEMM pairs), so the
index logic can be checked against the oracle without a GPU.  It shares no
code with the oracle.
"""
import numpy as np


def panel_qr(P):
    """Householder QR of P (m x nb) in place, one 'reduction' per column:
    s_k = sum_{r>i} a_ri a_rk, pivot row a_i., then the update.  Returns
    (V explicit, tau)."""
    m, nb = P.shape
    tau = np.zeros(nb)
    for i in range(nb):
        s = P[i + 1:, i] @ P[i + 1:, i:]      # s_k, k >= i
        piv = P[i, i:].copy()
        alpha, sig2 = piv[0], s[0]
        if sig2 == 0.0:
            continue
        nrm = np.sqrt(alpha * alpha + sig2)
        beta = nrm if alpha < 0 else -nrm
        t = (beta - alpha) / beta
        d = alpha - beta
        z = piv[1:] + s[1:] / d
        P[i + 1:, i] /= d
        P[i + 1:, i + 1:] -= np.outer(P[i + 1:, i], t * z)
        P[i, i + 1:] -= t * z
        P[i, i] = beta
        tau[i] = t
    V = np.tril(P, -1)[:, :nb].copy()
    V[np.arange(nb), np.arange(nb)] = 1.0
    return V, tau


def larft(S, tau):
    nb = len(tau)
    T = np.zeros((nb, nb))
    for i in range(nb):
        T[:i, i] = -tau[i] * (T[:i, :i] @ S[:i, i])
        T[i, i] = tau[i]
    return T


def sy2sb_blocked(A, w, b):
    """A: full symmetric (lower triangle used). Returns (lower Aout, tau)."""
    n = A.shape[0]
    A = np.tril(np.array(A, dtype=np.float64))
    tau = np.zeros(max(n - w, 0))
    nref = n - w - 1
    c = 0
    while c < nref:
        pb = min(b, nref - c)
        r = c + w
        j = n - r
        V, t = panel_qr(A[r:, c:c + pb])  # in place on the view
        tau[c:c + pb] = t
        T = larft(V.T @ V, t)
        if w - pb > 0:
            A1 = A[r:, c + pb:r]
            A1 -= V @ (T.T @ (V.T @ A1))
        A2s = np.tril(A[r:, r:]) + np.tril(A[r:, r:], -1).T  # symmetric view of lower storage
        X = (A2s @ V) @ T
        M = T.T @ (V.T @ X)
        W = X - 0.5 * V @ M
        U = W @ V.T + V @ W.T
        cn = c + b
        pbn = min(b, nref - cn) if cn < nref else 0
        a2L = max(0, cn + pbn - r) if cn < nref else 0
        L = np.tril(np.ones((j, j), dtype=bool))
        colmask = np.zeros((j, j), dtype=bool)
        colmask[:, :a2L] = True
        A2 = A[r:, r:]
        A2[L & colmask] -= U[L & colmask]
        A2[L & ~colmask] -= U[L & ~colmask]
        c += b
    return A, tau


def ge2gb_blocked(A, w, b):
    A = np.array(A, dtype=np.float64, order="F", copy=True)
    m, n = A.shape
    tauq = np.zeros(n)
    taup = np.zeros(n)
    c = 0
    while c < n:
        pb = min(b, n - c)
        Vq, tq = panel_qr(A[c:, c:c + pb])
        tauq[c:c + pb] = tq
        Tq = larft(Vq.T @ Vq, tq)
        if n - c - pb > 0:
            E = A[c:, c + pb:]
            E -= Vq @ (Tq.T @ (Vq.T @ E))
        pr = max(0, min(pb, n - w - 1 - c))
        if pr > 0:
            c0 = c + w
            Ct = A[c:c + pr, c0:].T.copy()
            U, tp = panel_qr(Ct)
            A[c:c + pr, c0:] = Ct.T
            taup[c:c + pr] = tp
            Tp = larft(U.T @ U, tp)
            D = A[c + pr:, c0:]
            D -= ((D @ U) @ Tp) @ U.T
        c += b
    return A, tauq, taup
