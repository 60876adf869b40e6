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


# ---------------------------------------------------------------------------
# CholeskyQR2 + Householder reconstruction (the default panel method of the
# GPU drivers), with the drivers' acceptance thresholds
# ---------------------------------------------------------------------------

CHOL1_REL = 1e-10  # first Cholesky: pivot > CHOL1_REL * original diagonal
CHOL2_REL = 1e-6   # second Cholesky: the same test


def _chol_checked(G, rel):
    """Upper Cholesky factor of G, right-looking, and whether every pivot
    (the Schur-complement diagonal) exceeded rel times the original diagonal.
    A failing pivot is replaced by 1 and the factorisation continues, as in
    the kernel."""
    G = np.array(G, dtype=np.float64, copy=True)
    b = G.shape[0]
    d0 = np.diag(G).copy()
    R = np.zeros_like(G)
    ok = True
    worst = np.inf
    for k in range(b):
        d = G[k, k]
        worst = min(worst, d / d0[k] if d0[k] > 0 else 0.0)
        ok = ok and d > rel * d0[k]
        if d <= 0.0:
            d = 1.0
        r = np.sqrt(d)
        R[k, k] = r
        R[k, k + 1:] = G[k, k + 1:] / r
        G[k + 1:, k + 1:] -= np.outer(R[k, k + 1:], R[k, k + 1:])
    return R, ok, worst


def cholqr2_recon(P):
    """Factor the m x b panel P (m > b) as the drivers do by default.

    Returns a dict with ``branch`` ("cholqr2" when both Cholesky factorisations
    pass their pivot tests, else "fallback-chol1" / "fallback-chol2": the
    drivers then factor the panel column by column), the smallest pivot
    ratios, and for the accepted branch V (explicit, unit lower trapezoidal),
    tau and beta (the diagonal of the Householder R).
    Reconstruction (Ballard et al.): LU without pivoting of Q(0:b,:) - S with
    S_k = -sign of the current pivot gives V = [L; Q(b:m,:) U^-1],
    T = -U S L^-T, R_householder = S R."""
    m, b = P.shape
    R1, ok1, w1 = _chol_checked(P.T @ P, CHOL1_REL)
    out = {"pivot_ratio1": w1}
    if not ok1:
        out["branch"] = "fallback-chol1"
        return out
    Q1 = np.linalg.solve(R1.T, P.T).T
    R2, ok2, w2 = _chol_checked(Q1.T @ Q1, CHOL2_REL)
    out["pivot_ratio2"] = w2
    if not ok2:
        out["branch"] = "fallback-chol2"
        return out
    Q = np.linalg.solve(R2.T, Q1.T).T
    R = R2 @ R1
    W = Q[:b, :].copy()
    L = np.eye(b)
    U = np.zeros((b, b))
    S = np.zeros(b)
    for k in range(b):
        S[k] = -1.0 if W[k, k] >= 0.0 else 1.0
        W[k, k] -= S[k]
        U[k, k:] = W[k, k:]
        L[k + 1:, k] = W[k + 1:, k] / W[k, k]
        W[k + 1:, k + 1:] -= np.outer(L[k + 1:, k], U[k, k + 1:])
    V = np.vstack([L, np.linalg.solve(U.T, Q[b:, :].T).T])
    T = -U @ np.diag(S) @ np.linalg.inv(L).T
    out.update(branch="cholqr2", V=V, tau=np.diag(T).copy(), beta=S * np.diag(R))
    return out


def conditioned_panel(m, b, kappa, kind, seed):
    """An m x b panel of condition number kappa.
      clustered: singular values 1 except the last four, 1/kappa;
      graded:    singular values kappa^(-i/(b-1));
      scaled:    a well-conditioned N(0,1) panel times diag(kappa^(-i/(b-1)))
                 (badly scaled columns; every column's angle to the span of
                 the others stays O(1), so no single pivot ratio is small)."""
    g = np.random.Generator(np.random.PCG64(seed))
    if kind == "scaled":
        return g.standard_normal((m, b)) * kappa ** (-np.arange(b) / (b - 1))
    Uq, _ = np.linalg.qr(g.standard_normal((m, b)))
    Vq, _ = np.linalg.qr(g.standard_normal((b, b)))
    if kind == "clustered":
        s = np.ones(b)
        s[-4:] = 1.0 / kappa
    else:
        s = kappa ** (-np.arange(b) / (b - 1))
    return (Uq * s) @ Vq.T


def sym_with_first_panel(P, w, seed):
    """Symmetric (m + w) x (m + w) matrix, N(0,1) elsewhere, whose first
    panel A[w:, :b] is P (so the reduction's first b reflectors are those of
    the Householder QR of P)."""
    m, b = P.shape
    n = m + w
    g = np.random.Generator(np.random.PCG64(seed))
    Z = np.triu(g.standard_normal((n, n)))
    A = Z + np.triu(Z, 1).T
    A[w:, :b] = P
    A[:b, w:] = P.T
    return np.asfortranarray(A)
