"""Conditional value functions and their associative combination (numpy, FP64).

TEST INFRASTRUCTURE ONLY.  Written from Sec. IV-A ("Efficiently solving
(primal_update) via associative scans") and Sec. IV-B of the paper.

A conditional value function (CVF, eq. (CVF)) from stage i to stage j is the
tuple e = (P, p, A, C, b) standing for
    V(x_i, x_j) = max_eta 1/2 x_i^T P x_i + p^T x_i - 1/2 eta^T C eta
                          - eta^T (x_j - A x_i - b).
``combine(e_ik, e_kj)`` returns e_ij by the combination rules
eq. (combination_rules), read as follows where the printed text is garbled:
  * the p-rule adds P_kj b_ik:  p_ij = Ups (p_kj + P_kj b_ik) + p_ik  (the
    printed minus sign does not reproduce the Riccati p_i; a pin test shows it);
  * Ups = A_ik^T (I + P_kj C_ik)^{-1},  Psi = A_kj (I + C_ik P_kj)^{-1}.
Element initialisation follows eq. (assoc_init) with the cross term
S_hat = S + rho D^T C.  The reverse scan's suffix s_i = e_i (x) ... (x) e_N
carries the Riccati terms P_i = P(s_i), p_i = p(s_i).

The forward "conditional optimal trajectory" (eq. (CVF_nominal) /
eq. (nom_recovery)) composes affine maps x -> Abar x + bbar.  Read with the
composition order that applies the earlier map first:
    Abar_ij = Abar_kj Abar_ik,  bbar_ij = Abar_kj bbar_ik + bbar_kj,
and the first element carrying the initial state through the closed loop:
    Abar_01 = 0,  bbar_01 = (A_0 + B_0 K_0) x_0 + B_0 k_0 + b_0.

The SLS scan (eq. (CVF_robust), eq. (robust_combin)) uses the matrix part of
the same rule on (P, A, D); its element init reads
    A~ = A - B Qu^{-1} Qux,  D~ = B Qu^{-1} B^T,  P~ = Qx - Qxu Qu^{-1} Qux,
with terminal element (Qx_N, 0, 0).
"""
from __future__ import annotations

import numpy as np


def identity(nx):
    """Identity element of the combination: (0, 0, I, 0, 0)."""
    return (np.zeros((nx, nx)), np.zeros(nx), np.eye(nx), np.zeros((nx, nx)), np.zeros(nx))


def combine(e_ik, e_kj, p_sign=+1.0):
    """e_ij = e_ik (x) e_kj by eq. (combination_rules).  ``p_sign`` = +1 is the
    reading used throughout; -1 reproduces the printed sign (tests only)."""
    P1, p1, A1, C1, b1 = e_ik
    P2, p2, A2, C2, b2 = e_kj
    n = P1.shape[0]
    I = np.eye(n)
    Ups = A1.T @ np.linalg.inv(I + P2 @ C1)
    Psi = A2 @ np.linalg.inv(I + C1 @ P2)
    P = Ups @ P2 @ A1 + P1
    p = Ups @ (p2 + p_sign * (P2 @ b1)) + p1
    A = Psi @ A1
    C = Psi @ C1 @ A2.T + C2
    b = Psi @ (b1 - C1 @ p2) + b2
    return (P, p, A, C, b)


def augmented(prob, rho, y, z):
    """Augmented costs eq. (augmented_matrices) and linear terms
    eq. (augmented_linear) for scaled duals y and split variable z."""
    N, nc = prob.N, prob.nc
    w = y - z
    Qh = prob.Q.copy(); qh = prob.q.copy()
    Rh = np.empty_like(prob.R); Sh = np.empty_like(prob.S); rh = np.empty_like(prob.r)
    for k in range(N):
        Ck, Dk, wk = prob.C[k], prob.D[k], w[k * nc:(k + 1) * nc]
        Qh[k] = prob.Q[k] + rho * Ck.T @ Ck
        Rh[k] = prob.R[k] + rho * Dk.T @ Dk
        Sh[k] = prob.S[k] + rho * Dk.T @ Ck
        qh[k] = prob.q[k] + rho * Ck.T @ wk
        rh[k] = prob.r[k] + rho * Dk.T @ wk
    Qh[N] = prob.Q[N] + rho * prob.CN.T @ prob.CN
    qh[N] = prob.q[N] + rho * prob.CN.T @ w[N * nc:]
    return Qh, Rh, Sh, qh, rh


def elements(prob, Qh, Rh, Sh, qh, rh):
    """Scan elements e_{i,i+1}, i = 0..N-1, and the terminal e_{N,N+1}, eq. (assoc_init)."""
    N, nx = prob.N, prob.nx
    out = []
    for i in range(N):
        Ri = np.linalg.inv(Rh[i])
        Om = Ri @ rh[i]
        B = prob.B[i]
        out.append((Qh[i] - Sh[i].T @ Ri @ Sh[i], qh[i] - Sh[i].T @ Om,
                    prob.A[i] - B @ Ri @ Sh[i], B @ Ri @ B.T, prob.b[i] - B @ Om))
    out.append((Qh[N].copy(), qh[N].copy(), np.zeros((nx, nx)), np.zeros((nx, nx)), np.zeros(nx)))
    return out


def suffix_scan(elems, op=combine):
    """All suffixes s_i = e_i (x) ... (x) e_last, sequentially from the right."""
    out = [None] * len(elems)
    acc = elems[-1]
    out[-1] = acc
    for i in range(len(elems) - 2, -1, -1):
        acc = op(elems[i], acc)
        out[i] = acc
    return out


def tree_suffix_scan(elems, op=combine):
    """Suffixes by the up-sweep / down-sweep tree of App. A (reversed), giving
    the same values as ``suffix_scan`` in a different association order."""
    n = len(elems)
    size = 1
    while size < n:
        size *= 2
    nx = elems[0][0].shape[0]
    e = identity(nx)
    # reverse the sequence so the suffix scan becomes a prefix scan of the
    # reversed operator a (x)' b = b (x) a
    rev = [elems[n - 1 - i] for i in range(n)] + [e] * (size - n)
    rop = lambda a, b: op(b, a)  # noqa: E731
    tree = [rev]
    while len(tree[-1]) > 1:
        lv = tree[-1]
        tree.append([rop(lv[2 * i], lv[2 * i + 1]) for i in range(len(lv) // 2)])
    pref = [e]
    for d in range(len(tree) - 2, -1, -1):
        lv = tree[d]
        nxt = []
        for i, pp in enumerate(pref):
            nxt.append(pp)                       # left child keeps the prefix
            nxt.append(rop(pp, lv[2 * i]))       # right child adds the left value
        pref = nxt
    incl = [rop(pref[i], rev[i]) for i in range(n)]
    return [incl[n - 1 - i] for i in range(n)]


def gains(prob, Rh, Sh, rh, P, p):
    """K_i, k_i, Gamma_i of eq. (controller_cache) from the scan's P_i, p_i."""
    N = prob.N
    K = []; k = []; Gam = []
    for i in range(N):
        A, B, b = prob.A[i], prob.B[i], prob.b[i]
        G = np.linalg.inv(Rh[i] + B.T @ P[i + 1] @ B)
        K.append(-G @ (Sh[i] + B.T @ P[i + 1] @ A))
        k.append(-G @ (B.T @ (p[i + 1] + P[i + 1] @ b) + rh[i]))
        Gam.append(G)
    return np.array(K), np.array(k), np.array(Gam)


def fwd_combine(h_ik, h_kj):
    """Compose affine maps: first h_ik, then h_kj."""
    A1, b1 = h_ik
    A2, b2 = h_kj
    return (A2 @ A1, A2 @ b1 + b2)


def forward_scan(prob, K, k, x0):
    """States x_0..x_N by the prefix composition of eq. (nom_recovery)."""
    N, nx = prob.N, prob.nx
    els = []
    for i in range(N):
        Ab = prob.A[i] + prob.B[i] @ K[i]
        bb = prob.B[i] @ k[i] + prob.b[i]
        if i == 0:
            els.append((np.zeros((nx, nx)), Ab @ x0 + bb))
        else:
            els.append((Ab, bb))
    X = [x0.copy()]
    acc = None
    for i in range(N):
        acc = els[i] if acc is None else fwd_combine(acc, els[i])
        X.append(acc[1].copy())
    X = np.array(X)
    U = np.array([K[i] @ X[i] + k[i] for i in range(N)])
    return X, U


def lqr_by_scan(prob, rho, y, z, tree=False):
    """The ADMM x-update solved by the reverse and forward scans."""
    Qh, Rh, Sh, qh, rh = augmented(prob, rho, y, z)
    els = elements(prob, Qh, Rh, Sh, qh, rh)
    suf = tree_suffix_scan(els) if tree else suffix_scan(els)
    P = np.array([s[0] for s in suf]); p = np.array([s[1] for s in suf])
    K, k, _ = gains(prob, Rh, Sh, rh, P, p)
    X, U = forward_scan(prob, K, k, prob.x0)
    return dict(P=P, p=p, K=K, k=k, X=X, U=U)


def robust_elements(prob, tau_col, j, Qbar, Rbar, QbarN):
    """SLS scan elements for disturbance column j over stages j+1..N-1 and the
    terminal element, from the tau-weighted costs eq. (sls_cost_matrices_tau).
    ``tau_col[k]`` is tau_{k,j} (length nc for k < N, nf for k = N)."""
    N, nx = prob.N, prob.nx
    out = []
    for k in range(j + 1, N):
        T = np.diag(tau_col[k])
        C, D, A, B = prob.C[k], prob.D[k], prob.A[k], prob.B[k]
        Qx = C.T @ T @ C + Qbar; Qu = D.T @ T @ D + Rbar; Qux = D.T @ T @ C
        Qi = np.linalg.inv(Qu)
        out.append((Qx - Qux.T @ Qi @ Qux, np.zeros(nx), A - B @ Qi @ Qux, B @ Qi @ B.T,
                    np.zeros(nx)))
    TN = np.diag(tau_col[N]) if prob.nf else np.zeros((0, 0))
    out.append((prob.CN.T @ TN @ prob.CN + QbarN, np.zeros(nx), np.zeros((nx, nx)),
                np.zeros((nx, nx)), np.zeros(nx)))
    return out
