"""Parallel (associative-scan) formulation of Sec. IV, evaluated on the CPU (test infrastructure).

Float64 numpy transcription of the filter elements and operator (Parallel IMKF,
eq. a-k-f and eq. op-filter) and of the smoother elements and operator (Parallel
IMS, eq. parallel-ak-smoothing and eq. op-smoother), with folds that evaluate
prefixes and suffixes either left to right or under an arbitrary bracketing.

Readings (also listed in the design notes):
  * B = 0, so every u-term drops.
  * The element tuple is (F, d, D, eta, J); the 'b_k' of the operator's preamble is d_k.
  * For k = 1 the paper gives F_1 = 0, d_1 = m^f_{1,l}, D_1 = P^f_{1,l}; eta_1 and J_1
    are not given and are taken as 0 (they never reach a filter output, because a_1
    is always the leftmost operand and d_ij, D_ij read only the left operand's F, d, D).
  * The printed smoother covariance S_k = P^f_{k,1} - E_k A P^f_{k,1,l} is taken as
    S_k = P^f_{k,1} - E_k A (P^f_{k,1,l})^T, the form that follows from
    E_k = P^f_{k,1,l} A^T (A P^f_{k,l} A^T + Q)^{-1} with
    P^f_{k,i,j} = Cov(x_{k,i}, x_{k,j} | y_{1:k}); `printed_S=True` gives the printed one.
"""
from __future__ import annotations

import numpy as np

from .srtm_oracle import slow_rate_model, batch_model, imkf, fast_filter_window


# ----------------------------------------------------------------------------- filter
def filter_elements(A, Q, C, R, L, m0, P0, y):
    """Elements a_k = (F_k, d_k, D_k, eta_k, J_k), k = 1..N (Parallel IMKF, eq. a-k-f).

    k > 1:  R_x = M_bar Q~ M_bar^T + R,  K_k = G_bar Q~ M_bar^T R_x^{-1},
            F_k = A_bar - K_k C_bar,  d_k = K_k y_k,  D_k = Q_bar - K_k M_bar Q~ G_bar^T,
            eta_k = C_bar^T R_x^{-1} y_k,  J_k = C_bar^T R_x^{-1} C_bar.
    k = 1:  one IMKF step from (m0, P0): F_1 = 0, d_1 = m^f_{1,l}, D_1 = P^f_{1,l}.
    """
    sr = slow_rate_model(A, Q, C, L)
    Abar, Gbar, Qt, Qbar, Cbar, Mbar = (sr[k] for k in ("Abar", "Gbar", "Qtilde", "Qbar", "Cbar", "Mbar"))
    nx = A.shape[0]
    Rx = Mbar @ Qt @ Mbar.T + R
    Rx_inv = np.linalg.inv(Rx)
    K = Gbar @ Qt @ Mbar.T @ Rx_inv
    F = Abar - K @ Cbar
    D = Qbar - K @ Mbar @ Qt @ Gbar.T
    J = Cbar.T @ Rx_inv @ Cbar
    m1, P1, _ = imkf(A, Q, C, R, L, m0, P0, y[:1])
    elems = [(np.zeros((nx, nx)), m1[0], P1[0], np.zeros(nx), np.zeros((nx, nx)))]
    for k in range(1, y.shape[0]):
        elems.append((F.copy(), K @ y[k], D.copy(), Cbar.T @ Rx_inv @ y[k], J.copy()))
    return elems


def generic_filter_element(A, Q, C, R, L, yk):
    """The k > 1 element of eq. a-k-f for measurement yk (used for any k, including 1)."""
    sr = slow_rate_model(A, Q, C, L)
    Abar, Gbar, Qt, Qbar, Cbar, Mbar = (sr[k] for k in ("Abar", "Gbar", "Qtilde", "Qbar", "Cbar", "Mbar"))
    Rx_inv = np.linalg.inv(Mbar @ Qt @ Mbar.T + R)
    K = Gbar @ Qt @ Mbar.T @ Rx_inv
    return (Abar - K @ Cbar, K @ yk, Qbar - K @ Mbar @ Qt @ Gbar.T,
            Cbar.T @ Rx_inv @ yk, Cbar.T @ Rx_inv @ Cbar)


def filter_op(ai, aj):
    """a_i (x) a_j of eq. op-filter."""
    Fi, di, Di, ei, Ji = ai
    Fj, dj, Dj, ej, Jj = aj
    nx = Fi.shape[0]
    I = np.eye(nx)
    W = np.linalg.inv(I + Di @ Jj)
    Wt = np.linalg.inv(I + Jj @ Di)
    F = Fj @ W @ Fi
    d = Fj @ W @ (di + Di @ ej) + dj
    D = Fj @ W @ Di @ Fj.T + Dj
    e = Fi.T @ Wt @ (ej - Jj @ di) + ei
    J = Fi.T @ Wt @ Jj @ Fi + Ji
    return (F, d, D, e, J)


def filter_identity(nx):
    """Neutral element of eq. op-filter: (I, 0, 0, 0, 0)."""
    return (np.eye(nx), np.zeros(nx), np.zeros((nx, nx)), np.zeros(nx), np.zeros((nx, nx)))


# ----------------------------------------------------------------------------- smoother
def window_filter_blocks(A, Q, C, R, L, m0, P0, y):
    """Per-window filter quantities the smoother elements need (Remark pf-k-1-l):
    m^f_{k,1}, P^f_{k,1}, the cross-covariance P^f_{k,1,l}, and m^f_{k,l}, P^f_{k,l}."""
    nx, N = A.shape[0], y.shape[0]
    m_slow, P_slow, _ = imkf(A, Q, C, R, L, m0, P0, y)
    bm = batch_model(A, Q, C, L)
    out = []
    for k in range(N):
        mp, Pp = (m0, P0) if k == 0 else (m_slow[k - 1], P_slow[k - 1])
        M_f, P_f = fast_filter_window(bm, R, mp, Pp, y[k])
        out.append(dict(mf1=M_f[:nx], Pf1=P_f[:nx, :nx], Pf1L=P_f[:nx, (L - 1) * nx:],
                        mfL=m_slow[k], PfL=P_slow[k]))
    return out


def smoother_elements(A, Q, C, R, L, m0, P0, y, *, printed_S=False):
    """Elements a_k = (E_k, g_k, S_k) of Parallel IMS (eq. parallel-ak-smoothing).

    k < N:  E_k = P^f_{k,1,l} A^T (A P^f_{k,l} A^T + Q)^{-1},
            g_k = m^f_{k,1} - E_k A m^f_{k,l},
            S_k = P^f_{k,1} - E_k A (P^f_{k,1,l})^T   (printed_S: without the transpose);
    k = N:  E_N = 0, g_N = m^f_{N,1}, S_N = P^f_{N,1}.
    """
    nx, N = A.shape[0], y.shape[0]
    blocks = window_filter_blocks(A, Q, C, R, L, m0, P0, y)
    elems = []
    for k, b in enumerate(blocks):
        if k == N - 1:
            elems.append((np.zeros((nx, nx)), b["mf1"], b["Pf1"]))
            continue
        Ppred = A @ b["PfL"] @ A.T + Q
        E = b["Pf1L"] @ A.T @ np.linalg.inv(Ppred)
        g = b["mf1"] - E @ (A @ b["mfL"])
        cross = b["Pf1L"] if printed_S else b["Pf1L"].T
        S = b["Pf1"] - E @ A @ cross
        elems.append((E, g, S))
    return elems


def smoother_op(ai, aj):
    """a_i (x) a_j of eq. op-smoother: E_ij = E_i E_j, g_ij = E_i g_j + g_i, S_ij = E_i S_j E_i^T + S_i."""
    Ei, gi, Si = ai
    Ej, gj, Sj = aj
    return (Ei @ Ej, Ei @ gj + gi, Ei @ Sj @ Ei.T + Si)


# ----------------------------------------------------------------------------- folds
def prefix_fold(elems, op):
    """All prefixes a_1 (x) ... (x) a_k, evaluated left to right."""
    out = [elems[0]]
    for a in elems[1:]:
        out.append(op(out[-1], a))
    return out


def suffix_fold(elems, op):
    """All suffixes a_k (x) ... (x) a_N, evaluated right to left."""
    out = [elems[-1]]
    for a in reversed(elems[:-1]):
        out.append(op(a, out[-1]))
    return out[::-1]


def bracketed_fold(elems, op, rng):
    """a_1 (x) ... (x) a_n under a random binary bracketing (associativity check)."""
    items = list(elems)
    while len(items) > 1:
        j = int(rng.integers(0, len(items) - 1))
        items[j:j + 2] = [op(items[j], items[j + 1])]
    return items[0]
