"""Sequential float64 reference for the SRTM filter and smoother (test infrastructure).

Written from Yaghoobi & Sarkka, arXiv 2410.00627, Sec. III, in the paper's order
and notation, with B = 0 (no inputs). Every function is a plain transcription of
the stated equations using dense matrices; nothing is blocked, fused or reduced.

Readings taken where the paper is silent (each also listed in the design notes):
  * Q~ = E[w_bar w_bar^T] = I_L (x) Q, because the w_t are iid N(0, Q) (eq. prediction).
  * Measurement window k holds x_{k,1..l}; x_{0,l} = x_0 is not measured (Sec. III).
  * "Fast-rate filter" means p(x_{k,i} | y_{1:k}), i.e. it includes the window's own
    measurement (eq. update-fast).
  * Covariances are symmetrised, P <- (P + P^T)/2, after each update (rounding only).
  * The log-likelihood is sum_k log N(y_k; C_bar m^f_{k-1,l}, C_bar P C_bar^T + R_x),
    the normaliser of the IMKF update (eq. m-h-k-l).
"""
from __future__ import annotations

import numpy as np


def _sym(P):
    return 0.5 * (P + P.T)


def _mpow(A, i):
    return np.linalg.matrix_power(A, i)


def _per_window(X, N):
    X = np.asarray(X, dtype=float)
    return X if X.ndim == 3 else np.broadcast_to(X, (N,) + X.shape)


def slow_rate_model(A, Q, C, L, B=None):
    """Slow-rate dynamic and measurement model of Sec. III-A.

    With inputs (x_t = A x_{t-1} + B u_{t-1} + w_{t-1}, eq. original-linear-SSM) the stacked
    window input u_bar_k = [u_{k,0}; ...; u_{k,l-1}] (u_{k,i-1} drives x_{k,i}) enters as
    B_bar u_bar_k in the state equation and D_bar u_bar_k in the measurement equation, with
    B_bar = G_bar (I_l (x) B) and D_bar = M_bar (I_l (x) B) (the input rides the same
    propagation as the process noise).

    eq. h-k-l-2:  x_{k,l} = A_bar x_{k-1,l} + G_bar w_bar_k,
                  A_bar = A^l, G_bar = [A^{l-1} ... A I], Q_bar = G_bar Q~ G_bar^T.
    eq. y-k-l-2:  y_k = C_bar x_{k-1,l} + M_bar w_bar_k + v_k,
                  C_bar = (C/l) sum_{i=1..l} A^i,
                  M_bar = (C/l) [sum_{i=0}^{l-1} A^i, sum_{i=0}^{l-2} A^i, ..., I].
    """
    nx = A.shape[0]
    Abar = _mpow(A, L)
    Gbar = np.hstack([_mpow(A, L - 1 - j) for j in range(L)])
    Qtilde = np.kron(np.eye(L), Q)
    Qbar = Gbar @ Qtilde @ Gbar.T
    Cbar = (C / L) @ sum(_mpow(A, i) for i in range(1, L + 1))
    Mbar = (C / L) @ np.hstack([sum(_mpow(A, i) for i in range(0, L - j)) for j in range(L)])
    out = dict(Abar=Abar, Gbar=Gbar, Qtilde=Qtilde, Qbar=Qbar, Cbar=Cbar, Mbar=Mbar, nx=nx, L=L)
    if B is not None:
        Btilde = np.kron(np.eye(L), B)
        out.update(Bbar=Gbar @ Btilde, Dbar=Mbar @ Btilde)
    return out


def batch_model(A, Q, C, L, B=None):
    """Stacked fast-rate window model of Sec. III-B (with inputs: calB = calG (I_l (x) B)).

    eq. params-fast:   calA = [A; A^2; ...; A^l] (l nx x nx),
                       calG = lower block-triangular Toeplitz with blocks A^{r-c}.
    eq. y-k-l-2-H:     calH = (1/l) [C ... C] (ny x l nx).
    """
    nx = A.shape[0]
    calA = np.vstack([_mpow(A, i) for i in range(1, L + 1)])
    calG = np.zeros((L * nx, L * nx))
    for r in range(L):
        for c in range(r + 1):
            calG[r * nx:(r + 1) * nx, c * nx:(c + 1) * nx] = _mpow(A, r - c)
    calH = np.hstack([C] * L) / L
    Qtilde = np.kron(np.eye(L), Q)
    out = dict(calA=calA, calG=calG, calH=calH, Qtilde=Qtilde, nx=nx, L=L)
    if B is not None:
        out["calB"] = calG @ np.kron(np.eye(L), B)
    return out


def imkf(A, Q, C, R, L, m0, P0, y, B=None, u=None):
    """Sequential slow-rate IMKF, eq. prediction and eq. m-h-k-l (Sec. III-A).

    Optional inputs: B (nx x nu) and u [N][l][nu], u[k-1][i-1] driving x_{k,i}.
    Time-varying model: A, Q, C, R given per window as arrays [N, ...]. Reading: window k's
    A_k, Q_k drive its fast steps x_{k,1} .. x_{k,l} (the step from x_{k-1,l} included) and
    C_k, R_k its measurement, so each window's slow-rate model (eq. h-k-l-2, eq. y-k-l-2) is
    built from its own matrices.
    Returns (m, P, loglik) with m[k-1] = m^f_{k,l}, P[k-1] = P^f_{k,l} for k = 1..N.
    """
    tv = np.ndim(A) == 3
    sr = None if tv else slow_rate_model(A, Q, C, L, B)
    N = y.shape[0]
    nx, ny = np.shape(A)[-1], np.shape(C)[-2]
    ms = np.zeros((N, nx))
    Ps = np.zeros((N, nx, nx))
    m, P = np.array(m0, dtype=float), np.array(P0, dtype=float)
    ll = 0.0
    for k in range(N):
        if tv:  # window k's own slow-rate model
            sr = slow_rate_model(A[k], Q[k], C[k], L)
        Abar, Gbar, Qt, Qbar, Cbar, Mbar = (sr[x] for x in ("Abar", "Gbar", "Qtilde", "Qbar", "Cbar", "Mbar"))
        Rk = R[k] if tv else R
        ub = None if B is None else np.asarray(u[k], dtype=float).reshape(-1)
        # prediction (eq. prediction)
        m_pred = Abar @ m + (0.0 if ub is None else sr["Bbar"] @ ub)
        P_pred = Abar @ P @ Abar.T + Qbar
        # update (eq. m-h-k-l): gain from the cross-covariance with the correlated noise term
        cross = Abar @ P @ Cbar.T + Gbar @ Qt @ Mbar.T
        S = Cbar @ P @ Cbar.T + Mbar @ Qt @ Mbar.T + Rk
        innov = y[k] - Cbar @ m - (0.0 if ub is None else sr["Dbar"] @ ub)
        gain = np.linalg.solve(S.T, cross.T).T
        m = m_pred + gain @ innov
        P = _sym(P_pred - gain @ cross.T)
        ms[k], Ps[k] = m, P
        _, logdet = np.linalg.slogdet(S)
        ll += -0.5 * (innov @ np.linalg.solve(S, innov) + logdet + ny * np.log(2 * np.pi))
    return ms, Ps, ll


def fast_filter_window(bm, R, m_prev, P_prev, yk, uk=None):
    """Window posterior p(X_{k,1:l} | y_{1:k}), eq. predict-fast and eq. update-fast.

    (m_prev, P_prev) = (m^f_{k-1,l}, P^f_{k-1,l}); returns the dense (l nx) mean and
    (l nx) x (l nx) covariance of the stacked window states.
    """
    calA, calG, calH, Qt = bm["calA"], bm["calG"], bm["calH"], bm["Qtilde"]
    M_pred = calA @ m_prev
    if uk is not None:   # stacked window input u_{k,0..l-1}
        M_pred = M_pred + bm["calB"] @ np.asarray(uk, dtype=float).reshape(-1)
    P_pred = calA @ P_prev @ calA.T + calG @ Qt @ calG.T
    S = calH @ P_pred @ calH.T + R
    gain = np.linalg.solve(S.T, (P_pred @ calH.T).T).T
    M_f = M_pred + gain @ (yk - calH @ M_pred)
    P_f = _sym(P_pred - gain @ calH @ P_pred)
    return M_f, P_f


def _blocks(M, P, nx, L):
    m = M.reshape(L, nx)
    Pd = np.stack([P[i * nx:(i + 1) * nx, i * nx:(i + 1) * nx] for i in range(L)])
    return m, Pd


def srtm_filter(A, Q, C, R, L, m0, P0, y, B=None, u=None):
    """Fast- and slow-rate filtering marginals (Sec. III-A, III-B and Remark fast-par-filter).

    Returns dict with
      m_fast[k-1, i-1] = E[x_{k,i} | y_{1:k}],  P_fast[k-1, i-1] = Cov[x_{k,i} | y_{1:k}],
      m_slow[k-1] = m^f_{k,l},  P_slow[k-1] = P^f_{k,l}  (the IMKF carry), and loglik.
    Per-window (time-varying) arrays as in imkf: window k's filter uses its own batch model.
    """
    tv = np.ndim(A) == 3
    nx, N = np.shape(A)[-1], y.shape[0]
    m_slow, P_slow, ll = imkf(A, Q, C, R, L, m0, P0, y, B, u)
    bm = None if tv else batch_model(A, Q, C, L, B)
    m_fast = np.zeros((N, L, nx))
    P_fast = np.zeros((N, L, nx, nx))
    for k in range(N):
        mp, Pp = (m0, P0) if k == 0 else (m_slow[k - 1], P_slow[k - 1])
        if tv:
            bm = batch_model(A[k], Q[k], C[k], L)
        M_f, P_f = fast_filter_window(bm, R[k] if tv else R, mp, Pp, y[k], None if B is None else u[k])
        m_fast[k], P_fast[k] = _blocks(M_f, P_f, nx, L)
    return dict(m_fast=m_fast, P_fast=P_fast, m_slow=m_slow, P_slow=P_slow, loglik=ll)


def srtm_smoother(A, Q, C, R, L, m0, P0, y, *, with_filter=False, B=None, u=None, lag1=False):
    """Fast- and slow-rate smoothing marginals by the proposed sequential smoother.

    eq. smoothing-dynamic / eq. seq-smoothing-all (Sec. III-C): for k = N-1..1,
      m^-_{k+1,1} = A_hat M^f_k,  P^-_{k+1,1} = A_hat P^f_k A_hat^T + Q,
      G_k = P^f_k A_hat^T [P^-_{k+1,1}]^{-1},
      M^s_k = M^f_k + G_k (m^s_{k+1,1} - m^-_{k+1,1}),
      P^s_k = P^f_k + G_k (P^s_{k+1,1} - P^-_{k+1,1}) G_k^T,
    with A_hat = [0 ... 0 A]; window N is smoothed = filtered. The window filter
    (M^f_k, P^f_k) is recomputed from the stored slow carry (Remark fast-par-filter).
    With inputs the prediction of x_{k+1,1} adds B u_{k+1,0} (the input driving it).

    Per-window (time-varying) arrays as in imkf: window k's filter uses its own batch model,
    and the prediction of x_{k+1,1} uses A_{k+1} and Q_{k+1}, the model of that step.

    Returns dict with ms_fast/Ps_fast [N, L, ...] = p(x_{k,i} | y_{1:N}) and
    ms_slow/Ps_slow [N, ...] = p(x_{k,1} | y_{1:N}) (the smoother's slow state).

    lag1: also Cs_fast [N, L, nx, nx], the lag-one smoothed cross-covariances
    Cov(x_{k,i}, x_{k,i-1} | y_{1:N}) with x_{k,0} = x_{k-1,l} and x_{1,0} = x_0 (Remark
    cross-covariances): inside a window the off-diagonal blocks of the smoothed window
    covariance; across a boundary the smoother's cross term Cov(window k, x_{k+1,1}) = G_k P^s_{k+1,1},
    and for x_0 the same with the one-step gain P0 A^T (A P0 A^T + Q)^{-1}.
    """
    tv = np.ndim(A) == 3
    nx, N = np.shape(A)[-1], y.shape[0]
    m_slow, P_slow, ll = imkf(A, Q, C, R, L, m0, P0, y, B, u)
    bm = None if tv else batch_model(A, Q, C, L, B)
    Ahat = np.hstack([np.zeros((nx, (L - 1) * nx)), A]) if not tv else None
    ms_fast = np.zeros((N, L, nx))
    Ps_fast = np.zeros((N, L, nx, nx))
    Cs_fast = np.zeros((N, L, nx, nx)) if lag1 else None
    out = {}
    if with_filter:
        out["m_fast"] = np.zeros((N, L, nx))
        out["P_fast"] = np.zeros((N, L, nx, nx))
    ms1 = Ps1 = None
    for k in range(N - 1, -1, -1):
        mp, Pp = (m0, P0) if k == 0 else (m_slow[k - 1], P_slow[k - 1])
        if tv:
            bm = batch_model(A[k], Q[k], C[k], L)
        M_f, P_f = fast_filter_window(bm, R[k] if tv else R, mp, Pp, y[k], None if B is None else u[k])
        if with_filter:
            out["m_fast"][k], out["P_fast"][k] = _blocks(M_f, P_f, nx, L)
        if k == N - 1:
            M_s, P_s = M_f, P_f
        else:
            if tv:  # the step into x_{k+1,1} belongs to window k+1
                Ahat = np.hstack([np.zeros((nx, (L - 1) * nx)), A[k + 1]])
            m_pred = Ahat @ M_f + (0.0 if B is None else B @ np.asarray(u[k + 1][0], dtype=float))
            P_pred = Ahat @ P_f @ Ahat.T + (Q[k + 1] if tv else Q)
            G = np.linalg.solve(P_pred.T, (P_f @ Ahat.T).T).T
            M_s = M_f + G @ (ms1 - m_pred)
            P_s = _sym(P_f + G @ (Ps1 - P_pred) @ G.T)
            if lag1:  # x_{k+1,1} with x_{k,l}: the last block row of G P^s_{k+1,1}, transposed
                Cs_fast[k + 1, 0] = (G @ Ps1)[(L - 1) * nx:, :].T
        ms_fast[k], Ps_fast[k] = _blocks(M_s, P_s, nx, L)
        if lag1:
            for i in range(1, L):
                Cs_fast[k, i] = P_s[i * nx:(i + 1) * nx, (i - 1) * nx:i * nx]
        ms1, Ps1 = ms_fast[k, 0].copy(), Ps_fast[k, 0].copy()
    if lag1:  # x_{1,1} with the prior state x_0
        A1, Q1 = (A[0], Q[0]) if tv else (A, Q)
        P_one = A1 @ P0 @ A1.T + Q1
        G0 = np.linalg.solve(P_one.T, (P0 @ A1.T).T).T
        Cs_fast[0, 0] = (G0 @ Ps_fast[0, 0]).T
        out["Cs_fast"] = Cs_fast
    out.update(ms_fast=ms_fast, Ps_fast=Ps_fast, ms_slow=ms_fast[:, 0].copy(),
               Ps_slow=Ps_fast[:, 0].copy(), m_slow=m_slow, P_slow=P_slow, loglik=ll)
    return out


def imkf_tv(A, Q, C, R, L, m0, P0, y):
    """IMKF with a time-varying model given per window (arrays [N, ...]); see imkf."""
    N = y.shape[0]
    return imkf(*(_per_window(X, N) for X in (A, Q, C, R)), L, m0, P0, y)


def srtm_filter_tv(A, Q, C, R, L, m0, P0, y):
    """srtm_filter with a per-window model (arrays [N, ...]); see srtm_filter."""
    N = y.shape[0]
    return srtm_filter(*(_per_window(X, N) for X in (A, Q, C, R)), L, m0, P0, y)


def srtm_smoother_tv(A, Q, C, R, L, m0, P0, y, *, with_filter=False):
    """srtm_smoother with a per-window model (arrays [N, ...]); see srtm_smoother."""
    N = y.shape[0]
    return srtm_smoother(*(_per_window(X, N) for X in (A, Q, C, R)), L, m0, P0, y, with_filter=with_filter)


def slow_rate_smoother(A, Q, C, R, L, m0, P0, y):
    """Slow-rate smoother for x_{k,1}, eq. seq-smoothing-1 (Sec. III-C).

      G_{k,1} = P^f_{k,1,l} A^T [P^-_{k+1,1}]^{-1},
      m^s_{k,1} = m^f_{k,1} + G_{k,1} (m^s_{k+1,1} - m^-_{k+1,1}),
      P^s_{k,1} = P^f_{k,1} + G_{k,1} (P^s_{k+1,1} - P^-_{k+1,1}) G_{k,1}^T,
    with m^-_{k+1,1} = A m^f_{k,l}, P^-_{k+1,1} = A P^f_{k,l} A^T + Q, and the
    first/last cross-covariance P^f_{k,1,l} read from the window filter
    (Remark pf-k-1-l). Returns (ms, Ps) with ms[k-1] = m^s_{k,1}.
    """
    nx, N = A.shape[0], y.shape[0]
    m_slow, P_slow, _ = imkf(A, Q, C, R, L, m0, P0, y)
    bm = batch_model(A, Q, C, L)
    ms = np.zeros((N, nx))
    Ps = np.zeros((N, nx, nx))
    for k in range(N - 1, -1, -1):
        mp, Pp = (m0, P0) if k == 0 else (m_slow[k - 1], P_slow[k - 1])
        M_f, P_f = fast_filter_window(bm, R, mp, Pp, y[k])
        mf1 = M_f[:nx]
        Pf1 = P_f[:nx, :nx]
        if k == N - 1:
            ms[k], Ps[k] = mf1, Pf1
            continue
        Pf1L = P_f[:nx, (L - 1) * nx:]
        m_pred = A @ m_slow[k]
        P_pred = A @ P_slow[k] @ A.T + Q
        G1 = np.linalg.solve(P_pred.T, (Pf1L @ A.T).T).T
        ms[k] = mf1 + G1 @ (ms[k + 1] - m_pred)
        Ps[k] = _sym(Pf1 + G1 @ (Ps[k + 1] - P_pred) @ G1.T)
    return ms, Ps


def loglik_grad_fd(A, Q, C, R, L, m0, P0, y, h=1e-6, B=None, u=None):
    """Central finite differences of the IMKF log-likelihood (imkf) with respect to the model.

    Returns (dA, dQ, dR): dA[i, j] = d loglik / d A[i, j]; Q and R are perturbed as symmetric
    matrices (entries (i, j) and (j, i) together), and the returned dQ, dR are the symmetric
    gradients G with d loglik = tr(G E) for a small symmetric change E, i.e. half the paired
    difference off the diagonal. Step h is relative to max(1, |entry|). Known inputs (B, u) are
    passed through to imkf unchanged.
    """
    def ll(a, q, r):
        return imkf(a, q, C, r, L, m0, P0, y, B=B, u=u)[2]

    A, Q, R = (np.array(x, dtype=float) for x in (A, Q, R))
    nx, ny = A.shape[0], R.shape[0]
    dA = np.zeros_like(A)
    for i in range(nx):
        for j in range(nx):
            s = h * max(1.0, abs(A[i, j]))
            Ap, Am = A.copy(), A.copy()
            Ap[i, j] += s
            Am[i, j] -= s
            dA[i, j] = (ll(Ap, Q, R) - ll(Am, Q, R)) / (2 * s)

    def sym_grad(M, which):
        n = M.shape[0]
        G = np.zeros_like(M)
        for i in range(n):
            for j in range(i, n):
                s = h * max(1.0, abs(M[i, j]))
                Mp, Mm = M.copy(), M.copy()
                Mp[i, j] += s
                Mm[i, j] -= s
                if i != j:
                    Mp[j, i] += s
                    Mm[j, i] -= s
                fp = ll(A, Mp, R) if which == "Q" else ll(A, Q, Mp)
                fm = ll(A, Mm, R) if which == "Q" else ll(A, Q, Mm)
                d = (fp - fm) / (2 * s)
                G[i, j] = G[j, i] = d if i == j else 0.5 * d
        return G

    return dA, sym_grad(Q, "Q"), sym_grad(R, "R")
