"""Brute-force posteriors of the SRTM model by conditioning one dense joint Gaussian.

Independent of the recursive filters: the prior over all stacked fast states
Z = [x_0; x_1; ...; x_{NL}] is written from x_t = A^t x_0 + sum_{s<=t} A^{t-s} w_{s-1},
the measurements as Y = Psi Z + v with y_k = (C/L) sum_{i} x_{(k-1)L+i} (Sec. III,
eq. original-linear-SSM), and marginals follow from the Gaussian conditioning rule.
Only usable for tiny problems (dimension (N L + 1) nx).

Time-varying models: A, Q, C, R may also be given per window as arrays [N, ...]; window k's
A and Q then drive the fast steps into x_{k,1} .. x_{k,L} and its C, R give y_k.
"""
from __future__ import annotations

import numpy as np


def _per_window(X, N):
    X = np.asarray(X, dtype=float)
    return X if X.ndim == 3 else np.broadcast_to(X, (N,) + X.shape)


def joint_prior(A, Q, C, R, L, m0, P0, N, B=None, u=None):
    As, Qs, Cs, Rs = (_per_window(X, N) for X in (A, Q, C, R))
    nx, ny = As.shape[1], Cs.shape[1]
    T = N * L
    dim = (T + 1) * nx
    # transition products Phi(t, s) = A_t ... A_{s+1}, with A_t the matrix of the window of step t
    step_A = [None] + [As[(t - 1) // L] for t in range(1, T + 1)]
    Phi = np.zeros((dim, nx))
    Gam = np.zeros((dim, T * nx))
    for s in range(T + 1):
        M = np.eye(nx)
        for t in range(s, T + 1):
            if t > s:
                M = step_A[t] @ M
            if s == 0:
                Phi[t * nx:(t + 1) * nx] = M
            else:                          # w_{s-1} enters x_s
                Gam[t * nx:(t + 1) * nx, (s - 1) * nx:s * nx] = M
    muZ = Phi @ m0
    if B is not None:   # u_{s-1} enters x_s like w_{s-1}: mean shift Gam (I_T (x) B) u
        muZ = muZ + Gam @ np.kron(np.eye(T), B) @ np.asarray(u, dtype=float).reshape(-1)
    Qw = np.zeros((T * nx, T * nx))       # Cov of the stacked w_0 .. w_{T-1}
    for s in range(1, T + 1):
        Qw[(s - 1) * nx:s * nx, (s - 1) * nx:s * nx] = Qs[(s - 1) // L]
    SZ = Phi @ P0 @ Phi.T + Gam @ Qw @ Gam.T
    Psi = np.zeros((N * ny, dim))
    Rv = np.zeros((N * ny, N * ny))
    for k in range(N):
        for i in range(1, L + 1):
            t = k * L + i
            Psi[k * ny:(k + 1) * ny, t * nx:(t + 1) * nx] = Cs[k] / L
        Rv[k * ny:(k + 1) * ny, k * ny:(k + 1) * ny] = Rs[k]
    SY = Psi @ SZ @ Psi.T + Rv
    return muZ, SZ, Psi, SY


def _condition(muZ, SZ, Psi, SY, y, rows):
    """Mean and covariance of Z given the measurement rows `rows` of Y."""
    SZY = (SZ @ Psi.T)[:, rows]
    Syy = SY[np.ix_(rows, rows)]
    r = y.reshape(-1)[rows] - (Psi @ muZ)[rows]
    K = np.linalg.solve(Syy, SZY.T).T
    return muZ + K @ r, SZ - K @ SZY.T


def posteriors(A, Q, C, R, L, m0, P0, y, B=None, u=None):
    """Exact filter and smoother marginals of every fast state x_{k,i}.

    Returns dict: m_fast/P_fast = p(x_{k,i} | y_{1:k}), ms_fast/Ps_fast = p(x_{k,i} | y_{1:N}),
    Cs_fast = Cov(x_{k,i}, x_{k,i-1} | y_{1:N}) (x_{k,0} = x_{k-1,L}, x_{1,0} = x_0),
    and loglik = log N(Y; Psi mu_Z, Psi S_Z Psi^T + I (x) R).
    """
    nx, ny = np.shape(A)[-1], np.shape(C)[-2]
    N = y.shape[0]
    muZ, SZ, Psi, SY = joint_prior(A, Q, C, R, L, m0, P0, N, B, u)
    m_fast = np.zeros((N, L, nx))
    P_fast = np.zeros((N, L, nx, nx))
    for k in range(N):
        mu, S = _condition(muZ, SZ, Psi, SY, y, np.arange((k + 1) * ny))
        for i in range(L):
            t = k * L + i + 1
            m_fast[k, i] = mu[t * nx:(t + 1) * nx]
            P_fast[k, i] = S[t * nx:(t + 1) * nx, t * nx:(t + 1) * nx]
    mu, S = _condition(muZ, SZ, Psi, SY, y, np.arange(N * ny))
    ms_fast = np.zeros((N, L, nx))
    Ps_fast = np.zeros((N, L, nx, nx))
    Cs_fast = np.zeros((N, L, nx, nx))   # Cov(x_t, x_{t-1} | y_{1:N}), t = (k-1) L + i
    for k in range(N):
        for i in range(L):
            t = k * L + i + 1
            ms_fast[k, i] = mu[t * nx:(t + 1) * nx]
            Ps_fast[k, i] = S[t * nx:(t + 1) * nx, t * nx:(t + 1) * nx]
            Cs_fast[k, i] = S[t * nx:(t + 1) * nx, (t - 1) * nx:t * nx]
    r = y.reshape(-1) - Psi @ muZ
    _, logdet = np.linalg.slogdet(SY)
    ll = -0.5 * (r @ np.linalg.solve(SY, r) + logdet + len(r) * np.log(2 * np.pi))
    return dict(m_fast=m_fast, P_fast=P_fast, ms_fast=ms_fast, Ps_fast=Ps_fast, Cs_fast=Cs_fast, loglik=ll)


def one_window_moments(A, Q, C, R, L):
    """Moments of one window given x_{k-1,l} = 0, read off the joint prior of a single window.

    Returns (Abar, Cbar, Qbar, Syx, Rx): the map x_{k-1,l} -> E[x_{k,l}], the map
    x_{k-1,l} -> E[y_k], Cov(x_{k,l}), Cov(x_{k,l}, y_k) and Cov(y_k), obtained by
    brute-force conditioning rather than by the slow-rate formulas.
    """
    nx, ny = A.shape[0], C.shape[0]
    zero = np.zeros(nx)
    muZ, SZ, Psi, SY = joint_prior(A, Q, C, R, L, zero, np.zeros((nx, nx)), 1)
    last = slice(L * nx, (L + 1) * nx)
    Qbar = SZ[last, last]
    Syx = (SZ @ Psi.T)[last]
    Rx = SY
    # mean maps: propagate unit initial states without noise
    Abar = np.zeros((nx, nx))
    Cbar = np.zeros((ny, nx))
    for j in range(nx):
        e = np.zeros(nx)
        e[j] = 1.0
        mu, _, Psi1, _ = joint_prior(A, Q, C, R, L, e, np.zeros((nx, nx)), 1)
        Abar[:, j] = mu[last]
        Cbar[:, j] = Psi1 @ mu
    return Abar, Cbar, Qbar, Syx, Rx
