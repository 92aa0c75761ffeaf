"""Seeded synthetic SRTM workloads (model matrices and simulated measurements).

This module is shared by the tests, the benchmark and the CPU reference. It holds
no filtering or smoothing arithmetic: it only draws a linear Gaussian model of the
form of Sec. III (eq. original-linear-SSM, with B = 0) and simulates data from it.

Conventions (the paper's, Sec. III):
  x_t = A x_{t-1} + w_{t-1},   w ~ N(0, Q)
  y_k = (C / L) * sum_{i=1..L} x_{k,i} + v_k,  v ~ N(0, R)
  window k holds fast steps (k-1)L+1 .. kL; x_0 ~ N(m0, P0) belongs to no window.
The C-ABI names the matrices (F, Q, H, R); F is the paper's A and H the paper's C.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Model:
    """A time-invariant linear Gaussian SRTM model (all float64)."""
    A: np.ndarray          # (nx, nx) fast-rate transition
    Q: np.ndarray          # (nx, nx) process-noise covariance
    C: np.ndarray          # (ny, nx) measurement matrix; y averages C x over a window
    R: np.ndarray          # (ny, ny) measurement-noise covariance
    L: int                 # window length (fast steps per measurement)
    m0: np.ndarray         # (nx,) initial mean
    P0: np.ndarray         # (nx, nx) initial covariance
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nx(self) -> int:
        return self.A.shape[0]

    @property
    def ny(self) -> int:
        return self.C.shape[0]


def _haar_orthogonal(rng: np.random.Generator, n: int) -> np.ndarray:
    """Haar-distributed orthogonal matrix: QR of an N(0,1) matrix, columns sign-fixed."""
    g = rng.standard_normal((n, n))
    q, r = np.linalg.qr(g)
    return q * np.sign(np.diag(r))[None, :]


def wna_model(dt: float = 0.01, q: float = 1.0, L: int = 10, r: float = 0.1) -> Model:
    """Position/velocity model with white-noise acceleration (the tiny FP64 case).

    The measurement is dt * sum_{window} [1, 0] x, i.e. in the paper's (C/L) sum
    convention C = L * dt * [1, 0].
    """
    A = np.array([[1.0, dt], [0.0, 1.0]])
    Q = q * np.array([[dt ** 3 / 3.0, dt ** 2 / 2.0], [dt ** 2 / 2.0, dt]])
    C = np.array([[L * dt, 0.0]])
    R = np.array([[r]])
    return Model(A, Q, C, R, L, np.zeros(2), np.eye(2), name="wna",
                 meta=dict(dt=dt, q=q))


def random_stable_model(nx: int, ny: int, L: int, seed: int, *, rho: float = 0.99,
                        q: float = 0.01, r: float = 0.05) -> Model:
    """A = rho * U (U Haar orthogonal), Q = q I, C ~ N(0,1)^{ny x nx}, R = r I, m0 = 0, P0 = I."""
    rng = np.random.Generator(np.random.PCG64(seed))
    A = rho * _haar_orthogonal(rng, nx)
    C = rng.standard_normal((ny, nx))
    return Model(A, q * np.eye(nx), C, r * np.eye(ny), L, np.zeros(nx), np.eye(nx),
                 name=f"rand_nx{nx}_ny{ny}_L{L}_s{seed}", meta=dict(seed=seed))


def random_spd(rng: np.random.Generator, n: int, scale: float = 1.0, floor: float = 0.1) -> np.ndarray:
    g = rng.standard_normal((n, n))
    return scale * (g @ g.T / n + floor * np.eye(n))


def random_general_model(nx: int, ny: int, L: int, seed: int) -> Model:
    """Non-orthogonal A, full Q, R, P0 and nonzero m0 (for pins that must not rely on structure)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    A = rng.standard_normal((nx, nx))
    A *= 0.95 / max(abs(np.linalg.eigvals(A)))
    Q = random_spd(rng, nx, 0.05)
    C = rng.standard_normal((ny, nx))
    R = random_spd(rng, ny, 0.2)
    m0 = rng.standard_normal(nx)
    P0 = random_spd(rng, nx, 1.0)
    return Model(A, Q, C, R, L, m0, P0, name=f"gen_nx{nx}_ny{ny}_L{L}_s{seed}",
                 meta=dict(seed=seed))


def headline_model(seed: int = 2024) -> Model:
    """One long sequence: nx=4, ny=2, L=20, A = 0.99 U, Q = 0.01 I, C Gaussian, R = 0.05 I."""
    return random_stable_model(4, 2, 20, seed, rho=0.99, q=0.01, r=0.05)


HEADLINE_N = 1 << 17
WNA_N = 100


def random_inputs(nx: int, nu: int, L: int, N: int, seed: int, scale: float = 0.5):
    """Input matrix B ~ N(0,1)^{nx x nu} and inputs u [N][L][nu]: a slow sinusoid plus
    N(0, scale^2) noise per fast step."""
    rng = np.random.Generator(np.random.PCG64(seed))
    B = rng.standard_normal((nx, nu))
    t = np.arange(N * L).reshape(N, L, 1)
    u = np.sin(2 * np.pi * t / (7.0 * L) + np.arange(nu)) + scale * rng.standard_normal((N, L, nu))
    return B, u


@dataclass
class TVModel:
    """A linear Gaussian SRTM model whose matrices change from window to window (float64):
    window k's A[k-1], Q[k-1] drive its fast steps x_{k,1} .. x_{k,L} (the step from x_{k-1,L}
    included) and C[k-1], R[k-1] give its measurement y_k."""
    A: np.ndarray          # (N, nx, nx)
    Q: np.ndarray          # (N, nx, nx)
    C: np.ndarray          # (N, ny, nx)
    R: np.ndarray          # (N, ny, ny)
    L: int
    m0: np.ndarray
    P0: np.ndarray
    name: str = ""

    @property
    def nx(self) -> int:
        return self.A.shape[1]

    @property
    def ny(self) -> int:
        return self.C.shape[1]

    @property
    def N(self) -> int:
        return self.A.shape[0]


def time_varying_model(nx: int, ny: int, L: int, N: int, seed: int, *, general: bool = False) -> TVModel:
    """Per-window matrices. Default: a slowly drifting version of the long-sequence model,
    A_k = rho_k U (U Haar orthogonal, rho_k = 0.97 + 0.02 sin(2 pi k / 50)),
    Q_k = 0.01 (1 + 0.5 sin(2 pi k / 37)) I, C_k = C0 + 0.2 sin(2 pi k / 29) C1 (C0, C1
    Gaussian), R_k = 0.05 (1 + 0.5 cos(2 pi k / 23)) I, m0 = 0, P0 = I. With general=True every
    window draws an unrelated random model (non-orthogonal A with spectral radius 0.95, full Q,
    R), with nonzero m0 and full P0: for pins that must not rely on structure."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if general:
        A = np.empty((N, nx, nx))
        Q = np.empty((N, nx, nx))
        C = rng.standard_normal((N, ny, nx))
        R = np.empty((N, ny, ny))
        for k in range(N):
            a = rng.standard_normal((nx, nx))
            A[k] = a * (0.95 / max(abs(np.linalg.eigvals(a))))
            Q[k] = random_spd(rng, nx, 0.05)
            R[k] = random_spd(rng, ny, 0.2)
        return TVModel(A, Q, C, R, L, rng.standard_normal(nx), random_spd(rng, nx, 1.0),
                       name=f"tvgen_nx{nx}_ny{ny}_L{L}_s{seed}")
    U = _haar_orthogonal(rng, nx)
    C0 = rng.standard_normal((ny, nx))
    C1 = rng.standard_normal((ny, nx))
    k = np.arange(1, N + 1)
    rho = 0.97 + 0.02 * np.sin(2 * np.pi * k / 50.0)
    q = 0.01 * (1.0 + 0.5 * np.sin(2 * np.pi * k / 37.0))
    r = 0.05 * (1.0 + 0.5 * np.cos(2 * np.pi * k / 23.0))
    A = rho[:, None, None] * U[None]
    Q = q[:, None, None] * np.eye(nx)[None]
    C = C0[None] + 0.2 * np.sin(2 * np.pi * k / 29.0)[:, None, None] * C1[None]
    R = r[:, None, None] * np.eye(ny)[None]
    return TVModel(A, Q, C, R, L, np.zeros(nx), np.eye(nx), name=f"tv_nx{nx}_ny{ny}_L{L}_s{seed}")


def simulate_tv(model: TVModel, seed: int, *, return_states: bool = False):
    """Draw x_0..x_{NL} and y_1..y_N from a per-window model (plain loop over fast steps)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nx, ny, L, N = model.nx, model.ny, model.L, model.N
    x = model.m0 + _chol_psd(model.P0) @ rng.standard_normal(nx)
    xs = [x]
    y = np.zeros((N, ny))
    for k in range(N):
        cq = _chol_psd(model.Q[k])
        acc = np.zeros(nx)
        for _ in range(L):
            x = model.A[k] @ x + cq @ rng.standard_normal(nx)
            acc += x
            xs.append(x)
        y[k] = model.C[k] @ acc / L + _chol_psd(model.R[k]) @ rng.standard_normal(ny)
    return (y, np.array(xs)) if return_states else y


def batched_specs(n_seq: int = 256, seed: int = 3030):
    """Many independent sequences of uneven length: per sequence nx in {2, 4, 6}, L in
    {5, 10, 20}, N = round(2^U(8, 14)) windows, ny = 1; returns (nx, L, N, model seed) tuples."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for j in range(n_seq):
        nx = int(rng.choice([2, 4, 6]))
        L = int(rng.choice([5, 10, 20]))
        N = int(round(2.0 ** rng.uniform(8.0, 14.0)))
        out.append((nx, L, N, seed * 1000 + j))
    return out


def batched_model(nx: int, L: int, seed: int) -> Model:
    """One sequence of the batched workload: A = 0.99 U, Q = 0.01 I, C Gaussian 1 x nx, R = 0.1."""
    return random_stable_model(nx, 1, L, seed, rho=0.99, q=0.01, r=0.1)


def _chol_psd(S: np.ndarray) -> np.ndarray:
    w, V = np.linalg.eigh(S)
    return V * np.sqrt(np.clip(w, 0.0, None))[None, :]


def simulate(model: Model, N: int, seed: int, *, return_states: bool = False, B=None, u=None):
    """Draw x_0..x_{NL} and y_1..y_N from the model (float64); with inputs, B (nx x nu) and
    u [N][L][nu] add B u[k-1][i-1] to the step into x_{k,i}.

    The fast-rate recursion is evaluated blockwise: within blocks of b steps it runs
    vectorised over all blocks from a zero start, then block-start states are chained
    and their free responses A^j x_start added back. This is plain linear algebra on
    the generative model, exact up to rounding.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    nx, ny, L = model.nx, model.ny, model.L
    T = N * L
    x0 = model.m0 + _chol_psd(model.P0) @ rng.standard_normal(nx)
    w = rng.standard_normal((T, nx)) @ _chol_psd(model.Q).T      # w_{t-1} drives x_t
    v = rng.standard_normal((N, ny)) @ _chol_psd(model.R).T
    if B is not None:
        w = w + np.asarray(u, dtype=float).reshape(T, -1) @ np.asarray(B, dtype=float).T
    A = model.A
    b = max(1, min(T, int(np.sqrt(T)) + 1))
    nb = -(-T // b)
    wp = np.zeros((nb * b, nx))
    wp[:T] = w
    wp = wp.reshape(nb, b, nx)
    loc = np.zeros((nb, b, nx))            # zero-start response inside each block
    cur = np.zeros((nb, nx))
    for j in range(b):
        cur = cur @ A.T + wp[:, j]
        loc[:, j] = cur
    starts = np.zeros((nb, nx))            # state just before each block
    s = x0.copy()
    Ab = np.linalg.matrix_power(A, b)
    for k in range(nb):
        starts[k] = s
        s = Ab @ s + loc[k, b - 1]
    Apows = np.empty((b, nx, nx))
    P = np.eye(nx)
    for j in range(b):
        P = A @ P
        Apows[j] = P
    x = loc + np.einsum("jab,kb->kja", Apows, starts)
    x = x.reshape(nb * b, nx)[:T]                     # x_1 .. x_T
    xw = x.reshape(N, L, nx)
    y = (xw.sum(axis=1) @ model.C.T) / L + v
    if return_states:
        return y, xw, x0
    return y
