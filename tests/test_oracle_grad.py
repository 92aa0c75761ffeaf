"""Pins of the finite-difference log-likelihood gradient (the reference for the GPU gradient).

* Scalar closed form: nx = ny = 1, L = 1, N = 1 reduces the model to y = c (a x_0 + w) + v,
  so log p(y) = log N(y; c a m0, c^2 (a^2 P0 + q) + r), whose derivatives in a, q and r are
  written out by hand below.
* Two step sizes agree (the difference quotient has converged).
* Symmetry: the Q and R gradients are symmetric.
"""
import numpy as np

import oracle
from paper_2410_00627_amd import workloads as wl


def test_fd_gradient_matches_scalar_closed_form():
    a, q, c, r, m0, P0, y = 0.9, 0.3, 1.7, 0.4, 0.5, 2.0, 1.3
    mu = c * a * m0
    s = c * c * (a * a * P0 + q) + r
    dll_ds = 0.5 * ((y - mu) ** 2 / s ** 2 - 1.0 / s)
    dll_dmu = (y - mu) / s
    da = dll_dmu * c * m0 + dll_ds * 2 * c * c * a * P0
    dq = dll_ds * c * c
    dr = dll_ds
    # the oracle's measurement model is y = (C / L) sum_i x_i + v with L = 1
    gA, gQ, gR = oracle.loglik_grad_fd(np.array([[a]]), np.array([[q]]), np.array([[c]]), np.array([[r]]), 1,
                                       np.array([m0]), np.array([[P0]]), np.array([[y]]))
    for got, want in ((gA[0, 0], da), (gQ[0, 0], dq), (gR[0, 0], dr)):
        assert abs(got - want) <= 1e-7 * max(1.0, abs(want))


def test_fd_gradient_converged_and_symmetric():
    m = wl.random_general_model(3, 2, 4, 71)
    y = wl.simulate(m, 30, 72)
    g1 = oracle.loglik_grad_fd(m.A, m.Q, m.C, m.R, m.L, m.m0, m.P0, y, h=1e-5)
    g2 = oracle.loglik_grad_fd(m.A, m.Q, m.C, m.R, m.L, m.m0, m.P0, y, h=1e-6)
    for a, b in zip(g1, g2):
        assert np.max(np.abs(a - b)) <= 1e-5 * max(1.0, np.max(np.abs(b)))
    assert np.array_equal(g2[1], g2[1].T) and np.array_equal(g2[2], g2[2].T)
