"""Writes wna_window_constants.txt: exact slow-rate window constants of the tiny
white-noise-acceleration model (dt = 1/100, q = 1, l = 10, y = dt * sum [1 0] x).

The model's Q(dt) is the exact discretisation of continuous white-noise acceleration,
so x_{k,i} are samples of integrated Brownian motion at t_i = i dt after x_{k-1,l}.
The constants of eq. h-k-l-2 and eq. y-k-l-2 then have closed forms:
  A_bar = A^l = [[1, T], [0, 1]],  T = l dt,
  Q_bar = q [[T^3/3, T^2/2], [T^2/2, T]],
  C_bar = (C/l) sum_i A^i = dt * [l, dt * l(l+1)/2],
  M_bar Q~ M_bar^T = dt^2 sum_{i,j} Cov(p(t_i), p(t_j)),
  G_bar Q~ M_bar^T = dt sum_j Cov(x(T), p(t_j)),
with Cov(p(s), p(t)) = q (a^2 b / 2 - a^3 / 6), a = min, b = max, and
Cov(v(T), p(t)) = q t^2 / 2 for t <= T. Run: python tests/golden/make_wna_constants.py
"""
import os
from fractions import Fraction as Fr

dt, q, L = Fr(1, 100), Fr(1), 10
T = L * dt
t = [i * dt for i in range(1, L + 1)]


def cpp(s, u):
    a, b = min(s, u), max(s, u)
    return q * (a * a * b / 2 - a ** 3 / 6)


def cvp(s, u):          # Cov(v(s), p(u)) for u <= s
    return q * u * u / 2


vals = {
    "Abar": [Fr(1), T, Fr(0), Fr(1)],
    "Qbar": [q * T ** 3 / 3, q * T ** 2 / 2, q * T ** 2 / 2, q * T],
    "Cbar": [dt * L, dt * dt * L * (L + 1) / 2],
    "Syy": [dt * dt * sum(cpp(a, b) for a in t for b in t)],
    "Sxy": [dt * sum(cpp(T, b) for b in t), dt * sum(cvp(T, b) for b in t)],
}

if __name__ == "__main__":
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "wna_window_constants.txt")
    with open(out, "w") as f:
        f.write("# Exact window constants of the white-noise-acceleration model (dt=1/100, q=1, l=10),\n")
        f.write("# slow-rate model of Sec. III-A (eq. h-k-l-2, eq. y-k-l-2); written by make_wna_constants.py\n")
        f.write("# from continuous-time closed forms. Matrices are row-major.\n")
        for k, v in vals.items():
            f.write(f"{k} = " + " ".join(str(x) for x in v) + "\n")
    print(open(out).read())
