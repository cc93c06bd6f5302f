"""Derive the ROK4 coefficient table used by the tests and the benchmark.

TEST INFRASTRUCTURE (CPU oracle side).  Writes rok_inputs/rok4_tableau.json
and rok_inputs/ros4_only_tableau.json.  Run:  python -m oracle.derive_rok4

The paper takes its ROK coefficients from its reference on Rosenbrock-Krylov
methods (Sec. 2.2.2), which is not reproduced in the paper.  This script
derives a four-stage, order-4 table from the conditions in oracle.conditions:

* gamma = 1/x_2, x_2 the second root of the Laguerre polynomial L_4, so the
  stability function on the Krylov space vanishes at infinity (the choice that
  makes a four-stage, order-4 Rosenbrock method L-stable);
* (alpha, b) = the classical fourth-order Runge-Kutta method, so that M = 0
  (the explicit limit named after eq. 9) is itself order 4;
* the six gamma_ij solve the five remaining conditions; the one free
  parameter is fixed by the minimum-norm solution.

A second, diagnostic table satisfies the eight classical Rosenbrock conditions
but violates the split condition 7a/7b; it must show order 4 only when the
Krylov space is the whole space.
"""
from __future__ import annotations

import json
import os

import mpmath as mp

mp.mp.dps = 60

S = 4
HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(os.path.dirname(HERE), "rok_inputs")


def laguerre_gamma():
    roots = sorted(mp.polyroots([1, -16, 72, -96, 24], maxsteps=200, extraprec=200), key=lambda r: mp.re(r))
    return 1 / mp.re(roots[1])


def unpack(x):
    al = mp.zeros(S, S)
    ga = mp.zeros(S, S)
    k = 0
    for i in range(S):
        for j in range(i):
            al[i, j] = x[k]
            k += 1
    for i in range(S):
        for j in range(i):
            ga[i, j] = x[k]
            k += 1
    b = [x[k + i] for i in range(S)]
    return al, ga, b


def conds(al, ga, b, g, split_offset=None):
    be = al + ga
    a = [sum(al[i, j] for j in range(S)) for i in range(S)]
    bp = [sum(be[i, j] for j in range(S)) for i in range(S)]
    a2 = [x * x for x in a]

    def mv(Mx, v):
        return [sum(Mx[i, j] * v[j] for j in range(S)) for i in range(S)]

    def dotb(v):
        return sum(b[i] * v[i] for i in range(S))

    c = [
        sum(b) - 1,
        dotb(bp) - (mp.mpf(1) / 2 - g),
        dotb(a2) - mp.mpf(1) / 3,
        dotb(mv(be, bp)) - (mp.mpf(1) / 6 - g + g * g),
        dotb([x**3 for x in a]) - mp.mpf(1) / 4,
        dotb([a[i] * mv(al, bp)[i] for i in range(S)]) - (mp.mpf(1) / 8 - g / 3),
        dotb(mv(be, mv(be, bp))) - (mp.mpf(1) / 24 - g / 2 + mp.mpf(3) / 2 * g * g - g**3),
    ]
    r7a = dotb(mv(al, a2)) - mp.mpf(1) / 12
    r7b = dotb(mv(ga, a2)) + g / 3
    if split_offset is None:
        c += [r7a, r7b]
    else:
        c += [r7a + r7b, r7a - split_offset]
    return c


def min_norm_newton(F, x0, iters=60):
    x = mp.matrix(x0)
    for _ in range(iters):
        r = mp.matrix(F(x))
        if mp.norm(r) < mp.mpf(10) ** (-55):
            break
        n, m = len(r), len(x)
        J = mp.zeros(n, m)
        h = mp.mpf(10) ** (-30)
        for k in range(m):
            xp = x.copy()
            xp[k] += h
            rp = mp.matrix(F(xp))
            for i in range(n):
                J[i, k] = (rp[i] - r[i]) / h
        dx = J.T * mp.lu_solve(J * J.T, r)
        x = x - dx
    return x, mp.norm(mp.matrix(F(x)))


def table_json(al, ga, b, g, note):
    return {
        "s": S,
        "gamma": float(g),
        "alpha": [[float(al[i, j]) for j in range(S)] for i in range(S)],
        "gam": [[float(ga[i, j]) for j in range(S)] for i in range(S)],
        "b": [float(x) for x in b],
        "note": note,
    }


def derive():
    g = laguerre_gamma()
    # (alpha, b): classical RK4
    al = mp.zeros(S, S)
    al[1, 0] = mp.mpf(1) / 2
    al[2, 1] = mp.mpf(1) / 2
    al[3, 2] = mp.mpf(1)
    b = [mp.mpf(1) / 6, mp.mpf(1) / 3, mp.mpf(1) / 3, mp.mpf(1) / 6]

    def F_gam(x):
        ga = mp.zeros(S, S)
        k = 0
        for i in range(S):
            for j in range(i):
                ga[i, j] = x[k]
                k += 1
        c = conds(al, ga, b, g)
        return [c[1], c[3], c[5], c[6], c[8]]  # the conditions that involve gamma_ij

    x, res = min_norm_newton(F_gam, [mp.mpf("-0.3")] * 6)
    ga = mp.zeros(S, S)
    k = 0
    for i in range(S):
        for j in range(i):
            ga[i, j] = x[k]
            k += 1
    res = mp.norm(mp.matrix(conds(al, ga, b, g)))
    rok4 = table_json(al, ga, b, g, "ROK4: classical RK4 (alpha, b), gamma = 1/x2 of L4, "
                      "min-norm gamma_ij solving the order-4 ROK conditions; residual %.1e" % float(res))

    # diagnostic: eight classical ROS4 conditions hold, 7a is violated by 0.25
    x0 = []
    for i in range(S):
        for j in range(i):
            x0.append(al[i, j])
    x0 += list(x)
    x0 += b
    x1, res1 = min_norm_newton(lambda z: conds(*unpack(z), g, split_offset=mp.mpf("0.25")), x0)
    al1, ga1, b1 = unpack(x1)
    ros4 = table_json(al1, ga1, b1, g, "diagnostic: classical ROS4 conditions hold, ROK split "
                      "condition 7a violated by 0.25; residual %.1e" % float(res1))
    return rok4, ros4


def main():
    rok4, ros4 = derive()
    os.makedirs(OUT, exist_ok=True)
    with open(os.path.join(OUT, "rok4_tableau.json"), "w") as fh:
        json.dump(rok4, fh, indent=1)
    with open(os.path.join(OUT, "ros4_only_tableau.json"), "w") as fh:
        json.dump(ros4, fh, indent=1)
    print(json.dumps(rok4, indent=1))
    print(json.dumps(ros4, indent=1))


if __name__ == "__main__":
    main()
