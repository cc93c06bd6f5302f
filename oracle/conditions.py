"""Order conditions and stability function for ROK coefficient tables.

TEST INFRASTRUCTURE ONLY (CPU oracle; see the package docstring).

The paper defers the ROK coefficients and order theory to its reference on
Rosenbrock-Krylov methods (Sec. 2.2.2).  The conditions used here are derived
as follows.  Substituting k_i = V lambda_i + h (I - V V^T) F_i into eq. (9)
gives (I - h gamma A) k_i = h F_i + h A sum_j gamma_ij k_j with A = V H V^T =
P J P (P = V V^T), i.e. a Rosenbrock-W method (Sec. 2.2.1) whose matrix is A.
Since f(y_n) lies in K_M, A^k f = J^k f for k < M, so for M >= 4 every
elementary differential of order <= 4 in which A occurs equals its exact-J
counterpart except A f''(f, f).  Order 4 therefore means the eight classical
Rosenbrock conditions (Hairer & Wanner, Solving ODEs II, Sec. IV.7) with the
one involving sum b_i beta_ij alpha_j^2 split into its J part and its A part.

Notation: beta_ij = alpha_ij + gamma_ij, a_i = sum_j alpha_ij,
bp_i = sum_j beta_ij (sums over j < i).
"""
from __future__ import annotations

import numpy as np


def _arrays(tab):
    s = tab["s"]
    al = np.array(tab["alpha"], dtype=np.float64).reshape(s, s)
    ga = np.array(tab["gam"], dtype=np.float64).reshape(s, s)
    b = np.array(tab["b"], dtype=np.float64).reshape(s)
    return al, ga, b, float(tab["gamma"])


def rok4_residuals(tab) -> dict:
    """Residuals of the nine order-4 ROK conditions (M >= 4)."""
    al, ga, b, g = _arrays(tab)
    be = al + ga
    a = al.sum(axis=1)
    bp = be.sum(axis=1)
    return {
        "1": b.sum() - 1.0,
        "2": b @ bp - (0.5 - g),
        "3": b @ a**2 - 1.0 / 3.0,
        "4": b @ (be @ bp) - (1.0 / 6.0 - g + g * g),
        "5": b @ a**3 - 0.25,
        "6": b @ (a * (al @ bp)) - (1.0 / 8.0 - g / 3.0),
        "7a": b @ (al @ a**2) - 1.0 / 12.0,
        "7b": b @ (ga @ a**2) + g / 3.0,
        "8": b @ (be @ (be @ bp)) - (1.0 / 24.0 - g / 2.0 + 1.5 * g * g - g**3),
    }


def ros4_residuals(tab) -> dict:
    """The eight classical Rosenbrock order-4 conditions (7a and 7b merged)."""
    r = rok4_residuals(tab)
    r7 = r.pop("7a") + r.pop("7b")
    r["7"] = r7
    return r


def erk4_residuals(tab) -> dict:
    """Order-4 conditions of the explicit method (alpha, b) used when M = 0."""
    al, _, b, _ = _arrays(tab)
    a = al.sum(axis=1)
    return {
        "1": b.sum() - 1.0,
        "2": b @ a - 0.5,
        "3": b @ a**2 - 1.0 / 3.0,
        "4": b @ (al @ a) - 1.0 / 6.0,
        "5": b @ a**3 - 0.25,
        "6": b @ (a * (al @ a)) - 1.0 / 8.0,
        "7": b @ (al @ a**2) - 1.0 / 12.0,
        "8": b @ (al @ (al @ a)) - 1.0 / 24.0,
    }


def stability(tab, z: complex) -> complex:
    """R(z) = 1 + z b^T (I - z B)^{-1} 1, B = beta + gamma I (linear problem, A = J)."""
    al, ga, b, g = _arrays(tab)
    s = len(b)
    B = al + ga + g * np.eye(s)
    k = np.linalg.solve(np.eye(s) - z * B, np.ones(s))
    return 1.0 + z * (b @ k)
