"""Modified Arnoldi and the reduced (M x M) solve of the ROK method.

TEST INFRASTRUCTURE ONLY (CPU oracle; see the package docstring).

Sec. 2.2.2: the ROK method builds, by modified Arnoldi iteration, an
orthonormal basis V (N x M) of the Krylov space K_M(J_n, f(y_n)) together with
the upper Hessenberg H = V^T J_n V, and solves (I_M - h gamma H) lambda = rhs
by a direct method.  Readings of what the paper leaves open:

* breakdown: if ||f(y_n)|| = 0 the basis is empty (M_eff = 0); if the new
  subdiagonal h_{j+1,j} <= tol * ||(h_{1j}, ..., h_{j+1,j})|| (the norm of
  J v_j before orthogonalisation, by Pythagoras), the space is invariant and
  M_eff = j; always M_eff <= min(M, N);
* H is the leading M x M block: the last column is orthogonalised but its
  subdiagonal and the vector v_{M+1} are not formed;
* inside Arnoldi the finite-difference increment uses ||v_j|| = 1;
* the direct method is LU with partial pivoting (row swap only when a later
  pivot is strictly larger in magnitude), done once per step since gamma is
  the same for all stages (the reason given for Rosenbrock methods, Sec. 2.2).
"""
from __future__ import annotations

import math

import torch

BREAKDOWN_TOL = 1e-13


def dot(a: torch.Tensor, b: torch.Tensor) -> float:
    return float(torch.dot(a, b))


def arnoldi(matvec, f0: torch.Tensor, M: int, tol: float = BREAKDOWN_TOL):
    """Modified Gram-Schmidt Arnoldi for K_M(J, f0).

    matvec(v) returns J v.  Returns (V, H, M_eff) with V of shape (N, M_eff)
    (columns are the basis vectors) and H of shape (M_eff, M_eff).
    """
    N = f0.numel()
    M = min(M, N)
    beta = math.sqrt(dot(f0, f0))
    H = torch.zeros(M + 1, M, dtype=torch.float64)
    cols = []
    if beta == 0.0 or M == 0:
        return torch.zeros(N, 0, dtype=torch.float64), torch.zeros(0, 0, dtype=torch.float64), 0
    cols.append(f0 / beta)
    m_eff = M
    for j in range(M):
        w = matvec(cols[j])
        for i in range(j + 1):
            hij = dot(cols[i], w)
            H[i, j] = hij
            w = w - hij * cols[i]
        if j + 1 == M:
            break
        hn = math.sqrt(dot(w, w))
        H[j + 1, j] = hn
        s = 0.0
        for i in range(j + 2):
            s = s + H[i, j].item() * H[i, j].item()
        if hn <= tol * math.sqrt(s):
            m_eff = j + 1
            break
        cols.append(w / hn)
    V = torch.stack(cols[:m_eff], dim=1)
    return V, H[:m_eff, :m_eff].clone(), m_eff


def lu_factor(A: torch.Tensor):
    """LU with partial pivoting, written out; returns (LU as nested lists, perm)."""
    n = A.shape[0]
    LU = [[float(A[i, j]) for j in range(n)] for i in range(n)]
    perm = list(range(n))
    for k in range(n):
        piv = k
        for r in range(k + 1, n):
            if abs(LU[r][k]) > abs(LU[piv][k]):
                piv = r
        if piv != k:
            LU[k], LU[piv] = LU[piv], LU[k]
            perm[k], perm[piv] = perm[piv], perm[k]
        for r in range(k + 1, n):
            LU[r][k] = LU[r][k] / LU[k][k]
            for c in range(k + 1, n):
                LU[r][c] = LU[r][c] - LU[r][k] * LU[k][c]
    return LU, perm


def lu_solve(LU, perm, b: torch.Tensor) -> torch.Tensor:
    n = len(LU)
    bl = [float(x) for x in b]
    x = [bl[perm[i]] for i in range(n)]
    for i in range(n):
        for c in range(i):
            x[i] = x[i] - LU[i][c] * x[c]
    for i in reversed(range(n)):
        for c in range(i + 1, n):
            x[i] = x[i] - LU[i][c] * x[c]
        x[i] = x[i] / LU[i][i]
    return torch.tensor(x, dtype=torch.float64)
