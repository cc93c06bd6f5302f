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
  the same for all stages (the reason given for Rosenbrock methods, Sec. 2.2);
* summation order.  The paper does not fix the order in which a dot product
  adds its N terms; floating-point sums depend on it, and the first-order
  difference quotient of Sec. 2.3, eq. 10, multiplies last-bit differences
  by 1/eps, so two correct implementations that add in different orders
  drift apart by ~1e-10 after one step.  The reading taken here is one
  canonical order, written out in `canonical_sum`: the terms are dealt
  round-robin over 262144 lanes, each lane adds its terms in index order,
  lanes are combined 256 at a time by a pairwise halving tree, and the 1024
  resulting sums are dealt over 256 lanes (four each, in order) and combined
  by the same tree.  Sums over the small Krylov index (V lambda, H g) are
  taken in column order.
"""
from __future__ import annotations

import math

import numpy as np
import torch

BREAKDOWN_TOL = 1e-13


RED_BLOCKS = 1024
RED_THREADS = 256
RED_LANES = RED_BLOCKS * RED_THREADS


def _halving_tree(s: np.ndarray) -> np.ndarray:
    """Pairwise sum along the last axis (length 256): s[i] += s[i + h], h = 128, 64, ..., 1."""
    s = s.copy()
    h = s.shape[-1] // 2
    while h >= 1:
        s[..., :h] = s[..., :h] + s[..., h:2 * h]
        h //= 2
    return s[..., 0]


def canonical_sum(terms: np.ndarray) -> float:
    """Sum of a float64 vector in the canonical order described in the module docstring.

    Lanes past the end of the data and blocks past the last used lane hold +0.0
    and are left out: adding +0.0 to a lane or block sum (never -0.0 when it
    starts from +0.0) leaves it unchanged.
    """
    n = terms.size
    used = max(1, min(n, RED_LANES))
    nb = -(-used // RED_THREADS)
    lane = np.zeros(nb * RED_THREADS, dtype=np.float64)
    for r in range(max(1, -(-n // RED_LANES))):
        seg = terms[r * RED_LANES:(r + 1) * RED_LANES]
        lane[:seg.size] = lane[:seg.size] + seg
    blocks = np.zeros(RED_BLOCKS, dtype=np.float64)
    blocks[:nb] = _halving_tree(lane.reshape(nb, RED_THREADS))
    fin = np.zeros(RED_THREADS, dtype=np.float64)
    for r in range(RED_BLOCKS // RED_THREADS):
        fin = fin + blocks[r * RED_THREADS:(r + 1) * RED_THREADS]
    return float(_halving_tree(fin[None, :])[0])


def dot(a: torch.Tensor, b: torch.Tensor) -> float:
    """<a, b>: products rounded once each, summed in the canonical order."""
    return canonical_sum((a * b).numpy())


def matvec_cols(V: torch.Tensor, c: torch.Tensor) -> torch.Tensor:
    """V c = sum_j c_j V[:, j], accumulated in column order from zero."""
    acc = torch.zeros(V.shape[0], dtype=torch.float64)
    for j in range(V.shape[1]):
        acc = acc + V[:, j] * float(c[j])
    return acc


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
