"""Eigenvalues of the Jacobian of f (the stiffness diagnostic of Sec. 4).

TEST INFRASTRUCTURE ONLY (CPU oracle; see the package docstring).

The paper estimates the largest-magnitude eigenvalues of J = df/dy
matrix-free with an implicitly restarted Arnoldi method (Sec. 4, the
eigenvalue figures).  What that estimates has a plain definition: the
eigenvalues of the Jacobian.  Here J is formed densely (column by column, by
forward-mode differentiation of the oracle's residual) and its eigenvalues
are LAPACK's (numpy.linalg.eigvals); grids must be small enough to hold J.
"""
from __future__ import annotations

import numpy as np
import torch

from . import fv


def dense_jacobian(P: fv.Problem, y: torch.Tensor) -> torch.Tensor:
    """J(y) as an N x N float64 matrix (exact derivative of fv.residual)."""
    return torch.func.jacfwd(lambda z: fv.residual(P, z))(y)


def eigenvalues(P: fv.Problem, y: torch.Tensor) -> np.ndarray:
    """All eigenvalues of J(y), ordered by decreasing magnitude."""
    ev = np.linalg.eigvals(dense_jacobian(P, y).numpy())
    return ev[np.argsort(-np.abs(ev), kind="stable")]


def largest(P: fv.Problem, y: torch.Tensor, k: int) -> np.ndarray:
    """The k eigenvalues of largest magnitude."""
    return eigenvalues(P, y)[:k]
