"""Host logic of the checkpointed reverse sweep (paper_1607_06834_amd.autograd),
on the CPU: a stand-in integrator whose step is a fixed linear map A, so the
gradient of <w, y_K> is (A^T)^K w for every trajectory length and checkpoint
interval (nsteps = 0 included: the identity)."""
import pytest
import torch

from paper_1607_06834_amd.autograd import rok_trajectory


class LinearStepper:
    """Duck-typed stand-in for Rok: step(y) = A y, step_vjp(y, g) = A^T g."""

    def __init__(self, n, seed=0):
        gen = torch.Generator().manual_seed(seed)
        self.A = torch.eye(n, dtype=torch.float64) + 0.3 * torch.randn(n, n, dtype=torch.float64, generator=gen)
        self.calls = 0

    def step(self, y, h, tableau, M, mode="tangent", out=None):
        self.calls += 1
        return self.A @ y

    def step_vjp(self, y, g, h, tableau, M, out=None):
        out.copy_(self.A.T @ g)
        return out

    def step_keep(self, y, h, tableau, M):
        return self.A @ y, ("rec",)

    def step_vjp_stored(self, rec, g, out=None):
        out.copy_(self.A.T @ g)
        return out


@pytest.mark.parametrize("nsteps", [0, 1, 3, 7])
@pytest.mark.parametrize("every", [None, 2, 3, 10])
def test_gradient_of_linear_trajectory(nsteps, every):
    n = 6
    st = LinearStepper(n)
    gen = torch.Generator().manual_seed(1)
    y0 = torch.randn(n, dtype=torch.float64, generator=gen, requires_grad=True)
    w = torch.randn(n, dtype=torch.float64, generator=gen)
    yK = rok_trajectory(st, y0, 0.1, {}, 4, nsteps, checkpoint_every=every)
    (w @ yK).backward()
    want = torch.linalg.matrix_power(st.A.T, nsteps) @ w
    assert torch.allclose(y0.grad, want, rtol=1e-13, atol=1e-13)
    assert torch.allclose(yK.detach(), torch.linalg.matrix_power(st.A, nsteps) @ y0.detach(), rtol=1e-13)


@pytest.mark.parametrize("nsteps", [0, 1, 4])
def test_gradient_stored_forward(nsteps):
    n = 5
    st = LinearStepper(n, seed=2)
    y0 = torch.randn(n, dtype=torch.float64, requires_grad=True)
    w = torch.randn(n, dtype=torch.float64)
    yK = rok_trajectory(st, y0, 0.1, {}, 4, nsteps, store_forward=True)
    (w @ yK).backward()
    assert torch.allclose(y0.grad, torch.linalg.matrix_power(st.A.T, nsteps) @ w, rtol=1e-13, atol=1e-13)


def test_zero_steps_output_is_not_the_input():
    st = LinearStepper(3)
    y0 = torch.ones(3, dtype=torch.float64, requires_grad=True)
    y = rok_trajectory(st, y0, 0.1, {}, 4, 0)
    assert y.data_ptr() != y0.data_ptr()
    assert st.calls == 0


def test_negative_steps_rejected():
    with pytest.raises(ValueError):
        rok_trajectory(LinearStepper(3), torch.ones(3, dtype=torch.float64), 0.1, {}, 4, -1)
