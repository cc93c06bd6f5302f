"""Checkpoint and resume of a fixed-step ROK trajectory on the GPU.

A run is resumed from a saved state y_n (written to disk with numpy.save and
read back with numpy.load) in a fresh library context and continued with the
same step size, tableau and M; the final state must equal that of the
uninterrupted run bit for bit (each step depends only on y_n, h, the tableau
and M, so nothing else needs saving).
"""
import sys

import numpy as np
import pytest
import torch

import rok_inputs as ri

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1607_06834_amd import load_library
    load_library()
    return torch.device("cuda", 0)


@pytest.mark.parametrize("recon,mode,M", [("muscl", "fd", 16), ("first", "tangent", 8), ("muscl", "fd", 0)])
def test_resume_from_saved_state_is_bitwise(dev, tmp_path, recon, mode, M):
    from paper_1607_06834_amd import Rok
    say("resume", recon, mode, M)
    pb = ri.vortex_problem(48, recon)
    y0 = ri.vortex_state(pb)
    tab = ri.rok4_tableau()
    h = ri.cfl_step(pb, y0, 2.0 if M else 0.5)
    K, k_save = 12, 5
    R = Rok(pb)
    y = torch.tensor(y0, device=dev)
    saved = None
    for n in range(K):
        if n == k_save:
            path = tmp_path / "y_n.npy"
            np.save(path, y.cpu().numpy())
            saved = path
        y = R.step(y, h, tab, M, mode=mode)
    straight = y.cpu()
    del R
    R2 = Rok(pb)
    y = torch.tensor(np.load(saved), device=dev)
    for n in range(k_save, K):
        y = R2.step(y, h, tab, M, mode=mode)
    assert torch.isfinite(straight).all()
    assert torch.equal(y.cpu(), straight)
