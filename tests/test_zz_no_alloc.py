"""rok_jvp_noalloc (the allocation-free Jacobian-vector product) through the
C-ABI against rok_jvp on the same inputs: bit for bit (the same kernels, the
reductions of the default finite-difference increment in the library's
per-device scratch array instead of a workspace).  Two calls in a row, the
second on a smaller problem (the array keeps the first call's contents, which
the second must not read), in both orders of FD and exact products, 2-D and
3-D, FP64 and the FP32 form."""
import sys

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


def _inputs(pb, dev, seed):
    y = torch.tensor(ri.smooth_random_state(pb, seed=seed, amplitude=0.2), device=dev)
    v = torch.tensor(ri.random_direction(ri.size(pb), seed + 7), device=dev)
    return y, v


PAIRS = [
    ("vortex 96^2 then 24^2", lambda: ri.vortex_problem(96, "muscl"), lambda: ri.vortex_problem(24, "muscl")),
    ("ns3d 20^3 then 7x5x3", lambda: ri.tgv_problem(20, 3),
     lambda: ri.problem((7, 5, 3), (0, 0, 0), (1.0, 0.9, 1.2), "ns", "muscl", mu=0.05)),
    # column-marching grids (n0, n1 multiples of 16)
    ("ns3d 32^3 then 16x16x5", lambda: ri.tgv_problem(32, 3),
     lambda: ri.problem((16, 16, 5), (0, 0, 0), (1.0, 0.9, 1.2), "ns", "muscl", mu=0.05)),
]


@pytest.mark.parametrize("label,big,small", PAIRS)
@pytest.mark.parametrize("eps", [0.0, 3e-7])
def test_fd_noalloc_equals_jvp(dev, label, big, small, eps):
    from paper_1607_06834_amd import Rok
    for k, mk in enumerate((big, small)):
        pb = mk()
        g = Rok(pb, "fp64")
        y, v = _inputs(pb, dev, 10 + k)
        F = g.residual(y)
        ref = g.jvp(y, v, "fd", fy=F, eps=eps)
        got = g.jvp_noalloc(y, v, "fd", fy=F, eps=eps)
        torch.cuda.synchronize()
        say(label, "call", k + 1, "N", g.N, "eps", eps, "bitwise", torch.equal(got, ref))
        assert torch.equal(got, ref)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_tangent_noalloc_equals_jvp(dev, precision):
    from paper_1607_06834_amd import Rok
    for k, pb in enumerate((ri.tgv_problem(48, 2), ri.tgv_problem(16, 2))):
        g = Rok(pb, precision)
        y, v = _inputs(pb, dev, 20 + k)
        ref = g.jvp(y, v, "tangent")
        got = g.jvp_noalloc(y, v, "tangent")
        say("tangent", precision, "call", k + 1, "N", g.N, "bitwise", torch.equal(got, ref))
        assert torch.equal(got, ref)


def test_noalloc_after_other_calls_and_repeated(dev):
    """Interleaved with workspace calls and repeated: every result equals rok_jvp's."""
    from paper_1607_06834_amd import Rok
    pb = ri.vortex_problem(40, "first")
    g = Rok(pb, "fp64")
    y, v = _inputs(pb, dev, 30)
    F = g.residual(y)
    ref = g.jvp(y, v, "fd", fy=F)
    for _ in range(3):
        g.step(y, 0.001, ri.rok4_tableau(), 4, "fd")
        assert torch.equal(g.jvp_noalloc(y, v, "fd", fy=F), ref)
    say("interleaved: bitwise")


def test_noalloc_rejects_bad_arguments(dev):
    from paper_1607_06834_amd import Rok, RokError
    pb = ri.vortex_problem(16, "first")
    g = Rok(pb, "fp64")
    y, v = _inputs(pb, dev, 40)
    with pytest.raises(ValueError):
        g.jvp_noalloc(y, v, "fd")          # FD without f(y)
    g32 = Rok(pb, "fp32")
    with pytest.raises(RokError):
        g32.jvp_noalloc(y, v, "fd", fy=g.residual(y))   # FD products are FP64 only
