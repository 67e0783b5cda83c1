"""Host-side checks of the torch layer: it imports without a GPU and refuses
CPU tensors (there is no CPU path)."""
import pytest
import torch

from paper_2004_01729_amd import autograd as A


class _FakeSolver:
    B = 1
    sizes = [2]


def test_cpu_tensors_are_refused():
    mu = torch.zeros(1, dtype=torch.float64)
    beta = torch.ones(1, dtype=torch.float64)
    h = torch.zeros(1, 2, 2, dtype=torch.float64, requires_grad=True)
    with pytest.raises(ValueError, match="no CPU path"):
        A.FTCCOmega.apply(mu, beta, h, _FakeSolver())


def test_solver_requires_hip_device():
    with pytest.raises(ValueError):
        A.OmegaSolver([torch.zeros(2, 2, 2, 2).numpy()], [torch.zeros(2).numpy()], device="cpu")
