"""Host-side argument checks of the autograd wrappers (no GPU needed: the
check runs before anything reaches the library)."""
import pytest
import torch

from paper_2312_02756_amd import autograd as ag


def test_broadcast_beta_requiring_grad_is_rejected():
    x = tuple(torch.ones(8, dtype=torch.float64) for _ in range(4))
    beta = tuple(torch.full((1,), 0.1, dtype=torch.float64, requires_grad=True) for _ in range(3))
    with pytest.raises(ValueError, match="broadcast beta"):
        ag.boost(x, beta)
