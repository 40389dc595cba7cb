"""CPU check of the closed-form gradient of the log-spectrum loss that the flow-control
workload applies every step: against torch autograd through the oracle's own shell
spectrum, in 2D and 3D, with and without shells below the clamp cutoff."""
import pytest
import torch

import synthetic
from oracle import spectrum as ospec
from paper_2106_12929_amd import spectrum as SP


@pytest.mark.parametrize("spatial", [(24, 20), (10, 12, 14)])
@pytest.mark.parametrize("cutoff", [1e-12, 3e-4])
def test_loss_gradient_matches_autograd_of_the_oracle_spectrum(spatial, cutoff):
    D = len(spatial)
    u = synthetic.random_normal((D,) + spatial, 91, 0.05)
    target = ospec.energy_spectrum(synthetic.random_normal((D,) + spatial, 92, 0.05))
    kmax = min(spatial) // 2
    uu = u.clone().requires_grad_(True)
    E = ospec.energy_spectrum(uu)
    a = torch.log(torch.clamp(E[1:kmax + 1], min=cutoff))
    b = torch.log(torch.clamp(target[1:kmax + 1], min=cutoff))
    R_ref = (a - b).square().sum()
    (g_ref,) = torch.autograd.grad(R_ref, uu)
    R, g = SP.log_spectrum_loss_and_grad(u, SP.shell_index(spatial, "cpu"), target, 1, kmax, cutoff)
    assert abs(float(R) - float(R_ref)) <= 1e-12 * float(R_ref)
    assert float((g - g_ref).abs().max()) <= 1e-12 * float(g_ref.abs().max())
    if cutoff > 1e-6:  # the case is meant to exercise the clamp
        assert int((E.detach()[1:kmax + 1] < cutoff).sum()) > 0
