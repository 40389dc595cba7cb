"""GPU checks of the flow-control loss head (lbm_shell_energy, lbm_log_spectrum_grad,
lbm_real_part behind spectrum.NativeLossHead) against the oracle: the shell spectrum
(Sec. 3.1 reading) against the oracle's scatter-add spectrum, the log-spectrum cost
(Sec. 3.2 reading) against the oracle's, and the gradient against autograd through the
oracle's spectrum on the CPU."""
import pytest
import torch

import synthetic
from oracle import spectrum as ospec

from _helpers import binding, need_gpu, say

pytestmark = pytest.mark.gpu


def _field(spatial, seed):
    D = len(spatial)
    return synthetic.random_normal((D,) + spatial, seed, 0.05)


@pytest.mark.parametrize("spatial", [(48, 40), (33, 30), (12, 10, 14)], ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("cut_quantile", [0.0, 0.5])
def test_native_loss_head_matches_oracle(spatial, cut_quantile):
    need_gpu()
    binding()
    from paper_2106_12929_amd import spectrum as SP

    say(f"loss head {spatial} cut quantile {cut_quantile}")
    u = _field(spatial, 5)
    target_field = _field(spatial, 6)
    E_ref = ospec.energy_spectrum(u)
    Et = ospec.energy_spectrum(target_field)
    # a cutoff that switches off some shells (the flat part of the clamp) or none
    c = float(torch.quantile(E_ref[1:], cut_quantile)) if cut_quantile > 0 else 1e-30
    k_lo, k_hi = 1, E_ref.numel() - 2
    # oracle: R and dR/du by autograd through the oracle's spectrum (FP64, CPU)
    uo = u.clone().requires_grad_(True)
    R_ref = ospec.log_spectrum_loss(ospec.energy_spectrum(uo), Et, k_lo, k_hi, c)
    R_ref.backward()
    g_ref = uo.grad

    shells = SP.shell_index(spatial, "cuda")
    head = SP.NativeLossHead(shells, Et.cuda(), k_lo, k_hi, c)
    out = torch.empty((len(spatial),) + spatial, dtype=torch.float64, device="cuda")
    head.scaled_grad(u.cuda(), 1.0, out, with_cost=True)
    E = head.E.cpu()
    assert E.numel() == E_ref.numel()
    assert float((E - E_ref).abs().max()) <= 1e-13 * float(E_ref.max())
    assert abs(float(head.R.cpu()) - float(R_ref)) <= 1e-11 * max(1.0, float(R_ref))
    scale = float(g_ref.abs().max())
    assert scale > 0
    assert float((out.cpu() - g_ref).abs().max()) <= 1e-10 * scale
    # the FP32 output is the FP64 one rounded
    out32 = torch.empty_like(out, dtype=torch.float32)
    head.scaled_grad(u.cuda(), -3.0, out32)
    assert torch.equal(out32.cpu(), (-3.0 * out.cpu()).to(torch.float32))


def test_native_loss_head_matches_torch_head():
    """The native head and the torch closed-form head (log_spectrum_loss_and_grad) give
    the same R and gradient to rounding, on the flow-control shape."""
    need_gpu()
    binding()
    from paper_2106_12929_amd import spectrum as SP

    u = synthetic.isotropic_turbulence(128, 4.0, 0.04, seed=3, dim=2, device="cuda").to(torch.float32)
    shells = SP.shell_index((128, 128), "cuda")
    # the synthetic turbulence prescribes its spectrum: a target with another peak
    # wavenumber, so that R is of order one
    Et = SP.energy_spectrum(synthetic.isotropic_turbulence(128, 9.0, 0.04, seed=4, dim=2, device="cuda"), shells)
    R_t, g_t = SP.log_spectrum_loss_and_grad(u, shells, Et, 1, 64, 2e-5)
    head = SP.NativeLossHead(shells, Et, 1, 64, 2e-5)
    out = torch.empty((2, 128, 128), dtype=torch.float64, device="cuda")
    head.scaled_grad(u, 1.0, out, with_cost=True)
    assert float(R_t) > 1.0
    assert abs(float(head.R) - float(R_t)) <= 1e-11 * float(R_t)
    assert float((out - g_t).abs().max()) <= 1e-10 * float(g_t.abs().max())



def test_flow_control_step_at_workload_size():
    """The flow-control configuration itself (D2Q9 FP32, 128^2, tau 0.5018, the paper's
    kappa and cutoff): the native loss head's shift du = -kappa dR/du against autograd
    through the oracle's spectrum, then lbm_step_shifted with that shift against the
    oracle's shifted step on the whole grid."""
    need_gpu()
    B = binding()
    from oracle import lbm as olbm
    from oracle import storage as ost
    from paper_2106_12929_amd import spectrum as SP
    from test_gpu_forward import _tolerance_ok

    n, tau, kappa, cutoff = 128, 0.5018, 5e-5, 2e-5
    st = olbm.stencil("D2Q9")
    grid = B.Grid("D2Q9", "f32", n, n)
    u0 = synthetic.isotropic_turbulence(n, 4.0, 0.04, seed=0, dim=2, device="cpu").double()
    s = ost.quantize(olbm.equilibrium(torch.ones((n, n), dtype=torch.float64), u0, st), st, "f32")
    _, u = olbm.state_moments(ost.dequantize(s, st, "f32"), st, None)
    u32 = u.to(torch.float32)
    target = ospec.energy_spectrum(_field((n, n), 9))
    kmax = n // 2
    # oracle shift: autograd through the oracle's spectrum and cost, at the FP32 field
    uo = u32.double().clone().requires_grad_(True)
    ospec.log_spectrum_loss(ospec.energy_spectrum(uo), target, 1, kmax, cutoff).backward()
    du_ref = -kappa * uo.grad
    head = SP.NativeLossHead(SP.shell_index((n, n), "cuda"), target.cuda(), 1, kmax, cutoff)
    du = torch.empty((2, n, n), dtype=torch.float32, device="cuda")
    head.scaled_grad(u32.cuda(), -kappa, du)
    du_cpu = du.cpu().double()
    assert float((du_cpu - du_ref).abs().max()) <= 1e-6 * float(du_ref.abs().max())  # FP32 output
    out = grid.empty_populations()
    assert B.lbm_step_shifted(grid, grid.to_layout(s).cuda(), out, tau, du, 1) == 0
    ref = ost.step_emulated(s, tau, st, "f32", du=du_cpu)
    excess, ratio, same = _tolerance_ok("f32", st, grid.from_layout(out.cpu()), ref, tau)
    say(f"flow-control step 128^2: max err / bound = {ratio:.3f}, bit-identical fraction = {same:.4f}")
    assert excess <= 0, ratio
