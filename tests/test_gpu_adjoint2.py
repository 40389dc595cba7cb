"""Two adjoint steps per launch (lbm_adjoint_step2_local).

The kernel chains two collision-local adjoint steps (Sec. 3.2) with the intermediate
chi on chip.  Each cell's arithmetic is that of lbm_adjoint_step_local, applied to the
same values, and the force gradient is added in the order of two one-step calls, so
chi and the force gradient must equal two one-step launches bit for bit.  The one-step
launches are tied to the oracle's autograd gradient by the adjoint tests; the rollout
test here ties the paired backward pass to the one-step backward pass bit for bit, and
the last test ties it to the oracle directly.

Shapes: one tile (every neighbour wraps onto the tile itself), several tiles in x and
y, the smallest nz (3), odd nz with a ragged last z chunk, padded rows, D3Q19.
"""
import pytest
import torch

import synthetic
from oracle import adjoint as oadj
from oracle import lbm as olbm
from oracle import storage as ost

from _helpers import binding, bits, need_gpu, say

pytestmark = pytest.mark.gpu

CASES = [  # lattice, (nx, ny, nz), pitch (None = nx)
    ("D3Q27", (32, 8, 3), None),
    ("D3Q27", (64, 16, 20), None),
    ("D3Q27", (96, 24, 37), None),
    ("D3Q27", (32, 40, 5), 96),
    ("D3Q19", (64, 16, 11), None),
    ("D3Q19", (32, 8, 4), 64),
    ("D3Q27", (128, 16, 5), None),
]


def _spatial(st, shape):
    nx, ny, nz = shape
    return (ny, nx) if st.D == 2 else (nz, ny, nx)


def _state(st, spatial, seed, kind):
    rho, u = synthetic.random_fields(spatial, st.D, seed, drho=0.03, umax=0.06)
    f = olbm.equilibrium(rho, u, st) * (1 + synthetic.random_normal((st.Q,) + spatial, seed + 1, 0.02))
    return ost.quantize(f, st, kind)


def _inputs(B, lat, shape, pitch, kind, mode, seed=41):
    st = olbm.stencil(lat)
    spatial = _spatial(st, shape)
    grid = B.Grid(lat, kind, *shape, pitch)
    gt = grid.to_layout(_state(st, spatial, seed, kind)).cuda()
    gtm1 = grid.to_layout(_state(st, spatial, seed + 2, kind)).cuda()
    chi = grid.to_layout(synthetic.random_normal((st.Q,) + spatial, seed + 4).to(grid.real_dtype)).cuda()
    F = dF = None
    if mode != "none":
        F = synthetic.random_normal((st.D,) + spatial, seed + 5, 1e-4).to(grid.real_dtype).cuda()
    if mode == "grad":
        dF = synthetic.random_normal((st.D,) + spatial, seed + 6, 1e-3).to(grid.real_dtype).cuda()
    return grid, gt, gtm1, chi, F, dF


def _two_singles(B, grid, gt, gtm1, chi, tau, F, dF):
    tmp = torch.zeros_like(chi)
    out = torch.zeros_like(chi)
    B.lbm_adjoint_step_local(grid, gt, chi, True, tmp, tau, F, dF)
    B.lbm_adjoint_step_local(grid, gtm1, tmp, True, out, tau, F, dF)
    return out


@pytest.mark.parametrize("lat,shape,pitch", CASES)
@pytest.mark.parametrize("kind", ["f32", "f32s", "f16s", "bf16s"])
@pytest.mark.parametrize("mode", ["none", "force", "grad"])
def test_two_adjoint_steps_equal_single_steps(lat, shape, pitch, kind, mode):
    need_gpu()
    B = binding()
    say(f"two adjoint steps {lat} {shape} pitch {pitch} {kind} {mode}")
    grid, gt, gtm1, chi, F, dF = _inputs(B, lat, shape, pitch, kind, mode)
    assert B.lbm_adjoint_step2_available(grid)
    tau = 0.56
    dF_ref = None if dF is None else dF.clone()
    ref = _two_singles(B, grid, gt, gtm1, chi, tau, F, dF_ref)
    out = torch.zeros_like(chi)
    B.lbm_adjoint_step2_local(grid, gt, gtm1, chi, out, tau, F, dF)
    torch.cuda.synchronize()
    assert torch.equal(bits(grid.from_layout(out.cpu())), bits(grid.from_layout(ref.cpu())))
    if dF is not None:
        assert torch.equal(bits(dF.cpu()), bits(dF_ref.cpu()))


def test_two_adjoint_steps_reject_other_grids():
    """Grids off the tile grid and FP64 storage raise instead of running another path."""
    need_gpu()
    B = binding()
    for lat, kind, shape in (("D3Q27", "f32", (48, 16, 6)), ("D3Q27", "f64", (32, 8, 6)),
                             ("D3Q27", "f32", (32, 8, 2)), ("D2Q9", "f32", (64, 16, 1))):
        grid = B.Grid(lat, kind, *shape)
        assert not B.lbm_adjoint_step2_available(grid)
        g = grid.empty_populations()
        c = torch.zeros(grid.population_shape(), dtype=grid.real_dtype, device="cuda")
        with pytest.raises(RuntimeError):
            B.lbm_adjoint_step2_local(grid, g, g, c, torch.zeros_like(c), 0.6)


@pytest.mark.parametrize("kind,mode,n,tuned", [("f32", "grad", 256, False), ("f16s", "none", 256, False),
                                               ("f16s", "grad", 512, True)])
def test_two_adjoint_steps_full_size(kind, mode, n, tuned):
    """256^3, and 512^3 on the rows of the full-scale adjoint workload (Grid.tuned, FP16
    state, force gradient), in the launch shape the rollout uses (tiles of 32 x 8
    columns, the z chunks the occupancy gives): every word of chi and of the force
    gradient compared with two one-step launches."""
    need_gpu()
    B = binding()
    grid = B.Grid.tuned("D3Q27", kind, n, n, n) if tuned else B.Grid("D3Q27", kind, n, n, n)
    say(f"two adjoint steps full size {kind} {mode} {n}^3 pitch {grid.row_pitch}")
    u = synthetic.taylor_green_3d_on("cuda", n, n, n, 0.05)
    gtm1 = grid.empty_populations()
    B.lbm_init_equilibrium(grid, None, u, gtm1)
    del u
    F = dF = None
    if mode == "grad":
        F = torch.full((3, n, n, n), 1e-5, dtype=grid.real_dtype, device="cuda")
        dF = torch.zeros_like(F)
    gt = grid.empty_populations()
    assert B.lbm_step(grid, gtm1, gt, 0.51, F, 1) == 0  # a non-equilibrium state
    chi = torch.empty(grid.population_shape(), dtype=grid.real_dtype, device="cuda")
    chi.copy_(gt.to(grid.real_dtype) if kind == "f32" else torch.ones_like(chi))
    dF_ref = None if dF is None else dF.clone()
    ref = _two_singles(B, grid, gt, gtm1, chi, 0.51, F, dF_ref)
    out = torch.empty_like(chi)
    B.lbm_adjoint_step2_local(grid, gt, gtm1, chi, out, 0.51, F, dF)
    torch.cuda.synchronize()
    assert torch.equal(bits(grid.from_layout(out)), bits(grid.from_layout(ref)))
    if dF is not None:
        assert torch.equal(bits(dF), bits(dF_ref))


@pytest.mark.parametrize("kind,K", [("f32", 4), ("f32", 3), ("f16s", 5)])
def test_rollout_backward_paired_equals_single_steps(kind, K):
    """The rollout's backward pass with two adjoint steps per launch (within each
    checkpoint segment) against the same backward pass with one step per launch:
    the input gradient and the force gradient, bit for bit.  K = 3 and 5 leave
    segments of odd length (a single step at each segment's end)."""
    need_gpu()
    B = binding()
    from paper_2106_12929_amd import autograd as AG

    lat, shape = "D3Q27", (64, 16, 9)
    st = olbm.stencil(lat)
    spatial = _spatial(st, shape)
    grid = B.Grid(lat, kind, *shape)
    say(f"rollout backward paired {kind} K={K}")
    g0 = grid.to_layout(_state(st, spatial, 51, kind)).cuda()
    F0 = synthetic.random_normal((st.D,) + spatial, 52, 1e-4).to(grid.real_dtype).cuda()
    w = grid.to_layout(synthetic.random_normal((st.Q,) + spatial, 53).to(grid.real_dtype)).cuda()
    grads = []
    for pair in (False, True):
        g = g0.clone()
        if kind == "f32":
            g.requires_grad_(True)
        F = F0.clone().requires_grad_(True)
        out = AG.LBMRollout.apply(g, F, grid, 0.56, 11, K, pair)
        (out.to(grid.real_dtype) * w).sum().backward()
        grads.append((g.grad.clone() if kind == "f32" else None, F.grad.clone()))
    (ga, fa), (gb, fb) = grads
    if ga is not None:
        assert torch.equal(bits(ga), bits(gb))
    assert torch.equal(bits(fa), bits(fb))


def test_paired_rollout_gradient_vs_oracle():
    """A 12-step rollout on 32 x 8 x 6 cells (FP32 storage, two adjoint steps per launch,
    checkpoint every 4) and a linear loss of the final moments: the gradients with
    respect to the initial state and the force against the oracle's autograd (FP64)."""
    need_gpu()
    B = binding()
    from paper_2106_12929_amd import autograd as AG

    lat, shape = "D3Q27", (32, 8, 6)
    st = olbm.stencil(lat)
    spatial = _spatial(st, shape)
    grid = B.Grid(lat, "f32", *shape)
    assert B.lbm_adjoint_step2_available(grid)
    tau, steps = 0.56, 12
    f0 = _state(st, spatial, 57, "f32")
    F0 = synthetic.random_normal((st.D,) + spatial, 58, 1e-4).float().double()
    wr = synthetic.random_normal(spatial, 59)
    wu = synthetic.random_normal((st.D,) + spatial, 60)
    L_ref, dg_ref, dF_ref = oadj.rollout_grad(ost.dequantize(f0, st, "f32"), F0, tau, st, steps,
                                              lambda rho, u: (rho * wr).sum() + (u * wu).sum())
    g = grid.to_layout(f0).cuda().requires_grad_(True)
    F = F0.float().cuda().requires_grad_(True)
    out = AG.LBMRollout.apply(g, F, grid, tau, steps, 4, True)
    rho, u = AG.moments(grid, out, F)
    L = (rho.double() * wr.cuda()).sum() + (u.double() * wu.cuda()).sum()
    L.backward()
    eF = float((F.grad.cpu().double() - dF_ref).abs().max() / dF_ref.abs().max())
    eg = float((grid.from_layout(g.grad.cpu()).double() - dg_ref).abs().max() / dg_ref.abs().max())
    say(f"  loss gpu {float(L):.8e} oracle {float(L_ref):.8e}; dF rel err {eF:.2e}, dg0 rel err {eg:.2e}")
    assert abs(float(L) - float(L_ref)) <= 1e-5 * abs(float(L_ref))
    assert eF < 1e-4 and eg < 1e-4


def test_paired_rollout_on_padded_rows_matches_dense():
    """The paired backward pass on padded rows (pitch 64 for 32 cells): loss, force
    gradient and state gradient equal the dense layout's bit for bit, and the state
    gradient's pad entries stay zero (the two-step adjoint writes live cells only)."""
    need_gpu()
    B = binding()
    from paper_2106_12929_amd import autograd as AG

    st = olbm.stencil("D3Q27")
    shape = (32, 8, 5)
    spatial = _spatial(st, shape)
    dense = B.Grid("D3Q27", "f32", *shape)
    pitched = B.Grid("D3Q27", "f32", *shape, 64)
    assert B.lbm_adjoint_step2_available(dense) and B.lbm_adjoint_step2_available(pitched)
    s = _state(st, spatial, 71, "f32")
    F0 = synthetic.random_normal((st.D,) + spatial, 72, 1e-4).float().cuda()
    out = []
    for grid in (dense, pitched):
        say(f"paired rollout, row pitch {grid.row_pitch}")
        g0 = grid.to_layout(s).cuda().requires_grad_(True)
        F = F0.clone().requires_grad_(True)
        gT = AG.rollout(grid, g0, F, 0.57, 9, checkpoint_every=4)
        rho, u = AG.moments(grid, gT, F)
        loss = (u.double() ** 2).sum() + (rho.double() - 1).pow(2).sum()
        loss.backward()
        out.append((loss.detach(), F.grad, g0.grad))
    (l0, f0, s0), (l1, f1, s1) = out
    assert torch.equal(bits(l0), bits(l1))
    assert torch.equal(bits(f0), bits(f1))
    assert torch.equal(bits(pitched.from_layout(s1.cpu())), bits(dense.from_layout(s0.cpu())))
    assert bool((s1.view(5 * 8, 27, 64)[:, :, 32:] == 0).all())
