"""GPU parity of the hand-written adjoint (lbm_adjoint_step, lbm_moments_adjoint and
the checkpointed autograd rollout) against the oracle's autograd gradient and
finite differences of the GPU FP64 forward path."""
import pytest
import torch

import synthetic
from oracle import adjoint as oadj
from oracle import lbm as olbm
from oracle import spectrum as ospec
from oracle import storage as ost

from _helpers import binding, need_gpu, say

pytestmark = pytest.mark.gpu

CASES = [("D2Q9", (37, 9, 1)), ("D3Q27", (17, 13, 11)), ("D3Q27", (130, 5, 3)), ("D3Q19", (21, 6, 5))]


def _spatial(lat, shape):
    nx, ny, nz = shape
    return (ny, nx) if lat == "D2Q9" else (nz, ny, nx)


def _state(st, spatial, seed):
    rho, u = synthetic.random_fields(spatial, st.D, seed, drho=0.03, umax=0.06)
    return olbm.equilibrium(rho, u, st) * (1 + synthetic.random_normal((st.Q,) + spatial, seed + 1, 0.02))


@pytest.mark.parametrize("lat,shape", CASES)
@pytest.mark.parametrize("kind", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("forced", [False, True])
def test_adjoint_step_vs_oracle_autograd(lat, shape, kind, forced):
    need_gpu()
    B = binding()
    st = olbm.stencil(lat)
    spatial = _spatial(lat, shape)
    grid = B.Grid(lat, kind, *shape)
    tau = 0.56
    say(f"adjoint {lat} {kind} {shape} forced={forced}")
    s = ost.quantize(_state(st, spatial, 61), st, kind)
    g64 = ost.dequantize(s, st, kind)
    F = synthetic.random_normal((st.D,) + spatial, 62, 1e-4).to(grid.real_dtype) if forced else None
    lam = synthetic.random_normal((st.Q,) + spatial, 63).to(grid.real_dtype)
    lam_out = torch.empty(grid.population_shape(), dtype=grid.real_dtype, device="cuda")
    dF = torch.zeros_like(F, device="cuda") if forced else None
    if forced:
        dF += 0.25  # accumulation: the kernel adds to what is there
    B.lbm_adjoint_step(grid, grid.to_layout(s).cuda(), grid.to_layout(lam).cuda(), lam_out, tau,
                       None if F is None else F.cuda(), dF)
    ref, ref_dF = oadj.step_vjp(g64, lam.double(), tau, st, None if F is None else F.double())
    tol = 1e-13 if kind == "f64" else 2e-6
    err = float((grid.from_layout(lam_out.cpu()).double() - ref).abs().max() / ref.abs().max())
    say(f"  lambda rel err {err:.2e}")
    assert err < tol
    if forced:
        errF = float(((dF.cpu().double() - 0.25) - ref_dF).abs().max() / ref_dF.abs().max())
        say(f"  dF rel err {errF:.2e}")
        assert errF < (1e-12 if kind == "f64" else 1e-5)


@pytest.mark.parametrize("lat,shape", CASES[:2])
@pytest.mark.parametrize("forced", [False, True])
def test_adjoint_transposition_fd(lat, shape, forced):
    """<lam', J dg> by a central finite difference of the GPU FP64 forward step
    against <J^T lam', dg> from the GPU adjoint."""
    need_gpu()
    B = binding()
    st = olbm.stencil(lat)
    spatial = _spatial(lat, shape)
    grid = B.Grid(lat, "f64", *shape)
    tau = 0.56
    g = grid.to_layout(_state(st, spatial, 71)).cuda()
    F = synthetic.random_normal((st.D,) + spatial, 72, 1e-4).cuda() if forced else None
    lam = grid.to_layout(synthetic.random_normal((st.Q,) + spatial, 73)).cuda()
    dg = grid.to_layout(synthetic.random_normal((st.Q,) + spatial, 74, 1e-3)).cuda()
    eps = 1e-4

    def fwd(x, FF=F):
        out = torch.empty_like(x)
        B.lbm_step(grid, x.contiguous(), out, tau, FF, 1)
        return out

    jvp = (fwd(g + eps * dg) - fwd(g - eps * dg)) / (2 * eps)
    lam_out = torch.empty_like(lam)
    dF = torch.zeros_like(F) if forced else None
    B.lbm_adjoint_step(grid, g, lam, lam_out, tau, F, dF)
    lhs, rhs = float((lam * jvp).sum()), float((lam_out * dg).sum())
    say(f"transposition {lat} forced={forced}: {lhs:.12e} vs {rhs:.12e}")
    assert abs(lhs - rhs) <= 1e-8 * abs(rhs)
    if forced:
        dFdir = synthetic.random_normal((st.D,) + spatial, 75, 1e-4).cuda()
        jvpF = (fwd(g, F + eps * dFdir) - fwd(g, F - eps * dFdir)) / (2 * eps)
        lhs, rhs = float((lam * jvpF).sum()), float((dF * dFdir).sum())
        assert abs(lhs - rhs) <= 1e-8 * abs(rhs)


@pytest.mark.parametrize("lat,shape", CASES)
@pytest.mark.parametrize("kind", ["f64", "f32"])
@pytest.mark.parametrize("forced", [False, True])
def test_moments_adjoint_vs_oracle(lat, shape, kind, forced):
    need_gpu()
    B = binding()
    st = olbm.stencil(lat)
    spatial = _spatial(lat, shape)
    grid = B.Grid(lat, kind, *shape)
    s = ost.quantize(_state(st, spatial, 81), st, kind)
    F = synthetic.random_normal((st.D,) + spatial, 82, 1e-4).to(grid.real_dtype) if forced else None
    a = synthetic.random_normal(spatial, 83).to(grid.real_dtype)
    b = synthetic.random_normal((st.D,) + spatial, 84).to(grid.real_dtype)
    lam = torch.empty(grid.population_shape(), dtype=grid.real_dtype, device="cuda")
    dF = torch.zeros_like(F, device="cuda") if forced else None
    sd = grid.to_layout(s).cuda()
    B.lbm_moments_adjoint(grid, sd, None if F is None else F.cuda(), a.cuda(), b.cuda(), lam, dF)
    ref, ref_dF = oadj.moments_vjp(ost.dequantize(s, st, kind), st, None if F is None else F.double(),
                                   a.double(), b.double())
    tol = 1e-13 if kind == "f64" else 2e-6
    assert float((grid.from_layout(lam.cpu()).double() - ref).abs().max() / ref.abs().max()) < tol
    if forced:
        assert float((dF.cpu().double() - ref_dF).abs().max() / ref_dF.abs().max()) < tol
    # NULL cotangents mean zero
    B.lbm_moments_adjoint(grid, sd, None if F is None else F.cuda(), None, None, lam, None)
    assert float(lam.abs().max()) == 0.0


def _spectral_loss_fn(n, k_hi=3):
    K = torch.arange(n, dtype=torch.float64).clamp(min=1)
    target = 1e-4 * K ** (-5.0 / 3.0)
    return target, k_hi


def test_rollout_gradient_vs_oracle_autograd():
    """Whole differentiated rollout (8^3, 12 steps, checkpoint every 5) through the
    autograd wrapper and the GPU spectral loss head, against the oracle's autograd
    through its own steps and spectrum, in FP64."""
    need_gpu()
    B = binding()
    from paper_2106_12929_amd import autograd as AG
    from paper_2106_12929_amd import spectrum as gspec

    st = olbm.stencil("D3Q27")
    n, tau, T = 8, 0.6, 12
    u0 = synthetic.isotropic_turbulence(n, 2.0, 0.03, seed=3)
    g0 = olbm.equilibrium(torch.ones(n, n, n, dtype=torch.float64), u0, st)
    F = synthetic.random_normal((3, n, n, n), 91, 1e-4)
    target, k_hi = _spectral_loss_fn(n)

    def oracle_loss(rho, u):
        return ospec.log_spectrum_loss(ospec.energy_spectrum(u), target, 1, k_hi, 1e-14)

    L_ref, dg_ref, dF_ref = oadj.rollout_grad(g0, F, tau, st, T, oracle_loss)

    grid = B.Grid("D3Q27", "f64", n, n, n)
    g0d = grid.to_layout(g0).cuda().requires_grad_(True)
    Fd = F.cuda().requires_grad_(True)
    gT = AG.rollout(grid, g0d, Fd, tau, T, checkpoint_every=5)
    rho, u = AG.moments(grid, gT, Fd)
    L = gspec.log_spectrum_loss(gspec.energy_spectrum(u), target.cuda(), 1, k_hi, 1e-14)
    L.backward()
    say(f"rollout loss gpu {float(L):.12e} oracle {float(L_ref):.12e}")
    assert abs(float(L) - float(L_ref)) <= 1e-10 * abs(float(L_ref))
    eF = float((Fd.grad.cpu() - dF_ref).abs().max() / dF_ref.abs().max())
    eg = float((grid.from_layout(g0d.grad.cpu()) - dg_ref).abs().max() / dg_ref.abs().max())
    say(f"  dF rel err {eF:.2e}, dg0 rel err {eg:.2e}")
    assert eF < 1e-10 and eg < 1e-10


def test_rollout_gradient_fd_32cube():
    """FD check of dL/dF along a random direction: 32^3 FP64, 100 steps (the forced
    workload's reduced copy), checkpoint every 10."""
    need_gpu()
    B = binding()
    from paper_2106_12929_amd import autograd as AG
    from paper_2106_12929_amd import spectrum as gspec

    n, tau, T = 32, 0.51, 100
    grid = B.Grid("D3Q27", "f64", n, n, n)
    u0 = synthetic.isotropic_turbulence(n, 4.0, 0.05, seed=0).cuda()
    g0 = grid.empty_populations()
    B.lbm_init_equilibrium(grid, None, u0, g0)
    E0 = gspec.energy_spectrum(u0)
    K = torch.arange(E0.numel(), dtype=torch.float64, device="cuda").clamp(min=1)
    target = K ** (-5.0 / 3.0)
    target = target * E0[2:17].sum() / target[2:17].sum()
    cut = 1e-12 * float(E0.sum())

    def loss_of(F, grad=False):
        gT = AG.rollout(grid, g0, F, tau, T, checkpoint_every=10)
        _, u = AG.moments(grid, gT, F)
        return gspec.log_spectrum_loss(gspec.energy_spectrum(u), target, 2, 16, cut)

    F = torch.zeros((3, n, n, n), dtype=torch.float64, device="cuda", requires_grad=True)
    L = loss_of(F)
    L.backward()
    d = synthetic.random_normal((3, n, n, n), 92, 1.0).cuda()
    eps = 1e-8
    with torch.no_grad():
        Lp = float(loss_of(F + eps * d))
        Lm = float(loss_of(F - eps * d))
    fd = (Lp - Lm) / (2 * eps)
    an = float((F.grad * d).sum())
    say(f"FD {fd:.10e} adjoint {an:.10e}")
    assert abs(fd - an) <= 1e-6 * abs(an)


def test_checkpoint_invariance_bitwise():
    need_gpu()
    B = binding()
    from paper_2106_12929_amd import autograd as AG

    n, tau, T = 24, 0.51, 40
    grid = B.Grid("D3Q27", "f32", n, n, n)
    u0 = synthetic.isotropic_turbulence(n, 4.0, 0.05, seed=1).cuda()
    g0 = grid.empty_populations()
    B.lbm_init_equilibrium(grid, None, u0, g0)
    grads = []
    for K in (1, 7, 40, 100):
        F = torch.zeros((3, n, n, n), dtype=torch.float32, device="cuda", requires_grad=True)
        gT = AG.rollout(grid, g0, F, tau, T, checkpoint_every=K)
        _, u = AG.moments(grid, gT, F)
        (0.5 * (u.double() ** 2).sum()).backward()
        grads.append(F.grad.clone())
    for g in grads[1:]:
        assert torch.equal(g, grads[0])


@pytest.mark.parametrize("lat,shape", CASES)
@pytest.mark.parametrize("kind", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("forced", [False, True])
def test_local_form_chain_matches_scatter_form_bitwise(lat, shape, kind, forced):
    """Five adjoint steps in the collision-local form followed by one unstream give
    the same words as five scatter-form steps (the same arithmetic, stored at other
    addresses), and the same force gradient."""
    need_gpu()
    B = binding()
    st = olbm.stencil(lat)
    spatial = _spatial(lat, shape)
    grid = B.Grid(lat, kind, *shape)
    tau = 0.53
    say(f"local-form chain {lat} {kind} {shape} forced={forced}")
    states = [grid.to_layout(ost.quantize(_state(st, spatial, 100 + k), st, kind)).cuda() for k in range(5)]
    F = synthetic.random_normal((st.D,) + spatial, 120, 1e-4).to(grid.real_dtype).cuda() if forced else None
    lamT = grid.to_layout(synthetic.random_normal((st.Q,) + spatial, 121).to(grid.real_dtype)).cuda()
    # scatter form
    lam = lamT.clone()
    out = torch.empty_like(lam)
    dF1 = torch.zeros_like(F) if forced else None
    for t in reversed(range(5)):
        B.lbm_adjoint_step(grid, states[t], lam, out, tau, F, dF1)
        lam, out = out, lam
    # local form
    bufs = [torch.empty_like(lamT), torch.empty_like(lamT)]
    cur, is_chi = lamT.clone(), False
    dF2 = torch.zeros_like(F) if forced else None
    for k, t in enumerate(reversed(range(5))):
        B.lbm_adjoint_step_local(grid, states[t], cur, is_chi, bufs[k & 1], tau, F, dF2)
        cur, is_chi = bufs[k & 1], True
    lam2 = torch.empty_like(lamT)
    B.lbm_adjoint_unstream(grid, cur, lam2)
    assert torch.equal(lam, lam2)
    if forced:
        assert torch.equal(dF1, dF2)


@pytest.mark.parametrize("kind,forced,n,tuned", [("f32", False, 256, False), ("f16s", False, 256, False),
                                                 ("f32", True, 256, False), ("f16s", True, 256, False),
                                                 ("f16s", True, 512, False), ("f16s", True, 512, True)])
def test_full_size_local_adjoint_sampled(kind, forced, n, tuned):
    """The collision-local adjoint step on the 256^3 D3Q27 grid the benchmark times (and
    at 512^3, the full-scale workload's size with an f16s state and a force), in
    its launch shape (chi input): chi_out(x) = J_C(h(x))^T lam'(x) with h(x) the gathered
    state and lam'_i(x) = chi_i(x + c_i), against the VJP of the oracle's collision at
    4096 sampled cells and the 8 corners; with a force, also dF there.  The tuned case
    takes Grid.tuned's 576-word rows, as the 512^3 workload does."""
    need_gpu()
    B = binding()
    st = olbm.stencil("D3Q27")
    Q, tau = 27, 0.51
    grid = B.Grid.tuned("D3Q27", kind, n, n, n) if tuned else B.Grid("D3Q27", kind, n, n, n)
    p = grid.row_pitch
    say(f"full-size local adjoint {kind} {n}^3 forced={forced} pitch {p}")
    a, b = grid.empty_populations(), grid.empty_populations()
    B.lbm_init_equilibrium(grid, None, synthetic.taylor_green_3d_on("cuda", n, n, n, 0.05), a)
    B.lbm_step(grid, a, b, tau, None, 2)  # non-equilibrium state in a
    del b
    gen = torch.Generator(device="cuda").manual_seed(64)
    chi = torch.randn(grid.population_shape(), generator=gen, device="cuda", dtype=torch.float32)
    F = (1e-4 * torch.randn((3, n, n, n), generator=gen, device="cuda")) if forced else None
    dF = torch.zeros_like(F) if forced else None
    out = torch.empty_like(chi)
    B.lbm_adjoint_step_local(grid, a, chi, True, out, tau, F, dF)
    torch.cuda.synchronize()
    cg = torch.Generator().manual_seed(65)
    cells = torch.cat([torch.randint(0, n, (4096, 3), generator=cg),
                       torch.tensor([[x, y, z] for x in (0, n - 1) for y in (0, n - 1) for z in (0, n - 1)])])
    x, y, z = (cells[:, k].cuda() for k in range(3))

    def word(i, dx, dy, dz):  # flat index of direction i at (x + dx, y + dy, z + dz), periodic
        return ((((z + dz) % n) * n + (y + dy) % n) * Q + i) * p + (x + dx) % n

    c = st.c.to(torch.int64)
    h = torch.stack([a.view(-1)[word(i, -c[i, 0], -c[i, 1], -c[i, 2])] for i in range(Q)]).cpu().double()
    if kind == "f16s":
        h = h + st.w.reshape(Q, 1)
    lam = torch.stack([chi.view(-1)[word(i, c[i, 0], c[i, 1], c[i, 2])] for i in range(Q)]).cpu().double()
    got = torch.stack([out.view(-1)[word(i, 0, 0, 0)] for i in range(Q)]).cpu().double()
    hh = h.requires_grad_(True)
    inputs = [hh]
    Fc = None
    if forced:
        flat = ((z * n + y) * n + x)
        Fc = torch.stack([F[k].reshape(-1)[flat] for k in range(3)]).cpu().double().requires_grad_(True)
        inputs.append(Fc)
    grads = torch.autograd.grad(olbm.bgk_collide(hh, tau, st, Fc), inputs, grad_outputs=lam)
    err = float((got - grads[0]).abs().max() / grads[0].abs().max())
    say(f"  chi rel err {err:.2e}")
    assert err < 2e-6
    if forced:
        gotF = torch.stack([dF[k].reshape(-1)[flat] for k in range(3)]).cpu().double()
        errF = float((gotF - grads[1]).abs().max() / grads[1].abs().max())
        say(f"  dF rel err {errF:.2e}")
        assert errF < 1e-5
