"""GPU checks of the workloads built on the C ABI: captured HIP-graph replays of the
step, the flow-control restraint, and the adjoint-driven forcing optimisation."""
import pytest
import torch

import synthetic
from oracle import lbm as olbm

from _helpers import binding, bits, need_gpu, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("lat,shape,plan", [("D3Q27", (40, 12, 9), (10, 0, 0)), ("D3Q27", (64, 16, 9), (2, 4, 0)),
                                            ("D2Q9", (128, 16, 1), (2, 0, 2))])
def test_graph_replay_matches_eager(lat, shape, plan):
    """A captured 10-step lbm_step replayed three times, with eager work and
    synchronisations in between, reproduces the eager result every time: single
    steps, and two- and four-step launches (the launch plan is checked)."""
    need_gpu()
    B = binding()
    grid = B.Grid(lat, "f32", *shape)
    assert B.lbm_step_launches(grid, 10) == plan
    spatial = (shape[1], shape[0]) if lat == "D2Q9" else (shape[2], shape[1], shape[0])
    u = synthetic.random_fields(spatial, grid.D, 7, umax=0.05)[1].cuda()
    a, b = grid.empty_populations(), grid.empty_populations()
    B.lbm_init_equilibrium(grid, None, u, a)
    start = a.clone()
    # eager reference: 10, 20 and 30 steps
    refs = []
    x, y = start.clone(), grid.empty_populations()
    for _ in range(3):
        B.lbm_step(grid, x, y, 0.55, None, 10)  # even: result back in x
        refs.append(x.clone())
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            B.lbm_step(grid, a, b, 0.55, None, 10)
    torch.cuda.current_stream().wait_stream(s)
    a.copy_(start)
    for k in range(3):
        graph.replay()
        torch.cuda.synchronize()
        _ = (a.float().sum() + 1).item()  # eager work between replays
        assert torch.equal(bits(a), bits(refs[k])), k


def test_graph_replay_of_two_adjoint_steps_matches_eager():
    """Two collision-local adjoint steps per launch (with a force gradient) captured in
    a graph and replayed three times against eager launches: chi and the accumulated
    force gradient every time."""
    need_gpu()
    B = binding()
    grid = B.Grid("D3Q27", "f32", 64, 16, 9)
    spatial = (9, 16, 64)
    u = synthetic.random_fields(spatial, 3, 8, umax=0.05)[1].cuda()
    g0, g1 = grid.empty_populations(), grid.empty_populations()
    B.lbm_init_equilibrium(grid, None, u, g0)
    B.lbm_step(grid, g0, g1, 0.55, None, 1)
    F = synthetic.random_normal((3,) + spatial, 9, 1e-4).float().cuda()
    chi0 = synthetic.random_normal((27,) + spatial, 10).float()
    chi0 = grid.to_layout(chi0).cuda()
    refs = []
    x, y = chi0.clone(), torch.empty_like(chi0)
    dF = torch.zeros_like(F)
    for _ in range(3):
        B.lbm_adjoint_step2_local(grid, g1, g0, x, y, 0.55, F, dF)
        x, y = y, x
        refs.append((x.clone(), dF.clone()))
    a, b = chi0.clone(), torch.empty_like(chi0)
    dG = torch.zeros_like(F)
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            B.lbm_adjoint_step2_local(grid, g1, g0, a, b, 0.55, F, dG)
            B.lbm_copy(b, a)
    torch.cuda.current_stream().wait_stream(s)
    for k in range(3):
        graph.replay()
        torch.cuda.synchronize()
        _ = (a.float().sum() + 1).item()  # eager work between replays
        assert torch.equal(bits(a), bits(refs[k][0])), k
        assert torch.equal(bits(dG), bits(refs[k][1])), k


def test_resume_from_saved_state_is_bit_identical(tmp_path):
    """Save after 7 steps, run 9 more; a Simulation restored from the file and run 9
    steps (in two calls) reaches the same live words bit for bit (padded rows, FP16
    storage, a body force)."""
    need_gpu()
    B = binding()
    from paper_2106_12929_amd.simulation import Simulation

    grid = B.Grid.padded("D3Q27", "f16s", 40, 12, 9)
    u = synthetic.random_fields((9, 12, 40), 3, 17, umax=0.05)[1]
    F = synthetic.random_normal((3, 9, 12, 40), 18, 1e-5).to(grid.real_dtype).cuda()
    sim = Simulation(grid, 0.53, F)
    sim.init_equilibrium(u)
    sim.step(7)
    path = str(tmp_path / "state.safetensors")
    sim.save(path)
    sim.step(9)
    ref = grid.from_layout(sim.f).cpu()
    back = Simulation.restore(path)
    assert back.steps_done == 7 and back.grid == grid and back.tau == 0.53
    back.step(4)
    back.step(5)
    assert back.steps_done == 16
    assert torch.equal(bits(grid.from_layout(back.f).cpu()), bits(ref))


def test_flow_control_restrains_the_spectrum():
    need_gpu()
    binding()
    from paper_2106_12929_amd import workloads as WL

    u = synthetic.isotropic_turbulence(64, 4.0, 0.04, seed=1, dim=2, device="cuda")
    out = WL.flow_control_2d(u, 0.51, 400, kappa=5e-3, record_every=100)
    R_free = out["free"]["history"][-1][1]
    R_ctrl = out["restrained"]["history"][-1][1]
    say(f"flow control 64^2: R free {R_free:.3f}, restrained {R_ctrl:.3f}")
    assert R_ctrl < 0.25 * R_free


def test_flow_control_graph_matches_eager():
    """The restrained run replaying its captured two-step HIP graph (moments, FFT loss
    head, shifted step, twice) gives the eager run's R and kinetic-energy history bit
    for bit after every replay (each recorded eagerly, with a synchronisation, between
    the replays)."""
    need_gpu()
    binding()
    from paper_2106_12929_amd import workloads as WL

    u = synthetic.isotropic_turbulence(64, 4.0, 0.04, seed=2, dim=2, device="cuda")
    eager = WL.flow_control_2d(u, 0.51, 40, kappa=5e-3, record_every=2, graph=False)
    graphed = WL.flow_control_2d(u, 0.51, 40, kappa=5e-3, record_every=2, graph=True)
    assert graphed["graph"] and not eager["graph"]
    assert len(graphed["restrained"]["history"]) == 21
    assert graphed["restrained"]["history"] == eager["restrained"]["history"]
    assert graphed["free"]["history"] == eager["free"]["history"]
    # the restraint acts: R stays below the free run's
    assert graphed["restrained"]["history"][-1][1] < graphed["free"]["history"][-1][1]


def test_forcing_optimisation_lowers_the_loss():
    need_gpu()
    binding()
    from paper_2106_12929_amd import workloads as WL

    u = synthetic.isotropic_turbulence(32, 4.0, 0.05, seed=0, device="cuda")
    out = WL.forcing_optimisation(u, 0.51, steps=20, checkpoint_every=5, iters=6, lr=1e-5, k_band=(2, 8))
    say(f"forcing 32^3: loss {out['loss_first']:.4f} -> {out['loss_last']:.4f}")
    assert out["loss_last"] < out["loss_first"]
    assert out["loss_min"] < 0.95 * out["loss_first"]


def test_simulation_driver_and_copy():
    """The ping-pong driver (Listing 1's Simulation.step usage) against the oracle,
    and the reference copy."""
    need_gpu()
    B = binding()
    from paper_2106_12929_amd.simulation import Simulation
    from oracle import storage as ost

    st = olbm.stencil("D2Q9")
    grid = B.Grid("D2Q9", "f64", 24, 20)
    u = synthetic.taylor_green_2d(24, 20, 0.04)
    sim = Simulation(grid, 0.7)
    sim.init_equilibrium(u)
    sim.step(3)
    sim.step(4)
    assert sim.steps_done == 7
    ref = olbm.run(olbm.equilibrium(torch.ones(20, 24, dtype=torch.float64), u, st), 0.7, st, 7)
    assert float((grid.from_layout(sim.f.cpu()) - ref).abs().max()) < 1e-15
    rho, uu = sim.moments()
    r_ref, u_ref = olbm.state_moments(ref, st)
    assert float((uu.cpu() - u_ref).abs().max()) < 1e-15
    red = sim.reductions()
    assert abs(red["mass"] - float(r_ref.sum())) < 1e-10
    assert red["nonfinite_cells"] == 0.0
    x = torch.randn(1 << 20, device="cuda")
    y = torch.empty_like(x)
    B.lbm_copy(x, y)
    assert torch.equal(x, y)


def test_run_monitor_raises_on_non_finite_cells():
    """Failure detection forced from the host: a NaN planted in one population spreads
    through streaming and collision, and Simulation.run raises Diverged at its first
    check; a clean run of the same length returns finite reductions."""
    need_gpu()
    B = binding()
    from paper_2106_12929_amd.simulation import Diverged, Simulation

    grid = B.Grid("D3Q27", "f32", 20, 12, 10)
    u = synthetic.taylor_green_3d(20, 12, 10, 0.04)
    sim = Simulation(grid, 0.6)
    sim.init_equilibrium(u)
    red = sim.run(30, check_every=10)
    assert red["nonfinite_cells"] == 0 and sim.steps_done == 30
    sim.init_equilibrium(u)
    sim.f[3, 4, 13, 5] = float("nan")  # plane 3, row 4, rest direction, x = 5
    with pytest.raises(Diverged) as info:
        sim.run(30, check_every=10)
    assert info.value.steps_done == 10
    assert info.value.reductions["nonfinite_cells"] > 1


def test_gradient_precision_fp32_matches_fp64():
    """The FP32 adjoint's force gradient points where the FP64 one does (48^3, 50
    steps): cosine >= 0.999."""
    need_gpu()
    binding()
    from paper_2106_12929_amd import workloads as WL

    u = synthetic.isotropic_turbulence(48, 4.0, 0.05, seed=2, device="cuda")
    out = WL.gradient_precision(u, 0.51, steps=50, checkpoint_every=10, storages=("f64", "f32", "f16s"),
                                k_band=(2, 12))
    c32 = out["runs"]["f32"]["cosine_vs_f64"]
    c16 = out["runs"]["f16s"]["cosine_vs_f64"]
    say(f"gradient cosine vs f64: f32 {c32:.8f}, f16s {c16:.6f}")
    assert c32 >= 0.999
    assert c16 >= 0.9
