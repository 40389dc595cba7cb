"""The three GPU workloads beyond the forward roofline run, built on the C ABI:

* `precision_study`: decaying isotropic turbulence (the paper's second flow,
  Sec. 3.1) on D3Q27 with shifted FP16/BF16 storage next to FP32 and FP64: the error
  of the kinetic energy, of the shell spectrum and of the velocity field against the
  FP64 run.
* `forcing_optimisation`: a per-cell body force (Guo scheme) optimised through the
  hand-written adjoint so that the shell spectrum after a rollout matches a target
  E(k) ~ k^-5/3 on a band of shells (the spectrum-holding flow control of Sec. 3.2,
  with a learnable force field in place of the velocity shift).
* `full_scale_adjoint`: a long FP16-shifted forward run at full HBM scale, then the
  checkpointed adjoint over its last steps; reports throughput and peak memory.
* `stability_study`: where and when a long forward run first speeds up beyond a
  threshold, per storage format (attribution of a BGK blow-up).
* `flow_control_2d`: the paper's own flow control (Sec. 3.2): every step the
  equilibrium is taken at u + du with du = -kappa grad_u R(u), R the log-spectrum
  deviation from the initial spectrum with cut-off c; a free run alongside.

Everything runs on the current GPU; inputs come from `synthetic`.
"""
from __future__ import annotations

import time

import torch

from . import autograd as AG
from . import binding as B
from . import spectrum as SP


def _sync_time(t0):
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def _reductions(grid, f):
    red = torch.zeros(B.NRED, dtype=torch.float64, device=f.device)
    ws = torch.empty(B.lbm_moments_workspace_size(grid), dtype=torch.uint8, device=f.device)
    B.lbm_moments(grid, f, None, None, None, red, ws)
    return dict(zip(B.RED_NAMES, red.cpu().tolist()))


def precision_study(u0: torch.Tensor, tau: float, steps: int, storages=("f64", "f32", "f16s", "bf16s"),
                    check_every: int = 250):
    """Runs the same initial field in each storage format; returns per-format
    throughput, kinetic-energy history and errors against the FP64 run.

    A run stops early when the reductions report non-finite cells (BGK blow-up); its
    `blew_up_at` gives the step.  Errors are only computed for runs that finished
    while the FP64 reference also finished."""
    n = u0.shape[-1]
    out = {"grid": [n, n, n], "tau": tau, "steps": steps, "runs": {}}
    ref = None
    shells = SP.shell_index((n, n, n), u0.device)
    for storage in storages:
        grid = B.Grid.tuned("D3Q27", storage, n, n, n)
        a, b = grid.empty_populations(), grid.empty_populations()
        B.lbm_init_equilibrium(grid, None, u0, a)
        ke_hist = []
        blew_up_at = None
        t_run = 0.0
        done = 0
        while done < steps:
            k = min(check_every, steps - done)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            where = B.lbm_step(grid, a, b, tau, None, k)
            t_run += _sync_time(t0)
            if where == 0:
                a, b = b, a
            done += k
            red = _reductions(grid, a)
            ke_hist.append((done, red["kinetic_energy"]))
            if red["nonfinite_cells"] > 0 or red["max_speed"] > 1.0:
                blew_up_at = done
                break
        run = {"mlups": n ** 3 * done / t_run / 1e6, "kinetic_energy": ke_hist, "blew_up_at": blew_up_at}
        if blew_up_at is None:
            u = grid.empty_real(3)
            B.lbm_moments(grid, a, None, None, u)
            u = u.double()
            E = SP.energy_spectrum(u, shells)
            if storage == storages[0]:
                ref = {"u": u, "E": E, "ke": dict(ke_hist)}
            elif ref is not None:
                kmax = n // 2
                rel_E = ((E[1:kmax] - ref["E"][1:kmax]).abs() / ref["E"][1:kmax]).cpu()
                ke_ref = ref["ke"][ke_hist[-1][0]]
                run.update({
                    "u_rel_l2": float((u - ref["u"]).norm() / ref["u"].norm()),
                    "ke_rel_err_final": abs(ke_hist[-1][1] - ke_ref) / ke_ref,
                    "ke_rel_err_max": max(abs(k - ref["ke"][t]) / ref["ke"][t] for t, k in ke_hist),
                    "spectrum_rel_err_max": float(rel_E.max()),
                    "spectrum_rel_err_median": float(rel_E.median()),
                })
            del u
        del a, b
        out["runs"][storage] = run
        torch.cuda.empty_cache()
    return out


def forcing_optimisation(u0: torch.Tensor, tau: float, steps: int = 100, checkpoint_every: int = 10,
                         iters: int = 30, lr: float = 1e-5, k_band=(2, 16)):
    """Adam on a per-cell force field F (FP32, constant in time, starting at zero) so
    that the shell spectrum after `steps` steps matches A k^-5/3 on k_band, with A
    matching the band energy of the initial spectrum.  Loss:
    sum_k (ln max(E,c) - ln max(E_t,c))^2 in FP64, c = 1e-12 E_total(0)."""
    n = u0.shape[-1]
    grid = B.Grid("D3Q27", "f32", n, n, n)
    g0 = grid.empty_populations()
    B.lbm_init_equilibrium(grid, None, u0, g0)
    shells = SP.shell_index((n, n, n), u0.device)
    E0 = SP.energy_spectrum(u0.double(), shells)
    K = torch.arange(E0.numel(), dtype=torch.float64, device=u0.device).clamp(min=1)
    lo, hi = k_band
    target = K ** (-5.0 / 3.0)
    target = target * E0[lo:hi + 1].sum() / target[lo:hi + 1].sum()
    cut = 1e-12 * float(E0.sum())
    F = torch.zeros((3, n, n, n), dtype=torch.float32, device=u0.device, requires_grad=True)
    opt = torch.optim.Adam([F], lr=lr)
    losses, times = [], []
    for it in range(iters):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        opt.zero_grad()
        gT = AG.rollout(grid, g0, F, tau, steps, checkpoint_every)
        _, u = AG.moments(grid, gT, F)
        L = SP.log_spectrum_loss(SP.energy_spectrum(u, shells), target, lo, hi, cut)
        L.backward()
        opt.step()
        times.append(_sync_time(t0))
        losses.append(float(L))
    # cell updates per iteration: forward rollout + replay + adjoint
    per_iter_s = sorted(times)[len(times) // 2]
    return {"grid": [n, n, n], "tau": tau, "steps": steps, "checkpoint_every": checkpoint_every, "iters": iters,
            "lr": lr, "loss_first": losses[0], "loss_last": losses[-1], "loss_min": min(losses),
            "loss_curve": losses, "seconds_per_iteration": per_iter_s,
            "forward_plus_backward_mlups": n ** 3 * steps / per_iter_s / 1e6,
            "max_abs_force": float(F.detach().abs().max())}


def stability_study(u0: torch.Tensor, tau: float, storage: str, steps: int, check_every: int = 25,
                    pitch: int | None = None, threshold: float = 0.2):
    """A forward run that records, every `check_every` steps, the kinetic energy, the
    largest speed and the cell where it occurs, with that cell's row offset in bytes in
    the population buffer; and the first check at which the largest speed passes
    `threshold`.  It tells a blow-up caused by the storage format from one tied to the
    addressing (row ends, high planes, words beyond 4 GiB of the buffer).  Rows take
    Grid.tuned's pitch unless `pitch` is given; the run stops at non-finite cells."""
    n = u0.shape[-1]
    grid = (B.Grid.tuned("D3Q27", storage, n, n, n) if pitch is None
            else B.Grid("D3Q27", storage, n, n, n, pitch))
    a, b = grid.empty_populations(), grid.empty_populations()
    B.lbm_init_equilibrium(grid, None, u0, a)
    word = a.element_size()
    hist, first_over = [], None
    done, t_run = 0, 0.0
    u = grid.empty_real(3)
    while done < steps:
        k = min(check_every, steps - done)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if B.lbm_step(grid, a, b, tau, None, k) == 0:
            a, b = b, a
        t_run += _sync_time(t0)
        done += k
        red = torch.zeros(B.NRED, dtype=torch.float64, device=u0.device)
        ws = torch.empty(B.lbm_moments_workspace_size(grid), dtype=torch.uint8, device=u0.device)
        B.lbm_moments(grid, a, None, None, u, red, ws)
        red = dict(zip(B.RED_NAMES, red.cpu().tolist()))
        speed2 = (u.double() ** 2).sum(dim=0)
        flat = int(torch.argmax(speed2))
        z, y, x = flat // (n * n), (flat // n) % n, flat % n
        row_bytes = ((z * n + y) * grid.Q) * grid.row_pitch * word
        rec = [done, red["kinetic_energy"], red["max_speed"], x, y, z, row_bytes]
        hist.append(rec)
        del speed2
        if first_over is None and red["max_speed"] > threshold:
            first_over = {"step": done, "max_speed": red["max_speed"], "cell_xyz": [x, y, z],
                          "row_byte_offset": row_bytes, "beyond_4GiB": row_bytes >= 1 << 32}
        if red["nonfinite_cells"] > 0:
            break
    out = {"grid": [n, n, n], "storage": storage, "tau": tau, "row_pitch": grid.row_pitch, "steps": done,
           "mlups": n ** 3 * done / t_run / 1e6, "buffer_bytes": a.numel() * word,
           "history_step_ke_maxspeed_xyz_rowbytes": hist, "first_over_threshold": first_over,
           "threshold": threshold}
    del a, b, u
    torch.cuda.empty_cache()
    return out


def full_scale_adjoint(u0: torch.Tensor, tau: float, forward_steps: int = 500, adjoint_steps: int = 50,
                       checkpoint_every: int = 10, pitch: int | None = None):
    """FP16-shifted forward run, then the gradient of the final kinetic energy
    1/2 sum |u|^2 with respect to the state `adjoint_steps` steps before the end and
    a zero force field active over those steps.

    Freed memory stays in torch's cache (no empty_cache) between calls: handing the
    ~185 GB of one call back to the driver and mapping it again made the next call's
    backward about 4x slower (same results), so repeated calls reuse the cached blocks.
    The populations take Grid.tuned's row pitch unless `pitch` is given."""
    n = u0.shape[-1]
    grid = B.Grid.tuned("D3Q27", "f16s", n, n, n) if pitch is None else B.Grid("D3Q27", "f16s", n, n, n, pitch)
    torch.cuda.reset_peak_memory_stats()
    a, b = grid.empty_populations(), grid.empty_populations()
    B.lbm_init_equilibrium(grid, None, u0, a)
    pre = forward_steps - adjoint_steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    where = B.lbm_step(grid, a, b, tau, None, pre)
    t_fwd = _sync_time(t0)
    g_start = (b if where == 0 else a).clone()
    del a, b
    red = _reductions(grid, g_start)
    if red["nonfinite_cells"] > 0 or red["max_speed"] > 1.0:
        del g_start
        return {"grid": [n, n, n], "tau": tau, "forward_steps": forward_steps, "diverged_before_step": pre,
                "forward_mlups": n ** 3 * pre / t_fwd / 1e6}
    F = torch.zeros((3, n, n, n), dtype=torch.float32, device=u0.device, requires_grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gT = AG.rollout(grid, g_start, F, tau, adjoint_steps, checkpoint_every)
    _, u = AG.moments(grid, gT, F)
    KE = 0.5 * (u.double() ** 2).sum()
    t_tail = _sync_time(t0)
    t0 = time.perf_counter()
    KE.backward()
    t_bwd = _sync_time(t0)
    peak = torch.cuda.max_memory_allocated()
    dF = F.grad
    if not bool(torch.isfinite(KE)) or not bool(torch.isfinite(dF).all()):
        # A forward run on its way to divergence (finite, but gaining energy) has an
        # adjoint that grows exponentially and overflows: counted as diverged too.
        res = {"grid": [n, n, n], "tau": tau, "forward_steps": forward_steps,
               "diverged_before_step": forward_steps, "finite_at_step": pre,
               "max_speed_at_step_%d" % pre: red["max_speed"], "forward_mlups": n ** 3 * pre / t_fwd / 1e6,
               "kinetic_energy_final": float(KE), "grad_finite": bool(torch.isfinite(dF).all())}
        del gT, u, F, g_start
        return res
    out = {"grid": [n, n, n], "row_pitch": grid.row_pitch, "storage": "f16s state, f32 adjoint", "tau": tau,
           "forward_steps": forward_steps, "adjoint_steps": adjoint_steps, "checkpoint_every": checkpoint_every,
           "forward_mlups": n ** 3 * pre / t_fwd / 1e6,
           "tail_forward_mlups": n ** 3 * adjoint_steps / t_tail / 1e6,
           "backward_mlups": n ** 3 * adjoint_steps / t_bwd / 1e6,
           "backward_seconds": t_bwd, "peak_memory_gb": peak / 1e9,
           "kinetic_energy_final": float(KE), "grad_force_norm": float(dF.double().norm()),
           "grad_finite": bool(torch.isfinite(dF).all())}
    del gT, u, F, g_start
    return out


def gradient_precision(u0: torch.Tensor, tau: float, steps: int = 100, checkpoint_every: int = 10,
                       storages=("f64", "f32", "f16s", "bf16s"), k_band=(2, 16)):
    """dL/dF of the spectral loss of `forcing_optimisation` at F = 0, computed through
    the adjoint in each storage format, compared with the FP64 gradient (cosine and
    relative L2)."""
    n = u0.shape[-1]
    shells = SP.shell_index((n, n, n), u0.device)
    E0 = SP.energy_spectrum(u0.double(), shells)
    K = torch.arange(E0.numel(), dtype=torch.float64, device=u0.device).clamp(min=1)
    lo, hi = k_band
    target = K ** (-5.0 / 3.0)
    target = target * E0[lo:hi + 1].sum() / target[lo:hi + 1].sum()
    cut = 1e-12 * float(E0.sum())
    out = {"grid": [n, n, n], "tau": tau, "steps": steps, "checkpoint_every": checkpoint_every, "runs": {}}
    ref = None
    for storage in storages:
        grid = B.Grid("D3Q27", storage, n, n, n)
        g0 = grid.empty_populations()
        B.lbm_init_equilibrium(grid, None, u0, g0)
        F = torch.zeros((3, n, n, n), dtype=grid.real_dtype, device=u0.device, requires_grad=True)
        gT = AG.rollout(grid, g0, F, tau, steps, checkpoint_every)
        _, u = AG.moments(grid, gT, F)
        L = SP.log_spectrum_loss(SP.energy_spectrum(u, shells), target, lo, hi, cut)
        L.backward()
        gF = F.grad.double().reshape(-1)
        if ref is None:
            ref = gF
            out["runs"][storage] = {"loss": float(L), "grad_norm": float(gF.norm())}
        else:
            out["runs"][storage] = {"loss": float(L), "grad_norm": float(gF.norm()),
                                    "cosine_vs_f64": float(torch.dot(gF, ref) / (gF.norm() * ref.norm())),
                                    "rel_l2_vs_f64": float((gF - ref).norm() / ref.norm())}
        del g0, F, gT, u, gF
        torch.cuda.empty_cache()
    return out


def flow_control_2d(u0: torch.Tensor, tau: float, steps: int, kappa: float = 5e-5, cutoff: float = 2e-5,
                    record_every: int = 250, storage: str = "f32", graph: bool = True,
                    modes=("free", "restrained")):
    """Free and restrained decaying turbulence on a periodic D2Q9 grid.

    R(u) = sum_K (ln max(sigma_K(u), c) - ln max(sigma0_K, c))^2 over shells
    K = 1 .. n/2, sigma0 the spectrum of the initial field; the restrained run takes
    every step with lbm_step_shifted and du = -kappa dR/du (the closed-form gradient
    through the FFT, two FFTs per step, with the spectrum, its gradient multiplier and
    the real part in the library's kernels: SP.NativeLossHead).  Returns R and the
    kinetic energy over time for both.

    With `graph` (and even `steps` and `record_every`), two restrained steps (a -> b,
    b -> a: moments, loss head, shifted step, twice) are captured once as a HIP graph
    and replayed; the free run takes record_every steps per lbm_step call.  `modes`
    selects the runs ("free", "restrained").
    """
    ny, nx = u0.shape[1:]
    grid = B.Grid("D2Q9", storage, nx, ny)
    shells = SP.shell_index((ny, nx), u0.device)
    sigma0 = SP.energy_spectrum(u0.double(), shells)
    kmax = min(nx, ny) // 2
    use_graph = graph and steps % 2 == 0 and record_every % 2 == 0

    def R_of(u):
        return SP.log_spectrum_loss(SP.energy_spectrum(u, shells), sigma0, 1, kmax, cutoff)

    head = SP.NativeLossHead(shells, sigma0, 1, kmax, cutoff)
    du = grid.empty_real(2)

    def controlled(src, dst, u):
        B.lbm_moments(grid, src, None, None, u)
        head.scaled_grad(u, -kappa, du)
        B.lbm_step_shifted(grid, src, dst, tau, du, 1)

    out = {"grid": [nx, ny], "tau": tau, "steps": steps, "kappa": kappa, "cutoff": cutoff, "storage": storage,
           "graph": use_graph}
    for mode in modes:
        if mode not in ("free", "restrained"):
            raise ValueError(f"unknown mode {mode!r}")
        a, b = grid.empty_populations(), grid.empty_populations()
        B.lbm_init_equilibrium(grid, None, u0, a)
        u = grid.empty_real(2)
        pair = None
        if mode == "restrained" and use_graph:
            # warm-up (FFT plans, allocator) on scratch buffers, then the capture
            x, y = a.clone(), grid.empty_populations()
            ux = grid.empty_real(2)
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                controlled(x, y, ux)
                controlled(y, x, ux)
                pair = torch.cuda.CUDAGraph()
                with torch.cuda.graph(pair, stream=side):
                    controlled(a, b, u)
                    controlled(b, a, u)
            torch.cuda.current_stream().wait_stream(side)
            del x, y, ux
        # one untimed step, its state thrown away, and one untimed record, so that first
        # launches (code loading, graph upload) stay out of the timing
        if pair is not None:
            keep = a.clone()
            pair.replay()
            a.copy_(keep)
            del keep
        elif mode == "free":
            B.lbm_step(grid, a.clone(), b, tau, None, 1)
        else:
            controlled(a.clone(), b, u)
        B.lbm_moments(grid, a, None, None, u)
        with torch.no_grad():
            float(R_of(u)), float(0.5 * (u.double() ** 2).sum())
        hist = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t = 0
        while True:
            if t % record_every == 0:
                B.lbm_moments(grid, a, None, None, u)
                with torch.no_grad():
                    hist.append((t, float(R_of(u)), float(0.5 * (u.double() ** 2).sum())))
            if t == steps:
                break
            if mode == "free":
                k = min(record_every - t % record_every, steps - t)
                if B.lbm_step(grid, a, b, tau, None, k) == 0:
                    a, b = b, a
                t += k
            elif pair is not None:
                pair.replay()  # two steps: the state is back in a
                t += 2
            else:
                controlled(a, b, u)
                a, b = b, a
                t += 1
        out[mode] = {"history": hist, "seconds": _sync_time(t0)}
        del a, b, pair
    return out


__all__ = ["precision_study", "forcing_optimisation", "gradient_precision", "full_scale_adjoint", "flow_control_2d"]
