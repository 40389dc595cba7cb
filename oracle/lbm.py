"""Plain FP64 CPU oracle of the lattice-Boltzmann stream-and-collide step.

Test infrastructure.  Only the test suite, the smoke check and the CPU-baseline leg
of the benchmark import this package; the product path (the HIP library and its
Python binding) never does, and the two share no code.

Source: Bedrunka et al., "Lettuce: PyTorch-based Lattice Boltzmann Framework"
(arXiv:2106.12929), Sec. 2.1, Eqs. (1)-(4), and the tau-nu relation in Sec. 3.1.
Where the paper is silent (lattice weights and velocity order, the Guo forcing
term, boundaries) the docstring names the textbook definition followed
(Krueger et al., "The Lattice Boltzmann Method", 2016, which the paper cites).

Everything here is written for readability, not speed: torch float64 tensors on the
CPU, one `torch.roll` per direction for streaming, no fusion.

Array layout
    populations  f[i, y, x]     (D2Q9)     f[i, z, y, x]  (D3Q27)
    velocity     u[a, y, x]  /  u[a, z, y, x]   with a = 0 (x), 1 (y), 2 (z)
    density      rho[y, x]   /  rho[z, y, x]
    force        F[a, ...]   same layout as u
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import torch

F64 = torch.float64

# Textbook D1Q3-derived lattice weights, indexed by |c|^2 (Krueger 2016, Table 3.2).
# The paper names the weights w_i and the sound speed c_s (Sec. 2.1, after Eq. 3)
# but prints no values.
_WEIGHTS = {
    "D2Q9": {0: 4.0 / 9.0, 1: 1.0 / 9.0, 2: 1.0 / 36.0},
    "D3Q19": {0: 1.0 / 3.0, 1: 1.0 / 18.0, 2: 1.0 / 36.0},
    "D3Q27": {0: 8.0 / 27.0, 1: 2.0 / 27.0, 2: 1.0 / 54.0, 3: 1.0 / 216.0},
}
CS2 = 1.0 / 3.0  # squared lattice sound speed c_s^2 of both stencils


@dataclass(frozen=True)
class Stencil:
    """Discrete velocity set: c[i] = (c_x, c_y[, c_z]) in {-1, 0, 1}^D, weights w[i]."""

    name: str
    D: int
    Q: int
    c: torch.Tensor  # [Q, D] int64
    w: torch.Tensor  # [Q] float64

    @property
    def opposite(self) -> list[int]:
        """opposite[i] = j with c_j = -c_i."""
        rows = [tuple(r) for r in self.c.tolist()]
        return [rows.index(tuple(-v for v in r)) for r in rows]


def stencil(name: str) -> Stencil:
    """D2Q9, D3Q19 or D3Q27 (the lattices of Sec. 2.1/3.1, Listing 1's example and the
    3D benchmark of Sec. 3.3).

    Velocity order: every c in {-1,0,1}^D (D3Q19: those with |c|^2 <= 2), with c_x
    varying fastest, then c_y, then c_z; for D2Q9 and D3Q27 that is
    i = 3(c_y+1) + (c_x+1) and i = 9(c_z+1) + 3(c_y+1) + (c_x+1).  The paper fixes no
    order; this one puts the rest velocity in the middle and makes
    opposite(i) = Q-1-i.
    """
    D = {"D2Q9": 2, "D3Q19": 3, "D3Q27": 3}[name]
    rows = []
    for tail in itertools.product((-1, 0, 1), repeat=D):
        # product() varies its last element fastest; reverse so that c_x is fastest.
        rows.append(tuple(reversed(tail)))
    if name == "D3Q19":
        rows = [r for r in rows if sum(v * v for v in r) <= 2]
    c = torch.tensor(rows, dtype=torch.int64)
    w = torch.tensor([_WEIGHTS[name][sum(v * v for v in r)] for r in rows], dtype=F64)
    return Stencil(name, D, len(rows), c, w)


def _bshape(st: Stencil, vec: torch.Tensor, ndim_spatial: int) -> torch.Tensor:
    """Reshape a per-direction vector [Q] to broadcast against [Q, *spatial]."""
    return vec.reshape((st.Q,) + (1,) * ndim_spatial)


def c_dot(st: Stencil, u: torch.Tensor) -> torch.Tensor:
    """(c_i . u)(x) for every direction i: returns [Q, *spatial]."""
    cf = st.c.to(F64)
    return torch.einsum("qa,a...->q...", cf, u)


def density(f: torch.Tensor) -> torch.Tensor:
    """rho = sum_i f_i  (Eq. 4, left)."""
    return f.sum(dim=0)


def momentum(f: torch.Tensor, st: Stencil) -> torch.Tensor:
    """rho u = sum_i c_i f_i  (Eq. 4, right): returns [D, *spatial]."""
    cf = st.c.to(F64)
    return torch.einsum("qa,q...->a...", cf, f)


def velocity(f: torch.Tensor, st: Stencil, force: torch.Tensor | None = None) -> torch.Tensor:
    """u = (sum_i c_i f_i) / rho (Eq. 4).

    With a body force F the Guo scheme uses the half-force corrected velocity
    u = (sum_i c_i f_i + F/2) / rho (Guo, Zheng & Shi 2002; Krueger 2016, Sec. 6.3).
    """
    j = momentum(f, st)
    if force is not None:
        j = j + 0.5 * force
    return j / density(f)


def equilibrium(rho: torch.Tensor, u: torch.Tensor, st: Stencil) -> torch.Tensor:
    """Second-order equilibrium (Eq. 3):

        f_i^eq = w_i rho (1 + u.c_i / c_s^2 + (u.c_i)^2 / (2 c_s^4) - u.u / (2 c_s^2)).
    """
    nd = rho.dim()
    cu = c_dot(st, u)
    uu = (u * u).sum(dim=0)
    w = _bshape(st, st.w, nd)
    return w * rho * (1.0 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2))


def guo_source(u: torch.Tensor, force: torch.Tensor, tau: float, st: Stencil) -> torch.Tensor:
    """Guo forcing term added to the collided populations (not in the paper; textbook,
    Guo, Zheng & Shi 2002; Krueger 2016, Eq. 6.14):

        S_i = (1 - 1/(2 tau)) w_i [ (c_i - u)/c_s^2 + (c_i.u) c_i / c_s^4 ] . F
    """
    nd = u.dim() - 1
    cf = st.c.to(F64)
    cu = c_dot(st, u)                                  # [Q, ...]
    cF = torch.einsum("qa,a...->q...", cf, force)      # c_i . F
    uF = (u * force).sum(dim=0)                        # u . F
    w = _bshape(st, st.w, nd)
    return (1.0 - 0.5 / tau) * w * ((cF - uF) / CS2 + cu * cF / (CS2 * CS2))


def bgk_collide(f: torch.Tensor, tau: float, st: Stencil, force: torch.Tensor | None = None) -> torch.Tensor:
    """BGK collision (Eq. 2): f_i + Omega_i with Omega_i = -(f_i - f_i^eq) / tau.

    f^eq is taken at the local rho and u of f (Eq. 4).  With a body force the Guo
    velocity u = (sum c f + F/2)/rho enters f^eq and the Guo source is added.
    """
    rho = density(f)
    u = velocity(f, st, force)
    feq = equilibrium(rho, u, st)
    out = f - (f - feq) / tau
    if force is not None:
        out = out + guo_source(u, force, tau, st)
    return out


def bgk_collide_shifted(f: torch.Tensor, tau: float, st: Stencil, du: torch.Tensor) -> torch.Tensor:
    """BGK collision with the flow-control forcing of Sec. 3.2: the equilibrium is
    expanded around the locally shifted velocity u + du, with u from Eq. 4:
        f_i - (f_i - f_i^eq(rho, u + du)) / tau.
    """
    rho = density(f)
    u = momentum(f, st) / rho
    return f - (f - equilibrium(rho, u + du, st)) / tau


def stream(f: torch.Tensor, st: Stencil) -> torch.Tensor:
    """Streaming (Eq. 1): the population moving with c_i travels from x to x + c_i,
    on a periodic grid.  out_i(x + c_i) = f_i(x), i.e. out_i(x) = f_i(x - c_i).
    """
    out = torch.empty_like(f)
    dims = tuple(-1 - a for a in range(st.D))  # x is the last axis, then y, then z
    for i in range(st.Q):
        shifts = tuple(int(v) for v in st.c[i])
        out[i] = torch.roll(f[i], shifts=shifts, dims=dims)
    return out


def step(g: torch.Tensor, tau: float, st: Stencil, force: torch.Tensor | None = None) -> torch.Tensor:
    """One time step in the pull (stream-then-collide) convention used for every
    comparison with the GPU path:  g(t+1) = C(S g(t)).

    g(t) holds the post-collision populations C(f(t)) of Eq. 1's state f(t); see
    `step_literal` for Eq. 1 as printed and the test that ties the two together.
    """
    return bgk_collide(stream(g, st), tau, st, force)


def step_shifted(g: torch.Tensor, tau: float, st: Stencil, du: torch.Tensor) -> torch.Tensor:
    """Pull-convention step with the shifted-velocity equilibrium: C_du(S g)."""
    return bgk_collide_shifted(stream(g, st), tau, st, du)


def step_literal(f: torch.Tensor, tau: float, st: Stencil, force: torch.Tensor | None = None) -> torch.Tensor:
    """Eq. 1 as printed: collide at x, then move to x + c_i:  f(t+1) = S(C(f(t)))."""
    return stream(bgk_collide(f, tau, st, force), st)


def run(g: torch.Tensor, tau: float, st: Stencil, n_steps: int, force: torch.Tensor | None = None) -> torch.Tensor:
    """n_steps applications of `step` (Listing 1's Simulation.step(num_steps))."""
    for _ in range(n_steps):
        g = step(g, tau, st, force)
    return g


def state_moments(g: torch.Tensor, st: Stencil, force: torch.Tensor | None = None):
    """Density and physical velocity of the pre-collision state f(t) that produced the
    stored post-collision populations g(t) = C(f(t)).

    Collision conserves mass, so rho = sum g.  It conserves momentum without a force;
    with the Guo force sum_i c_i g_i = sum_i c_i f_i + F, hence the physical momentum
    rho u = sum_i c_i f_i + F/2 = sum_i c_i g_i - F/2.
    """
    rho = density(g)
    j = momentum(g, st)
    if force is not None:
        j = j - 0.5 * force
    return rho, j / rho


def nu_from_tau(tau: float) -> float:
    """Kinematic viscosity in lattice units, nu = c_s^2 (tau - 1/2) (Sec. 3.1, with
    delta_t = 1)."""
    return CS2 * (tau - 0.5)


# --------------------------------------------------------------------------------------
# Pointwise evaluation for sampled parity at large grids
# --------------------------------------------------------------------------------------

def gather_at_cells(g: torch.Tensor, st: Stencil, cells: torch.Tensor) -> torch.Tensor:
    """The streamed populations h_i(x) = g_i(x - c_i) (periodic, as in `stream`) at
    the listed cells only.  cells: [M, D] int64 coordinates (x, y[, z]).  Returns
    [Q, M] float64 (g may have any dtype; values are converted exactly)."""
    spatial = g.shape[1:]
    sizes = [spatial[-1 - a] for a in range(st.D)]   # (nx, ny[, nz])
    M = cells.shape[0]
    h = torch.empty((st.Q, M), dtype=F64)
    for i in range(st.Q):
        src = [(cells[:, a] - int(st.c[i, a])) % sizes[a] for a in range(st.D)]
        idx = tuple(reversed(src))                      # (z, y, x) order for indexing
        h[i] = g[i][idx].to(F64)
    return h


def force_at_cells(force: torch.Tensor, st: Stencil, cells: torch.Tensor) -> torch.Tensor:
    """force[a](x) at the listed cells: [D, M] float64."""
    idx = tuple(cells[:, a] for a in reversed(range(st.D)))
    return torch.stack([force[a][idx].to(F64) for a in range(st.D)])


def step_at_cells(g: torch.Tensor, tau: float, st: Stencil, cells: torch.Tensor,
                  force: torch.Tensor | None = None) -> torch.Tensor:
    """`step` evaluated only at the listed cells: returns [Q, M] float64, the
    populations C(S g) there."""
    h = gather_at_cells(g, st, cells)
    F = None if force is None else force_at_cells(force, st, cells)
    return bgk_collide(h, tau, st, F)


# --------------------------------------------------------------------------------------
# Multiple-relaxation-time collision (Sec. 3.1, Eq. 5), D2Q9, Dellar moment basis
# --------------------------------------------------------------------------------------

def dellar_matrix(st: Stencil) -> torch.Tensor:
    """Moment matrix M of the D2Q9 basis m = M f = (rho, rho u, rho v, Pi_xx, Pi_xy,
    Pi_yy, N, J_x, J_y) (Sec. 3.1, following Dellar 2003).

    Rows: 1, c_x, c_y, c_x^2, c_x c_y, c_y^2, g, g c_x, g c_y with the non-hydrodynamic
    weight g = (3 c_x^2 - 1)(3 c_y^2 - 1), i.e. g = 1, -2, 4 on the rest, axis and
    diagonal velocities (Dellar's N and J moments).
    """
    if st.name != "D2Q9":
        raise ValueError("the Dellar basis is defined for D2Q9")
    cx = st.c[:, 0].to(F64)
    cy = st.c[:, 1].to(F64)
    g = (3.0 * cx * cx - 1.0) * (3.0 * cy * cy - 1.0)
    return torch.stack([torch.ones_like(cx), cx, cy, cx * cx, cx * cy, cy * cy, g, g * cx, g * cy])


def mrt_collide(f: torch.Tensor, taus, st: Stencil) -> torch.Tensor:
    """Eq. 5: f + Omega with Omega = -M^{-1} S^{-1} (M f - m^eq), m^eq = M f^eq(rho, u),
    S = diag(tau_0 .. tau_8).

    taus: 9 relaxation times (numbers or tensors broadcastable to the spatial shape;
    per-cell values for tau_6..8 model the neural collision's outputs).  The conserved
    moments (0..2) have m = m^eq, so their tau has no effect.
    """
    M = dellar_matrix(st)
    Minv = torch.linalg.inv(M)
    rho = density(f)
    u = momentum(f, st) / rho
    feq = equilibrium(rho, u, st)
    m = torch.einsum("kq,q...->k...", M, f)
    meq = torch.einsum("kq,q...->k...", M, feq)
    rel = torch.stack([(m[k] - meq[k]) / taus[k] for k in range(st.Q)])
    return f - torch.einsum("qk,k...->q...", Minv, rel)


def step_mrt(g: torch.Tensor, taus, st: Stencil) -> torch.Tensor:
    """Pull-convention step with the MRT collision: C_MRT(S g)."""
    return mrt_collide(stream(g, st), taus, st)
