"""CPU tests of the C ABI boundary: the library loads, exports every entry point the
header declares, publishes the oracle's lattice tables, and rejects invalid
arguments on the host before any HIP call (so no GPU is needed here)."""
import ctypes
import os
import re
import subprocess

import pytest

from oracle import lbm as olbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


@pytest.fixture(scope="module")
def B():
    from paper_2106_12929_amd import binding

    return binding


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = _declared()
    for need in ("lbm_init_equilibrium", "lbm_step", "lbm_moments", "lbm_adjoint_step",
                 "lbm_moments_adjoint", "lbm_stream_only", "lbm_lattice_info", "lbm_strerror"):
        assert need in names


def test_library_exports_every_declared_symbol(B):
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True, text=True, check=True)
    exported = set(re.findall(r"\sT\s+(\w+)", out.stdout))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    for n in _declared():
        assert hasattr(B._lib, n)


def test_every_exported_entry_point_is_declared(B):
    """The header is the whole boundary: no lbm_* symbol is exported undocumented."""
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True, text=True, check=True)
    exported = set(re.findall(r"\sT\s+(lbm_\w+)", out.stdout))
    undeclared = sorted(exported - set(_declared()))
    assert not undeclared, undeclared


@pytest.mark.parametrize("name", ["D2Q9", "D3Q19", "D3Q27"])
def test_lattice_info_matches_oracle_tables(B, name):
    D, Q, c, w = B.lbm_lattice_info(name)
    st = olbm.stencil(name)
    assert (D, Q) == (st.D, st.Q)
    assert [tuple(r) for r in st.c.tolist()] == c
    assert st.w.tolist() == w


def _grid(B, lattice="D3Q27", storage="f32", nx=8, ny=8, nz=8, pitch=0):
    return B._CGrid(B.LATTICES.get(lattice, lattice) if isinstance(lattice, str) else lattice,
                    B.STORAGES.get(storage, storage) if isinstance(storage, str) else storage, nx, ny, nz, pitch)


P1 = ctypes.c_void_p(0x10000)        # aligned fake device addresses: validation
P2 = ctypes.c_void_p(0x4000000000)   # fails before any of them is dereferenced
P3 = ctypes.c_void_p(0x8000000000)
MIS = ctypes.c_void_p(0x10004)


def _step(B, g, a, b, tau=0.6, force=None, n=1):
    return B._lib.lbm_step(ctypes.byref(g), a, b, tau, force, n, None)


def test_step_validation(B):
    lib = B._lib
    g = _grid(B)
    assert _step(B, g, P1, P2, tau=0.5) == -1           # tau <= 1/2
    assert _step(B, g, P1, P2, tau=float("nan")) == -1
    assert _step(B, g, P1, P2, tau=float("inf")) == -1
    assert _step(B, g, P1, P2, n=0) == -1                # n_steps < 1
    assert _step(B, g, None, P2) == -2
    assert _step(B, g, P1, None) == -2
    assert _step(B, g, MIS, P2) == -3
    assert _step(B, g, P1, P1) == -4                     # f_in == f_out
    assert _step(B, g, P1, ctypes.c_void_p(0x10000 + 16)) == -4  # overlapping ranges
    assert _step(B, g, P1, P2, force=P1) == -4           # force overlaps f_in
    assert b"overlap" in lib.lbm_last_error()
    assert lib.lbm_step(None, P1, P2, 0.6, None, 1, None) == -2


@pytest.mark.parametrize("dims,code", [((0, 4, 4), -1), ((4, -1, 4), -1), ((1 << 31, 1, 1), -6),
                                       ((1 << 16, 1 << 16, 1), -6)])
def test_grid_validation(B, dims, code):
    g = _grid(B, nx=dims[0], ny=dims[1], nz=dims[2])
    assert _step(B, g, P1, P2) == code


@pytest.mark.parametrize("storage,limit", [("f64", 1 << 29), ("f32", 1 << 30), ("f32s", 1 << 30),
                                           ("f16s", 1 << 30), ("bf16s", 1 << 30)])
def test_row_offsets_stay_32_bit(B, storage, limit):
    """A row (nx, or the pitch) whose byte length in the grid's widest element reaches
    2^32 is rejected: inside a row the kernels use 32-bit byte offsets.  One word less
    is accepted (checked through the validation-only workspace query)."""
    lib = B._lib
    need = ctypes.c_size_t()
    for nx, pitch, code in ((limit - 1, 0, 0), (limit, 0, -6), (limit + 1, 0, -6),
                            (8, limit - 1, 0), (8, limit, -6)):
        g = _grid(B, lattice="D2Q9", storage=storage, nx=nx, ny=1, nz=1, pitch=pitch)
        assert lib.lbm_moments_workspace_size(ctypes.byref(g), ctypes.byref(need)) == code, (nx, pitch)
        if code:
            assert _step(B, g, P1, P2) == code
            assert b"4 GiB" in lib.lbm_last_error()


def test_lattice_storage_validation(B):
    assert _step(B, _grid(B, lattice=5), P1, P2) == -1
    assert _step(B, _grid(B, storage=9), P1, P2) == -1
    assert _step(B, _grid(B, lattice="D2Q9", nz=2), P1, P2) == -1  # D2Q9 needs nz == 1


def test_other_entry_points_validate(B):
    lib = B._lib
    g = _grid(B)
    gp = ctypes.byref(g)
    assert lib.lbm_init_equilibrium(gp, None, None, P1, None) == -2       # u required
    assert lib.lbm_init_equilibrium(gp, None, P1, P1, None) == -4         # f_out overlaps u
    assert lib.lbm_stream_only(gp, P1, P1, None) == -4
    assert lib.lbm_moments(gp, None, None, None, None, None, None, 0, None) == -2
    red = ctypes.c_void_p(0x40000000)
    assert lib.lbm_moments(gp, P1, None, None, None, red, None, 0, None) == -2    # workspace needed
    need = ctypes.c_size_t()
    assert lib.lbm_moments_workspace_size(gp, ctypes.byref(need)) == 0
    # at most one partial per block of the cell launch (8-cell rows take 64-cell segments,
    # 4 rows per block: 16 blocks) plus one per 2048 of those: 17 entries of 8 doubles
    assert need.value == (16 + 1) * 8 * 8
    assert lib.lbm_moments(gp, P1, None, None, None, red, P2, need.value - 1, None) == -1
    assert lib.lbm_moments(gp, P1, None, P1, None, None, None, 0, None) == -4    # rho_out overlaps g
    assert lib.lbm_adjoint_step(gp, P1, P2, P2, 0.6, None, None, None) == -4     # lam_out == lam_next
    assert lib.lbm_adjoint_step(gp, P1, P2, P3, 0.6, None, ctypes.c_void_p(0xC000000000), None) == -5
    assert lib.lbm_adjoint_step(gp, P1, P2, P3, 0.4, None, None, None) == -1
    assert lib.lbm_moments_adjoint(gp, P1, None, None, None, P1, None, None) == -4
    assert lib.lbm_moments_adjoint(gp, P1, None, None, None, None, None, None) == -2


def test_shifted_step_validation(B):
    lib = B._lib
    g = _grid(B)
    gp = ctypes.byref(g)
    assert lib.lbm_step_shifted(gp, P1, P2, 0.6, None, 1, None) == -2   # du is required
    assert lib.lbm_step_shifted(gp, P1, P2, 0.6, P1, 1, None) == -4     # du overlaps f_in
    assert lib.lbm_step_shifted(gp, P1, P2, 0.5, P3, 1, None) == -1
    assert lib.lbm_step_shifted(gp, P1, P2, 0.6, P3, 0, None) == -1


def test_mrt_validation(B):
    lib = B._lib
    taus = (ctypes.c_double * 9)(1, 1, 1, 0.6, 0.6, 0.6, 1, 1, 1)
    bad = (ctypes.c_double * 9)(1, 1, 1, 0.6, 0.5, 0.6, 1, 1, 1)
    g3 = _grid(B)                                      # D3Q27
    g2 = _grid(B, lattice="D2Q9", nz=1)
    assert lib.lbm_step_mrt(ctypes.byref(g3), P1, P2, taus, None, 1, None) == -5
    assert lib.lbm_step_mrt(ctypes.byref(g2), P1, P2, None, None, 1, None) == -2
    assert lib.lbm_step_mrt(ctypes.byref(g2), P1, P2, bad, None, 1, None) == -1
    assert lib.lbm_step_mrt(ctypes.byref(g2), P1, P1, taus, None, 1, None) == -4
    assert lib.lbm_step_mrt(ctypes.byref(g2), P1, P2, taus, P1, 1, None) == -4
    assert lib.lbm_step_mrt(ctypes.byref(g2), P1, P2, taus, None, 0, None) == -1


def test_local_adjoint_validation(B):
    lib = B._lib
    g = _grid(B)
    gp = ctypes.byref(g)
    assert lib.lbm_adjoint_step_local(gp, P1, P2, 2, P3, 0.6, None, None, None) == -1   # adj_is_chi not 0/1
    assert lib.lbm_adjoint_step_local(gp, P1, P2, 1, P2, 0.6, None, None, None) == -4   # output == input
    assert lib.lbm_adjoint_step_local(gp, P1, P2, 0, None, 0.6, None, None, None) == -2
    assert lib.lbm_adjoint_step_local(gp, P1, P2, 0, P3, 0.5, None, None, None) == -1
    assert lib.lbm_adjoint_unstream(gp, P1, P1, None) == -4
    assert lib.lbm_adjoint_unstream(gp, None, P1, None) == -2


def test_two_step_adjoint_validation(B):
    lib = B._lib
    P4 = ctypes.c_void_p(0xC000000000)
    P5 = ctypes.c_void_p(0x10000000000)
    g = _grid(B, nx=64, ny=16, nz=8)
    gp = ctypes.byref(g)
    f = lib.lbm_adjoint_step2_local
    assert f(gp, None, P2, P3, P4, 0.6, None, None, None) == -2
    assert f(gp, P1, P2, P3, None, 0.6, None, None, None) == -2
    assert f(gp, P1, MIS, P3, P4, 0.6, None, None, None) == -3
    assert f(gp, P1, P2, P3, P4, 0.5, None, None, None) == -1
    assert f(gp, P1, P2, P3, P3, 0.6, None, None, None) == -4       # chi_out == chi_next
    assert f(gp, P1, P2, P3, P4, 0.6, None, P5, None) == -5         # dforce without force
    assert f(gp, P1, P2, P3, P4, 0.6, P5, P4, None) == -4           # dforce == chi_out
    for storage, dims in (("f64", (64, 16, 8)), ("f32", (48, 16, 8)), ("f32", (64, 12, 8)), ("f32", (64, 16, 2))):
        h = _grid(B, storage=storage, nx=dims[0], ny=dims[1], nz=dims[2])
        assert f(ctypes.byref(h), P1, P2, P3, P4, 0.6, None, None, None) == -5, (storage, dims)
    h = _grid(B, "D2Q9", nx=64, ny=16, nz=1)
    assert f(ctypes.byref(h), P1, P2, P3, P4, 0.6, None, None, None) == -5
    v = ctypes.c_int32(7)
    assert lib.lbm_adjoint_step2_available(gp, None) == -2
    assert lib.lbm_adjoint_step2_available(ctypes.byref(_grid(B, nx=0)), ctypes.byref(v)) == -1


@pytest.mark.parametrize("lattice,storage,dims,ok", [
    ("D3Q27", "f32", (64, 16, 8), True), ("D3Q19", "f16s", (32, 8, 3), True), ("D3Q27", "f32s", (32, 8, 3), True),
    ("D3Q27", "bf16s", (256, 256, 256), True), ("D3Q27", "f64", (64, 16, 8), False),
    ("D3Q27", "f32", (48, 16, 8), False), ("D3Q27", "f32", (32, 8, 2), False), ("D2Q9", "f32", (64, 16, 1), False)])
def test_two_step_adjoint_availability(B, lattice, storage, dims, ok):
    v = ctypes.c_int32(7)
    g = _grid(B, lattice, storage, *dims)
    assert B._lib.lbm_adjoint_step2_available(ctypes.byref(g), ctypes.byref(v)) == 0
    assert v.value == int(ok)
    assert B.lbm_adjoint_step2_available(B.Grid(lattice, storage, *dims)) == ok


def test_copy_validation(B):
    lib = B._lib
    assert lib.lbm_copy(P1, P2, 17, None) == -1      # not a multiple of 16
    assert lib.lbm_copy(P1, ctypes.c_void_p(0x10000 + 32), 64, None) == -4
    assert lib.lbm_copy(None, P2, 16, None) == -2
    assert lib.lbm_copy(MIS, P2, 16, None) == -3


def test_neural_step_validation(B):
    lib = B._lib
    g2 = _grid(B, "D2Q9", nz=1)

    def neural(grid=g2, a=P1, b=P2, tau=0.6, params=P3, act=0, n=1):
        return lib.lbm_step_neural(ctypes.byref(grid), a, b, tau, params, act, n, None)

    assert neural(grid=_grid(B)) == -5                  # D2Q9 only
    assert neural(tau=0.5) == -1
    assert neural(act=2) == -1
    assert neural(n=0) == -1
    assert neural(params=None) == -2
    assert neural(params=MIS) == -3
    assert neural(a=P1, b=P1) == -4
    assert neural(params=ctypes.c_void_p(0x10000 + 64)) == -4   # params inside f_in


def test_slab_step_validation(B):
    lib = B._lib
    g = _grid(B)  # 8 x 8 x 8 D3Q27 f32: slab buffers of 10 planes

    def step(grid, a=P1, b=P2, tau=0.6, force=None, z0=0, z1=8):
        return lib.lbm_step_slab(ctypes.byref(grid), a, b, tau, force, z0, z1, None)

    assert step(_grid(B, "D2Q9", nz=1), z1=1) == -5     # z-slabs need a 3D lattice
    for z0, z1 in ((0, 0), (-1, 4), (0, 9), (5, 3)):
        assert step(g, z0=z0, z1=z1) == -1              # empty or out-of-range plane range
    assert step(g, tau=0.5) == -1
    assert step(g, a=None) == -2
    assert step(g, b=None) == -2
    assert step(g, a=MIS) == -3
    assert step(g, a=P1, b=P1) == -4
    plane = 27 * 8 * 8 * 4
    # f_out starts inside the last ghost plane of f_in: the buffers overlap
    assert step(g, a=P1, b=ctypes.c_void_p(0x10000 + 9 * plane)) == -4
    assert step(g, force=ctypes.c_void_p(0x10000 + 16)) == -4


def test_slab_halo_validation(B):
    lib = B._lib
    g = _grid(B)

    def halo(src_grid=g, src=P1, dst_grid=g, dst=P2, face=0):
        return lib.lbm_slab_halo_copy(ctypes.byref(src_grid), src, ctypes.byref(dst_grid), dst, face, None)

    assert halo(src_grid=_grid(B, "D2Q9", nz=1), dst_grid=_grid(B, "D2Q9", nz=1)) == -5
    assert halo(dst_grid=_grid(B, nx=9)) == -1          # slabs must agree in nx, ny
    assert halo(dst_grid=_grid(B, storage="f16s")) == -1
    assert halo(dst_grid=_grid(B, "D3Q19")) == -1
    assert halo(face=2) == -1
    assert halo(src=None) == -2
    assert halo(dst=MIS) == -3
    plane = 27 * 8 * 8 * 4
    # LOW reads src plane 1 and writes dst plane nz + 1 = 9: a dst 8 planes below src
    # puts that ghost plane on top of the source plane
    assert halo(dst=ctypes.c_void_p(0x10000 - 8 * plane), face=0) == -4


def test_slab2_step_validation(B):
    lib = B._lib
    g = _grid(B, nx=32, ny=8, nz=8)  # slab buffers of 12 planes

    def step(grid=g, a=P1, b=P2, tau=0.6, force=None, z0=0, z1=None):
        z1 = grid.nz if z1 is None else z1
        return lib.lbm_step_slab2(ctypes.byref(grid), a, b, tau, force, z0, z1, None)

    assert step(_grid(B, "D2Q9", nx=64, ny=8, nz=1)) == -5   # z-slabs need a 3D lattice
    assert step(_grid(B, nx=32, ny=8, nz=1)) == -1           # nz < 2
    for z0, z1 in ((0, 0), (-1, 4), (0, 9), (5, 3)):
        assert step(z0=z0, z1=z1) == -1                     # empty or out-of-range plane range
    assert step(tau=0.5) == -1
    assert step(a=None) == -2
    assert step(b=MIS) == -3
    assert step(a=P1, b=P1) == -4
    plane = 27 * 32 * 8 * 4
    assert step(b=ctypes.c_void_p(0x10000 + 11 * plane)) == -4   # f_out inside f_in's top ghost plane
    assert step(force=ctypes.c_void_p(0x10000 + 16)) == -4
    assert step(_grid(B, nx=48, ny=8, nz=8)) == -5            # nx off the 32-cell tiles
    assert step(_grid(B, nx=32, ny=12, nz=8)) == -5           # ny off the 8-row tiles
    assert step(_grid(B, storage="f16s", nx=32, ny=8, nz=8)) == -5  # 2-byte words: 64 x 4 tiles
    v = ctypes.c_int32(7)
    for grid, ok in ((g, 1), (_grid(B, storage="f16s", nx=64, ny=4, nz=2), 1), (_grid(B, storage="f64", nx=32, ny=4, nz=3), 1),
                     (_grid(B, nx=32, ny=8, nz=1), 0), (_grid(B, "D2Q9", nx=64, ny=8, nz=1), 0),
                     (_grid(B, nx=48, ny=8, nz=8), 0)):
        assert lib.lbm_step_slab2_available(ctypes.byref(grid), ctypes.byref(v)) == 0
        assert v.value == ok
    assert lib.lbm_step_slab2_available(ctypes.byref(g), None) == -2


def test_slab2_halo_validation(B):
    lib = B._lib
    g = _grid(B)  # 8 x 8 x 8: buffers of 12 planes

    def halo(src_grid=g, src=P1, dst_grid=g, dst=P2, face=0):
        return lib.lbm_slab2_halo_copy(ctypes.byref(src_grid), src, ctypes.byref(dst_grid), dst, face, None)

    assert halo(src_grid=_grid(B, "D2Q9", nz=1), dst_grid=_grid(B, "D2Q9", nz=1)) == -5
    assert halo(dst_grid=_grid(B, nx=9)) == -1
    assert halo(dst_grid=_grid(B, nz=1)) == -1           # both slabs need two planes
    assert halo(src_grid=_grid(B, nz=1)) == -1
    assert halo(face=3) == -1
    assert halo(src=None) == -2
    assert halo(dst=MIS) == -3
    plane = 27 * 8 * 8 * 4
    # LOW reads src planes 2, 3 and writes dst planes nz + 2, nz + 3 = 10, 11: a dst 8
    # planes below src puts ghost plane 10 on source plane 2
    assert halo(dst=ctypes.c_void_p(0x10000 - 8 * plane), face=0) == -4
    # HIGH reads src planes nz, nz + 1 = 8, 9 and writes dst planes 0, 1
    assert halo(dst=ctypes.c_void_p(0x10000 + 8 * plane), face=1) == -4


def test_pitch_validation(B):
    lib = B._lib
    assert _step(B, _grid(B, nx=8, pitch=7), P1, P2) == -1      # 0 < pitch < nx
    assert _step(B, _grid(B, nx=8, pitch=2 ** 31), P1, P2) == -6
    # with pitch 16 a buffer spans 27*16*8*8*4 bytes: f_out that far past f_in is clear,
    # one word less overlaps (the unpadded size would not)
    size = 27 * 16 * 8 * 8 * 4
    assert _step(B, _grid(B, nx=8, pitch=16), P1, ctypes.c_void_p(0x10000 + size - 16)) == -4


def test_strerror(B):
    for code in range(-7, 1):
        assert B._lib.lbm_strerror(code)
    assert B._lib.lbm_strerror(-99) == b"unknown status"


def test_binding_rejects_host_tensors(B):
    import torch

    grid = B.Grid("D3Q27", "f32", 4, 4, 4)
    a = torch.zeros(grid.population_shape(), dtype=torch.float32)
    with pytest.raises(ValueError):
        B.lbm_step(grid, a, a.clone(), 0.6)


def test_loss_head_entry_points_validate(B):
    """The flow-control loss head's entry points reject bad tables, shell bands,
    cutoffs, output kinds and overlapping buffers on the host."""
    lib = B._lib
    sh = B._CShells(100, 8, 0x10000, 0x20000, 0x30000)
    sp = ctypes.byref(sh)
    assert lib.lbm_shell_energy(None, 2, P1, 0.01, P2, None) == -2
    assert lib.lbm_shell_energy(sp, 0, P1, 0.01, P2, None) == -1               # D in 1..3
    assert lib.lbm_shell_energy(sp, 4, P1, 0.01, P2, None) == -1
    assert lib.lbm_shell_energy(sp, 2, None, 0.01, P2, None) == -2
    assert lib.lbm_shell_energy(sp, 2, MIS, 0.01, P2, None) == -3               # misaligned uhat
    assert lib.lbm_shell_energy(sp, 2, P1, float("nan"), P2, None) == -1
    assert lib.lbm_shell_energy(sp, 2, P1, 0.01, ctypes.c_void_p(0x10000 + 3200 - 16), None) == -4  # E inside uhat
    bad = B._CShells(0, 8, 0x10000, 0x20000, 0x30000)
    assert lib.lbm_shell_energy(ctypes.byref(bad), 2, P1, 0.01, P2, None) == -1
    big = B._CShells(1 << 31, 8, 0x10000, 0x20000, 0x30000)
    assert lib.lbm_shell_energy(ctypes.byref(big), 2, P1, 0.01, P2, None) == -6
    nul = B._CShells(100, 8, 0x10000, None, 0x30000)
    assert lib.lbm_shell_energy(ctypes.byref(nul), 2, P1, 0.01, P2, None) == -2
    grad = lib.lbm_log_spectrum_grad
    assert grad(sp, 2, P1, P2, P3, 1, 8, 1e-5, 0.01, None, None) == -1         # k_hi >= nshell
    assert grad(sp, 2, P1, P2, P3, 3, 2, 1e-5, 0.01, None, None) == -1         # k_hi < k_lo
    assert grad(sp, 2, P1, P2, P3, -1, 2, 1e-5, 0.01, None, None) == -1
    assert grad(sp, 2, P1, P2, P3, 1, 7, 0.0, 0.01, None, None) == -1          # cutoff > 0
    assert grad(sp, 2, P1, P2, P3, 1, 7, float("inf"), 0.01, None, None) == -1
    assert grad(sp, 2, P1, P2, None, 1, 7, 1e-5, 0.01, None, None) == -2       # E_target required
    assert grad(sp, 2, P1, P1, P3, 1, 7, 1e-5, 0.01, None, None) == -4         # E overlaps uhat
    assert grad(sp, 2, P1, P2, P3, 1, 7, 1e-5, 0.01, P1, None) == -4           # R overlaps uhat
    assert grad(sp, 2, ctypes.c_void_p(0x30000), P2, P3, 1, 7, 1e-5, 0.01, None, None) == -4  # uhat on shell[]
    assert grad(sp, 2, P1, P2, P3, 1, 7, 1e-5, 0.01, ctypes.c_void_p(0x20010), None) == -4    # R on offsets[]
    assert grad(sp, 2, P1, P2, P3, 1, 7, 1e-5, 0.01, P2, None) == -4           # R overlaps E
    assert lib.lbm_shell_energy(sp, 2, P1, 0.01, ctypes.c_void_p(0x20000), None) == -4  # E on offsets[]
    real = lib.lbm_real_part
    assert real(P1, 100, 1.0, P2, 3, None) == -1                               # F32 or F64 only
    assert real(P1, 0, 1.0, P2, 1, None) == -1
    assert real(None, 100, 1.0, P2, 1, None) == -2
    assert real(P1, 100, 1.0, ctypes.c_void_p(0x10000 + 800), 1, None) == -4   # out inside z
    assert real(P1, 100, float("nan"), P2, 1, None) == -1


def test_moments_noalloc_validation(B):
    """lbm_moments_noalloc validates like lbm_moments, and rejects on the host a
    reduction whose partials would not fit the library's fixed scratch (a 512^3 D3Q27
    grid writing fields needs one partial per 256 cells: 524,544 > 131,072).  Only
    calls that fail before the first HIP call are made here."""
    lib = B._lib
    gp = ctypes.byref(_grid(B, nx=512, ny=512, nz=512))
    red = ctypes.c_void_p(0x100000)
    assert lib.lbm_moments_noalloc(gp, None, None, None, None, red, None) == -2            # g required
    assert lib.lbm_moments_noalloc(gp, MIS, None, None, None, red, None) == -3
    assert lib.lbm_moments_noalloc(gp, P1, None, P1, None, None, None) == -4              # rho_out overlaps g
    assert lib.lbm_moments_noalloc(gp, P1, None, P2, None, red, None) == -6               # scratch too small
    assert b"fixed scratch" in lib.lbm_last_error()
    assert lib.lbm_moments_noalloc(None, P1, None, None, None, red, None) == -2


def _launches(B, g, n):
    single, paired, quad = ctypes.c_int(-1), ctypes.c_int(-1), ctypes.c_int(-1)
    rc = B._lib.lbm_step_launches(ctypes.byref(g), n, ctypes.byref(single), ctypes.byref(paired), ctypes.byref(quad))
    return rc, single.value, paired.value, quad.value


@pytest.mark.parametrize("lattice,storage,dims,pitch,most", [
    ("D3Q27", "f32", (256, 256, 256), 0, 2),
    ("D3Q27", "f32s", (32, 8, 3), 0, 2),
    ("D3Q19", "f32", (64, 16, 11), 128, 2),
    ("D3Q27", "f16s", (256, 256, 256), 0, 2),    # 2-byte words: 64 x 4 tiles
    ("D3Q27", "f16s", (32, 8, 8), 0, 1),
    ("D3Q19", "f16s", (64, 4, 3), 0, 2),
    ("D3Q27", "bf16s", (256, 256, 256), 0, 2),   # shifted BF16: 64 x 4 tiles, as FP16
    ("D3Q27", "f64", (256, 256, 256), 0, 2),     # 8-byte words: 32 x 4 tiles
    ("D3Q27", "f64", (32, 4, 3), 0, 2),
    ("D3Q19", "f64", (64, 8, 5), 96, 2),
    ("D3Q27", "f64", (32, 6, 3), 0, 1),          # ny off the 4-row tiles
    ("D3Q27", "f64", (32, 4, 4), 4971027, 1),    # one z plane of words: 2^32 + 32 bytes
    ("D3Q27", "f64", (32, 4, 4), 4971026, 2),    # 2^32 - 832 bytes
    ("D2Q9", "f32", (256, 256, 1), 0, 4),        # 2D: four steps per launch
    ("D2Q9", "f64", (64, 64, 1), 0, 4),
    ("D2Q9", "f16s", (8192, 8192, 1), 0, 4),     # every kind: four steps per launch
    ("D2Q9", "f32", (128, 4, 1), 0, 2),          # ny < 5: two steps per launch
    ("D2Q9", "f32", (64, 3, 1), 192, 2),
    ("D2Q9", "f32", (96, 8, 1), 0, 1),           # nx off the 64-cell segments
    ("D2Q9", "f32", (64, 2, 1), 0, 1),           # ny < 3
    ("D2Q9", "bf16s", (256, 256, 1), 0, 4),
    ("D2Q9", "f64", (64, 8, 1), 59652324, 1),    # the 9 direction rows of a grid row: 2^32 + 32 bytes
    ("D2Q9", "f64", (64, 8, 1), 59652320, 4),    # 2^32 - 256 bytes
    ("D3Q27", "f32", (48, 16, 8), 0, 1),         # nx off the 32-cell tiles
    ("D3Q27", "f32", (32, 12, 8), 0, 1),         # ny off the 8-row tiles
    ("D3Q27", "f32", (32, 8, 2), 0, 1),          # nz < 3
    ("D3Q27", "f32", (32, 8, 4), 4971027, 1),    # one z plane of words: 2^32 + 32 bytes
    ("D3Q27", "f32", (32, 8, 4), 4971026, 2),    # 2^32 - 832 bytes
])
def test_step_launch_plan(B, lattice, storage, dims, pitch, most):
    """lbm_step's split into one-, two- and four-step launches: the multi-step
    launches in pairs of one kind (so that the result stays where single steps leave it)
    after n_steps mod 4 single steps, on the grids the kernels take; single steps
    everywhere else."""
    g = _grid(B, lattice=lattice, storage=storage, nx=dims[0], ny=dims[1], nz=dims[2], pitch=pitch)
    for n in (1, 2, 3, 4, 5, 6, 7, 8, 9, 12, 19, 1000, 1001, 1003):
        rc, single, paired, quad = _launches(B, g, n)
        assert rc == 0
        assert single + 2 * paired + 4 * quad == n
        if most == 4:
            assert (quad, paired, single) == (2 * (n // 8), 2 * ((n % 8) // 4), n % 4), n
        elif most == 2:
            assert (quad, paired, single) == (0, 2 * (n // 4), n % 4), n
        else:
            assert (quad, paired, single) == (0, 0, n), n
    expect = {4: (0, 0, 250), 2: (0, 500, 0), 1: (1000, 0, 0)}[most]
    assert B.lbm_step_launches(B.Grid(lattice, storage, *dims, pitch or None), 1000) == expect


def test_step_launch_plan_validation(B):
    g = _grid(B)
    assert _launches(B, g, 0)[0] == -1
    assert B._lib.lbm_step_launches(ctypes.byref(g), 4, None, None, None) == -2
    assert _launches(B, _grid(B, nx=0), 4)[0] == -1
