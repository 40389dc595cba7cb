"""Thin ctypes binding of liblbm.so (the C ABI in include/lbm.h).

Each function has the name of the C entry point it calls and only marshals
arguments: it checks that every tensor lives on the GPU, is contiguous and has the
dtype and element count the call reads or writes (so the kernels never index past
a buffer), then passes raw device pointers and the current HIP stream.  All
arithmetic happens in the HIP kernels.  There is no fallback: if the library is
missing, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LATTICES = {"D2Q9": 0, "D3Q27": 1, "D3Q19": 2}
STORAGES = {"f64": 0, "f32": 1, "f32s": 2, "f16s": 3, "bf16s": 4}
FACES = {"low": 0, "high": 1}
ACTIVATIONS = {"relu": 0, "tanh": 1}
NEURAL_PARAMS = 530
STORAGE_DTYPE = {"f64": torch.float64, "f32": torch.float32, "f32s": torch.float32,
                 "f16s": torch.float16, "bf16s": torch.bfloat16}
NRED = 8
RED_NAMES = ("mass", "momentum_x", "momentum_y", "momentum_z", "kinetic_energy",
             "nonfinite_cells", "max_speed", "min_density")


class LbmError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.lbm_strerror(status).decode()
        detail = _lib.lbm_last_error().decode()
        super().__init__(f"{where}: {msg} ({status}){': ' + detail if detail else ''}")


class _CGrid(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int32), ("storage", ctypes.c_int32),
                ("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("pitch", ctypes.c_int64)]


class _CShells(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nshell", ctypes.c_int32), ("order", ctypes.c_void_p),
                ("offsets", ctypes.c_void_p), ("shell", ctypes.c_void_p)]


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2106_12929_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, dbl, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    gp = ctypes.POINTER(_CGrid)
    sigs = {
        "lbm_strerror": (ctypes.c_char_p, [i32]),
        "lbm_last_error": (ctypes.c_char_p, []),
        "lbm_version": (i32, []),
        "lbm_lattice_info": (i32, [i32, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                   ctypes.POINTER(dbl)]),
        "lbm_init_equilibrium": (i32, [gp, vp, vp, vp, vp]),
        "lbm_step": (i32, [gp, vp, vp, dbl, vp, i32, vp]),
        "lbm_step_shifted": (i32, [gp, vp, vp, dbl, vp, i32, vp]),
        "lbm_step_launches": (i32, [gp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "lbm_step_mrt": (i32, [gp, vp, vp, ctypes.POINTER(dbl), vp, i32, vp]),
        "lbm_step_neural": (i32, [gp, vp, vp, dbl, vp, i32, i32, vp]),
        "lbm_stream_only": (i32, [gp, vp, vp, vp]),
        "lbm_moments_workspace_size": (i32, [gp, ctypes.POINTER(sz)]),
        "lbm_moments": (i32, [gp, vp, vp, vp, vp, vp, vp, sz, vp]),
        "lbm_moments_noalloc": (i32, [gp, vp, vp, vp, vp, vp, vp]),
        "lbm_adjoint_step": (i32, [gp, vp, vp, vp, dbl, vp, vp, vp]),
        "lbm_moments_adjoint": (i32, [gp, vp, vp, vp, vp, vp, vp, vp]),
        "lbm_adjoint_step_local": (i32, [gp, vp, vp, i32, vp, dbl, vp, vp, vp]),
        "lbm_adjoint_unstream": (i32, [gp, vp, vp, vp]),
        "lbm_adjoint_step2_local": (i32, [gp, vp, vp, vp, vp, dbl, vp, vp, vp]),
        "lbm_adjoint_step2_available": (i32, [gp, ctypes.POINTER(i32)]),
        "lbm_copy": (i32, [vp, vp, sz, vp]),
        "lbm_step_slab": (i32, [gp, vp, vp, dbl, vp, ctypes.c_int64, ctypes.c_int64, vp]),
        "lbm_slab_halo_copy": (i32, [gp, vp, gp, vp, i32, vp]),
        "lbm_step_slab2": (i32, [gp, vp, vp, dbl, vp, ctypes.c_int64, ctypes.c_int64, vp]),
        "lbm_step_slab2_available": (i32, [gp, ctypes.POINTER(i32)]),
        "lbm_slab2_halo_copy": (i32, [gp, vp, gp, vp, i32, vp]),
        "lbm_shell_energy": (i32, [ctypes.POINTER(_CShells), i32, vp, dbl, vp, vp]),
        "lbm_log_spectrum_grad": (i32, [ctypes.POINTER(_CShells), i32, vp, vp, vp, i32, i32, dbl, dbl, vp, vp]),
        "lbm_real_part": (i32, [vp, ctypes.c_int64, dbl, vp, i32, vp]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


@dataclass(frozen=True)
class Grid:
    """Grid descriptor: lattice "D2Q9"/"D3Q19"/"D3Q27", storage kind, nx, ny, nz cells,
    and the words between direction rows of population buffers (pitch; None = nx)."""

    lattice: str
    storage: str
    nx: int
    ny: int
    nz: int = 1
    pitch: int | None = None

    @staticmethod
    def padded(lattice: str, storage: str, nx: int, ny: int, nz: int = 1) -> "Grid":
        """A grid whose direction rows are padded to a multiple of 256 bytes (full
        bandwidth for any nx)."""
        per = 256 // torch.tensor([], dtype=STORAGE_DTYPE[storage]).element_size()
        return Grid(lattice, storage, nx, ny, nz, -(-nx // per) * per)

    @staticmethod
    def tuned(lattice: str, storage: str, nx: int, ny: int, nz: int = 1) -> "Grid":
        """`padded`, then one more 128-byte line on the rows of 3D lattices that measured
        slow on MI355X: 2- or 8-byte words, a row of a power-of-two length of 1 KB or
        more, split over several 256-cell blocks.  The D3Q27 step ran 10-11% faster with
        that line at 1 KB and 2 KB rows of 2-byte words and at 4 KB rows of 8-byte
        words (3% at 4 KB rows of 2-byte words; D3Q19 7%).  With 4-byte words, other
        row lengths and D2Q9 the extra line measured slower, so those keep `padded`."""
        g = Grid.padded(lattice, storage, nx, ny, nz)
        word = torch.tensor([], dtype=STORAGE_DTYPE[storage]).element_size()
        row = g.row_pitch * word
        if lattice != "D2Q9" and word in (2, 8) and nx > 256 and row >= 1024 and row & (row - 1) == 0:
            g = Grid(lattice, storage, nx, ny, nz, g.row_pitch + 128 // word)
        return g

    @property
    def row_pitch(self) -> int:
        return self.nx if self.pitch is None else self.pitch

    @property
    def pop_size(self) -> int:
        """Entries of a population buffer (and of an adjoint population array)."""
        return self.Q * self.row_pitch * self.ny * self.nz

    @property
    def D(self) -> int:
        return 2 if self.lattice == "D2Q9" else 3

    @property
    def Q(self) -> int:
        return {"D2Q9": 9, "D3Q19": 19, "D3Q27": 27}[self.lattice]

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def spatial(self) -> tuple:
        return (self.ny, self.nx) if self.D == 2 else (self.nz, self.ny, self.nx)

    @property
    def word_dtype(self) -> torch.dtype:
        return STORAGE_DTYPE[self.storage]

    @property
    def real_dtype(self) -> torch.dtype:
        return torch.float64 if self.storage == "f64" else torch.float32

    def population_shape(self) -> tuple:
        """Shape of a population buffer in the library's row-interleaved layout:
        (nz, ny, Q, pitch) for 3D lattices, (ny, Q, pitch) for D2Q9; word (i, x, y, z)
        sits at ((z*ny + y)*Q + i)*pitch + x (pitch = nx unless padded)."""
        p = self.row_pitch
        return (self.ny, self.Q, p) if self.D == 2 else (self.nz, self.ny, self.Q, p)

    def to_layout(self, f: torch.Tensor) -> torch.Tensor:
        """[Q, *spatial] (direction-major) -> the library layout (a contiguous copy;
        pad words are zero)."""
        g = f.permute(1, 0, 2) if self.D == 2 else f.permute(1, 2, 0, 3)
        if self.row_pitch == self.nx:
            return g.contiguous()
        out = torch.zeros(g.shape[:-1] + (self.row_pitch,), dtype=f.dtype, device=f.device)
        out[..., :self.nx] = g
        return out

    def from_layout(self, f: torch.Tensor) -> torch.Tensor:
        """The library layout -> [Q, *spatial] (a contiguous copy; pad words dropped)."""
        f = f[..., :self.nx]
        if self.D == 2:
            return f.permute(1, 0, 2).contiguous()
        return f.permute(2, 0, 1, 3).contiguous()

    def vector_shape(self) -> tuple:
        return (self.D,) + self.spatial

    def c_struct(self) -> _CGrid:
        if self.lattice not in LATTICES:
            raise ValueError(f"unknown lattice {self.lattice!r}")
        if self.storage not in STORAGES:
            raise ValueError(f"unknown storage {self.storage!r}")
        return _CGrid(LATTICES[self.lattice], STORAGES[self.storage], self.nx, self.ny, self.nz,
                      0 if self.pitch is None else self.pitch)

    def empty_populations(self, device="cuda") -> torch.Tensor:
        return torch.empty(self.population_shape(), dtype=self.word_dtype, device=device)

    def slab_population_shape(self, ghost: int = 1) -> tuple:
        """Shape of a z-slab buffer: the population layout of nz + 2 * ghost planes,
        `ghost` ghost planes below and above the slab's own (1: lbm_step_slab, 2:
        lbm_step_slab2)."""
        if self.D != 3:
            raise ValueError("z-slabs need a 3D lattice")
        if ghost not in (1, 2):
            raise ValueError("a slab has 1 or 2 ghost planes on each side")
        return (self.nz + 2 * ghost, self.ny, self.Q, self.row_pitch)

    def empty_slab_populations(self, device="cuda", ghost: int = 1) -> torch.Tensor:
        return torch.empty(self.slab_population_shape(ghost), dtype=self.word_dtype, device=device)

    def empty_real(self, components: int, device="cuda") -> torch.Tensor:
        shape = self.spatial if components == 0 else (components,) + self.spatial
        return torch.empty(shape, dtype=self.real_dtype, device=device)


def _dev_ptr(t: torch.Tensor | None, name: str, dtype: torch.dtype, numel: int, required: bool = True):
    if t is None:
        if required:
            raise ValueError(f"{name} is required")
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor (got {t.device})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype} (got {t.dtype})")
    if t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements (got {t.numel()})")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _check(rc: int, where: str) -> int:
    if rc < 0:
        raise LbmError(rc, where)
    return rc


def lbm_version() -> int:
    return _lib.lbm_version()


def lbm_lattice_info(lattice: str):
    """(D, Q, c [Q][D] as a list of tuples, w [Q]) of a lattice."""
    D, Q = ctypes.c_int(), ctypes.c_int()
    _check(_lib.lbm_lattice_info(LATTICES[lattice], ctypes.byref(D), ctypes.byref(Q), None, None),
           "lbm_lattice_info")
    c = (ctypes.c_int * (Q.value * D.value))()
    w = (ctypes.c_double * Q.value)()
    _check(_lib.lbm_lattice_info(LATTICES[lattice], None, None, c, w), "lbm_lattice_info")
    rows = [tuple(c[i * D.value:(i + 1) * D.value]) for i in range(Q.value)]
    return D.value, Q.value, rows, list(w)


def lbm_init_equilibrium(grid: Grid, rho: torch.Tensor | None, u: torch.Tensor, f_out: torch.Tensor,
                         stream=None) -> None:
    """f_out <- f^eq(rho, u); rho (or None for 1) and u are float64 GPU tensors."""
    N = grid.ncells
    g = grid.c_struct()
    args = (_dev_ptr(rho, "rho", torch.float64, N, required=False),
            _dev_ptr(u, "u", torch.float64, grid.D * N),
            _dev_ptr(f_out, "f_out", grid.word_dtype, grid.pop_size))
    _check(_lib.lbm_init_equilibrium(ctypes.byref(g), *args, _stream(stream)), "lbm_init_equilibrium")


def lbm_step(grid: Grid, f_in: torch.Tensor, f_out: torch.Tensor, tau: float,
             force: torch.Tensor | None = None, n_steps: int = 1, stream=None) -> int:
    """n_steps ping-pong steps; returns 0 if the result is in f_out, 1 if in f_in."""
    N = grid.ncells
    g = grid.c_struct()
    a = _dev_ptr(f_in, "f_in", grid.word_dtype, grid.pop_size)
    b = _dev_ptr(f_out, "f_out", grid.word_dtype, grid.pop_size)
    F = _dev_ptr(force, "force", grid.real_dtype, grid.D * N, required=False)
    return _check(_lib.lbm_step(ctypes.byref(g), a, b, float(tau), F, int(n_steps), _stream(stream)), "lbm_step")


def lbm_step_shifted(grid: Grid, f_in: torch.Tensor, f_out: torch.Tensor, tau: float, du: torch.Tensor,
                     n_steps: int = 1, stream=None) -> int:
    """n_steps steps with f^eq(rho, u + du); returns 0 (result in f_out) or 1 (in f_in)."""
    N = grid.ncells
    g = grid.c_struct()
    a = _dev_ptr(f_in, "f_in", grid.word_dtype, grid.pop_size)
    b = _dev_ptr(f_out, "f_out", grid.word_dtype, grid.pop_size)
    d = _dev_ptr(du, "du", grid.real_dtype, grid.D * N)
    return _check(_lib.lbm_step_shifted(ctypes.byref(g), a, b, float(tau), d, int(n_steps), _stream(stream)),
                  "lbm_step_shifted")


def lbm_step_mrt(grid: Grid, f_in: torch.Tensor, f_out: torch.Tensor, taus, tau_ghost: torch.Tensor | None = None,
                 n_steps: int = 1, stream=None) -> int:
    """D2Q9 MRT steps (Dellar basis); taus: 9 relaxation times; tau_ghost: optional
    [3, ny, nx] per-cell tau_6..8.  Returns 0 (result in f_out) or 1 (in f_in)."""
    N = grid.ncells
    g = grid.c_struct()
    t = (ctypes.c_double * 9)(*[float(v) for v in taus])
    a = _dev_ptr(f_in, "f_in", grid.word_dtype, grid.pop_size)
    b = _dev_ptr(f_out, "f_out", grid.word_dtype, grid.pop_size)
    tg = _dev_ptr(tau_ghost, "tau_ghost", grid.real_dtype, 3 * N, required=False)
    return _check(_lib.lbm_step_mrt(ctypes.byref(g), a, b, t, tg, int(n_steps), _stream(stream)), "lbm_step_mrt")


def lbm_step_neural(grid: Grid, f_in: torch.Tensor, f_out: torch.Tensor, tau_shear: float,
                    params: torch.Tensor, activation: str = "relu", n_steps: int = 1, stream=None) -> int:
    """D2Q9 steps with the neural collision (MRT with network-given tau_6..8);
    params: 530 reals (W1 [53][6], b1 [53], W2 [3][53]).  Returns 0 (result in f_out)
    or 1 (in f_in)."""
    N = grid.ncells
    g = grid.c_struct()
    a = _dev_ptr(f_in, "f_in", grid.word_dtype, grid.pop_size)
    b = _dev_ptr(f_out, "f_out", grid.word_dtype, grid.pop_size)
    p = _dev_ptr(params, "params", grid.real_dtype, NEURAL_PARAMS)
    return _check(_lib.lbm_step_neural(ctypes.byref(g), a, b, float(tau_shear), p, ACTIVATIONS[activation],
                                       int(n_steps), _stream(stream)), "lbm_step_neural")


def lbm_step_slab(slab: Grid, f_in: torch.Tensor, f_out: torch.Tensor, tau: float,
                  force: torch.Tensor | None = None, z_begin: int = 0, z_end: int | None = None,
                  stream=None) -> None:
    """One step of slab planes [z_begin, z_end) (default: all) of a z-slab; f_in and
    f_out are slab buffers (nz + 2 planes), force holds the slab's own D*N reals."""
    N = slab.ncells
    words = slab.Q * slab.row_pitch * slab.ny * (slab.nz + 2)
    g = slab.c_struct()
    a = _dev_ptr(f_in, "f_in", slab.word_dtype, words)
    b = _dev_ptr(f_out, "f_out", slab.word_dtype, words)
    F = _dev_ptr(force, "force", slab.real_dtype, slab.D * N, required=False)
    z1 = slab.nz if z_end is None else int(z_end)
    _check(_lib.lbm_step_slab(ctypes.byref(g), a, b, float(tau), F, int(z_begin), z1, _stream(stream)),
           "lbm_step_slab")


def lbm_slab_halo_copy(src_slab: Grid, src: torch.Tensor, dst_slab: Grid, dst: torch.Tensor, face: str,
                       stream=None) -> None:
    """Copies the populations leaving src through `face` ("low" or "high") into the
    matching ghost plane of dst, the neighbouring slab on that side."""
    gs, gd = src_slab.c_struct(), dst_slab.c_struct()
    a = _dev_ptr(src, "src", src_slab.word_dtype, src_slab.Q * src_slab.row_pitch * src_slab.ny * (src_slab.nz + 2))
    b = _dev_ptr(dst, "dst", dst_slab.word_dtype, dst_slab.Q * dst_slab.row_pitch * dst_slab.ny * (dst_slab.nz + 2))
    _check(_lib.lbm_slab_halo_copy(ctypes.byref(gs), a, ctypes.byref(gd), b, FACES[face], _stream(stream)),
           "lbm_slab_halo_copy")


def lbm_step_slab2(slab: Grid, f_in: torch.Tensor, f_out: torch.Tensor, tau: float,
                   force: torch.Tensor | None = None, z_begin: int = 0, z_end: int | None = None,
                   stream=None) -> None:
    """Two steps of slab planes [z_begin, z_end) (default: all) of a z-slab with two ghost
    planes on each side; f_in and f_out are slab buffers (nz + 4 planes), force holds
    D*nx*ny*(nz + 2) reals (planes -1 .. nz)."""
    words = slab.Q * slab.row_pitch * slab.ny * (slab.nz + 4)
    g = slab.c_struct()
    a = _dev_ptr(f_in, "f_in", slab.word_dtype, words)
    b = _dev_ptr(f_out, "f_out", slab.word_dtype, words)
    F = _dev_ptr(force, "force", slab.real_dtype, slab.D * slab.nx * slab.ny * (slab.nz + 2), required=False)
    z1 = slab.nz if z_end is None else int(z_end)
    _check(_lib.lbm_step_slab2(ctypes.byref(g), a, b, float(tau), F, int(z_begin), z1, _stream(stream)),
           "lbm_step_slab2")


def lbm_step_slab2_available(slab: Grid) -> bool:
    """Whether lbm_step_slab2 takes this slab and storage kind (host-only)."""
    g = slab.c_struct()
    v = ctypes.c_int32(0)
    _check(_lib.lbm_step_slab2_available(ctypes.byref(g), ctypes.byref(v)), "lbm_step_slab2_available")
    return bool(v.value)


def lbm_slab2_halo_copy(src_slab: Grid, src: torch.Tensor, dst_slab: Grid, dst: torch.Tensor, face: str,
                        stream=None) -> None:
    """Fills the two ghost planes of dst (the neighbouring slab on `face`'s side of src)
    from src's two planes at that face."""
    gs, gd = src_slab.c_struct(), dst_slab.c_struct()
    a = _dev_ptr(src, "src", src_slab.word_dtype, src_slab.Q * src_slab.row_pitch * src_slab.ny * (src_slab.nz + 4))
    b = _dev_ptr(dst, "dst", dst_slab.word_dtype, dst_slab.Q * dst_slab.row_pitch * dst_slab.ny * (dst_slab.nz + 4))
    _check(_lib.lbm_slab2_halo_copy(ctypes.byref(gs), a, ctypes.byref(gd), b, FACES[face], _stream(stream)),
           "lbm_slab2_halo_copy")


def lbm_stream_only(grid: Grid, f_in: torch.Tensor, f_out: torch.Tensor, stream=None) -> None:
    N = grid.ncells
    g = grid.c_struct()
    a = _dev_ptr(f_in, "f_in", grid.word_dtype, grid.pop_size)
    b = _dev_ptr(f_out, "f_out", grid.word_dtype, grid.pop_size)
    _check(_lib.lbm_stream_only(ctypes.byref(g), a, b, _stream(stream)), "lbm_stream_only")


def lbm_copy(src: torch.Tensor, dst: torch.Tensor, stream=None) -> None:
    """dst <- src byte for byte (same number of bytes, a multiple of 16)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("src and dst must have the same size in bytes")
    a = _dev_ptr(src, "src", src.dtype, src.numel())
    b = _dev_ptr(dst, "dst", dst.dtype, dst.numel())
    _check(_lib.lbm_copy(a, b, ctypes.c_size_t(nbytes), _stream(stream)), "lbm_copy")


def lbm_step_launches(grid: Grid, n_steps: int) -> tuple:
    """(single, paired, quad): how lbm_step splits n_steps into one-step, two-step and
    four-step launches (host-side, no device work)."""
    g = grid.c_struct()
    single, paired, quad = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(_lib.lbm_step_launches(ctypes.byref(g), int(n_steps), ctypes.byref(single), ctypes.byref(paired),
                                  ctypes.byref(quad)), "lbm_step_launches")
    return single.value, paired.value, quad.value


def lbm_moments_workspace_size(grid: Grid) -> int:
    g = grid.c_struct()
    n = ctypes.c_size_t()
    _check(_lib.lbm_moments_workspace_size(ctypes.byref(g), ctypes.byref(n)), "lbm_moments_workspace_size")
    return n.value


def lbm_moments(grid: Grid, f: torch.Tensor, force: torch.Tensor | None = None,
                rho_out: torch.Tensor | None = None, u_out: torch.Tensor | None = None,
                red: torch.Tensor | None = None, workspace: torch.Tensor | None = None, stream=None) -> None:
    """Density/velocity fields and (if red is given) the 8 FP64 reductions.

    red: float64 GPU tensor of 8 elements.  workspace: uint8 GPU tensor of at least
    lbm_moments_workspace_size(grid) bytes (required with red).
    """
    N = grid.ncells
    g = grid.c_struct()
    ws_ptr, ws_bytes = None, 0
    if red is not None:
        need = lbm_moments_workspace_size(grid)
        if workspace is None or workspace.dtype != torch.uint8 or workspace.numel() < need:
            raise ValueError(f"workspace must be a uint8 GPU tensor of >= {need} bytes")
        ws_ptr = _dev_ptr(workspace, "workspace", torch.uint8, workspace.numel())
        ws_bytes = workspace.numel()
    args = (_dev_ptr(f, "f", grid.word_dtype, grid.pop_size),
            _dev_ptr(force, "force", grid.real_dtype, grid.D * N, required=False),
            _dev_ptr(rho_out, "rho_out", grid.real_dtype, N, required=False),
            _dev_ptr(u_out, "u_out", grid.real_dtype, grid.D * N, required=False),
            _dev_ptr(red, "red", torch.float64, NRED, required=False))
    _check(_lib.lbm_moments(ctypes.byref(g), *args, ws_ptr, ctypes.c_size_t(ws_bytes), _stream(stream)),
           "lbm_moments")


def lbm_moments_noalloc(grid: Grid, f: torch.Tensor, force: torch.Tensor | None = None,
                        rho_out: torch.Tensor | None = None, u_out: torch.Tensor | None = None,
                        red: torch.Tensor | None = None, stream=None) -> None:
    """lbm_moments with the reduction partials in the library's fixed device scratch
    (no workspace, no allocation; calls on one GPU must not overlap)."""
    N = grid.ncells
    g = grid.c_struct()
    args = (_dev_ptr(f, "f", grid.word_dtype, grid.pop_size),
            _dev_ptr(force, "force", grid.real_dtype, grid.D * N, required=False),
            _dev_ptr(rho_out, "rho_out", grid.real_dtype, N, required=False),
            _dev_ptr(u_out, "u_out", grid.real_dtype, grid.D * N, required=False),
            _dev_ptr(red, "red", torch.float64, NRED, required=False))
    _check(_lib.lbm_moments_noalloc(ctypes.byref(g), *args, _stream(stream)), "lbm_moments_noalloc")


def lbm_adjoint_step(grid: Grid, g_t: torch.Tensor, lam_next: torch.Tensor, lam_out: torch.Tensor, tau: float,
                     force: torch.Tensor | None = None, dforce: torch.Tensor | None = None, stream=None) -> None:
    """lam_out <- (dg'/dg_t)^T lam_next; dforce += (dg'/dF)^T lam_next."""
    N = grid.ncells
    g = grid.c_struct()
    args = (_dev_ptr(g_t, "g_t", grid.word_dtype, grid.pop_size),
            _dev_ptr(lam_next, "lam_next", grid.real_dtype, grid.pop_size),
            _dev_ptr(lam_out, "lam_out", grid.real_dtype, grid.pop_size))
    F = _dev_ptr(force, "force", grid.real_dtype, grid.D * N, required=False)
    dF = _dev_ptr(dforce, "dforce", grid.real_dtype, grid.D * N, required=False)
    _check(_lib.lbm_adjoint_step(ctypes.byref(g), *args, float(tau), F, dF, _stream(stream)), "lbm_adjoint_step")


def lbm_adjoint_step_local(grid: Grid, g_t: torch.Tensor, adj_next: torch.Tensor, adj_is_chi: bool,
                           chi_out: torch.Tensor, tau: float, force: torch.Tensor | None = None,
                           dforce: torch.Tensor | None = None, stream=None) -> None:
    """chi_out <- J_C^T lam_{t+1} with lam_{t+1} = adj_next or S^T adj_next (adj_is_chi);
    dforce += (dC/dF)^T lam_{t+1}."""
    N = grid.ncells
    g = grid.c_struct()
    args = (_dev_ptr(g_t, "g_t", grid.word_dtype, grid.pop_size),
            _dev_ptr(adj_next, "adj_next", grid.real_dtype, grid.pop_size))
    out = _dev_ptr(chi_out, "chi_out", grid.real_dtype, grid.pop_size)
    F = _dev_ptr(force, "force", grid.real_dtype, grid.D * N, required=False)
    dF = _dev_ptr(dforce, "dforce", grid.real_dtype, grid.D * N, required=False)
    _check(_lib.lbm_adjoint_step_local(ctypes.byref(g), *args, 1 if adj_is_chi else 0, out, float(tau), F, dF,
                                       _stream(stream)), "lbm_adjoint_step_local")


def lbm_adjoint_step2_local(grid: Grid, g_t: torch.Tensor, g_tm1: torch.Tensor, chi_next: torch.Tensor,
                            chi_out: torch.Tensor, tau: float, force: torch.Tensor | None = None,
                            dforce: torch.Tensor | None = None, stream=None) -> None:
    """chi_out <- two collision-local adjoint steps (states g_t, then g_tm1) from chi_next;
    dforce += both steps' force gradients, in the order of two one-step calls."""
    N = grid.ncells
    g = grid.c_struct()
    a = _dev_ptr(g_t, "g_t", grid.word_dtype, grid.pop_size)
    b = _dev_ptr(g_tm1, "g_tm1", grid.word_dtype, grid.pop_size)
    c = _dev_ptr(chi_next, "chi_next", grid.real_dtype, grid.pop_size)
    out = _dev_ptr(chi_out, "chi_out", grid.real_dtype, grid.pop_size)
    F = _dev_ptr(force, "force", grid.real_dtype, grid.D * N, required=False)
    dF = _dev_ptr(dforce, "dforce", grid.real_dtype, grid.D * N, required=False)
    _check(_lib.lbm_adjoint_step2_local(ctypes.byref(g), a, b, c, out, float(tau), F, dF, _stream(stream)),
           "lbm_adjoint_step2_local")


def lbm_adjoint_step2_available(grid: Grid) -> bool:
    """Whether lbm_adjoint_step2_local takes this grid and storage kind (host-only)."""
    g = grid.c_struct()
    v = ctypes.c_int32(0)
    _check(_lib.lbm_adjoint_step2_available(ctypes.byref(g), ctypes.byref(v)), "lbm_adjoint_step2_available")
    return bool(v.value)


def lbm_adjoint_unstream(grid: Grid, chi: torch.Tensor, lam_out: torch.Tensor, stream=None) -> None:
    """lam_out <- S^T chi."""
    N = grid.ncells
    g = grid.c_struct()
    a = _dev_ptr(chi, "chi", grid.real_dtype, grid.pop_size)
    b = _dev_ptr(lam_out, "lam_out", grid.real_dtype, grid.pop_size)
    _check(_lib.lbm_adjoint_unstream(ctypes.byref(g), a, b, _stream(stream)), "lbm_adjoint_unstream")


def lbm_moments_adjoint(grid: Grid, f: torch.Tensor, force: torch.Tensor | None,
                        dL_drho: torch.Tensor | None, dL_du: torch.Tensor | None, lam_out: torch.Tensor,
                        dforce: torch.Tensor | None = None, stream=None) -> None:
    """lam_out <- d(rho, u)/dg ^T (dL_drho, dL_du); dforce += -dL_du/(2 rho)."""
    N = grid.ncells
    g = grid.c_struct()
    args = (_dev_ptr(f, "f", grid.word_dtype, grid.pop_size),
            _dev_ptr(force, "force", grid.real_dtype, grid.D * N, required=False),
            _dev_ptr(dL_drho, "dL_drho", grid.real_dtype, N, required=False),
            _dev_ptr(dL_du, "dL_du", grid.real_dtype, grid.D * N, required=False),
            _dev_ptr(lam_out, "lam_out", grid.real_dtype, grid.pop_size),
            _dev_ptr(dforce, "dforce", grid.real_dtype, grid.D * N, required=False))
    _check(_lib.lbm_moments_adjoint(ctypes.byref(g), *args, _stream(stream)), "lbm_moments_adjoint")


def bytes_per_cell_step(grid: Grid) -> int:
    """Algorithmic HBM bytes of one step per cell: read and write Q stored words."""
    return 2 * grid.Q * torch.tensor([], dtype=grid.word_dtype).element_size()


def mlups(grid: Grid, steps: int, seconds: float) -> float:
    return grid.ncells * steps / seconds / 1e6


@dataclass(frozen=True)
class ShellTable:
    """Wavevectors of a periodic grid grouped by shell, as lbm_shells wants them (int32
    device arrays): order sorts the flat wavevector indices by shell, shell K holds
    order[offsets[K]:offsets[K+1]], shell gives every wavevector's shell."""

    n: int
    nshell: int
    order: torch.Tensor
    offsets: torch.Tensor
    shell: torch.Tensor

    @staticmethod
    def from_shells(shell: torch.Tensor) -> "ShellTable":
        """From the shell index of every flat wavevector (non-negative integers, GPU)."""
        flat = shell.reshape(-1).to(torch.int64)
        counts = torch.bincount(flat)
        offsets = torch.zeros(counts.numel() + 1, dtype=torch.int64, device=flat.device)
        offsets[1:] = torch.cumsum(counts, 0)
        order = torch.argsort(flat, stable=True)
        return ShellTable(flat.numel(), counts.numel(), order.to(torch.int32).contiguous(),
                          offsets.to(torch.int32).contiguous(), flat.to(torch.int32).contiguous())

    def c_struct(self) -> _CShells:
        _dev_ptr(self.order, "order", torch.int32, self.n)
        _dev_ptr(self.offsets, "offsets", torch.int32, self.nshell + 1)
        _dev_ptr(self.shell, "shell", torch.int32, self.n)
        return _CShells(self.n, self.nshell, self.order.data_ptr(), self.offsets.data_ptr(), self.shell.data_ptr())


def _spectral_field(t: torch.Tensor, name: str, table: ShellTable) -> tuple[int, ctypes.c_void_p]:
    """(D, pointer) of a [D, ...] complex128 field over table.n wavevectors."""
    D = t.shape[0] if t.dim() > 0 else 0
    if D < 1 or D > 3:
        raise ValueError(f"{name} must be [D, ...] with D in 1..3")
    return D, _dev_ptr(t, name, torch.complex128, D * table.n)


def lbm_shell_energy(table: ShellTable, uhat: torch.Tensor, scale: float, E: torch.Tensor, stream=None) -> None:
    """E[K] <- scale^2/2 * sum over shell K of sum_a |uhat_a(k)|^2 (uhat: unnormalised
    FFT of u, [D, *spatial] complex128; E: nshell float64)."""
    D, p = _spectral_field(uhat, "uhat", table)
    e = _dev_ptr(E, "E", torch.float64, table.nshell)
    c = table.c_struct()
    _check(_lib.lbm_shell_energy(ctypes.byref(c), D, p, float(scale), e, _stream(stream)), "lbm_shell_energy")


def lbm_log_spectrum_grad(table: ShellTable, uhat: torch.Tensor, E: torch.Tensor, E_target: torch.Tensor,
                          k_lo: int, k_hi: int, cutoff: float, scale: float, R: torch.Tensor | None = None,
                          stream=None) -> None:
    """uhat *= scale * dR/dE at each wavevector's shell, in place (R the log-spectrum
    cost over shells k_lo..k_hi with cutoff c); R (one float64) receives the cost."""
    D, p = _spectral_field(uhat, "uhat", table)
    e = _dev_ptr(E, "E", torch.float64, table.nshell)
    et = _dev_ptr(E_target, "E_target", torch.float64, table.nshell)
    r = _dev_ptr(R, "R", torch.float64, 1, required=False)
    c = table.c_struct()
    _check(_lib.lbm_log_spectrum_grad(ctypes.byref(c), D, p, e, et, int(k_lo), int(k_hi), float(cutoff),
                                      float(scale), r, _stream(stream)), "lbm_log_spectrum_grad")


def lbm_real_part(z: torch.Tensor, scale: float, out: torch.Tensor, stream=None) -> None:
    """out <- scale * Re z elementwise (z complex128; out float32 or float64, same count)."""
    if out.dtype not in (torch.float32, torch.float64):
        raise TypeError("out must be float32 or float64")
    zp = _dev_ptr(z, "z", torch.complex128, z.numel())
    op = _dev_ptr(out, "out", out.dtype, z.numel())
    kind = STORAGES["f64"] if out.dtype == torch.float64 else STORAGES["f32"]
    _check(_lib.lbm_real_part(zp, ctypes.c_int64(z.numel()), float(scale), op, kind, _stream(stream)),
           "lbm_real_part")


__all__ = [n for n in dir() if n.startswith("lbm_")] + ["Grid", "LbmError", "NRED", "RED_NAMES", "LIB_PATH",
                                                        "ShellTable", "bytes_per_cell_step", "mlups"]
