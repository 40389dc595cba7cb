"""Population storage formats and the emulated reduced-precision step (oracle side).

Test infrastructure, like the rest of `oracle/`.

A stored population buffer holds, per storage kind:
    "f64"    f_i as float64
    "f32"    f_i as float32
    "f32s"   d_i = f_i - w_i as float32      ("shifted" storage)
    "f16s"   d_i = f_i - w_i as IEEE binary16
    "bf16s"  d_i = f_i - w_i as bfloat16
Rounding is IEEE round-to-nearest-even with subnormals kept, which is what torch's
dtype casts do.  The paper keeps populations in the working precision of PyTorch
(FP32 or FP64, Sec. 3.3); the shifted 16-bit forms are this library's extension and
are checked here by emulation: dequantise to FP64, take one exact FP64 step, round
the result back.
"""
from __future__ import annotations

import torch

from . import lbm
from . import neural as nn_oracle

KINDS = ("f64", "f32", "f32s", "f16s", "bf16s")
_DTYPE = {"f64": torch.float64, "f32": torch.float32, "f32s": torch.float32,
          "f16s": torch.float16, "bf16s": torch.bfloat16}


def is_shifted(kind: str) -> bool:
    return kind.endswith("s")


def dtype_of(kind: str) -> torch.dtype:
    return _DTYPE[kind]


def _w(st: lbm.Stencil, nd: int) -> torch.Tensor:
    return st.w.reshape((st.Q,) + (1,) * nd)


def quantize(f: torch.Tensor, st: lbm.Stencil, kind: str) -> torch.Tensor:
    """FP64 populations -> stored representation (one rounding)."""
    x = f.to(torch.float64)
    if is_shifted(kind):
        x = x - _w(st, f.dim() - 1)
    return x.to(_DTYPE[kind])


def dequantize(s: torch.Tensor, st: lbm.Stencil, kind: str) -> torch.Tensor:
    """Stored representation -> FP64 populations (exact)."""
    x = s.to(torch.float64)
    if is_shifted(kind):
        x = x + _w(st, s.dim() - 1)
    return x


def step_emulated(s: torch.Tensor, tau: float, st: lbm.Stencil, kind: str,
                  force: torch.Tensor | None = None, du: torch.Tensor | None = None,
                  mrt_taus=None, neural=None) -> torch.Tensor:
    """One pull step on stored populations: dequantise, exact FP64 step, quantise.
    With `du` the step uses the shifted-velocity equilibrium instead of a force; with
    `mrt_taus` (9 relaxation times) the MRT collision of Eq. 5; with
    `neural` = (params, activation) the neural collision of Sec. 3.1 with shear time
    `tau`."""
    f = dequantize(s, st, kind)
    if neural is not None:
        out = nn_oracle.step(f, tau, neural[0], neural[1], st)
    elif mrt_taus is not None:
        out = lbm.step_mrt(f, mrt_taus, st)
    elif du is not None:
        out = lbm.step_shifted(f, tau, st, du)
    else:
        out = lbm.step(f, tau, st, force)
    return quantize(out, st, kind)


def step_at_cells_emulated(s: torch.Tensor, tau: float, st: lbm.Stencil, kind: str, cells: torch.Tensor,
                           force: torch.Tensor | None = None) -> torch.Tensor:
    """`step_emulated` evaluated at the listed cells only ([M, D] coordinates):
    gathers the streamed stored words, dequantises, takes the FP64 collision and
    returns the FP64 populations [Q, M] (before the final rounding to storage)."""
    h = lbm.gather_at_cells(s, st, cells)
    if is_shifted(kind):
        h = h + st.w.reshape(st.Q, 1)
    F = None if force is None else lbm.force_at_cells(force, st, cells)
    return lbm.bgk_collide(h, tau, st, F)


def stream_stored(s: torch.Tensor, st: lbm.Stencil) -> torch.Tensor:
    """Streaming applied to the stored words themselves: a permutation, so no
    arithmetic and no rounding is involved, whatever the storage dtype."""
    return lbm.stream(s, st)


def ulp(x: torch.Tensor, kind: str) -> torch.Tensor:
    """Spacing of the storage format at |x| (the gap to the next larger magnitude),
    in FP64.  Subnormal spacing is used below the smallest normal."""
    dt = _DTYPE[kind]
    fi = torch.finfo(dt)
    mant_bits = {torch.float64: 52, torch.float32: 23, torch.float16: 10, torch.bfloat16: 7}[dt]
    a = x.abs().to(torch.float64)
    e = torch.floor(torch.log2(torch.clamp(a, min=fi.tiny)))
    return torch.pow(2.0, e - mant_bits).clamp(min=fi.tiny * 2.0 ** -mant_bits)
