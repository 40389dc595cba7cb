"""Shared helpers of the GPU parity tests (not collected by pytest)."""
import sys

import torch

INT_VIEW = {1: torch.int8, 2: torch.int16, 4: torch.int32, 8: torch.int64}


def bits(t: torch.Tensor) -> torch.Tensor:
    """Raw storage words of a tensor as signed integers (for bit-exact comparisons)."""
    return t.contiguous().view(INT_VIEW[t.element_size()])


def say(*args) -> None:
    """Print a line that names the case before GPU work, flushed at once."""
    print(*args, flush=True)
    sys.stdout.flush()


def need_gpu():
    import pytest

    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def binding():
    """The HIP binding; importing it loads liblbm.so (raises if it is not built)."""
    from paper_2106_12929_amd import binding as B

    return B


def rel_l2(a: torch.Tensor, b: torch.Tensor) -> float:
    a = a.double().cpu()
    b = b.double().cpu()
    return float((a - b).norm() / b.norm())


def err_in_ulps(got: torch.Tensor, ref: torch.Tensor, ulp: torch.Tensor) -> torch.Tensor:
    return (got.double().cpu() - ref.double().cpu()).abs() / ulp
