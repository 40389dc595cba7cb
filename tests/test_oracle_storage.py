"""Pins of the oracle's stored-population formats (shifted FP16/BF16/FP32 storage)."""
import numpy as np
import pytest
import torch

import synthetic
from oracle import lbm, storage


@pytest.mark.parametrize("name", ["D2Q9", "D3Q27"])
@pytest.mark.parametrize("kind", storage.KINDS)
def test_rest_state_exact(name, kind):
    # rho = 1, u = 0 is the equilibrium w_i: shifted storage holds exact zeros, and a
    # step moves the populations by FP64 roundoff only (sum_i w_i is 1 only to
    # roundoff in binary64), which binary16 rounds back to exact zeros.
    st = lbm.stencil(name)
    spatial = (3,) * st.D
    f = lbm.equilibrium(torch.ones(spatial, dtype=torch.float64),
                        torch.zeros((st.D,) + spatial, dtype=torch.float64), st)
    s = storage.quantize(f, st, kind)
    if storage.is_shifted(kind):
        assert torch.count_nonzero(s) == 0
    s1 = storage.step_emulated(s, 0.6, st, kind)
    diff = storage.dequantize(s1, st, kind) - storage.dequantize(s, st, kind)
    assert float(diff.abs().max()) <= 4 * 2.0 ** -52
    if kind == "f16s":  # below half the smallest binary16 subnormal
        assert torch.count_nonzero(s1) == 0


def test_f16_rounding_is_ieee_nearest_even():
    # numpy's float16 conversion is an independent IEEE binary16 implementation.
    st = lbm.stencil("D2Q9")
    d = synthetic.random_normal((st.Q, 16, 16), 41, 1e-3)
    d[0, 0, :4] = torch.tensor([1e-7, -3e-8, 6.0e-5, 65000.0], dtype=torch.float64)
    f = d + st.w.reshape(-1, 1, 1)
    s = storage.quantize(f, st, "f16s")
    ref = (f - st.w.reshape(-1, 1, 1)).numpy().astype(np.float32).astype(np.float16)
    assert np.array_equal(s.numpy().view(np.uint16), ref.view(np.uint16))


def test_bf16_rounding_is_nearest_even():
    # bfloat16 is the upper half of binary32; round-to-nearest-even on the dropped
    # 16 bits, written out with integer arithmetic.
    x = synthetic.random_normal((4096,), 42, 1e-2).to(torch.float32)
    bits = x.numpy().view(np.uint32).astype(np.uint64)
    lower = bits & 0xFFFF
    upper = bits >> 16
    up = (lower > 0x8000) | ((lower == 0x8000) & ((upper & 1) == 1))
    expect = (upper + up).astype(np.uint16)
    got = x.to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(got, expect)


@pytest.mark.parametrize("kind", storage.KINDS)
def test_quantize_dequantize(kind):
    st = lbm.stencil("D3Q27")
    rho, u = synthetic.random_fields((3, 4, 5), 3, 43)
    f = lbm.equilibrium(rho, u, st)
    s = storage.quantize(f, st, kind)
    assert s.dtype == storage.dtype_of(kind)
    back = storage.dequantize(s, st, kind)
    err = (back - f).abs()
    ref = (f - st.w.reshape(-1, 1, 1, 1)).abs() if storage.is_shifted(kind) else f.abs()
    assert bool((err <= 0.5 * storage.ulp(ref, kind) * (1 + 1e-12)).all())
    # and re-quantising the dequantised value is the identity (exact round trip)
    assert torch.equal(storage.quantize(back, st, kind).view(torch.uint8), s.view(torch.uint8))


def test_f64_emulated_step_is_the_step():
    st = lbm.stencil("D2Q9")
    rho, u = synthetic.random_fields((6, 7), 2, 44)
    f = lbm.equilibrium(rho, u, st)
    assert torch.equal(storage.step_emulated(f, 0.6, st, "f64"), lbm.step(f, 0.6, st))


def test_ulp_values():
    one = torch.tensor([1.0, 1e-3, 2.0 ** -20], dtype=torch.float64)
    assert storage.ulp(one, "f16s").tolist() == [2.0 ** -10, 2.0 ** -20, 2.0 ** -24]
    assert storage.ulp(one, "bf16s").tolist()[0] == 2.0 ** -7
    assert storage.ulp(one, "f32").tolist()[0] == 2.0 ** -23
