"""Pins of the oracle's emulated storage precisions (oracle/rounding.py and the
flow oracle's `emulate` option) against exact values and invariants."""
import struct

import numpy as np
import pytest

import seeded_inputs as si
from oracle import flow as of
from oracle.rounding import to_bf16, to_fp32


def _f32(bits):
    return struct.unpack("<f", struct.pack("<I", bits))[0]


@pytest.mark.parametrize("x,expect", [
    (1.0, 1.0),
    (1.0 + 2.0 ** -8, 1.0),                          # halfway, ties to even (down)
    (1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -6),          # halfway, ties to even (up)
    (1.0 + 2.0 ** -8 + 2.0 ** -20, 1.0 + 2.0 ** -7),  # above halfway
    (-(1.0 + 2.0 ** -8), -1.0),
    (0.1, _f32(0x3DCD0000)),                         # 0x3DCCCCCD rounds up
    (2.0 ** -133, 2.0 ** -133),                      # subnormal with only upper bits
    (2.0 ** -149, 0.0),                              # lowest subnormal bit rounds away
    (3.0 * 2.0 ** 100, 3.0 * 2.0 ** 100),
])
def test_bf16_exact_values(x, expect):
    assert to_bf16(np.array([x]))[0] == expect


def test_fp32_is_the_binary32_cast():
    x = np.random.default_rng(3).standard_normal(1000) * 10.0 ** np.random.default_rng(4).integers(-30, 30, 1000)
    ref = np.array([struct.unpack("<f", struct.pack("<f", v))[0] for v in x])
    assert np.array_equal(to_fp32(x), ref)


def test_bf16_is_nearest_and_idempotent():
    x = np.random.default_rng(5).standard_normal(4000) * 7.3
    r = to_bf16(x)
    assert np.array_equal(to_bf16(r), r)
    # nearest: no BF16 neighbour of r (one unit in the last place either side) is closer
    u = np.frexp(np.abs(r))[1]
    ulp = np.ldexp(1.0, u - 8)
    assert np.all(np.abs(x - r) <= 0.5 * ulp * (1 + 1e-12))


def test_emulation_changes_nothing_on_exact_operands():
    """With every conv operand representable in BF16 (fields in {0,1}, weights in
    {0, 1/4}, non-negative so LeakyReLU is the identity and the hidden values are
    short sums of quarters), the emulated network equals the FP64 one exactly."""
    fs = of.FlowShape(2, 4, 1, 8)
    rng = np.random.default_rng(11)
    p = np.where(rng.random(si.param_count(2, 1, 8)) < 0.1, 0.25, 0.0)
    lay = of.unpack(p, fs)[0]
    x = of.as_lattice(rng.integers(0, 2, (3, 16)).astype(np.float64), fs)
    mF = of.frozen_mask(fs, 0)
    def flat(out):  # (acts, hs, o, s, t) -> list of arrays
        acts, hs, *rest = out
        return list(acts) + list(hs) + rest

    plain = of.net(x, lay, mF, fs)
    h1, h2 = plain[1][1], plain[1][2]
    assert np.array_equal(to_bf16(h1), h1) and np.array_equal(to_bf16(h2), h2)
    for mode in ("bf16", "fp32"):
        emu = of.net(x, lay, mF, fs, emulate=mode)
        for a, b in zip(flat(plain), flat(emu)):
            assert np.array_equal(a, b)


def test_emulation_error_orders_by_precision():
    fs = of.FlowShape(2, 8, 4, 8)
    p = si.flow_params(2, 4, 8, seed=9, w_std=0.1, b_std=0.05).astype(np.float64)
    z = si.normal_fields(10, 4, 64)
    ref = of.flow_forward(p, z, fs)["phi"]
    e32 = np.max(np.abs(of.flow_forward(p, z, fs, emulate="fp32")["phi"] - ref))
    e16 = np.max(np.abs(of.flow_forward(p, z, fs, emulate="bf16")["phi"] - ref))
    assert 0 < e32 < 1e-5 * np.max(np.abs(ref)) and e32 * 100 < e16
