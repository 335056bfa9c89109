"""Rounding of FP64 arrays to FP32 and to BF16 values (returned as FP64) -- the
oracle's emulation of stored operand precisions.  TEST INFRASTRUCTURE ONLY.

The flow oracle can evaluate the method with the operands of every convolution
(inputs and weights) rounded to FP32 or to BF16 and the field kept in FP32
between layers, everything else in FP64.  The parity tests use it to size
tolerances: how far rounding the stored operands alone moves a result from the
FP64 value bounds how far any implementation that stores them so can be
expected to be.

  to_fp32: IEEE round-to-nearest-even to binary32 (numpy's cast).
  to_bf16: round-to-nearest-even of the binary32 value to its upper 16 bits
           (8 exponent bits, 7 fraction bits); FP64 inputs are first rounded to
           binary32, as a binary32 value would be.  Non-finite values are not
           expected and not treated specially.

Pinned by exact values: ties to even at 1 + 2^-8 and 1 + 3 2^-8, rounding of
0.1, halfway cases below the smallest normal, and agreement with the cast.
"""
from __future__ import annotations

import numpy as np


def to_fp32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def to_bf16(x):
    u = np.asarray(x, dtype=np.float64).astype(np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


ROUNDERS = {"fp32": to_fp32, "bf16": to_bf16}
