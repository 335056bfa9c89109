"""Pins for oracle.prior: Philox known answers, Box-Muller invariants, the N(0,1) law."""
import os

import numpy as np
import pytest
from scipy import stats

from oracle.prior import (box_muller, log_prior, philox4x32_10, prior_normal,
                          prior_uniforms, words_to_unit)

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def kat_rows():
    rows = []
    for line in open(GOLD):
        if line.strip() and not line.startswith("#"):
            rows.append([int(x, 16) for x in line.split()])
    return rows


@pytest.mark.parametrize("row", kat_rows())
def test_philox_known_answers(row):
    out = philox4x32_10(tuple(np.uint64(x) for x in row[:4]), tuple(np.uint64(x) for x in row[4:6]))
    assert [int(o) for o in out] == row[6:]


def test_unit_map_open_interval_and_fp32_exact():
    x = np.array([0, 1, 255, 256, 2**31, 2**32 - 1], dtype=np.uint64)
    u = words_to_unit(x)
    assert np.all(u > 0) and np.all(u < 1)
    assert np.array_equal(u.astype(np.float32).astype(np.float64), u)
    assert u[0] == 0.5 * 2.0 ** -23 and u[-1] == 1 - 0.5 * 2.0 ** -23


def test_box_muller_polar_invariants():
    rng = np.random.default_rng(0)
    ua, ub = rng.random(1000) * 0.999 + 0.0005, rng.random(1000)
    za, zb = box_muller(ua, ub)
    # radius and angle recover the two uniforms: this fixes the transform completely
    np.testing.assert_allclose(za ** 2 + zb ** 2, -2 * np.log(ua), rtol=1e-12)
    ang = np.mod(np.arctan2(zb, za), 2 * np.pi)
    d = np.abs(ang - 2 * np.pi * ub)
    assert np.all(np.minimum(d, 2 * np.pi - d) < 1e-9)


def test_prior_site_pairing_uses_stream_layout():
    key, c0, B, V = 12345, 7, 3, 16
    z = prior_normal(key, c0, B, V)
    u0, u1, u2, u3 = prior_uniforms(key, c0, B, V)
    np.testing.assert_allclose(z[:, 0::4] ** 2 + z[:, 1::4] ** 2, -2 * np.log(u0), rtol=1e-12)
    np.testing.assert_allclose(z[:, 2::4] ** 2 + z[:, 3::4] ** 2, -2 * np.log(u2), rtol=1e-12)
    # sample b of a draw at base c0 equals sample 0 of a draw at base c0 + b
    z2 = prior_normal(key, c0 + 2, 1, V)
    np.testing.assert_array_equal(z[2], z2[0])


def test_prior_is_standard_normal():
    z = prior_normal(12345, 0, 64, 1024).ravel()
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 5 / np.sqrt(z.size)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / z.size)
    zz = z.reshape(64, 1024)
    c = np.corrcoef(zz[:, :-1].ravel(), zz[:, 1:].ravel())[0, 1]
    assert abs(c) < 5 / np.sqrt(z.size)


def test_log_prior_matches_scipy():
    z = np.random.default_rng(1).standard_normal((5, 4, 4))
    ref = stats.norm.logpdf(z).reshape(5, -1).sum(axis=1)
    np.testing.assert_allclose(log_prior(z), ref, rtol=1e-13)
