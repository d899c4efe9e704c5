"""The bound the channel scan uses to skip null candidates.

An interpolated cumulative probability a + t (b - a) with 0 <= t <= 1,
evaluated in the particle precision with one rounding per operation, never
exceeds max(a, b) (1 + 2^-21) in FP32 (2^-50 in FP64) rounded to that
precision; so a random number at or above that bound hits no channel and
the scan may stop there without changing any selection.  Checked on random
and adversarial operands (equal, adjacent and far-apart rows, t at 0 and 1,
values spanning many binades).
"""
import numpy as np
import pytest


@pytest.mark.parametrize("dt,slack", [(np.float32, 2.0 ** -21), (np.float64, 2.0 ** -50)])
def test_interpolated_row_never_exceeds_the_bound(dt, slack):
    rng = np.random.default_rng(7)
    n = 1_000_000
    a = rng.random(n).astype(dt) * dt(0.3)
    b = rng.random(n).astype(dt) * dt(0.3)
    # adjacent values and equal rows
    k = n // 4
    b[:k] = np.nextafter(a[:k], dt(1.0))
    a[k:2 * k] = b[k:2 * k]
    # many binades
    e = rng.integers(-40, 0, size=n)
    sc = np.ldexp(np.ones(n), e).astype(dt)
    a[2 * k:3 * k] *= sc[2 * k:3 * k]
    b[2 * k:3 * k] *= sc[2 * k:3 * k]
    t = rng.random(n).astype(dt)
    t[:1000] = dt(0.0)
    t[1000:2000] = dt(1.0)
    t[2000:3000] = np.nextafter(dt(1.0), dt(0.0))
    p = a + t * (b - a)  # each operation rounded to dt
    assert p.dtype == dt
    top = np.maximum(a, b) * dt(1.0 + slack)
    assert top.dtype == dt
    assert np.all(p <= top)
