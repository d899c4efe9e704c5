"""Pins of the oracle's leapfrog push with linear gather (closed-form
trajectories) and of wall removal."""
import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("precision", [0, 1])
def test_free_streaming_is_exact_for_dyadic_velocities(precision):
    nc, steps = 1024, 200
    kdz = 2.0 ** -10
    rng = np.random.default_rng(precision)
    n = 500
    cell = rng.integers(300, 700, n)
    off = rng.integers(0, 256, n) / 256.0
    vz = rng.integers(-64, 65, n) * 2.0  # v kdz = k/512 cells per step, dyadic
    Ep = np.zeros(nc + 1)
    c2, o2, v2, st = oracle.push(precision, cell, off, vz, Ep, nc, kdz, steps)
    z_exact = cell + off + steps * vz * kdz
    assert (st == 0).all()
    np.testing.assert_array_equal(c2 + o2.astype(np.float64), z_exact)
    np.testing.assert_array_equal(v2, vz)
    assert (o2 >= 0).all() and (o2 < 1).all()


@pytest.mark.parametrize("precision", [0, 1])
def test_uniform_field_leapfrog_closed_form(precision):
    # Leapfrog is exact for constant acceleration:
    # v^{n+1/2} = v^{-1/2} + (n+1) a,  s^{n} = s^0 + kdz (n v^{-1/2} + a n (n+1) / 2).
    nc, steps = 4096, 100
    kdz = 2.0 ** -12
    a = 2.0 ** -3  # per-step velocity increment in the node array E'
    n = 64
    cell = np.full(n, 1500)
    off = np.arange(n) / 64.0
    v0 = np.arange(-32, 32) * 8.0  # dyadic, so every step is exact
    Ep = np.full(nc + 1, a)
    c2, o2, v2, st = oracle.push(precision, cell, off, v0, Ep, nc, kdz, steps)
    assert (st == 0).all()
    s_exact = cell + off + kdz * (steps * v0 + a * steps * (steps + 1) / 2)
    np.testing.assert_array_equal(v2, v0 + steps * a)
    np.testing.assert_array_equal(c2 + o2.astype(np.float64), s_exact)


def test_linear_gather_interpolates_between_nodes():
    nc, kdz = 8, 0.0
    Ep = np.arange(nc + 1, dtype=np.float64) * 0.5  # E'_j = j/2
    cell = np.array([0, 3, 3, 7])
    off = np.array([0.0, 0.25, 0.5, 0.75])
    c2, o2, v2, st = oracle.push(1, cell, off, np.zeros(4), Ep, nc, kdz, 1)
    np.testing.assert_array_equal(v2, 0.5 * (cell + off))


def test_walls_remove_at_predicted_step():
    nc, kdz = 16, 1.0
    # left-moving: from z = 3.5 cells at -0.25 cells/step, exits after 15 steps
    c2, o2, v2, st = oracle.push(1, [3], [0.5], [-0.25], np.zeros(nc + 1), nc, kdz, 14)
    assert st[0] == 0 and c2[0] == 0 and o2[0] == 0.0
    c2, o2, v2, st = oracle.push(1, [3], [0.5], [-0.25], np.zeros(nc + 1), nc, kdz, 15)
    assert st[0] == 1
    # right-moving: from 14.5 at +0.5 exits when s reaches 16 (3 steps)
    c2, o2, v2, st = oracle.push(1, [14], [0.5], [0.5], np.zeros(nc + 1), nc, kdz, 2)
    assert st[0] == 0 and c2[0] == 15 and o2[0] == 0.5
    c2, o2, v2, st = oracle.push(1, [14], [0.5], [0.5], np.zeros(nc + 1), nc, kdz, 3)
    assert st[0] == 2


def test_offset_rounding_to_one_stays_in_cell():
    # s = off + v kdz slightly below 0 -> floor = -1 and s - floor rounds to 1
    # in float: the particle is placed at (c, 0), never at off == 1.
    c2, o2, v2, st = oracle.push(0, [5], [0.0], [-1e-12], np.zeros(17), 16, 1.0, 1)
    assert st[0] == 0 and c2[0] == 5 and o2[0] == 0.0
