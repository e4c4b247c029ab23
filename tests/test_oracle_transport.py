"""Pins of the oracle's semi-Lagrangian state transport (paper §2.3 state
equation): identity at zero velocity, exact integer shifts, the discrete
maximum principle, convergence to the analytic solution, central differences
in closed form, and the incremental state at zero velocity."""

import numpy as np
import pytest

from oracle.transport import grad_h, incremental_transport, interpolate, sl_step, transport
from paper_1807_11560_amd import synth


def smooth_image(grid):
    X = np.meshgrid(*[np.arange(n) / n for n in grid], indexing="ij")
    f = np.ones(grid)
    for j, x in enumerate(X):
        f = f * (1.2 + np.sin(2 * np.pi * x + 0.3 * j))
    return f


@pytest.mark.parametrize("grid", [(16, 12), (8, 10, 6)])
def test_zero_velocity_is_identity(grid):
    rng = np.random.default_rng(0)
    I0 = rng.standard_normal(grid)
    v = np.zeros((len(grid),) + grid)
    ms = transport(I0, [v] * 5, 0.2)
    for m in ms:
        np.testing.assert_array_equal(m, I0)


def test_integer_shift_is_exact():
    """Constant velocity c with dt c_j N_j integer: a circular shift by c."""
    grid = (16, 12, 10)
    rng = np.random.default_rng(1)
    I0 = rng.standard_normal(grid)
    nt = 4
    shift = (1, -2, 3)  # voxels per step
    v = np.stack([np.full(grid, shift[j] * nt / grid[j]) for j in range(3)])
    m = transport(I0, [v] * nt, 1.0 / nt)[-1]
    expect = np.roll(I0, tuple(s * nt for s in shift), axis=(0, 1, 2))
    np.testing.assert_allclose(m, expect, atol=1e-12)


def test_maximum_principle():
    grid = (24, 24)
    rng = np.random.default_rng(2)
    I0 = synth.gaussian_blobs(rng, grid, count=5)
    vs = [0.05 * rng.standard_normal((2,) + grid) for _ in range(6)]
    for m in transport(I0, vs, 1.0 / 6):
        assert m.min() >= I0.min() - 1e-14 and m.max() <= I0.max() + 1e-14


def test_converges_to_analytic_translation():
    """Constant sub-voxel velocity: m_1 -> I0(x - c); error falls with h."""
    errs = []
    c = np.array([0.123, -0.071])
    for n in (32, 64, 128):
        grid = (n, n)
        I0 = smooth_image(grid)
        X = np.meshgrid(*[np.arange(k) / k for k in grid], indexing="ij")
        exact = np.ones(grid)
        for j in range(2):
            exact = exact * (1.2 + np.sin(2 * np.pi * (X[j] - c[j]) + 0.3 * j))
        v = np.stack([np.full(grid, c[j]) for j in range(2)])
        m = transport(I0, [v] * 4, 0.25)[-1]
        errs.append(np.abs(m - exact).max())
    assert errs[0] > errs[1] > errs[2]
    assert errs[0] / errs[2] > 4.0


def test_interpolation_at_nodes_and_midpoints():
    rng = np.random.default_rng(3)
    f = rng.standard_normal((6, 5, 4))
    nodes = np.stack(np.meshgrid(*[np.arange(n, dtype=float) for n in f.shape], indexing="ij"))
    np.testing.assert_allclose(interpolate(f, nodes), f, atol=1e-15)
    mid = nodes.copy()
    mid[1] += 0.5
    np.testing.assert_allclose(interpolate(f, mid), 0.5 * (f + np.roll(f, -1, axis=1)), atol=1e-14)
    wrap = nodes.copy()
    wrap[2] -= 4.0  # one period
    np.testing.assert_allclose(interpolate(f, wrap), f, atol=1e-14)


def test_central_difference_closed_form():
    """grad_h sin(2 pi k i/N) = N sin(2 pi k/N) cos(2 pi k i/N) along that axis."""
    N, k = 20, 3
    i = np.arange(N)
    f = np.tile(np.sin(2 * np.pi * k * i / N)[:, None], (1, 7))
    g = grad_h(f)
    np.testing.assert_allclose(g[0][:, 0], N * np.sin(2 * np.pi * k / N) * np.cos(2 * np.pi * k * i / N),
                               atol=1e-12)
    assert np.abs(g[1]).max() < 1e-12


def test_incremental_state_is_central_derivative_at_zero_velocity():
    """At v = 0 the incremental state equals the central finite difference of
    the discrete transport in the direction dv (one-sided interpolation slopes
    average to the central difference)."""
    grid = (16, 14)
    rng = np.random.default_rng(4)
    I0 = synth.gaussian_blobs(rng, grid, count=3)
    nt = 5
    dvs = [0.3 * rng.standard_normal((2,) + grid) for _ in range(nt)]
    zero = [np.zeros((2,) + grid)] * nt
    ms = transport(I0, zero, 1.0 / nt)
    dm = incremental_transport(ms, zero, dvs, 1.0 / nt)
    h = 1e-8  # the O(h) remainder carries slope jumps of the random dv
    mp = transport(I0, [h * d for d in dvs], 1.0 / nt)[-1]
    mm = transport(I0, [-h * d for d in dvs], 1.0 / nt)[-1]
    np.testing.assert_allclose(dm, (mp - mm) / (2 * h), atol=1e-6)


def test_sl_step_moves_with_velocity():
    grid = (32,)
    f = np.zeros(grid)
    f[10] = 1.0
    v = np.full((1,) + grid, 2.0 / 32)  # two voxels in unit time
    out = sl_step(f, v, 1.0)
    assert out[12] == 1.0 and out.sum() == 1.0
