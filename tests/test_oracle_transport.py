"""Pins of the oracle's semi-Lagrangian state transport (paper §2.3 state
equation): identity at zero velocity, exact integer shifts, the discrete
maximum principle, convergence to the analytic solution, central differences
in closed form, the incremental state at zero velocity, in closed form for
time-varying integer shifts, and its first-order convergence to the
derivative of the discrete transport at a nonzero velocity (paper §2.5
incremental state equation)."""

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


def _shift_velocity(shift, grid, dt):
    """Constant velocity that moves the image by ``shift`` voxels in one step."""
    return np.stack([np.full(grid, shift[j] / (dt * grid[j])) for j in range(len(grid))])


@pytest.mark.parametrize("grid", [(12, 10), (10, 8, 6)])
def test_incremental_state_closed_form_for_time_varying_shifts(grid):
    """Per-step constant velocities with integer-voxel steps s_n (a different
    shift at every step) make each SL step an exact circular shift, so
    m_n = I0(x - S_n) with S_n = s_0 + ... + s_{n-1}, and the incremental state
    (source at the nodes, then carried by the step) has the closed form
        dm_nt(x) = -dt sum_n grad_h I0(x - S_nt) . dv_n(x - S_nt + S_n).
    Written with array shifts only, no interpolation.  A slip between step n
    and n+1 in the state, the velocity or the direction changes the sum."""
    d = len(grid)
    nt = 4
    dt = 1.0 / nt
    rng = np.random.default_rng(11)
    shifts = [tuple(int(x) for x in rng.integers(-2, 3, size=d)) for _ in range(nt)]
    shifts[1] = tuple(3 if j == 0 else -1 for j in range(d))  # steps differ
    I0 = rng.standard_normal(grid)
    vgrid = [_shift_velocity(s, grid, dt) for s in shifts]
    dvs = [rng.standard_normal((d,) + grid) for _ in range(nt)]
    ms = transport(I0, vgrid, dt)
    dm = incremental_transport(ms, vgrid, dvs, dt)

    axes = tuple(range(d))
    S = [np.zeros(d, dtype=int)]
    for s in shifts:
        S.append(S[-1] + np.array(s))
    for n in range(nt + 1):  # the states themselves are the shifts
        np.testing.assert_allclose(ms[n], np.roll(I0, tuple(S[n]), axis=axes), atol=1e-12)
    gI0 = np.stack([(np.roll(I0, -1, axis=j) - np.roll(I0, 1, axis=j)) * (grid[j] / 2.0) for j in range(d)])
    g_end = np.stack([np.roll(gI0[j], tuple(S[nt]), axis=axes) for j in range(d)])
    expect = np.zeros(grid)
    for n in range(nt):
        dv_moved = np.stack([np.roll(dvs[n][j], tuple(S[nt] - S[n]), axis=axes) for j in range(d)])
        expect -= dt * np.sum(g_end * dv_moved, axis=0)
    np.testing.assert_allclose(dm, expect, atol=1e-11)


def _smooth_fields(grid, rng):
    """Smooth periodic image, velocity and direction (low sine modes)."""
    X = np.meshgrid(*[np.arange(n) / n for n in grid], indexing="ij")
    I0 = 0.5 + 0.3 * np.sin(2 * np.pi * X[0]) * np.cos(2 * np.pi * X[1] + 0.4)
    v = np.stack([0.08 * np.sin(2 * np.pi * (X[1] + 0.2)), 0.06 * np.cos(2 * np.pi * (X[0] - 0.1))])
    dv = np.stack([np.cos(2 * np.pi * (X[0] + X[1])), 0.7 * np.sin(2 * np.pi * (X[0] - 0.3))])
    return I0, v, dv


def test_incremental_state_converges_to_derivative_of_transport():
    """At a nonzero velocity the incremental state (node source, then
    transported; the paper's linearised state equation) differs from the
    exact derivative of the discrete transport by O(h) + O(dt).  Refining grid
    and time step together (dt proportional to h) shrinks the gap at first
    order."""
    gaps = []
    for n in (32, 64, 128):
        grid = (n, n)
        nt = n // 8
        dt = 1.0 / nt
        I0, v, dv = _smooth_fields(grid, None)
        vgrid = [v * (1.0 + 0.2 * k / nt) for k in range(nt)]  # time-varying
        dvs = [dv * (1.0 - 0.3 * k / nt) for k in range(nt)]
        ms = transport(I0, vgrid, dt)
        dm = incremental_transport(ms, vgrid, dvs, dt)
        h = 1e-7
        mp = transport(I0, [a + h * b for a, b in zip(vgrid, dvs)], dt)[-1]
        mm = transport(I0, [a - h * b for a, b in zip(vgrid, dvs)], dt)[-1]
        fd = (mp - mm) / (2 * h)
        gaps.append(np.linalg.norm(dm - fd) / np.linalg.norm(fd))
    assert gaps[0] > gaps[1] > gaps[2]
    for a, b in zip(gaps, gaps[1:]):
        assert 1.6 < a / b < 2.6, gaps  # first order
    assert gaps[-1] < 0.05
