"""Pins of the oracle's higher-order time integration: RK4 shooting against
SciPy's adaptive integrator and at fourth order in dt, conservation of the
geodesic energy <L v, v> (paper §2.2) to fourth order against the Euler
steps' first, and midpoint departure points at second order against
characteristics traced pointwise on the Fourier sum."""

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import Params
from oracle.band import freqs, iota_vec, symbol_L
from oracle.epdiff import energies, shoot, shoot_rk4
from oracle.highorder import forward_rk
from oracle.lie import ad_dagger
from oracle.transport import departure_points, departure_points_rk2, transport_rk2
from paper_1807_11560_amd import synth


def velocity(seed, band, amp):
    v = synth.random_band_field(np.random.default_rng(seed), band, 0.0025, 2)
    return v * (amp / np.abs(v).max())


def test_rk4_matches_an_independent_integrator():
    """The band EPDiff integrated by SciPy's DOP853 at tolerance 1e-12 on the
    flattened real system: RK4 converges to it at fourth order."""
    grid, band = (16, 16), (8, 8)
    p = Params(grid=grid, band=band, nt=40)
    Ls = symbol_L(band, p.alpha, p.s)
    v0 = velocity(3, band, 0.05)
    shape = v0.shape

    def rhs(t, y):
        v = (y[: y.size // 2] + 1j * y[y.size // 2:]).reshape(shape)
        f = -ad_dagger(v, v, Ls, p.spectral)
        return np.concatenate([f.real.ravel(), f.imag.ravel()])

    y0 = np.concatenate([v0.real.ravel(), v0.imag.ravel()])
    sol = solve_ivp(rhs, (0.0, 1.0), y0, method="DOP853", rtol=1e-12, atol=1e-14)
    ref = (sol.y[: y0.size // 2, -1] + 1j * sol.y[y0.size // 2:, -1]).reshape(shape)
    scale = np.abs(ref).max()
    v1 = shoot_rk4(v0, p)[-1]
    e40 = np.abs(v1 - ref).max() / scale
    e20 = np.abs(shoot_rk4(v0, Params(grid=grid, band=band, nt=20))[-1] - ref).max() / scale
    assert e40 < 3e-6 and 12.0 < e20 / e40 < 20.0
    # the Euler steps are much further away
    assert np.abs(shoot(v0, p)[-1] - ref).max() / scale > 1e4 * e40


def test_rk4_is_fourth_order():
    grid, band = (16, 16), (8, 8)
    v0 = velocity(4, band, 0.05)
    ref = shoot_rk4(v0, Params(grid=grid, band=band, nt=160))[-1]
    errs = [np.abs(shoot_rk4(v0, Params(grid=grid, band=band, nt=nt))[-1] - ref).max() for nt in (10, 20)]
    assert 12.0 < errs[0] / errs[1] < 20.0


def test_rk4_conserves_the_geodesic_energy_to_fourth_order():
    grid, band = (16, 16), (8, 8)
    v0 = velocity(11, band, 0.05)
    drift, drift_euler = [], []
    for nt in (10, 20, 40):
        p = Params(grid=grid, band=band, nt=nt)
        e = energies(shoot_rk4(v0, p), p)
        drift.append(abs(e[-1] - e[0]))
        e = energies(shoot(v0, p), p)
        drift_euler.append(abs(e[-1] - e[0]))
    assert drift[0] / drift[1] > 14.0 and drift[1] / drift[2] > 14.0
    assert drift[0] < 1e-3 * drift_euler[0]


def test_rk4_zero_and_constant_velocity():
    p = Params(grid=(16, 16, 16), band=(8, 8, 8), nt=4)
    v0 = np.zeros((3,) + p.band, dtype=complex)
    assert all(np.abs(v).max() == 0 for v in shoot_rk4(v0, p))
    v0[:, 0, 0, 0] = (0.1, -0.2, 0.05)
    for v in shoot_rk4(v0, p):
        np.testing.assert_allclose(v, v0, atol=1e-15)


def band_eval(v, X):
    """v(X) at arbitrary points by the direct Fourier sum over its nonzero modes."""
    K0, K1 = v.shape[1:]
    idx = np.argwhere(np.any(v != 0, axis=0))
    k = np.stack([freqs(K0)[idx[:, 0]], freqs(K1)[idx[:, 1]]]).astype(np.float64)  # (2, modes)
    ph = np.exp(2j * np.pi * (k.T @ X))  # (modes, points)
    c = v[:, idx[:, 0], idx[:, 1]]       # (comps, modes)
    return np.real(c @ ph)


def test_midpoint_departure_points_are_second_order():
    """One step of size dt with a steady field: the departure point error
    against the backward characteristic (RK4, 50 sub-steps, on the Fourier
    sum) falls as dt^3 for the midpoint rule and as dt^2 for the Euler
    departure point."""
    grid, band = (128, 128), (8, 8)
    v = synth.random_band_field(np.random.default_rng(7), band, 0.0025, 2)
    k = [np.abs(freqs(K)) for K in band]
    v = v * ((k[0][:, None] <= 1) & (k[1][None, :] <= 1))
    v = v * (0.3 / np.abs(v).max())
    vg = iota_vec(v, grid)
    nodes = np.meshgrid(*[np.arange(n) / n for n in grid], indexing="ij")
    X0 = np.stack([c.ravel() for c in nodes])
    e_rk2, e_eul = [], []
    for dt in (0.2, 0.1, 0.05):
        X = X0.copy()
        h = dt / 50
        f = lambda Y: -band_eval(v, Y)
        for _ in range(50):
            k1 = f(X)
            k2 = f(X + 0.5 * h * k1)
            k3 = f(X + 0.5 * h * k2)
            k4 = f(X + h * k3)
            X = X + h / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
        ref = (X * np.array(grid)[:, None]).reshape((2,) + grid)  # voxels
        e_rk2.append(np.abs(departure_points_rk2(vg, dt) - ref).max())
        e_eul.append(np.abs(departure_points(vg, dt) - ref).max())
    assert 6.5 < e_rk2[0] / e_rk2[1] < 9.5 and 6.5 < e_rk2[1] / e_rk2[2] < 9.5
    assert 3.3 < e_eul[0] / e_eul[1] < 4.7 and 3.3 < e_eul[1] / e_eul[2] < 4.7


@pytest.mark.parametrize("grid", [(16, 12), (8, 10, 6)])
def test_rk2_transport_zero_velocity_and_integer_shift(grid):
    rng = np.random.default_rng(2)
    I0 = rng.standard_normal(grid)
    d = len(grid)
    ms = transport_rk2(I0, [np.zeros((d,) + grid)] * 3, 0.25)
    for m in ms:
        np.testing.assert_array_equal(m, I0)
    # constant velocity of one voxel per step along the last axis
    dt = 0.25
    vm = np.zeros((d,) + grid)
    vm[-1] = 1.0 / (dt * grid[-1])
    m1 = transport_rk2(I0, [vm], dt)[-1]
    np.testing.assert_allclose(m1, np.roll(I0, 1, axis=d - 1), atol=1e-12)


def test_forward_rk_zero_velocity_is_identity():
    p = Params(grid=(12, 12, 12), band=(6, 6, 6), nt=3)
    I0 = np.random.default_rng(1).standard_normal(p.grid)
    vs, ms = forward_rk(np.zeros((3,) + p.band, dtype=complex), I0, p)
    assert all(np.array_equal(m, I0) for m in ms)
