"""Pins of the oracle's energy, adjoint Jacobi gradient and incremental
adjoint Jacobi Hessian-vector product (paper §3.2): exact adjointness of the
band sweep, pairing conservation, finite differences of the discrete energy
and of the sweeps, the zero-velocity closed forms, symmetry and the spectrum
of the assembled Gauss-Newton matrix."""

import numpy as np
import pytest

from oracle import Params
from oracle.band import inner, iota_vec, pi_vec, symbol_K, symbol_L
from oracle.epdiff import shoot
from oracle.jacobi import (backward_sweep, energy, forward, gradient, hessvec, incremental_backward,
                           incremental_shoot)
from oracle.lie import ad
from oracle.transport import grad_h
from paper_1807_11560_amd import synth


def problem(grid=(24, 24), band=(8, 8), nt=6, seed=1, dmax=1.5, s=2):
    p = Params(grid=grid, band=band, nt=nt, alpha=0.0025, s=s, sigma=0.03)
    rng = np.random.default_rng(seed)
    if len(grid) == 2:
        I0 = synth.gaussian_blobs(rng, grid, count=4) * 0.8
    else:
        I0 = synth.tissue_phantom(rng, grid)
    vstar = synth.scale_to_displacement(synth.random_band_field(rng, band, s=s), grid, dmax)
    I1 = forward(vstar, I0, p)[2][-1]
    return p, I0, I1, vstar


def energy_at(v, I0, I1, p):
    return energy(v, forward(v, I0, p)[2][-1], I1, p)[0]


def test_problem_is_not_degenerate():
    p, I0, I1, _ = problem()
    assert I0.std() > 0.1 and np.abs(I1 - I0).max() > 0.03


@pytest.mark.parametrize("dims", [2, 3])
def test_dot_product_of_the_band_sweep(dims):
    """<g_V - v0, dv0>_V = <U_nt, Y_nt>_V where Y_{n+1} = Y_n + dt (ad_{v_n}
    Y_n + dv_n), Y_0 = 0: the backward sweep is the exact transpose of the
    forward Jacobi recursion."""
    if dims == 2:
        p, I0, I1, vstar = problem()
    else:
        p, I0, I1, vstar = problem(grid=(12, 12, 12), band=(6, 6, 6), nt=4, dmax=1.0)
    Ls = symbol_L(p.band, p.alpha, p.s)
    v0 = 0.6 * vstar
    g, _, cache = gradient(v0, I0, I1, p)
    d = synth.random_direction(7, p.band)
    dvs = incremental_shoot(cache["vs"], d, p)
    Y = np.zeros_like(d)
    for n in range(p.nt):
        Y = Y + p.dt * (ad(cache["vs"][n], Y, p.spectral) + dvs[n])
    lhs = inner(Ls * (g - v0), d)
    rhs = inner(Ls * cache["Us"][p.nt], Y)
    assert abs(lhs - rhs) < 1e-11 * max(abs(lhs), 1e-3)


def test_pairing_conservation():
    """<U_n, Y_n>_V is constant along the sweep when Y_{n+1} = Y_n + dt ad_{v_n} Y_n."""
    p, I0, I1, vstar = problem()
    Ls = symbol_L(p.band, p.alpha, p.s)
    _, _, cache = gradient(0.6 * vstar, I0, I1, p)
    Y = synth.random_direction(8, p.band)
    vals = []
    for n in range(p.nt + 1):
        vals.append(inner(Ls * cache["Us"][n], Y))
        if n < p.nt:
            Y = Y + p.dt * ad(cache["vs"][n], Y, p.spectral)
    assert np.ptp(vals) < 1e-11 * max(abs(vals[0]), 1e-3)


@pytest.mark.parametrize("dims", [2, 3])
def test_gradient_at_zero_is_energy_derivative(dims):
    """At v0 = 0 the Jacobi gradient equals the central finite difference of
    the discrete energy (signs, 2/sigma^2, |N|^-1, K~ and the regulariser)."""
    if dims == 2:
        p, I0, I1, _ = problem()
    else:
        p, I0, I1, _ = problem(grid=(12, 12, 12), band=(6, 6, 6), nt=4, dmax=1.0)
    Ls = symbol_L(p.band, p.alpha, p.s)
    v0 = np.zeros((p.d,) + p.band, dtype=complex)
    g, E, _ = gradient(v0, I0, I1, p)
    assert E[1] == 0.0 and abs(E[0] - np.sum((I0 - I1) ** 2) / (p.sigma ** 2 * I0.size)) < 1e-12 * E[0]
    for seed in (9, 10):
        d = synth.random_direction(seed, p.band)
        h = 1e-7
        fd = (energy_at(h * d, I0, I1, p) - energy_at(-h * d, I0, I1, p)) / (2 * h)
        assert abs(inner(Ls * g, d) - fd) < 1e-4 * abs(fd)
    # closed form at zero velocity
    lam1 = -(2 / p.sigma ** 2) * (I0 - I1)
    np.testing.assert_allclose(g, symbol_K(p.band, p.alpha, p.s) * pi_vec(lam1 * grad_h(I0), p.band),
                               atol=1e-10 * np.abs(g).max())


def test_regulariser_gradient():
    """With I1 = m_1 (zero data term and residual) g_V = v0: the V-gradient of
    1/2 <L v0, v0>."""
    p, I0, _, vstar = problem()
    v0 = 0.5 * vstar
    m1 = forward(v0, I0, p)[2][-1]
    g, E, _ = gradient(v0, I0, m1, p)
    assert E[2] == 0.0
    np.testing.assert_allclose(g, v0, atol=1e-15)


def test_coupling_terms_are_the_derivative_of_the_sweep():
    """With a frozen terminal U*, the incremental backward sweep with dU_nt = 0
    (R1 coupling terms only) is the derivative of v0 -> w_0(v0; U*)."""
    p, I0, I1, vstar = problem(nt=4)
    v0 = 0.6 * vstar
    Ustar = synth.random_direction(11, p.band) * 50.0
    d = synth.random_direction(12, p.band)
    vs = shoot(v0, p)
    Us, ws = backward_sweep(vs, Ustar, p)
    dvs = incremental_shoot(vs, d, p)
    an = incremental_backward(vs, dvs, Us, ws, np.zeros_like(d), p, "R1")
    h = 1e-6
    wp = backward_sweep(shoot(v0 + h * d, p), Ustar, p)[1][0]
    wm = backward_sweep(shoot(v0 - h * d, p), Ustar, p)[1][0]
    fd = (wp - wm) / (2 * h)
    assert np.linalg.norm(an - fd) < 1e-6 * np.linalg.norm(fd)
    # and the dU_nt-driven part is the (linear) gradient sweep itself
    dU = synth.random_direction(13, p.band)
    r2 = incremental_backward(vs, dvs, Us, ws, dU, p, "R2")
    np.testing.assert_allclose(r2, backward_sweep(vs, dU, p)[1][0], atol=1e-13)


@pytest.mark.parametrize("mode", ["R1", "R2"])
def test_hessvec_at_zero_is_gradient_derivative(mode):
    """At v0 = 0 with I1 = I0 (zero residual) both Gauss-Newton modes equal
    the finite difference of the gradient, and the closed form
    dv + K~ pi((2/sigma^2)(grad I0 . iota dv) grad I0)."""
    p, I0, _, _ = problem()
    I1 = I0.copy()
    v0 = np.zeros((p.d,) + p.band, dtype=complex)
    _, _, cache = gradient(v0, I0, I1, p)
    d = synth.random_direction(14, p.band)
    Hd = hessvec(cache, d, p, mode)
    h = 1e-7
    fd = (gradient(h * d, I0, I1, p)[0] - gradient(-h * d, I0, I1, p)[0]) / (2 * h)
    assert np.linalg.norm(Hd - fd) < 1e-4 * np.linalg.norm(fd)
    gI = grad_h(I0)
    closed = d + symbol_K(p.band, p.alpha, p.s) * pi_vec(
        (2 / p.sigma ** 2) * np.sum(gI * iota_vec(d, p.grid), axis=0) * gI, p.band)
    np.testing.assert_allclose(Hd, closed, atol=1e-10 * np.abs(closed).max())


def hermitian_basis(band, d):
    """Real basis of Hermitian band vector fields: for each canonical
    frequency pair {k, -k} the real and imaginary unit fields."""
    from oracle.band import band_mask, reverse_index
    mask = band_mask(band)
    rev = [reverse_index(K) for K in band]
    seen = set()
    basis = []
    for c in range(d):
        for idx in map(tuple, np.argwhere(mask)):
            ridx = tuple(rev[j][idx[j]] for j in range(len(band)))
            if (c, ridx) in seen:
                continue
            seen.add((c, idx))
            e = np.zeros((d,) + band, dtype=complex)
            if ridx == idx:
                e[(c,) + idx] = 1.0
                basis.append(e)
            else:
                e[(c,) + idx] = 1.0
                e[(c,) + ridx] = 1.0
                basis.append(e)
                f = np.zeros_like(e)
                f[(c,) + idx] = 1j
                f[(c,) + ridx] = -1j
                basis.append(f)
    return basis


def test_assembled_gauss_newton_matrix_at_zero():
    """At v0 = 0 the R2 matrix is symmetric in V with every eigenvalue >= 1
    (identity plus a Gram matrix)."""
    p, I0, I1, _ = problem(grid=(16, 16), band=(6, 6), nt=3)
    Ls = symbol_L(p.band, p.alpha, p.s)
    v0 = np.zeros((p.d,) + p.band, dtype=complex)
    _, _, cache = gradient(v0, I0, I1, p)
    basis = hermitian_basis(p.band, p.d)
    assert len(basis) == p.d * 25
    H = [hessvec(cache, e, p, "R2") for e in basis]
    G = np.array([[inner(Ls * a, hb) for hb in H] for a in basis])
    D = np.array([inner(Ls * a, a) for a in basis])
    Gn = G / np.sqrt(np.outer(D, D))
    assert np.abs(Gn - Gn.T).max() < 1e-9 * np.abs(Gn).max()
    ev = np.linalg.eigvalsh(0.5 * (Gn + Gn.T))
    assert ev.min() > 1.0 - 1e-9


def test_method_gap_to_energy_derivative_is_reported():
    """The Jacobi gradient is not the exact derivative of the discrete energy
    away from v0 = 0 (band truncation of the Jacobi field); the gap shrinks as
    the grid and band are refined.  Measured, with a loose sanity bound."""
    gaps = []
    for grid, band in (((32, 32), (8, 8)), ((64, 64), (16, 16))):
        p, I0, I1, vstar = problem(grid=grid, band=band, nt=6, dmax=grid[0] / 16.0)
        Ls = symbol_L(p.band, p.alpha, p.s)
        v0 = 0.5 * vstar
        g, _, _ = gradient(v0, I0, I1, p)
        d = synth.random_direction(15, p.band)
        h = 1e-6
        fd = (energy_at(v0 + h * d, I0, I1, p) - energy_at(v0 - h * d, I0, I1, p)) / (2 * h)
        gaps.append(abs(inner(Ls * g, d) - fd) / abs(fd))
    print("Jacobi-gradient gap to the energy derivative:", gaps)
    assert gaps[1] < 0.5


def test_full_newton_at_zero_is_gradient_derivative():
    """At v0 = 0 with a nonzero residual the full Newton product ("FULL")
    is the derivative of the gradient: the central difference of the
    gradient approaches it linearly in the step (the trilinear interpolant
    has kinks at the nodes, so the difference is first order).  The
    Gauss-Newton product and the paper's printed sign of lambda_1 grad dm_1
    stay far from it."""
    p, I0, I1, _ = problem()
    v0 = np.zeros((p.d,) + p.band, dtype=complex)
    _, _, cache = gradient(v0, I0, I1, p)
    d = synth.random_direction(15, p.band)
    full = hessvec(cache, d, p, "FULL")
    r1 = hessvec(cache, d, p, "R1")
    printed_sign = 2 * r1 - full  # dU(1) with -lambda_1 grad dm_1
    errs = []
    for h in (1e-3, 1e-4):
        fd = (gradient(h * d, I0, I1, p)[0] - gradient(-h * d, I0, I1, p)[0]) / (2 * h)
        errs.append(np.linalg.norm(full - fd) / np.linalg.norm(fd))
        assert np.linalg.norm(r1 - fd) > 0.05 * np.linalg.norm(fd)
        assert np.linalg.norm(printed_sign - fd) > 0.15 * np.linalg.norm(fd)
    assert errs[1] < 5e-3 and errs[0] / errs[1] > 5.0


def test_full_newton_equals_gauss_newton_at_zero_residual():
    """With I1 = m_1(v0) (lambda_1 = 0) the full Newton product is the
    Gauss-Newton product of the paper reading."""
    p, I0, _, vstar = problem()
    v0 = 0.5 * vstar
    I1 = forward(v0, I0, p)[2][-1]
    _, _, cache = gradient(v0, I0, I1, p)
    d = synth.random_direction(16, p.band)
    np.testing.assert_array_equal(hessvec(cache, d, p, "FULL"), hessvec(cache, d, p, "R1"))
