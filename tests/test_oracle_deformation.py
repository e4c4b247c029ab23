"""Pins of the oracle's deformation-state variant (paper §3.3): the band
deformation state equation against characteristics traced independently,
the interpolant's derivatives against finite differences, exact
compositions, first-order consistency of the gradient with the discrete
energy, and the Hessian-vector products against central differences of the
gradient (classical Gauss-Newton at zero residual, full Newton anywhere)."""

import numpy as np
import pytest

from oracle import Params
from oracle import deformation as D
from oracle.band import freqs, inner, iota_vec, symbol_L
from oracle.transport import interpolate
from paper_1807_11560_amd import synth


def problem(grid=(24, 24), band=(8, 8), nt=6, seed=1, dmax=1.5, s=2):
    p = Params(grid=grid, band=band, nt=nt, alpha=0.0025, s=s, sigma=0.03)
    rng = np.random.default_rng(seed)
    if len(grid) == 2:
        I0 = synth.gaussian_blobs(rng, grid, count=4) * 0.8
    else:
        I0 = synth.tissue_phantom(rng, grid)
    vstar = synth.scale_to_displacement(synth.random_band_field(rng, band, s=s), grid, dmax)
    I1 = D.forward(vstar, I0, p)[2]
    return p, I0, I1, vstar


def energy_at(v, I0, I1, p):
    return D.energy(v, D.forward(v, I0, p)[2], I1, p)[0]


EXACT = "interpolant"  # image derivatives of the discrete m(1): exact pins


def band_eval(v, X):
    """v(X) at arbitrary points of the unit square by the direct Fourier sum
    (no grid, no interpolation).  X: (2, P)."""
    K0, K1 = v.shape[1:]
    k0 = freqs(K0).reshape(K0, 1, 1)
    k1 = freqs(K1).reshape(1, K1, 1)
    ph = np.exp(2j * np.pi * (k0 * X[0].reshape(1, 1, -1) + k1 * X[1].reshape(1, 1, -1)))
    return np.stack([np.real(np.sum(v[c][..., None] * ph, axis=(0, 1))) for c in range(v.shape[0])])


def characteristic_displacement(v, grid, steps=400):
    """phi(1)(x) - x for the steady field v: phi(1) is the flow of -v for unit
    time (d_t phi + D phi v = 0, phi(0) = id), traced with classical RK4."""
    nodes = np.meshgrid(*[np.arange(n) / n for n in grid], indexing="ij")
    X = np.stack([c.ravel() for c in nodes]).astype(np.float64)
    X0 = X.copy()
    h = 1.0 / steps
    f = lambda Y: -band_eval(v, Y)
    for _ in range(steps):
        k1 = f(X)
        k2 = f(X + 0.5 * h * k1)
        k3 = f(X + 0.5 * h * k2)
        k4 = f(X + h * k3)
        X = X + h / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
    return (X - X0).reshape((2,) + tuple(grid))


def test_transport_converges_to_characteristics():
    """With a steady velocity the band deformation state equation reproduces
    the flow of -v (traced pointwise by RK4 on the Fourier sum) to first
    order in dt."""
    grid, band = (16, 16), (16, 16)
    rng = np.random.default_rng(5)
    v = synth.random_band_field(rng, band, s=3)
    # keep |k| <= 1: the displacement's spectrum then decays fast enough
    # that the band truncation stays far below the time-stepping error
    k = [np.abs(freqs(K)) for K in band]
    v = v * ((k[0][:, None] <= 1) & (k[1][None, :] <= 1))
    v = synth.scale_to_displacement(v, grid, 1.0)
    ref = characteristic_displacement(v, grid)
    errs = []
    for nt in (16, 32, 64):
        p = Params(grid=grid, band=band, nt=nt)
        u = D.deformation_transport([v] * nt, p)[-1]
        errs.append(np.abs(iota_vec(u, grid) - ref).max())
    scale = np.abs(ref).max()
    assert scale > 0.05
    assert errs[2] < 0.01 * scale
    for a, b in zip(errs, errs[1:]):
        assert 0.4 < b / a < 0.6  # first order


def test_interpolant_derivatives_match_finite_differences():
    rng = np.random.default_rng(3)
    f = rng.standard_normal((7, 9, 8))
    X = np.stack([rng.uniform(-3.0, 12.0, 50) for _ in range(3)])
    frac = X - np.floor(X)
    keep = np.all((frac > 1e-3) & (frac < 1 - 1e-3), axis=0)
    X = X[:, keep]
    val, grad, hess = D.interpolate_derivatives(f, X)
    assert np.allclose(val, interpolate(f, X), atol=1e-13)
    h = 1e-6
    for a in range(3):
        e = np.zeros((3, 1))
        e[a] = h
        fd = (interpolate(f, X + e) - interpolate(f, X - e)) / (2 * h) * f.shape[a]
        assert np.allclose(grad[a], fd, atol=1e-7)
        for b in range(3):
            if a == b:
                assert np.all(hess[a, b] == 0.0)
                continue
            gp = D.interpolate_derivatives(f, X + e)[1][b]
            gm = D.interpolate_derivatives(f, X - e)[1][b]
            assert np.allclose(hess[a, b], (gp - gm) / (2 * h) * f.shape[a], atol=1e-5)


def test_composition_identity_and_integer_shift():
    rng = np.random.default_rng(4)
    I0 = rng.standard_normal((6, 10, 8))
    for sampling in ("central", EXACT):
        m, _, _ = D.compose(I0, np.zeros((3,) + I0.shape), sampling)
        assert np.array_equal(m, I0)
        s = (2, -3, 5)
        u = np.stack([np.full(I0.shape, s[j] / I0.shape[j]) for j in range(3)])
        m, _, _ = D.compose(I0, u, sampling)
        assert np.allclose(m, np.roll(I0, [-x for x in s], axis=(0, 1, 2)), atol=1e-12)


def test_central_sampling_at_nodes_is_the_central_difference():
    """At phi = id the central sampling returns grad_h I0 (closed form
    (I[i+1] - I[i-1]) N / 2) and the central second differences."""
    rng = np.random.default_rng(6)
    I0 = rng.standard_normal((6, 10, 8))
    _, g, h = D.compose(I0, np.zeros((3,) + I0.shape), "central")
    for a in range(3):
        n = I0.shape[a]
        ref = (np.roll(I0, -1, axis=a) - np.roll(I0, 1, axis=a)) * n / 2
        assert np.allclose(g[a], ref, atol=1e-12)
        wide = (np.roll(I0, -2, axis=a) - 2 * I0 + np.roll(I0, 2, axis=a)) * n * n / 4
        assert np.allclose(h[a, a], wide, atol=1e-10)
    assert np.allclose(h[0, 1], h[1, 0], atol=1e-10)


def test_samplings_agree_on_smooth_images():
    """The two samplings differ at first order in h (inside a cell the
    interpolant's gradient is a one-sided difference): a smooth periodic image
    on grids of 16 and 32 points."""
    errs = []
    for n in (16, 32):
        x = np.arange(n) / n
        X0, X1 = np.meshgrid(x, x, indexing="ij")
        I0 = np.sin(2 * np.pi * X0) * np.cos(4 * np.pi * X1)
        u = np.stack([0.3 / n + 0.1 * np.sin(2 * np.pi * X1), 0.2 / n + 0.05 * np.cos(2 * np.pi * X0)])
        _, gc, _ = D.compose(I0, u, "central")
        _, gi, _ = D.compose(I0, u, EXACT)
        errs.append(np.abs(gc - gi).max() / np.abs(gi).max())
    assert errs[0] < 0.4 and 0.4 < errs[1] / errs[0] < 0.6


def test_zero_velocity_keeps_the_source():
    p, I0, I1, _ = problem()
    vs, us, m1, _, _ = D.forward(np.zeros((2,) + p.band, dtype=complex), I0, p)
    assert all(np.abs(u).max() == 0.0 for u in us)
    assert np.array_equal(m1, I0)


def test_problem_is_not_degenerate():
    p, I0, I1, vstar = problem()
    assert np.abs(I1 - I0).max() > 0.05
    us = D.forward(vstar, I0, p)[1]
    assert np.abs(iota_vec(us[-1], p.grid)).max() * p.grid[0] > 0.5  # voxels


def test_gradient_is_consistent_with_the_energy():
    """The adjoint Jacobi gradient is the derivative of the continuous
    problem; against the discrete energy its error falls at first order."""
    errs = []
    for nt in (4, 8, 16):
        p, I0, I1, vstar = problem(nt=nt)
        Ls = symbol_L(p.band, p.alpha, p.s)
        v0 = 0.5 * vstar
        g = D.gradient(v0, I0, I1, p, EXACT)[0]
        d = synth.random_direction(7, p.band)
        h = 1e-6
        fd = (energy_at(v0 + h * d, I0, I1, p) - energy_at(v0 - h * d, I0, I1, p)) / (2 * h)
        errs.append(abs(inner(Ls * g, d) - fd) / abs(fd))
    assert errs[0] < 0.03
    assert errs[1] < 0.65 * errs[0] and errs[2] < 0.65 * errs[1]


def _fd_gradient(v0, d, I0, I1, p, h=1e-6, sampling=EXACT):
    gp = D.gradient(v0 + h * d, I0, I1, p, sampling)[0]
    gm = D.gradient(v0 - h * d, I0, I1, p, sampling)[0]
    return (gp - gm) / (2 * h)


@pytest.mark.parametrize("dims", [2, 3])
def test_gauss_newton_at_zero_residual_is_gradient_derivative(dims):
    """I1 = m(1)(v0): every mode equals the central difference of the gradient
    (the plus sign of D~phi * drho~, the incremental deformation state and
    both sweeps)."""
    if dims == 2:
        p, I0, _, vstar = problem()
    else:
        p, I0, _, vstar = problem(grid=(12, 12, 12), band=(6, 6, 6), nt=3, dmax=1.0)
    v0 = 0.5 * vstar
    I1 = D.forward(v0, I0, p)[2]
    _, _, cache = D.gradient(v0, I0, I1, p, EXACT)
    d = synth.random_direction(7, p.band)
    fd = _fd_gradient(v0, d, I0, I1, p)
    scale = np.abs(fd).max()
    for mode in ("R2", "R1", "FULL"):
        assert np.abs(D.hessvec(cache, d, p, mode) - fd).max() < 1e-7 * scale
    # a sign flip of D~phi * drho~ is caught
    assert np.abs(2 * d - D.hessvec(cache, d, p, "R2") - fd).max() > 0.5 * scale


def test_full_newton_is_gradient_derivative():
    """With a residual, the full Newton product equals the central difference
    of the gradient; the Gauss-Newton modes drop terms of visible size."""
    p, I0, I1, vstar = problem()
    v0 = 0.5 * vstar
    _, _, cache = D.gradient(v0, I0, I1, p, EXACT)
    d = synth.random_direction(7, p.band)
    fd = _fd_gradient(v0, d, I0, I1, p)
    scale = np.abs(fd).max()
    assert np.abs(D.hessvec(cache, d, p, "FULL") - fd).max() < 1e-7 * scale
    assert np.abs(D.hessvec(cache, d, p, "R1") - fd).max() > 1e-3 * scale
    assert np.abs(D.hessvec(cache, d, p, "R2") - fd).max() > 1e-2 * scale


def test_central_sampling_products_are_close_to_the_derivative():
    """With the product path's sampling the products are no longer exact
    derivatives of its gradient (the sampled Hessian is not the derivative of
    the sampled gradient) but stay within the sampling difference of them on
    this coarse problem; the sharp pins above use the exact sampling."""
    p, I0, I1, vstar = problem()
    v0 = 0.5 * vstar
    d = synth.random_direction(7, p.band)
    _, _, cache = D.gradient(v0, I0, I1, p)
    fd = _fd_gradient(v0, d, I0, I1, p, sampling="central")
    e = np.abs(D.hessvec(cache, d, p, "FULL") - fd).max() / np.abs(fd).max()
    assert e < 0.15
    Iz = D.forward(v0, I0, p)[2]
    _, _, cz = D.gradient(v0, I0, Iz, p)
    fdz = _fd_gradient(v0, d, I0, Iz, p, sampling="central")
    ez = np.abs(D.hessvec(cz, d, p, "R2") - fdz).max() / np.abs(fdz).max()
    assert ez < 0.15


def test_gauss_newton_modes_differ_by_the_coupling_terms_only():
    """R1 - R2 is the coupling part of the incremental sweep: with U = w = 0
    substituted into the cache the two modes agree."""
    p, I0, I1, vstar = problem()
    d = synth.random_direction(9, p.band)
    _, _, cache = D.gradient(0.5 * vstar, I0, I1, p)
    zeroed = dict(cache, Us=[np.zeros_like(u) for u in cache["Us"]], ws=[np.zeros_like(u) for u in cache["ws"]])
    assert np.allclose(D.hessvec(zeroed, d, p, "R1"), D.hessvec(zeroed, d, p, "R2"), atol=1e-12, rtol=0)


def test_modes_agree_only_at_zero_residual():
    p, I0, I1, vstar = problem()
    d = synth.random_direction(9, p.band)
    _, _, cache = D.gradient(0.5 * vstar, I0, I1, p)
    r1 = D.hessvec(cache, d, p, "R1")
    r2 = D.hessvec(cache, d, p, "R2")
    assert np.abs(r1 - r2).max() > 1e-3 * np.abs(r1).max()
    with pytest.raises(ValueError):
        D.hessvec(cache, d, p, "R3")
