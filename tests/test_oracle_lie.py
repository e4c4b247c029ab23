"""Pins of the oracle's band Lie operators (paper §3.1 ad~, and the bracket
of the band-limited EPDiff equation) and of shooting: closed forms, the
Jacobi identity, exact adjointness, the 1-D Camassa-Holm reduction, the
discrete Euler energy identity, momentum transport direction, symmetry."""

import numpy as np
import pytest
import sympy

from oracle import Params
from oracle.band import hermitian_part, inner, iota, pi, symbol_L
from oracle.epdiff import shoot
from oracle.lie import ad, ad_dagger, ad_star


def rand_field(seed, band, kmax=None):
    rng = np.random.default_rng(seed)
    d = len(band)
    f = rng.standard_normal((d,) + band) + 1j * rng.standard_normal((d,) + band)
    if kmax is not None:
        from oracle.band import freqs
        for j, K in enumerate(band):
            shape = [1] * (d + 1)
            shape[j + 1] = K
            f = f * (np.abs(freqs(K)) <= kmax).reshape(shape)
    return hermitian_part(f, band)


def grid_coords(grid):
    return np.meshgrid(*[np.arange(n) / n for n in grid], indexing="ij")


@pytest.mark.parametrize("band", [(8, 8), (6, 8, 6)])
def test_ad_star_is_l2_adjoint_of_ad(band):
    M = tuple(3 * K // 2 for K in band)
    a, b, mu = rand_field(1, band), rand_field(2, band), rand_field(3, band)
    lhs = inner(ad(a, b, M), mu)
    rhs = inner(b, ad_star(a, mu, M))
    assert abs(lhs - rhs) < 1e-11 * max(1.0, abs(lhs))


@pytest.mark.parametrize("band", [(8, 8), (6, 8, 6)])
def test_ad_antisymmetric(band):
    M = tuple(3 * K // 2 for K in band)
    a, b = rand_field(4, band), rand_field(5, band)
    np.testing.assert_allclose(ad(a, b, M), -ad(b, a, M), atol=1e-11)
    assert np.abs(ad(a, a, M)).max() < 1e-11


def test_ad_closed_form_2d():
    """a = (sin 2 pi y, 0), b = (0, sin 2 pi x):
    ad_a b = Da b - Db a = (2 pi cos 2 pi y sin 2 pi x, -2 pi cos 2 pi x sin 2 pi y)."""
    grid, band = (12, 12), (6, 6)
    X, Y = grid_coords(grid)
    tp = 2 * np.pi
    a = np.stack([pi(np.sin(tp * Y), band), pi(0 * X, band)])
    b = np.stack([pi(0 * X, band), pi(np.sin(tp * X), band)])
    expect = np.stack([pi(tp * np.cos(tp * Y) * np.sin(tp * X), band),
                       pi(-tp * np.cos(tp * X) * np.sin(tp * Y), band)])
    np.testing.assert_allclose(ad(a, b, (9, 9)), expect, atol=1e-12)


def test_jacobi_identity_low_frequency():
    """Exact for fields with |k| <= 1 in a band holding |k| <= 3 (no truncation)."""
    band = (8, 8, 8)
    M = (12, 12, 12)
    a, b, c = rand_field(6, band, 1), rand_field(7, band, 1), rand_field(8, band, 1)
    J = ad(a, ad(b, c, M), M) + ad(b, ad(c, a, M), M) + ad(c, ad(a, b, M), M)
    scale = np.abs(ad(a, ad(b, c, M), M)).max()
    assert np.abs(J).max() < 1e-12 * scale


def test_ad_star_camassa_holm_reduction():
    """d = 1 reduction: ad*_u m = 2 m u_x + u m_x (Camassa-Holm form)."""
    x = sympy.symbols("x", real=True)
    tp = 2 * sympy.pi
    u = sympy.sin(tp * x) + sympy.Rational(3, 10) * sympy.cos(2 * tp * x)
    m = sympy.cos(tp * x) + sympy.Rational(1, 2) * sympy.sin(2 * tp * x)
    rhs = 2 * m * sympy.diff(u, x) + u * sympy.diff(m, x)
    fu, fm, fr = (sympy.lambdify(x, e, "numpy") for e in (u, m, rhs))
    grid, band = (24, 8), (12, 4)
    X, _ = grid_coords(grid)
    zero = pi(0 * X, band)
    a = np.stack([pi(fu(X), band), zero])
    mu = np.stack([pi(fm(X), band), zero])
    out = ad_star(a, mu, (18, 6))
    np.testing.assert_allclose(out[0], pi(fr(X), band), atol=1e-12)
    assert np.abs(out[1]).max() < 1e-13


def test_ad_star_of_constant_field_is_advection():
    band, M = (8, 8), (12, 12)
    c = np.zeros((2,) + band, dtype=complex)
    c[0][0, 0], c[1][0, 0] = 0.3, -0.7
    mu = rand_field(9, band)
    out = ad_star(c, mu, M)
    from oracle.band import symbol_D
    adv = 0.3 * symbol_D(band, 0) * mu + -0.7 * symbol_D(band, 1) * mu
    np.testing.assert_allclose(out, adv, atol=1e-12)
    # and the momentum of a constant velocity is not moved: ad*_c (L c) = 0
    assert np.abs(ad_star(c, c, M)).max() < 1e-14


def params(grid, band, nt=10, s=2):
    return Params(grid=grid, band=band, nt=nt, alpha=0.0025, s=s, sigma=0.03)


def smooth_velocity(seed, band, amp=0.05, s=2):
    from paper_1807_11560_amd import synth
    v = synth.random_band_field(np.random.default_rng(seed), band, 0.0025, s)
    return v * (amp / np.abs(v).max())


def test_shoot_zero_and_constant():
    p = params((16, 16, 16), (8, 8, 8))
    v0 = np.zeros((3,) + p.band, dtype=complex)
    assert all(np.abs(v).max() == 0 for v in shoot(v0, p))
    v0[:, 0, 0, 0] = (0.1, -0.2, 0.05)
    for v in shoot(v0, p):
        np.testing.assert_allclose(v, v0, atol=1e-15)


@pytest.mark.parametrize("grid,band", [((16, 16), (8, 8)), ((12, 12, 12), (6, 6, 6))])
def test_euler_energy_identity(grid, band):
    """E_{n+1} - E_n = dt^2 <a_n, K a_n> with E_n = <L v_n, v_n> and
    a_n = ad*_{v_n} L v_n: the first-order term <ad*_v Lv, v> = <Lv, ad_v v>
    vanishes, the discrete form of momentum conservation (§2.2)."""
    p = params(grid, band)
    Ls = symbol_L(p.band, p.alpha, p.s)
    vs = shoot(smooth_velocity(10, band, 0.05), p)
    for n in range(p.nt):
        En, En1 = inner(Ls * vs[n], vs[n]), inner(Ls * vs[n + 1], vs[n + 1])
        a = ad_star(vs[n], Ls * vs[n], p.spectral)
        pred = p.dt ** 2 * inner(a, a / Ls)
        assert abs((En1 - En) - pred) < 1e-9 * En


def test_energy_drift_first_order_in_dt():
    grid, band = (16, 16), (8, 8)
    Ls = symbol_L(band, 0.0025, 2)
    v0 = smooth_velocity(11, band, 0.01)
    drift = []
    for nt in (10, 20, 40):
        vs = shoot(v0, params(grid, band, nt))
        drift.append(inner(Ls * vs[-1], vs[-1]) - inner(Ls * v0, v0))
    assert drift[0] > 0
    assert 1.8 < drift[0] / drift[1] < 2.2 and 1.8 < drift[1] / drift[2] < 2.2


def test_momentum_moves_with_velocity():
    """A velocity bump along x: its momentum L v travels in the direction of
    the velocity (EPDiff transports momentum with the flow; the opposite sign
    of the equation would move it against the velocity)."""
    grid, band = (64, 4), (16, 4)
    X, _ = grid_coords(grid)
    bump = np.exp(-((X - 0.5) ** 2) / (2 * 0.1 ** 2))
    p = params(grid, band, nt=40, s=1)
    Ls = symbol_L(band, p.alpha, p.s)

    def centroid(v):
        m = iota((Ls * v)[0], grid)[:, 0]
        z = np.sum(np.abs(m) * np.exp(2j * np.pi * np.arange(grid[0]) / grid[0]))
        return np.angle(z) / (2 * np.pi) % 1.0

    for amp in (0.1, -0.1):
        v0 = np.stack([pi(amp * bump, band), pi(0 * X, band)])
        vs = shoot(v0, p)
        c0, c1 = centroid(vs[0]), centroid(vs[-1])
        assert abs(c0 - 0.5) < 1e-9
        moved = (c1 - c0) * np.sign(amp)
        assert 0.05 < moved < 0.2


def test_axis_permutation_equivariance():
    p = params((12, 12, 12), (6, 6, 6))
    v0 = smooth_velocity(12, p.band, 0.05)
    perm = (2, 0, 1)
    vp = np.stack([np.transpose(v0[perm[c]], perm) for c in range(3)])
    out = shoot(v0, p)[-1]
    outp = shoot(vp, p)[-1]
    expect = np.stack([np.transpose(out[perm[c]], perm) for c in range(3)])
    np.testing.assert_allclose(outp, expect, atol=1e-12)


def test_ad_dagger_definition_consistency():
    """<ad_dagger_a b, c>_V = <b, ad_a c>_V: ad_dagger is the V-adjoint of ad."""
    band, M = (8, 8), (12, 12)
    Ls = symbol_L(band, 0.0025, 2)
    a, b, c = rand_field(13, band), rand_field(14, band), rand_field(15, band)
    lhs = inner(Ls * ad_dagger(a, b, Ls, M), c)
    rhs = inner(Ls * b, ad(a, c, M))
    assert abs(lhs - rhs) < 1e-10 * max(1.0, abs(lhs))


def test_ad_golden_sine_pair():
    """Hand-derived coefficients of ad_a b for a = (sin 2 pi x1, 0),
    b = (0, sin 2 pi x0) (tests/golden/ad_sine_pair_2d.txt), set up directly
    in band coefficients (no transform on the input side)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "ad_sine_pair_2d.txt")
    rows = [line.split() for line in open(path) if line.strip() and not line.startswith("#")]
    band = (8, 8)
    a = np.zeros((2,) + band, dtype=np.complex128)
    b = np.zeros((2,) + band, dtype=np.complex128)
    a[0, 0, 1], a[0, 0, -1] = -0.5j, 0.5j
    b[1, 1, 0], b[1, -1, 0] = -0.5j, 0.5j
    expect = np.zeros((2,) + band, dtype=np.complex128)
    for c, k0, k1, re, im in rows:
        expect[int(c), int(k0), int(k1)] = float(re) + 1j * float(im)
    assert len(rows) == 8
    np.testing.assert_allclose(ad(a, b, (12, 12)), expect, atol=1e-12)
