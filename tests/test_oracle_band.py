"""Pins of the oracle's band algebra (paper §3.1) against things other than
itself: numpy's FFT, symbolic differentiation, Parseval, brute-force
convolution and the alias bound of the padded product."""

import numpy as np
import pytest
import sympy

from oracle.band import (band_mask, brute_convolution, freqs, hermitian_part, inner, iota,
                         iota_complex, pi, star, symbol_D, symbol_K, symbol_L)
from paper_1807_11560_amd import synth


def rand_herm(seed, band):
    rng = np.random.default_rng(seed)
    f = rng.standard_normal(band) + 1j * rng.standard_normal(band)
    return hermitian_part(f, band)


@pytest.mark.parametrize("grid,band", [((12, 10), (6, 4)), ((8, 10, 6), (4, 6, 4)), ((16,), (8,))])
def test_iota_matches_numpy_ifft(grid, band):
    f = rand_herm(1, band)
    spec = np.zeros(grid, dtype=np.complex128)
    idx = np.ix_(*[freqs(K) % N for K, N in zip(band, grid)])
    spec[idx] = f
    ref = np.fft.ifftn(spec) * np.prod(grid)
    np.testing.assert_allclose(iota_complex(f, grid), ref, atol=1e-12)
    assert np.abs(ref.imag).max() < 1e-12  # Hermitian -> real field


@pytest.mark.parametrize("grid,band", [((12, 10), (6, 4)), ((8, 10, 6), (4, 6, 4))])
def test_pi_matches_numpy_fft_and_is_hermitian(grid, band):
    rng = np.random.default_rng(2)
    g = rng.standard_normal(grid)
    spec = np.fft.fftn(g) / np.prod(grid)
    idx = np.ix_(*[freqs(K) % N for K, N in zip(band, grid)])
    ref = spec[idx] * band_mask(band)
    out = pi(g, band)
    np.testing.assert_allclose(out, ref, atol=1e-13)
    np.testing.assert_allclose(hermitian_part(out, band), out, atol=1e-14)


def test_pi_iota_roundtrip_and_slot_zero():
    band, grid = (8, 6, 4), (16, 12, 10)
    f = rand_herm(3, band)
    np.testing.assert_allclose(pi(iota(f, grid), band), f, atol=1e-13)
    # the -K/2 slot of every axis is outside the effective band
    m = band_mask(band)
    assert not m[4].any() and not m[:, 3].any() and not m[:, :, 2].any()


def test_parseval():
    band, grid = (6, 8), (10, 12)
    rng = np.random.default_rng(4)
    g = rng.standard_normal(grid)
    a = rand_herm(5, band)
    lhs = inner(pi(g, band), a)
    rhs = float(np.sum(g * iota(a, grid))) / np.prod(grid)
    assert abs(lhs - rhs) < 1e-13 * max(1.0, abs(rhs))
    # l2 norm of the band = L2 norm of the synthesised field
    assert abs(inner(a, a) - np.sum(iota(a, grid) ** 2) / np.prod(grid)) < 1e-12


def test_symbols_by_symbolic_differentiation():
    """L = (Id - alpha Laplacian)^s applied to exp(2 pi i k.x) symbolically."""
    x, y, z = sympy.symbols("x y z", real=True)
    alpha = sympy.Rational(1, 400)
    band = (6, 6, 4)
    fr = [freqs(K) for K in band]
    Ls = symbol_L(band, 0.0025, 3)
    for q in [(1, 2, 1), (5, 0, 3), (2, 4, 0)]:
        k = [int(fr[j][q[j]]) for j in range(3)]
        e = sympy.exp(2 * sympy.pi * sympy.I * (k[0] * x + k[1] * y + k[2] * z))
        f = e
        for _ in range(3):
            f = f - alpha * (sympy.diff(f, x, 2) + sympy.diff(f, y, 2) + sympy.diff(f, z, 2))
        sym = complex(sympy.simplify(f / e))
        assert abs(sym - Ls[q]) < 1e-10 * abs(sym)
        for j, var in enumerate((x, y, z)):
            dsym = complex(sympy.simplify(sympy.diff(e, var) / e))
            assert abs(dsym - symbol_D(band, j)[tuple(q[i] if i == j else 0 for i in range(3))]) < 1e-12
    np.testing.assert_allclose(symbol_K(band, 0.0025, 3) * Ls, 1.0, rtol=1e-15)


@pytest.mark.parametrize("band", [(4, 4), (6, 6), (8, 8), (4, 6, 4)])
def test_star_equals_brute_force_convolution(band):
    f = rand_herm(6, band)
    g = rand_herm(7, band)
    ref = brute_convolution(f, g)
    M = tuple(3 * K // 2 - 2 for K in band)  # smallest alias-free grid
    np.testing.assert_allclose(star(f, g, M), ref, atol=1e-12)
    np.testing.assert_allclose(star(f, g, tuple(3 * K // 2 for K in band)), ref, atol=1e-12)


@pytest.mark.parametrize("band", [(6, 6), (8, 8)])
def test_star_alias_bound_is_tight(band):
    f = rand_herm(8, band)
    g = rand_herm(9, band)
    ref = brute_convolution(f, g)
    M = tuple(3 * K // 2 - 3 for K in band)
    assert np.abs(star(f, g, M) - ref).max() > 1e-3


def test_random_field_generator_is_hermitian_and_band_limited():
    v = synth.random_band_field(np.random.default_rng(0), (8, 6, 4), s=2)
    for c in v:
        np.testing.assert_allclose(hermitian_part(c, (8, 6, 4)), c, atol=1e-15)
    assert v[:, 0, 0, 0].tolist() == [0, 0, 0]
