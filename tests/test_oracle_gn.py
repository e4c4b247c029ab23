"""Pins of the oracle's Krylov solver and Gauss-Newton loop (paper §2.7):
V-metric CG equals textbook preconditioned CG on the equivalent system, the
curvature guard, and monotone energy decrease of a small registration."""

import numpy as np

from oracle import Params
from oracle.band import symbol_L
from oracle.gn import pcg, register
from oracle.jacobi import forward
from paper_1807_11560_amd import synth


def textbook_pcg(S, b, Minv, iters):
    """Preconditioned CG for S x = b (Saad, Iterative Methods, Alg. 9.1)."""
    x = np.zeros_like(b)
    r = b - S @ x
    z = Minv @ r
    p = z.copy()
    for _ in range(iters):
        Sp = S @ p
        a = (r @ z) / (p @ Sp)
        x = x + a * p
        r_new = r - a * Sp
        z_new = Minv @ r_new
        beta = (r_new @ z_new) / (r @ z)
        p = z_new + beta * p
        r, z = r_new, z_new
    return x


def test_v_metric_cg_is_preconditioned_cg():
    """CG on H p = -g in <a,b>_V = <L a, b> with H = L^-1 S (self-adjoint in
    V) is PCG on S p = -L g preconditioned by L^-1."""
    rng = np.random.default_rng(0)
    n = 30
    A = rng.standard_normal((n, n))
    S = A @ A.T + n * np.eye(n)
    Ldiag = rng.uniform(1.0, 20.0, n)
    g = rng.standard_normal(n)
    H = S / Ldiag[:, None]
    for iters in (3, 7):
        p, info = pcg(lambda d: H @ d, g, Ldiag, iters)
        ref = textbook_pcg(S, -Ldiag * g, np.diag(1.0 / Ldiag), iters)
        np.testing.assert_allclose(p, ref, rtol=1e-10, atol=1e-12)
        assert info["iters"] == iters and not info["guard"]
    p, _ = pcg(lambda d: H @ d, g, Ldiag, n)
    np.testing.assert_allclose(p, -np.linalg.solve(H, g), rtol=1e-8)


def test_curvature_guard():
    g = np.array([1.0, -2.0, 0.5])
    L = np.ones(3)
    p, info = pcg(lambda d: -d, g, L, 5)
    assert info["guard"] and info["iters"] == 0
    np.testing.assert_array_equal(p, -g)
    p, info = pcg(lambda d: d, np.zeros(3), L, 5)  # zero residual: nothing to do
    assert info["iters"] == 0 and not p.any()


def test_small_registration_decreases_energy():
    grid, band = (32, 32), (8, 8)
    p = Params(grid=grid, band=band, nt=5, alpha=0.0025, s=2, sigma=0.03)
    rng = np.random.default_rng(1000)
    I0 = synth.gaussian_blobs(rng, grid, count=5) * 0.9
    vstar = synth.scale_to_displacement(synth.random_band_field(rng, band, s=2), grid, 2.0)
    I1 = forward(vstar, I0, p)[2][-1]
    v, stats, status = register(I0, I1, p, gn_iters=3, pcg_iters=5)
    assert status == 0
    E = [s["E"] for s in stats]
    assert all(E[i + 1] < E[i] for i in range(len(E) - 1))
    m1 = forward(v, I0, p)[2][-1]
    mse = 100 * np.sum((m1 - I1) ** 2) / np.sum((I0 - I1) ** 2)
    assert mse < 50.0
    assert np.abs(v).max() > 0 and symbol_L(band, 0.0025, 2).shape == band
