"""Pins of the oracle's exact derivative of the discrete energy
(oracle/exact.py; paper §3.2 energy and constraints in their Euler /
semi-Lagrangian discretisation): central finite differences of the energy
itself, of the transport, and the transposes.

  * <g, d>_V equals the central difference of E along d to 1e-6 (FP64, step
    1e-7 of the iterate: the energy is smooth inside the trilinear cells and
    no departure point crosses a face over so small a step);
  * interpolate_transpose is the transpose of interpolate, and
    interpolant_gradient the derivative of interpolate (brute force);
  * the tangent transport equals the central difference of m_nt;
  * the Gauss-Newton product is symmetric in the V metric and at least the
    identity (J^T W J is positive semi-definite);
  * the paper's gradient (Jacobi module) differs from this one by the
    method gap that the Jacobi module's docstring describes: reported."""

import numpy as np
import pytest

from oracle import Params
from oracle import exact
from oracle.band import inner, symbol_L
from oracle.jacobi import energy, forward
from oracle.jacobi import gradient as paper_gradient
from oracle.transport import interpolate
from paper_1807_11560_amd import synth

CASES = {
    "2d": dict(grid=(20, 18), band=(8, 6), nt=4, s=2),
    "3d": dict(grid=(12, 10, 14), band=(6, 6, 4), nt=3, s=2),
}


def problem(name):
    c = CASES[name]
    p = Params(grid=c["grid"], band=c["band"], nt=c["nt"], alpha=0.0025, s=c["s"], sigma=0.03)
    rng = np.random.default_rng(21)
    x = np.meshgrid(*[np.arange(n) / n for n in c["grid"]], indexing="ij")
    I0 = 0.5 + 0.2 * np.sin(2 * np.pi * x[0] + 0.4) * np.cos(2 * np.pi * x[1] - 0.3)
    if len(c["grid"]) == 3:
        I0 = I0 + 0.1 * np.sin(2 * np.pi * (x[2] + x[0]))
    vstar = synth.scale_to_displacement(synth.random_band_field(rng, c["band"], s=2), c["grid"], 1.5)
    I1 = forward(vstar, I0, p)[2][-1]
    v0 = 0.6 * vstar + synth.scale_to_displacement(synth.random_band_field(rng, c["band"], s=2), c["grid"], 0.4)
    return p, I0, I1, v0, rng


def E_of(v, I0, I1, p):
    return energy(v, forward(v, I0, p)[2][-1], I1, p)[0]


@pytest.mark.parametrize("name", list(CASES))
def test_gradient_is_the_derivative_of_the_discrete_energy(name):
    p, I0, I1, v0, rng = problem(name)
    g, E, _ = exact.gradient(v0, I0, I1, p)
    assert abs(E[0] - E_of(v0, I0, I1, p)) <= 1e-14 * E[0]
    Lsym = symbol_L(p.band, p.alpha, p.s)
    for k in range(4):
        d = synth.random_direction(100 + k, p.band, s=1)
        h = 1e-7 * np.linalg.norm(v0) / np.linalg.norm(d)
        fd = (E_of(v0 + h * d, I0, I1, p) - E_of(v0 - h * d, I0, I1, p)) / (2 * h)
        an = inner(Lsym * g, d)
        assert abs(an - fd) <= 1e-6 * abs(fd), (k, an, fd)


def test_transpose_and_derivative_of_the_interpolation():
    rng = np.random.default_rng(5)
    shape = (5, 4, 6)
    f = rng.standard_normal(shape)
    lam = rng.standard_normal(shape)
    X = np.stack([rng.uniform(-3, 9, size=shape) for _ in range(3)])
    # <I[f], lam> = <f, I^T[lam]>
    assert abs(np.sum(interpolate(f, X) * lam) - np.sum(f * exact.interpolate_transpose(lam, X))) < 1e-12
    G = exact.interpolant_gradient(f, X)
    h = 1e-6
    for j in range(3):
        e = np.zeros_like(X)
        e[j] = h
        fd = (interpolate(f, X + e) - interpolate(f, X - e)) / (2 * h)
        np.testing.assert_allclose(G[j], fd, atol=1e-8)


@pytest.mark.parametrize("name", list(CASES))
def test_tangent_transport_is_the_derivative_of_the_state(name):
    p, I0, I1, v0, rng = problem(name)
    _, _, cache = exact.gradient(v0, I0, I1, p)
    from oracle.band import iota_vec
    from oracle.jacobi import incremental_shoot
    d = synth.random_direction(7, p.band, s=1)
    dvs = incremental_shoot(cache["vs"], d, p)
    dm = exact.tangent_transport(cache["ms"], cache["vgrid"], [iota_vec(x, p.grid) for x in dvs], p.dt)
    h = 1e-7 * np.linalg.norm(v0) / np.linalg.norm(d)
    fd = (forward(v0 + h * d, I0, p)[2][-1] - forward(v0 - h * d, I0, p)[2][-1]) / (2 * h)
    assert np.linalg.norm(dm - fd) <= 1e-6 * np.linalg.norm(fd)


@pytest.mark.parametrize("name", list(CASES))
def test_gauss_newton_product_is_symmetric_and_at_least_the_identity(name):
    p, I0, I1, v0, rng = problem(name)
    _, _, cache = exact.gradient(v0, I0, I1, p)
    Lsym = symbol_L(p.band, p.alpha, p.s)
    a = synth.random_direction(11, p.band, s=1)
    b = synth.random_direction(12, p.band, s=1)
    Ha = exact.gauss_newton_hessvec(cache, a, p)
    Hb = exact.gauss_newton_hessvec(cache, b, p)
    ab, ba = inner(Lsym * a, Hb), inner(Lsym * b, Ha)
    assert abs(ab - ba) <= 1e-12 * max(abs(ab), abs(ba))
    for x, Hx in ((a, Ha), (b, Hb)):
        assert inner(Lsym * x, Hx) >= inner(Lsym * x, x) * (1 - 1e-12)


def test_paper_gradient_gap_is_reported():
    """Not gated: the method gap between the paper's gradient and the exact
    one on the 3-D case (the band truncation of the coadjoint transport,
    O(dt) and O(h))."""
    p, I0, I1, v0, rng = problem("3d")
    gB, _, _ = exact.gradient(v0, I0, I1, p)
    gA, _, _ = paper_gradient(v0, I0, I1, p)
    gap = np.linalg.norm(gA - gB) / np.linalg.norm(gB)
    print(f"paper gradient vs exact: relative gap {gap:.3f}")
    assert np.isfinite(gap)


def test_exact_gauss_newton_loop_decreases_energy():
    """The Gauss-Newton-Krylov loop with the exact gradient and its
    (positive definite) Gauss-Newton product: CG is never stopped by the
    curvature guard and the energy decreases at every iteration."""
    from oracle.gn import register
    p, I0, I1, v0, rng = problem("2d")
    v, stats, status = register(I0, I1, p, gn_iters=4, pcg_iters=5, mode="EXACT")
    assert status == 0
    assert not any(s["pcg_guard"] for s in stats)
    assert all(stats[k + 1]["E"] < stats[k]["E"] for k in range(len(stats) - 1))


def test_single_precision_departure_points():
    """departure_points_fp32 rounds v, dt v and the departure point to single
    precision (within half an ulp of X plus 2^-23 of the displacement of the
    FP64 point) and leaves every
    derivative of the oracle a derivative of its energy: at FP64 departure
    points everything above holds; with FP32 ones only the cell decisions of
    a few points move (the gradient by 1e-5-1e-4 here)."""
    from oracle.transport import departure_points
    p, I0, I1, v0, rng = problem("3d")
    vg = forward(v0, I0, p)[1][0]
    X64 = departure_points(vg, p.dt)
    X32 = exact.departure_points_fp32(vg, p.dt)
    nodes = np.stack(np.meshgrid(*[np.arange(n, dtype=np.float64) for n in p.grid], indexing="ij"))
    ulp = np.spacing(np.abs(X64).astype(np.float32)).astype(np.float64)
    bound = 0.5 * ulp + 2.0 ** -23 * np.abs(X64 - nodes) * 1.01
    assert np.all(np.abs(X32 - X64) <= bound)
    assert np.any(X32 != X64)
    assert np.all(X32 == X32.astype(np.float32))
    g64, _, _ = exact.gradient(v0, I0, I1, p)
    g32, _, _ = exact.gradient(v0, I0, I1, p, decisions="fp32")
    gap = np.linalg.norm(g32 - g64) / np.linalg.norm(g64)
    print(f"FP32 cell decisions move the exact gradient by {gap:.1e}")
    assert gap < 1e-3
