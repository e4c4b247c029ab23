"""Pins of the oracle's Krylov solver and Gauss-Newton loop (paper §2.7):
V-metric CG equals textbook preconditioned CG on the equivalent system, the
curvature guard, monotone energy decrease of a small registration, the Armijo
search against a brute-force scan of the energy, the slope handed to it
against a central difference of the energy at v0 = 0, and a one-parameter
translation problem whose every iterate, energy, MSE_rel and gradient norm
follow from a scalar computation written without the oracle."""

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


# ---------------------------------------------------------------------------
# Armijo search and the Gauss-Newton loop against cases the mathematics fixes
# (paper §2.7: the update v0 + eps p and its step length).

from oracle import gn as GN  # noqa: E402
from oracle.jacobi import energy  # noqa: E402


def _small_problem():
    grid, band = (16, 14), (6, 6)
    p = Params(grid=grid, band=band, nt=4, alpha=0.0025, s=2, sigma=0.03)
    rng = np.random.default_rng(1007)
    x = np.meshgrid(*[np.arange(n) / n for n in grid], indexing="ij")
    I0 = (0.5 + 0.25 * np.sin(2 * np.pi * x[0] + 0.3) * np.cos(2 * np.pi * x[1] - 0.2)
          + 0.1 * np.sin(4 * np.pi * x[1] + 1.0))
    vstar = synth.scale_to_displacement(synth.random_band_field(rng, band, s=2), grid, 1.5)
    I1 = forward(vstar, I0, p)[2][-1]
    return p, I0, I1, vstar, rng


def _E(v, I0, I1, p):
    return energy(v, forward(v, I0, p)[2][-1], I1, p)[0]


def test_line_search_is_first_armijo_point_of_a_brute_force_scan():
    """The accepted step is the first eps in 1, 1/2, 1/4, ... of a scan of
    E(v0 + eps p) with E <= E0 + c1 eps slope; the search fails (eps = 0,
    no energy) when no trial passes.  Sufficient-decrease constants well above
    1e-4 make the threshold decide between trials."""
    p, I0, I1, vstar, rng = _small_problem()
    v0 = 0.2 * vstar
    E0 = _E(v0, I0, I1, p)
    direction = vstar - v0
    h = 1e-6
    slope = (_E(v0 + h * direction, I0, I1, p) - _E(v0 - h * direction, I0, I1, p)) / (2 * h)
    assert slope < 0
    scan = [(0.5 ** k, _E(v0 + 0.5 ** k * direction, I0, I1, p)) for k in range(10)]
    seen = set()
    for c1 in (1e-4, 0.3, 0.6, 0.8, 0.95):
        expect = next((k + 1 for k, (eps, E) in enumerate(scan) if E <= E0 + c1 * eps * slope), None)
        ok, eps, E, trials = GN.line_search(v0, direction, E0, slope, I0, I1, p, c1=c1)
        assert ok and trials == expect and eps == scan[expect - 1][0]
        assert abs(E[0] - scan[expect - 1][1]) <= 1e-13 * abs(E0)
        seen.add(expect)
    assert len(seen) >= 2  # the constants really select different trials
    ok, eps, E, trials = GN.line_search(v0, -direction, E0, -slope, I0, I1, p, max_trials=3)
    assert (ok, eps, E, trials) == (False, 0.0, None, 3)


def test_register_passes_the_v_metric_slope(monkeypatch):
    """At v0 = 0 the paper's gradient is the derivative of the discrete energy
    (central differences of the image, the average of the interpolant's
    one-sided slopes), so the slope that the loop hands to the Armijo search
    must equal the central difference of E along the search direction.  A
    slope taken in l2 (without L~) is off by the symbol's weights."""
    p, I0, I1, vstar, rng = _small_problem()
    seen = {}

    def spy(v0, p_dir, E0, slope, *args, **kw):
        seen.update(v0=v0.copy(), p_dir=p_dir.copy(), E0=E0, slope=slope)
        return real(v0, p_dir, E0, slope, *args, **kw)

    real = GN.line_search
    monkeypatch.setattr(GN, "line_search", spy)
    GN.register(I0, I1, p, gn_iters=1, pcg_iters=3)
    assert not seen["v0"].any()
    d = seen["p_dir"]
    scale = 1e-7 / np.abs(d).max()
    fd = (_E(scale * d, I0, I1, p) - _E(-scale * d, I0, I1, p)) / (2 * scale)
    assert seen["slope"] < 0
    assert abs(seen["slope"] - fd) <= 1e-5 * abs(fd), (seen["slope"], fd)
    assert abs(seen["E0"] - _E(np.zeros_like(d), I0, I1, p)) <= 1e-14 * seen["E0"]


# A one-parameter registration: an image that varies along axis 0 only as one
# sine, its target translated along that axis, band 4 x 4 (|k_j| <= 1).  The
# data-term products of two |k0| = 1 modes land at k0 = 0 or |k0| = 2, so the
# gradient, every Hessian-vector product and every iterate live on the k = 0
# coefficient u of component 0 (a constant velocity, which the band EPDiff
# keeps constant).  Shooting plus transport is then a 1-D linear-interpolation
# shift by dt u N0 voxels per step, written below without the oracle.
_N0, _N1, _SHIFT = 24, 6, 1.3


def _translation_problem():
    p = Params(grid=(_N0, _N1), band=(4, 4), nt=4, alpha=0.0025, s=2, sigma=0.03)
    x0 = np.arange(_N0)[:, None] / _N0 * np.ones((1, _N1))
    I0 = 0.5 + 0.3 * np.sin(2 * np.pi * x0)
    I1 = 0.5 + 0.3 * np.sin(2 * np.pi * (x0 - _SHIFT / _N0))
    return p, I0, I1


def _m1_1d(u, I0, nt):
    """nt steps of m(i) <- m at i - dt u N0 by linear interpolation."""
    f = I0[:, 0].copy()
    shift = u * _N0 / nt
    q = int(np.floor(shift))
    a = shift - q
    for _ in range(nt):
        f = (1 - a) * np.roll(f, q) + a * np.roll(f, q + 1)
    return f


def _E_1d(u, I0, I1, p):
    r = _m1_1d(u, I0, p.nt) - I1[:, 0]
    return 0.5 * u * u + float(np.mean(r * r)) / p.sigma ** 2


def test_translation_registration_follows_the_scalar_problem():
    p, I0, I1 = _translation_problem()
    h = 1e-6
    dE0 = (_E_1d(h, I0, I1, p) - _E_1d(-h, I0, I1, p)) / (2 * h)
    D = (_m1_1d(h, I0, p.nt) - _m1_1d(-h, I0, p.nt)) / (2 * h)  # dm1/du at u = 0
    hess = 1.0 + 2.0 / p.sigma ** 2 * float(np.mean(D * D))     # Gauss-Newton curvature
    pu = -dE0 / hess
    E0 = _E_1d(0.0, I0, I1, p)
    eps_expect = next(0.5 ** k for k in range(10)
                      if _E_1d(0.5 ** k * pu, I0, I1, p) <= E0 + 1e-4 * 0.5 ** k * dE0 * pu)

    v1, st1, status = GN.register(I0, I1, p, gn_iters=1, pcg_iters=2)
    assert status == 0
    u1 = v1[0, 0, 0].real
    rest = v1.copy()
    rest[0, 0, 0] = 0
    assert np.abs(rest).max() <= 1e-12 * abs(u1) and abs(v1[0, 0, 0].imag) <= 1e-12 * abs(u1)
    assert st1[0]["eps"] == eps_expect and st1[0]["trials"] == 1 + int(round(-np.log2(eps_expect)))
    assert abs(u1 - eps_expect * pu) <= 1e-6 * abs(pu)
    assert abs(st1[0]["E"] - E0) <= 1e-13 * E0
    assert st1[0]["mse_rel"] == 100.0 and st1[0]["g_inf_rel"] == 1.0
    assert st1[0]["pcg_iters"] >= 1 and not st1[0]["pcg_guard"]

    # MSE_rel and the gradient's sup norm of an iteration are those of its
    # starting iterate.  On this problem the paper's gradient reduces to one
    # number: pi at k = 0 is the mean, K~(0) = L~(0) = 1, the U and w sweeps
    # carry constants that every ad and ad* of constants annihilates, so
    # g(u) = u + mean(lambda_1 d0 m1) with lambda_1 = -(2/sigma^2)(m1 - I1)
    # and d0 the periodic central difference.
    def g_red(u):
        m1 = _m1_1d(u, I0, p.nt)
        d0 = (np.roll(m1, -1) - np.roll(m1, 1)) * (_N0 / 2.0)
        return u - 2.0 / p.sigma ** 2 * float(np.mean((m1 - I1[:, 0]) * d0))

    assert abs(g_red(0.0) - dE0) <= 1e-6 * abs(dE0)  # exact at u = 0
    v3, st3, status = GN.register(I0, I1, p, gn_iters=3, pcg_iters=2)
    assert status == 0
    r1 = _m1_1d(u1, I0, p.nt) - I1[:, 0]
    r0 = I0[:, 0] - I1[:, 0]
    assert abs(st3[1]["mse_rel"] - 100.0 * np.sum(r1 * r1) / np.sum(r0 * r0)) <= 1e-9 * st3[1]["mse_rel"]
    assert abs(st3[1]["E"] - _E_1d(u1, I0, I1, p)) <= 1e-12 * st3[1]["E"]
    assert abs(st3[1]["g_inf_rel"] - abs(g_red(u1)) / abs(g_red(0.0))) <= 1e-6 * st3[1]["g_inf_rel"]
    assert all(st3[k + 1]["E"] < st3[k]["E"] for k in range(2))

    # Gauss-Newton converges to the root of the paper's gradient (bisection on
    # the reduced form) ...
    a, b = 0.5 * _SHIFT / _N0, 1.5 * _SHIFT / _N0
    assert g_red(a) < 0 < g_red(b)
    for _ in range(100):
        c = 0.5 * (a + b)
        a, b = (c, b) if g_red(c) < 0 else (a, c)
    uA = 0.5 * (a + b)
    u3 = v3[0, 0, 0].real
    u2 = GN.register(I0, I1, p, gn_iters=2, pcg_iters=2)[0][0, 0, 0].real
    errs = [abs(u - uA) / uA for u in (u1, u2, u3)]
    assert errs[2] < 1e-4 and errs[1] < errs[0] / 5 and errs[2] < errs[1] / 5, errs

    # ... which sits near the minimiser of the scalar energy (a dense scan
    # refined by golden sections) but not on it: the paper's gradient uses the
    # central difference of m1, not the derivative of the interpolation.  From
    # there the Gauss-Newton direction does not decrease the energy: the search
    # fails and the loop keeps the last accepted iterate.
    us = np.linspace(0.0, 2.0 * _SHIFT / _N0, 401)
    k = int(np.argmin([_E_1d(u, I0, I1, p) for u in us]))
    a, b = us[max(k - 1, 0)], us[min(k + 1, len(us) - 1)]
    gr = (np.sqrt(5) - 1) / 2
    for _ in range(80):
        c, d = b - gr * (b - a), a + gr * (b - a)
        if _E_1d(c, I0, I1, p) < _E_1d(d, I0, I1, p):
            b = d
        else:
            a = c
    ustar = 0.5 * (a + b)
    assert 1e-4 * ustar < abs(u3 - ustar) <= 1e-2 * ustar, (u3, ustar)
    v6, st6, status = GN.register(I0, I1, p, gn_iters=6, pcg_iters=2)
    fails = [k for k, r in enumerate(st6) if r["eps"] == 0.0]
    assert status == 1 and fails == [len(st6) - 1] and st6[-1]["trials"] == 10
    assert v6[0, 0, 0].real == u3  # the last accepted iterate
