"""Exact derivative of the discrete band-limited energy (paper §3.2: the
energy E(v0) = 1/2 <L~ v0, v0> + sigma^-2 ||m(1) - I1||^2 subject to the
band-limited EPDiff equation and the state equation, here after the
discretisation of the Jacobi module: explicit Euler steps of the band EPDiff,
one first-order semi-Lagrangian step of the state per time step).  FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's gradient (§3.2, the Jacobi module) transports the adjoint of the
image only through its value at t = 1 and carries it backward in the band.
That is a discretisation of the continuous adjoint, not the derivative of the
discrete energy above; the two differ by the band truncation of the
coadjoint transport and by O(dt) and O(h) terms.  Here every discrete step is
differentiated in reverse order instead:

  state adjoint   lambda_nt = 2 / (sigma^2 |N|) (m_nt - I1)  (= dE/dm_nt),
                  lambda_n = I^T[lambda_{n+1}] at the departure points
                  X_n = x - dt v_n(x): the transpose of the trilinear
                  interpolation, a scatter of lambda_{n+1}(x) with the
                  interpolation weights onto the corners of X_n(x);
  velocity source dE/dv_n(x)_j = -dt N_j lambda_{n+1}(x) (d_j I[m_n])(X_n(x)),
                  with d_j I[m_n] the exact derivative of the interpolant
                  (the slope of the cell that holds X_n(x), per voxel of
                  axis j; X is in voxels, v in units of the unit cube);
                  in the band, iota_N^T of a real grid field g is
                  |N| pi_N(g) (the l2 gradient with respect to the band
                  coefficients);
  band adjoint    the transpose of each Euler step v_{n+1} = v_n + dt F(v_n),
                  F(v) = -K~ ad~*_v(L~ v), written in the V metric
                  w = K~ a (a the l2 adjoint):
                    w_n = w_{n+1} + dt [-ad~_{v_n} w_{n+1}
                                        + K~ ad~*_{w_{n+1}}(L~ v_n)] + S_n,
                    S_n = K~ |N| pi_N(dE/dv_n),   w_nt = 0,
                  which is the w recursion of the paper's sweep with the
                  source U_{n+1} replaced by the per-step transport source
                  and no U recursion;
  gradient        g_V = v_0 + w_0 (the regulariser's V gradient is v_0).

The Gauss-Newton product of this energy is J^T W J + Id in the V metric, with
J the derivative of m_nt with respect to v_0 (the incremental EPDiff of the
Jacobi module, then the tangent of each transport step,
  dm_{n+1}(x) = I[dm_n](X_n(x)) - dt sum_j N_j (d_j I[m_n])(X_n(x)) dv_n(x)_j,
dm_0 = 0) and W = 2 / (sigma^2 |N|): the adjoint above applied to
lambda_nt = W dm_nt.  It is symmetric positive definite in <., .>_V.
"""

import itertools

import numpy as np

from .band import iota_vec, pi_vec, symbol_K, symbol_L
from .jacobi import energy, forward, incremental_shoot
from .lie import ad, ad_dagger
from .transport import departure_points, interpolate


def departure_points_fp32(v, dt):
    """Departure points formed in single precision as the library's kernels
    form them: t = fl32(dt v_j), X_j = fl32(i_j - t N_j) with the product t N_j
    exact (one fused multiply-add).  The cell of a departure point is an
    integer that floating point decides; the exact derivative jumps with it
    (the slope of the interpolant is piecewise constant), so a comparison with
    a single-precision implementation takes that decision in single
    precision.  Returned as float64 values."""
    grid = v.shape[1:]
    d = len(grid)
    nodes = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in grid], indexing="ij")
    out = []
    for j in range(d):
        t = (np.float32(dt) * v[j].astype(np.float32)).astype(np.float64)
        out.append((nodes[j] - t * float(grid[j])).astype(np.float32).astype(np.float64))
    return np.stack(out)


def _departures(decisions):
    return departure_points_fp32 if decisions == "fp32" else departure_points


def _cells(X, shape):
    """Per axis: the lower corner index (periodic) and the fractional part."""
    base = [np.floor(X[j]) for j in range(len(shape))]
    frac = [X[j] - base[j] for j in range(len(shape))]
    idx0 = [base[j].astype(np.int64) % shape[j] for j in range(len(shape))]
    return idx0, frac


def interpolant_gradient(f, X):
    """(d_j I[f])(X) for every axis j: the derivative of the periodic
    multilinear interpolant of f with respect to voxel coordinate j at X."""
    d = f.ndim
    idx0, frac = _cells(X, f.shape)
    out = []
    for j in range(d):
        g = np.zeros(X.shape[1:])
        for corner in itertools.product((0, 1), repeat=d):
            w = np.ones(X.shape[1:])
            for i in range(d):
                if i == j:
                    w = w * (1.0 if corner[i] else -1.0)
                else:
                    w = w * (frac[i] if corner[i] else 1.0 - frac[i])
            ind = tuple((idx0[i] + corner[i]) % f.shape[i] for i in range(d))
            g = g + w * f[ind]
        out.append(g)
    return np.stack(out)


def interpolate_transpose(lam, X):
    """I^T[lam]: every lam(x) scattered onto the corners of the cell of X(x)
    with its interpolation weights (the transpose of ``interpolate``)."""
    d = lam.ndim
    idx0, frac = _cells(X, lam.shape)
    out = np.zeros(lam.size)
    for corner in itertools.product((0, 1), repeat=d):
        w = np.ones(X.shape[1:])
        for i in range(d):
            w = w * (frac[i] if corner[i] else 1.0 - frac[i])
        ind = tuple((idx0[i] + corner[i]) % lam.shape[i] for i in range(d))
        out += np.bincount(np.ravel_multi_index(ind, lam.shape).ravel(), weights=(w * lam).ravel(),
                           minlength=lam.size)
    return out.reshape(lam.shape)


def adjoint_sweep(vs, vgrid, ms, lam_nt, p, decisions="fp64"):
    """The reverse sweep above from the state adjoint lambda_nt: returns w_0
    (V metric) and the per-step band sources S_n.  decisions="fp32" forms the
    departure points as a single-precision implementation does (see
    departure_points_fp32)."""
    dep = _departures(decisions)
    Lsym = symbol_L(p.band, p.alpha, p.s)
    Ksym = symbol_K(p.band, p.alpha, p.s)
    nN = float(np.prod(p.grid))
    scale = np.array(p.grid, dtype=np.float64).reshape((p.d,) + (1,) * p.d)
    lam = lam_nt
    w = np.zeros_like(vs[0])
    sources = [None] * p.nt
    for n in range(p.nt - 1, -1, -1):
        X = dep(vgrid[n], p.dt)
        dEdv = -p.dt * scale * lam[None] * interpolant_gradient(ms[n], X)
        S = Ksym * nN * pi_vec(dEdv, p.band)
        sources[n] = S
        w = w + p.dt * (-ad(vs[n], w, p.spectral) + ad_dagger(w, vs[n], Lsym, p.spectral)) + S
        lam = interpolate_transpose(lam, X)
    return w, sources


def gradient(v0, I0, I1, p, decisions="fp64"):
    """V-metric gradient of the discrete energy, the energy and a cache."""
    vs, vgrid, ms = forward(v0, I0, p)
    E = energy(v0, ms[-1], I1, p)
    lam = 2.0 / (p.sigma ** 2 * float(np.prod(p.grid))) * (ms[-1] - I1)
    w, sources = adjoint_sweep(vs, vgrid, ms, lam, p, decisions)
    cache = dict(vs=vs, vgrid=vgrid, ms=ms, sources=sources)
    return v0 + w, E, cache


def tangent_transport(ms, vgrid, dvgrid, dt, decisions="fp64"):
    """dm_nt of the tangent of the transport steps, dm_0 = 0."""
    dep = _departures(decisions)
    grid = ms[0].shape
    scale = np.array(grid, dtype=np.float64).reshape((len(grid),) + (1,) * len(grid))
    dm = np.zeros(grid)
    for n in range(len(vgrid)):
        X = dep(vgrid[n], dt)
        dm = interpolate(dm, X) - dt * np.sum(scale * interpolant_gradient(ms[n], X) * dvgrid[n], axis=0)
    return dm


def gauss_newton_hessvec(cache, dv0, p, decisions="fp64"):
    """(J^T W J + Id) dv0 in the V metric (see the module docstring)."""
    vs, vgrid, ms = cache["vs"], cache["vgrid"], cache["ms"]
    dvs = incremental_shoot(vs, dv0, p)
    dvgrid = [iota_vec(dvs[n], p.grid) for n in range(p.nt)]
    dm = tangent_transport(ms, vgrid, dvgrid, p.dt, decisions)
    lam = 2.0 / (p.sigma ** 2 * float(np.prod(p.grid))) * dm
    w, _ = adjoint_sweep(vs, vgrid, ms, lam, p, decisions)
    return dv0 + w
