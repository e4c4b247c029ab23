"""Energy, gradient and Hessian-vector product of band-limited Jacobi
PDE-EPDiff LDDMM subject to the deformation state equation (paper §3.3).
FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The state is the deformation phi(t) = id + u(t), carried in the band; the
image only appears at t = 1 through m(1) = I0 o phi(1).  Steps, in the
paper's order:
  forward    band EPDiff shooting v_0..v_nt (as §3.2), then the band
             deformation state equation by explicit Euler steps,
               u_{n+1} = u_n - dt [v_n + D~u_n * v_n],   u_0 = 0,
             (D~u * v)_i = sum_j (d_j u_i) * v_j (truncated products), and
             m(1)(x) = I0(x + iota(u_nt)(x)) by periodic multilinear
             interpolation.
  energy     as §3.2, with this m(1).
  gradient   lambda_1 = -(2/sigma^2)(m(1) - I1),
             rho(1) = lambda_1 (grad I0)(phi(1)),  rho~ = pi(rho(1)),
             U_nt = K~ (D~phi(1) * rho~),
               (D~phi * r)_j = r_j + sum_i (d_j u_i) * r_i,
             then the reduced adjoint Jacobi sweep of §3.2 (§3.3 restates
             the same equations); g_V = v_0 + w_0.
  hessvec    incremental EPDiff (as §3.2), the incremental deformation state
               du_{n+1} = du_n - dt [D~du_n * v_n + dv_n + D~u_n * dv_n],
               du_0 = 0,
             dm(1) = (grad I0)(phi(1)) . iota(du_nt),
             dlambda_1 = -(2/sigma^2) dm(1),
             drho(1) = dlambda_1 (grad I0)(phi(1))
                       [+ lambda_1 (Hess I0)(phi(1)) iota(du_nt)],
             dU_nt = K~ ([D~du_nt * rho~] + D~phi(1) * pi(drho(1))),
               (D~du * r)_j = sum_i (d_j du_i) * r_i,
             then the incremental adjoint Jacobi sweep of §3.2;
             H_V dv_0 = dv_0 + dw_0.

Readings:
  * phi~ is read as the band-limited displacement u = phi - id (the identity
    is not periodic and has no band representation), so D~phi~ = Id + D~u.
    The interval of the state equation is printed both as (0,1] and [0,1);
    each Euler step uses the velocity at its start, as the image transport
    of §3.2 does.
  * rho(1) is not defined in §3.3.  It is read as the derivative of the
    image term with respect to phi(1), lambda_1 (grad I0)(phi(1)); then
    D phi(1)^T rho(1) = lambda_1 grad m(1), and U(1) is the band form of the
    U(1) of §3.2.  "D~phi~ * rho~" is read as the contraction with the
    transposed Jacobian (the derivative of <rho, D phi v> with respect to v).
  * How (grad I0)(phi(1)) and (Hess I0)(phi(1)) are sampled (``sampling``):
    "central" (the product path) interpolates the periodic central-difference
    gradient grad_h I0 and Hessian grad_h grad_h I0 multilinearly at
    phi(1)(x), the image gradient of §3.2 carried to phi(1); both are
    continuous in phi(1).  "interpolant" takes the gradient and Hessian of the
    multilinear interpolant of I0 itself, the exact derivatives of the
    discrete m(1) (pure second derivatives vanish inside a cell); with it the
    discrete gradient is differentiated exactly, which the tests use to pin
    every other step.  The two differ at first order in h on smooth images
    (inside a cell the interpolant's gradient is a one-sided difference), and
    the interpolant's gradient jumps across cell faces, which would make FP32
    and FP64 evaluations disagree where phi(1)(x) lies within rounding of a
    face.
  * The paper prints a minus before D~phi~(1) * drho~(1) in dU(1).  The
    derivative of U(1) has a plus, which is taken; a test pins it (at zero
    residual the classical Gauss-Newton product equals the central
    difference of the gradient).
  * Gauss-Newton (§2.7), as for §3.2, where the paper's reading drops the
    term lambda_1 grad(dm_1) of dU(1), the residual times a derivative of the
    increment: mode "R1" drops both such terms of dU(1) here, D~du * rho~
    (rho carries lambda_1) and lambda_1 (Hess I0) iota(du), and keeps every
    coupling term of the sweep; "R2" also drops the coupling terms; "FULL"
    keeps every term and is the derivative of the discrete gradient (away
    from cell faces of the interpolant).  Keeping D~du * rho~ without the
    Hessian term, as the printed dU(1) does, gives a product that is
    indefinite far from the minimum (the CG curvature guard stops the first
    Gauss-Newton iteration of a 32^3 registration and it converges several
    times slower).
"""

import itertools

import numpy as np

from .band import iota, iota_vec, pi, pi_vec, symbol_D, symbol_K
from .epdiff import shoot
from .jacobi import backward_sweep, energy, incremental_backward, incremental_shoot
from .transport import grad_h, interpolate


def jac_star(u, v, spectral):
    """D~u * v, component i: sum_j (d_j u_i) * v_j (§3.3 deformation state)."""
    d = u.shape[0]
    band = u.shape[1:]
    V = [iota(v[j], spectral) for j in range(d)]
    out = []
    for i in range(d):
        prod = sum(iota(symbol_D(band, j) * u[i], spectral) * V[j] for j in range(d))
        out.append(pi(prod, band))
    return np.stack(out)


def jac_t_star(u, r, spectral):
    """(D~u)^T * r, component j: sum_i (d_j u_i) * r_i (§3.3, U(1))."""
    d = u.shape[0]
    band = u.shape[1:]
    R = [iota(r[i], spectral) for i in range(d)]
    out = []
    for j in range(d):
        prod = sum(iota(symbol_D(band, j) * u[i], spectral) * R[i] for i in range(d))
        out.append(pi(prod, band))
    return np.stack(out)


def deformation_transport(vs, p):
    """Displacements u_0..u_nt of the band deformation state equation (§3.3),
    driven by the velocities vs[0..nt-1]."""
    us = [np.zeros_like(vs[0])]
    for n in range(p.nt):
        u = us[-1]
        us.append(u - p.dt * (vs[n] + jac_star(u, vs[n], p.spectral)))
    return us


def interpolate_derivatives(f, X):
    """Value, gradient and Hessian of the periodic multilinear interpolant of
    the grid field ``f`` at voxel coordinates ``X`` (shape (d,) + points).
    Derivatives are per unit length of the unit cube (voxel derivative times
    N_j).  The cell is floor(X), as in the image transport."""
    d = f.ndim
    grid = f.shape
    base = [np.floor(X[j]) for j in range(d)]
    frac = [X[j] - base[j] for j in range(d)]
    idx0 = [base[j].astype(np.int64) for j in range(d)]
    shape = X.shape[1:]
    val = np.zeros(shape)
    grad = np.zeros((d,) + shape)
    hess = np.zeros((d, d) + shape)
    for corner in itertools.product((0, 1), repeat=d):
        fc = f[tuple((idx0[j] + corner[j]) % grid[j] for j in range(d))]
        w = [frac[j] if corner[j] else 1.0 - frac[j] for j in range(d)]
        dw = [(1.0 if corner[j] else -1.0) * grid[j] for j in range(d)]

        def weight(skip):
            out = np.ones(shape)
            for j in range(d):
                if j not in skip:
                    out = out * w[j]
            return out

        val += fc * weight(())
        for a in range(d):
            grad[a] += fc * dw[a] * weight((a,))
            for b in range(d):
                if b != a:
                    hess[a, b] += fc * dw[a] * dw[b] * weight((a, b))
    return val, grad, hess


def compose(I0, ugrid, sampling="central"):
    """m = I0(x + u(x)) at every grid node with the image gradient and Hessian
    sampled there (§3.3, m(1) = I0 o phi(1); ``sampling`` as in the module
    doc)."""
    grid = I0.shape
    d = I0.ndim
    nodes = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in grid], indexing="ij")
    X = np.stack([nodes[j] + ugrid[j] * grid[j] for j in range(d)])
    if sampling == "interpolant":
        return interpolate_derivatives(I0, X)
    if sampling != "central":
        raise ValueError("sampling must be 'central' or 'interpolant'")
    G = grad_h(I0)
    H = np.stack([grad_h(G[b]) for b in range(d)], axis=1)  # H[a, b] = d_a d_b
    val = interpolate(I0, X)
    grad = np.stack([interpolate(G[a], X) for a in range(d)])
    hess = np.stack([np.stack([interpolate(H[a, b], X) for b in range(d)]) for a in range(d)])
    return val, grad, hess


def forward(v0, I0, p, sampling="central"):
    """Band trajectory, displacements and m(1) with the image derivatives
    sampled at phi(1)."""
    vs = shoot(v0, p)
    us = deformation_transport(vs, p)
    m1, gI, hI = compose(I0, iota_vec(us[-1], p.grid), sampling)
    return vs, us, m1, gI, hI


def gradient(v0, I0, I1, p, sampling="central"):
    """V-metric gradient g_V = v_0 + w_0 (§3.3) and the trajectories it used."""
    Ksym = symbol_K(p.band, p.alpha, p.s)
    vs, us, m1, gI, hI = forward(v0, I0, p, sampling)
    E = energy(v0, m1, I1, p)
    lam1 = -(2.0 / p.sigma ** 2) * (m1 - I1)
    rho = pi_vec(lam1 * gI, p.band)
    U_nt = Ksym * (rho + jac_t_star(us[-1], rho, p.spectral))
    Us, ws = backward_sweep(vs, U_nt, p)
    g = v0 + ws[0]
    cache = dict(vs=vs, us=us, m1=m1, gI=gI, hI=hI, lam1=lam1, rho=rho, Us=Us, ws=ws)
    return g, E, cache


def incremental_transport(vs, dvs, us, p):
    """du_nt of the incremental deformation state equation (§3.3), du_0 = 0."""
    du = np.zeros_like(vs[0])
    for n in range(p.nt):
        du = du - p.dt * (jac_star(du, vs[n], p.spectral) + dvs[n]
                          + jac_star(us[n], dvs[n], p.spectral))
    return du


def hessvec(cache, dv0, p, mode="R1"):
    """Hessian-vector product H_V dv_0 (§3.3, §2.7): Gauss-Newton modes "R1"
    and "R2", or the full Newton product "FULL"."""
    if mode not in ("R1", "R2", "FULL"):
        raise ValueError("mode must be 'R1', 'R2' or 'FULL'")
    Ksym = symbol_K(p.band, p.alpha, p.s)
    vs, us, Us, ws, gI = (cache[k] for k in ("vs", "us", "Us", "ws", "gI"))
    dvs = incremental_shoot(vs, dv0, p)
    du = incremental_transport(vs, dvs, us, p)
    dug = iota_vec(du, p.grid)
    dm = np.sum(gI * dug, axis=0)
    src = -(2.0 / p.sigma ** 2) * dm * gI
    if mode == "FULL":
        src = src + cache["lam1"] * np.einsum("ab...,b...->a...", cache["hI"], dug)
    drho = pi_vec(src, p.band)
    dU = drho + jac_t_star(us[-1], drho, p.spectral)
    if mode == "FULL":
        dU = dU + jac_t_star(du, cache["rho"], p.spectral)
    return dv0 + incremental_backward(vs, dvs, Us, ws, Ksym * dU, p, mode)
