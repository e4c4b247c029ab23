"""Energy, gradient and Hessian-vector product of band-limited Jacobi
PDE-EPDiff LDDMM subject to the state equation (paper §3.2).  FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Steps, in the paper's order:
  forward    band EPDiff shooting v_0..v_nt, then the state transport
             m_0 = I0, m_{n+1} = I[m_n](x - dt iota(v_n)(x))
  energy     E = 1/2 <L~ v_0, v_0>_l2 + sigma^-2 ||m_nt - I1||^2_L2 (§3.2,
             band-limited energy), ||f||^2_L2 = |N|^-1 sum_x f(x)^2
  gradient   lambda_1 = -(2/sigma^2)(m_nt - I1) (§2.3), U_nt = K~ pi(lambda_1
             grad_h m_nt) (§3.2), then the reduced adjoint Jacobi equations of
             §3.2 integrated backward with w_nt = 0:
               w_n = w_{n+1} + dt [U_{n+1} - ad~_{v_n} w_{n+1}
                                   + ad~dagger_{w_{n+1}} v_n]
               U_n = U_{n+1} + dt ad~dagger_{v_n} U_{n+1}
             gradient in the V metric g_V = v_0 + w_0.
  hessvec    incremental EPDiff forward (§2.5/§3.2),
               dv_{n+1} = dv_n - dt [ad~dagger_{dv_n} v_n + ad~dagger_{v_n} dv_n]
             incremental state transport (§2.5) to dm_nt, dlambda_1 =
             -(2/sigma^2) dm_nt (§2.3), dU_nt = K~ pi(dlambda_1 grad_h m_nt),
             then the reduced incremental adjoint Jacobi equations of §3.2
             backward with dw_nt = 0:
               dU_n = dU_{n+1} + dt [ad~dagger_{v_n} dU_{n+1}
                                     + ad~dagger_{dv_n} U_{n+1}]
               dw_n = dw_{n+1} + dt [dU_{n+1} - ad~_{dv_n} w_{n+1}
                                     - ad~_{v_n} dw_{n+1}
                                     + ad~dagger_{dw_{n+1}} v_n
                                     + ad~dagger_{w_{n+1}} dv_n]
             H_V dv_0 = dv_0 + dw_0.

Readings:
  * The third term of the w equation: the band equations of §3.2 print
    ad~dagger there, while the reduced adjoint Jacobi equations of §2.2 and
    both deformation-state variants print ad; ad is taken, which makes the
    discrete backward sweep the exact transpose of the forward Jacobi
    recursion Y_{n+1} = Y_n + dt (ad~_{v_n} Y_n + dv_n).
  * Each backward step is the transpose of the corresponding forward Euler
    step: it uses v_n (and dv_n) with the adjoint values at n+1.
  * Gauss-Newton (§2.7 drops unnamed terms of the Hessian): mode "R1" drops
    only the -lambda_1 grad(dm_1) term of dU(1) and keeps every coupling term
    of the incremental adjoint Jacobi equations; mode "R2" also drops the
    coupling terms that carry U or w (ad~dagger_{dv} U, ad~_{dv} w,
    ad~dagger_w dv).  The two coincide when lambda_1 = 0.
  * K~ and pi commute (both act per frequency), so the paper's K~(pi(.)) for
    U(1) and pi(K~(.)) for dU(1) are the same operation.
  * Full Newton (mode "FULL", the incremental equations of §2.3/§3.2 with no
    term dropped): dU(1) = K~ pi(dlambda_1 grad m_1 + lambda_1 grad dm_1),
    the derivative of U(1) = K~ pi(lambda_1 grad m_1).  The paper prints a
    minus before lambda_1 grad dm_1; with it the product is not the
    derivative of the gradient (a test pins the plus sign: at v_0 = 0 the
    "FULL" product equals the central difference of the gradient).
"""

import numpy as np

from .band import inner, iota_vec, pi_vec, symbol_K, symbol_L
from .epdiff import shoot
from .lie import ad, ad_dagger
from .transport import grad_h, incremental_transport, transport


def forward(v0, I0, p):
    """Band trajectory, its grid velocities (steps 0..nt-1) and the states."""
    vs = shoot(v0, p)
    vgrid = [iota_vec(vs[n], p.grid) for n in range(p.nt)]
    ms = transport(I0, vgrid, p.dt)
    return vs, vgrid, ms


def energy(v0, m1, I1, p):
    """(E, E_reg, E_data) of the band-limited energy (paper §3.2)."""
    Lsym = symbol_L(p.band, p.alpha, p.s)
    e_reg = 0.5 * inner(Lsym * v0, v0)
    e_data = float(np.sum((m1 - I1) ** 2)) / (p.sigma ** 2 * float(np.prod(p.grid)))
    return e_reg + e_data, e_reg, e_data


def backward_sweep(vs, U_nt, p):
    """Reduced adjoint Jacobi equations (§3.2) from U_nt, w_nt = 0.
    Returns the lists U_0..U_nt and w_0..w_nt."""
    Lsym = symbol_L(p.band, p.alpha, p.s)
    U = U_nt
    w = np.zeros_like(U)
    Us = [None] * (p.nt + 1)
    ws = [None] * (p.nt + 1)
    Us[p.nt], ws[p.nt] = U, w
    for n in range(p.nt - 1, -1, -1):
        v = vs[n]
        w_new = w + p.dt * (U - ad(v, w, p.spectral) + ad_dagger(w, v, Lsym, p.spectral))
        U = U + p.dt * ad_dagger(v, U, Lsym, p.spectral)
        w = w_new
        Us[n], ws[n] = U, w
    return Us, ws


def gradient(v0, I0, I1, p):
    """V-metric gradient g_V = v_0 + w_0 and the trajectories it used."""
    Ksym = symbol_K(p.band, p.alpha, p.s)
    vs, vgrid, ms = forward(v0, I0, p)
    E = energy(v0, ms[-1], I1, p)
    lam1 = -(2.0 / p.sigma ** 2) * (ms[-1] - I1)
    U_nt = Ksym * pi_vec(lam1 * grad_h(ms[-1]), p.band)
    Us, ws = backward_sweep(vs, U_nt, p)
    g = v0 + ws[0]
    cache = dict(vs=vs, vgrid=vgrid, ms=ms, Us=Us, ws=ws, lam1=lam1)
    return g, E, cache


def incremental_shoot(vs, dv0, p):
    """Incremental band EPDiff trajectory dv_0..dv_{nt-1} (paper §2.5/§3.2)."""
    Lsym = symbol_L(p.band, p.alpha, p.s)
    dvs = [dv0]
    for n in range(p.nt - 1):
        dv = dvs[n]
        dvs.append(dv - p.dt * (ad_dagger(dv, vs[n], Lsym, p.spectral)
                                + ad_dagger(vs[n], dv, Lsym, p.spectral)))
    return dvs


def incremental_backward(vs, dvs, Us, ws, dU_nt, p, mode="R1"):
    """Reduced incremental adjoint Jacobi equations (§3.2) from dU_nt,
    dw_nt = 0.  Returns dw_0."""
    if mode not in ("R1", "R2", "FULL"):
        raise ValueError("mode must be 'R1', 'R2' or 'FULL'")
    Lsym = symbol_L(p.band, p.alpha, p.s)
    dU = dU_nt
    dw = np.zeros_like(dU)
    coupling = mode != "R2"
    for n in range(p.nt - 1, -1, -1):
        v, dv = vs[n], dvs[n]
        rhs_w = dU - ad(v, dw, p.spectral) + ad_dagger(dw, v, Lsym, p.spectral)
        rhs_U = ad_dagger(v, dU, Lsym, p.spectral)
        if coupling:
            rhs_w = rhs_w - ad(dv, ws[n + 1], p.spectral) + ad_dagger(ws[n + 1], dv, Lsym, p.spectral)
            rhs_U = rhs_U + ad_dagger(dv, Us[n + 1], Lsym, p.spectral)
        dw = dw + p.dt * rhs_w
        dU = dU + p.dt * rhs_U
    return dw


def hessvec(cache, dv0, p, mode="R1"):
    """Hessian-vector product H_V dv_0 (paper §3.2, §2.7): Gauss-Newton
    modes "R1" and "R2", or the full Newton product "FULL"."""
    Ksym = symbol_K(p.band, p.alpha, p.s)
    vs, vgrid, ms, Us, ws = (cache[k] for k in ("vs", "vgrid", "ms", "Us", "ws"))
    dvs = incremental_shoot(vs, dv0, p)
    dvgrid = [iota_vec(dvs[n], p.grid) for n in range(p.nt)]
    dm = incremental_transport(ms, vgrid, dvgrid, p.dt)
    dlam1 = -(2.0 / p.sigma ** 2) * dm
    src = dlam1 * grad_h(ms[-1])
    if mode == "FULL":
        src = src + cache["lam1"] * grad_h(dm)
    dU = Ksym * pi_vec(src, p.band)
    return dv0 + incremental_backward(vs, dvs, Us, ws, dU, p, mode)
