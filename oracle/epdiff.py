"""Geodesic shooting on the band (paper §3.1/§3.2, band-limited EPDiff).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings:
  * Sign: the paper writes the band equation once as d_t v = ad~dagger v and
    then as d_t v + ad~dagger_v v = 0 (§3.2) in agreement with the continuous
    EPDiff of §2.2, d_t v = -K ad*_v L v.  The minus sign is taken.
  * Time discretisation: nt explicit Euler steps of size 1/nt,
        v_{n+1} = v_n - dt K~ ad~*_{v_n}(L~ v_n),   n = 0..nt-1.
  * Higher order (``shoot_rk4``): the classical four-stage Runge-Kutta
    method on the same right-hand side f(v) = -K~ ad~*_v(L~ v), each stage
    with the truncated product; it conserves <L~ v_t, v_t> (the geodesic
    energy of §2.2) to O(dt^4) instead of O(dt).
"""

import numpy as np

from .band import symbol_L
from .lie import ad_dagger


def shoot(v0, p):
    """Band trajectory v_0..v_nt of the Euler-discretised band EPDiff."""
    Lsym = symbol_L(p.band, p.alpha, p.s)
    vs = [v0]
    v = v0
    for _ in range(p.nt):
        v = v - p.dt * ad_dagger(v, v, Lsym, p.spectral)
        vs.append(v)
    return vs


def shoot_rk4(v0, p):
    """Band trajectory v_0..v_nt of the band EPDiff by classical fourth-order
    Runge-Kutta steps of size 1/nt."""
    Lsym = symbol_L(p.band, p.alpha, p.s)

    def f(v):
        return -ad_dagger(v, v, Lsym, p.spectral)

    vs = [v0]
    v = v0
    h = p.dt
    for _ in range(p.nt):
        k1 = f(v)
        k2 = f(v + 0.5 * h * k1)
        k3 = f(v + 0.5 * h * k2)
        k4 = f(v + h * k3)
        v = v + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        vs.append(v)
    return vs


def energies(vs, p):
    """<L~ v_n, v_n> along a trajectory (the conserved geodesic energy, §2.2)."""
    Lsym = symbol_L(p.band, p.alpha, p.s)
    return [float(np.real(np.vdot(Lsym * v, v))) for v in vs]
