"""Geodesic shooting on the band (paper §3.1/§3.2, band-limited EPDiff).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings:
  * Sign: the paper writes the band equation once as d_t v = ad~dagger v and
    then as d_t v + ad~dagger_v v = 0 (§3.2) in agreement with the continuous
    EPDiff of §2.2, d_t v = -K ad*_v L v.  The minus sign is taken.
  * Time discretisation: nt explicit Euler steps of size 1/nt,
        v_{n+1} = v_n - dt K~ ad~*_{v_n}(L~ v_n),   n = 0..nt-1.
"""

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
