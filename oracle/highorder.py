"""Shooting and state transport with higher-order time integration (paper
§2.2: the geodesic conserves <L v_t, v_t>; §3.2 state equation).  FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

forward_rk: the band EPDiff by classical RK4 (``epdiff.shoot_rk4``), then
the image transport with midpoint departure points whose mid-step velocity is
iota of the band average of v_n and v_{n+1} (``transport.transport_rk2``).
The adjoint sweeps of the gradient and the Hessian-vector product are the
transposes of Euler steps and are not integrated this way.
"""

from .band import iota_vec
from .epdiff import shoot_rk4
from .transport import transport_rk2


def forward_rk(v0, I0, p):
    """(v_0..v_nt, m_0..m_nt) of the higher-order forward model."""
    vs = shoot_rk4(v0, p)
    vmids = [iota_vec(0.5 * (vs[n] + vs[n + 1]), p.grid) for n in range(p.nt)]
    return vs, transport_rk2(I0, vmids, p.dt)
