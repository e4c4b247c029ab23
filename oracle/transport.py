"""Semi-Lagrangian transport on the periodic grid (paper §2.3 state equation
d_t m + grad m . v = 0, used in §3.2 with v = iota(v~_t); §2.5 incremental
state equation d_t dm + grad dm . v + grad m . dv = 0).  FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings (the paper gives the PDEs only):
  * One first-order semi-Lagrangian step per Euler step, with the velocity of
    the start of the step: departure point X(x) = x - dt v_n(x), value by
    periodic multilinear interpolation (trilinear in 3-D, bilinear in 2-D),
    cell = floor, weights = fractional parts.
  * The incremental-state source -dt grad_h m_n . dv_n is added at the grid
    nodes and transported with the step:
        dm_{n+1} = I[dm_n - dt grad_h m_n . dv_n](X(x)),   dm_0 = 0.
  * grad_h is the periodic central difference with spacing 1/N_j.
  * Higher order (``transport_rk2``): midpoint-rule departure points with the
    mid-step velocity v_{n+1/2} (on the band, the average of v_n and
    v_{n+1}): X_h = x - dt/2 v_{n+1/2}(x), X = x - dt v_{n+1/2}(X_h), the
    velocity at X_h by the same multilinear interpolation; the departure
    point is then second-order accurate in dt instead of first.
"""

import itertools

import numpy as np


def interpolate(f, X):
    """Periodic multilinear interpolation of grid field ``f`` at voxel
    coordinates ``X`` (shape (d,) + grid)."""
    d = f.ndim
    base = [np.floor(X[j]) for j in range(d)]
    frac = [X[j] - base[j] for j in range(d)]
    idx0 = [base[j].astype(np.int64) for j in range(d)]
    out = np.zeros(X.shape[1:])
    for corner in itertools.product((0, 1), repeat=d):
        w = np.ones(X.shape[1:])
        ind = []
        for j in range(d):
            if corner[j]:
                w = w * frac[j]
            else:
                w = w * (1.0 - frac[j])
            ind.append((idx0[j] + corner[j]) % f.shape[j])
        out += w * f[tuple(ind)]
    return out


def departure_points(v, dt):
    """Voxel coordinates of x - dt v(x) for every grid node x."""
    grid = v.shape[1:]
    d = len(grid)
    nodes = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in grid], indexing="ij")
    return np.stack([nodes[j] - dt * v[j] * grid[j] for j in range(d)])


def sl_step(f, v, dt):
    """One semi-Lagrangian step of the state equation: f(x - dt v(x))."""
    return interpolate(f, departure_points(v, dt))


def grad_h(f):
    """Periodic central differences, spacing 1/N_j along axis j."""
    return np.stack([(np.roll(f, -1, axis=j) - np.roll(f, 1, axis=j)) * (f.shape[j] / 2.0)
                     for j in range(f.ndim)])


def transport(I0, vgrid, dt):
    """State trajectory m_0 = I0, m_{n+1} = I[m_n](x - dt v_n(x))."""
    ms = [I0]
    for v in vgrid:
        ms.append(sl_step(ms[-1], v, dt))
    return ms


def incremental_transport(ms, vgrid, dvgrid, dt):
    """Incremental state dm_nt from dm_0 = 0 (reading in the module doc)."""
    dm = np.zeros_like(ms[0])
    for n in range(len(vgrid)):
        src = dm - dt * np.sum(grad_h(ms[n]) * dvgrid[n], axis=0)
        dm = sl_step(src, vgrid[n], dt)
    return dm


def departure_points_rk2(vmid, dt):
    """Voxel coordinates of the midpoint-rule departure point of every grid
    node for one step of size dt with the mid-step velocity ``vmid``."""
    grid = vmid.shape[1:]
    d = len(grid)
    nodes = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in grid], indexing="ij")
    Xh = np.stack([nodes[j] - 0.5 * dt * vmid[j] * grid[j] for j in range(d)])
    vh = [interpolate(vmid[j], Xh) for j in range(d)]
    return np.stack([nodes[j] - dt * vh[j] * grid[j] for j in range(d)])


def transport_rk2(I0, vmids, dt):
    """State trajectory with midpoint departure points: m_{n+1} = I[m_n](X_n)."""
    ms = [I0]
    for vm in vmids:
        ms.append(interpolate(ms[-1], departure_points_rk2(vm, dt)))
    return ms
