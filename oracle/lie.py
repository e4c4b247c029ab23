"""The band Lie algebra operators (paper §3.1: the band-limited EPDiff equation
and the adjoint operator ad~).  FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

With (Dv)_{ij} = d_j v_i and the truncated convolution *:
  ad~_a b          = D~a * b - D~b * a                      (paper §3.1)
      (ad~_a b)_i  = sum_j (d_j a_i) * b_j - (d_j b_i) * a_j
  ad~*_a mu        = (D~a)^T * mu + D~(mu) * a + mu (div~ * a)
      (ad~*_a mu)_i = sum_j (d_i a_j) * mu_j + (d_j mu_i) * a_j + mu_i * (d_j a_j)
                     (the bracket of the band-limited EPDiff equation, §3.1,
                      with the coadjoint operator of §2.2)
  ad~dagger_a b    = K~ ad~*_a (L~ b)                       (§2.2, §3.1)
ad~* is the exact l2-adjoint of ad~ on Hermitian band fields.

A sum of truncated products is evaluated as pi_M of the sum of the pointwise
products of the synthesised M-grid fields (pi_M is linear); each factor is
synthesised once per call.
"""

import numpy as np

from .band import iota, pi, symbol_D


def _grid_fields(a, spectral):
    """a_j and d_i a_j synthesised on the M-grid: (A[j], DA[i][j])."""
    d = a.shape[0]
    band = a.shape[1:]
    A = [iota(a[j], spectral) for j in range(d)]
    DA = [[iota(symbol_D(band, i) * a[j], spectral) for j in range(d)] for i in range(d)]
    return A, DA


def ad(a, b, spectral):
    """ad~_a b (paper §3.1, adjoint operator)."""
    d = a.shape[0]
    band = a.shape[1:]
    A, DA = _grid_fields(a, spectral)
    B, DB = _grid_fields(b, spectral)
    out = []
    for i in range(d):
        prod = sum(DA[j][i] * B[j] - DB[j][i] * A[j] for j in range(d))
        out.append(pi(prod, band))
    return np.stack(out)


def ad_star(a, mu, spectral):
    """ad~*_a mu (paper §3.1, bracket of the band-limited EPDiff equation)."""
    d = a.shape[0]
    band = a.shape[1:]
    A, DA = _grid_fields(a, spectral)
    MU, DMU = _grid_fields(mu, spectral)
    div_a = sum(DA[j][j] for j in range(d))
    out = []
    for i in range(d):
        prod = sum(DA[i][j] * MU[j] + DMU[j][i] * A[j] for j in range(d)) + MU[i] * div_a
        out.append(pi(prod, band))
    return np.stack(out)


def ad_dagger(a, b, Lsym, spectral):
    """ad~dagger_a b = K~ ad~*_a (L~ b) (paper §2.2 EPDiff, §3.1)."""
    return ad_star(a, Lsym * b, spectral) / Lsym
