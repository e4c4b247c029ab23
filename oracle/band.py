"""Band-limited algebra (paper §3.1, "Background on the space of band-limited
vector fields").  FP64, explicit DFT matrices applied one axis at a time.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings (the paper is silent or garbled here):
  * The domain is the periodic unit cube; iota sums exp(2 pi i k.x) over the
    band.  The paper prints the sum as running over k_j = 0..K_j, which cannot
    give a real field; it is read as the centred band in FFT storage order with
    the slot k_j = -K_j/2 held at zero, so |k_j| <= K_j/2 - 1 on every axis.
  * iota synthesises without normalisation; pi analyses with 1/|N|, so that
    pi(iota(v)) = v and <pi f, a>_l2 = |N|^-1 sum_x f(x) iota(a)(x) (Parseval),
    i.e. the L2 norm on the grid is h^d times the sum over grid points.
  * L~ is the Fourier symbol of (Id - alpha*Laplacian)^s on the unit cube,
    (1 + alpha*sum_j (2 pi k_j)^2)^s; K~ = 1/L~; D~_j = 2 pi i k_j.
  * The truncated convolution f * g is the product of the two synthesised
    fields on an M-grid with M_j >= 3K_j/2 - 2, analysed back onto the band;
    for such M the aliases of the product miss the band, so this equals the
    direct sum over p + q = k of f(p) g(q) (``brute_convolution``).
"""

from functools import lru_cache

import numpy as np


def freqs(K):
    """Integer frequency held in each storage slot of one axis."""
    q = np.arange(K)
    return np.where(q < K // 2, q, q - K)


def axis_mask(K):
    """True on the slots of the effective band |k| <= K/2 - 1."""
    return np.abs(freqs(K)) <= K // 2 - 1


def band_mask(band):
    m = np.ones(tuple(band), dtype=bool)
    for j, K in enumerate(band):
        shape = [1] * len(band)
        shape[j] = K
        m = m & axis_mask(K).reshape(shape)
    return m


def _axis_freqs(band, j):
    shape = [1] * len(band)
    shape[j] = band[j]
    return freqs(band[j]).reshape(shape).astype(np.float64)


def symbol_L(band, alpha, s):
    """Band symbol of L = (Id - alpha*Laplacian)^s (paper §2.1 and §3.1)."""
    lap = sum((2.0 * np.pi * _axis_freqs(band, j)) ** 2 for j in range(len(band)))
    return (1.0 + alpha * lap) ** s


def symbol_K(band, alpha, s):
    """Band symbol of K = L^-1 (paper §2.1)."""
    return 1.0 / symbol_L(band, alpha, s)


def symbol_D(band, j):
    """Band symbol of the partial derivative along axis j: 2 pi i k_j."""
    return 2j * np.pi * _axis_freqs(band, j)


@lru_cache(maxsize=None)
def synthesis_matrix(K, N):
    """E[x, q] = exp(2 pi i k_q x / N) on the band slots, zero on slot -K/2."""
    x = np.arange(N).reshape(N, 1)
    k = freqs(K).reshape(1, K)
    E = np.exp(2j * np.pi * k * x / N)
    E[:, ~axis_mask(K)] = 0.0
    return E


@lru_cache(maxsize=None)
def analysis_matrix(K, N):
    """A[q, x] = exp(-2 pi i k_q x / N) / N on the band slots."""
    x = np.arange(N).reshape(1, N)
    k = freqs(K).reshape(K, 1)
    A = np.exp(-2j * np.pi * k * x / N) / N
    A[~axis_mask(K), :] = 0.0
    return A


def _apply_axis(mat, f, axis):
    return np.moveaxis(np.tensordot(mat, f, axes=([1], [axis])), 0, axis)


def iota_complex(f, grid):
    """Inclusion iota of one band scalar onto the grid, before taking the
    real part (paper §3.1, definition of iota)."""
    g = np.asarray(f, dtype=np.complex128)
    for j, N in enumerate(grid):
        g = _apply_axis(synthesis_matrix(g.shape[j], N), g, j)
    return g


def iota(f, grid):
    """iota of a Hermitian band scalar: a real grid field (paper §3.1)."""
    return iota_complex(f, grid).real


def pi(f, band):
    """Projection pi of a grid scalar onto the band (paper §3.1)."""
    g = np.asarray(f, dtype=np.complex128)
    for j, K in enumerate(band):
        g = _apply_axis(analysis_matrix(K, g.shape[j]), g, j)
    return g


def iota_vec(v, grid):
    return np.stack([iota(c, grid) for c in v])


def pi_vec(f, band):
    return np.stack([pi(c, band) for c in f])


def reverse_index(K):
    """Storage slot holding frequency -k for the slot holding k."""
    return (-np.arange(K)) % K


def hermitian_part(f, band):
    """Orthogonal projection of a band array onto the Hermitian fields
    f(-k) = conj f(k) supported on the effective band.  ``f`` is a scalar of
    shape ``band`` or a vector field of shape ``(d,) + band``."""
    f = np.asarray(f, dtype=np.complex128)
    band = tuple(band)
    idx = np.ix_(*[reverse_index(K) for K in band])
    if f.shape == band:
        g = 0.5 * (f + np.conj(f[idx]))
    else:
        g = np.stack([0.5 * (c + np.conj(c[idx])) for c in f])
    return g * band_mask(band)


def inner(a, b):
    """l2 inner product of band fields: Re sum conj(a) b (paper §3.1)."""
    return float(np.real(np.vdot(a, b)))


def inner_V(a, b, Lsym):
    """V inner product <L~ a, b>_l2 (paper §3.1, scalar product on V~)."""
    return inner(Lsym * a, b)


def star(f, g, spectral):
    """Truncated convolution of two band scalars, evaluated on the M-grid."""
    band = f.shape
    return pi(iota(f, spectral) * iota(g, spectral), band)


def brute_convolution(f, g):
    """Direct truncated convolution sum_{p+q=k} f(p) g(q) over the effective
    band, by enumeration.  Only for tiny bands (used to pin ``star``)."""
    band = f.shape
    mask = band_mask(band)
    out = np.zeros(band, dtype=np.complex128)
    slots = [tuple(i) for i in np.argwhere(mask)]
    fr = [freqs(K) for K in band]
    half = [K // 2 - 1 for K in band]
    for p in slots:
        kp = [fr[j][p[j]] for j in range(len(band))]
        for q in slots:
            kq = [fr[j][q[j]] for j in range(len(band))]
            k = [kp[j] + kq[j] for j in range(len(band))]
            if any(abs(k[j]) > half[j] for j in range(len(band))):
                continue
            r = tuple(k[j] % band[j] for j in range(len(band)))
            out[r] += f[p] * g[q]
    return out
