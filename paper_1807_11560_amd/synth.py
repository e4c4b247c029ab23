"""Seeded synthetic workloads shaped like the paper's brain-MRI registrations.

This module only draws random numbers and builds images; it holds none of the
registration arithmetic (no shooting, transport, gradient or Hessian), so the
library and the FP64 oracle can both be fed from it.  Targets are produced by
shooting a random initial velocity with whichever implementation is under
test or serves as the checker.

Band arrays are complex128 of shape (d,) + band in FFT storage order (slot q
holds frequency q for q < K/2 and q - K otherwise; the slot -K/2 is zero),
Hermitian (v(-k) = conj v(k)), with the k = 0 mode zeroed (no translation).
"""

import numpy as np

# ---------------------------------------------------------------- problem set
# The workloads: 2-D Gaussian blobs, 3-D nested ellipsoids, 3-D tissue
# phantom (the measured workload), the large volume; the batch is below.
CONFIGS = {
    1: dict(grid=(64, 64), band=(16, 16), s=2, nt=10, dmax=4.0, gn=5, pcg=10),
    2: dict(grid=(64, 64, 64), band=(16, 16, 16), s=2, nt=10, dmax=5.0, gn=10, pcg=20),
    3: dict(grid=(128, 128, 128), band=(32, 32, 32), s=3, nt=10, dmax=8.0, gn=10, pcg=20),
    4: dict(grid=(160, 192, 160), band=(32, 32, 32), s=3, nt=20, dmax=5.0, gn=0, pcg=0),
}
ALPHA = 0.0025
SIGMA = 0.03


def seed_for(config, pair=0):
    return 1000 * config + pair


def _freqs(K):
    q = np.arange(K)
    return np.where(q < K // 2, q, q - K)


def _band_support(band):
    m = np.ones(tuple(band), dtype=bool)
    for j, K in enumerate(band):
        shape = [1] * len(band)
        shape[j] = K
        m &= (np.abs(_freqs(K)) <= K // 2 - 1).reshape(shape)
    return m


def _hermitian(f):
    idx = np.ix_(*[(-np.arange(K)) % K for K in f.shape])
    return 0.5 * (f + np.conj(f[idx]))


def random_band_field(rng, band, alpha=ALPHA, s=2, zero_mean=True):
    """Complex normal coefficients on the band, Hermitian, damped by the
    spectral weight (1 + alpha |2 pi k|^2)^-s (smooth random velocities)."""
    band = tuple(band)
    d = len(band)
    lap = np.zeros(band)
    for j, K in enumerate(band):
        shape = [1] * d
        shape[j] = K
        lap = lap + (2 * np.pi * _freqs(K).reshape(shape)) ** 2
    weight = (1.0 + alpha * lap) ** (-s)
    sup = _band_support(band)
    comps = []
    for _ in range(d):
        xi = rng.standard_normal(band) + 1j * rng.standard_normal(band)
        xi = _hermitian(xi * sup) * weight
        if zero_mean:
            xi[(0,) * d] = 0.0
        comps.append(xi)
    return np.stack(comps)


def band_to_grid_fft(v, grid):
    """Evaluate a band field on the grid with numpy's FFT (used only to size
    the random velocities; not part of the registration arithmetic)."""
    d = v.shape[0]
    out = []
    for c in range(d):
        spec = np.zeros(tuple(grid), dtype=np.complex128)
        idx = np.ix_(*[_freqs(K) % N for K, N in zip(v.shape[1:], grid)])
        spec[idx] = v[c]
        out.append(np.fft.ifftn(spec).real * float(np.prod(grid)))
    return np.stack(out)


def scale_to_displacement(v, grid, dmax):
    """Scale v so that its largest displacement over unit time, measured in
    voxels (max_x |(v_j(x) N_j)_j|), equals dmax."""
    g = band_to_grid_fft(v, grid)
    mag = np.sqrt(sum((g[j] * grid[j]) ** 2 for j in range(len(grid))))
    return v * (dmax / float(mag.max()))


# ------------------------------------------------------------------- phantoms
def gaussian_blobs(rng, grid, count=12):
    """2-D: clipped sum of isotropic Gaussians, centres in the central 60 %,
    widths (std) 3-8 px, amplitudes U[0.3, 1], periodic minimum-image
    distance."""
    grid = tuple(grid)
    img = np.zeros(grid)
    coords = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in grid], indexing="ij")
    for _ in range(count):
        c = [rng.uniform(0.2 * n, 0.8 * n) for n in grid]
        w = rng.uniform(3.0, 8.0)
        a = rng.uniform(0.3, 1.0)
        r2 = 0.0
        for j, n in enumerate(grid):
            dx = np.abs(coords[j] - c[j])
            dx = np.minimum(dx, n - dx)
            r2 = r2 + dx ** 2
        img += a * np.exp(-r2 / (2.0 * w * w))
    return np.clip(img, 0.0, 1.0)


def nested_ellipsoids(rng, grid, noise=0.02):
    """3-D: three nested ellipsoids centred at N/2 with semi-axes U[12, 28]
    voxels (sorted per axis so they nest), intensities 0.2 / 0.5 / 0.8 from
    the outer shell to the core, background 0, plus N(0, noise^2)."""
    grid = tuple(grid)
    axes = np.sort(rng.uniform(12.0, 28.0, size=(3, len(grid))), axis=0)[::-1]
    coords = np.meshgrid(*[np.arange(n, dtype=np.float64) - n / 2.0 for n in grid], indexing="ij")
    img = np.zeros(grid)
    for level, value in enumerate((0.2, 0.5, 0.8)):
        r = sum((coords[j] / axes[level][j]) ** 2 for j in range(len(grid)))
        img[r <= 1.0] = value
    return img + noise * rng.standard_normal(grid)


def tissue_phantom(rng, grid, noise=0.02, kmax=6):
    """3-D brain-like phantom: a smooth random Fourier series g (modes with
    |k|_inf <= kmax, weight exp(-|k|^2/18)) thresholded at its 20 % / 60 %
    quantiles inside an ellipsoidal mask (semi-axes 0.40, 0.45, 0.38 of the
    grid) into CSF 0.2 / GM 0.5 / WM 0.8, zero outside, then Rician noise
    I = sqrt((I + n1)^2 + n2^2) with n ~ N(0, noise^2).  The series is
    resolution independent, so one atlas can be sampled at any grid."""
    grid = tuple(grid)
    d = len(grid)
    ks = np.arange(-kmax, kmax + 1)
    kk = np.meshgrid(*([ks] * d), indexing="ij")
    k2 = sum(k.astype(np.float64) ** 2 for k in kk)
    coef = (rng.standard_normal(k2.shape) + 1j * rng.standard_normal(k2.shape)) * np.exp(-k2 / 18.0)
    coef = 0.5 * (coef + np.conj(coef[(slice(None, None, -1),) * d]))
    spec = np.zeros(grid, dtype=np.complex128)
    idx = np.ix_(*[ks % n for n in grid])
    spec[idx] = coef
    g = np.fft.ifftn(spec).real
    coords = np.meshgrid(*[(np.arange(n, dtype=np.float64) - n / 2.0) / n for n in grid], indexing="ij")
    semi = (0.40, 0.45, 0.38)[:d]
    mask = sum((coords[j] / semi[j]) ** 2 for j in range(d)) <= 1.0
    inside = g[mask]
    q20, q60 = np.quantile(inside, [0.2, 0.6])
    img = np.zeros(grid)
    img[mask & (g <= q20)] = 0.2
    img[mask & (g > q20) & (g <= q60)] = 0.5
    img[mask & (g > q60)] = 0.8
    n1 = noise * rng.standard_normal(grid)
    n2 = noise * rng.standard_normal(grid)
    return np.sqrt((img + n1) ** 2 + n2 ** 2)


def make_source(config, rng, grid=None):
    grid = tuple(grid or CONFIGS[config]["grid"])
    if config == 1:
        return gaussian_blobs(rng, grid)
    if config == 2:
        return nested_ellipsoids(rng, grid)
    return tissue_phantom(rng, grid)


def workload(config, pair=0, grid=None, band=None):
    """Source image and target velocity of one registration pair.

    Returns dict(I0, v_star, params) where v_star is the random band-limited
    initial velocity whose geodesic warps I0 into the target."""
    c = dict(CONFIGS[config])
    if grid is not None:
        c["grid"] = tuple(grid)
    if band is not None:
        c["band"] = tuple(band)
    rng = np.random.default_rng(seed_for(config, pair))
    I0 = make_source(config, rng, c["grid"])
    v = random_band_field(rng, c["band"], ALPHA, c["s"])
    v = scale_to_displacement(v, c["grid"], c["dmax"])
    params = dict(grid=c["grid"], band=c["band"], nt=c["nt"], alpha=ALPHA, s=c["s"],
                  sigma=SIGMA, gn=c["gn"], pcg=c["pcg"])
    return dict(I0=I0, v_star=v, params=params)


# The batched serving workload: pairs warped from one atlas, each with a grid
# and a band drawn from these sets and a maximal displacement in [4, 10] voxels.
BATCH = dict(grids=((96, 96, 96), (128, 128, 128), (144, 176, 144), (160, 192, 160)),
             bands=((24, 24, 24), (32, 32, 32)), dmax=(4.0, 10.0), s=3, nt=10, gn=10, pcg=20)
BATCH_SEED = 5000


def batch_workload(pairs=16, seed=BATCH_SEED):
    """Source images and target velocities of `pairs` atlas registrations.
    The atlas is one tissue phantom (its random series is drawn from the same
    seed for every grid, so all sources are samplings of one image).  Returns a
    list of dicts like ``workload``."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(pairs):
        grid = BATCH["grids"][int(rng.integers(len(BATCH["grids"])))]
        band = BATCH["bands"][int(rng.integers(len(BATCH["bands"])))]
        dmax = float(rng.uniform(*BATCH["dmax"]))
        I0 = tissue_phantom(np.random.default_rng(seed + 1), grid)
        v = scale_to_displacement(random_band_field(rng, band, ALPHA, BATCH["s"]), grid, dmax)
        params = dict(grid=grid, band=band, nt=BATCH["nt"], alpha=ALPHA, s=BATCH["s"], sigma=SIGMA,
                      gn=BATCH["gn"], pcg=BATCH["pcg"])
        out.append(dict(I0=I0, v_star=v, params=params))
    return out


def random_direction(seed, band, s=2, alpha=ALPHA):
    """Random Hermitian band direction of unit l2 norm."""
    rng = np.random.default_rng(seed)
    v = random_band_field(rng, band, alpha, s, zero_mean=False)
    return v / np.sqrt(np.real(np.vdot(v, v)))
