"""Problem parameters of the oracle (paper §3.2 problem statement: I0, I1,
L = (Id - alpha*Laplacian)^s, sigma, band size, time steps).

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""

from dataclasses import dataclass, field
from typing import Tuple


@dataclass(frozen=True)
class Params:
    """Parameters of one registration problem.

    grid      N_j, grid points per axis of the periodic unit cube [0,1)^d
    band      K_j, band storage per axis (even); frequency of slot q is q for
              q < K/2 and q - K otherwise; the slot k = -K/2 is held at zero
    spectral  M_j, the padded grid on which the truncated convolution is
              evaluated pseudo-spectrally (None: 3*K_j/2); must be >= 3K/2-2
    nt        number of explicit Euler time steps on [0, 1]
    alpha, s  L = (Id - alpha*Laplacian)^s (paper §2.1)
    sigma     weight of the image term (paper §3.2, band-limited energy)
    """

    grid: Tuple[int, ...]
    band: Tuple[int, ...]
    nt: int = 10
    alpha: float = 0.0025
    s: int = 2
    sigma: float = 0.03
    spectral: Tuple[int, ...] = field(default=None)

    def __post_init__(self):
        if len(self.grid) != len(self.band):
            raise ValueError("grid and band must have the same length")
        if self.spectral is None:
            object.__setattr__(self, "spectral", tuple(3 * k // 2 for k in self.band))
        for n, k, m in zip(self.grid, self.band, self.spectral):
            if k % 2 or k < 2 or k > n:
                raise ValueError("band sizes must be even and at most the grid size")
            if m < 3 * k // 2 - 2:
                raise ValueError("spectral grid too small for an alias-free product")

    @property
    def d(self) -> int:
        return len(self.grid)

    @property
    def dt(self) -> float:
        return 1.0 / self.nt
