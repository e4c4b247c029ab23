"""The workloads' geodesics have the maximal displacement their recipe
names.  The input generators scale the random initial velocity by its
largest grid value (max_x |v(x) N| in voxels over unit time: they hold none
of the method's arithmetic); the displacement of the geodesic itself,
u(1) = phi(1) - id of the deformation state equation integrated by the FP64
oracle (paper §3.3), must come out within 15 % of the nominal value."""

import numpy as np
import pytest

from oracle import Params, deformation
from oracle.band import iota_vec
from paper_1807_11560_amd import synth


@pytest.mark.parametrize("config", [1, 2, 3])
def test_geodesic_displacement_matches_the_recipe(config):
    w = synth.workload(config)
    pp = w["params"]
    p = Params(grid=pp["grid"], band=pp["band"], nt=pp["nt"], alpha=pp["alpha"], s=pp["s"], sigma=pp["sigma"])
    us = deformation.forward(w["v_star"], w["I0"], p)[1]
    ug = iota_vec(us[-1], p.grid)
    dmax = float(np.sqrt(sum((ug[j] * p.grid[j]) ** 2 for j in range(p.d))).max())
    nominal = synth.CONFIGS[config]["dmax"]
    print(f"config {config}: geodesic displacement {dmax:.3f} voxels (nominal {nominal})")
    assert 0.85 * nominal <= dmax <= 1.15 * nominal
