"""Edge and degenerate cases of the HIP library against the FP64 oracle and
against what the method fixes exactly.

* smallest sizes the library accepts (grid 8, band 4) and odd grid sizes;
* padded grids other than the default 3K/2: the smallest alias-free one
  (3K/2 - 2) and a larger one (2K), which change the convolution grid but not
  the result on the band;
* zero velocity: the identity map (m_1 = I0, v_1 = 0) exactly;
* zero residual (I1 = m_1 of the same v0): gradient = v0, data energy = 0,
  exactly;
* zero direction: H 0 = 0 exactly;
* the Gauss-Newton loop with the classical Gauss-Newton Hessian (GN_CLASSICAL)
  per iteration against the oracle's mode R2.
Tolerances as in test_gpu_parity (relative L2 1e-4, energies 1e-5)."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import Params  # noqa: E402
from oracle.gn import register  # noqa: E402
from oracle.jacobi import forward, gradient, hessvec  # noqa: E402
from paper_1807_11560_amd import synth  # noqa: E402


def L():
    from paper_1807_11560_amd import lddmm
    return lddmm


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128 if t.is_complex() else np.float64)


def setup(grid, band, nt, spectral=None, dmax=1.0, s=2):
    # the tissue phantom (a random Fourier series) keeps its structure at any grid size
    w = synth.workload(3, grid=grid, band=band)
    p = Params(grid=grid, band=band, nt=nt, alpha=synth.ALPHA, s=s, sigma=synth.SIGMA, spectral=spectral)
    vstar = synth.scale_to_displacement(w["v_star"], grid, dmax)
    I0 = w["I0"]
    I1 = forward(vstar, I0, p)[2][-1]
    prob = L().Problem(grid=grid, band=band, time_steps=nt, alpha=synth.ALPHA, s=s, sigma=synth.SIGMA,
                       spectral=tuple(spectral) if spectral else (0, 0, 0))
    return p, prob, I0, I1, vstar


SHAPES = {
    "min": dict(grid=(8, 8, 8), band=(4, 4, 4), nt=3, dmax=0.5),
    "odd": dict(grid=(13, 17, 15), band=(6, 8, 6), nt=3, dmax=1.0),
    "alias_bound": dict(grid=(20, 18, 16), band=(8, 6, 8), nt=3, spectral=(10, 7, 10), dmax=1.0),
    "wide_pad": dict(grid=(20, 18, 16), band=(8, 6, 8), nt=3, spectral=(16, 12, 16), dmax=1.0),
}


@pytest.mark.parametrize("name", list(SHAPES))
def test_shapes_against_oracle(name):
    c = SHAPES[name]
    print(f"\n[edge shape {name}]", flush=True)
    p, prob, I0, I1, vstar = setup(c["grid"], c["band"], c["nt"], c.get("spectral"), c["dmax"])
    v0 = 0.5 * vstar
    vs, _, ms = forward(v0, I0, p)
    g_ref, E_ref, cache = gradient(v0, I0, I1, p)
    d = synth.random_direction(91, p.band)
    h_ref = hessvec(cache, d, p, "R1")
    ws = L().Workspace(prob)
    m1, v1 = L().shoot(prob, dev(I0, torch.float32), dev(v0, torch.complex64), ws, want_v1=True)
    g, e3 = L().gradient(prob, dev(I0, torch.float32), dev(I1, torch.float32), dev(v0, torch.complex64), ws)
    h = L().hessvec(prob, dev(d, torch.complex64), ws)
    errs = dict(v1=rel(host(v1), vs[-1]), m1=rel(host(m1), ms[-1]), g=rel(host(g), g_ref), h=rel(host(h), h_ref))
    e3 = host(e3)
    eE = max(abs(e3[i] - E_ref[i]) / max(abs(E_ref[i]), 1e-30) for i in range(3))
    print(f"{name}: {errs} energy {eE:.2e}")
    assert max(errs.values()) < 1e-4 and eE < 1e-5


def test_zero_velocity_is_the_identity():
    p, prob, I0, I1, vstar = setup((24, 20, 18), (8, 8, 6), 4)
    ws = L().Workspace(prob)
    tI0 = dev(I0, torch.float32)
    m1, v1 = L().shoot(prob, tI0, torch.zeros(prob.band_shape, dtype=torch.complex64, device="cuda"), ws,
                       want_v1=True)
    torch.cuda.synchronize()
    assert torch.equal(m1, tI0)
    assert not torch.any(v1)


def test_zero_residual_gives_the_regulariser_gradient():
    p, prob, I0, I1, vstar = setup((24, 20, 18), (8, 8, 6), 4)
    ws = L().Workspace(prob)
    tI0 = dev(I0, torch.float32)
    v0 = dev(0.5 * vstar, torch.complex64)
    m1 = L().shoot(prob, tI0, v0, ws)
    g, e3 = L().gradient(prob, tI0, m1, v0, ws)
    e3 = host(e3)
    print(f"zero residual: E_data {e3[2]:.3e}, |g - v0| {float((g - v0).abs().max()):.3e}")
    assert e3[2] == 0.0
    assert torch.equal(g, v0)


def test_zero_direction_gives_zero():
    p, prob, I0, I1, vstar = setup((24, 20, 18), (8, 8, 6), 4)
    ws = L().Workspace(prob)
    L().gradient(prob, dev(I0, torch.float32), dev(I1, torch.float32), dev(0.5 * vstar, torch.complex64), ws)
    h = L().hessvec(prob, torch.zeros(prob.band_shape, dtype=torch.complex64, device="cuda"), ws)
    torch.cuda.synchronize()
    assert not torch.any(h)


def test_register_classical_matches_oracle():
    p, prob0, I0, I1, vstar = setup((24, 20, 18), (8, 8, 6), 4, dmax=1.5)
    import dataclasses
    prob = dataclasses.replace(prob0, hessian=L().GN_CLASSICAL)
    v_ref, st_ref, status_ref = register(I0, I1, p, 3, 4, mode="R2")
    ws = L().Workspace(prob)
    v, stats, rc, hvps = L().register(prob, dev(I0, torch.float32), dev(I1, torch.float32), ws, gn_iters=3,
                                      pcg_iters=4)
    assert rc == status_ref and len(stats) == len(st_ref)
    for k, (a, b) in enumerate(zip(stats, st_ref)):
        print(f"classical GN {k}: E {a['energy']:.6f}/{b['E']:.6f} pcg {a['pcg_iters']}/{b['pcg_iters']} "
              f"eps {a['step']}/{b['eps']}")
        assert abs(a["energy"] - b["E"]) <= 1e-4 * abs(b["E"])
        assert a["pcg_iters"] == b["pcg_iters"] and a["step"] == b["eps"] and a["trials"] == b["trials"]
    assert rel(host(v), v_ref) < 1e-3
