"""Parity with the FP64 oracle at the measured problem size: 128^3 grid,
band 32^3 (padded grid 48^3), s = 3, 10 Euler steps, the tissue phantom and a
random geodesic of 8 voxels.  This runs the kernel instantiations tuned for
that shape, in the launch configuration bench.py times.  The oracle takes
about half a minute per call here, so the whole field is compared once for
shooting, energy, gradient and one Hessian-vector product; the gradient at
v0 = 0 is also checked against its closed form K~ pi(lambda_1 grad I0).
Tolerances as in test_gpu_parity (relative L2 1e-4, energies 1e-5)."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import Params  # noqa: E402
from oracle.band import pi_vec, symbol_K  # noqa: E402
from oracle.jacobi import forward, gradient, hessvec  # noqa: E402
from oracle.transport import grad_h  # noqa: E402
from paper_1807_11560_amd import synth  # noqa: E402


def L():
    from paper_1807_11560_amd import lddmm
    return lddmm


def rel(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128 if t.is_complex() else np.float64)


@pytest.fixture(scope="module")
def problem():
    print("\n[full size 128^3 band 32^3]", flush=True)
    w = synth.workload(3)
    pp = w["params"]
    p = Params(grid=pp["grid"], band=pp["band"], nt=pp["nt"], alpha=pp["alpha"], s=pp["s"], sigma=pp["sigma"])
    prob = L().Problem(grid=pp["grid"], band=pp["band"], time_steps=pp["nt"], alpha=pp["alpha"], s=pp["s"],
                       sigma=pp["sigma"])
    I0, vstar = w["I0"], w["v_star"]
    vs, _, ms = forward(vstar, I0, p)
    return dict(p=p, prob=prob, I0=I0, vstar=vstar, I1=ms[-1], v1=vs[-1])


def test_full_size_shoot(problem):
    s = problem
    ws = L().Workspace(s["prob"])
    m1, v1 = L().shoot(s["prob"], dev(s["I0"], torch.float32), dev(s["vstar"], torch.complex64), ws,
                       want_v1=True)
    ev, em = rel(host(v1), s["v1"]), rel(host(m1), s["I1"])
    print(f"full: v_nt rel {ev:.2e}  m_nt rel {em:.2e}")
    assert ev < 1e-4 and em < 1e-4


def test_full_size_gradient_at_zero_closed_form(problem):
    s = problem
    p = s["p"]
    ws = L().Workspace(s["prob"])
    v0 = np.zeros((3,) + tuple(p.band), dtype=np.complex128)
    g, e3 = L().gradient(s["prob"], dev(s["I0"], torch.float32), dev(s["I1"], torch.float32),
                         dev(v0, torch.complex64), ws)
    lam1 = -(2 / p.sigma ** 2) * (s["I0"] - s["I1"])
    ref = symbol_K(p.band, p.alpha, p.s) * pi_vec(lam1 * grad_h(s["I0"]), p.band)
    e = rel(host(g), ref)
    print(f"full: gradient at zero rel {e:.2e}")
    assert e < 1e-4


def test_full_size_gradient_and_hessvec(problem):
    s = problem
    p = s["p"]
    v0 = 0.5 * s["vstar"]
    g_ref, E_ref, cache = gradient(v0, s["I0"], s["I1"], p)
    d = synth.random_direction(3077, p.band, s=p.s)
    h_ref = hessvec(cache, d, p, "R1")
    ws = L().Workspace(s["prob"])
    g, e3 = L().gradient(s["prob"], dev(s["I0"], torch.float32), dev(s["I1"], torch.float32),
                         dev(v0, torch.complex64), ws)
    h = L().hessvec(s["prob"], dev(d, torch.complex64), ws)
    eg, eh = rel(host(g), g_ref), rel(host(h), h_ref)
    e3 = host(e3)
    eE = max(abs(e3[i] - E_ref[i]) / abs(E_ref[i]) for i in range(3))
    print(f"full: gradient rel {eg:.2e}  hessvec rel {eh:.2e}  energy rel {eE:.2e}")
    assert eg < 1e-4 and eh < 1e-4 and eE < 1e-5
    # the full Newton product on the same gradient state
    import dataclasses
    hf_ref = hessvec(cache, d, p, "FULL")
    probn = dataclasses.replace(s["prob"], hessian=L().NEWTON)
    wsn = L().Workspace(probn)
    L().gradient(probn, dev(s["I0"], torch.float32), dev(s["I1"], torch.float32), dev(v0, torch.complex64), wsn)
    ehf = rel(host(L().hessvec(probn, dev(d, torch.complex64), wsn)), hf_ref)
    print(f"full: full Newton hessvec rel {ehf:.2e}")
    assert ehf < 1e-4
