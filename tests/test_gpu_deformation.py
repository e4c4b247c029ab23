"""Parity of the deformation-state variant (paper §3.3) of the HIP library,
through its C-ABI, with the FP64 oracle on seeded synthetic inputs:
shooting with the band displacement and m(1) = I0 o phi(1), energy,
gradient and the three Hessian-vector products, on shapes with ragged
tiles, the 64^3 / band 16^3 problem and the 128^3 / band 32^3 problem.

Tolerances as for the image state (relative L2 against FP64): final
velocity, m(1), gradient and Hessian-vector product 1e-4, energies 1e-5."""

import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import Params  # noqa: E402
from oracle import deformation as D  # noqa: E402
from paper_1807_11560_amd import synth  # noqa: E402


def L():
    from paper_1807_11560_amd import lddmm
    return lddmm


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128 if t.is_complex() else np.float64)


CASES = {
    "small": dict(grid=(24, 20, 18), band=(8, 8, 6), nt=4, s=2, dmax=1.5, cfg=2),
    "aniso": dict(grid=(40, 36, 32), band=(12, 16, 8), nt=5, s=2, dmax=2.0, cfg=2),
    "one_step": dict(grid=(32, 32, 32), band=(8, 8, 8), nt=1, s=2, dmax=1.5, cfg=2),
    "cfg2": dict(grid=(64, 64, 64), band=(16, 16, 16), nt=10, s=2, dmax=5.0, cfg=2),
    "cfg3": dict(grid=(128, 128, 128), band=(32, 32, 32), nt=10, s=3, dmax=8.0, cfg=3),
    # large bands on the generic kernels (LDS tiles up to the 160 KiB of a workgroup)
    "wide_aniso": dict(grid=(64, 56, 64), band=(48, 40, 56), nt=3, s=2, dmax=3.0, cfg=2),
    "band64": dict(grid=(64, 64, 64), band=(64, 64, 64), nt=2, s=2, dmax=3.0, cfg=2),
}


def make_case(name):
    c = CASES[name]
    w = synth.workload(c["cfg"], grid=c["grid"], band=c["band"])
    p = Params(grid=c["grid"], band=c["band"], nt=c["nt"], alpha=synth.ALPHA, s=c["s"], sigma=synth.SIGMA)
    vstar = synth.scale_to_displacement(w["v_star"], c["grid"], c["dmax"])
    I0 = w["I0"]
    I1 = D.forward(vstar, I0, p)[2]
    prob = L().Problem(grid=c["grid"], band=c["band"], time_steps=c["nt"], alpha=synth.ALPHA, s=c["s"],
                       sigma=synth.SIGMA, state=L().STATE_DEFORMATION)
    return p, prob, I0, I1, vstar


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    print(f"\n[deformation case {request.param}]", flush=True)
    return (request.param,) + make_case(request.param)


def test_shoot(case):
    name, p, prob, I0, I1, vstar = case
    vs, us, m1, _, _ = D.forward(vstar, I0, p)
    ws = L().Workspace(prob)
    gm1, v1 = L().shoot(prob, dev(I0, torch.float32), dev(vstar, torch.complex64), ws, want_v1=True)
    ev, em = rel(host(v1), vs[-1]), rel(host(gm1), m1)
    print(f"{name}: v_nt rel {ev:.2e}  m(1) rel {em:.2e}")
    assert ev < 1e-4 and em < 1e-4


@pytest.fixture(scope="module")
def grad_state(case):
    name, p, prob, I0, I1, vstar = case
    v0 = 0.5 * vstar
    g, E, cache = D.gradient(v0, I0, I1, p)
    ws = L().Workspace(prob)
    args = (dev(I0, torch.float32), dev(I1, torch.float32), dev(v0, torch.complex64))
    gg, e3 = L().gradient(prob, *args, ws)
    return dict(name=name, p=p, prob=prob, g=g, E=E, cache=cache, ws=ws, gg=host(gg), e3=host(e3),
                args=args)


def test_energy_and_gradient(grad_state):
    s = grad_state
    eg = rel(s["gg"], s["g"])
    eE = [abs(s["e3"][i] - s["E"][i]) / max(abs(s["E"][i]), 1e-30) for i in range(3)]
    print(f"{s['name']}: gradient rel {eg:.2e}  energy rel {eE}")
    assert eg < 1e-4
    assert max(eE) < 1e-5


@pytest.mark.parametrize("mode", ["R1", "R2", "FULL"])
def test_hessvec(grad_state, mode):
    s = grad_state
    d = synth.random_direction(77, s["p"].band)
    ref = D.hessvec(s["cache"], d, s["p"], mode)
    if mode == "R1":
        prob, ws = s["prob"], s["ws"]
    else:
        hess = L().GN_CLASSICAL if mode == "R2" else L().NEWTON
        prob = dataclasses.replace(s["prob"], hessian=hess)
        ws = L().Workspace(prob)
        L().gradient(prob, *s["args"], ws)
    out = L().hessvec(prob, dev(d, torch.complex64), ws)
    e = rel(host(out), ref)
    print(f"{s['name']}: hessvec {mode} rel {e:.2e}")
    assert e < 1e-4


def test_hessvec_is_repeatable(grad_state):
    s = grad_state
    d = dev(synth.random_direction(78, s["p"].band), torch.complex64)
    a = host(L().hessvec(s["prob"], d, s["ws"]))
    b = host(L().hessvec(s["prob"], d, s["ws"]))
    assert np.array_equal(a, b)


def test_zero_velocity_keeps_the_source():
    p, prob, I0, I1, vstar = make_case("small")
    ws = L().Workspace(prob)
    m1, v1 = L().shoot(prob, dev(I0, torch.float32), torch.zeros(prob.band_shape, dtype=torch.complex64,
                                                                   device="cuda"), ws, want_v1=True)
    assert np.array_equal(host(m1), I0.astype(np.float32).astype(np.float64))
    assert np.abs(host(v1)).max() == 0.0
