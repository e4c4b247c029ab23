"""Parity of the HIP library (through its C-ABI) with the FP64 oracle on
seeded synthetic inputs: shooting, transport, energy, gradient and both
Gauss-Newton Hessian-vector products and the full Newton one, at sizes whose padded-grid and grid
tiles have ragged tails, on the 64^3 / band 16^3 problem and on the
128^3 / band 32^3 problem used for measurement.

Tolerances (relative L2 against FP64): one Euler step of the band EPDiff
1e-5; final velocity, warped image, gradient and Hessian-vector product
1e-4.  The library computes in FP32 with FP64 reductions."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import Params  # noqa: E402
from oracle.jacobi import forward, gradient, hessvec  # noqa: E402
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
    # the smallest problem the library takes: grid 8^3, band 4^3 (effective
    # band |k| <= 1), padded grid 6^3
    "tiny": dict(grid=(8, 8, 8), band=(4, 4, 4), nt=2, s=2, dmax=1.0, cfg=2),
    # anisotropic, odd padded axis (M2 = 9), ragged grid rows
    "small": dict(grid=(24, 20, 18), band=(8, 8, 6), nt=4, s=2, dmax=1.5, cfg=2),
    # ragged padded-grid rows (M1 = 18 with 21-row tiles -> one tile; M = 24 with 10-row tiles)
    "aniso": dict(grid=(40, 36, 32), band=(12, 16, 8), nt=5, s=2, dmax=2.0, cfg=2),
    # the 64^3, band 16^3 problem
    "cfg2": dict(grid=(64, 64, 64), band=(16, 16, 16), nt=10, s=2, dmax=5.0, cfg=2),
    # band 24^3 on the tuned 36^3 padded-grid kernels (odd depth halves in the column step)
    "band24": dict(grid=(48, 48, 48), band=(24, 24, 24), nt=3, s=2, dmax=3.0, cfg=2),
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
    I1 = forward(vstar, I0, p)[2][-1]
    prob = L().Problem(grid=c["grid"], band=c["band"], time_steps=c["nt"], alpha=synth.ALPHA, s=c["s"],
                       sigma=synth.SIGMA)
    return p, prob, I0, I1, vstar


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    print(f"\n[case {request.param}]", flush=True)
    return (request.param,) + make_case(request.param)


def test_one_euler_step(case):
    name, p, prob, I0, I1, vstar = case
    import dataclasses
    p1 = dataclasses.replace(p, nt=1)
    prob1 = dataclasses.replace(prob, time_steps=1)
    vs = forward(vstar, I0, p1)[0]
    ws = L().Workspace(prob1)
    m1, v1 = L().shoot(prob1, dev(I0, torch.float32), dev(vstar, torch.complex64), ws, want_v1=True)
    e = rel(host(v1), vs[1])
    print(f"{name}: one Euler step rel err {e:.2e}")
    assert e < 1e-5


def test_shoot_and_transport(case):
    name, p, prob, I0, I1, vstar = case
    vs, _, ms = forward(vstar, I0, p)
    ws = L().Workspace(prob)
    m1, v1 = L().shoot(prob, dev(I0, torch.float32), dev(vstar, torch.complex64), ws, want_v1=True)
    ev, em = rel(host(v1), vs[-1]), rel(host(m1), ms[-1])
    print(f"{name}: v_nt rel {ev:.2e}  m_nt rel {em:.2e}")
    assert ev < 1e-4 and em < 1e-4


@pytest.fixture(scope="module")
def grad_state(case):
    name, p, prob, I0, I1, vstar = case
    v0 = 0.5 * vstar
    g, E, cache = gradient(v0, I0, I1, p)
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
    import dataclasses
    s = grad_state
    d = synth.random_direction(77, s["p"].band)
    ref = hessvec(s["cache"], d, s["p"], mode)
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


def test_hessvec_before_gradient_is_rejected():
    prob = L().Problem(grid=(32, 32, 32), band=(8, 8, 8))
    ws = L().Workspace(prob)
    d = torch.zeros(prob.band_shape, dtype=torch.complex64, device="cuda")
    with pytest.raises(L().LddmmError) as e:
        L().hessvec(prob, d, ws)
    assert e.value.code == L().E_NOT_PREPARED
