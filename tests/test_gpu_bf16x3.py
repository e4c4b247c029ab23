"""Parity of the compensated-BF16 mode (LDDMM_FP32_BF16X3: every partial-DFT
contraction on the matrix cores as hi/lo BF16 products, paper §3.1 transforms
and truncated convolution) with the FP64 oracle, stated separately from the
FP32 mode: every Euler step of a shooting, the final velocity and warped
image, the gradient, the Hessian-vector product, and the Gauss-Newton loop
iteration by iteration.

Tolerances are those the FP32 mode is held to (relative L2 1e-5 per Euler
step, 1e-4 for the final velocity, warped image, gradient and product,
energies 1e-5): one split product carries a relative error of about 2^-16
instead of 2^-24, and a contraction of depth K about sqrt(K) 2^-16 ~ 1e-4
in the worst case, averaging down over the stages.  Outputs must be exactly
Hermitian, and must differ from the FP32 mode's (the mode is in effect)."""

import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import Params  # noqa: E402
from oracle.epdiff import shoot as oracle_shoot  # noqa: E402
from oracle.gn import register as oracle_register  # noqa: E402
from oracle.jacobi import forward, gradient, hessvec  # noqa: E402
from paper_1807_11560_amd import synth  # noqa: E402


def L():
    from paper_1807_11560_amd import lddmm
    return lddmm


def rel(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()


def raw(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def hermitian_exact(o, band):
    rev = np.ix_(range(o.shape[0]), *[(-np.arange(K)) % K for K in band])
    return np.array_equal(o, np.conj(o[rev]))


CASES = {
    "small": dict(grid=(24, 20, 18), band=(8, 8, 6), nt=4, s=2, dmax=1.5, cfg=2),
    "cfg2": dict(grid=(64, 64, 64), band=(16, 16, 16), nt=10, s=2, dmax=5.0, cfg=2),
    "band24": dict(grid=(48, 48, 48), band=(24, 24, 24), nt=3, s=2, dmax=3.0, cfg=2),
    "full": dict(grid=(128, 128, 128), band=(32, 32, 32), nt=10, s=3, dmax=8.0, cfg=3),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    name = request.param
    c = CASES[name]
    print(f"\n[bf16x3 case {name}]", flush=True)
    w = synth.workload(c["cfg"], grid=c["grid"], band=c["band"])
    p = Params(grid=c["grid"], band=c["band"], nt=c["nt"], alpha=synth.ALPHA, s=c["s"], sigma=synth.SIGMA)
    vstar = synth.scale_to_displacement(w["v_star"], c["grid"], c["dmax"])
    I0 = w["I0"]
    vs, _, ms = forward(vstar, I0, p)
    probs = {prec: L().Problem(grid=c["grid"], band=c["band"], time_steps=c["nt"], alpha=synth.ALPHA, s=c["s"],
                               sigma=synth.SIGMA, precision=prec) for prec in (L().FP32, L().FP32_BF16X3)}
    return dict(name=name, c=c, p=p, I0=I0, I1=ms[-1], vstar=vstar, vs=vs, ms=ms, probs=probs)


def test_every_euler_step(case):
    c, vs = case["c"], case["vs"]
    dt = 1.0 / c["nt"]
    prob1 = dataclasses.replace(case["probs"][L().FP32_BF16X3], time_steps=1)
    ws = L().Workspace(prob1)
    I0 = dev(case["I0"], torch.float32)
    errs = []
    for n in range(c["nt"]):
        _, out = L().shoot(prob1, I0, dev(dt * vs[n], torch.complex64), ws, want_v1=True)
        o = raw(out)
        assert hermitian_exact(o, c["band"])
        errs.append(rel(o.astype(np.complex128) / dt, vs[n + 1]))
    print(f"{case['name']} bf16x3: worst Euler step rel {max(errs):.2e}")
    assert max(errs) < 1e-5


def test_shoot(case):
    c = case["c"]
    out = {}
    for prec, prob in case["probs"].items():
        ws = L().Workspace(prob)
        m1, v1 = L().shoot(prob, dev(case["I0"], torch.float32), dev(case["vstar"], torch.complex64), ws,
                           want_v1=True)
        out[prec] = (raw(m1), raw(v1))
    m1, v1 = out[L().FP32_BF16X3]
    assert hermitian_exact(v1, c["band"])
    assert not np.array_equal(v1, out[L().FP32][1])  # the mode is in effect
    ev, em = rel(v1.astype(np.complex128), case["vs"][-1]), rel(m1.astype(np.float64), case["ms"][-1])
    ev32 = rel(out[L().FP32][1].astype(np.complex128), case["vs"][-1])
    print(f"{case['name']} bf16x3: v_nt rel {ev:.2e} (fp32 {ev32:.2e}), m_nt rel {em:.2e}")
    assert ev < 1e-4 and em < 1e-4


def test_gradient_and_hessvec(case):
    c, p = case["c"], case["p"]
    v0 = 0.5 * case["vstar"]
    g, E, cache = gradient(v0, case["I0"], case["I1"], p)
    d = synth.random_direction(77, c["band"], s=c["s"])
    ref = {mode: hessvec(cache, d, p, mode) for mode in ("R1", "R2")}
    prob = case["probs"][L().FP32_BF16X3]
    ws = L().Workspace(prob)
    args = (dev(case["I0"], torch.float32), dev(case["I1"], torch.float32), dev(v0, torch.complex64))
    gg, e3 = L().gradient(prob, *args, ws)
    gg, e3 = raw(gg), raw(e3)
    assert hermitian_exact(gg, c["band"])
    eg = rel(gg.astype(np.complex128), g)
    eE = max(abs(e3[i] - E[i]) / abs(E[i]) for i in range(3))
    h = raw(L().hessvec(prob, dev(d, torch.complex64), ws))
    assert hermitian_exact(h, c["band"])
    eh = rel(h.astype(np.complex128), ref["R1"])
    prob2 = dataclasses.replace(prob, hessian=L().GN_CLASSICAL)
    ws2 = L().Workspace(prob2)
    L().gradient(prob2, *args, ws2)
    eh2 = rel(raw(L().hessvec(prob2, dev(d, torch.complex64), ws2)).astype(np.complex128), ref["R2"])
    print(f"{case['name']} bf16x3: gradient rel {eg:.2e}, energy rel {eE:.1e}, hessvec R1 rel {eh:.2e}, "
          f"R2 rel {eh2:.2e}")
    assert eg < 1e-4 and eE < 1e-5 and eh < 1e-4 and eh2 < 1e-4


def test_registration_loop_bf16x3():
    """The Gauss-Newton loop (paper §2.7) in the compensated mode against the
    oracle's, iteration by iteration (decisions exact, energies 1e-4)."""
    print("\n[bf16x3 register]", flush=True)
    grid, band, nt = (24, 20, 18), (8, 8, 6), 4
    w = synth.workload(2, grid=grid, band=band)
    p = Params(grid=grid, band=band, nt=nt, alpha=synth.ALPHA, s=2, sigma=synth.SIGMA)
    vstar = synth.scale_to_displacement(w["v_star"], grid, 1.5)
    I0 = w["I0"]
    I1 = forward(vstar, I0, p)[2][-1]
    v_ref, st_ref, status_ref = oracle_register(I0, I1, p, 3, 4)
    prob = L().Problem(grid=grid, band=band, time_steps=nt, alpha=synth.ALPHA, s=2, sigma=synth.SIGMA,
                       precision=L().FP32_BF16X3)
    ws = L().Workspace(prob)
    v, st, rc, hv = L().register(prob, dev(I0, torch.float32), dev(I1, torch.float32), ws, gn_iters=3, pcg_iters=4)
    assert rc == status_ref and len(st) == len(st_ref)
    for a, b in zip(st, st_ref):
        assert a["pcg_iters"] == b["pcg_iters"] and bool(a["pcg_guard"]) == bool(b["pcg_guard"])
        assert a["trials"] == b["trials"] and a["step"] == b["eps"]
        assert abs(a["energy"] - b["E"]) <= 1e-4 * abs(b["E"])
        assert abs(a["mse_rel"] - b["mse_rel"]) <= 1e-4 * max(abs(b["mse_rel"]), 1e-12)
    ev = rel(raw(v).astype(np.complex128), v_ref)
    print(f"bf16x3 register: final v0 rel {ev:.2e}")
    assert ev < 1e-3
