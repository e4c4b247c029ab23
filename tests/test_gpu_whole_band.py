"""Parity with the FP64 oracle that sees the whole band (paper §3.1: the
truncated Fourier domain, iota/pi and the truncated convolution; §3.2: the
shooting, gradient and Hessian-vector product built on them).

The other parity tests feed smooth inputs (coefficients damped by the
inverse symbol of L), whose outer band carries a fraction of a per cent of
the norm, and compare one relative-L2 number.  Here the inputs are white
(undamped: every coefficient of the effective band drawn with the same
variance), every output is compared shell by shell (|k|_inf = r) with the
largest error of the shell bounded by the shell's largest reference value,
every output is checked to be exactly Hermitian with the k = -K/2 slots
exactly zero, and every Euler step of a shooting is checked, not only the
first: one step of size dt from v_n equals 1/dt times one step of size 1
from dt v_n (the right-hand side is quadratic in v), so a one-step call
on dt v_n gives step n of the trajectory.

Tolerances: relative L2 1e-5 per Euler step and 1e-4 for shooting, gradient
and Hessian-vector product, as elsewhere; per shell 1e-3 of the shell's
largest reference value.  The Hessian-vector product in a white direction
dv is the exception at the large bands: L~ dv then spans the whole range of
the symbol over the band, L^(k) from 1 to (1 + alpha |2 pi k|^2)^s at the
band's corner (8e4 at band 64, s = 2; 4e6 at band 48, s = 3), and the
pseudo-spectral products spread the FP32 rounding of its largest values over
every frequency.  The measured error follows that range (at band 64 it is
2e-4 with s = 2 and 3e-6 with s = 1 for the same direction, and 3e-7 for a
smooth direction), so those two cases carry their own bounds (5e-4 and 5e-3
in relative L2, ten times that per shell)."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import Params  # noqa: E402
from oracle.epdiff import shoot as oracle_shoot  # noqa: E402
from oracle.jacobi import forward, gradient, hessvec  # noqa: E402
from paper_1807_11560_amd import synth  # noqa: E402

SHELL_TOL = 1e-3


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


def freqs(K):
    q = np.arange(K)
    return np.where(q < K // 2, q, q - K)


def shell_of(band):
    r = np.zeros(tuple(band), dtype=int)
    for j, K in enumerate(band):
        shape = [1] * len(band)
        shape[j] = K
        r = np.maximum(r, np.abs(freqs(K)).reshape(shape))
    return r


def shell_errors(out, ref, band):
    """max |out - ref| / max |ref| over each shell |k|_inf = r of the
    effective band (r = 0 .. max_j K_j/2 - 1).  A shell whose reference is
    below 1e-2 of the field's largest value is measured against that floor
    instead: the k = 0 shell of a shooting is zero in exact arithmetic (the
    band EPDiff conserves the zero mean), and in FP32 holds the rounding of
    sums over the whole band that cancel there."""
    r = shell_of(band)
    eff = np.ones(tuple(band), dtype=bool)
    for j, K in enumerate(band):
        shape = [1] * len(band)
        shape[j] = K
        eff &= (np.abs(freqs(K)) <= K // 2 - 1).reshape(shape)
    errs = []
    floor = 1e-2 * np.abs(ref).max()
    for s in range(int(r[eff].max()) + 1):
        m = eff & (r == s)
        if not m.any():
            continue
        d = np.abs(out[:, m] - ref[:, m]).max()
        errs.append(float(d / max(np.abs(ref[:, m]).max(), floor)))
    return errs


def assert_exact_band_form(out, band):
    """Bitwise Hermitian, and zero in every k = -K/2 slot."""
    rev = np.ix_(range(out.shape[0]), *[(-np.arange(K)) % K for K in band])
    assert np.array_equal(out, np.conj(out[rev])), "output is not exactly Hermitian"
    for j, K in enumerate(band):
        assert not np.take(out, K // 2, axis=1 + j).any(), f"slot -K/2 of axis {j} is not zero"


def white(seed, p, inc):
    """Undamped Hermitian band field (k = 0 zeroed), scaled so that the first
    Euler step changes it by the fraction `inc` (relative L2).  A white field
    of a few voxels' displacement grows without bound under explicit steps at
    the larger bands; the right-hand side is quadratic, so the change of one
    step is proportional to the scale, which one oracle step of size 1 fixes."""
    import dataclasses
    v = synth.random_band_field(np.random.default_rng(seed), p.band, s=0)
    one = oracle_shoot(v, dataclasses.replace(p, nt=1))[1]
    ratio = np.linalg.norm(one - v) / np.linalg.norm(v)  # ||F(v)|| / ||v||
    return v * (inc / (p.dt * ratio))


def white_direction(seed, band):
    v = synth.random_band_field(np.random.default_rng(seed), band, s=0, zero_mean=False)
    return v / np.sqrt(np.real(np.vdot(v, v)))


CASES = {
    "small": dict(grid=(24, 20, 18), band=(8, 8, 6), nt=4, s=2, dmax=1.5, cfg=2),
    "aniso": dict(grid=(40, 36, 32), band=(12, 16, 8), nt=5, s=2, dmax=2.0, cfg=2),
    "cfg2": dict(grid=(64, 64, 64), band=(16, 16, 16), nt=10, s=2, dmax=5.0, cfg=2),
    "band24": dict(grid=(48, 48, 48), band=(24, 24, 24), nt=3, s=2, dmax=3.0, cfg=2),
    "band64": dict(grid=(64, 64, 64), band=(64, 64, 64), nt=2, s=2, dmax=3.0, cfg=2, hvp_tol=5e-4),
    # band 32 on the shape-generic kernels (padded grid 50 instead of the tuned 48)
    "band32_generic": dict(grid=(64, 64, 64), band=(32, 32, 32), spectral=(50, 50, 50), nt=4, s=2, dmax=3.0, cfg=2),
    # the band-sweep shape of band 48 on the measured grid (generic kernels)
    "band48_128": dict(grid=(128, 128, 128), band=(48, 48, 48), nt=5, s=3, dmax=8.0, cfg=3, hvp_tol=5e-3),
    "full": dict(grid=(128, 128, 128), band=(32, 32, 32), nt=10, s=3, dmax=8.0, cfg=3),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    name = request.param
    c = CASES[name]
    print(f"\n[whole-band case {name}]", flush=True)
    w = synth.workload(c["cfg"], grid=c["grid"], band=c["band"])
    spec = c.get("spectral")
    p = Params(grid=c["grid"], band=c["band"], nt=c["nt"], alpha=synth.ALPHA, s=c["s"], sigma=synth.SIGMA,
               spectral=spec)
    vstar = synth.scale_to_displacement(w["v_star"], c["grid"], c["dmax"])
    I0 = w["I0"]
    I1 = forward(vstar, I0, p)[2][-1]
    prob = L().Problem(grid=c["grid"], band=c["band"], time_steps=c["nt"], alpha=synth.ALPHA, s=c["s"],
                       sigma=synth.SIGMA, spectral=spec or (0, 0, 0))
    return dict(name=name, c=c, p=p, prob=prob, I0=I0, I1=I1, vstar=vstar)


def test_every_euler_step_of_a_white_velocity(case):
    import dataclasses
    c, p = case["c"], case["p"]
    v0 = white(31, p, 0.1)
    vs = oracle_shoot(v0, p)
    dt = 1.0 / c["nt"]
    prob1 = dataclasses.replace(case["prob"], time_steps=1)
    ws = L().Workspace(prob1)
    I0 = dev(case["I0"], torch.float32)
    worst, worst_inc, worst_shell, at = 0.0, 0.0, 0.0, None
    for n in range(c["nt"]):
        _, out = L().shoot(prob1, I0, dev(dt * vs[n], torch.complex64), ws, want_v1=True)
        o = raw(out)
        assert_exact_band_form(o, c["band"])
        step = o.astype(np.complex128) / dt
        e = rel(step, vs[n + 1])
        inc = rel(step - vs[n], vs[n + 1] - vs[n])
        she = shell_errors(step, vs[n + 1], c["band"])
        if max(she) > worst_shell:
            worst_shell, at = max(she), (n, int(np.argmax(she)))
        worst, worst_inc = max(worst, e), max(worst_inc, inc)
    print(f"{case['name']}: worst step rel {worst:.2e}, increment rel {worst_inc:.2e}, "
          f"shell {worst_shell:.2e} (step, shell) {at}")
    assert worst < 1e-5
    assert worst_inc < 1e-3
    assert worst_shell < SHELL_TOL


def test_shoot_of_a_white_velocity(case):
    c, p = case["c"], case["p"]
    v0 = white(32, p, 0.1)
    vs, _, ms = forward(v0, case["I0"], p)
    ws = L().Workspace(case["prob"])
    m1, v1 = L().shoot(case["prob"], dev(case["I0"], torch.float32), dev(v0, torch.complex64), ws, want_v1=True)
    o = raw(v1)
    assert_exact_band_form(o, c["band"])
    ev, em = rel(o.astype(np.complex128), vs[-1]), rel(raw(m1).astype(np.float64), ms[-1])
    sh = shell_errors(o.astype(np.complex128), vs[-1], c["band"])
    print(f"{case['name']}: white v_nt rel {ev:.2e} m_nt rel {em:.2e} shells max {max(sh):.2e} "
          f"at shell {int(np.argmax(sh))}")
    assert ev < 1e-4 and em < 1e-4
    assert max(sh) < SHELL_TOL


@pytest.fixture(scope="module")
def white_grad(case):
    p = case["p"]
    v0 = white(33, p, 0.05)
    g, E, cache = gradient(v0, case["I0"], case["I1"], p)
    ws = L().Workspace(case["prob"])
    gg, e3 = L().gradient(case["prob"], dev(case["I0"], torch.float32), dev(case["I1"], torch.float32),
                          dev(v0, torch.complex64), ws)
    return dict(g=g, E=E, cache=cache, ws=ws, gg=raw(gg), e3=raw(e3), v0=v0)


def test_gradient_at_a_white_velocity(case, white_grad):
    s = white_grad
    band = case["c"]["band"]
    assert_exact_band_form(s["gg"], band)
    out = s["gg"].astype(np.complex128)
    e = rel(out, s["g"])
    sh = shell_errors(out, s["g"], band)
    eE = max(abs(s["e3"][i] - s["E"][i]) / abs(s["E"][i]) for i in range(3))
    print(f"{case['name']}: white gradient rel {e:.2e} shells max {max(sh):.2e} energy {eE:.1e}")
    assert e < 1e-4 and eE < 1e-5
    assert max(sh) < SHELL_TOL


@pytest.mark.parametrize("mode", ["R1", "FULL"])
def test_hessvec_in_a_white_direction(case, white_grad, mode):
    import dataclasses
    band = case["c"]["band"]
    d = white_direction(34, band)
    ref = hessvec(white_grad["cache"], d, case["p"], mode)
    if mode == "R1":
        prob, ws = case["prob"], white_grad["ws"]
    else:
        prob = dataclasses.replace(case["prob"], hessian=L().NEWTON)
        ws = L().Workspace(prob)
        L().gradient(prob, dev(case["I0"], torch.float32), dev(case["I1"], torch.float32),
                     dev(white_grad["v0"], torch.complex64), ws)
    o = raw(L().hessvec(prob, dev(d, torch.complex64), ws))
    assert_exact_band_form(o, band)
    out = o.astype(np.complex128)
    e = rel(out, ref)
    sh = shell_errors(out, ref, band)
    # the increment dw_0 alone, whose outer shells the identity term would hide
    ew = rel(out - d, ref - d)
    shw = shell_errors(out - d, ref - d, band)
    print(f"{case['name']}: white hessvec {mode} rel {e:.2e} shells max {max(sh):.2e}; "
          f"dw0 rel {ew:.2e} shells {' '.join(f'{x:.1e}' for x in shw)}")
    tol = case["c"].get("hvp_tol", 1e-4)
    assert e < tol and ew < tol
    assert max(sh) < 10 * tol and max(shw) < 10 * tol
