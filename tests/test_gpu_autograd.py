"""The torch.autograd form of the energy (paper_1807_11560_amd.autograd):
its backward is L~ g_V of lddmm_gradient, equals the FP64 oracle's l2
gradient (1e-4), agrees with central differences of the library's own energy
as the oracle's gradient does with the oracle's energy (the method gap of the
adjoint Jacobi gradient), and runs on the 160x192x160 / band 32^3 / 20-step
volume against the oracle."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import Params  # noqa: E402
from oracle.band import symbol_L  # noqa: E402
from oracle.jacobi import forward, gradient  # noqa: E402
from paper_1807_11560_amd import synth  # noqa: E402


def L():
    from paper_1807_11560_amd import lddmm
    return lddmm


def A():
    from paper_1807_11560_amd import autograd
    return autograd


def rel(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def setup(grid, band, nt, s, dmax, cfg):
    w = synth.workload(cfg, grid=grid, band=band)
    p = Params(grid=grid, band=band, nt=nt, alpha=synth.ALPHA, s=s, sigma=synth.SIGMA)
    vstar = synth.scale_to_displacement(w["v_star"], grid, dmax)
    I0 = w["I0"]
    I1 = forward(vstar, I0, p)[2][-1]
    prob = L().Problem(grid=grid, band=band, time_steps=nt, alpha=synth.ALPHA, s=s, sigma=synth.SIGMA)
    return p, prob, I0, I1, vstar


def test_backward_is_the_l2_gradient():
    p, prob, I0, I1, vstar = setup((40, 36, 32), (12, 16, 8), 5, 2, 2.0, 2)
    v0n = 0.5 * vstar
    g, E, _ = gradient(v0n, I0, I1, p)
    ref = symbol_L(p.band, p.alpha, p.s) * g
    ws = L().Workspace(prob)
    tI0 = torch.from_numpy(I0).float().cuda()
    tI1 = torch.from_numpy(I1).float().cuda()
    v0 = torch.from_numpy(v0n).to(torch.complex64).cuda().requires_grad_(True)
    e = A().energy(prob, v0, tI0, tI1, ws)
    e.backward()
    torch.cuda.synchronize()
    got = v0.grad.detach().cpu().numpy().astype(np.complex128)
    eg, eE = rel(got, ref), abs(float(e.detach()) - E[0]) / E[0]
    print(f"autograd l2 gradient rel {eg:.2e}, energy rel {eE:.2e}")
    assert eg < 1e-4 and eE < 1e-5
    # the chain rule through a scalar factor
    v0.grad = None
    (3.0 * A().energy(prob, v0, tI0, tI1, ws)).backward()
    assert rel(v0.grad.detach().cpu().numpy(), 3.0 * ref) < 1e-4


def test_gradient_against_central_differences():
    """<grad, d> against (E(v0 + h d) - E(v0 - h d)) / 2h of the library's own
    energy for 8 random directions.  The library's differences equal the FP64
    oracle's (FP32 noise of E aside).  At v0 = 0 the adjoint Jacobi gradient is
    the derivative up to a few percent (this checks the autograd convention:
    sign, factor, real and imaginary parts).  Away from 0 it is the paper's
    method, not the exact derivative: the band truncation of the coadjoint
    transport leaves a gap of tens of percent that does not shrink with nt,
    which is reported, as the oracle's tests do."""
    from oracle.band import inner
    from oracle.jacobi import energy as oracle_energy
    p, prob, I0, I1, vstar = setup((40, 36, 32), (12, 16, 8), 5, 2, 2.0, 2)
    ws = L().Workspace(prob)
    tI0 = torch.from_numpy(I0).float().cuda()
    tI1 = torch.from_numpy(I1).float().cuda()
    h = 2e-4  # a fraction of a voxel along iota(d), well above the FP32 noise of E
    for fac in (0.0, 0.5):
        v0n = fac * vstar
        v0 = torch.from_numpy(v0n).to(torch.complex64).cuda().requires_grad_(True)
        A().energy(prob, v0, tI0, tI1, ws).backward()
        grad = v0.grad.detach()
        an_all, fd_all, fdo_all = [], [], []
        for seed in range(8):
            dn = synth.random_direction(300 + seed, prob.band)
            d = torch.from_numpy(dn).to(torch.complex64).cuda()
            with torch.no_grad():
                ep = float(A().energy(prob, v0.detach() + h * d, tI0, tI1, ws))
                em = float(A().energy(prob, v0.detach() - h * d, tI0, tI1, ws))
            fd_all.append((ep - em) / (2 * h))
            an_all.append(float(torch.sum(grad.real * d.real + grad.imag * d.imag)))
            fdo_all.append((oracle_energy(v0n + h * dn, forward(v0n + h * dn, I0, p)[2][-1], I1, p)[0]
                            - oracle_energy(v0n - h * dn, forward(v0n - h * dn, I0, p)[2][-1], I1, p)[0]) / (2 * h))
        an, fd, fdo = np.array(an_all), np.array(fd_all), np.array(fdo_all)
        gaps = np.abs(an - fd) / np.abs(fd)
        print(f"v0 = {fac} v*: gap to central differences", ["%.3f" % x for x in gaps],
              "library - oracle difference", "%.2e" % (np.abs(fd - fdo).max() / np.abs(fdo).max()))
        assert np.abs(fd - fdo).max() < 1e-2 * np.abs(fdo).max()
        if fac == 0.0:
            assert np.median(gaps) < 0.05


def test_large_volume_gradient_matches_oracle():
    """160x192x160, band 32^3, 20 time steps (the autograd workload): the whole
    trajectory stays resident; the backward equals the oracle's l2 gradient."""
    p, prob, I0, I1, vstar = setup((160, 192, 160), (32, 32, 32), 20, 3, 5.0, 4)
    v0n = 0.5 * vstar
    g, E, _ = gradient(v0n, I0, I1, p)
    ref = symbol_L(p.band, p.alpha, p.s) * g
    ws = L().Workspace(prob)
    print(f"workspace {ws.nbytes / 2**30:.2f} GiB")
    v0 = torch.from_numpy(v0n).to(torch.complex64).cuda().requires_grad_(True)
    e = A().energy(prob, v0, torch.from_numpy(I0).float().cuda(), torch.from_numpy(I1).float().cuda(), ws)
    e.backward()
    torch.cuda.synchronize()
    eg = rel(v0.grad.detach().cpu().numpy().astype(np.complex128), ref)
    print(f"160x192x160: l2 gradient rel {eg:.2e}, energy rel {abs(float(e) - E[0]) / E[0]:.2e}")
    assert eg < 1e-4
