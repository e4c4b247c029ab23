"""The torch.autograd form of the energy (paper_1807_11560_amd.autograd):
forward lddmm_energy, backward the exact derivative of the discrete energy
(lddmm_gradient_exact) turned into the l2 gradient L~ g_V.

  * the backward equals the FP64 oracle's exact l2 gradient (1e-4) and obeys
    the chain rule;
  * <grad, d> equals FP64 central differences of the discrete energy (the
    oracle's, step 1e-7 |v0| / |d|) on 16 random directions to 1e-3;
  * the 160x192x160 / band 32^3 / 20-step volume at a random v0 of 5 voxels
    (not 0: there every departure point sits on a node, where the
    interpolant's slope is one-sided) with the state checkpointed every 5
    steps: the backward against the oracle's exact gradient (1e-3; that
    gradient is itself pinned by FP64 differences to 1e-6), the workspace
    and peak memory against the unchecked layout, and central differences of
    the library's own FP32 energy with step h = 1e-4 |v0| / |d| on 16
    directions, reported.

The differences of the FP32 energy are not held to 1e-3: a trilinear
transport has a slope jump wherever a departure point crosses a cell face,
and with this step about 3e-3 of the departure points of the 20 steps cross
one, which moves the difference by 1e-3 to 1e-2 of its value (the FP64
oracle's differences at step 1e-7 cross none); at smaller steps the FP32
rounding of the energy takes over.  They are held to 5e-2 of the largest
directional derivative, which catches a wrong sign, factor or missing term.
Errors are measured against the largest |<grad, d>| of the directions, since
a random direction can be nearly orthogonal to the gradient."""

import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import Params  # noqa: E402
from oracle import exact  # noqa: E402
from oracle.band import symbol_L  # noqa: E402
from oracle.jacobi import forward  # noqa: E402
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


def directional(grad, d):
    return float(torch.sum(grad.real * d.real + grad.imag * d.imag))


def fd_gaps(prob, ws, v0, grad, tI0, tI1, seeds, rel_step):
    """|<grad, d> - central difference| / max_d |central difference|, FP32
    energies of the library."""
    an, fd = [], []
    for seed in seeds:
        dn = synth.random_direction(seed, prob.band)
        d = torch.from_numpy(dn).to(torch.complex64).cuda()
        h = rel_step * float(torch.linalg.vector_norm(v0)) / float(torch.linalg.vector_norm(d))
        with torch.no_grad():
            ep = float(A().energy(prob, v0.detach() + h * d, tI0, tI1, ws))
            em = float(A().energy(prob, v0.detach() - h * d, tI0, tI1, ws))
        fd.append((ep - em) / (2 * h))
        an.append(directional(grad, d))
    an, fd = np.array(an), np.array(fd)
    return np.abs(an - fd) / np.abs(fd).max()


def test_backward_is_the_exact_l2_gradient():
    p, prob, I0, I1, vstar = setup((40, 36, 32), (12, 16, 8), 5, 2, 2.0, 2)
    v0n = 0.5 * vstar
    g, E, _ = exact.gradient(v0n, I0, I1, p)
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
    print(f"autograd exact l2 gradient rel {eg:.2e}, energy rel {eE:.2e}")
    assert eg < 1e-4 and eE < 1e-5
    v0.grad = None
    (3.0 * A().energy(prob, v0, tI0, tI1, ws)).backward()
    assert rel(v0.grad.detach().cpu().numpy(), 3.0 * ref) < 1e-4


def test_gradient_against_fp64_central_differences():
    from oracle.jacobi import energy as oracle_energy
    p, prob, I0, I1, vstar = setup((40, 36, 32), (12, 16, 8), 5, 2, 2.0, 2)
    ws = L().Workspace(prob)
    tI0 = torch.from_numpy(I0).float().cuda()
    tI1 = torch.from_numpy(I1).float().cuda()
    v0n = 0.5 * vstar
    v0 = torch.from_numpy(v0n).to(torch.complex64).cuda().requires_grad_(True)
    A().energy(prob, v0, tI0, tI1, ws).backward()
    grad = v0.grad.detach()

    def E(v):
        return oracle_energy(v, forward(v, I0, p)[2][-1], I1, p)[0]

    an, fd = [], []
    for seed in range(300, 316):
        dn = synth.random_direction(seed, prob.band)
        h = 1e-7 * np.linalg.norm(v0n) / np.linalg.norm(dn)
        fd.append((E(v0n + h * dn) - E(v0n - h * dn)) / (2 * h))
        an.append(directional(grad, torch.from_numpy(dn).to(torch.complex64).cuda()))
    an, fd = np.array(an), np.array(fd)
    gaps = np.abs(an - fd) / np.abs(fd).max()
    print("gaps to FP64 central differences", ["%.1e" % x for x in gaps])
    assert gaps.max() < 1e-3
    fp32 = fd_gaps(prob, ws, v0, grad, tI0, tI1, range(300, 308), 1e-4)
    print("gaps to the library's FP32 differences (step 1e-4)", ["%.1e" % x for x in fp32])


def test_large_volume_checkpointed_against_oracle_and_differences():
    p, prob, I0, I1, vstar = setup((160, 192, 160), (32, 32, 32), 20, 3, 5.0, 4)
    v0n = 0.6 * vstar
    probc = dataclasses.replace(prob, checkpoint=5)
    plain_bytes = prob.workspace_bytes()
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    ws = L().Workspace(probc)
    print(f"workspace {ws.nbytes / 2**30:.3f} GiB with checkpoints every 5 steps, "
          f"{plain_bytes / 2**30:.3f} GiB without", flush=True)
    assert ws.nbytes < 0.5 * plain_bytes
    tI0 = torch.from_numpy(I0).float().cuda()
    tI1 = torch.from_numpy(I1).float().cuda()
    v0 = torch.from_numpy(v0n).to(torch.complex64).cuda().requires_grad_(True)
    e = A().energy(probc, v0, tI0, tI1, ws)
    e.backward()
    torch.cuda.synchronize()
    print(f"peak device memory of energy + backward: {torch.cuda.max_memory_allocated() / 2**30:.3f} GiB",
          flush=True)
    grad = v0.grad.detach()
    gaps = fd_gaps(probc, ws, v0, grad, tI0, tI1, range(400, 416), 1e-4)
    print("step 1e-4: gaps to the library's FP32 differences", ["%.1e" % x for x in gaps], flush=True)
    g, E, _ = exact.gradient(v0n, I0, I1, p)
    ref = symbol_L(p.band, p.alpha, p.s) * g
    eg = rel(grad.cpu().numpy().astype(np.complex128), ref)
    print(f"160x192x160: exact l2 gradient rel {eg:.2e}, energy rel {abs(float(e) - E[0]) / E[0]:.2e}")
    assert eg < 1e-3
    assert gaps.max() < 5e-2
