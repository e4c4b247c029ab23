"""The exact derivative of the discrete energy on the GPU
(lddmm_gradient_exact; paper §3.2 energy and constraints in their Euler /
semi-Lagrangian discretisation) against the FP64 oracle's (oracle/exact.py,
pinned by finite differences), with and without state checkpoints, and
lddmm_energy against the gradient's energy.

Tolerances: gradient relative L2 1e-4 and energy 1e-5 against FP64, as for
the paper's gradient; checkpointed against plain 1e-5 (the same arithmetic,
except that the scatter of the state adjoint adds in a different order).

The exact derivative holds the slope of the interpolant's cell at each
departure point, and the cell is an integer that floating point decides: the
kernels form X = i - (dt v) N in single precision.  Where a departure point
lies within rounding of a cell face, single and double precision pick
different cells and the exact derivative differs by a whole slope jump there.
So the library is compared with the oracle taking its cell decisions in single
precision as the kernels do (exact.departure_points_fp32) at 1e-5 (measured
2e-7 to 1.3e-6: FP32 arithmetic and the order of the scatter's additions
only), and with the all-FP64 oracle at a bar that allows
for those decisions: the gradient 1e-4 still, the Gauss-Newton product 5e-4
(at 64^3 / band 16^3 / 10 steps the oracle's own product moves by 1.6e-4 when
only its cell decisions are made in single precision, the gradient by
2.9e-5)."""

import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import Params  # noqa: E402
from oracle import exact  # noqa: E402
from oracle.jacobi import forward  # noqa: E402
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


CASES = {
    "small": dict(grid=(24, 20, 18), band=(8, 8, 6), nt=4, s=2, dmax=1.5, cfg=2, ckpt=3),
    "aniso": dict(grid=(40, 36, 32), band=(12, 16, 8), nt=5, s=2, dmax=2.0, cfg=2, ckpt=2),
    "cfg2": dict(grid=(64, 64, 64), band=(16, 16, 16), nt=10, s=2, dmax=5.0, cfg=2, ckpt=4),
    "full": dict(grid=(128, 128, 128), band=(32, 32, 32), nt=10, s=3, dmax=8.0, cfg=3, ckpt=5),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    name = request.param
    c = CASES[name]
    print(f"\n[exact gradient case {name}]", flush=True)
    w = synth.workload(c["cfg"], grid=c["grid"], band=c["band"])
    p = Params(grid=c["grid"], band=c["band"], nt=c["nt"], alpha=synth.ALPHA, s=c["s"], sigma=synth.SIGMA)
    vstar = synth.scale_to_displacement(w["v_star"], c["grid"], c["dmax"])
    I0 = w["I0"]
    I1 = forward(vstar, I0, p)[2][-1]
    v0 = 0.6 * vstar
    g, E, cache = exact.gradient(v0, I0, I1, p)
    g32 = v0 + exact.adjoint_sweep(cache["vs"], cache["vgrid"], cache["ms"],
                                   2.0 / (p.sigma ** 2 * float(np.prod(p.grid))) * (cache["ms"][-1] - I1), p,
                                   decisions="fp32")[0]
    prob = L().Problem(grid=c["grid"], band=c["band"], time_steps=c["nt"], alpha=synth.ALPHA, s=c["s"],
                       sigma=synth.SIGMA)
    args = (dev(I0, torch.float32), dev(I1, torch.float32), dev(v0, torch.complex64))
    return dict(name=name, c=c, p=p, g=g, g32=g32, E=E, cache=cache, prob=prob, args=args, vstar=vstar,
                I0=I0, I1=I1)


def test_exact_gradient_matches_oracle(case):
    ws = L().Workspace(case["prob"])
    gg, e3 = L().gradient_exact(case["prob"], *case["args"], ws)
    gh = host(gg)
    eg, eg32 = rel(gh, case["g"]), rel(gh, case["g32"])
    e3 = host(e3)
    eE = max(abs(e3[i] - case["E"][i]) / abs(case["E"][i]) for i in range(3))
    print(f"{case['name']}: exact gradient rel {eg32:.2e} (single-precision cell decisions), "
          f"{eg:.2e} (FP64), energy rel {eE:.1e}")
    assert eg32 < 1e-5 and eg < 1e-4 and eE < 1e-5
    e_only = host(L().energy(case["prob"], *case["args"], ws))
    assert np.max(np.abs(e_only - e3) / np.abs(e3)) < 1e-12


def test_checkpointed_equals_plain(case):
    prob_c = dataclasses.replace(case["prob"], checkpoint=case["c"]["ckpt"])
    ws_c = L().Workspace(prob_c)
    ws = L().Workspace(case["prob"])
    g0, _ = L().gradient_exact(case["prob"], *case["args"], ws)
    g1, _ = L().gradient_exact(prob_c, *case["args"], ws_c)
    e = rel(host(g1), host(g0))
    print(f"{case['name']}: checkpoint {case['c']['ckpt']}: rel {e:.1e}; workspace "
          f"{ws_c.nbytes / 2**20:.1f} MiB instead of {ws.nbytes / 2**20:.1f} MiB")
    assert e < 1e-5
    assert ws_c.nbytes < ws.nbytes


def test_exact_gauss_newton_product_matches_oracle_and_is_symmetric(case):
    """LDDMM_GN_EXACT: (J^T W J + Id) dv against the oracle (1e-5 with the
    cell decisions in single precision, 5e-4 all FP64; see the module doc),
    and <a, H b>_V = <b, H a>_V on random pairs (relative to
    sqrt(<a,Ha><b,Hb>), 1e-5: the product is symmetric up to FP32
    rounding)."""
    from oracle.band import inner, symbol_L
    p = case["p"]
    cache = case["cache"]
    prob = dataclasses.replace(case["prob"], hessian=L().GN_EXACT)
    ws = L().Workspace(prob)
    L().gradient(prob, *case["args"], ws)
    Lsym = symbol_L(p.band, p.alpha, p.s)
    dirs = [synth.random_direction(500 + k, p.band, s=p.s) for k in range(4)]
    H = [host(L().hessvec(prob, dev(d, torch.complex64), ws)) for d in dirs]
    e = rel(H[0], exact.gauss_newton_hessvec(cache, dirs[0], p))
    e32 = rel(H[0], exact.gauss_newton_hessvec(cache, dirs[0], p, decisions="fp32"))
    sym = []
    for i, j in ((0, 1), (2, 3), (0, 3)):
        ab, ba = inner(Lsym * dirs[i], H[j]), inner(Lsym * dirs[j], H[i])
        sym.append(abs(ab - ba) / np.sqrt(inner(Lsym * dirs[i], H[i]) * inner(Lsym * dirs[j], H[j])))
    print(f"{case['name']}: exact Gauss-Newton product rel {e32:.2e} (single-precision cell decisions), "
          f"{e:.2e} (FP64), symmetry {['%.1e' % x for x in sym]}")
    assert e32 < 1e-5 and e < 5e-4 and max(sym) < 1e-5


def test_exact_registration_loop_matches_oracle():
    """The Gauss-Newton-Krylov loop in LDDMM_GN_EXACT against the oracle's
    mode "EXACT" (decisions exact, energies 1e-4, final iterate 1e-3)."""
    from oracle.gn import register as oracle_register
    print("\n[exact Gauss-Newton loop]", flush=True)
    grid, band, nt = (24, 20, 18), (8, 8, 6), 4
    w = synth.workload(2, grid=grid, band=band)
    p = Params(grid=grid, band=band, nt=nt, alpha=synth.ALPHA, s=2, sigma=synth.SIGMA)
    vstar = synth.scale_to_displacement(w["v_star"], grid, 1.5)
    I0 = w["I0"]
    I1 = forward(vstar, I0, p)[2][-1]
    v_ref, st_ref, status_ref = oracle_register(I0, I1, p, 3, 4, mode="EXACT")
    prob = L().Problem(grid=grid, band=band, time_steps=nt, alpha=synth.ALPHA, s=2, sigma=synth.SIGMA,
                       hessian=L().GN_EXACT)
    ws = L().Workspace(prob)
    v, st, rc, hv = L().register(prob, dev(I0, torch.float32), dev(I1, torch.float32), ws, gn_iters=3, pcg_iters=4)
    assert rc == status_ref and len(st) == len(st_ref)
    for a, b in zip(st, st_ref):
        print(f"library pcg {a['pcg_iters']} guard {a['pcg_guard']} step {a['step']} E {a['energy']:.6f} | "
              f"oracle pcg {b['pcg_iters']} guard {b['pcg_guard']} step {b['eps']} E {b['E']:.6f}")
        assert a["pcg_iters"] == b["pcg_iters"] and bool(a["pcg_guard"]) == bool(b["pcg_guard"])
        assert a["trials"] == b["trials"] and a["step"] == b["eps"]
        assert abs(a["energy"] - b["E"]) <= 1e-4 * abs(b["E"])
    ev = rel(host(v), v_ref)
    print(f"exact loop: final v0 rel {ev:.2e}")
    assert ev < 1e-3


def test_exact_product_symmetry_at_the_autograd_volume():
    """160x192x160 / band 32^3 / 20 steps at a random v0 of 5 voxels: the
    exact Gauss-Newton product on random pairs (relative asymmetry 1e-5)."""
    from oracle.band import inner, symbol_L
    print("\n[exact product 160x192x160]", flush=True)
    grid, band, nt = (160, 192, 160), (32, 32, 32), 20
    w = synth.workload(4)
    vstar = w["v_star"]
    prob = L().Problem(grid=grid, band=band, time_steps=nt, alpha=synth.ALPHA, s=3, sigma=synth.SIGMA,
                       hessian=L().GN_EXACT)
    ws = L().Workspace(prob)
    tI0 = dev(w["I0"], torch.float32)
    tI1 = L().shoot(dataclasses.replace(prob, hessian=L().GN_PAPER), tI0, dev(vstar, torch.complex64),
                    L().Workspace(dataclasses.replace(prob, hessian=L().GN_PAPER)))
    L().gradient(prob, tI0, tI1, dev(0.6 * vstar, torch.complex64), ws)
    Lsym = symbol_L(band, synth.ALPHA, 3)
    dirs = [synth.random_direction(600 + k, band, s=3) for k in range(4)]
    H = [host(L().hessvec(prob, dev(d, torch.complex64), ws)) for d in dirs]
    sym = []
    for i, j in ((0, 1), (2, 3), (1, 2)):
        ab, ba = inner(Lsym * dirs[i], H[j]), inner(Lsym * dirs[j], H[i])
        sym.append(abs(ab - ba) / np.sqrt(inner(Lsym * dirs[i], H[i]) * inner(Lsym * dirs[j], H[j])))
    print("asymmetry on random pairs", ["%.1e" % x for x in sym])
    assert max(sym) < 1e-5
