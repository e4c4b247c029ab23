"""The tile table and the autotuner (lddmm_tiles_set, lddmm_autotune): every
launch shape the table can select gives bitwise the gradient and the
Hessian-vector product of the built-in rule (the shapes change which blocks
compute what, not the arithmetic), at the measured 128^3 / band 32^3 shape
(lean and general column kernels) and at 64^3 / band 16^3; the autotuner
returns a valid entry, stores it, leaves the workspace prepared, and its
choice is never slower than the built-in rule on its own measurement."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_1807_11560_amd import synth  # noqa: E402


def L():
    from paper_1807_11560_amd import lddmm
    return lddmm


CASES = {
    "128cubed_band32": dict(cfg=3, grid=(128, 128, 128), band=(32, 32, 32), s=3, nt=10),
    "64cubed_band16": dict(cfg=2, grid=(64, 64, 64), band=(16, 16, 16), s=2, nt=10),
}

TILES = [dict(sl_threads=64), dict(sl_threads=128), dict(prod_rows=1), dict(prod_rows=3), dict(col_split=1),
         dict(col_split=2), dict(col_split=3), dict(prod_rows=2, col_split=1, sl_threads=128)]


def setup(name):
    c = CASES[name]
    w = synth.workload(c["cfg"], grid=c["grid"], band=c["band"])
    prob = L().Problem(grid=c["grid"], band=c["band"], time_steps=c["nt"], alpha=synth.ALPHA, s=c["s"],
                       sigma=synth.SIGMA)
    vstar = synth.scale_to_displacement(w["v_star"], c["grid"], 4.0)
    ws = L().Workspace(prob)
    I0 = torch.from_numpy(w["I0"]).float().cuda()
    I1 = L().shoot(prob, I0, torch.from_numpy(vstar).to(torch.complex64).cuda(), ws)
    v0 = torch.from_numpy(0.5 * vstar).to(torch.complex64).cuda()
    d = torch.from_numpy(synth.random_direction(11, c["band"], s=c["s"])).to(torch.complex64).cuda()
    return prob, ws, I0, I1, v0, d


def grad_and_hvp(prob, ws, I0, I1, v0, d):
    g, _ = L().gradient(prob, I0, I1, v0, ws)
    h = L().hessvec(prob, d, ws)
    torch.cuda.synchronize()
    return g.cpu().numpy(), h.cpu().numpy()


@pytest.mark.parametrize("name", list(CASES))
def test_every_tile_choice_is_bitwise_the_built_in_rule(name):
    print(f"\n[tiles {name}]", flush=True)
    prob, ws, I0, I1, v0, d = setup(name)
    L().tiles_clear()
    try:
        g0, h0 = grad_and_hvp(prob, ws, I0, I1, v0, d)
        for t in TILES:
            if t.get("prod_rows", 0) > 256 // (3 * prob.band[2] // 2):
                continue
            L().tiles_set(prob, t)
            g, h = grad_and_hvp(prob, ws, I0, I1, v0, d)
            print(f"{t}: gradient equal {np.array_equal(g, g0)}, product equal {np.array_equal(h, h0)}", flush=True)
            assert np.array_equal(g, g0) and np.array_equal(h, h0)
    finally:
        L().tiles_clear()


def test_autotune_stores_a_valid_entry_and_keeps_the_results():
    print("\n[autotune 128^3 / band 32^3]", flush=True)
    prob, ws, I0, I1, v0, d = setup("128cubed_band32")
    L().tiles_clear()
    try:
        g0, h0 = grad_and_hvp(prob, ws, I0, I1, v0, d)
        best, ms_best, ms_default = L().autotune(prob, I0, I1, v0, ws, reps=10)
        print(f"autotune: {best}, {ms_best:.3f} ms per product (built-in rule {ms_default:.3f} ms)", flush=True)
        assert 0 < ms_best <= ms_default
        assert 0 <= best["prod_rows"] <= 5 and 0 <= best["col_split"] <= 3 and best["sl_threads"] in (0, 64, 128)
        assert L().tiles_get(prob) == best
        # the workspace is prepared at v0: a product right away equals the built-in rule's
        h = L().hessvec(prob, d, ws)
        torch.cuda.synchronize()
        assert np.array_equal(h.cpu().numpy(), h0)
        g, h = grad_and_hvp(prob, ws, I0, I1, v0, d)
        assert np.array_equal(g, g0) and np.array_equal(h, h0)
    finally:
        L().tiles_clear()
