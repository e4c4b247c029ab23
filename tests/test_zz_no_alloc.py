"""lddmm_shoot_static (the entry point for callers that cannot allocate)
against lddmm_shoot through the C-ABI: two calls in a row, the second on a
smaller problem, each equal to lddmm_shoot on the same inputs (the same
kernels run in a different workspace, so the results are expected to be
identical; the bound is the 1e-6 relative L2 of FP32 rounding), and a
problem too large for its fixed array is rejected before anything runs."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_1807_11560_amd import synth  # noqa: E402


def L():
    from paper_1807_11560_amd import lddmm
    return lddmm


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def test_static_shoot_equals_shoot_twice_then_smaller():
    cases = [((64, 64, 64), (16, 16, 16), 10, 2), ((24, 20, 18), (8, 8, 6), 4, 2)]
    for grid, band, nt, cfg in cases:
        print(f"\n[static shoot {grid} band {band} nt {nt}]", flush=True)
        w = synth.workload(cfg, grid=grid, band=band)
        prob = L().Problem(grid=grid, band=band, time_steps=nt, alpha=synth.ALPHA, s=2, sigma=synth.SIGMA)
        assert prob.workspace_bytes() <= L().STATIC_SCRATCH_BYTES
        I0 = torch.from_numpy(w["I0"]).float().cuda()
        v0 = torch.from_numpy(synth.scale_to_displacement(w["v_star"], grid, 2.0)).to(torch.complex64).cuda()
        m_ref, v_ref = L().shoot(prob, I0, v0, L().Workspace(prob), want_v1=True)
        m_st, v_st = L().shoot_static(prob, I0, v0, want_v1=True)
        torch.cuda.synchronize()
        a, b = m_st.cpu().numpy(), m_ref.cpu().numpy()
        c, d = v_st.cpu().numpy(), v_ref.cpu().numpy()
        em, ev = rel(a.astype(np.float64), b.astype(np.float64)), rel(c.astype(np.complex128), d.astype(np.complex128))
        print(f"m1 rel {em:.1e} (bitwise {np.array_equal(a, b)}), v1 rel {ev:.1e} (bitwise {np.array_equal(c, d)})")
        assert em <= 1e-6 and ev <= 1e-6
    # too large for the fixed array: rejected, nothing enqueued
    big = L().Problem(grid=(128, 128, 128), band=(32, 32, 32), time_steps=10)
    assert big.workspace_bytes() > L().STATIC_SCRATCH_BYTES
    I0 = torch.zeros(big.grid, dtype=torch.float32, device="cuda")
    v0 = torch.zeros(big.band_shape, dtype=torch.complex64, device="cuda")
    with pytest.raises(L().LddmmError) as e:
        L().shoot_static(big, I0, v0)
    assert e.value.code == L().E_WORKSPACE
