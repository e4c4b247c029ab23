"""A steady stream of Hessian-vector products for a profiler: the measured
128^3 / band 32^3 problem (synthetic tissue phantom, its warp by the band
geodesic as the target), one gradient at v0 = v*/2, then N products in one
direction, back to back on the current stream.

    rocprofv3 --kernel-trace --output-format csv -d DIR -o hvp -- python3 -m paper_1807_11560_amd.profile_products --products 40
"""

import argparse
import os
import sys


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--products", type=int, default=40)
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import torch
    from paper_1807_11560_amd import lddmm as L
    from paper_1807_11560_amd import synth

    w = synth.workload(3)
    pp = w["params"]
    prob = L.Problem(grid=pp["grid"], band=pp["band"], time_steps=pp["nt"], alpha=pp["alpha"], s=pp["s"],
                     sigma=pp["sigma"])
    ws = L.Workspace(prob)
    I0 = torch.from_numpy(w["I0"]).float().cuda()
    vstar = torch.from_numpy(w["v_star"]).to(torch.complex64).cuda()
    I1 = L.shoot(prob, I0, vstar, ws)
    L.gradient(prob, I0, I1, 0.5 * vstar, ws)
    d = torch.from_numpy(synth.random_direction(1, prob.band, s=pp["s"])).to(torch.complex64).cuda()
    out = torch.empty_like(d)
    for _ in range(args.products):
        L.hessvec(prob, d, ws, out=out)
    torch.cuda.synchronize()
    print(f"{args.products} products done", flush=True)


if __name__ == "__main__":
    main()
