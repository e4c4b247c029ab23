"""Conjugate gradients in the V metric and the Gauss-Newton-Krylov loop
(paper §2.7, the Newton update and the Krylov system H dv_0 = -grad E, with
"CG with the gradient and the Hessian computed on V").  FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings:
  * Sign: the paper's update v - eps dv with H dv = -grad E would ascend; the
    system H_V p = -g_V is solved and the update is v_0 + eps p (a descent
    step whenever H_V is positive definite).
  * CG starts from p = 0 and runs a fixed number of iterations with all
    inner products <a, b>_V = <L~ a, b>_l2.  Curvature guard: if
    <d, H d>_V <= 0 the loop stops; at the first iteration p = -g_V.
    It also stops when the residual is exactly zero.
  * Step length: Armijo backtracking, eps = 1, 1/2, 1/4, ... at most
    ``max_trials`` trials, sufficient decrease c1 = 1e-4.  If p is not a
    descent direction (<g_V, p>_V >= 0) it is replaced by -g_V.
  * MSE_rel = 100 ||m_1 - I1||^2 / ||I0 - I1||^2 and
    ||g||_inf,rel = ||g_k||_inf / ||g_0||_inf (reported in §4, not defined
    there).
"""

import numpy as np

from . import deformation, exact, jacobi
from .band import inner, symbol_L
from .jacobi import energy

# the constrained problem: image state (§3.2) or deformation state (§3.3)
STATES = ("image", "deformation")


def final_state(v, I0, p, state="image"):
    """m(1) of the forward model of the given state."""
    if state == "image":
        return jacobi.forward(v, I0, p)[2][-1]
    return deformation.forward(v, I0, p)[2]


def pcg(apply_H, g, Lsym, iters):
    """CG on H_V p = -g_V in the V metric.  Returns (p, info)."""
    p = np.zeros_like(g)
    r = -g
    d = r.copy()
    rr = inner(Lsym * r, r)
    info = {"iters": 0, "guard": False, "res": [np.sqrt(max(rr, 0.0))]}
    for it in range(iters):
        if rr <= 0.0:
            break
        Hd = apply_H(d)
        dHd = inner(Lsym * d, Hd)
        if dHd <= 0.0:
            info["guard"] = True
            if it == 0:
                p = -g
            break
        a = rr / dHd
        p = p + a * d
        r = r - a * Hd
        rr_new = inner(Lsym * r, r)
        d = r + (rr_new / rr) * d
        rr = rr_new
        info["iters"] = it + 1
        info["res"].append(np.sqrt(max(rr, 0.0)))
    return p, info


def line_search(v0, p_dir, E0, slope, I0, I1, p, c1=1e-4, max_trials=10, state="image"):
    """Armijo backtracking.  Returns (accepted, eps, E, trials)."""
    eps = 1.0
    for trial in range(1, max_trials + 1):
        v_try = v0 + eps * p_dir
        E = energy(v_try, final_state(v_try, I0, p, state), I1, p)
        if E[0] <= E0 + c1 * eps * slope:
            return True, eps, E, trial
        eps *= 0.5
    return False, 0.0, None, max_trials


def register(I0, I1, p, gn_iters, pcg_iters, v0=None, mode="R1", max_trials=10, state="image"):
    """Gauss-Newton-Krylov registration from v0 (zero by default) for the
    problem subject to the image state (§3.2) or the deformation state (§3.3).
    mode: the Hessian of the paper's method ("R1", "R2", "FULL"), or "EXACT":
    the exact derivative of the discrete energy and its Gauss-Newton product
    (oracle/exact.py)."""
    if state not in STATES:
        raise ValueError("state must be 'image' or 'deformation'")
    model = jacobi if state == "image" else deformation
    if mode == "EXACT":
        # the exact derivative of the discrete energy and its Gauss-Newton product
        if state != "image":
            raise ValueError("mode 'EXACT' is for the image state")
        grad_fn, hess_fn = exact.gradient, (lambda cache, d: exact.gauss_newton_hessvec(cache, d, p))
    else:
        grad_fn, hess_fn = model.gradient, (lambda cache, d: model.hessvec(cache, d, p, mode))
    Lsym = symbol_L(p.band, p.alpha, p.s)
    if v0 is None:
        v0 = np.zeros((p.d,) + tuple(p.band), dtype=np.complex128)
    denom = float(np.sum((I0 - I1) ** 2))
    stats = []
    g0_inf = None
    status = 0
    for it in range(gn_iters):
        g, E, cache = grad_fn(v0, I0, I1, p)
        m1 = cache["ms"][-1] if state == "image" else cache["m1"]
        g_inf = float(np.max(np.abs(g)))
        if g0_inf is None:
            g0_inf = g_inf
        p_dir, info = pcg(lambda dvec: hess_fn(cache, dvec), g, Lsym, pcg_iters)
        slope = inner(Lsym * g, p_dir)
        if slope >= 0.0:
            p_dir = -g
            slope = inner(Lsym * g, p_dir)
        ok, eps, E_new, trials = line_search(v0, p_dir, E[0], slope, I0, I1, p,
                                             max_trials=max_trials, state=state)
        rec = {"E": E[0], "E_reg": E[1], "E_data": E[2],
               "mse_rel": 100.0 * float(np.sum((m1 - I1) ** 2)) / denom if denom > 0 else 0.0,
               "g_inf_rel": g_inf / g0_inf if g0_inf > 0 else 0.0,
               "pcg_iters": info["iters"], "pcg_guard": info["guard"],
               "eps": eps, "trials": trials}
        stats.append(rec)
        if not ok:
            status = 1
            break
        v0 = v0 + eps * p_dir
    return v0, stats, status
