"""Python binding of liblddmm.so (include/lddmm.h): argument marshalling only.

Every step of shooting, transport, gradient, Hessian-vector product and
registration runs in the HIP library; torch provides device memory and the
stream.  Importing this module fails loudly if the library has not been
built (``python -m paper_1807_11560_amd.build``).
"""

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblddmm.so")

# torch is imported first so that the library's HIP calls bind to the HIP
# runtime torch has loaded: device memory and streams come from torch, and a
# second runtime in the same process would not see them.
import torch  # noqa: E402,F401

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build the HIP library first (python -m paper_1807_11560_amd.build)")
_lib = ctypes.CDLL(LIB_PATH)

OK = 0
W_LINESEARCH = 1
E_INVALID_ARG = -1
E_SHAPE = -2
E_WORKSPACE = -3
E_HIP = -4
E_NOT_PREPARED = -5
E_NONFINITE = -6
FP32 = 0
FP32_BF16X3 = 1
GN_PAPER = 0
GN_CLASSICAL = 1
NEWTON = 2
GN_EXACT = 3
STATE_IMAGE = 0
STATE_DEFORMATION = 1
EULER = 0
RK4 = 1
SYMBOL_L = 0
SYMBOL_K = 1
KF_SYNTH, KF_GRID, KF_SL, KF_INV0, KF_COLUMN, KF_PRODS = 1, 2, 3, 4, 5, 6
KF_INV0_GRID, KF_FWD1_GRID, KF_FWD0_GRID, KF_SRC = 7, 8, 9, 10
KERNEL_FAMILIES = {KF_SYNTH: "k_synth", KF_GRID: "k_gridstep", KF_SL: "k_sl", KF_INV0: "k_inv0 (padded grid)",
                   KF_COLUMN: "k_colstep", KF_PRODS: "k_prods", KF_INV0_GRID: "k_inv0 (image grid)",
                   KF_FWD1_GRID: "k_fwd1", KF_FWD0_GRID: "k_fwd0", KF_SRC: "k_src_fwd2"}


class LddmmParams(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("grid", ctypes.c_int32 * 3),
        ("band", ctypes.c_int32 * 3),
        ("spectral", ctypes.c_int32 * 3),
        ("time_steps", ctypes.c_int32),
        ("s", ctypes.c_int32),
        ("alpha", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("hessian", ctypes.c_int32),
        ("state", ctypes.c_int32),
        ("integrator", ctypes.c_int32),
        ("checkpoint", ctypes.c_int32),
    ]


class LddmmStats(ctypes.Structure):
    _fields_ = [
        ("energy", ctypes.c_double),
        ("energy_reg", ctypes.c_double),
        ("energy_data", ctypes.c_double),
        ("mse_rel", ctypes.c_double),
        ("grad_inf_rel", ctypes.c_double),
        ("step", ctypes.c_double),
        ("trials", ctypes.c_int32),
        ("pcg_iters", ctypes.c_int32),
        ("pcg_guard", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class LddmmTiles(ctypes.Structure):
    _fields_ = [
        ("prod_rows", ctypes.c_int32),
        ("col_split", ctypes.c_int32),
        ("sl_threads", ctypes.c_int32),
    ]


_vp = ctypes.c_void_p
_P = ctypes.POINTER(LddmmParams)
_T = ctypes.POINTER(LddmmTiles)
_SIGS = {
    "lddmm_workspace_bytes": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t)]),
    "lddmm_shoot": (ctypes.c_int, [_P, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "lddmm_shoot_static": (ctypes.c_int, [_P, _vp, _vp, _vp, _vp, _vp]),
    "lddmm_gradient": (ctypes.c_int, [_P, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "lddmm_geodesic_energy": (ctypes.c_int, [_P, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "lddmm_apply_symbol": (ctypes.c_int, [_P, ctypes.c_int32, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "lddmm_hessvec": (ctypes.c_int, [_P, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "lddmm_gradient_exact": (ctypes.c_int, [_P, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "lddmm_energy": (ctypes.c_int, [_P, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "lddmm_register": (ctypes.c_int, [_P, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.POINTER(LddmmStats), ctypes.c_int32, _vp,
                                      ctypes.c_size_t, _vp]),
    "lddmm_last_register_hvps": (ctypes.c_int64, []),
    "lddmm_batch_workspace_bytes": (ctypes.c_int, [ctypes.c_int32, _P, ctypes.POINTER(ctypes.c_size_t)]),
    "lddmm_register_batch": (ctypes.c_int, [ctypes.c_int32, _P, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_int32, ctypes.POINTER(LddmmStats), ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                                            _vp, ctypes.c_size_t, _vp]),
    "lddmm_kernel_timer": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32]),
    "lddmm_kernel_timer_read": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int64),
                                               ctypes.POINTER(ctypes.c_double),
                                               ctypes.POINTER(ctypes.c_double),
                                               ctypes.POINTER(ctypes.c_double)]),
    "lddmm_use_graphs": (ctypes.c_int, [ctypes.c_int32]),
    "lddmm_tiles_set": (ctypes.c_int, [_P, ctypes.c_char_p, _T]),
    "lddmm_tiles_get": (ctypes.c_int, [_P, ctypes.c_char_p, _T, ctypes.POINTER(ctypes.c_int32)]),
    "lddmm_tiles_clear": (ctypes.c_int, []),
    "lddmm_tiles_save": (ctypes.c_int, [ctypes.c_char_p]),
    "lddmm_tiles_load": (ctypes.c_int, [ctypes.c_char_p]),
    "lddmm_autotune": (ctypes.c_int, [_P, _vp, _vp, _vp, ctypes.c_int32, _T, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double), _vp, ctypes.c_size_t, _vp]),
    "lddmm_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "lddmm_last_error": (ctypes.c_char_p, []),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class LddmmError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        detail = _lib.lddmm_last_error().decode()
        super().__init__(f"{where}: {_lib.lddmm_status_string(code).decode()} ({code}): {detail}")


def _check(code, where):
    if code < 0:
        raise LddmmError(code, where)
    return code


@dataclass(frozen=True)
class Problem:
    """Parameters of one registration problem (paper §3.2 problem statement;
    ``state`` selects the image state of §3.2 or the deformation state of §3.3)."""

    grid: Tuple[int, int, int]
    band: Tuple[int, int, int]
    time_steps: int = 10
    alpha: float = 0.0025
    s: int = 2
    sigma: float = 0.03
    spectral: Tuple[int, int, int] = (0, 0, 0)
    hessian: int = GN_PAPER
    state: int = STATE_IMAGE
    integrator: int = EULER
    precision: int = FP32
    checkpoint: int = 0

    def c_params(self) -> LddmmParams:
        p = LddmmParams()
        p.ndim = len(self.grid)
        for j in range(3):
            p.grid[j] = int(self.grid[j]) if j < len(self.grid) else 1
            p.band[j] = int(self.band[j]) if j < len(self.band) else 1
            p.spectral[j] = int(self.spectral[j]) if j < len(self.spectral) else 0
        p.time_steps = int(self.time_steps)
        p.s = int(self.s)
        p.alpha = float(self.alpha)
        p.sigma = float(self.sigma)
        p.precision = int(self.precision)
        p.checkpoint = int(self.checkpoint)
        p.hessian = int(self.hessian)
        p.state = int(self.state)
        p.integrator = int(self.integrator)
        return p

    def workspace_bytes(self) -> int:
        n = ctypes.c_size_t(0)
        _check(_lib.lddmm_workspace_bytes(ctypes.byref(self.c_params()), ctypes.byref(n)),
               "lddmm_workspace_bytes")
        return n.value

    @property
    def band_shape(self):
        # one component per axis: [3][K0][K1][K2], or [2][K0][K1] in the plane
        return (len(self.grid),) + tuple(self.band)


def _torch():
    import torch
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _need(t, dtype, shape, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Workspace:
    """Device workspace owned by torch; carries the gradient -> hessvec state."""

    def __init__(self, problem: Problem, device=None):
        torch = _torch()
        self.problem = problem
        self.nbytes = problem.workspace_bytes()
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=device or "cuda")

    @property
    def ptr(self):
        return ctypes.c_void_p(self.buf.data_ptr())


def shoot(problem: Problem, I0, v0, ws: Workspace, want_v1=False, stream=None):
    """m_1 (and v_1) of the band geodesic from v0 (lddmm_shoot)."""
    torch = _torch()
    _need(I0, torch.float32, problem.grid, "I0")
    _need(v0, torch.complex64, problem.band_shape, "v0")
    m1 = torch.empty_like(I0)
    v1 = torch.empty_like(v0) if want_v1 else None
    _check(_lib.lddmm_shoot(ctypes.byref(problem.c_params()), _ptr(I0), _ptr(v0), _ptr(m1), _ptr(v1),
                            ws.ptr, ws.nbytes, _stream(stream)), "lddmm_shoot")
    return (m1, v1) if want_v1 else m1


STATIC_SCRATCH_BYTES = 128 << 20


def shoot_static(problem: Problem, I0, v0, want_v1=False, stream=None):
    """lddmm_shoot in the library's own device array (lddmm_shoot_static):
    no workspace, nothing allocated by the library (the outputs here are
    torch tensors)."""
    torch = _torch()
    _need(I0, torch.float32, problem.grid, "I0")
    _need(v0, torch.complex64, problem.band_shape, "v0")
    m1 = torch.empty_like(I0)
    v1 = torch.empty_like(v0) if want_v1 else None
    _check(_lib.lddmm_shoot_static(ctypes.byref(problem.c_params()), _ptr(I0), _ptr(v0), _ptr(m1), _ptr(v1),
                                   _stream(stream)), "lddmm_shoot_static")
    return (m1, v1) if want_v1 else m1


def apply_symbol(problem: Problem, which: int, x, ws: Workspace, out=None, stream=None):
    """L~ x (which = SYMBOL_L) or K~ x (SYMBOL_K) on a band field (lddmm_apply_symbol)."""
    torch = _torch()
    _need(x, torch.complex64, problem.band_shape, "x")
    if out is None:
        out = torch.empty_like(x)
    _check(_lib.lddmm_apply_symbol(ctypes.byref(problem.c_params()), int(which), _ptr(x), _ptr(out), ws.ptr,
                                   ws.nbytes, _stream(stream)), "lddmm_apply_symbol")
    return out


def geodesic_energy(problem: Problem, v0, ws: Workspace, stream=None):
    """<L~ v_n, v_n> for n = 0..nt along the shot trajectory (lddmm_geodesic_energy):
    a float64 device tensor of nt + 1 values."""
    torch = _torch()
    _need(v0, torch.complex64, problem.band_shape, "v0")
    out = torch.empty(problem.time_steps + 1, dtype=torch.float64, device=v0.device)
    _check(_lib.lddmm_geodesic_energy(ctypes.byref(problem.c_params()), _ptr(v0), _ptr(out), ws.ptr, ws.nbytes,
                                      _stream(stream)), "lddmm_geodesic_energy")
    return out


def gradient(problem: Problem, I0, I1, v0, ws: Workspace, stream=None):
    """(g_V, energy[3] float64 on the device) at v0 (lddmm_gradient)."""
    torch = _torch()
    _need(I0, torch.float32, problem.grid, "I0")
    _need(I1, torch.float32, problem.grid, "I1")
    _need(v0, torch.complex64, problem.band_shape, "v0")
    g = torch.empty_like(v0)
    e3 = torch.empty(3, dtype=torch.float64, device=v0.device)
    _check(_lib.lddmm_gradient(ctypes.byref(problem.c_params()), _ptr(I0), _ptr(I1), _ptr(v0), _ptr(g),
                               _ptr(e3), ws.ptr, ws.nbytes, _stream(stream)), "lddmm_gradient")
    return g, e3


def energy(problem: Problem, I0, I1, v0, ws: Workspace, stream=None):
    """energy[3] (E, E_reg, E_data; float64 on the device) at v0 (lddmm_energy)."""
    torch = _torch()
    _need(I0, torch.float32, problem.grid, "I0")
    _need(I1, torch.float32, problem.grid, "I1")
    _need(v0, torch.complex64, problem.band_shape, "v0")
    e3 = torch.empty(3, dtype=torch.float64, device=v0.device)
    _check(_lib.lddmm_energy(ctypes.byref(problem.c_params()), _ptr(I0), _ptr(I1), _ptr(v0), _ptr(e3), ws.ptr,
                             ws.nbytes, _stream(stream)), "lddmm_energy")
    return e3


def gradient_exact(problem: Problem, I0, I1, v0, ws: Workspace, stream=None):
    """(g_V, energy[3] float64 on the device): the exact derivative of the
    discrete energy at v0 (lddmm_gradient_exact; honours problem.checkpoint)."""
    torch = _torch()
    _need(I0, torch.float32, problem.grid, "I0")
    _need(I1, torch.float32, problem.grid, "I1")
    _need(v0, torch.complex64, problem.band_shape, "v0")
    g = torch.empty_like(v0)
    e3 = torch.empty(3, dtype=torch.float64, device=v0.device)
    _check(_lib.lddmm_gradient_exact(ctypes.byref(problem.c_params()), _ptr(I0), _ptr(I1), _ptr(v0), _ptr(g),
                                     _ptr(e3), ws.ptr, ws.nbytes, _stream(stream)), "lddmm_gradient_exact")
    return g, e3


def hessvec(problem: Problem, dv0, ws: Workspace, out=None, stream=None):
    """Gauss-Newton H_V dv0 at the v0 of the last gradient on ws (lddmm_hessvec)."""
    torch = _torch()
    _need(dv0, torch.complex64, problem.band_shape, "dv0")
    if out is None:
        out = torch.empty_like(dv0)
    else:
        _need(out, torch.complex64, problem.band_shape, "out")
    _check(_lib.lddmm_hessvec(ctypes.byref(problem.c_params()), _ptr(dv0), _ptr(out), ws.ptr, ws.nbytes,
                              _stream(stream)), "lddmm_hessvec")
    return out


def register(problem: Problem, I0, I1, ws: Workspace, gn_iters=10, pcg_iters=20, v0=None,
             stream=None):
    """Gauss-Newton-Krylov registration (lddmm_register).

    Returns (v0, stats, status, hvps): the result, one dict per GN iteration,
    OK or W_LINESEARCH, and the number of Hessian-vector products."""
    torch = _torch()
    _need(I0, torch.float32, problem.grid, "I0")
    _need(I1, torch.float32, problem.grid, "I1")
    if v0 is None:
        v0 = torch.zeros(problem.band_shape, dtype=torch.complex64, device=I0.device)
    else:
        _need(v0, torch.complex64, problem.band_shape, "v0")
    stats = (LddmmStats * max(gn_iters, 1))()
    rc = _check(_lib.lddmm_register(ctypes.byref(problem.c_params()), _ptr(I0), _ptr(I1), _ptr(v0),
                                    int(gn_iters), int(pcg_iters), stats, int(gn_iters), ws.ptr,
                                    ws.nbytes, _stream(stream)), "lddmm_register")
    recs = []
    for i in range(gn_iters):
        s = stats[i]
        if s.trials == 0:
            break
        recs.append({f: getattr(s, f) for f, _ in LddmmStats._fields_ if f != "reserved"})
    return v0, recs, rc, int(_lib.lddmm_last_register_hvps())


def batch_workspace_bytes(problems: Sequence[Problem]) -> int:
    """Workspace bytes of register_batch over these problems (lddmm_batch_workspace_bytes)."""
    arr = (LddmmParams * len(problems))(*[q.c_params() for q in problems])
    n = ctypes.c_size_t(0)
    _check(_lib.lddmm_batch_workspace_bytes(len(problems), arr, ctypes.byref(n)), "lddmm_batch_workspace_bytes")
    return n.value


class BatchWorkspace:
    """One device workspace for register_batch over a list of problems."""

    def __init__(self, problems: Sequence[Problem], device=None):
        torch = _torch()
        self.nbytes = batch_workspace_bytes(problems)
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=device or "cuda")

    @property
    def ptr(self):
        return self.buf.data_ptr()


def register_batch(problems: Sequence[Problem], I0s, I1s, ws: BatchWorkspace, gn_iters=10, pcg_iters=20,
                   v0s=None, concurrency=0, stream=None):
    """Independent registrations in one call (lddmm_register_batch).

    Returns (v0s, stats, status, hvps, rc): per pair the result, one dict per GN
    iteration, the return code and the number of Hessian-vector products."""
    torch = _torch()
    n = len(problems)
    if not (len(I0s) == len(I1s) == n):
        raise ValueError("one I0 and one I1 per problem")
    for q, a, b in zip(problems, I0s, I1s):
        _need(a, torch.float32, q.grid, "I0")
        _need(b, torch.float32, q.grid, "I1")
    if v0s is None:
        v0s = [torch.zeros(q.band_shape, dtype=torch.complex64, device=a.device) for q, a in zip(problems, I0s)]
    for q, v in zip(problems, v0s):
        _need(v, torch.complex64, q.band_shape, "v0")
    arr = (LddmmParams * n)(*[q.c_params() for q in problems])
    p0 = (ctypes.c_void_p * n)(*[_ptr(a) for a in I0s])
    p1 = (ctypes.c_void_p * n)(*[_ptr(b) for b in I1s])
    pv = (ctypes.c_void_p * n)(*[_ptr(v) for v in v0s])
    slen = max(gn_iters, 1)
    stats = (LddmmStats * (n * slen))()
    status = (ctypes.c_int32 * n)()
    hv = (ctypes.c_int64 * n)()
    rc = _check(_lib.lddmm_register_batch(n, arr, p0, p1, pv, int(gn_iters), int(pcg_iters), int(concurrency),
                                          stats, slen, status, hv, ws.ptr, ws.nbytes, _stream(stream)),
                "lddmm_register_batch")
    recs = []
    for i in range(n):
        r = []
        for k in range(gn_iters):
            s_ = stats[i * slen + k]
            if s_.trials == 0:
                break
            r.append({f: getattr(s_, f) for f, _ in LddmmStats._fields_ if f != "reserved"})
        recs.append(r)
    return v0s, recs, [int(x) for x in status], [int(x) for x in hv], rc


def kernel_timer(family: int, every: int = 1):
    """Time one launch in `every` of kernel family `family` (0 switches the timer off)."""
    _check(_lib.lddmm_kernel_timer(int(family), int(every)), "lddmm_kernel_timer")


def kernel_timer_read():
    """(launches, total ms, algorithmic flops, algorithmic bytes) of the timed family."""
    n = ctypes.c_int64(0)
    ms = ctypes.c_double(0.0)
    fl = ctypes.c_double(0.0)
    by = ctypes.c_double(0.0)
    _check(_lib.lddmm_kernel_timer_read(ctypes.byref(n), ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(by)),
           "lddmm_kernel_timer_read")
    return n.value, ms.value, fl.value, by.value


def use_graphs(enable: bool):
    """Graph replay of the launch-bound sequences on or off (default; lddmm_use_graphs)."""
    _check(_lib.lddmm_use_graphs(1 if enable else 0), "lddmm_use_graphs")


def raw():
    """The loaded ctypes library (for tests of the C-ABI itself)."""
    return _lib


TILE_FIELDS = ("prod_rows", "col_split", "sl_threads")


def _arch(arch):
    return arch.encode() if arch is not None else None


def tiles_set(problem: Problem, tiles: dict, arch: Optional[str] = None):
    """Sets the tile-table entry of the problem's shape (lddmm_tiles_set)."""
    t = LddmmTiles(*(int(tiles.get(k, 0)) for k in TILE_FIELDS))
    _check(_lib.lddmm_tiles_set(ctypes.byref(problem.c_params()), _arch(arch), ctypes.byref(t)), "lddmm_tiles_set")


def tiles_get(problem: Problem, arch: Optional[str] = None):
    """The tile-table entry of the problem's shape, or None (lddmm_tiles_get)."""
    t = LddmmTiles()
    found = ctypes.c_int32(0)
    _check(_lib.lddmm_tiles_get(ctypes.byref(problem.c_params()), _arch(arch), ctypes.byref(t),
                                ctypes.byref(found)), "lddmm_tiles_get")
    return {k: getattr(t, k) for k in TILE_FIELDS} if found.value else None


def tiles_clear():
    _check(_lib.lddmm_tiles_clear(), "lddmm_tiles_clear")


def tiles_save(path: str):
    _check(_lib.lddmm_tiles_save(os.fsencode(path)), "lddmm_tiles_save")


def tiles_load(path: str):
    _check(_lib.lddmm_tiles_load(os.fsencode(path)), "lddmm_tiles_load")


def autotune(problem: Problem, I0, I1, v0, ws: Workspace, reps: int = 10, stream=None):
    """Tunes the tile table for this problem (lddmm_autotune): returns the
    chosen tiles, their ms per Hessian-vector product and the built-in
    rule's.  Leaves ws prepared for hessvec at v0."""
    torch = _torch()
    _need(I0, torch.float32, problem.grid, "I0")
    _need(I1, torch.float32, problem.grid, "I1")
    _need(v0, torch.complex64, problem.band_shape, "v0")
    t = LddmmTiles()
    mb, md = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(_lib.lddmm_autotune(ctypes.byref(problem.c_params()), _ptr(I0), _ptr(I1), _ptr(v0), int(reps),
                               ctypes.byref(t), ctypes.byref(mb), ctypes.byref(md), ws.ptr, ws.nbytes,
                               _stream(stream)), "lddmm_autotune")
    return {k: getattr(t, k) for k in TILE_FIELDS}, mb.value, md.value
