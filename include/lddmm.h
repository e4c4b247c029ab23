/*
 * lddmm.h -- C-ABI of the MI355X library for band-limited Jacobi PDE-EPDiff
 * LDDMM subject to the state equation, solved by Gauss-Newton-Krylov
 * (M. Hernandez, "Efficient Gauss-Newton-Krylov momentum conservation
 * constrained PDE-LDDMM using the band-limited vector field
 * parameterization", arXiv 1807.11560).
 *
 * Problem (paper §3.2, band-limited energy): minimise over the band-limited
 * initial velocity v0
 *     E(v0) = 1/2 <L~ v0, v0>_l2 + sigma^-2 || m(1) - I1 ||^2_L2
 * subject to the band-limited EPDiff equation d_t v + ad~dagger_v v = 0
 * (paper §3.1) and the state equation d_t m + grad m . iota(v_t) = 0 with
 * m(0) = I0 (paper §2.3, §3.2), L = (Id - alpha Laplacian)^s (paper §2.1).
 *
 * Conventions used by every entry point
 *   - Domain: the periodic unit cube [0,1)^3; grid point i_j sits at i_j/N_j.
 *   - Grid images (I0, I1, m1): float32, shape [N0][N1][N2], C order (last
 *     axis fastest), device memory.
 *   - Band vector fields (v0, v1, gradients, directions, products): complex64
 *     interleaved (re, im), shape [3][K0][K1][K2], device memory.  Slot q of
 *     axis j holds frequency k = q for q < K_j/2 and q - K_j otherwise; the
 *     slot k = -K_j/2 is zero, so the effective band is |k_j| <= K_j/2 - 1
 *     (paper §3.1, truncated Fourier domain).  iota(v)(x) = sum_k v(k)
 *     exp(2 pi i k.x) (no normalisation), pi(f)(k) = |N|^-1 sum_x f(x)
 *     exp(-2 pi i k.x).  Fields are real, i.e. Hermitian: v(-k) = conj v(k).
 *     Inputs are projected onto Hermitian fields supported on the effective
 *     band (never rejected for violating it); outputs are exactly Hermitian.
 *   - Inner products: <a,b>_l2 = Re sum conj(a) b; the V metric (paper §3.1)
 *     is <a,b>_V = <L~ a, b>_l2 with L~(k) = (1 + alpha sum_j (2 pi k_j)^2)^s.
 *   - Time: nt explicit Euler steps of size 1/nt.  The state is moved by one
 *     first-order semi-Lagrangian step per time step (periodic trilinear
 *     interpolation at x - dt iota(v_n)(x)).
 *   - Streams: every call enqueues its work on `stream` (a hipStream_t; NULL
 *     is the legacy default stream).  lddmm_shoot, lddmm_gradient and
 *     lddmm_hessvec are asynchronous; lddmm_register synchronises `stream`.
 *   - Ownership: the caller owns every buffer, including the workspace
 *     `ws` of `ws_bytes` >= lddmm_workspace_bytes() bytes of device memory.
 *     The library allocates no device memory.  It keeps, per workspace
 *     pointer, a small host record (parameters, prepared flag); the
 *     workspace must not be shared by calls that run concurrently.
 *   - Errors: arguments are validated before anything is enqueued, so a
 *     negative return means nothing was enqueued (except LDDMM_E_HIP, which
 *     reports a failed launch or copy).  lddmm_last_error() gives a
 *     thread-local detail string for the last failure.
 */
#ifndef LDDMM_H
#define LDDMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LDDMM_OK = 0,
  LDDMM_W_LINESEARCH = 1,     /* register: Armijo search failed; v0 holds the last accepted iterate */
  LDDMM_E_INVALID_ARG = -1,   /* null pointer, non-positive alpha/sigma, unknown enum value */
  LDDMM_E_SHAPE = -2,         /* unsupported ndim, odd band, band > grid, spectral grid too small */
  LDDMM_E_WORKSPACE = -3,     /* ws_bytes smaller than lddmm_workspace_bytes() */
  LDDMM_E_HIP = -4,           /* a HIP runtime call or kernel launch failed */
  LDDMM_E_NOT_PREPARED = -5,  /* hessvec without a preceding gradient on this workspace/params */
  LDDMM_E_NONFINITE = -6      /* register: energy or gradient is not finite */
};

/* Arithmetic of the partial-DFT contractions on the matrix cores (paper §3.1: the
 * band <-> grid transforms iota and pi and the truncated convolution, evaluated as
 * separable partial DFTs).  LDDMM_FP32: FP32 operands and accumulation.
 * LDDMM_FP32_BF16X3: each FP32 operand x is split into hi = bf16(x) and
 * lo = bf16(x - hi) (round to nearest even), every product a*b is formed as
 * ah*bh + ah*bl + al*bh on BF16 matrix instructions with FP32 accumulation (the
 * dropped al*bl is about 2^-16 of a*b), so each contraction carries a relative
 * error of about 2^-16 instead of 2^-24.  Everything else (pointwise Lie products,
 * interpolation, symbols, updates) stays FP32, and all inner products, energies
 * and line-search reductions are FP64 in both modes.  Shapes that run on the
 * shape-generic (non-matrix-core) kernels compute those stages in FP32 in both
 * modes. */
enum { LDDMM_FP32 = 0, LDDMM_FP32_BF16X3 = 1 };
/* Hessian of the Krylov solves, see lddmm_params */
enum { LDDMM_GN_PAPER = 0, LDDMM_GN_CLASSICAL = 1, LDDMM_NEWTON = 2, LDDMM_GN_EXACT = 3 };
/* State that carries the deformation, see lddmm_params */
enum { LDDMM_STATE_IMAGE = 0, LDDMM_STATE_DEFORMATION = 1 };
/* Time integration of shooting and transport, see lddmm_params */
enum { LDDMM_EULER = 0, LDDMM_RK4 = 1 };

typedef struct lddmm_params {
  int32_t ndim;         /* spatial dimension, 3 or 2.  With ndim == 2 only grid[0..1],
                           band[0..1] and spectral[0..1] are read; images are [N0][N1],
                           band fields [2][K0][K1] (same slot convention), the domain the
                           periodic unit square.  The single-problem entry points take
                           planar problems (run as the volume problem of depth 8, band
                           depth 4, whose fields do not depend on the new first coordinate;
                           lddmm_workspace_bytes adds staging for two images of that depth
                           and two band fields); lddmm_shoot_static, the batch, the tile
                           table and the autotuner take volumes only (LDDMM_E_SHAPE). */
  int32_t grid[3];      /* N_j >= 8, C order; the last axis at most 256 */
  int32_t band[3];      /* K_j even, 4 <= K_j <= min(N_j, 64) */
  int32_t spectral[3];  /* M_j, padded grid of the truncated convolution; 0 selects 3*K_j/2.
                           Must satisfy 3*K_j/2 - 2 <= M_j <= 256 so that the product of two
                           band fields is alias-free on the band (paper §3.1, truncated
                           convolution). */
  int32_t time_steps;   /* nt >= 1 */
  int32_t s;            /* exponent of L, 1 <= s <= 8 */
  double alpha;         /* > 0 */
  double sigma;         /* > 0, weight of the image term */
  int32_t precision;    /* LDDMM_FP32 or LDDMM_FP32_BF16X3 */
  int32_t hessian;      /* LDDMM_GN_PAPER: Gauss-Newton drops only the -lambda(1) grad dm(1) term
                           of dU(1) and keeps every coupling term of the incremental adjoint
                           Jacobi equations; LDDMM_GN_CLASSICAL also drops the coupling terms
                           that carry U or w (paper §2.7: "dropping expressions" of the Hessian);
                           LDDMM_NEWTON keeps every term, with
                           dU(1) = K~ pi(dlambda(1) grad m(1) + lambda(1) grad dm(1)), the
                           derivative of the gradient's U(1) (the paper prints a minus before
                           lambda(1) grad dm(1) in §2.3/§3.2; the plus sign is the derivative,
                           see the oracle's pins).  This Hessian need not be positive definite:
                           the CG of lddmm_register stops on non-positive curvature.
                           LDDMM_GN_EXACT (image state, Euler): the exact derivative of the
                           discrete energy instead of the paper's adjoint Jacobi one, for
                           lddmm_gradient, lddmm_hessvec and lddmm_register alike: the gradient
                           of lddmm_gradient_exact and the Gauss-Newton product J^T W J + Id
                           (V metric) of that energy, J the derivative of m_nt (the linearised
                           Euler steps and the tangent of every transport step,
                           dm_{n+1} = I[dm_n](X_n) - dt sum_j N_j (d_j I[m_n])(X_n) dv_n,j),
                           W = 2/(sigma^2 |N|); symmetric positive definite, so CG runs its
                           iterations to the end. */
  int32_t state;        /* LDDMM_STATE_IMAGE: the image is transported on the grid (paper §3.2,
                           everything documented above).  LDDMM_STATE_DEFORMATION: the
                           deformation phi = id + u is transported in the band and the image
                           is only formed at t = 1 (paper §3.3):
                             u_{n+1} = u_n - dt [v_n + D~u_n * v_n],  u_0 = 0,
                             (D~u * v)_i = sum_j (d_j u_i) * v_j (truncated products),
                             m(1)(x) = I0(x + iota(u_nt)(x)) (periodic trilinear interpolation),
                           gradient: U(1) = K~(D~phi(1) * rho~), rho~ = pi(lambda(1)
                           (grad I0)(phi(1))), (D~phi * r)_j = r_j + sum_i (d_j u_i) * r_i;
                           the adjoint sweeps are those of §3.2.  Hessian-vector product: the
                           incremental deformation du_{n+1} = du_n - dt [D~du_n * v_n + dv_n
                           + D~u_n * dv_n], dm(1) = (grad I0)(phi(1)) . iota(du_nt) and
                           dU(1) = K~([D~du_nt * rho~] + D~phi(1) * pi(dlambda(1)
                           (grad I0)(phi(1)) [+ lambda(1) (Hess I0)(phi(1)) iota(du_nt)])).
                           LDDMM_GN_PAPER drops both bracketed terms (the residual times a
                           derivative of the increment, like lambda(1) grad dm(1) of the image
                           state) and keeps the coupling terms, LDDMM_GN_CLASSICAL also drops
                           the coupling terms, LDDMM_NEWTON keeps everything.  grad I0 and
                           Hess I0 are the periodic central differences of I0, interpolated
                           trilinearly at phi(1).  The plus signs are the derivative of U(1)
                           (the paper prints a minus before D~phi(1) * drho~(1)).  No per-step
                           image or grid velocity is kept, so the workspace is smaller. */
  int32_t integrator;   /* LDDMM_EULER: nt explicit Euler steps everywhere (as documented above).
                           LDDMM_RK4 (lddmm_shoot and lddmm_geodesic_energy only, image state):
                           the band EPDiff by classical fourth-order Runge-Kutta steps, which
                           conserve the geodesic energy <L~ v_t, v_t> of §2.2 to O(dt^4), and the
                           image transport with midpoint departure points
                           X_h = x - dt/2 v_h(x), X = x - dt v_h(X_h), v_h = iota((v_n + v_{n+1})/2)
                           interpolated trilinearly at X_h (second order in dt).  The gradient,
                           Hessian-vector product and registration integrate the adjoint sweeps
                           as transposes of Euler steps and reject LDDMM_RK4. */
  int32_t checkpoint;   /* 0: the forward keeps every state m_n and grid velocity (the workspace
                           layout of every entry point).  c >= 1 (lddmm_gradient_exact,
                           lddmm_energy, lddmm_apply_symbol and lddmm_workspace_bytes only;
                           image state, Euler): only the states
                           m_0, m_c, m_2c, ... and m_nt are kept; the backward sweep transports
                           each segment of c steps again from its first state and synthesises
                           the grid velocities again from the band trajectory, so the workspace
                           holds about nt/c + c states instead of 4 nt + 1 grid fields (states and
                           grid velocities) and no sweep caches beyond the shooting's.
                           lddmm_energy accepts it too (the forward pass of the same layout). */
} lddmm_params;

/* One Gauss-Newton iteration of lddmm_register (host memory). */
typedef struct lddmm_stats {
  double energy, energy_reg, energy_data; /* at the start of the iteration */
  double mse_rel;       /* 100 ||m1 - I1||^2 / ||I0 - I1||^2 at the start of the iteration */
  double grad_inf_rel;  /* max |g_V(k)| relative to the first iteration */
  double step;          /* accepted Armijo step eps (0 if none) */
  int32_t trials;       /* line-search trials */
  int32_t pcg_iters;    /* CG iterations that updated the solution */
  int32_t pcg_guard;    /* 1 if CG stopped on non-positive curvature */
  int32_t reserved;
} lddmm_stats;

/* Bytes of device workspace needed for these parameters.  Host only, no side
 * effects.  Returns LDDMM_OK or a validation error. */
int lddmm_workspace_bytes(const lddmm_params* p, size_t* bytes);

/* Geodesic shooting and state transport (paper §3.2, the two constraints):
 * v_{n+1} = v_n - dt K~ ad~*_{v_n}(L~ v_n) on the band (band-limited EPDiff,
 * §3.1, explicit Euler), m_{n+1} = I[m_n](x - dt iota(v_n)(x)), m_0 = I0.
 *   I0  [N0][N1][N2] float32 (device, read)
 *   v0  [3][K0][K1][K2] complex64 (device, read)
 *   m1  [N0][N1][N2] float32 (device, written): m_nt
 *   v1  [3][K0][K1][K2] complex64 (device, written) or NULL: v_nt */
int lddmm_shoot(const lddmm_params* p, const float* I0, const void* v0, float* m1, void* v1,
                void* ws, size_t ws_bytes, void* stream);

/* Bytes of the library's own device array that lddmm_shoot_static works in. */
#define LDDMM_STATIC_SCRATCH_BYTES ((size_t)128 << 20)

/* lddmm_shoot without a workspace argument, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid allocation): the same computation, arguments and outputs as
 * lddmm_shoot, working in LDDMM_STATIC_SCRATCH_BYTES of device memory that
 * the library holds as a fixed array, one copy per GPU, from its first use
 * on that GPU until the process ends (problems whose lddmm_workspace_bytes
 * exceeds that size, e.g. beyond 64^3 / band 16^3 / 10 steps, return
 * LDDMM_E_WORKSPACE before anything is enqueued).  It allocates nothing and
 * creates no stream or event: all work is enqueued on `stream`.  Every call
 * on one GPU uses that GPU's array and leaves its contents behind; nothing
 * in it needs to start at zero, and calls that overlap on one GPU (from
 * several host threads or streams) race. */
int lddmm_shoot_static(const lddmm_params* p, const float* I0, const void* v0, float* m1, void* v1,
                       void* stream);

/* Band symbols of lddmm_apply_symbol */
enum { LDDMM_SYMBOL_L = 0, LDDMM_SYMBOL_K = 1 };

/* out = L~ in (which = LDDMM_SYMBOL_L) or K~ in (LDDMM_SYMBOL_K) on a band field
 * (paper §3.1: the band symbols of L = (Id - alpha Laplacian)^s and K = L^-1).
 * Converts a V-metric gradient g_V into the l2 gradient L~ g_V that is the
 * derivative of the energy with respect to the real and imaginary parts of
 * v0 (and back).  in and out: [3][K0][K1][K2] complex64 (device); in is
 * projected onto Hermitian fields on the effective band; out may alias in.
 * Overwrites the workspace's scratch fields (not the trajectories that
 * lddmm_hessvec uses). */
int lddmm_apply_symbol(const lddmm_params* p, int32_t which, const void* in, void* out, void* ws,
                       size_t ws_bytes, void* stream);

/* Geodesic energies E_n = <L~ v_n, v_n>_l2, n = 0..nt, in FP64, along the band
 * trajectory that lddmm_shoot would follow from v0 with the same parameters
 * (paper §2.2: constant along the exact geodesic; an Euler step changes it by
 * dt^2 <a_n, K~ a_n>, a_n = ad~*_{v_n}(L~ v_n), an RK4 step by O(dt^5)).  The
 * conservation check of the shooting; no image is involved.
 *   v0        [3][K0][K1][K2] complex64 (device, read)
 *   energies  nt + 1 doubles (device, written) */
int lddmm_geodesic_energy(const lddmm_params* p, const void* v0, double* energies, void* ws,
                          size_t ws_bytes, void* stream);

/* Energy and gradient in the V metric (paper §3.2: energy, the reduced
 * adjoint Jacobi equations in the band with U(1) = K~ pi(lambda(1) grad
 * m(1)), lambda(1) = -(2/sigma^2)(m(1) - I1) from §2.3), integrated backward
 * by the transpose of the Euler steps:
 *   w_n = w_{n+1} + dt [U_{n+1} - ad~_{v_n} w_{n+1} + K~ ad~*_{w_{n+1}}(L~ v_n)],
 *   U_n = U_{n+1} + dt K~ ad~*_{v_n}(L~ U_{n+1}),  g_V = v0 + w_0.
 * grad m(1) is the periodic central difference.
 *   I0, I1   [N0][N1][N2] float32 (device, read)
 *   v0       [3][K0][K1][K2] complex64 (device, read)
 *   grad     [3][K0][K1][K2] complex64 (device, written): g_V
 *   energy3  3 doubles (device, written): E, E_reg, E_data; may be NULL
 * Leaves in `ws` the trajectories lddmm_hessvec needs (prepares it). */
int lddmm_gradient(const lddmm_params* p, const float* I0, const float* I1, const void* v0,
                   void* grad, double* energy3, void* ws, size_t ws_bytes, void* stream);

/* Energy only (paper §3.2, band-limited energy): E, E_reg, E_data of v0,
 * by shooting and transport without the caches of the gradient (the
 * forward pass of the autograd form, whose backward is
 * lddmm_gradient_exact).  Arguments as for lddmm_gradient; energy3 (device,
 * 3 doubles) is required.  Accepts params->checkpoint, so that one
 * checkpointed workspace serves both passes. */
int lddmm_energy(const lddmm_params* p, const float* I0, const float* I1, const void* v0, double* energy3,
                 void* ws, size_t ws_bytes, void* stream);

/* Energy and the exact derivative of the discrete energy in the V metric
 * (paper §3.2 energy and constraints as discretised here: explicit Euler
 * steps of the band EPDiff, one semi-Lagrangian transport step per time
 * step): every step is differentiated in reverse order,
 *   state adjoint     lam_nt = 2/(sigma^2 |N|) (m_nt - I1), lam_n = I^T[lam_{n+1}]
 *                     (transpose of the trilinear interpolation at X_n = x - dt v_n(x)),
 *   velocity source   S_n = K~ |N| pi(-dt N_j lam_{n+1} (d_j I[m_n])(X_n)), the exact
 *                     slope of the interpolant in the cell of X_n,
 *   band adjoint      w_n = w_{n+1} + dt [-ad~_{v_n} w_{n+1} + K~ ad~*_{w_{n+1}}(L~ v_n)] + S_n,
 *                     w_nt = 0, g_V = v0 + w_0.
 * This is the derivative that finite differences of the energy see (the
 * gradient of lddmm_gradient is the paper's adjoint Jacobi gradient, which
 * discretises the continuous adjoint instead; the two differ by the band
 * truncation of the coadjoint transport and by O(dt) and O(h)).  The
 * scatter uses FP32 atomic additions, so the last bits vary between runs.
 * Honours params->checkpoint (see lddmm_params).  Arguments as for
 * lddmm_gradient; does not prepare the workspace for lddmm_hessvec. */
int lddmm_gradient_exact(const lddmm_params* p, const float* I0, const float* I1, const void* v0,
                         void* grad, double* energy3, void* ws, size_t ws_bytes, void* stream);

/* Hessian-vector product in the V metric at the v0 of the last
 * lddmm_gradient on this workspace with equal parameters (paper §3.2: the
 * incremental EPDiff and incremental state equations forward, then the
 * reduced incremental adjoint Jacobi equations backward from
 * dU(1) = K~ pi(dlambda(1) grad m(1)), dlambda(1) = -(2/sigma^2) dm(1)):
 *   dv_{n+1} = dv_n - dt K~[ad~*_{dv_n}(L~ v_n) + ad~*_{v_n}(L~ dv_n)]
 *   dm_{n+1} = I[dm_n - dt grad m_n . iota(dv_n)](x - dt iota(v_n)(x)), dm_0 = 0
 *   dU_n = dU_{n+1} + dt K~[ad~*_{v_n}(L~ dU_{n+1}) + ad~*_{dv_n}(L~ U_{n+1})]
 *   dw_n = dw_{n+1} + dt[dU_{n+1} - ad~_{v_n} dw_{n+1} - ad~_{dv_n} w_{n+1}
 *                       + K~ ad~*_{dw_{n+1}}(L~ v_n) + K~ ad~*_{w_{n+1}}(L~ dv_n)]
 *   Hdv = dv0 + dw_0
 * (terms with U or w are dropped under LDDMM_GN_CLASSICAL; LDDMM_NEWTON adds
 * lambda(1) grad dm(1) to the source of dU(1), lambda(1) = -(2/sigma^2)(m(1) - I1)
 * from the gradient's I1).
 *   dv0  [3][K0][K1][K2] complex64 (device, read)
 *   Hdv  [3][K0][K1][K2] complex64 (device, written; may not alias dv0)
 * Returns LDDMM_E_NOT_PREPARED if no such gradient preceded it. */
int lddmm_hessvec(const lddmm_params* p, const void* dv0, void* Hdv, void* ws, size_t ws_bytes,
                  void* stream);

/* Gauss-Newton-Krylov registration (paper §2.7): for each iteration, the
 * gradient, then `pcg_iters` iterations of CG in the V metric on
 * H_V p = -g_V from p = 0 (stopping early on non-positive curvature, in which
 * case the first iteration returns p = -g_V), then an Armijo search
 * (eps = 1, 1/2, ..., at most 10 trials, c1 = 1e-4) and v0 <- v0 + eps p.
 *   I0, I1    [N0][N1][N2] float32 (device, read)
 *   v0_inout  [3][K0][K1][K2] complex64 (device, read and written): the start
 *             iterate (zero for a fresh registration) and the result
 *   stats     host array of `stats_len` entries (one per iteration) or NULL
 * Synchronous: the host takes the loop's decisions from scalars that a
 * kernel writes to 512 bytes of pinned host memory that the calling host
 * thread holds until it exits (the block then serves a later thread; blocks
 * are kept until the process ends; copies and stream synchronisation instead
 * if that memory cannot be allocated).  Returns LDDMM_OK, LDDMM_W_LINESEARCH
 * (stopped early on a failed search; v0 holds the last accepted iterate) or
 * an error. */
int lddmm_register(const lddmm_params* p, const float* I0, const float* I1, void* v0_inout,
                   int32_t gn_iters, int32_t pcg_iters, lddmm_stats* stats, int32_t stats_len,
                   void* ws, size_t ws_bytes, void* stream);

/* Number of Hessian-vector products the last lddmm_register (or, summed over
 * its pairs, lddmm_register_batch) on this thread evaluated (host only). */
int64_t lddmm_last_register_hvps(void);

/* Bytes of device workspace for lddmm_register_batch on these n parameter
 * sets: the sum over pairs of lddmm_workspace_bytes rounded up to 256.  Host
 * only.  Returns LDDMM_OK or the first validation error (detail names the
 * pair). */
int lddmm_batch_workspace_bytes(int32_t n, const lddmm_params* p, size_t* bytes);

/* Many independent registrations in one call (the atlas-serving form of the
 * Gauss-Newton-Krylov loop of §2.7): pair i has its own parameters p[i]
 * (sizes, band, state and Hessian mode may differ), images I0[i], I1[i] and
 * iterate v0_inout[i], and runs exactly the loop of lddmm_register, so its
 * results equal those of lddmm_register on the same inputs.  Up to
 * `concurrency` pairs run at a time (0 selects 8), each on one library stream
 * of its own (a pair's grid chain follows its band chain on that stream), so
 * that the launches of different pairs share the compute units; pairs start
 * largest first (by workspace size).  The calling thread drives every pair:
 * each pair's loop is suspended while it waits for a value from the device
 * and resumed once that value is there, so no pair's host work waits for
 * another's device work.  With lddmm_use_graphs(1) each pair replays its
 * captured sequences (Gauss-Newton head, CG iteration, line-search trials);
 * pair i takes the i-th block of pinned host words from the library's pool
 * (allocated on first use, kept until the process ends), so a repeated call
 * on the same workspace replays the graphs of the previous one.
 *   n          1 <= n <= 4096
 *   p, I0, I1, v0_inout   host arrays of n entries; the images and iterates are
 *              device buffers laid out as for lddmm_register
 *   stats      host array [n][stats_len] or NULL; status: host array [n] or
 *              NULL (per-pair return code); hvps: host array [n] or NULL
 *   ws         one device workspace of ws_bytes >= lddmm_batch_workspace_bytes();
 *              pair i uses the slice that starts after the slices of pairs < i
 * The pairs start after the work already enqueued on `stream`; the call is
 * synchronous.  Returns LDDMM_OK, LDDMM_W_LINESEARCH if a pair stopped on a
 * failed search, or the error of the lowest-numbered failing pair (every pair
 * is still attempted; argument errors are found before anything runs). */
int lddmm_register_batch(int32_t n, const lddmm_params* p, const float* const* I0, const float* const* I1,
                         void* const* v0_inout, int32_t gn_iters, int32_t pcg_iters, int32_t concurrency,
                         lddmm_stats* stats, int32_t stats_len, int32_t* status, int64_t* hvps, void* ws,
                         size_t ws_bytes, void* stream);

/* Launch timing of one kernel, for roofline accounting.  While enabled,
 * one launch in `every` on average (all of them for every = 1; otherwise
 * those whose sequence number among the launches of that kernel this
 * process makes hashes to a multiple of `every`, so that the sample does not
 * follow a period of the launch sequence) of kernel family `family`
 * (LDDMM_KF_*) is bracketed by HIP events on its stream, and the
 * algorithmic work of those launches (flops of the partial DFT contractions,
 * Lie products and interpolation; HBM bytes of their inputs and outputs, each
 * read or written once) is summed.  lddmm_kernel_timer_read synchronises the
 * events and returns the number of timed launches, their summed duration in
 * milliseconds and their summed algorithmic flops and bytes.  Enabling (or
 * LDDMM_KF_NONE) resets the counters.  `every` must be in [1, 1000] and
 * `family` in [0, LDDMM_KF_SRC] (else LDDMM_E_INVALID_ARG).  With graphs on
 * (lddmm_use_graphs), the sampled launches are fixed when a sequence is
 * captured and carry event nodes in its graph.  Host only; not thread-safe
 * against concurrent enabling. */
enum {
  LDDMM_KF_NONE = 0,
  LDDMM_KF_SYNTH = 1,      /* k_synth: padded-grid synthesis of new fields (inverse stages 1-2, MFMA) */
  LDDMM_KF_GRID = 2,       /* k_gridstep: grid velocity / incremental-state source (inverse stages 1-2) */
  LDDMM_KF_SL = 3,         /* k_sl: semi-Lagrangian transport step */
  LDDMM_KF_INV0 = 4,       /* k_inv0 (padded grid): inverse stage 0 at the start of a sweep */
  LDDMM_KF_COLUMN = 5,     /* k_colstep: forward stages 1-0, band update, next inverse stage 0 */
  LDDMM_KF_PRODS = 6,      /* k_prods: Lie products and forward stage 2 on the padded grid */
  LDDMM_KF_INV0_GRID = 7,  /* k_inv0 (image grid): inverse stage 0 of a grid velocity */
  LDDMM_KF_FWD1_GRID = 8,  /* k_fwd1: forward stage 1 of a grid field */
  LDDMM_KF_FWD0_GRID = 9,  /* k_fwd0: forward stage 0 of a grid field and its band epilogue */
  LDDMM_KF_SRC = 10        /* k_src_fwd2: image-matching source and forward stage 2 */
};
int lddmm_kernel_timer(int32_t family, int32_t every);
int lddmm_kernel_timer_read(int64_t* launches, double* total_ms, double* flops, double* bytes);

/* Graph replay of the launch-bound sequences (default off).  With graphs on,
 * lddmm_hessvec and the per-iteration sequences of lddmm_register (the
 * gradient at the head of a Gauss-Newton iteration, one CG iteration, one
 * line-search trial) are captured into a HIP graph on a library-owned stream
 * the first time they run for a given device, workspace, problem, external
 * input pointers and timed kernel family, and replayed on the caller's
 * stream afterwards; the kernels and their order are the same as without.
 * Captures run one at a time across host threads (the pairs of
 * lddmm_register_batch capture their own graphs in turn).  The CG iteration's
 * graph also holds the calling thread's pinned host words (see
 * lddmm_register), so each block of words has its own; successive batched
 * calls give pair i the same block and therefore the same graphs.  The
 * graphs are keyed by the state and integrator too, so calls on one
 * workspace that differ only in those never share a graph.  The captured graphs hold workspace addresses: a workspace that is freed
 * and reallocated at the same address with the same problem reuses them,
 * which is correct because all of its buffers are recomputed.  Graphs live
 * until the process ends.  `enable` must be 0 or 1 (else
 * LDDMM_E_INVALID_ARG).  Process-wide; host only. */
int lddmm_use_graphs(int32_t enable);

/* Launch shapes of three kernel families for one problem shape (the tile
 * table).  They change which thread blocks compute what, never the
 * arithmetic of an output: results are bitwise those of the built-in rule.
 *   prod_rows   padded-grid rows per block of the pointwise Lie products
 *               (1 .. floor(256 / M2), capped at M1; 0: the largest)
 *   col_split   band column steps: 0 the built-in rule, 1 one block per
 *               column tile, 2 two blocks per tile sharing its next-stage
 *               outputs, 3 as 2 with the lean kernel for the forward
 *               sweeps where the shape has one (bands 24^3 and 32^3)
 *   sl_threads  threads per block of the semi-Lagrangian transport step:
 *               64, 128 or 256 (0: 256) */
typedef struct {
  int32_t prod_rows;
  int32_t col_split;
  int32_t sl_threads;
} lddmm_tiles;

/* The tile table: one entry per (grid, band, spectral grid, precision,
 * arch), e.g. arch "gfx950".  Every call reads the entry for its parameters
 * on the current device, if any; else the built-in rule applies.
 * lddmm_tiles_set: sets the entry for p's shape and precision (the other
 * fields of p are only validated); arch NULL names the current device's.
 * LDDMM_E_INVALID_ARG for fields out of range.
 * lddmm_tiles_get: *found = 1 and the entry, or *found = 0 and zeros.
 * lddmm_tiles_clear: empties the table.
 * lddmm_tiles_save / lddmm_tiles_load: the table as a JSON file
 *   {"format": "lddmm-tiles-1", "entries": [{"arch": "gfx950",
 *    "grid": [N0, N1, N2], "band": [K0, K1, K2], "spectral": [M0, M1, M2],
 *    "precision": "fp32" | "bf16x3", "prod_rows": r, "col_split": c,
 *    "sl_threads": t, "ms_per_hvp": x}, ...]}
 * (load merges into the table; every entry is validated before any is
 * taken, and a malformed file changes nothing and returns
 * LDDMM_E_INVALID_ARG).  Process-wide, thread-safe; host only. */
int lddmm_tiles_set(const lddmm_params* p, const char* arch, const lddmm_tiles* t);
int lddmm_tiles_get(const lddmm_params* p, const char* arch, lddmm_tiles* t, int32_t* found);
int lddmm_tiles_clear(void);
int lddmm_tiles_save(const char* path);
int lddmm_tiles_load(const char* path);

/* Autotuner of the tile table for one problem (the Hessian-vector product of
 * §2.7's CG is the measure): runs the gradient at v0 with the built-in rule
 * (leaving ws prepared for lddmm_hessvec, as lddmm_gradient does), then times
 * `reps` products (direction v0, after one untimed product) for the built-in
 * rule and for each candidate of one field at a time (sl_threads 64, 128;
 * prod_rows 1 .. max - 1; col_split 1, 2, 3), keeping a candidate when it is
 * at least 1 % faster than the choice so far.  The winner is stored in the
 * table for p's shape on the current device and returned in *best, its time
 * per product (ms) in *ms_best and the built-in rule's in *ms_default (each
 * may be NULL).  Synchronous.
 *   I0, I1  [N0][N1][N2] float32 (device, read); v0 [3][K0][K1][K2]
 *           complex64 (device, read); 1 <= reps <= 1000 */
int lddmm_autotune(const lddmm_params* p, const float* I0, const float* I1, const void* v0, int32_t reps,
                   lddmm_tiles* best, double* ms_best, double* ms_default, void* ws, size_t ws_bytes,
                   void* stream);

/* Static description of a status code. */
const char* lddmm_status_string(int code);
/* Thread-local detail of the last failure on this thread ("" if none). */
const char* lddmm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LDDMM_H */
