// Shared declarations of the HIP library: problem dimensions, kernel job
// descriptors and the launch wrappers the host engine calls.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lddmm {

constexpr int kMaxBand = 64;   // K_j upper bound
constexpr size_t kMaxLds = 160 * 1024;  // LDS of one workgroup on gfx950
constexpr int kMaxJobs = 32;   // jobs per batched launch

// Problem sizes.  Band fields are kept internally as the half spectrum
// [3][Kh][K0][K1] (k2 = 0..K2/2-1 slowest, k1 fastest), complex float; the
// negative-k2 half follows from Hermitian symmetry.  A column step owns one
// k2 and 16 k1, so its band reads and writes are rows of 16 consecutive k1.
struct Dims {
  int N[3], K[3], M[3];
  int Kh;           // K[2] / 2
  int nb;           // K0 * K1 * Kh, complex values per component
  long long nN;     // grid points
  long long nM;     // padded spectral grid points
  int nt;
  int s;
  double alpha, sigma;
  int hessian;      // 0: couplings kept (paper reading), 1: dropped, 2: full Newton
  int state;        // 0: image state on the grid; 1: deformation state in the band
  int integrator;   // 0: Euler; 1: RK4 shooting with midpoint transport (shooting only)
  int prec;         // 0: FP32 matrix-core products; 1: compensated BF16 (three products)
  int ckpt;         // 0: every state kept; c > 0: states every c steps (exact gradient only)
  // launch shapes from the tile table (0: the built-in rule); they change
  // which blocks do what, never the arithmetic of an output
  int tile_prod_rows;  // padded-grid rows per block of k_prods
  int tile_col;        // column step: 1 one block per column tile, 2 two (general kernel), 3 two (lean kernel where it applies)
  int tile_sl;         // threads per block of k_sl (64, 128 or 256)
};

// Valid range of the tile fields for a shape (host only).
int prod_rows_max(const Dims& d);

// ---------------------------------------------------------------- tables
// Twiddle tables for one transform direction set (grid G = M or N).
struct Twiddles {
  const float2* inv0;  // [2][G0][K0]  exp(+2 pi i k x/G), variant 1 times 2 pi i k
  const float2* inv1;  // [2][G1][K1]
  const float2* inv2;  // [2][G2][Kh]  weight 1 (k2 = 0) or 2 folded in
  const float2* fwd0;  // [K0][G0]     exp(-2 pi i k x/G)
  const float2* fwd1;  // [K1][G1]
  const float2* fwd2;  // [Kh][G2]
  int G[3];
};

// ---------------------------------------------------------------- jobs
struct Inv0Job {
  const float2* in;   // band half spectrum of one component [Kh][K0][K1]
  float2* out;        // [nvar][G0][Kh][K1]
  int lflag;          // multiply the input by L~ on load
};
struct Inv0Jobs { Inv0Job j[kMaxJobs]; };

// Program of the padded-grid products kernel: which band-limited Lie
// products to form at each point.
enum MProg {
  PROG_STORE = 0,   // only synthesise (and store) the new groups
  PROG_SHOOT = 1,   // out0 = ad*_V(LV)                         new: V, LV
  PROG_H1 = 2,      // out0 = ad*_dV(LV) + ad*_V(LdV)           new: dV, LdV; cached: V, LV
  PROG_GRAD = 3,    // out0 = ad*_V(LU), out1 = ad_V(W), out2 = ad*_W(LV)
                    //                                          new: LU, W; cached: V, LV
  PROG_H5 = 4,      // out0 = ad*_V(LdU) + ad*_dV(LU)
                    // out1 = ad_V(dW) + ad_dV(W)
                    // out2 = ad*_dW(LV) + ad*_W(LdV)
                    //                   new: LdU, dW; cached: V, LV, LU, W, dV, LdV
  PROG_H5_NOCOUPLE = 5, // out0 = ad*_V(LdU), out1 = ad_V(dW), out2 = ad*_dW(LV)
  // deformation state (D~A * B)_i = sum_j (d_j A_i) B_j, ((D~A)^T * B)_j = sum_i (d_j A_i) B_i:
  PROG_DEF_FWD = 6,     // out0 = D~Phi * V                             new: Phi; cached: V
  PROG_DEF_H = 7,       // out0 = D~dPhi * V + D~Phi * dV               new: dPhi; cached: V, Phi, dV
  PROG_DEF_TAIL = 8,    // out0 = (D~A)^T * R                           new: A and/or R
  PROG_DEF_HTAIL = 9,   // out0 = (D~dPhi)^T * R + (D~Phi)^T * dR       new: dPhi, dR; cached: Phi, R
  // exact adjoint sweep (no U recursion):
  PROG_ADJ = 10         // out0 = ad_V(W), out1 = ad*_W(LV)              new: W; cached: V, LV
  // k_prods group order: SHOOT (V, LV); H1 (dV, LdV, V, LV); GRAD (LU, W, V, LV);
  // H5 (LdU, dW, V, LV, LU, W, dV, LdV); H5_NOCOUPLE (LdU, dW, V, LV);
  // DEF_FWD (Phi, V); DEF_H (dPhi, V, Phi, dV); DEF_TAIL (A, R); DEF_HTAIL (dPhi, dR, Phi, R).
  // Of a group that enters through its Jacobian only the nine derivative
  // fields are read, of one that enters through its values only the three values.
};

// Lie products on the padded grid (k_prods): group pointers ([3][nM][4]:
// per component and point the value and its three derivatives) in the
// order the program names them (see MProg).
struct ProdArgs {
  const float* g[8];
  float2* s1;  // [nout][Kh][M0][M1]
  int nout, prog;
};

// Band-side step of one output component (k_colstep): forward stages 1 and
// 0 of one or two product fields s1 ([Kh][M0][M1] each), the update
// out = base + ca*(K~ if syma)*F(a) + cb*(K~ if symb)*F(b) + ce*extra, the
// inverse stage 0 of out (of L~ out where t1l) into up to two padded-grid
// stage-0 buffers [2 vars][M0][Kh][K1] for the next step, and, if t1n is
// set, the image-grid inverse stage 0 of out into t1n [N0][Kh][K1].
struct ColJob {
  const float2* a;
  const float2* b;
  const float2* base;
  const float2* extra;
  float2* out;
  float2* t1[2];       // [2 vars][M0][Kh][K1]
  float2* t1n;         // [N0][Kh][K1] or null
  float ca, cb, ce;
  int syma, symb;
  int t1l[2];
  int nt1;
};
struct ColJobs {
  ColJob j[8];
  const float2* w0n;   // image-grid stage-0 inverse twiddles [N0][K0] (for t1n)
  int N0;
};

struct Fwd1Job { const float2* in; float2* out; };   // [G0][G1][Kh] -> [G0][Kh][K1]
struct Fwd1Jobs { Fwd1Job j[kMaxJobs]; };

// out = base + ca*(K~ if syma)*F(a) + cb*(K~ if symb)*F(b) + ce*extra, per
// band point; F is the last forward stage with the 1/|G| normalisation.
struct Fwd0Job {
  const float2* a;
  const float2* b;
  const float2* base;
  const float2* extra;
  float2* out;
  float2* out2;  // optional (a alone, syma = 0): ca K~ F(a) / |N| beside out
  float ca, cb, ce;
  int syma, symb;
};
struct Fwd0Jobs { Fwd0Job j[kMaxJobs]; };

struct GridStepArgs {
  const float2* t1;   // [3][N0][Kh][K1]
  int op;             // 0: write the velocity; 1: incremental-state source
  float* vout;        // op 0: [3][nN]
  const float* m;     // op 1: state m_n
  const float* dm;    // op 1: incremental state dm_n (null: zero)
  float* q;           // op 1: dm_n - dt grad_h m_n . dv_n
  float dt;
};

// ------------------------------------------------------- launch wrappers
// Each returns hipSuccess or the launch error.
hipError_t launch_twiddles(float2* dst, int K, int G, int mode, hipStream_t st);
hipError_t launch_symbols(float* Lsym, float* Ksym, const Dims& d, hipStream_t st);
hipError_t launch_full_to_half(const float2* full, float2* half, const Dims& d, hipStream_t st);
// full = expand(a + cb b), times the band symbol sym when given
hipError_t launch_half_to_full(const float2* a, const float2* b, float cb, float2* full,
                               const Dims& d, hipStream_t st, const float* sym = nullptr);
// Inverse stage 0; `trans` writes the padded-grid layout [v][x0][kh][k1]
// instead of [v][x0][k1][kh].
// Output [nvar][G0][Kh][K1]; image_grid selects the timer family of the launch.
hipError_t launch_inv0(const Inv0Jobs& jobs, int njobs, int nvar, const float2* tw, const float* Lsym,
                       int K0, int C, int G0, int Kh, bool image_grid, hipStream_t st);
hipError_t launch_synth_tables(const Twiddles& tw, float* tables, const Dims& d, hipStream_t st);
size_t synth_table_floats(const Dims& d);
size_t synth_shared_bytes(const Dims& d);
// Synthesis of group 0 and, when t1g1 is set, group 1.
hipError_t launch_synth(const float2* t1g0, const float2* t1g1, float* dst0, float* dst1,
                        const float* tables, const Dims& d, hipStream_t st);
size_t prods_shared_bytes(const Dims& d, int nout);
hipError_t launch_prods(const ProdArgs& a, const Dims& d, const Twiddles& tw, hipStream_t st);
hipError_t launch_colstep(const ColJobs& jobs, int njobs, const Dims& d, const Twiddles& tw,
                          const float2* coltab, const float* Lsym, const float* Ksym, hipStream_t st);
size_t col_table_count(const Dims& d);
// Whether the column kernel can form the image-grid stage 0 (t1n) for this shape.
bool colstep_fuses_grid0(const Dims& d);
hipError_t launch_col_tables(const Twiddles& tw, float2* tab, const Dims& d, hipStream_t st);
size_t colstep_shared_bytes(const Dims& d);
hipError_t launch_fwd1(const Fwd1Jobs& jobs, int njobs, const float2* tw, int G0, int G1, int K1,
                       int Kh, hipStream_t st);
hipError_t launch_fwd0(const Fwd0Jobs& jobs, int njobs, const float2* tw, const float* Ksym, int G0,
                       int K0, int K1, int Kh, float invG, hipStream_t st);
hipError_t launch_gridstep(const GridStepArgs& a, const Dims& d, const Twiddles& tw, hipStream_t st);
hipError_t launch_sl(const float* src, const float* vel, float* dst, float dt, const Dims& d,
                     hipStream_t st);
// One transport step with midpoint departure points: vel is the mid-step
// velocity [3][nN]; dst(x) = src(x - dt vel(x - dt/2 vel(x))).
hipError_t launch_sl_rk2(const float* src, const float* vel, float* dst, float dt, const Dims& d,
                         hipStream_t st);
// Fused t = 1 tail on the tuned shapes: image-matching source (with the
// r d_j a term of the full Newton product when r is given), forward
// stages 2 and 1 (partial over 64-row chunks of x1) into P
// [nparts][3][Kh][N0][K1], then forward stage 0 with the K~/|N| epilogue into
// the band field `out`, and the padded-grid stage-0 buffers of the first
// backward step: group 0 from L~ out (t1u), group 1 zero (t1z).
bool tail_fused(const Dims& d);
size_t tail_parts_bytes(const Dims& d);
hipError_t launch_tail(const float* a, const float* b, const float* r, const float* m, float coef, float2* P,
                       float2* out,
                       float2* const t1u[3], float2* const t1z[3], const Dims& d, const Twiddles& twN,
                       const float2* coltab, const float* Lsym, const float* Ksym, hipStream_t st);
// s_j = coef [(a - b) d_j m + r d_j a]; b and r may be null.
hipError_t launch_src_fwd2(const float* a, const float* b, const float* r, const float* m, float coef,
                           float2* s1,
                           const Dims& d, const Twiddles& tw, hipStream_t st);
// Tangent of one transport step (see k_sl_tangent): out = I[dm](X) -
// dt sum_j N_j (d_j I[m])(X) dvel_j, X = x - dt vel(x); dm may be null (zero).
hipError_t launch_sl_tangent(const float* dm, const float* m, const float* vel, const float* dvel, float* out,
                             float dt, const Dims& d, hipStream_t st);
// Exact adjoint of one transport step (see k_adj_src_fwd2): lam_out += I^T
// [lam] (lam_out zeroed by the caller), and forward stage 2 of
// s_j = -dt N_j coef lam (d_j I[m])(x - dt vel(x)) into s1 [3][N0][N1][Kh].
hipError_t launch_adj_src_fwd2(const float* lam, const float* m, const float* vel, float* lam_out, float coef,
                               float dt, float2* s1, const Dims& d, const Twiddles& tw, hipStream_t st);
// Deformation state at t = 1 (see k_rho_fwd2): the image-term source at
// phi(1) = id + u and its forward stage 2 into s1 [3][N0][N1][Kh].
struct RhoArgs {
  const float* I0;
  const float* G;     // [nN][4]: I0 and its central-difference gradient per point
  const float* H;     // [nN][8]: its Hessian (00, 01, 02, 11, 12, 22, 0, 0), full Newton only
  const float* u;     // [3][nN] displacement iota(u_nt)
  const float* I1;    // op 0
  const float* du;    // op 1: [3][nN] iota(du_nt)
  const float* res;   // op 1, full Newton: m(1) - I1, or null
  float coef;
  int op;
};
// I0 with its central differences, G [nN][4] = (I0, d0, d1, d2), and, when H
// is set, H [nN][8] = (d00, d01, d02, d11, d12, d22, 0, 0).
hipError_t launch_image_derivs(const float* I0, float* G, float* H, const Dims& d, hipStream_t st);
hipError_t launch_rho_fwd2(const RhoArgs& a, float2* s1, const Dims& d, const Twiddles& tw, hipStream_t st);
hipError_t launch_fill(float* p, long long n, float v, hipStream_t st);
hipError_t launch_copy(const float* src, float* dst, long long n, hipStream_t st);
// Two-dimensional problems on the three-dimensional path: out [depth][plane] =
// in [plane] per plane; band out [3][kd][plane2] = in [2][plane2] placed in
// components 1, 2 at first-axis slot 0, zero elsewhere; and back.
hipError_t launch_embed_image(const float* in, float* out, long long plane, int depth, hipStream_t st);
// *out += number of i < n with a[i] and b[i] different bit for bit
hipError_t launch_count_ne(const float* a, const float* b, long long n, unsigned* out, hipStream_t st);
hipError_t launch_embed_band(const float2* in, float2* out, int kd, long long plane2, hipStream_t st);
hipError_t launch_extract_band(const float2* in, float2* out, int kd, long long plane2, hipStream_t st);
hipError_t launch_diff(const float* a, const float* b, float* out, long long n, hipStream_t st);  // a - b
hipError_t launch_axpy_band(const float2* x, const float2* y, float a, float2* out, int n,
                            hipStream_t st);   // out = x + a*y
// Reductions, deterministic two-pass; results in double on the device.
hipError_t launch_sqdiff(const float* a, const float* b, long long n, double* partial, double* out,
                         double scale, hipStream_t st);
// With `count` (a zero counter of the caller, left zero), one launch: the
// last block to finish sums the partials in the same order as the second pass
// and then, for post = 1 or 2, runs CG scalar phase a or b on `pcg` (phase b
// with the optional pinned host pair `host`).
hipError_t launch_band_dot(const float2* a, const float2* b, const float* Lsym, const Dims& d,
                           double* partial, double* out, double scale, hipStream_t st,
                           unsigned* count = nullptr, double* pcg = nullptr, int post = 0,
                           double* host = nullptr);
hipError_t launch_band_maxabs(const float2* a, const Dims& d, double* partial, double* out,
                              hipStream_t st);
hipError_t launch_scalar_copy(const double* src, double* dst, int n, hipStream_t st);
hipError_t launch_energy_combine(double* sc, hipStream_t st);  // sc[0] = sc[1] + sc[2]
size_t gridstep_shared_bytes(const Dims& d);
size_t src_shared_bytes(const Dims& d);
// CG in the V metric, all scalars on the device (see engine).
hipError_t launch_pcg_reset(double* sc, hipStream_t st);
hipError_t launch_pcg_init(const float2* g, float2* p, float2* r, float2* dvec, int n,
                           hipStream_t st);
hipError_t launch_pcg_update_pr(const double* sc, const float2* dvec, const float2* Hd, float2* p,
                                float2* r, int n, hipStream_t st);
// Copies a[0 .. na) and b[0 .. nb) (na + nb <= 63) of device memory to
// host[1 ..] of pinned host memory, then sets host[0] = 1.
hipError_t launch_host_copy(const double* a, int na, const double* b, int nb, double* host, hipStream_t st);
hipError_t launch_pcg_update_d(const double* sc, const float2* r, float2* dvec, int n,
                               hipStream_t st);

// Kernel-family timing (see lddmm_kernel_timer); one family per kernel.
enum KernelFamily {
  KF_SYNTH = 1, KF_GRID = 2, KF_SL = 3, KF_INV0 = 4, KF_COLUMN = 5, KF_PRODS = 6, KF_INV0_GRID = 7,
  KF_FWD1_GRID = 8, KF_FWD0_GRID = 9, KF_SRC = 10, KF_LAST = 10
};
// timer_work records the algorithmic flops and HBM bytes of the launch that
// follows and decides whether that launch is sampled; timer_events hands out
// the start/stop events a sampled launch carries (false when the launch is
// not sampled or a graph is being captured); timer_captured, after the
// launch, hands the kernel node of a sampled launch in a capture to the
// timer.  Each timed launch calls the three in this order.
void timer_work(int family, double flops, double bytes);
bool timer_events(int family, hipEvent_t* start, hipEvent_t* stop);
void timer_captured(int family, hipStream_t st);

// Scalar slots of the CG state.
enum PcgSlot {
  SC_RR = 0, SC_DHD = 1, SC_RRNEW = 2, SC_ALPHA = 3, SC_BETA = 4, SC_STOPPED = 5, SC_GUARD = 6,
  SC_ITERS = 7, SC_NEGG = 8, SC_DOUPD = 9, SC_COUNT = 16
};

}  // namespace lddmm
