// Host engine: workspace layout and the time loops of shooting, transport,
// the adjoint Jacobi gradient, the incremental adjoint Jacobi
// Hessian-vector product and the Gauss-Newton-Krylov loop.
#pragma once

#include <functional>
#include <vector>

#include "common.h"

namespace lddmm {

// Carves named buffers out of the caller's workspace.  With base == nullptr
// it only accumulates the size.
struct Carver {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

// Destroys the auxiliary streams and events of the calling thread (worker
// threads that end call it; the stream must be idle).
void release_thread_streams();

class Engine {
 public:
  Engine(const Dims& d, void* ws, hipStream_t st);
  static size_t workspace_bytes(const Dims& d);

  hipError_t init_tables();
  // band I/O in the caller's full layout
  hipError_t load_band(const void* full, float2* half);
  hipError_t store_band(const float2* a, const float2* b, float cb, void* full, const float* sym = nullptr);

  // Called after the band step that produces v_n has been enqueued.
  using StepHook = std::function<hipError_t(int)>;
  // Band shooting from V[0] (fills V[1..nt]; caches the padded-grid fields
  // when `cache`); `hook(n)` after the step that makes V[n].
  hipError_t shoot_band(bool cache, const StepHook& hook = StepHook());
  // Shooting with caches, grid velocities vg[n] and states m[0..nt].
  hipError_t forward(const float* I0);
  // Shooting and transport without caches; *m_out = m_nt.
  hipError_t forward_light(const float* I0, const float** m_out);
  // Band shooting by classical RK4 steps from V[0] (no caches).
  hipError_t shoot_band_rk4();
  // <L~ v_n, v_n> (FP64) for n = 0..nt into out[0..nt] (device), after shooting
  // with the integrator of the parameters.
  hipError_t geodesic_energies(double* out);
  // E, E_reg, E_data of (V[0], m_nt) into scal[0..2] (device).
  hipError_t energy(const float* mnt, const float* I1);
  // U, W sweeps from m_nt; g_V = V[0] + W[0] into g_out (half) if non-null.
  hipError_t backward(const float* I1, float2* g_out);
  // Hessian-vector product on half-spectrum vectors.
  hipError_t hessvec(const float2* dvh, float2* out);
  // Exact derivative of the discrete energy (reverse sweep of every Euler and
  // transport step) after `forward` (or `forward_ckpt` with checkpoints):
  // g_V = V[0] + W[0] into g_out (half); the per-step band sources go to U[n].
  hipError_t backward_exact(const float* I1, float2* g_out);
  // Gauss-Newton product of the exact discrete energy, (J^T W J + Id) dv in
  // the V metric, at the v0 of the last forward (no checkpoints): the
  // linearised Euler steps and the tangent of every transport step, then the
  // reverse sweep of backward_exact from the state adjoint W dm_nt.
  hipError_t hessvec_exact(const float2* dvh, float2* out);
  // Shooting with caches; with checkpoints only the states m_{kc} and m_nt
  // are kept (final_state() is m_nt).
  hipError_t forward_ckpt(const float* I0);

  // m(1) of the last forward: m_nt (image state) or I0 o phi(1) (deformation state).
  const float* final_state() const { return d_.state ? m1 : (d_.ckpt ? mfin_ : m[d_.nt]); }

  const Dims& dims() const { return d_; }
  // Second stream of this thread and device for the grid chain, and events.
  hipError_t aux_init(int nevents);
  hipStream_t stream() const { return st_; }
  // Redirects all further work (used while capturing a graph).
  void set_stream(hipStream_t s) { st_ = s; }
  // Runs the grid chain on the caller's stream too (the host enqueues every
  // step after the work it depends on, so one stream keeps the order).
  void set_one_stream(bool on) { one_stream_ = on; }

  // buffers
  std::vector<float2*> V, U, W, dV;
  float2 *dU[2], *dW[2];
  float2 *gh, *ph, *rh, *dh, *Hdh, *v0h, *vtry, *tmph;
  std::vector<float*> VG, UG, WG, dVG;
  std::vector<float*> m, vg;
  float *dm[2], *q;
  float* resid;  // m(1) - I1 of the last gradient (full Newton only)
  // deformation state: band displacements u_0..u_nt, incremental pair,
  // their padded-grid groups (PG[1..nt]), rho~ (R, K~ R), its group, drho~,
  // iota(u_nt) and iota(du_nt) on the image grid, m(1), a copy of I0 and its
  // derivatives
  std::vector<float2*> Phi;
  float2* dPhi[2];
  std::vector<float*> PG;
  float* RG;
  float2 *R, *KR, *dR, *KdR;
  float *ug, *dug, *m1, *I0c, *IG, *IH;  // IG [nN][4]: I0 and its central differences; IH [nN][8]: Hessian
  float *mlight[2];
  double *partial, *scal, *pcg;
  unsigned* count;  // zero counter of the one-launch reductions (zeroed with the tables)
  float *Lsym, *Ksym;

 private:
  void layout(Carver& c);
  float2* t1(int g, int c) const;
  const float2* s1(int o) const;
  const float2* s2n(int o) const;
  hipError_t inv0_groups(const float2* in0, int l0, const float2* in1, int l1);
  hipError_t mstep(int prog, int nout, float* store0, float* store1, const float* const* cached);
  ColJob col_job(int c, int oa, float ca, int syma, int ob, float cb, int symb, const float2* base,
                 const float2* extra, float ce, float2* out, int g0, int l0, int g1, int l1,
                 float2* t1n = nullptr) const;
  hipError_t colstep(const ColJob* jobs, int n);
  hipError_t fwd_grid(Fwd0Job* jobs, int njobs, hipStream_t s);

  hipError_t record(hipStream_t s, int ev);
  hipError_t wait(hipStream_t s, int ev);
  hipError_t grid_stage0(const float2* band, float2* t1n, hipStream_t s);
  hipError_t tail(const float* a, const float* b, const float* r, float coef, float2* out,
                  const float2* zero_band, hipStream_t s);
  hipError_t grid_t1(int n, const float2* band, hipStream_t s);
  hipError_t grid_velocity(int n, float* out, hipStream_t s);
  hipError_t grid_source(int n, const float* dmn, hipStream_t s);
  // deformation state (paper §3.3)
  hipError_t forward_def(const float* I0);
  hipError_t forward_rk(const float* I0, const float** m_out);
  hipError_t tail_def(const float* I1);
  hipError_t hessvec_def(const float2* dvh, float2* out);
  hipError_t hessvec_sweep(float2* out);
  hipError_t inv0_group(const float2* in, int g, int lflag, hipStream_t s);
  hipError_t colstep_on(const ColJob* jobs, int n, hipStream_t s);
  hipError_t prods_on(int prog, const float* const* g, int ng, float2* out, hipStream_t s);
  hipError_t grid_field(const float2* band, bool have_t1n, float* out, hipStream_t s);
  hipError_t band_pair(float2* plain, float2* smooth, hipStream_t s);
  hipError_t def_head(int prog, const float* const* g, int ng, const float2* base, float2* out);

  Dims d_;
  hipStream_t st_;
  hipStream_t aux_ = nullptr;
  bool one_stream_ = false;
  std::vector<hipEvent_t>* ev_ = nullptr;
  Twiddles twM_{}, twN_{};
  float2* twbuf_ = nullptr;
  float2 *T1_ = nullptr, *S1_ = nullptr, *S1N_ = nullptr, *S2N_ = nullptr;
  float2 *T1NA_ = nullptr, *S1A_ = nullptr;  // displacement chain: image-grid stage 0, products
  float* NGA_ = nullptr;                     // displacement chain: scratch for two groups
  std::vector<float2*> T1N;     // image-grid stage-0 output of each time step [3][N0][Kh][K1]
  bool fuse_grid0_ = false;     // the column kernel forms T1N[n + 1]
  float* NG_ = nullptr;         // scratch for new groups that are not cached
  // with checkpoints (d_.ckpt = c > 0): m[k] = m_{kc}; mseg_[i] = m_{sc+i} of the
  // segment being recomputed; mfin_ = m_nt
  std::vector<float*> mseg_;
  float* mfin_ = nullptr;
  // where state n lives in the checkpointed layout (nullptr: not kept now)
  float* ckpt_state(int n) const;
  hipError_t grid_velocity_ckpt(int n, float* out, hipStream_t s);
  // reverse sweep of backward_exact from the state adjoint (over coef) in dm[cur]
  hipError_t adjoint_exact(int cur);
  float* dvg_ = nullptr;  // grid velocity increment of one step [3][nN] (exact product)
  float* synth_tab_ = nullptr;  // MFMA-form stage-1/2 twiddles of the padded grid
  float2* col_tab_ = nullptr;   // MFMA-form twiddles of the column step
};

}  // namespace lddmm
