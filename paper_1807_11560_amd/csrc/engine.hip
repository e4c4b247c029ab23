// Host engine of band-limited Jacobi PDE-EPDiff LDDMM (paper §3.2).
//
// Per Euler step on the padded grid the engine issues three launches: the
// MFMA synthesis of the new fields (inverse stages 1-2; k_synth), their Lie
// products with forward stage 2 (k_prods) and the column kernel (forward
// stages 1-0, the band update, and stage 0 of the next step's inverse
// transforms; k_colstep).  The first step of a sweep gets its stage 0 from k_inv0.
// Fields of the trajectory that later sweeps reuse are cached on the padded
// grid when they are first synthesised.
#include "engine.h"

#include <algorithm>
#include <map>

namespace lddmm {

#define TRY(x)                            \
  do {                                    \
    hipError_t e_ = (x);                  \
    if (e_ != hipSuccess) return e_;      \
  } while (0)

namespace {

size_t twiddle_count(const int* G, const Dims& d) {
  return 2 * (size_t)G[0] * d.K[0] + 2 * (size_t)G[1] * d.K[1] + 2 * (size_t)G[2] * d.Kh +
         (size_t)d.K[0] * G[0] + (size_t)d.K[1] * G[1] + (size_t)d.Kh * G[2];
}
}  // namespace

// Per thread and device: the auxiliary stream (default priority) and a
// pool of timing-free events; created on first use, kept for the process.
struct AuxRes {
  hipStream_t stream = nullptr;
  std::vector<hipEvent_t> events;
};
static thread_local std::map<int, AuxRes> t_aux;

hipError_t Engine::aux_init(int nevents) {
  if (one_stream_) {  // everything on the caller's stream: nothing to order, nothing to create
    aux_ = st_;
    ev_ = nullptr;
    return hipSuccess;
  }
  int dev = 0;
  TRY(hipGetDevice(&dev));
  AuxRes& r = t_aux[dev];
  if (!r.stream && !one_stream_) TRY(hipStreamCreateWithFlags(&r.stream, hipStreamNonBlocking));
  // The events only order the two streams of one device: a device-scope
  // release suffices (runtimes without that flag get the default).
  while ((int)r.events.size() < nevents) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming | hipEventReleaseToDevice) != hipSuccess) {
      (void)hipGetLastError();
      TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    r.events.push_back(e);
  }
  aux_ = one_stream_ ? st_ : r.stream;
  ev_ = &r.events;
  return hipSuccess;
}

void release_thread_streams() {
  for (auto& kv : t_aux) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev != kv.first) (void)hipSetDevice(kv.first);
    for (hipEvent_t e : kv.second.events) (void)hipEventDestroy(e);
    if (kv.second.stream) (void)hipStreamDestroy(kv.second.stream);
  }
  t_aux.clear();
}

hipError_t Engine::record(hipStream_t s, int ev) { return one_stream_ ? hipSuccess : hipEventRecord((*ev_)[ev], s); }
hipError_t Engine::wait(hipStream_t s, int ev) { return one_stream_ ? hipSuccess : hipStreamWaitEvent(s, (*ev_)[ev], 0); }

void Engine::layout(Carver& c) {
  const Dims& d = d_;
  const size_t nbv = 3 * (size_t)d.nb;
  const int nt = d.nt;
  const bool ck = d.ckpt > 0 && d.state == 0;
  V.resize(nt + 1); U.resize(nt + 1); W.resize(nt + 1); dV.resize(ck ? 0 : nt);
  for (auto& p : V) p = c.take<float2>(nbv);
  for (auto& p : U) p = c.take<float2>(nbv);
  for (auto& p : W) p = c.take<float2>(nbv);
  for (auto& p : dV) p = c.take<float2>(nbv);
  for (int i = 0; i < 2; ++i) { dU[i] = c.take<float2>(nbv); dW[i] = c.take<float2>(nbv); }
  gh = c.take<float2>(nbv); ph = c.take<float2>(nbv); rh = c.take<float2>(nbv);
  dh = c.take<float2>(nbv); Hdh = c.take<float2>(nbv); v0h = c.take<float2>(nbv);
  vtry = c.take<float2>(nbv); tmph = c.take<float2>(nbv);
  // with checkpoints only the exact gradient runs: no sweep caches but VG
  VG.resize(nt); UG.resize(ck ? 0 : nt); WG.resize(ck ? 0 : nt); dVG.resize(ck ? 0 : nt);
  for (auto& p : VG) p = c.take<float>(24 * (size_t)d.nM);
  for (auto& p : UG) p = c.take<float>(12 * (size_t)d.nM);
  for (auto& p : WG) p = c.take<float>(12 * (size_t)d.nM);
  for (auto& p : dVG) p = c.take<float>(24 * (size_t)d.nM);
  // the image state keeps m_n and the grid velocities of every step; the
  // deformation state needs neither
  const bool def = d.state == 1;
  if (ck) {
    // states m_0, m_c, m_2c, ... < nt; one segment of c recomputed states;
    // m_nt; one grid velocity, recomputed when needed
    m.assign((nt + d.ckpt - 1) / d.ckpt, nullptr);
    mseg_.assign(d.ckpt, nullptr);
    vg.assign(1, nullptr);
  } else {
    m.assign(def ? 0 : nt + 1, nullptr);
    mseg_.clear();
    vg.assign(def ? 0 : nt, nullptr);
  }
  for (auto& p : m) p = c.take<float>((size_t)d.nN);
  for (auto& p : mseg_) p = c.take<float>((size_t)d.nN);
  mfin_ = ck ? c.take<float>((size_t)d.nN) : nullptr;
  for (auto& p : vg) p = c.take<float>(3 * (size_t)d.nN);
  dm[0] = dm[1] = q = mlight[0] = mlight[1] = nullptr;
  if (!def) {
    dm[0] = c.take<float>((size_t)d.nN);  // also the state adjoint of the exact gradient
    dm[1] = c.take<float>((size_t)d.nN);
    if (!ck) {
      dvg_ = c.take<float>(3 * (size_t)d.nN);
      q = c.take<float>((size_t)d.nN);
      mlight[0] = c.take<float>((size_t)d.nN);
      mlight[1] = c.take<float>((size_t)d.nN);
    }
  }
  resid = c.take<float>(d.hessian == 2 ? (size_t)d.nN : 1);
  partial = c.take<double>(1024);
  count = c.take<unsigned>(64);
  scal = c.take<double>(64);
  pcg = c.take<double>(SC_COUNT);
  Lsym = c.take<float>((size_t)d.nb);
  Ksym = c.take<float>((size_t)d.nb);
  twbuf_ = c.take<float2>(twiddle_count(d.M, d) + twiddle_count(d.N, d));
  const size_t C = (size_t)d.K[1] * d.Kh;
  T1_ = c.take<float2>((def ? 4 : 2) * 3 * 2 * (size_t)d.M[0] * C);
  NG_ = c.take<float>(24 * (size_t)d.nM);
  synth_tab_ = c.take<float>(synth_table_floats(d));
  col_tab_ = c.take<float2>(col_table_count(d));
  S1_ = c.take<float2>(9 * (size_t)d.M[0] * d.M[1] * d.Kh);
  T1N.assign(def ? 0 : (ck ? 1 : nt), nullptr);
  for (auto& p : T1N) p = c.take<float2>(3 * (size_t)d.N[0] * C);
  S1N_ = c.take<float2>(3 * (size_t)d.N[0] * d.N[1] * d.Kh);
  S2N_ = c.take<float2>(3 * (size_t)d.N[0] * C);
  Phi.assign(def ? nt + 1 : 0, nullptr);
  PG.assign(def ? nt + 1 : 0, nullptr);
  dPhi[0] = dPhi[1] = R = KR = dR = KdR = nullptr;
  RG = ug = dug = m1 = I0c = IG = IH = NGA_ = nullptr;
  T1NA_ = S1A_ = nullptr;
  if (def) {
    for (auto& p : Phi) p = c.take<float2>(nbv);
    for (int k = 1; k <= nt; ++k) PG[k] = c.take<float>(12 * (size_t)d.nM);  // u_0 = 0 has no group
    dPhi[0] = c.take<float2>(nbv);
    dPhi[1] = c.take<float2>(nbv);
    R = c.take<float2>(nbv);
    KR = c.take<float2>(nbv);
    dR = c.take<float2>(nbv);
    KdR = c.take<float2>(nbv);
    RG = c.take<float>(12 * (size_t)d.nM);
    NGA_ = c.take<float>(24 * (size_t)d.nM);
    S1A_ = c.take<float2>(3 * (size_t)d.M[0] * d.M[1] * d.Kh);
    T1NA_ = c.take<float2>(3 * (size_t)d.N[0] * C);
    ug = c.take<float>(3 * (size_t)d.nN);
    dug = c.take<float>(3 * (size_t)d.nN);
    m1 = c.take<float>((size_t)d.nN);
    I0c = c.take<float>((size_t)d.nN);
    IG = c.take<float>(4 * (size_t)d.nN);
    if (d.hessian == 2) IH = c.take<float>(8 * (size_t)d.nN);
  }
}

Engine::Engine(const Dims& d, void* ws, hipStream_t st)
    : d_(d), st_(st), fuse_grid0_(colstep_fuses_grid0(d) && d.ckpt == 0) {
  Carver c{static_cast<char*>(ws)};
  layout(c);
  // twiddle table views
  float2* t = twbuf_;
  for (int pass = 0; pass < 2; ++pass) {
    Twiddles& tw = pass == 0 ? twM_ : twN_;
    const int* G = pass == 0 ? d.M : d.N;
    for (int j = 0; j < 3; ++j) tw.G[j] = G[j];
    tw.inv0 = t; t += 2 * (size_t)G[0] * d.K[0];
    tw.inv1 = t; t += 2 * (size_t)G[1] * d.K[1];
    tw.inv2 = t; t += 2 * (size_t)G[2] * d.Kh;
    tw.fwd0 = t; t += (size_t)d.K[0] * G[0];
    tw.fwd1 = t; t += (size_t)d.K[1] * G[1];
    tw.fwd2 = t; t += (size_t)d.Kh * G[2];
  }
}

size_t Engine::workspace_bytes(const Dims& d) {
  Engine e(d, nullptr, nullptr);
  Carver c{nullptr};
  e.layout(c);
  return c.off + 256;
}

hipError_t Engine::init_tables() {
  for (int pass = 0; pass < 2; ++pass) {
    const Twiddles& tw = pass == 0 ? twM_ : twN_;
    const int* G = tw.G;
    TRY(launch_twiddles(const_cast<float2*>(tw.inv0), d_.K[0], G[0], 0, st_));
    TRY(launch_twiddles(const_cast<float2*>(tw.inv1), d_.K[1], G[1], 0, st_));
    TRY(launch_twiddles(const_cast<float2*>(tw.inv2), d_.K[2], G[2], 1, st_));
    TRY(launch_twiddles(const_cast<float2*>(tw.fwd0), d_.K[0], G[0], 2, st_));
    TRY(launch_twiddles(const_cast<float2*>(tw.fwd1), d_.K[1], G[1], 2, st_));
    TRY(launch_twiddles(const_cast<float2*>(tw.fwd2), d_.K[2], G[2], 3, st_));
  }
  TRY(launch_fill(reinterpret_cast<float*>(count), 64, 0.f, st_));
  TRY(launch_synth_tables(twM_, synth_tab_, d_, st_));
  TRY(launch_col_tables(twM_, col_tab_, d_, st_));
  return launch_symbols(Lsym, Ksym, d_, st_);
}

hipError_t Engine::load_band(const void* full, float2* half) {
  return launch_full_to_half(static_cast<const float2*>(full), half, d_, st_);
}

hipError_t Engine::store_band(const float2* a, const float2* b, float cb, void* full, const float* sym) {
  return launch_half_to_full(a, b, cb, static_cast<float2*>(full), d_, st_, sym);
}

float2* Engine::t1(int g, int c) const {
  return T1_ + (size_t)(g * 3 + c) * 2 * d_.M[0] * d_.K[1] * d_.Kh;
}

const float2* Engine::s1(int o) const { return S1_ + (size_t)o * d_.Kh * d_.M[0] * d_.M[1]; }

// Inverse stage 0 of the new groups of a step (at the start of a sweep;
// later steps get it from the column kernel of the previous step).
hipError_t Engine::inv0_groups(const float2* in0, int l0, const float2* in1, int l1) {
  const int C = d_.K[1] * d_.Kh;
  Inv0Jobs jobs{};
  int nj = 0;
  const float2* ins[2] = {in0, in1};
  const int lf[2] = {l0, l1};
  for (int g = 0; g < 2; ++g)
    for (int c = 0; c < 3; ++c) {
      jobs.j[nj].in = ins[g] + (size_t)c * d_.nb;
      jobs.j[nj].out = t1(g, c);
      jobs.j[nj].lflag = lf[g];
      ++nj;
    }
  return launch_inv0(jobs, nj, 2, twM_.inv0, Lsym, d_.K[0], C, d_.M[0], d_.Kh, false, st_);
}

// Synthesis of the two new groups (into the cache when given, else into
// scratch), then the Lie products of the program (when nout > 0).
hipError_t Engine::mstep(int prog, int nout, float* store0, float* store1, const float* const* cached) {
  const size_t nM = (size_t)d_.nM;
  float* g0 = store0 ? store0 : NG_;
  float* g1 = store1 ? store1 : NG_ + 12 * nM;
  TRY(launch_synth(t1(0, 0), t1(1, 0), g0, g1, synth_tab_, d_, st_));
  if (nout == 0) return hipSuccess;
  ProdArgs a{};
  a.g[0] = g0;
  a.g[1] = g1;
  if (cached)
    for (int k = 0; k < 6; ++k) a.g[2 + k] = cached[k];
  a.s1 = S1_;
  a.nout = nout;
  a.prog = prog;
  return launch_prods(a, d_, twM_, st_);
}

// One column job: out_c = base + ca S F(s1[oa]) (+ cb S F(s1[ob])) + ce extra;
// next-step stage 0 into group g0 (L flag l0) and optionally g1 (l1).
ColJob Engine::col_job(int c, int oa, float ca, int syma, int ob, float cb, int symb,
                       const float2* base, const float2* extra, float ce, float2* out, int g0, int l0,
                       int g1, int l1, float2* t1n) const {
  ColJob j{};
  j.t1n = t1n ? t1n + (size_t)c * d_.N[0] * d_.K[1] * d_.Kh : nullptr;
  j.a = s1(oa);
  j.ca = ca;
  j.syma = syma;
  if (ob >= 0) {
    j.b = s1(ob);
    j.cb = cb;
    j.symb = symb;
  }
  j.base = base ? base + (size_t)c * d_.nb : nullptr;
  j.extra = extra ? extra + (size_t)c * d_.nb : nullptr;
  j.ce = ce;
  j.out = out + (size_t)c * d_.nb;
  j.nt1 = 0;
  if (g0 >= 0) { j.t1[j.nt1] = t1(g0, c); j.t1l[j.nt1] = l0; ++j.nt1; }
  if (g1 >= 0) { j.t1[j.nt1] = t1(g1, c); j.t1l[j.nt1] = l1; ++j.nt1; }
  return j;
}

hipError_t Engine::colstep(const ColJob* jobs, int n) { return colstep_on(jobs, n, st_); }

hipError_t Engine::colstep_on(const ColJob* jobs, int n, hipStream_t s) {
  ColJobs js{};
  for (int i = 0; i < n; ++i) js.j[i] = jobs[i];
  js.w0n = twN_.inv0;  // value variant [N0][K0]
  js.N0 = d_.N[0];
  return launch_colstep(js, n, d_, twM_, col_tab_, Lsym, Ksym, s);
}

// Forward stages 1 and 0 of the three grid fields in S1N with the given
// band epilogues.
hipError_t Engine::fwd_grid(Fwd0Job* jobs, int njobs, hipStream_t s) {
  const int C = d_.K[1] * d_.Kh;
  const int* G = d_.N;
  Fwd1Jobs j1{};
  for (int o = 0; o < 3; ++o) {
    j1.j[o].in = S1N_ + (size_t)o * G[0] * G[1] * d_.Kh;
    j1.j[o].out = S2N_ + (size_t)o * G[0] * C;
  }
  TRY(launch_fwd1(j1, 3, twN_.fwd1, G[0], G[1], d_.K[1], d_.Kh, s));
  Fwd0Jobs j0{};
  for (int k = 0; k < njobs; ++k) j0.j[k] = jobs[k];
  const float invG = (float)(1.0 / ((double)G[0] * G[1] * G[2]));
  return launch_fwd0(j0, njobs, twN_.fwd0, Ksym, G[0], d_.K[0], d_.K[1], d_.Kh, invG, s);
}

const float2* Engine::s2n(int o) const { return S2N_ + (size_t)o * d_.N[0] * d_.K[1] * d_.Kh; }

// Image-grid inverse stage 0 of one band field into t1n [3][N0][Kh][K1].
hipError_t Engine::grid_stage0(const float2* band, float2* t1n, hipStream_t s) {
  const int C = d_.K[1] * d_.Kh;
  Inv0Jobs jobs{};
  for (int c = 0; c < 3; ++c) {
    jobs.j[c].in = band + (size_t)c * d_.nb;
    jobs.j[c].out = t1n + (size_t)c * d_.N[0] * C;
    jobs.j[c].lflag = 0;
  }
  return launch_inv0(jobs, 3, 1, twN_.inv0, Lsym, d_.K[0], C, d_.N[0], d_.Kh, true, s);
}

// Stage-0 buffer of the grid step of time step n: formed by the column
// kernel of step n-1 (fused), or here (step 0, or shapes without fusion).
hipError_t Engine::grid_t1(int n, const float2* band, hipStream_t s) {
  if (n == 0 || !fuse_grid0_) return grid_stage0(band, T1N[n], s);
  return hipSuccess;
}

// Grid velocity of time step n (band field V[n]) on stream s.
hipError_t Engine::grid_velocity(int n, float* out, hipStream_t s) {
  TRY(grid_t1(n, V[n], s));
  GridStepArgs a{};
  a.t1 = T1N[n];
  a.op = 0;
  a.vout = out;
  return launch_gridstep(a, d_, twN_, s);
}

// Incremental transport source q = dm_n - dt grad_h m_n . dv_n of time step n
// on stream s.
hipError_t Engine::grid_source(int n, const float* dmn, hipStream_t s) {
  TRY(grid_t1(n, dV[n], s));
  GridStepArgs a{};
  a.t1 = T1N[n];
  a.op = 1;
  a.m = m[n];
  a.dm = dmn;
  a.q = q;
  a.dt = 1.0f / d_.nt;
  return launch_gridstep(a, d_, twN_, s);
}

// t = 1 tail: out = K~ pi(coef [(a - b) grad_h m_nt + r grad_h a]) (b, r may be null), then the
// padded-grid stage-0 buffers of the first backward step from (out with L~,
// zero_band) on stream s.
hipError_t Engine::tail(const float* a, const float* b, const float* r, float coef, float2* out,
                        const float2* zero_band, hipStream_t s) {
  const float* mnt = m[d_.nt];
  if (tail_fused(d_)) {
    float2* t1u[3];
    float2* t1z[3];
    for (int c = 0; c < 3; ++c) {
      t1u[c] = t1(0, c);
      t1z[c] = t1(1, c);
    }
    return launch_tail(a, b, r, mnt, coef, S1N_, out, t1u, t1z, d_, twN_, col_tab_, Lsym, Ksym, s);
  }
  TRY(launch_src_fwd2(a, b, r, mnt, coef, S1N_, d_, twN_, s));
  Fwd0Job fj[3];
  for (int c = 0; c < 3; ++c) {
    fj[c] = Fwd0Job{};
    fj[c].a = s2n(c);
    fj[c].ca = 1.f;
    fj[c].syma = 1;
    fj[c].out = out + (size_t)c * d_.nb;
  }
  TRY(fwd_grid(fj, 3, s));
  const int C = d_.K[1] * d_.Kh;
  Inv0Jobs jobs{};
  int nj = 0;
  const float2* ins[2] = {out, zero_band};
  for (int g = 0; g < 2; ++g)
    for (int c = 0; c < 3; ++c) {
      jobs.j[nj].in = ins[g] + (size_t)c * d_.nb;
      jobs.j[nj].out = t1(g, c);
      jobs.j[nj].lflag = g == 0;
      ++nj;
    }
  return launch_inv0(jobs, nj, 2, twM_.inv0, Lsym, d_.K[0], C, d_.M[0], d_.Kh, false, s);
}

hipError_t Engine::shoot_band(bool cache, const StepHook& hook) {
  const float dt = 1.0f / d_.nt;
  TRY(inv0_groups(V[0], 0, V[0], 1));
  for (int n = 0; n < d_.nt; ++n) {
    float* st0 = cache ? VG[n] : nullptr;
    float* st1 = cache ? VG[n] + 12 * (size_t)d_.nM : nullptr;
    TRY(mstep(PROG_SHOOT, 3, st0, st1, nullptr));
    const bool next = n + 1 < d_.nt;
    ColJob jobs[3];
    for (int c = 0; c < 3; ++c)
      jobs[c] = col_job(c, c, -dt, 1, -1, 0.f, 0, V[n], nullptr, 0.f, V[n + 1], next ? 0 : -1, 0,
                        next ? 1 : -1, 1, next && fuse_grid0_ && !d_.state ? T1N[n + 1] : nullptr);
    TRY(colstep(jobs, 3));
    if (ev_) TRY(record(st_, n + 1));
    if (hook) TRY(hook(n + 1));
  }
  return hipSuccess;
}

// Shooting on the caller's stream; the grid chain (velocity of step n, then
// the transport step) on the auxiliary stream.  Each grid step is enqueued
// right after the band step that produces v_n, so that the host issues both
// streams' work in the order the device can run it.
hipError_t Engine::forward(const float* I0) {
  if (d_.state) return forward_def(I0);
  const float dt = 1.0f / d_.nt;
  const int nt = d_.nt;
  TRY(aux_init(nt + 2));
  TRY(record(st_, 0));
  auto grid_step = [&](int n) -> hipError_t {
    if (n >= nt) return hipSuccess;
    TRY(wait(aux_, n));
    if (n == 0) TRY(launch_copy(I0, m[0], d_.nN, aux_));
    TRY(grid_velocity(n, vg[n], aux_));
    return launch_sl(m[n], vg[n], m[n + 1], dt, d_, aux_);
  };
  TRY(grid_step(0));
  TRY(shoot_band(true, grid_step));
  TRY(record(aux_, nt + 1));
  return wait(st_, nt + 1);
}

// Shooting and transport without the caches; returns m_nt in *m_out.
hipError_t Engine::forward_light(const float* I0, const float** m_out) {
  if (d_.integrator == 1) return forward_rk(I0, m_out);
  if (d_.state) {
    // the displacement chain reads the cached trajectory fields, so the
    // deformation state always runs the caching forward
    TRY(forward_def(I0));
    *m_out = m1;
    return hipSuccess;
  }
  const float dt = 1.0f / d_.nt;
  const int nt = d_.nt;
  TRY(aux_init(nt + 2));
  TRY(record(st_, 0));
  const float* cur = I0;
  auto grid_step = [&](int n) -> hipError_t {
    if (n >= nt) return hipSuccess;
    TRY(wait(aux_, n));
    TRY(grid_velocity(n, vg[0], aux_));
    float* dst = mlight[n & 1];
    TRY(launch_sl(cur, vg[0], dst, dt, d_, aux_));
    cur = dst;
    return hipSuccess;
  };
  TRY(grid_step(0));
  TRY(shoot_band(false, grid_step));
  TRY(record(aux_, nt + 1));
  TRY(wait(st_, nt + 1));
  *m_out = cur;
  return hipSuccess;
}

// Classical RK4 steps of the band EPDiff, f(v) = -K~ F(ad*_v(L~ v)): each stage
// is the usual synthesis and products launch pair and one column launch;
// the column launches of stages 1-3 form the next stage value (with its
// stage-0 groups) and the running sum v_n + dt/6 k1 + dt/3 k2 + dt/3 k3,
// that of stage 4 adds dt/6 k4 into V[n+1] and forms the next step's groups.
hipError_t Engine::shoot_band_rk4() {
  const float dt = 1.0f / d_.nt;
  const float cst[3] = {0.5f * dt, 0.5f * dt, dt};                // stage value = v_n + c k
  const float wsum[4] = {dt / 6.0f, dt / 3.0f, dt / 3.0f, dt / 6.0f};  // weights of the sum
  float2* va = dU[0];
  float2* acc[2] = {dU[1], dW[0]};
  TRY(inv0_groups(V[0], 0, V[0], 1));
  for (int n = 0; n < d_.nt; ++n) {
    const bool next = n + 1 < d_.nt;
    int cur = 0;
    for (int stg = 0; stg < 4; ++stg) {
      TRY(mstep(PROG_SHOOT, 3, nullptr, nullptr, nullptr));
      ColJob jobs[6];
      int nj = 0;
      if (stg < 3) {
        for (int c = 0; c < 3; ++c)
          jobs[nj++] = col_job(c, c, -cst[stg], 1, -1, 0.f, 0, V[n], nullptr, 0.f, va, 0, 0, 1, 1);
        const float2* base = stg == 0 ? V[n] : acc[cur];
        for (int c = 0; c < 3; ++c)
          jobs[nj++] = col_job(c, c, -wsum[stg], 1, -1, 0.f, 0, base, nullptr, 0.f, acc[1 - cur], -1, 0, -1, 0);
        cur = 1 - cur;
      } else {
        for (int c = 0; c < 3; ++c)
          jobs[nj++] = col_job(c, c, -wsum[3], 1, -1, 0.f, 0, acc[cur], nullptr, 0.f, V[n + 1], next ? 0 : -1, 0,
                               next ? 1 : -1, 1);
      }
      TRY(colstep(jobs, nj));
    }
  }
  return hipSuccess;
}

// RK4 shooting, then the image transport with midpoint departure points
// whose mid-step velocity is iota of the band average of v_n and v_{n+1}.
hipError_t Engine::forward_rk(const float* I0, const float** m_out) {
  const float dt = 1.0f / d_.nt;
  TRY(shoot_band_rk4());
  float2* diff = dW[1];
  float2* vmid = dV[0];
  const float* cur = I0;
  for (int n = 0; n < d_.nt; ++n) {
    TRY(launch_axpy_band(V[n + 1], V[n], -1.f, diff, 3 * d_.nb, st_));
    TRY(launch_axpy_band(V[n], diff, 0.5f, vmid, 3 * d_.nb, st_));
    TRY(grid_stage0(vmid, T1N[0], st_));
    GridStepArgs a{};
    a.t1 = T1N[0];
    a.op = 0;
    a.vout = vg[0];
    TRY(launch_gridstep(a, d_, twN_, st_));
    float* dst = mlight[n & 1];
    TRY(launch_sl_rk2(cur, vg[0], dst, dt, d_, st_));
    cur = dst;
  }
  *m_out = cur;
  return hipSuccess;
}

hipError_t Engine::geodesic_energies(double* out) {
  if (d_.integrator == 1)
    TRY(shoot_band_rk4());
  else
    TRY(shoot_band(false));
  for (int n = 0; n <= d_.nt; ++n) TRY(launch_band_dot(V[n], V[n], Lsym, d_, partial, out + n, 1.0, st_));
  return hipSuccess;
}

hipError_t Engine::energy(const float* mnt, const float* I1) {
  const double sdata = 1.0 / (d_.sigma * d_.sigma * (double)d_.nN);
  TRY(launch_sqdiff(mnt, I1, d_.nN, partial, scal + 2, sdata, st_));
  TRY(launch_band_dot(V[0], V[0], Lsym, d_, partial + 512, scal + 1, 0.5, st_));
  return launch_energy_combine(scal, st_);
}

hipError_t Engine::backward(const float* I1, float2* g_out) {
  if (d_.hessian == 3) return backward_exact(I1, g_out);
  const float dt = 1.0f / d_.nt;
  const int nt = d_.nt;
  const float coef = (float)(-2.0 / (d_.sigma * d_.sigma));
  // U_nt = K~ pi(lambda_1 grad_h m_nt), lambda_1 = -(2/sigma^2)(m_nt - I1); W_nt = 0
  TRY(launch_fill(reinterpret_cast<float*>(W[nt]), 6LL * d_.nb, 0.f, st_));
  if (d_.state)
    TRY(tail_def(I1));
  else
    TRY(tail(m[nt], I1, nullptr, coef, U[nt], W[nt], st_));
  // the full Newton product needs lambda_1 (as m(1) - I1) in later hessvec calls
  if (d_.hessian == 2) TRY(launch_diff(final_state(), I1, resid, d_.nN, st_));
  for (int n = nt - 1; n >= 0; --n) {
    const float* cached[6] = {VG[n], VG[n] + 12 * (size_t)d_.nM, nullptr, nullptr, nullptr, nullptr};
    TRY(mstep(PROG_GRAD, 9, UG[n], WG[n], cached));
    const bool next = n > 0;
    ColJob jobs[6];
    for (int c = 0; c < 3; ++c) {
      // U_n = U_{n+1} + dt K~ F(ad*_V LU)
      jobs[c] = col_job(c, c, dt, 1, -1, 0.f, 0, U[n + 1], nullptr, 0.f, U[n], next ? 0 : -1, 1, -1, 0);
      // W_n = W_{n+1} - dt F(ad_V W) + dt K~ F(ad*_W LV) + dt U_{n+1}
      jobs[3 + c] = col_job(c, 3 + c, -dt, 0, 6 + c, dt, 1, W[n + 1], U[n + 1], dt, W[n],
                            next ? 1 : -1, 0, -1, 0);
    }
    TRY(colstep(jobs, 6));
  }
  if (g_out) TRY(launch_axpy_band(V[0], W[0], 1.f, g_out, 3 * d_.nb, st_));
  return hipSuccess;
}

hipError_t Engine::hessvec(const float2* dvh, float2* out) {
  if (d_.state) return hessvec_def(dvh, out);
  if (d_.hessian == 3) return hessvec_exact(dvh, out);
  const float dt = 1.0f / d_.nt;
  const int nt = d_.nt;
  const bool coupled = d_.hessian != 1;  // paper reading and full Newton keep the coupling terms
  const size_t nM = (size_t)d_.nM;
  TRY(aux_init(nt + 3));
  if (dvh != dV[0]) TRY(launch_copy(reinterpret_cast<const float*>(dvh), reinterpret_cast<float*>(dV[0]),
                                    6LL * d_.nb, st_));
  TRY(record(st_, 0));
  // Incremental state transport on the auxiliary stream: step n waits for
  // dv_n (event n) and is enqueued as soon as the band step that makes dv_n
  // has been, so the two streams overlap.
  const float coef = (float)(-2.0 / (d_.sigma * d_.sigma));
  const float* dmcur = nullptr;
  auto grid_step = [&](int n) -> hipError_t {
    TRY(wait(aux_, n));
    TRY(grid_source(n, dmcur, aux_));
    float* dst = dm[n & 1];
    TRY(launch_sl(q, vg[n], dst, dt, d_, aux_));
    dmcur = dst;
    return hipSuccess;
  };
  TRY(grid_step(0));
  // incremental EPDiff forward (caller's stream); event n+1 marks dv_{n+1}
  TRY(inv0_groups(dV[0], 0, dV[0], 1));
  for (int n = 0; n < nt; ++n) {
    const bool last = n == nt - 1;
    if (last && !coupled) break;
    const float* cached[6] = {VG[n], VG[n] + 12 * nM, nullptr, nullptr, nullptr, nullptr};
    float* st0 = coupled ? dVG[n] : nullptr;
    float* st1 = coupled ? dVG[n] + 12 * nM : nullptr;
    TRY(mstep(last ? PROG_STORE : PROG_H1, last ? 0 : 3, st0, st1, cached));
    if (!last) {
      ColJob jobs[3];
      for (int c = 0; c < 3; ++c)
        jobs[c] = col_job(c, c, -dt, 1, -1, 0.f, 0, dV[n], nullptr, 0.f, dV[n + 1], 0, 0, 1, 1,
                          fuse_grid0_ ? T1N[n + 1] : nullptr);
      TRY(colstep(jobs, 3));
      TRY(record(st_, n + 1));
      TRY(grid_step(n + 1));
    }
  }
  // dU_nt = K~ pi(dlambda_1 grad_h m_nt), dlambda_1 = -(2/sigma^2) dm_nt, on the
  // auxiliary stream after the last transport step; dW_nt = 0.  The fused
  // tail also writes the padded-grid stage-0 buffers, which the main stream
  // reads until its last step above: it waits for that (event nt + 2).
  TRY(launch_fill(reinterpret_cast<float*>(dW[0]), 6LL * d_.nb, 0.f, st_));
  TRY(record(st_, nt + 2));
  TRY(wait(aux_, nt + 2));
  TRY(tail(dmcur, nullptr, d_.hessian == 2 ? resid : nullptr, coef, dU[0], dW[0], aux_));
  TRY(record(aux_, nt + 1));
  TRY(wait(st_, nt + 1));
  return hessvec_sweep(out);
}

// Incremental adjoint Jacobi sweep backward from dU[0] (dU_nt) and dW[0] = 0
// with the stage-0 buffers of its first step in place; Hdv = dv0 + dw_0.
hipError_t Engine::hessvec_sweep(float2* out) {
  const float dt = 1.0f / d_.nt;
  const int nt = d_.nt;
  const bool coupled = d_.hessian != 1;
  const size_t nM = (size_t)d_.nM;
  int cur = 0;
  for (int n = nt - 1; n >= 0; --n) {
    const float* cached[6] = {VG[n], VG[n] + 12 * nM, UG[n], WG[n], dVG[n], dVG[n] + 12 * nM};
    TRY(mstep(coupled ? PROG_H5 : PROG_H5_NOCOUPLE, 9, nullptr, nullptr, cached));
    const bool next = n > 0;
    ColJob jobs[6];
    for (int c = 0; c < 3; ++c) {
      jobs[c] = col_job(c, c, dt, 1, -1, 0.f, 0, dU[cur], nullptr, 0.f, dU[1 - cur], next ? 0 : -1, 1, -1, 0);
      jobs[3 + c] = col_job(c, 3 + c, -dt, 0, 6 + c, dt, 1, dW[cur], dU[cur], dt, dW[1 - cur],
                            next ? 1 : -1, 0, -1, 0);
    }
    TRY(colstep(jobs, 6));
    cur = 1 - cur;
  }
  return launch_axpy_band(dV[0], dW[cur], 1.f, out, 3 * d_.nb, st_);
}

// ------------------------------------- exact derivative of the discrete energy
// The reverse of every step of `forward`: the state adjoint lam (held as
// lam / coef, lam_nt / coef = m_nt - I1, coef = 2 / sigma^2 with the 1/|N| of
// the energy's mean folded into pi) is carried back through the transpose
// of each transport step, and each step's velocity sensitivity goes to the
// band as S_n = K~ pi(s_n) (k_adj_src_fwd2, then forward stages 1 and 0);
// then the transpose of each Euler step of the band EPDiff in the V metric,
// w_n = w_{n+1} - dt ad~_{v_n} w_{n+1} + dt K~ ad~*_{w_{n+1}}(L~ v_n) + S_n,
// w_nt = 0, g_V = v_0 + w_0.  With checkpoints the states of each segment of
// c steps are transported again from its first state, and the grid
// velocities are synthesised again from the band trajectory.

float* Engine::ckpt_state(int n) const {
  const int c = d_.ckpt;
  if (n == d_.nt) return mfin_;
  if (n % c == 0) return m[n / c];
  return mseg_[n % c];
}

hipError_t Engine::grid_velocity_ckpt(int n, float* out, hipStream_t s) {
  TRY(grid_stage0(V[n], T1N[0], s));
  GridStepArgs a{};
  a.t1 = T1N[0];
  a.op = 0;
  a.vout = out;
  return launch_gridstep(a, d_, twN_, s);
}

hipError_t Engine::forward_ckpt(const float* I0) {
  if (d_.ckpt == 0) return forward(I0);
  const float dt = 1.0f / d_.nt;
  const int nt = d_.nt;
  TRY(aux_init(nt + 2));
  TRY(record(st_, 0));
  auto grid_step = [&](int n) -> hipError_t {
    if (n >= nt) return hipSuccess;
    TRY(wait(aux_, n));
    if (n == 0) TRY(launch_copy(I0, m[0], d_.nN, aux_));
    TRY(grid_velocity_ckpt(n, vg[0], aux_));
    return launch_sl(ckpt_state(n), vg[0], ckpt_state(n + 1), dt, d_, aux_);
  };
  TRY(grid_step(0));
  TRY(shoot_band(true, grid_step));
  TRY(record(aux_, nt + 1));
  return wait(st_, nt + 1);
}

hipError_t Engine::backward_exact(const float* I1, float2* g_out) {
  TRY(launch_diff(final_state(), I1, dm[0], d_.nN, st_));
  TRY(adjoint_exact(0));
  if (g_out) TRY(launch_axpy_band(V[0], W[0], 1.f, g_out, 3 * d_.nb, st_));
  return hipSuccess;
}

hipError_t Engine::hessvec_exact(const float2* dvh, float2* out) {
  const float dt = 1.0f / d_.nt;
  const int nt = d_.nt;
  const size_t nM = (size_t)d_.nM;
  if (dvh != dV[0])
    TRY(launch_copy(reinterpret_cast<const float*>(dvh), reinterpret_cast<float*>(dV[0]), 6LL * d_.nb, st_));
  // the linearised Euler steps dv_{n+1} = dv_n - dt K~[ad*_{dv_n}(L~ v_n) + ad*_{v_n}(L~ dv_n)],
  // each step's grid increment iota(dv_n) and the tangent of transport step n
  TRY(inv0_groups(dV[0], 0, dV[0], 1));
  int cur = 0;
  for (int n = 0; n < nt; ++n) {
    TRY(grid_t1(n, dV[n], st_));
    GridStepArgs ga{};
    ga.t1 = T1N[n];
    ga.op = 0;
    ga.vout = dvg_;
    TRY(launch_gridstep(ga, d_, twN_, st_));
    TRY(launch_sl_tangent(n == 0 ? nullptr : dm[cur], m[n], vg[n], dvg_, dm[1 - cur], dt, d_, st_));
    cur = 1 - cur;
    if (n == nt - 1) break;
    const float* cached[6] = {VG[n], VG[n] + 12 * nM, nullptr, nullptr, nullptr, nullptr};
    TRY(mstep(PROG_H1, 3, nullptr, nullptr, cached));
    ColJob jobs[3];
    for (int c = 0; c < 3; ++c)
      jobs[c] = col_job(c, c, -dt, 1, -1, 0.f, 0, dV[n], nullptr, 0.f, dV[n + 1], 0, 0, 1, 1,
                        fuse_grid0_ ? T1N[n + 1] : nullptr);
    TRY(colstep(jobs, 3));
  }
  // lam_nt / coef = dm_nt (W = 2 / (sigma^2 |N|), the 1/|N| folded into pi)
  TRY(adjoint_exact(cur));
  return launch_axpy_band(dV[0], W[0], 1.f, out, 3 * d_.nb, st_);
}

hipError_t Engine::adjoint_exact(int cur) {
  const float dt = 1.0f / d_.nt;
  const int nt = d_.nt;
  const int c = d_.ckpt;
  const size_t nM = (size_t)d_.nM;
  const float coef = (float)(2.0 / (d_.sigma * d_.sigma));
  // grid chain, backward: S_n into U[n]
  for (int n = nt - 1; n >= 0; --n) {
    const float* mn;
    const float* vn;
    if (c == 0) {
      mn = m[n];
      vn = vg[n];
    } else {
      // entering a segment from its end: transport its states again
      const int s0 = (n / c) * c;
      if (n == nt - 1 || n % c == c - 1)
        for (int k = s0; k < n; ++k) {
          TRY(grid_velocity_ckpt(k, vg[0], st_));
          TRY(launch_sl(ckpt_state(k), vg[0], mseg_[(k + 1) - s0], dt, d_, st_));
        }
      mn = ckpt_state(n);
      TRY(grid_velocity_ckpt(n, vg[0], st_));
      vn = vg[0];
    }
    TRY(launch_fill(dm[1 - cur], d_.nN, 0.f, st_));
    TRY(launch_adj_src_fwd2(dm[cur], mn, vn, dm[1 - cur], coef, dt, S1N_, d_, twN_, st_));
    Fwd0Job fj[3];
    for (int k = 0; k < 3; ++k) {
      fj[k] = Fwd0Job{};
      fj[k].a = s2n(k);
      fj[k].ca = 1.f;
      fj[k].syma = 1;
      fj[k].out = U[n] + (size_t)k * d_.nb;
    }
    TRY(fwd_grid(fj, 3, st_));
    cur = 1 - cur;
  }
  // band sweep, backward from w_nt = 0
  TRY(launch_fill(reinterpret_cast<float*>(W[nt]), 6LL * d_.nb, 0.f, st_));
  TRY(inv0_group(W[nt], 0, 0, st_));
  for (int n = nt - 1; n >= 0; --n) {
    TRY(launch_synth(t1(0, 0), nullptr, NG_, nullptr, synth_tab_, d_, st_));
    ProdArgs a{};
    a.g[0] = NG_;
    a.g[1] = VG[n];
    a.g[2] = VG[n] + 12 * nM;
    a.s1 = S1_;
    a.nout = 6;
    a.prog = PROG_ADJ;
    TRY(launch_prods(a, d_, twM_, st_));
    const bool next = n > 0;
    ColJob jobs[3];
    for (int k = 0; k < 3; ++k)
      jobs[k] = col_job(k, k, -dt, 0, 3 + k, dt, 1, W[n + 1], U[n], 1.f, W[n], next ? 0 : -1, 0, -1, 0);
    TRY(colstep(jobs, 3));
  }
  return hipSuccess;
}

// ------------------------------------------------ deformation state (§3.3)
// Stage-0 group 2 belongs to the displacement chain (u_k or du_k), group 3
// to rho~ / drho~ at t = 1; groups 0 and 1 stay with the main chain.

hipError_t Engine::inv0_group(const float2* in, int g, int lflag, hipStream_t s) {
  const int C = d_.K[1] * d_.Kh;
  Inv0Jobs jobs{};
  for (int c = 0; c < 3; ++c) {
    jobs.j[c].in = in + (size_t)c * d_.nb;
    jobs.j[c].out = t1(g, c);
    jobs.j[c].lflag = lflag;
  }
  return launch_inv0(jobs, 3, 2, twM_.inv0, Lsym, d_.K[0], C, d_.M[0], d_.Kh, false, s);
}

hipError_t Engine::prods_on(int prog, const float* const* g, int ng, float2* out, hipStream_t s) {
  ProdArgs a{};
  for (int k = 0; k < ng; ++k) a.g[k] = g[k];
  a.s1 = out;
  a.nout = 3;
  a.prog = prog;
  return launch_prods(a, d_, twM_, s);
}

// iota of a band field on the image grid into out [3][nN], through the
// image-grid stage-0 buffer of the chain (already formed when have_t1n).
hipError_t Engine::grid_field(const float2* band, bool have_t1n, float* out, hipStream_t s) {
  if (!have_t1n) TRY(grid_stage0(band, T1NA_, s));
  GridStepArgs a{};
  a.t1 = T1NA_;
  a.op = 0;
  a.vout = out;
  return launch_gridstep(a, d_, twN_, s);
}

// Forward stages 1 and 0 of the three fields in S1N: pi(s) into `plain` and
// K~ pi(s) into `smooth`.
hipError_t Engine::band_pair(float2* plain, float2* smooth, hipStream_t s) {
  Fwd0Job fj[3];
  for (int c = 0; c < 3; ++c) {
    Fwd0Job& j = fj[c];
    j = Fwd0Job{};
    j.a = s2n(c);
    j.ca = 1.f;
    j.syma = 0;
    j.out = plain + (size_t)c * d_.nb;
    j.out2 = smooth + (size_t)c * d_.nb;
  }
  return fwd_grid(fj, 3, s);
}

// out = base + K~ F(products of the program) on the caller's stream, with the
// stage-0 buffers of the first backward step: group 0 from L~ out, group 1
// zero (w = 0 at t = 1).
hipError_t Engine::def_head(int prog, const float* const* g, int ng, const float2* base, float2* out) {
  TRY(prods_on(prog, g, ng, S1_, st_));
  TRY(launch_fill(reinterpret_cast<float*>(t1(1, 0)), 12LL * d_.M[0] * d_.K[1] * d_.Kh, 0.f, st_));
  ColJob jobs[3];
  for (int c = 0; c < 3; ++c) jobs[c] = col_job(c, c, 1.f, 1, -1, 0.f, 0, base, nullptr, 0.f, out, 0, 1, -1, 0);
  return colstep_on(jobs, 3, st_);
}

// Shooting on the caller's stream; the band displacement chain
//   u_{k+1} = u_k - dt [v_k + D~u_k * v_k],  u_0 = 0,
// on the auxiliary stream, step k enqueued right after the band step that
// makes v_{k+1} (the fields of v_k are cached by then); then iota(u_nt) on
// the image grid and m(1) = I0(x + iota(u_nt)(x)).
hipError_t Engine::forward_def(const float* I0) {
  const float dt = 1.0f / d_.nt;
  const int nt = d_.nt;
  const size_t ns1 = (size_t)d_.Kh * d_.M[0] * d_.M[1];
  TRY(aux_init(nt + 3));
  TRY(record(st_, 0));
  TRY(wait(aux_, 0));
  TRY(launch_fill(reinterpret_cast<float*>(Phi[0]), 6LL * d_.nb, 0.f, aux_));
  TRY(launch_copy(I0, I0c, d_.nN, aux_));
  TRY(launch_image_derivs(I0c, IG, IH, d_, aux_));
  auto chain = [&](int n) -> hipError_t {  // v_n exists: displacement step n - 1
    const int k = n - 1;
    TRY(wait(aux_, n));
    if (k == 0) {  // D~u_0 = 0
      TRY(launch_axpy_band(Phi[0], V[0], -dt, Phi[1], 3 * d_.nb, aux_));
      return inv0_group(Phi[1], 2, 0, aux_);
    }
    TRY(launch_synth(t1(2, 0), nullptr, PG[k], nullptr, synth_tab_, d_, aux_));
    const float* g[2] = {PG[k], VG[k]};
    TRY(prods_on(PROG_DEF_FWD, g, 2, S1A_, aux_));
    const bool last = k + 1 == nt;
    ColJob jobs[3];
    for (int c = 0; c < 3; ++c) {
      jobs[c] = col_job(c, c, -dt, 0, -1, 0.f, 0, Phi[k], V[k], -dt, Phi[k + 1], 2, 0, -1, 0,
                        last && fuse_grid0_ ? T1NA_ : nullptr);
      jobs[c].a = S1A_ + c * ns1;
    }
    return colstep_on(jobs, 3, aux_);
  };
  TRY(shoot_band(true, chain));
  TRY(grid_field(Phi[nt], nt > 1 && fuse_grid0_, ug, aux_));
  TRY(launch_sl(I0c, ug, m1, -1.0f, d_, aux_));
  TRY(record(aux_, nt + 1));
  return wait(st_, nt + 1);
}

// t = 1 of the gradient: rho~ = pi(lambda_1 (grad I0)(phi(1))) and
// U_nt = K~ rho~ + K~ ((D~u_nt)^T * rho~).
hipError_t Engine::tail_def(const float* I1) {
  const int nt = d_.nt;
  RhoArgs ra{};
  ra.I0 = I0c;
  ra.G = IG;
  ra.u = ug;
  ra.I1 = I1;
  ra.coef = (float)(-2.0 / (d_.sigma * d_.sigma));
  ra.op = 0;
  TRY(launch_rho_fwd2(ra, S1N_, d_, twN_, st_));
  TRY(band_pair(R, KR, st_));
  TRY(inv0_group(R, 3, 0, st_));
  TRY(launch_synth(t1(2, 0), t1(3, 0), PG[nt], RG, synth_tab_, d_, st_));
  const float* g[2] = {PG[nt], RG};
  return def_head(PROG_DEF_TAIL, g, 2, KR, U[nt]);
}

// Incremental EPDiff on the caller's stream (every step's fields kept), the
// incremental displacement chain
//   du_{k+1} = du_k - dt [D~du_k * v_k + dv_k + D~u_k * dv_k],  du_0 = 0,
// on the auxiliary stream, then drho~ and dU_nt and the incremental sweep.
hipError_t Engine::hessvec_def(const float2* dvh, float2* out) {
  const float dt = 1.0f / d_.nt;
  const int nt = d_.nt;
  const size_t nM = (size_t)d_.nM;
  const size_t ns1 = (size_t)d_.Kh * d_.M[0] * d_.M[1];
  TRY(aux_init(nt + 3));
  if (dvh != dV[0]) TRY(launch_copy(reinterpret_cast<const float*>(dvh), reinterpret_cast<float*>(dV[0]),
                                    6LL * d_.nb, st_));
  TRY(record(st_, 0));
  int cur = 0;  // dPhi[cur] holds du_k
  auto chain = [&](int k) -> hipError_t {  // dv_k and its fields exist (event k + 1)
    TRY(wait(aux_, k + 1));
    if (k == 0) {  // du_0 = 0 and u_0 = 0
      TRY(launch_axpy_band(Phi[0], dV[0], -dt, dPhi[0], 3 * d_.nb, aux_));
      return inv0_group(dPhi[0], 2, 0, aux_);
    }
    TRY(launch_synth(t1(2, 0), nullptr, NGA_, nullptr, synth_tab_, d_, aux_));
    const float* g[4] = {NGA_, VG[k], PG[k], dVG[k]};
    TRY(prods_on(PROG_DEF_H, g, 4, S1A_, aux_));
    const bool last = k + 1 == nt;
    ColJob jobs[3];
    for (int c = 0; c < 3; ++c) {
      jobs[c] = col_job(c, c, -dt, 0, -1, 0.f, 0, dPhi[cur], dV[k], -dt, dPhi[1 - cur], 2, 0, -1, 0,
                        last && fuse_grid0_ ? T1NA_ : nullptr);
      jobs[c].a = S1A_ + c * ns1;
    }
    TRY(colstep_on(jobs, 3, aux_));
    cur = 1 - cur;
    return hipSuccess;
  };
  TRY(inv0_groups(dV[0], 0, dV[0], 1));
  for (int n = 0; n < nt; ++n) {
    const bool last = n == nt - 1;
    const float* cached[6] = {VG[n], VG[n] + 12 * nM, nullptr, nullptr, nullptr, nullptr};
    TRY(mstep(last ? PROG_STORE : PROG_H1, last ? 0 : 3, dVG[n], dVG[n] + 12 * nM, cached));
    TRY(record(st_, n + 1));
    TRY(chain(n));
    if (!last) {
      ColJob jobs[3];
      for (int c = 0; c < 3; ++c)
        jobs[c] = col_job(c, c, -dt, 1, -1, 0.f, 0, dV[n], nullptr, 0.f, dV[n + 1], 0, 0, 1, 1);
      TRY(colstep(jobs, 3));
    }
  }
  // t = 1 on the auxiliary stream: iota(du_nt), drho~ = pi(dlambda_1 (grad I0)(phi(1))
  // [+ lambda_1 (Hess I0)(phi(1)) iota(du_nt)]) and its stage 0
  TRY(grid_field(dPhi[cur], nt > 1 && fuse_grid0_, dug, aux_));
  RhoArgs ra{};
  ra.I0 = I0c;
  ra.G = IG;
  ra.H = IH;
  ra.u = ug;
  ra.du = dug;
  ra.res = d_.hessian == 2 ? resid : nullptr;
  ra.coef = (float)(-2.0 / (d_.sigma * d_.sigma));
  ra.op = 1;
  TRY(launch_rho_fwd2(ra, S1N_, d_, twN_, aux_));
  TRY(band_pair(dR, KdR, aux_));
  TRY(inv0_group(dR, 3, 0, aux_));
  TRY(record(aux_, nt + 1));
  TRY(wait(st_, nt + 1));
  // dU_nt = K~ drho~ + K~ ((D~u_nt)^T * drho~ [+ (D~du_nt)^T * rho~, full Newton])
  TRY(launch_fill(reinterpret_cast<float*>(dW[0]), 6LL * d_.nb, 0.f, st_));
  if (d_.hessian != 2) {
    TRY(launch_synth(t1(3, 0), nullptr, NGA_, nullptr, synth_tab_, d_, st_));
    const float* g[2] = {PG[nt], NGA_};
    TRY(def_head(PROG_DEF_TAIL, g, 2, KdR, dU[0]));
  } else {
    TRY(launch_synth(t1(2, 0), t1(3, 0), NGA_, NGA_ + 12 * nM, synth_tab_, d_, st_));
    const float* g[4] = {NGA_, NGA_ + 12 * nM, PG[nt], RG};
    TRY(def_head(PROG_DEF_HTAIL, g, 4, KdR, dU[0]));
  }
  return hessvec_sweep(out);
}

}  // namespace lddmm
