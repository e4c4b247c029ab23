// Host engine of band-limited Jacobi PDE-EPDiff LDDMM (paper §3.2).
//
// Per Euler step on the padded grid the engine issues four launches:
// stage 0 of the inverse transforms of the new fields (k_inv0), the fused
// step kernel (inverse stages 1-2, Lie products, forward stage 2; k_mstep),
// and forward stages 1 and 0 with the band update as epilogue (k_fwd1,
// k_fwd0).  Fields of the trajectory that later sweeps reuse are cached on
// the padded grid when they are first synthesised.
#include "engine.h"

#include <algorithm>

namespace lddmm {

#define TRY(x)                            \
  do {                                    \
    hipError_t e_ = (x);                  \
    if (e_ != hipSuccess) return e_;      \
  } while (0)

namespace {
constexpr int kGridChunk = 10;  // time steps per batched band->grid stage-0 launch

size_t twiddle_count(const int* G, const Dims& d) {
  return 2 * (size_t)G[0] * d.K[0] + 2 * (size_t)G[1] * d.K[1] + 2 * (size_t)G[2] * d.Kh +
         (size_t)d.K[0] * G[0] + (size_t)d.K[1] * G[1] + (size_t)d.Kh * G[2];
}
}  // namespace

void Engine::layout(Carver& c) {
  const Dims& d = d_;
  const size_t nbv = 3 * (size_t)d.nb;
  const int nt = d.nt;
  V.resize(nt + 1); U.resize(nt + 1); W.resize(nt + 1); dV.resize(nt);
  for (auto& p : V) p = c.take<float2>(nbv);
  for (auto& p : U) p = c.take<float2>(nbv);
  for (auto& p : W) p = c.take<float2>(nbv);
  for (auto& p : dV) p = c.take<float2>(nbv);
  for (int i = 0; i < 2; ++i) { dU[i] = c.take<float2>(nbv); dW[i] = c.take<float2>(nbv); }
  gh = c.take<float2>(nbv); ph = c.take<float2>(nbv); rh = c.take<float2>(nbv);
  dh = c.take<float2>(nbv); Hdh = c.take<float2>(nbv); v0h = c.take<float2>(nbv);
  vtry = c.take<float2>(nbv); tmph = c.take<float2>(nbv);
  VG.resize(nt); UG.resize(nt); WG.resize(nt); dVG.resize(nt);
  for (auto& p : VG) p = c.take<float>(24 * (size_t)d.nM);
  for (auto& p : UG) p = c.take<float>(12 * (size_t)d.nM);
  for (auto& p : WG) p = c.take<float>(12 * (size_t)d.nM);
  for (auto& p : dVG) p = c.take<float>(24 * (size_t)d.nM);
  m.resize(nt + 1); vg.resize(nt);
  for (auto& p : m) p = c.take<float>((size_t)d.nN);
  for (auto& p : vg) p = c.take<float>(3 * (size_t)d.nN);
  dm[0] = c.take<float>((size_t)d.nN);
  dm[1] = c.take<float>((size_t)d.nN);
  q = c.take<float>((size_t)d.nN);
  mlight[0] = c.take<float>((size_t)d.nN);
  mlight[1] = c.take<float>((size_t)d.nN);
  partial = c.take<double>(1024);
  scal = c.take<double>(64);
  pcg = c.take<double>(SC_COUNT);
  Lsym = c.take<float>((size_t)d.nb);
  Ksym = c.take<float>((size_t)d.nb);
  twbuf_ = c.take<float2>(twiddle_count(d.M, d) + twiddle_count(d.N, d));
  const size_t C = (size_t)d.K[1] * d.Kh;
  T1_ = c.take<float2>(2 * 3 * 2 * (size_t)d.M[0] * C);
  S1_ = c.take<float2>(9 * (size_t)d.M[0] * d.M[1] * d.Kh);
  S2_ = c.take<float2>(9 * (size_t)d.M[0] * C);
  const int chunk = std::min(nt, kGridChunk);
  T1N_ = c.take<float2>((size_t)chunk * 3 * d.N[0] * C);
  S1N_ = c.take<float2>(3 * (size_t)d.N[0] * d.N[1] * d.Kh);
  S2N_ = c.take<float2>(3 * (size_t)d.N[0] * C);
}

Engine::Engine(const Dims& d, void* ws, hipStream_t st) : d_(d), st_(st) {
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
  return launch_symbols(Lsym, Ksym, d_, st_);
}

hipError_t Engine::load_band(const void* full, float2* half) {
  return launch_full_to_half(static_cast<const float2*>(full), half, d_, st_);
}

hipError_t Engine::store_band(const float2* a, const float2* b, float cb, void* full) {
  return launch_half_to_full(a, b, cb, static_cast<float2*>(full), d_, st_);
}

// Stage 0 for the new groups, then the fused step kernel.
hipError_t Engine::mstep_step(int prog, int nout, const float2* in0, int l0, const float2* in1,
                              int l1, float* store0, float* store1, const float* const* cached) {
  const int C = d_.K[1] * d_.Kh;
  const size_t t1comp = 2 * (size_t)d_.M[0] * C;
  Inv0Jobs jobs{};
  int nj = 0;
  const float2* ins[2] = {in0, in1};
  const int lf[2] = {l0, l1};
  const int nnew = in1 ? 2 : 1;
  for (int g = 0; g < nnew; ++g)
    for (int c = 0; c < 3; ++c) {
      jobs.j[nj].in = ins[g] + (size_t)c * d_.nb;
      jobs.j[nj].out = T1_ + (size_t)(g * 3 + c) * t1comp;
      jobs.j[nj].lflag = lf[g];
      ++nj;
    }
  TRY(launch_inv0(jobs, nj, 2, twM_.inv0, Lsym, d_.K[0], C, d_.M[0], st_));
  MStepArgs a{};
  for (int g = 0; g < nnew; ++g) a.t1[g] = T1_ + (size_t)g * 3 * t1comp;
  a.store[0] = store0;
  a.store[1] = store1;
  for (int k = 0; k < 6; ++k) a.cached[k] = cached ? cached[k] : nullptr;
  a.s1 = S1_;
  a.nnew = nnew;
  a.nout = nout;
  a.prog = prog;
  return launch_mstep(a, d_, twM_, st_);
}

// Forward stages 1 and 0 of `nout` padded-grid fields (or of the three
// grid fields when gridN) with the given band epilogues.
hipError_t Engine::fwd_batch(int nout, Fwd0Job* jobs, int njobs, bool gridN) {
  const int C = d_.K[1] * d_.Kh;
  const int* G = gridN ? d_.N : d_.M;
  float2* S1 = gridN ? S1N_ : S1_;
  float2* S2 = gridN ? S2N_ : S2_;
  const Twiddles& tw = gridN ? twN_ : twM_;
  Fwd1Jobs j1{};
  for (int o = 0; o < nout; ++o) {
    j1.j[o].in = S1 + (size_t)o * G[0] * G[1] * d_.Kh;
    j1.j[o].out = S2 + (size_t)o * G[0] * C;
  }
  TRY(launch_fwd1(j1, nout, tw.fwd1, G[0], G[1], d_.K[1], d_.Kh, st_));
  Fwd0Jobs j0{};
  for (int k = 0; k < njobs; ++k) j0.j[k] = jobs[k];
  const float invG = (float)(1.0 / ((double)G[0] * G[1] * G[2]));
  return launch_fwd0(j0, njobs, tw.fwd0, Ksym, G[0], d_.K[0], d_.K[1], d_.Kh, invG, st_);
}

const float2* Engine::s2(int o, bool gridN) const {
  const int C = d_.K[1] * d_.Kh;
  return (gridN ? S2N_ : S2_) + (size_t)o * (gridN ? d_.N[0] : d_.M[0]) * C;
}

// Band fields -> grid velocities vg[n] for the first `count` entries.
hipError_t Engine::grid_velocities(const std::vector<float2*>& bands, int count,
                                   std::vector<float*>& out) {
  const int C = d_.K[1] * d_.Kh;
  const size_t t1 = (size_t)d_.N[0] * C;
  for (int s0 = 0; s0 < count; s0 += kGridChunk) {
    const int ns = std::min(kGridChunk, count - s0);
    Inv0Jobs jobs{};
    int nj = 0;
    for (int s = 0; s < ns; ++s)
      for (int c = 0; c < 3; ++c) {
        jobs.j[nj].in = bands[s0 + s] + (size_t)c * d_.nb;
        jobs.j[nj].out = T1N_ + (size_t)(s * 3 + c) * t1;
        jobs.j[nj].lflag = 0;
        ++nj;
      }
    TRY(launch_inv0(jobs, nj, 1, twN_.inv0, Lsym, d_.K[0], C, d_.N[0], st_));
    for (int s = 0; s < ns; ++s) {
      GridStepArgs a{};
      a.t1 = T1N_ + (size_t)s * 3 * t1;
      a.op = 0;
      a.vout = out[s0 + s];
      TRY(launch_gridstep(a, d_, twN_, st_));
    }
  }
  return hipSuccess;
}

hipError_t Engine::shoot_band(bool cache) {
  const float dt = 1.0f / d_.nt;
  for (int n = 0; n < d_.nt; ++n) {
    float* st0 = cache ? VG[n] : nullptr;
    float* st1 = cache ? VG[n] + 12 * (size_t)d_.nM : nullptr;
    TRY(mstep_step(PROG_SHOOT, 3, V[n], 0, V[n], 1, st0, st1, nullptr));
    Fwd0Job jobs[3];
    for (int c = 0; c < 3; ++c) {
      jobs[c] = Fwd0Job{};
      jobs[c].a = s2(c, false);
      jobs[c].ca = -dt;
      jobs[c].syma = 1;
      jobs[c].base = V[n] + (size_t)c * d_.nb;
      jobs[c].out = V[n + 1] + (size_t)c * d_.nb;
    }
    TRY(fwd_batch(3, jobs, 3, false));
  }
  return hipSuccess;
}

hipError_t Engine::forward(const float* I0) {
  const float dt = 1.0f / d_.nt;
  TRY(shoot_band(true));
  TRY(grid_velocities(V, d_.nt, vg));
  TRY(launch_copy(I0, m[0], d_.nN, st_));
  for (int n = 0; n < d_.nt; ++n) TRY(launch_sl(m[n], vg[n], m[n + 1], dt, d_, st_));
  return hipSuccess;
}

// Shooting and transport without the caches; returns m_nt in *m_out.
hipError_t Engine::forward_light(const float* I0, const float** m_out) {
  const float dt = 1.0f / d_.nt;
  TRY(shoot_band(false));
  std::vector<float*> one(1, vg[0]);
  const float* cur = I0;
  for (int n = 0; n < d_.nt; ++n) {
    std::vector<float2*> b(1, V[n]);
    TRY(grid_velocities(b, 1, one));
    float* dst = mlight[n & 1];
    TRY(launch_sl(cur, vg[0], dst, dt, d_, st_));
    cur = dst;
  }
  *m_out = cur;
  return hipSuccess;
}

hipError_t Engine::energy(const float* mnt, const float* I1) {
  const double sdata = 1.0 / (d_.sigma * d_.sigma * (double)d_.nN);
  TRY(launch_sqdiff(mnt, I1, d_.nN, partial, scal + 2, sdata, st_));
  TRY(launch_band_dot(V[0], V[0], Lsym, d_, partial + 512, scal + 1, 0.5, st_));
  return launch_energy_combine(scal, st_);
}

hipError_t Engine::backward(const float* I1, float2* g_out) {
  const float dt = 1.0f / d_.nt;
  const int nt = d_.nt;
  const float coef = (float)(-2.0 / (d_.sigma * d_.sigma));
  // U_nt = K~ pi(lambda_1 grad_h m_nt), lambda_1 = -(2/sigma^2)(m_nt - I1)
  TRY(launch_src_fwd2(m[nt], I1, m[nt], coef, S1N_, d_, twN_, st_));
  Fwd0Job jobs[9];
  for (int c = 0; c < 3; ++c) {
    jobs[c] = Fwd0Job{};
    jobs[c].a = s2(c, true);
    jobs[c].ca = 1.f;
    jobs[c].syma = 1;
    jobs[c].out = U[nt] + (size_t)c * d_.nb;
  }
  TRY(fwd_batch(3, jobs, 3, true));
  TRY(launch_fill(reinterpret_cast<float*>(W[nt]), 6LL * d_.nb, 0.f, st_));
  for (int n = nt - 1; n >= 0; --n) {
    const float* cached[6] = {VG[n], VG[n] + 12 * (size_t)d_.nM, nullptr, nullptr, nullptr, nullptr};
    TRY(mstep_step(PROG_GRAD, 9, U[n + 1], 1, W[n + 1], 0, UG[n], WG[n], cached));
    for (int c = 0; c < 3; ++c) {
      Fwd0Job& ju = jobs[c];
      ju = Fwd0Job{};
      ju.a = s2(c, false);
      ju.ca = dt;
      ju.syma = 1;
      ju.base = U[n + 1] + (size_t)c * d_.nb;
      ju.out = U[n] + (size_t)c * d_.nb;
      Fwd0Job& jw = jobs[3 + c];
      jw = Fwd0Job{};
      jw.a = s2(3 + c, false);
      jw.ca = -dt;
      jw.syma = 0;
      jw.b = s2(6 + c, false);
      jw.cb = dt;
      jw.symb = 1;
      jw.base = W[n + 1] + (size_t)c * d_.nb;
      jw.extra = U[n + 1] + (size_t)c * d_.nb;
      jw.ce = dt;
      jw.out = W[n] + (size_t)c * d_.nb;
    }
    TRY(fwd_batch(9, jobs, 6, false));
  }
  if (g_out) TRY(launch_axpy_band(V[0], W[0], 1.f, g_out, 3 * d_.nb, st_));
  return hipSuccess;
}

hipError_t Engine::hessvec(const float2* dvh, float2* out) {
  const float dt = 1.0f / d_.nt;
  const int nt = d_.nt;
  const bool coupled = d_.hessian == 0;
  const size_t nM = (size_t)d_.nM;
  if (dvh != dV[0]) TRY(launch_copy(reinterpret_cast<const float*>(dvh), reinterpret_cast<float*>(dV[0]),
                                    6LL * d_.nb, st_));
  // incremental EPDiff forward
  for (int n = 0; n < nt; ++n) {
    const bool last = n == nt - 1;
    if (last && !coupled) break;
    const float* cached[6] = {VG[n], VG[n] + 12 * nM, nullptr, nullptr, nullptr, nullptr};
    float* st0 = coupled ? dVG[n] : nullptr;
    float* st1 = coupled ? dVG[n] + 12 * nM : nullptr;
    TRY(mstep_step(last ? PROG_STORE : PROG_H1, last ? 0 : 3, dV[n], 0, dV[n], 1, st0, st1, cached));
    if (!last) {
      Fwd0Job jobs[3];
      for (int c = 0; c < 3; ++c) {
        jobs[c] = Fwd0Job{};
        jobs[c].a = s2(c, false);
        jobs[c].ca = -dt;
        jobs[c].syma = 1;
        jobs[c].base = dV[n] + (size_t)c * d_.nb;
        jobs[c].out = dV[n + 1] + (size_t)c * d_.nb;
      }
      TRY(fwd_batch(3, jobs, 3, false));
    }
  }
  // incremental state transport
  {
    const int C = d_.K[1] * d_.Kh;
    const size_t t1 = (size_t)d_.N[0] * C;
    const float* dmcur = nullptr;
    for (int s0 = 0; s0 < nt; s0 += kGridChunk) {
      const int ns = std::min(kGridChunk, nt - s0);
      Inv0Jobs jobs{};
      int nj = 0;
      for (int s = 0; s < ns; ++s)
        for (int c = 0; c < 3; ++c) {
          jobs.j[nj].in = dV[s0 + s] + (size_t)c * d_.nb;
          jobs.j[nj].out = T1N_ + (size_t)(s * 3 + c) * t1;
          jobs.j[nj].lflag = 0;
          ++nj;
        }
      TRY(launch_inv0(jobs, nj, 1, twN_.inv0, Lsym, d_.K[0], C, d_.N[0], st_));
      for (int s = 0; s < ns; ++s) {
        const int n = s0 + s;
        GridStepArgs a{};
        a.t1 = T1N_ + (size_t)s * 3 * t1;
        a.op = 1;
        a.m = m[n];
        a.dm = dmcur;
        a.q = q;
        a.dt = dt;
        TRY(launch_gridstep(a, d_, twN_, st_));
        float* dst = dm[n & 1];
        TRY(launch_sl(q, vg[n], dst, dt, d_, st_));
        dmcur = dst;
      }
    }
    // dU_nt = K~ pi(dlambda_1 grad_h m_nt), dlambda_1 = -(2/sigma^2) dm_nt
    const float coef = (float)(-2.0 / (d_.sigma * d_.sigma));
    TRY(launch_src_fwd2(dmcur, nullptr, m[nt], coef, S1N_, d_, twN_, st_));
    Fwd0Job jobs[3];
    for (int c = 0; c < 3; ++c) {
      jobs[c] = Fwd0Job{};
      jobs[c].a = s2(c, true);
      jobs[c].ca = 1.f;
      jobs[c].syma = 1;
      jobs[c].out = dU[0] + (size_t)c * d_.nb;
    }
    TRY(fwd_batch(3, jobs, 3, true));
  }
  // incremental adjoint Jacobi sweep backward
  TRY(launch_fill(reinterpret_cast<float*>(dW[0]), 6LL * d_.nb, 0.f, st_));
  int cur = 0;
  for (int n = nt - 1; n >= 0; --n) {
    const float* cached[6] = {VG[n], VG[n] + 12 * nM, UG[n], WG[n], dVG[n], dVG[n] + 12 * nM};
    TRY(mstep_step(coupled ? PROG_H5 : PROG_H5_NOCOUPLE, 9, dU[cur], 1, dW[cur], 0, nullptr, nullptr,
                   cached));
    Fwd0Job jobs[6];
    for (int c = 0; c < 3; ++c) {
      Fwd0Job& ju = jobs[c];
      ju = Fwd0Job{};
      ju.a = s2(c, false);
      ju.ca = dt;
      ju.syma = 1;
      ju.base = dU[cur] + (size_t)c * d_.nb;
      ju.out = dU[1 - cur] + (size_t)c * d_.nb;
      Fwd0Job& jw = jobs[3 + c];
      jw = Fwd0Job{};
      jw.a = s2(3 + c, false);
      jw.ca = -dt;
      jw.syma = 0;
      jw.b = s2(6 + c, false);
      jw.cb = dt;
      jw.symb = 1;
      jw.base = dW[cur] + (size_t)c * d_.nb;
      jw.extra = dU[cur] + (size_t)c * d_.nb;
      jw.ce = dt;
      jw.out = dW[1 - cur] + (size_t)c * d_.nb;
    }
    TRY(fwd_batch(9, jobs, 6, false));
    cur = 1 - cur;
  }
  return launch_axpy_band(dV[0], dW[cur], 1.f, out, 3 * d_.nb, st_);
}

}  // namespace lddmm
