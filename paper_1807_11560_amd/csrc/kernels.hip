// Device kernels of band-limited Jacobi PDE-EPDiff LDDMM for CDNA4 (gfx950).
//
// Transforms between the band (paper §3.1, truncated Fourier domain) and a
// grid are separable partial DFTs: one contraction per axis, axis 0 first
// (k0 -> x0), then axis 1, then the real-output contraction over the half
// spectrum along axis 2.  The truncated convolution of the band Lie algebra
// (paper §3.1) is evaluated on the padded grid M >= 3K/2 - 2 where it is
// alias-free on the band.  Partial derivatives are folded into the twiddle
// tables of the axis they act on.
#include "common.h"

#include <hip/hip_ext.h>

#include <math.h>

#include <algorithm>
#include <type_traits>

namespace lddmm {

__device__ __forceinline__ void cmac(float2& acc, float2 a, float2 b) {
  acc.x = fmaf(a.x, b.x, acc.x);
  acc.x = fmaf(-a.y, b.y, acc.x);
  acc.y = fmaf(a.x, b.y, acc.y);
  acc.y = fmaf(a.y, b.x, acc.y);
}

// Fills n elements with kBatch loads in flight per thread before their
// stores (a load-then-store loop would wait one memory latency per element):
// load(i) gives the value of flat index i, store(i, v) puts it.
constexpr int kBatch = 8;
template <class T, class Load, class Store>
__device__ __forceinline__ void batched_fill(int n, Load load, Store store) {
  const int stride = blockDim.x;
  for (int i0 = threadIdx.x; i0 < n; i0 += stride * kBatch) {
    T v[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int i = i0 + u * stride;
      if (i < n) v[u] = load(i);
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int i = i0 + u * stride;
      if (i < n) store(i, v[u]);
    }
  }
}

// Two-phase copy for 256-thread blocks with every load of a thread in
// flight at once: load() fills r[u] for element i = threadIdx.x + 256 u
// (u < CAP, i < n), store() puts them.  The caller guarantees n <= 256 CAP.
// Every lane of a slot with any element loads (a lane past the end reads
// element n - 1 again): loads under a per-lane branch would make the
// branch's merge wait for every load in flight, which serialises the
// caller's later loads behind them.  Slots past the end are skipped (a
// condition that is the same for the whole block).
template <int CAP, class T>
struct RegStage {
  T r[CAP];
  template <class Load>
  __device__ __forceinline__ void load(int n, Load f) {
#pragma unroll
    for (int u = 0; u < CAP; ++u) {
      if (256 * u >= n) break;
      const int i = threadIdx.x + 256 * u;
      r[u] = f(i < n ? i : n - 1);
    }
  }
  template <class Store>
  __device__ __forceinline__ void store(int n, Store f) const {
#pragma unroll
    for (int u = 0; u < CAP; ++u) {
      const int i = threadIdx.x + 256 * u;
      if (i < n) f(i, r[u]);
    }
  }
};

__device__ __forceinline__ float4 ld4(const float2* p) { return *reinterpret_cast<const float4*>(p); }
__device__ __forceinline__ void st4(float2* p, float4 v) { *reinterpret_cast<float4*>(p) = v; }
// two complex values to an 8-byte aligned LDS address (rows of odd complex
// stride, which keep an MFMA operand's 16 rows in distinct banks)
__device__ __forceinline__ void st22(float2* p, float4 v) {
  p[0] = make_float2(v.x, v.y);
  p[1] = make_float2(v.z, v.w);
}

// ---------------------------------------------------------------- shapes
// Sizes seen by a kernel: compile-time for the shapes this library is tuned
// for (index arithmetic then folds into constants), runtime otherwise.
struct BandDyn {
  static constexpr bool kStatic = false;
  int k0, k1, kh, m0, m1, m2;
  __device__ __forceinline__ int K0() const { return k0; }
  __device__ __forceinline__ int K1() const { return k1; }
  __device__ __forceinline__ int Kh() const { return kh; }
  __device__ __forceinline__ int M0() const { return m0; }
  __device__ __forceinline__ int M1() const { return m1; }
  __device__ __forceinline__ int M2() const { return m2; }
};
template <int K, int M>
struct BandIso {
  static constexpr bool kStatic = true;
  __device__ static constexpr int K0() { return K; }
  __device__ static constexpr int K1() { return K; }
  __device__ static constexpr int Kh() { return K / 2; }
  __device__ static constexpr int M0() { return M; }
  __device__ static constexpr int M1() { return M; }
  __device__ static constexpr int M2() { return M; }
};
struct GridDyn {
  static constexpr bool kStatic = false;
  int n0, n1, n2, k1, kh;
  __device__ __forceinline__ int N0() const { return n0; }
  __device__ __forceinline__ int N1() const { return n1; }
  __device__ __forceinline__ int N2() const { return n2; }
  __device__ __forceinline__ int K1() const { return k1; }
  __device__ __forceinline__ int Kh() const { return kh; }
};
template <int A, int B, int C, int K>
struct GridShape {
  static constexpr bool kStatic = true;
  __device__ static constexpr int N0() { return A; }
  __device__ static constexpr int N1() { return B; }
  __device__ static constexpr int N2() { return C; }
  __device__ static constexpr int K1() { return K; }
  __device__ static constexpr int Kh() { return K / 2; }
};
template <int N, int K>
using GridIso = GridShape<N, N, N, K>;

// ------------------------------------------------------------- tables
// mode 0: inverse, full axis  [2][G][K]
// mode 1: inverse, half axis  [2][G][K/2], weight 1 at k = 0 else 2
// mode 2: forward, full axis  [K][G]
// mode 3: forward, half axis  [K/2][G]
__global__ void k_twiddles(float2* dst, int K, int G, int mode) {
  const int Kq = (mode == 1 || mode == 3) ? K / 2 : K;
  const int total = (mode <= 1) ? 2 * G * Kq : Kq * G;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  int v = 0, x, q;
  if (mode <= 1) {
    v = i / (G * Kq);
    x = (i / Kq) % G;
    q = i % Kq;
  } else {
    q = i / G;
    x = i % G;
  }
  const bool half = (mode == 1 || mode == 3);
  const int k = half ? q : (q < K / 2 ? q : q - K);
  if (!half && q == K / 2) { dst[i] = make_float2(0.f, 0.f); return; }
  long long r = ((long long)k * x) % G;
  if (r < 0) r += G;
  double s, c;
  sincospi(2.0 * (double)r / (double)G, &s, &c);
  double re = c, im = (mode >= 2) ? -s : s;
  if (mode <= 1 && v == 1) {  // times 2 pi i k
    const double w = 2.0 * M_PI * (double)k;
    const double nre = -w * im, nim = w * re;
    re = nre;
    im = nim;
  }
  if (mode == 1 && q > 0) { re *= 2.0; im *= 2.0; }
  dst[i] = make_float2((float)re, (float)im);
}

// L~ and K~ = 1 / L~ at the band slot (q0, q1, k2) (FP64, rounded once);
// kernels that need a few symbols per thread form them here instead of
// loading them from the tables.
__device__ __forceinline__ float2 band_symbols(int q0, int q1, int k2, int K0, int K1, int s, double alpha) {
  const int k0 = q0 < K0 / 2 ? q0 : q0 - K0;
  const int k1 = q1 < K1 / 2 ? q1 : q1 - K1;
  const double tp = 2.0 * M_PI;
  const double lap = tp * tp * ((double)k0 * k0 + (double)k1 * k1 + (double)k2 * k2);
  const double base = 1.0 + alpha * lap;
  double L = 1.0;
  for (int e = 0; e < s; ++e) L *= base;
  return make_float2((float)L, (float)(1.0 / L));
}

__global__ void k_symbols(float* Lsym, float* Ksym, int K0, int K1, int Kh, int s, double alpha) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K0 * K1 * Kh) return;
  // band layout [Kh][K0][K1]
  const float2 lk = band_symbols((i / K1) % K0, i % K1, i / (K0 * K1), K0, K1, s, alpha);
  Lsym[i] = lk.x;
  Ksym[i] = lk.y;
}

// ------------------------------------------------------- layout changes
// full [3][K0][K1][K2] -> half [3][Kh][K0][K1], projecting onto Hermitian
// fields on the effective band.
__global__ void k_full_to_half(const float2* __restrict__ full, float2* __restrict__ half, int K0,
                               int K1, int K2) {
  const int Kh = K2 / 2;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * K0 * K1 * Kh) return;
  int c = i / (K0 * K1 * Kh);
  int q2 = (i / (K0 * K1)) % Kh, q0 = (i / K1) % K0, q1 = i % K1;
  if (q0 == K0 / 2 || q1 == K1 / 2) { half[i] = make_float2(0.f, 0.f); return; }
  const float2* f = full + (size_t)c * K0 * K1 * K2;
  float2 a = f[((size_t)q0 * K1 + q1) * K2 + q2];
  int r0 = (K0 - q0) % K0, r1 = (K1 - q1) % K1, r2 = (K2 - q2) % K2;
  float2 b = f[((size_t)r0 * K1 + r1) * K2 + r2];
  half[i] = make_float2(0.5f * (a.x + b.x), 0.5f * (a.y - b.y));
}

// full = expand(a + cb*b)
__global__ void k_half_to_full(const float2* __restrict__ a, const float2* __restrict__ b, float cb,
                               const float* __restrict__ sym, float2* __restrict__ full, int K0, int K1,
                               int K2) {
  const int Kh = K2 / 2;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * K0 * K1 * K2) return;
  int c = i / (K0 * K1 * K2);
  int q0 = (i / (K1 * K2)) % K0, q1 = (i / K2) % K1, q2 = i % K2;
  if (q0 == K0 / 2 || q1 == K1 / 2 || q2 == K2 / 2) { full[i] = make_float2(0.f, 0.f); return; }
  bool conj = q2 > Kh;
  int s0 = conj ? (K0 - q0) % K0 : q0, s1 = conj ? (K1 - q1) % K1 : q1, s2 = conj ? K2 - q2 : q2;
  auto value = [&](int t0, int t1, int t2) {
    const size_t jb = ((size_t)t2 * K0 + t0) * K1 + t1;  // band layout [Kh][K0][K1]
    const size_t j = (size_t)c * K0 * K1 * Kh + jb;
    float2 v = a[j];
    if (b) { v.x += cb * b[j].x; v.y += cb * b[j].y; }
    if (sym) {
      const float w = sym[jb];
      v.x *= w;
      v.y *= w;
    }
    return v;
  };
  float2 v = value(s0, s1, s2);
  if (q2 == 0) {
    // the k2 = 0 plane holds both v(k0, k1, 0) and v(-k0, -k1, 0): its
    // Hermitian part, formed so that the two results are exact conjugates
    const float2 w = value((K0 - q0) % K0, (K1 - q1) % K1, 0);
    v = make_float2(0.5f * (v.x + w.x), 0.5f * (v.y - w.y));
  }
  if (conj) v.y = -v.y;
  full[i] = v;
}

// ------------------------------------------------- inverse stage 0 (k0)
// out[v][x0][kh][k1] = sum_k0 tw[v][x0][k0] * in[kh][k0][k1] (optionally in * L~):
// column c = kh K1 + k1 of the output reads in[c / K1][k0][c % K1].
// KC > 0: compile-time K0 = KC (all loads of a column issued before use).
template <int NV, int XT, int KC>
__global__ void __launch_bounds__(128) k_inv0(Inv0Jobs jobs, const float2* __restrict__ tw,
                                              const float* __restrict__ Lsym, int K0r, int C,
                                              int G0, int Kh) {
  const int K0 = KC > 0 ? KC : K0r;
  extern __shared__ float2 sh[];
  const Inv0Job job = jobs.j[blockIdx.z];
  const int xb = blockIdx.y * XT;
  batched_fill<float2>(NV * XT * K0, [&](int i) {
    int v = i / (XT * K0), t = (i / K0) % XT, k = i % K0;
    int x = xb + t;
    return (x < G0) ? tw[((size_t)v * G0 + x) * K0 + k] : make_float2(0.f, 0.f);
  }, [&](int i, float2 v) { sh[i] = v; });
  __syncthreads();
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const int K1 = C / Kh;
  const size_t cin = (size_t)(c / K1) * K0 * K1 + c % K1;  // (kh, k1) of column c, k0 = 0
  float2 acc[NV][XT];
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int t = 0; t < XT; ++t) acc[v][t] = make_float2(0.f, 0.f);
  // columns in chunks of eight: the chunk's loads are in flight together
#pragma unroll 1
  for (int k0 = 0; k0 < K0; k0 += 8) {
    float2 col[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) col[u] = (k0 + u < K0) ? job.in[cin + (size_t)(k0 + u) * K1] : make_float2(0.f, 0.f);
    if (job.lflag) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        float l = (k0 + u < K0) ? Lsym[cin + (size_t)(k0 + u) * K1] : 0.f;
        col[u].x *= l;
        col[u].y *= l;
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (k0 + u >= K0) break;
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int t = 0; t < XT; ++t) cmac(acc[v][t], sh[(v * XT + t) * K0 + k0 + u], col[u]);
    }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int t = 0; t < XT; ++t) {
      int x = xb + t;
      if (x < G0) job.out[((size_t)v * G0 + x) * C + c] = acc[v][t];
    }
}

// --------------------------------------------- band Lie algebra products
// Group layout: 12 scalar fields of one vector field f: f_c at index c,
// d_i f_c at index 3 + 3c + i.
// (ad*_a mu)_i = sum_j (d_i a_j) mu_j + (d_j mu_i) a_j + mu_i (d_j a_j)
__device__ __forceinline__ void adstar_acc(float* o, const float* a, const float* mu, float s) {
  const float diva = a[3] + a[7] + a[11];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    float r = mu[i] * diva;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      r = fmaf(a[3 + 3 * j + i], mu[j], r);
      r = fmaf(mu[3 + 3 * i + j], a[j], r);
    }
    o[i] = fmaf(s, r, o[i]);
  }
}

// (ad_a b)_i = sum_j (d_j a_i) b_j - (d_j b_i) a_j
__device__ __forceinline__ void ad_acc(float* o, const float* a, const float* b, float s) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    float r = 0.f;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      r = fmaf(a[3 + 3 * i + j], b[j], r);
      r = fmaf(-b[3 + 3 * i + j], a[j], r);
    }
    o[i] = fmaf(s, r, o[i]);
  }
}

// (D~a * b)_i += sum_j (d_j a_i) b_j; ja[3 i + j] = d_j a_i
__device__ __forceinline__ void jac_acc(float* o, const float* ja, const float* b) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) o[i] = fmaf(ja[3 * i + j], b[j], o[i]);
}

// ((D~a)^T * r)_j += sum_i (d_j a_i) r_i
__device__ __forceinline__ void jact_acc(float* o, const float* ja, const float* r) {
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int i = 0; i < 3; ++i) o[j] = fmaf(ja[3 * i + j], r[i], o[j]);
}

// ------------------------------------------- MFMA synthesis on the padded grid
// One block per (x0 plane, new field (g, c)), four waves.  The inverse
// stages 1 (k1 -> x1, complex) and 2 (half spectrum k2 -> real x2) are two
// real GEMMs on the matrix cores (v_mfma_f32_16x16x4f32, FP32 in, FP32
// accumulate):
//   T2 = [W1r | -W1i] [[T1r, T1i], [T1i, -T1r]]        rows x1, cols (kh re | kh im)
//   f  = [T2r | T2i] [[w2r], [-w2i]]                   rows x1, cols x2
// for the variants value, d/dx2 (pp with the derivative stage-2 table), d/dx1
// (stage-1 derivative table) and d/dx0 (stage-0 derivative input).  The
// four results go to the group's field array [3][nM][4]: per component and
// padded-grid point (value, d/dx0, d/dx1, d/dx2).
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef short shortx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

// Compensated BF16 products on the matrix cores (precision LDDMM_FP32_BF16X3):
// each FP32 operand x is split as hi = bf16(x), lo = bf16(x - hi) (round to
// nearest even both times), and a b is formed as ah bh + ah bl + al bh with
// FP32 accumulation; the dropped al bl is about 2^-16 of a b.  One FP32
// k-step of v_mfma_f32_16x16x4f32 becomes one v_mfma_f32_16x16x16_bf16 whose
// four k slots per lane hold the three terms and a zero: the A operand
// (ah, ah, al, 0), the B operand (bh, bl, bh, 0).  Both operands index k
// by (lane / 16, slot) alike, so the slot order only has to pair the terms.
__device__ __forceinline__ shortx4 bf3_a(float x) {
  const __bf16 h = (__bf16)x;
  const __bf16 l = (__bf16)(x - (float)h);
  const bf16x4 v = {h, h, l, (__bf16)0.f};
  return __builtin_bit_cast(shortx4, v);
}
__device__ __forceinline__ shortx4 bf3_b(float x) {
  const __bf16 h = (__bf16)x;
  const __bf16 l = (__bf16)(x - (float)h);
  const bf16x4 v = {h, l, h, (__bf16)0.f};
  return __builtin_bit_cast(shortx4, v);
}
__device__ __forceinline__ floatx4 mma_bf3(shortx4 a, shortx4 b, floatx4 acc) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
}
// acc += a b over one k-step of a 16x16 tile (lane layout of
// v_mfma_f32_16x16x4f32: A[row = lane % 16][k = lane / 16], B[k][col = lane % 16]).
template <bool BF3>
__device__ __forceinline__ floatx4 mma(float a, float b, floatx4 acc) {
  if constexpr (BF3)
    return mma_bf3(bf3_a(a), bf3_b(b), acc);
  else
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
}

struct SynthArgs {
  const float2* t1[2];  // stage-0 output of group g: [3][2][M0][K1*Kh]
  float* dst[2];        // fields of group g: [3][nM][4] (value, d0, d1, d2)
  const float* w1a;     // [2][M1p][2K1]    real block form of the stage-1 twiddles
  const float* w2b;     // [2][2Khp][M2p]   real block form of the stage-2 twiddles
};

constexpr int kSynthW2Pre = 16;
constexpr int kSynthT = 3;  // tiles a wave computes together
template <class S, bool BF3>
__global__ void __launch_bounds__(256) k_synth(SynthArgs a, S sh) {
  extern __shared__ float sms[];
  const int M0 = sh.M0(), M1 = sh.M1(), M2 = sh.M2(), K1 = sh.K1(), Kh = sh.Kh();
  const int M1p = (M1 + 15) & ~15, M2p = (M2 + 15) & ~15, Khp = (Kh + 7) & ~7;
  const int x0 = blockIdx.x;
  const int g = blockIdx.y / 3, c = blockIdx.y % 3;
  const int rt = blockIdx.z;  // 16-row tile of x1
  const int C = K1 * Kh;
  const int K2r = 2 * K1;    // GEMM1 depth
  const int N1 = 2 * Khp;    // GEMM1 width = GEMM2 depth
  // LDS strides: the 16 rows an MFMA operand reads lie in distinct banks
  // (row strides of 2 mod 4 floats for operands read along rows, 16 mod 32
  // for the stage-2 table read across rows)
  const int lda1 = K2r + 2, ldt2 = N1 + 2, ldbT = K2r + 2;
  const int ldw2 = (M2p % 32 == 0) ? M2p + 16 : M2p;
  const int nbt = 2 * N1 * (ldbT > ldw2 ? ldbT : ldw2);
  float* w1s = sms;                          // [2][16][lda1]   stage-1 rows of this tile
  float* bt1 = w1s + 2 * 16 * lda1;          // [2][N1][ldbT]   stage-0 input, transposed; then [2][N1][ldw2]
  float* t2s = bt1 + nbt;                    // [3][16][ldt2]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  (void)M1p;
  // The stage-2 table w2b [2][N1][M2p] is loaded into registers during GEMM1
  // (issued after the first barrier, which then waits for GEMM1's operands
  // alone) and put into the LDS of bt1 once GEMM1 has consumed it (when it
  // fits; else GEMM2 reads it from global memory).
  const int nw2 = 2 * N1 * M2p;
  const bool w2_lds = nw2 <= 256 * kSynthW2Pre;
  RegStage<kSynthW2Pre / 4, float4> rw2;
  const float2* src = a.t1[g] + (size_t)c * 2 * M0 * C;
  auto put_t1 = [&](int vs, int k1, int kh, float2 t) {  // B[k][col] kept as bT[col][k]
    float* b = bt1 + (size_t)vs * N1 * ldbT;
    b[(size_t)kh * ldbT + k1] = t.x;
    b[(size_t)(Khp + kh) * ldbT + k1] = t.y;
    b[(size_t)kh * ldbT + K1 + k1] = t.y;
    b[(size_t)(Khp + kh) * ldbT + K1 + k1] = -t.x;
  };
  // stage-1 table rows of this tile: w1a [2][M1p][K2r]
  const float* w1rows = a.w1a + (size_t)rt * 16 * K2r;
  const size_t w1var = (size_t)M1p * K2r;
  if constexpr (S::kStatic) {
    // the loads of GEMM1's operands in flight at once, four floats per load
    constexpr int sM1p = (S::M1() + 15) & ~15, sK1 = S::K1(), sKh = S::Kh(), sKhp = (sKh + 7) & ~7;
    constexpr int sK2r = 2 * sK1, KP = sK1 / 2, R4 = sK2r / 4;
    constexpr int NW1 = 2 * 16 * R4, NT1 = 2 * sKhp * KP;
    static_assert(sK1 % 2 == 0, "pairs of k1 per load");
    RegStage<(NW1 + 255) / 256, float4> rw1;
    RegStage<(NT1 + 255) / 256, float4> rt1;
    rw1.load(NW1, [&](int i) {
      const int vv = i / (16 * R4), row = (i / R4) % 16, k = 4 * (i % R4);
      return *reinterpret_cast<const float4*>(w1rows + vv * (size_t)sM1p * sK2r + (size_t)row * sK2r + k);
    });
    // the padding columns kh >= Kh load a valid row and are zeroed when stored
    // (a load under a per-lane condition would wait for every load in flight)
    rt1.load(NT1, [&](int i) {
      const int vs = i / (sKhp * KP), kh = (i / KP) % sKhp, k1 = 2 * (i % KP);
      return ld4(src + ((size_t)vs * M0 + x0) * C + (size_t)(kh < sKh ? kh : sKh - 1) * sK1 + k1);
    });
    rw1.store(NW1, [&](int i, float4 v) {
      const int vv = i / (16 * R4), row = (i / R4) % 16, k = 4 * (i % R4);
      float* d = w1s + ((size_t)vv * 16 + row) * lda1 + k;
      d[0] = v.x;
      d[1] = v.y;
      d[2] = v.z;
      d[3] = v.w;
    });
    rt1.store(NT1, [&](int i, float4 v) {
      const int vs = i / (sKhp * KP), kh = (i / KP) % sKhp, k1 = 2 * (i % KP);
      if (kh >= sKh) v = make_float4(0.f, 0.f, 0.f, 0.f);
      put_t1(vs, k1, kh, make_float2(v.x, v.y));
      put_t1(vs, k1 + 1, kh, make_float2(v.z, v.w));
    });
  } else {
    batched_fill<float>(2 * 16 * K2r, [&](int i) {
      const int vv = i / (16 * K2r), row = (i / K2r) % 16, k = i % K2r;
      return w1rows[vv * w1var + (size_t)row * K2r + k];
    }, [&](int i, float v) {
      const int vv = i / (16 * K2r), row = (i / K2r) % 16, k = i % K2r;
      w1s[((size_t)vv * 16 + row) * lda1 + k] = v;
    });
    batched_fill<float2>(2 * K1 * Khp, [&](int i) {
      int vs = i / (K1 * Khp), k1 = (i / Khp) % K1, kh = i % Khp;
      return (kh < Kh) ? src[((size_t)vs * M0 + x0) * C + (size_t)kh * K1 + k1] : make_float2(0.f, 0.f);
    }, [&](int i, float2 t) {
      int vs = i / (K1 * Khp), k1 = (i / Khp) % K1, kh = i % Khp;
      put_t1(vs, k1, kh, t);
    });
  }
  __syncthreads();
  if (w2_lds) rw2.load(nw2 / 4, [&](int i) { return reinterpret_cast<const float4*>(a.w2b)[i]; });
  // GEMM1 on this tile's 16 rows: var 0 = pp (plain stage 0, plain stage 1),
  // 1 = p1 (d1), 2 = 0p (d0 input).  Wave w takes tiles w, w + 4, w + 8, ...
  // and runs up to kSynthT of them at once, their matrix instructions
  // interleaved, operands fetched four k-steps ahead.
  const int tj1 = N1 / 16, nj1 = 3 * tj1;
  auto gemm1 = [&](auto TT, int j0) {
    constexpr int T = decltype(TT)::value;
    const float* A[T];
    const float* B[T];
    floatx4 acc[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int job = j0 + 4 * t;
      const int var = job / tj1, tj = job % tj1;
      const int vs = (var == 2), vt = (var == 1);
      A[t] = w1s + ((size_t)vt * 16 + li) * lda1 + lk;
      B[t] = bt1 + ((size_t)vs * N1 + tj * 16 + li) * ldbT + lk;
      acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
    for (int k0 = 0; k0 < K2r / 4; k0 += 4) {
      float av[T][4], bv[T][4];
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int ks = k0 + u;
          av[t][u] = (ks < K2r / 4) ? A[t][4 * ks] : 0.f;
          bv[t][u] = (ks < K2r / 4) ? B[t][4 * ks] : 0.f;
        }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int t = 0; t < T; ++t)
          acc[t] = mma<BF3>(av[t][u], bv[t][u], acc[t]);
    }
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int job = j0 + 4 * t;
      const int var = job / tj1, tj = job % tj1;
      float* Tp = t2s + ((size_t)var * 16 + 4 * lk) * ldt2 + tj * 16 + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) Tp[(size_t)r * ldt2] = acc[t][r];
    }
  };
  static_assert(kSynthT == 3, "tile groups of one to three");
  for (int j0 = wave; j0 < nj1; j0 += 4 * kSynthT) {
    const int cnt = min(kSynthT, (nj1 - j0 + 3) / 4);
    if (cnt == 3)
      gemm1(std::integral_constant<int, 3>{}, j0);
    else if (cnt == 2)
      gemm1(std::integral_constant<int, 2>{}, j0);
    else
      gemm1(std::integral_constant<int, 1>{}, j0);
  }
  __syncthreads();
  const float* w2src = a.w2b;
  int w2ld = M2p;
  if (w2_lds) {
    rw2.store(nw2 / 4, [&](int i, float4 v) {
      *reinterpret_cast<float4*>(bt1 + (size_t)((4 * i) / M2p) * ldw2 + (4 * i) % M2p) = v;
    });
    __syncthreads();
    w2src = bt1;
    w2ld = ldw2;
  }
  // GEMM2: ov 0 = value (pp, plain), 1 = d2 (pp, derivative table), 2 = d1 (p1), 3 = d0 (0p).
  // A wave forms all four for one 16-column tile, so that each point's
  // (value, d0, d1, d2) leaves as one 16-byte store.
  const int tj2 = M2p / 16;
  const long long nM = (long long)M0 * M1 * M2;
  float* out = a.dst[g] + (size_t)c * nM * 4;
  for (int tj = wave; tj < tj2; tj += 4) {
    const float* A[4];
    const float* B[4];
    floatx4 acc[4];
#pragma unroll
    for (int ov = 0; ov < 4; ++ov) {
      const int srcv = (ov <= 1) ? 0 : (ov == 2 ? 1 : 2);
      const int wv = (ov == 1);
      A[ov] = t2s + ((size_t)srcv * 16 + li) * ldt2 + lk;
      B[ov] = w2src + ((size_t)wv * N1 + lk) * w2ld + tj * 16 + li;
      acc[ov] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
    for (int k0 = 0; k0 < N1 / 4; k0 += 4) {
      float av[4][4], bv[4][4];
#pragma unroll
      for (int ov = 0; ov < 4; ++ov)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int ks = k0 + u;
          bv[ov][u] = (ks < N1 / 4) ? B[ov][(size_t)4 * ks * w2ld] : 0.f;
          av[ov][u] = (ks < N1 / 4) ? A[ov][4 * ks] : 0.f;
        }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int ov = 0; ov < 4; ++ov)
          acc[ov] = mma<BF3>(av[ov][u], bv[ov][u], acc[ov]);
    }
    const int x2 = tj * 16 + li;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int x1 = rt * 16 + 4 * lk + r;
      if (x1 < M1 && x2 < M2)
        *reinterpret_cast<float4*>(out + 4 * (((long long)x0 * M1 + x1) * M2 + x2)) =
            make_float4(acc[0][r], acc[3][r], acc[2][r], acc[1][r]);
    }
  }
}

// MFMA-friendly real forms of the stage-1 and stage-2 inverse twiddles.
__global__ void k_synth_tables(const float2* inv1, const float2* inv2, float* w1a, float* w2b, int M1,
                               int M2, int K1, int Kh, int M1p, int M2p, int Khp) {
  const int n1 = 2 * M1p * 2 * K1;
  const int n2 = 2 * 2 * Khp * M2p;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n1) {
    int v = i / (M1p * 2 * K1), row = (i / (2 * K1)) % M1p, k = i % (2 * K1);
    float val = 0.f;
    if (row < M1) {
      float2 w = inv1[((size_t)v * M1 + row) * K1 + (k < K1 ? k : k - K1)];
      val = (k < K1) ? w.x : -w.y;
    }
    w1a[i] = val;
  } else if (i < n1 + n2) {
    int e = i - n1;
    int v = e / (2 * Khp * M2p), j = (e / M2p) % (2 * Khp), x2 = e % M2p;
    int kh = (j < Khp) ? j : j - Khp;
    float val = 0.f;
    if (x2 < M2 && kh < Kh) {
      float2 w = inv2[((size_t)v * M2 + x2) * Kh + kh];
      val = (j < Khp) ? w.x : -w.y;
    }
    w2b[e] = val;
  }
}

// ------------------------------------------------ Lie products on the padded grid
// One block per (x0, R rows), one thread per point (R*M2 threads).  Reads
// the new and cached groups, forms the products of the program and
// contracts them over x2 (forward stage 2) into s1[o][kh][x0][x1]: on the
// matrix cores when M2 % 4 == 0 (rows (o, r) x columns (kh re | kh im), depth
// x2), else one thread per output.
template <class S, bool BF3>
__global__ void __launch_bounds__(256) k_prods(ProdArgs a, Twiddles tw, S sh, int R) {
  // R: padded-grid rows of this block (R M2 <= blockDim.x rounded to waves)
  extern __shared__ float smp[];
  const int M0 = sh.M0(), M1 = sh.M1(), M2 = sh.M2(), Kh = sh.Kh();
  const int x0 = blockIdx.y;
  const int x1b = blockIdx.x * R;
  const int rv = min(R, M1 - x1b);
  const int P = R * M2;
  const int LV = M2 + 2;  // product rows: 2 mod 4 floats, an MFMA A operand read along rows
  const long long nM = (long long)M0 * M1 * M2;
  float2* wfx = (float2*)smp;                  // [M2][Kh]
  float* outv = (float*)(wfx + M2 * Kh);       // [nout][R][LV]
  // the stage-2 table goes to LDS after the products (its loads overlap theirs)
  const int nw = M2 * Kh;
  const bool wreg = nw <= 256 * 4 && blockDim.x == 256;  // the register stage covers 256 threads
  RegStage<4, float2> rw;
  if (wreg) rw.load(nw, [&](int i) { return tw.fwd2[(size_t)(i % Kh) * M2 + i / Kh]; });
  for (int p = threadIdx.x; p < P; p += blockDim.x) {
    const int r = p / M2;
    float o[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) o[i] = 0.f;
    if (r < rv) {
      const long long gp = ((long long)x0 * M1 + x1b) * M2 + p;
      // a group is [3][nM][4]: per component i and point (a_i, d_0 a_i, d_1 a_i, d_2 a_i)
      auto get = [&](const float* base, float* dst) {  // dst[i] = a_i, dst[3 + 3 i + j] = d_j a_i
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const float4 v = *reinterpret_cast<const float4*>(base + ((size_t)i * nM + gp) * 4);
          dst[i] = v.x;
          dst[3 + 3 * i] = v.y;
          dst[4 + 3 * i] = v.z;
          dst[5 + 3 * i] = v.w;
        }
      };
      auto get_jac = [&](const float* base, float* dst) {  // dst[3 i + j] = d_j a_i
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const float4 v = *reinterpret_cast<const float4*>(base + ((size_t)i * nM + gp) * 4);
          dst[3 * i] = v.y;
          dst[3 * i + 1] = v.z;
          dst[3 * i + 2] = v.w;
        }
      };
      auto get_val = [&](const float* base, float* dst) {
#pragma unroll
        for (int i = 0; i < 3; ++i) dst[i] = base[((size_t)i * nM + gp) * 4];
      };
      // every group the program needs is loaded before any product is formed
      switch (a.prog) {
        case PROG_SHOOT: {  // g: V, LV
          float gV[12], gLV[12];
          get(a.g[0], gV);
          get(a.g[1], gLV);
          adstar_acc(o, gV, gLV, 1.f);
          break;
        }
        case PROG_H1: {  // g: dV, LdV, V, LV
          float gdV[12], gLdV[12], gV[12], gLV[12];
          get(a.g[0], gdV);
          get(a.g[1], gLdV);
          get(a.g[2], gV);
          get(a.g[3], gLV);
          adstar_acc(o, gdV, gLV, 1.f);   // ad*_dV(LV)
          adstar_acc(o, gV, gLdV, 1.f);   // ad*_V(LdV)
          break;
        }
        case PROG_GRAD:           // g: LU, W, V, LV
        case PROG_H5_NOCOUPLE: {  // g: LdU, dW, V, LV
          float gLU[12], gW[12], gV[12], gLV[12];
          get(a.g[0], gLU);
          get(a.g[1], gW);
          get(a.g[2], gV);
          get(a.g[3], gLV);
          adstar_acc(o, gV, gLU, 1.f);     // ad*_V(LU)
          ad_acc(o + 3, gV, gW, 1.f);      // ad_V(W)
          adstar_acc(o + 6, gW, gLV, 1.f); // ad*_W(LV)
          break;
        }
        case PROG_ADJ: {  // g: W, V, LV
          float gW[12], gV[12], gLV[12];
          get(a.g[0], gW);
          get(a.g[1], gV);
          get(a.g[2], gLV);
          ad_acc(o, gV, gW, 1.f);          // ad_V(W)
          adstar_acc(o + 3, gW, gLV, 1.f); // ad*_W(LV)
          break;
        }
        case PROG_H5: {  // g: LdU, dW, V, LV, LU, W, dV, LdV
          float gLdU[12], gdW[12], gV[12], gLV[12], gLU[12], gW[12], gdV[12], gLdV[12];
          get(a.g[0], gLdU);
          get(a.g[1], gdW);
          get(a.g[2], gV);
          get(a.g[3], gLV);
          get(a.g[4], gLU);
          get(a.g[5], gW);
          get(a.g[6], gdV);
          get(a.g[7], gLdV);
          adstar_acc(o, gV, gLdU, 1.f);      // ad*_V(LdU)
          ad_acc(o + 3, gV, gdW, 1.f);       // ad_V(dW)
          adstar_acc(o + 6, gdW, gLV, 1.f);  // ad*_dW(LV)
          adstar_acc(o, gdV, gLU, 1.f);      // ad*_dV(LU)
          ad_acc(o + 3, gdV, gW, 1.f);       // ad_dV(W)
          adstar_acc(o + 6, gW, gLdV, 1.f);  // ad*_W(LdV)
          break;
        }
        case PROG_DEF_FWD: {  // g: Phi, V
          float jP[9], gV[3];
          get_jac(a.g[0], jP);
          get_val(a.g[1], gV);
          jac_acc(o, jP, gV);
          break;
        }
        case PROG_DEF_H: {  // g: dPhi, V, Phi, dV
          float jdP[9], gV[3], jP[9], gdV[3];
          get_jac(a.g[0], jdP);
          get_val(a.g[1], gV);
          get_jac(a.g[2], jP);
          get_val(a.g[3], gdV);
          jac_acc(o, jdP, gV);
          jac_acc(o, jP, gdV);
          break;
        }
        case PROG_DEF_TAIL: {  // g: A, R
          float jA[9], gR[3];
          get_jac(a.g[0], jA);
          get_val(a.g[1], gR);
          jact_acc(o, jA, gR);
          break;
        }
        case PROG_DEF_HTAIL: {  // g: dPhi, dR, Phi, R
          float jdP[9], gdR[3], jP[9], gR[3];
          get_jac(a.g[0], jdP);
          get_val(a.g[1], gdR);
          get_jac(a.g[2], jP);
          get_val(a.g[3], gR);
          jact_acc(o, jdP, gR);
          jact_acc(o, jP, gdR);
          break;
        }
        default:
          break;
      }
    }
    if (p < P)
      for (int i = 0; i < a.nout; ++i) outv[((size_t)i * R + p / M2) * LV + p % M2] = o[i];
  }
  if (wreg)
    rw.store(nw, [&](int i, float2 v) { wfx[i] = v; });
  else
    batched_fill<float2>(nw, [&](int i) { return tw.fwd2[(size_t)(i % Kh) * M2 + i / Kh]; },
                         [&](int i, float2 v) { wfx[i] = v; });
  __syncthreads();
  if (M2 % 4 == 0) {
    // forward stage 2 on the matrix cores: D[row][kh] = sum_x2 outv[row][x2] fwd2[kh][x2],
    // row = o R + r, one 16-row tile (re and im columns of 16 kh) per wave and step
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const int rows = a.nout * R, trow = (rows + 15) / 16, tcol = (Kh + 15) / 16;
    for (int t = wave; t < trow * tcol; t += (int)(blockDim.x >> 6)) {
      const int ti = t / tcol, tj = t % tcol;
      const int arow = ti * 16 + li, kh = tj * 16 + li;
      const float* A = outv + (size_t)(arow < rows ? arow : 0) * LV + lk;
      const float2* B = wfx + (size_t)lk * Kh + (kh < Kh ? kh : 0);
      floatx4 dre = {0.f, 0.f, 0.f, 0.f}, dim = {0.f, 0.f, 0.f, 0.f};
      for (int ks = 0; ks < M2 / 4; ++ks) {
        const float av = (arow < rows) ? A[4 * ks] : 0.f;
        const float2 bv = (kh < Kh) ? B[(size_t)4 * ks * Kh] : make_float2(0.f, 0.f);
        dre = mma<BF3>(av, bv.x, dre);
        dim = mma<BF3>(av, bv.y, dim);
      }
      if (kh < Kh) {
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const int row = ti * 16 + 4 * lk + rr;
          const int o = row / R, r = row % R;
          if (row < rows && r < rv)
            a.s1[(((size_t)o * Kh + kh) * M0 + x0) * M1 + x1b + r] = make_float2(dre[rr], dim[rr]);
        }
      }
    }
    return;
  }
  // forward stage 2: one thread per (o, r, kh)
  for (int i = threadIdx.x; i < a.nout * rv * Kh; i += blockDim.x) {
    const int o = i / (rv * Kh), r = (i / Kh) % rv, kh = i % Kh;
    const float* row = outv + ((size_t)o * R + r) * LV;
    float2 acc = make_float2(0.f, 0.f);
    for (int x2 = 0; x2 < M2; ++x2) {
      const float2 w = wfx[(size_t)x2 * Kh + kh];
      acc.x = fmaf(row[x2], w.x, acc.x);
      acc.y = fmaf(row[x2], w.y, acc.y);
    }
    a.s1[(((size_t)o * Kh + kh) * M0 + x0) * M1 + x1b + r] = acc;
  }
}

// --------------------------------------- column step on the band side
// One block per (job, kh, group of KG k1 values): forward stage 1 (x1 -> k1)
// and stage 0 (x0 -> k0) of the job's one or two product fields at this kh,
// the band update out = base + ca S_a F(a) + cb S_b F(b) + ce extra (S = K~
// or 1), and the next step's inverse stage 0 (k0 -> x0, value and d0
// variants, optionally of L~ out) for the same columns.
template <int KG, class S>
__global__ void __launch_bounds__(256) k_colstep(ColJobs jobs, Twiddles tw, const float* __restrict__ Lsym,
                                                 const float* __restrict__ Ksym, S sh, float invG, int xsz,
                                                 int stage_w0) {
  extern __shared__ float2 shc[];
  const int M0 = sh.M0(), M1 = sh.M1(), K0 = sh.K0(), K1 = sh.K1(), Kh = sh.Kh();
  const ColJob job = jobs.j[blockIdx.z];
  const int kh = blockIdx.y;
  const int kb = blockIdx.x * KG;
  const int C = K1 * Kh;
  const int nterm = job.b ? 2 : 1;
  // region X: one S1 slice at a time (and later the inverse twiddles, when
  // they fit; else phase 3 reads them from global memory); region Y: the rest
  float2* sx = shc;                       // [M0][M1]
  float2* w0s = shc;                      // [2][M0][K0] (phase 3, when staged)
  float2* wf1 = shc + xsz;                // [KG][M1]
  float2* s2 = wf1 + KG * M1;             // [2][M0][KG]
  float2* wf0 = s2 + 2 * M0 * KG;         // [K0][M0]
  float2* bnd = wf0 + K0 * M0;            // [2][K0][KG]  (out, L~ out)

  batched_fill<float2>(KG * M1, [&](int i) {
    int kk = i / M1, x = i % M1;
    int k1 = kb + kk;
    return (k1 < K1) ? tw.fwd1[(size_t)k1 * M1 + x] : make_float2(0.f, 0.f);
  }, [&](int i, float2 v) { wf1[i] = v; });
  batched_fill<float2>(K0 * M0, [&](int i) { return tw.fwd0[i]; }, [&](int i, float2 v) { wf0[i] = v; });
  // stage 1', one term at a time: s2[t][x0][kk] = sum_x1 wf1[kk][x1] S[t][x0][x1]
  for (int t = 0; t < nterm; ++t) {
    const float2* src = (t ? job.b : job.a) + (size_t)kh * M0 * M1;
    if (t) __syncthreads();  // the previous slice has been consumed
    batched_fill<float2>(M0 * M1, [&](int i) { return src[i]; }, [&](int i, float2 v) { sx[i] = v; });
    __syncthreads();
    for (int i = threadIdx.x; i < M0 * KG; i += blockDim.x) {
      int x0 = i / KG, kk = i % KG;
      const float2* row = sx + (size_t)x0 * M1;
      const float2* w = wf1 + (size_t)kk * M1;
      float2 acc = make_float2(0.f, 0.f);
      for (int x = 0; x < M1; ++x) cmac(acc, w[x], row[x]);
      s2[(size_t)t * M0 * KG + i] = acc;
    }
  }
  __syncthreads();
  // stage 0' + band update
  for (int i = threadIdx.x; i < K0 * KG; i += blockDim.x) {
    int k0 = i / KG, kk = i % KG;
    int k1 = kb + kk;
    float2 res = make_float2(0.f, 0.f);
    if (k1 < K1 && k0 != K0 / 2 && k1 != K1 / 2) {
      const size_t idx = ((size_t)kh * K0 + k0) * K1 + k1;
      float2 fa = make_float2(0.f, 0.f), fb = make_float2(0.f, 0.f);
      const float2* w = wf0 + (size_t)k0 * M0;
      for (int x0 = 0; x0 < M0; ++x0) cmac(fa, w[x0], s2[(size_t)x0 * KG + kk]);
      if (nterm == 2)
        for (int x0 = 0; x0 < M0; ++x0) cmac(fb, w[x0], s2[((size_t)M0 + x0) * KG + kk]);
      if (job.base) res = job.base[idx];
      const float ks = Ksym[idx];
      const float sa = job.ca * invG * (job.syma ? ks : 1.f);
      res.x = fmaf(sa, fa.x, res.x);
      res.y = fmaf(sa, fa.y, res.y);
      if (nterm == 2) {
        const float sb = job.cb * invG * (job.symb ? ks : 1.f);
        res.x = fmaf(sb, fb.x, res.x);
        res.y = fmaf(sb, fb.y, res.y);
      }
      if (job.extra) {
        const float2 e = job.extra[idx];
        res.x = fmaf(job.ce, e.x, res.x);
        res.y = fmaf(job.ce, e.y, res.y);
      }
    }
    if (k1 < K1) job.out[((size_t)kh * K0 + k0) * K1 + k1] = res;
    bnd[i] = res;
    float l = (k1 < K1) ? Lsym[((size_t)kh * K0 + k0) * K1 + k1] : 0.f;
    bnd[K0 * KG + i] = make_float2(l * res.x, l * res.y);
  }
  if (job.nt1 == 0 && !job.t1n) return;
  __syncthreads();
  if (job.t1n) {
    // image-grid stage 0 of out: t1n[x0][kh][k1] = sum_k0 w0n[x0][k0] out[k0][k1]
    const int N0 = jobs.N0;
    for (int i = threadIdx.x; i < N0 * KG; i += blockDim.x) {
      const int x0 = i / KG, kk = i % KG, k1 = kb + kk;
      if (k1 >= K1) continue;
      const float2* w = jobs.w0n + (size_t)x0 * K0;
      float2 acc = make_float2(0.f, 0.f);
      for (int k0 = 0; k0 < K0; ++k0) cmac(acc, w[k0], bnd[(size_t)k0 * KG + kk]);
      job.t1n[((size_t)x0 * Kh + kh) * K1 + k1] = acc;
    }
  }
  if (job.nt1 == 0) return;
  const float2* w0t = tw.inv0;
  if (stage_w0) {
    batched_fill<float2>(2 * M0 * K0, [&](int i) { return tw.inv0[i]; }, [&](int i, float2 v) { w0s[i] = v; });
    w0t = w0s;
  }
  __syncthreads();
  // next inverse stage 0: t1[v][x0][k1][kh] = sum_k0 w0[v][x0][k0] b[k0]
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    if (u >= job.nt1) break;
    const float2* bsrc = bnd + ((u == 0 ? job.t1l[0] : job.t1l[1]) ? K0 * KG : 0);
    float2* dst = (u == 0) ? job.t1[0] : job.t1[1];
    for (int i = threadIdx.x; i < 2 * M0 * KG; i += blockDim.x) {
      int v = i / (M0 * KG), x0 = (i / KG) % M0, kk = i % KG;
      int k1 = kb + kk;
      if (k1 >= K1) continue;
      const float2* w = w0t + ((size_t)v * M0 + x0) * K0;
      float2 acc = make_float2(0.f, 0.f);
      for (int k0 = 0; k0 < K0; ++k0) cmac(acc, w[k0], bsrc[(size_t)k0 * KG + kk]);
      dst[((size_t)v * M0 + x0) * C + (size_t)kh * K1 + k1] = acc;
    }
  }
}

// ------------------------------------------ MFMA column step (tuned shapes)
// Complex 16x16 output tile by four real MFMAs per k-step of four:
// acc0 += Ar Br, acc1 += Ai Bi, acc2 += Ar Bi, acc3 += Ai Br, so the tile is
// (acc0 - acc1) + i (acc2 + acc3).  A(row, k) = A[row * lda + k] and
// B(k, col) = B[k * ldb + col] for the tile's 16 rows / 16 columns.
template <int KSTEPS, bool BF3>
__device__ __forceinline__ void ctile(const float2* __restrict__ A, int lda, const float2* __restrict__ B,
                                      int ldb, floatx4* acc) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const float2* a = A + li * lda + lk;
  const float2* b = B + lk * ldb + li;
#pragma unroll
  for (int k0 = 0; k0 < KSTEPS; k0 += 4) {
    float2 av[4], bv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (k0 + u < KSTEPS) {
        av[u] = a[4 * (k0 + u)];
        bv[u] = b[4 * (k0 + u) * ldb];
      }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (k0 + u < KSTEPS) {
        if constexpr (BF3) {  // each operand split once for its two products
          const shortx4 ar = bf3_a(av[u].x), ai = bf3_a(av[u].y), br = bf3_b(bv[u].x), bi = bf3_b(bv[u].y);
          acc[0] = mma_bf3(ar, br, acc[0]);
          acc[1] = mma_bf3(ai, bi, acc[1]);
          acc[2] = mma_bf3(ar, bi, acc[2]);
          acc[3] = mma_bf3(ai, br, acc[3]);
        } else {
          acc[0] = mma<BF3>(av[u].x, bv[u].x, acc[0]);
          acc[1] = mma<BF3>(av[u].y, bv[u].y, acc[1]);
          acc[2] = mma<BF3>(av[u].x, bv[u].y, acc[2]);
          acc[3] = mma<BF3>(av[u].y, bv[u].x, acc[3]);
        }
      }
  }
}

__device__ __forceinline__ void zero_acc(floatx4* acc, int n) {
  for (int i = 0; i < n; ++i) acc[i] = floatx4{0.f, 0.f, 0.f, 0.f};
}

// Logical block index (x, y, z) of a launch whose workgroups the command
// processor hands round-robin to the eight XCDs (workgroup p to XCD p % 8):
// with the block count a multiple of 8, XCD x takes the contiguous logical
// range [x T/8, (x + 1) T/8), so blocks that are neighbours in the logical
// order run on one XCD and meet in its L2.  The logical order runs x fastest,
// or with ZFirst z fastest, then x, then y (for launches whose z blocks of
// one (x, y) read the same input: the column steps' k1 tiles and parts of one
// kh read the same stage-1 input, and neighbouring kh share 32-byte granules
// of the band).
template <bool ZFirst>
__device__ __forceinline__ uint3 xcd_block3() {
  const unsigned gx = gridDim.x, gy = gridDim.y, gz = gridDim.z, total = gx * gy * gz;
  unsigned p = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  if (total % 8u == 0) p = (p % 8u) * (total / 8u) + p / 8u;
  if constexpr (ZFirst) return make_uint3((p / gz) % gx, p / (gz * gx), p % gz);
  return make_uint3(p % gx, (p / gx) % gy, p / (gx * gy));
}

// Tables for the MFMA column step: w1t[x1][k1] = fwd1[k1][x1] (columns padded
// to Kp), w0f[k0][x0] = fwd0 (rows padded to Kp), w0i[v][x0][k0] = inv0 (rows
// padded to Mp); padding is zero.
__global__ void k_col_tables(const float2* fwd1, const float2* fwd0, const float2* inv0, float2* w1t,
                             float2* w0f, float2* w0i, int M, int K, int Mp, int Kp) {
  const int n1 = M * Kp, n2 = Kp * M, n3 = 2 * Mp * K;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  const float2 z = make_float2(0.f, 0.f);
  if (i < n1) {
    int x1 = i / Kp, k1 = i % Kp;
    w1t[i] = (k1 < K) ? fwd1[(size_t)k1 * M + x1] : z;
  } else if (i < n1 + n2) {
    int e = i - n1, k0 = e / M, x0 = e % M;
    w0f[e] = (k0 < K) ? fwd0[(size_t)k0 * M + x0] : z;
  } else if (i < n1 + n2 + n3) {
    int e = i - n1 - n2, v = e / (Mp * K), x0 = (e / K) % Mp, k0 = e % K;
    w0i[e] = (x0 < M) ? inv0[((size_t)v * M + x0) * K + k0] : z;
  }
}

// One block per (kh, job, 16-wide tile of k1, part), four waves; same contract
// as k_colstep: every phase after the stage-1 input is separable along k1.
// With nparts > 1 the blocks of one tile all form the band update (only part
// 0 stores it) and split the output tiles of the next inverse stage 0 between
// them in contiguous ranges, which multiplies the blocks of launches that
// would leave most compute units idle.  The loads that stage 1' needs (the
// stage-1 input, its table, the band values of the update) are issued at the
// start, two complex values per load; the stage-0 tables and the image-grid
// table after the first barrier, arriving during stage 1' and waiting in
// registers until their LDS is free.
// Band values of the column step's update at (k0 = 16 tile + 4 lk + r, k1):
// the base and extra terms (the block's 16 k1 of one k2 are a 128-byte row
// of the band layout [Kh][K0][K1]) and the L~ / K~ symbols (formed in FP64);
// zero outside the band.  The loads are unconditional (a job without an
// extra term reads its base again, the same cache lines; one without a base
// reads its stage-1 input, which is longer than a band field, at a clamped
// index): a load under a branch makes the merge wait for every load in
// flight, so base_or_zero / extra_or_zero drop the missing terms where the
// values are used.
template <int K, int Kh>
__device__ __forceinline__ void update_values(const ColJob& job, int tile, int lk, int k1, int kh, int spow,
                                              double alpha, float2 (&pbase)[4], float2 (&pextra)[4],
                                              float (&pks)[4], float (&pls)[4]) {
  const float2* pb = job.base ? job.base : job.a;
  const float2* pe = job.extra ? job.extra : pb;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int k0 = tile * 16 + 4 * lk + r;
    const bool ok = k0 < K && k1 < K;
    const size_t idx = ((size_t)kh * K + (ok ? k0 : 0)) * K + (ok ? k1 : 0);
    pbase[r] = pb[idx];
    pextra[r] = pe[idx];
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int k0 = tile * 16 + 4 * lk + r;
    const bool ok = k0 < K && k1 < K;
    const float2 sym = band_symbols(ok ? k0 : 0, ok ? k1 : 0, kh, K, K, spow, alpha);
    pks[r] = ok ? sym.y : 0.f;
    pls[r] = ok ? sym.x : 0.f;
  }
}

__device__ __forceinline__ float2 base_or_zero(const ColJob& job, float2 v) {
  return job.base ? v : make_float2(0.f, 0.f);
}
__device__ __forceinline__ float2 extra_or_zero(const ColJob& job, float2 v) {
  return job.extra ? v : make_float2(0.f, 0.f);
}

constexpr int kGrid0Pre = 16;  // image-grid stage-0 table: complex values per thread
template <class S, bool BF3>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2))) k_colstep_mfma(ColJobs jobs, const float2* __restrict__ w1t,
                                                      const float2* __restrict__ w0f,
                                                      const float2* __restrict__ w0i,
                                                      double alpha, int spow, float invG,
                                                      int nparts) {
  constexpr int K = S::K0(), M = S::M0(), Kh = S::Kh();
  constexpr int Mp = (M + 15) & ~15, Kp = (K + 15) & ~15;
  // A operands (read along rows) get odd complex strides, B operands 18
  constexpr int LS1 = M + 1, LS2 = 18, LOB = 18;
  constexpr int C = K * Kh;
  constexpr int LW1 = 18, LW0F = M + 1, LW0I = K + 1, LG = K + 1;
  static_assert(M % 2 == 0 && K % 2 == 0, "pairs of complex values per load");
  __shared__ __align__(16) float2 s1[2][Mp][LS1];
  __shared__ __align__(16) float2 s2[2][M][LS2];
  __shared__ __align__(16) float2 ob[2][K][LOB];
  __shared__ __align__(16) float2 w1s[M][LW1];        // w1t columns of this k1 tile
  __shared__ __align__(16) float2 w0fs[Kp][LW0F];     // w0f
  __shared__ __align__(16) float2 w0is[2][Mp][LW0I];  // w0i
  float2* g0s = &s1[0][0][0];           // [N0][LG] image-grid stage-0 table, after stage 1'
  const uint3 lb = xcd_block3<true>();
  const ColJob& job = jobs.j[lb.y];
  const int kh = lb.x;
  constexpr int T0 = Kp / 16;
  const int kc = (lb.z % T0) * 16;  // first k1 of the tile
  const int part = lb.z / T0;
  const int nterm = job.b ? 2 : 1;
  const bool grid0 = job.t1n != nullptr;
  const int N0 = jobs.N0;
  // this part's range [jb0, jb1) of the next-stage output tiles: padded-grid
  // tiles first, then the image-grid ones
  constexpr int TIR = Mp / 16;
  const int njb = job.nt1 * 2 * TIR;
  const int ngb = grid0 ? N0 / 16 : 0;
  const int jb0 = (njb + ngb) * part / nparts, jb1 = (njb + ngb) * (part + 1) / nparts;
  const bool my_grid0 = grid0 && jb1 > njb;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const int k1 = kc + li;

  // ---- loads
  constexpr int H = M / 2, KH2 = K / 2;
  const int ns1 = nterm * Mp * H;
  const float2* sa = job.a + (size_t)kh * M * M;
  const float2* sb = job.b ? job.b + (size_t)kh * M * M : sa;
  RegStage<(2 * Mp * H + 255) / 256, float4> rs1;
  RegStage<(M * 8 + 255) / 256, float4> rw1;
  RegStage<(Kp * H + 255) / 256, float4> rw0f;
  RegStage<(2 * Mp * KH2 + 255) / 256, float4> rw0i;
  RegStage<kGrid0Pre / 2, float4> rg;
  const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
  // padding rows x0 >= M load a valid row and are zeroed when stored
  rs1.load(ns1, [&](int i) {
    const int t = i / (Mp * H), x0 = (i / H) % Mp, x1 = 2 * (i % H);
    return ld4((t ? sb : sa) + (x0 < M ? x0 : M - 1) * M + x1);
  });
  rw1.load(M * 8, [&](int i) { return ld4(w1t + (i / 8) * Kp + kc + 2 * (i % 8)); });
  // band values of the update at (k0 = 16 wave + 4 lk + r, k1)
  float2 pbase[4], pextra[4];
  float pks[4], pls[4];
  if (wave < T0) update_values<K, Kh>(job, wave, lk, k1, kh, spow, alpha, pbase, pextra, pks, pls);
  // ---- stores of what stage 1' reads
  rs1.store(ns1, [&](int i, float4 v) {
    const int t = i / (Mp * H), x0 = (i / H) % Mp, x1 = 2 * (i % H);
    st22(&s1[t][x0][x1], x0 < M ? v : z4);
  });
  rw1.store(M * 8, [&](int i, float4 v) { st4(&w1s[i / 8][2 * (i % 8)], v); });
  __syncthreads();
  // the stage-0 tables arrive during stage 1' (issued after the first
  // barrier, which then waits for the stage-1 input alone), waiting in
  // registers until its products are done
  rw0f.load(Kp * H, [&](int i) { return ld4(w0f + 2 * i); });
  rw0i.load(2 * Mp * KH2, [&](int i) { return ld4(w0i + 2 * i); });
  const int ng = my_grid0 ? N0 * KH2 : 0;
  rg.load(ng, [&](int i) { return ld4(jobs.w0n + 2 * i); });
  // stage 1': s2[t][x0][j] = sum_x1 s1[t][x0][x1] w1t[x1][kc + j]
  constexpr int T1R = Mp / 16;
  for (int jb = wave; jb < nterm * T1R; jb += 4) {
    const int t = jb / T1R, ti = jb % T1R;
    floatx4 acc[4];
    zero_acc(acc, 4);
    ctile<M / 4, BF3>(&s1[t][ti * 16][0], LS1, &w1s[0][0], LW1, acc);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int x0 = ti * 16 + 4 * lk + r;
      if (x0 < M) s2[t][x0][li] = make_float2(acc[0][r] - acc[1][r], acc[2][r] + acc[3][r]);
    }
  }
  rw0f.store(Kp * H, [&](int i, float4 v) { st22(&w0fs[i / H][2 * (i % H)], v); });
  rw0i.store(2 * Mp * KH2, [&](int i, float4 v) {
    st22(&w0is[i / (Mp * KH2)][(i / KH2) % Mp][2 * (i % KH2)], v);
  });
  __syncthreads();
  rg.store(ng, [&](int i, float4 v) { st22(g0s + (2 * i / K) * LG + (2 * i) % K, v); });
  // stage 0' and the band update (one k0 tile per wave).  With two k0 tiles
  // the other two waves take half of the products: the second term, or with
  // one term the second half of the x0 depth, and hand their sums over
  // through the LDS of the stage-1 table (unused after stage 1').
  constexpr bool kSplit0 = (T0 == 2);
  [[maybe_unused]] float2 own[4], other[4];
  if constexpr (kSplit0) {
    const int ti = wave & 1, h = wave >> 1;
    constexpr int SD = M / 4, S1 = SD / 2;
    floatx4 acc[4];
    zero_acc(acc, 4);
    if (nterm == 2)
      ctile<SD, BF3>(&w0fs[ti * 16][0], LW0F, &s2[h][0][0], LS2, acc);
    else if (h == 0)
      ctile<S1, BF3>(&w0fs[ti * 16][0], LW0F, &s2[0][0][0], LS2, acc);
    else
      ctile<SD - S1, BF3>(&w0fs[ti * 16][4 * S1], LW0F, &s2[0][4 * S1][0], LS2, acc);
    static_assert(M * LW1 >= 2 * 4 * 64, "hand-over buffer fits the stage-1 table");
    float2* red = &w1s[0][0];  // [tile][r][lane]
#pragma unroll
    for (int r = 0; r < 4; ++r) own[r] = make_float2(acc[0][r] - acc[1][r], acc[2][r] + acc[3][r]);
    if (h == 1) {
#pragma unroll
      for (int r = 0; r < 4; ++r) red[(ti * 4 + r) * 64 + lane] = own[r];
    }
    __syncthreads();
    if (h == 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) other[r] = red[(ti * 4 + r) * 64 + lane];
    }
  }
  if (wave < T0) {
    const int ti = wave;
    floatx4 aa[4], bb[4];
    if constexpr (!kSplit0) {
      zero_acc(aa, 4);
      zero_acc(bb, 4);
      ctile<M / 4, BF3>(&w0fs[ti * 16][0], LW0F, &s2[0][0][0], LS2, aa);
      if (nterm == 2) ctile<M / 4, BF3>(&w0fs[ti * 16][0], LW0F, &s2[1][0][0], LS2, bb);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int k0 = ti * 16 + 4 * lk + r;
      if (k0 >= K || k1 >= K) continue;
      const size_t idx = ((size_t)kh * K + k0) * K + k1;
      float2 res = make_float2(0.f, 0.f);
      if (k0 != K / 2 && k1 != K / 2) {
        res = base_or_zero(job, pbase[r]);
        const float sa_ = job.ca * invG * (job.syma ? pks[r] : 1.f);
        if constexpr (kSplit0) {
          const float2 ta = (nterm == 2) ? own[r] : make_float2(own[r].x + other[r].x, own[r].y + other[r].y);
          res.x = fmaf(sa_, ta.x, res.x);
          res.y = fmaf(sa_, ta.y, res.y);
          if (nterm == 2) {
            const float sb_ = job.cb * invG * (job.symb ? pks[r] : 1.f);
            res.x = fmaf(sb_, other[r].x, res.x);
            res.y = fmaf(sb_, other[r].y, res.y);
          }
        } else {
          res.x = fmaf(sa_, aa[0][r] - aa[1][r], res.x);
          res.y = fmaf(sa_, aa[2][r] + aa[3][r], res.y);
          if (nterm == 2) {
            const float sb_ = job.cb * invG * (job.symb ? pks[r] : 1.f);
            res.x = fmaf(sb_, bb[0][r] - bb[1][r], res.x);
            res.y = fmaf(sb_, bb[2][r] + bb[3][r], res.y);
          }
        }
        const float2 ex = extra_or_zero(job, pextra[r]);
        res.x = fmaf(job.ce, ex.x, res.x);
        res.y = fmaf(job.ce, ex.y, res.y);
      }
      if (part == 0) job.out[idx] = res;
      ob[0][k0][li] = res;
      ob[1][k0][li] = make_float2(pls[r] * res.x, pls[r] * res.y);
    }
  }
  if (jb0 == jb1) return;
  __syncthreads();
  // next inverse stage 0 on the padded grid: t1[v][x0][kh][k1] = sum_k0 w0i[v][x0][k0] ob[L][k0][k1],
  // then on the image grid: t1n[x0][kh][k1] = sum_k0 w0n[x0][k0] ob[0][k0][k1]
  for (int jb = jb0 + wave; jb < jb1; jb += 4) {
    floatx4 acc[4];
    zero_acc(acc, 4);
    if (jb >= njb) {
      const int ti = jb - njb;
      ctile<K / 4, BF3>(g0s + ti * 16 * LG, LG, &ob[0][0][0], LOB, acc);
      if (k1 >= K) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int x0 = ti * 16 + 4 * lk + r;
        job.t1n[((size_t)x0 * Kh + kh) * K + k1] = make_float2(acc[0][r] - acc[1][r], acc[2][r] + acc[3][r]);
      }
      continue;
    }
    const int u = jb / (2 * TIR), v = (jb / TIR) % 2, ti = jb % TIR;
    const int lsel = (u == 0) ? job.t1l[0] : job.t1l[1];
    float2* dst = (u == 0) ? job.t1[0] : job.t1[1];
    ctile<K / 4, BF3>(&w0is[v][ti * 16][0], LW0I, &ob[lsel][0][0], LOB, acc);
    if (k1 >= K) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int x0 = ti * 16 + 4 * lk + r;
      if (x0 < M)
        dst[((size_t)v * M + x0) * C + (size_t)kh * K + k1] = make_float2(acc[0][r] - acc[1][r], acc[2][r] + acc[3][r]);
    }
  }
}

// Lean form of k_colstep_mfma for the launches of the forward sweeps (one
// product field per job, the image-grid stage 0 fused, two parts per column
// tile), which run beside the grid chain: part 0 forms the next padded-grid
// stage 0 and stores the band update, part 1 the image-grid stage 0.  One LDS
// region holds in turn the stage-1 input, the stage-0 table and the part's
// next-stage table, so the block needs about half the LDS of k_colstep_mfma
// and can share a compute unit with grid-step blocks.  The tables are issued
// after the first barrier and wait in registers until their turn.
template <class S, bool BF3>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2))) k_colstep_lean(
    ColJobs jobs, const float2* __restrict__ w1t, const float2* __restrict__ w0f, const float2* __restrict__ w0i,
    double alpha, int spow, float invG) {
  constexpr int K = S::K0(), M = S::M0(), Kh = S::Kh();
  constexpr int Mp = (M + 15) & ~15, Kp = (K + 15) & ~15;
  constexpr int LS1 = M + 1, LS2 = 18, LOB = 18;
  constexpr int C = K * Kh;
  constexpr int LW1 = 18, LW0F = M + 1, LW0I = K + 1, LG = K + 1;
  constexpr int T0 = Kp / 16, TIR = Mp / 16;
  constexpr int NG0MAX = 256 * kGrid0Pre / K;  // image-grid rows the table may hold
  constexpr int NA1 = Mp * LS1, NA2 = Kp * LW0F, NA3 = 2 * Mp * LW0I, NA4 = NG0MAX * LG;
  constexpr int NA = NA1 > NA2 ? (NA1 > NA3 ? (NA1 > NA4 ? NA1 : NA4) : (NA3 > NA4 ? NA3 : NA4))
                               : (NA2 > NA3 ? (NA2 > NA4 ? NA2 : NA4) : (NA3 > NA4 ? NA3 : NA4));
  static_assert(M % 2 == 0 && K % 2 == 0 && T0 == 2, "pairs of complex values per load, two k0 tiles");
  __shared__ __align__(16) float2 ra[NA];          // s1 | w0fs | w0is or g0s
  __shared__ __align__(16) float2 s2[M][LS2];
  __shared__ __align__(16) float2 ob[2][K][LOB];
  __shared__ __align__(16) float2 w1s[M][LW1];      // stage-1 table; then the stage-0' hand-over
  float2(*s1)[LS1] = reinterpret_cast<float2(*)[LS1]>(ra);
  float2(*w0fs)[LW0F] = reinterpret_cast<float2(*)[LW0F]>(ra);
  float2(*w0is)[Mp][LW0I] = reinterpret_cast<float2(*)[Mp][LW0I]>(ra);
  float2* g0s = ra;
  const uint3 lb = xcd_block3<true>();
  const ColJob& job = jobs.j[lb.y];
  const int kh = lb.x;
  const int kc = (lb.z % T0) * 16;
  const int part = lb.z / T0;  // 0: padded-grid stage 0 and the store; 1: image-grid stage 0
  const int N0 = jobs.N0;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const int k1 = kc + li;
  constexpr int H = M / 2, KH2 = K / 2;
  const float2* sa = job.a + (size_t)kh * M * M;
  RegStage<(Mp * H + 255) / 256, float4> rs1;
  RegStage<(M * 8 + 255) / 256, float4> rw1;
  RegStage<(Kp * H + 255) / 256, float4> rw0f;
  constexpr int NT_I = 2 * Mp * KH2, NT_G = NG0MAX * KH2;
  RegStage<((NT_I > NT_G ? NT_I : NT_G) + 255) / 256, float4> rt;
  const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
  // padding rows x0 >= M load a valid row and are zeroed when stored
  rs1.load(Mp * H, [&](int i) {
    const int x0 = i / H, x1 = 2 * (i % H);
    return ld4(sa + (x0 < M ? x0 : M - 1) * M + x1);
  });
  rw1.load(M * 8, [&](int i) { return ld4(w1t + (i / 8) * Kp + kc + 2 * (i % 8)); });
  float2 pbase[4], pextra[4];
  float pks[4], pls[4];
  if (wave < T0) update_values<K, Kh>(job, wave, lk, k1, kh, spow, alpha, pbase, pextra, pks, pls);
  rs1.store(Mp * H, [&](int i, float4 v) { st22(&s1[i / H][2 * (i % H)], i / H < M ? v : z4); });
  rw1.store(M * 8, [&](int i, float4 v) { st4(&w1s[i / 8][2 * (i % 8)], v); });
  __syncthreads();
  // the tables are issued after the first barrier (which then waits for the
  // stage-1 input alone) and arrive during stage 1'; one load path for both
  // parts' next-stage tables
  rw0f.load(Kp * H, [&](int i) { return ld4(w0f + 2 * i); });
  const int nt_tab = part == 0 ? NT_I : N0 * KH2;
  const float2* tsrc = part == 0 ? w0i : jobs.w0n;
  rt.load(nt_tab, [&](int i) { return ld4(tsrc + 2 * i); });
  // stage 1': s2[x0][j] = sum_x1 s1[x0][x1] w1t[x1][kc + j]
  for (int ti = wave; ti < TIR; ti += 4) {
    floatx4 acc[4];
    zero_acc(acc, 4);
    ctile<M / 4, BF3>(&s1[ti * 16][0], LS1, &w1s[0][0], LW1, acc);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int x0 = ti * 16 + 4 * lk + r;
      if (x0 < M) s2[x0][li] = make_float2(acc[0][r] - acc[1][r], acc[2][r] + acc[3][r]);
    }
  }
  __syncthreads();
  rw0f.store(Kp * H, [&](int i, float4 v) { st22(&w0fs[i / H][2 * (i % H)], v); });
  __syncthreads();
  // stage 0' on all four waves: waves 2-3 take the second half of the x0
  // depth and hand their sums over through w1s; waves 0-1 form the update
  float2 own[4], other[4];
  {
    const int ti = wave & 1, h = wave >> 1;
    constexpr int SD = M / 4, S1 = SD / 2;
    floatx4 acc[4];
    zero_acc(acc, 4);
    if (h == 0)
      ctile<S1, BF3>(&w0fs[ti * 16][0], LW0F, &s2[0][0], LS2, acc);
    else
      ctile<SD - S1, BF3>(&w0fs[ti * 16][4 * S1], LW0F, &s2[4 * S1][0], LS2, acc);
    static_assert(M * LW1 >= 2 * 4 * 64, "hand-over buffer fits the stage-1 table");
    float2* red = &w1s[0][0];
#pragma unroll
    for (int r = 0; r < 4; ++r) own[r] = make_float2(acc[0][r] - acc[1][r], acc[2][r] + acc[3][r]);
    if (h == 1) {
#pragma unroll
      for (int r = 0; r < 4; ++r) red[(ti * 4 + r) * 64 + lane] = own[r];
    }
    __syncthreads();
    if (h == 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) other[r] = red[(ti * 4 + r) * 64 + lane];
    }
  }
  if (wave < T0) {
    const int ti = wave;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int k0 = ti * 16 + 4 * lk + r;
      if (k0 >= K || k1 >= K) continue;
      const size_t idx = ((size_t)kh * K + k0) * K + k1;
      float2 res = make_float2(0.f, 0.f);
      if (k0 != K / 2 && k1 != K / 2) {
        res = base_or_zero(job, pbase[r]);
        const float sa_ = job.ca * invG * (job.syma ? pks[r] : 1.f);
        res.x = fmaf(sa_, own[r].x + other[r].x, res.x);
        res.y = fmaf(sa_, own[r].y + other[r].y, res.y);
        const float2 ex = extra_or_zero(job, pextra[r]);
        res.x = fmaf(job.ce, ex.x, res.x);
        res.y = fmaf(job.ce, ex.y, res.y);
      }
      if (part == 0) job.out[idx] = res;
      ob[0][k0][li] = res;
      ob[1][k0][li] = make_float2(pls[r] * res.x, pls[r] * res.y);
    }
  }
  __syncthreads();
  if (part == 0)
    rt.store(nt_tab, [&](int i, float4 v) {
      st22(&w0is[i / (Mp * KH2)][(i / KH2) % Mp][2 * (i % KH2)], v);
    });
  else
    rt.store(nt_tab, [&](int i, float4 v) { st22(g0s + (2 * i / K) * LG + (2 * i) % K, v); });
  __syncthreads();
  if (part == 0) {
    // next inverse stage 0 on the padded grid: t1[v][x0][kh][k1] = sum_k0 w0i[v][x0][k0] ob[L][k0][k1]
    const int njb = job.nt1 * 2 * TIR;
    for (int jb = wave; jb < njb; jb += 4) {
      floatx4 acc[4];
      zero_acc(acc, 4);
      const int u = jb / (2 * TIR), v = (jb / TIR) % 2, ti = jb % TIR;
      const int lsel = (u == 0) ? job.t1l[0] : job.t1l[1];
      float2* dst = (u == 0) ? job.t1[0] : job.t1[1];
      ctile<K / 4, BF3>(&w0is[v][ti * 16][0], LW0I, &ob[lsel][0][0], LOB, acc);
      if (k1 >= K) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int x0 = ti * 16 + 4 * lk + r;
        if (x0 < M)
          dst[((size_t)v * M + x0) * C + (size_t)kh * K + k1] =
              make_float2(acc[0][r] - acc[1][r], acc[2][r] + acc[3][r]);
      }
    }
  } else {
    // image grid: t1n[x0][kh][k1] = sum_k0 w0n[x0][k0] ob[0][k0][k1]
    for (int ti = wave; ti < N0 / 16; ti += 4) {
      floatx4 acc[4];
      zero_acc(acc, 4);
      ctile<K / 4, BF3>(g0s + ti * 16 * LG, LG, &ob[0][0][0], LOB, acc);
      if (k1 >= K) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int x0 = ti * 16 + 4 * lk + r;
        job.t1n[((size_t)x0 * Kh + kh) * K + k1] = make_float2(acc[0][r] - acc[1][r], acc[2][r] + acc[3][r]);
      }
    }
  }
}

// ----------------------------------------------- forward stage 1 (x1)
template <int QT>
__global__ void __launch_bounds__(128) k_fwd1(Fwd1Jobs jobs, const float2* __restrict__ tw, int G0,
                                              int G1, int K1, int Kh) {
  extern __shared__ float2 sh[];
  const Fwd1Job job = jobs.j[blockIdx.z];
  const int qb = blockIdx.y * QT;
  batched_fill<float2>(QT * G1, [&](int i) {
    int t = i / G1, x = i % G1;
    int q = qb + t;
    return (q < K1) ? tw[(size_t)q * G1 + x] : make_float2(0.f, 0.f);
  }, [&](int i, float2 v) { sh[i] = v; });
  __syncthreads();
  const int e = blockIdx.x * blockDim.x + threadIdx.x;  // (x0, kh)
  if (e >= G0 * Kh) return;
  const int x0 = e / Kh, kh = e % Kh;
  float2 acc[QT];
#pragma unroll
  for (int t = 0; t < QT; ++t) acc[t] = make_float2(0.f, 0.f);
  const float2* src = job.in + (size_t)x0 * G1 * Kh + kh;
  for (int x = 0; x < G1; ++x) {
    float2 val = src[(size_t)x * Kh];
#pragma unroll
    for (int t = 0; t < QT; ++t) cmac(acc[t], sh[t * G1 + x], val);
  }
#pragma unroll
  for (int t = 0; t < QT; ++t) {
    int q = qb + t;
    if (q < K1) job.out[((size_t)x0 * Kh + kh) * K1 + q] = acc[t];
  }
}

// ------------------------------------- forward stage 0 (x0) + epilogue
template <int QT>
__global__ void __launch_bounds__(128) k_fwd0(Fwd0Jobs jobs, const float2* __restrict__ tw,
                                              const float* __restrict__ Ksym, int G0, int K0,
                                              int K1, int Kh, float invG) {
  extern __shared__ float2 sh[];
  const Fwd0Job job = jobs.j[blockIdx.z];
  const int qb = blockIdx.y * QT;
  batched_fill<float2>(QT * G0, [&](int i) {
    int t = i / G0, x = i % G0;
    int q = qb + t;
    return (q < K0) ? tw[(size_t)q * G0 + x] : make_float2(0.f, 0.f);
  }, [&](int i, float2 v) { sh[i] = v; });
  __syncthreads();
  const int C = K1 * Kh;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  float2 aa[QT], bb[QT];
#pragma unroll
  for (int t = 0; t < QT; ++t) { aa[t] = make_float2(0.f, 0.f); bb[t] = make_float2(0.f, 0.f); }
  for (int x = 0; x < G0; ++x) {
    float2 va = job.a[(size_t)x * C + c];
#pragma unroll
    for (int t = 0; t < QT; ++t) cmac(aa[t], sh[t * G0 + x], va);
  }
  if (job.b) {
    for (int x = 0; x < G0; ++x) {
      float2 vb = job.b[(size_t)x * C + c];
#pragma unroll
      for (int t = 0; t < QT; ++t) cmac(bb[t], sh[t * G0 + x], vb);
    }
  }
  const int q1 = c % K1, kh = c / K1;  // input column c = kh K1 + q1
#pragma unroll
  for (int t = 0; t < QT; ++t) {
    int q0 = qb + t;
    if (q0 >= K0) continue;
    size_t idx = ((size_t)kh * K0 + q0) * K1 + q1;
    float2 r = make_float2(0.f, 0.f);
    if (q0 != K0 / 2 && q1 != K1 / 2) {
      if (job.base) r = job.base[idx];
      float ks = Ksym[idx];
      float sa = job.ca * invG * (job.syma ? ks : 1.f);
      r.x = fmaf(sa, aa[t].x, r.x);
      r.y = fmaf(sa, aa[t].y, r.y);
      if (job.b) {
        float sb = job.cb * invG * (job.symb ? ks : 1.f);
        r.x = fmaf(sb, bb[t].x, r.x);
        r.y = fmaf(sb, bb[t].y, r.y);
      }
      if (job.extra) {
        float2 e = job.extra[idx];
        r.x = fmaf(job.ce, e.x, r.x);
        r.y = fmaf(job.ce, e.y, r.y);
      }
    }
    job.out[idx] = r;
    if (job.out2) {
      float2 r2 = make_float2(0.f, 0.f);
      if (q0 != K0 / 2 && q1 != K1 / 2) {
        const float s2 = job.ca * invG * Ksym[idx];
        r2.x = fmaf(s2, aa[t].x, 0.f);
        r2.y = fmaf(s2, aa[t].y, 0.f);
      }
      job.out2[idx] = r2;
    }
  }
}

// ----------------------------------------------------- grid step (N)
// One block per (x0, 16 consecutive x1 rows), 256 threads = 16 rows x 16
// lanes: inverse stage 1 of the three velocity components from their
// stage-0 output, then stage 2 register-blocked (lane l owns x2 = l + 16 j),
// then either the velocity itself or the incremental-state source.
constexpr int kGridRows = 16;

__device__ __forceinline__ float central_diff(const float* __restrict__ m, int x0, int x1, int x2,
                                              int N0, int N1, int N2, int axis) {
  if (axis == 0) {
    int p = (x0 + 1 == N0) ? 0 : x0 + 1, q = (x0 == 0) ? N0 - 1 : x0 - 1;
    return (m[((long long)p * N1 + x1) * N2 + x2] - m[((long long)q * N1 + x1) * N2 + x2]) * (0.5f * N0);
  }
  if (axis == 1) {
    int p = (x1 + 1 == N1) ? 0 : x1 + 1, q = (x1 == 0) ? N1 - 1 : x1 - 1;
    return (m[((long long)x0 * N1 + p) * N2 + x2] - m[((long long)x0 * N1 + q) * N2 + x2]) * (0.5f * N1);
  }
  int p = (x2 + 1 == N2) ? 0 : x2 + 1, q = (x2 == 0) ? N2 - 1 : x2 - 1;
  return (m[((long long)x0 * N1 + x1) * N2 + p] - m[((long long)x0 * N1 + x1) * N2 + q]) * (0.5f * N2);
}

template <int JN, class G>
__global__ void __launch_bounds__(256) k_gridstep(GridStepArgs a, Twiddles tw, G gs) {
  extern __shared__ float2 sh2[];
  const int N0 = gs.N0(), N1 = gs.N1(), N2 = gs.N2(), K1 = gs.K1(), Kh = gs.Kh();
  constexpr int R = kGridRows;
  const int C = K1 * Kh;
  const int x0 = blockIdx.y;
  const int x1b = blockIdx.x * R;
  float2* t1s = sh2;                 // [3][K1][Kh]
  float2* t2s = t1s + 3 * C;         // [3][R][Kh]
  float2* w1s = t2s + 3 * R * Kh;    // [R][K1]
  float2* w2t = w1s + R * K1;        // [Kh][N2]
  batched_fill<float2>(3 * C, [&](int i) {  // global [c][x0][kh][k1] -> t1s[c][k1][kh]
    return a.t1[((size_t)(i / C) * N0 + x0) * C + i % C];
  }, [&](int i, float2 v) {
    const int c = i / C, kh = (i % C) / K1, k1 = i % K1;
    t1s[(size_t)c * C + k1 * Kh + kh] = v;
  });
  batched_fill<float2>(R * K1, [&](int i) {
    int r = i / K1, k = i % K1;
    int x1 = x1b + r;
    return (x1 < N1) ? tw.inv1[(size_t)x1 * K1 + k] : make_float2(0.f, 0.f);
  }, [&](int i, float2 v) { w1s[i] = v; });
  batched_fill<float2>(N2 * Kh, [&](int i) {
    int kh = i / N2, x2 = i % N2;
    return tw.inv2[(size_t)x2 * Kh + kh];
  }, [&](int i, float2 v) { w2t[i] = v; });
  __syncthreads();
  for (int i = threadIdx.x; i < 3 * R * Kh; i += blockDim.x) {
    int c = i / (R * Kh), r = (i / Kh) % R, kh = i % Kh;
    float2 acc = make_float2(0.f, 0.f);
    const float2* wr = w1s + (size_t)r * K1;
    const float2* tc = t1s + (size_t)c * C + kh;
    for (int k = 0; k < K1; ++k) cmac(acc, wr[k], tc[(size_t)k * Kh]);
    t2s[i] = acc;
  }
  __syncthreads();
  const int r = threadIdx.x >> 4, lane = threadIdx.x & 15;
  const int x1 = x1b + r;
  float acc[3][JN];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int j = 0; j < JN; ++j) acc[c][j] = 0.f;
  for (int kh = 0; kh < Kh; ++kh) {
    float2 t[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) t[c] = t2s[((size_t)c * R + r) * Kh + kh];
    const float2* w = w2t + (size_t)kh * N2;
#pragma unroll
    for (int j = 0; j < JN; ++j) {
      int x2 = lane + 16 * j;
      float2 ww = (x2 < N2) ? w[x2] : make_float2(0.f, 0.f);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        acc[c][j] = fmaf(t[c].x, ww.x, acc[c][j]);
        acc[c][j] = fmaf(-t[c].y, ww.y, acc[c][j]);
      }
    }
  }
  if (x1 >= N1) return;
  const long long nN = (long long)N0 * N1 * N2;
#pragma unroll
  for (int j = 0; j < JN; ++j) {
    const int x2 = lane + 16 * j;
    if (x2 >= N2) continue;
    const long long gi = ((long long)x0 * N1 + x1) * N2 + x2;
    if (a.op == 0) {
#pragma unroll
      for (int c = 0; c < 3; ++c) a.vout[(size_t)c * nN + gi] = acc[c][j];
    } else {
      float g0 = central_diff(a.m, x0, x1, x2, N0, N1, N2, 0);
      float g1 = central_diff(a.m, x0, x1, x2, N0, N1, N2, 1);
      float g2 = central_diff(a.m, x0, x1, x2, N0, N1, N2, 2);
      float dot = g0 * acc[0][j] + g1 * acc[1][j] + g2 * acc[2][j];
      float base = a.dm ? a.dm[gi] : 0.f;
      a.q[gi] = fmaf(-a.dt, dot, base);
    }
  }
}

// Grid step on the matrix cores (tuned shapes): same contract as
// k_gridstep.  Stage 1 is a complex GEMM per component (16 rows x Kh),
// stage 2 the real part of a complex GEMM per (component, 16-column tile);
// a wave owns the three components of its column tiles, so the source
// term is formed in registers.
template <class G, bool BF3>
__global__ void __launch_bounds__(256) k_gridstep_mfma(GridStepArgs a, Twiddles tw) {
  constexpr int N0 = G::N0(), N1 = G::N1(), N2 = G::N2(), K1 = G::K1(), Kh = G::Kh();
  constexpr int R = kGridRows;
  constexpr int Khp = (Kh + 15) & ~15;  // half-spectrum columns padded to whole tiles (zero)
  constexpr int LT1 = Khp + 2, LW1 = K1 + 1, LT2 = Khp + 1, LW2 = N2 + 2;  // A operands: odd strides
  constexpr int KP = K1 / 2, KHP = Kh / 2;
  static_assert(K1 % 4 == 0 && Kh % 2 == 0 && N2 % 16 == 0, "tuned grid shape");
  __shared__ __align__(16) float2 t1s[3][K1][LT1];
  __shared__ __align__(16) float2 w1s[R][LW1];
  __shared__ __align__(16) float2 t2s[3][R][LT2];
  __shared__ __align__(16) float2 w2t[Khp][LW2];
  // source: rows x1b - 1 .. x1b + R of m in plane x0 (periodic), for the x1
  // and x2 differences; the x0 differences are read directly
  constexpr int LM = N2 + 4;
  __shared__ __align__(16) float mrow[R + 2][LM];
  static_assert(N1 % R == 0, "whole row tiles");
  // the row tiles of one plane read the same stage-0 input: one XCD each
  const uint3 lb = xcd_block3<false>();
  const int x0 = lb.y;
  const int x1b = lb.x * R;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
  // ---- all global loads of the block at once: the stage-0 input of this
  // plane, the stage-1 rows, the stage-2 table, and (source) the neighbours
  // of the points this lane will write
  RegStage<(3 * Kh * KP + 255) / 256, float4> rt;
  RegStage<(R * KP + 255) / 256, float4> rw1;
  RegStage<(N2 * KHP + 255) / 256, float4> rw2;
  rt.load(3 * Kh * KP, [&](int i) {
    const int c = i / (Kh * KP), kh = (i / KP) % Kh, k1 = 2 * (i % KP);
    return ld4(a.t1 + (((size_t)c * N0 + x0) * Kh + kh) * K1 + k1);
  });
  rw1.load(R * KP, [&](int i) {  // rows past N1 load a valid row and are zeroed when stored
    const int x1 = x1b + i / KP;
    return ld4(tw.inv1 + (size_t)(x1 < N1 ? x1 : N1 - 1) * K1 + 2 * (i % KP));
  });
  rw2.load(N2 * KHP, [&](int i) { return ld4(tw.inv2 + (size_t)(i / KHP) * Kh + 2 * (i % KHP)); });
  constexpr int NTJ = N2 / 16, TPW = (NTJ + 3) / 4, NM4 = (R + 2) * N2 / 4;
  RegStage<(NM4 + 255) / 256, float4> rm;
  if (a.op == 1) rm.load(NM4, [&](int i) {
    const int x1 = (x1b - 1 + i / (N2 / 4) + N1) % N1;
    return *reinterpret_cast<const float4*>(a.m + ((size_t)x0 * N1 + x1) * N2 + 4 * (i % (N2 / 4)));
  });
  float nb[TPW][4][2], dmv[TPW][4];
  if (a.op == 1) {
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      const int tj = wave + 4 * q;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int x1 = x1b + 4 * lk + r, x2 = tj * 16 + li;
        if (tj >= NTJ || x1 >= N1) continue;
        const int xp0 = (x0 + 1 == N0) ? 0 : x0 + 1, xm0 = (x0 == 0) ? N0 - 1 : x0 - 1;
        auto at = [&](int i0, int i1, int i2) { return a.m[((long long)i0 * N1 + i1) * N2 + i2]; };
        nb[q][r][0] = at(xp0, x1, x2);
        nb[q][r][1] = at(xm0, x1, x2);
        dmv[q][r] = a.dm ? a.dm[((long long)x0 * N1 + x1) * N2 + x2] : 0.f;
      }
    }
  }
  // ---- stores
  rt.store(3 * Kh * KP, [&](int i, float4 v) {
    const int c = i / (Kh * KP), kh = (i / KP) % Kh, k1 = 2 * (i % KP);
    t1s[c][k1][kh] = make_float2(v.x, v.y);
    t1s[c][k1 + 1][kh] = make_float2(v.z, v.w);
  });
  rw1.store(R * KP, [&](int i, float4 v) { st22(&w1s[i / KP][2 * (i % KP)], x1b + i / KP < N1 ? v : z4); });
  rw2.store(N2 * KHP, [&](int i, float4 v) {
    const int x2 = i / KHP, kh = 2 * (i % KHP);
    w2t[kh][x2] = make_float2(v.x, v.y);
    w2t[kh + 1][x2] = make_float2(v.z, v.w);
  });
  if (a.op == 1) rm.store(NM4, [&](int i, float4 v) {
    *reinterpret_cast<float4*>(&mrow[i / (N2 / 4)][4 * (i % (N2 / 4))]) = v;
  });
  if constexpr (Khp > Kh) {  // zero padding columns of the half spectrum
    for (int i = threadIdx.x; i < 3 * K1 * (Khp - Kh); i += 256)
      t1s[i / (K1 * (Khp - Kh))][(i / (Khp - Kh)) % K1][Kh + i % (Khp - Kh)] = make_float2(0.f, 0.f);
    for (int i = threadIdx.x; i < (Khp - Kh) * N2; i += 256) w2t[Kh + i / N2][i % N2] = make_float2(0.f, 0.f);
  }
  __syncthreads();
  // stage 1: one 16 x Kh complex tile per component (waves 0..2 when Kh = 16)
  for (int jb = wave; jb < 3 * (Khp / 16); jb += 4) {
    const int c = jb % 3, tj = jb / 3;
    floatx4 acc[4];
    zero_acc(acc, 4);
    ctile<K1 / 4, BF3>(&w1s[0][0], LW1, &t1s[c][0][tj * 16], LT1, acc);
#pragma unroll
    for (int r = 0; r < 4; ++r)
      t2s[c][4 * lk + r][tj * 16 + li] = make_float2(acc[0][r] - acc[1][r], acc[2][r] + acc[3][r]);
  }
  __syncthreads();
  // stage 2 + epilogue: a wave takes whole column tiles (all components)
  const long long nN = (long long)N0 * N1 * N2;
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    const int tj = wave + 4 * q;
    if (tj >= NTJ) break;
    floatx4 vel[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      floatx4 acc[4];
      zero_acc(acc, 4);
      // only the real part is needed: acc0 - acc1
      const float2* A = &t2s[c][0][0] + li * LT2 + lk;
      const float2* B = &w2t[0][0] + lk * LW2 + tj * 16 + li;
#pragma unroll
      for (int ks = 0; ks < Khp / 4; ++ks) {
        const float2 av = A[4 * ks], bv = B[4 * ks * LW2];
        acc[0] = mma<BF3>(av.x, bv.x, acc[0]);
        acc[1] = mma<BF3>(av.y, bv.y, acc[1]);
      }
      vel[c] = acc[0] - acc[1];
    }
    const int x2 = tj * 16 + li;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int x1 = x1b + 4 * lk + r;
      if (x1 >= N1) continue;
      const long long gi = ((long long)x0 * N1 + x1) * N2 + x2;
      if (a.op == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) a.vout[(size_t)c * nN + gi] = vel[c][r];
      } else {
        const int lr = 4 * lk + r + 1;  // row of x1 in mrow
        const int xp2 = (x2 + 1 == N2) ? 0 : x2 + 1, xm2 = (x2 == 0) ? N2 - 1 : x2 - 1;
        const float g0 = (nb[q][r][0] - nb[q][r][1]) * (0.5f * N0);
        const float g1 = (mrow[lr + 1][x2] - mrow[lr - 1][x2]) * (0.5f * N1);
        const float g2 = (mrow[lr][xp2] - mrow[lr][xm2]) * (0.5f * N2);
        const float dot = g0 * vel[0][r] + g1 * vel[1][r] + g2 * vel[2][r];
        a.q[gi] = fmaf(-a.dt, dot, dmv[q][r]);
      }
    }
  }
}

// ----------------------------------------- semi-Lagrangian step (N)
// dst(x) = src(x - dt v(x)) by periodic trilinear interpolation; v in
// domain units, converted to voxels per axis.
template <class G>
__global__ void __launch_bounds__(256) k_sl(const float* __restrict__ src,
                                            const float* __restrict__ vel, float* __restrict__ dst,
                                            float dt, G gs) {
  const int N0 = gs.N0(), N1 = gs.N1(), N2 = gs.N2();
  const long long nN = (long long)N0 * N1 * N2;
  long long gi = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= nN) return;
  int i2 = (int)(gi % N2);
  int i1 = (int)((gi / N2) % N1);
  int i0 = (int)(gi / ((long long)N1 * N2));
  float X0 = (float)i0 - dt * vel[gi] * (float)N0;
  float X1 = (float)i1 - dt * vel[nN + gi] * (float)N1;
  float X2 = (float)i2 - dt * vel[2 * nN + gi] * (float)N2;
  // a non-finite velocity must not turn into an out-of-range index
  if (!isfinite(X0)) X0 = (float)i0;
  if (!isfinite(X1)) X1 = (float)i1;
  if (!isfinite(X2)) X2 = (float)i2;
  float f0 = floorf(X0), f1 = floorf(X1), f2 = floorf(X2);
  float w0 = X0 - f0, w1 = X1 - f1, w2 = X2 - f2;
  int a0 = (int)f0 % N0; if (a0 < 0) a0 += N0;
  int a1 = (int)f1 % N1; if (a1 < 0) a1 += N1;
  int a2 = (int)f2 % N2; if (a2 < 0) a2 += N2;
  int b0 = (a0 + 1 == N0) ? 0 : a0 + 1;
  int b1 = (a1 + 1 == N1) ? 0 : a1 + 1;
  int b2 = (a2 + 1 == N2) ? 0 : a2 + 1;
  auto at = [&](int u, int v, int w) { return src[((long long)u * N1 + v) * N2 + w]; };
  float c00 = at(a0, a1, a2) + w2 * (at(a0, a1, b2) - at(a0, a1, a2));
  float c01 = at(a0, b1, a2) + w2 * (at(a0, b1, b2) - at(a0, b1, a2));
  float c10 = at(b0, a1, a2) + w2 * (at(b0, a1, b2) - at(b0, a1, a2));
  float c11 = at(b0, b1, a2) + w2 * (at(b0, b1, b2) - at(b0, b1, a2));
  float c0 = c00 + w1 * (c01 - c00);
  float c1 = c10 + w1 * (c11 - c10);
  dst[gi] = c0 + w0 * (c1 - c0);
}

// Periodic trilinear interpolation of f at voxel coordinates X (floor cell).
template <class G>
__device__ __forceinline__ float trilinear(const float* __restrict__ f, float X0, float X1, float X2, int i0,
                                           int i1, int i2, G gs) {
  const int N0 = gs.N0(), N1 = gs.N1(), N2 = gs.N2();
  // a non-finite coordinate must not turn into an out-of-range index
  if (!isfinite(X0)) X0 = (float)i0;
  if (!isfinite(X1)) X1 = (float)i1;
  if (!isfinite(X2)) X2 = (float)i2;
  const float f0 = floorf(X0), f1 = floorf(X1), f2 = floorf(X2);
  const float w0 = X0 - f0, w1 = X1 - f1, w2 = X2 - f2;
  int a0 = (int)f0 % N0; if (a0 < 0) a0 += N0;
  int a1 = (int)f1 % N1; if (a1 < 0) a1 += N1;
  int a2 = (int)f2 % N2; if (a2 < 0) a2 += N2;
  const int b0 = (a0 + 1 == N0) ? 0 : a0 + 1;
  const int b1 = (a1 + 1 == N1) ? 0 : a1 + 1;
  const int b2 = (a2 + 1 == N2) ? 0 : a2 + 1;
  auto at = [&](int u, int v, int w) { return f[((long long)u * N1 + v) * N2 + w]; };
  const float c00 = at(a0, a1, a2) + w2 * (at(a0, a1, b2) - at(a0, a1, a2));
  const float c01 = at(a0, b1, a2) + w2 * (at(a0, b1, b2) - at(a0, b1, a2));
  const float c10 = at(b0, a1, a2) + w2 * (at(b0, a1, b2) - at(b0, a1, a2));
  const float c11 = at(b0, b1, a2) + w2 * (at(b0, b1, b2) - at(b0, b1, a2));
  const float c0 = c00 + w1 * (c01 - c00);
  const float c1 = c10 + w1 * (c11 - c10);
  return c0 + w0 * (c1 - c0);
}

// One transport step with midpoint departure points: X_h = x - dt/2 v(x),
// X = x - dt v(X_h) (v trilinear at X_h), dst = src(X).
template <class G>
__global__ void __launch_bounds__(256) k_sl_rk2(const float* __restrict__ src, const float* __restrict__ vel,
                                                float* __restrict__ dst, float dt, G gs) {
  const int N0 = gs.N0(), N1 = gs.N1(), N2 = gs.N2();
  const long long nN = (long long)N0 * N1 * N2;
  const long long gi = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= nN) return;
  const int i2 = (int)(gi % N2), i1 = (int)((gi / N2) % N1), i0 = (int)(gi / ((long long)N1 * N2));
  const float h0 = (float)i0 - 0.5f * dt * vel[gi] * (float)N0;
  const float h1 = (float)i1 - 0.5f * dt * vel[nN + gi] * (float)N1;
  const float h2 = (float)i2 - 0.5f * dt * vel[2 * nN + gi] * (float)N2;
  const float v0 = trilinear(vel, h0, h1, h2, i0, i1, i2, gs);
  const float v1 = trilinear(vel + nN, h0, h1, h2, i0, i1, i2, gs);
  const float v2 = trilinear(vel + 2 * nN, h0, h1, h2, i0, i1, i2, gs);
  dst[gi] = trilinear(src, (float)i0 - dt * v0 * (float)N0, (float)i1 - dt * v1 * (float)N1,
                      (float)i2 - dt * v2 * (float)N2, i0, i1, i2, gs);
}

// ------------------- image-term source and forward stage 2 (N grid)
// s_j = coef * [(a - b) * d_j m + res * d_j a] (periodic central
// differences; b and res may be null) at the points of 16 x1 rows of plane x0, contracted
// over x2: s1[j][x0][x1][kh].
template <class G>
__global__ void __launch_bounds__(256) k_src_fwd2(const float* __restrict__ a,
                                                  const float* __restrict__ b,
                                                  const float* __restrict__ res,
                                                  const float* __restrict__ m, float coef,
                                                  float2* __restrict__ s1, Twiddles tw, G gs) {
  extern __shared__ float shs[];
  const int N0 = gs.N0(), N1 = gs.N1(), N2 = gs.N2(), Kh = gs.Kh();
  constexpr int R = kGridRows;
  const int x0 = blockIdx.y;
  const int x1b = blockIdx.x * R;
  const int rv = min(R, N1 - x1b);
  const int P = R * N2;
  float* vals = shs;                                   // [3][R][N2]
  float2* wfx = (float2*)(vals + ((3 * P + 3) & ~3));  // [N2][Kh]
  batched_fill<float2>(Kh * N2, [&](int i) {
    int x2 = i / Kh, kh = i % Kh;
    return tw.fwd2[(size_t)kh * N2 + x2];
  }, [&](int i, float2 v) { wfx[i] = v; });
  for (int p = threadIdx.x; p < R * N2; p += blockDim.x) {
    int r = p / N2, x2 = p % N2;
    int x1 = x1b + r;
    float v0 = 0.f, v1 = 0.f, v2 = 0.f;
    if (r < rv) {
      long long gi = ((long long)x0 * N1 + x1) * N2 + x2;
      float s = coef * (a[gi] - (b ? b[gi] : 0.f));
      v0 = s * central_diff(m, x0, x1, x2, N0, N1, N2, 0);
      v1 = s * central_diff(m, x0, x1, x2, N0, N1, N2, 1);
      v2 = s * central_diff(m, x0, x1, x2, N0, N1, N2, 2);
      if (res) {
        const float t = coef * res[gi];
        v0 = fmaf(t, central_diff(a, x0, x1, x2, N0, N1, N2, 0), v0);
        v1 = fmaf(t, central_diff(a, x0, x1, x2, N0, N1, N2, 1), v1);
        v2 = fmaf(t, central_diff(a, x0, x1, x2, N0, N1, N2, 2), v2);
      }
    }
    vals[p] = v0;
    vals[P + p] = v1;
    vals[2 * P + p] = v2;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 3 * rv * Kh; i += blockDim.x) {
    int j = i / (rv * Kh), r = (i / Kh) % rv, kh = i % Kh;
    const float* row = vals + (size_t)j * P + r * N2;
    float2 acc = make_float2(0.f, 0.f);
    for (int x2 = 0; x2 < N2; ++x2) {
      float2 w = wfx[(size_t)x2 * Kh + kh];
      acc.x = fmaf(row[x2], w.x, acc.x);
      acc.y = fmaf(row[x2], w.y, acc.y);
    }
    s1[(((size_t)j * N0 + x0) * N1 + x1b + r) * Kh + kh] = acc;
  }
}

// ------------------------------ tangent of one semi-Lagrangian step (N)
// The derivative of m_{n+1}(x) = I[m_n](X(x)), X(x) = x - dt v(x), in the
// direction (dm_n, dv): dm_{n+1}(x) = I[dm_n](X) - dt sum_j N_j
// (d_j I[m_n])(X) dv_j(x), with the interpolant's exact slope in the cell of
// X (dm_n null: zero).
template <class G>
__global__ void __launch_bounds__(256) k_sl_tangent(const float* __restrict__ dm, const float* __restrict__ m,
                                                    const float* __restrict__ vel,
                                                    const float* __restrict__ dvel, float* __restrict__ out,
                                                    float dt, G gs) {
  const int N0 = gs.N0(), N1 = gs.N1(), N2 = gs.N2();
  const long long nN = (long long)N0 * N1 * N2;
  const long long gi = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= nN) return;
  const int i2 = (int)(gi % N2), i1 = (int)((gi / N2) % N1), i0 = (int)(gi / ((long long)N1 * N2));
  float X0 = (float)i0 - dt * vel[gi] * (float)N0;
  float X1 = (float)i1 - dt * vel[nN + gi] * (float)N1;
  float X2 = (float)i2 - dt * vel[2 * nN + gi] * (float)N2;
  if (!isfinite(X0)) X0 = (float)i0;
  if (!isfinite(X1)) X1 = (float)i1;
  if (!isfinite(X2)) X2 = (float)i2;
  const float f0 = floorf(X0), f1 = floorf(X1), f2 = floorf(X2);
  const float w0 = X0 - f0, w1 = X1 - f1, w2 = X2 - f2;
  int a0 = (int)f0 % N0; if (a0 < 0) a0 += N0;
  int a1 = (int)f1 % N1; if (a1 < 0) a1 += N1;
  int a2 = (int)f2 % N2; if (a2 < 0) a2 += N2;
  const int b0 = (a0 + 1 == N0) ? 0 : a0 + 1;
  const int b1 = (a1 + 1 == N1) ? 0 : a1 + 1;
  const int b2 = (a2 + 1 == N2) ? 0 : a2 + 1;
  auto idx = [&](int u, int v, int w) { return ((long long)u * N1 + v) * N2 + w; };
  const float m000 = m[idx(a0, a1, a2)], m001 = m[idx(a0, a1, b2)];
  const float m010 = m[idx(a0, b1, a2)], m011 = m[idx(a0, b1, b2)];
  const float m100 = m[idx(b0, a1, a2)], m101 = m[idx(b0, a1, b2)];
  const float m110 = m[idx(b0, b1, a2)], m111 = m[idx(b0, b1, b2)];
  const float c00 = m000 + w2 * (m001 - m000), c01 = m010 + w2 * (m011 - m010);
  const float c10 = m100 + w2 * (m101 - m100), c11 = m110 + w2 * (m111 - m110);
  const float c0 = c00 + w1 * (c01 - c00), c1 = c10 + w1 * (c11 - c10);
  const float d0 = c1 - c0;
  const float d1 = (c01 - c00) + w0 * ((c11 - c10) - (c01 - c00));
  const float e00 = m001 - m000, e01 = m011 - m010, e10 = m101 - m100, e11 = m111 - m110;
  const float e0 = e00 + w1 * (e01 - e00), e1 = e10 + w1 * (e11 - e10);
  const float d2 = e0 + w0 * (e1 - e0);
  float r = -dt * ((float)N0 * d0 * dvel[gi] + (float)N1 * d1 * dvel[nN + gi] + (float)N2 * d2 * dvel[2 * nN + gi]);
  if (dm) {
    const float q00 = dm[idx(a0, a1, a2)] + w2 * (dm[idx(a0, a1, b2)] - dm[idx(a0, a1, a2)]);
    const float q01 = dm[idx(a0, b1, a2)] + w2 * (dm[idx(a0, b1, b2)] - dm[idx(a0, b1, a2)]);
    const float q10 = dm[idx(b0, a1, a2)] + w2 * (dm[idx(b0, a1, b2)] - dm[idx(b0, a1, a2)]);
    const float q11 = dm[idx(b0, b1, a2)] + w2 * (dm[idx(b0, b1, b2)] - dm[idx(b0, b1, a2)]);
    const float q0 = q00 + w1 * (q01 - q00), q1 = q10 + w1 * (q11 - q10);
    r += q0 + w0 * (q1 - q0);
  }
  out[gi] = r;
}

// ----------- exact adjoint of one semi-Lagrangian step, forward stage 2
// The reverse of m_{n+1}(x) = I[m_n](X(x)), X(x) = x - dt v(x) (voxels per
// axis, the departure point k_sl computes).  For the state adjoint lam of
// m_{n+1} (held as lam / coef): the transpose of the interpolation scatters
// lam(x) with the trilinear weights onto the eight corners of X(x) in
// lam_out (zero on entry; atomic adds), and the derivative with respect to
// the grid velocity, s_j(x) = -dt N_j coef lam(x) (d_j I[m_n])(X(x)) with the
// interpolant's exact slope in the cell of X, is contracted over x2 as in
// k_src_fwd2: s1[j][x0][x1][kh].
template <class G>
__global__ void __launch_bounds__(256) k_adj_src_fwd2(const float* __restrict__ lam,
                                                      const float* __restrict__ m,
                                                      const float* __restrict__ vel,
                                                      float* __restrict__ lam_out, float coef, float dt,
                                                      float2* __restrict__ s1, Twiddles tw, G gs) {
  extern __shared__ float shs[];
  const int N0 = gs.N0(), N1 = gs.N1(), N2 = gs.N2(), Kh = gs.Kh();
  const long long nN = (long long)N0 * N1 * N2;
  constexpr int R = kGridRows;
  const int x0 = blockIdx.y;
  const int x1b = blockIdx.x * R;
  const int rv = min(R, N1 - x1b);
  const int P = R * N2;
  float* vals = shs;                                   // [3][R][N2]
  float2* wfx = (float2*)(vals + ((3 * P + 3) & ~3));  // [N2][Kh]
  batched_fill<float2>(Kh * N2, [&](int i) {
    int x2 = i / Kh, kh = i % Kh;
    return tw.fwd2[(size_t)kh * N2 + x2];
  }, [&](int i, float2 v) { wfx[i] = v; });
  for (int p = threadIdx.x; p < R * N2; p += blockDim.x) {
    const int r = p / N2, x2 = p % N2;
    const int x1 = x1b + r;
    float g0 = 0.f, g1 = 0.f, g2 = 0.f;
    if (r < rv) {
      const long long gi = ((long long)x0 * N1 + x1) * N2 + x2;
      float X0 = (float)x0 - dt * vel[gi] * (float)N0;
      float X1 = (float)x1 - dt * vel[nN + gi] * (float)N1;
      float X2 = (float)x2 - dt * vel[2 * nN + gi] * (float)N2;
      if (!isfinite(X0)) X0 = (float)x0;
      if (!isfinite(X1)) X1 = (float)x1;
      if (!isfinite(X2)) X2 = (float)x2;
      const float f0 = floorf(X0), f1 = floorf(X1), f2 = floorf(X2);
      const float w0 = X0 - f0, w1 = X1 - f1, w2 = X2 - f2;
      int a0 = (int)f0 % N0; if (a0 < 0) a0 += N0;
      int a1 = (int)f1 % N1; if (a1 < 0) a1 += N1;
      int a2 = (int)f2 % N2; if (a2 < 0) a2 += N2;
      const int b0 = (a0 + 1 == N0) ? 0 : a0 + 1;
      const int b1 = (a1 + 1 == N1) ? 0 : a1 + 1;
      const int b2 = (a2 + 1 == N2) ? 0 : a2 + 1;
      auto idx = [&](int u, int v, int w) { return ((long long)u * N1 + v) * N2 + w; };
      const float m000 = m[idx(a0, a1, a2)], m001 = m[idx(a0, a1, b2)];
      const float m010 = m[idx(a0, b1, a2)], m011 = m[idx(a0, b1, b2)];
      const float m100 = m[idx(b0, a1, a2)], m101 = m[idx(b0, a1, b2)];
      const float m110 = m[idx(b0, b1, a2)], m111 = m[idx(b0, b1, b2)];
      // the interpolant's slopes in the cell (lerps of the edge differences)
      const float c00 = m000 + w2 * (m001 - m000), c01 = m010 + w2 * (m011 - m010);
      const float c10 = m100 + w2 * (m101 - m100), c11 = m110 + w2 * (m111 - m110);
      const float c0 = c00 + w1 * (c01 - c00), c1 = c10 + w1 * (c11 - c10);
      const float d0 = c1 - c0;
      const float d1 = (c01 - c00) + w0 * ((c11 - c10) - (c01 - c00));
      const float e00 = m001 - m000, e01 = m011 - m010, e10 = m101 - m100, e11 = m111 - m110;
      const float e0 = e00 + w1 * (e01 - e00), e1 = e10 + w1 * (e11 - e10);
      const float d2 = e0 + w0 * (e1 - e0);
      const float l = lam[gi];
      const float s = -dt * coef * l;
      g0 = s * (float)N0 * d0;
      g1 = s * (float)N1 * d1;
      g2 = s * (float)N2 * d2;
      // transpose of the interpolation
      const float u0 = 1.f - w0, u1 = 1.f - w1, u2 = 1.f - w2;
      atomicAdd(lam_out + idx(a0, a1, a2), l * u0 * u1 * u2);
      atomicAdd(lam_out + idx(a0, a1, b2), l * u0 * u1 * w2);
      atomicAdd(lam_out + idx(a0, b1, a2), l * u0 * w1 * u2);
      atomicAdd(lam_out + idx(a0, b1, b2), l * u0 * w1 * w2);
      atomicAdd(lam_out + idx(b0, a1, a2), l * w0 * u1 * u2);
      atomicAdd(lam_out + idx(b0, a1, b2), l * w0 * u1 * w2);
      atomicAdd(lam_out + idx(b0, b1, a2), l * w0 * w1 * u2);
      atomicAdd(lam_out + idx(b0, b1, b2), l * w0 * w1 * w2);
    }
    vals[p] = g0;
    vals[P + p] = g1;
    vals[2 * P + p] = g2;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 3 * rv * Kh; i += blockDim.x) {
    int j = i / (rv * Kh), r = (i / Kh) % rv, kh = i % Kh;
    const float* row = vals + (size_t)j * P + r * N2;
    float2 acc = make_float2(0.f, 0.f);
    for (int x2 = 0; x2 < N2; ++x2) {
      float2 w = wfx[(size_t)x2 * Kh + kh];
      acc.x = fmaf(row[x2], w.x, acc.x);
      acc.y = fmaf(row[x2], w.y, acc.y);
    }
    s1[(((size_t)j * N0 + x0) * N1 + x1b + r) * Kh + kh] = acc;
  }
}

// ------------- deformation-state image term and forward stage 2 (N grid)
// Central differences of I0 at every node: G_a = d_a I0 and, when H is set,
// H = (d0d0, d0d1, d0d2, d1d1, d1d2, d2d2) I0 (the same central difference
// applied twice; per unit length).
template <class G>
__global__ void __launch_bounds__(256) k_image_derivs(const float* __restrict__ I0, float* __restrict__ Gr,
                                                      float* __restrict__ H, G gs) {
  const int N0 = gs.N0(), N1 = gs.N1(), N2 = gs.N2();
  const long long nN = (long long)N0 * N1 * N2;
  const long long gi = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= nN) return;
  const int x2 = (int)(gi % N2), x1 = (int)((gi / N2) % N1), x0 = (int)(gi / ((long long)N1 * N2));
  const int n[3] = {N0, N1, N2}, x[3] = {x0, x1, x2};
  auto at = [&](int d0, int d1, int d2) {
    int i = x0 + d0, j = x1 + d1, k = x2 + d2;
    i = (i % N0 + N0) % N0;
    j = (j % N1 + N1) % N1;
    k = (k % N2 + N2) % N2;
    return I0[((long long)i * N1 + j) * N2 + k];
  };
  (void)x;
  (void)nN;
  const float c = at(0, 0, 0);
  reinterpret_cast<float4*>(Gr)[gi] =
      make_float4(c, (at(1, 0, 0) - at(-1, 0, 0)) * (0.5f * N0), (at(0, 1, 0) - at(0, -1, 0)) * (0.5f * N1),
                  (at(0, 0, 1) - at(0, 0, -1)) * (0.5f * N2));
  if (!H) return;
  reinterpret_cast<float4*>(H)[2 * gi] =
      make_float4((at(2, 0, 0) - 2.f * c + at(-2, 0, 0)) * (0.25f * n[0] * n[0]),
                  (at(1, 1, 0) - at(1, -1, 0) - at(-1, 1, 0) + at(-1, -1, 0)) * (0.25f * n[0] * n[1]),
                  (at(1, 0, 1) - at(1, 0, -1) - at(-1, 0, 1) + at(-1, 0, -1)) * (0.25f * n[0] * n[2]),
                  (at(0, 2, 0) - 2.f * c + at(0, -2, 0)) * (0.25f * n[1] * n[1]));
  reinterpret_cast<float4*>(H)[2 * gi + 1] =
      make_float4((at(0, 1, 1) - at(0, 1, -1) - at(0, -1, 1) + at(0, -1, -1)) * (0.25f * n[1] * n[2]),
                  (at(0, 0, 2) - 2.f * c + at(0, 0, -2)) * (0.25f * n[2] * n[2]), 0.f, 0.f);
}

// At phi(x) = x + u(x) (voxel coordinates x_j + N_j u_j) the periodic
// trilinear interpolation of I0, of its central-difference gradient G and
// (full Newton) of its central-difference Hessian H gives m, g and h.
// op 0: s_j = coef (m - I1) g_j.  op 1: s_j = coef (g . du) g_j
// [+ coef res (h du)_j when res is set].  Then forward stage 2 of the three
// sources like k_src_fwd2.
template <class G>
__global__ void __launch_bounds__(256) k_rho_fwd2(RhoArgs a, float2* __restrict__ s1, Twiddles tw, G gs) {
  extern __shared__ float shs[];
  const int N0 = gs.N0(), N1 = gs.N1(), N2 = gs.N2(), Kh = gs.Kh();
  const long long nN = (long long)N0 * N1 * N2;
  constexpr int R = kGridRows;
  const int x0 = blockIdx.y;
  const int x1b = blockIdx.x * R;
  const int rv = min(R, N1 - x1b);
  const int P = R * N2;
  float* vals = shs;                                   // [3][R][N2]
  float2* wfx = (float2*)(vals + ((3 * P + 3) & ~3));  // [N2][Kh]
  batched_fill<float2>(Kh * N2, [&](int i) {
    int x2 = i / Kh, kh = i % Kh;
    return tw.fwd2[(size_t)kh * N2 + x2];
  }, [&](int i, float2 v) { wfx[i] = v; });
  // two points per iteration, so that two chains of dependent loads are in flight
#pragma unroll 2
  for (int p = threadIdx.x; p < R * N2; p += blockDim.x) {
    const int r = p / N2, x2 = p % N2;
    const int x1 = x1b + r;
    float v0 = 0.f, v1 = 0.f, v2 = 0.f;
    if (r < rv) {
      const long long gi = ((long long)x0 * N1 + x1) * N2 + x2;
      float X0 = (float)x0 + a.u[gi] * (float)N0;
      float X1 = (float)x1 + a.u[nN + gi] * (float)N1;
      float X2 = (float)x2 + a.u[2 * nN + gi] * (float)N2;
      // a non-finite displacement must not turn into an out-of-range index
      if (!isfinite(X0)) X0 = (float)x0;
      if (!isfinite(X1)) X1 = (float)x1;
      if (!isfinite(X2)) X2 = (float)x2;
      const float f0 = floorf(X0), f1 = floorf(X1), f2 = floorf(X2);
      const float w0 = X0 - f0, w1 = X1 - f1, w2 = X2 - f2;
      int a0 = (int)f0 % N0; if (a0 < 0) a0 += N0;
      int a1 = (int)f1 % N1; if (a1 < 0) a1 += N1;
      int a2 = (int)f2 % N2; if (a2 < 0) a2 += N2;
      const int b0 = (a0 + 1 == N0) ? 0 : a0 + 1;
      const int b1 = (a1 + 1 == N1) ? 0 : a1 + 1;
      const int b2 = (a2 + 1 == N2) ? 0 : a2 + 1;
      const long long r00 = ((long long)a0 * N1 + a1) * N2, r01 = ((long long)a0 * N1 + b1) * N2;
      const long long r10 = ((long long)b0 * N1 + a1) * N2, r11 = ((long long)b0 * N1 + b1) * N2;
      // the four (or eight) channels of a point are one 16-byte load per corner
      auto lerp4 = [](float4 p, float4 q, float w) {
        return make_float4(p.x + w * (q.x - p.x), p.y + w * (q.y - p.y), p.z + w * (q.z - p.z),
                           p.w + w * (q.w - p.w));
      };
      auto interp4 = [&](const float4* f, int stride) {
        const float4 c00 = lerp4(f[stride * (r00 + a2)], f[stride * (r00 + b2)], w2);
        const float4 c01 = lerp4(f[stride * (r01 + a2)], f[stride * (r01 + b2)], w2);
        const float4 c10 = lerp4(f[stride * (r10 + a2)], f[stride * (r10 + b2)], w2);
        const float4 c11 = lerp4(f[stride * (r11 + a2)], f[stride * (r11 + b2)], w2);
        return lerp4(lerp4(c00, c01, w1), lerp4(c10, c11, w1), w0);
      };
      const float4 ig = interp4(reinterpret_cast<const float4*>(a.G), 1);  // (I0, d0, d1, d2)
      const float g0 = ig.y, g1 = ig.z, g2 = ig.w;
      if (a.op == 0) {
        const float l = a.coef * (ig.x - a.I1[gi]);
        v0 = l * g0;
        v1 = l * g1;
        v2 = l * g2;
      } else {
        const float du0 = a.du[gi], du1 = a.du[nN + gi], du2 = a.du[2 * nN + gi];
        const float l = a.coef * (g0 * du0 + g1 * du1 + g2 * du2);
        v0 = l * g0;
        v1 = l * g1;
        v2 = l * g2;
        if (a.res) {
          const float4 ha = interp4(reinterpret_cast<const float4*>(a.H), 2);      // (00, 01, 02, 11)
          const float4 hb = interp4(reinterpret_cast<const float4*>(a.H) + 1, 2);  // (12, 22, -, -)
          const float h00 = ha.x, h01 = ha.y, h02 = ha.z, h11 = ha.w, h12 = hb.x, h22 = hb.y;
          const float t = a.coef * a.res[gi];
          v0 = fmaf(t, h00 * du0 + h01 * du1 + h02 * du2, v0);
          v1 = fmaf(t, h01 * du0 + h11 * du1 + h12 * du2, v1);
          v2 = fmaf(t, h02 * du0 + h12 * du1 + h22 * du2, v2);
        }
      }
    }
    vals[p] = v0;
    vals[P + p] = v1;
    vals[2 * P + p] = v2;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 3 * rv * Kh; i += blockDim.x) {
    int j = i / (rv * Kh), r = (i / Kh) % rv, kh = i % Kh;
    const float* row = vals + (size_t)j * P + r * N2;
    float2 acc = make_float2(0.f, 0.f);
    for (int x2 = 0; x2 < N2; ++x2) {
      float2 w = wfx[(size_t)x2 * Kh + kh];
      acc.x = fmaf(row[x2], w.x, acc.x);
      acc.y = fmaf(row[x2], w.y, acc.y);
    }
    s1[(((size_t)j * N0 + x0) * N1 + x1b + r) * Kh + kh] = acc;
  }
}

// ------------------------------------------------- fused t = 1 tail (tuned)
// k_srcfwd: one block per (64-row chunk of x1, x0 plane), four waves, in
// sub-chunks of 32 rows: the source s_j = coef [(a - b) d_j m + res d_j a]
// (periodic central differences; the res term with FULL), forward stage 2
// (x2 -> kh) on the matrix cores, and
// the chunk's part of forward stage 1 (x1 -> k1), accumulated in the matrix
// accumulators over the sub-chunks: P[part][j][kh][x0][k1].
constexpr int kTailRows = 64, kTailSub = 32;
template <class G, bool FULL, bool BF3>
__global__ void __launch_bounds__(256) k_srcfwd(const float* __restrict__ a, const float* __restrict__ b,
                                                const float* __restrict__ res, const float* __restrict__ m,
                                                float coef, float2* __restrict__ P, Twiddles tw) {
  constexpr int N0 = G::N0(), N1 = G::N1(), N2 = G::N2(), K1 = G::K1(), Kh = G::Kh();
  constexpr int SR = kTailSub, RC = kTailRows < N1 ? kTailRows : N1, NSUB = RC / SR;
  constexpr int Q = N2 / 4;  // float4 per grid row
  // MFMA A operands: rows 2 mod 32 floats (vals) or odd complex strides (w1f);
  // the stage-2 table (a B operand) 16 mod 32
  constexpr int LM = N2 + 4, LV = N2 + 2, LW2 = ((2 * Kh) % 32 == 16) ? 2 * Kh : 2 * Kh + 16;
  constexpr int Khp = (Kh + 15) & ~15, LO = Khp + 2, LW1 = RC + 1;
  constexpr int TR = SR / 16, TC = 2 * Kh / 16;
  constexpr int TK1 = K1 / 16, TKH = Khp / 16, NT1 = 3 * TK1 * TKH, TPW = (NT1 + 3) / 4;
  static_assert(N2 % 4 == 0 && N1 % RC == 0 && RC % SR == 0 && (2 * Kh) % 16 == 0 && K1 % 16 == 0 &&
                    N2 % 2 == 0 && RC % 2 == 0,
                "tail shape");
  __shared__ __align__(16) float mr[SR + 2][LM];   // m rows x1 - 1 .. x1 + SR of the sub-chunk
  __shared__ __align__(16) float ar[FULL ? SR + 2 : 1][LM];  // the same rows of a (FULL)
  __shared__ __align__(16) float vals[3][SR][LV];  // source fields
  __shared__ __align__(16) float w2r[N2][LW2];     // forward stage 2: re (j < Kh) | im (j >= Kh)
  __shared__ __align__(16) float2 o2[3][SR][LO];   // stage-2 output, kh columns padded with zero
  __shared__ __align__(16) float2 w1f[K1][LW1];    // forward stage-1 columns of this chunk
  const int x0 = blockIdx.y, part = blockIdx.x, x1c = part * RC;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
  {
    RegStage<(Kh * N2 / 2 + 255) / 256, float4> r2;
    RegStage<(K1 * RC / 2 + 255) / 256, float4> r1;
    r2.load(Kh * N2 / 2, [&](int i) { return ld4(tw.fwd2 + 2 * i); });
    r1.load(K1 * RC / 2, [&](int i) {
      return ld4(tw.fwd1 + (size_t)(i / (RC / 2)) * N1 + x1c + 2 * (i % (RC / 2)));
    });
    // columns XOR-swizzled by (x2 / 2) % 16 within their 16-column group, so
    // that these stores (consecutive threads: consecutive even x2) spread
    // over the banks while the MFMA reads below stay conflict free
    r2.store(Kh * N2 / 2, [&](int i, float4 v) {
      const int kh = (2 * i) / N2, x2 = (2 * i) % N2, sw = (x2 >> 1) & 15;
      w2r[x2][kh ^ sw] = v.x;
      w2r[x2][(Kh + kh) ^ sw] = v.y;
      w2r[x2 + 1][kh ^ sw] = v.z;
      w2r[x2 + 1][(Kh + kh) ^ sw] = v.w;
    });
    r1.store(K1 * RC / 2, [&](int i, float4 v) { st22(&w1f[i / (RC / 2)][2 * (i % (RC / 2))], v); });
    if constexpr (Khp > Kh)
      for (int i = threadIdx.x; i < 3 * SR * (Khp - Kh); i += 256)
        o2[i / (SR * (Khp - Kh))][(i / (Khp - Kh)) % SR][Kh + i % (Khp - Kh)] = make_float2(0.f, 0.f);
  }
  floatx4 acc[TPW][4];
#pragma unroll
  for (int q = 0; q < TPW; ++q) zero_acc(acc[q], 4);
  const int xp0 = (x0 + 1 == N0) ? 0 : x0 + 1, xm0 = (x0 == 0) ? N0 - 1 : x0 - 1;
  auto row4 = [&](const float* f, int plane, int x1, int q) {
    return *reinterpret_cast<const float4*>(f + ((size_t)plane * N1 + x1) * N2 + 4 * q);
  };
  for (int sub = 0; sub < NSUB; ++sub) {
    const int x1s = x1c + sub * SR;
    RegStage<(SR * Q + 255) / 256, float4> ra, rb, rp, rn;
    RegStage<((SR + 2) * Q + 255) / 256, float4> rm;
    ra.load(SR * Q, [&](int i) { return row4(a, x0, x1s + i / Q, i % Q); });
    if (b) rb.load(SR * Q, [&](int i) { return row4(b, x0, x1s + i / Q, i % Q); });
    rp.load(SR * Q, [&](int i) { return row4(m, xp0, x1s + i / Q, i % Q); });
    rn.load(SR * Q, [&](int i) { return row4(m, xm0, x1s + i / Q, i % Q); });
    auto wrap1 = [&](int x1) { return (x1 < 0) ? x1 + N1 : (x1 >= N1 ? x1 - N1 : x1); };
    rm.load((SR + 2) * Q, [&](int i) { return row4(m, x0, wrap1(x1s - 1 + i / Q), i % Q); });
    RegStage<FULL ? (SR * Q + 255) / 256 : 1, float4> rres, rap, ran;
    RegStage<FULL ? ((SR + 2) * Q + 255) / 256 : 1, float4> ram;
    if constexpr (FULL) {
      rres.load(SR * Q, [&](int i) { return row4(res, x0, x1s + i / Q, i % Q); });
      rap.load(SR * Q, [&](int i) { return row4(a, xp0, x1s + i / Q, i % Q); });
      ran.load(SR * Q, [&](int i) { return row4(a, xm0, x1s + i / Q, i % Q); });
      ram.load((SR + 2) * Q, [&](int i) { return row4(a, x0, wrap1(x1s - 1 + i / Q), i % Q); });
      ram.store((SR + 2) * Q, [&](int i, float4 v) {
        *reinterpret_cast<float4*>(&ar[i / Q][4 * (i % Q)]) = v;
      });
    }
    rm.store((SR + 2) * Q, [&](int i, float4 v) {
      *reinterpret_cast<float4*>(&mr[i / Q][4 * (i % Q)]) = v;
    });
    __syncthreads();
#pragma unroll
    for (int u = 0; u < (SR * Q + 255) / 256; ++u) {
      const int i = threadIdx.x + 256 * u;
      if (i >= SR * Q) continue;
      const int r0 = i / Q, q = i % Q;
      const float av[4] = {ra.r[u].x, ra.r[u].y, ra.r[u].z, ra.r[u].w};
      const float4 bw = b ? rb.r[u] : z4;
      const float bv[4] = {bw.x, bw.y, bw.z, bw.w};
      const float pv[4] = {rp.r[u].x, rp.r[u].y, rp.r[u].z, rp.r[u].w};
      const float nv[4] = {rn.r[u].x, rn.r[u].y, rn.r[u].z, rn.r[u].w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int x2 = 4 * q + e;
        const int x2p = (x2 + 1 == N2) ? 0 : x2 + 1, x2m = (x2 == 0) ? N2 - 1 : x2 - 1;
        const float sv = coef * (av[e] - bv[e]);
        float s0 = sv * ((pv[e] - nv[e]) * (0.5f * N0));
        float s1 = sv * ((mr[r0 + 2][x2] - mr[r0][x2]) * (0.5f * N1));
        float s2 = sv * ((mr[r0 + 1][x2p] - mr[r0 + 1][x2m]) * (0.5f * N2));
        if constexpr (FULL) {
          const float rv[4] = {rres.r[u].x, rres.r[u].y, rres.r[u].z, rres.r[u].w};
          const float apv[4] = {rap.r[u].x, rap.r[u].y, rap.r[u].z, rap.r[u].w};
          const float anv[4] = {ran.r[u].x, ran.r[u].y, ran.r[u].z, ran.r[u].w};
          const float t = coef * rv[e];
          s0 = fmaf(t, (apv[e] - anv[e]) * (0.5f * N0), s0);
          s1 = fmaf(t, (ar[r0 + 2][x2] - ar[r0][x2]) * (0.5f * N1), s1);
          s2 = fmaf(t, (ar[r0 + 1][x2p] - ar[r0 + 1][x2m]) * (0.5f * N2), s2);
        }
        vals[0][r0][x2] = s0;
        vals[1][r0][x2] = s1;
        vals[2][r0][x2] = s2;
      }
    }
    __syncthreads();
    // forward stage 2: o2[j][r][kh] = sum_x2 vals[j][r][x2] fwd2[kh][x2]
    for (int jb = wave; jb < 3 * TR * TC; jb += 4) {
      const int c = jb / (TR * TC), ti = (jb / TC) % TR, tj = jb % TC;
      floatx4 a2 = {0.f, 0.f, 0.f, 0.f};
      const float* A = &vals[c][ti * 16][0] + li * LV + lk;
      const float* B = &w2r[0][0] + lk * LW2 + tj * 16;
#pragma unroll 8
      for (int ks = 0; ks < N2 / 4; ++ks)  // row 4 ks + lk, swizzle (2 ks + lk / 2) % 16
        a2 = mma<BF3>(A[4 * ks], B[4 * ks * LW2 + (li ^ ((2 * ks + (lk >> 1)) & 15))], a2);
      const int j = tj * 16 + li;
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int r = ti * 16 + 4 * lk + rr;
        if (j < Kh) o2[c][r][j].x = a2[rr];
        else o2[c][r][j - Kh].y = a2[rr];
      }
    }
    __syncthreads();
    // this sub-chunk's part of forward stage 1: acc += w1f[k1][x1] o2[j][x1][kh]
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      const int t = wave + 4 * q;
      if (t >= NT1) break;
      const int c = t / (TK1 * TKH), ti = (t / TKH) % TK1, tj = t % TKH;
      ctile<SR / 4, BF3>(&w1f[ti * 16][sub * SR], LW1, &o2[c][0][tj * 16], LO, acc[q]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    const int t = wave + 4 * q;
    if (t >= NT1) break;
    const int c = t / (TK1 * TKH), ti = (t / TKH) % TK1, tj = t % TKH;
    const int kh = tj * 16 + li;
    if (kh >= Kh) continue;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int k1 = ti * 16 + 4 * lk + rr;
      P[((((size_t)part * 3 + c) * Kh + kh) * N0 + x0) * K1 + k1] =
          make_float2(acc[q][0][rr] - acc[q][1][rr], acc[q][2][rr] + acc[q][3][rr]);
    }
  }
}

// k_fwd0_mfma: one block per (kh, component, 16-wide tile of k1), four
// waves: forward stage 0 over (part, x0) of P (the parts add up), split over
// the waves of each output tile; the epilogue out = ca K~ F / |N| (zero on
// the k = -K/2 slots); the padded-grid inverse stage 0 of L~ out into the
// group-0 stage-0 buffer and zero into the group-1 buffer.
struct TailJobs {
  const float2* P;
  float2* out;       // band field [3][Kh][K0][K1]
  float2* t1u[3];    // [2][M0][Kh][K1] per component
  float2* t1z[3];
  float ca;
};
template <class S, int NG0, int NP, bool BF3>
__global__ void __launch_bounds__(256) k_fwd0_mfma(TailJobs tj, const float2* __restrict__ w0n,
                                                   const float2* __restrict__ w0i, double alpha,
                                                   int spow, float invG) {
  constexpr int K = S::K0(), M = S::M0(), Kh = S::Kh();
  constexpr int Mp = (M + 15) & ~15, Kp = (K + 15) & ~15, C = K * Kh;
  constexpr int LB = 18, LA = NG0 + 1, LW0I = K + 1, LOB = 18;  // A operands: odd complex strides
  constexpr int T0 = Kp / 16, SPL = 4 / T0, DEPTH = NP * NG0, LEN = DEPTH / SPL;
  static_assert(K % 16 == 0, "whole k1 tiles");
  static_assert(4 % T0 == 0 && DEPTH % SPL == 0 && (LEN <= NG0 ? NG0 % LEN == 0 : LEN % NG0 == 0) &&
                    LEN % 4 == 0 && LEN <= NG0 && NG0 % 2 == 0 && K % 2 == 0,
                "tail stage-0 shape");
  __shared__ __align__(16) float2 bs[DEPTH][LB];     // P rows (part, x0) of this column tile
  __shared__ __align__(16) float2 as[Kp][LA];        // forward stage-0 table [k0][x0]
  __shared__ __align__(16) float2 w0is[2][Mp][LW0I];
  __shared__ __align__(16) float2 ob[2][K][LOB];
  __shared__ __align__(16) floatx4 red[4][4][64];
  const int kh = blockIdx.x, c = blockIdx.y, kc = blockIdx.z * 16;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const int k1 = kc + li;
  const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
  RegStage<(DEPTH * 8 + 255) / 256, float4> rb;
  RegStage<(Kp * NG0 / 2 + 255) / 256, float4> ra;
  RegStage<(2 * Mp * K / 2 + 255) / 256, float4> rw;
  rb.load(DEPTH * 8, [&](int i) {
    const int row = i / 8, p = row / NG0, x0 = row % NG0;
    return ld4(tj.P + ((((size_t)p * 3 + c) * Kh + kh) * NG0 + x0) * K + kc + 2 * (i % 8));
  });
  ra.load(Kp * NG0 / 2, [&](int i) {  // rows past K load a valid row and are zeroed when stored
    const int k0 = i / (NG0 / 2);
    return ld4(w0n + (size_t)(k0 < K ? k0 : K - 1) * NG0 + 2 * (i % (NG0 / 2)));
  });
  rw.load(2 * Mp * K / 2, [&](int i) { return ld4(w0i + 2 * i); });
  float pks[4], pls[4];
  if (wave < T0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int k0 = wave * 16 + 4 * lk + r;
      const bool ok = k0 < K && k1 < K;
      const float2 sym = band_symbols(ok ? k0 : 0, ok ? k1 : 0, kh, K, K, spow, alpha);
      pks[r] = ok ? sym.y : 0.f;
      pls[r] = ok ? sym.x : 0.f;
    }
  }
  rb.store(DEPTH * 8, [&](int i, float4 v) { st4(&bs[i / 8][2 * (i % 8)], v); });
  ra.store(Kp * NG0 / 2, [&](int i, float4 v) {
    st22(&as[i / (NG0 / 2)][2 * (i % (NG0 / 2))], i / (NG0 / 2) < K ? v : z4);
  });
  rw.store(2 * Mp * K / 2, [&](int i, float4 v) {
    st22(&w0is[i / (Mp * K / 2)][(i / (K / 2)) % Mp][2 * (i % (K / 2))], v);
  });
  __syncthreads();
  {  // tile ti = wave % T0, depth split h = wave / T0
    const int ti = wave % T0, h = wave / T0, d0 = h * LEN;
    floatx4 acc[4];
    zero_acc(acc, 4);
    ctile<LEN / 4, BF3>(&as[ti * 16][d0 % NG0], LA, &bs[d0][0], LB, acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) red[wave][i][lane] = acc[i];
  }
  __syncthreads();
  if (wave < T0) {
    const int ti = wave;
    floatx4 acc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      acc[i] = red[ti][i][lane];
#pragma unroll
      for (int h = 1; h < SPL; ++h) acc[i] += red[ti + T0 * h][i][lane];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int k0 = ti * 16 + 4 * lk + r;
      if (k0 >= K || k1 >= K) continue;
      float2 res = make_float2(0.f, 0.f);
      if (k0 != K / 2 && k1 != K / 2) {
        const float sc = tj.ca * invG * pks[r];
        res = make_float2(sc * (acc[0][r] - acc[1][r]), sc * (acc[2][r] + acc[3][r]));
      }
      tj.out[(size_t)c * K * C + ((size_t)kh * K + k0) * K + k1] = res;
      ob[0][k0][li] = res;
      ob[1][k0][li] = make_float2(pls[r] * res.x, pls[r] * res.y);
    }
  }
  __syncthreads();
  // padded-grid inverse stage 0 of L~ out (both variants); group 1 is zero
  constexpr int TIR = Mp / 16;
  for (int jb = wave; jb < 2 * TIR; jb += 4) {
    const int v = jb / TIR, ti = jb % TIR;
    floatx4 acc[4];
    zero_acc(acc, 4);
    ctile<K / 4, BF3>(&w0is[v][ti * 16][0], LW0I, &ob[1][0][0], LOB, acc);
    if (k1 >= K) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int x0 = ti * 16 + 4 * lk + r;
      if (x0 >= M) continue;
      const size_t o = ((size_t)v * M + x0) * C + (size_t)kh * K + k1;
      tj.t1u[c][o] = make_float2(acc[0][r] - acc[1][r], acc[2][r] + acc[3][r]);
      tj.t1z[c][o] = make_float2(0.f, 0.f);
    }
  }
}

// ------------------------------------------------------ elementwise
__global__ void k_fill(float* p, long long n, float v) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_copy(const float* __restrict__ s, float* __restrict__ d, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = s[i];
}
__global__ void k_diff(const float* __restrict__ a, const float* __restrict__ b, float* __restrict__ d,
                       long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = a[i] - b[i];
}
__global__ void k_axpy_band(const float2* x, const float2* y, float a, float2* out, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float2 u = x[i], v = y[i];
  out[i] = make_float2(fmaf(a, v.x, u.x), fmaf(a, v.y, u.y));
}

// ------------------------------------------------------- reductions
constexpr int kRedBlocks = 512;
constexpr int kRedThreads = 256;

__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += sh[w];
  return r;
}

__global__ void __launch_bounds__(kRedThreads) k_sqdiff(const float* a, const float* b, long long n,
                                                        double* partial) {
  __shared__ double sh[kRedThreads / 64];
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    double d = (double)a[i] - (double)(b ? b[i] : 0.f);
    s += d * d;
  }
  double r = block_sum(s, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

// sum_c sum_k w(k2) (L~ if given) Re(conj a b), w = 1 at k2 = 0 else 2 (band layout [3][Kh][K0][K1])
__global__ void __launch_bounds__(kRedThreads) k_band_dot(const float2* a, const float2* b,
                                                          const float* Lsym, int nb, int Kh,
                                                          double* partial) {
  __shared__ double sh[kRedThreads / 64];
  double s = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < 3 * nb; i += gridDim.x * blockDim.x) {
    int e = i % nb;
    double w = (e < nb / Kh) ? 1.0 : 2.0;  // layout [Kh][K0][K1]: k2 = 0 first
    if (Lsym) w *= (double)Lsym[e];
    s += w * ((double)a[i].x * b[i].x + (double)a[i].y * b[i].y);
  }
  double r = block_sum(s, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

// k_band_dot and k_final in one launch: each block stores its partial sum,
// and the block that finishes last (by a device-wide counter) adds the
// partials in k_final's order and resets the counter.
__device__ void pcg_phase_a_body(double* sc);
__device__ void pcg_phase_b_body(double* sc, double* host);

// post: 0, or the CG scalar phase that follows the sum (1: phase a, 2: phase
// b with the optional host pair), run by the last block once the sum is in *out
__global__ void __launch_bounds__(kRedThreads) k_band_dot_once(const float2* a, const float2* b,
                                                               const float* Lsym, int nb, int Kh, double* partial,
                                                               unsigned* count, double* out, double scale,
                                                               double* pcg, int post, double* host) {
  __shared__ double sh[kRedThreads];
  __shared__ bool last;
  double s = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < 3 * nb; i += gridDim.x * blockDim.x) {
    int e = i % nb;
    double w = (e < nb / Kh) ? 1.0 : 2.0;  // layout [Kh][K0][K1]: k2 = 0 first
    if (Lsym) w *= (double)Lsym[e];
    s += w * ((double)a[i].x * b[i].x + (double)a[i].y * b[i].y);
  }
  const double r = block_sum(s, sh);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = r;
    __threadfence();
    last = atomicAdd(count, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  const volatile double* vp = partial;
  double v = 0.0;
  for (int i = threadIdx.x; i < (int)gridDim.x; i += blockDim.x) v = v + vp[i];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *out = scale * sh[0];
    *count = 0u;
    if (post == 1) pcg_phase_a_body(pcg);
    if (post == 2) pcg_phase_b_body(pcg, host);
  }
}

__global__ void __launch_bounds__(kRedThreads) k_band_maxabs(const float2* a, int n,
                                                             double* partial) {
  __shared__ double sh[kRedThreads];
  double m = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    m = fmax(m, sqrt((double)a[i].x * a[i].x + (double)a[i].y * a[i].y));
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(kRedThreads) k_final(const double* partial, int n, double* out,
                                                       double scale, int is_max) {
  __shared__ double sh[kRedThreads];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s = is_max ? fmax(s, partial[i]) : s + partial[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      sh[threadIdx.x] = is_max ? fmax(sh[threadIdx.x], sh[threadIdx.x + o])
                               : sh[threadIdx.x] + sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = scale * sh[0];
}

__global__ void k_energy_combine(double* sc) {
  if (threadIdx.x == 0) sc[0] = sc[1] + sc[2];
}

__global__ void k_pcg_reset(double* sc) {
  int i = threadIdx.x;
  if (i < SC_COUNT && i != SC_RR) sc[i] = 0.0;
}

__global__ void k_scalar_copy(const double* s, double* d, int n) {
  int i = threadIdx.x;
  if (i < n) d[i] = s[i];
}

// ------------------------------------------------------------- CG
__global__ void k_pcg_init(const float2* g, float2* p, float2* r, float2* dv, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float2 v = make_float2(-g[i].x, -g[i].y);
  p[i] = make_float2(0.f, 0.f);
  r[i] = v;
  dv[i] = v;
}

// After <d, H d>_V: decide whether this iteration updates.  The first
// iteration is the one before any update (SC_ITERS == 0 and not stopped).
__device__ void pcg_phase_a_body(double* sc) {
  sc[SC_DOUPD] = 0.0;
  sc[SC_NEGG] = 0.0;
  if (sc[SC_STOPPED] != 0.0) return;
  if (!(sc[SC_RR] > 0.0)) { sc[SC_STOPPED] = 1.0; return; }
  if (!(sc[SC_DHD] > 0.0)) {
    sc[SC_STOPPED] = 1.0;
    sc[SC_GUARD] = 1.0;
    if (sc[SC_ITERS] == 0.0) sc[SC_NEGG] = 1.0;
    return;
  }
  sc[SC_ALPHA] = sc[SC_RR] / sc[SC_DHD];
  sc[SC_DOUPD] = 1.0;
}

__global__ void k_pcg_update_pr(const double* sc, const float2* dv, const float2* Hd, float2* p,
                                float2* r, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (sc[SC_NEGG] != 0.0) { p[i] = dv[i]; return; }  // first iteration: d = -g
  if (sc[SC_DOUPD] == 0.0) return;
  float al = (float)sc[SC_ALPHA];
  float2 pv = p[i], rv = r[i], dd = dv[i], hd = Hd[i];
  p[i] = make_float2(fmaf(al, dd.x, pv.x), fmaf(al, dd.y, pv.y));
  r[i] = make_float2(fmaf(-al, hd.x, rv.x), fmaf(-al, hd.y, rv.y));
}

// After <r, r>_V: beta = <r, r>_new / <r, r>_old for an iteration that
// updated.  host (optional, pinned host memory): host[1] = the stop flag of
// this iteration, then host[0] = 1, both visible system-wide.
__device__ void pcg_phase_b_body(double* sc, double* host) {
  if (host) {
    host[1] = sc[SC_STOPPED];
    __threadfence_system();
    __hip_atomic_store(host, 1.0, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
  if (sc[SC_DOUPD] == 0.0) return;
  sc[SC_BETA] = sc[SC_RRNEW] / sc[SC_RR];
  sc[SC_RR] = sc[SC_RRNEW];
  sc[SC_ITERS] += 1.0;
}

__global__ void k_pcg_update_d(const double* sc, const float2* r, float2* dv, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (sc[SC_DOUPD] == 0.0) return;
  float be = (float)sc[SC_BETA];
  float2 rv = r[i], dd = dv[i];
  dv[i] = make_float2(fmaf(be, dd.x, rv.x), fmaf(be, dd.y, rv.y));
}

// ================================================= launch wrappers
// Launch of a kernel the timer may sample: a sampled launch carries the
// timer's start and stop events in its dispatch (they then hold the times the
// dispatch began and completed, which include the command processor's
// per-dispatch work around the kernel); while a graph is being captured, the
// kernel node is handed to the timer instead.
#define LAUNCH_TIMED(fam, kernel, grid, block, shm, st, ...)                              \
  do {                                                                                     \
    hipEvent_t ev0_ = nullptr, ev1_ = nullptr;                                             \
    if (timer_events((fam), &ev0_, &ev1_))                                                 \
      hipExtLaunchKernelGGL(kernel, grid, block, shm, st, ev0_, ev1_, 0, __VA_ARGS__);    \
    else                                                                                   \
      hipLaunchKernelGGL(kernel, grid, block, shm, st, __VA_ARGS__);                       \
    timer_captured((fam), st);                                                             \
  } while (0)

static inline unsigned nblk(long long n, int t) { return (unsigned)((n + t - 1) / t); }

static bool band_iso(const Dims& d, int K, int M) {
  return d.K[0] == K && d.K[1] == K && d.K[2] == K && d.M[0] == M && d.M[1] == M && d.M[2] == M;
}
static bool grid_iso(const Dims& d, int N, int K) {
  return d.N[0] == N && d.N[1] == N && d.N[2] == N && d.K[1] == K && d.K[2] == K;
}
static bool grid_is(const Dims& d, int A, int B, int C, int K) {
  return d.N[0] == A && d.N[1] == B && d.N[2] == C && d.K[1] == K && d.K[2] == K;
}
// Calls f with the band shape type for these sizes.
template <class F>
static hipError_t with_band(const Dims& d, F&& f) {
  if (band_iso(d, 32, 48)) return f(BandIso<32, 48>{});
  if (band_iso(d, 16, 24)) return f(BandIso<16, 24>{});
  if (band_iso(d, 24, 36)) return f(BandIso<24, 36>{});
  return f(BandDyn{d.K[0], d.K[1], d.Kh, d.M[0], d.M[1], d.M[2]});
}
template <class F>
static hipError_t with_grid(const Dims& d, F&& f) {
  // the measured volume, the 64^3 problem and the grids of the atlas
  // batch and of the differentiation volume, with bands 24^3 and 32^3
  if (grid_iso(d, 128, 32)) return f(GridIso<128, 32>{});
  if (grid_iso(d, 64, 16)) return f(GridIso<64, 16>{});
  if (grid_iso(d, 128, 24)) return f(GridIso<128, 24>{});
  if (grid_iso(d, 96, 24)) return f(GridIso<96, 24>{});
  if (grid_iso(d, 96, 32)) return f(GridIso<96, 32>{});
  if (grid_is(d, 144, 176, 144, 24)) return f(GridShape<144, 176, 144, 24>{});
  if (grid_is(d, 144, 176, 144, 32)) return f(GridShape<144, 176, 144, 32>{});
  if (grid_is(d, 160, 192, 160, 24)) return f(GridShape<160, 192, 160, 24>{});
  if (grid_is(d, 160, 192, 160, 32)) return f(GridShape<160, 192, 160, 32>{});
  return f(GridDyn{d.N[0], d.N[1], d.N[2], d.K[1], d.Kh});
}

hipError_t launch_twiddles(float2* dst, int K, int G, int mode, hipStream_t st) {
  int Kq = (mode == 1 || mode == 3) ? K / 2 : K;
  int total = (mode <= 1) ? 2 * G * Kq : Kq * G;
  hipLaunchKernelGGL(k_twiddles, dim3(nblk(total, 256)), dim3(256), 0, st, dst, K, G, mode);
  return hipGetLastError();
}

hipError_t launch_symbols(float* Lsym, float* Ksym, const Dims& d, hipStream_t st) {
  hipLaunchKernelGGL(k_symbols, dim3(nblk(d.nb, 256)), dim3(256), 0, st, Lsym, Ksym, d.K[0], d.K[1],
                     d.Kh, d.s, d.alpha);
  return hipGetLastError();
}

hipError_t launch_full_to_half(const float2* full, float2* half, const Dims& d, hipStream_t st) {
  hipLaunchKernelGGL(k_full_to_half, dim3(nblk(3LL * d.nb, 256)), dim3(256), 0, st, full, half,
                     d.K[0], d.K[1], d.K[2]);
  return hipGetLastError();
}

hipError_t launch_half_to_full(const float2* a, const float2* b, float cb, float2* full,
                               const Dims& d, hipStream_t st, const float* sym) {
  long long n = 3LL * d.K[0] * d.K[1] * d.K[2];
  hipLaunchKernelGGL(k_half_to_full, dim3(nblk(n, 256)), dim3(256), 0, st, a, b, cb, sym, full, d.K[0],
                     d.K[1], d.K[2]);
  return hipGetLastError();
}

hipError_t launch_inv0(const Inv0Jobs& jobs, int njobs, int nvar, const float2* tw, const float* Lsym,
                       int K0, int C, int G0, int Kh, bool image_grid, hipStream_t st) {
  const int fam = image_grid ? KF_INV0_GRID : KF_INV0;
  const int T = 128;
  {
    double fl = 0, by = 0;
    for (int i = 0; i < njobs; ++i) {
      fl += 8.0 * nvar * G0 * K0 * (double)C;
      by += 8.0 * K0 * (double)C * (1 + nvar * (double)G0 / K0) + (jobs.j[i].lflag ? 4.0 * K0 * C : 0.0);
    }
    timer_work(fam, fl, by);
  }
  auto go = [&](auto nv_tag, auto xt_tag, auto kc_tag) {
    constexpr int NV = decltype(nv_tag)::value, XT = decltype(xt_tag)::value, KC = decltype(kc_tag)::value;
    dim3 grid(nblk(C, T), nblk(G0, XT), njobs);
    size_t shm = NV * XT * K0 * sizeof(float2);
    LAUNCH_TIMED(fam, (k_inv0<NV, XT, KC>), grid, dim3(T), shm, st, jobs, tw, Lsym, K0, C, G0, Kh);
  };
  using I2 = std::integral_constant<int, 2>;
  using I1 = std::integral_constant<int, 1>;
  using X2 = std::integral_constant<int, 2>;
  using X4 = std::integral_constant<int, 4>;
  if (nvar == 2) {
    if (K0 == 32) go(I2{}, X2{}, std::integral_constant<int, 32>{});
    else if (K0 == 16) go(I2{}, X2{}, std::integral_constant<int, 16>{});
    else go(I2{}, X2{}, std::integral_constant<int, 0>{});
  } else {
    if (K0 == 32) go(I1{}, X4{}, std::integral_constant<int, 32>{});
    else if (K0 == 16) go(I1{}, X4{}, std::integral_constant<int, 16>{});
    else go(I1{}, X4{}, std::integral_constant<int, 0>{});
  }
  return hipGetLastError();
}

static inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

void synth_padding(const Dims& d, int* M1p, int* M2p, int* Khp) {
  *M1p = round_up(d.M[1], 16);
  *M2p = round_up(d.M[2], 16);
  *Khp = round_up(d.Kh, 8);
}

size_t synth_table_floats(const Dims& d) {
  int M1p, M2p, Khp;
  synth_padding(d, &M1p, &M2p, &Khp);
  return 2 * (size_t)M1p * 2 * d.K[1] + 2 * 2 * (size_t)Khp * M2p;
}

size_t synth_shared_bytes(const Dims& d) {
  int M1p, M2p, Khp;
  synth_padding(d, &M1p, &M2p, &Khp);
  const int K2r = 2 * d.K[1], N1 = 2 * Khp;
  const int ldbT = K2r + 2, ldw2 = (M2p % 32 == 0) ? M2p + 16 : M2p;
  return (2 * 16 * (size_t)(K2r + 2) + 2 * (size_t)N1 * (ldbT > ldw2 ? ldbT : ldw2) + 3 * 16 * (size_t)(N1 + 2)) *
         sizeof(float);
}

hipError_t launch_synth_tables(const Twiddles& tw, float* tables, const Dims& d, hipStream_t st) {
  int M1p, M2p, Khp;
  synth_padding(d, &M1p, &M2p, &Khp);
  const size_t n = synth_table_floats(d);
  float* w1a = tables;
  float* w2b = tables + 2 * (size_t)M1p * 2 * d.K[1];
  hipLaunchKernelGGL(k_synth_tables, dim3(nblk((long long)n, 256)), dim3(256), 0, st, tw.inv1, tw.inv2, w1a,
                     w2b, d.M[1], d.M[2], d.K[1], d.Kh, M1p, M2p, Khp);
  return hipGetLastError();
}

hipError_t launch_synth(const float2* t1g0, const float2* t1g1, float* dst0, float* dst1,
                        const float* tables, const Dims& d, hipStream_t st) {
  int M1p, M2p, Khp;
  synth_padding(d, &M1p, &M2p, &Khp);
  SynthArgs a{};
  a.t1[0] = t1g0;
  a.t1[1] = t1g1;
  a.dst[0] = dst0;
  a.dst[1] = dst1;
  a.w1a = tables;
  a.w2b = tables + 2 * (size_t)M1p * 2 * d.K[1];
  const double nM = (double)d.nM;
  const int nf = t1g1 ? 6 : 3;  // new fields (group, component)
  timer_work(KF_SYNTH, nf * (3.0 * d.M[0] * d.M[1] * d.Kh * d.K[1] * 8.0 + 4.0 * nM * d.Kh * 4.0),
             nf * (2.0 * d.M[0] * d.K[1] * d.Kh * 8.0 + 4.0 * nM * 4.0));
  (void)Khp;
  (void)M2p;
  hipError_t e = with_band(d, [&](auto sh) {
    do {
      if (d.prec)
        LAUNCH_TIMED(KF_SYNTH, (k_synth<decltype(sh), true>), dim3(d.M[0], nf, M1p / 16), dim3(256), synth_shared_bytes(d), st,
                   a, sh);
      else
        LAUNCH_TIMED(KF_SYNTH, (k_synth<decltype(sh), false>), dim3(d.M[0], nf, M1p / 16), dim3(256), synth_shared_bytes(d), st,
                   a, sh);
    } while (0);
    return hipGetLastError();
  });
  return e;
}

int prod_rows_max(const Dims& d) {
  int R = 256 / d.M[2];
  if (R < 1) R = 1;
  if (R > d.M[1]) R = d.M[1];
  return R;
}

static int prod_rows(const Dims& d) {
  const int R = prod_rows_max(d);
  return (d.tile_prod_rows > 0 && d.tile_prod_rows < R) ? d.tile_prod_rows : R;
}

size_t prods_shared_bytes(const Dims& d, int nout) {
  return (size_t)d.M[2] * d.Kh * sizeof(float2) + (size_t)nout * prod_rows(d) * (d.M[2] + 2) * sizeof(float);
}

hipError_t launch_prods(const ProdArgs& a, const Dims& d, const Twiddles& tw, hipStream_t st) {
  const int R = prod_rows(d);
  dim3 grid(nblk(d.M[1], R), d.M[0]);
  size_t shm = prods_shared_bytes(d, a.nout);
  {
    static const double prog_flops[11] = {0, 47, 94, 136, 272, 136, 18, 36, 18, 36, 89};
    static const int prog_fields[11] = {0, 24, 48, 48, 96, 48, 12, 24, 12, 24, 36};
    const double nM = (double)d.nM;
    double fl = prog_flops[a.prog] * nM + a.nout * nM * d.Kh * 4.0;
    double by = prog_fields[a.prog] * nM * 4.0 + a.nout * (double)d.M[0] * d.M[1] * d.Kh * 8.0;
    timer_work(KF_PRODS, fl, by);
  }
  int threads = ((R * d.M[2] + 63) / 64) * 64;
  if (threads > 256) threads = 256;
  hipError_t e = with_band(d, [&](auto sh) {
    do {
      if (d.prec)
        LAUNCH_TIMED(KF_PRODS, (k_prods<decltype(sh), true>), grid, dim3(threads), shm, st, a, tw, sh, R);
      else
        LAUNCH_TIMED(KF_PRODS, (k_prods<decltype(sh), false>), grid, dim3(threads), shm, st, a, tw, sh, R);
    } while (0);
    return hipGetLastError();
  });
  return e;
}

constexpr int kColGroup = 8;

// LDS plan of the generic column kernel: region X holds one S1 slice and,
// when the total stays within the LDS of a workgroup, the inverse twiddles
// of phase 3.
static void colstep_lds_plan(const Dims& d, int* xsz, int* stage_w0, size_t* bytes) {
  const int M0 = d.M[0], M1 = d.M[1], K0 = d.K[0];
  const size_t rest = (size_t)kColGroup * M1 + 2 * (size_t)M0 * kColGroup + (size_t)K0 * M0 +
                      2 * (size_t)K0 * kColGroup;
  const size_t staged = (size_t)std::max(M0 * M1, 2 * M0 * K0);
  const bool st = (staged + rest) * sizeof(float2) <= kMaxLds;
  *xsz = st ? (int)staged : M0 * M1;
  *stage_w0 = st ? 1 : 0;
  *bytes = ((size_t)*xsz + rest) * sizeof(float2);
}

size_t colstep_shared_bytes(const Dims& d) {
  int xsz, sw;
  size_t b;
  colstep_lds_plan(d, &xsz, &sw, &b);
  return b;
}

size_t col_table_count(const Dims& d) {
  const int M = d.M[0], K = d.K[0];
  const int Mp = round_up(M, 16), Kp = round_up(K, 16);
  return (size_t)M * Kp + (size_t)Kp * M + 2 * (size_t)Mp * K;
}

hipError_t launch_col_tables(const Twiddles& tw, float2* tab, const Dims& d, hipStream_t st) {
  const int M = d.M[0], K = d.K[0];
  const int Mp = round_up(M, 16), Kp = round_up(K, 16);
  // the MFMA column kernel runs for shapes with K0 = K1 and M0 = M1 only
  if (d.M[1] != M || d.K[1] != K) return hipSuccess;
  float2* w1t = tab;
  float2* w0f = w1t + (size_t)M * Kp;
  float2* w0i = w0f + (size_t)Kp * M;
  hipLaunchKernelGGL(k_col_tables, dim3(nblk((long long)col_table_count(d), 256)), dim3(256), 0, st, tw.fwd1,
                     tw.fwd0, tw.inv0, w1t, w0f, w0i, M, K, Mp, Kp);
  return hipGetLastError();
}

static bool colstep_mfma_shape(const Dims& d) {
  return band_iso(d, 32, 48) || band_iso(d, 16, 24) || band_iso(d, 24, 36);
}

bool colstep_fuses_grid0(const Dims& d) {
  if (!colstep_mfma_shape(d)) return true;  // the generic kernel reads the table from global memory
  const int K = d.K[0], M = d.M[0], Mp = round_up(M, 16);
  return d.N[0] % 16 == 0 && d.N[0] * K <= 256 * kGrid0Pre && d.N[0] * (K + 2) <= 2 * Mp * (M + 2);
}

hipError_t launch_colstep(const ColJobs& jobs, int njobs, const Dims& d, const Twiddles& tw,
                          const float2* coltab, const float* Lsym, const float* Ksym, hipStream_t st) {
  for (int i = 0; i < njobs; ++i) {
    if (jobs.j[i].t1n && (!colstep_fuses_grid0(d) || jobs.N0 != d.N[0] || !jobs.w0n)) return hipErrorInvalidValue;
    // the tuned kernel loads pairs of complex values
    if (colstep_mfma_shape(d) && (((uintptr_t)jobs.j[i].a | (uintptr_t)jobs.j[i].b | (uintptr_t)coltab |
                                   (uintptr_t)jobs.w0n) & 15))
      return hipErrorInvalidValue;
  }
  {
    const double M0 = d.M[0], M1 = d.M[1], K0 = d.K[0], K1 = d.K[1], Kh = d.Kh;
    double fl = 0, by = 0;
    for (int i = 0; i < njobs; ++i) {
      const ColJob& j = jobs.j[i];
      int terms = 1 + (j.b != nullptr);
      const double N0 = j.t1n ? d.N[0] : 0.0;
      fl += terms * (M0 * M1 * K1 + K0 * K1 * M0) * Kh * 8.0 + j.nt1 * 2.0 * M0 * K0 * K1 * Kh * 8.0 +
            N0 * K0 * K1 * Kh * 8.0;
      by += terms * M0 * M1 * Kh * 8.0 + K0 * K1 * Kh * 8.0 * (1 + (j.base != nullptr) + (j.extra != nullptr)) +
            j.nt1 * 2.0 * M0 * K1 * Kh * 8.0 + N0 * K1 * Kh * 8.0;
    }
    timer_work(KF_COLUMN, fl, by);
  }
  const float invG = (float)(1.0 / ((double)d.M[0] * d.M[1] * d.M[2]));
  const int M = d.M[0], K = d.K[0];
  const float2* w1t = coltab;
  const float2* w0f = w1t + (size_t)M * round_up(K, 16);
  const float2* w0i = w0f + (size_t)round_up(K, 16) * M;
  hipError_t e;
  // split the next-stage tiles over two blocks per column tile when the
  // launch would otherwise fill fewer than half of the compute units and
  // every job has at least 8 such tiles
  const int ktiles = round_up(d.K[0], 16) / 16;
  int min_tiles = 1 << 30;
  for (int i = 0; i < njobs; ++i) {
    const ColJob& j = jobs.j[i];
    const int t = j.nt1 * 2 * (round_up(d.M[0], 16) / 16) + (j.t1n ? d.N[0] / 16 : 0);
    min_tiles = t < min_tiles ? t : min_tiles;
  }
  // (or as the tile table says: tile_col 1 / 2 / 3 = one part, two parts, two
  // parts with the lean kernel where it applies)
  const int nparts = d.tile_col == 1 ? 1
                     : d.tile_col >= 2 ? 2
                                       : ((d.Kh * njobs * ktiles <= 128 && min_tiles >= 8) ? 2 : 1);
  const dim3 cgrid(d.Kh, njobs, ktiles * nparts);
  // the forward sweeps' launches (one product field per job, image-grid stage
  // 0 fused, two parts) take the lean kernel
  bool lean = nparts == 2 && d.tile_col != 2 && (band_iso(d, 32, 48) || band_iso(d, 24, 36));
  for (int i = 0; i < njobs && lean; ++i) lean = jobs.j[i].b == nullptr && jobs.j[i].t1n != nullptr;
  if (lean) {
    if (band_iso(d, 32, 48))
      do {
        if (d.prec)
          LAUNCH_TIMED(KF_COLUMN, (k_colstep_lean<BandIso<32, 48>, true>), cgrid, dim3(256), 0, st, jobs, w1t, w0f, w0i,
                     d.alpha, d.s, invG);
        else
          LAUNCH_TIMED(KF_COLUMN, (k_colstep_lean<BandIso<32, 48>, false>), cgrid, dim3(256), 0, st, jobs, w1t, w0f, w0i,
                     d.alpha, d.s, invG);
      } while (0);
    else
      do {
        if (d.prec)
          LAUNCH_TIMED(KF_COLUMN, (k_colstep_lean<BandIso<24, 36>, true>), cgrid, dim3(256), 0, st, jobs, w1t, w0f, w0i,
                     d.alpha, d.s, invG);
        else
          LAUNCH_TIMED(KF_COLUMN, (k_colstep_lean<BandIso<24, 36>, false>), cgrid, dim3(256), 0, st, jobs, w1t, w0f, w0i,
                     d.alpha, d.s, invG);
      } while (0);
    return hipGetLastError();
  }
  if (band_iso(d, 32, 48)) {
    do {
      if (d.prec)
        LAUNCH_TIMED(KF_COLUMN, (k_colstep_mfma<BandIso<32, 48>, true>), cgrid, dim3(256), 0, st, jobs, w1t, w0f, w0i, d.alpha,
                   d.s, invG, nparts);
      else
        LAUNCH_TIMED(KF_COLUMN, (k_colstep_mfma<BandIso<32, 48>, false>), cgrid, dim3(256), 0, st, jobs, w1t, w0f, w0i, d.alpha,
                   d.s, invG, nparts);
    } while (0);
    e = hipGetLastError();
  } else if (band_iso(d, 16, 24)) {
    do {
      if (d.prec)
        LAUNCH_TIMED(KF_COLUMN, (k_colstep_mfma<BandIso<16, 24>, true>), cgrid, dim3(256), 0, st, jobs, w1t, w0f, w0i, d.alpha,
                   d.s, invG, nparts);
      else
        LAUNCH_TIMED(KF_COLUMN, (k_colstep_mfma<BandIso<16, 24>, false>), cgrid, dim3(256), 0, st, jobs, w1t, w0f, w0i, d.alpha,
                   d.s, invG, nparts);
    } while (0);
    e = hipGetLastError();
  } else if (band_iso(d, 24, 36)) {
    do {
      if (d.prec)
        LAUNCH_TIMED(KF_COLUMN, (k_colstep_mfma<BandIso<24, 36>, true>), cgrid, dim3(256), 0, st, jobs, w1t, w0f, w0i, d.alpha,
                   d.s, invG, nparts);
      else
        LAUNCH_TIMED(KF_COLUMN, (k_colstep_mfma<BandIso<24, 36>, false>), cgrid, dim3(256), 0, st, jobs, w1t, w0f, w0i, d.alpha,
                   d.s, invG, nparts);
    } while (0);
    e = hipGetLastError();
  } else {
    dim3 grid(nblk(d.K[1], kColGroup), d.Kh, njobs);
    int xsz, stage_w0;
    size_t shm;
    colstep_lds_plan(d, &xsz, &stage_w0, &shm);
    BandDyn sh{d.K[0], d.K[1], d.Kh, d.M[0], d.M[1], d.M[2]};
    LAUNCH_TIMED(KF_COLUMN, (k_colstep<kColGroup, BandDyn>), grid, dim3(256), shm, st, jobs, tw, Lsym, Ksym, sh, invG,
                 xsz, stage_w0);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_fwd1(const Fwd1Jobs& jobs, int njobs, const float2* tw, int G0, int G1, int K1,
                       int Kh, hipStream_t st) {
  constexpr int QT = 2;
  const int T = 128;
  dim3 grid(nblk((long long)G0 * Kh, T), nblk(K1, QT), njobs);
  size_t shm = QT * G1 * sizeof(float2);
  timer_work(KF_FWD1_GRID, njobs * 8.0 * G0 * Kh * (double)K1 * G1,
             njobs * 8.0 * ((double)G0 * G1 * Kh + (double)G0 * K1 * Kh));
  LAUNCH_TIMED(KF_FWD1_GRID, (k_fwd1<QT>), grid, dim3(T), shm, st, jobs, tw, G0, G1, K1, Kh);
  return hipGetLastError();
}

hipError_t launch_fwd0(const Fwd0Jobs& jobs, int njobs, const float2* tw, const float* Ksym, int G0,
                       int K0, int K1, int Kh, float invG, hipStream_t st) {
  constexpr int QT = 2;
  const int T = 128;
  dim3 grid(nblk((long long)K1 * Kh, T), nblk(K0, QT), njobs);
  size_t shm = QT * G0 * sizeof(float2);
  {
    const double C = (double)K1 * Kh;
    double fl = 0, by = 0;
    for (int i = 0; i < njobs; ++i) {
      const Fwd0Job& j = jobs.j[i];
      int terms = 1 + (j.b != nullptr);
      fl += terms * 8.0 * K0 * C * G0;
      by += terms * 8.0 * G0 * C +
            8.0 * K0 * C * (1 + (j.base != nullptr) + (j.extra != nullptr) + (j.out2 != nullptr)) + 4.0 * K0 * C;
    }
    timer_work(KF_FWD0_GRID, fl, by);
  }
  LAUNCH_TIMED(KF_FWD0_GRID, (k_fwd0<QT>), grid, dim3(T), shm, st, jobs, tw, Ksym, G0, K0, K1, Kh, invG);
  return hipGetLastError();
}

size_t gridstep_shared_bytes(const Dims& d) {
  const int C = d.K[1] * d.Kh;
  return (3 * (size_t)C + 3 * (size_t)kGridRows * d.Kh + (size_t)kGridRows * d.K[1] +
          (size_t)d.N[2] * d.Kh) * sizeof(float2);
}

size_t src_shared_bytes(const Dims& d) {
  return (size_t)((3 * kGridRows * d.N[2] + 3) & ~3) * sizeof(float) +
         (size_t)d.Kh * d.N[2] * sizeof(float2);
}

hipError_t launch_gridstep(const GridStepArgs& a, const Dims& d, const Twiddles& tw, hipStream_t st) {
  const int C = d.K[1] * d.Kh;
  dim3 grid(nblk(d.N[1], kGridRows), d.N[0]);
  size_t shm = gridstep_shared_bytes(d);
  {
    const double nN = (double)d.nN;
    double fl = 3.0 * d.N[0] * d.N[1] * d.Kh * d.K[1] * 8.0 + 3.0 * nN * d.Kh * 4.0 + (a.op ? 15.0 * nN : 0.0);
    double by = 3.0 * d.N[0] * (double)C * 8.0 + (a.op ? (a.dm ? 12.0 : 8.0) * nN : 12.0 * nN);
    timer_work(KF_GRID, fl, by);
  }
  hipError_t e;
  // the compile-time grid shapes take the matrix-core kernel
  bool done = false;
  e = with_grid(d, [&](auto gs) -> hipError_t {
    using G = decltype(gs);
    if constexpr (G::kStatic) {
      static_assert(G::N1() % kGridRows == 0 && G::N2() % 16 == 0 && G::K1() % 4 == 0, "matrix-core grid shape");
      done = true;
      if (d.prec)
        LAUNCH_TIMED(KF_GRID, (k_gridstep_mfma<G, true>), grid, dim3(256), 0, st, a, tw);
      else
        LAUNCH_TIMED(KF_GRID, (k_gridstep_mfma<G, false>), grid, dim3(256), 0, st, a, tw);
      return hipGetLastError();
    }
    return hipSuccess;
  });
  if (!done) {
    const int jn = (d.N[2] + 15) / 16;
    GridDyn gs{d.N[0], d.N[1], d.N[2], d.K[1], d.Kh};
    if (jn <= 2)
      LAUNCH_TIMED(KF_GRID, (k_gridstep<2, GridDyn>), grid, dim3(256), shm, st, a, tw, gs);
    else if (jn <= 4)
      LAUNCH_TIMED(KF_GRID, (k_gridstep<4, GridDyn>), grid, dim3(256), shm, st, a, tw, gs);
    else if (jn <= 8)
      LAUNCH_TIMED(KF_GRID, (k_gridstep<8, GridDyn>), grid, dim3(256), shm, st, a, tw, gs);
    else
      LAUNCH_TIMED(KF_GRID, (k_gridstep<16, GridDyn>), grid, dim3(256), shm, st, a, tw, gs);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_sl(const float* src, const float* vel, float* dst, float dt, const Dims& d,
                     hipStream_t st) {
  timer_work(KF_SL, 40.0 * (double)d.nN, 20.0 * (double)d.nN);
  const int T = (d.tile_sl == 64 || d.tile_sl == 128) ? d.tile_sl : 256;
  hipError_t e = with_grid(d, [&](auto gs) {
    LAUNCH_TIMED(KF_SL, (k_sl<decltype(gs)>), dim3(nblk(d.nN, T)), dim3(T), 0, st, src, vel, dst, dt, gs);
    return hipGetLastError();
  });
  return e;
}

hipError_t launch_sl_rk2(const float* src, const float* vel, float* dst, float dt, const Dims& d,
                         hipStream_t st) {
  timer_work(KF_SL, 140.0 * (double)d.nN, 20.0 * (double)d.nN);
  return with_grid(d, [&](auto gs) {
    LAUNCH_TIMED(KF_SL, (k_sl_rk2<decltype(gs)>), dim3(nblk(d.nN, 256)), dim3(256), 0, st, src, vel, dst, dt, gs);
    return hipGetLastError();
  });
}

hipError_t launch_src_fwd2(const float* a, const float* b, const float* r, const float* m, float coef,
                           float2* s1, const Dims& d, const Twiddles& tw, hipStream_t st) {
  dim3 grid(nblk(d.N[1], kGridRows), d.N[0]);
  size_t shm = src_shared_bytes(d);
  {
    // gradient of m (6 flops / point / axis), the source, forward stage 2 of 3 fields
    const double nN = (double)d.nN;
    timer_work(KF_SRC, 3.0 * nN * d.Kh * 4.0 + (r ? 43.0 : 25.0) * nN,
               (b ? 12.0 : 8.0) * nN + (r ? 4.0 : 0.0) * nN + 3.0 * d.N[0] * (double)d.N[1] * d.Kh * 8.0);
  }
  hipError_t e = with_grid(d, [&](auto gs) {
    LAUNCH_TIMED(KF_SRC, (k_src_fwd2<decltype(gs)>), grid, dim3(256), shm, st, a, b, r, m, coef, s1, tw, gs);
    return hipGetLastError();
  });
  return e;
}

hipError_t launch_sl_tangent(const float* dm, const float* m, const float* vel, const float* dvel, float* out,
                             float dt, const Dims& d, hipStream_t st) {
  timer_work(KF_SL, 90.0 * (double)d.nN, ((dm ? 8.0 : 4.0) + 12.0 + 12.0 + 4.0) * (double)d.nN);
  return with_grid(d, [&](auto gs) {
    LAUNCH_TIMED(KF_SL, (k_sl_tangent<decltype(gs)>), dim3(nblk(d.nN, 256)), dim3(256), 0, st, dm, m, vel, dvel,
                 out, dt, gs);
    return hipGetLastError();
  });
}

hipError_t launch_adj_src_fwd2(const float* lam, const float* m, const float* vel, float* lam_out, float coef,
                               float dt, float2* s1, const Dims& d, const Twiddles& tw, hipStream_t st) {
  dim3 grid(nblk(d.N[1], kGridRows), d.N[0]);
  size_t shm = src_shared_bytes(d);
  {
    // departure point, 8 gathers, slopes, 8 scattered weights, forward stage 2 of 3 fields
    const double nN = (double)d.nN;
    timer_work(KF_SRC, 3.0 * nN * d.Kh * 4.0 + 80.0 * nN,
               (4.0 + 12.0 + 4.0 + 8.0 * 4.0) * nN + 3.0 * d.N[0] * (double)d.N[1] * d.Kh * 8.0);
  }
  hipError_t e = with_grid(d, [&](auto gs) {
    LAUNCH_TIMED(KF_SRC, (k_adj_src_fwd2<decltype(gs)>), grid, dim3(256), shm, st, lam, m, vel, lam_out, coef, dt,
                 s1, tw, gs);
    return hipGetLastError();
  });
  return e;
}

hipError_t launch_image_derivs(const float* I0, float* G, float* H, const Dims& d, hipStream_t st) {
  return with_grid(d, [&](auto gs) {
    hipLaunchKernelGGL((k_image_derivs<decltype(gs)>), dim3(nblk(d.nN, 256)), dim3(256), 0, st, I0, G, H, gs);
    return hipGetLastError();
  });
}

hipError_t launch_rho_fwd2(const RhoArgs& a, float2* s1, const Dims& d, const Twiddles& tw, hipStream_t st) {
  dim3 grid(nblk(d.N[1], kGridRows), d.N[0]);
  size_t shm = src_shared_bytes(d);
  {
    // trilinear interpolation of 4 (op 0), 3 or 9 (op 1) fields, the source,
    // forward stage 2 of 3 fields; point reads u (3) and I1 | du (3), res
    const double nN = (double)d.nN;
    const bool full = a.op == 1 && a.res;
    const double nf = a.op == 0 ? 4.0 : (full ? 9.0 : 3.0);
    const double rd = a.op == 0 ? 4.0 : (full ? 7.0 : 6.0);
    timer_work(KF_SRC, 3.0 * nN * d.Kh * 4.0 + (nf * 14.0 + (full ? 30.0 : 12.0)) * nN,
               (nf + rd) * 4.0 * nN + 3.0 * d.N[0] * (double)d.N[1] * d.Kh * 8.0);
  }
  hipError_t e = with_grid(d, [&](auto gs) {
    LAUNCH_TIMED(KF_SRC, (k_rho_fwd2<decltype(gs)>), grid, dim3(256), shm, st, a, s1, tw, gs);
    return hipGetLastError();
  });
  return e;
}

bool tail_fused(const Dims& d) {
  return (band_iso(d, 32, 48) && grid_iso(d, 128, 32)) || (band_iso(d, 16, 24) && grid_iso(d, 64, 16));
}

size_t tail_parts_bytes(const Dims& d) {
  const int np = d.N[1] > kTailRows ? d.N[1] / kTailRows : 1;
  return (size_t)np * 3 * d.N[0] * d.K[1] * d.Kh * sizeof(float2);
}

hipError_t launch_tail(const float* a, const float* b, const float* r, const float* m, float coef, float2* P,
                       float2* out, float2* const t1u[3], float2* const t1z[3], const Dims& d,
                       const Twiddles& twN, const float2* coltab, const float* Lsym, const float* Ksym,
                       hipStream_t st) {
  if (!tail_fused(d)) return hipErrorInvalidValue;
  const int K = d.K[0], M = d.M[0], N = d.N[0], Kh = d.Kh;
  const int np = N > kTailRows ? N / kTailRows : 1;
  const double nN = (double)d.nN, C = (double)K * Kh;
  if ((((uintptr_t)a | (uintptr_t)m | (uintptr_t)(b ? b : a) | (uintptr_t)(r ? r : a) | (uintptr_t)P |
        (uintptr_t)twN.fwd1 |
        (uintptr_t)twN.fwd2 | (uintptr_t)twN.fwd0 | (uintptr_t)coltab) & 15))
    return hipErrorInvalidValue;
  timer_work(KF_SRC, (r ? 43.0 : 25.0) * nN + 3.0 * nN * Kh * 4.0 + 3.0 * N * (double)N * K * Kh * 8.0,
             (b ? 12.0 : 8.0) * nN + (r ? 4.0 : 0.0) * nN + np * 3.0 * N * C * 8.0);
  hipError_t e;
  const dim3 g1(N > kTailRows ? N / kTailRows : 1, N);
  if (N == 128 && r)
    do {
      if (d.prec)
        LAUNCH_TIMED(KF_SRC, (k_srcfwd<GridIso<128, 32>, true, true>), g1, dim3(256), 0, st, a, b, r, m, coef, P, twN);
      else
        LAUNCH_TIMED(KF_SRC, (k_srcfwd<GridIso<128, 32>, true, false>), g1, dim3(256), 0, st, a, b, r, m, coef, P, twN);
    } while (0);
  else if (N == 128)
    do {
      if (d.prec)
        LAUNCH_TIMED(KF_SRC, (k_srcfwd<GridIso<128, 32>, false, true>), g1, dim3(256), 0, st, a, b, r, m, coef, P, twN);
      else
        LAUNCH_TIMED(KF_SRC, (k_srcfwd<GridIso<128, 32>, false, false>), g1, dim3(256), 0, st, a, b, r, m, coef, P, twN);
    } while (0);
  else if (r)
    do {
      if (d.prec)
        LAUNCH_TIMED(KF_SRC, (k_srcfwd<GridIso<64, 16>, true, true>), g1, dim3(256), 0, st, a, b, r, m, coef, P, twN);
      else
        LAUNCH_TIMED(KF_SRC, (k_srcfwd<GridIso<64, 16>, true, false>), g1, dim3(256), 0, st, a, b, r, m, coef, P, twN);
    } while (0);
  else
    do {
      if (d.prec)
        LAUNCH_TIMED(KF_SRC, (k_srcfwd<GridIso<64, 16>, false, true>), g1, dim3(256), 0, st, a, b, r, m, coef, P, twN);
      else
        LAUNCH_TIMED(KF_SRC, (k_srcfwd<GridIso<64, 16>, false, false>), g1, dim3(256), 0, st, a, b, r, m, coef, P, twN);
    } while (0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  TailJobs tj{};
  tj.P = P;
  tj.out = out;
  for (int c = 0; c < 3; ++c) {
    tj.t1u[c] = t1u[c];
    tj.t1z[c] = t1z[c];
  }
  tj.ca = 1.f;
  const float2* w0i = coltab + (size_t)M * round_up(K, 16) + (size_t)round_up(K, 16) * M;
  const float invG = (float)(1.0 / d.nN);
  timer_work(KF_FWD0_GRID, 3.0 * K * C * N * np * 8.0 + 3.0 * 2.0 * M * K * C * 8.0,
             np * 3.0 * N * C * 8.0 + 3.0 * K * C * 8.0 + 3.0 * 2.0 * 2.0 * M * C * 8.0);
  const dim3 grid(Kh, 3, round_up(K, 16) / 16);
  if (N == 128)
    do {
      if (d.prec)
        LAUNCH_TIMED(KF_FWD0_GRID, (k_fwd0_mfma<BandIso<32, 48>, 128, 2, true>), grid, dim3(256), 0, st, tj, twN.fwd0, w0i,
                   d.alpha, d.s, invG);
      else
        LAUNCH_TIMED(KF_FWD0_GRID, (k_fwd0_mfma<BandIso<32, 48>, 128, 2, false>), grid, dim3(256), 0, st, tj, twN.fwd0, w0i,
                   d.alpha, d.s, invG);
    } while (0);
  else
    do {
      if (d.prec)
        LAUNCH_TIMED(KF_FWD0_GRID, (k_fwd0_mfma<BandIso<16, 24>, 64, 1, true>), grid, dim3(256), 0, st, tj, twN.fwd0, w0i,
                   d.alpha, d.s, invG);
      else
        LAUNCH_TIMED(KF_FWD0_GRID, (k_fwd0_mfma<BandIso<16, 24>, 64, 1, false>), grid, dim3(256), 0, st, tj, twN.fwd0, w0i,
                   d.alpha, d.s, invG);
    } while (0);
  return hipGetLastError();
}

hipError_t launch_fill(float* p, long long n, float v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill, dim3(nblk(n, 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_diff(const float* a, const float* b, float* out, long long n, hipStream_t st) {
  hipLaunchKernelGGL(k_diff, dim3(nblk(n, 256)), dim3(256), 0, st, a, b, out, n);
  return hipGetLastError();
}

hipError_t launch_copy(const float* s, float* dd, long long n, hipStream_t st) {
  hipLaunchKernelGGL(k_copy, dim3(nblk(n, 256)), dim3(256), 0, st, s, dd, n);
  return hipGetLastError();
}

// Two-dimensional problems as three-dimensional ones independent of the
// first coordinate: images repeated over `depth` planes, band fields placed
// in components 1.. at first-axis frequency slot 0 (component 0 and the other
// slots zero), and the inverse of the band placement.
__global__ void k_embed_image(const float* __restrict__ in, float* __restrict__ out, long long plane, int depth) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= plane * depth) return;
  out[i] = in[i % plane];
}

__global__ void k_embed_band(const float2* __restrict__ in, float2* __restrict__ out, int kd, long long plane2) {
  // out [3][kd][plane2], in [2][plane2]
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * kd * plane2) return;
  const long long c = i / (kd * plane2), slot = (i / plane2) % kd, r = i % plane2;
  out[i] = (c > 0 && slot == 0) ? in[(c - 1) * plane2 + r] : make_float2(0.f, 0.f);
}

__global__ void k_extract_band(const float2* __restrict__ in, float2* __restrict__ out, int kd, long long plane2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * plane2) return;
  const long long c = i / plane2, r = i % plane2;
  out[i] = in[((c + 1) * kd) * plane2 + r];
}

// Number of positions where a and b differ bit for bit (NaN never equals).
__global__ void k_count_ne(const float* __restrict__ a, const float* __restrict__ b, long long n, unsigned* out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && __float_as_uint(a[i]) != __float_as_uint(b[i])) atomicAdd(out, 1u);
}

hipError_t launch_count_ne(const float* a, const float* b, long long n, unsigned* out, hipStream_t st) {
  hipLaunchKernelGGL(k_count_ne, dim3(nblk(n, 256)), dim3(256), 0, st, a, b, n, out);
  return hipGetLastError();
}

hipError_t launch_embed_image(const float* in, float* out, long long plane, int depth, hipStream_t st) {
  hipLaunchKernelGGL(k_embed_image, dim3(nblk(plane * depth, 256)), dim3(256), 0, st, in, out, plane, depth);
  return hipGetLastError();
}

hipError_t launch_embed_band(const float2* in, float2* out, int kd, long long plane2, hipStream_t st) {
  hipLaunchKernelGGL(k_embed_band, dim3(nblk(3 * kd * plane2, 256)), dim3(256), 0, st, in, out, kd, plane2);
  return hipGetLastError();
}

hipError_t launch_extract_band(const float2* in, float2* out, int kd, long long plane2, hipStream_t st) {
  hipLaunchKernelGGL(k_extract_band, dim3(nblk(2 * plane2, 256)), dim3(256), 0, st, in, out, kd, plane2);
  return hipGetLastError();
}

hipError_t launch_axpy_band(const float2* x, const float2* y, float a, float2* out, int n,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_axpy_band, dim3(nblk(n, 256)), dim3(256), 0, st, x, y, a, out, n);
  return hipGetLastError();
}

hipError_t launch_sqdiff(const float* a, const float* b, long long n, double* partial, double* out,
                         double scale, hipStream_t st) {
  hipLaunchKernelGGL(k_sqdiff, dim3(kRedBlocks), dim3(kRedThreads), 0, st, a, b, n, partial);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedThreads), 0, st, partial, kRedBlocks, out, scale, 0);
  return hipGetLastError();
}

hipError_t launch_band_dot(const float2* a, const float2* b, const float* Lsym, const Dims& d,
                           double* partial, double* out, double scale, hipStream_t st, unsigned* count,
                           double* pcg, int post, double* host) {
  if (post && (!count || !pcg)) return hipErrorInvalidValue;
  const int blocks = 64;
  if (count) {
    hipLaunchKernelGGL(k_band_dot_once, dim3(blocks), dim3(kRedThreads), 0, st, a, b, Lsym, d.nb, d.Kh, partial,
                       count, out, scale, pcg, post, host);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_band_dot, dim3(blocks), dim3(kRedThreads), 0, st, a, b, Lsym, d.nb, d.Kh,
                     partial);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedThreads), 0, st, partial, blocks, out, scale, 0);
  return hipGetLastError();
}

hipError_t launch_band_maxabs(const float2* a, const Dims& d, double* partial, double* out,
                              hipStream_t st) {
  const int blocks = 64;
  hipLaunchKernelGGL(k_band_maxabs, dim3(blocks), dim3(kRedThreads), 0, st, a, 3 * d.nb, partial);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedThreads), 0, st, partial, blocks, out, 1.0, 1);
  return hipGetLastError();
}

hipError_t launch_scalar_copy(const double* src, double* dst, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_scalar_copy, dim3(1), dim3(64), 0, st, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_energy_combine(double* sc, hipStream_t st) {
  hipLaunchKernelGGL(k_energy_combine, dim3(1), dim3(64), 0, st, sc);
  return hipGetLastError();
}
hipError_t launch_pcg_reset(double* sc, hipStream_t st) {
  hipLaunchKernelGGL(k_pcg_reset, dim3(1), dim3(64), 0, st, sc);
  return hipGetLastError();
}

hipError_t launch_pcg_init(const float2* g, float2* p, float2* r, float2* dv, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_pcg_init, dim3(nblk(n, 256)), dim3(256), 0, st, g, p, r, dv, n);
  return hipGetLastError();
}
hipError_t launch_pcg_update_pr(const double* sc, const float2* dv, const float2* Hd, float2* p,
                                float2* r, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_pcg_update_pr, dim3(nblk(n, 256)), dim3(256), 0, st, sc, dv, Hd, p, r, n);
  return hipGetLastError();
}
// host[1 .. na] = a, host[1 + na .. na + nb] = b, then host[0] = 1, visible
// system-wide (host: pinned host memory)
__global__ void k_host_copy(const double* a, int na, const double* b, int nb, double* host) {
  const int i = threadIdx.x;
  if (i < na) host[1 + i] = a[i];
  if (i < nb) host[1 + na + i] = b[i];
  __threadfence_system();
  __syncthreads();
  if (i == 0) __hip_atomic_store(host, 1.0, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

hipError_t launch_host_copy(const double* a, int na, const double* b, int nb, double* host, hipStream_t st) {
  if (na < 0 || nb < 0 || na + nb > 63) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_host_copy, dim3(1), dim3(64), 0, st, a, na, b, nb, host);
  return hipGetLastError();
}

hipError_t launch_pcg_update_d(const double* sc, const float2* r, float2* dv, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_pcg_update_d, dim3(nblk(n, 256)), dim3(256), 0, st, sc, r, dv, n);
  return hipGetLastError();
}

}  // namespace lddmm
