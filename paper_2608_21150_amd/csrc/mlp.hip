// Learned stand-in for the vn diffusion step: an 18 -> 64 -> 64 -> 1
// perceptron with GELU, BF16 operands on the matrix cores (FP32
// accumulation) and FP32 master weights.  Training (forward, backward) uses
// v_mfma_f32_16x16x16_bf16 and the erf form of GELU; inference uses
// v_mfma_f32_16x16x32_bf16 in the transposed orientation described at
// forward_t and a polynomial GELU within 4.6e-5 of the erf form.
// The paper motivates coupling the dynamical core to machine-learning
// workflows (Sections 3 and 6); the features, the network, its training and
// the per-column fallback to the plain diffusion are readings of this
// library, not the paper's design.
//
// Wave-level layout of the 16x16x16 instruction (lane l, i = l % 16,
// q = l / 16): A fragment = row i, columns 4q..4q+3; B fragment = column i,
// rows 4q..4q+3; result = rows 4q..4q+3 of column i.  A wave owns 64
// samples (4 row tiles); features (padded to 32) and hidden activations are
// staged in LDS as BF16 (round to nearest even) and the weights transposed,
// so that every fragment is one 8-byte LDS read.  In the backward pass the
// forward results are already in the fragment layout that the weight
// gradients (samples as the contraction axis) need.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "bodies.h"
#include "internal.h"
#include "kernels.h"
#include "state.h"

using namespace dc;
using namespace dc::bodies;

namespace {

constexpr int NIN = 18, NH = 64, XK = 32;
constexpr int OFF_W1 = 0, OFF_B1 = NIN * NH, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH, OFF_W3 = OFF_B2 + NH,
              OFF_B3 = OFF_W3 + NH, NPAR = OFF_B3 + 1;
static_assert(NPAR == DC_MLP_NPARAMS, "parameter count");
constexpr int XS = 40, HS = 72;  // LDS row strides (bf16 elements)
constexpr int NFLOW = 16;        // features 0..15 change sign with the flow

struct Norm {
  float mean[NIN], istd[NIN], fmin[NIN], fmax[NIN];
  float tstd;
};

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned short bf16;

// FP32 -> BF16, round to nearest even (gfx950 converts natively)
__device__ __forceinline__ bf16 to_bf16(float x) { return __builtin_bit_cast(bf16, (__bf16)x); }

// erf for x >= 0 by Abramowitz & Stegun 7.1.26 (absolute error <= 1.5e-7,
// far below the BF16 resolution of the network's activations), branch-free;
// e = exp(-x^2) is passed in so that GELU and its derivative share it.
__device__ __forceinline__ float erf_pos(float ax, float e) {
  const float t = __builtin_amdgcn_rcpf(1.0f + 0.3275911f * ax);
  const float poly = t * (0.254829592f + t * (-0.284496736f + t * (1.421413741f + t * (-1.453152027f + t * 1.061405429f))));
  return 1.0f - poly * e;
}
// Phi(x) = (1 + erf(x / sqrt 2)) / 2 and phi(x) = exp(-x^2 / 2) / sqrt(2 pi)
__device__ __forceinline__ void normal_cdf_pdf(float x, float& cdf, float& pdf) {
  const float u = x * 0.70710678118654752f;
  const float e = __expf(-u * u);
  const float er = erf_pos(fabsf(u), e);
  cdf = 0.5f * (1.0f + copysignf(er, u));
  pdf = e * 0.39894228040143268f;
}
// exact-erf GELU x Phi(x) and its derivative Phi(x) + x phi(x)
__device__ __forceinline__ void gelu_and_grad(float x, float& g, float& gd) {
  float c, d;
  normal_cdf_pdf(x, c, d);
  g = x * c;
  gd = c + x * d;
}
__device__ __forceinline__ s4 frag(const bf16* m, int ld, int r0, int k0) {
  const int l = threadIdx.x & 63;
  return *reinterpret_cast<const s4*>(m + (r0 + (l & 15)) * ld + k0 + 4 * (l >> 4));
}
__device__ __forceinline__ f4 mfma(s4 a, s4 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0); }
__device__ __forceinline__ s4 pack(f4 v) {
  s4 r;
  r[0] = (short)to_bf16(v[0]);
  r[1] = (short)to_bf16(v[1]);
  r[2] = (short)to_bf16(v[2]);
  r[3] = (short)to_bf16(v[3]);
  return r;
}
// Orders a wave's LDS writes before its later LDS reads of other lanes'
// entries: LDS executes one wave's instructions in issue order, and the
// wave barrier keeps the compiler from moving them across.  For LDS rows
// that only this wave uses.
__device__ __forceinline__ void wave_lds_sync() { __builtin_amdgcn_wave_barrier(); }

__device__ __forceinline__ float sum16(float v) {
  v += __shfl_xor(v, 1, 16);
  v += __shfl_xor(v, 2, 16);
  v += __shfl_xor(v, 4, 16);
  v += __shfl_xor(v, 8, 16);
  return v;
}
__device__ __forceinline__ float sumq(float v) {
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}

// Block-shared weights in BF16: W1t[h][f] (f padded to 32), W2t[o][i].
struct SW {
  alignas(16) bf16 w1t[NH * XS];
  alignas(16) bf16 w2t[NH * HS];
  float b1[NH], b2[NH], w3[NH];
  float b3;
};

__device__ void stage_weights(SW& s, const float* __restrict__ p, bf16* w2n) {
  for (int x = threadIdx.x; x < NH * XK; x += blockDim.x) {
    const int h = x / XK, f = x % XK;
    s.w1t[h * XS + f] = f < NIN ? to_bf16(p[OFF_W1 + f * NH + h]) : (bf16)0;
  }
  for (int x = threadIdx.x; x < NH * NH; x += blockDim.x) {
    const int i = x / NH, o = x % NH;
    const bf16 v = to_bf16(p[OFF_W2 + i * NH + o]);
    s.w2t[o * HS + i] = v;
    if (w2n) w2n[i * HS + o] = v;
  }
  for (int x = threadIdx.x; x < NH; x += blockDim.x) {
    s.b1[x] = p[OFF_B1 + x];
    s.b2[x] = p[OFF_B2 + x];
    s.w3[x] = p[OFF_W3 + x];
  }
  if (threadIdx.x == 0) s.b3 = p[OFF_B3];
}

// ---------------------------------------------------------------------------
// Inference forward (no gradients) in the transposed orientation: hidden
// units are the rows and samples the columns of every product, so that a
// layer-1 result tile is already the B operand of layer 2 and activations
// never pass through LDS.  v_mfma_f32_16x16x32_bf16: lane l = 16 q + j holds
// row j of A and column j of B, eight k slots each, and receives rows
// 4q..4q+3 of column j.  Any map of (q, slot) to k serves when A and B share
// it: layer 1 takes feature 8q + slot; layer 2's k step m takes hidden units
// 32m + 4q + slot (slot < 4) and 32m + 16 + 4q + slot - 4 (slot >= 4), which
// are exactly the outputs of layer-1 tiles 2m and 2m+1 in the same lane.  The
// weight fragments, biases (the accumulators' initial values) and w3 stay in
// registers for the whole kernel.
// ---------------------------------------------------------------------------
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f4 mfma32(bf8 a, bf8 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }

// GELU(x) = x Phi(x) with Phi(x) = 1/2 + x Q(x^2): Q is a degree-8 polynomial
// in s = min(x^2, T^2) (T = 4.25) and Phi is clamped to [0, 1]; largest
// deviation from the erf form 4.6e-5 (at |x| = T; 1.7e-5 for |x| < 3.5),
// below the BF16 resolution of the activations.  The coefficients are
// printed by gelu_fit.py beside this package's sources.
constexpr float kGeluT2 = 18.0625f;
constexpr float kGeluQ[9] = {3.988192976e-01f, -6.619048119e-02f, 9.718909860e-03f, -1.079113572e-03f,
                             8.849387086e-05f, -5.147835964e-06f, 1.986260969e-07f, -4.515380070e-09f,
                             4.546895846e-11f};
__device__ __forceinline__ float gelu_poly(float x) {
  const float s = fminf(x * x, kGeluT2);
  float a = kGeluQ[8];
#pragma unroll
  for (int i = 7; i >= 0; --i) a = fmaf(a, s, kGeluQ[i]);
  return x * __builtin_amdgcn_fmed3f(fmaf(x, a, 0.5f), 0.0f, 1.0f);
}

__device__ __forceinline__ int l2_unit(int m, int q, int slot) { return 32 * m + 4 * q + (slot < 4 ? slot : 12 + slot); }

struct RegNet {
  bf8 w1[4];               // hidden tile nt: W1[8q + slot][16 nt + j]
  bf8 w2[4][2];            // output tile nt, k step m: W2[l2_unit(m, q, slot)][16 nt + j]
  f4 b1[4], b2[4], w3[4];  // unit 16 nt + 4 q + t
  float b3;
};

__device__ void load_net(RegNet& n, const float* __restrict__ p) {
  const int l = threadIdx.x & 63, j = l & 15, q = l >> 4;
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
#pragma unroll
    for (int sl = 0; sl < 8; ++sl) {
      const int f = 8 * q + sl;
      n.w1[nt][sl] = (__bf16)(f < NIN ? p[OFF_W1 + f * NH + 16 * nt + j] : 0.0f);
#pragma unroll
      for (int m = 0; m < 2; ++m) n.w2[nt][m][sl] = (__bf16)p[OFF_W2 + l2_unit(m, q, sl) * NH + 16 * nt + j];
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int u = 16 * nt + 4 * q + t;
      n.b1[nt][t] = p[OFF_B1 + u];
      n.b2[nt][t] = p[OFF_B2 + u];
      n.w3[nt][t] = p[OFF_W3 + u];
    }
  }
  n.b3 = p[OFF_B3];
}

// Output (normalised) of the wave's 64 samples: xs row r (stride XS) holds
// sample r's normalised BF16 features in columns 0..31 (zero beyond NIN);
// lane l returns sample l's output.  Reads only the wave's own LDS rows.
__device__ float forward_t(const RegNet& n, const bf16* xs) {
  const int l = threadIdx.x & 63, j = l & 15, q = l >> 4;
  float y = 0.f;
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const bf8 xb = *reinterpret_cast<const bf8*>(xs + (16 * st + j) * XS + 8 * q);
    f4 a1[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) a1[nt] = mfma32(n.w1[nt], xb, n.b1[nt]);
    bf8 hb[2];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        hb[m][t] = (__bf16)gelu_poly(a1[2 * m][t]);
        hb[m][4 + t] = (__bf16)gelu_poly(a1[2 * m + 1][t]);
      }
    float yp = 0.f;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      f4 a2 = mfma32(n.w2[nt][0], hb[0], n.b2[nt]);
      a2 = mfma32(n.w2[nt][1], hb[1], a2);
#pragma unroll
      for (int t = 0; t < 4; ++t) yp = fmaf(gelu_poly(a2[t]), n.w3[nt][t], yp);
    }
    yp = sumq(yp);
    if (q == st) y = yp;
  }
  return y + n.b3;
}

// Writes lane l's normalised BF16 feature row (columns 0..31) into xs row l.
__device__ __forceinline__ void put_row(bf16* xs, const float* v) {
  const int l = threadIdx.x & 63;
  bf8 r[4];
#pragma unroll
  for (int c = 0; c < 32; ++c) r[c >> 3][c & 7] = (__bf16)(c < NIN ? v[c] : 0.0f);
  bf8* d = reinterpret_cast<bf8*>(xs + l * XS);
#pragma unroll
  for (int c = 0; c < 4; ++c) d[c] = r[c];
}

// The 18 raw features of edge e at level k, from vn (edges; vt formed here
// with the step's tangential-wind stencil), D = div vn (cells), DL = div L1
// (cells), CL = curl L1 (vertices) and the vertex quantities V (vertex
// vector and Z = curl vn, laid out as VertexQ says); the fields are those of
// the plain diffusion.  Stencil values enter as centred pairs, the mean of
// the two points and their difference over their distance, formed in the
// path's precision before the network's BF16 rounding: vn_e, vt_e; D at c0,
// c1; Z at the end vertices v0, v1; div L1 at c0, c1; curl L1 at v0, v1; the
// four rhombus derivatives; Z at the two opposite rhombus vertices;
// l_e / mean l, d_e / mean d.
struct FeatIn {
  const void *vn, *D, *DL, *CL, *V;
};
template <typename R>
__device__ __forceinline__ void features(const DevGrid& g, const FeatIn& in, int e, int k, double lbar, double dbar,
                                         float f[NIN]) {
  const R* dr = static_cast<const R*>(in.D) + (size_t)k * g.cs;
  const R* dlr = static_cast<const R*>(in.DL) + (size_t)k * g.cs;
  const R* clr = static_cast<const R*>(in.CL) + (size_t)k * g.vs;
  Edge1Geo<R> q;
  q.load_rhombus(g, e);
  VVec<R> qv[4];
  q.gather(g, static_cast<const R*>(in.V), k, qv);
  const int c0 = g.e2c[e], c1 = g.e2c[g.es + e];
  const int v0 = q.rv[0], v1 = q.rv[1];
  const R invd = (R)g.invd[e], invl = q.invl, invlr = q.invlr;
  const R half = R(0.5);
  const R* vnr = static_cast<const R*>(in.vn) + (size_t)k * g.es;
  VtStencil<R> vs;
  vs.load(g, e);
  f[0] = (float)vnr[e];
  f[1] = (float)vs.apply(vnr, e);
  f[2] = (float)(half * (dr[c0] + dr[c1]));
  f[3] = (float)((dr[c1] - dr[c0]) * invd);
  f[4] = (float)(half * (qv[0].zeta + qv[1].zeta));
  f[5] = (float)((qv[1].zeta - qv[0].zeta) * invl);
  f[6] = (float)(half * (dlr[c0] + dlr[c1]));
  f[7] = (float)((dlr[c1] - dlr[c0]) * invd);
  f[8] = (float)(half * (clr[v0] + clr[v1]));
  f[9] = (float)((clr[v1] - clr[v0]) * invl);
  R d[4];
  q.rhombus(qv, d);
#pragma unroll
  for (int i = 0; i < 4; ++i) f[10 + i] = (float)d[i];
  f[14] = (float)(half * (qv[2].zeta + qv[3].zeta));
  f[15] = (float)((qv[3].zeta - qv[2].zeta) * invlr);
  f[16] = (float)(1.0 / (g.invl[e] * lbar));
  f[17] = (float)(1.0 / (g.invd[e] * dbar));
}

// ---------------------------------------------------------------------------
// inference: features -> normalised BF16 -> MLP -> T (denormalised).  Every
// wave works alone on tiles of 64 consecutive edges of one level, taken in
// level-major order with a stride of the grid's wave count.  A column with any
// feature outside the training range gets flag_range[e] = 1 (plain stores
// of one value: order independent).
// ---------------------------------------------------------------------------
constexpr int kInferWaves = 4;
constexpr int kInferBlocks = 2048;  // persistent: each wave loads the weights once
template <typename R>
__global__ void __launch_bounds__(64 * kInferWaves) k_infer(DevGrid g, FeatIn fin, const float* __restrict__ par,
                                                            const Norm* __restrict__ nrm, double lbar, double dbar,
                                                            R* __restrict__ tout, int* __restrict__ flag_range) {
  __shared__ alignas(16) bf16 xs_all[kInferWaves][64 * XS];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  bf16* xs = xs_all[w];
  RegNet n;
  load_net(n, par);
  const int ntx = (g.ne + 63) / 64;
  const int total = ntx * g.K;
  const int nwave = gridDim.x * kInferWaves;
  for (int tile = blockIdx.x * kInferWaves + w; tile < total; tile += nwave) {
    const int k = tile / ntx, e = (tile % ntx) * 64 + l;
    float f[NIN];
    if (e < g.ne) {
      features<R>(g, fin, e, k, lbar, dbar, f);
      bool out = false;
#pragma unroll
      for (int i = 0; i < NIN; ++i) out |= !(f[i] >= nrm->fmin[i] && f[i] <= nrm->fmax[i]);
      if (out) flag_range[e] = 1;
#pragma unroll
      for (int i = 0; i < NIN; ++i) f[i] = (f[i] - nrm->mean[i]) * nrm->istd[i];
    } else {
#pragma unroll
      for (int i = 0; i < NIN; ++i) f[i] = 0.0f;
    }
    put_row(xs, f);
    wave_lds_sync();
    const float y = forward_t(n, xs);
    if (e < g.ne) tout[(size_t)k * g.es + e] = (R)(y * nrm->tstd);
    wave_lds_sync();
  }
}

// Adds the wave's count of lanes with pred set to *c (one atomic per wave;
// integer sums are order independent).  Every lane of the wave must call it.
__device__ __forceinline__ void wave_count(bool pred, int* c) {
  const unsigned long long b = __ballot(pred);
  if ((threadIdx.x & 63) == 0 && b) atomicAdd(c, (int)__popcll(b));
}
__device__ __forceinline__ void wave_count64(bool pred, unsigned long long* c) {
  const unsigned long long b = __ballot(pred);
  if ((threadIdx.x & 63) == 0 && b) atomicAdd(c, (unsigned long long)__popcll(b));
}

// apply: vn += dt T_mlp, or on flagged columns the plain update from the
// fields of the plain diffusion's front (the expressions of its last
// kernel).  cnt[1] counts range flags, cnt[2] fallback columns of this step;
// the 64-bit counter at cnt + 4 sums the fallback columns since the network
// was set.
template <typename R>
__global__ void __launch_bounds__(256) k_apply(DevGrid g, R* __restrict__ vn, const R* __restrict__ tmlp,
                                               const R* __restrict__ l1, const R* __restrict__ nu,
                                               const R* __restrict__ dl1, const R* __restrict__ cl1,
                                               const int* __restrict__ fj, const int* __restrict__ fr,
                                               int* __restrict__ cnt, StepCoef cf) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = e < g.ne;
  const bool rf = in && fr[e] != 0;
  const bool fb = in && (rf || fj[e] != 0);
  wave_count(rf, &cnt[1]);
  wave_count(fb, &cnt[2]);
  wave_count64(fb, reinterpret_cast<unsigned long long*>(cnt + 4));
  if (!in) return;
  const R dt = (R)cf.dt;
  if (fb) {
    const int c0 = g.e2c[e], c1 = g.e2c[g.es + e];
    const int v0 = g.e2v[e], v1 = g.e2v[g.es + e];
    const double ae = g.ae[e];
    const R k4a2 = (R)(cf.k4 * ae * ae);
    const R invd = (R)g.invd[e], invl = (R)g.invl[e];
    for (int k = 0; k < g.K; ++k) {
      const R* dr = dl1 + (size_t)k * g.cs;
      const R* zr = cl1 + (size_t)k * g.vs;
      const R l2 = dif_l2<R>(invd, invl, dr[c0], dr[c1], zr[v0], zr[v1]);
      const size_t r = (size_t)k * g.es + e;
      vn[r] = dif_update<R>(vn[r], dt, nu[r], l1[r], k4a2, l2);
    }
  } else {
    for (int k = 0; k < g.K; ++k) {
      const size_t r = (size_t)k * g.es + e;
      vn[r] = vn[r] + dt * tmlp[r];
    }
  }
}

// judge: residual of the surrogate against the plain tendency per column,
// r_e = dt |T_mlp - T_plain|_2 / max(|vn|_2, sqrt(K) m/s); cnt[0] counts flags
template <typename R>
__global__ void __launch_bounds__(256) k_judge(DevGrid g, const R* __restrict__ vn_new, const R* __restrict__ vn_old,
                                               const R* __restrict__ tmlp, double dt, double thr,
                                               int* __restrict__ fj, int* __restrict__ cnt) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = e < g.ne;
  double num = 0.0, den = 0.0;
  for (int k = 0; in && k < g.K; ++k) {
    const size_t r = (size_t)k * g.es + e;
    const double tp = ((double)vn_new[r] - (double)vn_old[r]) / dt;
    const double d = (double)tmlp[r] - tp;
    num += d * d;
    den += (double)vn_old[r] * (double)vn_old[r];
  }
  const double res = dt * sqrt(num) / fmax(sqrt(den), sqrt((double)g.K));
  const int f = (in && (res > thr || !(res == res))) ? 1 : 0;
  wave_count(f != 0, &cnt[0]);
  if (in) fj[e] = f;
}

__global__ void k_fill_int(int* __restrict__ p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

template <typename T>
__global__ void k_copy(const T* __restrict__ a, T* __restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) b[i] = a[i];
}

// ---------------------------------------------------------------------------
// sampler: a counter-based Feistel permutation of [0, n) (sampling without
// replacement): four rounds of a 32-bit integer mixer on the two halves of
// an even-width index, cycle-walking back into [0, n)
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ unsigned mix32(unsigned x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}
__host__ __device__ __forceinline__ unsigned long long feistel(unsigned long long x, unsigned long long n,
                                                               unsigned long long key) {
  int bits = 2;
  while ((1ull << bits) < n) bits += 2;
  const int hb = bits / 2;
  const unsigned long long mask = (1ull << hb) - 1;
  do {
    unsigned long long L = x >> hb, Rr = x & mask;
    for (int r = 0; r < 4; ++r) {
      const unsigned kr = mix32((unsigned)(key >> (32 * (r & 1))) + 0x9e3779b9u * (unsigned)(r + 1));
      const unsigned f = mix32((unsigned)Rr ^ kr);
      const unsigned long long nl = Rr;
      Rr = (L ^ f) & mask;
      L = nl;
    }
    x = (L << hb) | Rr;
  } while (x >= n);
  return x;
}

// features of the sampled points (pre-diffusion fields); idx_out keeps the
// flat internal index k * ne + e of every sample
template <typename R>
__global__ void __launch_bounds__(256) k_sample_feat(DevGrid g, FeatIn fin, double lbar,
                                                     double dbar, unsigned long long key, long long nsamp,
                                                     float* __restrict__ buf, long long stride, long long offset,
                                                     long long* __restrict__ idx_out) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= nsamp) return;
  const unsigned long long N = (unsigned long long)g.K * g.ne;
  const unsigned long long idx = feistel((unsigned long long)i, N, key);
  const int k = (int)(idx / g.ne), e = (int)(idx % g.ne);
  float f[NIN];
  features<R>(g, fin, e, k, lbar, dbar, f);
  for (int x = 0; x < NIN; ++x) buf[x * stride + offset + i] = f[x];
  if (idx_out) idx_out[i] = (long long)idx;
}

// target of the sampled points: (vn after the diffusion - vn before) / dt
template <typename R>
__global__ void __launch_bounds__(256) k_sample_target(DevGrid g, const R* __restrict__ vn_old,
                                                       const R* __restrict__ vn_new, double dt, unsigned long long key,
                                                       long long nsamp, float* __restrict__ buf, long long stride,
                                                       long long offset) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= nsamp) return;
  const unsigned long long idx = feistel((unsigned long long)i, (unsigned long long)g.K * g.ne, key);
  const int k = (int)(idx / g.ne), e = (int)(idx % g.ne);
  const size_t r = (size_t)k * g.es + e;
  buf[NIN * stride + offset + i] = (float)(((double)vn_new[r] - (double)vn_old[r]) / dt);
}

// ---------------------------------------------------------------------------
// statistics of a training set (19 rows: 18 features + target): per block
// and row, sum and sum of squares (double), min and max
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_stats(const float* __restrict__ buf, long long stride, long long n,
                                               double* __restrict__ part) {
  __shared__ double sh[256];
  const int row = blockIdx.y;
  double s = 0.0, s2 = 0.0, mn = 1e300, mx = -1e300;
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += 256ll * gridDim.x) {
    const double v = buf[row * stride + i];
    s += v;
    s2 += v * v;
    mn = fmin(mn, v);
    mx = fmax(mx, v);
  }
  const double vals[4] = {s, s2, mn, mx};
  for (int m = 0; m < 4; ++m) {
    sh[threadIdx.x] = vals[m];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) {
        const double a = sh[threadIdx.x], b = sh[threadIdx.x + w];
        sh[threadIdx.x] = m < 2 ? a + b : (m == 2 ? fmin(a, b) : fmax(a, b));
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) part[((size_t)row * gridDim.x + blockIdx.x) * 4 + m] = sh[0];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// training: forward and backward of 128 samples per block (64 per wave);
// every wave writes its partial gradients (NPAR) and its partial sum of
// squared residuals (one more slot) to part[wave].  Sample p of the epoch
// is row feistel(p) of the set (identity with key 0); augment flips the
// sign of the flow features and the target of a hashed half of the rows.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(128) k_train(const float* __restrict__ par, const Norm* __restrict__ nrm,
                                               const float* __restrict__ buf, long long stride, long long n,
                                               unsigned long long key, long long base, int batch, int augment,
                                               float* __restrict__ part) {
  __shared__ SW s;
  __shared__ alignas(16) bf16 w2n[NH * HS];
  __shared__ alignas(16) bf16 xs_all[2][64 * XS];
  __shared__ alignas(16) bf16 hs_all[2][16 * HS];
  __shared__ alignas(16) bf16 ds_all[2][16 * HS];
  __shared__ float tsh[2][64];
  stage_weights(s, par, w2n);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, j = l & 15, q = l >> 4;
  bf16* xs = xs_all[w];
  bf16* hs = hs_all[w];
  bf16* ds = ds_all[w];
  const long long pos = base + blockIdx.x * 128ll + w * 64 + l;
  const unsigned long long idx =
      key ? feistel((unsigned long long)(pos % n), (unsigned long long)n, key) : (unsigned long long)(pos % n);
  const float sgn = (augment && (mix32((unsigned)idx ^ mix32((unsigned)key)) & 1u)) ? -1.f : 1.f;
#pragma unroll
  for (int i = 0; i < XK; ++i) {
    float v = 0.f;
    if (i < NIN) {
      v = buf[i * stride + idx];
      if (i < NFLOW) v *= sgn;
      v = (v - nrm->mean[i]) * nrm->istd[i];
    }
    xs[l * XS + i] = to_bf16(v);
  }
  tsh[w][l] = sgn * buf[NIN * stride + idx] / nrm->tstd;
  __syncthreads();
  f4 dw2[4][4], dw1[2][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) dw2[a][b] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) dw1[a][b] = f4{0.f, 0.f, 0.f, 0.f};
  float db1[4] = {0.f, 0.f, 0.f, 0.f}, db2[4] = {0.f, 0.f, 0.f, 0.f}, dw3[4] = {0.f, 0.f, 0.f, 0.f};
  float db3 = 0.f, loss = 0.f;
  const float scale = 2.0f / (float)batch;
  // forward and backward of one 16-row tile at a time; the gradients of the
  // weights accumulate over the tiles
  for (int st = 0; st < 4; ++st) {
    // layer 1: keep gelu'(z1) and the BF16 h1 fragments
    f4 gd1[4];
    s4 h1f[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) acc = mfma(frag(xs, XS, 16 * st, 16 * ks), frag(s.w1t, XS, 16 * nt, 16 * ks), acc);
      f4 h;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        float hv, gv;
        gelu_and_grad(acc[t] + s.b1[16 * nt + j], hv, gv);
        h[t] = hv;
        gd1[nt][t] = gv;
      }
      h1f[nt] = pack(h);
#pragma unroll
      for (int t = 0; t < 4; ++t) hs[(4 * q + t) * HS + 16 * nt + j] = (bf16)h1f[nt][t];
    }
    __syncthreads();
    // layers 2 and 3, residual, dz2; dW2 += h1^T dz2
    f4 h2v[4], g2v[4];
    float yp[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) acc = mfma(frag(hs, HS, 0, 16 * ks), frag(s.w2t, HS, 16 * nt, 16 * ks), acc);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        float hv, gv;
        gelu_and_grad(acc[t] + s.b2[16 * nt + j], hv, gv);
        h2v[nt][t] = hv;
        g2v[nt][t] = gv;
        yp[t] += hv * s.w3[16 * nt + j];
      }
    }
    float dy[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const float r = sum16(yp[t]) + s.b3 - tsh[w][16 * st + 4 * q + t];
      dy[t] = scale * r;
      if (j == 0) {
        loss += r * r;
        db3 += dy[t];
      }
    }
    s4 dzf[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      f4 dz;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        dw3[nt] += h2v[nt][t] * dy[t];
        dz[t] = dy[t] * s.w3[16 * nt + j] * g2v[nt][t];
        db2[nt] += dz[t];
      }
      dzf[nt] = pack(dz);
#pragma unroll
      for (int t = 0; t < 4; ++t) ds[(4 * q + t) * HS + 16 * nt + j] = (bf16)dzf[nt][t];
    }
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
      for (int nj = 0; nj < 4; ++nj) dw2[mi][nj] = mfma(h1f[mi], dzf[nj], dw2[mi][nj]);
    __syncthreads();
    // dh1 = dz2 W2^T, dz1 = dh1 gelu'(z1); dW1 += x^T dz1
    s4 xt[2];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi) {
      s4 a;
#pragma unroll
      for (int t = 0; t < 4; ++t) a[t] = (short)xs[(16 * st + 4 * q + t) * XS + 16 * mi + j];
      xt[mi] = a;
    }
#pragma unroll
    for (int nj = 0; nj < 4; ++nj) {
      f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) acc = mfma(frag(ds, HS, 0, 16 * ks), frag(w2n, HS, 16 * nj, 16 * ks), acc);
      f4 dz;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        dz[t] = acc[t] * gd1[nj][t];
        db1[nj] += dz[t];
      }
      const s4 dzp = pack(dz);
#pragma unroll
      for (int mi = 0; mi < 2; ++mi) dw1[mi][nj] = mfma(xt[mi], dzp, dw1[mi][nj]);
    }
    __syncthreads();
  }
  // sums over the four row groups, then the partial writes
  float* out = part + (size_t)(blockIdx.x * 2 + w) * (NPAR + 1);
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const float a = sumq(db1[nt]), b = sumq(db2[nt]), c = sumq(dw3[nt]);
    if (q == 0) {
      out[OFF_B1 + 16 * nt + j] = a;
      out[OFF_B2 + 16 * nt + j] = b;
      out[OFF_W3 + 16 * nt + j] = c;
    }
  }
  db3 = sumq(db3);
  loss = sumq(loss);
  if (l == 0) {
    out[OFF_B3] = db3;
    out[NPAR] = loss;
  }
#pragma unroll
  for (int mi = 0; mi < 4; ++mi)
#pragma unroll
    for (int nj = 0; nj < 4; ++nj)
#pragma unroll
      for (int t = 0; t < 4; ++t) out[OFF_W2 + (16 * mi + 4 * q + t) * NH + 16 * nj + j] = dw2[mi][nj][t];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int nj = 0; nj < 4; ++nj)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int f = 16 * mi + 4 * q + t;
        if (f < NIN) out[OFF_W1 + f * NH + 16 * nj + j] = dw1[mi][nj][t];
      }
}

// Sum of the wave partials (fixed order), optional Adam update (0.9, 0.999,
// 1e-8, bias-corrected), mean loss of the batch.
__global__ void __launch_bounds__(256) k_adam(const float* __restrict__ part, int nw, float* __restrict__ par,
                                              float* __restrict__ m, float* __restrict__ v, float* __restrict__ grad,
                                              int step, float lr, int update, float* __restrict__ loss_out,
                                              int batch) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p <= NPAR; p += gridDim.x * blockDim.x) {
    float gs = 0.f;
    for (int w = 0; w < nw; ++w) gs += part[(size_t)w * (NPAR + 1) + p];
    if (p == NPAR) {
      if (loss_out) *loss_out = gs / (float)batch;
      continue;
    }
    if (grad) grad[p] = gs;
    if (update) {
      const float mm = b1 * m[p] + (1.0f - b1) * gs;
      const float vv = b2 * v[p] + (1.0f - b2) * gs * gs;
      m[p] = mm;
      v[p] = vv;
      par[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    }
  }
}

// forward of raw feature rows [n][18] (tests and evaluation): y = T, by the
// inference path (one wave per 64 rows)
__global__ void __launch_bounds__(64 * kInferWaves) k_forward_rows(const float* __restrict__ par,
                                                                   const Norm* __restrict__ nrm,
                                                                   const float* __restrict__ x, long long n,
                                                                   float* __restrict__ y) {
  __shared__ alignas(16) bf16 xs_all[kInferWaves][64 * XS];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  bf16* xs = xs_all[w];
  RegNet net;
  load_net(net, par);
  const long long r = (blockIdx.x * (long long)kInferWaves + w) * 64 + l;
  float v[NIN];
#pragma unroll
  for (int i = 0; i < NIN; ++i) v[i] = r < n ? (x[r * NIN + i] - nrm->mean[i]) * nrm->istd[i] : 0.0f;
  put_row(xs, v);
  wave_lds_sync();
  const float yy = forward_t(net, xs);
  if (r < n) y[r] = yy * nrm->tstd;
}

}  // namespace

// ===========================================================================
// host side
// ===========================================================================
struct dc_mlp {
  int device = -1;
  float* par = nullptr;  // NPAR master weights
  float* m = nullptr;
  float* v = nullptr;
  Norm* nrm = nullptr;
  Norm hnrm{};
  long long adam_step = 0;
  std::vector<float> loss_trace;
};

namespace dc {

struct SurCtx {
  const dc_mlp* mlp = nullptr;
  double thr = 1e-3;
  int judge_every = 10;
  long long steps = 0, judge_steps = 0;
};

}  // namespace dc

namespace {

#define ML_TRY(expr)                                                \
  do {                                                              \
    hipError_t _e = (expr);                                         \
    if (_e != hipSuccess) {                                         \
      set_error(std::string(#expr) + ": " + hipGetErrorString(_e)); \
      return DC_EHIP;                                               \
    }                                                               \
  } while (0)

dc_status mfail(dc_status c, const std::string& msg) {
  set_error(msg);
  return c;
}

// mean primal and dual edge length of the grid (feature scales)
void mean_lengths(const HostGrid& h, double* lbar, double* dbar) {
  double sl = 0, sd = 0;
  for (int e = 0; e < h.ne; ++e) {
    sl += h.l[e];
    sd += h.d[e];
  }
  *lbar = sl / h.ne;
  *dbar = sd / h.ne;
}

// The plain diffusion's front on the current vn (w diffused into the state's
// w with the fresh viscosity; curl L1 into its own buffer so that the
// vorticity survives); the features read its fields.
template <typename R>
FeatIn front_and_features(dc_state* s, const StepCoef& c, hipStream_t st) {
  const DevGrid& g = s->d;
  const dc_fields& cur = s->buf[s->cur];
  R* vn = static_cast<R*>(cur.vn);
  launch_diffusion_front<R>(g, vn, s->wtmp, static_cast<double*>(cur.w), static_cast<R*>(s->vt),
                            static_cast<R*>(s->tvn0), static_cast<R*>(s->kc), static_cast<R*>(s->d2),
                            static_cast<R*>(s->zeta), static_cast<R*>(s->sur_cl), static_cast<R*>(s->vv), c, s->tiles,
                            st, nullptr);
  return FeatIn{vn, s->kc, s->d2, s->sur_cl, s->vv};
}

}  // namespace

namespace dc {

// One diffusion step of a surrogate-mode state on its current buffer set.
// The plain diffusion's front runs every step (ν, L1, div and curl of L1 and
// the w diffusion); every judge_every-th step (the first included) then
// runs its last kernel and flags the columns whose surrogate residual
// exceeds the threshold; the other steps apply the surrogate tendency except
// on flagged columns and on columns with out-of-range features, which take
// the plain update.
template <typename R>
void surrogate_diffusion(dc_state* s, const StepCoef& c) {
  SurCtx& sc = *s->sur;
  hipStream_t st = s->stream;
  const DevGrid& g = s->d;
  R* vn = static_cast<R*>(s->buf[s->cur].vn);
  R* tm = static_cast<R*>(s->sur_tmlp);
  const bool judge = sc.steps % sc.judge_every == 0;
  ++sc.steps;
  const FeatIn fin = front_and_features<R>(s, c, st);
  k_fill_int<<<(g.ne + 255) / 256, 256, 0, st>>>(s->sur_fr, g.ne, 0);
  const int tiles = ((g.ne + 63) / 64) * g.K;
  const int blocks = std::min((tiles + kInferWaves - 1) / kInferWaves, kInferBlocks);
  k_infer<R><<<blocks, 64 * kInferWaves, 0, st>>>(g, fin, sc.mlp->par, sc.mlp->nrm, s->sur_lbar, s->sur_dbar, tm,
                                                  s->sur_fr);
  const R* l1 = static_cast<const R*>(s->vt);
  const R* nu = static_cast<const R*>(s->tvn0);
  const R* dl1 = static_cast<const R*>(s->d2);
  const R* cl1 = static_cast<const R*>(s->sur_cl);
  if (judge) {
    ++sc.judge_steps;
    R* old = static_cast<R*>(s->vns);  // substep workspace, idle during the diffusion
    k_copy<R><<<1024, 256, 0, st>>>(vn, old, (size_t)g.K * g.es);
    launch_diffusion_back<R>(g, vn, l1, nu, dl1, cl1, c, s->tiles, st, nullptr);
    k_fill_int<<<1, 64, 0, st>>>(s->sur_cnt, 1, 0);
    k_judge<R><<<(g.ne + 255) / 256, 256, 0, st>>>(g, vn, old, tm, c.dt, sc.thr, s->sur_fj, s->sur_cnt);
  } else {
    k_fill_int<<<1, 64, 0, st>>>(s->sur_cnt + 1, 2, 0);
    k_apply<R><<<(g.ne + 255) / 256, 256, 0, st>>>(g, vn, tm, l1, nu, dl1, cl1, s->sur_fj, s->sur_fr, s->sur_cnt, c);
  }
}

template void surrogate_diffusion<double>(dc_state*, const StepCoef&);
template void surrogate_diffusion<float>(dc_state*, const StepCoef&);

void surrogate_free(dc_state* s) {
  delete s->sur;
  s->sur = nullptr;
}

void surrogate_geometry(dc_state* s) { mean_lengths(s->grid->h, &s->sur_lbar, &s->sur_dbar); }

// One plain step that records training pairs: features of the state before
// the diffusion and target (vn after - vn before) / dt at n sampled points.
template <typename R>
dc_status collect_impl(dc_state* s, double dt, int nsub, unsigned long long key, long long nsamp, float* buf,
                       long long stride, long long offset, long long* idx_dev) {
  const StepCoef c = make_coef(s, dt, std::max(nsub, 1));
  hipStream_t st = s->stream;
  const DevGrid& g = s->d;
  if (nsub > 0) {
    enqueue_substeps<R>(s, c, nsub, true);
  } else {
    const dc_fields& f = s->buf[s->cur];
    k_copy<double><<<1024, 256, 0, st>>>(static_cast<const double*>(f.w), s->wtmp, (size_t)(g.K + 1) * g.cs);
  }
  R* vn = static_cast<R*>(s->buf[s->cur].vn);
  R* old = static_cast<R*>(s->sur_tmlp);
  const FeatIn fin = front_and_features<R>(s, c, st);
  k_sample_feat<R><<<(unsigned)((nsamp + 255) / 256), 256, 0, st>>>(g, fin, s->sur_lbar, s->sur_dbar, key, nsamp, buf,
                                                                    stride, offset, idx_dev);
  k_copy<R><<<1024, 256, 0, st>>>(vn, old, (size_t)g.K * g.es);
  launch_diffusion_back<R>(g, vn, static_cast<const R*>(s->vt), static_cast<const R*>(s->tvn0),
                           static_cast<const R*>(s->d2), static_cast<const R*>(s->sur_cl), c, s->tiles, st, nullptr);
  k_sample_target<R><<<(unsigned)((nsamp + 255) / 256), 256, 0, st>>>(g, old, vn, dt, key, nsamp, buf, stride, offset);
  ML_TRY(hipGetLastError());
  return DC_OK;
}

}  // namespace dc

extern "C" {

dc_status dc_mlp_create(uint64_t seed, dc_mlp** out) {
  if (!out) return mfail(DC_EINVAL, "out is NULL");
  *out = nullptr;
  dc_mlp* M = new (std::nothrow) dc_mlp();
  if (!M) return mfail(DC_ENOMEM, "host allocation failed");
  auto bad = [&](hipError_t e) {
    (void)hipFree(M->par);
    (void)hipFree(M->m);
    (void)hipFree(M->v);
    (void)hipFree(M->nrm);
    delete M;
    return mfail(DC_EHIP, std::string("mlp allocation: ") + hipGetErrorString(e));
  };
  hipError_t e;
  if ((e = hipGetDevice(&M->device)) != hipSuccess) return bad(e);
  if ((e = hipMalloc(&M->par, NPAR * sizeof(float))) != hipSuccess) return bad(e);
  if ((e = hipMalloc(&M->m, NPAR * sizeof(float))) != hipSuccess) return bad(e);
  if ((e = hipMalloc(&M->v, NPAR * sizeof(float))) != hipSuccess) return bad(e);
  if ((e = hipMalloc(&M->nrm, sizeof(Norm))) != hipSuccess) return bad(e);
  // Kaiming-uniform (fan-in, gain sqrt 2) weights, zero biases
  std::mt19937_64 rng(seed);
  std::vector<float> p(NPAR, 0.0f);
  auto ku = [&](int off, int count, int fan_in) {
    std::uniform_real_distribution<double> u(-std::sqrt(6.0 / fan_in), std::sqrt(6.0 / fan_in));
    for (int i = 0; i < count; ++i) p[off + i] = (float)u(rng);
  };
  ku(OFF_W1, NIN * NH, NIN);
  ku(OFF_W2, NH * NH, NH);
  ku(OFF_W3, NH, NH);
  const std::vector<float> z(NPAR, 0.0f);
  Norm id{};
  for (int i = 0; i < NIN; ++i) {
    id.mean[i] = 0.f;
    id.istd[i] = 1.f;
    id.fmin[i] = -INFINITY;
    id.fmax[i] = INFINITY;
  }
  id.tstd = 1.f;
  M->hnrm = id;
  if ((e = hipMemcpy(M->par, p.data(), NPAR * 4, hipMemcpyHostToDevice)) != hipSuccess) return bad(e);
  if ((e = hipMemcpy(M->m, z.data(), NPAR * 4, hipMemcpyHostToDevice)) != hipSuccess) return bad(e);
  if ((e = hipMemcpy(M->v, z.data(), NPAR * 4, hipMemcpyHostToDevice)) != hipSuccess) return bad(e);
  if ((e = hipMemcpy(M->nrm, &id, sizeof(Norm), hipMemcpyHostToDevice)) != hipSuccess) return bad(e);
  *out = M;
  return DC_OK;
}

dc_status dc_mlp_destroy(dc_mlp* M) {
  if (!M) return mfail(DC_EINVAL, "mlp is NULL");
  const hipError_t e = hipDeviceSynchronize();
  (void)hipFree(M->par);
  (void)hipFree(M->m);
  (void)hipFree(M->v);
  (void)hipFree(M->nrm);
  delete M;
  if (e != hipSuccess) return mfail(DC_EHIP, std::string("pending work failed: ") + hipGetErrorString(e));
  return DC_OK;
}

dc_status dc_mlp_get_params(dc_mlp* M, float* host, int64_t n) {
  if (!M || !host || n != NPAR) return mfail(DC_EINVAL, "need a host array of DC_MLP_NPARAMS floats");
  ML_TRY(hipDeviceSynchronize());
  ML_TRY(hipMemcpy(host, M->par, NPAR * 4, hipMemcpyDeviceToHost));
  return DC_OK;
}

dc_status dc_mlp_set_params(dc_mlp* M, const float* host, int64_t n) {
  if (!M || !host || n != NPAR) return mfail(DC_EINVAL, "need a host array of DC_MLP_NPARAMS floats");
  ML_TRY(hipDeviceSynchronize());
  ML_TRY(hipMemcpy(M->par, host, NPAR * 4, hipMemcpyHostToDevice));
  const std::vector<float> z(NPAR, 0.0f);
  ML_TRY(hipMemcpy(M->m, z.data(), NPAR * 4, hipMemcpyHostToDevice));
  ML_TRY(hipMemcpy(M->v, z.data(), NPAR * 4, hipMemcpyHostToDevice));
  M->adam_step = 0;
  return DC_OK;
}

dc_status dc_mlp_set_norm(dc_mlp* M, const float* mean, const float* sd, const float* fmin, const float* fmax,
                          float tstd) {
  if (!M || !mean || !sd || !fmin || !fmax) return mfail(DC_EINVAL, "NULL argument");
  if (!(tstd > 0.f) || !std::isfinite(tstd)) return mfail(DC_EINVAL, "target scale must be finite and > 0");
  Norm nr{};
  for (int i = 0; i < NIN; ++i) {
    if (!(sd[i] > 0.f) || !std::isfinite(sd[i]) || !std::isfinite(1.0f / sd[i]) || !std::isfinite(mean[i]))
      return mfail(DC_EINVAL, "feature scales must be finite and > 0");
    if (!(fmin[i] <= fmax[i])) return mfail(DC_EINVAL, "feature range must have min <= max");
    nr.mean[i] = mean[i];
    nr.istd[i] = 1.0f / sd[i];
    nr.fmin[i] = fmin[i];
    nr.fmax[i] = fmax[i];
  }
  nr.tstd = tstd;
  ML_TRY(hipDeviceSynchronize());
  ML_TRY(hipMemcpy(M->nrm, &nr, sizeof(Norm), hipMemcpyHostToDevice));
  M->hnrm = nr;
  return DC_OK;
}

dc_status dc_mlp_get_norm(const dc_mlp* M, float* out, int64_t n) {
  if (!M || !out || n != 4 * NIN + 1) return mfail(DC_EINVAL, "need a host array of 73 floats");
  for (int i = 0; i < NIN; ++i) {
    out[i] = M->hnrm.mean[i];
    out[NIN + i] = 1.0f / M->hnrm.istd[i];
    out[2 * NIN + i] = M->hnrm.fmin[i];
    out[3 * NIN + i] = M->hnrm.fmax[i];
  }
  out[4 * NIN] = M->hnrm.tstd;
  return DC_OK;
}

dc_status dc_mlp_fit_norm(dc_mlp* M, const float* dev_buf, int64_t stride, int64_t n) {
  if (!M || !dev_buf || n < 2 || stride < n) return mfail(DC_EINVAL, "bad training buffer (n >= 2, stride >= n)");
  const int nb = 256;
  double* part = nullptr;
  ML_TRY(hipMalloc(&part, (size_t)(NIN + 1) * nb * 4 * sizeof(double)));
  k_stats<<<dim3(nb, NIN + 1), 256>>>(dev_buf, stride, n, part);
  std::vector<double> h((size_t)(NIN + 1) * nb * 4);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpy(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost);
  (void)hipFree(part);
  if (e != hipSuccess) return mfail(DC_EHIP, std::string("fit_norm: ") + hipGetErrorString(e));
  float mean[NIN], sd[NIN], mn[NIN], mx[NIN], tstd = 1.f;
  for (int r = 0; r <= NIN; ++r) {
    double s = 0, s2 = 0, lo = 1e300, hi = -1e300;
    for (int b = 0; b < nb; ++b) {
      const double* p = &h[((size_t)r * nb + b) * 4];
      s += p[0];
      s2 += p[1];
      lo = std::min(lo, p[2]);
      hi = std::max(hi, p[3]);
    }
    if (!std::isfinite(s2) || !std::isfinite(lo) || !std::isfinite(hi))
      return mfail(DC_ENONFINITE, "training buffer holds non-finite values");
    // flow features and the target: symmetric set (sign augmentation)
    const bool flow = r < NFLOW || r == NIN;
    const double mu = flow ? 0.0 : s / n;
    // the physical features span tens of orders of magnitude (div L1 is
    // ~1e-17 s^-1 m^-2 on a global grid): only a vanishing or non-finite
    // spread counts as constant
    double var = s2 / n - mu * mu;
    if (!(var > 0.0) || !std::isfinite(var) || !std::isfinite((float)(1.0 / std::sqrt(var)))) var = 1.0;
    if (r == NIN) {
      tstd = (float)std::sqrt(var);
      continue;
    }
    mean[r] = (float)mu;
    sd[r] = (float)std::sqrt(var);
    const double amax = std::max(std::fabs(lo), std::fabs(hi));
    mn[r] = (float)(flow ? -amax : lo);
    mx[r] = (float)(flow ? amax : hi);
  }
  return dc_mlp_set_norm(M, mean, sd, mn, mx, tstd);
}

dc_status dc_mlp_train(dc_mlp* M, const float* dev_buf, int64_t stride, int64_t n, const dc_train_cfg* cfg) {
  if (!M || !dev_buf || !cfg) return mfail(DC_EINVAL, "NULL argument");
  if (cfg->batch < 128 || cfg->batch % 128 || cfg->epochs < 1 || n < cfg->batch || stride < n)
    return mfail(DC_EINVAL, "batch must be a positive multiple of 128, n >= batch, stride >= n, epochs >= 1");
  if (!(cfg->lr0 > 0) || !(cfg->lr1 >= 0)) return mfail(DC_EINVAL, "learning rates must be positive");
  const int nw = cfg->batch / 64;
  float* part = nullptr;
  float* loss_d = nullptr;
  const long long iters_per_epoch = n / cfg->batch;
  const long long total = iters_per_epoch * cfg->epochs;
  ML_TRY(hipMalloc(&part, (size_t)nw * (NPAR + 1) * sizeof(float)));
  hipError_t e = hipMalloc(&loss_d, (size_t)total * sizeof(float));
  if (e != hipSuccess) {
    (void)hipFree(part);
    return mfail(DC_ENOMEM, "loss trace allocation failed");
  }
  long long it = 0;
  for (int ep = 0; ep < cfg->epochs && e == hipSuccess; ++ep) {
    const unsigned long long key =
        cfg->shuffle ? (cfg->seed * 0x9e3779b97f4a7c15ull + 0x2545f4914f6cdd1dull * (unsigned long long)(ep + 1)) | 1ull
                     : 0ull;
    for (long long b = 0; b < iters_per_epoch; ++b, ++it) {
      const double lr = cfg->lr1 + 0.5 * (cfg->lr0 - cfg->lr1) * (1.0 + std::cos(M_PI * (double)it / (double)total));
      k_train<<<cfg->batch / 128, 128>>>(M->par, M->nrm, dev_buf, stride, n, key, b * (long long)cfg->batch,
                                         cfg->batch, cfg->augment, part);
      ++M->adam_step;
      k_adam<<<22, 256>>>(part, nw, M->par, M->m, M->v, nullptr, (int)std::min<long long>(M->adam_step, 1 << 30),
                          (float)lr, 1, loss_d + it, cfg->batch);
    }
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess) {
    M->loss_trace.resize(total);
    e = hipMemcpy(M->loss_trace.data(), loss_d, (size_t)total * sizeof(float), hipMemcpyDeviceToHost);
  }
  (void)hipFree(part);
  (void)hipFree(loss_d);
  if (e != hipSuccess) return mfail(DC_EHIP, std::string("training: ") + hipGetErrorString(e));
  return DC_OK;
}

dc_status dc_mlp_loss_trace(const dc_mlp* M, float* host, int64_t cap, int64_t* n_out) {
  if (!M || !n_out || cap < 0) return mfail(DC_EINVAL, "NULL argument");
  *n_out = (int64_t)M->loss_trace.size();
  if (host) std::memcpy(host, M->loss_trace.data(), sizeof(float) * std::min<size_t>(cap, M->loss_trace.size()));
  return DC_OK;
}

dc_status dc_mlp_forward(dc_mlp* M, const float* host_x, int64_t n, float* host_y) {
  if (!M || !host_x || !host_y || n < 1) return mfail(DC_EINVAL, "bad arguments");
  float *x = nullptr, *y = nullptr;
  ML_TRY(hipMalloc(&x, (size_t)n * NIN * 4));
  hipError_t e = hipMalloc(&y, (size_t)n * 4);
  if (e == hipSuccess) e = hipMemcpy(x, host_x, (size_t)n * NIN * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    k_forward_rows<<<(unsigned)((n + 64 * kInferWaves - 1) / (64 * kInferWaves)), 64 * kInferWaves>>>(M->par, M->nrm, x, n, y);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpy(host_y, y, (size_t)n * 4, hipMemcpyDeviceToHost);
  (void)hipFree(x);
  (void)hipFree(y);
  if (e != hipSuccess) return mfail(DC_EHIP, std::string("forward: ") + hipGetErrorString(e));
  return DC_OK;
}

dc_status dc_mlp_grad(dc_mlp* M, const float* host_x, const float* host_t, int64_t n, float* host_grad, float* loss) {
  if (!M || !host_x || !host_t || !host_grad || n < 128 || n % 128) return mfail(DC_EINVAL, "n must be a multiple of 128");
  std::vector<float> soa((size_t)(NIN + 1) * n);
  for (int64_t r = 0; r < n; ++r) {
    for (int f = 0; f < NIN; ++f) soa[(size_t)f * n + r] = host_x[r * NIN + f];
    soa[(size_t)NIN * n + r] = host_t[r];
  }
  float *buf = nullptr, *part = nullptr, *g = nullptr, *l = nullptr;
  const int nw = (int)(n / 64);
  ML_TRY(hipMalloc(&buf, soa.size() * 4));
  hipError_t e = hipMalloc(&part, (size_t)nw * (NPAR + 1) * 4);
  if (e == hipSuccess) e = hipMalloc(&g, NPAR * 4);
  if (e == hipSuccess) e = hipMalloc(&l, 4);
  if (e == hipSuccess) e = hipMemcpy(buf, soa.data(), soa.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    k_train<<<(unsigned)(n / 128), 128>>>(M->par, M->nrm, buf, n, n, 0, 0, (int)n, 0, part);
    k_adam<<<22, 256>>>(part, nw, M->par, M->m, M->v, g, 1, 0.f, 0, l, (int)n);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpy(host_grad, g, NPAR * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess && loss) e = hipMemcpy(loss, l, 4, hipMemcpyDeviceToHost);
  (void)hipFree(buf);
  (void)hipFree(part);
  (void)hipFree(g);
  (void)hipFree(l);
  if (e != hipSuccess) return mfail(DC_EHIP, std::string("grad: ") + hipGetErrorString(e));
  return DC_OK;
}

dc_status dc_state_set_mlp(dc_state* s, const dc_mlp* M, double threshold, int32_t judge_every) {
  if (!s || !M) return mfail(DC_EINVAL, "NULL argument");
  if (s->diff != DC_DIFF_SURROGATE) return mfail(DC_ESTATE, "state was not created with DC_DIFF_SURROGATE");
  if (judge_every < 1 || !(threshold >= 0.0)) return mfail(DC_EINVAL, "need judge_every >= 1 and threshold >= 0");
  if (M->device != s->grid->device) return mfail(DC_EINVAL, "mlp and state on different devices");
  if (!s->sur) s->sur = new (std::nothrow) SurCtx();
  if (!s->sur) return mfail(DC_ENOMEM, "host allocation failed");
  s->sur->mlp = M;
  s->sur->thr = threshold;
  s->sur->judge_every = judge_every;
  s->sur->steps = 0;
  s->sur->judge_steps = 0;
  k_fill_int<<<1, 64, 0, s->stream>>>(s->sur_cnt, 6, 0);
  ML_TRY(hipGetLastError());
  return DC_OK;
}

dc_status dc_surrogate_stats(dc_state* s, dc_surrogate_info* out) {
  if (!s || !out) return mfail(DC_EINVAL, "NULL argument");
  if (s->diff != DC_DIFF_SURROGATE) return mfail(DC_ESTATE, "state was not created with DC_DIFF_SURROGATE");
  int cnt[6] = {0, 0, 0, 0, 0, 0};
  ML_TRY(hipStreamSynchronize(s->stream));
  ML_TRY(hipMemcpy(cnt, s->sur_cnt, sizeof(cnt), hipMemcpyDeviceToHost));
  unsigned long long total;
  std::memcpy(&total, cnt + 4, sizeof(total));
  out->steps = s->sur ? s->sur->steps : 0;
  out->judge_steps = s->sur ? s->sur->judge_steps : 0;
  out->judge_flagged = cnt[0];
  out->range_flagged = cnt[1];
  out->fallback = cnt[2];
  out->fallback_total = (int64_t)total;
  out->n_columns = s->grid->h.ne;
  return DC_OK;
}

dc_status dc_surrogate_collect(dc_state* s, double dt, int32_t nsub, uint64_t seed, int64_t n_samples, float* dev_buf,
                               int64_t stride, int64_t offset, int64_t* host_index) {
  if (!s || !dev_buf) return mfail(DC_EINVAL, "NULL argument");
  if (s->diff != DC_DIFF_SURROGATE) return mfail(DC_ESTATE, "state was not created with DC_DIFF_SURROGATE");
  const HostGrid& h = s->grid->h;
  if (n_samples < 1 || offset < 0 || offset + n_samples > stride) return mfail(DC_EINVAL, "bad sample buffer extent");
  if ((unsigned long long)n_samples > (unsigned long long)h.K * h.ne)
    return mfail(DC_EINVAL, "more samples than (edge, level) points");
  if (!(dt > 0.0) || !std::isfinite(dt) || nsub < 0 || nsub > 1000) return mfail(DC_EINVAL, "bad dt or nsubsteps");
  long long* idx = nullptr;
  if (host_index) ML_TRY(hipMalloc(&idx, (size_t)n_samples * sizeof(long long)));
  const unsigned long long key = seed * 0x9e3779b97f4a7c15ull + 0x632be59bd9b4e019ull;
  s->part = 0;  // the workspace is overwritten
  const dc_status st = s->prec == DC_PREC_MIXED
                           ? collect_impl<float>(s, dt, nsub, key, n_samples, dev_buf, stride, offset, idx)
                           : collect_impl<double>(s, dt, nsub, key, n_samples, dev_buf, stride, offset, idx);
  if (idx) {
    std::vector<long long> hi(n_samples);
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e == hipSuccess) e = hipMemcpy(hi.data(), idx, (size_t)n_samples * sizeof(long long), hipMemcpyDeviceToHost);
    (void)hipFree(idx);
    if (e != hipSuccess) return mfail(DC_EHIP, std::string("collect: ") + hipGetErrorString(e));
    if (st == DC_OK)
      for (int64_t i = 0; i < n_samples; ++i) {
        const long long k = hi[i] / h.ne, ie = hi[i] % h.ne;
        host_index[i] = k * h.ne + h.perm_e[ie];
      }
  }
  return st;
}

}  // extern "C"
