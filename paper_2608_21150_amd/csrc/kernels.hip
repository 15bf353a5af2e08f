// Single-state launches of the dycore step (see bodies.h for the kernels).

#include <hip/hip_runtime.h>

#include <algorithm>

#include "bodies.h"
#include "internal.h"
#include "kernels.h"

namespace dc {

namespace {

using bodies::vt_row;

// ---------------------------------------------------------------------------
// conservation diagnostics: fixed-order block partials, then one block
// ---------------------------------------------------------------------------
constexpr int kDiagThreads = 256;

template <typename T>
__device__ T block_sum(T v, T* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = kDiagThreads / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] = sh[t] + sh[t + s];
    __syncthreads();
  }
  const T r = sh[0];
  __syncthreads();
  return r;
}
__device__ double block_max(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = kDiagThreads / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] = fmax(sh[t], sh[t + s]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// partial layout: [5][nblocks]: mass, theta-mass, max|w|, max|vn|, nonfinite
template <typename R>
__global__ void __launch_bounds__(kDiagThreads) k_diag(DevGrid g, const R* __restrict__ vn,
                                                       const double* __restrict__ w, const double* __restrict__ rho,
                                                       const double* __restrict__ th, const double* __restrict__ ex,
                                                       double* __restrict__ part, int ncb) {
  __shared__ double sh[kDiagThreads];
  const int nblk = gridDim.x;
  const int K = g.K;
  const double* dzf = vt_row(g, VT_DZF);
  double m = 0.0, tm = 0.0, mw = 0.0, mv = 0.0, nf = 0.0;
  if ((int)blockIdx.x < ncb) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < g.nc) {
      double sr = 0.0, srt = 0.0;
      for (int j = 0; j < K; ++j) {
        const size_t r = (size_t)j * g.cs + c;
        const double a = rho[r], t = th[r], x = ex[r];
        sr += a * dzf[j];
        srt += a * t * dzf[j];
        nf += (!isfinite(a)) + (!isfinite(t)) + (!isfinite(x));
      }
      for (int k = 0; k <= K; ++k) {
        const double x = w[(size_t)k * g.cs + c];
        nf += !isfinite(x);
        mw = fmax(mw, fabs(x));
      }
      m = g.area[c] * sr;
      tm = g.area[c] * srt;
    }
  } else {
    const int e = (blockIdx.x - ncb) * blockDim.x + threadIdx.x;
    if (e < g.ne) {
      for (int j = 0; j < K; ++j) {
        const double x = (double)vn[(size_t)j * g.es + e];
        nf += !isfinite(x);
        mv = fmax(mv, fabs(x));
      }
    }
  }
  const double bm = block_sum(m, sh), btm = block_sum(tm, sh);
  const double bw = block_max(mw, sh), bv = block_max(mv, sh);
  const double bn = block_sum(nf, sh);
  if (threadIdx.x == 0) {
    part[0 * nblk + blockIdx.x] = bm;
    part[1 * nblk + blockIdx.x] = btm;
    part[2 * nblk + blockIdx.x] = bw;
    part[3 * nblk + blockIdx.x] = bv;
    part[4 * nblk + blockIdx.x] = bn;
  }
}

__global__ void __launch_bounds__(kDiagThreads) k_diag_final(const double* __restrict__ part, int nblk,
                                                             double* __restrict__ out) {
  __shared__ double sh[kDiagThreads];
  double s0 = 0.0, s1 = 0.0, s4 = 0.0, m2 = 0.0, m3 = 0.0;
  for (int i = threadIdx.x; i < nblk; i += kDiagThreads) {
    s0 += part[i];
    s1 += part[nblk + i];
    m2 = fmax(m2, part[2 * nblk + i]);
    m3 = fmax(m3, part[3 * nblk + i]);
    s4 += part[4 * nblk + i];
  }
  const double a = block_sum(s0, sh), b = block_sum(s1, sh);
  const double c = block_max(m2, sh), d = block_max(m3, sh);
  const double e = block_sum(s4, sh);
  if (threadIdx.x == 0) {
    out[0] = a;
    out[1] = b;
    out[2] = c;
    out[3] = d;
    out[4] = e;
  }
}

}  // namespace

const char* const kKernelNames[K_COUNT] = {
    "vort_ke_pred", "edge_pred", "column_pred",
    "vort_ke_corr", "edge_corr", "column_corr",
    "diff_vertex", "diff_div", "diff_edge1", "diff_cell_vertex2", "diff_edge2",
    "edge_upwind"};


int diag_partial_count(const DevGrid& g) {
  return (g.nc + kDiagThreads - 1) / kDiagThreads + (g.ne + kDiagThreads - 1) / kDiagThreads;
}

namespace {

template <typename B>
void one(int id, const DevGrid& g, const typename B::Args& a, const Tile* T, hipStream_t s, Prof* prof) {
  const bodies::Geom geo = bodies::geom_of(id, g, T, sizeof(typename B::Real));
  if (geo.nbx == 0) return;  // nothing to do (the vorticity pass of a fused grid)
  const bool rec = prof && prof->wants(id);
  if (rec) prof->mark(s, id);
  bodies::k_one<B><<<dim3(geo.nbx, geo.nby), geo.threads, geo.smem, s>>>(g, a);
  if (rec) prof->mark(s, -1);
}

template <typename R, bool CORR>
void one_col(int id, const DevGrid& g, const bodies::ColPhaseArgs<R>& a, const Tile* T, hipStream_t s, Prof* prof) {
  int lm;
  bodies::col_chunks_lm(g.K, CORR, &lm);
  if (lm == 8)
    one<bodies::BCol<R, CORR, 8>>(id, g, a, T, s, prof);
  else if (lm == 12)
    one<bodies::BCol<R, CORR, 12>>(id, g, a, T, s, prof);
  else
    one<bodies::BCol<R, CORR, 16>>(id, g, a, T, s, prof);
}

}  // namespace

template <typename R>
void launch_predictor(const DevGrid& g, const Bufs<R>& b, const StepCoef& c, const Tile* T, hipStream_t s,
                      Prof* prof) {
  using namespace bodies;
  const SubstepArgs<R> a = substep_args<R>(g, b, c, T);
  // advective tendencies at the substep start, momentum, column
  one<BVc<R, false>>(K_VC_P, g, a.vc_p, T, s, prof);
  if (c.miura) one<BMiura<R>>(K_MIURA, g, a.mi, T, s, prof);  // needs vt of the start vn
  one<BEdge<R, false>>(K_EDGE_P, g, a.e_p, T, s, prof);
  one_col<R, false>(K_COL_P, g, a.c_p, T, s, prof);
}

template <typename R>
void launch_corrector(const DevGrid& g, const Bufs<R>& b, const StepCoef& c, const Tile* T, hipStream_t s,
                      Prof* prof) {
  using namespace bodies;
  const SubstepArgs<R> a = substep_args<R>(g, b, c, T);
  // tendencies at the predicted state, damping, momentum, column
  one<BVc<R, true>>(K_VC_C, g, a.vc_c, T, s, prof);
  one<BEdge<R, true>>(K_EDGE_C, g, a.e_c, T, s, prof);
  one_col<R, true>(K_COL_C, g, a.c_c, T, s, prof);
}

template <typename R>
void launch_substep(const DevGrid& g, const Bufs<R>& b, const StepCoef& c, const Tile* T, hipStream_t s, Prof* prof) {
  launch_predictor<R>(g, b, c, T, s, prof);
  launch_corrector<R>(g, b, c, T, s, prof);
}

template <typename R>
void launch_diffusion(const DevGrid& g, R* vn, const double* w_in, double* w_out, R* l1, R* nu, R* dv, R* dl1,
                      R* zeta, R* vv, const ThetaDiff& td, const StepCoef& c, const Tile* T, hipStream_t s,
                      Prof* prof) {
  using namespace bodies;
  const DiffusionArgs<R> d = diffusion_args<R>(g, vn, w_in, w_out, l1, nu, dv, dl1, zeta, vv, c, T, td);
  one<BDvert<R>>(K_DVERT, g, d.dv, T, s, prof);
  one<BDiv<R>>(K_DDIV, g, d.dd, T, s, prof);
  one<BDedge1<R>>(K_DEDGE1, g, d.d1, T, s, prof);
  one<BDcv2<R>>(K_DCV2, g, d.cv, T, s, prof);  // cells (K+1 half levels) and vertices in one launch
  one<BDedge2<R>>(K_DEDGE2, g, d.d2, T, s, prof);
}

template <typename R>
void launch_diffusion_front(const DevGrid& g, const R* vn, const double* w_in, double* w_out, R* l1, R* nu, R* dv,
                            R* dl1, R* zeta, R* curll1, R* vv, const StepCoef& c, const Tile* T, hipStream_t s,
                            Prof* prof) {
  using namespace bodies;
  DiffusionArgs<R> d = diffusion_args<R>(g, const_cast<R*>(vn), w_in, w_out, l1, nu, dv, dl1, zeta, vv, c, T);
  d.cv.curll1 = curll1;
  one<BDvert<R>>(K_DVERT, g, d.dv, T, s, prof);
  one<BDiv<R>>(K_DDIV, g, d.dd, T, s, prof);
  one<BDedge1<R>>(K_DEDGE1, g, d.d1, T, s, prof);
  one<BDcv2<R>>(K_DCV2, g, d.cv, T, s, prof);
}

template <typename R>
void launch_diffusion_back(const DevGrid& g, R* vn, const R* l1, const R* nu, const R* dl1, const R* curll1,
                           const StepCoef& c, const Tile* T, hipStream_t s, Prof* prof) {
  using namespace bodies;
  const typename BDedge2<R>::Args a{vn, l1, nu, dl1, curll1, c, T[T_DEDGE].kb};
  one<BDedge2<R>>(K_DEDGE2, g, a, T, s, prof);
}

template <typename R>
void launch_diag(const DevGrid& g, const R* vn, const double* w, const double* rho, const double* th,
                 const double* ex, double* partial, double* out, hipStream_t s) {
  const int ncb = (g.nc + kDiagThreads - 1) / kDiagThreads;
  const int neb = (g.ne + kDiagThreads - 1) / kDiagThreads;
  k_diag<R><<<ncb + neb, kDiagThreads, 0, s>>>(g, vn, w, rho, th, ex, partial, ncb);
  k_diag_final<<<1, kDiagThreads, 0, s>>>(partial, ncb + neb, out);
}

template void launch_predictor<double>(const DevGrid&, const Bufs<double>&, const StepCoef&, const Tile*,
                                       hipStream_t, Prof*);
template void launch_predictor<float>(const DevGrid&, const Bufs<float>&, const StepCoef&, const Tile*, hipStream_t,
                                      Prof*);
template void launch_corrector<double>(const DevGrid&, const Bufs<double>&, const StepCoef&, const Tile*,
                                       hipStream_t, Prof*);
template void launch_corrector<float>(const DevGrid&, const Bufs<float>&, const StepCoef&, const Tile*, hipStream_t,
                                      Prof*);
template void launch_substep<double>(const DevGrid&, const Bufs<double>&, const StepCoef&, const Tile*, hipStream_t,
                                     Prof*);
template void launch_substep<float>(const DevGrid&, const Bufs<float>&, const StepCoef&, const Tile*, hipStream_t,
                                    Prof*);
template void launch_diffusion<double>(const DevGrid&, double*, const double*, double*, double*, double*, double*,
                                       double*, double*, double*, const ThetaDiff&, const StepCoef&, const Tile*,
                                       hipStream_t, Prof*);
template void launch_diffusion<float>(const DevGrid&, float*, const double*, double*, float*, float*, float*, float*,
                                      float*, float*, const ThetaDiff&, const StepCoef&, const Tile*, hipStream_t,
                                      Prof*);
template void launch_diffusion_front<double>(const DevGrid&, const double*, const double*, double*, double*,
                                             double*, double*, double*, double*, double*, double*, const StepCoef&,
                                             const Tile*, hipStream_t, Prof*);
template void launch_diffusion_front<float>(const DevGrid&, const float*, const double*, double*, float*, float*,
                                            float*, float*, float*, float*, float*, const StepCoef&, const Tile*,
                                            hipStream_t, Prof*);
template void launch_diffusion_back<double>(const DevGrid&, double*, const double*, const double*, const double*,
                                            const double*, const StepCoef&, const Tile*, hipStream_t, Prof*);
template void launch_diffusion_back<float>(const DevGrid&, float*, const float*, const float*, const float*,
                                           const float*, const StepCoef&, const Tile*, hipStream_t, Prof*);
template void launch_diag<double>(const DevGrid&, const double*, const double*, const double*, const double*,
                                  const double*, double*, double*, hipStream_t);
template void launch_diag<float>(const DevGrid&, const float*, const double*, const double*, const double*,
                                 const double*, double*, double*, hipStream_t);

}  // namespace dc
