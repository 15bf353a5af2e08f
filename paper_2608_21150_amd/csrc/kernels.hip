// HIP kernels (gfx950) of the non-hydrostatic dycore step.
//
// Layout: every field is [level][entity], entity index fastest, each level
// padded to a multiple of 64 entities; a thread owns one entity and walks a
// block of levels, so the neighbour indices and stencil weights are loaded
// once per thread and every level access of the own entity is a coalesced
// 64-wide row.  Gathers go through the lookup tables (paper, Section 4.2.1).
// Blocks are remapped so that the 8 XCDs each sweep a contiguous range of
// tiles (neighbour halos then mostly hit the same XCD's L2).
//
// Template parameter R is the type of vn and of the horizontal-stencil
// intermediates: double for the FP64 path, float for the mixed path.  The
// column solver, w/rho/exner/theta_v and flux-divergence sums are always
// FP64.  No floating-point atomics: results do not depend on scheduling.

#include "internal.h"
#include "kernels.h"

namespace dc {

namespace {

__device__ __forceinline__ void tile_coords(int& bx, int& by) {
  const int nbx = gridDim.x;
  const int n = gridDim.x * gridDim.y;
  const int lin = blockIdx.x + blockIdx.y * nbx;
  const int q = n >> 3, r = n & 7, x = lin & 7, i = lin >> 3;
  const int lp = (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
  bx = lp % nbx;
  by = lp / nbx;
}

__device__ __forceinline__ const double* vt_row(const DevGrid& g, int tab) { return g.vert + (size_t)tab * (g.K + 1); }

// ---------------------------------------------------------------------------
// vertex: relative vorticity zeta_v = (1/A_v) sum sig d_e vn_e
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(256) k_curl(DevGrid g, const R* __restrict__ vn, R* __restrict__ zeta, int kb) {
  int bx, by;
  tile_coords(bx, by);
  const int v = bx * blockDim.x + threadIdx.x;
  if (v >= g.nv) return;
  int idx[6];
  R cf[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    idx[s] = g.v2e[s * g.vs + v];
    cf[s] = (R)g.kcurl[s * g.vs + v];
  }
  const int k0 = by * kb, k1 = min(g.K, k0 + kb);
  for (int k = k0; k < k1; ++k) {
    const R* row = vn + (size_t)k * g.es;
    R acc = cf[0] * row[idx[0]];
#pragma unroll
    for (int s = 1; s < 6; ++s) acc += cf[s] * row[idx[s]];
    zeta[(size_t)k * g.vs + v] = acc;
  }
}

// ---------------------------------------------------------------------------
// edge: tangential wind by Perot reconstruction (weights precomputed)
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(256) k_vt(DevGrid g, const R* __restrict__ vn, R* __restrict__ vt, int kb) {
  int bx, by;
  tile_coords(bx, by);
  const int e = bx * blockDim.x + threadIdx.x;
  if (e >= g.ne) return;
  int idx[4];
  R cf[5];
  cf[0] = (R)g.kvt[e];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    idx[s] = g.e2c2e[s * g.es + e];
    cf[1 + s] = (R)g.kvt[(1 + s) * g.es + e];
  }
  const int k0 = by * kb, k1 = min(g.K, k0 + kb);
  for (int k = k0; k < k1; ++k) {
    const R* row = vn + (size_t)k * g.es;
    R acc = cf[0] * row[e];
#pragma unroll
    for (int s = 0; s < 4; ++s) acc += cf[1 + s] * row[idx[s]];
    vt[(size_t)k * g.es + e] = acc;
  }
}

// ---------------------------------------------------------------------------
// cell: kinetic energy K_c, vertical-wind advection T_w (half levels) and,
// in the corrector, the divergence-damping field D2 = laps(div vn).
// Grid y covers the K+1 half levels.
// ---------------------------------------------------------------------------
template <typename R, bool CORR>
__global__ void __launch_bounds__(256) k_cell_adv(DevGrid g, const R* __restrict__ vn, const R* __restrict__ vt,
                                                  const double* __restrict__ w, R* __restrict__ kc,
                                                  R* __restrict__ tw, R* __restrict__ d2, int kb) {
  int bx, by;
  tile_coords(bx, by);
  const int c = bx * blockDim.x + threadIdx.x;
  if (c >= g.nc) return;
  const int K = g.K;
  int ie[3], nb[3];
  R kd[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    ie[i] = g.c2e[i * g.cs + c];
    nb[i] = g.c2e2c[i * g.cs + c];
    kd[i] = (R)g.kdiv[i * g.cs + c];
  }
  int ie2[3][3];
  R kd2[3][3], kl[3];
  if (CORR) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      kl[i] = (R)g.klap[i * g.cs + c];
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        ie2[i][m] = g.c2e[m * g.cs + nb[i]];
        kd2[i][m] = (R)g.kdiv[m * g.cs + nb[i]];
      }
    }
  }
  const double* idzc2 = vt_row(g, VT_IDZC2);
  const int k0 = by * kb, k1 = min(K + 1, k0 + kb);
  for (int k = k0; k < k1; ++k) {
    if (k < K) {
      const R* vrow = vn + (size_t)k * g.es;
      const R* trow = vt + (size_t)k * g.es;
      R ke = R(0);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const R a = vrow[ie[i]], b = trow[ie[i]];
        ke += R(0.5) * (a * a + b * b);
      }
      kc[(size_t)k * g.cs + c] = ke / R(3);
      if (CORR) {
        R dc = kd[0] * vrow[ie[0]] + kd[1] * vrow[ie[1]] + kd[2] * vrow[ie[2]];
        R acc = R(0);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const R dn = kd2[i][0] * vrow[ie2[i][0]] + kd2[i][1] * vrow[ie2[i][1]] + kd2[i][2] * vrow[ie2[i][2]];
          acc += kl[i] * (dn - dc);
        }
        d2[(size_t)k * g.cs + c] = acc;
      }
    }
    R t = R(0);
    if (k >= 1 && k <= K - 1) {
      const R* va = vn + (size_t)(k - 1) * g.es;
      const R* vb = vn + (size_t)k * g.es;
      const double* wr = w + (size_t)k * g.cs;
      const double wc = wr[c];
      R h = R(0);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const R vie = R(0.5) * (va[ie[i]] + vb[ie[i]]);
        h += kd[i] * vie * (R)(wr[nb[i]] - wc);
      }
      const double dwdz = (w[(size_t)(k - 1) * g.cs + c] - w[(size_t)(k + 1) * g.cs + c]) * idzc2[k];
      t = R(-0.5) * h - (R)(wc * dwdz);
    }
    tw[(size_t)k * g.cs + c] = t;
  }
}

// ---------------------------------------------------------------------------
// edge: advective tendency T_vn and the horizontal momentum update.
//  predictor: vn* = vn + dtau (T_vn - cpd theta_e grad pi')       -> tvn0, vns
//  corrector: vn' = vn_now + dtau (a0 T0 + a1 T* - cpd theta_e grad pi')
//                   - c4 Abar^2 grad(D2)                             -> vn_out
// The pressure-gradient term is formed from the state at the start of the
// substep in both passes.
// ---------------------------------------------------------------------------
template <typename R, bool CORR>
__global__ void __launch_bounds__(256) k_edge(DevGrid g, const R* __restrict__ vn, const R* __restrict__ vt,
                                              const R* __restrict__ zeta, const R* __restrict__ kc,
                                              const double* __restrict__ w, const double* __restrict__ ex,
                                              const double* __restrict__ th, R* __restrict__ tvn0,
                                              R* __restrict__ vout, const R* __restrict__ vn_now,
                                              const R* __restrict__ d2, StepCoef cf, int kb) {
  int bx, by;
  tile_coords(bx, by);
  const int e = bx * blockDim.x + threadIdx.x;
  if (e >= g.ne) return;
  const int K = g.K;
  const int c0 = g.e2c[e], c1 = g.e2c[g.es + e];
  const int v0 = g.e2v[e], v1 = g.e2v[g.es + e];
  const double invd = g.invd[e];
  const R invd_r = (R)invd;
  const R fe = (R)g.fe[e];
  const double* idzf = vt_row(g, VT_IDZF);
  const double* exref = vt_row(g, VT_EXREF);
  const int k0 = by * kb, k1 = min(K, k0 + kb);
  for (int j = k0; j < k1; ++j) {
    const size_t re = (size_t)j * g.es + e;
    const R vj = vn[re];
    const R vup = j > 0 ? vn[re - g.es] : vj;
    const R vdn = j < K - 1 ? vn[re + g.es] : vj;
    const R ie_top = j > 0 ? R(0.5) * (vup + vj) : vj;
    const R ie_bot = j < K - 1 ? R(0.5) * (vj + vdn) : vj;
    const R* zr = zeta + (size_t)j * g.vs;
    const R ze = R(0.5) * (zr[v0] + zr[v1]);
    const R* kr = kc + (size_t)j * g.cs;
    const R kgrad = (kr[c1] - kr[c0]) * invd_r;
    const double* wa = w + (size_t)j * g.cs;
    const double* wb = wa + g.cs;
    const R wef = (R)(0.5 * (0.5 * (wa[c0] + wa[c1]) + 0.5 * (wb[c0] + wb[c1])));
    const R tvn = (ze + fe) * vt[re] - kgrad - wef * (ie_top - ie_bot) * (R)idzf[j];
    const size_t rc = (size_t)j * g.cs;
    const double exr = exref[j];
    const R gex = (R)((ex[rc + c1] - exr) - (ex[rc + c0] - exr)) * invd_r;
    const R the = (R)(0.5 * (th[rc + c0] + th[rc + c1]));
    const R pgf = (R)cf.cpd * the * gex;
    if (!CORR) {
      tvn0[re] = tvn;
      vout[re] = vj + (R)cf.dtau * (tvn - pgf);
    } else {
      const R dd = (d2[rc + c1] - d2[rc + c0]) * invd_r;
      vout[re] = vn_now[re] + (R)cf.dtau * ((R)cf.a0 * tvn0[re] + (R)cf.a1 * tvn - pgf) - (R)cf.c4a2 * dd;
    }
  }
}

// ---------------------------------------------------------------------------
// column: flux divergences, explicit parts, tridiagonal w solve (Thomas,
// no pivoting: every pivot is >= 1 for this matrix), sponge, and in the
// corrector the increment updates of rho, exner, theta_v.  One thread owns
// one column and sweeps it top to bottom and back; the elimination factors
// are kept in a [K+1][cs] scratch (coalesced rows).
// ---------------------------------------------------------------------------
template <typename R, bool CORR>
__global__ void __launch_bounds__(64) k_col(DevGrid g, const double* __restrict__ w, const double* __restrict__ rho,
                                            const double* __restrict__ ex, const double* __restrict__ th,
                                            const R* __restrict__ vnf, const R* __restrict__ tw0,
                                            const R* __restrict__ tw1, double* __restrict__ w_out,
                                            double* __restrict__ rho_out, double* __restrict__ ex_out,
                                            double* __restrict__ th_out, double* __restrict__ cpv,
                                            double* __restrict__ dpv, double* __restrict__ drxv,
                                            double* __restrict__ dxxv, StepCoef cf) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.nc) return;
  const int K = g.K, cs = g.cs;
  int ie[3], nb[3];
  double kd[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    ie[i] = g.c2e[i * cs + c];
    nb[i] = g.c2e2c[i * cs + c];
    kd[i] = g.kdiv[i * cs + c];
  }
  const double* idzf = vt_row(g, VT_IDZF);
  const double* idzh = vt_row(g, VT_IDZH);
  const double* exref = vt_row(g, VT_EXREF);
  const double* thref = vt_row(g, VT_THREF);
  const double* thric = vt_row(g, VT_THREFIC);
  const double* dxric = vt_row(g, VT_DEXREFIC);
  const double eta = cf.eta, dtau = cf.dtau, cpd = cf.cpd;
  const double oneme = 1.0 - eta;

  // sliding window: full levels j (cur) and j+1 (nxt); half levels j and j+1
  double rho_c = rho[c], th_c = th[c], ex_c = ex[c];
  double thp_c = th_c - thref[0], exp_c = ex_c - exref[0];
  double ric_c = rho_c, atil_c = 0.0;  // half level 0
  double gam_c = 0.0, zth_c = 0.0;     // half level 0 (unused)
  double w_c = w[c];
  double beta_p = 0.0, e_p = 0.0, aeta_p = 0.0;  // full level j-1 / half level j-1
  double cp_p = 0.0, dp_p = 0.0;
  for (int j = 0; j < K; ++j) {
    // half level j+1
    double rho_n = 0.0, th_n = 0.0, ex_n = 0.0, thp_n = 0.0, exp_n = 0.0;
    double ric_n, atil_n, gam_n = 0.0, zth_n = 0.0;
    if (j + 1 < K) {
      const size_t r = (size_t)(j + 1) * cs + c;
      rho_n = rho[r];
      th_n = th[r];
      ex_n = ex[r];
      thp_n = th_n - thref[j + 1];
      exp_n = ex_n - exref[j + 1];
      ric_n = 0.5 * (rho_c + rho_n);
      const double thp_ic = 0.5 * (thp_c + thp_n);
      const double th_ic = thric[j + 1] + thp_ic;
      atil_n = th_ic * ric_n;
      gam_n = dtau * cpd * eta * th_ic * idzh[j + 1];
      zth_n = oneme * th_ic * (exp_c - exp_n) * idzh[j + 1] + thp_ic * dxric[j + 1];
    } else {
      ric_n = rho_c;
      atil_n = 0.0;
    }
    const double w_n = w[(size_t)(j + 1) * cs + c];
    // flux divergences at full level j
    const R* vr = vnf + (size_t)j * g.es;
    const double* rr = rho + (size_t)j * cs;
    const double* tr = th + (size_t)j * cs;
    double dm = 0.0, dth = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const R rho_e = (R)(0.5 * (rho_c + rr[nb[i]]));
      const R th_e = (R)(0.5 * (th_c + tr[nb[i]]));
      const R fm = rho_e * vr[ie[i]];
      const R ft = fm * th_e;
      dm += kd[i] * (double)fm;
      dth += kd[i] * (double)ft;
    }
    const double b = dtau * cf.rd_cvd * ex_c / (rho_c * th_c);
    const double beta = b * idzf[j];
    const double drx = -dtau * (dm + oneme * (ric_c * w_c - ric_n * w_n) * idzf[j]);
    const double dxx = -b * (dth + oneme * (atil_c * w_c - atil_n * w_n) * idzf[j]);
    const double e_c = exp_c + dxx;
    if (CORR) {
      drxv[(size_t)j * cs + c] = drx;
      dxxv[(size_t)j * cs + c] = dxx;
    }
    const double aeta_c = eta * atil_c, aeta_n = eta * atil_n;
    if (j >= 1) {
      // row of half level j
      double tw = (double)tw0[(size_t)j * cs + c];
      if (CORR) tw = cf.a0 * tw + cf.a1 * (double)tw1[(size_t)j * cs + c];
      const double wx = w_c + dtau * (tw - cpd * zth_c);
      const double A = -gam_c * beta_p * aeta_p;
      const double B = 1.0 + gam_c * aeta_c * (beta_p + beta);
      const double C = -gam_c * beta * aeta_n;
      const double rhs = wx - gam_c * (e_p - e_c);
      const double den = B - A * cp_p;
      const double cpk = C / den;
      const double dpk = (rhs - A * dp_p) / den;
      cpv[(size_t)j * cs + c] = cpk;
      dpv[(size_t)j * cs + c] = dpk;
      cp_p = cpk;
      dp_p = dpk;
    }
    // shift the window
    beta_p = beta;
    e_p = e_c;
    aeta_p = aeta_c;
    rho_c = rho_n;
    th_c = th_n;
    ex_c = ex_n;
    thp_c = thp_n;
    exp_c = exp_n;
    ric_c = ric_n;
    atil_c = atil_n;
    gam_c = gam_n;
    zth_c = zth_n;
    w_c = w_n;
  }
  // back substitution, sponge; corrector: increment updates level by level
  const double* tau = g.tau;
  w_out[(size_t)K * cs + c] = 0.0;
  double x_n = 0.0;    // undamped solution at half level k+1
  double ws_n = 0.0;   // damped w at half level k+1
  // window for the corrector updates (full level k and half levels k, k+1)
  double rho_k = 0.0, th_k = 0.0, ex_k = 0.0, thp_k = 0.0;
  double ric_kn = 0.0, atil_kn = 0.0;  // half level k+1
  if (CORR) {
    const size_t r = (size_t)(K - 1) * cs + c;
    rho_k = rho[r];
    th_k = th[r];
    ex_k = ex[r];
    thp_k = th_k - thref[K - 1];
    ric_kn = rho_k;
    atil_kn = 0.0;
  }
  for (int k = K - 1; k >= 0; --k) {
    double ws_k = 0.0;
    if (k >= 1) {
      const double x = dpv[(size_t)k * cs + c] - cpv[(size_t)k * cs + c] * x_n;
      x_n = x;
      ws_k = x / (1.0 + dtau * tau[k]);
    }
    w_out[(size_t)k * cs + c] = ws_k;
    if (CORR) {
      // half level k quantities need full level k-1
      double rho_m = 0.0, th_m = 0.0, thp_m = 0.0, ric_k, atil_k;
      if (k >= 1) {
        const size_t r = (size_t)(k - 1) * cs + c;
        rho_m = rho[r];
        th_m = th[r];
        thp_m = th_m - thref[k - 1];
        ric_k = 0.5 * (rho_m + rho_k);
        atil_k = (thric[k] + 0.5 * (thp_m + thp_k)) * ric_k;
      } else {
        ric_k = rho_k;
        atil_k = 0.0;
      }
      const size_t r = (size_t)k * cs + c;
      const double b = dtau * cf.rd_cvd * ex_k / (rho_k * th_k);
      const double beta = b * idzf[k];
      const double drho = drxv[r] - dtau * eta * (ric_k * ws_k - ric_kn * ws_n) * idzf[k];
      const double dex = dxxv[r] - beta * (eta * atil_k * ws_k - eta * atil_kn * ws_n);
      const double rho_new = rho_k + drho;
      rho_out[r] = rho_new;
      ex_out[r] = ex_k + dex;
      th_out[r] = th_k + (rho_k * th_k * cf.cvd_rd * dex / ex_k - th_k * drho) / rho_new;
      rho_k = rho_m;
      th_k = th_m;
      thp_k = thp_m;
      if (k >= 1) ex_k = ex[(size_t)(k - 1) * cs + c];
      ric_kn = ric_k;
      atil_kn = atil_k;
    }
    ws_n = ws_k;
  }
}

// ---------------------------------------------------------------------------
// diffusion
// ---------------------------------------------------------------------------
// vertex: least-squares vertex vector V_v (3 components) and vorticity.
template <typename R>
__global__ void __launch_bounds__(256) k_dvert(DevGrid g, const R* __restrict__ vn, R* __restrict__ vv,
                                               R* __restrict__ zeta, int kb) {
  int bx, by;
  tile_coords(bx, by);
  const int v = bx * blockDim.x + threadIdx.x;
  if (v >= g.nv) return;
  int idx[6];
  R cc[6], lw[3][6];
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    idx[s] = g.v2e[s * g.vs + v];
    cc[s] = (R)g.kcurl[s * g.vs + v];
#pragma unroll
    for (int j = 0; j < 3; ++j) lw[j][s] = (R)g.klsq[(j * 6 + s) * g.vs + v];
  }
  const size_t plane = (size_t)g.K * g.vs;
  const int k0 = by * kb, k1 = min(g.K, k0 + kb);
  for (int k = k0; k < k1; ++k) {
    const R* row = vn + (size_t)k * g.es;
    R x[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) x[s] = row[idx[s]];
    R z = R(0), a = R(0), b = R(0), d = R(0);
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      z += cc[s] * x[s];
      a += lw[0][s] * x[s];
      b += lw[1][s] * x[s];
      d += lw[2][s] * x[s];
    }
    const size_t o = (size_t)k * g.vs + v;
    zeta[o] = z;
    vv[o] = a;
    vv[plane + o] = b;
    vv[2 * plane + o] = d;
  }
}

// cell: divergence of an edge field (first pass: div vn)
template <typename R>
__global__ void __launch_bounds__(256) k_div(DevGrid g, const R* __restrict__ f, R* __restrict__ out, int kb) {
  int bx, by;
  tile_coords(bx, by);
  const int c = bx * blockDim.x + threadIdx.x;
  if (c >= g.nc) return;
  int ie[3];
  R kd[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    ie[i] = g.c2e[i * g.cs + c];
    kd[i] = (R)g.kdiv[i * g.cs + c];
  }
  const int k0 = by * kb, k1 = min(g.K, k0 + kb);
  for (int k = k0; k < k1; ++k) {
    const R* row = f + (size_t)k * g.es;
    out[(size_t)k * g.cs + c] = kd[0] * row[ie[0]] + kd[1] * row[ie[1]] + kd[2] * row[ie[2]];
  }
}

// edge: L1 = grad(div vn) - gradt(curl vn) and the Smagorinsky viscosity
// from the rhombus deformation of the vertex vectors.
template <typename R>
__global__ void __launch_bounds__(256) k_dedge1(DevGrid g, const R* __restrict__ dv, const R* __restrict__ zeta,
                                                const R* __restrict__ vv, R* __restrict__ l1, R* __restrict__ nu,
                                                StepCoef cf, int kb) {
  int bx, by;
  tile_coords(bx, by);
  const int e = bx * blockDim.x + threadIdx.x;
  if (e >= g.ne) return;
  const int c0 = g.e2c[e], c1 = g.e2c[g.es + e];
  int rv[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) rv[i] = g.e2c2v[i * g.es + e];
  const R invd = (R)g.invd[e], invl = (R)g.invl[e], invlr = (R)g.invlr[e];
  const R n0 = (R)g.nrm[e], n1 = (R)g.nrm[g.es + e], n2 = (R)g.nrm[2 * g.es + e];
  const R t0 = (R)g.tan[e], t1 = (R)g.tan[g.es + e], t2 = (R)g.tan[2 * g.es + e];
  const double ae = g.ae[e];
  const R smag = (R)(cf.cs * ae);
  const R cap = (R)(ae / (cf.cap * cf.dt));
  const size_t plane = (size_t)g.K * g.vs;
  const int k0 = by * kb, k1 = min(g.K, k0 + kb);
  for (int k = k0; k < k1; ++k) {
    const R* dr = dv + (size_t)k * g.cs;
    const R* zr = zeta + (size_t)k * g.vs;
    l1[(size_t)k * g.es + e] = (dr[c1] - dr[c0]) * invd - (zr[rv[1]] - zr[rv[0]]) * invl;
    const R* vx = vv + (size_t)k * g.vs;
    const R* vy = vx + plane;
    const R* vz = vy + plane;
    const R tx = vx[rv[1]] - vx[rv[0]], ty = vy[rv[1]] - vy[rv[0]], tz = vz[rv[1]] - vz[rv[0]];
    const R nx = vx[rv[3]] - vx[rv[2]], ny = vy[rv[3]] - vy[rv[2]], nz = vz[rv[3]] - vz[rv[2]];
    const R dvn_dt = (tx * n0 + ty * n1 + tz * n2) * invl;
    const R dvt_dt = (tx * t0 + ty * t1 + tz * t2) * invl;
    const R dvn_dn = (nx * n0 + ny * n1 + nz * n2) * invlr;
    const R dvt_dn = (nx * t0 + ny * t1 + nz * t2) * invlr;
    const R a = dvn_dn - dvt_dt, b = dvt_dn + dvn_dt;
    const R def = sqrt(a * a + b * b);
    nu[(size_t)k * g.es + e] = fmin(smag * def, cap);
  }
}

// cell + vertex (one launch): div(L1) at cells, curl(L1) at vertices, and the
// Smagorinsky diffusion of w at cells (reads w_in, writes w_out).
template <typename R>
__global__ void __launch_bounds__(256) k_dcv2(DevGrid g, const R* __restrict__ l1, const R* __restrict__ nu,
                                              const double* __restrict__ w_in, double* __restrict__ w_out,
                                              R* __restrict__ divl1, R* __restrict__ curll1, int ncb, StepCoef cf,
                                              int kb) {
  int bx, by;
  tile_coords(bx, by);
  const int K = g.K;
  if (bx < ncb) {
    const int c = bx * blockDim.x + threadIdx.x;
    if (c >= g.nc) return;
    int ie[3], nb[3];
    R kd[3];
    double kl[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      ie[i] = g.c2e[i * g.cs + c];
      nb[i] = g.c2e2c[i * g.cs + c];
      kd[i] = (R)g.kdiv[i * g.cs + c];
      kl[i] = g.klap[i * g.cs + c];
    }
    const int k0 = by * kb, k1 = min(K + 1, k0 + kb);
    for (int k = k0; k < k1; ++k) {
      if (k < K) {
        const R* row = l1 + (size_t)k * g.es;
        divl1[(size_t)k * g.cs + c] = kd[0] * row[ie[0]] + kd[1] * row[ie[1]] + kd[2] * row[ie[2]];
      }
      const size_t r = (size_t)k * g.cs + c;
      double wn = w_in[r];
      if (cf.diffuse_w && k >= 1 && k <= K - 1) {
        const R* na = nu + (size_t)(k - 1) * g.es;
        const R* nbr = nu + (size_t)k * g.es;
        R nuc = R(0);
#pragma unroll
        for (int i = 0; i < 3; ++i) nuc += R(0.5) * (na[ie[i]] + nbr[ie[i]]);
        nuc = nuc / R(3);
        const double* wr = w_in + (size_t)k * g.cs;
        double lw = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) lw += kl[i] * (wr[nb[i]] - wn);
        wn = wn + cf.dt * (double)nuc * lw;
      }
      w_out[r] = wn;
    }
  } else {
    const int v = (bx - ncb) * blockDim.x + threadIdx.x;
    if (v >= g.nv) return;
    int idx[6];
    R cc[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      idx[s] = g.v2e[s * g.vs + v];
      cc[s] = (R)g.kcurl[s * g.vs + v];
    }
    const int k0 = by * kb, k1 = min(K, k0 + kb);
    for (int k = k0; k < k1; ++k) {
      const R* row = l1 + (size_t)k * g.es;
      R z = cc[0] * row[idx[0]];
#pragma unroll
      for (int s = 1; s < 6; ++s) z += cc[s] * row[idx[s]];
      curll1[(size_t)k * g.vs + v] = z;
    }
  }
}

// edge: L2 = lapv(L1) and vn += dt nu L1 - k4 A_e^2 L2 (in place).
template <typename R>
__global__ void __launch_bounds__(256) k_dedge2(DevGrid g, R* __restrict__ vn, const R* __restrict__ l1,
                                                const R* __restrict__ nu, const R* __restrict__ divl1,
                                                const R* __restrict__ curll1, StepCoef cf, int kb) {
  int bx, by;
  tile_coords(bx, by);
  const int e = bx * blockDim.x + threadIdx.x;
  if (e >= g.ne) return;
  const int c0 = g.e2c[e], c1 = g.e2c[g.es + e];
  const int v0 = g.e2v[e], v1 = g.e2v[g.es + e];
  const R invd = (R)g.invd[e], invl = (R)g.invl[e];
  const double ae = g.ae[e];
  const R k4a2 = (R)(cf.k4 * ae * ae);
  const R dt = (R)cf.dt;
  const int k0 = by * kb, k1 = min(g.K, k0 + kb);
  for (int k = k0; k < k1; ++k) {
    const R* dr = divl1 + (size_t)k * g.cs;
    const R* zr = curll1 + (size_t)k * g.vs;
    const R l2 = (dr[c1] - dr[c0]) * invd - (zr[v1] - zr[v0]) * invl;
    const size_t r = (size_t)k * g.es + e;
    vn[r] = vn[r] + dt * nu[r] * l1[r] - k4a2 * l2;
  }
}

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

inline dim3 grid2(int n, int levels, const Tile& t) {
  const int nbx = (n + t.threads - 1) / t.threads;
  const int nby = (levels + t.kb - 1) / t.kb;
  return dim3(nbx, nby);
}

}  // namespace

const char* const kKernelNames[K_COUNT] = {
    "curl_pred", "vt_pred", "cell_adv_pred", "edge_pred", "column_pred",
    "curl_corr", "vt_corr", "cell_adv_corr", "edge_corr", "column_corr",
    "diff_vertex", "diff_div", "diff_edge1", "diff_cell_vertex2", "diff_edge2"};

#define LAUNCH(id, ...)                     \
  do {                                      \
    if (prof) prof->mark(s, id);            \
    __VA_ARGS__;                            \
    if (prof) prof->mark(s, -1);            \
  } while (0)

int diag_partial_count(const DevGrid& g) {
  return (g.nc + kDiagThreads - 1) / kDiagThreads + (g.ne + kDiagThreads - 1) / kDiagThreads;
}

template <typename R>
void launch_substep(const DevGrid& g, const Bufs<R>& b, const StepCoef& c, const Tile* T, hipStream_t s, Prof* prof) {
  const int K = g.K;
  // predictor: advective tendencies at the substep start, momentum, column
  LAUNCH(K_CURL_P, k_curl<R><<<grid2(g.nv, K, T[T_CURL]), T[T_CURL].threads, 0, s>>>(g, b.vn, b.zeta, T[T_CURL].kb));
  LAUNCH(K_VT_P, k_vt<R><<<grid2(g.ne, K, T[T_VT]), T[T_VT].threads, 0, s>>>(g, b.vn, b.vt, T[T_VT].kb));
  LAUNCH(K_CELL_P, k_cell_adv<R, false><<<grid2(g.nc, K + 1, T[T_CELLADV]), T[T_CELLADV].threads, 0, s>>>(
                       g, b.vn, b.vt, b.w, b.kc, b.tw0, nullptr, T[T_CELLADV].kb));
  LAUNCH(K_EDGE_P, k_edge<R, false><<<grid2(g.ne, K, T[T_EDGE]), T[T_EDGE].threads, 0, s>>>(
                       g, b.vn, b.vt, b.zeta, b.kc, b.w, b.ex, b.th, b.tvn0, b.vns, nullptr, nullptr, c, T[T_EDGE].kb));
  const int ncol = (g.nc + T[T_COL].threads - 1) / T[T_COL].threads;
  LAUNCH(K_COL_P, k_col<R, false><<<ncol, T[T_COL].threads, 0, s>>>(g, b.w, b.rho, b.ex, b.th, b.vns, b.tw0, nullptr,
                                                                      b.ws, nullptr, nullptr, nullptr, b.cp, b.dp,
                                                                      nullptr, nullptr, c));
  // corrector: tendencies at the predicted state, damping, momentum, column
  LAUNCH(K_CURL_C, k_curl<R><<<grid2(g.nv, K, T[T_CURL]), T[T_CURL].threads, 0, s>>>(g, b.vns, b.zeta, T[T_CURL].kb));
  LAUNCH(K_VT_C, k_vt<R><<<grid2(g.ne, K, T[T_VT]), T[T_VT].threads, 0, s>>>(g, b.vns, b.vt, T[T_VT].kb));
  LAUNCH(K_CELL_C, k_cell_adv<R, true><<<grid2(g.nc, K + 1, T[T_CELLADV]), T[T_CELLADV].threads, 0, s>>>(
                       g, b.vns, b.vt, b.ws, b.kc, b.tw1, b.d2, T[T_CELLADV].kb));
  LAUNCH(K_EDGE_C, k_edge<R, true><<<grid2(g.ne, K, T[T_EDGE]), T[T_EDGE].threads, 0, s>>>(
                       g, b.vns, b.vt, b.zeta, b.kc, b.ws, b.ex, b.th, b.tvn0, b.vn_out, b.vn, b.d2, c, T[T_EDGE].kb));
  LAUNCH(K_COL_C, k_col<R, true><<<ncol, T[T_COL].threads, 0, s>>>(g, b.w, b.rho, b.ex, b.th, b.vn_out, b.tw0, b.tw1,
                                                                     b.w_out, b.rho_out, b.ex_out, b.th_out, b.cp, b.dp,
                                                                     b.drx, b.dxx, c));
}

template <typename R>
void launch_diffusion(const DevGrid& g, R* vn, const double* w_in, double* w_out, R* l1, R* nu, R* dv, R* dl1,
                      R* zeta, R* vv, const StepCoef& c, const Tile* T, hipStream_t s, Prof* prof) {
  const int K = g.K;
  LAUNCH(K_DVERT, k_dvert<R><<<grid2(g.nv, K, T[T_DVERT]), T[T_DVERT].threads, 0, s>>>(g, vn, vv, zeta, T[T_DVERT].kb));
  LAUNCH(K_DDIV, k_div<R><<<grid2(g.nc, K, T[T_DCELL]), T[T_DCELL].threads, 0, s>>>(g, vn, dv, T[T_DCELL].kb));
  LAUNCH(K_DEDGE1, k_dedge1<R><<<grid2(g.ne, K, T[T_DEDGE]), T[T_DEDGE].threads, 0, s>>>(g, dv, zeta, vv, l1, nu, c,
                                                                                         T[T_DEDGE].kb));
  // cells (K+1 half levels for w) and vertices share one launch
  const Tile& t = T[T_DCELL];
  const int ncb = (g.nc + t.threads - 1) / t.threads;
  const int nvb = (g.nv + t.threads - 1) / t.threads;
  const dim3 gr(ncb + nvb, (K + 1 + t.kb - 1) / t.kb);
  LAUNCH(K_DCV2, k_dcv2<R><<<gr, t.threads, 0, s>>>(g, l1, nu, w_in, w_out, dl1, zeta, ncb, c, t.kb));
  LAUNCH(K_DEDGE2, k_dedge2<R><<<grid2(g.ne, K, T[T_DEDGE]), T[T_DEDGE].threads, 0, s>>>(g, vn, l1, nu, dl1, zeta, c,
                                                                                         T[T_DEDGE].kb));
}

template <typename R>
void launch_diag(const DevGrid& g, const R* vn, const double* w, const double* rho, const double* th,
                 const double* ex, double* partial, double* out, hipStream_t s) {
  const int ncb = (g.nc + kDiagThreads - 1) / kDiagThreads;
  const int neb = (g.ne + kDiagThreads - 1) / kDiagThreads;
  k_diag<R><<<ncb + neb, kDiagThreads, 0, s>>>(g, vn, w, rho, th, ex, partial, ncb);
  k_diag_final<<<1, kDiagThreads, 0, s>>>(partial, ncb + neb, out);
}

template void launch_substep<double>(const DevGrid&, const Bufs<double>&, const StepCoef&, const Tile*, hipStream_t,
                                     Prof*);
template void launch_substep<float>(const DevGrid&, const Bufs<float>&, const StepCoef&, const Tile*, hipStream_t,
                                    Prof*);
template void launch_diffusion<double>(const DevGrid&, double*, const double*, double*, double*, double*, double*,
                                       double*, double*, double*, const StepCoef&, const Tile*, hipStream_t, Prof*);
template void launch_diffusion<float>(const DevGrid&, float*, const double*, double*, float*, float*, float*, float*,
                                      float*, float*, const StepCoef&, const Tile*, hipStream_t, Prof*);
template void launch_diag<double>(const DevGrid&, const double*, const double*, const double*, const double*,
                                  const double*, double*, double*, hipStream_t);
template void launch_diag<float>(const DevGrid&, const float*, const double*, const double*, const double*,
                                 const double*, double*, double*, hipStream_t);

}  // namespace dc
