// Device bodies of the dycore kernels, shared by the single-state launches
// (kernels.hip) and the batched ensemble launches (ensemble.hip).
//
// Layout: every field is [level][entity], entity index fastest, each level
// padded to a multiple of 64 entities; a thread owns one entity and walks a
// block of levels, so the neighbour indices and stencil weights are loaded
// once per thread and every level access of the own entity is a coalesced
// 64-wide row.  Gathers go through the lookup tables (paper, Section 4.2.1).
// Single-state launches remap blocks so that the 8 XCDs each sweep a
// contiguous range of tiles (neighbour halos then mostly hit one XCD's L2);
// bodies with kXcdRanges = false keep the hardware's round-robin order
// instead (the vorticity, edge and cell-vertex diffusion passes, whose edge
// and vertex tiles read the same rows and run faster when every XCD works
// on every part of the grid at once).
//
// Template parameter R is the type of vn and of the horizontal-stencil
// intermediates: double for the FP64 path, float for the mixed path.  The
// column solver, w/rho/exner/theta_v and flux-divergence sums are always
// FP64.  No floating-point atomics: results do not depend on the launch
// geometry, so tuned and batched launches give bit-identical results.
//
// Each body is a struct with an Args type (its pointers and scalars),
// kThreads (the largest block it is compiled for) and a device function
// run(grid, args, bx, by) for one tile.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "internal.h"
#include "kernels.h"

namespace dc {
namespace bodies {


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
// Tangential wind at edge e by Perot reconstruction: a 5-point stencil over
// the edge and its four e2c2e neighbours (weights precomputed on the host).
// ---------------------------------------------------------------------------
template <typename R>
struct VtStencil {
  int idx[4];
  R w[5];
  __device__ __forceinline__ void load(const DevGrid& g, int e) {
    w[0] = (R)g.kvt[e];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      idx[s] = g.e2c2e[s * g.es + e];
      w[1 + s] = (R)g.kvt[(1 + s) * g.es + e];
    }
  }
  __device__ __forceinline__ R apply(const R* __restrict__ row, int e) const {
    R acc = w[0] * row[e];
#pragma unroll
    for (int s = 0; s < 4; ++s) acc += w[1 + s] * row[idx[s]];
    return acc;
  }
};

// ---------------------------------------------------------------------------
// edge + vertex (+ cell) pass, one launch: blocks [0, neb) are edges, the
// next nvb blocks vertices, and in the corrector the rest cells.
//  edges:    tangential wind vt (Perot) and kinetic energy K_e = (vn^2 + vt^2)/2
//  vertices: relative vorticity zeta_v = (1/A_v) sum sig d_e vn_e
//  cells:    (corrector) the divergence-damping field D2 = laps(D) from
//            D = div vn*, which the predictor's column kernel stored.
// The cell kinetic energy K_c = mean of K_e over the cell's edges is not
// stored: the edge kernel forms grad K_c from K_e of the rhombus edges.
// ---------------------------------------------------------------------------
template <typename R, bool CORR>
struct BVc {
  using Real = R;
  struct Args {
    const R* vn;
    R* zeta;
    R* vt;
    R* ke;
    R* d2;
    const R* dv;  // corrector: D = div vn*
    int neb, nvb;
    int kb;
  };
  static constexpr bool kXcdRanges = false;  // round-robin tile order (see the top of this file)
  static constexpr int kThreads = 256;
  __device__ static void run(const DevGrid& g, const Args& args, int bx, int by) {
    const R* __restrict__ vn = args.vn;
    const int kb = args.kb;
    const int k0 = by * kb, k1 = min(g.K, k0 + kb);
    if (bx < args.neb) {
      // the block's own vn row goes through LDS (double-buffered by level
      // parity, one barrier per level); the four neighbour edges of the vt
      // stencil that lie in the block (~87 % for 256 edges) are read there.
      // Every thread reaches every barrier.
      __shared__ R s_row[2][kThreads];
      const int base = bx * blockDim.x;
      const int e = base + threadIdx.x;
      const bool in = e < g.ne;
      R* __restrict__ vt = args.vt;
      R* __restrict__ ke = args.ke;
      VtStencil<R> vts;
      if (in) vts.load(g, e);
      for (int k = k0; k < k1; ++k) {
        const R* row = vn + (size_t)k * g.es;
        const R a = in ? row[e] : R(0);
        s_row[k & 1][threadIdx.x] = a;
        __syncthreads();
        if (in) {
          R b = vts.w[0] * a;
  #pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int l = vts.idx[q] - base;
            R x = s_row[k & 1][l & (kThreads - 1)];
            x = (unsigned)l < (unsigned)blockDim.x ? x : row[vts.idx[q]];
            b += vts.w[1 + q] * x;
          }
          const size_t r = (size_t)k * g.es + e;
          vt[r] = b;
          ke[r] = R(0.5) * (a * a + b * b);
        }
      }
      __syncthreads();  // the next tile of a persistent block reuses s_row
      return;
    }
    if (bx < args.neb + args.nvb) {
      R* __restrict__ zeta = args.zeta;
      const int v = (bx - args.neb) * blockDim.x + threadIdx.x;
      if (v >= g.nv) return;
      int idx[6];
      R cf[6];
  #pragma unroll
      for (int s = 0; s < 6; ++s) {
        idx[s] = g.v2e[s * g.vs + v];
        cf[s] = (R)g.kcurl[s * g.vs + v];
      }
      for (int k = k0; k < k1; ++k) {
        const R* row = vn + (size_t)k * g.es;
        R acc = cf[0] * row[idx[0]];
  #pragma unroll
        for (int s = 1; s < 6; ++s) acc += cf[s] * row[idx[s]];
        zeta[(size_t)k * g.vs + v] = acc;
      }
      return;
    }
    if (CORR) {
      R* __restrict__ d2 = args.d2;
      const int c = (bx - args.neb - args.nvb) * blockDim.x + threadIdx.x;
      if (c >= g.nc) return;
      int nb[3];
      R kl[3];
  #pragma unroll
      for (int i = 0; i < 3; ++i) {
        nb[i] = g.c2e2c[i * g.cs + c];
        kl[i] = (R)g.klap[i * g.cs + c];
      }
      for (int k = k0; k < k1; ++k) {
        const R* drow = args.dv + (size_t)k * g.cs;
        const R dc = drow[c];
        R acc = R(0);
  #pragma unroll
        for (int i = 0; i < 3; ++i) acc += kl[i] * (drow[nb[i]] - dc);
        d2[(size_t)k * g.cs + c] = acc;
      }
    }
  }
};

// ---------------------------------------------------------------------------
// edge (option): rho and theta_v at the edges by second-order upwind (Miura)
// reconstruction from the state at the start of the substep and its winds
// vn, vt: q_e = q_up + sum_i w_i (q_i - q_up) over the upwind cell's three
// neighbours, w_i = a_i - dtau (vn b_i + vt c_i) from the host's per-edge,
// per-side coefficients (the least-squares gradient dotted with the offset
// from the upwind cell centre to the departure point of the edge midpoint).
// In FP64 in both forms; stored for the edge and column kernels of both
// passes.
// ---------------------------------------------------------------------------
template <typename R>
struct BMiura {
  using Real = R;
  struct Args {
    const R* vn;
    const double* rho;
    const double* th;
    double* rhoe;
    double* the;
    double dtau;
    int kb;
  };
  static constexpr int kThreads = 256;
  __device__ static void run(const DevGrid& g, const Args& args, int bx, int by) {
    const int e = bx * blockDim.x + threadIdx.x;
    if (e >= g.ne) return;
    const R* __restrict__ vn = args.vn;
    const double* __restrict__ rho = args.rho;
    const double* __restrict__ th = args.th;
    double* __restrict__ rhoe = args.rhoe;
    double* __restrict__ the = args.the;
    int cu[2], nb[2][3];
    double ca[2][3], cb[2][3], cc[2][3];
  #pragma unroll
    for (int s = 0; s < 2; ++s) {
      cu[s] = g.e2c[s * g.es + e];
  #pragma unroll
      for (int i = 0; i < 3; ++i) {
        nb[s][i] = g.c2e2c[i * g.cs + cu[s]];
        ca[s][i] = g.kmiura[(9 * s + i) * g.es + e];
        cb[s][i] = g.kmiura[(9 * s + 3 + i) * g.es + e];
        cc[s][i] = g.kmiura[(9 * s + 6 + i) * g.es + e];
      }
    }
    VtStencil<R> vts;  // vt of the start vn, formed here
    vts.load(g, e);
    const double dtau = args.dtau;
    const int kb = args.kb;
    const int k0 = by * kb, k1 = min(g.K, k0 + kb);
    for (int k = k0; k < k1; ++k) {
      const size_t re = (size_t)k * g.es + e;
      const double v = (double)vn[re], t = (double)vts.apply(vn + (size_t)k * g.es, e);
      const bool s0 = v >= 0.0;  // the normal points c0 -> c1: c0 is upwind
      const int up = s0 ? cu[0] : cu[1];
      const double* rr = rho + (size_t)k * g.cs;
      const double* tr = th + (size_t)k * g.cs;
      const double r0 = rr[up], t0 = tr[up];
      double ra = r0, ta = t0;
  #pragma unroll
      for (int i = 0; i < 3; ++i) {
        const int n = s0 ? nb[0][i] : nb[1][i];
        const double w = (s0 ? ca[0][i] : ca[1][i]) - dtau * (v * (s0 ? cb[0][i] : cb[1][i]) + t * (s0 ? cc[0][i] : cc[1][i]));
        ra += w * (rr[n] - r0);
        ta += w * (tr[n] - t0);
      }
      rhoe[re] = ra;
      the[re] = ta;
    }
  }
};

// ---------------------------------------------------------------------------
// edge: advective tendency T_vn and the horizontal momentum update.
//  predictor: vn* = vn + dtau (T_vn - cpd theta_e grad pi')       -> vns, and
//             Y = vn + dtau (a0 T_vn - cpd theta_e grad pi')        -> tvn0
//  corrector: vn' = Y + (dtau a1 T* - c4 Abar^2 grad(D2))          -> vn_out
// The pressure-gradient term is formed from the state at the start of the
// substep in both passes.
// ---------------------------------------------------------------------------
template <typename R, bool CORR>
struct BEdge {
  using Real = R;
  struct Args {
    const R* vn;
    const R* zeta;
    const R* ke;  // K_e of this pass's vn
    const R* vt;  // vt of this pass's vn
    const double* w;
    const double* ex;
    const double* th;
    R* tvn0;
    R* vout;
    const R* d2;
    R* gw;  // out: l_e vn_ie (w_c1 - w_c0) at the half levels 1..K-1
    const double* the;  // Miura theta_v at the edges (option; predictor)
    StepCoef cf;
    int kb;
  };
  static constexpr bool kXcdRanges = false;  // round-robin tile order (see the top of this file)
  static constexpr int kThreads = EdgeTiles::kTileE;
  // LDS of the fused form: per level parity, vn of the staged edges, vt and
  // K_e of the tile and its rhombus edges, vorticity at the tile's vertices
  static constexpr int kBuf = EdgeTiles::XM + 2 * EdgeTiles::XV + EdgeTiles::VM;
  static constexpr size_t kSmem = 2 * kBuf * sizeof(R);

  // per-edge constants of the edge a thread owns
  struct Own {
    int e, c0, c1;
    bool in;
    R invd_r, fe, le;
  };
  __device__ __forceinline__ static Own own(const DevGrid& g, int e, bool in) {
    Own o;
    o.e = e;
    o.in = in;
    o.c0 = g.e2c[e];
    o.c1 = g.e2c[g.es + e];
    o.invd_r = (R)g.invd[e];
    o.fe = (R)g.fe[e];
    o.le = (R)(1.0 / g.invl[e]);
    return o;
  }

  // Cell and edge values of the momentum update at level j: the predictor's
  // exner and theta_v at c0, c1 (with the Miura option theta_v at the edge
  // in t0), the corrector's damping field at c0, c1 and its stored Y.
  struct EdgeIn {
    double x0, x1, t0, t1;
    R d0, d1, y;
  };
  __device__ __forceinline__ static EdgeIn edge_in(const DevGrid& g, const StepCoef& cf, const Own& o, int j,
                                                   const double* __restrict__ ex, const double* __restrict__ th,
                                                   const double* __restrict__ the_m, const R* __restrict__ d2,
                                                   const R* __restrict__ tvn0) {
    EdgeIn v{};
    const size_t rc = (size_t)j * g.cs, re = (size_t)j * g.es + o.e;
    if (!CORR) {
      v.x0 = ex[rc + o.c0];
      v.x1 = ex[rc + o.c1];
      if (cf.miura) {
        v.t0 = the_m[re];
      } else {
        v.t0 = th[rc + o.c0];
        v.t1 = th[rc + o.c1];
      }
    } else {
      v.d0 = d2[rc + o.c0];
      v.d1 = d2[rc + o.c1];
      v.y = tvn0[re];
    }
    return v;
  }

  // The edge's work at full level j from vn at j - 1, j, j + 1, w at c0, c1
  // on half levels j and j + 1, the vorticity at the edge, the K_e of its
  // four rhombus edges, its vt and the values of edge_in.
  // The fields are restrict parameters: no buffer is both read and written
  // by one launch, so loads of later levels may move above earlier stores.
  __device__ __forceinline__ static void level(const DevGrid& g, const StepCoef& cf, const Own& o, int j, R vup,
                                               R vj, R vdn, double wa0, double wa1, double wb0, double wb1, R ze,
                                               const R kq[4], R vt, const EdgeIn& in_v, R* __restrict__ gw,
                                               R* __restrict__ tvn0, R* __restrict__ vout) {
    const int K = g.K;
    const size_t re = (size_t)j * g.es + o.e;
    const R ie_top = j > 0 ? R(0.5) * (vup + vj) : vj;
    const R ie_bot = j < K - 1 ? R(0.5) * (vj + vdn) : vj;
    // the other two edges of c0, then of c1: K_c1 - K_c0 is a third of the
    // difference of their kinetic energies (the edge's own K_e cancels)
    const R kgrad = ((kq[2] + kq[3]) - (kq[0] + kq[1])) * (R(1) / R(3)) * o.invd_r;
    const R wef = (R)(0.5 * (0.5 * (wa0 + wa1) + 0.5 * (wb0 + wb1)));
    // this edge's share of the horizontal advection of w at half level j:
    // both neighbouring cells take l_e vn_ie (w_c1 - w_c0) / A_c
    if (j > 0 && o.in) gw[re] = o.le * ie_top * (R)(wa1 - wa0);
    const R tvn = (ze + o.fe) * vt - kgrad - wef * (ie_top - ie_bot) * (R)vt_row(g, VT_IDZF)[j];
    if (!CORR) {
      // the pressure-gradient term comes from the substep's start state in
      // both passes: the predictor forms it once and stores the start vn
      // advanced by it and by its share of the tendency,
      // vn + dtau (a0 T_vn0 - cpd theta_e grad pi'), which is all the
      // corrector needs of the three
      const double exr = vt_row(g, VT_EXREF)[j];
      const R gex = (R)((in_v.x1 - exr) - (in_v.x0 - exr)) * o.invd_r;
      const R the = cf.miura ? (R)in_v.t0 : (R)(0.5 * (in_v.t0 + in_v.t1));
      const R pgf = (R)cf.cpd * the * gex;
      if (o.in) {
        tvn0[re] = vj + (R)cf.dtau * ((R)cf.a0 * tvn - pgf);
        vout[re] = vj + (R)cf.dtau * (tvn - pgf);
      }
    } else {
      const R dd = (in_v.d1 - in_v.d0) * o.invd_r;
      if (o.in) vout[re] = in_v.y + ((R)cf.dtau * (R)cf.a1 * tvn - (R)cf.c4a2 * dd);
    }
  }

  __device__ static void run(const DevGrid& g, const Args& args, int bx, int by) {
    if (g.et_ok)
      fused(g, args, bx, by);
    else
      gather(g, args, bx, by);
  }

  // Fused form: the block's tile of kTileE edges stages, at every level, vn of
  // the tile, of its rhombus edges, of their rhombus edges and of the edges
  // around the tile's vertices in LDS (host tables list them), forms vt and
  // K_e on the tile and its rhombus edges and the vorticity at the tile's
  // vertices there, then each thread does its edge's work.  No vt, K_e or
  // vorticity field goes through memory.  Threads past the last edge of the
  // grid do the staging and reach every barrier but store nothing.
  __device__ static void fused(const DevGrid& g, const Args& args, int bx, int by) {
    using T = EdgeTiles;
    extern __shared__ double s_dyn[];
    R* const sb = reinterpret_cast<R*>(s_dyn);
    const R* __restrict__ vn = args.vn;
    const double* __restrict__ w = args.w;
    const int t = bx, tid = threadIdx.x;
    const size_t tt = (size_t)t;
    const int n_own = g.et_n[4 * tt], n_vt = g.et_n[4 * tt + 1], n_ext = g.et_n[4 * tt + 2],
              n_v = g.et_n[4 * tt + 3];
    // staged positions tid, tid + 256, tid + 512 of this thread
    int gx[3];
  #pragma unroll
    for (int r = 0; r < 3; ++r) {
      const int p = tid + r * T::kTileE;
      gx[r] = p < n_ext ? g.et_x[tt * T::XM + p] : -1;
    }
    // vt and K_e at local positions tid and tid + 256 (the vt set is a
    // prefix of the staged set, so its global ids are gx[0], gx[1])
    int nbl[2][4];
    R wv[2][5];
    bool hv[2];
  #pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int l = tid + q * T::kTileE;
      hv[q] = l < n_vt;
      const int ge = hv[q] ? gx[q] : 0;
  #pragma unroll
      for (int s = 0; s < 4; ++s) nbl[q][s] = hv[q] ? (int)g.et_nb[(tt * 4 + s) * T::XV + l] : 0;
  #pragma unroll
      for (int s = 0; s < 5; ++s) wv[q][s] = (R)g.kvt[s * g.es + ge];
    }
    // vorticity at local vertex tid
    const bool hz = tid < n_v;
    int vl[6];
    R kc[6];
    {
      const int gv = hz ? g.et_vx[tt * T::VM + tid] : 0;
  #pragma unroll
      for (int s = 0; s < 6; ++s) {
        vl[s] = hz ? (int)g.et_vl[(tt * 6 + s) * T::VM + tid] : 0;
        kc[s] = (R)g.kcurl[s * g.vs + gv];
      }
    }
    // the own edge (local position tid; its rhombus positions are nbl[0])
    const bool in = tid < n_own;
    const Own o = own(g, in ? t * T::kTileE + tid : 0, in);
    const int lv0 = in ? (int)g.et_ev[(tt * 2) * T::kTileE + tid] : 0;
    const int lv1 = in ? (int)g.et_ev[(tt * 2 + 1) * T::kTileE + tid] : 0;
    const int K = g.K, kb = args.kb;
    const int k0 = by * kb, k1 = min(K, k0 + kb);
    R vup = vn[(size_t)max(k0 - 1, 0) * g.es + o.e];
    double wa0 = w[(size_t)k0 * g.cs + o.c0], wa1 = w[(size_t)k0 * g.cs + o.c1];
    for (int j = k0; j < k1; ++j) {
      R* sv = sb + (j & 1) * kBuf;
      R* svt = sv + T::XM;
      R* ske = svt + T::XV;
      R* sz = ske + T::XV;
      const R* row = vn + (size_t)j * g.es;
      // FP32: every load of the level first and the LDS stores after them
      // (staged positions past the tile's list load edge 0 and fill entries
      // that nothing reads, so neither needs a branch): one memory round
      // trip per level (mixed R2B8 edge_pred -6 %, edge_corr -3 %).  FP64
      // stages under a branch per position, which serialises the staging
      // loads but measured faster (the branch-free form: +5 % and +7 %).
      R st[3];
      if constexpr (sizeof(R) == 4) {
  #pragma unroll
        for (int r = 0; r < 3; ++r) st[r] = row[gx[r] >= 0 ? gx[r] : 0];
      } else {
  #pragma unroll
        for (int r = 0; r < 3; ++r)
          if (gx[r] >= 0) sv[tid + r * T::kTileE] = row[gx[r]];
      }
      // loads that do not wait for the staging
      const size_t re = (size_t)j * g.es + o.e;
      const R vdn = j < K - 1 ? vn[re + g.es] : vn[re];
      const double wb0 = w[(size_t)(j + 1) * g.cs + o.c0], wb1 = w[(size_t)(j + 1) * g.cs + o.c1];
      const EdgeIn in_v = edge_in(g, args.cf, o, j, args.ex, args.th, args.the, args.d2, args.tvn0);
      if constexpr (sizeof(R) == 4) {
  #pragma unroll
        for (int r = 0; r < 3; ++r) sv[tid + r * T::kTileE] = st[r];
      }
      __syncthreads();
  #pragma unroll
      for (int q = 0; q < 2; ++q)
        if (hv[q]) {
          const int l = tid + q * T::kTileE;
          const R a = sv[l];
          R b = wv[q][0] * a;
  #pragma unroll
          for (int s = 0; s < 4; ++s) b += wv[q][1 + s] * sv[nbl[q][s]];
          svt[l] = b;
          ske[l] = R(0.5) * (a * a + b * b);
        }
      if (hz) {
        R z = kc[0] * sv[vl[0]];
  #pragma unroll
        for (int s = 1; s < 6; ++s) z += kc[s] * sv[vl[s]];
        sz[tid] = z;
      }
      __syncthreads();
      const R vj = sv[tid];
      const R ze = R(0.5) * (sz[lv0] + sz[lv1]);
      R kq[4];
  #pragma unroll
      for (int q = 0; q < 4; ++q) kq[q] = ske[nbl[0][q]];
      level(g, args.cf, o, j, vup, vj, vdn, wa0, wa1, wb0, wb1, ze, kq, svt[tid], in_v, args.gw, args.tvn0, args.vout);
      vup = vj;
      wa0 = wb0;
      wa1 = wb1;
    }
    __syncthreads();  // the next tile of a persistent block reuses the LDS
  }

  // Gather form, for grids whose tiles do not fit the fused form's LDS: vt,
  // K_e and the vorticity come from the vorticity pass through memory; the
  // rhombus edges' K_e from the block's row in LDS where they lie in the
  // block.  Threads past the last edge compute edge 0 and store nothing:
  // every thread reaches the per-level barriers.
  __device__ static void gather(const DevGrid& g, const Args& args, int bx, int by) {
    const R* __restrict__ vn = args.vn;
    const R* __restrict__ zeta = args.zeta;
    const R* __restrict__ ke = args.ke;
    const R* __restrict__ vtf = args.vt;
    const double* __restrict__ w = args.w;
    const int base = bx * blockDim.x;
    const bool in = base + (int)threadIdx.x < g.ne;
    const Own o = own(g, in ? base + (int)threadIdx.x : 0, in);
    __shared__ R s_ke[2][kThreads];
    const int v0 = g.e2v[o.e], v1 = g.e2v[g.es + o.e];
    int rh[4];
  #pragma unroll
    for (int s = 0; s < 4; ++s) rh[s] = g.e2c2e[s * g.es + o.e];
    const int K = g.K, kb = args.kb;
    const int k0 = by * kb, k1 = min(K, k0 + kb);
    R vup = vn[(size_t)max(k0 - 1, 0) * g.es + o.e];
    R vj = vn[(size_t)k0 * g.es + o.e];
    double wa0 = w[(size_t)k0 * g.cs + o.c0], wa1 = w[(size_t)k0 * g.cs + o.c1];
    for (int j = k0; j < k1; ++j) {
      const size_t re = (size_t)j * g.es + o.e;
      const R vdn = j < K - 1 ? vn[re + g.es] : vj;
      const double wb0 = w[(size_t)(j + 1) * g.cs + o.c0], wb1 = w[(size_t)(j + 1) * g.cs + o.c1];
      const R* zr = zeta + (size_t)j * g.vs;
      const R ze = R(0.5) * (zr[v0] + zr[v1]);
      const R* kr = ke + (size_t)j * g.es;
      s_ke[j & 1][threadIdx.x] = kr[o.e];
      __syncthreads();
      R kq[4];
  #pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int l = rh[q] - base;
        const R x = s_ke[j & 1][l & (kThreads - 1)];
        kq[q] = (unsigned)l < (unsigned)blockDim.x ? x : kr[rh[q]];
      }
      const EdgeIn in_v = edge_in(g, args.cf, o, j, args.ex, args.th, args.the, args.d2, args.tvn0);
      level(g, args.cf, o, j, vup, vj, vdn, wa0, wa1, wb0, wb1, ze, kq, vtf[re], in_v, args.gw, args.tvn0, args.vout);
      vup = vj;
      vj = vdn;
      wa0 = wb0;
      wa1 = wb1;
    }
    __syncthreads();  // the next tile of a persistent block reuses s_ke
  }
};

// ---------------------------------------------------------------------------
// column: vertical-wind advection T_w, flux divergences, explicit parts, the
// tridiagonal w solve, sponge and (corrector) the increment updates of rho,
// exner and theta_v.
// Layout: a block holds 64 neighbouring columns (one per lane, so every
// level row is one coalesced 512-byte access) and P waves; wave p owns a
// chunk of at most LM consecutive half levels (rows) of those columns.
// Solve: partition method.  Each wave eliminates its chunk in registers
// (down sweep, then up sweep), leaving every row expressed through the last
// row of the chunk above and the first row of the chunk below; the interface
// unknowns form a 2x2-block tridiagonal system of P-1 blocks that wave 0
// solves through LDS; every wave then back-substitutes its rows.  The matrix
// is diagonally similar to I + symmetric positive semi-definite, so no
// pivoting is needed anywhere.  No HBM scratch.  Rows 0 and K are the w = 0
// boundaries.
// ---------------------------------------------------------------------------
template <typename R>
struct ColArgs {
  const double *w, *rho, *ex, *th;  // state at the start of the substep
  const R* gw;                       // edge terms of T_w of this pass (from the edge kernel)
  const R* vnf;                      // vn of the mass fluxes (vn* / new vn)
  R* tw0;                            // T_w at the substep start: written (predictor), read (corrector);
                                     // T_w is formed in R, so R storage is exact
  R* dv_out;                         // predictor: D = div vn* at the full levels
  const double* ws;                  // corrector: predicted w* (T_w*)
  double *w_out, *rho_out, *ex_out, *th_out;
  const double *rhoe, *the;          // Miura rho, theta_v at the edges (option)
};

// T_w at half level k (1 <= k <= K-1) of column c: horizontal part from the
// three edge terms l_e vn_ie (w_c1 - w_c0) of the cell (gw, over A_c), vertical
// part from the column's own w at half levels k-1, k, k+1 (w_up, w_k, w_dn).
template <typename R>
__device__ __forceinline__ double col_tw(const R* gw, const double* vert, int K1, int es, double w_up, double w_k,
                                         double w_dn, int k, const int* ie, R inv_area) {
  const R* gr = gw + (size_t)k * es;
  const R hs = (gr[ie[0]] + gr[ie[1]] + gr[ie[2]]) * inv_area;
  const double dwdz = (w_up - w_dn) * vert[VT_IDZC2 * K1 + k];
  return (double)(R(-0.5) * hs - (R)(w_k * dwdz));
}

// The same from the three edge terms already loaded.
template <typename R>
__device__ __forceinline__ double col_tw_g(const R g[3], const double* vert, int K1, double w_up, double w_k,
                                           double w_dn, int k, R inv_area) {
  const R hs = (g[0] + g[1] + g[2]) * inv_area;
  const double dwdz = (w_up - w_dn) * vert[VT_IDZC2 * K1 + k];
  return (double)(R(-0.5) * hs - (R)(w_k * dwdz));
}

// Memory inputs of one step of the predictor's forward sweep at full level
// j: the level below (rho, theta_v, exner at j + 1, clamped at the bottom;
// w at half level j + 1), vn* at the cell's edges, the neighbours' rho and
// theta_v (with the Miura option the edge values) and the edge terms of T_w
// at half level j (ws and tw0 are the corrector's and stay unused).  A wave
// loads the next level's inputs before it computes the current one, so the
// memory latency of a level overlaps the previous level's arithmetic
// (column_pred -7 % in FP64, -15 % mixed on R2B8).  The corrector keeps its
// loads where they are used: its registers are full, and the same prefetch
// spilled there and made it slower.
template <typename R>
struct LevIn {
  double rho, th, ex, w, ws;
  R vq[3];
  double rn[3], tn[3];
  R gq[3];
  R tw0;
};

// 1 / x for the column solve's positive divisors (pivots >= 1, rho theta_v,
// exner rho, 1 + dtau tau): the hardware's reciprocal estimate refined by two
// Newton-Raphson steps, e <- 1 - x r, r <- r + r e (each step doubles the
// correct bits), within about an ulp of the rounded quotient and shorter on
// the solve's recurrence than a correctly rounded division.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// State of one level of a column: full level j and half level j.
struct ColLev {
  double rho, th, ex, thp, exp_;  // full level j
  double w, ws;                    // w, w* at half level j
  double ric, atil, gam, zth;      // half level j
};

__device__ __forceinline__ void col_load(const double* rho, const double* th, const double* ex, const double* vert,
                                         int K1, int cs, int j, int c, ColLev& L) {
  const size_t r = (size_t)j * cs + c;
  L.rho = rho[r];
  L.th = th[r];
  L.ex = ex[r];
  L.thp = L.th - vert[VT_THREF * K1 + j];
  L.exp_ = L.ex - vert[VT_EXREF * K1 + j];
}

// half-level quantities of level b (= j1) from full levels j1-1 (a) and j1 (b)
__device__ __forceinline__ void col_half(const double* vert, int K1, const ColLev& a, ColLev& b, int j1, double dtau,
                                         double cpd, double eta) {
  b.ric = 0.5 * (a.rho + b.rho);
  const double thp_ic = 0.5 * (a.thp + b.thp);
  const double th_ic = vert[VT_THREFIC * K1 + j1] + thp_ic;
  b.atil = th_ic * b.ric;
  const double idzh = vert[VT_IDZH * K1 + j1];
  b.gam = dtau * cpd * eta * th_ic * idzh;
  b.zth = (1.0 - eta) * th_ic * (a.exp_ - b.exp_) * idzh + thp_ic * vert[VT_DEXREFIC * K1 + j1];
}

template <typename R>
struct ColPhaseArgs {
  ColArgs<R> a;
  StepCoef cf;
  int P;
};

template <typename R, bool CORR, int LM>
struct BCol {
  using Real = R;
  using Args = ColPhaseArgs<R>;
  // the predictor runs up to 12 waves per block, the corrector up to 8 (its
  // registers allow two waves per SIMD only)
  static constexpr int kThreads = CORR ? 512 : 768;
  __device__ static void run(const DevGrid& g, const Args& args, int bx, int by) {
    const ColArgs<R>& a = args.a;
    body(g, args.cf, args.P, bx, g.vert, g.tau, a.w, a.rho, a.ex, a.th, a.gw, a.vnf, a.tw0, a.dv_out, a.ws, a.w_out,
         a.rho_out, a.ex_out, a.th_out, a.rhoe, a.the);
  }
  // The fields as restrict parameters: the compiler may then move the loads
  // of later levels above the stores of earlier ones (no buffer is both read
  // and written by one launch).
  __device__ __forceinline__ static void body(const DevGrid& g, const StepCoef cf, const int P, const int bx,
                                              const double* __restrict__ vert, const double* __restrict__ tau,
                                              const double* __restrict__ pw, const double* __restrict__ prho,
                                              const double* __restrict__ pex, const double* __restrict__ pth,
                                              const R* __restrict__ pgw, const R* __restrict__ pvn,
                                              R* __restrict__ ptw0, R* __restrict__ pdv,
                                              const double* __restrict__ pws, double* __restrict__ pw_out,
                                              double* __restrict__ prho_out, double* __restrict__ pex_out,
                                              double* __restrict__ pth_out, const double* __restrict__ prhoe,
                                              const double* __restrict__ pthe) {
    // LDS: [6][P][64] interface system; s_stg (corrector): each wave's row
    // of rho and theta_v at its current level (neighbour gathers inside the
    // tile)
    extern __shared__ double s_red[];
    __shared__ double s_stg[8][2][64];
    const int K = g.K, cs = g.cs;
    // the wave index is uniform across the wave: let the compiler keep it,
    // the chunk bounds and every row address derived from them in scalar
    // registers
    const int cl = threadIdx.x & 63, p = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c0 = bx * 64 + cl;
    const bool ok = c0 < g.nc;
    // padding lanes (c0 >= nc, still inside the padded row) compute column 0
    // and store it into their own padding entry, which nothing reads: the
    // stores need no branch, and the loads of later levels may be issued
    // above them
    const int c = ok ? c0 : 0;
    // rows (half levels 1..K-1) of this chunk: [s, s + n)
    const int nrow = K - 1;
    const int base = nrow / P, extra = nrow - base * P;
    const int n = base + (p < extra ? 1 : 0);
    const int s = 1 + p * base + min(p, extra);
    const int h = s - 1;  // full level above the first row (halo; chunk 0 owns it)
    const int K1 = K + 1;
    const double* idzf = vert + VT_IDZF * K1;
    const double eta = cf.eta, dtau = cf.dtau, cpd = cf.cpd, oneme = 1.0 - eta;
    int ie[3], nb[3];
    double kd[3];
  #pragma unroll
    for (int q = 0; q < 3; ++q) {
      ie[q] = g.c2e[q * cs + c];
      nb[q] = g.c2e2c[q * cs + c];
      kd[q] = g.kdiv[q * cs + c];
    }
    const R inv_area = (R)(1.0 / g.area[c]);

    // ---- forward sweep over levels h..h+n: explicit parts, rows, down sweep ----
    double cpv[LM], dpv[LM], lpv[LM];
    double drxv[LM + 1], dxxv[LM + 1];

    ColLev cur;
    col_load(prho, pth, pex, vert, K1, cs, h, c, cur);
    cur.w = pw[(size_t)h * cs + c];
    cur.ws = CORR ? pws[(size_t)h * cs + c] : 0.0;
    double w_up = 0.0, ws_up = 0.0;
    if (h >= 1) {
      ColLev up;
      col_load(prho, pth, pex, vert, K1, cs, h - 1, c, up);
      col_half(vert, K1, up, cur, h, dtau, cpd, eta);
      w_up = pw[(size_t)(h - 1) * cs + c];
      if (CORR) ws_up = pws[(size_t)(h - 1) * cs + c];
    } else {
      cur.ric = cur.rho;
      cur.atil = 0.0;
      cur.gam = 0.0;
      cur.zth = 0.0;
    }
    // corrector with chunks of up to 12 rows: the full levels' rho, theta_v,
    // exner stay in registers for the increment updates after the solve
    // instead of being read again (16-row chunks would spill heavily)
    constexpr bool kKeep = CORR && LM <= 12;
    // 12-row chunks keep rho and theta_v but read exner again: keeping all
    // three spilled (R2B8 column_corr -1 % FP64, -4 % mixed without them);
    // 8-row chunks keep all three (reading exner again: +4 %)
    constexpr bool kKeepEx = kKeep && LM <= 8;
    double sv_r[LM + 2], sv_t[LM + 2], sv_e[LM + 2];
    const double ric0 = cur.ric, atil0 = cur.atil;
    sv_r[0] = cur.rho;
    sv_t[0] = cur.th;
    sv_e[0] = cur.ex;
    double beta_p = 0.0, e_p = 0.0, atil_p = 0.0;
    if constexpr (CORR) {
    #pragma unroll
      for (int i = 0; i <= LM; ++i) {
        if (i <= n) {
          const int j = h + i;
          // the level below, clamped at the bottom (no branch: the last full
          // level takes its own values and then overrides them)
          const bool bottom = j + 1 >= K;
          const int jn = bottom ? K - 1 : j + 1;
          ColLev nx;
          col_load(prho, pth, pex, vert, K1, cs, jn, c, nx);
          col_half(vert, K1, cur, nx, jn, dtau, cpd, eta);
          nx.w = pw[(size_t)(j + 1) * cs + c];
          nx.ws = CORR ? pws[(size_t)(j + 1) * cs + c] : 0.0;
          if (bottom) {
            nx.ric = cur.rho;
            nx.atil = 0.0;
            nx.ws = 0.0;
          }
          sv_r[i + 1] = nx.rho;
          sv_t[i + 1] = nx.th;
          sv_e[i + 1] = nx.ex;
          // mass and theta fluxes, explicit parts at full level j.  Neighbour
          // rho, theta_v: the corrector takes those inside the 64-column tile
          // from the other lanes' rows through LDS, the others from memory;
          // the predictor reads them all from memory (the tile's rows were
          // just read by the other lanes, so mostly from cache), which measured
          // faster there
          double dm = 0.0, dth = 0.0;
          // this level's edge and own loads first: the wave barriers of the
          // LDS exchange below keep later loads from moving above them
          const R* vr = pvn + (size_t)j * g.es;
          R vq[3], gq[3] = {R(0), R(0), R(0)};
          R tw0v = R(0);
    #pragma unroll
          for (int q = 0; q < 3; ++q) vq[q] = vr[ie[q]];
          if (i >= 1) {
            const R* gr = pgw + (size_t)j * g.es;
    #pragma unroll
            for (int q = 0; q < 3; ++q) gq[q] = gr[ie[q]];
            tw0v = ptw0[(size_t)j * cs + c];
          }
          {
            const double* rr = prho + (size_t)j * cs;
            const double* tr = pth + (size_t)j * cs;
            if (CORR) {
              s_stg[p][0][cl] = cur.rho;
              s_stg[p][1][cl] = cur.th;
              __builtin_amdgcn_wave_barrier();
            }
            if (cf.miura) {
              // Miura edge values stored by the upwind pass
              const double* er = prhoe + (size_t)j * g.es;
              const double* et = pthe + (size_t)j * g.es;
    #pragma unroll
              for (int q = 0; q < 3; ++q) {
                const double fm = er[ie[q]] * (double)vq[q];
                dm += kd[q] * fm;
                dth += kd[q] * (fm * et[ie[q]]);
              }
            } else {
      #pragma unroll
              for (int q = 0; q < 3; ++q) {
                double rn, tn;
                if (CORR) {
                  // the LDS read is unconditional (masked index), the memory
                  // read only for neighbours outside the tile (written as
                  // selects: an if-statement form makes the gfx950 backend fail
                  // machine verification)
                  const int lq = nb[q] - bx * 64;
                  rn = s_stg[p][0][lq & 63];
                  tn = s_stg[p][1][lq & 63];
                  rn = (unsigned)lq >= 64u ? rr[nb[q]] : rn;
                  tn = (unsigned)lq >= 64u ? tr[nb[q]] : tn;
                } else {
                  rn = rr[nb[q]];
                  tn = tr[nb[q]];
                }
                // edge means and fluxes in FP64 in both forms (mixed: from the
                // FP32 vn): an FP32 rounding of the fluxes would add to the
                // divergence errors that drive w and rho
                const double rho_e = 0.5 * (cur.rho + rn);
                const double th_e = 0.5 * (cur.th + tn);
                const double fm = rho_e * (double)vq[q];
                const double ft = fm * th_e;
                dm += kd[q] * fm;
                dth += kd[q] * ft;
              }
            }
            if (CORR) __builtin_amdgcn_wave_barrier();
            // predictor: divergence of vn* for the corrector's damping (each
            // full level is stored by the chunk that owns it)
            // (level h of chunk p > 0 is also stored by chunk p - 1: the same value)
            if (!CORR) pdv[(size_t)j * cs + c0] = (R)kd[0] * vq[0] + (R)kd[1] * vq[1] + (R)kd[2] * vq[2];
          }
          const double b = dtau * cf.rd_cvd * cur.ex * rcp_nr(cur.rho * cur.th);
          const double beta = b * idzf[j];
          const double drx = -dtau * (dm + oneme * (cur.ric * cur.w - nx.ric * nx.w) * idzf[j]);
          const double dxx = -b * (dth + oneme * (cur.atil * cur.w - nx.atil * nx.w) * idzf[j]);
          const double e_c = cur.exp_ + dxx;
          drxv[i] = drx;
          dxxv[i] = dxx;
          if (i >= 1) {
            // row of half level j, then one step of the down sweep
            double tw;
            if (CORR) {
              tw = cf.a0 * (double)tw0v + cf.a1 * col_tw_g<R>(gq, vert, K1, ws_up, cur.ws, nx.ws, j, inv_area);
            } else {
              tw = col_tw<R>(pgw, vert, K1, g.es, w_up, cur.w, nx.w, j, ie, inv_area);
              ptw0[(size_t)j * cs + c0] = (R)tw;
            }
            const double wx = cur.w + dtau * (tw - cpd * cur.zth);
            const double A = -cur.gam * beta_p * (eta * atil_p);
            const double B = 1.0 + cur.gam * (eta * cur.atil) * (beta_p + beta);
            const double C = -cur.gam * beta * (eta * nx.atil);
            const double rhs = wx - cur.gam * (e_p - e_c);
            // one reciprocal per row: the pivots are >= 1, so multiplying by
            // it loses nothing against three divisions
            if (i == 1) {
              const double r = rcp_nr(B);
              cpv[0] = C * r;
              dpv[0] = rhs * r;
              lpv[0] = A * r;
            } else {
              const double r = rcp_nr(B - A * cpv[i - 2]);
              cpv[i - 1] = C * r;
              dpv[i - 1] = (rhs - A * dpv[i - 2]) * r;
              lpv[i - 1] = -A * lpv[i - 2] * r;
            }
          }
          beta_p = beta;
          e_p = e_c;
          atil_p = cur.atil;
          w_up = cur.w;
          ws_up = cur.ws;
          cur = nx;
        }
      }
    } else {
      // the predictor loads the next level's inputs before it computes
      // the current level (see LevIn)
      auto load_in = [&](int j, LevIn<R>& L) {
        const int jn = j + 1 >= K ? K - 1 : j + 1;
        const size_t r = (size_t)jn * cs + c;
        L.rho = prho[r];
        L.th = pth[r];
        L.ex = pex[r];
        L.w = pw[(size_t)(j + 1) * cs + c];
        L.ws = CORR ? pws[(size_t)(j + 1) * cs + c] : 0.0;
        const R* vr = pvn + (size_t)j * g.es;
        const R* gr = pgw + (size_t)j * g.es;
    #pragma unroll
        for (int q = 0; q < 3; ++q) {
          L.vq[q] = vr[ie[q]];
          L.gq[q] = gr[ie[q]];
        }
        if (cf.miura) {
    #pragma unroll
          for (int q = 0; q < 3; ++q) {
            L.rn[q] = prhoe[(size_t)j * g.es + ie[q]];
            L.tn[q] = pthe[(size_t)j * g.es + ie[q]];
          }
        } else if (!CORR) {
    #pragma unroll
          for (int q = 0; q < 3; ++q) {
            L.rn[q] = prho[(size_t)j * cs + nb[q]];
            L.tn[q] = pth[(size_t)j * cs + nb[q]];
          }
        }
        L.tw0 = CORR ? ptw0[(size_t)j * cs + c] : R(0);
      };
      LevIn<R> in_a;
      load_in(h, in_a);
    #pragma unroll
      for (int i = 0; i <= LM; ++i) {
        if (i <= n) {
          const int j = h + i;
          LevIn<R> in_b = in_a;
          if (i + 1 <= n) load_in(j + 1, in_b);
          // the level below, clamped at the bottom (no branch: the last full
          // level takes its own values and then overrides them)
          const bool bottom = j + 1 >= K;
          const int jn = bottom ? K - 1 : j + 1;
          ColLev nx;
          nx.rho = in_a.rho;
          nx.th = in_a.th;
          nx.ex = in_a.ex;
          nx.thp = nx.th - vert[VT_THREF * K1 + jn];
          nx.exp_ = nx.ex - vert[VT_EXREF * K1 + jn];
          col_half(vert, K1, cur, nx, jn, dtau, cpd, eta);
          nx.w = in_a.w;
          nx.ws = in_a.ws;
          if (bottom) {
            nx.ric = cur.rho;
            nx.atil = 0.0;
            nx.ws = 0.0;
          }
          sv_r[i + 1] = nx.rho;
          sv_t[i + 1] = nx.th;
          sv_e[i + 1] = nx.ex;
          // mass and theta fluxes, explicit parts at full level j.  Neighbour
          // rho, theta_v: the corrector takes those inside the 64-column tile
          // from the other lanes' rows through LDS, the others from memory;
          // the predictor reads them all from memory (the tile's rows were
          // just read by the other lanes, so mostly from cache), which measured
          // faster there
          double dm = 0.0, dth = 0.0;
          {
            const double* rr = prho + (size_t)j * cs;
            const double* tr = pth + (size_t)j * cs;
            if (CORR) {
              s_stg[p][0][cl] = cur.rho;
              s_stg[p][1][cl] = cur.th;
              __builtin_amdgcn_wave_barrier();
            }
            const R* vq = in_a.vq;
    #pragma unroll
            for (int q = 0; q < 3; ++q) {
              double rho_e, th_e;
              if (cf.miura) {
                // Miura edge values stored by the upwind pass
                rho_e = in_a.rn[q];
                th_e = in_a.tn[q];
              } else {
                double rn, tn;
                if (CORR) {
                  // the LDS read is unconditional (masked index), the memory
                  // read only for neighbours outside the tile (written as
                  // selects: an if-statement form makes the gfx950 backend
                  // fail machine verification)
                  const int lq = nb[q] - bx * 64;
                  rn = s_stg[p][0][lq & 63];
                  tn = s_stg[p][1][lq & 63];
                  rn = (unsigned)lq >= 64u ? rr[nb[q]] : rn;
                  tn = (unsigned)lq >= 64u ? tr[nb[q]] : tn;
                } else {
                  rn = in_a.rn[q];
                  tn = in_a.tn[q];
                }
                rho_e = 0.5 * (cur.rho + rn);
                th_e = 0.5 * (cur.th + tn);
              }
              // edge means and fluxes in FP64 in both forms (mixed: from the
              // FP32 vn): an FP32 rounding of the fluxes would add to the
              // divergence errors that drive w and rho
              const double fm = rho_e * (double)vq[q];
              const double ft = fm * th_e;
              dm += kd[q] * fm;
              dth += kd[q] * ft;
            }
            if (CORR) __builtin_amdgcn_wave_barrier();
            // predictor: divergence of vn* for the corrector's damping (each
            // full level is stored by the chunk that owns it)
            // (level h of chunk p > 0 is also stored by chunk p - 1: the same value)
            if (!CORR) pdv[(size_t)j * cs + c0] = (R)kd[0] * vq[0] + (R)kd[1] * vq[1] + (R)kd[2] * vq[2];
          }
          const double b = dtau * cf.rd_cvd * cur.ex * rcp_nr(cur.rho * cur.th);
          const double beta = b * idzf[j];
          const double drx = -dtau * (dm + oneme * (cur.ric * cur.w - nx.ric * nx.w) * idzf[j]);
          const double dxx = -b * (dth + oneme * (cur.atil * cur.w - nx.atil * nx.w) * idzf[j]);
          const double e_c = cur.exp_ + dxx;
          drxv[i] = drx;
          dxxv[i] = dxx;
          if (i >= 1) {
            // row of half level j, then one step of the down sweep
            double tw;
            if (CORR) {
              tw = cf.a0 * (double)in_a.tw0 + cf.a1 * col_tw_g<R>(in_a.gq, vert, K1, ws_up, cur.ws, nx.ws, j, inv_area);
            } else {
              tw = col_tw_g<R>(in_a.gq, vert, K1, w_up, cur.w, nx.w, j, inv_area);
              ptw0[(size_t)j * cs + c0] = (R)tw;
            }
            const double wx = cur.w + dtau * (tw - cpd * cur.zth);
            const double A = -cur.gam * beta_p * (eta * atil_p);
            const double B = 1.0 + cur.gam * (eta * cur.atil) * (beta_p + beta);
            const double C = -cur.gam * beta * (eta * nx.atil);
            const double rhs = wx - cur.gam * (e_p - e_c);
            // one reciprocal per row: the pivots are >= 1, so multiplying by
            // it loses nothing against three divisions
            if (i == 1) {
              const double r = rcp_nr(B);
              cpv[0] = C * r;
              dpv[0] = rhs * r;
              lpv[0] = A * r;
            } else {
              const double r = rcp_nr(B - A * cpv[i - 2]);
              cpv[i - 1] = C * r;
              dpv[i - 1] = (rhs - A * dpv[i - 2]) * r;
              lpv[i - 1] = -A * lpv[i - 2] * r;
            }
          }
          beta_p = beta;
          e_p = e_c;
          atil_p = cur.atil;
          w_up = cur.w;
          ws_up = cur.ws;
          cur = nx;
          in_a = in_b;
        }
      }
    }
    // ---- up sweep: row i of the chunk = d_i - u_i x_below - v_i x_above ----
  #pragma unroll
    for (int i = LM - 2; i >= 0; --i) {
      if (i < n - 1) {
        dpv[i] = dpv[i] - cpv[i] * dpv[i + 1];
        lpv[i] = lpv[i] - cpv[i] * lpv[i + 1];
        cpv[i] = -cpv[i] * cpv[i + 1];
      }
    }
    // ---- interface system (2x2 blocks), solved by wave 0 ----
    const int sP = P * 64;
    double xa = 0.0, xb = 0.0;  // x in the last row of the chunk above, first row of the chunk below
    if (P > 1) {
      double dl = 0.0, ul = 0.0, vl = 0.0;
  #pragma unroll
      for (int i = 0; i < LM; ++i)
        if (i == n - 1) {
          dl = dpv[i];
          ul = cpv[i];
          vl = lpv[i];
        }
      const int o = p * 64 + cl;
      s_red[0 * sP + o] = dl;
      s_red[1 * sP + o] = ul;
      s_red[2 * sP + o] = vl;
      s_red[3 * sP + o] = dpv[0];
      s_red[4 * sP + o] = cpv[0];
      s_red[5 * sP + o] = lpv[0];
      __syncthreads();
      if (p == 0) {
        double c0p = 0.0, g0p = 0.0;
        for (int q = 0; q < P - 1; ++q) {
          const int oq = q * 64 + cl, on = (q + 1) * 64 + cl;
          const double dz = s_red[0 * sP + oq], uz = s_red[1 * sP + oq], vz = s_red[2 * sP + oq];
          const double df = s_red[3 * sP + on], uf = s_red[4 * sP + on], vf = s_red[5 * sP + on];
          const double bq = uz - vz * c0p;
          const double det = 1.0 - bq * vf;
          const double r0 = dz - vz * g0p, r1 = df;
          const double g0 = (r0 - bq * r1) / det, g1 = (r1 - vf * r0) / det;
          const double k0 = -bq * uf / det, k1 = uf / det;
          s_red[0 * sP + oq] = k0;
          s_red[1 * sP + oq] = k1;
          s_red[2 * sP + oq] = g0;
          s_red[3 * sP + oq] = g1;
          c0p = k0;
          g0p = g0;
        }
        double fnext = 0.0;
        for (int q = P - 2; q >= 0; --q) {
          const int oq = q * 64 + cl;
          const double y0 = s_red[2 * sP + oq] - s_red[0 * sP + oq] * fnext;
          const double y1 = s_red[3 * sP + oq] - s_red[1 * sP + oq] * fnext;
          s_red[4 * sP + oq] = y0;  // last row of chunk q
          s_red[5 * sP + oq] = y1;  // first row of chunk q + 1
          fnext = y1;
        }
      }
      __syncthreads();
      if (p > 0) xa = s_red[4 * sP + (p - 1) * 64 + cl];
      if (p < P - 1) xb = s_red[5 * sP + p * 64 + cl];
      // every wave has read its interface values before any wave of a
      // persistent block writes the next tile's system into s_red (P is
      // uniform over the block, so every wave reaches this barrier)
      __syncthreads();
    }
    // ---- back substitution and sponge: w* at half levels s..s+n-1 ----
    // (row i of the chunk is half level s + i; w*(h) of the chunk above is
    // needed only by chunk 0, where it is the w = 0 boundary)
    const int e = s + n;
    const double w_below = (e < K) ? xb * rcp_nr(1.0 + dtau * tau[e]) : 0.0;
    if (!CORR) {
  #pragma unroll
      for (int i = 0; i < LM; ++i) {
        if (i < n) {
          const double x = dpv[i] - cpv[i] * xb - lpv[i] * xa;
          pw_out[(size_t)(s + i) * cs + c0] = x * rcp_nr(1.0 + dtau * tau[s + i]);
        }
      }
    }
    if (ok && p == 0) pw_out[c] = 0.0;
    if (ok && p == P - 1) pw_out[(size_t)K * cs + c] = 0.0;

    // ---- corrector: w*, and increment updates of rho, exner, theta_v at
    // full levels h..h+n (level h only in chunk 0) ----
    if (CORR) {
      ColLev lv;
      if (kKeep) {
        lv.rho = sv_r[0];
        lv.th = sv_t[0];
        lv.ex = kKeepEx ? sv_e[0] : pex[(size_t)h * cs + c];
        lv.thp = lv.th - vert[VT_THREF * K1 + h];
        lv.exp_ = lv.ex - vert[VT_EXREF * K1 + h];
        lv.ric = ric0;
        lv.atil = atil0;
      } else {
        col_load(prho, pth, pex, vert, K1, cs, h, c, lv);
        if (h >= 1) {
          ColLev up;
          col_load(prho, pth, pex, vert, K1, cs, h - 1, c, up);
          col_half(vert, K1, up, lv, h, dtau, cpd, eta);
        } else {
          lv.ric = lv.rho;
          lv.atil = 0.0;
        }
      }
      double w0 = 0.0;  // w* at half level h (used by chunk 0 only: the top boundary)
  #pragma unroll
      for (int i = 0; i <= LM; ++i) {
        if (i <= n) {
          const int j = h + i;
          double w1 = w_below;
          if (i < n) {
            const double x = dpv[i] - cpv[i] * xb - lpv[i] * xa;
            w1 = x * rcp_nr(1.0 + dtau * tau[s + i]);
            pw_out[(size_t)(s + i) * cs + c0] = w1;
          }
          const bool bottom = j + 1 >= K;
          const int jn = bottom ? K - 1 : j + 1;
          ColLev nx;
          if (kKeep) {
            nx.rho = sv_r[i + 1];
            nx.th = sv_t[i + 1];
            nx.ex = kKeepEx ? sv_e[i + 1] : pex[(size_t)jn * cs + c];
            nx.thp = nx.th - vert[VT_THREF * K1 + jn];
            nx.exp_ = nx.ex - vert[VT_EXREF * K1 + jn];
          } else {
            col_load(prho, pth, pex, vert, K1, cs, jn, c, nx);
          }
          col_half(vert, K1, lv, nx, jn, dtau, cpd, eta);
          if (bottom) {
            nx.ric = lv.rho;
            nx.atil = 0.0;
          }
          if (i >= 1 || p == 0) {
            const double b = dtau * cf.rd_cvd * lv.ex * rcp_nr(lv.rho * lv.th);
            const double beta = b * idzf[j];
            const double drho = drxv[i] - dtau * eta * (lv.ric * w0 - nx.ric * w1) * idzf[j];
            const double dex = dxxv[i] - beta * (eta * lv.atil * w0 - eta * nx.atil * w1);
            const double rho_new = lv.rho + drho;
            {
              const size_t r = (size_t)j * cs + c0;
              prho_out[r] = rho_new;
              pex_out[r] = lv.ex + dex;
              pth_out[r] = lv.th + lv.th * (lv.rho * cf.cvd_rd * dex - drho * lv.ex) * rcp_nr(lv.ex * rho_new);
            }
          }
          w0 = w1;
          lv = nx;
        }
      }
    }
  }
};

// ---------------------------------------------------------------------------
// diffusion
// ---------------------------------------------------------------------------
// vertex: least-squares vertex vector V_v (3 components) and vorticity.
// ---------------------------------------------------------------------------
// diffusion arithmetic shared by the plain kernels and the per-column
// fallback of the surrogate (identical expressions, identical results)
// ---------------------------------------------------------------------------
// Each helper holds the stencil geometry of one entity in registers: a
// thread loads it once and applies it at every level of its block (the
// double-precision tables would otherwise be fetched again at each level,
// since the compiler cannot prove that the stores leave them unchanged).
//
// first vector Laplacian at edge e, grad(div vn) - gradt(curl vn), and the
// Smagorinsky viscosity from the rhombus deformation of the vertex vectors
// Vertex quantities of the diffusion's first pass: the least-squares vertex
// vector (x, y, z) and the relative vorticity.  FP32 keeps them interleaved
// per vertex, one 16-byte record that one load brings in (diff_edge1 -46 %
// on R2B8); FP64 keeps two planes of 16-byte pairs, (x, y) then (z,
// vorticity), each [K][vs]: two loads per vertex (diff_edge1 -10 % against
// four planes), where 32-byte records were slower than four planes.  Index
// i = level * vs + vertex; plane = K * vs values.
template <typename R>
struct alignas(4 * sizeof(R)) VVec {
  R x, y, z, zeta;
};
template <typename R>
struct VertexQ {
  static constexpr bool kInterleaved = sizeof(R) == 4;
  __device__ __forceinline__ static VVec<R> load(const R* __restrict__ base, size_t plane, size_t i) {
    if constexpr (kInterleaved) {
      return reinterpret_cast<const VVec<R>*>(base)[i];
    } else {
      using R2 = R __attribute__((ext_vector_type(2)));
      const R2 a = reinterpret_cast<const R2*>(base)[i];
      const R2 b = reinterpret_cast<const R2*>(base + 2 * plane)[i];
      return VVec<R>{a.x, a.y, b.x, b.y};
    }
  }
  __device__ __forceinline__ static void store(R* __restrict__ base, size_t plane, size_t i, const VVec<R>& v) {
    if constexpr (kInterleaved) {
      reinterpret_cast<VVec<R>*>(base)[i] = v;
    } else {
      using R2 = R __attribute__((ext_vector_type(2)));
      reinterpret_cast<R2*>(base)[i] = R2{v.x, v.y};
      reinterpret_cast<R2*>(base + 2 * plane)[i] = R2{v.z, v.zeta};
    }
  }
};

template <typename R>
struct Edge1Geo {
  int c0, c1, rv[4];
  R invd, invl, invlr, n[3], t[3], smag, cap;
  __device__ __forceinline__ void load_rhombus(const DevGrid& g, int e) {
#pragma unroll
    for (int i = 0; i < 4; ++i) rv[i] = g.e2c2v[i * g.es + e];
    invl = (R)g.invl[e];
    invlr = (R)g.invlr[e];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      n[i] = (R)g.nrm[i * g.es + e];
      t[i] = (R)g.tan[i * g.es + e];
    }
  }
  __device__ __forceinline__ void load(const DevGrid& g, int e, const StepCoef& cf) {
    load_rhombus(g, e);
    c0 = g.e2c[e];
    c1 = g.e2c[g.es + e];
    invd = (R)g.invd[e];
    const double ae = g.ae[e];
    smag = (R)(cf.cs * ae);
    cap = (R)(ae / (cf.cap * cf.dt));
  }
  // the rhombus vertices' quantities at level k
  __device__ __forceinline__ void gather(const DevGrid& g, const R* vv, int k, VVec<R> q[4]) const {
    const size_t plane = (size_t)g.K * g.vs, row = (size_t)k * g.vs;
#pragma unroll
    for (int i = 0; i < 4; ++i) q[i] = VertexQ<R>::load(vv, plane, row + rv[i]);
  }
  __device__ __forceinline__ R l1(const R* dr, const VVec<R> q[4]) const {
    return (dr[c1] - dr[c0]) * invd - (q[1].zeta - q[0].zeta) * invl;
  }
  // derivatives of the normal and tangential wind across the rhombus from the
  // vertex vectors: d = {dvn/dt, dvt/dt, dvn/dn, dvt/dn}
  __device__ __forceinline__ void rhombus(const VVec<R> q[4], R d[4]) const {
    const R tx = q[1].x - q[0].x, ty = q[1].y - q[0].y, tz = q[1].z - q[0].z;
    const R nx = q[3].x - q[2].x, ny = q[3].y - q[2].y, nz = q[3].z - q[2].z;
    d[0] = (tx * n[0] + ty * n[1] + tz * n[2]) * invl;
    d[1] = (tx * t[0] + ty * t[1] + tz * t[2]) * invl;
    d[2] = (nx * n[0] + ny * n[1] + nz * n[2]) * invlr;
    d[3] = (nx * t[0] + ny * t[1] + nz * t[2]) * invlr;
  }
  __device__ __forceinline__ R nu(const VVec<R> q[4]) const {
    R d[4];
    rhombus(q, d);
    const R a = d[2] - d[1], b = d[3] + d[0];
    const R def = sqrt(a * a + b * b);
    return fmin(smag * def, cap);
  }
};
// divergence at cell c of an edge field row
template <typename R>
struct DivGeo {
  int ie[3];
  R kd[3];
  __device__ __forceinline__ void load(const DevGrid& g, int c) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      ie[i] = g.c2e[i * g.cs + c];
      kd[i] = (R)g.kdiv[i * g.cs + c];
    }
  }
  __device__ __forceinline__ R apply(const R* row) const { return kd[0] * row[ie[0]] + kd[1] * row[ie[1]] + kd[2] * row[ie[2]]; }
};
// relative vorticity at vertex v of an edge field row
template <typename R>
struct CurlGeo {
  int ie[6];
  R kc[6];
  __device__ __forceinline__ void load(const DevGrid& g, int v) {
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      ie[s] = g.v2e[s * g.vs + v];
      kc[s] = (R)g.kcurl[s * g.vs + v];
    }
  }
  __device__ __forceinline__ R apply(const R* row) const {
    R z = kc[0] * row[ie[0]];
#pragma unroll
    for (int s = 1; s < 6; ++s) z += kc[s] * row[ie[s]];
    return z;
  }
};
// second Laplacian at edge e from div(L1) at cells and curl(L1) at vertices
template <typename R>
__device__ __forceinline__ R dif_l2(R invd, R invl, R dl1_c0, R dl1_c1, R cl1_v0, R cl1_v1) {
  return (dl1_c1 - dl1_c0) * invd - (cl1_v1 - cl1_v0) * invl;
}
template <typename R>
__device__ __forceinline__ R dif_update(R vn, R dt, R nu, R l1, R k4a2, R l2) {
  return vn + dt * nu * l1 - k4a2 * l2;
}
// w at cell c, half level k after Smagorinsky diffusion with the edge
// viscosity (na, nb: nu on the cell's three edges at the full levels k-1 and
// k, averaged to the cell and the half level); the cell's neighbours and the
// weights of the scalar Laplacian are held in registers
struct LapGeo {
  int nb[3];
  double kl[3];
  __device__ __forceinline__ void load(const DevGrid& g, int c) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      nb[i] = g.c2e2c[i * g.cs + c];
      kl[i] = g.klap[i * g.cs + c];
    }
  }
};
template <typename R>
__device__ __forceinline__ double dif_w(const DevGrid& g, const LapGeo& q, const double* w_in, const R* na,
                                        const R* nb, int c, int k, const StepCoef& cf) {
  const size_t r = (size_t)k * g.cs + c;
  double wn = w_in[r];
  if (cf.diffuse_w && k >= 1 && k <= g.K - 1) {
    R nuc = R(0);
#pragma unroll
    for (int i = 0; i < 3; ++i) nuc += R(0.5) * (na[i] + nb[i]);
    nuc = nuc / R(3);
    const double* wr = w_in + (size_t)k * g.cs;
    double lw = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) lw += q.kl[i] * (wr[q.nb[i]] - wn);
    wn = wn + cf.dt * (double)nuc * lw;
  }
  return wn;
}

template <typename R>
struct BDvert {
  using Real = R;
  struct Args {
    const R* vn;
    R* vv;
    int kb;
  };
  static constexpr int kThreads = 256;
  __device__ static void run(const DevGrid& g, const Args& args, int bx, int by) {
    const R* __restrict__ vn = args.vn;
    R* __restrict__ vv = args.vv;
    const int kb = args.kb;
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
      VertexQ<R>::store(vv, (size_t)g.K * g.vs, (size_t)k * g.vs + v, VVec<R>{a, b, d, z});
    }
  }
};

// cell: divergence of an edge field (first pass: div vn)
template <typename R>
struct BDiv {
  using Real = R;
  struct Args {
    const R* f;
    R* out;
    int kb;
  };
  static constexpr int kThreads = 256;
  __device__ static void run(const DevGrid& g, const Args& args, int bx, int by) {
    const R* __restrict__ f = args.f;
    R* __restrict__ out = args.out;
    const int kb = args.kb;
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
};

// edge: L1 = grad(div vn) - gradt(curl vn) and the Smagorinsky viscosity
// from the rhombus deformation of the vertex vectors.
template <typename R>
struct BDedge1 {
  using Real = R;
  struct Args {
    const R* dv;
    const R* vv;
    R* l1;
    R* nu;
    StepCoef cf;
    int kb;
  };
  static constexpr int kThreads = 256;
  __device__ static void run(const DevGrid& g, const Args& args, int bx, int by) {
    const R* __restrict__ dv = args.dv;
    const R* __restrict__ vv = args.vv;
    R* __restrict__ l1 = args.l1;
    R* __restrict__ nu = args.nu;
    const StepCoef cf = args.cf;
    const int kb = args.kb;
    const int e = bx * blockDim.x + threadIdx.x;
    if (e >= g.ne) return;
    Edge1Geo<R> q;
    q.load(g, e, cf);
    const int k0 = by * kb, k1 = min(g.K, k0 + kb);
    for (int k = k0; k < k1; ++k) {
      VVec<R> qv[4];
      q.gather(g, vv, k, qv);
      l1[(size_t)k * g.es + e] = q.l1(dv + (size_t)k * g.cs, qv);
      nu[(size_t)k * g.es + e] = q.nu(qv);
    }
  }
};

// cell + vertex (one launch): div(L1) at cells, curl(L1) at vertices, and the
// Smagorinsky diffusion of w at cells (reads w_in, writes w_out).
template <typename R>
struct BDcv2 {
  using Real = R;
  struct Args {
    const R* l1;
    const R* nu;
    const double* w_in;
    double* w_out;
    R* divl1;
    R* curll1;
    const double* th_in;  // theta_v diffusion (cf.diffuse_theta): theta_v in,
    double* th_out;       // theta_v out,
    double* ex;           // exner, updated in place
    int ncb;
    StepCoef cf;
    int kb;
  };
  static constexpr bool kXcdRanges = false;  // round-robin tile order (see the top of this file)
  static constexpr int kThreads = 256;
  __device__ static void run(const DevGrid& g, const Args& args, int bx, int by) {
    const R* __restrict__ l1 = args.l1;
    const R* __restrict__ nu = args.nu;
    const double* __restrict__ w_in = args.w_in;
    double* __restrict__ w_out = args.w_out;
    R* __restrict__ divl1 = args.divl1;
    R* __restrict__ curll1 = args.curll1;
    const int ncb = args.ncb;
    const StepCoef cf = args.cf;
    const int kb = args.kb;
    const int K = g.K;
    if (bx < ncb) {
      const int c = bx * blockDim.x + threadIdx.x;
      if (c >= g.nc) return;
      DivGeo<R> dq;
      dq.load(g, c);
      LapGeo lq;
      lq.load(g, c);
      const int* ie = dq.ie;
      const int k0 = by * kb, k1 = min(K + 1, k0 + kb);
      // near-surface floor on the theta_v coefficient: the Smagorinsky
      // stability cap averaged over the cell's edges, reached by cells
      // colder than their neighbours' mean by twice the threshold
      const int k_enh = K - cf.theta_enh_nlev;
      double capc = 0.0;
      if (cf.diffuse_theta && k1 > k_enh)
        capc = (g.ae[ie[0]] + g.ae[ie[1]] + g.ae[ie[2]]) / 3.0 / (cf.cap * cf.dt);
      // nu on the cell's edges at full level k - 1, carried from one half
      // level to the next
      R nup[3] = {R(0), R(0), R(0)};
      if (k0 >= 1) {
  #pragma unroll
        for (int i = 0; i < 3; ++i) nup[i] = nu[(size_t)(k0 - 1) * g.es + ie[i]];
      }
      for (int k = k0; k < k1; ++k) {
        R nuk[3] = {R(0), R(0), R(0)};
        const size_t r = (size_t)k * g.cs + c;
        if (k < K) {
          const R* row = l1 + (size_t)k * g.es;
          divl1[r] = dq.apply(row);
  #pragma unroll
          for (int i = 0; i < 3; ++i) nuk[i] = nu[(size_t)k * g.es + ie[i]];
          if (cf.diffuse_theta) {
            // theta_v at full level k: the Smagorinsky form of w with nu
            // averaged over the cell's edges; exner by the equation of state
            // at fixed rho, dpi/pi = (R_d/c_vd) dtheta_v/theta_v
            const double* tr = args.th_in + (size_t)k * g.cs;
            const double tc = tr[c];
            const R nuf = (nuk[0] + nuk[1] + nuk[2]) / R(3);
            double nud = (double)nuf;
            double tn[3];
  #pragma unroll
            for (int i = 0; i < 3; ++i) tn[i] = tr[lq.nb[i]];
            if (k >= k_enh) {
              const double cold = (tn[0] + tn[1] + tn[2]) / 3.0 - tc;
              const double sr = fmin(fmax((cold - cf.theta_enh_thr) / cf.theta_enh_thr, 0.0), 1.0);
              nud = fmax(nud, sr * capc);
            }
            double lt = 0.0;
  #pragma unroll
            for (int i = 0; i < 3; ++i) lt += lq.kl[i] * (tn[i] - tc);
            const double dth = cf.dt * nud * lt;
            args.th_out[r] = tc + dth;
            args.ex[r] = args.ex[r] * (1.0 + cf.rd_cvd * dth / tc);
          }
        }
        w_out[r] = dif_w<R>(g, lq, w_in, nup, nuk, c, k, cf);
  #pragma unroll
        for (int i = 0; i < 3; ++i) nup[i] = nuk[i];
      }
    } else {
      const int v = (bx - ncb) * blockDim.x + threadIdx.x;
      if (v >= g.nv) return;
      CurlGeo<R> q;
      q.load(g, v);
      const int k0 = by * kb, k1 = min(K, k0 + kb);
      for (int k = k0; k < k1; ++k) curll1[(size_t)k * g.vs + v] = q.apply(l1 + (size_t)k * g.es);
    }
  }
};

// edge: L2 = lapv(L1) and vn += dt nu L1 - k4 A_e^2 L2 (in place).
template <typename R>
struct BDedge2 {
  using Real = R;
  struct Args {
    R* vn;
    const R* l1;
    const R* nu;
    const R* divl1;
    const R* curll1;
    StepCoef cf;
    int kb;
  };
  static constexpr int kThreads = 256;
  __device__ static void run(const DevGrid& g, const Args& args, int bx, int by) {
    R* __restrict__ vn = args.vn;
    const R* __restrict__ l1 = args.l1;
    const R* __restrict__ nu = args.nu;
    const R* __restrict__ divl1 = args.divl1;
    const R* __restrict__ curll1 = args.curll1;
    const StepCoef cf = args.cf;
    const int kb = args.kb;
    const int e = bx * blockDim.x + threadIdx.x;
    if (e >= g.ne) return;
    const int c0 = g.e2c[e], c1 = g.e2c[g.es + e];
    const int v0 = g.e2v[e], v1 = g.e2v[g.es + e];
    const double ae = g.ae[e];
    const R k4a2 = (R)(cf.k4 * ae * ae);
    const R dt = (R)cf.dt;
    const R invd = (R)g.invd[e], invl = (R)g.invl[e];
    const int k0 = by * kb, k1 = min(g.K, k0 + kb);
    for (int k = k0; k < k1; ++k) {
      const R* dr = divl1 + (size_t)k * g.cs;
      const R* zr = curll1 + (size_t)k * g.vs;
      const R l2 = dif_l2<R>(invd, invl, dr[c0], dr[c1], zr[v0], zr[v1]);
      const size_t r = (size_t)k * g.es + e;
      vn[r] = dif_update<R>(vn[r], dt, nu[r], l1[r], k4a2, l2);
    }
  }
};


// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
// one state: 2-D grid of tiles, XCD-aware order
template <typename B, typename = void>
struct xcd_ranges : std::true_type {};
template <typename B>
struct xcd_ranges<B, std::void_t<decltype(B::kXcdRanges)>> : std::bool_constant<B::kXcdRanges> {};

template <typename B>
__global__ void __launch_bounds__(B::kThreads) k_one(DevGrid g, typename B::Args a) {
  int bx, by;
  if constexpr (xcd_ranges<B>::value) {
    tile_coords(bx, by);
  } else {
    bx = blockIdx.x;
    by = blockIdx.y;
  }
  B::run(g, a, bx, by);
}

// many states: a persistent grid walks the (member, tile) work table;
// tstart[m] is the first tile of member m, tstart[nm] the total.
template <typename A>
struct Job {
  DevGrid g;
  A a;
  int nbx;  // tiles along the entity axis
};

template <typename B>
__global__ void __launch_bounds__(B::kThreads) k_many(const Job<typename B::Args>* __restrict__ jobs,
                                                       const int* __restrict__ tstart, int nm) {
  const int total = tstart[nm];
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    int m = 0;
    while (t >= tstart[m + 1]) ++m;
    const int lt = t - tstart[m];
    const int nbx = jobs[m].nbx;
    B::run(jobs[m].g, jobs[m].a, lt % nbx, lt / nbx);
  }
}

// ---------------------------------------------------------------------------
// host-side argument builders and launch geometry (shared by the single and
// batched launch paths, so both run identical per-tile work)
// ---------------------------------------------------------------------------
struct Geom {
  int nbx, nby, threads;
  size_t smem;
};

inline int cdiv(int a, int b) { return (a + b - 1) / b; }

// Column chunking: chunk length LM in {8, 12, 16}, chunks hold >= 2 rows
// whenever there is more than one; supports n_lev <= 129.  The corrector (at
// most 8 waves per block: its registers allow two waves per SIMD) takes the
// smallest LM that fits in 8 chunks.  The predictor, at three waves per SIMD,
// takes up to 12 chunks: 8-row chunks up to 96 rows, 12-row chunks beyond,
// so deep columns get more waves and shorter serial sweeps.
inline int col_chunks_lm(int K, bool corr, int* lm) {
  const int nrow = std::max(K - 1, 0);
  if (corr)
    *lm = nrow <= 64 ? 8 : (nrow <= 96 ? 12 : 16);
  else
    *lm = nrow <= 96 ? 8 : 12;
  return std::max(1, (nrow + *lm - 1) / *lm);
}

// rbytes: bytes of the stencil precision (the fused edge pass's LDS holds it)
inline Geom geom_of(int phase, const DevGrid& g, const Tile* T, size_t rbytes) {
  int lm;
  switch (phase) {
    case K_VC_P:
    case K_VC_C: {
      // with the fused edge pass only the corrector's damping field is left
      const Tile& t = T[T_VC];
      const int nbx = (g.et_ok ? 0 : cdiv(g.ne, t.threads) + cdiv(g.nv, t.threads)) +
                      (phase == K_VC_C ? cdiv(g.nc, t.threads) : 0);
      return {nbx, cdiv(g.K, t.kb), t.threads, 0};
    }
    case K_EDGE_P:
    case K_EDGE_C: {
      // tiles of EdgeTiles::kTileE edges in both forms (the fused form's
      // host tables are built for them); only the level blocks are tuned
      const Tile& t = T[T_EDGE];
      return {cdiv(g.ne, EdgeTiles::kTileE), cdiv(g.K, t.kb), EdgeTiles::kTileE,
              g.et_ok ? BEdge<double, false>::kSmem / sizeof(double) * rbytes : 0};
    }
    case K_MIURA: {
      const Tile& t = T[T_EDGE];
      return {cdiv(g.ne, t.threads), cdiv(g.K, t.kb), t.threads, 0};
    }
    case K_COL_P:
    case K_COL_C: {
      const int P = col_chunks_lm(g.K, phase == K_COL_C, &lm);
      return {cdiv(g.nc, 64), 1, 64 * P, P > 1 ? 6 * sizeof(double) * 64 * (size_t)P : 0};
    }
    case K_DVERT: {
      const Tile& t = T[T_DVERT];
      return {cdiv(g.nv, t.threads), cdiv(g.K, t.kb), t.threads, 0};
    }
    case K_DDIV: {
      const Tile& t = T[T_DCELL];
      return {cdiv(g.nc, t.threads), cdiv(g.K, t.kb), t.threads, 0};
    }
    case K_DCV2: {
      const Tile& t = T[T_DCELL];
      return {cdiv(g.nc, t.threads) + cdiv(g.nv, t.threads), cdiv(g.K + 1, t.kb), t.threads, 0};
    }
    default: {  // K_DEDGE1, K_DEDGE2
      const Tile& t = T[T_DEDGE];
      return {cdiv(g.ne, t.threads), cdiv(g.K, t.kb), t.threads, 0};
    }
  }
}

template <typename R>
struct SubstepArgs {
  typename BVc<R, false>::Args vc_p;
  typename BMiura<R>::Args mi;
  typename BEdge<R, false>::Args e_p;
  ColPhaseArgs<R> c_p;
  typename BVc<R, true>::Args vc_c;
  typename BEdge<R, true>::Args e_c;
  ColPhaseArgs<R> c_c;
};

template <typename R>
SubstepArgs<R> substep_args(const DevGrid& g, const Bufs<R>& b, const StepCoef& c, const Tile* T) {
  SubstepArgs<R> s;
  int lm;
  const int Pp = col_chunks_lm(g.K, false, &lm), Pc = col_chunks_lm(g.K, true, &lm);
  const int neb = g.et_ok ? 0 : cdiv(g.ne, T[T_VC].threads), nvb = g.et_ok ? 0 : cdiv(g.nv, T[T_VC].threads);
  s.vc_p = {b.vn, b.zeta, b.vt, b.kc, nullptr, nullptr, neb, nvb, T[T_VC].kb};
  s.mi = {b.vn, b.rho, b.th, b.rhoe, b.the, c.dtau, T[T_EDGE].kb};
  s.e_p = {b.vn, b.zeta, b.kc, b.vt, b.w, b.ex, b.th, b.tvn0, b.vns, nullptr, b.gw, b.the, c, T[T_EDGE].kb};
  s.c_p = {{b.w, b.rho, b.ex, b.th, b.gw, b.vns, b.tw0, b.dvn, nullptr, b.ws, nullptr, nullptr, nullptr, b.rhoe, b.the},
           c, Pp};
  s.vc_c = {b.vns, b.zeta, b.vt, b.kc, b.d2, b.dvn, neb, nvb, T[T_VC].kb};
  s.e_c = {b.vns, b.zeta, b.kc, b.vt, b.ws, b.ex, b.th, b.tvn0, b.vn_out, b.d2, b.gw, nullptr, c, T[T_EDGE].kb};
  s.c_c = {{b.w, b.rho, b.ex, b.th, b.gw, b.vn_out, b.tw0, nullptr, b.ws, b.w_out, b.rho_out, b.ex_out, b.th_out, b.rhoe,
            b.the},
           c, Pc};
  return s;
}

template <typename R>
struct DiffusionArgs {
  typename BDvert<R>::Args dv;
  typename BDiv<R>::Args dd;
  typename BDedge1<R>::Args d1;
  typename BDcv2<R>::Args cv;
  typename BDedge2<R>::Args d2;
};

// vn updated in place; w read from w_in, written to w_out; l1, nu, dv, dl1,
// zeta (curl L1), vv are workspace fields (edge, edge, cell, cell, vertex,
// 4 x vertex: vertex vector and vorticity of vn, laid out as VertexQ says)
template <typename R>
DiffusionArgs<R> diffusion_args(const DevGrid& g, R* vn, const double* w_in, double* w_out, R* l1, R* nu, R* dv,
                                R* dl1, R* zeta, R* vv, const StepCoef& c, const Tile* T,
                                const ThetaDiff& td = ThetaDiff{nullptr, nullptr, nullptr}) {
  DiffusionArgs<R> d;
  d.dv = {vn, vv, T[T_DVERT].kb};
  d.dd = {vn, dv, T[T_DCELL].kb};
  d.d1 = {dv, vv, l1, nu, c, T[T_DEDGE].kb};
  d.cv = {l1, nu, w_in, w_out, dl1, zeta, td.th_in, td.th_out, td.ex, cdiv(g.nc, T[T_DCELL].threads), c,
          T[T_DCELL].kb};
  d.d2 = {vn, l1, nu, dl1, zeta, c, T[T_DEDGE].kb};
  return d;
}

}  // namespace bodies
}  // namespace dc
