// Device-side views and kernel launchers of the dycore library.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

namespace dc {

// Kernel identifiers for per-launch timing.
enum KernelId {
  K_VC_P = 0, K_EDGE_P, K_COL_P,
  K_VC_C, K_EDGE_C, K_COL_C,
  K_DVERT, K_DDIV, K_DEDGE1, K_DCV2, K_DEDGE2,
  K_MIURA,  // upwind edge values of rho and theta_v (option), once per substep
  K_COUNT
};
extern const char* const kKernelNames[K_COUNT];

// Optional HIP-event timer: mark(id) before a launch, mark(-1) after it.
struct Prof {
  bool on = false;
  unsigned mask = ~0u;  // kernels (1u << id) whose launches are recorded
  bool wants(int id) const { return on && ((mask >> id) & 1u); }
  std::vector<hipEvent_t> ev;
  std::vector<int> kid;
  size_t used = 0;
  void mark(hipStream_t s, int id) {
    if (!on) return;
    if (used == ev.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) { on = false; return; }
      ev.push_back(e);
      kid.push_back(0);
    }
    kid[used] = id;
    (void)hipEventRecord(ev[used], s);
    ++used;
  }
};

// Read-only grid view handed to every kernel by value.  Tables are
// slot-major ([slot][entity]) with padded strides so that neighbouring
// threads read neighbouring table entries.
struct DevGrid {
  int nc, ne, nv, K, cs, es, vs;
  const int* c2e;       // [3][cs]
  const int* c2e2c;     // [3][cs]
  const double* kdiv;   // [3][cs]  s l / A_c
  const double* klap;   // [3][cs]  l / (d A_c)
  const double* area;   // [cs]
  const int* e2c;       // [2][es]
  const int* e2v;       // [2][es]  ordered along the tangent
  const int* e2c2e;     // [4][es]
  const int* e2c2v;     // [4][es]
  const double* kvt;    // [5][es]  tangential-wind weights: self, e2c2e[0..3]
  const double* invd;   // [es] 1/d_e
  const double* invl;   // [es] 1/l_e
  const double* ae;     // [es] l_e d_e / 2
  const double* invlr;  // [es] 1/(rhombus diagonal length)
  const double* nrm;    // [3][es]
  const double* tan;    // [3][es]
  const int* v2e;       // [6][vs]
  const double* kcurl;  // [6][vs] sig d / A_v
  const double* klsq;   // [18][vs]
  const double* vert;   // [VT_COUNT][K+1]
  const double* fe;     // [es] Coriolis parameter (per state)
  const double* tau;    // [K+1] sponge rate (per state)
  const double* kmiura; // [18][es] Miura upwind coefficients (per state; null when off)
  // tiles of the fused edge pass (et_ok = 0: separate vorticity pass)
  int et_ok, et_ntile;
  const int* et_n;        // [ntile][4] own, vt set, staged set, vertices
  const int* et_x;        // [ntile][XM] staged edge ids
  const int* et_vx;       // [ntile][VM] vertex ids
  const unsigned short* et_nb;  // [ntile][4][XV] local positions of e2c2e
  const unsigned short* et_vl;  // [ntile][6][VM] local positions of v2e
  const unsigned short* et_ev;  // [ntile][2][256] local ids of the own edges' end vertices
};

// Launch geometry of a level-blocked stencil kernel.
struct Tile {
  int threads;  // threads per block (entities)
  int kb;       // levels per block
};

struct StepCoef {
  double dtau, dt, eta, a0, a1, cpd, rd_cvd, cvd_rd, c4a2, cs, cap, k4;
  int diffuse_w, diffuse_theta;
  int miura;             // rho and theta_v at edges by Miura upwind reconstruction
  int theta_enh_nlev;    // lowest levels with the near-surface floor on the theta_v coefficient
  double theta_enh_thr;  // its threshold [K]
};

// Pointers of one predictor/corrector/diffusion pass; the meaning of each
// member is given at the launcher that uses it.
template <typename R>
struct Bufs {
  // state at the start of the substep
  const R* vn;
  const double *w, *rho, *ex, *th;
  // workspace (kc: K_e at edges [K][es] during the substeps)
  R *vt, *tvn0, *vns, *kc, *d2, *zeta, *vv;
  double *ws, *wtmp;
  R* gw;        // [K+1][es] edge terms of the horizontal advection of w
  R* dvn;       // [K][cs] div vn* (predictor column kernel -> corrector damping)
  R* tw0;       // [K+1][cs] T_w at the substep start (predictor -> corrector), formed in R
  double* rhoe;  // [K][es] Miura rho at edges (option; written by the upwind pass, read by the columns)
  double* the;   // [K][es] Miura theta_v at edges (also the pressure-gradient term's theta_v)
  // outputs of the corrector
  R* vn_out;
  double *w_out, *rho_out, *ex_out, *th_out;
};

template <typename R>
void launch_substep(const DevGrid& g, const Bufs<R>& b, const StepCoef& c, const Tile* tiles, hipStream_t s,
                    Prof* prof);
// the two halves of a substep: the predictor writes only workspace fields
// (vn*, Y, w*, T_w at the start, div vn*, the edge terms of T_w); the
// corrector reads them and writes the next buffer set
template <typename R>
void launch_predictor(const DevGrid& g, const Bufs<R>& b, const StepCoef& c, const Tile* tiles, hipStream_t s,
                      Prof* prof);
template <typename R>
void launch_corrector(const DevGrid& g, const Bufs<R>& b, const StepCoef& c, const Tile* tiles, hipStream_t s,
                      Prof* prof);
// theta_v diffusion (optional): theta_v read from th_in, written to th_out,
// exner updated in place; all null when it is off
struct ThetaDiff {
  const double* th_in;
  double* th_out;
  double* ex;
};
template <typename R>
void launch_diffusion(const DevGrid& g, R* vn, const double* w_in, double* w_out, R* vt_l1, R* nu, R* kc_div,
                      R* d2_divl1, R* zeta, R* vv, const ThetaDiff& td, const StepCoef& c, const Tile* tiles,
                      hipStream_t s, Prof* prof);
// The diffusion in two parts: the front (vertex vectors and vorticity, div vn,
// L1 and the viscosity, div L1 and curl L1, the w diffusion) and the back
// (L2 and the vn update).  curll1 may differ from zeta so that the vorticity
// survives the front.
template <typename R>
void launch_diffusion_front(const DevGrid& g, const R* vn, const double* w_in, double* w_out, R* l1, R* nu, R* dv,
                            R* dl1, R* zeta, R* curll1, R* vv, const StepCoef& c, const Tile* tiles, hipStream_t s,
                            Prof* prof);
template <typename R>
void launch_diffusion_back(const DevGrid& g, R* vn, const R* l1, const R* nu, const R* dl1, const R* curll1,
                           const StepCoef& c, const Tile* tiles, hipStream_t s, Prof* prof);
template <typename R>
void launch_diag(const DevGrid& g, const R* vn, const double* w, const double* rho, const double* th,
                 const double* ex, double* partial, double* out, hipStream_t s);
int diag_partial_count(const DevGrid& g);

// indices into the tile table
enum TileId { T_VC = 0, T_EDGE, T_DVERT, T_DCELL, T_DEDGE, T_COUNT };

}  // namespace dc
