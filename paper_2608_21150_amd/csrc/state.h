// Internal definitions of the grid and state handles (shared by the C-ABI
// implementation files; not part of the public interface).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <vector>

#include "dycore.h"
#include "internal.h"
#include "kernels.h"

namespace dc {
struct SurCtx;  // surrogate settings of a state (defined with the surrogate)
}

struct dc_grid {
  using HostGrid = dc::HostGrid;
  using DevGrid = dc::DevGrid;
  HostGrid h;
  DevGrid d{};
  bool uploaded = false;
  int device = -1;
  std::vector<void*> allocs;
  std::atomic<int> states{0};
  // tables of the optional schemes, uploaded on first use
  const double* kvt_rbf = nullptr;  // [5][es] RBF tangential-wind weights
  const double* kmiura = nullptr;   // [18][es] Miura upwind coefficients
};

struct dc_state {
  using DevGrid = dc::DevGrid;
  using Tile = dc::Tile;
  using Prof = dc::Prof;
  static constexpr int kTiles = dc::T_COUNT;
  dc_grid* grid = nullptr;
  dc_params p{};
  dc_precision prec = DC_PREC_FP64;
  dc_diffusion diff = DC_DIFF_PLAIN;
  dc_fields buf[2]{};
  int cur = 0;
  hipStream_t stream = nullptr;
  DevGrid d{};  // grid view plus per-state Coriolis and sponge tables
  Tile tiles[kTiles];
  Prof prof;
  // workspace carve-up
  char* ws = nullptr;
  size_t ws_bytes = 0;
  void *vt, *tvn0, *vns, *kc, *d2, *zeta, *vv, *gw, *dvn;
  double *wstar, *wtmp, *ttmp, *fe, *tau, *diag_part, *diag_out;
  void* tw0;  // [K+1][cs] T_w of the predictor, in the stencil precision
  double *rhoe = nullptr, *the = nullptr;  // [K][es] Miura edge values (option)
  // surrogate diffusion (DC_DIFF_SURROGATE only): network tendency [K][es],
  // curl L1 of the diffusion front [K][vs], judge and range flags [es],
  // counters (4 int, then one 64-bit)
  dc::SurCtx* sur = nullptr;
  void* sur_tmlp = nullptr;
  void* sur_cl = nullptr;
  int* sur_fj = nullptr;
  int* sur_fr = nullptr;
  int* sur_cnt = nullptr;
  double sur_lbar = 1.0, sur_dbar = 1.0;  // mean primal / dual edge length
  // the step in parts: 1 after a predictor (its workspace fields readable, a
  // corrector may follow), 2 after that corrector, 0 once anything else has
  // run over the workspace
  int part = 0;
};


namespace dc {

inline StepCoef make_coef(const dc_state* s, double dt, int nsub) {
  StepCoef c{};
  c.dtau = dt / nsub;
  c.dt = dt;
  c.eta = s->p.eta;
  c.a0 = s->p.adv_w0;
  c.a1 = s->p.adv_w1;
  c.cpd = s->p.cpd;
  c.rd_cvd = s->p.rd / s->p.cvd;
  c.cvd_rd = s->p.cvd / s->p.rd;
  c.c4a2 = s->p.divdamp_c4 * s->grid->h.mean_area * s->grid->h.mean_area;
  c.cs = s->p.smag_cs;
  c.cap = s->p.smag_cap;
  c.k4 = s->p.hdiff_k4;
  c.diffuse_w = s->p.diffuse_w;
  c.diffuse_theta = s->p.diffuse_theta;
  c.theta_enh_nlev = s->p.theta_enh_nlev;
  c.theta_enh_thr = s->p.theta_enh_thresh;
  c.miura = s->p.miura;
  return c;
}

// Buffers of substep i of a step that starts in buffer set `cur`; the last
// substep writes w to the diffusion staging field when diffusion follows.
template <typename R>
Bufs<R> substep_bufs(const dc_state* s, int cur_idx, bool w_to_staging) {
  const dc_fields& cur = s->buf[cur_idx];
  const dc_fields& nxt = s->buf[1 - cur_idx];
  Bufs<R> b{};
  b.vn = static_cast<const R*>(cur.vn);
  b.w = static_cast<const double*>(cur.w);
  b.rho = static_cast<const double*>(cur.rho);
  b.ex = static_cast<const double*>(cur.exner);
  b.th = static_cast<const double*>(cur.theta_v);
  b.vt = static_cast<R*>(s->vt);
  b.tvn0 = static_cast<R*>(s->tvn0);
  b.vns = static_cast<R*>(s->vns);
  b.kc = static_cast<R*>(s->kc);
  b.d2 = static_cast<R*>(s->d2);
  b.zeta = static_cast<R*>(s->zeta);
  b.vv = static_cast<R*>(s->vv);
  b.ws = s->wstar;
  b.wtmp = s->wtmp;
  b.gw = static_cast<R*>(s->gw);
  b.dvn = static_cast<R*>(s->dvn);
  b.tw0 = static_cast<R*>(s->tw0);
  b.rhoe = s->rhoe;
  b.the = s->the;
  b.vn_out = static_cast<R*>(nxt.vn);
  b.w_out = w_to_staging ? s->wtmp : static_cast<double*>(nxt.w);
  b.rho_out = static_cast<double*>(nxt.rho);
  b.ex_out = static_cast<double*>(nxt.exner);
  // theta_v goes to its staging field too when the diffusion diffuses it
  b.th_out = w_to_staging && s->p.diffuse_theta ? s->ttmp : static_cast<double*>(nxt.theta_v);
  return b;
}

// The nsub dynamic substeps of one step (flipping the buffer set after
// each); the last writes w to the diffusion staging field if to_staging.
template <typename R>
void enqueue_substeps(dc_state* s, const StepCoef& c, int nsub, bool to_staging) {
  for (int i = 0; i < nsub; ++i) {
    const Bufs<R> b = substep_bufs<R>(s, s->cur, i == nsub - 1 && to_staging);
    launch_substep<R>(s->d, b, c, s->tiles, s->stream, &s->prof);
    s->cur ^= 1;
  }
}

// surrogate diffusion of the current buffer set (a state with an MLP set)
template <typename R>
void surrogate_diffusion(dc_state* s, const StepCoef& c);
void surrogate_free(dc_state* s);
void surrogate_geometry(dc_state* s);

// Default launch tiles (dc_state_autotune replaces them by measured ones).
// The levels are split into near-equal blocks: a short last block leaves
// much of its wave's time unused.  Shapes from timings of the 81920-cell,
// 65-level grid on one MI355X: thin edge-momentum tiles running deep in the
// column, wide vorticity and diffusion tiles with a few levels each.
inline void default_tiles(const HostGrid& h, Tile* t) {
  auto kb_of = [&](int nby) {
    nby = std::max(1, std::min(nby, h.K));
    return (h.K + nby - 1) / nby;
  };
  t[T_VC] = {256, kb_of(6)};
  t[T_EDGE] = {64, kb_of(2)};
  t[T_DVERT] = {256, kb_of(3)};
  t[T_DCELL] = {256, kb_of(11)};
  t[T_DEDGE] = {128, kb_of(5)};
}

}  // namespace dc
