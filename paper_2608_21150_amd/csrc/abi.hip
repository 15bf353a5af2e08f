// C-ABI entry points of the dycore library: grid and state lifecycle, the
// time step (dynamic substeps, then diffusion), host copies and diagnostics.
// The call conventions follow the paper's Fortran/C bridge (Section 4.3.1):
// scalars by value, arrays by reference without copies, double-buffered
// prognostic fields flipped by the library, and nothing of the kernel
// implementation visible in the interface.

#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "kernels.h"
#include "state.h"

namespace dc {

thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

}  // namespace dc

using namespace dc;

namespace {

#define DC_TRY(expr)                                                                  \
  do {                                                                                \
    hipError_t _e = (expr);                                                           \
    if (_e != hipSuccess) {                                                           \
      set_error(std::string(#expr) + ": " + hipGetErrorString(_e));                   \
      return DC_EHIP;                                                                 \
    }                                                                                 \
  } while (0)

dc_status fail(dc_status code, const std::string& msg) {
  set_error(msg);
  return code;
}

size_t elem_size(dc_precision prec) { return prec == DC_PREC_MIXED ? sizeof(float) : sizeof(double); }

struct Layout {
  size_t vt, tvn0, vns, kc, d2, zeta, vv, gw, dvn, wstar, wtmp, ttmp, tw0, fe, tau, dpart, dout;
  size_t rhoe, the;  // Miura option only
  size_t s_tmlp, s_cl, s_fj, s_fr, s_cnt;  // surrogate mode only
  size_t total;
};

Layout workspace_layout(const HostGrid& h, dc_precision prec, dc_diffusion diff, bool miura) {
  const size_t r = elem_size(prec);
  const size_t K = h.K, K1 = h.K + 1;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  };
  Layout L;
  L.vt = take(K * h.es * r);
  L.tvn0 = take(K * h.es * r);
  L.vns = take(K * h.es * r);
  L.kc = take(K * std::max(h.es, h.cs) * r);  // K_e [K][es] in substeps, div vn [K][cs] in diffusion
  L.d2 = take(K1 * h.cs * r);
  L.zeta = take(K * h.vs * r);
  L.vv = take(4 * K * h.vs * r);  // vertex vector and vorticity (bodies::VertexQ)
  L.gw = take(K1 * h.es * r);
  L.dvn = take(K * h.cs * r);
  L.wstar = take(K1 * h.cs * 8);
  L.wtmp = take(K1 * h.cs * 8);
  L.ttmp = take(K * h.cs * 8);  // theta_v staged for its diffusion
  L.tw0 = take(K1 * h.cs * r);
  L.fe = take(h.es * 8);
  L.tau = take(K1 * 8);
  const int nblk = (h.nc + 255) / 256 + (h.ne + 255) / 256;
  L.dpart = take(5 * (size_t)nblk * 8);
  L.dout = take(8 * 8);
  L.rhoe = L.the = 0;
  if (miura) {
    L.rhoe = take(K * h.es * 8);
    L.the = take(K * h.es * 8);
  }
  L.s_tmlp = L.s_cl = L.s_fj = L.s_fr = L.s_cnt = 0;
  if (diff == DC_DIFF_SURROGATE) {
    L.s_tmlp = take(K * h.es * r);
    L.s_cl = take(K * h.vs * r);  // curl L1 of the diffusion front
    L.s_fj = take((size_t)h.es * 4);
    L.s_fr = take((size_t)h.es * 4);
    L.s_cnt = take(8 * 4);  // 4 int counters, then one 64-bit counter
  }
  L.total = off;
  return L;
}

template <typename T>
dc_status upload(dc_grid* g, const std::vector<T>& v, const T** out) {
  void* p = nullptr;
  const size_t bytes = std::max<size_t>(v.size() * sizeof(T), 256);
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) return fail(DC_ENOMEM, std::string("hipMalloc(grid table): ") + hipGetErrorString(e));
  g->allocs.push_back(p);
  if (!v.empty()) DC_TRY(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  *out = static_cast<const T*>(p);
  return DC_OK;
}

dc_status ensure_uploaded(dc_grid* g) {
  if (g->uploaded) return DC_OK;
  const HostGrid& h = g->h;
  DevGrid& d = g->d;
  d.nc = h.nc;
  d.ne = h.ne;
  d.nv = h.nv;
  d.K = h.K;
  d.cs = h.cs;
  d.es = h.es;
  d.vs = h.vs;
  dc_status st;
#define UP(vec, field) \
  if ((st = upload(g, vec, &d.field)) != DC_OK) return st;
  UP(h.t_c2e, c2e);
  UP(h.t_c2e2c, c2e2c);
  UP(h.k_div, kdiv);
  UP(h.k_lap, klap);
  UP(h.k_area, area);
  UP(h.t_e2c, e2c);
  UP(h.t_e2v, e2v);
  UP(h.t_e2c2e, e2c2e);
  UP(h.t_e2c2v, e2c2v);
  UP(h.k_vt, kvt);
  UP(h.k_invd, invd);
  UP(h.k_invl, invl);
  UP(h.k_ae, ae);
  UP(h.k_invlr, invlr);
  UP(h.k_nrm, nrm);
  UP(h.k_tan, tan);
  UP(h.t_v2e, v2e);
  UP(h.k_curl, kcurl);
  UP(h.k_lsq, klsq);
  UP(h.vert, vert);
#undef UP
  d.fe = nullptr;
  d.tau = nullptr;
  d.kmiura = nullptr;
  d.et_ok = h.et_ok;
  d.et_ntile = h.et_ntile;
  d.et_n = d.et_x = d.et_vx = nullptr;
  d.et_nb = d.et_vl = d.et_ev = nullptr;
  if (h.et_ok) {
    if ((st = upload(g, h.et_n, &d.et_n)) != DC_OK) return st;
    if ((st = upload(g, h.et_x, &d.et_x)) != DC_OK) return st;
    if ((st = upload(g, h.et_vx, &d.et_vx)) != DC_OK) return st;
    if ((st = upload(g, h.et_nb, &d.et_nb)) != DC_OK) return st;
    if ((st = upload(g, h.et_vl, &d.et_vl)) != DC_OK) return st;
    if ((st = upload(g, h.et_ev, &d.et_ev)) != DC_OK) return st;
  }
  DC_TRY(hipGetDevice(&g->device));
  g->uploaded = true;
  return DC_OK;
}

// tables of the optional schemes a state asks for, built and uploaded once
dc_status ensure_options(dc_grid* g, const dc_params& p) {
  dc_status st;
  if (p.vt_rbf && !g->kvt_rbf) {
    bool ok = false;
    try {
      ok = build_rbf_vt(&g->h);
    } catch (const std::bad_alloc&) {
      return fail(DC_ENOMEM, "host allocation failed");
    }
    if (!ok) return fail(DC_EGRID, "singular RBF system at an edge");
    if ((st = upload(g, g->h.k_vt_rbf, &g->kvt_rbf)) != DC_OK) return st;
    std::vector<double>().swap(g->h.k_vt_rbf);
  }
  if (p.miura && !g->kmiura) {
    try {
      build_miura(&g->h);
    } catch (const std::bad_alloc&) {
      return fail(DC_ENOMEM, "host allocation failed");
    }
    if ((st = upload(g, g->h.k_miura, &g->kmiura)) != DC_OK) return st;
    std::vector<double>().swap(g->h.k_miura);
  }
  return DC_OK;
}

bool aligned(const void* p) { return p && (reinterpret_cast<uintptr_t>(p) % 256 == 0); }

size_t field_elems(const HostGrid& h, int field) {
  switch (field) {
    case DC_FIELD_VN: return (size_t)h.K * h.es;
    case DC_FIELD_W: return (size_t)(h.K + 1) * h.cs;
    default: return (size_t)h.K * h.cs;
  }
}
size_t field_host_elems(const HostGrid& h, int field) {
  switch (field) {
    case DC_FIELD_VN: return (size_t)h.K * h.ne;
    case DC_FIELD_W: return (size_t)(h.K + 1) * h.nc;
    default: return (size_t)h.K * h.nc;
  }
}
void* field_ptr(const dc_fields& f, int field) {
  switch (field) {
    case DC_FIELD_VN: return f.vn;
    case DC_FIELD_W: return f.w;
    case DC_FIELD_RHO: return f.rho;
    case DC_FIELD_EXNER: return f.exner;
    default: return f.theta_v;
  }
}

// the theta_v diffusion's fields: theta_v staged by the last substep, the
// current buffer set's theta_v and exner (null when it is off)
ThetaDiff theta_diff(const dc_state* s, const dc_fields& cur) {
  if (!s->p.diffuse_theta) return ThetaDiff{nullptr, nullptr, nullptr};
  return ThetaDiff{s->ttmp, static_cast<double*>(cur.theta_v), static_cast<double*>(cur.exner)};
}

template <typename R>
void enqueue_step(dc_state* s, double dt, int nsub) {
  const StepCoef c = make_coef(s, dt, nsub);
  const bool diffuse = s->diff != DC_DIFF_NONE;
  enqueue_substeps<R>(s, c, nsub, diffuse);
  if (s->diff == DC_DIFF_SURROGATE) {
    surrogate_diffusion<R>(s, c);
  } else if (diffuse) {
    const dc_fields& cur = s->buf[s->cur];
    launch_diffusion<R>(s->d, static_cast<R*>(cur.vn), s->wtmp, static_cast<double*>(cur.w), static_cast<R*>(s->vt),
                        static_cast<R*>(s->tvn0), static_cast<R*>(s->kc), static_cast<R*>(s->d2),
                        static_cast<R*>(s->zeta), static_cast<R*>(s->vv), theta_diff(s, cur), c, s->tiles, s->stream,
                        &s->prof);
  }
}

// One step with the plain diffusion (or none), whatever the state's mode: the
// timing trials of the tuner leave the surrogate's flags and counters alone.
template <typename R>
void enqueue_trial_step(dc_state* s, double dt, int nsub) {
  const StepCoef c = make_coef(s, dt, nsub);
  const bool diffuse = s->diff != DC_DIFF_NONE;
  enqueue_substeps<R>(s, c, nsub, diffuse);
  if (diffuse) {
    const dc_fields& cur = s->buf[s->cur];
    launch_diffusion<R>(s->d, static_cast<R*>(cur.vn), s->wtmp, static_cast<double*>(cur.w), static_cast<R*>(s->vt),
                        static_cast<R*>(s->tvn0), static_cast<R*>(s->kc), static_cast<R*>(s->d2),
                        static_cast<R*>(s->zeta), static_cast<R*>(s->vv), theta_diff(s, cur), c, s->tiles, s->stream,
                        &s->prof);
  }
}

// One part of a step (dc_dycore_part): the predictor or the corrector of one
// substep on the current buffer set, or the plain diffusion with its inputs
// first staged where the last substep of a step would have put them.
template <typename R>
hipError_t enqueue_part(dc_state* s, int part, double dt, int nsub) {
  const StepCoef c = make_coef(s, dt, nsub);
  if (part == DC_PART_PREDICTOR) {
    launch_predictor<R>(s->d, substep_bufs<R>(s, s->cur, false), c, s->tiles, s->stream, &s->prof);
    s->part = 1;
  } else if (part == DC_PART_CORRECTOR) {
    launch_corrector<R>(s->d, substep_bufs<R>(s, s->cur, false), c, s->tiles, s->stream, &s->prof);
    s->cur ^= 1;
    s->part = 2;
  } else {
    const dc_fields& cur = s->buf[s->cur];
    const size_t K = s->grid->h.K, cs = s->grid->h.cs;
    s->part = 0;
    hipError_t e = hipMemcpyAsync(s->wtmp, cur.w, (K + 1) * cs * 8, hipMemcpyDeviceToDevice, s->stream);
    if (e == hipSuccess && s->p.diffuse_theta)
      e = hipMemcpyAsync(s->ttmp, cur.theta_v, K * cs * 8, hipMemcpyDeviceToDevice, s->stream);
    if (e != hipSuccess) return e;
    launch_diffusion<R>(s->d, static_cast<R*>(cur.vn), s->wtmp, static_cast<double*>(cur.w), static_cast<R*>(s->vt),
                        static_cast<R*>(s->tvn0), static_cast<R*>(s->kc), static_cast<R*>(s->d2),
                        static_cast<R*>(s->zeta), static_cast<R*>(s->vv), theta_diff(s, cur), c, s->tiles, s->stream,
                        &s->prof);
  }
  return hipSuccess;
}

dc_status run_diag(dc_state* s, dc_diag* out) {
  const dc_fields& f = s->buf[s->cur];
  if (s->prec == DC_PREC_MIXED)
    launch_diag<float>(s->d, static_cast<const float*>(f.vn), static_cast<const double*>(f.w),
                       static_cast<const double*>(f.rho), static_cast<const double*>(f.theta_v),
                       static_cast<const double*>(f.exner), s->diag_part, s->diag_out, s->stream);
  else
    launch_diag<double>(s->d, static_cast<const double*>(f.vn), static_cast<const double*>(f.w),
                        static_cast<const double*>(f.rho), static_cast<const double*>(f.theta_v),
                        static_cast<const double*>(f.exner), s->diag_part, s->diag_out, s->stream);
  DC_TRY(hipGetLastError());
  double h[5];
  DC_TRY(hipMemcpyAsync(h, s->diag_out, sizeof(h), hipMemcpyDeviceToHost, s->stream));
  DC_TRY(hipStreamSynchronize(s->stream));
  out->fallback_fraction = 0.0;
  if (s->diff == DC_DIFF_SURROGATE) {
    int cnt[3];
    DC_TRY(hipMemcpy(cnt, s->sur_cnt, sizeof(cnt), hipMemcpyDeviceToHost));
    out->fallback_fraction = (double)cnt[2] / s->grid->h.ne;
  }
  out->mass = h[0];
  out->theta_mass = h[1];
  out->max_abs_w = h[2];
  out->max_abs_vn = h[3];
  out->n_nonfinite = (int64_t)h[4];
  return DC_OK;
}

}  // namespace

extern "C" {

const char* dc_last_error(void) { return g_last_error.c_str(); }

dc_status dc_params_default(dc_params* p) {
  if (!p) return fail(DC_EINVAL, "params is NULL");
  p->eta = 0.65;
  p->adv_w0 = 0.25;
  p->adv_w1 = 0.75;
  p->divdamp_c4 = 0.0025;
  p->rayleigh_tau0 = 0.05;
  p->rayleigh_zfrac = 2.0 / 3.0;
  p->smag_cs = 0.015;
  p->smag_cap = 16.0;
  p->hdiff_k4 = 1.0 / 128.0;
  p->rd = 287.04;
  p->cpd = 1004.64;
  p->cvd = 1004.64 - 287.04;
  p->omega = 7.29212e-5;
  p->diffuse_w = 1;
  p->check_finite = 0;
  p->diffuse_theta = 0;
  p->theta_enh_nlev = 0;
  p->theta_enh_thresh = 5.0;
  p->miura = 0;
  p->vt_rbf = 0;
  return DC_OK;
}

dc_status dc_grid_create(const dc_grid_desc* desc, dc_grid** out) {
  if (!out) return fail(DC_EINVAL, "out is NULL");
  *out = nullptr;
  dc_grid* g = new (std::nothrow) dc_grid();
  if (!g) return fail(DC_ENOMEM, "host allocation failed");
  std::string err;
  int rc;
  try {
    rc = build_host_grid(desc, &g->h, &err);
  } catch (const std::bad_alloc&) {
    rc = DC_ENOMEM;
    err = "host allocation failed";
  }
  if (rc != DC_OK) {
    delete g;
    return fail((dc_status)rc, err);
  }
  *out = g;
  set_error("");
  return DC_OK;
}

dc_status dc_grid_info_get(const dc_grid* g, dc_grid_info* info) {
  if (!g || !info) return fail(DC_EINVAL, "NULL argument");
  info->n_cells = g->h.nc;
  info->n_edges = g->h.ne;
  info->n_verts = g->h.nv;
  info->n_lev = g->h.K;
  info->cell_stride = g->h.cs;
  info->edge_stride = g->h.es;
  info->vert_stride = g->h.vs;
  info->fused_edge_pass = g->h.et_ok;
  return DC_OK;
}

dc_status dc_grid_table(const dc_grid* g, int32_t id, int32_t* out, size_t n) {
  if (!g || !out) return fail(DC_EINVAL, "NULL argument");
  const HostGrid& h = g->h;
  const std::vector<int32_t>* t = nullptr;
  switch (id) {
    case DC_TAB_E2C: t = &h.e2c; break;
    case DC_TAB_C2E: t = &h.c2e; break;
    case DC_TAB_E2V: t = &h.e2v; break;
    case DC_TAB_C2E2C: t = &h.c2e2c; break;
    case DC_TAB_C2V: t = &h.c2v; break;
    case DC_TAB_V2E: t = &h.v2e; break;
    case DC_TAB_V2C: t = &h.v2c; break;
    case DC_TAB_E2C2E: t = &h.e2c2e; break;
    case DC_TAB_E2C2V: t = &h.e2c2v; break;
    case DC_TAB_PERM_CELL: t = &h.perm_c; break;
    case DC_TAB_PERM_EDGE: t = &h.perm_e; break;
    case DC_TAB_PERM_VERT: t = &h.perm_v; break;
    default: return fail(DC_EINVAL, "unknown table id");
  }
  if (n != t->size()) return fail(DC_EINVAL, "table size mismatch: expected " + std::to_string(t->size()));
  std::memcpy(out, t->data(), n * sizeof(int32_t));
  return DC_OK;
}

dc_status dc_grid_destroy(dc_grid* g) {
  if (!g) return fail(DC_EINVAL, "grid is NULL");
  if (g->states.load() > 0) return fail(DC_EBUSY, "grid still has live states");
  for (void* p : g->allocs) (void)hipFree(p);
  delete g;
  return DC_OK;
}

dc_status dc_field_bytes(const dc_grid* g, dc_precision prec, int32_t field, size_t* bytes) {
  if (!g || !bytes) return fail(DC_EINVAL, "NULL argument");
  if (prec != DC_PREC_FP64 && prec != DC_PREC_MIXED) return fail(DC_EINVAL, "bad precision");
  if (field < 0 || field >= DC_FIELD_COUNT) return fail(DC_EINVAL, "bad field id");
  const size_t es = (field == DC_FIELD_VN && prec == DC_PREC_MIXED) ? 4 : 8;
  *bytes = field_elems(g->h, field) * es;
  return DC_OK;
}

dc_status dc_state_workspace_bytes(const dc_grid* g, dc_precision prec, dc_diffusion diff, size_t* bytes) {
  if (!g || !bytes) return fail(DC_EINVAL, "NULL argument");
  if (prec != DC_PREC_FP64 && prec != DC_PREC_MIXED) return fail(DC_EINVAL, "bad precision");
  if (diff != DC_DIFF_PLAIN && diff != DC_DIFF_NONE && diff != DC_DIFF_SURROGATE)
    return fail(DC_EINVAL, "bad diffusion mode");
  *bytes = workspace_layout(g->h, prec, diff, false).total;
  return DC_OK;
}

dc_status dc_state_workspace_bytes_params(const dc_grid* g, const dc_params* params, dc_precision prec,
                                          dc_diffusion diff, size_t* bytes) {
  if (!g || !params || !bytes) return fail(DC_EINVAL, "NULL argument");
  if (prec != DC_PREC_FP64 && prec != DC_PREC_MIXED) return fail(DC_EINVAL, "bad precision");
  if (diff != DC_DIFF_PLAIN && diff != DC_DIFF_NONE && diff != DC_DIFF_SURROGATE)
    return fail(DC_EINVAL, "bad diffusion mode");
  *bytes = workspace_layout(g->h, prec, diff, params->miura != 0).total;
  return DC_OK;
}

dc_status dc_state_create(const dc_grid* gc, const dc_params* params, dc_precision prec, dc_diffusion diff,
                          dc_fields a, dc_fields b, void* workspace, size_t ws_bytes, void* stream, dc_state** out) {
  if (!gc || !params || !out) return fail(DC_EINVAL, "NULL argument");
  *out = nullptr;
  dc_grid* g = const_cast<dc_grid*>(gc);
  if (prec != DC_PREC_FP64 && prec != DC_PREC_MIXED) return fail(DC_EINVAL, "bad precision");
  if (diff != DC_DIFF_PLAIN && diff != DC_DIFF_NONE && diff != DC_DIFF_SURROGATE)
    return fail(DC_EINVAL, "bad diffusion mode");
  const dc_fields* bs[2] = {&a, &b};
  for (int i = 0; i < 2; ++i)
    for (int f = 0; f < DC_FIELD_COUNT; ++f)
      if (!aligned(field_ptr(*bs[i], f))) return fail(DC_EINVAL, "field buffers must be non-NULL and 256-byte aligned");
  if ((params->miura != 0 && params->miura != 1) || (params->vt_rbf != 0 && params->vt_rbf != 1))
    return fail(DC_EINVAL, "miura and vt_rbf must be 0 or 1");
  const Layout L = workspace_layout(g->h, prec, diff, params->miura != 0);
  if (!aligned(workspace)) return fail(DC_EINVAL, "workspace must be non-NULL and 256-byte aligned");
  if (ws_bytes < L.total) return fail(DC_EINVAL, "workspace too small: need " + std::to_string(L.total) + " bytes");
  const dc_params& p = *params;
  if (!(p.eta >= 0.5 && p.eta <= 1.0) || !(p.rd > 0 && p.cpd > p.rd && p.cvd > 0) || !(p.smag_cap > 0) ||
      !(p.rayleigh_zfrac > 0 && p.rayleigh_zfrac < 1) || p.rayleigh_tau0 < 0 || p.divdamp_c4 < 0 || p.hdiff_k4 < 0 ||
      p.smag_cs < 0 || !std::isfinite(p.omega) || (p.diffuse_theta != 0 && p.diffuse_theta != 1))
    return fail(DC_EINVAL, "parameter out of range");
  if (p.theta_enh_nlev < 0 || p.theta_enh_nlev > g->h.K || !(p.theta_enh_thresh > 0) ||
      !std::isfinite(p.theta_enh_thresh))
    return fail(DC_EINVAL, "theta_enh_nlev must lie in 0..n_lev and theta_enh_thresh be positive");
  if (p.theta_enh_nlev > 0 && !p.diffuse_theta)
    return fail(DC_EINVAL, "theta_enh_nlev needs diffuse_theta");
  if (p.diffuse_theta && diff == DC_DIFF_SURROGATE)
    return fail(DC_EINVAL, "theta_v diffusion is available with the plain diffusion only");
  dc_status st = ensure_uploaded(g);
  if (st != DC_OK) return st;
  if ((st = ensure_options(g, p)) != DC_OK) return st;
  int dev = -1;
  DC_TRY(hipGetDevice(&dev));
  if (dev != g->device) return fail(DC_EINVAL, "state must be created on the grid's device");

  dc_state* s = new (std::nothrow) dc_state();
  if (!s) return fail(DC_ENOMEM, "host allocation failed");
  s->grid = g;
  s->p = p;
  s->prec = prec;
  s->diff = diff;
  s->buf[0] = a;
  s->buf[1] = b;
  s->stream = static_cast<hipStream_t>(stream);
  s->ws = static_cast<char*>(workspace);
  s->ws_bytes = ws_bytes;
  char* w = s->ws;
  s->vt = w + L.vt;
  s->tvn0 = w + L.tvn0;
  s->vns = w + L.vns;
  s->kc = w + L.kc;
  s->d2 = w + L.d2;
  s->zeta = w + L.zeta;
  s->vv = w + L.vv;
  s->gw = w + L.gw;
  s->dvn = w + L.dvn;
  s->wstar = reinterpret_cast<double*>(w + L.wstar);
  s->wtmp = reinterpret_cast<double*>(w + L.wtmp);
  s->ttmp = reinterpret_cast<double*>(w + L.ttmp);
  s->tw0 = w + L.tw0;
  s->fe = reinterpret_cast<double*>(w + L.fe);
  s->tau = reinterpret_cast<double*>(w + L.tau);
  s->diag_part = reinterpret_cast<double*>(w + L.dpart);
  s->diag_out = reinterpret_cast<double*>(w + L.dout);
  if (p.miura) {
    s->rhoe = reinterpret_cast<double*>(w + L.rhoe);
    s->the = reinterpret_cast<double*>(w + L.the);
  }
  if (diff == DC_DIFF_SURROGATE) {
    s->sur_tmlp = w + L.s_tmlp;
    s->sur_cl = w + L.s_cl;
    s->sur_fj = reinterpret_cast<int*>(w + L.s_fj);
    s->sur_fr = reinterpret_cast<int*>(w + L.s_fr);
    s->sur_cnt = reinterpret_cast<int*>(w + L.s_cnt);
    surrogate_geometry(s);
  }
  // per-state tables: Coriolis parameter and sponge profile
  const HostGrid& h = g->h;
  std::vector<double> fe(h.es, 0.0), tau(h.K + 1, 0.0);
  for (int e = 0; e < h.ne; ++e) fe[e] = 2.0 * p.omega * h.xe[3 * e + 2];
  const double ztop = h.z_half[0], zd = p.rayleigh_zfrac * ztop;
  for (int k = 0; k <= h.K; ++k) {
    const double z = h.z_half[k];
    if (z > zd) {
      const double sn = std::sin(0.5 * M_PI * (z - zd) / (ztop - zd));
      tau[k] = p.rayleigh_tau0 * sn * sn;
    }
  }
  hipError_t e1 = hipMemcpy(s->fe, fe.data(), fe.size() * 8, hipMemcpyHostToDevice);
  hipError_t e2 = hipMemcpy(s->tau, tau.data(), tau.size() * 8, hipMemcpyHostToDevice);
  if (e1 == hipSuccess && e2 == hipSuccess && diff == DC_DIFF_SURROGATE) {
    // flags and counters start cleared (the first surrogate step judges)
    e1 = hipMemset(w + L.s_fj, 0, L.s_cnt + 32 - L.s_fj);
  }
  if (e1 != hipSuccess || e2 != hipSuccess) {
    delete s;
    return fail(DC_EHIP, std::string("hipMemcpy(state tables): ") + hipGetErrorString(e1 != hipSuccess ? e1 : e2));
  }
  s->d = g->d;
  s->d.fe = s->fe;
  s->d.tau = s->tau;
  if (p.vt_rbf) s->d.kvt = g->kvt_rbf;
  s->d.kmiura = p.miura ? g->kmiura : nullptr;
  default_tiles(h, s->tiles);
  g->states.fetch_add(1);
  *out = s;
  return DC_OK;
}

dc_status dc_state_current(const dc_state* s, int32_t* which) {
  if (!s || !which) return fail(DC_EINVAL, "NULL argument");
  *which = s->cur;
  return DC_OK;
}

dc_status dc_state_read(dc_state* s, int32_t field, double* host, size_t n) {
  if (!s || !host) return fail(DC_EINVAL, "NULL argument");
  if (field < 0 || field >= DC_FIELD_COUNT) return fail(DC_EINVAL, "bad field id");
  const HostGrid& h = s->grid->h;
  if (n != field_host_elems(h, field)) return fail(DC_EINVAL, "host array size mismatch");
  const size_t ne_pad = field_elems(h, field);
  const bool f32 = field == DC_FIELD_VN && s->prec == DC_PREC_MIXED;
  std::vector<double> tmp(ne_pad);
  std::vector<float> tmpf(f32 ? ne_pad : 0);
  DC_TRY(hipStreamSynchronize(s->stream));
  void* src = field_ptr(s->buf[s->cur], field);
  if (f32)
    DC_TRY(hipMemcpy(tmpf.data(), src, ne_pad * 4, hipMemcpyDeviceToHost));
  else
    DC_TRY(hipMemcpy(tmp.data(), src, ne_pad * 8, hipMemcpyDeviceToHost));
  const int stride = field == DC_FIELD_VN ? h.es : h.cs;
  const int nent = field == DC_FIELD_VN ? h.ne : h.nc;
  const std::vector<int32_t>& perm = field == DC_FIELD_VN ? h.perm_e : h.perm_c;
  const int levels = field == DC_FIELD_W ? h.K + 1 : h.K;
  for (int k = 0; k < levels; ++k)
    for (int i = 0; i < nent; ++i) {
      const size_t src_i = (size_t)k * stride + i;
      host[(size_t)k * nent + perm[i]] = f32 ? (double)tmpf[src_i] : tmp[src_i];
    }
  return DC_OK;
}

dc_status dc_state_write(dc_state* s, int32_t field, const double* host, size_t n) {
  if (!s || !host) return fail(DC_EINVAL, "NULL argument");
  if (field < 0 || field >= DC_FIELD_COUNT) return fail(DC_EINVAL, "bad field id");
  const HostGrid& h = s->grid->h;
  if (n != field_host_elems(h, field)) return fail(DC_EINVAL, "host array size mismatch");
  const size_t ne_pad = field_elems(h, field);
  const bool f32 = field == DC_FIELD_VN && s->prec == DC_PREC_MIXED;
  const int stride = field == DC_FIELD_VN ? h.es : h.cs;
  const int nent = field == DC_FIELD_VN ? h.ne : h.nc;
  const std::vector<int32_t>& perm = field == DC_FIELD_VN ? h.perm_e : h.perm_c;
  const int levels = field == DC_FIELD_W ? h.K + 1 : h.K;
  std::vector<double> tmp(f32 ? 0 : ne_pad, 0.0);
  std::vector<float> tmpf(f32 ? ne_pad : 0, 0.0f);
  for (int k = 0; k < levels; ++k)
    for (int i = 0; i < nent; ++i) {
      const double x = host[(size_t)k * nent + perm[i]];
      const size_t dst = (size_t)k * stride + i;
      if (f32)
        tmpf[dst] = (float)x;
      else
        tmp[dst] = x;
    }
  DC_TRY(hipStreamSynchronize(s->stream));
  void* dstp = field_ptr(s->buf[s->cur], field);
  if (f32)
    DC_TRY(hipMemcpy(dstp, tmpf.data(), ne_pad * 4, hipMemcpyHostToDevice));
  else
    DC_TRY(hipMemcpy(dstp, tmp.data(), ne_pad * 8, hipMemcpyHostToDevice));
  return DC_OK;
}

dc_status dc_dycore_step(dc_state* s, double dt, int32_t nsub) {
  if (!s) return fail(DC_EINVAL, "state is NULL");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(DC_EINVAL, "dt must be finite and > 0");
  if (nsub < 1 || nsub > 1000) return fail(DC_EINVAL, "nsubsteps must be in [1, 1000]");
  if (s->diff == DC_DIFF_SURROGATE && !s->sur) return fail(DC_ESTATE, "surrogate mode needs dc_state_set_mlp first");
  s->part = 0;
  if (s->prec == DC_PREC_MIXED)
    enqueue_step<float>(s, dt, nsub);
  else
    enqueue_step<double>(s, dt, nsub);
  DC_TRY(hipGetLastError());
  if (s->p.check_finite) {
    dc_diag d;
    dc_status st = run_diag(s, &d);
    if (st != DC_OK) return st;
    if (d.n_nonfinite > 0) return fail(DC_ENONFINITE, "state holds non-finite values");
  }
  return DC_OK;
}

dc_status dc_dycore_part(dc_state* s, int32_t part, double dt, int32_t nsub) {
  if (!s) return fail(DC_EINVAL, "state is NULL");
  if (part < DC_PART_PREDICTOR || part > DC_PART_DIFFUSION) return fail(DC_EINVAL, "bad part");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(DC_EINVAL, "dt must be finite and > 0");
  if (nsub < 1 || nsub > 1000) return fail(DC_EINVAL, "nsubsteps must be in [1, 1000]");
  if (part == DC_PART_CORRECTOR && s->part != 1) return fail(DC_ESTATE, "the corrector needs a predictor just before");
  if (part == DC_PART_DIFFUSION && s->diff != DC_DIFF_PLAIN)
    return fail(DC_ESTATE, "the diffusion part needs a state with the plain diffusion");
  DC_TRY(s->prec == DC_PREC_MIXED ? enqueue_part<float>(s, part, dt, nsub) : enqueue_part<double>(s, part, dt, nsub));
  DC_TRY(hipGetLastError());
  return DC_OK;
}

dc_status dc_state_read_work(dc_state* s, int32_t which, double* host, size_t n) {
  if (!s || !host) return fail(DC_EINVAL, "NULL argument");
  if (which < 0 || which >= DC_WORK_COUNT) return fail(DC_EINVAL, "bad workspace field id");
  if (s->part == 0) return fail(DC_ESTATE, "no predictor part ran since the workspace was last overwritten");
  const HostGrid& h = s->grid->h;
  const bool edge = which == DC_WORK_VN_PRED || which == DC_WORK_Y;
  const bool half = which == DC_WORK_W_PRED || which == DC_WORK_T_W;
  const int levels = half ? h.K + 1 : h.K;
  const int nent = edge ? h.ne : h.nc, stride = edge ? h.es : h.cs;
  if (n != (size_t)levels * nent) return fail(DC_EINVAL, "host array size mismatch");
  const bool f32 = which != DC_WORK_W_PRED && s->prec == DC_PREC_MIXED;
  const void* src = which == DC_WORK_VN_PRED ? s->vns
                    : which == DC_WORK_Y     ? s->tvn0
                    : which == DC_WORK_W_PRED ? static_cast<const void*>(s->wstar)
                    : which == DC_WORK_T_W   ? s->tw0
                                             : s->dvn;
  const size_t np = (size_t)levels * stride;
  std::vector<double> tmp(f32 ? 0 : np);
  std::vector<float> tmpf(f32 ? np : 0);
  DC_TRY(hipStreamSynchronize(s->stream));
  if (f32)
    DC_TRY(hipMemcpy(tmpf.data(), src, np * 4, hipMemcpyDeviceToHost));
  else
    DC_TRY(hipMemcpy(tmp.data(), src, np * 8, hipMemcpyDeviceToHost));
  const std::vector<int32_t>& perm = edge ? h.perm_e : h.perm_c;
  for (int k = 0; k < levels; ++k) {
    // T_w lives on the interior half levels only
    const bool zero = which == DC_WORK_T_W && (k == 0 || k == h.K);
    for (int i = 0; i < nent; ++i) {
      const size_t si = (size_t)k * stride + i;
      host[(size_t)k * nent + perm[i]] = zero ? 0.0 : (f32 ? (double)tmpf[si] : tmp[si]);
    }
  }
  return DC_OK;
}

dc_status dc_diag_conservation(dc_state* s, dc_diag* out) {
  if (!s || !out) return fail(DC_EINVAL, "NULL argument");
  return run_diag(s, out);
}

dc_status dc_state_profile(dc_state* s, int32_t enable) {
  if (!s) return fail(DC_EINVAL, "state is NULL");
  DC_TRY(hipStreamSynchronize(s->stream));
  s->prof.on = enable != 0;
  s->prof.used = 0;
  return DC_OK;
}

dc_status dc_state_profile_select(dc_state* s, uint32_t kernel_mask) {
  if (!s) return fail(DC_EINVAL, "state is NULL");
  DC_TRY(hipStreamSynchronize(s->stream));
  s->prof.mask = kernel_mask == 0 ? ~0u : kernel_mask;
  return DC_OK;
}


dc_status dc_state_autotune(dc_state* s, double dt, int32_t nsub) {
  if (!s) return fail(DC_EINVAL, "state is NULL");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(DC_EINVAL, "dt must be finite and > 0");
  if (nsub < 1 || nsub > 1000) return fail(DC_EINVAL, "nsubsteps must be in [1, 1000]");
  s->part = 0;  // the trial steps overwrite the workspace
  DC_TRY(hipStreamSynchronize(s->stream));
  // the trial steps advance the state: keep a copy of the current fields
  const int parity = s->cur;
  void* saved[DC_FIELD_COUNT] = {};
  size_t bytes[DC_FIELD_COUNT] = {};
  auto release = [&]() {
    for (void* p : saved)
      if (p) (void)hipFree(p);
  };
  for (int f = 0; f < DC_FIELD_COUNT; ++f) {
    dc_field_bytes(s->grid, s->prec, f, &bytes[f]);
    if (hipMalloc(&saved[f], bytes[f]) != hipSuccess) {
      saved[f] = nullptr;
      release();
      return fail(DC_ENOMEM, "autotune: no memory for the copy of the fields");
    }
    if (hipMemcpyAsync(saved[f], field_ptr(s->buf[parity], f), bytes[f], hipMemcpyDeviceToDevice, s->stream) !=
        hipSuccess) {
      release();
      return fail(DC_EHIP, "autotune: copy of the fields failed");
    }
  }
  // candidates: threads x near-equal level blocks
  const int K = s->grid->h.K;
  std::vector<Tile> cands;
  for (int th : {64, 128, 256}) {
    int last = 0;
    for (int nby : {1, 2, 3, 4, 5, 6, 8, 11}) {
      const int kb = (K + nby - 1) / nby;
      if (kb != last) cands.push_back({th, kb});
      last = kb;
    }
  }
  static const std::vector<std::vector<int>> uses = {
      {K_VC_P, K_VC_C}, {K_EDGE_P, K_EDGE_C, K_MIURA}, {K_DVERT}, {K_DDIV, K_DCV2}, {K_DEDGE1, K_DEDGE2}};
  const Tile tile0[T_COUNT] = {s->tiles[0], s->tiles[1], s->tiles[2], s->tiles[3], s->tiles[4]};
  const bool prof_on = s->prof.on;
  const unsigned prof_mask = s->prof.mask;
  std::vector<double> best(T_COUNT, 1e300);
  std::vector<Tile> best_tile(tile0, tile0 + T_COUNT);
  hipError_t err = hipSuccess;
  for (size_t ci = 0; ci < cands.size() && err == hipSuccess; ++ci) {
    for (int t = 0; t < T_COUNT; ++t) s->tiles[t] = cands[ci];
    double per[K_COUNT];
    for (int rep = 0; rep < 2 && err == hipSuccess; ++rep) {
      s->prof.on = true;
      s->prof.mask = ~0u;
      s->prof.used = 0;
      if (s->prec == DC_PREC_MIXED)
        enqueue_trial_step<float>(s, dt, nsub);
      else
        enqueue_trial_step<double>(s, dt, nsub);
      s->prof.on = false;
      err = hipGetLastError();
      if (err == hipSuccess) err = hipStreamSynchronize(s->stream);
      double cur[K_COUNT] = {0};
      for (size_t i = 0; i + 1 < s->prof.used && err == hipSuccess; ++i)
        if (s->prof.kid[i] >= 0 && s->prof.kid[i + 1] == -1) {
          float ms = 0.f;
          err = hipEventElapsedTime(&ms, s->prof.ev[i], s->prof.ev[i + 1]);
          cur[s->prof.kid[i]] += ms;
        }
      for (int k = 0; k < K_COUNT; ++k) per[k] = rep == 0 ? cur[k] : std::min(per[k], cur[k]);
    }
    for (int t = 0; t < T_COUNT && err == hipSuccess; ++t) {
      double sum = 0.0;
      for (int k : uses[t]) sum += per[k];
      if (sum < best[t]) {
        best[t] = sum;
        best_tile[t] = cands[ci];
      }
    }
  }
  // restore the fields, the parity and the profiler
  s->cur = parity;
  for (int f = 0; f < DC_FIELD_COUNT && err == hipSuccess; ++f)
    err = hipMemcpyAsync(field_ptr(s->buf[parity], f), saved[f], bytes[f], hipMemcpyDeviceToDevice, s->stream);
  if (err == hipSuccess) err = hipStreamSynchronize(s->stream);
  release();
  s->prof.on = prof_on;
  s->prof.mask = prof_mask;
  s->prof.used = 0;
  if (err != hipSuccess) {
    std::copy(tile0, tile0 + T_COUNT, s->tiles);
    return fail(DC_EHIP, std::string("autotune trial failed: ") + hipGetErrorString(err));
  }
  std::copy(best_tile.begin(), best_tile.end(), s->tiles);
  return DC_OK;
}

dc_status dc_state_tiles(const dc_state* s, int32_t* out, int32_t n) {
  if (!s || !out) return fail(DC_EINVAL, "NULL argument");
  if (n < 2 * T_COUNT) return fail(DC_EINVAL, "need room for 10 values");
  for (int t = 0; t < T_COUNT; ++t) {
    out[2 * t] = s->tiles[t].threads;
    out[2 * t + 1] = s->tiles[t].kb;
  }
  return DC_OK;
}

dc_status dc_state_profile_read(dc_state* s, dc_kernel_stat* out, int32_t cap, int32_t* n_out) {
  if (!s || !out || !n_out || cap < K_COUNT) return fail(DC_EINVAL, "NULL argument or capacity < kernel count");
  DC_TRY(hipStreamSynchronize(s->stream));
  for (int k = 0; k < K_COUNT; ++k) {
    std::memset(out[k].name, 0, sizeof(out[k].name));
    std::strncpy(out[k].name, kKernelNames[k], sizeof(out[k].name) - 1);
    out[k].calls = 0;
    out[k].total_ms = 0.0;
  }
  const Prof& p = s->prof;
  for (size_t i = 0; i + 1 < p.used; ++i) {
    if (p.kid[i] >= 0 && p.kid[i + 1] == -1) {
      float ms = 0.f;
      DC_TRY(hipEventElapsedTime(&ms, p.ev[i], p.ev[i + 1]));
      out[p.kid[i]].calls += 1;
      out[p.kid[i]].total_ms += ms;
    }
  }
  *n_out = K_COUNT;
  return DC_OK;
}

dc_status dc_state_destroy(dc_state* s) {
  if (!s) return fail(DC_EINVAL, "state is NULL");
  hipError_t e = hipStreamSynchronize(s->stream);
  for (hipEvent_t ev : s->prof.ev) (void)hipEventDestroy(ev);
  s->grid->states.fetch_sub(1);
  surrogate_free(s);
  delete s;
  if (e != hipSuccess) return fail(DC_EHIP, std::string("pending work failed: ") + hipGetErrorString(e));
  return DC_OK;
}

}  // extern "C"
