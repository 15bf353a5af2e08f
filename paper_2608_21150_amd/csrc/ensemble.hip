// Batched ensemble stepping: members on any grids (same precision, same
// number of levels) advance together.  Every phase of the step is ONE
// persistent kernel launch whose blocks walk a (member, tile) work table;
// the whole step (nsub substeps and diffusion, i.e. 6 * nsub + 5 phases) is
// captured once into a hipGraph and replayed with a single hipGraphLaunch.
// This removes the per-member, per-kernel launch overhead that the paper
// hides by launching asynchronously from Python (Section 4.3.3).
//
// The tile and grid schedules come from a small autotuner that times each
// candidate on the ensemble itself and keeps the winner in a plain-text
// cache file keyed by precision, levels and member sizes.  Every candidate
// computes bit-identical results (per-entity arithmetic does not depend on
// the launch geometry), so tuning never changes the answer.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "bodies.h"
#include "internal.h"
#include "kernels.h"
#include "state.h"

using namespace dc;
using namespace dc::bodies;

namespace {

// One phase launch of a planned step: a work table in the device blob.
struct Rec {
  int phase;  // KernelId
  int lm;     // column chunk length (column phases)
  size_t jobs_off, ts_off;
  int nm, total, threads;
  size_t smem;
};

struct GraphEntry {
  double dt;
  int nsub, parity;
  hipGraph_t graph;
  hipGraphExec_t exec;
  void* blob;
};

}  // namespace

struct dc_ensemble {
  std::vector<dc_state*> m;
  dc_precision prec;
  int K = 0;
  hipStream_t stream = nullptr;
  Tile tiles[T_COUNT];
  int gfac[K_COUNT];  // persistent grid: blocks per CU; 0 = one block per tile
  int n_cu = 256;
  std::vector<GraphEntry> graphs;
  hipEvent_t done = nullptr;   // recorded after each ensemble step
  hipEvent_t ready = nullptr;  // member stream -> ensemble stream ordering
  Prof prof;
};

namespace {

#define EN_TRY(expr)                                                    \
  do {                                                                  \
    hipError_t _e = (expr);                                             \
    if (_e != hipSuccess) {                                             \
      set_error(std::string(#expr) + ": " + hipGetErrorString(_e));     \
      return DC_EHIP;                                                   \
    }                                                                   \
  } while (0)

dc_status efail(dc_status c, const std::string& m) {
  set_error(m);
  return c;
}

template <typename A>
size_t append_table(std::vector<char>& blob, const std::vector<Job<A>>& jobs, const std::vector<int>& ts,
                    size_t* ts_off) {
  auto put = [&](const void* p, size_t n) {
    const size_t off = (blob.size() + 255) / 256 * 256;
    blob.resize(off + n);
    std::memcpy(blob.data() + off, p, n);
    return off;
  };
  const size_t off = put(jobs.data(), jobs.size() * sizeof(Job<A>));
  *ts_off = put(ts.data(), ts.size() * sizeof(int));
  return off;
}

// Build the job tables of every phase of one step of every member.
template <typename R>
void plan_step(dc_ensemble* E, double dt, int nsub, int parity, std::vector<char>& blob, std::vector<Rec>& recs) {
  const int nm = (int)E->m.size();
  const bool diffuse = E->m[0]->diff != DC_DIFF_NONE;
  auto table = [&](int phase, auto&& args_of) {
    using A = std::decay_t<decltype(args_of(0))>;
    std::vector<Job<A>> jobs(nm);
    std::vector<int> ts(nm + 1, 0);
    Geom geo{};
    size_t smem = 0;  // the largest member's need (fused edge passes use LDS)
    for (int i = 0; i < nm; ++i) {
      const dc_state* s = E->m[i];
      geo = geom_of(phase, s->d, E->tiles, sizeof(R));
      smem = std::max(smem, geo.smem);
      jobs[i].g = s->d;
      jobs[i].a = args_of(i);
      jobs[i].nbx = geo.nbx;
      ts[i + 1] = ts[i] + geo.nbx * geo.nby;
    }
    Rec r{};
    r.phase = phase;
    col_chunks_lm(E->K, phase == K_COL_C, &r.lm);
    r.jobs_off = append_table(blob, jobs, ts, &r.ts_off);
    r.nm = nm;
    r.total = ts[nm];
    r.threads = geo.threads;
    r.smem = smem;
    recs.push_back(r);
  };
  for (int i = 0; i < nsub; ++i) {
    std::vector<SubstepArgs<R>> sa(nm);
    for (int k = 0; k < nm; ++k) {
      const dc_state* s = E->m[k];
      const Bufs<R> b = substep_bufs<R>(s, (parity + i) & 1, i == nsub - 1 && diffuse);
      sa[k] = substep_args<R>(s->d, b, make_coef(s, dt, nsub), E->tiles);
    }
    table(K_VC_P, [&](int k) { return sa[k].vc_p; });
    if (E->m[0]->p.miura) table(K_MIURA, [&](int k) { return sa[k].mi; });
    table(K_EDGE_P, [&](int k) { return sa[k].e_p; });
    table(K_COL_P, [&](int k) { return sa[k].c_p; });
    table(K_VC_C, [&](int k) { return sa[k].vc_c; });
    table(K_EDGE_C, [&](int k) { return sa[k].e_c; });
    table(K_COL_C, [&](int k) { return sa[k].c_c; });
  }
  if (diffuse) {
    const int fin = (parity + nsub) & 1;
    std::vector<DiffusionArgs<R>> da(nm);
    for (int k = 0; k < nm; ++k) {
      dc_state* s = E->m[k];
      const dc_fields& f = s->buf[fin];
      da[k] = diffusion_args<R>(s->d, static_cast<R*>(f.vn), s->wtmp, static_cast<double*>(f.w),
                                static_cast<R*>(s->vt), static_cast<R*>(s->tvn0), static_cast<R*>(s->kc),
                                static_cast<R*>(s->d2), static_cast<R*>(s->zeta), static_cast<R*>(s->vv),
                                make_coef(s, dt, nsub), E->tiles,
                                s->p.diffuse_theta ? ThetaDiff{s->ttmp, static_cast<double*>(f.theta_v),
                                                               static_cast<double*>(f.exner)}
                                                   : ThetaDiff{nullptr, nullptr, nullptr});
    }
    table(K_DVERT, [&](int k) { return da[k].dv; });
    table(K_DDIV, [&](int k) { return da[k].dd; });
    table(K_DEDGE1, [&](int k) { return da[k].d1; });
    table(K_DCV2, [&](int k) { return da[k].cv; });
    table(K_DEDGE2, [&](int k) { return da[k].d2; });
  }
}

template <typename B>
void many(const Rec& r, const char* base, int grid, hipStream_t s) {
  using J = Job<typename B::Args>;
  k_many<B><<<grid, r.threads, r.smem, s>>>(reinterpret_cast<const J*>(base + r.jobs_off),
                                           reinterpret_cast<const int*>(base + r.ts_off), r.nm);
}

template <typename R, bool CORR>
void many_col(const Rec& r, const char* base, int grid, hipStream_t s) {
  if (r.lm == 8)
    many<BCol<R, CORR, 8>>(r, base, grid, s);
  else if (r.lm == 12)
    many<BCol<R, CORR, 12>>(r, base, grid, s);
  else
    many<BCol<R, CORR, 16>>(r, base, grid, s);
}

template <typename R>
void launch_recs(dc_ensemble* E, const std::vector<Rec>& recs, const char* base, hipStream_t s, Prof* prof) {
  for (const Rec& r : recs) {
    const int g = E->gfac[r.phase] > 0 ? std::min(r.total, E->gfac[r.phase] * E->n_cu) : r.total;
    if (g <= 0) continue;
    if (prof) prof->mark(s, r.phase);
    switch (r.phase) {
      case K_VC_P: many<BVc<R, false>>(r, base, g, s); break;
      case K_EDGE_P: many<BEdge<R, false>>(r, base, g, s); break;
      case K_COL_P: many_col<R, false>(r, base, g, s); break;
      case K_VC_C: many<BVc<R, true>>(r, base, g, s); break;
      case K_EDGE_C: many<BEdge<R, true>>(r, base, g, s); break;
      case K_COL_C: many_col<R, true>(r, base, g, s); break;
      case K_DVERT: many<BDvert<R>>(r, base, g, s); break;
      case K_DDIV: many<BDiv<R>>(r, base, g, s); break;
      case K_DEDGE1: many<BDedge1<R>>(r, base, g, s); break;
      case K_DCV2: many<BDcv2<R>>(r, base, g, s); break;
      case K_MIURA: many<BMiura<R>>(r, base, g, s); break;
      default: many<BDedge2<R>>(r, base, g, s); break;
    }
    if (prof) prof->mark(s, -1);
  }
}

void free_graphs(dc_ensemble* E) {
  for (GraphEntry& g : E->graphs) {
    (void)hipGraphExecDestroy(g.exec);
    (void)hipGraphDestroy(g.graph);
    (void)hipFree(g.blob);
  }
  E->graphs.clear();
}

// Upload a plan; returns the device blob (caller frees).
dc_status upload_plan(const std::vector<char>& blob, void** dev) {
  *dev = nullptr;
  EN_TRY(hipMalloc(dev, std::max<size_t>(blob.size(), 256)));
  EN_TRY(hipMemcpy(*dev, blob.data(), blob.size(), hipMemcpyHostToDevice));
  return DC_OK;
}

// ---------------------------------------------------------------------------
// allocation-free eager step: the step's work tables go into a file-scope
// device array instead of memory allocated per call.  Each GPU holds its own
// copy of the array; its address comes from hipGetSymbolAddress once per
// device (the array's name is a host-side stand-in, never a device address)
// ---------------------------------------------------------------------------
constexpr size_t kStaticPlanBytes = (size_t)DC_STATIC_PLAN_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticPlanBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on device dev (looked up on first use, with dev
// current)
dc_status scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (dev < 0 || dev >= kMaxDevices) return efail(DC_EINVAL, "device id out of range for the static work table");
  if (!g_scratch_ptr[dev]) {
    int cur = -1;
    EN_TRY(hipGetDevice(&cur));
    if (cur != dev) EN_TRY(hipSetDevice(dev));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p)
      return efail(DC_EHIP, std::string("hipGetSymbolAddress(static work table): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return DC_OK;
}

enum class StepMode { Graph, Eager, Static };

template <typename R>
dc_status step_impl(dc_ensemble* E, double dt, int nsub, StepMode mode, Prof* prof) {
  const int parity = E->m[0]->cur;
  // eager modes: plan on the host first, so that a plan too large for the
  // static table is refused before anything is enqueued
  std::vector<char> blob;
  std::vector<Rec> recs;
  void* table = nullptr;
  if (mode != StepMode::Graph) plan_step<R>(E, dt, nsub, parity, blob, recs);
  if (mode == StepMode::Static) {
    if (blob.size() > kStaticPlanBytes)
      return efail(DC_EINVAL, "the step's work tables (" + std::to_string(blob.size()) +
                                  " bytes) exceed the static table of " + std::to_string(kStaticPlanBytes) +
                                  " bytes: use fewer members or substeps, or dc_ensemble_step_eager");
    const dc_status st = scratch_address(E->m[0]->grid->device, &table);
    if (st != DC_OK) return st;
  }
  // the ensemble stream waits for work already queued on the members' streams
  for (size_t i = 0; i < E->m.size(); ++i) {
    bool seen = false;
    for (size_t j = 0; j < i; ++j) seen |= E->m[j]->stream == E->m[i]->stream;
    if (seen) continue;
    EN_TRY(hipEventRecord(E->ready, E->m[i]->stream));
    EN_TRY(hipStreamWaitEvent(E->stream, E->ready, 0));
  }
  if (mode != StepMode::Graph) {
    if (mode == StepMode::Eager) {
      const dc_status st = upload_plan(blob, &table);
      if (st != DC_OK) return st;
    } else {
      // the host blob outlives the copy: the stream is synchronised below
      EN_TRY(hipMemcpyAsync(table, blob.data(), blob.size(), hipMemcpyHostToDevice, E->stream));
    }
    launch_recs<R>(E, recs, static_cast<const char*>(table), E->stream, prof);
    hipError_t e = hipGetLastError();
    hipError_t e2 = hipStreamSynchronize(E->stream);
    if (mode == StepMode::Eager) (void)hipFree(table);
    if (e != hipSuccess || e2 != hipSuccess)
      return efail(DC_EHIP, std::string("batched step: ") + hipGetErrorString(e != hipSuccess ? e : e2));
  } else {
    GraphEntry* ge = nullptr;
    for (GraphEntry& g : E->graphs)
      if (g.dt == dt && g.nsub == nsub && g.parity == parity) ge = &g;
    if (!ge) {
      std::vector<char> blob;
      std::vector<Rec> recs;
      plan_step<R>(E, dt, nsub, parity, blob, recs);
      GraphEntry g{dt, nsub, parity, nullptr, nullptr, nullptr};
      dc_status st = upload_plan(blob, &g.blob);
      if (st != DC_OK) return st;
      EN_TRY(hipStreamBeginCapture(E->stream, hipStreamCaptureModeThreadLocal));
      launch_recs<R>(E, recs, static_cast<const char*>(g.blob), E->stream, nullptr);
      EN_TRY(hipStreamEndCapture(E->stream, &g.graph));
      EN_TRY(hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0));
      E->graphs.push_back(g);
      ge = &E->graphs.back();
    }
    EN_TRY(hipGraphLaunch(ge->exec, E->stream));
  }
  // later work on any member's own stream is ordered after the ensemble step
  EN_TRY(hipEventRecord(E->done, E->stream));
  for (dc_state* s : E->m) {
    s->cur = (parity + nsub) & 1;
    EN_TRY(hipStreamWaitEvent(s->stream, E->done, 0));
  }
  return DC_OK;
}

dc_status ens_step(dc_ensemble* E, double dt, int nsub, StepMode mode, Prof* prof) {
  for (dc_state* s : E->m) s->part = 0;  // the members' workspaces are overwritten
  if (E->prec == DC_PREC_MIXED) return step_impl<float>(E, dt, nsub, mode, prof);
  return step_impl<double>(E, dt, nsub, mode, prof);
}

std::string tune_key(const dc_ensemble* E) {
  std::vector<int> nc;
  for (const dc_state* s : E->m) nc.push_back(s->grid->h.nc);
  std::sort(nc.begin(), nc.end());
  std::ostringstream k;
  k << "prec=" << (int)E->prec << ";K=" << E->K << ";diff=" << (int)E->m[0]->diff << ";cells=";
  for (size_t i = 0; i < nc.size(); ++i) k << (i ? "," : "") << nc[i];
  return k.str();
}

std::string schedule_text(const dc_ensemble* E) {
  std::ostringstream o;
  for (int t = 0; t < T_COUNT; ++t) o << E->tiles[t].threads << "x" << E->tiles[t].kb << " ";
  o << "|";
  for (int p = 0; p < K_COUNT; ++p) o << " " << E->gfac[p];
  return o.str();
}

bool parse_schedule(const std::string& txt, dc_ensemble* E) {
  std::istringstream in(txt);
  Tile t[T_COUNT];
  int gf[K_COUNT];
  for (int i = 0; i < T_COUNT; ++i) {
    std::string tok;
    if (!(in >> tok)) return false;
    if (std::sscanf(tok.c_str(), "%dx%d", &t[i].threads, &t[i].kb) != 2) return false;
    if (t[i].threads <= 0 || t[i].threads > 256 || t[i].threads % 64 || t[i].kb <= 0) return false;
  }
  std::string bar;
  if (!(in >> bar) || bar != "|") return false;
  for (int p = 0; p < K_COUNT; ++p)
    if (!(in >> gf[p]) || gf[p] < 0) return false;
  std::copy(t, t + T_COUNT, E->tiles);
  std::copy(gf, gf + K_COUNT, E->gfac);
  return true;
}

}  // namespace

extern "C" {

dc_status dc_ensemble_create(dc_state* const* members, int32_t n, dc_ensemble** out) {
  if (!out) return efail(DC_EINVAL, "out is NULL");
  *out = nullptr;
  if (!members || n < 1 || n > 4096) return efail(DC_EINVAL, "need 1..4096 members");
  for (int i = 0; i < n; ++i) {
    if (!members[i]) return efail(DC_EINVAL, "NULL member");
    if (members[i]->prec != members[0]->prec) return efail(DC_EINVAL, "members must share the precision");
    if (members[i]->grid->h.K != members[0]->grid->h.K) return efail(DC_EINVAL, "members must share n_lev");
    if (members[i]->diff != members[0]->diff || members[i]->diff == DC_DIFF_SURROGATE)
      return efail(DC_EINVAL, "members must share a plain or disabled diffusion mode");
    if (members[i]->cur != members[0]->cur) return efail(DC_EINVAL, "members must start in the same buffer set");
    if (members[i]->p.miura != members[0]->p.miura)
      return efail(DC_EINVAL, "members must share the Miura upwind option");
    if (members[i]->grid->device != members[0]->grid->device) return efail(DC_EINVAL, "members on different devices");
    for (int j = 0; j < i; ++j)
      if (members[j] == members[i]) return efail(DC_EINVAL, "a member appears twice");
  }
  dc_ensemble* E = new (std::nothrow) dc_ensemble();
  if (!E) return efail(DC_ENOMEM, "host allocation failed");
  E->m.assign(members, members + n);
  E->prec = members[0]->prec;
  E->K = members[0]->grid->h.K;
  // graphs cannot be captured on the legacy null stream: the ensemble owns a
  // non-blocking stream (default priority) ordered against the members' streams
  if (hipStreamCreateWithFlags(&E->stream, hipStreamNonBlocking) != hipSuccess) {
    delete E;
    return efail(DC_EHIP, "hipStreamCreate failed");
  }
  // default schedule: the largest member's default tiles, one block per tile
  const dc_state* big = members[0];
  for (int i = 1; i < n; ++i)
    if (members[i]->grid->h.nc > big->grid->h.nc) big = members[i];
  std::copy(big->tiles, big->tiles + T_COUNT, E->tiles);
  std::fill(E->gfac, E->gfac + K_COUNT, 0);
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    E->n_cu = prop.multiProcessorCount;
  if (hipEventCreateWithFlags(&E->done, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&E->ready, hipEventDisableTiming) != hipSuccess) {
    (void)hipStreamDestroy(E->stream);
    delete E;
    return efail(DC_EHIP, "hipEventCreate failed");
  }
  for (int i = 0; i < n; ++i)
    if (hipStreamSynchronize(members[i]->stream) != hipSuccess) {
      (void)hipEventDestroy(E->done);
      (void)hipEventDestroy(E->ready);
      (void)hipStreamDestroy(E->stream);
      delete E;
      return efail(DC_EHIP, "member stream synchronisation failed");
    }
  *out = E;
  return DC_OK;
}

dc_status dc_ensemble_step(dc_ensemble* E, double dt, int32_t nsub) {
  if (!E) return efail(DC_EINVAL, "ensemble is NULL");
  if (!(dt > 0.0) || !std::isfinite(dt)) return efail(DC_EINVAL, "dt must be finite and > 0");
  if (nsub < 1 || nsub > 1000) return efail(DC_EINVAL, "nsubsteps must be in [1, 1000]");
  for (const dc_state* s : E->m)
    if (s->cur != E->m[0]->cur) return efail(DC_ESTATE, "members were stepped individually (buffer sets differ)");
  return ens_step(E, dt, nsub, StepMode::Graph, nullptr);
}

dc_status dc_ensemble_step_eager(dc_ensemble* E, double dt, int32_t nsub) {
  if (!E) return efail(DC_EINVAL, "ensemble is NULL");
  if (!(dt > 0.0) || !std::isfinite(dt)) return efail(DC_EINVAL, "dt must be finite and > 0");
  if (nsub < 1 || nsub > 1000) return efail(DC_EINVAL, "nsubsteps must be in [1, 1000]");
  for (const dc_state* s : E->m)
    if (s->cur != E->m[0]->cur) return efail(DC_ESTATE, "members were stepped individually (buffer sets differ)");
  return ens_step(E, dt, nsub, StepMode::Eager, nullptr);
}

dc_status dc_ensemble_step_noalloc(dc_ensemble* E, double dt, int32_t nsub) {
  if (!E) return efail(DC_EINVAL, "ensemble is NULL");
  if (!(dt > 0.0) || !std::isfinite(dt)) return efail(DC_EINVAL, "dt must be finite and > 0");
  if (nsub < 1 || nsub > 1000) return efail(DC_EINVAL, "nsubsteps must be in [1, 1000]");
  for (const dc_state* s : E->m)
    if (s->cur != E->m[0]->cur) return efail(DC_ESTATE, "members were stepped individually (buffer sets differ)");
  return ens_step(E, dt, nsub, StepMode::Static, nullptr);
}

dc_status dc_ensemble_autotune(dc_ensemble* E, double dt, int32_t nsub, const char* cache_path) {
  if (!E) return efail(DC_EINVAL, "ensemble is NULL");
  if (!(dt > 0.0) || nsub < 1 || nsub > 1000) return efail(DC_EINVAL, "bad dt or nsubsteps");
  const std::string key = tune_key(E);
  if (cache_path && *cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      const size_t bar = line.find('\t');
      if (bar != std::string::npos && line.substr(0, bar) == key && parse_schedule(line.substr(bar + 1), E)) {
        free_graphs(E);
        return DC_OK;
      }
    }
  }
  // snapshot the members' current state: the trial steps advance it.  The
  // copies run on the null stream, which is not ordered against the
  // ensemble's non-blocking stream or the members' streams: let the work
  // queued there finish first
  if (hipStreamSynchronize(E->stream) != hipSuccess) return efail(DC_EHIP, "ensemble stream synchronisation failed");
  for (dc_state* s : E->m)
    if (hipStreamSynchronize(s->stream) != hipSuccess) return efail(DC_EHIP, "member stream synchronisation failed");
  std::vector<std::vector<void*>> saved(E->m.size());
  const int parity = E->m[0]->cur;
  auto release = [&]() {
    for (auto& v : saved)
      for (void* p : v) (void)hipFree(p);
  };
  for (size_t i = 0; i < E->m.size(); ++i) {
    dc_state* s = E->m[i];
    for (int f = 0; f < DC_FIELD_COUNT; ++f) {
      size_t bytes = 0;
      dc_field_bytes(s->grid, s->prec, f, &bytes);
      void* p = nullptr;
      if (hipMalloc(&p, bytes) != hipSuccess) {
        release();
        return efail(DC_ENOMEM, "autotune snapshot allocation failed");
      }
      saved[i].push_back(p);
      const dc_fields& cur = s->buf[parity];
      const void* src = f == 0 ? cur.vn : f == 1 ? cur.w : f == 2 ? cur.rho : f == 3 ? cur.exner : cur.theta_v;
      if (hipMemcpy(p, src, bytes, hipMemcpyDeviceToDevice) != hipSuccess) {
        release();
        return efail(DC_EHIP, "autotune snapshot copy failed");
      }
    }
  }
  struct Cand {
    int threads, kb, gfac;
  };
  // threads x the levels split into near-equal blocks (a short last level
  // block wastes most of its wave's time), each with one block per tile and
  // with a persistent grid of 8 blocks per compute unit
  std::vector<Cand> cands;
  for (int gf : {0, 8})
    for (int th : {256, 128, 64}) {
      int last = 0;
      for (int nby : {1, 2, 3, 4, 5, 6, 8, 11}) {
        const int kb = (E->K + nby - 1) / nby;
        if (kb != last) cands.push_back({th, kb, gf});
        last = kb;
      }
    }
  const Tile tile0[T_COUNT] = {E->tiles[0], E->tiles[1], E->tiles[2], E->tiles[3], E->tiles[4]};
  // per tile kind: phases that use it
  const std::vector<std::vector<int>> uses = {
      {K_VC_P, K_VC_C}, {K_EDGE_P, K_EDGE_C, K_MIURA}, {K_DVERT}, {K_DDIV, K_DCV2}, {K_DEDGE1, K_DEDGE2}};
  std::vector<double> best_t(T_COUNT, 1e300), best_col(2, 1e300);
  std::vector<Cand> best_c(T_COUNT, cands[0]);
  int best_colg[2] = {0, 0};
  dc_status st = DC_OK;
  // warm-up
  st = ens_step(E, dt, nsub, StepMode::Eager, nullptr);
  for (size_t ci = 0; ci < cands.size() && st == DC_OK; ++ci) {
    for (int t = 0; t < T_COUNT; ++t) E->tiles[t] = {cands[ci].threads, cands[ci].kb};
    std::fill(E->gfac, E->gfac + K_COUNT, cands[ci].gfac);
    double ph[K_COUNT] = {0};
    for (int rep = 0; rep < 2 && st == DC_OK; ++rep) {
      E->prof.on = true;
      E->prof.used = 0;
      st = ens_step(E, dt, nsub, StepMode::Eager, &E->prof);
      E->prof.on = false;
      double cur[K_COUNT] = {0};
      for (size_t i = 0; i + 1 < E->prof.used; ++i)
        if (E->prof.kid[i] >= 0 && E->prof.kid[i + 1] == -1) {
          float ms = 0.f;
          if (hipEventElapsedTime(&ms, E->prof.ev[i], E->prof.ev[i + 1]) == hipSuccess) cur[E->prof.kid[i]] += ms;
        }
      for (int p = 0; p < K_COUNT; ++p) ph[p] = rep == 0 ? cur[p] : std::min(ph[p], cur[p]);
    }
    for (int t = 0; t < T_COUNT; ++t) {
      double sum = 0;
      for (int p : uses[t]) sum += ph[p];
      if (sum < best_t[t]) {
        best_t[t] = sum;
        best_c[t] = cands[ci];
      }
    }
    for (int q = 0; q < 2; ++q) {
      const double v = ph[q == 0 ? K_COL_P : K_COL_C];
      // the column phases have no tile: only the persistent grid differs
      if (v < best_col[q]) {
        best_col[q] = v;
        best_colg[q] = cands[ci].gfac;
      }
    }
  }
  // restore the snapshot
  for (size_t i = 0; i < E->m.size(); ++i) {
    dc_state* s = E->m[i];
    s->cur = parity;
    const dc_fields& cur = s->buf[parity];
    for (int f = 0; f < DC_FIELD_COUNT; ++f) {
      size_t bytes = 0;
      dc_field_bytes(s->grid, s->prec, f, &bytes);
      void* dst = f == 0 ? cur.vn : f == 1 ? cur.w : f == 2 ? cur.rho : f == 3 ? cur.exner : cur.theta_v;
      if (hipMemcpy(dst, saved[i][f], bytes, hipMemcpyDeviceToDevice) != hipSuccess) st = DC_EHIP;
    }
  }
  release();
  if (st != DC_OK) {
    std::copy(tile0, tile0 + T_COUNT, E->tiles);
    std::fill(E->gfac, E->gfac + K_COUNT, 0);
    return st == DC_EHIP ? efail(DC_EHIP, "autotune trial failed") : st;
  }
  for (int t = 0; t < T_COUNT; ++t) E->tiles[t] = {best_c[t].threads, best_c[t].kb};
  std::fill(E->gfac, E->gfac + K_COUNT, 0);
  for (int t = 0; t < T_COUNT; ++t)
    for (int p : uses[t]) E->gfac[p] = best_c[t].gfac;
  E->gfac[K_COL_P] = best_colg[0];
  E->gfac[K_COL_C] = best_colg[1];
  free_graphs(E);
  if (cache_path && *cache_path) {
    std::ofstream out(cache_path, std::ios::app);
    out << key << '\t' << schedule_text(E) << '\n';
  }
  return DC_OK;
}

dc_status dc_ensemble_schedule(const dc_ensemble* E, char* buf, size_t n) {
  if (!E || !buf || n == 0) return efail(DC_EINVAL, "NULL argument");
  const std::string s = schedule_text(E);
  std::strncpy(buf, s.c_str(), n - 1);
  buf[n - 1] = 0;
  return s.size() < n ? DC_OK : efail(DC_EINVAL, "buffer too small");
}

dc_status dc_ensemble_destroy(dc_ensemble* E) {
  if (!E) return efail(DC_EINVAL, "ensemble is NULL");
  hipError_t e = hipStreamSynchronize(E->stream);
  free_graphs(E);
  (void)hipEventDestroy(E->done);
  (void)hipEventDestroy(E->ready);
  (void)hipStreamDestroy(E->stream);
  for (hipEvent_t ev : E->prof.ev) (void)hipEventDestroy(ev);
  delete E;
  if (e != hipSuccess) return efail(DC_EHIP, std::string("pending work failed: ") + hipGetErrorString(e));
  return DC_OK;
}

}  // extern "C"
