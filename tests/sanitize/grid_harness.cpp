// Host grid layer under AddressSanitizer and UndefinedBehaviorSanitizer: a
// CPU-only driver of dc::build_host_grid (validation, canonical tables,
// space-filling curve, stencil coefficients, fused-edge tiles) and of the
// optional schemes' tables (RBF weights, Miura coefficients).  It reads one
// grid description per file, builds it and prints the status; any invalid
// memory access or undefined operation aborts with the sanitizer's report.
//
// usage: grid_harness FILE...
// FILE, little-endian: int32 C, E, V, K, sfc; double radius; int32 e2c [E][2],
// c2e [C][3], e2v [E][2], c2e2c [C][3]; double vert_xyz [V][3],
// cell_xyz [C][3], edge_xyz [E][3], edge_length [E], dual_edge_length [E],
// cell_area [C], dual_area [V], edge_normal_xyz [E][3], z_half [K+1],
// exner_ref_full [K], theta_ref_full [K], theta_ref_half [K+1],
// dexner_dz_ref_half [K+1].  Arrays are allocated at exactly their size.
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "internal.h"

namespace dc {
void set_error(const std::string&) {}
}

template <typename T>
static bool rd(FILE* f, std::vector<T>& v, size_t n) {
  v.resize(n);
  return n == 0 || std::fread(v.data(), sizeof(T), n, f) == n;
}

int main(int argc, char** argv) {
  for (int a = 1; a < argc; ++a) {
    FILE* f = std::fopen(argv[a], "rb");
    if (!f) return 2;
    int32_t h[5];
    double radius = 0;
    if (std::fread(h, 4, 5, f) != 5 || std::fread(&radius, 8, 1, f) != 1) return 2;
    const size_t C = h[0], E = h[1], V = h[2], K = h[3];
    std::vector<int32_t> e2c, c2e, e2v, c2e2c;
    std::vector<double> vx, cx, ex, l, d, ac, av, nrm, zh, exf, thf, thh, dexh;
    bool ok = rd(f, e2c, 2 * E) && rd(f, c2e, 3 * C) && rd(f, e2v, 2 * E) && rd(f, c2e2c, 3 * C) &&
              rd(f, vx, 3 * V) && rd(f, cx, 3 * C) && rd(f, ex, 3 * E) && rd(f, l, E) && rd(f, d, E) &&
              rd(f, ac, C) && rd(f, av, V) && rd(f, nrm, 3 * E) && rd(f, zh, K + 1) && rd(f, exf, K) &&
              rd(f, thf, K) && rd(f, thh, K + 1) && rd(f, dexh, K + 1);
    std::fclose(f);
    if (!ok) return 2;
    dc_grid_desc g{};
    g.n_cells = h[0];
    g.n_edges = h[1];
    g.n_verts = h[2];
    g.n_lev = h[3];
    g.e2c = e2c.data();
    g.c2e = c2e.data();
    g.e2v = e2v.data();
    g.c2e2c = c2e2c.data();
    g.vert_xyz = vx.data();
    g.cell_xyz = cx.data();
    g.edge_xyz = ex.data();
    g.edge_length = l.data();
    g.dual_edge_length = d.data();
    g.cell_area = ac.data();
    g.dual_area = av.data();
    g.edge_normal_xyz = nrm.data();
    g.z_half = zh.data();
    g.exner_ref_full = exf.data();
    g.theta_ref_full = thf.data();
    g.theta_ref_half = thh.data();
    g.dexner_dz_ref_half = dexh.data();
    g.radius = radius;
    g.sfc_reorder = h[4];
    dc::HostGrid hg;
    std::string err;
    const int rc = dc::build_host_grid(&g, &hg, &err);
    int rbf = -1, tiles = -1;
    if (rc == DC_OK) {
      rbf = dc::build_rbf_vt(&hg) ? 1 : 0;
      dc::build_miura(&hg);
      tiles = hg.et_ok;
    }
    std::printf("%s %d %d %d\n", argv[a], rc, rbf, tiles);
  }
  return 0;
}
