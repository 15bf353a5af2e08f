// Internal declarations of the dycore library (not part of the public ABI).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "dycore.h"

namespace dc {

constexpr int kPad = 64;  // level stride granularity (entities)

inline int pad_to(int n, int m) { return (n + m - 1) / m * m; }

// Host-side grid: renumbered inputs, canonical tables, geometry and the
// stencil coefficients in slot-major ("SoA") layout with padded strides.
struct HostGrid {
  int nc = 0, ne = 0, nv = 0, K = 0;
  int cs = 0, es = 0, vs = 0;  // padded strides
  double radius = 0.0, mean_area = 0.0;
  // canonical tables, row-major [entity][slot] (what dc_grid_table returns)
  std::vector<int32_t> e2c, c2e, e2v, c2e2c, c2v, v2e, v2c, e2c2e, e2c2v;
  std::vector<int32_t> perm_c, perm_e, perm_v;  // internal id -> original id
  std::vector<int32_t> sgn_c, sgn_v;            // [C][3], [V][6]
  // geometry in internal numbering
  std::vector<double> xv, xe, xc, nrm, tan;     // [.][3]
  std::vector<double> l, d, ac, av;
  // vertical column
  std::vector<double> z_half, ex_ref, th_ref, th_ref_ic, dex_ref_ic;
  // stencil coefficients, slot-major with padded strides
  std::vector<int32_t> t_c2e, t_c2e2c;            // [3][cs]
  std::vector<double> k_div, k_lap, k_area;       // [3][cs], [3][cs], [cs]
  std::vector<int32_t> t_e2c, t_e2v, t_e2c2e, t_e2c2v;  // [2][es], [2][es], [4][es], [4][es]
  std::vector<double> k_vt;                       // [5][es] self, e2c2e[0..3]
  std::vector<double> k_invd, k_invl, k_f, k_ae, k_invlr;  // [es]
  std::vector<double> k_nrm, k_tan;               // [3][es]
  std::vector<int32_t> t_v2e;                     // [6][vs] (pentagon slot 5 -> slot 0)
  std::vector<double> k_curl;                     // [6][vs] (0 in pentagon slot 5)
  std::vector<double> k_lsq;                      // [18][vs] row j*6+s: component j, slot s
  std::vector<double> vert;                       // vertical tables, see VertTab
  // tiles of the fused edge pass (see EdgeTiles below), tile-major so that a
  // block reads its rows contiguously: counts [ntile][4] (own, vt set,
  // staged set, vertices), staged edge ids [ntile][XM], local stencil
  // positions [ntile][4][XV], vertex ids [ntile][VM], local v2e positions
  // [ntile][6][VM], local end-vertex ids [ntile][2][256]
  int et_ok = 0, et_ntile = 0;
  std::vector<int32_t> et_n, et_x, et_vx;
  std::vector<uint16_t> et_nb, et_vl, et_ev;
  // optional schemes, built on first use by a state that asks for them
  std::vector<double> k_vt_rbf;                   // [5][es] RBF tangential-wind weights
  std::vector<double> k_miura;                    // [18][es] Miura upwind coefficients
};

// Offsets (in units of K+1 doubles) of the per-level vertical tables.
enum VertTab {
  VT_DZF = 0,    // dz_full[j]
  VT_IDZF,       // 1/dz_full[j]
  VT_IDZH,       // 1/(z_full[k-1]-z_full[k]), interior half levels
  VT_IDZC2,      // 1/(z_half[k-1]-z_half[k+1]), interior half levels
  VT_EXREF,      // pi0 full
  VT_THREF,      // theta0 full
  VT_THREFIC,    // theta0 half
  VT_DEXREFIC,   // d pi0/dz half
  VT_COUNT
};

// Fused edge pass: a tile is kTileE consecutive edges; its block stages vn of
// the tile, of the rhombus edges of the tile (R1), of their rhombus edges
// (R2) and of the edges around the tile's vertices in LDS, and forms vt and
// K_e on tile + R1 and the vorticity at the tile's vertices there.  The
// staged sets of one tile must fit the fixed capacities below; grids whose
// numbering scatters neighbours further (et_ok = 0) keep separate
// vorticity/kinetic-energy and edge passes.
// Tiles of 512 edges: against 256, the staged halo is a smaller share of a
// tile (R2B8 FP64 edge_pred 10.1 -> 9.4 ms, edge_corr 8.5 -> 7.9 ms; mixed
// unchanged overall); the FP64 buffers fill the 64 KB of LDS of a block.
struct EdgeTiles {
  static constexpr int kTileE = 512;  // edges per tile (= threads per block)
  static constexpr int XM = 1536;     // staged edges per tile
  static constexpr int XV = 1024;     // edges with vt and K_e per tile
  static constexpr int VM = 512;      // vertices per tile
};

int build_host_grid(const dc_grid_desc* desc, HostGrid* g, std::string* err);
void build_edge_tiles(HostGrid* g);
bool build_rbf_vt(HostGrid* g);
void build_miura(HostGrid* g);
void lsq_vertex_weights(const HostGrid& g, int v, double w[3][6]);

void set_error(const std::string& msg);

}  // namespace dc
