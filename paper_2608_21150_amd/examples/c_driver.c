/* A host time loop in plain C over the library's C ABI: no Python, no
 * PyTorch.  It plays the role of the host model that calls the dynamical
 * core through its C interface (the paper's Section 4.3.1: scalars by
 * value, arrays by reference, double buffers flipped by the library): it
 * builds the grid, allocates the field buffers and the workspace on the
 * device itself, writes an initial state, runs the steps and reads the
 * state back.
 *
 * usage: c_driver IN OUT
 *
 * IN, little-endian binary:
 *   int32  n_cells C, n_edges E, n_verts V, n_lev K, precision (0 FP64,
 *          1 mixed), sfc_reorder, nsub, steps
 *   double radius, dt
 *   int32  e2c [E][2], c2e [C][3], e2v [E][2], c2e2c [C][3]
 *   double vert_xyz [V][3], cell_xyz [C][3], edge_xyz [E][3],
 *          edge_length [E], dual_edge_length [E], cell_area [C],
 *          dual_area [V], edge_normal_xyz [E][3],
 *          z_half [K+1], exner_ref_full [K], theta_ref_full [K],
 *          theta_ref_half [K+1], dexner_dz_ref_half [K+1],
 *          vn [K][E], w [K+1][C], rho [K][C], exner [K][C], theta_v [K][C]
 * OUT: the five fields after the steps, in the same order and layout, then
 *      the conservation diagnostics (mass, theta mass, max |w|, max |vn|,
 *      non-finite count as a double).
 * Exit status 0 on success, 1 on a library or I/O error (the message is
 * printed), 2 on bad usage.
 */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "dycore.h"

static int fail_io(const char* what) {
  fprintf(stderr, "c_driver: %s\n", what);
  return 1;
}

#define DC_CHECK(call)                                                                  \
  do {                                                                                  \
    dc_status st_ = (call);                                                             \
    if (st_ != DC_OK) {                                                                 \
      fprintf(stderr, "c_driver: %s failed (%d): %s\n", #call, (int)st_, dc_last_error()); \
      return 1;                                                                         \
    }                                                                                   \
  } while (0)

static void* read_block(FILE* f, size_t bytes) {
  void* p = malloc(bytes ? bytes : 1);
  if (p && bytes && fread(p, 1, bytes, f) != bytes) {
    free(p);
    return NULL;
  }
  return p;
}

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: c_driver IN OUT\n");
    return 2;
  }
  FILE* f = fopen(argv[1], "rb");
  if (!f) return fail_io("cannot open the input file");
  int32_t hdr[8];
  double hdr2[2];
  if (fread(hdr, sizeof(int32_t), 8, f) != 8 || fread(hdr2, sizeof(double), 2, f) != 2)
    return fail_io("short header");
  const int32_t C = hdr[0], E = hdr[1], V = hdr[2], K = hdr[3];
  const dc_precision prec = hdr[4] ? DC_PREC_MIXED : DC_PREC_FP64;
  const int32_t nsub = hdr[6], steps = hdr[7];
  const double dt = hdr2[1];
  if (C <= 0 || E <= 0 || V <= 0 || K <= 0 || steps < 0) return fail_io("bad counts");

  dc_grid_desc d;
  memset(&d, 0, sizeof(d));
  d.n_cells = C;
  d.n_edges = E;
  d.n_verts = V;
  d.n_lev = K;
  d.radius = hdr2[0];
  d.sfc_reorder = hdr[5];
  const size_t i4 = sizeof(int32_t), f8 = sizeof(double);
  int32_t* e2c = read_block(f, 2 * (size_t)E * i4);
  int32_t* c2e = read_block(f, 3 * (size_t)C * i4);
  int32_t* e2v = read_block(f, 2 * (size_t)E * i4);
  int32_t* c2e2c = read_block(f, 3 * (size_t)C * i4);
  double* vxyz = read_block(f, 3 * (size_t)V * f8);
  double* cxyz = read_block(f, 3 * (size_t)C * f8);
  double* exyz = read_block(f, 3 * (size_t)E * f8);
  double* el = read_block(f, (size_t)E * f8);
  double* del = read_block(f, (size_t)E * f8);
  double* ca = read_block(f, (size_t)C * f8);
  double* da = read_block(f, (size_t)V * f8);
  double* en = read_block(f, 3 * (size_t)E * f8);
  double* zh = read_block(f, (size_t)(K + 1) * f8);
  double* exf = read_block(f, (size_t)K * f8);
  double* thf = read_block(f, (size_t)K * f8);
  double* thh = read_block(f, (size_t)(K + 1) * f8);
  double* dexh = read_block(f, (size_t)(K + 1) * f8);
  const size_t n_field[5] = {(size_t)K * E, (size_t)(K + 1) * C, (size_t)K * C, (size_t)K * C, (size_t)K * C};
  double* field[5];
  for (int i = 0; i < 5; ++i) field[i] = read_block(f, n_field[i] * f8);
  fclose(f);
  if (!e2c || !c2e || !e2v || !c2e2c || !vxyz || !cxyz || !exyz || !el || !del || !ca || !da || !en || !zh ||
      !exf || !thf || !thh || !dexh || !field[0] || !field[1] || !field[2] || !field[3] || !field[4])
    return fail_io("short input");
  d.e2c = e2c;
  d.c2e = c2e;
  d.e2v = e2v;
  d.c2e2c = c2e2c;
  d.vert_xyz = vxyz;
  d.cell_xyz = cxyz;
  d.edge_xyz = exyz;
  d.edge_length = el;
  d.dual_edge_length = del;
  d.cell_area = ca;
  d.dual_area = da;
  d.edge_normal_xyz = en;
  d.z_half = zh;
  d.exner_ref_full = exf;
  d.theta_ref_full = thf;
  d.theta_ref_half = thh;
  d.dexner_dz_ref_half = dexh;

  dc_grid* grid = NULL;
  DC_CHECK(dc_grid_create(&d, &grid));
  dc_params params;
  DC_CHECK(dc_params_default(&params));

  /* device buffers: two sets of the five fields and the workspace */
  void* bufs[2][5];
  for (int b = 0; b < 2; ++b)
    for (int i = 0; i < 5; ++i) {
      size_t bytes = 0;
      DC_CHECK(dc_field_bytes(grid, prec, i, &bytes));
      if (hipMalloc(&bufs[b][i], bytes) != hipSuccess) return fail_io("hipMalloc of a field failed");
    }
  size_t ws_bytes = 0;
  DC_CHECK(dc_state_workspace_bytes(grid, prec, DC_DIFF_PLAIN, &ws_bytes));
  void* ws = NULL;
  if (hipMalloc(&ws, ws_bytes) != hipSuccess) return fail_io("hipMalloc of the workspace failed");
  hipStream_t stream;
  if (hipStreamCreate(&stream) != hipSuccess) return fail_io("hipStreamCreate failed");
  dc_fields fa = {bufs[0][0], bufs[0][1], bufs[0][2], bufs[0][3], bufs[0][4]};
  dc_fields fb = {bufs[1][0], bufs[1][1], bufs[1][2], bufs[1][3], bufs[1][4]};
  dc_state* st = NULL;
  DC_CHECK(dc_state_create(grid, &params, prec, DC_DIFF_PLAIN, fa, fb, ws, ws_bytes, (void*)stream, &st));
  for (int i = 0; i < 5; ++i) DC_CHECK(dc_state_write(st, i, field[i], n_field[i]));

  for (int s = 0; s < steps; ++s) DC_CHECK(dc_dycore_step(st, dt, nsub));
  dc_diag diag;
  DC_CHECK(dc_diag_conservation(st, &diag));
  for (int i = 0; i < 5; ++i) DC_CHECK(dc_state_read(st, i, field[i], n_field[i]));

  FILE* o = fopen(argv[2], "wb");
  if (!o) return fail_io("cannot open the output file");
  for (int i = 0; i < 5; ++i)
    if (fwrite(field[i], f8, n_field[i], o) != n_field[i]) return fail_io("short write");
  const double dg[5] = {diag.mass, diag.theta_mass, diag.max_abs_w, diag.max_abs_vn, (double)diag.n_nonfinite};
  if (fwrite(dg, f8, 5, o) != 5) return fail_io("short write");
  fclose(o);

  DC_CHECK(dc_state_destroy(st));
  DC_CHECK(dc_grid_destroy(grid));
  for (int b = 0; b < 2; ++b)
    for (int i = 0; i < 5; ++i) hipFree(bufs[b][i]);
  hipFree(ws);
  hipStreamDestroy(stream);
  printf("c_driver: %d steps of dt %g s (%d substeps), %d cells x %d levels, %s: mass %.17g, non-finite %lld\n",
         steps, dt, nsub, C, K, prec == DC_PREC_MIXED ? "mixed" : "fp64", diag.mass, (long long)diag.n_nonfinite);
  return 0;
}
