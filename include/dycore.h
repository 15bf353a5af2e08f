/*
 * dycore.h -- C ABI of the MI355X (gfx950) ICON-style non-hydrostatic
 * dynamical-core time step.
 *
 * The operation: one time step of length dt = nsub dynamic substeps of length
 * dt/nsub (each a predictor and a corrector that start with the advective
 * tendencies, update the horizontal momentum with pressure gradient and
 * advection, damp divergence in the corrector only and advance w, rho, Exner
 * and theta_v with a vertically implicit column solver), followed by one
 * diffusion step (Smagorinsky plus fourth-order background on vn, second
 * order on w).  Paper: Section 4.1 and the caption of Fig. 1 (time-step
 * structure), Section 5.1 "Experimental setup" (substep / diffusion split,
 * RnBk icosahedral grids), Section 4.3.1 (C-ABI conventions: scalars by value,
 * arrays by reference without copies, double-buffered prognostic arrays, an
 * interface independent of the implementation).
 *
 * Conventions shared by every entry point
 *  - Every call returns a dc_status.  A call that fails validation returns
 *    its error without enqueuing work or changing any state; the message is
 *    available from dc_last_error() (thread-local).
 *  - Device errors of asynchronous work surface at the next synchronising
 *    call (dc_state_read/write, dc_diag_conservation, destroy) as DC_EHIP.
 *  - Host arrays are plain C arrays, row-major.  Device field buffers are
 *    [level][entity] with the entity index fastest and each level padded to
 *    the stride reported by dc_grid_info_get (a multiple of 64 entities).
 *  - One host thread per state at a time; different states are independent.
 *  - GPU: the library uses the current HIP device at dc_grid_create.
 */
#ifndef DYCORE_H
#define DYCORE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dc_grid dc_grid;
typedef struct dc_state dc_state;
typedef struct dc_ensemble dc_ensemble;
typedef struct dc_mlp dc_mlp;

typedef enum {
  DC_OK = 0,
  DC_EINVAL = -1,      /* NULL pointer, bad size, bad enum, misaligned buffer   */
  DC_EGRID = -2,       /* inconsistent connectivity or geometry                 */
  DC_EHIP = -3,        /* a HIP runtime call or kernel failed                   */
  DC_ENOMEM = -4,      /* device or host allocation failed                      */
  DC_ENONFINITE = -5,  /* check_finite set and the state holds NaN/Inf          */
  DC_EBUSY = -6,       /* grid destroyed while states still use it              */
  DC_ESTATE = -7       /* operation not valid in the state's configuration      */
} dc_status;

typedef enum { DC_PREC_FP64 = 0, DC_PREC_MIXED = 1 } dc_precision;
/* DC_DIFF_NONE skips the diffusion step (used to measure what diffusion adds). */
typedef enum { DC_DIFF_PLAIN = 0, DC_DIFF_SURROGATE = 1, DC_DIFF_NONE = 2 } dc_diffusion;

/*
 * Grid description (all host pointers; dc_grid_create copies everything).
 * Horizontal: the RnBk triangular grid of the paper's Section 5.1.
 *   e2c   [E][2] the two cells of an edge; the normal points e2c[e][0] -> e2c[e][1]
 *   c2e   [C][3] the three edges of a cell (any order; canonicalised)
 *   e2v   [E][2] the two vertices of an edge (any order; ordered along the tangent)
 *   c2e2c [C][3] the three neighbour cells (any order; validated as a set)
 *   vert_xyz, cell_xyz, edge_xyz [.][3] unit position vectors (cell = circumcentre,
 *                                  edge = normalised vertex midpoint)
 *   edge_length l_e, dual_edge_length d_e [E] metres; cell_area [C], dual_area [V] m^2
 *   edge_normal_xyz [E][3] unit normal, tangent to the sphere at edge_xyz
 * Vertical: height-based column, level 0 at the model top.
 *   z_half [K+1] strictly decreasing; exner_ref_full, theta_ref_full [K];
 *   theta_ref_half, dexner_dz_ref_half [K+1]: the reference atmosphere
 *   (pi0, theta0 at full levels, theta0 and d pi0/dz at half levels).
 * sfc_reorder = 1 renumbers cells, edges and vertices along a space-filling
 * curve of the circumcentres for locality of the neighbour gathers: the keys
 * descend a recursive 4-way subdivision of a fixed icosahedron (poles on the
 * z axis), so runs of 4^j consecutive cells are spherical triangles; edges
 * follow their lower new cell, vertices the lowest new cell around them.  Host arrays passed to
 * dc_state_read/write always use the caller's original numbering.
 */
typedef struct {
  int32_t n_cells, n_edges, n_verts, n_lev;
  const int32_t *e2c, *c2e, *e2v, *c2e2c;
  const double *vert_xyz, *cell_xyz, *edge_xyz;
  const double *edge_length, *dual_edge_length;
  const double *cell_area, *dual_area;
  const double *edge_normal_xyz;
  const double *z_half;
  const double *exner_ref_full, *theta_ref_full;
  const double *theta_ref_half, *dexner_dz_ref_half;
  double radius;
  int32_t sfc_reorder;
} dc_grid_desc;

typedef struct {
  int32_t n_cells, n_edges, n_verts, n_lev;
  int32_t cell_stride, edge_stride, vert_stride; /* padded level strides, entities */
  int32_t fused_edge_pass; /* 1: every tile of 256 consecutive edges has its stencil
                              neighbourhood within the fused edge pass's LDS (a local
                              numbering, e.g. the generator's or the curve's); 0: the
                              vorticity/kinetic-energy pass runs separately (same results) */
} dc_grid_info;

/* Table ids for dc_grid_table (internal numbering; int32, row-major). */
enum {
  DC_TAB_E2C = 0,   /* [E][2]                                                     */
  DC_TAB_C2E,       /* [C][3] counter-clockwise; c2e[c][i] joins c2v[i], c2v[i+1] */
  DC_TAB_E2V,       /* [E][2] ordered along the tangent t = r x n                 */
  DC_TAB_C2E2C,     /* [C][3] cell across c2e[c][i]                               */
  DC_TAB_C2V,       /* [C][3] counter-clockwise seen from outside                 */
  DC_TAB_V2E,       /* [V][6] counter-clockwise from the smallest id, -1 padded   */
  DC_TAB_V2C,       /* [V][6] cell between v2e[i] and v2e[i+1], -1 padded         */
  DC_TAB_E2C2E,     /* [E][4] other edges of c0, then of c1, in c2e order         */
  DC_TAB_E2C2V,     /* [E][4] v0, v1, vertex of c0 off e, vertex of c1 off e      */
  DC_TAB_PERM_CELL, /* [C] original id of internal cell i (identity without SFC)  */
  DC_TAB_PERM_EDGE, /* [E]                                                        */
  DC_TAB_PERM_VERT, /* [V]                                                        */
  DC_TAB_COUNT
};

/*
 * Scheme parameters.  Defaults (dc_params_default) are the documented
 * readings of the paper's unstated constants.
 */
typedef struct {
  double eta;            /* implicit weight of the column solver (0.65)                 */
  double adv_w0, adv_w1; /* corrector weights of the two advective tendencies (.25/.75)  */
  double divdamp_c4;     /* 4th-order divergence damping: c4 * mean_cell_area^2 (0.0025)  */
  double rayleigh_tau0;  /* sponge rate [1/s] (0.05)                                      */
  double rayleigh_zfrac; /* sponge starts at this fraction of the model top (2/3)         */
  double smag_cs;        /* Smagorinsky constant (0.015)                                  */
  double smag_cap;       /* nu <= A_e / (smag_cap * dt) (16)                              */
  double hdiff_k4;       /* background 4th-order diffusion k4 * A_e^2 (1/128)             */
  double rd, cpd, cvd;   /* gas constant, heat capacities of dry air                      */
  double omega;          /* planetary angular velocity [1/s]                              */
  int32_t diffuse_w;     /* 1: diffuse w with the Smagorinsky viscosity                   */
  int32_t check_finite;  /* 1: dc_dycore_step checks the state and returns DC_ENONFINITE  */
  int32_t diffuse_theta; /* 1: the diffusion step also diffuses theta_v (Smagorinsky, as w,
                            at full levels with nu averaged over the cell's edges) and
                            moves exner with it, dpi/pi = (R_d/c_vd) dtheta_v/theta_v
                            (the equation of state at fixed rho); plain diffusion only */
  int32_t theta_enh_nlev;   /* with diffuse_theta: in this many lowest levels (0..n_lev; 0 off)
                               the theta_v coefficient of a cell colder than the mean of its
                               three neighbours by dT > theta_enh_thresh is raised to at least
                               s * mean_e(A_e) / (smag_cap * dt), s = min(1, dT / thresh - 1):
                               the paper's larger coefficients for strong near-surface
                               temperature contrasts (Section 4.1)                        */
  double theta_enh_thresh;  /* that threshold [K] (> 0; 5)                                     */
  /* Fuller ICON numerics (Section 4.1: the dynamical core keeps ICON's
   * discretisation); both off by default. */
  int32_t miura;   /* 1: rho and theta_v at the edges (mass and theta fluxes of both passes,
                      theta_v of the pressure-gradient term) by second-order upwind (Miura)
                      reconstruction: the value at the departure point of the edge midpoint
                      over the substep, x* = x_e - dtau (vn n + vt t), extrapolated linearly
                      from the upwind cell (c0 when vn >= 0) with its least-squares gradient
                      over the three neighbour cells; 0: means of the two cells.  Needs the
                      larger workspace of dc_state_workspace_bytes_params.               */
  int32_t vt_rbf;  /* 1: tangential wind by vector radial-basis-function reconstruction over
                      the edge and its four e2c2e neighbours (inverse multiquadric of scale
                      0.5 l_e, plus a constant vector tangent at the edge, so uniform tangent
                      flow is exact); 0: Perot's cell-based reconstruction.               */
} dc_params;

/* Device pointers of the five prognostic fields, [level][entity] padded.
 * FP64 mode: all double.  Mixed mode: vn float, the others double.
 * vn [K][edge_stride], w [K+1][cell_stride], rho/exner/theta_v [K][cell_stride].
 * Every pointer must be 256-byte aligned.  The padding entries of each level
 * (entities n .. stride-1) belong to the library: a step may write them and
 * no result depends on them. */
typedef struct { void *vn, *w, *rho, *exner, *theta_v; } dc_fields;

enum { DC_FIELD_VN = 0, DC_FIELD_W, DC_FIELD_RHO, DC_FIELD_EXNER, DC_FIELD_THETA_V, DC_FIELD_COUNT };

typedef struct {
  double mass;        /* sum_c A_c sum_j rho dz_j                 [kg]  */
  double theta_mass;  /* sum_c A_c sum_j rho theta_v dz_j         [kg K] */
  double max_abs_w, max_abs_vn;
  int64_t n_nonfinite; /* NaN/Inf entries over the five fields           */
  double fallback_fraction; /* surrogate mode: share of edge columns that ran
                               the plain diffusion in the last non-judge step */
} dc_diag;

/* Validate the description, derive canonical tables, orientation and
 * stencil coefficients on the host, upload them to the current device.
 * DC_EGRID when: an index is out of range; e2c/c2e/e2v/c2e2c disagree; an
 * edge is not in exactly two cells; V - E + C != 2; a length or area <= 0;
 * n_e . (x_c1 - x_c0) <= 0; a vertex has more than 6 edges.  Memory owned by
 * the grid is released by dc_grid_destroy.  DC_EINVAL for counts <= 0 or
 * n_lev outside [1, 129] (the column solver's limit). */
dc_status dc_grid_create(const dc_grid_desc *desc, dc_grid **out);
dc_status dc_grid_info_get(const dc_grid *grid, dc_grid_info *info);
/* Copy a derived table (see DC_TAB_*) to host_out, which holds n int32. */
dc_status dc_grid_table(const dc_grid *grid, int32_t table_id, int32_t *host_out, size_t n);
/* DC_EBUSY while states created on the grid are alive. */
dc_status dc_grid_destroy(dc_grid *grid);

dc_status dc_params_default(dc_params *p);

/* Bytes of one device field buffer (padded) in the given precision. */
dc_status dc_field_bytes(const dc_grid *grid, dc_precision prec, int32_t field, size_t *bytes);
/* Bytes of the caller-provided device workspace a state needs with the
 * default parameters; dc_state_workspace_bytes_params for given parameters
 * (the Miura option adds two edge fields in FP64). */
dc_status dc_state_workspace_bytes(const dc_grid *grid, dc_precision prec, dc_diffusion diff, size_t *bytes);
dc_status dc_state_workspace_bytes_params(const dc_grid *grid, const dc_params *params, dc_precision prec,
                                          dc_diffusion diff, size_t *bytes);

/* Create a state over caller-owned device buffers (borrowed, never freed
 * by the library; keep them alive until dc_state_destroy).  bufA holds the
 * initial state; each substep writes the other buffer set and flips.
 * stream: a hipStream_t (NULL = the null stream); all work is enqueued
 * there asynchronously.  The workspace belongs to the state until
 * dc_state_destroy: besides the step's scratch fields it holds per-state
 * tables written here (Coriolis parameter, sponge profile), so the caller
 * must not write it. */
dc_status dc_state_create(const dc_grid *grid, const dc_params *params, dc_precision prec,
                          dc_diffusion diff, dc_fields bufA, dc_fields bufB, void *workspace,
                          size_t workspace_bytes, void *stream, dc_state **out);
/* 0: bufA holds the latest state, 1: bufB. */
dc_status dc_state_current(const dc_state *st, int32_t *which);
/* Synchronising host copies of one field in FP64, unpadded [level][entity],
 * original numbering; n must equal the field's element count. */
dc_status dc_state_read(dc_state *st, int32_t field, double *host, size_t n);
dc_status dc_state_write(dc_state *st, int32_t field, const double *host, size_t n);
/* One time step: nsubsteps predictor-corrector substeps of dt/nsubsteps,
 * then diffusion with dt.  Asynchronous on the state's stream.
 * DC_EINVAL: dt <= 0 or not finite, nsubsteps < 1. */
dc_status dc_dycore_step(dc_state *st, double dt, int32_t nsubsteps);
/* The step in parts, for verification of the segments that lie between
 * halo exchanges one at a time against a reference given the same input
 * fields (paper, Section 4.4, first level of the verification hierarchy).
 * dc_dycore_part runs one part with the coefficients of a step (dt,
 * nsubsteps), asynchronously on the state's stream:
 *   DC_PART_PREDICTOR  the predictor of one substep of dt/nsubsteps from
 *                      the current buffer set (advective tendencies at the
 *                      substep start, the momentum update to vn*, the
 *                      vertically implicit solve for w*).  Writes workspace
 *                      fields only; the buffer set and its contents are
 *                      unchanged.
 *   DC_PART_CORRECTOR  the corrector of that substep: reads the current
 *                      buffer set and what the last DC_PART_PREDICTOR left
 *                      in the workspace, writes the other buffer set and
 *                      makes it current.  PREDICTOR then CORRECTOR equals
 *                      one substep bit for bit.
 *   DC_PART_DIFFUSION  the plain diffusion of one step of dt on the current
 *                      buffer set, in place (w, and theta_v with the theta_v
 *                      diffusion option, are first copied to the staging
 *                      fields that the last substep of a step fills).
 * DC_EINVAL: bad part, dt <= 0 or not finite, nsubsteps outside [1, 1000].
 * DC_ESTATE: DC_PART_DIFFUSION on a state created without the plain
 * diffusion, DC_PART_CORRECTOR before any DC_PART_PREDICTOR (or after a
 * step or another corrector). */
enum { DC_PART_PREDICTOR = 0, DC_PART_CORRECTOR = 1, DC_PART_DIFFUSION = 2 };
dc_status dc_dycore_part(dc_state *st, int32_t part, double dt, int32_t nsubsteps);
/* Synchronising host copy, in FP64 (unpadded [level][entity], original
 * numbering, like dc_state_read), of a workspace field that the last
 * DC_PART_PREDICTOR wrote:
 *   DC_WORK_VN_PRED  vn* = vn + dtau (T_vn - cpd theta_e grad pi')   [K][E]
 *   DC_WORK_Y        vn + dtau (a0 T_vn - cpd theta_e grad pi'), the
 *                    part of the corrector's vn that the predictor forms [K][E]
 *   DC_WORK_W_PRED   w* from the implicit solve                      [K+1][C]
 *   DC_WORK_T_W      T_w at the substep start on the half levels
 *                    1..K-1 (rows 0 and K are returned as 0)         [K+1][C]
 *   DC_WORK_DIV      div vn* (input of the corrector's damping)      [K][C]
 * Mixed precision: vn*, Y, T_w and div vn* are stored in FP32.  n must equal
 * the element count.  DC_ESTATE if no DC_PART_PREDICTOR ran since the
 * state was created or its workspace was last overwritten (by a step, a
 * diffusion part, tuning, an ensemble step or a surrogate collection). */
enum { DC_WORK_VN_PRED = 0, DC_WORK_Y, DC_WORK_W_PRED, DC_WORK_T_W, DC_WORK_DIV, DC_WORK_COUNT };
dc_status dc_state_read_work(dc_state *st, int32_t which, double *host, size_t n);
/* Synchronising conservation diagnostics of the current buffer (fixed
 * reduction order: reproducible run to run). */
dc_status dc_diag_conservation(dc_state *st, dc_diag *out);
dc_status dc_state_destroy(dc_state *st);

/* Per-kernel timing with HIP events recorded on the state's stream around
 * every launch of dc_dycore_step (paper, Section 4.3.3: the profile of one
 * substep, launch versus execution).  enable != 0 clears and starts the
 * record, 0 stops it.  dc_state_profile_read synchronises and fills one
 * entry per kernel kind (cap >= 12), in kernel-id order: name, launches,
 * summed duration.  dc_state_profile_select limits later records to the
 * kernels whose bit (1u << kernel id) is set in kernel_mask (0 or all ones:
 * every kernel), so that one kernel can be timed inside a run with little
 * disturbance of the others. */
typedef struct {
  char name[32];
  int64_t calls;
  double total_ms;
} dc_kernel_stat;
dc_status dc_state_profile(dc_state *st, int32_t enable);
dc_status dc_state_profile_read(dc_state *st, dc_kernel_stat *out, int32_t cap, int32_t *n_out);
dc_status dc_state_profile_select(dc_state *st, uint32_t kernel_mask);

/* Launch tiles.  The stencil kernels run 2-D grids of tiles: a block of
 * `threads` consecutive entities times `levels` consecutive levels.  Five
 * families share a tile each: 0 vorticity and kinetic energy, 1 edge
 * momentum update, 2 diffusion vertex pass, 3 diffusion cell passes,
 * 4 diffusion edge passes.  No result depends on the tiles.
 * dc_state_autotune times candidate tiles (64, 128 or 256 threads; the
 * levels split into 1 to 11 near-equal blocks) with trial steps of
 * (dt, nsubsteps) on the state's own fields, keeps the fastest per family,
 * and restores the fields and the buffer parity: later steps give the same
 * bits as without tuning.  It synchronises, allocates a copy of the five
 * fields for the duration of the call, and takes about 50 trial steps.
 * dc_state_tiles writes threads and levels of family t to out[2t], out[2t+1]
 * (n >= 10). */
dc_status dc_state_autotune(dc_state *st, double dt, int32_t nsubsteps);
dc_status dc_state_tiles(const dc_state *st, int32_t *out, int32_t n);

/* Batched ensemble (paper, Section 4.3.3: launch overhead must not show).
 * Members on any grids, sharing precision, n_lev and diffusion mode, and
 * starting in the same buffer set, advance together: every phase of the
 * step is one persistent kernel whose blocks walk a (member, tile) work
 * table, and the whole step is captured into a hipGraph (cached per dt,
 * nsubsteps and buffer set) that dc_ensemble_step replays with one
 * hipGraphLaunch on a stream the ensemble owns; events order it after work
 * already queued on the members' streams and later member work after it.  Members keep their own buffers and stay
 * valid single states; stepping a member alone in between makes
 * dc_ensemble_step return DC_ESTATE until the buffer sets agree again.
 * Each member's result is bit-identical to stepping it alone.
 * Destroy the ensemble before its members. */
dc_status dc_ensemble_create(dc_state *const *members, int32_t n_members, dc_ensemble **out);
dc_status dc_ensemble_step(dc_ensemble *ens, double dt, int32_t nsubsteps);
/* The same step launched eagerly (no graph), synchronising. */
dc_status dc_ensemble_step_eager(dc_ensemble *ens, double dt, int32_t nsubsteps);
/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): dc_ensemble_step_eager without its
 * per-call allocation.  The step's work tables (one (member, tile) table per
 * phase) are copied into a static device array of DC_STATIC_PLAN_BYTES
 * that each GPU the library runs on holds until the process ends, instead
 * of into memory allocated for the call; nothing is allocated or freed on
 * the device.  Same kernels, same results as dc_ensemble_step_eager, bit for
 * bit.  Synchronising.  DC_EINVAL, with nothing enqueued, when the tables
 * exceed the array (about 9 KB per phase for 24 members; a step has
 * 6 nsubsteps + 5 phases).  Every call on one GPU shares that GPU's array
 * and overwrites it: calls that overlap on one GPU (other host threads, or
 * ensembles on streams not ordered against each other) race. */
#define DC_STATIC_PLAN_BYTES (2u << 20)
dc_status dc_ensemble_step_noalloc(dc_ensemble *ens, double dt, int32_t nsubsteps);
/* Pick the tile/grid schedule of every phase by timing candidates on the
 * ensemble itself (members' states are restored afterwards).  cache_path
 * (may be NULL): a text file of "key<TAB>schedule" lines; a matching key is
 * reused without timing, a new result is appended. */
dc_status dc_ensemble_autotune(dc_ensemble *ens, double dt, int32_t nsubsteps, const char *cache_path);
/* Text form of the current schedule ("threads x levels" per tile kind, then
 * blocks per CU of every phase, 0 = one block per tile). */
dc_status dc_ensemble_schedule(const dc_ensemble *ens, char *buf, size_t n);
dc_status dc_ensemble_destroy(dc_ensemble *ens);

/*
 * Learned diffusion surrogate (DC_DIFF_SURROGATE).  The paper motivates a
 * dynamical core that couples to machine-learning workflows (Sections 3
 * and 6); the network is this library's reading: per (edge, level) an
 * 18 -> 64 -> 64 -> 1 perceptron with exact (erf) GELU, BF16 operands on the
 * matrix cores and FP32 accumulation, predicting T = (vn after the vn
 * diffusion - vn before) / dt from 18 stencil features.  Stencil values
 * enter as centred pairs (mean of the two points, difference over their
 * distance, formed before the BF16 rounding), in this order:
 *   0 vn_e, 1 vt_e; 2, 3 D = div vn at e2c[0..1]; 4, 5 Z = curl vn at the
 *   end vertices e2c2v[0..1]; 6, 7 div L1 at the two cells; 8, 9 curl L1 at
 *   the two end vertices (L1 = grad D - gradt Z); 10..13 the rhombus
 *   derivatives dvn/dt, dvt/dt, dvn/dn, dvt/dn of the least-squares vertex
 *   vectors (the Smagorinsky deformation); 14, 15 Z at the opposite rhombus
 *   vertices e2c2v[2..3] (difference over the rhombus diagonal);
 *   16 l_e / mean(l), 17 d_e / mean(d).
 * Features 0..15 are odd in vn; the plain tendency is nu L1 - k4 A_e^2 L2 / dt
 * with L1 = f3 - f5, L2 = f7 - f9 and nu a function of f10..f13 and A_e.
 * Parameters (DC_MLP_NPARAMS floats, row-major): W1 [18][64], b1 [64],
 * W2 [64][64], b2 [64], w3 [64], b3 [1]; y = W3 gelu(W2 gelu(W1 x' + b1) + b2)
 * + b3 with x' = (x - mean) / std, and T = y * target_std.
 * Surrogate step: the plain diffusion's front runs every step (viscosity,
 * L1, div L1 and curl L1, which the features use, and the w diffusion); the
 * network then stands in for the vn update (the second Laplacian term and
 * the update itself).  Every judge_every-th step (the first included) runs
 * the plain vn update and flags every edge column whose residual
 * dt |T_mlp - T_plain|_2 / max(|vn|_2, sqrt(K) m/s) exceeds the threshold
 * (flags hold until the next judge step).  The other steps add dt T_mlp to
 * vn except on flagged columns and on columns with a feature outside the
 * normalisation range, which take the plain vn update.  An MLP must
 * outlive the states it is set on.
 */
#define DC_MLP_NFEATURES 18
#define DC_MLP_NPARAMS 5441

typedef struct {
  int32_t batch;   /* samples per Adam step, a multiple of 128 (4096)      */
  int32_t epochs;  /* passes over the set (2)                              */
  double lr0, lr1; /* cosine decay from lr0 to lr1 over all steps (1e-3, 1e-5) */
  uint64_t seed;   /* epoch shuffles                                       */
  int32_t shuffle; /* 1: permute the set every epoch                       */
  int32_t augment; /* 1: flip the sign of the 16 flow features and the
                      target of a hashed half of the samples (the diffusion
                      is odd in vn)                                        */
} dc_train_cfg;

typedef struct {
  int64_t steps, judge_steps; /* surrogate steps since dc_state_set_mlp, judge steps among them */
  int64_t judge_flagged;      /* columns flagged by the last judge step                        */
  int64_t range_flagged;      /* columns with out-of-range features in the last non-judge step  */
  int64_t fallback;           /* columns that ran the plain diffusion in that step              */
  int64_t fallback_total;     /* the same summed over the non-judge steps since dc_state_set_mlp */
  int64_t n_columns;          /* edge columns of the grid                                        */
} dc_surrogate_info;

/* Seeded Kaiming-uniform weights (fan-in, gain sqrt 2), zero biases, identity
 * normalisation with an unbounded range, on the current device. */
dc_status dc_mlp_create(uint64_t seed, dc_mlp **out);
dc_status dc_mlp_destroy(dc_mlp *mlp);
/* Host copies of the parameters (n must be DC_MLP_NPARAMS); set resets Adam. */
dc_status dc_mlp_get_params(dc_mlp *mlp, float *host, int64_t n);
dc_status dc_mlp_set_params(dc_mlp *mlp, const float *host, int64_t n);
/* Normalisation: per-feature mean, std (> 0), range [min, max] and the
 * target scale.  get fills 73 floats: mean[18], std[18], min[18], max[18], tstd. */
dc_status dc_mlp_set_norm(dc_mlp *mlp, const float *mean, const float *std_, const float *fmin,
                          const float *fmax, float target_std);
dc_status dc_mlp_get_norm(const dc_mlp *mlp, float *host, int64_t n);
/* Training sets live in device memory, row-major [19][stride] float:
 * rows 0..17 the features, row 18 the target T, samples 0..n-1 used.
 * fit_norm sets the normalisation from the set (synchronising): the 16 flow
 * features and the target get mean 0 and their root mean square as scale
 * with the symmetric range [-max|x|, max|x|] (the set under sign
 * augmentation); the two length ratios get mean, standard deviation and
 * [min, max].  DC_ENONFINITE if the set holds NaN/Inf. */
dc_status dc_mlp_fit_norm(dc_mlp *mlp, const float *dev_buf, int64_t stride, int64_t n);
/* MSE in normalised units, Adam (0.9, 0.999, 1e-8), synchronising; the
 * per-step mean batch loss is kept for dc_mlp_loss_trace.  The set's
 * floor(n / batch) * batch first positions of every epoch order are used. */
dc_status dc_mlp_train(dc_mlp *mlp, const float *dev_buf, int64_t stride, int64_t n, const dc_train_cfg *cfg);
dc_status dc_mlp_loss_trace(const dc_mlp *mlp, float *host, int64_t cap, int64_t *n_out);
/* Synchronising host-to-host evaluation: host_x [n][18] raw features ->
 * host_y [n] = T.  (Testing and offline evaluation.) */
dc_status dc_mlp_forward(dc_mlp *mlp, const float *host_x, int64_t n, float *host_y);
/* Gradient of mean((y - t / target_std)^2) over n rows (n a multiple of
 * 128, no augmentation) with respect to every parameter; loss may be NULL. */
dc_status dc_mlp_grad(dc_mlp *mlp, const float *host_x, const float *host_t, int64_t n, float *host_grad,
                      float *loss);
/* Attach an MLP to a DC_DIFF_SURROGATE state (restarts the judge cycle).
 * DC_ESTATE for other modes; dc_dycore_step on a surrogate state without an
 * MLP returns DC_ESTATE. */
dc_status dc_state_set_mlp(dc_state *st, const dc_mlp *mlp, double resid_threshold, int32_t judge_every);
dc_status dc_surrogate_stats(dc_state *st, dc_surrogate_info *out);
/* One plain step of a DC_DIFF_SURROGATE state (nsubsteps >= 0; 0 = the
 * diffusion alone) that records n_samples training pairs: features of the
 * state before the diffusion and T, at (edge, level) points drawn without
 * replacement by a seeded Feistel permutation, into columns
 * offset .. offset + n_samples - 1 of dev_buf ([19][stride], see above).
 * host_index (may be NULL) receives k * n_edges + e of every sample in the
 * caller's numbering (synchronising). */
dc_status dc_surrogate_collect(dc_state *st, double dt, int32_t nsubsteps, uint64_t seed, int64_t n_samples,
                               float *dev_buf, int64_t stride, int64_t offset, int64_t *host_index);

/* Thread-local message of the last failing call ("" if none). */
const char *dc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DYCORE_H */
