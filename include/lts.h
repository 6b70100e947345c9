/*
 * liblts — LTS3 local time stepping for the TRiSK shallow water equations on
 * Voronoi C-grid meshes, on AMD Instinct MI355X (gfx950).
 *
 * Method: Capodaglio & Petersen, "Local time stepping for the shallow water
 * equations in MPAS" (arXiv 2106.07154): Algorithm 2.2 (LTS3, with LTS2 as its
 * second-order branch) over the discrete system of eq:sweTimeStepping, whose
 * right-hand side is the TRiSK discretisation of Appendix B.
 *
 * Conventions
 *   - Every call returns lts_status (0 = LTS_OK, < 0 = error); the message of
 *     the last error is available from lts_last_error().  A context is not
 *     thread-safe: calls on one context must not overlap.
 *   - Host arrays passed in are owned by the caller and copied during the call.
 *     Device buffers are owned by the context and freed by lts_destroy().
 *   - Indices are 0-based int32 in the caller's numbering; unused slots of
 *     per-cell tables hold -1.  Layout is row-major: edges_on_cell[i*max_edges+j],
 *     cells_on_edge[2*e+s], edges_on_vertex[3*v+k].
 *   - Orientation: n_e points from cells_on_edge[e][0] to cells_on_edge[e][1]
 *     (n_{e,c0} = +1, n_{e,c1} = -1, the sign correction of Appendix B);
 *     t_e = k x n_e points from vertices_on_edge[e][0] to vertices_on_edge[e][1]
 *     (t_{e,v1} = +1).  edges_on_cell lists a cell's edges counter-clockwise;
 *     vertices_on_cell[i][j] is the vertex shared by edges_on_cell[i][j] and
 *     edges_on_cell[i][j+1]; cells_on_cell[i][j] is the cell across
 *     edges_on_cell[i][j].  Any flip of n_e (with u_e negated) is equivalent.
 *   - State: thickness h at cells, normal velocity u at edges, always passed as
 *     double on the host; on the device the context keeps it in its precision
 *     (LTS_FP64 or LTS_FP32), permuted so every LTS region is a contiguous range.
 *   - All work is enqueued on the context's HIP stream.  Calls that return host
 *     data (lts_diagnostics, lts_get_state, lts_get_regions, lts_eval_rhs)
 *     synchronise that stream; lts_step and lts_step_rk3 do not.
 */
#ifndef LTS_H
#define LTS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LTS_OK = 0,
    LTS_EINVAL = -1,     /* bad argument (NULL pointer, M < 1, dt <= 0, ...)   */
    LTS_EMESH = -2,      /* inconsistent mesh connectivity or geometry         */
    LTS_ELABEL = -3,     /* unusable LTS regions (no fine cell, all fine, ...) */
    LTS_ENONFINITE = -4, /* a step produced Inf/NaN; state invalid until init  */
    LTS_EDEVICE = -5,    /* HIP runtime error                                  */
    LTS_ESTATE = -6,     /* call out of order (no mesh, no state)              */
    LTS_ENOMEM = -7      /* device or host allocation failed                   */
} lts_status;

typedef enum { LTS_FP64 = 0, LTS_FP32 = 1 } lts_precision;

/* Region labels, eq:indexSetsCells / eq:indexSetsEdges. */
typedef enum { LTS_C = 0, LTS_I2 = 1, LTS_I1 = 2, LTS_F = 3 } lts_region;

/* Largest number of edges a cell may have: the slot capacity of the cell
   kernels (8 lanes per cell up to 8 edges, 16 lanes above). */
#define LTS_MAX_EDGES 16
#define LTS_MAX_LEVELS 8  /* LTS levels of lts_upload_mesh_levels (fine levels + 1) */

typedef struct lts_ctx lts_ctx;

/* MPAS-style mesh (Appendix B sets EC, EV, CE, VE; EE is derived). */
typedef struct {
    int32_t n_cells, n_edges, n_vertices, max_edges;
    const int32_t *n_edges_on_cell;      /* [n_cells]                          */
    const int32_t *edges_on_cell;        /* [n_cells][max_edges], ccw          */
    const int32_t *cells_on_cell;        /* [n_cells][max_edges]               */
    const int32_t *vertices_on_cell;     /* [n_cells][max_edges]               */
    const int32_t *cells_on_edge;        /* [n_edges][2]                       */
    const int32_t *vertices_on_edge;     /* [n_edges][2]                       */
    const int32_t *edges_on_vertex;      /* [n_vertices][3]                    */
    const int32_t *cells_on_vertex;      /* [n_vertices][3]                    */
    const double *kite_areas_on_vertex;  /* [n_vertices][3]: A_{i,v}, i = cells_on_vertex[v][k] */
    const double *area_cell;             /* [n_cells]    A_i                   */
    const double *area_triangle;         /* [n_vertices] A_v                   */
    const double *dc_edge;               /* [n_edges]    d_e (cell-to-cell)    */
    const double *dv_edge;               /* [n_edges]    l_e (primal edge)     */
    const double *f_vertex;              /* [n_vertices] Coriolis parameter    */
    const double *bottom;                /* [n_cells]    topography b_i        */
    const double *cell_xyz;              /* [n_cells][3] or NULL: positions, used
                                            only to order cells for locality     */
    /* Optional MPAS tables of eq:discPV (all three NULL, or all three given
       with max_edges2 >= 1).  The library derives the weights of eq:weights
       itself from the kite areas and never reads these in a step; when they
       are given, lts_upload_mesh and lts_plan check them against the derived
       ones: edges_on_edge[e] must list EE(e) (the other edges of both cells
       of e, n_edges_on_edge[e] = n_i + n_j - 2 of them, in any order) and
       |w - w_derived| <= 1e-9 (1 + |w_derived|) for each, with
       w_derived = -n_{e,i} n_{e',i} (R - 1/2), R the kite fractions
       A_{i,v}/A_i summed counter-clockwise around the shared cell i from e'
       to e.  A mismatch is LTS_EMESH naming the edge. */
    int32_t max_edges2;
    const int32_t *n_edges_on_edge;      /* [n_edges]                          */
    const int32_t *edges_on_edge;        /* [n_edges][max_edges2]              */
    const double *weights_on_edge;       /* [n_edges][max_edges2]              */
    /* Optional sign tables (each NULL or given).  The library derives both
       signs from the orientation convention above and never reads these in
       a step; given tables are checked against it: edge_sign_on_cell[i][j]
       must be n_{e,i} of e = edges_on_cell[i][j] (+1 when cells_on_edge[e][0]
       is i, else -1) and edge_sign_on_vertex[v][k] must be t_{e,v} of
       e = edges_on_vertex[v][k] (+1 when vertices_on_edge[e][1] is v, else
       -1).  A mismatch is LTS_EMESH naming the cell or vertex.  (A table
       with the opposite convention is the negation of these.) */
    const int8_t *edge_sign_on_cell;     /* [n_cells][max_edges]               */
    const int8_t *edge_sign_on_vertex;   /* [n_vertices][3]                    */
} lts_mesh;

typedef struct {
    double t;             /* simulated time                                     */
    double mass;          /* sum_i A_i h_i, FP64 on the device                  */
    double energy;        /* sum_i A_i (h_i K_i + g (h_i^2/2 + h_i b_i)), FP64  */
    double h_min, h_max, u_absmax;
    int64_t n_nonfinite;  /* non-finite h or u values in the state              */
    int64_t steps;        /* coarse steps (LTS) or steps (RK3) taken            */
    int64_t gate_fallbacks; /* surrogate steps the residual gate rejected and
                               the plain LTS3 step recomputed (lts_sur_step),
                               since the last lts_init_state                   */
} lts_diag;

/* Create a context on HIP device `device`, computing in `prec`.  hip_stream is
   a hipStream_t to enqueue on (it must outlive the context) or NULL for a
   context-owned stream. */
lts_status lts_create(lts_ctx **out, int device, lts_precision prec, void *hip_stream);

/* Advance n_layers independent copies of the system on the same mesh (the
   vertical layers of an ocean-like workload; default 1).  Call before
   lts_upload_mesh (LTS_ESTATE afterwards).  With L layers every state array
   passed to or returned by the library (lts_init_state, lts_get_state,
   lts_eval_rhs and their device forms) holds the L fields one after another:
   h[l * n_cells + i], u[l * n_edges + e].  Diagnostics sum or reduce over all
   layers.  On the device each per-element array is [element][layer], so a
   wave works on consecutive layers of one element and reads its mesh
   coefficients once. */
lts_status lts_set_layers(lts_ctx *ctx, int n_layers);

/* Validate and upload the mesh, label the LTS regions (F = cells with
   fine_mask != 0; I1 = n_if1_rings breadth-first cell rings around F; I2 = the
   next n_if2_rings; C = the rest; underlined F = the two fine rings nearest
   I1; each edge takes the finest region of its two cells) and fold the TRiSK
   coefficients, including the weights of eq:weights, from the kite areas.
   LTS_EMESH on inconsistent connectivity, LTS_ELABEL on unusable regions.
   Replaces any previous mesh and invalidates the state. */
lts_status lts_upload_mesh(lts_ctx *ctx, const lts_mesh *mesh, const uint8_t *fine_mask,
                           int n_if1_rings, int n_if2_rings, double gravity);

/* More than two LTS levels (Remark 3.1: regions of several resolutions,
   each neighbouring pair with an integer step ratio).  fine_masks holds
   n_fine_levels nested masks of n_cells bytes one after another, outermost
   first: level l's fine region F_l = cells with fine_masks[l][i] != 0, each
   labelled as lts_upload_mesh labels one fine region (n_if1_rings and
   n_if2_rings interface rings at every level).  Every fine, interface-1 and
   interface-2 cell of level l >= 1 must lie at least four cell rings inside
   F_{l-1} (LTS_ELABEL otherwise: three rings are what the method needs, the
   fourth keeps every level's evaluation sets contiguous in device order).
   n_fine_levels = 1 is lts_upload_mesh.  Layered contexts (lts_set_layers)
   advance every layer through the same levels.  Level 0's labels are the ones lts_get_regions and
   lts_region_counts report, and lts_step runs the two-level scheme on them. */
lts_status lts_upload_mesh_levels(lts_ctx *ctx, const lts_mesh *mesh, int n_fine_levels,
                                  const uint8_t *fine_masks, int n_if1_rings, int n_if2_rings,
                                  double gravity);

/* Labels of level `level` (0 .. n_fine_levels - 1), as lts_get_regions. */
lts_status lts_get_level_regions(lts_ctx *ctx, int level, int8_t *cell_region,
                                 int8_t *edge_region, uint8_t *cell_fbar, uint8_t *edge_fbar);

/* Advance n_steps coarse steps of multi-level LTS3 on a mesh uploaded with
   lts_upload_mesh_levels: M[l] (l = 0 .. n_fine_levels - 1, each >= 1) is the
   step ratio of level l to level l+1.  Level l's M[l] fine substeps on F_l
   are LTS3 steps of level l+1 (the deepest level takes SSPRK3 substeps);
   each level's Steps 1, 2 and 4 also evaluate the enclosing level's
   interface, which accumulates those right-hand sides (Steps 3.s.2) for its
   correction (Step 5).  Conserves mass exactly; the innermost fine cells
   take steps of dt_coarse / (M[0] M[1] ... M[n_fine_levels - 1]).  Asynchronous.
   LTS_EINVAL for a two-level mesh, a NULL M, a ratio < 1 or dt_coarse <= 0. */
lts_status lts_step_levels(lts_ctx *ctx, double dt_coarse, const int32_t *M, int n_steps);

/* Region labels in the caller's numbering (host arrays, any may be NULL). */
lts_status lts_get_regions(lts_ctx *ctx, int8_t *cell_region, int8_t *edge_region,
                           uint8_t *cell_fbar, uint8_t *edge_fbar);

/* Set the state from host arrays h[n_cells], u[n_edges] (caller numbering). */
lts_status lts_init_state(lts_ctx *ctx, const double *h, const double *u, double t0);

/* Same from device arrays in the context precision (caller numbering); they
   are read only during the call.  A set-up path, not a fast path: the arrays
   are staged through host memory (synchronous copies), where the FP32 form's
   reference thickness is derived from them exactly as for lts_init_state. */
lts_status lts_init_state_device(lts_ctx *ctx, const void *d_h, const void *d_u, double t0);

/* Advance n_steps coarse steps of LTS3 (Algorithm 2.2, order 3) with coarse
   step dt_coarse and fine step dt_coarse/M.  Asynchronous.  LTS_EINVAL when
   M < 1 or dt_coarse <= 0. */
lts_status lts_step(lts_ctx *ctx, double dt_coarse, int M, int n_steps);

/* Advance n_steps steps of global SSPRK3 (Algorithm 2.1) with step dt over the
   whole mesh; an independent code path from lts_step. */
lts_status lts_step_rk3(lts_ctx *ctx, double dt, int n_steps);

/* Time integration schemes of lts_step_scheme. */
typedef enum {
    LTS_SCHEME_LTS3 = 0,   /* Algorithm 2.2, third-order branch (= lts_step)      */
    LTS_SCHEME_LTS2 = 1,   /* Algorithm 2.2, second-order branch                  */
    LTS_SCHEME_SSPRK3 = 2, /* Algorithm 2.1, three stages (= lts_step_rk3)        */
    LTS_SCHEME_SSPRK2 = 3, /* Algorithm 2.1, two stages                           */
    LTS_SCHEME_RK4 = 4     /* classical RK4, the paper's reference and competitor */
} lts_scheme;

/* Advance n_steps steps of `scheme` with step dt (the coarse step for LTS2/3,
   fine step dt/M; M is ignored by the global schemes).  Asynchronous. */
lts_status lts_step_scheme(lts_ctx *ctx, int scheme, double dt, int M, int n_steps);

/* Evaluate the right-hand side (H, U) of eq:sweTimeStepping at the given host
   state (caller numbering) over the whole mesh.  Does not change the state. */
lts_status lts_eval_rhs(lts_ctx *ctx, const double *h, const double *u,
                        double *dh, double *du);

/* FP64 diagnostics of the current state (synchronises).  Returns
   LTS_ENONFINITE, sticky until the next init, when a step produced Inf/NaN. */
lts_status lts_diagnostics(lts_ctx *ctx, lts_diag *out);

/* Copy the state to host doubles (caller numbering; synchronises). */
lts_status lts_get_state(lts_ctx *ctx, double *h, double *u);

/* Copy the state to device arrays in the context precision (caller numbering;
   staged through host memory like lts_init_state_device; synchronises). */
lts_status lts_get_state_device(lts_ctx *ctx, void *d_h, void *d_u);

/* Per-kernel timing: when enabled, steps launch without graphs and every
   kernel is launched with start/stop events stamped by the GPU at the kernel's
   own start and end; lts_kernel_stats reports per kernel class the number of
   launches, total milliseconds and algorithmic bytes (every array element a
   launch needs, read or written once).  Classes: 0 vertex potential vorticity,
   1 cell tendency, 2 edge tendency (with the interface prediction and
   correction blocks it carries).  Returns the number of classes written. */
lts_status lts_set_timing(lts_ctx *ctx, int enable);
int lts_kernel_stats(lts_ctx *ctx, int max_classes, int64_t *launches, double *ms,
                     double *bytes);

/* Element counts of the LTS regions after upload: cells[4] and edges[4] in
   lts_region order (C, I2, I1, F), fbar[2] = underlined-F cells, edges. */
lts_status lts_region_counts(lts_ctx *ctx, int64_t *cells, int64_t *edges, int64_t *fbar);

/* Host-only planning, no device needed: validate `mesh`, label the regions
   and compute the device ordering exactly as lts_upload_mesh does.  Outputs
   (any may be NULL): region labels and underlined-F flags in caller numbering;
   cell/edge/vertex order (position -> caller index); ranges[54] = 8 cell class
   starts (F minus underlined F, F2, F1, I1, I2, C1, rest of C, end), 6 edge
   class starts (F minus underlined F, underlined F, I1, I2, C, end), then for
   each of the 5 pass kinds (full mesh, Step 1, Step 2, Step 3, Step 4) the
   cell-kernel range, vertex range, target cells and target edges (8 ints).
   On error the message goes to errbuf (errlen bytes, may be NULL). */
lts_status lts_plan(const lts_mesh *mesh, const uint8_t *fine_mask, int n_if1_rings,
                    int n_if2_rings, int8_t *cell_region, int8_t *edge_region,
                    uint8_t *cell_fbar, uint8_t *edge_fbar, int32_t *cell_order,
                    int32_t *edge_order, int32_t *vertex_order, int32_t *ranges,
                    char *errbuf, int errlen);

/* Host-only planning of a multi-level mesh (no device needed): the device
   ordering and, per level l (0 .. n_fine_levels - 1), 46 int32 ranges:
   cell class starts [8] (F interior, F2, F1, I1, I2, C1, rest of C, end of
   the level's domain), edge class starts [6] (F-interior edges, underlined-F
   edges, I1, I2, C, end of the domain), then four passes (Steps 1, 2, 3, 4;
   Steps 1, 2 and 4 of level l >= 1 also target level l-1's interface) of 8
   entries each: cell kernel range, vertex range, target cells, target
   edges (lo, hi pairs).  fine_masks, rings and errors as
   lts_upload_mesh_levels; errbuf receives the message. */
lts_status lts_plan_levels(const lts_mesh *mesh, int n_fine_levels, const uint8_t *fine_masks,
                           int n_if1_rings, int n_if2_rings, int32_t *cell_order,
                           int32_t *edge_order, int32_t *vertex_order, int32_t *ranges,
                           char *errbuf, int errlen);

const char *lts_last_error(const lts_ctx *ctx);
void lts_destroy(lts_ctx *ctx);

/* ------------------------------------------------------------------------
   Ensembles: many independent LTS3 runs of uneven size advanced together.
   Each member has its own mesh, regions, coarse step dt and ratio M; one
   ensemble step advances every member by one coarse step.  The members'
   passes are batched into shared launches over device work lists (one per
   phase, kernel class and member class: size < 30k cells, < 120k, larger,
   each split by whether some cell has more than 8 edges), the classes run as
   concurrent branches of one hipGraph, and an autotuner picks block and grid
   size per (kernel class, member class).
   Results equal lts_step on each member alone (same kernels and arithmetic).
   Call order: create, add_member..., init_member (every member), build,
   step..., get_member / diagnostics, destroy.  Not thread-safe. */
typedef struct lts_ens lts_ens;

lts_status lts_ens_create(lts_ens **out, int device, lts_precision prec, void *hip_stream);
/* Add a member (arguments as lts_upload_mesh, plus its coarse step and M);
   *member receives its index.  LTS_ESTATE after lts_ens_build. */
lts_status lts_ens_add_member(lts_ens *ens, const lts_mesh *mesh, const uint8_t *fine_mask,
                              int n_if1_rings, int n_if2_rings, double gravity, double dt_coarse,
                              int M, int *member);
/* Add a multi-level member (Remark 3.1; mesh, masks and rings as
   lts_upload_mesh_levels, M[l] for l = 0 .. n_fine_levels - 1 as
   lts_step_levels): each ensemble step advances it by one multi-level coarse
   step, its passes batched with the other members' (results equal
   lts_step_levels on the member alone).  In the SSPRK3 mode
   (lts_ens_set_scheme) it takes prod M[l] steps of dt_coarse / prod M[l].
   LTS_EINVAL for a NULL M, a ratio < 1, ratios whose product exceeds 2^20 or
   n_fine_levels outside 1 .. LTS_MAX_LEVELS - 1; labelling errors as
   lts_upload_mesh_levels; LTS_ESTATE after lts_ens_build. */
lts_status lts_ens_add_member_levels(lts_ens *ens, const lts_mesh *mesh, int n_fine_levels,
                                     const uint8_t *fine_masks, int n_if1_rings,
                                     int n_if2_rings, double gravity, double dt_coarse,
                                     const int32_t *M, int *member);
/* Host state of one member (caller numbering), as lts_init_state. */
lts_status lts_ens_init_member(lts_ens *ens, int member, const double *h, const double *u);
/* Plan the work lists, autotune when autotune != 0 (member states are
   restored afterwards), capture the step graph.  Every member must be
   initialised. */
lts_status lts_ens_build(lts_ens *ens, int autotune);
/* Advance every member by n_steps coarse steps.  Asynchronous. */
lts_status lts_ens_step(lts_ens *ens, int n_steps);
/* Choose what one ensemble step does and drop the current build (call
   lts_ens_build again; autotune = 0 keeps the previous tuning): scheme 0
   (LTS3, the default) advances member j by one LTS3 coarse step of
   dt_coarse[j] with its M; scheme 2 (global SSPRK3, Algorithm 2.1) advances
   it over the same dt_coarse[j] in M_j SSPRK3 steps of dt_coarse[j]/M_j,
   through the same batched work lists.  dt_coarse[n_members] (may be NULL:
   keep each member's) replaces the coarse steps.  Member states are kept.
   LTS_EINVAL for another scheme or a step <= 0. */
lts_status lts_ens_set_scheme(lts_ens *ens, int scheme, const double *dt_coarse);
/* Run each ensemble step as one persistent fused kernel (enable != 0) or as
   the batched launches per (phase, kernel class, size class) (enable = 0, the
   default), and drop the current build (call lts_ens_build again).  The
   fused kernel is one cooperative launch of 256-thread blocks, as many as
   fit on the device at once, that works through every phase of every
   member's step, the vertex, cell and edge work of a phase separated by
   grid-wide barriers on device-scope atomics; it is captured into the step's
   hipGraph when the runtime accepts that, else launched directly.  Every
   barrier wait is bounded by spin_limit polls (0: 2^22); one that runs out
   makes every block leave the kernel, and lts_ens_step (which synchronises
   in this mode) returns LTS_EDEVICE with the member states undefined until
   they are re-initialised.  Results are those of the batched launches (same
   arithmetic per element).  LTS_EINVAL for spin_limit < 0. */
lts_status lts_ens_set_fused(lts_ens *ens, int enable, int spin_limit);
/* Timing mode: advance every member by n_steps ensemble steps with each
   batched launch stamped by HIP events (launches issued one after another on
   the ensemble's stream, no graph), and return per kernel class (vertex,
   cell, edge) the launch count, the summed kernel time in ms and the summed
   algorithmic bytes (every array element a launch needs, read or written
   once).  With the fused kernel every step is one launch, reported in the
   cell entry (index 1) with the bytes of all three classes; the other two
   entries are zero.  Synchronises.  LTS_ESTATE before lts_ens_build. */
lts_status lts_ens_kernel_stats(lts_ens *ens, int n_steps, int64_t *launches, double *ms,
                                double *bytes);
lts_status lts_ens_get_member(lts_ens *ens, int member, double *h, double *u);
lts_status lts_ens_diagnostics(lts_ens *ens, int member, lts_diag *out);
/* Autotuner choices: tuned[(k*3+s)*2 + {0,1}] = block size, grid factor (grid =
   factor x compute units) for kernel class k (0 vertex, 1 cell, 2 edge) and
   size class s; tuned_us[k*3+s] = the timed microseconds of that choice;
   class_cells[s] = cells per size class; *n_launches = launches per step;
   step_bytes[k] = algorithmic bytes of kernel class k in one ensemble step
   (every array element a launch needs, read or written once).  Any pointer
   may be NULL. */
lts_status lts_ens_info(lts_ens *ens, int32_t *tuned, double *tuned_us, int64_t *class_cells,
                        int32_t *n_launches, double *step_bytes);
const char *lts_ens_last_error(const lts_ens *ens);
void lts_ens_destroy(lts_ens *ens);

#ifdef __cplusplus
}
#endif
#endif
