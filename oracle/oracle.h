/*
 * FP64 CPU oracle for LTS3/LTS2 local time stepping of the TRiSK shallow water
 * equations (Capodaglio & Petersen, "Local time stepping for the shallow water
 * equations in MPAS", arXiv 2106.07154).
 *
 * TEST INFRASTRUCTURE.  This code exists only to check the GPU library.  Only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no code, header or table with the GPU library.
 *
 * Everything is plain, unblocked double-precision loops that follow the
 * paper's definitions:
 *   - discrete operators: Appendix B (TRiSK), equation for the PV flux
 *     (eq:discPV), the perpendicular flux (eq:Feperp), the weights (eq:weights),
 *     kinetic energy, divergence and gradient;
 *   - SSPRK2/SSPRK3: Algorithm 2.1;
 *   - LTS2/LTS3: Algorithm 2.2 with the index sets of eq:indexSetsCells,
 *     eq:index_sets_cells and eq:indexSetsEdges;
 *   - RK4: the classical four-stage scheme the paper uses as reference solver
 *     (Section 3.1) and competitor.
 *
 * Mesh orientation conventions (same as the input generator documents):
 *   cellsOnEdge[e] = (c0, c1): n_e points from c0 to c1, n_{e,c0}=+1, n_{e,c1}=-1.
 *   verticesOnEdge[e] = (v0, v1): t_e = k x n_e points from v0 to v1,
 *     t_{e,v1}=+1, t_{e,v0}=-1.
 *   edgesOnCell[i][*] counter-clockwise; verticesOnCell[i][j] is shared by
 *     edgesOnCell[i][j] and edgesOnCell[i][j+1].
 * Arrays are row-major: edgesOnCell[i*maxEdges + j], cellsOnEdge[2*e + s],
 * edgesOnVertex[3*v + k].
 */
#ifndef LTS_ORACLE_H
#define LTS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct om_ctx om_ctx;

/* Region labels (cells and edges). */
enum { OM_C = 0, OM_I2 = 1, OM_I1 = 2, OM_F = 3 };

om_ctx *om_create(int nCells, int nEdges, int nVertices, int maxEdges,
                  const int32_t *nEdgesOnCell, const int32_t *edgesOnCell,
                  const int32_t *cellsOnCell, const int32_t *verticesOnCell,
                  const int32_t *cellsOnEdge, const int32_t *verticesOnEdge,
                  const int32_t *edgesOnVertex, const int32_t *cellsOnVertex,
                  const double *kiteAreasOnVertex, const double *areaCell,
                  const double *areaTriangle, const double *dcEdge,
                  const double *dvEdge, const double *fVertex,
                  const double *bottom, double gravity);
void om_destroy(om_ctx *c);

/* Number of entries in EE(e) (edges of both cells of e, minus e). */
int om_n_edges_on_edge(const om_ctx *c, int e);
/* TRiSK weights w_{e,e'} of eq:weights: out[k] for the k-th member of EE(e),
   members written to ee[k].  Returns the count. */
int om_weights_on_edge(const om_ctx *c, int e, int32_t *ee, double *w);

/* Discrete right-hand side (eq:sweTimeStepping / eq:sweDiscrete):
   dh[i] = H_i(h,u) = -[div F]_i, du[e] = U_e(h,u) = -F_perp[q] - [grad(g(h+b)+K)]_e. */
void om_rhs(const om_ctx *c, const double *h, const double *u,
            double *dh, double *du);
/* Intermediate diagnostics of the same evaluation (for operator pins). */
void om_diag_fields(const om_ctx *c, const double *h, const double *u,
                    double *K /*cells*/, double *q /*vertices*/,
                    double *zeta /*vertices*/, double *fperp /*edges: F_perp_e*/);

/* LTS region sets.  fine_mask[i] != 0 marks F.  I1 is n1 breadth-first cell
   rings around F, I2 the next n2 rings, C the rest.  fbar marks the two fine
   rings nearest I1 (cells) and the underlined-F edge set.  Returns 0, or -1 when
   the labels are unusable (no fine cell, every cell fine, n1 < 1 or n2 < 1). */
int om_regions(const om_ctx *c, const uint8_t *fine_mask, int n1, int n2,
               int8_t *cell_region, int8_t *edge_region,
               uint8_t *cell_fbar, uint8_t *edge_fbar);

/* One step of global SSPRK2 (order 2) or SSPRK3 (order 3), in place. */
void om_ssprk_step(const om_ctx *c, int order, double *h, double *u, double dt);
/* One step of classical RK4, in place. */
void om_rk4_step(const om_ctx *c, double *h, double *u, double dt);
/* One coarse step of LTS2 (order 2) or LTS3 (order 3) with fine step dt/M,
   in place.  Region arrays as produced by om_regions. */
void om_lts_step(const om_ctx *c, int order, const int8_t *cell_region,
                 const int8_t *edge_region, const uint8_t *cell_fbar,
                 const uint8_t *edge_fbar, double *h, double *u,
                 double dt, int M);

/* More than two LTS levels (Remark 3.1), LTS3 only.  nlev >= 2 levels; level
   l < nlev - 1 has the fine region masks[l*nCells ...] (nested: each inside
   the previous one) and the step ratio M[l] to level l+1.  om_mlts_regions
   labels every level (arrays of nlev-1 blocks of nCells / nEdges entries, as
   om_regions) and returns -1 unless every fine, interface-1 and interface-2
   cell of level l >= 1 lies at least three cell rings inside the fine region
   of level l-1.  om_mlts_step advances one coarse step dt in place: level l's
   fine substeps are LTS3 steps of level l+1 (see oracle.c); with nlev = 2 it
   is om_lts_step of order 3. */
int om_mlts_regions(const om_ctx *c, int nlev, const uint8_t *masks, int n1, int n2,
                    int8_t *cell_region, int8_t *edge_region, uint8_t *cell_fbar,
                    uint8_t *edge_fbar);
void om_mlts_step(const om_ctx *c, int nlev, const int8_t *cell_region,
                  const int8_t *edge_region, const uint8_t *cell_fbar,
                  const uint8_t *edge_fbar, const int32_t *M, double *h, double *u,
                  double dt);

/* Interface-1 prediction coefficients (a, b, c) such that the predicted value
   is a*x_old + b*x_1st + c*x_2nd, for stage s in {0,1,2} of fine substep k. */
void om_lts_predict_coeffs(int order, int stage, int k, int M, double out[3]);

/* Select a reading of the garbled passages (0 = the defended one; see
   oracle.c).  Test-only: lets tests show the literal text fails the pins. */
void om_set_reading(int r);
int om_get_reading(void);

/* Diagnostics: mass = sum A_i h_i (compensated), energy =
   sum_i A_i (h_i K_i + g (h_i^2/2 + h_i b_i)) (compensated). */
void om_diagnostics(const om_ctx *c, const double *h, const double *u,
                    double *mass, double *energy);

#ifdef __cplusplus
}
#endif
#endif
