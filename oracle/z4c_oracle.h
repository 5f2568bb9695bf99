/*
 * Z4c reference oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded FP64 implementation of the discrete Z4c
 * method described in "Performance-Portable Numerical Relativity with
 * AthenaK" (arXiv 2409.10383): cell-centred finite differences inside
 * ghost-zoned MeshBlocks (Sec. 3), per-stage ghost filling from neighbour
 * active zones or boundary conditions (Sec. 3), Lagrange restriction and
 * prolongation at refinement boundaries (Sec. 3.1, Eqs. 1-2), the Z4c
 * evolution system with 1+log lapse and Gamma-driver shift (Sec. 2; the
 * equations are the standard published Z4c system the paper defers to),
 * classic RK4 (Sec. 4.3), constraint monitors and the chi-based refinement
 * criteria (Sec. 3.3).
 *
 * Only the test-suite, the package smoke check and the benchmark's CPU
 * baseline may load this code.  The GPU library shares nothing with it.
 *
 * Storage: block b holds Z4C_ONF fields, each a cube of E=n_b+2g cells per
 * axis, x fastest: u[off_b + ((f*E + k)*E + j)*E + i], with
 * off_b = sum_{c<b} Z4C_ONF*E_c^3.  Interior-only outputs use the same order
 * with E=n_b and no ghosts.
 */
#ifndef Z4C_ORACLE_H
#define Z4C_ORACLE_H

#include <stdint.h>

#define ONF 22   /* number of evolved Z4c fields */

/* field order */
enum { O_CHI = 0, O_GXX, O_GXY, O_GXZ, O_GYY, O_GYZ, O_GZZ, O_KHAT,
       O_AXX, O_AXY, O_AXZ, O_AYY, O_AYZ, O_AZZ, O_GAMX, O_GAMY, O_GAMZ,
       O_THETA, O_ALPHA, O_BETAX, O_BETAY, O_BETAZ };

/* term-mask bits (the full method is all four) */
enum { OT_PHYS = 1, OT_GAUGE = 2, OT_ADVECT = 4, OT_DISSIP = 8 };

typedef struct {
    int32_t nb;          /* number of MeshBlocks                            */
    const int32_t *level;/* [nb] refinement level, 0 = root                  */
    const int32_t *n;    /* [nb] interior cells per axis (cubic blocks)      */
    const int32_t *ilo;  /* [3*nb] lower interior corner, in cells of level  */
    int32_t g;           /* ghost layers                                     */
    int32_t nroot[3];    /* root-level cells per axis over the whole domain  */
    int32_t bc;          /* 0 periodic, 1 outflow, 2 user (ghosts untouched) */
    int32_t pad;
    double lo[3];        /* domain lower corner                              */
    double dx0;          /* root-level cell size                             */
} or_mesh;

typedef struct {
    int32_t fd_order;    /* 4, 6 or 8                                        */
    uint32_t terms;      /* OT_* mask                                        */
    int32_t enforce;     /* 1: algebraic constraints + floors after writes   */
    int32_t pad;
    double ko_sigma, kappa1, kappa2, eta, mu_S, chi_floor, alpha_floor;
} or_params;

/* 1D finite-difference weights (Fornberg recurrence). */
int or_fd_weights(int deriv, int npts, const double *pts, double *w);

/* offsets/sizes */
int64_t or_block_offset(const or_mesh *m, int b);
int64_t or_total_size(const or_mesh *m);

/* ghost fill of every block of a register (all fields) */
int or_fill_ghosts(const or_mesh *m, double *u);
/* the ghosts of the blocks with only[b] != 0 (all when NULL) written into u,
 * every value computed from the active zones of src (a copy of u): disjoint
 * block sets may run concurrently */
int or_fill_ghosts_from(const or_mesh *m, const double *src, double *u, const int8_t *only);

/* RHS of all interior zones; u must have ghosts filled. rhs: interior layout */
int or_rhs(const or_mesh *m, const or_params *p, const double *u, double *rhs);
/* same, only for blocks with only[b] != 0 (others left untouched) */
int or_rhs_blocks(const or_mesh *m, const or_params *p, const double *u, double *rhs,
                  const int8_t *only);

/* one classic RK4 stage on registers U,S1,S2,A (ghosted layout, all FP64):
 * fills ghosts of the stage input itself. */
int or_rk4_stage(const or_mesh *m, const or_params *p, int stage, double dt,
                 double *U, double *S1, double *S2, double *A);
/* the register update of one stage (the writes above, with enforcement)
 * from a precomputed RHS k (interior layout), only for blocks with
 * only[b] != 0 (every block when only is NULL); ghosts are not touched, so
 * disjoint block sets may run concurrently */
int or_rk4_update(const or_mesh *m, const or_params *p, int stage, double dt, const double *k,
                  double *U, double *S1, double *S2, double *A, const int8_t *only);

/* constraints; out: interior layout with 8 components per zone
 * (H, Mx, My, Mz, Theta, Gx, Gy, Gz); norms[6] = H_L2, H_Linf, M_L2, M_Linf,
 * Theta_L2, G_L2 over zones outside r_exc of the centres (nexc may be 0). */
int or_constraints(const or_mesh *m, const or_params *p, const double *u,
                   double *out, int nexc, const double *exc_centres,
                   double r_exc, double *norms);

/* refinement flags, one int8 per block */
int or_refine_flags(const or_mesh *m, const or_params *p, const double *u,
                    int criterion, double chi_thr, double dchi_thr,
                    int level_max, double radius, const double *centre,
                    int radius_level, int8_t *flags);

/* Psi4 (Re, Im) at every interior zone, coordinate tetrad about origin[3];
 * u must have ghosts filled; out: interior layout with 2 components */
int or_psi4(const or_mesh *m, const or_params *p, const double *u, const double *origin, double *out);

/* 16 raw per-block features for the learned refinement indicator */
int or_block_features(const or_mesh *m, const or_params *p, const double *u, double *feat);

#endif
