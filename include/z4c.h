/*
 * z4c.h -- C ABI of the MI355X Z4c hot-path library (libz4c.so).
 *
 * The library evolves the vacuum Z4c system of "Performance-Portable
 * Numerical Relativity with AthenaK" (arXiv 2409.10383) on a MeshBlockPack:
 * a Mesh of cubic MeshBlocks, each an active region plus g ghost layers,
 * grouped so that one launch covers all of them (Sec. 3).  Ghosts are filled
 * at every Runge-Kutta stage from neighbour active zones, from boundary
 * conditions, or at refinement boundaries by Lagrange restriction and
 * prolongation with n = g+1 points per axis (Sec. 3.1, Eqs. 1-2).  The
 * right-hand side uses cell-centred finite differences of order 2(g-1) or
 * lower (Sec. 3 footnote, Sec. 3.2), Kreiss-Oliger dissipation, the 1+log
 * lapse and Gamma-driver shift, and constraint damping (Sec. 2, Sec. 4.3);
 * time integration is classic RK4 (Sec. 4.3).
 *
 * Conventions shared by every call:
 *  - Return value: Z4C_OK (0) or a negative Z4C_E* status.  Nothing aborts,
 *    prints or throws.  z4c_last_error() gives a message for the last failure
 *    on a pack.
 *  - Memory: the CALLER owns all device memory.  The library never allocates
 *    or frees device memory; z4c_pack_query reports the bytes needed for the
 *    four registers and for a workspace, and z4c_pack_bind takes device
 *    pointers to them.  Host-side pack metadata is allocated by
 *    z4c_pack_create and freed by z4c_pack_destroy.
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = the default
 *    stream).  Calls enqueue work and return; only calls that return host
 *    values (norms, flags, features) synchronise that stream.
 *  - Arguments are validated before anything is enqueued; a rejected call
 *    has no effect (Z4C_EINVAL).
 *  - A pack is not thread-safe; calls on one pack must be serialised.
 *
 * Register layout (device memory, one allocation per register):
 *  - State registers U, S1, S2: block b starts at element offset
 *    z4c_block_offset (its state offset); it holds Z4C_NFIELDS fields, field f at
 *    offset + f*slab_b, each a cube of E_b = n_b + 2g cells, x fastest:
 *    index ((k*E + j)*E + i), i,j,k in [0,E), active cells at [g, g+n).
 *    slab_b = E_b^3 rounded up to a multiple of 256 bytes.  Elements are
 *    double (Z4C_FP64) or float (Z4C_FP32_MIXED).
 *  - Accumulator A: always double, active cells only: block b at the
 *    interior offset of z4c_block_offset, field f at + f*n_b^3, x fastest.
 *  - Interior outputs (z4c_rhs, per-zone constraints) use the layout of A.
 * Field order (f = 0..21):
 *   chi, gxx, gxy, gxz, gyy, gyz, gzz, Khat, Axx, Axy, Axz, Ayy, Ayz, Azz,
 *   Gamx, Gamy, Gamz, Theta, alpha, betax, betay, betaz
 */
#ifndef Z4C_H
#define Z4C_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define Z4C_NFIELDS 22
#define Z4C_NREG 4
#define Z4C_NNORM 6
#define Z4C_NFEAT 16
#define Z4C_MAXTRACK 8

enum {
    Z4C_OK = 0,
    Z4C_EINVAL = -1,       /* invalid argument or pack description          */
    Z4C_ENOMEM = -2,       /* host allocation failed / workspace too small   */
    Z4C_EDEVICE = -3,      /* a HIP call failed                              */
    Z4C_ESTATE = -4,       /* call out of order (e.g. not bound)             */
    Z4C_ENONFINITE = -5,   /* non-finite value found (finite check enabled)  */
    Z4C_EUNSUPPORTED = -6  /* valid but not supported by this library        */
};

enum { Z4C_REG_U = 0, Z4C_REG_S1 = 1, Z4C_REG_S2 = 2, Z4C_REG_A = 3 };
enum { Z4C_BC_PERIODIC = 0, Z4C_BC_OUTFLOW = 1, Z4C_BC_USER = 2 };
enum { Z4C_FP64 = 0, Z4C_FP32_MIXED = 1 };
/* term mask: the full method is Z4C_TERM_ALL; subsets exist for tests */
enum {
    Z4C_TERM_PHYS = 1,    /* Z4c terms of chi, g~, Khat, A~, Gamma~, Theta  */
    Z4C_TERM_GAUGE = 2,   /* 1+log lapse and Gamma-driver shift terms       */
    Z4C_TERM_ADVECT = 4,  /* beta^k d_k (lapse/shift only with GAUGE)       */
    Z4C_TERM_DISSIP = 8,  /* Kreiss-Oliger on all 22 fields                 */
    Z4C_TERM_ALL = 15
};
enum {
    Z4C_FLAG_ENFORCE = 1,       /* det g~ = 1, tr A~ = 0, floors after writes */
    Z4C_FLAG_CHECK_FINITE = 2,  /* z4c_rk4_step checks U for non-finite values */
    Z4C_FLAG_GRAPH = 4          /* z4c_rk4_step replays a captured hipGraph  */
};

/* One MeshBlock: cubic, n^3 active cells at refinement `level`, lower
 * active corner `ilo` in cells of that level (cell size dx0 / 2^level). */
typedef struct {
    int32_t level;
    int32_t n;
    int32_t ilo[3];
} z4c_block;

typedef struct {
    int32_t fd_order;      /* 4, 6 or 8 (centred order 2N)                   */
    int32_t nghost;        /* g >= N + 1                                     */
    int32_t precision;     /* Z4C_FP64 or Z4C_FP32_MIXED                     */
    int32_t bc;            /* Z4C_BC_*                                       */
    int32_t nroot[3];      /* root-level cells per axis over the domain      */
    int32_t pad0;
    double lo[3];          /* domain lower corner                            */
    double dx0;            /* root-level cell size                           */
    double ko_sigma;       /* Kreiss-Oliger strength (paper: 0.5)            */
    double kappa1;         /* constraint damping (paper: 0.02)               */
    double kappa2;         /* (paper: 0)                                     */
    double eta;            /* Gamma-driver damping (2/M)                     */
    double mu_S;           /* Gamma-driver coefficient (1)                   */
    double chi_floor;      /* floor of chi, also used wherever chi divides   */
    double alpha_floor;    /* floor of the lapse                             */
    uint32_t terms;        /* Z4C_TERM_* mask                                */
    uint32_t flags;        /* Z4C_FLAG_* mask                                */
} z4c_params;

typedef struct {
    size_t reg_bytes[Z4C_NREG]; /* bytes of U, S1, S2, A                      */
    size_t workspace_bytes;     /* bytes of the workspace                     */
    int64_t nblocks;
    int64_t zones;              /* active cells of the pack                   */
    int32_t state_elem_bytes;   /* 8 (FP64) or 4 (FP32_MIXED)                 */
    int32_t nwork;              /* work items of the fused stage kernel       */
    int64_t nxfer;              /* cross-level copies/restrictions per fill   */
    int64_t nprolong;           /* cross-level prolongated ghost cells        */
} z4c_layout;

/* Norm region for z4c_constraints: zones with centre within r_exc of any
 * listed centre are left out of the norms (ncentres may be 0). */
typedef struct {
    int32_t ncentres;
    int32_t pad;
    double centres[8][3];
    double r_exc;
} z4c_norm_region;

/* Refinement criteria (Sec. 3.3). */
enum { Z4C_CRIT_CHI_MIN = 0, Z4C_CRIT_DCHI_MAX = 1, Z4C_CRIT_RADIUS = 2 };
typedef struct {
    int32_t criterion;     /* Z4C_CRIT_*                                     */
    int32_t level_max;     /* no +1 at or above this level                   */
    double chi_thr;        /* chi-min: refine if min chi < chi_thr (0.3)     */
    double dchi_thr;       /* dchi-max: refine if max |grad chi| > dchi_thr  */
    double radius;         /* radius: zones within `radius` of `centre` ...  */
    double centre[3];
    int32_t radius_level;  /* ... require level >= radius_level              */
    int32_t pad;
} z4c_refine_params;

/* ------------------------------------------------------------------ pack */

/* Validate a pack description and build its host metadata (Sec. 3: Mesh,
 * MeshBlocks, MeshBlockPack).  Checks: fd_order in {4,6,8}; nghost >= N+1
 * (the Kreiss-Oliger and lopsided stencils reach N+1 cells); nblocks >= 1;
 * every n a multiple of 8 (the stage kernel's tiles), 8 <= n <= 512 and
 * n >= nghost; levels 0..7; blocks inside
 * the domain, not overlapping, covering it; neighbouring levels differ by at
 * most one (the 2:1 rule, Sec. 3.3) with refinement-boundary stencils that
 * stay within one level.  Returns Z4C_EINVAL on any violation.  `blocks` is
 * host memory, copied.  On success *out owns host memory only. */
int z4c_pack_create(const z4c_params *params, const z4c_block *blocks, int32_t nblocks,
                    struct z4c_pack **out);

/* Sizes of the registers and the workspace the caller must allocate. */
int z4c_pack_query(const struct z4c_pack *pack, z4c_layout *out);

/* Element offset of block b in a state register (ghosted layout) and in the
 * accumulator / interior layout. */
int z4c_block_offset(const struct z4c_pack *pack, int32_t b, int64_t *state_off,
                     int64_t *interior_off);

/* Attach caller-owned device memory: regs[Z4C_NREG] (U, S1, S2, A) of at
 * least reg_bytes[r] each, 256-byte aligned; workspace of at least
 * workspace_bytes.  Uploads the block, neighbour and interpolation tables
 * into the workspace on `stream` (the call returns after the upload has been
 * enqueued; the workspace must not be reused while the pack is bound).
 * Packs with more than one refinement level also create, on the first bind
 * and on the current device, one non-blocking stream of default priority and
 * two events: each ghost fill forks its same-level copies onto that stream
 * beside the cross-level work and joins back to the caller's stream before
 * the call's next launch, so the caller sees stream-ordered results.
 * Z4C_EDEVICE if the stream or events cannot be created. */
int z4c_pack_bind(struct z4c_pack *pack, void *const regs[Z4C_NREG], void *workspace,
                  size_t workspace_bytes, void *stream);

/* Free host metadata; waits for the side stream of a multi-level pack and
 * destroys it.  Device memory stays the caller's. */
void z4c_pack_destroy(struct z4c_pack *pack);

/* Message of the last failed call on `pack` ("" if none). */
const char *z4c_last_error(const struct z4c_pack *pack);

/* ------------------------------------------------------------- hot path */

/* Fill every ghost cell of state register `reg` (U, S1 or S2): copies of
 * same-level neighbour active zones, periodic wrap or outflow copy of the
 * nearest active zone at the domain boundary, and Lagrange restriction /
 * prolongation at refinement boundaries (Sec. 3, Sec. 3.1).  With
 * Z4C_BC_USER nothing is written. */
int z4c_fill_ghosts(struct z4c_pack *pack, int32_t reg, void *stream);

/* Z4c right-hand side (Sec. 2; Sec. 4.3 parameters) of state register
 * src_reg at every active zone, written as double to rhs_out (device, the
 * interior layout, 22 fields).  Ghosts of src_reg must already be filled. */
int z4c_rhs(struct z4c_pack *pack, int32_t src_reg, void *rhs_out, void *stream);

/* One classic RK4 stage (stage = 1..4), fused with the RHS and, unless the
 * boundary condition is USER, preceded by the ghost fill of the stage input
 * (where a block's neighbour region in some direction is one block of the
 * same level and size, the stage reads that neighbour's active cells
 * directly and those ghost cells are not written; with outflow boundaries
 * the same holds where the direction's y or z leaves the domain and the
 * remaining components name such a block, or none, the read being clamped
 * to the active range.  Two kinds of ghosts are written by the stage kernel
 * itself, into the register it writes: a same-level neighbour's x-face
 * ghosts for FP32 storage or an odd FP64 ghost depth, and the ghost columns
 * beyond an outflow x face, in the block and in its same-level neighbours
 * across y and z.  The fill of stages 2-4 leaves those alone when the
 * previous call of this function on the pack was the preceding stage, so
 * the input register must then hold what that stage wrote; z4c_fill_ghosts
 * always writes every ghost cell):
 *   1: k1=F(U):  S1 = U + dt/2 k1, A  = U + dt/6 k1
 *   2: k2=F(S1): S2 = U + dt/2 k2, A += dt/3 k2
 *   3: k3=F(S2): S1 = U + dt k3,   A += dt/3 k3
 *   4: k4=F(S1): U  = A + dt/6 k4
 * followed, with Z4C_FLAG_ENFORCE, by det g~ = 1, trace-free A~ and the
 * chi/alpha floors on the written state.  A accumulates in double. */
int z4c_rk4_stage(struct z4c_pack *pack, int32_t stage, double dt, void *stream);

/* nsteps full RK4 steps of U (four stages each).  From the second step of
 * the call on, stage 1's fill also leaves alone the ghosts of U that the
 * previous step's stage 4 wrote.  With Z4C_FLAG_GRAPH and a non-NULL stream,
 * the four stages (ghost fills included) are captured once per (dt, stream)
 * into two hipGraphs, the step for a call's first step and the step for the
 * later ones, and replayed (captured again after a re-bind, a variant or a
 * tracker change).  With
 * Z4C_FLAG_CHECK_FINITE, after the steps every value of U's active cells is
 * checked (one read of U, then the stream is synchronised); Z4C_ENONFINITE
 * if any is NaN or infinite (U is left as computed). */
int z4c_rk4_step(struct z4c_pack *pack, double dt, int32_t nsteps, void *stream);

/* Launch configuration of the fused stage kernel (batching, Sec. 3:
 * MeshBlockPacks exist to cut kernel launches): tile-shape variant
 * (0: 8x8x4, 1: 16x4x4, 2: 8x4x8, 3: 16x8x2 active cells per workgroup)
 * and persistent mode (one grid sized to the resident workgroups, each
 * looping over its XCD's contiguous share of the tiles).  Every variant
 * computes bitwise-identical results.  Z4C_EUNSUPPORTED if the shape does
 * not divide every block.  Synchronises the stream. */
int z4c_set_variant(struct z4c_pack *pack, int32_t variant, int32_t persistent, void *stream);

/* Autotuner: times `reps` RK4 stage-1 launches with dt = 0 (ghost fill
 * included) of every (variant, persistent) pair that fits the pack,
 * times_ms[2*variant + persistent] (host, 8 doubles, -1 where not
 * applicable, nullable), selects the fastest and returns its index in
 * *chosen.  Overwrites S1 and the accumulator, leaves U unchanged (call
 * between RK4 steps).  Synchronises the stream. */
int z4c_autotune(struct z4c_pack *pack, int32_t reps, double *times_ms, int32_t *chosen,
                 void *stream);
/* z4c_autotune with a persistent cache of winners (a text file of JSON
 * lines at `path`, host): a record whose key matches this pack (device
 * architecture, FD order, precision, ghost depth, number of levels, block
 * sizes and their counts) is applied without timing (*from_cache = 1,
 * times_ms all -1); otherwise every variant is timed as by z4c_autotune and
 * the winner appended to the file (*from_cache = 0).  Z4C_EINVAL if the
 * file cannot be written.  from_cache nullable. */
int z4c_autotune_cached(struct z4c_pack *pack, const char *path, int32_t reps, double *times_ms,
                        int32_t *chosen, int32_t *from_cache, void *stream);

/* Constraint monitors in double: Hamiltonian H, momentum M^i, Theta and
 * G^i = Gamma~^i - Gamma~_d^i at every active zone of state register `reg`
 * (ghosts filled first unless USER).  per_zone_out (device, nullable):
 * interior layout with 8 components (H, Mx, My, Mz, Theta, Gx, Gy, Gz).
 * norms_out (host, Z4C_NNORM doubles): H_L2, H_Linf, M_L2, M_Linf,
 * Theta_L2, G_L2, volume-weighted (dV = dx^3) over the zones kept by
 * `region` (nullable: all).  Synchronises the stream. */
int z4c_constraints(struct z4c_pack *pack, int32_t reg, void *per_zone_out,
                    const z4c_norm_region *region, double *norms_out, void *stream);

/* Refinement flags per block (Sec. 3.3): +1 refine, 0 keep, -1 derefine,
 * from per-block reductions over active zones of state register `reg`.
 * flags_out: host int8[nblocks].  Synchronises the stream. */
int z4c_refine_flags(struct z4c_pack *pack, int32_t reg, const z4c_refine_params *rp,
                     int8_t *flags_out, void *stream);

/* ------------------------------------------------------------- regrid */

/* Regrid plan (Sec. 3.3: the refinement criteria drive the mesh; the 2:1
 * rule between neighbouring MeshBlocks).  flags (host, one per block of
 * `pack`, as z4c_refine_flags writes them): +1 refine, -1 derefine, 0 keep.
 * A refined block becomes its eight children (same n, level + 1, corners
 * 2*ilo + n*{0,1}^3), unless it is already at level_max.  Eight leaves
 * flagged -1 that are the aligned children of one parent (same level >= 1
 * and n, ilo = 2*P.ilo + n*{0,1}^3) merge into that parent.  Blocks within
 * reach of each other's ghost stencils (2g cells of the finer one,
 * periodic images included) end at most one level apart: refinement
 * spreads to coarser neighbours, merges that would break the rule are
 * cancelled.  Writes the new blocks (host) in the old order, children in
 * place of their parent (z, y, x order), a merged parent in place of its
 * first child.  *out_n receives the count; Z4C_ENOMEM (nothing written
 * past out_cap) if it exceeds out_cap.  Host only, no stream. */
int z4c_regrid_plan(const struct z4c_pack *pack, const int8_t *flags, int32_t level_max,
                    z4c_block *out_blocks, int32_t out_cap, int32_t *out_n);

/* Regrid transfer (Sec. 3.1, Eqs. 1-2): fills the active cells of state
 * register dst_reg of `dst` (a bound pack of the same parameters whose
 * blocks come from z4c_regrid_plan on `src`'s blocks) from state register
 * src_reg of `src`: a block present in both is copied; a block one level
 * finer than the src block containing it is prolongated from that block
 * (np = g+1 coarse centres nearest each fine centre per axis, the operator
 * of the fine ghost fill, reading the src block's ghosts); a block whose
 * eight children (same n) are src blocks is restricted from them (np fine
 * centres inside the owning child, the window of the coarse ghost fill).
 * Fills the ghosts of src_reg first (src's ghost cells are written).
 * Ghosts of dst_reg are left to the next fill.  Z4C_EINVAL if a dst block
 * is none of the three.  Enqueued on `stream`.  The interpolants are not
 * limited and no enforcement or floor is applied: prolongated through a
 * puncture, chi can come out negative next to it, so a block holding a
 * puncture should not be refined by transfer (set its data instead). */
int z4c_regrid_transfer(struct z4c_pack *src, int32_t src_reg, struct z4c_pack *dst, int32_t dst_reg,
                        void *stream);

/* ---------------------------------------- wave extraction, trackers */

/* Outgoing Weyl scalar (Sec. 3.4 wave extraction) of state register `reg`
 * at every active zone, in the coordinate tetrad about origin[3] (host):
 * from the physical metric gamma_ij = g~_ij / chi and extrinsic curvature
 * K_ij = A~_ij / chi + gamma_ij (Khat + 2 Theta)/3 (derivatives by the
 * centred order-2N stencils and the product rule), E_ij = R_ij - K_ik K^k_j
 * + K K_ij, B_ij = symmetric part of eps_i^kl D_k K_lj; tetrad vectors
 * x - origin, eps(u, x - origin), u = (-y, x, 0) orthonormalised in that
 * order (e_r, e_theta, e_phi), m = (e_theta + i e_phi)/sqrt 2; written is
 * Psi4 = -(E_ij - i B_ij) mbar^i mbar^j (= d2h+/dt2 - i d2hx/dt2 for an
 * outgoing linear wave).  0 where u vanishes (the tetrad's z axis).  out
 * (device): interior layout, 2 components (Re, Im), double.  Fills the
 * ghosts of `reg` first. */
int z4c_psi4(struct z4c_pack *pack, int32_t reg, const double origin[3], void *out, void *stream);

/* Cubic Lagrange interpolation (Sec. 3.4: quantities on extraction spheres,
 * at punctures) of interior-layout double data with ncomp components per
 * zone (device `src`, e.g. z4c_psi4's output) at npts points (device, x y z
 * per point): each point takes the finest block whose active cells contain
 * it and, per axis, the 4 cell centres nearest to it inside that block.
 * out (device): npts x ncomp doubles, NaN for points outside the mesh.
 * npts = 0 does nothing (the pointers may then be NULL). */
int z4c_interp(struct z4c_pack *pack, const void *src, int32_t ncomp, const double *pts, int32_t npts,
               double *out, void *stream);

/* The same for fields first .. first+nfield-1 of state register `reg`
 * (its active cells). */
int z4c_interp_state(struct z4c_pack *pack, int32_t reg, int32_t first, int32_t nfield, const double *pts,
                     int32_t npts, double *out, void *stream);

/* Spin-weight -2 spherical-harmonic decomposition (Sec. 3.4) of complex
 * values (device, Re Im per point) on a quadrature sphere: points (device,
 * npts x 3) with weights (device) about centre[3] (host); for l = 2..lmax
 * (lmax <= 12) and m = -l..l in that order,
 * modes[2q], modes[2q+1] (device) = sum_p w_p v_p conj(-2Y_lm(theta_p, phi_p)),
 * -2Y_22 = sqrt(5/(64 pi)) (1 + cos theta)^2 e^{2 i phi}. */
int z4c_swsh_project(const double *values, const double *pts, const double *weights, int32_t npts,
                     const double centre[3], int32_t lmax, double *modes, void *stream);

/* Puncture trackers (Sec. 3.4): n <= Z4C_MAXTRACK positions (host) advected
 * by dx/dt = -beta(x) with the classic RK4 of the evolution: every RK4 stage
 * of z4c_rk4_stage / z4c_rk4_step first evaluates beta of that stage's input
 * state at x + c_s dt k_(s-1) by z4c_interp_state's interpolation.  Setting
 * replaces the punctures (n = 0 stops tracking) and drops a captured step
 * graph.  Enqueued on `stream`. */
int z4c_tracker_set(struct z4c_pack *pack, int32_t n, const double *pos, void *stream);
/* Current positions (host, 3 per puncture).  Synchronises the stream. */
int z4c_tracker_get(struct z4c_pack *pack, double *pos, void *stream);

/* ----------------------------------------------- learned refinement */
/* The learned indicator predicts, per MeshBlock, the truncation error the
 * chi-based criteria of Sec. 3.3 stand in for, from cheap block features;
 * the plain dchi-max criterion stays as fallback and reference.  Features (16
 * per block, double): 0 max|d chi| 1 mean|d chi| 2 max|d alpha|
 * 3 mean|d alpha| 4 max|dd g~| 5 mean|dd g~| 6 min alpha 7 min chi
 * 8 max|Khat| 9 max|A~| 10 max|Theta| 11 max|Gamma~| 12 max|beta|
 * 13 max|dd chi| 14 max|d Khat| 15 log2 dx, reduced over active zones
 * (centred derivatives of the pack's order; vector and tensor norms
 * Euclidean, |dd f| the largest component). */
#define Z4C_MLP_NPARAM 5313   /* W1[64][16] b1[64] W2[64][64] b2[64] W3[64] b3[1] */

/* Features of state register `reg` (ghosts filled first unless USER) into
 * feat_dev (device double[nblocks*16], nullable) and/or feat_host (host,
 * nullable; synchronises the stream). */
int z4c_features(struct z4c_pack *pack, int32_t reg, void *feat_dev, double *feat_host,
                 void *stream);

/* Injection onto the even sublattice: active cell J of block b of pack_2h's
 * register reg_2h gets active cell 2J of block b of pack_h's register
 * reg_h.  pack_2h must have the same number of blocks, each with n/2 cells
 * and corner ilo/2 at the same level (its cell size 2h, its domain shifted
 * by -h/2 so that its centres are the even fine centres). */
int z4c_pack_inject_2h(struct z4c_pack *pack_h, int32_t reg_h, struct z4c_pack *pack_2h,
                       int32_t reg_2h, void *stream);

/* Truncation-error labels: y_b = log10(sqrt(mean over the active cells J of
 * block b of pack_2h and the 22 fields of (rhs_h(2J) - rhs_2h(J))^2) + 1e-30)
 * from two z4c_rhs outputs (device, interior layout).  labels_out: host
 * double[nblocks].  Synchronises the stream. */
int z4c_labels(struct z4c_pack *pack_h, const void *rhs_h, struct z4c_pack *pack_2h,
               const void *rhs_2h, double *labels_out, void *stream);

/* phi(raw) statistics over a batch of B feature rows (device double
 * raw[B*16]; phi = log10(|x| + 1e-12) for features 0..14, identity for 15):
 * stats (device double[64]) = mean[16], std[16], min[16], max[16]. */
int z4c_feature_stats(const void *raw, int32_t B, void *stats, void *stream);
/* Network inputs X[b][k] = (phi(raw[b][k]) - mean[k]) / std[k] (device float). */
int z4c_mlp_normalize(const void *raw, int32_t B, const void *stats, void *X, void *stream);

/* 16 -> 64 -> 64 -> 1 perceptron, ReLU hidden layers, linear output.
 * Inputs, weights and hidden activations are rounded to bfloat16 (nearest
 * even); sums accumulate in float32.  params: device float[Z4C_MLP_NPARAM]
 * (float32 master weights).  X: device float[B*16]; Y: device float[B];
 * cache (nullable for inference): device float[B*128] pre-activations. */
int z4c_mlp_forward(const void *params, const void *X, int32_t B, void *Y, void *cache,
                    void *stream);
/* Gradient of the mean squared error (Y from z4c_mlp_forward with cache,
 * targets T device float[B]) with respect to the master weights (through
 * the rounding as identity): grad device float[Z4C_MLP_NPARAM]; loss device
 * float[1] (nullable); work device float[Z4C_MLP_WORK(B)]: per-sample deltas
 * (129 per sample), then partial sums of the gradient over slices of
 * Z4C_MLP_SLICE samples, reduced in slice order (deterministic). */
#define Z4C_MLP_SLICE 64
#define Z4C_MLP_WORK(B) ((int64_t)(B) * 129 + (((int64_t)(B) + Z4C_MLP_SLICE - 1) / Z4C_MLP_SLICE) * Z4C_MLP_NPARAM)
int z4c_mlp_backward(const void *params, const void *X, const void *Y, const void *T,
                     const void *cache, int32_t B, void *grad, void *loss, void *work,
                     void *stream);
/* z4c_mlp_backward without the work argument, for callers that cannot
 * allocate device memory (code under hipGraph capture, serving loops,
 * harnesses that forbid hipMalloc): the work buffer is a library-owned
 * device array of Z4C_MLP_WORK(Z4C_MLP_NOALLOC_MAXB) floats (3.5 MB), one
 * per GPU, kept until the process ends; the call itself allocates nothing.
 * B > Z4C_MLP_NOALLOC_MAXB returns Z4C_EINVAL.  Every call on one GPU uses
 * that GPU's array: calls that overlap on one GPU (other streams, other
 * threads) race and must be ordered by the caller.  Same kernels and
 * results as z4c_mlp_backward. */
#define Z4C_MLP_NOALLOC_MAXB 4096
int z4c_mlp_backward_noalloc(const void *params, const void *X, const void *Y, const void *T,
                             const void *cache, int32_t B, void *grad, void *loss, void *stream);
/* One Adam step (step counts from 1) on params with moments m, v (device
 * float[Z4C_MLP_NPARAM] each). */
int z4c_mlp_adam(void *params, const void *grad, void *m, void *v, int32_t step, float lr,
                 float beta1, float beta2, float eps, void *stream);

typedef struct {
    const void *params;    /* device float[Z4C_MLP_NPARAM]                    */
    const void *stats;     /* device double[64] from z4c_feature_stats        */
    const double *range;   /* host double[32]: phi min[16], max[16] of training */
    double tau_ref;        /* predicted log10 error above which to refine     */
    double tau_deref;      /* ... below which to derefine                     */
    double chi_thr;        /* chi-min safety: min chi < chi_thr forces +1     */
    double dchi_thr;       /* dchi-max threshold of the fallback              */
    int32_t level_max;
    int32_t pad;
} z4c_mlp_model;

/* Learned refinement flags: features -> network -> +1 if prediction >
 * tau_ref, -1 if < tau_deref, else 0; min chi < chi_thr forces +1; a block
 * whose features are non-finite or outside the training range widened by
 * 10% takes the dchi-max flag instead (fallback_out[b] = 1, nullable).
 * Level limits as z4c_refine_flags.  Synchronises the stream. */
int z4c_refine_flags_learned(struct z4c_pack *pack, int32_t reg, const z4c_mlp_model *model,
                             int8_t *flags_out, int8_t *fallback_out, void *stream);

/* Kernel timing for benchmarks.  With enable = 1, every later stage-kernel
 * and ghost-fill launch on this pack is bracketed by a pair of HIP events
 * recorded on the launch stream; z4c_profile_read waits for them and
 * returns out[0] total stage-kernel milliseconds, out[1] stage launches,
 * out[2] ghost-fill milliseconds, out[3] fill launches, out[4] captured-step
 * (hipGraph) milliseconds, out[5] graph launches (reset != 0 clears the
 * totals).  Events are host-side HIP objects; no device memory. */
int z4c_profile(struct z4c_pack *pack, int32_t enable);
int z4c_profile_read(struct z4c_pack *pack, double *out, int32_t reset);

/* Finite-difference weights the kernels use (for inspection): centred first
 * derivative (N+1 values, k = 0..N), centred second derivative (N+1 values),
 * lopsided (+) first derivative on -(N-1)..N+1 (2N+1 values).  Host only. */
int z4c_stencil_weights(int32_t fd_order, double *d1, double *d2, double *lop);

#ifdef __cplusplus
}
#endif
#endif
