// Launch interfaces of the libz4c kernels (host side).
#pragma once
#include <hip/hip_runtime.h>
#include "z4c_dev.hpp"

namespace z4c {

struct StageArgs {
    const void* src;          // stage input (ghosted state register)
    const void* U;            // step state (ghosted)
    void* dst;                // stage output (ghosted state register)
    double* A;                // accumulator (interior layout)
    double* rhs_out;          // z4c_rhs only (interior layout)
    const BlockDev* blocks;
    const WorkItem* work;
    const int64_t* vnbr;      // per block, 27 direction offsets of the staged halo
    const uint32_t* cmask;    // per block (2 b, 2 b + 1), directions read with y, z clamped (outflow)
    const uint32_t* pmask;    // per block, x directions pushed to a same-level neighbour
    const uint32_t* omask;    // per block, outflow x faces pushed: bits 0, 1 low / high x face;
                              // 2-5 low / high y, z faces on the domain face; 8 + e: target
                              // block across (0, e % 3 - 1, e / 3 - 1) (e = 4: the block itself)
    int32_t virt_x;           // 0: a staged cell's halo direction ignores x
    ParamsDev P;
    double dt;
    int32_t stage;            // 1..4, 0 = RHS only
    int32_t g;
    int32_t nwork;            // work items
    int32_t persistent;       // 1: grid smaller than nwork, workgroups loop
};

constexpr int NVARIANT = 4;
extern const int TILE_SHAPES[NVARIANT][3];

struct FillArgs {
    void* reg;
    const BlockDev* blocks;
    const int32_t* map;       // lookup map (all levels)
    LookupDev L;
    int32_t g, bc;
    int32_t nroot[3];
    int32_t maxghost;         // ghost cells of the largest block
    const uint32_t* skip;     // per block, directions left alone (virtual halos); null = none
    const uint32_t* skip2;    // per block, further directions left alone (written by the
                              // stage kernel that produced the register); null = none
};

// Restriction window of coarse cell kc (0 <= kc < n/2) inside a fine block
// of n active cells per axis: first fine cell o of the np-point window and
// the weight set d (evaluation point at the fine face o + d).  Centred where
// it fits; for odd np the extra point goes towards the block's interior;
// clamped to the block's active cells.
// Workgroup slot -> work index for a 1-D launch of xcd_grid(nwork) slots:
// slot b runs on XCD b % 8 (each XCD has its own L2), so that XCD receives
// the contiguous run x*per .. x*per+per-1 of the work list and neighbouring
// items, which read overlapping source lines, share one L2.  Indices >= nwork
// are padding slots and do nothing.
__device__ __forceinline__ int64_t xcd_run(int64_t slot, int64_t nwork)
{
    const int64_t per = (nwork + 7) / 8;
    return (slot % 8) * per + slot / 8;
}
inline unsigned xcd_grid(int64_t nwork) { return (unsigned)((nwork + 7) / 8 * 8); }

__device__ __forceinline__ void rwin(int kc, int n, int np, int& o, int& d)
{
    const int c = 2 * kc;
    int st = (np % 2 == 0) ? c - np / 2 + 1 : ((2 * kc + 1 < n / 2) ? c - (np - 1) / 2 + 1 : c - (np - 1) / 2);
    st = st < 0 ? 0 : st;
    st = st + np > n ? n - np : st;
    o = st;
    d = c + 1 - st;
}

// LDS budget of the image restriction (doubles): x-pass and y-pass partials
constexpr int RI_XMAX = 2048, RI_YMAX = 1536;

struct XlevelArgs {
    void* reg;                // register being filled
    void* shadow;             // shadow boxes (same element type)
    void* image;              // coarse images of restriction sources (same element type)
    const ImageSlice* islice;
    const BlockDev* blocks;
    const XferItem* xfer;
    const ProlongItem* prol;
    const ProlongGroup* pgrp;
    const double* rw;         // restriction weights [8][8]: set d, point q
    const double* pw;         // prolongation weights [2][8]: parity, point q
    int64_t nxfer, nprol, npgrp, nislice;
    int32_t npts;             // g + 1
};

// Regrid transfer: active cells of the destination pack's register from
// the source pack's (ghost-filled) register
struct RegridArgs {
    const void* src;          // source register
    void* dst;                // destination register
    const BlockDev* sblocks;  // source block table
    const BlockDev* dblocks;  // destination block table
    const RegridDesc* desc;   // per destination block
    int32_t g, npts;
    double rw[64];            // restriction weights [set d][point]
    double pw[16];            // prolongation weights [parity][point]
};

struct DiagArgs {
    const void* src;
    double* per_zone;         // nullable
    double* partial;          // [nwork][8]
    const BlockDev* blocks;
    const WorkItem* work;
    ParamsDev P;
    double lo[3];
    int32_t ncentres;
    int32_t mode;             // 0 constraints, 1 flag reductions
    double centres[8][3];
    double r_exc;
    int32_t g;
};

// finite-value check of a state register's active cells
struct FiniteArgs {
    const void* src;
    const BlockDev* blocks;
    const WorkItem* work;
    int32_t* flag;            // set to 1 where a value is not finite
    int32_t g;
};

struct FeatArgs {
    const void* src;
    const BlockDev* blocks;
    const WorkItem* work;
    const int32_t* first_work;  // [nblocks + 1]: first work item of each block
    double* partial;            // [nwork][16]
    double* feat;               // [nblocks][16]
    int32_t g, nblocks;
};

struct InjectArgs {
    const void* src;            // h-pack register
    void* dst;                  // 2h-pack register
    const BlockDev* blocks1;    // h pack
    const BlockDev* blocks2;    // 2h pack
    int32_t g1, g2;
};

struct LabelArgs {
    const double* rhs1;         // h-pack RHS (interior layout)
    const double* rhs2;         // 2h-pack RHS
    const BlockDev* blocks1;
    const BlockDev* blocks2;
    const WorkItem* work2;
    double* partial;            // [nwork2]
};

hipError_t launch_features(int N, int prec, const FeatArgs& a, int nwork, hipStream_t s);
hipError_t launch_inject(int prec, const InjectArgs& a, int nblocks, int maxcells, hipStream_t s);
hipError_t launch_labels(const LabelArgs& a, int nwork2, hipStream_t s);
hipError_t launch_mlp_forward(const float* P, const float* X, int B, float* Y, float* cache, hipStream_t s);
hipError_t launch_mlp_backward(const float* P, const float* X, const float* Y, const float* T,
                               const float* cache, int B, float* G, float* loss, float* work, hipStream_t s);
hipError_t launch_mlp_adam(float* P, const float* G, float* M, float* V, int step, float lr, float b1,
                           float b2, float eps, hipStream_t s);
hipError_t launch_normalize(const double* raw, int B, const double* stats, float* X, hipStream_t s);
// the rules of the learned refinement flags (training range of phi per
// feature, thresholds, level limit)
struct LearnedRule {
    double lo[16], hi[16];
    double tau_ref, tau_deref, chi_thr, dchi_thr;
    int32_t level_max, pad;
};
hipError_t launch_learned_flags(const double* feat, const float* Y, const BlockDev* blocks, int nb,
                                const LearnedRule& r, int8_t* flags, int8_t* fallback, hipStream_t s);
hipError_t launch_feat_stats(const double* raw, int B, double* stats, hipStream_t s);

hipError_t launch_stage(int N, int prec, int variant, const StageArgs& a, int grid, hipStream_t s);
int stage_occupancy(int N, int prec, int variant);
hipError_t launch_fill(int prec, const FillArgs& a, int nblocks, hipStream_t s);
hipError_t launch_diag(int N, int prec, const DiagArgs& a, int nwork, hipStream_t s);
hipError_t launch_check_finite(int prec, const FiniteArgs& a, int nwork, hipStream_t s);
// phases of the cross-level fill, in this order: restriction of the images,
// copies a.xfer[0 .. a.nxfer), prolongation
enum : int { XL_RESTRICT = 1, XL_XFER = 2, XL_PROLONG = 4 };
hipError_t launch_xlevel(int prec, const XlevelArgs& a, hipStream_t s, int phases);
hipError_t launch_regrid(int prec, const RegridArgs& a, int nblocks, int maxn, hipStream_t s);

}  // namespace z4c
