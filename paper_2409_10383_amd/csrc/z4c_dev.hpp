// Device-side data structures shared by the host runtime and the kernels of
// libz4c.  The layout of registers is described in include/z4c.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace z4c {

constexpr int NF = 22;

// field indices
enum : int {
    F_CHI = 0, F_GXX, F_GXY, F_GXZ, F_GYY, F_GYZ, F_GZZ, F_KH,
    F_AXX, F_AXY, F_AXZ, F_AYY, F_AYZ, F_AZZ, F_GAMX, F_GAMY, F_GAMZ,
    F_TH, F_ALPHA, F_BETAX, F_BETAY, F_BETAZ
};

// one MeshBlock as the kernels see it
struct BlockDev {
    int64_t off;      // element offset in a state register
    int64_t ioff;     // element offset in the interior layout (A, RHS)
    int64_t slab;     // elements per field in a state register (padded)
    int32_t n, E;     // active cells per axis, cells per axis with ghosts
    int32_t level, pad;
    int32_t ilo[3];
    int32_t pad2;
    double h;         // cell size
    double x0[3];     // centre of active cell (0,0,0)
};

// one tile of the fused stage kernel: a box of active cells in one block
struct WorkItem {
    int32_t block;
    int16_t i0, j0, k0;   // tile origin (active-cell indices)
    int16_t ni, nj, nk;   // tile extent
};

// lookup from a unit cell of a level to the leaf block covering it
struct LookupDev {
    int32_t unit;         // cells per lookup unit (gcd of sizes/corners)
    int32_t nlev;
    int32_t dim[8][3];    // per level: units per axis
    int64_t base[8];      // per level: start in `map`
};

// cross-level ghost fill (refinement boundaries)
// A transfer writes 22 values: a copy of one active cell, or the Lagrange
// restriction (n = g+1 points per axis) of a window of fine active cells,
// into a ghost cell of a register or into a block's coarse shadow box.
struct XferItem {
    int64_t dst;          // element offset of field 0 at the destination
    int64_t dst_stride;   // element stride between fields at the destination
    int64_t src;          // element offset (field 0) of the source cell / window origin
    int32_t src_block;    // source block (field stride and row length)
    uint8_t kind;         // bit0: restriction (else copy); bit1: destination is a shadow box
    uint8_t d[3];         // per-axis restriction weight set
};
// A prolongation fills one fine ghost cell from the (g+1)^3 coarse values
// of its block's shadow box.
struct ProlongItem {
    int64_t dst;          // register element offset of field 0
    int64_t sh;           // shadow element offset of the stencil origin (field 0)
    int32_t block;        // destination block (field stride)
    int32_t se;           // shadow box extent per axis
    int32_t parity;       // bit a: fine index along axis a is odd
    int32_t pad;          // field stride of the shadow box (elements)
};

// Prolongation of the (up to) 8 fine ghost children of one coarse parent:
// they share the union of their stencils, (g+2)^3 coarse values for even
// g+1 (the two parities' windows differ by one cell), (g+1)^3 for odd.
struct ProlongGroup {
    int64_t dst;          // register element offset of child (0,0,0), field 0
    int64_t sh;           // shadow element offset of the union stencil origin
    int32_t block;        // destination block (field stride, row length)
    int32_t se;           // shadow box extent per axis
    int32_t mask;         // bit (cz*4 + cy*2 + cx): child is a ghost to fill
    int32_t fstride;      // field stride of the shadow box (elements)
};

// physics / method parameters as the kernels read them
struct ParamsDev {
    double ko_sigma, kappa1, kappa2, eta, mu_S, chi_floor, alpha_floor;
    uint32_t terms;
    int32_t enforce;
};

}  // namespace z4c
