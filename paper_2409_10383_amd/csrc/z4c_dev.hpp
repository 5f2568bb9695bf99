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
// Restriction: the value of coarse cell K restricted from fine block F (the
// leaf that owns fine cell 2K) is a Lagrange interpolation (n = g+1 points
// per axis) over a window of F's active cells that depends only on K's
// position inside F.  Each fill first restricts every source block as a
// whole into its coarse image; a transfer then copies 22 values, from an
// active cell or an image cell, into a ghost cell of a register or into a
// block's coarse shadow box.
struct XferItem {
    int64_t dst;          // element offset of field 0 at the destination
    int64_t src;          // element offset of field 0 at the source
    int32_t dst_stride;   // element stride between fields at the destination
    int32_t src_stride;   // element stride between fields at the source
    int32_t kind;         // bit0: source is a coarse image; bit1: destination is a shadow box
    int32_t pad;
};
// One workgroup of the image restriction: coarse cells x0 .. x0+nx-1 of
// rows y0 .. y0+ny-1 of the coarse z-planes kz .. kz+nkz-1 of block `block`.
struct ImageSlice {
    int64_t img;          // element offset of the block's image (field 0)
    int32_t block;
    int32_t fstride;      // field stride of the image (elements)
    int16_t kz, nkz, y0, ny, x0, nx, pad[2];
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
    int32_t mask;         // bit (cz*4 + cy*2 + cx): child is a ghost to fill; bits 8-15
                          // the same for the parent one coarse cell further in y, and
                          // bits 16-23, 24-31 for those further in z, in y and z
    int32_t fstride;      // field stride of the shadow box (elements)
};

// How a block of a regridded pack gets its active data from the old pack:
// kind 0 copy of block src[0] (same geometry), 1 prolongation from the
// coarser block src[0] that contains it, 2 restriction from its eight
// children src[cz*4 + cy*2 + cx] (same cell count).
struct RegridDesc {
    int32_t kind;
    int32_t src[8];
    int32_t pad;
};

// physics / method parameters as the kernels read them
struct ParamsDev {
    double ko_sigma, kappa1, kappa2, eta, mu_S, chi_floor, alpha_floor;
    uint32_t terms;
    int32_t enforce;
};

}  // namespace z4c
