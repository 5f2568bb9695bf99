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

// physics / method parameters as the kernels read them
struct ParamsDev {
    double ko_sigma, kappa1, kappa2, eta, mu_S, chi_floor, alpha_floor;
    uint32_t terms;
    int32_t enforce;
};

}  // namespace z4c
