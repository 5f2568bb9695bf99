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
    ParamsDev P;
    double dt;
    int32_t stage;            // 1..4, 0 = RHS only
    int32_t g;
};

struct FillArgs {
    void* reg;
    const BlockDev* blocks;
    const int32_t* map;       // lookup map (all levels)
    LookupDev L;
    int32_t g, bc;
    int32_t nroot[3];
    int32_t maxghost;         // ghost cells of the largest block
};

struct XlevelArgs {
    void* reg;                // register being filled
    void* shadow;             // shadow boxes (same element type)
    const BlockDev* blocks;
    const XferItem* xfer;
    const ProlongItem* prol;
    const double* rw;         // restriction weights [8][8]: set d, point q
    const double* pw;         // prolongation weights [2][8]: parity, point q
    int64_t nxfer, nprol;
    int32_t npts;             // g + 1
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

hipError_t launch_stage(int N, int prec, const StageArgs& a, int nwork, hipStream_t s);
hipError_t launch_fill(int prec, const FillArgs& a, int nblocks, hipStream_t s);
hipError_t launch_diag(int N, int prec, const DiagArgs& a, int nwork, hipStream_t s);
hipError_t launch_xlevel(int prec, const XlevelArgs& a, hipStream_t s);

}  // namespace z4c
