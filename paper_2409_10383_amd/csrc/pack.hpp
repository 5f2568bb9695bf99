// Host-side state of a MeshBlockPack (struct z4c_pack of the C ABI) and the
// helpers the host runtime's translation units share.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/z4c.h"
#include "kernels.hpp"

using namespace z4c;

struct z4c_pack {
    z4c_params p;
    std::vector<z4c_block> blk;
    std::vector<BlockDev> bdev;
    std::vector<WorkItem> work;
    std::vector<int32_t> map;
    LookupDev L;
    bool multilevel = false;
    // cross-level fill tables
    std::vector<XferItem> xfer;       // copies from active cells first, then from images
    int64_t nxfer_direct = 0;         // of which from active cells
    // the stage path's fill stops at these counts: the items after them write
    // ghosts of directions the stage kernel reads in place or never reads
    int64_t nxfer_stage = 0, nprol_stage = 0, npgrp_stage = 0;
    std::vector<ProlongItem> prol;
    std::vector<ProlongGroup> pgrp;   // parents by four (y and z, FP64), by two (y), then single
    int64_t nparent = 0;              // coarse parents of grouped prolongations
    std::vector<ImageSlice> islice;
    std::vector<RegridDesc> regrid_desc;  // last regrid into this pack (kept for the upload)
    std::vector<int64_t> img_off;     // per block: offset of its coarse image, -1 if none
    std::vector<int32_t> img_fstride;
    int64_t image_elems = 0;
    std::vector<double> rw, pw, wtab;
    int64_t shadow_elems = 0;
    size_t ws_xfer = 0, ws_prol = 0, ws_pgrp = 0, ws_islice = 0, ws_w = 0, ws_shadow = 0, ws_image = 0;
    size_t ws_regrid = 0, ws_vnbr = 0, ws_vmask = 0;
    std::vector<int64_t> vnbr;    // virtual halos: 27 offsets per block
    std::vector<uint32_t> vmask;  // directions the stage path's fill skips, per block
    std::vector<uint32_t> cmask;  // of those, per block the directions read with y (2 b) and z (2 b + 1) clamped
    size_t ws_cmask = 0;
    int virt_x = 1;               // 1: directions with dx != 0 are read in place too
    std::vector<uint32_t> pmask;  // per block, x directions whose ghosts the stage kernel pushes
    size_t ws_pmask = 0;
    std::vector<uint32_t> omask;  // per block, outflow x faces whose ghost columns the stage kernel writes
    size_t ws_omask = 0;
    std::vector<uint32_t> fskip;  // per block, directions written by the previous stage kernel
    size_t ws_fskip = 0;
    bool fill_pushed_empty = false;   // after a stage, the same-level fill has nothing left to do
    int last_stage = 0;           // last RK stage run on the pack (0: none, or other work since)
    // puncture tracker: device state (x, k_prev, acc) per puncture in the workspace
    int ntrack = 0;
    size_t ws_track = 0;
    size_t ws_flag = 0;       // finite-value check flag (int32)
    std::vector<double> track_host;
    size_t ws_first = 0, ws_feat = 0, ws_x = 0, ws_y = 0, ws_lflag = 0;
    std::vector<int32_t> first_work;
    int maxghost = 0;
    int64_t zones = 0;
    size_t reg_bytes[Z4C_NREG] = {0, 0, 0, 0};
    // workspace carve-up (byte offsets)
    size_t ws_blocks = 0, ws_work = 0, ws_map = 0, ws_part = 0, ws_total = 0;
    // bound memory
    bool bound = false;
    void* reg[Z4C_NREG] = {nullptr, nullptr, nullptr, nullptr};
    char* ws = nullptr;
    std::vector<double> part_host;
    std::string err;
    // stage-kernel variant (tile shape) and launch mode
    int variant = 0;
    bool persistent = false;
    int grid_persistent = 0;
    // captured RK4 step (hipGraph), valid for one (dt, stream); graph2: the
    // same step for the second and later steps of a call (its stage 1 finds
    // the ghosts the previous step's stage 4 wrote)
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph2 = nullptr;
    hipGraphExec_t gexec2 = nullptr;
    double graph_dt = 0.0;
    hipStream_t graph_stream = nullptr;
    // multi-level packs: the same-level fill runs on a side stream beside the
    // cross-level chain (fork and join through events on the caller's stream)
    hipStream_t side = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    // optional kernel timing
    bool prof = false;
    struct EvPair { hipEvent_t a, b; int kind; };
    std::vector<EvPair> ev;
    double prof_acc[6] = {0, 0, 0, 0, 0, 0};
};

// drop the captured step graphs (their kernel arguments hold the registers,
// workspace, launch variant and tracker count they were captured with)
inline void drop_graphs(z4c_pack* pk)
{
    if (pk->gexec) { (void)hipGraphExecDestroy(pk->gexec); pk->gexec = nullptr; }
    if (pk->graph) { (void)hipGraphDestroy(pk->graph); pk->graph = nullptr; }
    if (pk->gexec2) { (void)hipGraphExecDestroy(pk->gexec2); pk->gexec2 = nullptr; }
    if (pk->graph2) { (void)hipGraphDestroy(pk->graph2); pk->graph2 = nullptr; }
}


namespace z4c_host {

// record a message on the pack and return `code`
int fail(z4c_pack* pk, int code, const char* fmt, ...);
hipStream_t as_stream(void* s);
// floor division
int64_t floor_div(int64_t a, int64_t b);
// Lagrange weights of the nodes q + 1/2, q = 0..n-1, at t
void lagrange_half(int n, double t, double* w);
// RK4 stage `stage` of the puncture tracker (no-op without punctures)
hipError_t track_stage(z4c_pack* pk, int stage, int reg, double dt, hipStream_t s);

}  // namespace z4c_host
