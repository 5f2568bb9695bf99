// Adaptive regrid of a MeshBlockPack (Sec. 3.3: refinement criteria drive
// the mesh; the 2:1 rule between neighbours, Sec. 3).  The plan turns
// per-block flags into a new list of octree leaves: a refined block becomes
// its eight children (same cell count, one level finer), eight flagged
// sibling leaves merge into their parent; refinement spreads to coarser
// neighbours and merges are cancelled wherever the 2:1 rule would break.
// The transfer fills the active cells of a register of the new pack from
// the old one: copies where a block is unchanged, Lagrange prolongation
// (n = g+1 coarse points per axis, the fine ghosts' operator) into refined
// blocks, Lagrange restriction (the coarse ghosts' window) into merged ones
// (Sec. 3.1, Eqs. 1-2).
#include <algorithm>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>

#include "pack.hpp"

namespace z4c {

// one thread per active cell of a destination block (blockIdx.y)
template <class T, int NP>
__global__ __launch_bounds__(256) void k_regrid(const RegridArgs a)
{
    const BlockDev D = a.dblocks[blockIdx.y];
    const int n = D.n, g = a.g, np = NP ? NP : a.npts;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)n * n * n) return;
    const int i = (int)(q % n), j = (int)((q / n) % n), k = (int)(q / ((int64_t)n * n));
    const int G[3] = {D.ilo[0] + i, D.ilo[1] + j, D.ilo[2] + k};
    const RegridDesc ds = a.desc[blockIdx.y];
    T* dst = (T*)a.dst + D.off + ((int64_t)(k + g) * D.E + (j + g)) * D.E + (i + g);
    const T* __restrict__ src = (const T*)a.src;
    if (ds.kind == 0) {
        const BlockDev S = a.sblocks[ds.src[0]];
        const T* p = src + S.off + ((int64_t)(G[2] - S.ilo[2] + g) * S.E + (G[1] - S.ilo[1] + g)) * S.E +
                     (G[0] - S.ilo[0] + g);
#pragma unroll
        for (int f = 0; f < NF; ++f) dst[(int64_t)f * D.slab] = p[(int64_t)f * S.slab];
        return;
    }
    int o[3];
    const double* w[3];
    const T* p;
    BlockDev S;
    if (ds.kind == 1) {
        // fine cell G of the parent cell G >> 1: stencil of the np coarse
        // centres nearest the fine centre, in the parent's ghosted data
        S = a.sblocks[ds.src[0]];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int J = G[d] >> 1, par = G[d] & 1;
            const int s0 = (np % 2) ? J - (np - 1) / 2 : (par ? J - np / 2 + 1 : J - np / 2);
            o[d] = s0 - S.ilo[d] + g;
            w[d] = a.pw + 8 * par;
        }
    } else {
        // coarse cell G from the child block owning fine cell 2G
        const int cx = (2 * (G[0] - D.ilo[0])) / n, cy = (2 * (G[1] - D.ilo[1])) / n,
                  cz = (2 * (G[2] - D.ilo[2])) / n;
        S = a.sblocks[ds.src[cz * 4 + cy * 2 + cx]];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            int ow, dw;
            rwin(G[d] - S.ilo[d] / 2, S.n, np, ow, dw);
            o[d] = ow + g;
            w[d] = a.rw + 8 * dw;
        }
    }
    p = src + S.off + ((int64_t)o[2] * S.E + o[1]) * S.E + o[0];
    for (int f = 0; f < NF; ++f) {
        const T* pf = p + (int64_t)f * S.slab;
        double acc = 0.0;
#pragma unroll 1
        for (int kz = 0; kz < np; ++kz) {
            double az = 0.0;
#pragma unroll
            for (int jy = 0; jy < np; ++jy) {
                const T* row = pf + ((int64_t)kz * S.E + jy) * S.E;
                double ay = 0.0;
#pragma unroll
                for (int ix = 0; ix < np; ++ix) ay += w[0][ix] * (double)row[ix];
                az += w[1][jy] * ay;
            }
            acc += w[2][kz] * az;
        }
        dst[(int64_t)f * D.slab] = (T)acc;
    }
}

template <class T>
static void launch_regrid_t(const RegridArgs& a, dim3 grid, hipStream_t s)
{
    switch (a.npts) {
    case 4: hipLaunchKernelGGL((k_regrid<T, 4>), grid, dim3(256), 0, s, a); break;
    case 5: hipLaunchKernelGGL((k_regrid<T, 5>), grid, dim3(256), 0, s, a); break;
    case 6: hipLaunchKernelGGL((k_regrid<T, 6>), grid, dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((k_regrid<T, 0>), grid, dim3(256), 0, s, a); break;
    }
}

hipError_t launch_regrid(int prec, const RegridArgs& a, int nblocks, int maxn, hipStream_t s)
{
    const int64_t cells = (int64_t)maxn * maxn * maxn;
    const dim3 grid((unsigned)((cells + 255) / 256), (unsigned)nblocks);
    if (prec == 0) launch_regrid_t<double>(a, grid, s);
    else launch_regrid_t<float>(a, grid, s);
    return hipGetLastError();
}

}  // namespace z4c

using namespace z4c_host;

namespace {

// Blocks within the reach of each other's ghost stencils (the finer one's
// 2g cells), periodic images included: the pairs the 2:1 rule constrains.
struct Near {
    const z4c_params* p;
    int F;                         // finest level of the comparison units
    bool operator()(const z4c_block& a, int la, const z4c_block& b, int lb) const
    {
        const int64_t sa = int64_t(1) << (F - a.level), sb = int64_t(1) << (F - b.level);
        const int lf = std::max(la, lb);
        const int64_t reach = (int64_t)2 * p->nghost * (int64_t(1) << (F - lf));
        for (int d = 0; d < 3; ++d) {
            const int64_t a0 = a.ilo[d] * sa, a1 = (a.ilo[d] + a.n) * sa;
            const int64_t b0 = b.ilo[d] * sb, b1 = (b.ilo[d] + b.n) * sb;
            const int64_t N = (int64_t)p->nroot[d] << F;
            bool hit = false;
            const int nimg = p->bc == Z4C_BC_PERIODIC ? 1 : 0;
            for (int m = -nimg; m <= nimg && !hit; ++m)
                hit = (a0 - reach < b1 + m * N) && (b0 + m * N < a1 + reach);
            if (!hit) return false;
        }
        return true;
    }
};

}  // namespace

extern "C" {

int z4c_regrid_plan(const z4c_pack* pk, const int8_t* flags, int32_t level_max, z4c_block* out,
                    int32_t out_cap, int32_t* out_n)
{
    if (!pk || !flags || !out_n || out_cap < 0 || (out_cap > 0 && !out)) return Z4C_EINVAL;
    if (level_max < 0 || level_max > 7) return Z4C_EINVAL;
    const std::vector<z4c_block>& B = pk->blk;
    const int nb = (int)B.size();
    std::vector<int> t(nb);
    int F = 0;
    for (int b = 0; b < nb; ++b) {
        if (flags[b] < -1 || flags[b] > 1) return Z4C_EINVAL;
        t[b] = B[b].level + ((flags[b] > 0 && B[b].level < level_max) ? 1 : 0);
        F = std::max(F, t[b]);
    }
    const Near near{&pk->p, F};
    // refinement: a block two levels coarser than a near target refines too
    for (bool changed = true; changed;) {
        changed = false;
        for (int b = 0; b < nb; ++b)
            for (int c = 0; c < nb; ++c)
                if (c != b && t[b] > t[c] + 1 && near(B[b], t[b], B[c], t[c])) {
                    t[c] = t[b] - 1;
                    changed = true;
                }
    }
    for (int b = 0; b < nb; ++b)
        if (t[b] > B[b].level + 1 || t[b] > 7) return Z4C_EINVAL;  // input mesh broke the 2:1 rule
    // merges: eight aligned same-size leaves of one level, all flagged -1
    std::map<std::tuple<int, int, int, int, int>, std::vector<int>> groups;
    for (int b = 0; b < nb; ++b) {
        const z4c_block& q = B[b];
        if (flags[b] >= 0 || t[b] != q.level || q.level < 1) continue;
        if (q.ilo[0] % q.n || q.ilo[1] % q.n || q.ilo[2] % q.n) continue;
        const int m = 2 * q.n;
        groups[std::make_tuple(q.level, q.n, q.ilo[0] / m, q.ilo[1] / m, q.ilo[2] / m)].push_back(b);
    }
    std::vector<int> gid(nb, -1);
    std::vector<std::vector<int>> merge;
    std::vector<z4c_block> parent;
    for (auto& kv : groups) {
        if (kv.second.size() != 8) continue;
        const z4c_block& q = B[kv.second[0]];
        z4c_block P;
        P.level = q.level - 1;
        P.n = q.n;
        P.ilo[0] = std::get<2>(kv.first) * q.n;
        P.ilo[1] = std::get<3>(kv.first) * q.n;
        P.ilo[2] = std::get<4>(kv.first) * q.n;
        for (int b : kv.second) gid[b] = (int)merge.size();
        merge.push_back(kv.second);
        parent.push_back(P);
    }
    std::vector<char> live(merge.size(), 1);
    for (size_t m = 0; m < merge.size(); ++m)
        for (int b : merge[m]) t[b] = B[b].level - 1;
    // cancel merges whose parent would sit two levels below a near block
    for (bool changed = true; changed;) {
        changed = false;
        for (size_t m = 0; m < merge.size(); ++m) {
            if (!live[m]) continue;
            const int lp = parent[m].level;
            for (int c = 0; c < nb && live[m]; ++c) {
                if (gid[c] == (int)m) continue;
                if (t[c] > lp + 1 && near(parent[m], lp, B[c], t[c])) {
                    live[m] = 0;
                    for (int b : merge[m]) t[b] = B[b].level;
                    changed = true;
                }
            }
        }
    }
    // emit: children in place of a refined block, the parent in place of a
    // merged group's first member
    int64_t cnt = 0;
    for (int b = 0; b < nb; ++b) {
        if (gid[b] >= 0 && live[gid[b]]) cnt += (merge[gid[b]][0] == b) ? 1 : 0;
        else cnt += (t[b] > B[b].level) ? 8 : 1;
    }
    *out_n = (int32_t)cnt;
    if (cnt > out_cap) return Z4C_ENOMEM;
    int64_t o = 0;
    for (int b = 0; b < nb; ++b) {
        const z4c_block& q = B[b];
        if (gid[b] >= 0 && live[gid[b]]) {
            if (merge[gid[b]][0] == b) out[o++] = parent[gid[b]];
        } else if (t[b] > q.level) {
            for (int cz = 0; cz < 2; ++cz)
                for (int cy = 0; cy < 2; ++cy)
                    for (int cx = 0; cx < 2; ++cx) {
                        z4c_block c;
                        c.level = q.level + 1;
                        c.n = q.n;
                        c.ilo[0] = 2 * q.ilo[0] + cx * q.n;
                        c.ilo[1] = 2 * q.ilo[1] + cy * q.n;
                        c.ilo[2] = 2 * q.ilo[2] + cz * q.n;
                        out[o++] = c;
                    }
        } else {
            out[o++] = q;
        }
    }
    return Z4C_OK;
}

int z4c_regrid_transfer(z4c_pack* src, int32_t src_reg, z4c_pack* dst, int32_t dst_reg, void* stream)
{
    if (!src || !dst || src == dst) return Z4C_EINVAL;
    if (src_reg < Z4C_REG_U || src_reg > Z4C_REG_S2 || dst_reg < Z4C_REG_U || dst_reg > Z4C_REG_S2)
        return fail(dst, Z4C_EINVAL, "regrid: bad register");
    if (!src->bound || !dst->bound) return fail(dst, Z4C_ESTATE, "regrid: pack not bound");
    const z4c_params &a = src->p, &b = dst->p;
    bool same = a.fd_order == b.fd_order && a.nghost == b.nghost && a.precision == b.precision &&
                a.bc == b.bc && a.dx0 == b.dx0;
    for (int d = 0; d < 3; ++d) same = same && a.nroot[d] == b.nroot[d] && a.lo[d] == b.lo[d];
    if (!same) return fail(dst, Z4C_EINVAL, "regrid: packs describe different meshes or methods");
    dst->last_stage = 0;   // a register of dst is rewritten
    // per destination block: where its data comes from
    std::map<std::tuple<int, int, int, int, int>, int> at;
    for (size_t s = 0; s < src->blk.size(); ++s) {
        const z4c_block& q = src->blk[s];
        at[std::make_tuple(q.level, q.n, q.ilo[0], q.ilo[1], q.ilo[2])] = (int)s;
    }
    const int nd = (int)dst->blk.size();
    std::vector<RegridDesc>& desc = dst->regrid_desc;
    desc.assign(nd, RegridDesc{});
    int maxn = 0;
    for (int d = 0; d < nd; ++d) {
        const z4c_block& q = dst->blk[d];
        RegridDesc& r = desc[d];
        std::memset(&r, 0, sizeof(r));
        maxn = std::max(maxn, q.n);
        auto it = at.find(std::make_tuple(q.level, q.n, q.ilo[0], q.ilo[1], q.ilo[2]));
        if (it != at.end()) {
            r.kind = 0;
            r.src[0] = it->second;
            continue;
        }
        int par = -1;
        for (size_t s = 0; s < src->blk.size() && par < 0; ++s) {
            const z4c_block& c = src->blk[s];
            if (c.level != q.level - 1) continue;
            bool in = true;
            for (int k = 0; k < 3; ++k)
                in = in && 2 * c.ilo[k] <= q.ilo[k] && q.ilo[k] + q.n <= 2 * (c.ilo[k] + c.n);
            if (in) par = (int)s;
        }
        if (par >= 0) {
            r.kind = 1;
            r.src[0] = par;
            continue;
        }
        r.kind = 2;
        for (int c = 0; c < 8; ++c) {
            const int cx = c & 1, cy = (c >> 1) & 1, cz = c >> 2;
            auto ic = at.find(std::make_tuple(q.level + 1, q.n, 2 * q.ilo[0] + cx * q.n,
                                              2 * q.ilo[1] + cy * q.n, 2 * q.ilo[2] + cz * q.n));
            if (ic == at.end())
                return fail(dst, Z4C_EINVAL, "regrid: block %d is neither kept, refined nor merged", d);
            r.src[c] = ic->second;
        }
        if (q.n < a.nghost + 1) return fail(dst, Z4C_EUNSUPPORTED, "regrid: blocks smaller than the stencil");
    }
    hipStream_t s = as_stream(stream);
    int rc = z4c_fill_ghosts(src, src_reg, stream);
    if (rc) return fail(dst, rc, "regrid: ghost fill of the source failed: %s", src->err.c_str());
    hipError_t e = hipMemcpyAsync(dst->ws + dst->ws_regrid, desc.data(), sizeof(RegridDesc) * nd,
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return fail(dst, Z4C_EDEVICE, "regrid upload: %s", hipGetErrorString(e));
    RegridArgs ra;
    std::memset(&ra, 0, sizeof(ra));
    ra.src = src->reg[src_reg];
    ra.dst = dst->reg[dst_reg];
    ra.sblocks = reinterpret_cast<const BlockDev*>(src->ws + src->ws_blocks);
    ra.dblocks = reinterpret_cast<const BlockDev*>(dst->ws + dst->ws_blocks);
    ra.desc = reinterpret_cast<const RegridDesc*>(dst->ws + dst->ws_regrid);
    ra.g = a.nghost;
    ra.npts = a.nghost + 1;
    if (ra.npts > 8) return fail(dst, Z4C_EUNSUPPORTED, "regrid: stencil wider than 8");
    // the cross-level fill's weights: restriction set d evaluates at the fine
    // face d of an np-point window; prolongation at the fine centres of
    // parity 0 / 1 within the prolongation window
    const int np = ra.npts;
    for (int d = 1; d < np; ++d) lagrange_half(np, (double)d, &ra.rw[8 * d]);
    {
        const double t0 = (np % 2 == 0) ? np / 2 + 0.25 : (np - 1) / 2 + 0.25;
        const double t1 = (np % 2 == 0) ? np / 2 - 0.25 : (np - 1) / 2 + 0.75;
        lagrange_half(np, t0, &ra.pw[0]);
        lagrange_half(np, t1, &ra.pw[8]);
    }
    e = launch_regrid(a.precision, ra, nd, maxn, s);
    if (e != hipSuccess) return fail(dst, Z4C_EDEVICE, "regrid launch: %s", hipGetErrorString(e));
    return Z4C_OK;
}

}  // extern "C"
