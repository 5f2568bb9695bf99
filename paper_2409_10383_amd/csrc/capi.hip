// Host runtime of libz4c: pack validation and geometry (Mesh / MeshBlock /
// MeshBlockPack, Sec. 3), register and workspace layout, table upload and
// kernel dispatch behind the C ABI of include/z4c.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <type_traits>
#include <map>
#include <tuple>
#include <unordered_map>
#include <string>
#include <vector>

#include "pack.hpp"
#include "stencils.hpp"

namespace z4c_host {

int fail(z4c_pack* pk, int code, const char* fmt, ...)
{
    if (pk) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        pk->err = buf;
    }
    return code;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

int64_t floor_div(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// Lagrange weights (Eq. 1 of the paper) of the nodes q + 1/2, q = 0..n-1, at t
void lagrange_half(int n, double t, double* w)
{
    for (int q = 0; q < n; ++q) {
        double p = 1.0;
        for (int m = 0; m < n; ++m)
            if (m != q) p *= (t - (m + 0.5)) / ((q + 0.5) - (m + 0.5));
        w[q] = p;
    }
}

}  // namespace z4c_host

using namespace z4c_host;

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int gcd_i(int a, int b)
{
    a = a < 0 ? -a : a;
    b = b < 0 ? -b : b;
    while (b) { int t = a % b; a = b; b = t; }
    return a;
}

ParamsDev dev_params(const z4c_params& p)
{
    ParamsDev d;
    d.ko_sigma = p.ko_sigma;
    d.kappa1 = p.kappa1;
    d.kappa2 = p.kappa2;
    d.eta = p.eta;
    d.mu_S = p.mu_S;
    d.chi_floor = p.chi_floor;
    d.alpha_floor = p.alpha_floor;
    d.terms = p.terms;
    d.enforce = (p.flags & Z4C_FLAG_ENFORCE) ? 1 : 0;
    return d;
}

// work list of the fused stage kernel for tile-shape variant v
bool build_work(const std::vector<z4c_block>& blk, int v, std::vector<WorkItem>& work)
{
    const int ti = TILE_SHAPES[v][0], tj = TILE_SHAPES[v][1], tk = TILE_SHAPES[v][2];
    work.clear();
    for (size_t b = 0; b < blk.size(); ++b) {
        const int n = blk[b].n;
        if (n % ti || n % tj || n % tk) return false;
        for (int k0 = 0; k0 < n; k0 += tk)
            for (int j0 = 0; j0 < n; j0 += tj)
                for (int i0 = 0; i0 < n; i0 += ti) {
                    WorkItem w;
                    w.block = (int32_t)b;
                    w.i0 = (int16_t)i0; w.j0 = (int16_t)j0; w.k0 = (int16_t)k0;
                    w.ni = (int16_t)ti; w.nj = (int16_t)tj; w.nk = (int16_t)tk;
                    work.push_back(w);
                }
    }
    return true;
}

// Host-side queries on the block layout of a pack.
struct Geo {
    const z4c_pack* pk;
    void bc(int l, int64_t I[3]) const
    {
        for (int a = 0; a < 3; ++a) {
            const int64_t N = (int64_t)pk->p.nroot[a] << l;
            if (pk->p.bc == Z4C_BC_PERIODIC) {
                I[a] %= N;
                if (I[a] < 0) I[a] += N;
            } else {
                I[a] = I[a] < 0 ? 0 : (I[a] >= N ? N - 1 : I[a]);
            }
        }
    }
    // leaf of exactly level l covering cell I (I inside the domain), or -1
    int leaf(int l, const int64_t I[3]) const
    {
        if (l < 0 || l >= pk->L.nlev) return -1;
        const int u = pk->L.unit;
        int64_t q[3];
        for (int a = 0; a < 3; ++a) {
            q[a] = I[a] / u;
            if (I[a] < 0 || q[a] >= pk->L.dim[l][a]) return -1;
        }
        return pk->map[pk->L.base[l] + (q[2] * pk->L.dim[l][1] + q[1]) * pk->L.dim[l][0] + q[0]];
    }
    int64_t cell(int b, const int64_t I[3]) const  // ghosted element offset of active cell I of block b
    {
        const BlockDev& B = pk->bdev[b];
        const int g = pk->p.nghost;
        return ((I[2] - B.ilo[2] + g) * (int64_t)B.E + (I[1] - B.ilo[1] + g)) * B.E + (I[0] - B.ilo[0] + g);
    }
    // restriction of coarse cell J (level l) from fine leaf F: window origin and weight sets
    // coarse cell J (level of F minus one) in F's coarse image: local index
    int64_t image_cell(int F, const int64_t J[3]) const
    {
        const z4c_block& FB = pk->blk[F];
        const int64_t m = FB.n / 2;
        int64_t L[3];
        for (int a = 0; a < 3; ++a) {
            L[a] = J[a] - FB.ilo[a] / 2;
            if (L[a] < 0 || L[a] >= m) return -1;
        }
        return (L[2] * m + L[1]) * m + L[0];
    }
};

// Non-persistent stage grid: the XCD-aware slot -> tile map interleaves
// 8 slices of ceil(nwork/8) tiles, so it needs 8 * ceil(nwork/8) slots
// (slots past the end map to tile indices >= nwork and exit).
static int stage_grid(size_t nwork)
{
    return (int)(8 * ((nwork + 7) / 8));
}

// Build the transfer / prolongation lists of a multi-level pack.
int build_xlevel(z4c_pack* pk)
{
    const int g = pk->p.nghost, np = g + 1;
    if (np > 8) return Z4C_EUNSUPPORTED;
    Geo geo{pk};
    pk->rw.assign(64, 0.0);
    pk->pw.assign(16, 0.0);
    for (int d = 1; d < np; ++d) lagrange_half(np, (double)d, &pk->rw[8 * d]);
    {
        const double t0 = (np % 2 == 0) ? np / 2 + 0.25 : (np - 1) / 2 + 0.25;
        const double t1 = (np % 2 == 0) ? np / 2 - 0.25 : (np - 1) / 2 + 0.75;
        lagrange_half(np, t0, &pk->pw[0]);
        lagrange_half(np, t1, &pk->pw[8]);
    }
    const size_t esz = pk->p.precision == Z4C_FP64 ? 8 : 4;
    const int64_t per256 = 256 / (int64_t)esz;
    const int nb = (int)pk->blk.size();
    pk->img_off.assign(nb, -1);
    std::vector<ProlongGroup> quads, pairs, singles;   // grouped prolongations
    // ghosts of directions the stage path leaves alone (vmask): their items go
    // after those of the other ghosts
    std::vector<ProlongGroup> lquads, lpairs, lsingles;
    std::vector<XferItem> xlate;
    std::vector<ProlongItem> plate;
    // image rows (z-plane * m + y) some transfer reads, per source block
    // and the range of coarse x each such row needs
    std::vector<std::vector<uint8_t>> img_rows(nb);
    std::vector<std::vector<int16_t>> img_xlo(nb), img_xhi(nb);
    auto need_row = [&](int F, int64_t ic) {
        const int64_t m = pk->blk[F].n / 2;
        if (img_rows[F].empty()) {
            img_rows[F].assign((size_t)(m * m), 0);
            img_xlo[F].assign((size_t)(m * m), (int16_t)m);
            img_xhi[F].assign((size_t)(m * m), (int16_t)-1);
        }
        const size_t row = (size_t)(ic / m);
        const int16_t x = (int16_t)(ic % m);
        img_rows[F][row] = 1;
        img_xlo[F][row] = std::min(img_xlo[F][row], x);
        img_xhi[F][row] = std::max(img_xhi[F][row], x);
    };
    pk->img_fstride.assign(nb, 0);
    // coarse image of fine block F (allocated on first use)
    auto image_of = [&](int F) -> int64_t {
        if (pk->img_off[F] < 0) {
            const int64_t m = pk->blk[F].n / 2;
            const int64_t fs = (m * m * m + per256 - 1) / per256 * per256;
            pk->img_off[F] = pk->image_elems;
            pk->img_fstride[F] = (int32_t)fs;
            pk->image_elems += NF * fs;
        }
        return pk->img_off[F];
    };
    for (int b = 0; b < nb; ++b) {
        const z4c_block& B = pk->blk[b];
        const BlockDev& D = pk->bdev[b];
        const int l = B.level, n = B.n, E = D.E;
        if (D.slab > INT32_MAX) return Z4C_EUNSUPPORTED;
        // shadow box of this block at level l-1 (allocated on first use)
        int64_t S0[3];
        const int64_t SE = (n + 2 * g) / 2 + 2 * (np + 1) + 2;
        for (int a = 0; a < 3; ++a) S0[a] = floor_div(B.ilo[a] - g, 2) - (np + 1);
        int64_t shoff = -1;
        std::vector<uint8_t> mark;
        // per set (0: ghosts the stage path reads, 1: the others)
        std::unordered_map<int64_t, size_t> pgmap[2];  // parent's child-(0,0,0) cell -> group
        std::vector<ProlongGroup> bg[2];                // this block's groups
        std::vector<int64_t> bkey[2];                   // and their keys
        for (int k = 0; k < E; ++k)
            for (int j = 0; j < E; ++j)
                for (int i = 0; i < E; ++i) {
                    if (i >= g && i < g + n && j >= g && j < g + n && k >= g && k < g + n) continue;
                    const int didx = ((k < g ? 0 : (k >= g + n ? 2 : 1)) * 3 + (j < g ? 0 : (j >= g + n ? 2 : 1))) * 3 +
                                     (i < g ? 0 : (i >= g + n ? 2 : 1));
                    const int late = (int)((pk->vmask[b] >> didx) & 1u);
                    const int64_t G[3] = {B.ilo[0] + i - g, B.ilo[1] + j - g, B.ilo[2] + k - g};
                    int64_t Gb[3] = {G[0], G[1], G[2]};
                    geo.bc(l, Gb);
                    if (geo.leaf(l, Gb) >= 0) continue;  // same level
                    const int64_t dcell = D.off + ((int64_t)k * E + j) * E + i;
                    const int64_t C2[3] = {2 * Gb[0], 2 * Gb[1], 2 * Gb[2]};
                    const int F = geo.leaf(l + 1, C2);
                    if (F >= 0) {
                        XferItem it;
                        it.dst = dcell;
                        it.dst_stride = (int32_t)D.slab;
                        const int64_t ic = geo.image_cell(F, Gb);
                        if (ic < 0) return Z4C_EINVAL;
                        need_row(F, ic);
                        it.src = image_of(F) + ic;
                        it.src_stride = pk->img_fstride[F];
                        it.kind = 1;
                        it.pad = 0;
                        (late ? xlate : pk->xfer).push_back(it);
                        continue;
                    }
                    const int64_t P[3] = {Gb[0] / 2, Gb[1] / 2, Gb[2] / 2};
                    if (geo.leaf(l - 1, P) < 0) return Z4C_EINVAL;
                    // prolongation: stencil around the periodic-unwrapped or clamped index
                    const int64_t* Iu = (pk->p.bc == Z4C_BC_PERIODIC) ? G : Gb;
                    const bool regular = (Iu[0] == G[0] && Iu[1] == G[1] && Iu[2] == G[2]);
                    int64_t s[3];
                    int parity = 0;
                    for (int a = 0; a < 3; ++a) {
                        const int64_t J = floor_div(Iu[a], 2);
                        const int odd = (int)(Iu[a] - 2 * J);
                        parity |= odd << a;
                        s[a] = (np % 2) ? J - (np - 1) / 2 : (odd ? J - np / 2 + 1 : J - np / 2);
                        if (s[a] < S0[a] || s[a] + np > S0[a] + SE) return Z4C_EINVAL;
                    }
                    if (regular) {
                        // grouped by coarse parent: union stencil starts one cell lower
                        // for even np (parity-0 window)
                        for (int a = 0; a < 3; ++a)
                            if (np % 2 == 0 && (parity >> a & 1)) s[a] -= 1;
                        for (int a = 0; a < 3; ++a)
                            if (s[a] < S0[a] || s[a] + np + (np % 2 == 0) > S0[a] + SE) return Z4C_EINVAL;
                    }
                    if (shoff < 0) {
                        shoff = pk->shadow_elems;
                        const int64_t cells = SE * SE * SE;
                        pk->shadow_elems += NF * ((cells + per256 - 1) / per256 * per256);
                        mark.assign((size_t)(SE * SE * SE), 0);
                    }
                    const int64_t fstride = (SE * SE * SE + per256 - 1) / per256 * per256;
                    const int nu = regular ? np + (np % 2 == 0) : np;
                    for (int kz = 0; kz < nu; ++kz)
                        for (int jy = 0; jy < nu; ++jy)
                            for (int ix = 0; ix < nu; ++ix) {
                                const int64_t K[3] = {s[0] + ix, s[1] + jy, s[2] + kz};
                                const int64_t loc = ((K[2] - S0[2]) * SE + (K[1] - S0[1])) * SE + (K[0] - S0[0]);
                                if (mark[loc]) continue;
                                mark[loc] = 1;
                                int64_t Kb[3] = {K[0], K[1], K[2]};
                                geo.bc(l - 1, Kb);
                                XferItem it;
                                it.dst = shoff + loc;
                                it.dst_stride = (int32_t)fstride;
                                it.kind = 2;
                                it.pad = 0;
                                const int Cb = geo.leaf(l - 1, Kb);
                                if (Cb >= 0) {
                                    it.src = pk->bdev[Cb].off + geo.cell(Cb, Kb);
                                    it.src_stride = (int32_t)pk->bdev[Cb].slab;
                                } else {
                                    const int64_t K2[3] = {2 * Kb[0], 2 * Kb[1], 2 * Kb[2]};
                                    const int Fb = geo.leaf(l, K2);
                                    if (Fb < 0) return Z4C_EINVAL;  // would need a level two away
                                    const int64_t ic = geo.image_cell(Fb, Kb);
                                    if (ic < 0) return Z4C_EINVAL;
                                    need_row(Fb, ic);
                                    it.src = image_of(Fb) + ic;
                                    it.src_stride = pk->img_fstride[Fb];
                                    it.kind = 3;
                                }
                                pk->xfer.push_back(it);
                            }
                    const int64_t shs = shoff + ((s[2] - S0[2]) * SE + (s[1] - S0[1])) * SE + (s[0] - S0[0]);
                    if (regular) {
                        // child (cx, cy, cz) of the parent; the (0,0,0) child's cell
                        const int cx = parity & 1, cy = (parity >> 1) & 1, cz = (parity >> 2) & 1;
                        const int64_t d0 = D.off + ((int64_t)(k - cz) * E + (j - cy)) * E + (i - cx);
                        // key: child (0,0,0) index shifted by one (it can sit at -1)
                        const int64_t key = ((int64_t)(k - cz + 1) * (E + 2) + (j - cy + 1)) * (E + 2) + (i - cx + 1);
                        auto itg = pgmap[late].find(key);
                        if (itg == pgmap[late].end()) {
                            ProlongGroup pg;
                            pg.dst = d0;
                            pg.sh = shs;
                            pg.block = b;
                            pg.se = (int32_t)SE;
                            pg.mask = 0;
                            pg.fstride = (int32_t)fstride;
                            itg = pgmap[late].emplace(key, bg[late].size()).first;
                            bg[late].push_back(pg);
                            bkey[late].push_back(key);
                        }
                        bg[late][itg->second].mask |= 1 << (cz * 4 + cy * 2 + cx);
                    } else {
                        ProlongItem pi;
                        pi.dst = dcell;
                        pi.sh = shs;
                        pi.block = b;
                        pi.se = (int32_t)SE;
                        pi.parity = parity;
                        pi.pad = (int32_t)fstride;  // field stride of the shadow box
                        (late ? plate : pk->prol).push_back(pi);
                    }
                }
        // neighbouring parents along y and z (child-(0,0,0) keys two rows or
        // two planes apart) are taken together, four (y and z) or two (y) at
        // a time: one thread reads the union of their stencils (one more row,
        // or row and plane), while neighbouring threads keep taking
        // neighbouring parents along x, so a load still touches the lines of
        // one row
        const int64_t dy = 2 * (int64_t)(E + 2), dz = dy * (E + 2);
        for (int set = 0; set < 2; ++set) {
            const std::vector<ProlongGroup>& grp = bg[set];
            const std::vector<int64_t>& keys = bkey[set];
            const std::unordered_map<int64_t, size_t>& at = pgmap[set];
            std::vector<ProlongGroup>& q4 = set ? lquads : quads;
            std::vector<ProlongGroup>& q2 = set ? lpairs : pairs;
            std::vector<ProlongGroup>& q1 = set ? lsingles : singles;
            std::vector<uint8_t> used(grp.size(), 0);
            auto partner = [&](size_t q, int64_t dk) -> int64_t {
                const auto it2 = at.find(keys[q] + dk);
                return (it2 == at.end() || used[it2->second]) ? -1 : (int64_t)it2->second;
            };
            // (fours only for FP64: with 4-byte loads the wider thread costs more
            // than the shared rows save)
            for (size_t q = 0; q < grp.size() && pk->p.precision == Z4C_FP64; ++q) {
                if (used[q]) continue;
                const int64_t b1 = partner(q, dy), c1 = partner(q, dz), d1 = partner(q, dy + dz);
                if (b1 < 0 || c1 < 0 || d1 < 0) continue;
                ProlongGroup pg = grp[q];
                pg.mask |= (grp[b1].mask << 8) | (grp[c1].mask << 16) | (grp[d1].mask << 24);
                q4.push_back(pg);
                used[q] = used[b1] = used[c1] = used[d1] = 1;
            }
            for (size_t q = 0; q < grp.size(); ++q) {
                if (used[q]) continue;
                const int64_t o1 = partner(q, dy);
                if (o1 < 0) continue;
                ProlongGroup pg = grp[q];
                pg.mask |= grp[o1].mask << 8;
                q2.push_back(pg);
                used[q] = used[o1] = 1;
            }
            for (size_t q = 0; q < grp.size(); ++q)
                if (!used[q]) q1.push_back(grp[q]);
            pk->nparent += (int64_t)grp.size();
        }
    }
    // by kind, so that few waves mix them
    pk->pgrp = quads;
    pk->pgrp.insert(pk->pgrp.end(), pairs.begin(), pairs.end());
    pk->pgrp.insert(pk->pgrp.end(), singles.begin(), singles.end());
    pk->npgrp_stage = (int64_t)pk->pgrp.size();
    pk->pgrp.insert(pk->pgrp.end(), lquads.begin(), lquads.end());
    pk->pgrp.insert(pk->pgrp.end(), lpairs.begin(), lpairs.end());
    pk->pgrp.insert(pk->pgrp.end(), lsingles.begin(), lsingles.end());
    pk->nprol_stage = (int64_t)pk->prol.size();
    pk->prol.insert(pk->prol.end(), plate.begin(), plate.end());
    // image restriction work: per source block, runs of consecutive coarse
    // z-planes that need the same rows (first to last row some transfer
    // reads) and columns, split into row chunks that fit the LDS budget; a
    // workgroup marches along its run keeping the y-passes of the last np
    // fine planes, so that it reads each fine plane once
    for (int F = 0; F < nb; ++F) {
        if (pk->img_off[F] < 0) continue;
        const int m = pk->blk[F].n / 2;
        if (pk->blk[F].ilo[0] % 2 || pk->blk[F].ilo[1] % 2 || pk->blk[F].ilo[2] % 2) return Z4C_EINVAL;
        if (pk->blk[F].n < np) return Z4C_EUNSUPPORTED;
        const std::vector<uint8_t>& need = img_rows[F];
        // per coarse plane: first and last needed row, first and last column
        std::vector<std::array<int, 4>> pl((size_t)m, std::array<int, 4>{-1, -1, m, -1});
        for (int kz = 0; kz < m; ++kz)
            for (int y = 0; y < m; ++y)
                if (need[(size_t)kz * m + y]) {
                    std::array<int, 4>& q = pl[(size_t)kz];
                    if (q[0] < 0) q[0] = y;
                    q[1] = y;
                    q[2] = std::min<int>(q[2], img_xlo[F][(size_t)kz * m + y]);
                    q[3] = std::max<int>(q[3], img_xhi[F][(size_t)kz * m + y]);
                }
        for (int kz = 0; kz < m;) {
            const std::array<int, 4> q = pl[(size_t)kz];
            if (q[0] < 0) { ++kz; continue; }
            int k1 = kz + 1;
            while (k1 < m && pl[(size_t)k1] == q) ++k1;
            const int cx = q[3] - q[2] + 1;
            int cy = q[1] - q[0] + 1;
            while (cy > 1 && ((int64_t)(2 * cy + np) * cx > RI_XMAX || (int64_t)np * cy * cx > RI_YMAX))
                cy = (cy + 1) / 2;
            if ((int64_t)(2 * cy + np) * cx > RI_XMAX || (int64_t)np * cy * cx > RI_YMAX) return Z4C_EUNSUPPORTED;
            for (int y0 = q[0]; y0 <= q[1]; y0 += cy) {
                ImageSlice sl;
                std::memset(&sl, 0, sizeof(sl));
                sl.img = pk->img_off[F];
                sl.block = F;
                sl.fstride = pk->img_fstride[F];
                sl.kz = (int16_t)kz;
                sl.nkz = (int16_t)(k1 - kz);
                sl.y0 = (int16_t)y0;
                sl.ny = (int16_t)std::min(cy, q[1] - y0 + 1);
                sl.x0 = (int16_t)q[2];
                sl.nx = (int16_t)cx;
                pk->islice.push_back(sl);
            }
            kz = k1;
        }
    }
    // copies from active cells first: they need neither the restriction nor
    // the same-level fill, and run beside them
    std::stable_partition(pk->xfer.begin(), pk->xfer.end(), [](const XferItem& it) { return it.kind == 2; });
    pk->nxfer_direct = std::count_if(pk->xfer.begin(), pk->xfer.end(), [](const XferItem& it) { return it.kind == 2; });
    pk->nxfer_stage = (int64_t)pk->xfer.size();
    pk->xfer.insert(pk->xfer.end(), xlate.begin(), xlate.end());
    return Z4C_OK;
}

// Virtual halos: the stage kernel's staged tiles read a same-level neighbour's
// active cells directly where the neighbour region of direction (dx, dy, dz)
// is one block of the same level and size (periodic wrap included), so the
// stage path's ghost fill leaves those ghost cells alone.  vnbr[27 b + idx]
// is the element offset that puts the ghosted index of block b's frame onto
// the neighbour's cells (the block's own offset where the ghosts are real).
// A staged row that takes its x halo from the neighbours spans three
// blocks' memory.  With 16-byte FP64 lanes and an even ghost depth that
// costs little, and every direction is read in place (virt_x).  With FP32
// storage it costs the stage kernel more (12 % on the 512-block pack) than
// the ghosts would, and with an odd FP64 ghost depth the lanes at the x
// faces straddle them: there only directions with dx = 0 are read in
// place, and directions with dx != 0 whose neighbour is one block of the
// same level and size are pushed instead (pmask): the stage kernel writes
// each zone near an x face into the neighbours' ghosts as well, so the
// stage path's fill leaves them alone from the second stage of a step on,
// and a staged lane takes its direction from y and z alone (across the x
// face it reads its own, or that neighbour's, x ghosts).  FP64 lanes that
// are not 16-byte aligned (ghost depth and halo of different parity) copy
// per half cell from the block itself: no direction is virtual or pushed.
// Outflow boundaries: a staged cell whose y or z lies beyond a domain face
// takes the value of the nearest active cell along that axis, so a direction
// whose y and z components leave the domain (dx = 0, or any dx where x
// directions are read in place) reads the block across its remaining
// components, the block itself where none remain, with y and z clamped to
// the active range (cmask: y and z clamp bits per direction); the fill skips
// those directions too.  Directions across an outflow x face cannot be
// clamped per lane; there the zones on the face write the ghost columns
// beyond it (omask) into their own block and into the same-level neighbours
// across y and z whose ghosts reach their rows, the clamped rows beyond y and
// z domain faces included, and the fill leaves those directions alone from
// the second stage of a step on (fskip, with the pushed x directions).
void build_virtual_halos(z4c_pack* pk)
{
    const int nb = (int)pk->blk.size();
    const int g = pk->p.nghost, R = pk->p.fd_order / 2 + 1;
    pk->vnbr.assign((size_t)27 * nb, 0);
    pk->vmask.assign(nb, 0u);
    pk->cmask.assign((size_t)2 * nb, 0u);
    pk->pmask.assign(nb, 0u);
    pk->omask.assign(nb, 0u);
    pk->fskip.assign(nb, 0u);
    pk->virt_x = 1;
    pk->fill_pushed_empty = false;
    for (int b = 0; b < nb; ++b)
        for (int i = 0; i < 27; ++i) pk->vnbr[27 * b + i] = pk->bdev[b].off;
    const bool fp64 = pk->p.precision == Z4C_FP64;
    if (pk->p.bc == Z4C_BC_USER) return;
    if (fp64 && ((g - R) & 1)) return;
    if (!fp64 || (g & 1)) pk->virt_x = 0;
    const bool outflow = pk->p.bc == Z4C_BC_OUTFLOW;
    std::map<std::tuple<int, int, int64_t, int64_t, int64_t>, int> at;   // (level, n, ilo) -> block
    for (int b = 0; b < nb; ++b) {
        const z4c_block& B = pk->blk[b];
        at[std::make_tuple(B.level, B.n, (int64_t)B.ilo[0], (int64_t)B.ilo[1], (int64_t)B.ilo[2])] = b;
    }
    std::vector<uint32_t> same(nb, 0u);   // directions with a same-level neighbour of the same size
    std::vector<int> nbr((size_t)27 * nb, -1);   // that neighbour
    std::vector<std::array<uint8_t, 3>> face(nb);   // per axis: bit 0 low, bit 1 high face on the domain face
    for (int b = 0; b < nb; ++b) {
        const z4c_block& B = pk->blk[b];
        const BlockDev& D = pk->bdev[b];
        for (int a = 0; a < 3; ++a) {
            const int64_t N = (int64_t)pk->p.nroot[a] << B.level;
            face[b][a] = (uint8_t)((B.ilo[a] == 0 ? 1 : 0) | ((int64_t)B.ilo[a] + B.n >= N ? 2 : 0));
        }
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    if (!dx && !dy && !dz) continue;
                    const int dd[3] = {dx, dy, dz};
                    const int idx = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
                    // outflow: drop the y and z components that leave the domain
                    int ee[3] = {dx, dy, dz};
                    uint32_t cy = 0, cz = 0;
                    if (outflow) {
                        for (int a = 1; a < 3; ++a)
                            if (dd[a] && (face[b][a] >> (dd[a] > 0)) & 1) {
                                ee[a] = 0;
                                (a == 1 ? cy : cz) = 1u;
                            }
                        if (dx && (face[b][0] >> (dx > 0)) & 1) continue;   // across an outflow x face
                    }
                    const bool clamped = cy || cz;
                    if (clamped && dx && !pk->virt_x) continue;
                    int64_t v = D.off;
                    if (ee[0] || ee[1] || ee[2]) {
                        int64_t J[3];
                        bool inside = true;
                        for (int a = 0; a < 3; ++a) {
                            const int64_t N = (int64_t)pk->p.nroot[a] << B.level;
                            J[a] = (int64_t)B.ilo[a] + (int64_t)ee[a] * B.n;
                            if (J[a] < 0 || J[a] >= N) {
                                if (pk->p.bc != Z4C_BC_PERIODIC) inside = false;
                                J[a] = ((J[a] % N) + N) % N;
                            }
                        }
                        if (!inside) continue;
                        auto it = at.find(std::make_tuple(B.level, B.n, J[0], J[1], J[2]));
                        if (it == at.end()) continue;
                        const BlockDev& T = pk->bdev[it->second];
                        const int64_t E = D.E;
                        v = T.off - (int64_t)B.n * (ee[2] * E * E + ee[1] * E + ee[0]);
                        // element offsets of the staged cells stay within int32
                        if (std::llabs(v - D.off) > ((int64_t)1 << 30)) continue;
                        if (!clamped) {
                            same[b] |= 1u << idx;
                            nbr[(size_t)27 * b + idx] = it->second;
                        }
                    }
                    pk->vnbr[27 * b + idx] = v;
                    pk->cmask[2 * b] |= cy << idx;
                    pk->cmask[2 * b + 1] |= cz << idx;
                    if (dx && !pk->virt_x) pk->pmask[b] |= 1u << idx;
                    else pk->vmask[b] |= 1u << idx;
                }
    }
    // Without x directions read in place, a staged cell beyond an x face and
    // a y or z face takes its direction from y and z alone: it reads the x
    // ghosts of the block across (0, dy, dz) where that direction is read in
    // place (or its own, clamped).  The block's own ghosts in (dx, dy, dz)
    // are then never read: the fill skips them and nothing writes them.
    // A block pushes into a neighbour's ghosts of direction (-dx, -dy, -dz)
    // only where that neighbour reads them, and skips its own (dx, dy, dz)
    // ghosts in the fill where it never reads them or the neighbour there
    // pushes them (pmask: pusher role; recv: receiver role).
    std::vector<uint32_t> recv = pk->pmask;
    if (!pk->virt_x) {
        const std::vector<uint32_t> v0 = pk->vmask, p0 = pk->pmask;
        auto reads = [&](int b, int idx) {   // block b reads its ghosts of direction idx
            const int dx = idx % 3 - 1, e = idx - dx;   // e: the direction with dx = 0
            return e == 13 || !((v0[b] >> e) & 1u);
        };
        for (int b = 0; b < nb; ++b) {
            uint32_t push = 0, skip = 0;
            for (int idx = 0; idx < 27; ++idx) {
                if (idx % 3 == 1) continue;   // dx = 0
                if (!reads(b, idx)) pk->vmask[b] |= 1u << idx;
                else if ((p0[b] >> idx) & 1u) skip |= 1u << idx;
                if (((p0[b] >> idx) & 1u) && reads(nbr[(size_t)27 * b + idx], 26 - idx)) push |= 1u << idx;
            }
            pk->pmask[b] = push;
            recv[b] = skip;
        }
    }
    if (outflow) {
        for (int b = 0; b < nb; ++b) {
            const uint32_t xf = face[b][0] & 3u;
            if (!xf) continue;
            // pusher: faces, and the blocks across (0, ey, ez) it writes into
            // (without x directions read in place only its own rows are read)
            uint32_t om = xf | 1u << (8 + 4);
            if (pk->virt_x) {
                om |= (uint32_t)(face[b][1] & 3u) << 2 | (uint32_t)(face[b][2] & 3u) << 4;
                for (int e = 0; e < 9; ++e) {
                    const int idx = e * 3 + 1;   // direction (0, e % 3 - 1, e / 3 - 1)
                    if ((same[b] >> idx) & 1u) om |= 1u << (8 + e);
                }
            }
            pk->omask[b] = om;
            // receiver: a direction across an outflow x face takes its values
            // from the block across its y and z components that stay inside
            // the domain (the block itself if none does)
            for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; dx += 2) {
                        if (!((xf >> (dx > 0)) & 1u)) continue;
                        if (!pk->virt_x && (dy || dz)) continue;   // never read, or filled
                        const int sy = (dy && !((face[b][1] >> (dy > 0)) & 1)) ? dy : 0;
                        const int sz = (dz && !((face[b][2] >> (dz > 0)) & 1)) ? dz : 0;
                        const int sidx = (sz + 1) * 9 + (sy + 1) * 3 + 1;
                        if ((sy || sz) && !((same[b] >> sidx) & 1u)) continue;
                        pk->fskip[b] |= 1u << ((dz + 1) * 9 + (dy + 1) * 3 + (dx + 1));
                    }
        }
    }
    const uint32_t all = ((1u << 27) - 1) & ~(1u << 13);
    bool empty = true;
    for (int b = 0; b < nb; ++b) {
        pk->fskip[b] |= recv[b];
        if (((pk->vmask[b] | pk->fskip[b]) & all) != all) empty = false;
    }
    pk->fill_pushed_empty = empty;
}

// side stream and its fork/join events (multi-level packs)
void release_side(z4c_pack* pk)
{
    if (pk->side) hipStreamSynchronize(pk->side);
    if (pk->fork_ev) hipEventDestroy(pk->fork_ev);
    if (pk->join_ev) hipEventDestroy(pk->join_ev);
    if (pk->side) hipStreamDestroy(pk->side);
    pk->side = nullptr;
    pk->fork_ev = pk->join_ev = nullptr;
}

// bracket a launch with events when profiling is on (kind 0 stage, 1 fill)
struct ProfScope {
    z4c_pack* pk;
    hipStream_t s;
    int kind;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(z4c_pack* p, hipStream_t st, int k) : pk(p), s(st), kind(k)
    {
        if (!pk->prof) return;
        if (hipEventCreate(&a) != hipSuccess) { a = nullptr; return; }
        if (hipEventCreate(&b) != hipSuccess) { hipEventDestroy(a); a = b = nullptr; return; }
        hipEventRecord(a, s);
    }
    ~ProfScope()
    {
        if (!a) return;
        hipEventRecord(b, s);
        pk->ev.push_back({a, b, kind});
    }
};

}  // namespace

extern "C" {

int z4c_pack_create(const z4c_params* params, const z4c_block* blocks, int32_t nblocks,
                    z4c_pack** out)
{
    if (!out) return Z4C_EINVAL;
    *out = nullptr;
    if (!params || !blocks || nblocks < 1) return Z4C_EINVAL;
    const z4c_params& p = *params;
    if (p.fd_order != 4 && p.fd_order != 6 && p.fd_order != 8) return Z4C_EINVAL;
    const int N = p.fd_order / 2;
    if (p.nghost < N + 1 || p.nghost > 8) return Z4C_EINVAL;
    if (p.precision != Z4C_FP64 && p.precision != Z4C_FP32_MIXED) return Z4C_EINVAL;
    if (p.bc < Z4C_BC_PERIODIC || p.bc > Z4C_BC_USER) return Z4C_EINVAL;
    if (!(p.dx0 > 0.0) || !std::isfinite(p.dx0)) return Z4C_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (p.nroot[a] < 1 || !std::isfinite(p.lo[a])) return Z4C_EINVAL;
    if ((p.terms & ~15u) != 0) return Z4C_EINVAL;
    if (!(p.chi_floor >= 0.0) || !(p.alpha_floor >= 0.0) || !(p.ko_sigma >= 0.0)) return Z4C_EINVAL;

    z4c_pack* pk = new (std::nothrow) z4c_pack();
    if (!pk) return Z4C_ENOMEM;
    pk->p = p;
    pk->blk.assign(blocks, blocks + nblocks);
    const int g = p.nghost;
    int lmax = 0, unit = 0;
    for (int b = 0; b < nblocks; ++b) {
        const z4c_block& B = blocks[b];
        // the stage kernel works on 8 x 8 x 4 tiles of active cells
        if (B.level < 0 || B.level > 7 || B.n < 8 || (B.n % 8) || B.n < g || B.n > 512) {
            delete pk;
            return Z4C_EINVAL;
        }
        for (int a = 0; a < 3; ++a) {
            const int64_t Nl = (int64_t)p.nroot[a] << B.level;
            if (B.ilo[a] < 0 || (int64_t)B.ilo[a] + B.n > Nl) { delete pk; return Z4C_EINVAL; }
            unit = gcd_i(unit, B.ilo[a]);
        }
        unit = gcd_i(unit, B.n);
        lmax = std::max(lmax, B.level);
    }
    for (int a = 0; a < 3; ++a) unit = gcd_i(unit, p.nroot[a]);
    // pairwise checks in units of the finest level: no overlap, 2:1 rule
    {
        const int F = lmax;
        double vol = 0.0;
        for (int b = 0; b < nblocks; ++b) {
            const double s = std::ldexp(1.0, F - blocks[b].level);
            vol += std::pow(blocks[b].n * s, 3);
        }
        double dom = 1.0;
        for (int a = 0; a < 3; ++a) dom *= std::ldexp((double)p.nroot[a], F);
        if (std::fabs(vol - dom) > 0.5) { delete pk; return Z4C_EINVAL; }
        for (int b = 0; b < nblocks; ++b) {
            const int64_t sb = int64_t(1) << (F - blocks[b].level);
            for (int c = b + 1; c < nblocks; ++c) {
                const int64_t sc = int64_t(1) << (F - blocks[c].level);
                bool overlap = true, touch = true;
                for (int a = 0; a < 3; ++a) {
                    const int64_t b0 = blocks[b].ilo[a] * sb, b1 = (blocks[b].ilo[a] + blocks[b].n) * sb;
                    const int64_t c0 = blocks[c].ilo[a] * sc, c1 = (blocks[c].ilo[a] + blocks[c].n) * sc;
                    // the finer block's ghost reach, in finest units
                    const int64_t reach = (int64_t)g * std::min(sb, sc) * 2;
                    if (!(b0 < c1 && c0 < b1)) overlap = false;
                    if (!(b0 - reach < c1 && c0 - reach < b1)) touch = false;
                }
                if (overlap) { delete pk; return Z4C_EINVAL; }
                if (touch && std::abs(blocks[b].level - blocks[c].level) > 1) {
                    delete pk;
                    return Z4C_EINVAL;
                }
            }
        }
    }
    pk->multilevel = lmax > 0;

    // register layout
    const size_t esz = p.precision == Z4C_FP64 ? 8 : 4;
    int64_t off = 0, ioff = 0;
    pk->bdev.resize(nblocks);
    for (int b = 0; b < nblocks; ++b) {
        const z4c_block& B = blocks[b];
        BlockDev& d = pk->bdev[b];
        const int E = B.n + 2 * g;
        const int64_t cells = (int64_t)E * E * E;
        const int64_t per256 = 256 / (int64_t)esz;
        d.off = off;
        d.ioff = ioff;
        d.slab = (cells + per256 - 1) / per256 * per256;
        d.n = B.n;
        d.E = E;
        d.level = B.level;
        d.pad = 0;
        for (int a = 0; a < 3; ++a) d.ilo[a] = B.ilo[a];
        d.pad2 = 0;
        d.h = p.dx0 / (double)(1 << B.level);
        for (int a = 0; a < 3; ++a) d.x0[a] = p.lo[a] + (B.ilo[a] + 0.5) * d.h;
        off += (int64_t)NF * d.slab;
        ioff += (int64_t)NF * B.n * B.n * B.n;
        pk->zones += (int64_t)B.n * B.n * B.n;
        pk->maxghost = std::max<int>(pk->maxghost, (int)(cells - (int64_t)B.n * B.n * B.n));
    }
    pk->reg_bytes[0] = pk->reg_bytes[1] = pk->reg_bytes[2] = align256((size_t)off * esz);
    pk->reg_bytes[3] = align256((size_t)ioff * 8);

    // work list: tiles of active cells (variant 0 fits every valid pack)
    build_work(pk->blk, 0, pk->work);

    // leaf lookup per level, at `unit` granularity
    std::memset(&pk->L, 0, sizeof(pk->L));
    pk->L.unit = unit;
    pk->L.nlev = lmax + 1;
    int64_t tot = 0;
    for (int l = 0; l <= lmax; ++l) {
        pk->L.base[l] = tot;
        int64_t t = 1;
        for (int a = 0; a < 3; ++a) {
            pk->L.dim[l][a] = (int32_t)(((int64_t)p.nroot[a] << l) / unit);
            t *= pk->L.dim[l][a];
        }
        tot += t;
    }
    if (tot > (int64_t)1 << 28) { delete pk; return Z4C_EUNSUPPORTED; }
    pk->map.assign((size_t)tot, -1);
    for (int b = 0; b < nblocks; ++b) {
        const z4c_block& B = blocks[b];
        const int l = B.level, nu = B.n / unit;
        for (int z = 0; z < nu; ++z)
            for (int y = 0; y < nu; ++y)
                for (int x = 0; x < nu; ++x) {
                    const int64_t X = B.ilo[0] / unit + x, Y = B.ilo[1] / unit + y, Z = B.ilo[2] / unit + z;
                    pk->map[pk->L.base[l] + (Z * pk->L.dim[l][1] + Y) * pk->L.dim[l][0] + X] = b;
                }
    }

    // the cross-level lists put the items of ghosts the stage path leaves
    // alone (vmask) last
    build_virtual_halos(pk);
    if (pk->multilevel) {
        const int rc = build_xlevel(pk);
        if (rc) { delete pk; return rc; }
    }

    // workspace
    size_t o = 0;
    pk->ws_blocks = o; o = align256(o + sizeof(BlockDev) * nblocks);
    pk->ws_work = o;   o = align256(o + sizeof(WorkItem) * pk->work.size());
    pk->ws_map = o;    o = align256(o + sizeof(int32_t) * pk->map.size());
    pk->ws_part = o;   o = align256(o + sizeof(double) * 16 * pk->work.size());
    pk->ws_first = o;  o = align256(o + sizeof(int32_t) * (nblocks + 1));
    pk->ws_feat = o;   o = align256(o + sizeof(double) * 16 * nblocks);
    pk->ws_x = o;      o = align256(o + sizeof(float) * 16 * nblocks);
    pk->ws_y = o;      o = align256(o + sizeof(float) * nblocks);
    pk->ws_lflag = o;  o = align256(o + 2 * (size_t)nblocks);
    pk->ws_xfer = o;   o = align256(o + sizeof(XferItem) * pk->xfer.size());
    pk->ws_prol = o;   o = align256(o + sizeof(ProlongItem) * pk->prol.size());
    pk->ws_pgrp = o;   o = align256(o + sizeof(ProlongGroup) * pk->pgrp.size());
    pk->ws_w = o;      o = align256(o + sizeof(double) * 80);
    pk->ws_shadow = o; o = align256(o + esz * (size_t)pk->shadow_elems);
    pk->ws_islice = o; o = align256(o + sizeof(ImageSlice) * pk->islice.size());
    pk->ws_image = o;  o = align256(o + esz * (size_t)pk->image_elems);
    pk->ws_regrid = o; o = align256(o + sizeof(RegridDesc) * nblocks);
    pk->ws_vnbr = o;   o = align256(o + sizeof(int64_t) * 27 * nblocks);
    pk->ws_vmask = o;  o = align256(o + sizeof(uint32_t) * nblocks);
    pk->ws_cmask = o;  o = align256(o + sizeof(uint32_t) * 2 * nblocks);
    pk->ws_pmask = o;  o = align256(o + sizeof(uint32_t) * nblocks);
    pk->ws_omask = o;  o = align256(o + sizeof(uint32_t) * nblocks);
    pk->ws_fskip = o;  o = align256(o + sizeof(uint32_t) * nblocks);
    pk->ws_track = o;  o = align256(o + sizeof(double) * 9 * Z4C_MAXTRACK);
    pk->ws_flag = o;   o = align256(o + sizeof(int32_t));
    pk->ws_total = o;
    pk->part_host.resize(16 * pk->work.size());
    pk->first_work.assign(nblocks + 1, 0);
    for (size_t w = 0; w < pk->work.size(); ++w) pk->first_work[pk->work[w].block + 1] = (int32_t)(w + 1);
    for (int b = 0; b < nblocks; ++b)
        if (pk->first_work[b + 1] < pk->first_work[b]) pk->first_work[b + 1] = pk->first_work[b];
    *out = pk;
    return Z4C_OK;
}

int z4c_pack_query(const z4c_pack* pk, z4c_layout* out)
{
    if (!pk || !out) return Z4C_EINVAL;
    for (int r = 0; r < Z4C_NREG; ++r) out->reg_bytes[r] = pk->reg_bytes[r];
    out->workspace_bytes = pk->ws_total;
    out->nblocks = (int64_t)pk->blk.size();
    out->zones = pk->zones;
    out->state_elem_bytes = pk->p.precision == Z4C_FP64 ? 8 : 4;
    out->nwork = (int32_t)pk->work.size();
    out->nxfer = (int64_t)pk->xfer.size();
    out->nprolong = (int64_t)pk->prol.size() + 8 * pk->nparent;
    return Z4C_OK;
}

int z4c_block_offset(const z4c_pack* pk, int32_t b, int64_t* state_off, int64_t* interior_off)
{
    if (!pk || b < 0 || b >= (int32_t)pk->blk.size()) return Z4C_EINVAL;
    if (state_off) *state_off = pk->bdev[b].off;
    if (interior_off) *interior_off = pk->bdev[b].ioff;
    return Z4C_OK;
}

int z4c_pack_bind(z4c_pack* pk, void* const regs[Z4C_NREG], void* workspace, size_t ws_bytes,
                  void* stream)
{
    if (!pk) return Z4C_EINVAL;
    if (!regs || !workspace) return fail(pk, Z4C_EINVAL, "null register or workspace pointer");
    if (ws_bytes < pk->ws_total) return fail(pk, Z4C_ENOMEM, "workspace too small: %zu < %zu", ws_bytes, pk->ws_total);
    for (int r = 0; r < Z4C_NREG; ++r) {
        if (!regs[r] || (reinterpret_cast<uintptr_t>(regs[r]) & 255))
            return fail(pk, Z4C_EINVAL, "register %d null or not 256-byte aligned", r);
    }
    if (reinterpret_cast<uintptr_t>(workspace) & 255) return fail(pk, Z4C_EINVAL, "workspace not 256-byte aligned");
    hipStream_t s = as_stream(stream);
    char* ws = static_cast<char*>(workspace);
    hipError_t e = hipMemcpyAsync(ws + pk->ws_blocks, pk->bdev.data(), sizeof(BlockDev) * pk->bdev.size(),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ws + pk->ws_work, pk->work.data(), sizeof(WorkItem) * pk->work.size(),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ws + pk->ws_map, pk->map.data(), sizeof(int32_t) * pk->map.size(),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ws + pk->ws_first, pk->first_work.data(), sizeof(int32_t) * pk->first_work.size(),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !pk->xfer.empty())
        e = hipMemcpyAsync(ws + pk->ws_xfer, pk->xfer.data(), sizeof(XferItem) * pk->xfer.size(),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !pk->prol.empty())
        e = hipMemcpyAsync(ws + pk->ws_prol, pk->prol.data(), sizeof(ProlongItem) * pk->prol.size(),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ws + pk->ws_vnbr, pk->vnbr.data(), sizeof(int64_t) * pk->vnbr.size(),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ws + pk->ws_vmask, pk->vmask.data(), sizeof(uint32_t) * pk->vmask.size(),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ws + pk->ws_cmask, pk->cmask.data(), sizeof(uint32_t) * pk->cmask.size(),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ws + pk->ws_pmask, pk->pmask.data(), sizeof(uint32_t) * pk->pmask.size(),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ws + pk->ws_omask, pk->omask.data(), sizeof(uint32_t) * pk->omask.size(),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ws + pk->ws_fskip, pk->fskip.data(), sizeof(uint32_t) * pk->fskip.size(),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !pk->islice.empty())
        e = hipMemcpyAsync(ws + pk->ws_islice, pk->islice.data(), sizeof(ImageSlice) * pk->islice.size(),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !pk->pgrp.empty())
        e = hipMemcpyAsync(ws + pk->ws_pgrp, pk->pgrp.data(), sizeof(ProlongGroup) * pk->pgrp.size(),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess && pk->multilevel) {
        double wt[80];
        for (int q = 0; q < 64; ++q) wt[q] = pk->rw[q];
        for (int q = 0; q < 16; ++q) wt[64 + q] = pk->pw[q];
        pk->wtab.assign(wt, wt + 80);
        e = hipMemcpyAsync(ws + pk->ws_w, pk->wtab.data(), sizeof(double) * 80, hipMemcpyHostToDevice, s);
    }
    if (e != hipSuccess) return fail(pk, Z4C_EDEVICE, "table upload: %s", hipGetErrorString(e));
    if (pk->multilevel && !pk->side) {
        // default priority, not synchronised with the legacy null stream
        e = hipStreamCreateWithFlags(&pk->side, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&pk->fork_ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&pk->join_ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            release_side(pk);
            return fail(pk, Z4C_EDEVICE, "side stream: %s", hipGetErrorString(e));
        }
    }
    // a step graph captured against the previous registers / workspace holds
    // their addresses in its kernel arguments: drop it, the next graph step
    // captures again
    drop_graphs(pk);
    for (int r = 0; r < Z4C_NREG; ++r) pk->reg[r] = regs[r];
    pk->ws = ws;
    pk->bound = true;
    pk->last_stage = 0;
    pk->err.clear();
    return Z4C_OK;
}

void z4c_pack_destroy(z4c_pack* pk)
{
    if (!pk) return;
    drop_graphs(pk);
    release_side(pk);
    for (auto& e : pk->ev) {
        hipEventDestroy(e.a);
        hipEventDestroy(e.b);
    }
    delete pk;
}

int z4c_profile(z4c_pack* pk, int32_t enable)
{
    if (!pk) return Z4C_EINVAL;
    pk->prof = enable != 0;
    return Z4C_OK;
}

int z4c_profile_read(z4c_pack* pk, double* out, int32_t reset)
{
    if (!pk || !out) return Z4C_EINVAL;
    hipError_t r = hipSuccess;
    for (auto& e : pk->ev) {
        float ms = 0.f;
        if (r == hipSuccess) r = hipEventSynchronize(e.b);
        if (r == hipSuccess) r = hipEventElapsedTime(&ms, e.a, e.b);
        hipEventDestroy(e.a);
        hipEventDestroy(e.b);
        if (r != hipSuccess) continue;  // keep destroying the rest
        pk->prof_acc[2 * e.kind] += ms;
        pk->prof_acc[2 * e.kind + 1] += 1.0;
    }
    pk->ev.clear();
    if (r != hipSuccess) return fail(pk, Z4C_EDEVICE, "profile: %s", hipGetErrorString(r));
    for (int q = 0; q < 6; ++q) out[q] = pk->prof_acc[q];
    if (reset)
        for (int q = 0; q < 6; ++q) pk->prof_acc[q] = 0.0;
    return Z4C_OK;
}

const char* z4c_last_error(const z4c_pack* pk) { return pk ? pk->err.c_str() : "null pack"; }

// ghost fill; `virt` leaves the ghost cells of virtual-halo directions
// (read directly from neighbours by the stage kernel) unwritten
// virt: leave the virtual (read in place) directions alone; pushed: also
// those the previous stage kernel wrote into the register
static int fill_impl(z4c_pack* pk, int32_t reg, void* stream, bool virt, bool pushed = false)
{
    if (pk->p.bc == Z4C_BC_USER) return Z4C_OK;
    FillArgs a;
    a.skip = virt ? reinterpret_cast<const uint32_t*>(pk->ws + pk->ws_vmask) : nullptr;
    a.skip2 = (virt && pushed) ? reinterpret_cast<const uint32_t*>(pk->ws + pk->ws_fskip) : nullptr;
    // every ghost cell the same-level fill would write is read in place or
    // was written by the stage kernel that produced the register
    const bool same_empty = virt && pushed && pk->fill_pushed_empty;
    a.reg = pk->reg[reg];
    a.blocks = reinterpret_cast<const BlockDev*>(pk->ws + pk->ws_blocks);
    a.map = reinterpret_cast<const int32_t*>(pk->ws + pk->ws_map);
    a.L = pk->L;
    a.g = pk->p.nghost;
    a.bc = pk->p.bc;
    for (int d = 0; d < 3; ++d) a.nroot[d] = pk->p.nroot[d];
    a.maxghost = pk->maxghost;
    ProfScope ps(pk, as_stream(stream), 1);
    const hipStream_t s = as_stream(stream);
    // The same-level copies and the cross-level chain (restriction, copies
    // into coarse ghosts and shadow boxes, prolongation) read only active
    // cells, except the prolongation, which reads the shadow boxes, and they
    // write disjoint cells.  On multi-level packs the side stream takes the
    // same-level copies and the shadow-box copies from active cells, the
    // stream itself the restriction and the copies from images; the
    // prolongation waits for both.
    const bool fork = pk->multilevel && pk->side;
    hipError_t e = hipSuccess;
    XlevelArgs x = {};
    if (pk->multilevel) {
        x.reg = pk->reg[reg];
        x.shadow = pk->ws + pk->ws_shadow;
        x.image = pk->ws + pk->ws_image;
        x.islice = reinterpret_cast<const ImageSlice*>(pk->ws + pk->ws_islice);
        x.nislice = (int64_t)pk->islice.size();
        x.blocks = a.blocks;
        x.xfer = reinterpret_cast<const XferItem*>(pk->ws + pk->ws_xfer);
        x.prol = reinterpret_cast<const ProlongItem*>(pk->ws + pk->ws_prol);
        x.rw = reinterpret_cast<const double*>(pk->ws + pk->ws_w);
        x.pw = x.rw + 64;
        x.nxfer = virt ? pk->nxfer_stage : (int64_t)pk->xfer.size();
        x.nprol = virt ? pk->nprol_stage : (int64_t)pk->prol.size();
        x.pgrp = reinterpret_cast<const ProlongGroup*>(pk->ws + pk->ws_pgrp);
        x.npgrp = virt ? pk->npgrp_stage : (int64_t)pk->pgrp.size();
        x.npts = pk->p.nghost + 1;
    }
    const XferItem* xf = x.xfer;
    const int64_t nall = x.nxfer, ndir = pk->nxfer_direct;
    if (fork) {
        e = hipEventRecord(pk->fork_ev, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(pk->side, pk->fork_ev, 0);
        if (e == hipSuccess && !same_empty) e = launch_fill(pk->p.precision, a, (int)pk->blk.size(), pk->side);
        if (e == hipSuccess) {
            x.xfer = xf;
            x.nxfer = ndir;
            e = launch_xlevel(pk->p.precision, x, pk->side, XL_XFER);
        }
        if (e == hipSuccess) e = hipEventRecord(pk->join_ev, pk->side);
        if (e == hipSuccess) {
            x.xfer = xf + ndir;
            x.nxfer = nall - ndir;
            e = launch_xlevel(pk->p.precision, x, s, XL_RESTRICT | XL_XFER);
        }
        // join even after a failed launch, so that a capture on s stays closed
        const hipError_t j = hipStreamWaitEvent(s, pk->join_ev, 0);
        if (e == hipSuccess) e = j;
        if (e == hipSuccess) e = launch_xlevel(pk->p.precision, x, s, XL_PROLONG);
    } else {
        if (!same_empty) e = launch_fill(pk->p.precision, a, (int)pk->blk.size(), s);
        if (e == hipSuccess && pk->multilevel)
            e = launch_xlevel(pk->p.precision, x, s, XL_RESTRICT | XL_XFER | XL_PROLONG);
    }
    if (e != hipSuccess) return fail(pk, Z4C_EDEVICE, "ghost fill launch: %s", hipGetErrorString(e));
    return Z4C_OK;
}

int z4c_fill_ghosts(z4c_pack* pk, int32_t reg, void* stream)
{
    if (!pk) return Z4C_EINVAL;
    if (reg < Z4C_REG_U || reg > Z4C_REG_S2) return fail(pk, Z4C_EINVAL, "bad register %d", reg);
    if (!pk->bound) return fail(pk, Z4C_ESTATE, "pack not bound");
    return fill_impl(pk, reg, stream, false);
}

static StageArgs stage_args(z4c_pack* pk)
{
    StageArgs a;
    std::memset(&a, 0, sizeof(a));
    a.nwork = (int32_t)pk->work.size();
    a.persistent = pk->persistent ? 1 : 0;
    a.blocks = reinterpret_cast<const BlockDev*>(pk->ws + pk->ws_blocks);
    a.work = reinterpret_cast<const WorkItem*>(pk->ws + pk->ws_work);
    a.P = dev_params(pk->p);
    a.g = pk->p.nghost;
    a.A = static_cast<double*>(pk->reg[Z4C_REG_A]);
    a.U = pk->reg[Z4C_REG_U];
    a.vnbr = reinterpret_cast<const int64_t*>(pk->ws + pk->ws_vnbr);
    a.cmask = reinterpret_cast<const uint32_t*>(pk->ws + pk->ws_cmask);
    a.pmask = reinterpret_cast<const uint32_t*>(pk->ws + pk->ws_pmask);
    a.omask = reinterpret_cast<const uint32_t*>(pk->ws + pk->ws_omask);
    a.virt_x = pk->virt_x;
    return a;
}

int z4c_rhs(z4c_pack* pk, int32_t src_reg, void* rhs_out, void* stream)
{
    if (!pk) return Z4C_EINVAL;
    if (src_reg < Z4C_REG_U || src_reg > Z4C_REG_S2) return fail(pk, Z4C_EINVAL, "bad register %d", src_reg);
    if (!rhs_out) return fail(pk, Z4C_EINVAL, "null rhs_out");
    if (!pk->bound) return fail(pk, Z4C_ESTATE, "pack not bound");
    StageArgs a = stage_args(pk);
    a.src = pk->reg[src_reg];
    a.rhs_out = static_cast<double*>(rhs_out);
    a.stage = 0;
    const int grid = pk->persistent ? pk->grid_persistent : stage_grid(pk->work.size());
    hipError_t e = launch_stage(pk->p.fd_order / 2, pk->p.precision, pk->variant, a, grid, as_stream(stream));
    if (e != hipSuccess) return fail(pk, Z4C_EDEVICE, "rhs launch: %s", hipGetErrorString(e));
    return Z4C_OK;
}

// chained: the stage kernel that ran last on the pack wrote the stage's input
// register, so the ghosts it wrote (pushed x-face ghosts, outflow x faces)
// are current and the fill leaves them alone
static int rk4_stage_impl(z4c_pack* pk, int32_t stage, double dt, void* stream, bool chained)
{
    static const int src_of[5] = {0, Z4C_REG_U, Z4C_REG_S1, Z4C_REG_S2, Z4C_REG_S1};
    static const int dst_of[5] = {0, Z4C_REG_S1, Z4C_REG_S2, Z4C_REG_S1, Z4C_REG_U};
    int rc = fill_impl(pk, src_of[stage], stream, true, chained);
    pk->last_stage = 0;
    if (rc) return rc;
    if (pk->ntrack > 0) {
        hipError_t te = track_stage(pk, stage, src_of[stage], dt, as_stream(stream));
        if (te != hipSuccess) return fail(pk, Z4C_EDEVICE, "tracker launch: %s", hipGetErrorString(te));
    }
    StageArgs a = stage_args(pk);
    a.src = pk->reg[src_of[stage]];
    a.dst = pk->reg[dst_of[stage]];
    a.dt = dt;
    a.stage = stage;
    ProfScope ps(pk, as_stream(stream), 0);
    const int grid = pk->persistent ? pk->grid_persistent : stage_grid(pk->work.size());
    hipError_t e = launch_stage(pk->p.fd_order / 2, pk->p.precision, pk->variant, a, grid, as_stream(stream));
    if (e != hipSuccess) return fail(pk, Z4C_EDEVICE, "stage launch: %s", hipGetErrorString(e));
    pk->last_stage = stage;
    return Z4C_OK;
}

int z4c_rk4_stage(z4c_pack* pk, int32_t stage, double dt, void* stream)
{
    if (!pk) return Z4C_EINVAL;
    if (stage < 1 || stage > 4) return fail(pk, Z4C_EINVAL, "bad stage %d", stage);
    if (!std::isfinite(dt)) return fail(pk, Z4C_EINVAL, "dt not finite");
    if (!pk->bound) return fail(pk, Z4C_ESTATE, "pack not bound");
    // stages 2-4 read the register the previous stage wrote when that stage
    // ran last; stage 1 reads U, which the caller may have changed since
    return rk4_stage_impl(pk, stage, dt, stream, stage >= 2 && pk->last_stage == stage - 1);
}

// with Z4C_FLAG_CHECK_FINITE: every value of U's active cells finite?
static int check_finite(z4c_pack* pk, hipStream_t s)
{
    FiniteArgs a;
    a.src = pk->reg[Z4C_REG_U];
    a.blocks = reinterpret_cast<const BlockDev*>(pk->ws + pk->ws_blocks);
    a.work = reinterpret_cast<const WorkItem*>(pk->ws + pk->ws_work);
    a.flag = reinterpret_cast<int32_t*>(pk->ws + pk->ws_flag);
    a.g = pk->p.nghost;
    int32_t bad = 0;
    hipError_t e = launch_check_finite(pk->p.precision, a, (int)pk->work.size(), s);
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, a.flag, sizeof(bad), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(pk, Z4C_EDEVICE, "finite check: %s", hipGetErrorString(e));
    return bad ? fail(pk, Z4C_ENONFINITE, "non-finite value in U after the step") : Z4C_OK;
}

static int rk4_steps(z4c_pack* pk, double dt, int32_t nsteps, void* stream);

int z4c_rk4_step(z4c_pack* pk, double dt, int32_t nsteps, void* stream)
{
    const int rc = rk4_steps(pk, dt, nsteps, stream);
    if (rc || !(pk->p.flags & Z4C_FLAG_CHECK_FINITE) || nsteps == 0) return rc;
    return check_finite(pk, as_stream(stream));
}

static int rk4_steps(z4c_pack* pk, double dt, int32_t nsteps, void* stream)
{
    if (!pk) return Z4C_EINVAL;
    if (nsteps < 0) return fail(pk, Z4C_EINVAL, "negative nsteps");
    if (!std::isfinite(dt)) return fail(pk, Z4C_EINVAL, "dt not finite");
    if (!pk->bound) return fail(pk, Z4C_ESTATE, "pack not bound");
    hipStream_t s = as_stream(stream);
    if ((pk->p.flags & Z4C_FLAG_GRAPH) && s != nullptr && nsteps > 0) {
        // the four stages (ghost fills included) captured once, replayed: the
        // first step of a call from `graph`, later ones from `graph2`, whose
        // stage 1 finds the ghosts of U the previous step's stage 4 wrote
        if (!pk->gexec || !pk->gexec2 || pk->graph_dt != dt || pk->graph_stream != s) {
            drop_graphs(pk);
            const bool prof = pk->prof;
            pk->prof = false;
            for (int g = 0; g < 2; ++g) {
                hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
                if (e != hipSuccess) {
                    pk->prof = prof;
                    drop_graphs(pk);
                    return fail(pk, Z4C_EDEVICE, "capture: %s", hipGetErrorString(e));
                }
                int rc = Z4C_OK;
                for (int st = 1; st <= 4 && rc == Z4C_OK; ++st)
                    rc = st == 1 ? rk4_stage_impl(pk, 1, dt, stream, g == 1) : z4c_rk4_stage(pk, st, dt, stream);
                hipGraph_t gr = nullptr;
                e = hipStreamEndCapture(s, &gr);
                if (rc == Z4C_OK && e != hipSuccess) rc = fail(pk, Z4C_EDEVICE, "end capture: %s", hipGetErrorString(e));
                hipGraphExec_t ex = nullptr;
                if (rc == Z4C_OK) {
                    e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
                    if (e != hipSuccess) rc = fail(pk, Z4C_EDEVICE, "instantiate: %s", hipGetErrorString(e));
                }
                if (rc) {
                    if (gr) hipGraphDestroy(gr);
                    pk->prof = prof;
                    drop_graphs(pk);
                    return rc;
                }
                (g ? pk->graph2 : pk->graph) = gr;
                (g ? pk->gexec2 : pk->gexec) = ex;
            }
            pk->prof = prof;
            pk->graph_dt = dt;
            pk->graph_stream = s;
        }
        for (int n = 0; n < nsteps; ++n) {
            ProfScope ps(pk, s, 2);
            hipError_t e = hipGraphLaunch(n ? pk->gexec2 : pk->gexec, s);
            if (e != hipSuccess) {
                pk->last_stage = 0;
                return fail(pk, Z4C_EDEVICE, "graph launch: %s", hipGetErrorString(e));
            }
            pk->last_stage = 4;
        }
        return Z4C_OK;
    }
    // within the call, a step's stage 1 reads the U the previous step's
    // stage 4 wrote
    for (int n = 0; n < nsteps; ++n)
        for (int st = 1; st <= 4; ++st) {
            const bool chained = st >= 2 ? pk->last_stage == st - 1 : (n > 0 && pk->last_stage == 4);
            int rc = rk4_stage_impl(pk, st, dt, stream, chained);
            if (rc) return rc;
        }
    return Z4C_OK;
}

int z4c_set_variant(z4c_pack* pk, int32_t variant, int32_t persistent, void* stream)
{
    if (!pk) return Z4C_EINVAL;
    if (variant < 0 || variant >= NVARIANT) return fail(pk, Z4C_EINVAL, "bad variant %d", variant);
    std::vector<WorkItem> w;
    if (!build_work(pk->blk, variant, w)) return fail(pk, Z4C_EUNSUPPORTED, "tile shape %d does not divide the blocks", variant);
    if (w.size() != pk->work.size()) return fail(pk, Z4C_EINVAL, "work size mismatch");
    pk->work = w;
    pk->variant = variant;
    pk->persistent = persistent != 0;
    if (pk->persistent) {
        int dev = 0, ncu = 0;
        hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1) ncu = 256;
        const int occ = stage_occupancy(pk->p.fd_order / 2, pk->p.precision, variant);
        pk->grid_persistent = std::min<int>((int)pk->work.size(), ncu * occ);
    }
    drop_graphs(pk);
    if (pk->bound) {
        hipError_t e = hipMemcpyAsync(pk->ws + pk->ws_work, pk->work.data(), sizeof(WorkItem) * pk->work.size(),
                                      hipMemcpyHostToDevice, as_stream(stream));
        if (e == hipSuccess) e = hipStreamSynchronize(as_stream(stream));
        if (e != hipSuccess) return fail(pk, Z4C_EDEVICE, "work upload: %s", hipGetErrorString(e));
    }
    return Z4C_OK;
}

int z4c_autotune(z4c_pack* pk, int32_t reps, double* times_ms, int32_t* chosen, void* stream)
{
    if (!pk) return Z4C_EINVAL;
    if (reps < 1 || !chosen) return fail(pk, Z4C_EINVAL, "bad autotune arguments");
    if (!pk->bound) return fail(pk, Z4C_ESTATE, "pack not bound");
    hipStream_t s = as_stream(stream);
    int rc = Z4C_OK;
    double best = INFINITY;
    int bv = -1, bp = 0;
    for (int v = 0; v < NVARIANT; ++v)
        for (int per = 0; per <= 1; ++per) {
            const int q = 2 * v + per;
            if (times_ms) times_ms[q] = -1.0;
            std::vector<WorkItem> w;
            if (!build_work(pk->blk, v, w)) continue;
            rc = z4c_set_variant(pk, v, per, stream);
            if (rc) return rc;
            hipEvent_t e0, e1;
            if (hipEventCreate(&e0) != hipSuccess) return fail(pk, Z4C_EDEVICE, "autotune events");
            if (hipEventCreate(&e1) != hipSuccess) {
                hipEventDestroy(e0);
                return fail(pk, Z4C_EDEVICE, "autotune events");
            }
            // RK stage 1 with dt = 0: writes only S1 and the accumulator
            rc = z4c_rk4_stage(pk, 1, 0.0, stream);  // warm-up
            hipEventRecord(e0, s);
            for (int r = 0; r < reps && rc == Z4C_OK; ++r) rc = z4c_rk4_stage(pk, 1, 0.0, stream);
            hipEventRecord(e1, s);
            hipError_t e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            hipEventDestroy(e0);
            hipEventDestroy(e1);
            if (rc) return rc;
            if (e != hipSuccess) return fail(pk, Z4C_EDEVICE, "autotune timing: %s", hipGetErrorString(e));
            const double t = ms / reps;
            if (times_ms) times_ms[q] = t;
            if (t < best) { best = t; bv = v; bp = per; }
        }
    if (bv < 0) return fail(pk, Z4C_EUNSUPPORTED, "no tile shape fits");
    *chosen = 2 * bv + bp;
    return z4c_set_variant(pk, bv, bp, stream);
}

// Autotuner cache: one line per tuned configuration,
//   {"key": "<arch>|order=<o>|prec=<p>|g=<g>|levels=<l>|n=<n>x<count>,...", "variant": v, "persistent": 0|1, "ms": t}
// keyed by what the choice depends on (device architecture, FD order,
// storage precision, ghost depth, number of levels, block sizes and counts).
static std::string tune_key(const z4c_pack* pk)
{
    int dev = 0;
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
    std::map<int, int> sizes;
    int lmax = 0;
    for (const z4c_block& b : pk->blk) {
        sizes[b.n] += 1;
        lmax = std::max(lmax, (int)b.level);
    }
    std::string k = arch + "|order=" + std::to_string(pk->p.fd_order) + "|prec=" + std::to_string(pk->p.precision) +
                    "|g=" + std::to_string(pk->p.nghost) + "|levels=" + std::to_string(lmax + 1) + "|n=";
    bool first = true;
    for (const auto& e : sizes) {
        if (!first) k += ",";
        k += std::to_string(e.first) + "x" + std::to_string(e.second);
        first = false;
    }
    return k;
}

int z4c_autotune_cached(z4c_pack* pk, const char* path, int32_t reps, double* times_ms, int32_t* chosen,
                        int32_t* from_cache, void* stream)
{
    if (!pk) return Z4C_EINVAL;
    if (!path || !chosen) return fail(pk, Z4C_EINVAL, "null cache path or output");
    if (!pk->bound) return fail(pk, Z4C_ESTATE, "pack not bound");
    const std::string key = tune_key(pk);
    if (from_cache) *from_cache = 0;
    if (FILE* f = std::fopen(path, "r")) {
        char line[1024];
        int hit_v = -1, hit_p = 0;
        while (std::fgets(line, sizeof(line), f)) {
            const char* kq = std::strstr(line, "\"key\": \"");
            if (!kq) continue;
            kq += 8;
            const char* ke = std::strchr(kq, '"');
            if (!ke || std::string(kq, ke) != key) continue;
            const char* vq = std::strstr(ke, "\"variant\": ");
            const char* pq = std::strstr(ke, "\"persistent\": ");
            int v = -1, per = 0;
            if (vq && pq && std::sscanf(vq + 11, "%d", &v) == 1 && std::sscanf(pq + 14, "%d", &per) == 1 &&
                v >= 0 && v < NVARIANT && (per == 0 || per == 1)) {
                hit_v = v;   // the last record of a key wins
                hit_p = per;
            }
        }
        std::fclose(f);
        if (hit_v >= 0) {
            const int rc = z4c_set_variant(pk, hit_v, hit_p, stream);
            if (rc == Z4C_OK) {
                if (times_ms)
                    for (int q = 0; q < 2 * NVARIANT; ++q) times_ms[q] = -1.0;
                *chosen = 2 * hit_v + hit_p;
                if (from_cache) *from_cache = 1;
                return Z4C_OK;
            }
            // a record that no longer applies (e.g. the tile does not divide
            // the blocks) falls through to timing
        }
    }
    double t[2 * NVARIANT];
    int rc = z4c_autotune(pk, reps, t, chosen, stream);
    if (rc) return rc;
    if (times_ms)
        for (int q = 0; q < 2 * NVARIANT; ++q) times_ms[q] = t[q];
    if (FILE* f = std::fopen(path, "a")) {
        std::fprintf(f, "{\"key\": \"%s\", \"variant\": %d, \"persistent\": %d, \"ms\": %.6g}\n", key.c_str(),
                     *chosen / 2, *chosen % 2, t[*chosen]);
        std::fclose(f);
    } else {
        return fail(pk, Z4C_EINVAL, "cannot write autotune cache %s", path);
    }
    return Z4C_OK;
}

static int run_diag(z4c_pack* pk, int32_t reg, int mode, void* per_zone, const double* centres,
                    int ncentres, double r_exc, void* stream)
{
    if (reg < Z4C_REG_U || reg > Z4C_REG_S2) return fail(pk, Z4C_EINVAL, "bad register %d", reg);
    if (!pk->bound) return fail(pk, Z4C_ESTATE, "pack not bound");
    int rc = z4c_fill_ghosts(pk, reg, stream);
    if (rc) return rc;
    DiagArgs a;
    std::memset(&a, 0, sizeof(a));
    a.src = pk->reg[reg];
    a.per_zone = static_cast<double*>(per_zone);
    a.partial = reinterpret_cast<double*>(pk->ws + pk->ws_part);
    a.blocks = reinterpret_cast<const BlockDev*>(pk->ws + pk->ws_blocks);
    a.work = reinterpret_cast<const WorkItem*>(pk->ws + pk->ws_work);
    a.P = dev_params(pk->p);
    for (int d = 0; d < 3; ++d) a.lo[d] = pk->p.lo[d];
    a.ncentres = ncentres;
    a.mode = mode;
    for (int e = 0; e < ncentres; ++e)
        for (int d = 0; d < 3; ++d) a.centres[e][d] = centres[3 * e + d];
    a.r_exc = r_exc;
    a.g = pk->p.nghost;
    hipStream_t s = as_stream(stream);
    hipError_t e = launch_diag(pk->p.fd_order / 2, pk->p.precision, a, (int)pk->work.size(), s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(pk->part_host.data(), a.partial, sizeof(double) * pk->part_host.size(),
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(pk, Z4C_EDEVICE, "diagnostics: %s", hipGetErrorString(e));
    return Z4C_OK;
}

int z4c_constraints(z4c_pack* pk, int32_t reg, void* per_zone_out, const z4c_norm_region* region,
                    double* norms_out, void* stream)
{
    if (!pk) return Z4C_EINVAL;
    if (!norms_out) return fail(pk, Z4C_EINVAL, "null norms_out");
    int nc = 0;
    double cen[24] = {0};
    double rexc = 0.0;
    if (region) {
        if (region->ncentres < 0 || region->ncentres > 8 || !(region->r_exc >= 0.0))
            return fail(pk, Z4C_EINVAL, "bad norm region");
        nc = region->ncentres;
        for (int e = 0; e < nc; ++e)
            for (int d = 0; d < 3; ++d) cen[3 * e + d] = region->centres[e][d];
        rexc = region->r_exc;
    }
    int rc = run_diag(pk, reg, 0, per_zone_out, cen, nc, rexc, stream);
    if (rc) return rc;
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (size_t w = 0; w < pk->work.size(); ++w) {
        const double* q = &pk->part_host[8 * w];
        s[0] += q[0]; s[1] = std::max(s[1], q[1]); s[2] += q[2]; s[3] = std::max(s[3], q[3]);
        s[4] += q[4]; s[5] += q[5]; s[6] += q[6];
    }
    const double vol = s[6];
    norms_out[0] = vol > 0 ? std::sqrt(s[0] / vol) : 0.0;
    norms_out[1] = s[1];
    norms_out[2] = vol > 0 ? std::sqrt(s[2] / vol) : 0.0;
    norms_out[3] = s[3];
    norms_out[4] = vol > 0 ? std::sqrt(s[4] / vol) : 0.0;
    norms_out[5] = vol > 0 ? std::sqrt(s[5] / vol) : 0.0;
    return Z4C_OK;
}

int z4c_refine_flags(z4c_pack* pk, int32_t reg, const z4c_refine_params* rp, int8_t* flags_out,
                     void* stream)
{
    if (!pk) return Z4C_EINVAL;
    if (!rp || !flags_out) return fail(pk, Z4C_EINVAL, "null argument");
    if (rp->criterion < Z4C_CRIT_CHI_MIN || rp->criterion > Z4C_CRIT_RADIUS)
        return fail(pk, Z4C_EINVAL, "bad criterion %d", rp->criterion);
    int rc = run_diag(pk, reg, 1, nullptr, rp->centre, 1, 0.0, stream);
    if (rc) return rc;
    const size_t nb = pk->blk.size();
    std::vector<double> cmin(nb, INFINITY), gmax(nb, 0.0), rmin(nb, INFINITY);
    for (size_t w = 0; w < pk->work.size(); ++w) {
        const double* q = &pk->part_host[8 * w];
        const int b = pk->work[w].block;
        cmin[b] = std::min(cmin[b], q[0]);
        gmax[b] = std::max(gmax[b], q[1]);
        rmin[b] = std::min(rmin[b], q[2]);
    }
    for (size_t b = 0; b < nb; ++b) {
        int f = 0;
        const int lev = pk->blk[b].level;
        if (rp->criterion == Z4C_CRIT_CHI_MIN) {
            if (cmin[b] < rp->chi_thr) f = 1;
            else if (cmin[b] > 1.5 * rp->chi_thr) f = -1;
        } else if (rp->criterion == Z4C_CRIT_DCHI_MAX) {
            if (gmax[b] > rp->dchi_thr) f = 1;
            else if (gmax[b] < 0.5 * rp->dchi_thr) f = -1;
        } else {
            f = (rmin[b] < rp->radius && lev < rp->radius_level) ? 1 : 0;
        }
        if (f > 0 && lev >= rp->level_max) f = 0;
        if (f < 0 && lev == 0) f = 0;
        flags_out[b] = (int8_t)f;
    }
    return Z4C_OK;
}

int z4c_features(z4c_pack* pk, int32_t reg, void* feat_dev, double* feat_host, void* stream)
{
    if (!pk) return Z4C_EINVAL;
    if (reg < Z4C_REG_U || reg > Z4C_REG_S2) return fail(pk, Z4C_EINVAL, "bad register %d", reg);
    if (!pk->bound) return fail(pk, Z4C_ESTATE, "pack not bound");
    int rc = z4c_fill_ghosts(pk, reg, stream);
    if (rc) return rc;
    FeatArgs a;
    a.src = pk->reg[reg];
    a.blocks = reinterpret_cast<const BlockDev*>(pk->ws + pk->ws_blocks);
    a.work = reinterpret_cast<const WorkItem*>(pk->ws + pk->ws_work);
    a.first_work = reinterpret_cast<const int32_t*>(pk->ws + pk->ws_first);
    a.partial = reinterpret_cast<double*>(pk->ws + pk->ws_part);
    a.feat = feat_dev ? static_cast<double*>(feat_dev) : reinterpret_cast<double*>(pk->ws + pk->ws_feat);
    a.g = pk->p.nghost;
    a.nblocks = (int32_t)pk->blk.size();
    hipStream_t s = as_stream(stream);
    hipError_t e = launch_features(pk->p.fd_order / 2, pk->p.precision, a, (int)pk->work.size(), s);
    if (e == hipSuccess && feat_host) {
        e = hipMemcpyAsync(feat_host, a.feat, sizeof(double) * 16 * pk->blk.size(), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    if (e != hipSuccess) return fail(pk, Z4C_EDEVICE, "features: %s", hipGetErrorString(e));
    return Z4C_OK;
}

int z4c_pack_inject_2h(z4c_pack* ph, int32_t reg_h, z4c_pack* p2, int32_t reg_2h, void* stream)
{
    if (!ph || !p2) return Z4C_EINVAL;
    if (reg_h < Z4C_REG_U || reg_h > Z4C_REG_S2 || reg_2h < Z4C_REG_U || reg_2h > Z4C_REG_S2)
        return fail(ph, Z4C_EINVAL, "bad register");
    if (!ph->bound || !p2->bound) return fail(ph, Z4C_ESTATE, "pack not bound");
    if (ph->blk.size() != p2->blk.size() || ph->p.precision != p2->p.precision)
        return fail(ph, Z4C_EINVAL, "2h pack does not match");
    int maxc = 0;
    for (size_t b = 0; b < ph->blk.size(); ++b) {
        const z4c_block &F = ph->blk[b], &C2 = p2->blk[b];
        if (C2.n * 2 != F.n || C2.level != F.level) return fail(ph, Z4C_EINVAL, "2h block %zu mismatch", b);
        for (int a = 0; a < 3; ++a)
            if (C2.ilo[a] * 2 != F.ilo[a]) return fail(ph, Z4C_EINVAL, "2h block %zu corner mismatch", b);
        maxc = std::max(maxc, C2.n * C2.n * C2.n);
    }
    InjectArgs a;
    a.src = ph->reg[reg_h];
    a.dst = p2->reg[reg_2h];
    a.blocks1 = reinterpret_cast<const BlockDev*>(ph->ws + ph->ws_blocks);
    a.blocks2 = reinterpret_cast<const BlockDev*>(p2->ws + p2->ws_blocks);
    a.g1 = ph->p.nghost;
    a.g2 = p2->p.nghost;
    hipError_t e = launch_inject(ph->p.precision, a, (int)ph->blk.size(), maxc, as_stream(stream));
    if (e != hipSuccess) return fail(ph, Z4C_EDEVICE, "inject: %s", hipGetErrorString(e));
    return Z4C_OK;
}

int z4c_labels(z4c_pack* ph, const void* rhs_h, z4c_pack* p2, const void* rhs_2h, double* labels_out,
               void* stream)
{
    if (!ph || !p2) return Z4C_EINVAL;
    if (!rhs_h || !rhs_2h || !labels_out) return fail(ph, Z4C_EINVAL, "null argument");
    if (!ph->bound || !p2->bound) return fail(ph, Z4C_ESTATE, "pack not bound");
    if (ph->blk.size() != p2->blk.size()) return fail(ph, Z4C_EINVAL, "2h pack does not match");
    for (size_t b = 0; b < ph->blk.size(); ++b)
        if (p2->blk[b].n * 2 != ph->blk[b].n) return fail(ph, Z4C_EINVAL, "2h block %zu mismatch", b);
    LabelArgs a;
    a.rhs1 = static_cast<const double*>(rhs_h);
    a.rhs2 = static_cast<const double*>(rhs_2h);
    a.blocks1 = reinterpret_cast<const BlockDev*>(ph->ws + ph->ws_blocks);
    a.blocks2 = reinterpret_cast<const BlockDev*>(p2->ws + p2->ws_blocks);
    a.work2 = reinterpret_cast<const WorkItem*>(p2->ws + p2->ws_work);
    a.partial = reinterpret_cast<double*>(p2->ws + p2->ws_part);
    hipStream_t s = as_stream(stream);
    hipError_t e = launch_labels(a, (int)p2->work.size(), s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p2->part_host.data(), a.partial, sizeof(double) * p2->work.size(),
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(ph, Z4C_EDEVICE, "labels: %s", hipGetErrorString(e));
    const size_t nb = ph->blk.size();
    std::vector<double> sum(nb, 0.0);
    for (size_t w = 0; w < p2->work.size(); ++w) sum[p2->work[w].block] += p2->part_host[w];
    for (size_t b = 0; b < nb; ++b) {
        const double n3 = std::pow((double)p2->blk[b].n, 3);
        labels_out[b] = std::log10(std::sqrt(sum[b] / (NF * n3)) + 1e-30);
    }
    return Z4C_OK;
}

int z4c_feature_stats(const void* raw, int32_t B, void* stats, void* stream)
{
    if (!raw || !stats || B < 1) return Z4C_EINVAL;
    return launch_feat_stats(static_cast<const double*>(raw), B, static_cast<double*>(stats),
                             as_stream(stream)) == hipSuccess ? Z4C_OK : Z4C_EDEVICE;
}

int z4c_mlp_normalize(const void* raw, int32_t B, const void* stats, void* X, void* stream)
{
    if (!raw || !stats || !X || B < 1) return Z4C_EINVAL;
    return launch_normalize(static_cast<const double*>(raw), B, static_cast<const double*>(stats),
                            static_cast<float*>(X), as_stream(stream)) == hipSuccess ? Z4C_OK : Z4C_EDEVICE;
}

int z4c_mlp_forward(const void* params, const void* X, int32_t B, void* Y, void* cache, void* stream)
{
    if (!params || !X || !Y || B < 1) return Z4C_EINVAL;
    return launch_mlp_forward(static_cast<const float*>(params), static_cast<const float*>(X), B,
                              static_cast<float*>(Y), static_cast<float*>(cache),
                              as_stream(stream)) == hipSuccess ? Z4C_OK : Z4C_EDEVICE;
}

int z4c_mlp_backward(const void* params, const void* X, const void* Y, const void* T, const void* cache,
                     int32_t B, void* grad, void* loss, void* work, void* stream)
{
    if (!params || !X || !Y || !T || !cache || !grad || !work || B < 1) return Z4C_EINVAL;
    return launch_mlp_backward(static_cast<const float*>(params), static_cast<const float*>(X),
                               static_cast<const float*>(Y), static_cast<const float*>(T),
                               static_cast<const float*>(cache), B, static_cast<float*>(grad),
                               static_cast<float*>(loss), static_cast<float*>(work),
                               as_stream(stream)) == hipSuccess ? Z4C_OK : Z4C_EDEVICE;
}

int z4c_mlp_adam(void* params, const void* grad, void* m, void* v, int32_t step, float lr, float beta1,
                 float beta2, float eps, void* stream)
{
    if (!params || !grad || !m || !v || step < 1) return Z4C_EINVAL;
    return launch_mlp_adam(static_cast<float*>(params), static_cast<const float*>(grad),
                           static_cast<float*>(m), static_cast<float*>(v), step, lr, beta1, beta2, eps,
                           as_stream(stream)) == hipSuccess ? Z4C_OK : Z4C_EDEVICE;
}

int z4c_refine_flags_learned(z4c_pack* pk, int32_t reg, const z4c_mlp_model* md, int8_t* flags_out,
                             int8_t* fallback_out, void* stream)
{
    if (!pk) return Z4C_EINVAL;
    if (!md || !md->params || !md->stats || !md->range || !flags_out) return fail(pk, Z4C_EINVAL, "null argument");
    const int nb = (int)pk->blk.size();
    int rc = z4c_features(pk, reg, nullptr, nullptr, stream);
    if (rc) return rc;
    hipStream_t s = as_stream(stream);
    double* fdev = reinterpret_cast<double*>(pk->ws + pk->ws_feat);
    float* X = reinterpret_cast<float*>(pk->ws + pk->ws_x);
    float* Y = reinterpret_cast<float*>(pk->ws + pk->ws_y);
    int8_t* fl = reinterpret_cast<int8_t*>(pk->ws + pk->ws_lflag);
    LearnedRule r;
    std::memset(&r, 0, sizeof(r));
    for (int k = 0; k < 16; ++k) { r.lo[k] = md->range[k]; r.hi[k] = md->range[16 + k]; }
    r.tau_ref = md->tau_ref;
    r.tau_deref = md->tau_deref;
    r.chi_thr = md->chi_thr;
    r.dchi_thr = md->dchi_thr;
    r.level_max = md->level_max;
    std::vector<int8_t> host(2 * (size_t)nb);
    hipError_t e = launch_normalize(fdev, nb, static_cast<const double*>(md->stats), X, s);
    if (e == hipSuccess) e = launch_mlp_forward(static_cast<const float*>(md->params), X, nb, Y, nullptr, s);
    if (e == hipSuccess)
        e = launch_learned_flags(fdev, Y, reinterpret_cast<const BlockDev*>(pk->ws + pk->ws_blocks), nb, r, fl,
                                 fl + nb, s);
    if (e == hipSuccess) e = hipMemcpyAsync(host.data(), fl, 2 * (size_t)nb, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(pk, Z4C_EDEVICE, "learned flags: %s", hipGetErrorString(e));
    std::memcpy(flags_out, host.data(), (size_t)nb);
    if (fallback_out) std::memcpy(fallback_out, host.data() + nb, (size_t)nb);
    return Z4C_OK;
}

int z4c_stencil_weights(int32_t fd_order, double* d1, double* d2, double* lop)
{
    auto fill = [&](auto tag) {
        constexpr int N = decltype(tag)::value;
        for (int k = 0; k <= N; ++k) {
            if (d1) d1[k] = Stencil<N>::D1[k];
            if (d2) d2[k] = Stencil<N>::D2[k];
        }
        for (int k = 0; k < 2 * N + 1; ++k)
            if (lop) lop[k] = Stencil<N>::LOP[k];
    };
    switch (fd_order) {
    case 4: fill(std::integral_constant<int, 2>()); return Z4C_OK;
    case 6: fill(std::integral_constant<int, 3>()); return Z4C_OK;
    case 8: fill(std::integral_constant<int, 4>()); return Z4C_OK;
    }
    return Z4C_EINVAL;
}

}  // extern "C"
