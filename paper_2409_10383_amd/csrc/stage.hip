// Fused Z4c RHS + classic RK4 stage kernel.
//
// One launch per RK stage covers the whole MeshBlockPack: each workgroup
// (256 threads, one zone each) owns an 8 x 8 x 4 tile of active cells of
// one MeshBlock and streams the 22 fields through LDS one at a time: the
// field's tile plus an (N+1)-cell halo is staged (coalesced, x fastest),
// then every derivative the method needs of that field is taken from LDS:
//   - per axis, one pass over the 2(N+1) neighbours gives the centred first
//     and second derivatives, the odd (advective) and even (advective +
//     Kreiss-Oliger) parts of the upwind-biased operator;
//   - mixed second derivatives in two passes, d_x f then d_y(d_x f),
//     d_z(d_x f), d_z(d_y f), through LDS intermediates (the first pass
//     covers only the halo points; the tile's own d_x f, d_y f are the
//     axis sweep's);
//   - second derivatives are contracted into the Ricci tensor and the shift
//     terms as soon as they are produced, so only first derivatives and a
//     few accumulators stay live in registers.
// The per-zone algebra then builds the 22 RHS values (equations listed in
// z4c_rhs.hpp), the RK4 update runs in double against the FP64 accumulator,
// and the algebraic constraints and floors are applied before the store.
#include "kernels.hpp"
#include "z4c_rhs.hpp"

namespace z4c {

// Tile shapes the autotuner chooses from (x, y, z extents; 256 zones each).
// The per-zone arithmetic does not depend on the shape, so every variant
// gives bitwise-identical results.
template <int N, int TX, int TY, int TZ> struct TileGeom {
    static constexpr int R = N + 1;                 // halo of the staged tile
    static constexpr int SX = TX + 2 * R, SY = TY + 2 * R, SZ = TZ + 2 * R;
    static constexpr int NS = SX * SY * SZ;         // staged cells
    static constexpr int DXY = TY + 2 * N, DXZ = TZ + 2 * N;
    static constexpr int NDX = TX * DXY * DXZ;      // d_x f box over the y, z halos
    static constexpr int NDY = TX * TY * DXZ;       // d_y f box over the z halo
    // points of those boxes the mixed derivatives read outside the tile:
    // d_x f on the y halo (TX x 2N x TZ) and the z halo (TX x TY x 2N), d_y f
    // on the z halo; the tile's own values come from the axis sweeps
    static constexpr int NHXY = TX * 2 * N * TZ;
    static constexpr int NHX = NHXY + TX * TY * 2 * N;
    static constexpr int NHY = TX * TY * 2 * N;
};

// LDS per workgroup: NBUF staged-field buffers, the mixed-derivative
// intermediates and the per-zone advection + dissipation slots.  Two
// buffers (the next field streams in while the current one is used) when
// they fit in a CU's 160 KB, else one.
template <class G, class C> struct StageLds {
    static constexpr int REST = (G::NDX + G::NDY + NF * 256) * (int)sizeof(C) + 27 * 4;
    static constexpr int NBUF = (2 * G::NS * (int)sizeof(C) + REST <= 160 * 1024) ? 2 : 1;
};

typedef __attribute__((address_space(1))) const void* gptr_t;
typedef __attribute__((address_space(3))) void* lptr_t;

// Asynchronous copy of one staged field (global -> LDS, no registers): the
// staged tile is dense in LDS (x fastest), so slot u of S bytes lands at
// byte S*u; lane l of a wave writes S bytes at the wave's LDS base + S*l.
// soff holds the element offset (from the field's base in this block's
// ghosted frame) of the first element of each of this thread's slots.
template <int S, int ESZ, int NSLOT, int NR>
__device__ __forceinline__ void dma_field(const char* gbase, char* lbase, const int (&soff)[NR])
{
    const int t = threadIdx.x, w = t >> 6;
#pragma unroll
    for (int r = 0; r < NR; ++r)
        if (r * 256 + t < NSLOT) {
            const gptr_t src = (gptr_t)(gbase + (int64_t)soff[r] * ESZ);
            const lptr_t dst = (lptr_t)(lbase + (r * 256 + w * 64) * S);
            if constexpr (S == 16) __builtin_amdgcn_global_load_lds(src, dst, 16, 0, 0);
            else __builtin_amdgcn_global_load_lds(src, dst, 4, 0, 0);
        }
}

// wait for this wave's outstanding vector memory operations (the LDS
// copies above count there), before the barrier that publishes them
__device__ __forceinline__ void wait_vmem()
{
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0), expcnt and lgkmcnt unconstrained
}

// workgroup barrier over this wave's LDS reads and writes only: the next
// field's copy (counted as vector memory) stays in flight across it.  A
// fence would also wait for that copy, since it targets LDS; the memory
// clobber keeps the compiler from moving memory accesses across.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// one axis of a staged field: centred d1, d2 (both optional) and the
// advection + dissipation contribution; no 1/h factors
// va is the advection speed along the axis (0 when advection is off) and
// sig the dissipation strength: ad += va*odd + |va|*even_lop + sig*even_ko
template <int N, class C, bool D1, bool D2>
__device__ __forceinline__ void axis_pass(const C* __restrict__ s, int c, int st, C va, C sig,
                                          C& d1, C& d2, C& ad)
{
    const C f0 = s[c];
    C a1 = 0, a2 = 0, odd = 0, el = 0, ek = 0;
#pragma unroll
    for (int k = 1; k <= N + 1; ++k) {
        const C fp = s[c + k * st], fm = s[c - k * st];
        const C dk = fp - fm;
        const C sk = (fp - f0) + (fm - f0);
        if (k <= N) {
            if (D1) a1 += (C)Stencil<N>::D1[k] * dk;
            if (D2) a2 += (C)Stencil<N>::D2[k] * sk;
        }
        odd += (C)lop_odd<N>(k) * dk;
        el += (C)lop_even<N>(k) * sk;
        ek += (C)Stencil<N>::KO[k] * sk;
    }
    d1 = a1;
    d2 = a2;
    ad += va * odd + (C)fabs((double)va) * el + sig * ek;
}

// The work items are spread so that each of the 8 XCDs (each with its own
// L2) receives a contiguous run of tiles: workgroup b runs on XCD b % 8.
__device__ __forceinline__ int work_index(int slot, int nwork)
{
    const int per = (nwork + 7) / 8;
    const int x = slot % 8, k = slot / 8;
    return x * per + k;
}

template <int N, class T, class C, int TX, int TY, int TZ, int SW>
__device__ __forceinline__ void stage_tile(const StageArgs& a, const WorkItem w, C* tile, C* dxs,
                                           C* dys, C* adks, int* vtab);

// Waves per SIMD the compiler is asked to fit: FP32 storage fits two (the
// 8th-order kernels would otherwise take 289 registers, one wave; asking for
// two spills 31 of them, the tile's copy offsets, to scratch, and the stage
// takes 3.9 instead of 6.3 ms on the 512-block pack); the FP64 kernels need
// about 440 registers and stay at one.
template <class T> struct StageWaves {
    static constexpr int value = sizeof(T) == 4 ? 2 : 1;
};

// One launch per stage.  With a.persistent the grid is sized to the
// resident workgroups and each loops over its XCD's share of the work.
// W: the staged tiles are copied in 16-byte pieces (FP32 storage always;
// FP64 when the ghost depth and the halo differ by an even count, which the
// launch checks), else FP64 fields go as 4-byte halves.
template <int N, class T, class C, int TX, int TY, int TZ, int SW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(StageWaves<T>::value))) void k_stage(
    const StageArgs a)
{
    using G = TileGeom<N, TX, TY, TZ>;
    __shared__ __align__(16) C tile[StageLds<G, C>::NBUF * G::NS];
    __shared__ C dxs[G::NDX];
    __shared__ C dys[G::NDY];
    __shared__ C adks[NF * 256];   // advection + dissipation, per field and zone
    __shared__ int vtab[27];       // the tile's block: halo offsets per direction
    if (!a.persistent) {
        const int w = work_index(blockIdx.x, a.nwork);
        if (w < a.nwork) stage_tile<N, T, C, TX, TY, TZ, SW>(a, a.work[w], tile, dxs, dys, adks, vtab);
        return;
    }
    // persistent: XCD x = blockIdx % 8 walks items x*per .. x*per+per-1
    const int per = (a.nwork + 7) / 8;
    const int x = blockIdx.x % 8, k0 = blockIdx.x / 8, nk = (gridDim.x - x + 7) / 8;
    for (int k = k0; k < per; k += nk) {
        const int w = x * per + k;
        if (w >= a.nwork) break;
        stage_tile<N, T, C, TX, TY, TZ, SW>(a, a.work[w], tile, dxs, dys, adks, vtab);
        lds_barrier();
    }
}

template <int N, class T, class C, int TX, int TY, int TZ, int SW>
__device__ __forceinline__ void stage_tile(const StageArgs& a, const WorkItem w, C* tile, C* dxs,
                                           C* dys, C* adks, int* vtab)
{
    using G = TileGeom<N, TX, TY, TZ>;
    constexpr int R = G::R, SX = G::SX, SY = G::SY;
    const BlockDev B = a.blocks[w.block];
    const int t = threadIdx.x;
    const int tx = t % TX, ty = (t / TX) % TY, tz = t / (TX * TY);
    const int i = w.i0 + tx, j = w.j0 + ty, k = w.k0 + tz;
    const int g = a.g, E = B.E, n = B.n;
    const int64_t slab = B.slab;
    const T* __restrict__ srcb = (const T*)a.src + B.off;
    const int64_t cz = ((int64_t)(k + g) * E + (j + g)) * E + (i + g);  // zone, ghosted index
    const C ih = (C)(1.0 / B.h), ih2 = ih * ih;
    const ParamsDev& P = a.P;

    // staged-tile index of this zone and its strides
    const int c = ((tz + R) * SY + (ty + R)) * SX + (tx + R);
    const int sxy = SX * SY;
    C* cur = tile;   // LDS buffer holding the field being processed

    // origin of the staged tile (tile + halo R) in the ghosted block
    const int64_t base0 = ((int64_t)(w.k0 - R + g) * E + (w.j0 - R + g)) * E + (w.i0 - R + g);
    // d_x f on the y/z halos and d_y f on the z halo (for mixed derivatives):
    // each of this thread's halo points keeps its staged-tile index (high 16
    // bits) and its index in the d_x f / d_y f box (low 16 bits), fixed per tile
    static_assert(G::NS < 65536 && G::NDX < 65536, "halo point indices must fit 16 bits");
    constexpr int NQX = (G::NHX + 255) / 256, NQY = (G::NHY + 255) / 256;
    constexpr int N2 = 2 * N;
    int ccx[NQX], ccy[NQY];
    auto halo = [](int zz, int ext) { return zz < N ? zz - N : ext + zz - N; };
#pragma unroll
    for (int r = 0; r < NQX; ++r) {
        const int q = t + 256 * r;
        int x, y, z;
        if (q < G::NHXY) {
            x = q % TX; y = halo((q / TX) % N2, TY); z = q / (TX * N2);
        } else {
            const int u = q - G::NHXY;
            x = u % TX; y = (u / TX) % TY; z = halo(u / (TX * TY), TZ);
        }
        ccx[r] = ((((z + R) * SY + (y + R)) * SX + (x + R)) << 16) | (((z + N) * G::DXY + (y + N)) * TX + x);
    }
#pragma unroll
    for (int r = 0; r < NQY; ++r) {
        const int q = t + 256 * r;
        const int x = q % TX, y = (q / TX) % TY, z = halo(q / (TX * TY), TZ);
        ccy[r] = ((((z + R) * SY + (y + R)) * SX + (x + R)) << 16) | (((z + N) * TY + y) * TX + x);
    }
    auto first_pass = [&]() {
#pragma unroll
        for (int r = 0; r < NQX; ++r)
            if (t + 256 * r < G::NHX) dxs[ccx[r] & 0xFFFF] = fd1<N, C>(cur + (ccx[r] >> 16), 1);
#pragma unroll
        for (int r = 0; r < NQY; ++r)
            if (t + 256 * r < G::NHY) dys[ccy[r] & 0xFFFF] = fd1<N, C>(cur + (ccy[r] >> 16), SX);
    };
    // this zone's own entries of the two boxes (written by the axis sweep)
    const int own_x = ((tz + N) * G::DXY + (ty + N)) * TX + tx;
    const int own_y = ((tz + N) * TY + ty) * TX + tx;
    // mixed derivatives of the staged field at this zone: xy, xz, yz
    auto mixed = [&](C& mxy, C& mxz, C& myz) {
        mxy = fd1<N, C>(dxs + own_x, TX);
        mxz = fd1<N, C>(dxs + own_x, TX * G::DXY);
        myz = fd1<N, C>(dys + own_y, TX * TY);
    };

    // centre values needed by the sweep: shift, conformal metric and its
    // inverse (loaded once the first field's copy is under way)
    C be[3], gdn[6], gu[6];
    const bool adv = (P.terms & 4u) != 0;
    const bool adv_gauge = adv && (P.terms & 2u);
    const C sig = (P.terms & 8u) ? (C)P.ko_sigma : (C)0;
    const int st3[3] = {1, SX, sxy};

    C dg[3][6], Rt[6];   // d_a g~_p ; Ricci accumulator
    C dchi[3], ddchi[6], dal[3], ddal[6], dbe[3][3], Lb[3], Bj[3], eK[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) { Lb[q] = 0; Bj[q] = 0; eK[q] = 0; }

    // generic per-field sweep: first derivatives d1[3], pure second d2[3]
    // advection + dissipation of field f at this zone, kept in LDS.  Fields
    // with second derivatives also need mixed ones: the sweep then leaves the
    // zone's d_x f and d_y f (no 1/h) in the boxes the mixed pass reads.
    auto put_adk = [&](int f, C v) { adks[f * 256 + t] = v; };
    auto sweep = [&](int f, bool gauge_field, C* d1, C* d2, auto D1tag, auto D2tag) {
        constexpr bool WD1 = decltype(D1tag)::value, WD2 = decltype(D2tag)::value;
        const bool a_on = gauge_field ? adv_gauge : adv;
        C ad = 0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            C x1, x2;
            axis_pass<N, C, WD1, WD2>(cur, c, st3[d], a_on ? be[d] : (C)0, sig, x1, x2, ad);
            if (WD2 && d == 0) dxs[own_x] = x1;
            if (WD2 && d == 1) dys[own_y] = x1;
            if (WD1) d1[d] = x1 * ih;
            if (WD2) d2[d] = x2 * ih2;
        }
        put_adk(f, ad * ih);
    };
    using T1 = std::integral_constant<bool, true>;
    using F0 = std::integral_constant<bool, false>;

    // ---- the 22 fields stream through LDS in the order below.  Each field's
    // staged tile is copied global -> LDS asynchronously (no registers); with
    // two buffers the next field's copy is issued before the current field is
    // processed, so its latency overlaps the stencil work.
    constexpr int NBUF = StageLds<G, C>::NBUF;
    // bytes per lane and copy (SW): a staged row splits into whole slots, each
    // of one row's consecutive cells.  16-byte copies need a 16-byte aligned
    // tile origin (E, every field base and the tile's x origin), which the
    // launch checks; otherwise FP64 fields go as 4-byte halves and FP32 ones
    // cell by cell
    constexpr int SLOT = sizeof(T) == 8 ? 16 : SW;
    constexpr bool wide = sizeof(T) == 4 || SW == 16;
    static_assert(!wide || (G::SX * (int)sizeof(T)) % SLOT == 0, "copy slots must not cross a staged row");
    constexpr int NSLOT = G::NS * (int)sizeof(T) / SLOT;
    constexpr int NRS = (NSLOT + 255) / 256;
    // staged cells outside the block read a same-level neighbour directly
    // where the pack provides a virtual halo for that direction (the offset
    // table then points the block's ghosted index at the neighbour's cells);
    // in pushed x directions the table gives the neighbour the zones near a
    // face write their state to
    // (one load per direction into LDS: the copy offsets below then read the
    // table there instead of waiting on one global load per slot)
    if (t < 27) vtab[t] = (int)(a.vnbr[(int64_t)w.block * 27 + t] - B.off);
    lds_barrier();
    // outflow directions whose y or z leaves the domain read the block across
    // the remaining components (the table's offset), with that y or z of the
    // staged cell clamped to the active range
    const uint32_t cmy = a.cmask[2 * w.block], cmz = a.cmask[2 * w.block + 1];
    int soff[NRS];
#pragma unroll
    for (int r = 0; r < NRS; ++r) {
        const int q = (r * 256 + t) * (SLOT / (int)sizeof(T));   // first element of the slot
        const int x = q % SX, y = (q / SX) % SY, z = q / sxy;
        const int lx = x + w.i0 - R, ly = y + w.j0 - R, lz = z + w.k0 - R;
        // without virtual x directions the x halo is read from the block's
        // own ghosts (same-level neighbours push them), so that a staged row
        // stays one block's memory
        const int dir = ((lz < 0 ? 0 : (lz >= n ? 2 : 1)) * 3 + (ly < 0 ? 0 : (ly >= n ? 2 : 1))) * 3 +
                        (a.virt_x ? (lx < 0 ? 0 : (lx >= n ? 2 : 1)) : 1);
        const int cy = ((cmy >> dir) & 1u) ? (ly < 0 ? 0 : (ly >= n ? n - 1 : ly)) : ly;
        const int cz = ((cmz >> dir) & 1u) ? (lz < 0 ? 0 : (lz >= n ? n - 1 : lz)) : lz;
        soff[r] = vtab[dir] + ((cz + g) * E + (cy + g)) * E + (lx + g);
    }
    auto issue = [&](int f, C* buf) {
        if (wide) {
            dma_field<SLOT, (int)sizeof(T), NSLOT, NRS>((const char*)(srcb + f * slab), (char*)buf, soff);
        } else {
            const char* gb = (const char*)(srcb + f * slab + base0);
            constexpr int NS4 = G::NS * (int)sizeof(T) / 4, NR4 = (NS4 + 255) / 256;
            const int wv = t >> 6;
#pragma unroll 4
            for (int r = 0; r < NR4; ++r) {
                const int u = r * 256 + t;
                if (u < NS4) {
                    const int q = u * 4 / (int)sizeof(T), hb = (u * 4) % (int)sizeof(T);
                    const int x = q % SX, y = (q / SX) % SY, z = q / sxy;
                    const int off = ((z * E + y) * E + x) * (int)sizeof(T) + hb;
                    __builtin_amdgcn_global_load_lds((gptr_t)(gb + off),
                                                     (lptr_t)((char*)buf + (r * 256 + wv * 64) * 4), 4, 0, 0);
                }
            }
        }
    };
    // slot -> field: g~ (6), chi, alpha, beta (3), Gamma~ (3), Khat, Theta, A~ (6)
    auto field_of = [](int sl) {
        return sl < 6 ? F_GXX + sl : sl == 6 ? F_CHI : sl == 7 ? F_ALPHA : sl < 11 ? F_BETAX + (sl - 8)
             : sl < 14 ? F_GAMX + (sl - 11) : sl == 14 ? F_KH : sl == 15 ? F_TH : F_AXX + (sl - 16);
    };
    // processing of field slot sl, staged in LDS at cur
    auto process = [&](int sl) __attribute__((always_inline)) {
        if (sl < 6) {
            // conformal metric: first derivatives, Ricci second-derivative term
            const int p = sl;
            first_pass();
            C d1[3], d2[3], mxy, mxz, myz;
            sweep(F_GXX + p, false, d1, d2, T1(), T1());
            lds_barrier();
            mixed(mxy, mxz, myz);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
#pragma unroll
                for (int pp = 0; pp < 6; ++pp)
                    if (pp == p) dg[d][pp] = d1[d];
            }
            const C r = -(C)0.5 * (gu[0] * d2[0] + gu[3] * d2[1] + gu[5] * d2[2] +
                                   (C)2 * ih2 * (gu[1] * mxy + gu[2] * mxz + gu[4] * myz));
#pragma unroll
            for (int pp = 0; pp < 6; ++pp)
                if (pp == p) Rt[pp] = r;
        } else if (sl < 8) {
            // chi and alpha: first and second derivatives
            first_pass();
            C d1[3], d2[3], mxy, mxz, myz;
            const bool is_chi = sl == 6;
            sweep(is_chi ? F_CHI : F_ALPHA, !is_chi, d1, d2, T1(), T1());
            lds_barrier();
            mixed(mxy, mxz, myz);
            C* dd = is_chi ? ddchi : ddal;
            C* d = is_chi ? dchi : dal;
            d[0] = d1[0]; d[1] = d1[1]; d[2] = d1[2];
            dd[0] = d2[0]; dd[3] = d2[1]; dd[5] = d2[2];
            dd[1] = mxy * ih2; dd[2] = mxz * ih2; dd[4] = myz * ih2;
        } else if (sl < 11) {
            // shift: first derivatives, g~^jk d_j d_k beta^i and d_j d_k beta^k
            const int q = sl - 8;
            first_pass();
            C d1[3], d2[3], mxy, mxz, myz;
            sweep(F_BETAX + q, true, d1, d2, T1(), T1());
            lds_barrier();
            mixed(mxy, mxz, myz);
            mxy *= ih2; mxz *= ih2; myz *= ih2;
            const C dd[6] = {d2[0], mxy, mxz, d2[1], myz, d2[2]};
            const C lb = gu[0] * dd[0] + gu[3] * dd[3] + gu[5] * dd[5] +
                         (C)2 * (gu[1] * dd[1] + gu[2] * dd[2] + gu[4] * dd[4]);
#pragma unroll
            for (int qq = 0; qq < 3; ++qq)
                if (qq == q) {
                    Lb[qq] = lb;
#pragma unroll
                    for (int d = 0; d < 3; ++d) dbe[d][qq] = d1[d];
                    // B_j += d_j d_q beta^q
                    Bj[0] += dd[S(0, qq)];
                    Bj[1] += dd[S(1, qq)];
                    Bj[2] += dd[S(2, qq)];
                }
        } else if (sl < 14) {
            // Gamma~: its first derivatives enter R~_ij only
            const int q = sl - 11;
            C d1[3], d2[3];
            sweep(F_GAMX + q, false, d1, d2, T1(), F0());
            // R~_ij += 1/2 (g~_qi d_j G^q + g~_qj d_i G^q)
#pragma unroll
            for (int qq = 0; qq < 3; ++qq)
                if (qq == q) {
#pragma unroll
                    for (int pp = 0; pp < 6; ++pp) {
                        const int ii = SA(pp), jj = SB(pp);
                        Rt[pp] += (C)0.5 * (gdn[S(qq, ii)] * d1[jj] + gdn[S(qq, jj)] * d1[ii]);
                    }
                }
        } else if (sl < 16) {
            // Khat and Theta: 2 d Khat + d Theta
            C d1[3], d2[3];
            sweep(sl == 14 ? F_KH : F_TH, false, d1, d2, T1(), F0());
            if (sl == 14) {
#pragma unroll
                for (int d = 0; d < 3; ++d) eK[d] = (C)2 * d1[d];
            } else {
#pragma unroll
                for (int d = 0; d < 3; ++d) eK[d] += d1[d];
            }
        } else {
            // A~_ij: advection and dissipation only
            C ad = 0;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                C x1, x2;
                axis_pass<N, C, false, false>(cur, c, st3[d], adv ? be[d] : (C)0, sig, x1, x2, ad);
            }
            put_adk(F_AXX + (sl - 16), ad * ih);
        }
    };
    issue(field_of(0), tile);
#pragma unroll
    for (int q = 0; q < 3; ++q) be[q] = (C)srcb[(F_BETAX + q) * slab + cz];
#pragma unroll
    for (int q = 0; q < 6; ++q) gdn[q] = (C)srcb[(F_GXX + q) * slab + cz];
    {
        const C c0 = gdn[3] * gdn[5] - gdn[4] * gdn[4];
        const C c1 = gdn[2] * gdn[4] - gdn[1] * gdn[5];
        const C c2 = gdn[1] * gdn[4] - gdn[2] * gdn[3];
        const C id = (C)1 / (gdn[0] * c0 + gdn[1] * c1 + gdn[2] * c2);
        gu[0] = c0 * id; gu[1] = c1 * id; gu[2] = c2 * id;
        gu[3] = (gdn[0] * gdn[5] - gdn[2] * gdn[2]) * id;
        gu[4] = (gdn[1] * gdn[2] - gdn[0] * gdn[4]) * id;
        gu[5] = (gdn[0] * gdn[3] - gdn[1] * gdn[1]) * id;
    }
#pragma unroll 1
    for (int sl = 0; sl < NF - 1; ++sl) {
        cur = (NBUF == 2 && (sl & 1)) ? tile + G::NS : tile;
        wait_vmem();
        __syncthreads();   // field sl in LDS; every wave is done with field sl-1
        if (NBUF == 2) issue(field_of(sl + 1), (sl & 1) ? tile : tile + G::NS);
        process(sl);
        if (NBUF == 1) {
            lds_barrier();     // every wave is done with the single buffer
            issue(field_of(sl + 1), tile);
        }
    }
    // the last field (a component of A~, light on registers), with the
    // centre values of the per-zone algebra loaded at its start so that their
    // latency overlaps it
    C chi, Kh, Th, al, A[6], Gam[3];
    {
        constexpr int sl = NF - 1;
        cur = (NBUF == 2 && (sl & 1)) ? tile + G::NS : tile;
        wait_vmem();
        __syncthreads();
        chi = (C)srcb[F_CHI * slab + cz];
        Kh = (C)srcb[F_KH * slab + cz];
        Th = (C)srcb[F_TH * slab + cz];
        al = (C)srcb[F_ALPHA * slab + cz];
#pragma unroll
        for (int q = 0; q < 6; ++q) A[q] = (C)srcb[(F_AXX + q) * slab + cz];
#pragma unroll
        for (int q = 0; q < 3; ++q) Gam[q] = (C)srcb[(F_GAMX + q) * slab + cz];
        process(sl);
    }

    // ---- the per-zone algebra

    // RK inputs of this zone (U for stages 1-3, the accumulator for 2-4).
    // FP64: loaded before the algebra so that their latency overlaps it (the
    // values wait in the AGPR half of the register file).  FP32 storage keeps
    // them out of the registers (its kernels fit two waves per SIMD) and
    // loads them in the update.
    constexpr bool EARLY = sizeof(T) == 8;
    const int64_t n3 = (int64_t)n * n * n;
    const int64_t ci = B.ioff + ((int64_t)k * n + j) * n + i;
    const T* __restrict__ U0 = (const T*)a.U + B.off + cz;
    double upre[EARLY ? NF : 1], apre[EARLY ? NF : 1];
    if constexpr (EARLY) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            upre[f] = (a.stage >= 1 && a.stage <= 3) ? (double)U0[f * slab] : 0.0;
            apre[f] = (a.stage >= 2) ? a.A[ci + f * n3] : 0.0;
        }
    }
    C rhs[NF];
    z4c_algebra<C>(P, chi, gdn, gu, Kh, A, Gam, Th, al, be, dg, dchi, ddchi, dal, ddal, dbe, Lb,
                   Bj, eK, Rt, rhs);
#pragma unroll
    for (int f = 0; f < NF; ++f) rhs[f] += adks[f * 256 + t];

    // ---- RK4 stage update
    if (a.stage == 0) {
#pragma unroll
        for (int f = 0; f < NF; ++f) a.rhs_out[ci + f * n3] = (double)rhs[f];
        return;
    }
    const double dt = a.dt;
    double out[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const double kf = (double)rhs[f];
        double* Af = a.A + ci + f * n3;
        if constexpr (EARLY) {
            switch (a.stage) {
            case 1:
                out[f] = upre[f] + 0.5 * dt * kf;
                *Af = upre[f] + dt / 6.0 * kf;
                break;
            case 2:
                out[f] = upre[f] + 0.5 * dt * kf;
                *Af = apre[f] + dt / 3.0 * kf;
                break;
            case 3:
                out[f] = upre[f] + dt * kf;
                *Af = apre[f] + dt / 3.0 * kf;
                break;
            default:
                out[f] = apre[f] + dt / 6.0 * kf;
            }
        } else {
            switch (a.stage) {
            case 1: {
                const double u = (double)U0[f * slab];
                out[f] = u + 0.5 * dt * kf;
                *Af = u + dt / 6.0 * kf;
            } break;
            case 2: {
                const double u = (double)U0[f * slab];
                out[f] = u + 0.5 * dt * kf;
                *Af += dt / 3.0 * kf;
            } break;
            case 3: {
                const double u = (double)U0[f * slab];
                out[f] = u + dt * kf;
                *Af += dt / 3.0 * kf;
            } break;
            default:
                out[f] = *Af + dt / 6.0 * kf;
            }
        }
    }
    if (P.enforce) enforce_zone(out, P);
    T* __restrict__ dst = (T*)a.dst + B.off + cz;
#pragma unroll
    for (int f = 0; f < NF; ++f) dst[f * slab] = (T)out[f];
    // A zone within g of an x face is a ghost of the same-level neighbour
    // across that face, and of the diagonal neighbours across it and a y or
    // z face the zone is also near (a zone may be near both faces of an axis
    // when n < 2g): the written state goes there too, so that the next
    // stage finds those ghosts filled (the pack's fill leaves them alone)
    // and stages every row from one block.
    const uint32_t pm = a.pmask[w.block];
    const int sxm = (i < g ? 1 : 0) | (i >= n - g ? 4 : 0);   // bit s: near the face of side s
    if (pm && sxm) {
        const int sym = 2 | (j < g ? 1 : 0) | (j >= n - g ? 4 : 0);
        const int szm = 2 | (k < g ? 1 : 0) | (k >= n - g ? 4 : 0);
#pragma unroll 1
        for (int d = 0; d < 27; ++d) {
            const int sx = d % 3, sy = (d / 3) % 3, sz = d / 9;
            if (!((pm >> d) & 1u) || !((sxm >> sx) & 1) || !((sym >> sy) & 1) || !((szm >> sz) & 1)) continue;
            T* __restrict__ gh = (T*)a.dst + B.off + vtab[d] + cz;
#pragma unroll
            for (int f = 0; f < NF; ++f) gh[f * slab] = (T)out[f];
        }
    }
    // A tile on an outflow x face: its face zones are the nearest active cells
    // of the g ghost columns beyond them in their rows and, at a y or z domain
    // face, of those of the rows beyond that face.  The face zones put their
    // new state in their own slots of the advection store (read above, each
    // thread its own slot only), and the workgroup writes those ghost cells in
    // this block and in the same-level neighbours across y and z whose ghost
    // layers hold them, one thread per ghost cell.
    const uint32_t om = a.omask[w.block];
#pragma unroll 1
    for (int side = 0; side < 2; ++side) {
        if (!((om >> side) & 1u) || (side ? w.i0 + TX != n : w.i0 != 0)) continue;
        const int fx = side ? TX - 1 : 0;    // the tile's face column
        if (tx == fx) {
#pragma unroll
            for (int f = 0; f < NF; ++f) adks[f * 256 + t] = (C)(T)out[f];
        }
        lds_barrier();
        const int xg = side ? n + g : 0;     // first ghost column, ghosted index
        const int ya = (w.j0 == 0 && (om & 4u)) ? -g : w.j0;
        const int yb = (w.j0 + TY == n && (om & 8u)) ? n + g - 1 : w.j0 + TY - 1;
        const int za = (w.k0 == 0 && (om & 16u)) ? -g : w.k0;
        const int zb = (w.k0 + TZ == n && (om & 32u)) ? n + g - 1 : w.k0 + TZ - 1;
#pragma unroll 1
        for (int e = 0; e < 9; ++e) {
            if (!((om >> (8 + e)) & 1u)) continue;
            const int ey = e % 3 - 1, ez = e / 3 - 1;
            // rows and planes of the target's ghosted range, in this block's frame
            const int y0 = max(ya, ey * n - g), y1 = min(yb, ey * n + n + g - 1);
            const int z0 = max(za, ez * n - g), z1 = min(zb, ez * n + n + g - 1);
            if (y0 > y1 || z0 > z1) continue;
            const int ny = y1 - y0 + 1, ncell = (z1 - z0 + 1) * ny * g;
            T* __restrict__ tb = (T*)a.dst + B.off + vtab[e * 3 + 1] + xg;
            for (int q = t; q < ncell; q += 256) {
                const int xc = q % g, r = q / g, yy = y0 + r % ny, zz = z0 + r / ny;
                const int sy = min(max(yy, w.j0), w.j0 + TY - 1) - w.j0;
                const int sz = min(max(zz, w.k0), w.k0 + TZ - 1) - w.k0;
                const C* __restrict__ sv = adks + (sz * TY + sy) * TX + fx;
                T* __restrict__ gh = tb + ((int64_t)(zz + g) * E + (yy + g)) * E + xc;
#pragma unroll
                for (int f = 0; f < NF; ++f) gh[f * slab] = (T)sv[f * 256];
            }
        }
    }
}

// FP32 copy width of a tile shape: 16 bytes where a staged row is a multiple
// of four cells (the launch also needs a 16-byte aligned origin), else 4;
// and the width when the origin is not aligned
template <int N, int TX> struct Fp32Slot {
    static constexpr int SX = TX + 2 * (N + 1);
    static constexpr int best = SX % 4 == 0 ? 16 : 4;
    static constexpr int fallback = 4;
};

template <int N, int TX, int TY, int TZ>
static hipError_t launch_v(int prec, const StageArgs& a, int grid, hipStream_t s)
{
    const int R = N + 1;
    if (prec == 0) {
        // 16-byte FP64 copies when the ghost depth and the halo N+1 differ by
        // an even count
        if (((a.g - R) & 1) == 0)
            hipLaunchKernelGGL((k_stage<N, double, double, TX, TY, TZ, 16>), dim3(grid), dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((k_stage<N, double, double, TX, TY, TZ, 4>), dim3(grid), dim3(256), 0, s, a);
    } else {
        // 16-byte FP32 copies: E = n + 2g a multiple of 4 cells (n is a
        // multiple of 8: g even) and the tile origin i0 - R + g too (i0 is a
        // multiple of 8)
        using S = Fp32Slot<N, TX>;
        if constexpr (S::best != 16) {
            hipLaunchKernelGGL((k_stage<N, float, float, TX, TY, TZ, S::best>), dim3(grid), dim3(256), 0, s, a);
        } else if ((a.g % 2 == 0) && ((a.g - R) % 4 == 0)) {
            hipLaunchKernelGGL((k_stage<N, float, float, TX, TY, TZ, 16>), dim3(grid), dim3(256), 0, s, a);
        } else {
            hipLaunchKernelGGL((k_stage<N, float, float, TX, TY, TZ, S::fallback>), dim3(grid), dim3(256), 0, s, a);
        }
    }
    return hipGetLastError();
}

template <int N>
static hipError_t launch_n(int prec, int variant, const StageArgs& a, int grid, hipStream_t s)
{
    switch (variant) {
    case 0: return launch_v<N, 8, 8, 4>(prec, a, grid, s);
    case 1: return launch_v<N, 16, 4, 4>(prec, a, grid, s);
    case 2: return launch_v<N, 8, 4, 8>(prec, a, grid, s);
    case 3: return launch_v<N, 16, 8, 2>(prec, a, grid, s);
    }
    return hipErrorInvalidValue;
}

const int TILE_SHAPES[NVARIANT][3] = {{8, 8, 4}, {16, 4, 4}, {8, 4, 8}, {16, 8, 2}};

hipError_t launch_stage(int N, int prec, int variant, const StageArgs& a, int grid, hipStream_t s)
{
    switch (N) {
    case 2: return launch_n<2>(prec, variant, a, grid, s);
    case 3: return launch_n<3>(prec, variant, a, grid, s);
    case 4: return launch_n<4>(prec, variant, a, grid, s);
    }
    return hipErrorInvalidValue;
}

// resident workgroups per CU of a variant (for the persistent grid; taken
// from the kernel with the widest copies the variant has: the FP64 kernels
// hold one workgroup per CU either way)
int stage_occupancy(int N, int prec, int variant)
{
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
#define Z4C_OCC(NN, TT, X, Y, Z) \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(                               \
        &nb, k_stage<NN, TT, TT, X, Y, Z, sizeof(TT) == 8 ? 16 : Fp32Slot<NN, X>::best>, 256, 0)
#define Z4C_OCCV(NN, TT)                                                     \
    switch (variant) {                                                        \
    case 0: Z4C_OCC(NN, TT, 8, 8, 4); break;                                  \
    case 1: Z4C_OCC(NN, TT, 16, 4, 4); break;                                 \
    case 2: Z4C_OCC(NN, TT, 8, 4, 8); break;                                  \
    case 3: Z4C_OCC(NN, TT, 16, 8, 2); break;                                 \
    }
    if (prec == 0) {
        if (N == 2) { Z4C_OCCV(2, double) } else if (N == 3) { Z4C_OCCV(3, double) } else { Z4C_OCCV(4, double) }
    } else {
        if (N == 2) { Z4C_OCCV(2, float) } else if (N == 3) { Z4C_OCCV(3, float) } else { Z4C_OCCV(4, float) }
    }
#undef Z4C_OCCV
#undef Z4C_OCC
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

}  // namespace z4c
