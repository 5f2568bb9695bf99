// Same-level ghost fill: every ghost cell of every block takes the value of
// the active cell that covers its centre, after the domain boundary
// condition (periodic wrap, or outflow = clamp to the nearest active cell).
// Ghost cells covered by another refinement level are left to the
// cross-level fill.
#include "kernels.hpp"

namespace z4c {

// ghost cell q of a block (0 <= q < E^3 - n^3) -> (i, j, k) in [0, E)
__device__ __forceinline__ bool ghost_cell(int64_t q, int n, int g, int E, int& i, int& j, int& k)
{
    const int64_t nz = 2LL * g * E * E, ny = 2LL * g * E * n, nx = 2LL * g * n * n;
    if (q < nz) {
        k = (int)(q / ((int64_t)E * E));
        const int64_t r = q % ((int64_t)E * E);
        j = (int)(r / E);
        i = (int)(r % E);
        if (k >= g) k += n;
        return true;
    }
    q -= nz;
    if (q < ny) {
        k = g + (int)(q / (2LL * g * E));
        const int64_t r = q % (2LL * g * E);
        j = (int)(r / E);
        i = (int)(r % E);
        if (j >= g) j += n;
        return true;
    }
    q -= ny;
    if (q < nx) {
        k = g + (int)(q / (2LL * g * n));
        const int64_t r = q % (2LL * g * n);
        j = g + (int)(r / (2 * g));
        i = (int)(r % (2 * g));
        if (i >= g) i += n;
        return true;
    }
    return false;
}

__device__ __forceinline__ int leaf_lookup(const FillArgs& a, int level, const int64_t G[3])
{
    if (level >= a.L.nlev) return -1;
    const int u = a.L.unit;
    const int64_t q0 = G[0] / u, q1 = G[1] / u, q2 = G[2] / u;
    return a.map[a.L.base[level] + (q2 * a.L.dim[level][1] + q1) * a.L.dim[level][0] + q0];
}

template <class T>
__global__ __launch_bounds__(256) void k_fill_same(const FillArgs a)
{
    const int b = blockIdx.y;
    const BlockDev B = a.blocks[b];
    const int n = B.n, g = a.g, E = B.E;
    int i, j, k;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (!ghost_cell(q, n, g, E, i, j, k)) return;
    if (a.skip) {
        const int dx = i < g ? 0 : (i >= g + n ? 2 : 1), dy = j < g ? 0 : (j >= g + n ? 2 : 1),
                  dz = k < g ? 0 : (k >= g + n ? 2 : 1);
        const uint32_t sk = a.skip[b] | (a.skip2 ? a.skip2[b] : 0u);
        if ((sk >> ((dz * 3 + dy) * 3 + dx)) & 1u) return;
    }
    int64_t G[3] = {(int64_t)B.ilo[0] + i - g, (int64_t)B.ilo[1] + j - g, (int64_t)B.ilo[2] + k - g};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int64_t N = (int64_t)a.nroot[d] << B.level;
        if (a.bc == 0) {
            G[d] = G[d] % N;
            if (G[d] < 0) G[d] += N;
        } else {
            G[d] = G[d] < 0 ? 0 : (G[d] >= N ? N - 1 : G[d]);
        }
    }
    const int s = leaf_lookup(a, B.level, G);
    if (s < 0) return;  // covered by another level
    const BlockDev SB = a.blocks[s];
    const int64_t so = SB.off + ((G[2] - SB.ilo[2] + g) * SB.E + (G[1] - SB.ilo[1] + g)) * SB.E +
                       (G[0] - SB.ilo[0] + g);
    const int64_t d = B.off + ((int64_t)k * E + j) * E + i;
    T* r = (T*)a.reg;
#pragma unroll
    for (int f = 0; f < NF; ++f) r[d + f * B.slab] = r[so + f * SB.slab];
}

// Coarse image of a fine block: separable x, y, z passes through LDS (the
// same association order as a direct triple sum: x innermost).  A workgroup
// takes one field of a run of coarse z-planes and marches along it: each
// fine plane a window needs is read once, restricted in x and then in y
// into a ring of the last np planes' y-passes (several new planes per pass
// as the x-pass buffer allows), and every coarse plane is the z-pass over
// its window's np ring entries.  Windows (clamped to the block, as the
// restriction reads only the block's own cells) never move back, so the
// ring holds them.
template <class T, int NP>
__global__ __launch_bounds__(256) void k_restrict_image(const XlevelArgs a)
{
    __shared__ double X[RI_XMAX];    // x-passes of new fine planes: plane, row, column
    __shared__ double Y[RI_YMAX];    // y-passes of the last np fine planes
    const int64_t wi = xcd_run(blockIdx.x, a.nislice * NF);
    if (wi >= a.nislice * NF) return;
    const ImageSlice sl = a.islice[wi / NF];
    const int f = (int)(wi % NF);
    const BlockDev F = a.blocks[sl.block];
    const int n = F.n, m = n >> 1, np = NP ? NP : a.npts, E = F.E, g = (E - n) >> 1;
    const int t = threadIdx.x, ny = sl.ny, x0 = sl.x0, cx = sl.nx;
    int oy0, dy0, oy1, dy1;
    rwin(sl.y0, n, np, oy0, dy0);
    rwin(sl.y0 + ny - 1, n, np, oy1, dy1);
    const int R = oy1 + np - oy0;    // fine rows read per plane
    const int nxq = cx * R, nyq = cx * ny;
    const int pmax = RI_XMAX / nxq;  // new planes per x-pass (the pack checks >= 1)
    T* img = (T*)a.image + sl.img + (int64_t)f * sl.fstride;
    // fine plane 0, row oy0, column 0 of field f
    const T* p = (const T*)a.reg + F.off + (int64_t)f * F.slab + ((int64_t)g * E + (oy0 + g)) * E + g;
    int hi = 0;                      // fine planes below hi are in the ring
    for (int kz = sl.kz; kz < sl.kz + sl.nkz; ++kz) {
        int oz, dz;
        rwin(kz, n, np, oz, dz);
        if (kz == sl.kz) hi = oz;
        while (hi < oz + np) {
            const int nnew = min(oz + np - hi, pmax);
            for (int q = t; q < nnew * nxq; q += 256) {
                const int pl = q / nxq, u = q - pl * nxq, kx = u % cx, r = u / cx;
                int ox, dx;
                rwin(x0 + kx, n, np, ox, dx);
                const T* row = p + ((int64_t)(hi + pl) * E + r) * E + ox;
                const double* wx = a.rw + 8 * dx;
                double s = 0.0;
#pragma unroll
                for (int ix = 0; ix < np; ++ix) s += wx[ix] * (double)row[ix];
                X[q] = s;
            }
            // also orders the previous z-pass's ring reads before the
            // y-pass below overwrites entries
            __syncthreads();
            for (int q = t; q < nnew * nyq; q += 256) {
                const int pl = q / nyq, u = q - pl * nyq, kx = u % cx, cy = u / cx;
                int oy, dy;
                rwin(sl.y0 + cy, n, np, oy, dy);
                const double* wy = a.rw + 8 * dy;
                const double* Xp = X + pl * nxq;
                double s = 0.0;
#pragma unroll
                for (int jy = 0; jy < np; ++jy) s += wy[jy] * Xp[(oy - oy0 + jy) * cx + kx];
                Y[((hi + pl) % np) * nyq + u] = s;
            }
            __syncthreads();
            hi += nnew;
        }
        const double* wz = a.rw + 8 * dz;
        for (int q = t; q < nyq; q += 256) {
            const int kx = q % cx, cy = q / cx;
            double s = 0.0;
#pragma unroll
            for (int kk = 0; kk < np; ++kk) s += wz[kk] * Y[((oz + kk) % np) * nyq + q];
            img[((int64_t)kz * m + (sl.y0 + cy)) * m + x0 + kx] = (T)s;
        }
    }
}

// copies into ghost cells and shadow boxes (sources: active cells, images)
template <class T>
__global__ __launch_bounds__(256) void k_xfer(const XlevelArgs a, int64_t nwork)
{
    const int64_t w = xcd_run(blockIdx.x, nwork);
    const int64_t q = w * blockDim.x + threadIdx.x;
    if (q >= a.nxfer) return;
    const XferItem it = a.xfer[q];
    const T* __restrict__ src = (const T*)((it.kind & 1) ? a.image : a.reg) + it.src;
    T* dst = (T*)((it.kind & 2) ? a.shadow : a.reg) + it.dst;
#pragma unroll
    for (int f = 0; f < NF; ++f) dst[(int64_t)f * it.dst_stride] = src[(int64_t)f * it.src_stride];
}

// prolongation of fine ghosts from the shadow boxes
template <class T>
__global__ __launch_bounds__(256) void k_prolong(const XlevelArgs a)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.nprol) return;
    const ProlongItem it = a.prol[q];
    const BlockDev B = a.blocks[it.block];
    const T* __restrict__ sh = (const T*)a.shadow + it.sh;
    T* dst = (T*)a.reg + it.dst;
    const int np = a.npts;
    const int64_t se = it.se, se3 = it.pad;  // field stride of the shadow box
    const double* wx = a.pw + 8 * (it.parity & 1);
    const double* wy = a.pw + 8 * ((it.parity >> 1) & 1);
    const double* wz = a.pw + 8 * ((it.parity >> 2) & 1);
    for (int f = 0; f < NF; ++f) {
        const T* p = sh + f * se3;
        double acc = 0.0;
        for (int kz = 0; kz < np; ++kz) {
            double az = 0.0;
            for (int jy = 0; jy < np; ++jy) {
                const T* row = p + (kz * se + jy) * se;
                double ay = 0.0;
                for (int ix = 0; ix < np; ++ix) ay += wx[ix] * (double)row[ix];
                az += wy[jy] * ay;
            }
            acc += wz[kz] * az;
        }
        dst[f * B.slab] = (T)acc;
    }
}

// grouped prolongation: one coarse parent, up to 8 fine children, separable
// (x, then y, then z) over the union stencil; one thread per group and field.
// A group may also hold the parent one coarse cell further in y (mask byte
// 1), or those further in y, in z and in both (bytes 1-3): their stencils
// are the first one's shifted by a row, a plane or both, so the thread reads
// the union once (one more row, or row and plane) and every parent's sums
// run in the same order as on its own.
template <class T, int NP>
__global__ __launch_bounds__(256) void k_prolong_group(const XlevelArgs a, int64_t ngx, int64_t nwork)
{
    const int64_t w = xcd_run(blockIdx.x, nwork);
    if (w >= nwork) return;
    const int64_t q = (w % ngx) * blockDim.x + threadIdx.x;
    if (q >= a.npgrp) return;
    const ProlongGroup it = a.pgrp[q];
    const BlockDev B = a.blocks[it.block];
    const T* __restrict__ sh = (const T*)a.shadow + it.sh;
    T* dst = (T*)a.reg + it.dst;
    const int np = NP ? NP : a.npts;
    const int even = (np % 2 == 0);
    const int nu = np + even;          // union stencil points per axis
    const int64_t se = it.se, E = B.E;
    const double* w0 = a.pw;           // parity 0 weights, union points 0..np-1
    const double* w1 = a.pw + 8;       // parity 1 weights, union points even..even+np-1
    const uint32_t mask = (uint32_t)it.mask;
    const int f = (int)(w / ngx);
    const T* p = sh + (int64_t)f * it.fstride;
    // x-pass of one union row
    auto xpass = [&](const T* row, double& ax0, double& ax1) {
        ax0 = 0.0;
        ax1 = 0.0;
#pragma unroll
        for (int ix = 0; ix < (NP ? NP + 1 : 9); ++ix) {
            if (ix >= nu) continue;
            const double v = (double)row[ix];
            if (ix < np) ax0 += w0[ix] * v;
            if (ix >= even) ax1 += w1[ix - even] * v;
        }
    };
    // y-pass term of union row jj of a parent's stencil
    auto yterm = [&](int jj, double ax0, double ax1, double (&ay)[2][2]) {
        if (jj < 0 || jj >= nu) return;
        if (jj < np) { ay[0][0] += w0[jj] * ax0; ay[0][1] += w0[jj] * ax1; }
        if (jj >= even) { ay[1][0] += w1[jj - even] * ax0; ay[1][1] += w1[jj - even] * ax1; }
    };
    // z-pass term of union plane kk of a parent's stencil
    auto zterm = [&](int kk, const double (&ay)[2][2], double (&ac)[2][2][2]) {
        if (kk < 0 || kk >= nu) return;
#pragma unroll
        for (int cy = 0; cy < 2; ++cy)
#pragma unroll
            for (int cx = 0; cx < 2; ++cx) {
                if (kk < np) ac[0][cy][cx] += w0[kk] * ay[cy][cx];
                if (kk >= even) ac[1][cy][cx] += w1[kk - even] * ay[cy][cx];
            }
    };
    // children of parent pb (0: this one, 1: +y, 2: +z, 3: +y+z)
    auto store = [&](int pb, const double (&ac)[2][2][2]) {
        for (int cz = 0; cz < 2; ++cz)
            for (int cy = 0; cy < 2; ++cy)
                for (int cx = 0; cx < 2; ++cx)
                    if (mask & (1u << (8 * pb + cz * 4 + cy * 2 + cx)))
                        dst[((cz + 2 * (pb >> 1)) * E + cy + 2 * (pb & 1)) * E + cx + (int64_t)f * B.slab] =
                            (T)ac[cz][cy][cx];
    };
    if constexpr (sizeof(T) == 8) if (mask >> 16) {
        // four parents (FP64 packs only): nu + 1 planes of nu + 1 rows
        double acc[4][2][2][2] = {};
#pragma unroll 1
        for (int kz = 0; kz <= nu; ++kz) {
            double ay[2][2][2] = {};   // [row shift][cy][cx]
#pragma unroll
            for (int jy = 0; jy < (NP ? NP + 2 : 10); ++jy) {
                if (jy > nu) continue;
                double ax0, ax1;
                xpass(p + (kz * se + jy) * se, ax0, ax1);
                yterm(jy, ax0, ax1, ay[0]);
                yterm(jy - 1, ax0, ax1, ay[1]);
            }
#pragma unroll
            for (int pb = 0; pb < 4; ++pb) zterm(kz - (pb >> 1), ay[pb & 1], acc[pb]);
        }
#pragma unroll
        for (int pb = 0; pb < 4; ++pb) store(pb, acc[pb]);
        return;
    }
    if (mask >> 8) {
        // two parents along y: nu planes of nu + 1 rows
        double acc[2][2][2][2] = {};
#pragma unroll 1
        for (int kz = 0; kz < nu; ++kz) {
            double ay[2][2][2] = {};
#pragma unroll
            for (int jy = 0; jy < (NP ? NP + 2 : 10); ++jy) {
                if (jy > nu) continue;
                double ax0, ax1;
                xpass(p + (kz * se + jy) * se, ax0, ax1);
                yterm(jy, ax0, ax1, ay[0]);
                yterm(jy - 1, ax0, ax1, ay[1]);
            }
            zterm(kz, ay[0], acc[0]);
            zterm(kz, ay[1], acc[1]);
        }
        store(0, acc[0]);
        store(1, acc[1]);
    } else {
        double acc[2][2][2] = {};
#pragma unroll 1
        for (int kz = 0; kz < nu; ++kz) {
            double ay[2][2] = {};
#pragma unroll
            for (int jy = 0; jy < (NP ? NP + 1 : 9); ++jy) {
                if (jy >= nu) continue;
                double ax0, ax1;
                xpass(p + (kz * se + jy) * se, ax0, ax1);
                yterm(jy, ax0, ax1, ay);
            }
            zterm(kz, ay, acc);
        }
        store(0, acc);
    }
}

template <class T, int NP>
static void launch_xlevel_np(const XlevelArgs& a, hipStream_t s, int ph)
{
    const unsigned gx = (unsigned)((a.nxfer + 255) / 256), gp = (unsigned)((a.nprol + 255) / 256);
    const unsigned gg = (unsigned)((a.npgrp + 255) / 256);
    if ((ph & XL_RESTRICT) && a.nislice)
        hipLaunchKernelGGL((k_restrict_image<T, NP>), dim3(xcd_grid(a.nislice * NF)), dim3(256), 0, s, a);
    if ((ph & XL_XFER) && gx) hipLaunchKernelGGL(k_xfer<T>, dim3(xcd_grid(gx)), dim3(256), 0, s, a, (int64_t)gx);
    if ((ph & XL_PROLONG) && gp) hipLaunchKernelGGL(k_prolong<T>, dim3(gp), dim3(256), 0, s, a);
    if ((ph & XL_PROLONG) && gg)
        hipLaunchKernelGGL((k_prolong_group<T, NP>), dim3(xcd_grid((int64_t)gg * NF)), dim3(256), 0, s, a,
                           (int64_t)gg, (int64_t)gg * NF);
}

template <class T>
static void launch_xlevel_t(const XlevelArgs& a, hipStream_t s, int ph)
{
    // stencil widths of the 4th/6th/8th-order ghost depths get unrolled kernels
    switch (a.npts) {
    case 4: launch_xlevel_np<T, 4>(a, s, ph); break;
    case 5: launch_xlevel_np<T, 5>(a, s, ph); break;
    case 6: launch_xlevel_np<T, 6>(a, s, ph); break;
    default: launch_xlevel_np<T, 0>(a, s, ph); break;
    }
}

hipError_t launch_xlevel(int prec, const XlevelArgs& a, hipStream_t s, int phases)
{
    if (prec == 0) launch_xlevel_t<double>(a, s, phases);
    else launch_xlevel_t<float>(a, s, phases);
    return hipGetLastError();
}

hipError_t launch_fill(int prec, const FillArgs& a, int nblocks, hipStream_t s)
{
    dim3 grid((unsigned)((a.maxghost + 255) / 256), (unsigned)nblocks);
    if (prec == 0)
        hipLaunchKernelGGL(k_fill_same<double>, grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_fill_same<float>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace z4c
