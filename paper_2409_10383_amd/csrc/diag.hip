// Constraint monitors and refinement-criterion reductions.
// Per work item (tile) the kernels write fixed-order partial results; the
// host combines them in work-item order, so results are deterministic.
#include "kernels.hpp"
#include "z4c_rhs.hpp"

namespace z4c {

constexpr int NPART = 8;

// any non-finite value among the 22 fields of the active cells of a tile
// sets the flag (cleared by k_clear_flag, launched just before on the same
// stream)
template <class T>
__global__ __launch_bounds__(256) void k_check_finite(const FiniteArgs a)
{
    const WorkItem w = a.work[blockIdx.x];
    const BlockDev B = a.blocks[w.block];
    const int t = threadIdx.x;
    const int li = t % w.ni, lj = (t / w.ni) % w.nj, lk = t / (w.ni * w.nj);
    if (lk >= w.nk) return;
    const int g = a.g, E = B.E;
    const int64_t cc = ((int64_t)(w.k0 + lk + g) * E + (w.j0 + lj + g)) * E + (w.i0 + li + g);
    const T* p = (const T*)a.src + B.off + cc;
    bool bad = false;
#pragma unroll
    for (int f = 0; f < NF; ++f) bad |= !__builtin_isfinite((double)p[f * B.slab]);
    if (bad) atomicOr(a.flag, 1);
}

__global__ void k_clear_flag(int32_t* flag)
{
    if (threadIdx.x == 0) *flag = 0;
}

hipError_t launch_check_finite(int prec, const FiniteArgs& a, int nwork, hipStream_t s)
{
    hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(64), 0, s, a.flag);
    if (prec == 0)
        hipLaunchKernelGGL(k_check_finite<double>, dim3((unsigned)nwork), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_check_finite<float>, dim3((unsigned)nwork), dim3(256), 0, s, a);
    return hipGetLastError();
}

// fixed-order workgroup reduction of 256 values (sum or max / min)
template <int OP>
__device__ double wg_reduce(double x, double* sh)
{
    const int t = threadIdx.x;
    sh[t] = x;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) {
            const double o = sh[t + s];
            sh[t] = OP == 0 ? sh[t] + o : (OP == 1 ? (o > sh[t] ? o : sh[t]) : (o < sh[t] ? o : sh[t]));
        }
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

template <int N, class T>
__global__ __launch_bounds__(256) void k_constraints(const DiagArgs a)
{
    __shared__ double sh[256];
    const WorkItem w = a.work[blockIdx.x];
    const BlockDev B = a.blocks[w.block];
    const int t = threadIdx.x;
    const int li = t % w.ni, lj = (t / w.ni) % w.nj, lk = t / (w.ni * w.nj);
    const bool live = lk < w.nk;
    const int i = w.i0 + li, j = w.j0 + lj, k = w.k0 + lk;
    const int g = a.g, E = B.E, n = B.n;
    double c[8];
    double H = 0, M2 = 0, T2 = 0, G2 = 0, dv = 0;
    if (live) {
        const int64_t cc = ((int64_t)(k + g) * E + (j + g)) * E + (i + g);
        const T* src = (const T*)a.src + B.off + cc;
        zone_constraints<N, T>(src, B.slab, E, E * E, 1.0 / B.h, a.P, c);
        if (a.per_zone) {
            const int64_t n3 = (int64_t)n * n * n;
            const int64_t ci = (B.ioff / NF) * 8 + ((int64_t)k * n + j) * n + i;
            for (int q = 0; q < 8; ++q) a.per_zone[ci + q * n3] = c[q];
        }
        const double x = B.x0[0] + i * B.h, y = B.x0[1] + j * B.h, zz = B.x0[2] + k * B.h;
        bool keep = true;
        for (int e = 0; e < a.ncentres; ++e) {
            const double dx = x - a.centres[e][0], dy = y - a.centres[e][1], dz = zz - a.centres[e][2];
            if (dx * dx + dy * dy + dz * dz < a.r_exc * a.r_exc) keep = false;
        }
        if (keep) {
            H = c[0];
            M2 = c[1] * c[1] + c[2] * c[2] + c[3] * c[3];
            T2 = c[4] * c[4];
            G2 = c[5] * c[5] + c[6] * c[6] + c[7] * c[7];
            dv = B.h * B.h * B.h;
        }
    }
    double* out = a.partial + (int64_t)blockIdx.x * NPART;
    const double r0 = wg_reduce<0>(H * H * dv, sh);
    const double r1 = wg_reduce<1>(fabs(H), sh);
    const double r2 = wg_reduce<0>(M2 * dv, sh);
    const double r3 = wg_reduce<1>(sqrt(M2), sh);
    const double r4 = wg_reduce<0>(T2 * dv, sh);
    const double r5 = wg_reduce<0>(G2 * dv, sh);
    const double r6 = wg_reduce<0>(dv, sh);
    if (t == 0) {
        out[0] = r0; out[1] = r1; out[2] = r2; out[3] = r3;
        out[4] = r4; out[5] = r5; out[6] = r6; out[7] = 0.0;
    }
}

// per tile: min chi, max |grad chi| (centred, order 2N), min distance to centre
template <int N, class T>
__global__ __launch_bounds__(256) void k_flag_reduce(const DiagArgs a)
{
    __shared__ double sh[256];
    const WorkItem w = a.work[blockIdx.x];
    const BlockDev B = a.blocks[w.block];
    const int t = threadIdx.x;
    const int li = t % w.ni, lj = (t / w.ni) % w.nj, lk = t / (w.ni * w.nj);
    const bool live = lk < w.nk;
    const int i = w.i0 + li, j = w.j0 + lj, k = w.k0 + lk;
    const int g = a.g, E = B.E;
    double cmin = INFINITY, gmax = 0.0, rmin = INFINITY;
    if (live) {
        const int64_t cc = ((int64_t)(k + g) * E + (j + g)) * E + (i + g);
        const T* p = (const T*)a.src + B.off + cc;  // chi is field 0
        cmin = (double)p[0];
        const double ih = 1.0 / B.h;
        const double gx = ih * fd1<N, double>(p, 1), gy = ih * fd1<N, double>(p, E),
                     gz = ih * fd1<N, double>(p, E * E);
        gmax = sqrt(gx * gx + gy * gy + gz * gz);
        const double x = B.x0[0] + i * B.h - a.centres[0][0], y = B.x0[1] + j * B.h - a.centres[0][1],
                     zz = B.x0[2] + k * B.h - a.centres[0][2];
        rmin = sqrt(x * x + y * y + zz * zz);
    }
    const double r0 = wg_reduce<2>(cmin, sh);
    const double r1 = wg_reduce<1>(gmax, sh);
    const double r2 = wg_reduce<2>(rmin, sh);
    if (t == 0) {
        double* out = a.partial + (int64_t)blockIdx.x * NPART;
        out[0] = r0; out[1] = r1; out[2] = r2;
    }
}

template <int N>
static hipError_t launch_diag_n(int prec, const DiagArgs& a, int nwork, hipStream_t s)
{
    if (a.mode == 0) {
        if (prec == 0) hipLaunchKernelGGL((k_constraints<N, double>), dim3(nwork), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_constraints<N, float>), dim3(nwork), dim3(256), 0, s, a);
    } else {
        if (prec == 0) hipLaunchKernelGGL((k_flag_reduce<N, double>), dim3(nwork), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_flag_reduce<N, float>), dim3(nwork), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_diag(int N, int prec, const DiagArgs& a, int nwork, hipStream_t s)
{
    switch (N) {
    case 2: return launch_diag_n<2>(prec, a, nwork, s);
    case 3: return launch_diag_n<3>(prec, a, nwork, s);
    case 4: return launch_diag_n<4>(prec, a, nwork, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace z4c
