// Fused Z4c RHS + classic RK4 stage kernel (one launch per stage covers the
// whole MeshBlockPack; work items are tiles of active cells).
#include "kernels.hpp"
#include "z4c_rhs.hpp"

namespace z4c {

template <int N, class T, class C>
__global__ __launch_bounds__(256) void k_stage(const StageArgs a)
{
    const WorkItem w = a.work[blockIdx.x];
    const BlockDev B = a.blocks[w.block];
    const int t = threadIdx.x;
    const int li = t % w.ni, lj = (t / w.ni) % w.nj, lk = t / (w.ni * w.nj);
    if (lk >= w.nk) return;
    const int i = w.i0 + li, j = w.j0 + lj, k = w.k0 + lk;
    const int g = a.g, E = B.E, n = B.n;
    const int64_t c = ((int64_t)(k + g) * E + (j + g)) * E + (i + g);
    const T* __restrict__ src = (const T*)a.src + B.off + c;
    C rhs[NF], v[NF];
    zone_rhs<N, T, C>(src, B.slab, E, E * E, (C)(1.0 / B.h), a.P, rhs, v);

    const int64_t n3 = (int64_t)n * n * n;
    const int64_t ci = B.ioff + ((int64_t)k * n + j) * n + i;
    if (a.stage == 0) {
#pragma unroll
        for (int f = 0; f < NF; ++f) a.rhs_out[ci + f * n3] = (double)rhs[f];
        return;
    }
    const double dt = a.dt;
    double out[NF];
    const T* __restrict__ U = (const T*)a.U + B.off + c;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const double kf = (double)rhs[f];
        double* Af = a.A + ci + f * n3;
        switch (a.stage) {
        case 1: {
            const double u = (double)v[f];
            out[f] = u + 0.5 * dt * kf;
            *Af = u + dt / 6.0 * kf;
        } break;
        case 2: {
            const double u = (double)U[f * B.slab];
            out[f] = u + 0.5 * dt * kf;
            *Af += dt / 3.0 * kf;
        } break;
        case 3: {
            const double u = (double)U[f * B.slab];
            out[f] = u + dt * kf;
            *Af += dt / 3.0 * kf;
        } break;
        default:
            out[f] = *Af + dt / 6.0 * kf;
        }
    }
    if (a.P.enforce) enforce_zone(out, a.P);
    T* __restrict__ dst = (T*)a.dst + B.off + c;
#pragma unroll
    for (int f = 0; f < NF; ++f) dst[f * B.slab] = (T)out[f];
}

template <int N>
static hipError_t launch_n(int prec, const StageArgs& a, int nwork, hipStream_t s)
{
    if (prec == 0)
        hipLaunchKernelGGL((k_stage<N, double, double>), dim3(nwork), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_stage<N, float, float>), dim3(nwork), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_stage(int N, int prec, const StageArgs& a, int nwork, hipStream_t s)
{
    switch (N) {
    case 2: return launch_n<2>(prec, a, nwork, s);
    case 3: return launch_n<3>(prec, a, nwork, s);
    case 4: return launch_n<4>(prec, a, nwork, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace z4c
