// Learned refinement indicator: per-block features, injection onto the even
// sublattice (the 2h pack), h-vs-2h RHS labels, feature normalisation and
// the 16 -> 64 -> 64 -> 1 perceptron (bfloat16 weights and activations,
// float32 accumulation): forward, backward and Adam.
#include "../../include/z4c.h"
#include <mutex>
#include "kernels.hpp"
#include "z4c_rhs.hpp"

namespace z4c {

constexpr int NFEAT = 16;

// ---------------------------------------------------------------- features
// per tile partials: 0 max|d chi| 1 sum|d chi| 2 max|d alpha| 3 sum|d alpha|
// 4 max|dd g~| 5 sum|dd g~| 6 min alpha 7 min chi 8 max|Khat| 9 max|A~|
// 10 max|Theta| 11 max|Gamma~| 12 max|beta| 13 max|dd chi| 14 max|d Khat|
// 15 zone count
template <int N, class T>
__global__ __launch_bounds__(256) void k_features(const FeatArgs a)
{
    __shared__ double sh[256];
    const WorkItem w = a.work[blockIdx.x];
    const BlockDev B = a.blocks[w.block];
    const int t = threadIdx.x;
    const int li = t % w.ni, lj = (t / w.ni) % w.nj, lk = t / (w.ni * w.nj);
    const bool live = lk < w.nk;
    const int g = a.g, E = B.E;
    double v[NFEAT];
    for (int q = 0; q < NFEAT; ++q) v[q] = 0.0;
    v[6] = INFINITY;
    v[7] = INFINITY;
    if (live) {
        const int i = w.i0 + li, j = w.j0 + lj, k = w.k0 + lk;
        const int64_t cz = ((int64_t)(k + g) * E + (j + g)) * E + (i + g);
        const T* z = (const T*)a.src + B.off + cz;
        const int64_t sl = B.slab;
        const int st[3] = {1, E, E * E};
        const double ih = 1.0 / B.h, ih2 = ih * ih;
        double gc = 0, ga = 0, gk = 0;
        for (int d = 0; d < 3; ++d) {
            const double x = ih * fd1<N, double>(z + F_CHI * sl, st[d]);
            const double y = ih * fd1<N, double>(z + F_ALPHA * sl, st[d]);
            const double q = ih * fd1<N, double>(z + F_KH * sl, st[d]);
            gc += x * x; ga += y * y; gk += q * q;
        }
        gc = sqrt(gc); ga = sqrt(ga); gk = sqrt(gk);
        double ddg = 0, ddc = 0;
        for (int fi = 0; fi < 7; ++fi) {
            const T* p = z + (fi == 6 ? F_CHI : F_GXX + fi) * sl;
            for (int qq = 0; qq < 6; ++qq) {
                const int aa = SA(qq), bb = SB(qq);
                const double s = ih2 * ((aa == bb) ? fd2<N, double>(p, st[aa]) : fdmix<N, double>(p, st[aa], st[bb]));
                if (fi == 6) ddc = fmax(ddc, fabs(s));
                else ddg = fmax(ddg, fabs(s));
            }
        }
        double A2 = 0, G2 = 0, b2 = 0;
        for (int qq = 0; qq < 6; ++qq) {
            const double x = (double)z[(F_AXX + qq) * sl];
            A2 += SW(qq) * x * x;
        }
        for (int d = 0; d < 3; ++d) {
            const double x = (double)z[(F_GAMX + d) * sl], y = (double)z[(F_BETAX + d) * sl];
            G2 += x * x; b2 += y * y;
        }
        v[0] = gc; v[1] = gc; v[2] = ga; v[3] = ga; v[4] = ddg; v[5] = ddg;
        v[6] = (double)z[F_ALPHA * sl]; v[7] = (double)z[F_CHI * sl];
        v[8] = fabs((double)z[F_KH * sl]); v[9] = sqrt(A2); v[10] = fabs((double)z[F_TH * sl]);
        v[11] = sqrt(G2); v[12] = sqrt(b2); v[13] = ddc; v[14] = gk; v[15] = 1.0;
    }
    double* out = a.partial + (int64_t)blockIdx.x * NFEAT;
    for (int q = 0; q < NFEAT; ++q) {
        // op: 0 sum, 1 max, 2 min
        const int op = (q == 1 || q == 3 || q == 5 || q == 15) ? 0 : ((q == 6 || q == 7) ? 2 : 1);
        sh[t] = v[q];
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (t < s) {
                const double o = sh[t + s];
                sh[t] = op == 0 ? sh[t] + o : (op == 1 ? fmax(sh[t], o) : fmin(sh[t], o));
            }
            __syncthreads();
        }
        if (t == 0) out[q] = sh[0];
        __syncthreads();
    }
}

// combine the tiles of each block in work-list order
__global__ void k_feat_combine(const FeatArgs a)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.nblocks) return;
    double f[NFEAT];
    for (int q = 0; q < NFEAT; ++q) f[q] = 0.0;
    f[6] = INFINITY;
    f[7] = INFINITY;
    for (int w = a.first_work[b]; w < a.first_work[b + 1]; ++w) {
        const double* p = a.partial + (int64_t)w * NFEAT;
        for (int q = 0; q < NFEAT; ++q) {
            if (q == 1 || q == 3 || q == 5 || q == 15) f[q] += p[q];
            else if (q == 6 || q == 7) f[q] = fmin(f[q], p[q]);
            else f[q] = fmax(f[q], p[q]);
        }
    }
    const double cnt = f[15];
    f[1] /= cnt; f[3] /= cnt; f[5] /= cnt;
    f[15] = log2(a.blocks[b].h);
    for (int q = 0; q < NFEAT; ++q) a.feat[(int64_t)b * NFEAT + q] = f[q];
}

// ----------------------------------------------------- 2h injection, labels
template <class T>
__global__ __launch_bounds__(256) void k_inject(const InjectArgs a)
{
    const int b = blockIdx.y;
    const BlockDev C2 = a.blocks2[b], F = a.blocks1[b];
    const int n2 = C2.n;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)n2 * n2 * n2) return;
    const int i = (int)(q % n2), j = (int)((q / n2) % n2), k = (int)(q / ((int64_t)n2 * n2));
    const int64_t s = F.off + ((int64_t)(2 * k + a.g1) * F.E + (2 * j + a.g1)) * F.E + (2 * i + a.g1);
    const int64_t d = C2.off + ((int64_t)(k + a.g2) * C2.E + (j + a.g2)) * C2.E + (i + a.g2);
    const T* src = (const T*)a.src;
    T* dst = (T*)a.dst;
    for (int f = 0; f < NF; ++f) dst[d + f * C2.slab] = src[s + f * F.slab];
}

// per 2h tile: sum over fields and active cells of (rhs_h(2J) - rhs_2h(J))^2
__global__ __launch_bounds__(256) void k_labels(const LabelArgs a)
{
    __shared__ double sh[256];
    const WorkItem w = a.work2[blockIdx.x];
    const BlockDev C2 = a.blocks2[w.block], F = a.blocks1[w.block];
    const int t = threadIdx.x;
    const int li = t % w.ni, lj = (t / w.ni) % w.nj, lk = t / (w.ni * w.nj);
    double s = 0.0;
    if (lk < w.nk) {
        const int i = w.i0 + li, j = w.j0 + lj, k = w.k0 + lk;
        const int n2 = C2.n, n1 = F.n;
        const int64_t c2 = C2.ioff + ((int64_t)k * n2 + j) * n2 + i;
        const int64_t c1 = F.ioff + ((int64_t)(2 * k) * n1 + 2 * j) * n1 + 2 * i;
        const int64_t s2 = (int64_t)n2 * n2 * n2, s1 = (int64_t)n1 * n1 * n1;
        for (int f = 0; f < NF; ++f) {
            const double d = a.rhs1[c1 + f * s1] - a.rhs2[c2 + f * s2];
            s += d * d;
        }
    }
    sh[t] = s;
    __syncthreads();
    for (int r = 128; r > 0; r >>= 1) {
        if (t < r) sh[t] += sh[t + r];
        __syncthreads();
    }
    if (t == 0) a.partial[blockIdx.x] = sh[0];
}

// ------------------------------------------------------------------- MLP
__device__ __forceinline__ float bf16r(float x)
{
    // round to bfloat16, nearest with ties to even (inputs are finite)
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xFFFF0000u);
}

constexpr int H = 64;
// samples per partial-gradient slice of the backward pass
constexpr int MLP_SLICE = Z4C_MLP_SLICE;
constexpr int OW1 = 0, OB1 = OW1 + H * NFEAT, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H,
              OB3 = OW3 + H, NPARAM = OB3 + 1;

// features -> network inputs: phi(raw) z-scored, phi = log10(|x| + 1e-12)
// for features 0..14, identity for log2 dx
__global__ void k_normalize(const double* raw, int B, const double* stats, float* X)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)B * NFEAT) return;
    const int k = (int)(q % NFEAT);
    const double r = raw[q];
    const double phi = k < 15 ? log10(fabs(r) + 1e-12) : r;
    X[q] = (float)((phi - stats[k]) / stats[16 + k]);
}

// per-feature mean, standard deviation, min, max of phi over the batch
__global__ void k_feat_stats(const double* raw, int B, double* stats)
{
    __shared__ double s1[256], s2[256], mn[256], mx[256];
    const int k = blockIdx.x, t = threadIdx.x;
    double a = 0, b = 0, lo = INFINITY, hi = -INFINITY;
    for (int i = t; i < B; i += 256) {
        const double r = raw[(int64_t)i * NFEAT + k];
        const double phi = k < 15 ? log10(fabs(r) + 1e-12) : r;
        a += phi; b += phi * phi; lo = fmin(lo, phi); hi = fmax(hi, phi);
    }
    s1[t] = a; s2[t] = b; mn[t] = lo; mx[t] = hi;
    __syncthreads();
    for (int r = 128; r > 0; r >>= 1) {
        if (t < r) {
            s1[t] += s1[t + r]; s2[t] += s2[t + r];
            mn[t] = fmin(mn[t], mn[t + r]); mx[t] = fmax(mx[t], mx[t + r]);
        }
        __syncthreads();
    }
    if (t == 0) {
        const double mu = s1[0] / B;
        double var = s2[0] / B - mu * mu;
        const double sd = var > 1e-24 ? sqrt(var) : 1.0;
        stats[k] = mu; stats[16 + k] = sd; stats[32 + k] = mn[0]; stats[48 + k] = mx[0];
    }
}

// forward: one sample per thread, rounded weights staged in LDS
__global__ __launch_bounds__(256) void k_mlp_fwd(const float* P, const float* X, int B, float* Y,
                                                 float* cache)
{
    __shared__ float w1[H * NFEAT], w2[H * H], w3[H], b1[H], b2[H];
    for (int q = threadIdx.x; q < H * H; q += 256) w2[q] = bf16r(P[OW2 + q]);
    for (int q = threadIdx.x; q < H * NFEAT; q += 256) w1[q] = bf16r(P[OW1 + q]);
    for (int q = threadIdx.x; q < H; q += 256) {
        w3[q] = bf16r(P[OW3 + q]);
        b1[q] = P[OB1 + q];
        b2[q] = P[OB2 + q];
    }
    __syncthreads();
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B) return;
    float x[NFEAT], h1[H];
    for (int k = 0; k < NFEAT; ++k) x[k] = bf16r(X[(int64_t)s * NFEAT + k]);
    for (int o = 0; o < H; ++o) {
        float acc = b1[o];
        for (int k = 0; k < NFEAT; ++k) acc += w1[o * NFEAT + k] * x[k];
        if (cache) cache[(int64_t)s * 2 * H + o] = acc;
        h1[o] = bf16r(acc > 0.f ? acc : 0.f);
    }
    float y = P[OB3];
    for (int o = 0; o < H; ++o) {
        float acc = b2[o];
        for (int k = 0; k < H; ++k) acc += w2[o * H + k] * h1[k];
        if (cache) cache[(int64_t)s * 2 * H + H + o] = acc;
        y += w3[o] * bf16r(acc > 0.f ? acc : 0.f);
    }
    Y[s] = y;
}

// backward, step 1: per-sample output error and hidden-layer deltas
// work layout per sample: [0,H) delta1, [H,2H) delta2, [2H] dy
__global__ __launch_bounds__(256) void k_mlp_bwd_delta(const float* P, const float* Y, const float* T,
                                                       const float* cache, int B, float* work)
{
    __shared__ float w2[H * H], w3[H];
    for (int q = threadIdx.x; q < H * H; q += 256) w2[q] = bf16r(P[OW2 + q]);
    for (int q = threadIdx.x; q < H; q += 256) w3[q] = bf16r(P[OW3 + q]);
    __syncthreads();
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B) return;
    const float* a = cache + (int64_t)s * 2 * H;
    float* wk = work + (int64_t)s * (2 * H + 1);
    const float dy = 2.f * (Y[s] - T[s]) / (float)B;
    float d2[H];
    for (int o = 0; o < H; ++o) d2[o] = a[H + o] > 0.f ? dy * w3[o] : 0.f;
    for (int k = 0; k < H; ++k) {
        float acc = 0.f;
        for (int o = 0; o < H; ++o) acc += w2[o * H + k] * d2[o];
        wk[k] = a[k] > 0.f ? acc : 0.f;
    }
    for (int o = 0; o < H; ++o) wk[H + o] = d2[o];
    wk[2 * H] = dy;
}

// backward, step 2: partial sums of the weight gradients over slices of
// MLP_SLICE samples (dW = delta^T x per layer, db = sum of delta), one
// workgroup per slice; the slice's deltas and layer inputs are staged in LDS
// and each thread sums its parameters over the slice's samples in order.
// partial layout: [slice][NPARAM]
__global__ __launch_bounds__(256) void k_mlp_bwd_partial(const float* X, const float* cache,
                                                         const float* work, int B, float* partial)
{
    constexpr int W = 2 * H + 1;              // deltas per sample in work
    __shared__ float d[MLP_SLICE][W];         // delta1, delta2, dy
    __shared__ float x[MLP_SLICE][NFEAT];     // bf16 inputs
    __shared__ float h[MLP_SLICE][2 * H];     // bf16 relu(a1), relu(a2)
    const int s0 = blockIdx.x * MLP_SLICE;
    const int ns = min(MLP_SLICE, B - s0);
    for (int q = threadIdx.x; q < ns * W; q += 256) d[q / W][q % W] = work[(int64_t)s0 * W + q];
    for (int q = threadIdx.x; q < ns * NFEAT; q += 256)
        x[q / NFEAT][q % NFEAT] = bf16r(X[(int64_t)s0 * NFEAT + q]);
    for (int q = threadIdx.x; q < ns * 2 * H; q += 256) {
        const float v = cache[(int64_t)s0 * 2 * H + q];
        h[q / (2 * H)][q % (2 * H)] = bf16r(v > 0.f ? v : 0.f);
    }
    __syncthreads();
    float* out = partial + (int64_t)blockIdx.x * NPARAM;
    for (int q = threadIdx.x; q < NPARAM; q += 256) {
        float acc = 0.f;
        if (q < OB1) {  // W1[o][k] : delta1_o * x_k
            const int o = q / NFEAT, k = q % NFEAT;
            for (int s = 0; s < ns; ++s) acc += d[s][o] * x[s][k];
        } else if (q < OW2) {
            const int o = q - OB1;
            for (int s = 0; s < ns; ++s) acc += d[s][o];
        } else if (q < OB2) {  // W2[o][k] : delta2_o * h1_k
            const int o = (q - OW2) / H, k = (q - OW2) % H;
            for (int s = 0; s < ns; ++s) acc += d[s][H + o] * h[s][k];
        } else if (q < OW3) {
            const int o = q - OB2;
            for (int s = 0; s < ns; ++s) acc += d[s][H + o];
        } else if (q < OB3) {  // W3[k] : dy * h2_k
            const int k = q - OW3;
            for (int s = 0; s < ns; ++s) acc += d[s][2 * H] * h[s][H + k];
        } else {
            for (int s = 0; s < ns; ++s) acc += d[s][2 * H];
        }
        out[q] = acc;
    }
}

// backward, step 3: one thread per parameter sums the slices in order
__global__ __launch_bounds__(256) void k_mlp_bwd_reduce(const float* partial, int nslice, float* G)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= NPARAM) return;
    float acc = 0.f;
    for (int sl = 0; sl < nslice; ++sl) acc += partial[(int64_t)sl * NPARAM + q];
    G[q] = acc;
}

__global__ void k_mlp_loss(const float* Y, const float* T, int B, float* loss)
{
    __shared__ float sh[256];
    float a = 0.f;
    for (int s = threadIdx.x; s < B; s += 256) {
        const float d = Y[s] - T[s];
        a += d * d;
    }
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int r = 128; r > 0; r >>= 1) {
        if ((int)threadIdx.x < r) sh[threadIdx.x] += sh[threadIdx.x + r];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = sh[0] / (float)B;
}

__global__ void k_mlp_adam(float* P, const float* G, float* M, float* V, int n, float lr, float b1,
                           float b2, float eps, float c1, float c2)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const float g = G[q];
    const float m = b1 * M[q] + (1.f - b1) * g;
    const float v = b2 * V[q] + (1.f - b2) * g * g;
    M[q] = m;
    V[q] = v;
    P[q] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// ------------------------------------------------------------------ launch
hipError_t launch_features(int N, int prec, const FeatArgs& a, int nwork, hipStream_t s)
{
#define Z4C_FEAT(NN)                                                                              \
    if (prec == 0) hipLaunchKernelGGL((k_features<NN, double>), dim3(nwork), dim3(256), 0, s, a); \
    else hipLaunchKernelGGL((k_features<NN, float>), dim3(nwork), dim3(256), 0, s, a);
    switch (N) {
    case 2: Z4C_FEAT(2) break;
    case 3: Z4C_FEAT(3) break;
    case 4: Z4C_FEAT(4) break;
    default: return hipErrorInvalidValue;
    }
#undef Z4C_FEAT
    hipLaunchKernelGGL(k_feat_combine, dim3((a.nblocks + 127) / 128), dim3(128), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_inject(int prec, const InjectArgs& a, int nblocks, int maxcells, hipStream_t s)
{
    dim3 grid((unsigned)((maxcells + 255) / 256), (unsigned)nblocks);
    if (prec == 0) hipLaunchKernelGGL(k_inject<double>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_inject<float>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_labels(const LabelArgs& a, int nwork2, hipStream_t s)
{
    hipLaunchKernelGGL(k_labels, dim3(nwork2), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* P, const float* X, int B, float* Y, float* cache, hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_fwd, dim3((B + 255) / 256), dim3(256), 0, s, P, X, B, Y, cache);
    return hipGetLastError();
}

hipError_t launch_mlp_backward(const float* P, const float* X, const float* Y, const float* T,
                               const float* cache, int B, float* G, float* loss, float* work, hipStream_t s)
{
    const int nslice = (B + MLP_SLICE - 1) / MLP_SLICE;
    float* partial = work + (int64_t)B * (2 * H + 1);
    hipLaunchKernelGGL(k_mlp_bwd_delta, dim3((B + 255) / 256), dim3(256), 0, s, P, Y, T, cache, B, work);
    hipLaunchKernelGGL(k_mlp_bwd_partial, dim3(nslice), dim3(256), 0, s, X, cache, work, B, partial);
    hipLaunchKernelGGL(k_mlp_bwd_reduce, dim3((NPARAM + 255) / 256), dim3(256), 0, s, partial, nslice, G);
    if (loss) hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(256), 0, s, Y, T, B, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float* P, const float* G, float* M, float* V, int step, float lr, float b1,
                           float b2, float eps, hipStream_t s)
{
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_mlp_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, s, P, G, M, V, NPARAM, lr,
                       b1, b2, eps, c1, c2);
    return hipGetLastError();
}

// Learned refinement flags of one block per thread: +1 if the prediction
// exceeds tau_ref, -1 below tau_deref, else 0; a block whose prediction or
// phi(features) is non-finite or outside the training range widened by 10 %
// takes the dchi-max flag instead (max|d chi| > thr: +1, < thr/2: -1);
// min chi < chi_thr forces +1; no +1 at level_max, no -1 at level 0.
__global__ void k_learned_flags(const double* feat, const float* Y, const BlockDev* blocks, int nb,
                                const LearnedRule r, int8_t* flags, int8_t* fallback)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const double* f = feat + (int64_t)b * NFEAT;
    const double y = (double)Y[b];
    bool ood = !isfinite(y);
    for (int k = 0; k < NFEAT; ++k) {
        const double phi = k < 15 ? log10(fabs(f[k]) + 1e-12) : f[k];
        const double lo = r.lo[k], hi = r.hi[k], pad = 0.1 * (hi - lo);
        if (!isfinite(phi) || phi < lo - pad || phi > hi + pad) ood = true;
    }
    int fl;
    if (ood) fl = f[0] > r.dchi_thr ? 1 : (f[0] < 0.5 * r.dchi_thr ? -1 : 0);
    else fl = y > r.tau_ref ? 1 : (y < r.tau_deref ? -1 : 0);
    if (f[7] < r.chi_thr) fl = 1;
    const int lev = blocks[b].level;
    if (fl > 0 && lev >= r.level_max) fl = 0;
    if (fl < 0 && lev == 0) fl = 0;
    flags[b] = (int8_t)fl;
    fallback[b] = ood ? 1 : 0;
}

hipError_t launch_learned_flags(const double* feat, const float* Y, const BlockDev* blocks, int nb,
                                const LearnedRule& r, int8_t* flags, int8_t* fallback, hipStream_t s)
{
    hipLaunchKernelGGL(k_learned_flags, dim3((nb + 255) / 256), dim3(256), 0, s, feat, Y, blocks, nb, r,
                       flags, fallback);
    return hipGetLastError();
}

hipError_t launch_normalize(const double* raw, int B, const double* stats, float* X, hipStream_t s)
{
    hipLaunchKernelGGL(k_normalize, dim3((B * NFEAT + 255) / 256), dim3(256), 0, s, raw, B, stats, X);
    return hipGetLastError();
}

hipError_t launch_feat_stats(const double* raw, int B, double* stats, hipStream_t s)
{
    hipLaunchKernelGGL(k_feat_stats, dim3(NFEAT), dim3(256), 0, s, raw, B, stats);
    return hipGetLastError();
}

}  // namespace z4c

// ------------------------------------------------ allocation-free backward
// Work buffer of z4c_mlp_backward_noalloc for up to Z4C_MLP_NOALLOC_MAXB
// samples: every GPU the library runs on holds its own copy until the
// process ends.  Host code never passes the array's name to a kernel: it
// takes the device address hipGetSymbolAddress returns on each device.
static __device__ __align__(256) float scratch[Z4C_MLP_WORK(Z4C_MLP_NOALLOC_MAXB)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
float* scratch_dev[kMaxDevices];   // address of `scratch` on each device
}  // namespace

extern "C" int z4c_mlp_backward_noalloc(const void* params, const void* X, const void* Y, const void* T,
                                        const void* cache, int32_t B, void* grad, void* loss, void* stream)
{
    if (!params || !X || !Y || !T || !cache || !grad || B < 1) return Z4C_EINVAL;
    if (B > Z4C_MLP_NOALLOC_MAXB) return Z4C_EINVAL;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return Z4C_EDEVICE;
    float* work = nullptr;
    {
        std::lock_guard<std::mutex> lock(scratch_mu);
        if (!scratch_dev[dev]) {
            void* ptr = nullptr;
            if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return Z4C_EDEVICE;
            scratch_dev[dev] = static_cast<float*>(ptr);
        }
        work = scratch_dev[dev];
    }
    // every value the kernels read from the work buffer is written earlier in
    // the same call (deltas, then every slice's partial sums): nothing to clear
    return z4c::launch_mlp_backward(static_cast<const float*>(params), static_cast<const float*>(X),
                                    static_cast<const float*>(Y), static_cast<const float*>(T),
                                    static_cast<const float*>(cache), B, static_cast<float*>(grad),
                                    static_cast<float*>(loss), work, static_cast<hipStream_t>(stream)) ==
                   hipSuccess
               ? Z4C_OK
               : Z4C_EDEVICE;
}
