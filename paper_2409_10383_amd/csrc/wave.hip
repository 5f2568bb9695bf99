// Wave extraction and puncture tracking (Sec. 3.4): the outgoing Weyl
// scalar Psi4 at every zone in a coordinate tetrad, cubic Lagrange
// interpolation of zone data at arbitrary points (spheres, punctures),
// spin-weight -2 spherical-harmonic projection on a quadrature sphere, and
// an RK4 puncture tracker advanced with the evolution's own stages.
#include <cmath>
#include <cstring>

#include "pack.hpp"
#include "z4c_rhs.hpp"

namespace z4c {

// Psi4 = -(E_ij - i B_ij) mbar^i mbar^j at one zone (pointer to its cell in
// the ghosted block, derivatives by the order-2N centred stencils).
//   gamma_ij = g~_ij / chi, K_ij = A~_ij / chi + gamma_ij (Khat + 2 Theta) / 3,
//   E_ij = R_ij - K_ik K^k_j + trK K_ij, B_ij = sym(eps_i^kl D_k K_lj),
//   tetrad: Gram-Schmidt of (x - origin), eps(u, x - origin), u = (-y, x, 0)
//   -> e_r, e_th, e_ph;  m = (e_th + i e_ph) / sqrt 2.
template <int N, class T>
__device__ void zone_psi4(const T* __restrict__ z, int64_t slab, int sy, int sz, double ih,
                          const double x[3], double out[2])
{
    using C = double;
    const int st[3] = {1, sy, sz};
    auto cen = [&](int f) { return (C)z[f * slab]; };
    const C chi = cen(F_CHI), Kt = cen(F_KH) + 2.0 * cen(F_TH), ic = 1.0 / chi;
    C gam[6], A[6], dgam[3][6], dA[3][6], dchi[3], dK[3], ddchi[6], ddgam[6][6];
#pragma unroll
    for (int p = 0; p < 6; ++p) {
        gam[p] = cen(F_GXX + p) * ic;
        A[p] = cen(F_AXX + p);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        dchi[a] = ih * fd1<N, C>(z + F_CHI * slab, st[a]);
        dK[a] = ih * (fd1<N, C>(z + F_KH * slab, st[a]) + 2.0 * fd1<N, C>(z + F_TH * slab, st[a]));
#pragma unroll
        for (int p = 0; p < 6; ++p) {
            dgam[a][p] = (ih * fd1<N, C>(z + (F_GXX + p) * slab, st[a]) - gam[p] * dchi[a]) * ic;
            dA[a][p] = ih * fd1<N, C>(z + (F_AXX + p) * slab, st[a]);
        }
    }
    const C ih2 = ih * ih;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const int a = SA(q), b = SB(q);
        const T* pc = z + F_CHI * slab;
        ddchi[q] = ih2 * ((a == b) ? fd2<N, C>(pc, st[a]) : fdmix<N, C>(pc, st[a], st[b]));
#pragma unroll
        for (int p = 0; p < 6; ++p) {
            const T* pf = z + (F_GXX + p) * slab;
            const C dd = ih2 * ((a == b) ? fd2<N, C>(pf, st[a]) : fdmix<N, C>(pf, st[a], st[b]));
            ddgam[q][p] = (dd - dgam[a][p] * dchi[b] - dgam[b][p] * dchi[a] - gam[p] * ddchi[q]) * ic;
        }
    }
    C Kij[6], dKij[3][6];
#pragma unroll
    for (int p = 0; p < 6; ++p) Kij[p] = A[p] * ic + gam[p] * Kt * (1.0 / 3.0);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int p = 0; p < 6; ++p)
            dKij[a][p] = (dA[a][p] - A[p] * dchi[a] * ic) * ic + dgam[a][p] * Kt * (1.0 / 3.0) +
                         gam[p] * dK[a] * (1.0 / 3.0);
    // inverse metric, sqrt det
    C gu[6];
    const C c0 = gam[3] * gam[5] - gam[4] * gam[4], c1 = gam[2] * gam[4] - gam[1] * gam[5],
            c2 = gam[1] * gam[4] - gam[2] * gam[3];
    const C det = gam[0] * c0 + gam[1] * c1 + gam[2] * c2, idt = 1.0 / det;
    gu[0] = c0 * idt; gu[1] = c1 * idt; gu[2] = c2 * idt;
    gu[3] = (gam[0] * gam[5] - gam[2] * gam[2]) * idt;
    gu[4] = (gam[1] * gam[2] - gam[0] * gam[4]) * idt;
    gu[5] = (gam[0] * gam[3] - gam[1] * gam[1]) * idt;
    const C sg = sqrt(det);
    // Christoffels: Gl[l][p] = (d_i g_jl + d_j g_il - d_l g_ij)/2, Gu[k][p] = g^kl Gl[l][p]
    C Gl[3][6], Gu[3][6];
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
        for (int p = 0; p < 6; ++p) {
            const int i = SA(p), j = SB(p);
            Gl[l][p] = 0.5 * (dgam[i][S(j, l)] + dgam[j][S(i, l)] - dgam[l][p]);
        }
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int p = 0; p < 6; ++p)
            Gu[k][p] = gu[S(k, 0)] * Gl[0][p] + gu[S(k, 1)] * Gl[1][p] + gu[S(k, 2)] * Gl[2][p];
    // Ricci: R_ij = d_k G^k_ij - d_j G^k_ik + G^k_kq G^q_ij - G^k_jq G^q_ik, with
    // d_m G^k_ij = (d_m g^kl) Gl[l][ij] + g^kl d_m Gl[l][ij]
    C R[6];
#pragma unroll
    for (int p = 0; p < 6; ++p) R[p] = 0.0;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        // d_m g^kl = -g^ka g^lb d_m g_ab
        C dgu[6];
#pragma unroll
        for (int r = 0; r < 6; ++r) {
            const int k = SA(r), l = SB(r);
            C s = 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) s -= gu[S(k, a)] * gu[S(l, b)] * dgam[m][S(a, b)];
            dgu[r] = s;
        }
        // d_m Gl[l][p]
        C dGl[3][6];
#pragma unroll
        for (int l = 0; l < 3; ++l)
#pragma unroll
            for (int p = 0; p < 6; ++p) {
                const int i = SA(p), j = SB(p);
                dGl[l][p] = 0.5 * (ddgam[S(m, i)][S(j, l)] + ddgam[S(m, j)][S(i, l)] - ddgam[S(m, l)][p]);
            }
        // d_m G^k_(p) for all k, p
#pragma unroll
        for (int p = 0; p < 6; ++p) {
            const int i = SA(p), j = SB(p);
            // + d_k G^k_ij with k = m
            {
                C s = 0.0;
#pragma unroll
                for (int l = 0; l < 3; ++l) s += dgu[S(m, l)] * Gl[l][p] + gu[S(m, l)] * dGl[l][p];
                R[p] += s;
            }
            // - d_j G^k_ik with j = m: contributes to R_ij for this i (and R_ji)
            if (j == m) {
                C s = 0.0;
#pragma unroll
                for (int k = 0; k < 3; ++k)
#pragma unroll
                    for (int l = 0; l < 3; ++l) s += dgu[S(k, l)] * Gl[l][S(i, k)] + gu[S(k, l)] * dGl[l][S(i, k)];
                R[p] -= s;
            }
        }
    }
#pragma unroll
    for (int p = 0; p < 6; ++p) {
        const int i = SA(p), j = SB(p);
        C s = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int q = 0; q < 3; ++q) s += Gu[k][S(k, q)] * Gu[q][p] - Gu[k][S(j, q)] * Gu[q][S(i, k)];
        R[p] += s;
    }
    C trK = 0.0;
#pragma unroll
    for (int p = 0; p < 6; ++p) trK += SW(p) * gu[p] * Kij[p];
    C E[6];
#pragma unroll
    for (int p = 0; p < 6; ++p) {
        const int i = SA(p), j = SB(p);
        C kk = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int l = 0; l < 3; ++l) kk += Kij[S(i, k)] * gu[S(k, l)] * Kij[S(l, j)];
        E[p] = R[p] - kk + trK * Kij[p];
    }
    // D_k K_lj (symmetric in l, j)
    C DK[3][6];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int p = 0; p < 6; ++p) {
            const int l = SA(p), j = SB(p);
            C s = dKij[k][p];
#pragma unroll
            for (int m = 0; m < 3; ++m) s -= Gu[m][S(k, l)] * Kij[S(m, j)] + Gu[m][S(k, j)] * Kij[S(l, m)];
            DK[k][p] = s;
        }
    // B_ij = sym(gamma_im eps^mkl D_k K_lj), eps^mkl = [mkl] / sqrt(det)
    C Braw[3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        // c^m_j = eps^mkl D_k K_lj
        C cm[3];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const int k1 = (m + 1) % 3, l1 = (m + 2) % 3;
            cm[m] = (DK[k1][S(l1, j)] - DK[l1][S(k1, j)]) / sg;
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) Braw[i][j] = gam[S(i, 0)] * cm[0] + gam[S(i, 1)] * cm[1] + gam[S(i, 2)] * cm[2];
    }
    C Bm[6];
#pragma unroll
    for (int p = 0; p < 6; ++p) Bm[p] = 0.5 * (Braw[SA(p)][SB(p)] + Braw[SB(p)][SA(p)]);
    // tetrad
    auto dot = [&](const C* a, const C* b) {
        return gam[0] * a[0] * b[0] + gam[3] * a[1] * b[1] + gam[5] * a[2] * b[2] +
               gam[1] * (a[0] * b[1] + a[1] * b[0]) + gam[2] * (a[0] * b[2] + a[2] * b[0]) +
               gam[4] * (a[1] * b[2] + a[2] * b[1]);
    };
    const C v[3] = {x[0], x[1], x[2]}, u[3] = {-x[1], x[0], 0.0};
    // w_d = sqrt(det) [dbc] u^b v^c, w^a = g^ad w_d
    const C wl[3] = {sg * (u[1] * v[2] - u[2] * v[1]), sg * (u[2] * v[0] - u[0] * v[2]),
                     sg * (u[0] * v[1] - u[1] * v[0])};
    C w[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) w[a] = gu[S(a, 0)] * wl[0] + gu[S(a, 1)] * wl[1] + gu[S(a, 2)] * wl[2];
    const C uu = dot(u, u), vv = dot(v, v);
    if (!(uu > 1e-24 * vv) || !(vv > 0.0)) { out[0] = out[1] = 0.0; return; }
    C er[3], et[3], ep[3];
    const C iv = 1.0 / sqrt(vv);
#pragma unroll
    for (int a = 0; a < 3; ++a) er[a] = v[a] * iv;
    const C wr = dot(w, er);
#pragma unroll
    for (int a = 0; a < 3; ++a) et[a] = w[a] - wr * er[a];
    const C it = 1.0 / sqrt(dot(et, et));
#pragma unroll
    for (int a = 0; a < 3; ++a) et[a] *= it;
    const C ur = dot(u, er), ut = dot(u, et);
#pragma unroll
    for (int a = 0; a < 3; ++a) ep[a] = u[a] - ur * er[a] - ut * et[a];
    const C ipn = 1.0 / sqrt(dot(ep, ep));
#pragma unroll
    for (int a = 0; a < 3; ++a) ep[a] *= ipn;
    C EP = 0, EQ = 0, BP = 0, BQ = 0;
#pragma unroll
    for (int p = 0; p < 6; ++p) {
        const int i = SA(p), j = SB(p);
        // P^ij = (e_th^i e_th^j - e_ph^i e_ph^j)/2, Q^ij = (e_th^i e_ph^j + e_ph^i e_th^j)/2
        const C w2 = SW(p);
        const C P = 0.5 * (et[i] * et[j] - ep[i] * ep[j]);
        const C Q = 0.5 * (et[i] * ep[j] + ep[i] * et[j]);
        EP += w2 * E[p] * P; EQ += w2 * E[p] * Q;
        BP += w2 * Bm[p] * P; BQ += w2 * Bm[p] * Q;
    }
    out[0] = -EP + BQ;
    out[1] = EQ + BP;
}

template <int N, class T>
__global__ __launch_bounds__(256) void k_psi4(const DiagArgs a, double* out)
{
    const WorkItem w = a.work[blockIdx.x];
    const BlockDev B = a.blocks[w.block];
    const int t = threadIdx.x;
    const int li = t % w.ni, lj = (t / w.ni) % w.nj, lk = t / (w.ni * w.nj);
    if (lk >= w.nk) return;
    const int i = w.i0 + li, j = w.j0 + lj, k = w.k0 + lk;
    const int g = a.g, E = B.E, n = B.n;
    const int64_t cc = ((int64_t)(k + g) * E + (j + g)) * E + (i + g);
    const double x[3] = {B.x0[0] + i * B.h - a.centres[0][0], B.x0[1] + j * B.h - a.centres[0][1],
                         B.x0[2] + k * B.h - a.centres[0][2]};
    double ps[2];
    zone_psi4<N, T>((const T*)a.src + B.off + cc, B.slab, E, E * E, 1.0 / B.h, x, ps);
    const int64_t n3 = (int64_t)n * n * n;
    const int64_t ci = (B.ioff / NF) * 2 + ((int64_t)k * n + j) * n + i;
    out[ci] = ps[0];
    out[ci + n3] = ps[1];
}

// ------------------------------------------------------------ points

struct PointArgs {
    const BlockDev* blocks;
    const int32_t* map;
    LookupDev L;
    double lo[3], dx0;
    int32_t nroot[3], g;
};

// finest block whose active cells contain p (-1 if none)
__device__ int locate(const PointArgs& a, const double p[3])
{
    for (int l = a.L.nlev - 1; l >= 0; --l) {
        const double h = a.dx0 / (double)(1 << l);
        int64_t c[3];
        bool in = true;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            c[d] = (int64_t)floor((p[d] - a.lo[d]) / h);
            in = in && c[d] >= 0 && c[d] < ((int64_t)a.nroot[d] << l);
        }
        if (!in) continue;
        const int u = a.L.unit;
        const int b = a.map[a.L.base[l] + ((c[2] / u) * a.L.dim[l][1] + c[1] / u) * a.L.dim[l][0] + c[0] / u];
        if (b >= 0) return b;
    }
    return -1;
}

// cubic Lagrange window (local index of the first of 4 nodes) and weights
__device__ __forceinline__ int cubic(double xt, int n, double w[4])
{
    int i0 = (int)floor(xt) - 1;
    i0 = i0 < 0 ? 0 : (i0 > n - 4 ? n - 4 : i0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        double s = 1.0;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (r != q) s *= (xt - (i0 + r)) / (double)(q - r);
        w[q] = s;
    }
    return i0;
}

// value of component(s) at point p from a block's cells: `get(b, i, j, k, c)`
template <class Get>
__device__ bool interp_at(const PointArgs& a, const double p[3], int ncomp, double* out, Get get)
{
    const int b = locate(a, p);
    if (b < 0) return false;
    const BlockDev B = a.blocks[b];
    double w[3][4];
    int i0[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) i0[d] = cubic((p[d] - a.lo[d]) / B.h - 0.5 - B.ilo[d], B.n, w[d]);
    for (int c = 0; c < ncomp; ++c) {
        double acc = 0.0;
        for (int kz = 0; kz < 4; ++kz) {
            double az = 0.0;
            for (int jy = 0; jy < 4; ++jy) {
                double ay = 0.0;
#pragma unroll
                for (int ix = 0; ix < 4; ++ix) ay += w[0][ix] * get(B, i0[0] + ix, i0[1] + jy, i0[2] + kz, c);
                az += w[1][jy] * ay;
            }
            acc += w[2][kz] * az;
        }
        out[c] = acc;
    }
    return true;
}

// interior-layout source (double, ncomp components per block)
__global__ __launch_bounds__(256) void k_interp(const PointArgs a, const double* __restrict__ src, int ncomp,
                                                const double* __restrict__ pts, int npts, double* out)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= npts) return;
    const double p[3] = {pts[3 * q], pts[3 * q + 1], pts[3 * q + 2]};
    double v[8];
    auto get = [&](const BlockDev& B, int i, int j, int k, int c) {
        const int64_t n = B.n;
        return src[(B.ioff / NF) * ncomp + (((int64_t)c * n + k) * n + j) * n + i];
    };
    bool ok = true;
    for (int c0 = 0; c0 < ncomp && ok; c0 += 8) {
        const int nc = ncomp - c0 < 8 ? ncomp - c0 : 8;
        auto g2 = [&](const BlockDev& B, int i, int j, int k, int c) { return get(B, i, j, k, c0 + c); };
        ok = interp_at(a, p, nc, v, g2);
        for (int c = 0; c < nc; ++c) out[(int64_t)q * ncomp + c0 + c] = ok ? v[c] : NAN;
    }
}

// state-register source (ghosted layout, element type T): fields first..first+nf-1
template <class T>
__device__ bool interp_state(const PointArgs& a, const T* __restrict__ reg, int first, int nf,
                             const double p[3], double* v)
{
    const int g = a.g;
    auto get = [&](const BlockDev& B, int i, int j, int k, int c) {
        return (double)reg[B.off + (int64_t)(first + c) * B.slab + (((int64_t)(k + g) * B.E + (j + g)) * B.E + (i + g))];
    };
    return interp_at(a, p, nf, v, get);
}

template <class T>
__global__ __launch_bounds__(256) void k_interp_state(const PointArgs a, const void* reg, int first, int nf,
                                                      const double* __restrict__ pts, int npts, double* out)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= npts) return;
    const double p[3] = {pts[3 * q], pts[3 * q + 1], pts[3 * q + 2]};
    double v[Z4C_NFIELDS];
    const bool ok = interp_state<T>(a, (const T*)reg, first, nf, p, v);
    for (int c = 0; c < nf; ++c) out[(int64_t)q * nf + c] = ok ? v[c] : NAN;
}

// puncture tracker, stage s (1..4) of classic RK4: k_s = -beta(stage input,
// x + c_s dt k_(s-1)); state per puncture: x, k_prev, acc
template <class T>
__global__ void k_track(const PointArgs a, const void* reg, int stage, double dt, double* st, int np)
{
    const int q = threadIdx.x;
    if (q >= np) return;
    double* x = st + 9 * q;
    double* kp = x + 3;
    double* acc = x + 6;
    const double c = stage == 1 ? 0.0 : (stage == 4 ? 1.0 : 0.5);
    const double b = (stage == 1 || stage == 4) ? 1.0 / 6.0 : 1.0 / 3.0;
    double p[3];
    for (int d = 0; d < 3; ++d) p[d] = x[d] + c * dt * kp[d];
    double beta[3];
    if (!interp_state<T>(a, (const T*)reg, F_BETAX, 3, p, beta))
        for (int d = 0; d < 3; ++d) beta[d] = NAN;
    for (int d = 0; d < 3; ++d) {
        const double k = -beta[d];
        acc[d] = (stage == 1 ? 0.0 : acc[d]) + b * k;
        kp[d] = k;
    }
    if (stage == 4)
        for (int d = 0; d < 3; ++d) x[d] = x[d] + dt * acc[d];
}

// ----------------------------------------------------- harmonics

// sY_lm(theta, phi) = (-1)^s sqrt((2l+1)/(4 pi)) d^l_{m,-s}(theta) e^{i m phi};
// the explicit sum below is d^l_{-s,m} = (-1)^(m+s) d^l_{m,-s}
__device__ void swsh_dev(int s, int l, int m, double th, double ph, double& re, double& im)
{
    double f[2 * 12 + 2];
    f[0] = 1.0;
    for (int q = 1; q < 2 * 12 + 2; ++q) f[q] = f[q - 1] * q;
    const int mp = -s;
    const double ch = cos(0.5 * th), sh = sin(0.5 * th);
    const double pre = sqrt(f[l + m] * f[l - m] * f[l + mp] * f[l - mp]);
    double d = 0.0;
    const int kmin = (m - mp > 0) ? m - mp : 0, kmax = (l + m < l - mp) ? l + m : l - mp;
    for (int k = kmin; k <= kmax; ++k) {
        const double den = f[l + m - k] * f[k] * f[l - k - mp] * f[k - m + mp];
        const double sg = ((k - m + mp) & 1) ? -1.0 : 1.0;
        d += sg * pow(ch, 2 * l + m - mp - 2 * k) * pow(sh, 2 * k - m + mp) / den;
    }
    d *= pre;
    const double amp = (((m + s) & 1) ? -1.0 : 1.0) * sqrt((2 * l + 1) / (4.0 * M_PI)) * d;
    re = amp * cos(m * ph);
    im = amp * sin(m * ph);
}

// one workgroup per mode (l, m), l = 2..lmax: sum_p w_p psi_p conj(Y)
__global__ __launch_bounds__(256) void k_swsh(const double* __restrict__ val, const double* __restrict__ pts,
                                              const double* __restrict__ wts, int npts, double cx, double cy,
                                              double cz, double* modes)
{
    __shared__ double sr[256], si[256];
    const int mode = blockIdx.x;
    int l = 2, m;
    {
        int r = mode;
        while (r >= 2 * l + 1) { r -= 2 * l + 1; ++l; }
        m = r - l;
    }
    double ar = 0.0, ai = 0.0;
    for (int q = threadIdx.x; q < npts; q += 256) {
        const double dx = pts[3 * q] - cx, dy = pts[3 * q + 1] - cy, dz = pts[3 * q + 2] - cz;
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        double c = dz / r;
        c = c > 1.0 ? 1.0 : (c < -1.0 ? -1.0 : c);
        const double th = acos(c), ph = atan2(dy, dx);
        double yr, yi;
        swsh_dev(-2, l, m, th, ph, yr, yi);
        const double vr = val[2 * q], vi = val[2 * q + 1], w = wts[q];
        // psi * conj(Y)
        ar += w * (vr * yr + vi * yi);
        ai += w * (vi * yr - vr * yi);
    }
    const int t = threadIdx.x;
    sr[t] = ar;
    si[t] = ai;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) { sr[t] += sr[t + s]; si[t] += si[t + s]; }
        __syncthreads();
    }
    if (t == 0) { modes[2 * mode] = sr[0]; modes[2 * mode + 1] = si[0]; }
}

}  // namespace z4c

using namespace z4c_host;

namespace {

PointArgs point_args(const z4c_pack* pk)
{
    PointArgs a;
    std::memset(&a, 0, sizeof(a));
    a.blocks = reinterpret_cast<const BlockDev*>(pk->ws + pk->ws_blocks);
    a.map = reinterpret_cast<const int32_t*>(pk->ws + pk->ws_map);
    a.L = pk->L;
    for (int d = 0; d < 3; ++d) { a.lo[d] = pk->p.lo[d]; a.nroot[d] = pk->p.nroot[d]; }
    a.dx0 = pk->p.dx0;
    a.g = pk->p.nghost;
    return a;
}

}  // namespace

namespace z4c_host {

// tracker stage launched by z4c_rk4_stage before the stage kernel
hipError_t track_stage(z4c_pack* pk, int stage, int reg, double dt, hipStream_t s)
{
    if (pk->ntrack <= 0) return hipSuccess;
    const PointArgs a = point_args(pk);
    double* st = reinterpret_cast<double*>(pk->ws + pk->ws_track);
    if (pk->p.precision == Z4C_FP64)
        hipLaunchKernelGGL(k_track<double>, dim3(1), dim3(64), 0, s, a, pk->reg[reg], stage, dt, st, pk->ntrack);
    else
        hipLaunchKernelGGL(k_track<float>, dim3(1), dim3(64), 0, s, a, pk->reg[reg], stage, dt, st, pk->ntrack);
    return hipGetLastError();
}

}  // namespace z4c_host

extern "C" {

int z4c_psi4(z4c_pack* pk, int32_t reg, const double origin[3], void* out, void* stream)
{
    if (!pk || !origin || !out) return Z4C_EINVAL;
    if (reg < Z4C_REG_U || reg > Z4C_REG_S2) return fail(pk, Z4C_EINVAL, "bad register %d", reg);
    if (!pk->bound) return fail(pk, Z4C_ESTATE, "pack not bound");
    int rc = z4c_fill_ghosts(pk, reg, stream);
    if (rc) return rc;
    DiagArgs a;
    std::memset(&a, 0, sizeof(a));
    a.src = pk->reg[reg];
    a.blocks = reinterpret_cast<const BlockDev*>(pk->ws + pk->ws_blocks);
    a.work = reinterpret_cast<const WorkItem*>(pk->ws + pk->ws_work);
    a.g = pk->p.nghost;
    for (int d = 0; d < 3; ++d) a.centres[0][d] = origin[d];
    hipStream_t s = as_stream(stream);
    const dim3 grid((unsigned)pk->work.size());
    const int N = pk->p.fd_order / 2;
    double* o = static_cast<double*>(out);
#define Z4C_PSI4(NN)                                                                                    \
    if (pk->p.precision == Z4C_FP64) hipLaunchKernelGGL((k_psi4<NN, double>), grid, dim3(256), 0, s, a, o); \
    else hipLaunchKernelGGL((k_psi4<NN, float>), grid, dim3(256), 0, s, a, o);
    if (N == 2) { Z4C_PSI4(2) } else if (N == 3) { Z4C_PSI4(3) } else { Z4C_PSI4(4) }
#undef Z4C_PSI4
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(pk, Z4C_EDEVICE, "psi4 launch: %s", hipGetErrorString(e));
    return Z4C_OK;
}

int z4c_interp(z4c_pack* pk, const void* src, int32_t ncomp, const double* pts, int32_t npts, double* out,
               void* stream)
{
    if (!pk || ncomp < 1 || npts < 0) return Z4C_EINVAL;
    if (!pk->bound) return fail(pk, Z4C_ESTATE, "pack not bound");
    for (const z4c_block& B : pk->blk)
        if (B.n < 4) return fail(pk, Z4C_EUNSUPPORTED, "interpolation needs 4 cells per block");
    if (npts == 0) return Z4C_OK;   // nothing to do; the pointers may be NULL
    if (!src || !pts || !out) return fail(pk, Z4C_EINVAL, "NULL pointer");
    const PointArgs a = point_args(pk);
    hipLaunchKernelGGL(k_interp, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, as_stream(stream), a,
                       static_cast<const double*>(src), (int)ncomp, pts, (int)npts, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(pk, Z4C_EDEVICE, "interp launch: %s", hipGetErrorString(e));
    return Z4C_OK;
}

int z4c_interp_state(z4c_pack* pk, int32_t reg, int32_t first, int32_t nfield, const double* pts, int32_t npts,
                     double* out, void* stream)
{
    if (!pk || npts < 0) return Z4C_EINVAL;
    if (reg < Z4C_REG_U || reg > Z4C_REG_S2) return fail(pk, Z4C_EINVAL, "bad register %d", reg);
    if (first < 0 || nfield < 1 || first + nfield > Z4C_NFIELDS) return fail(pk, Z4C_EINVAL, "bad fields");
    if (!pk->bound) return fail(pk, Z4C_ESTATE, "pack not bound");
    if (npts == 0) return Z4C_OK;   // nothing to do; the pointers may be NULL
    if (!pts || !out) return fail(pk, Z4C_EINVAL, "NULL pointer");
    const PointArgs a = point_args(pk);
    const dim3 grid((unsigned)((npts + 255) / 256));
    if (pk->p.precision == Z4C_FP64)
        hipLaunchKernelGGL(k_interp_state<double>, grid, dim3(256), 0, as_stream(stream), a, pk->reg[reg],
                           (int)first, (int)nfield, pts, (int)npts, out);
    else
        hipLaunchKernelGGL(k_interp_state<float>, grid, dim3(256), 0, as_stream(stream), a, pk->reg[reg],
                           (int)first, (int)nfield, pts, (int)npts, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(pk, Z4C_EDEVICE, "interp launch: %s", hipGetErrorString(e));
    return Z4C_OK;
}

int z4c_swsh_project(const double* values, const double* pts, const double* weights, int32_t npts,
                     const double centre[3], int32_t lmax, double* modes, void* stream)
{
    if (!values || !pts || !weights || !centre || !modes || npts < 1 || lmax < 2 || lmax > 12)
        return Z4C_EINVAL;
    const int nmodes = (lmax + 1) * (lmax + 1) - 4;
    hipLaunchKernelGGL(k_swsh, dim3((unsigned)nmodes), dim3(256), 0, as_stream(stream), values, pts, weights,
                       (int)npts, centre[0], centre[1], centre[2], modes);
    return hipGetLastError() == hipSuccess ? Z4C_OK : Z4C_EDEVICE;
}

int z4c_tracker_set(z4c_pack* pk, int32_t n, const double* pos, void* stream)
{
    if (!pk || n < 0 || n > Z4C_MAXTRACK || (n > 0 && !pos)) return Z4C_EINVAL;
    if (!pk->bound) return fail(pk, Z4C_ESTATE, "pack not bound");
    pk->track_host.assign(9 * Z4C_MAXTRACK, 0.0);
    for (int q = 0; q < n; ++q)
        for (int d = 0; d < 3; ++d) pk->track_host[9 * q + d] = pos[3 * q + d];
    hipError_t e = hipMemcpyAsync(pk->ws + pk->ws_track, pk->track_host.data(), sizeof(double) * 9 * Z4C_MAXTRACK,
                                  hipMemcpyHostToDevice, as_stream(stream));
    if (e != hipSuccess) return fail(pk, Z4C_EDEVICE, "tracker upload: %s", hipGetErrorString(e));
    pk->ntrack = n;
    // a captured step graph does not hold the tracker launches of the new count
    drop_graphs(pk);
    return Z4C_OK;
}

int z4c_tracker_get(z4c_pack* pk, double* pos, void* stream)
{
    if (!pk || !pos) return Z4C_EINVAL;
    if (!pk->bound) return fail(pk, Z4C_ESTATE, "pack not bound");
    if (pk->ntrack == 0) return Z4C_OK;
    std::vector<double> h(9 * Z4C_MAXTRACK);
    hipStream_t s = as_stream(stream);
    hipError_t e = hipMemcpyAsync(h.data(), pk->ws + pk->ws_track, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(pk, Z4C_EDEVICE, "tracker read: %s", hipGetErrorString(e));
    for (int q = 0; q < pk->ntrack; ++q)
        for (int d = 0; d < 3; ++d) pos[3 * q + d] = h[9 * q + d];
    return Z4C_OK;
}

}  // extern "C"
