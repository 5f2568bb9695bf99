// Per-zone Z4c right-hand side for the HIP kernels.
//
// Equations: the vacuum Z4c system with 1+log lapse and Gamma-driver shift
// that the paper adopts (Sec. 2), with its Sec. 4.3 parameters:
//   d_t chi   = (2/3) chi (alpha K - d_k beta^k)
//   d_t g~_ij = -2 alpha A~_ij + g~_ik d_j beta^k + g~_jk d_i beta^k
//               - (2/3) g~_ij d_k beta^k
//   d_t Khat  = -D^i D_i alpha + alpha (A~_ij A~^ij + K^2/3)
//               + kappa1 (1 - kappa2) alpha Theta
//   d_t A~_ij = chi [-D_i D_j alpha + alpha R_ij]^TF
//               + alpha (K A~_ij - 2 A~_ik g~^kl A~_lj)
//               + A~_ik d_j beta^k + A~_jk d_i beta^k - (2/3) A~_ij d_k beta^k
//   d_t G~^i  = -G~d^j d_j beta^i + (2/3) G~d^i d_j beta^j + g~^jk d_j d_k beta^i
//               + (1/3) g~^ij d_j d_k beta^k - 2 A~^ij d_j alpha
//               + 2 alpha (G~^i_jk A~^jk - (3/2) A~^ij d_j chi / chi
//                          - (1/3) g~^ij d_j (2 Khat + Theta))
//               - 2 alpha kappa1 (G~^i - G~d^i)
//   d_t Theta = (alpha/2)(R - A~_ij A~^ij + (2/3) K^2) - alpha kappa1 (2+kappa2) Theta
//   d_t alpha = -2 alpha Khat,   d_t beta^i = mu_S G~^i - eta beta^i
// plus beta^k d_k (lopsided) advection and Kreiss-Oliger dissipation,
// with K = Khat + 2 Theta, R_ij = R~_ij + R^chi_ij, R = chi g~^ij R_ij, the
// metric-derived G~d^i = g~^jk G~^i_jk, and chi floored where it divides.
// The evolved G~^i enters only where differentiated, in the damping term
// and in the shift equation.
#pragma once
#include "stencils.hpp"
#include "z4c_dev.hpp"

namespace z4c {

// symmetric index: xx xy xz yy yz zz
__host__ __device__ constexpr int S(int i, int j)
{
    return (i == j) ? (i == 0 ? 0 : (i == 1 ? 3 : 5)) : (i + j == 1 ? 1 : (i + j == 2 ? 2 : 4));
}
// weight of a symmetric pair in a full double contraction
__host__ __device__ constexpr double SW(int p) { return (p == 0 || p == 3 || p == 5) ? 1.0 : 2.0; }
__host__ __device__ constexpr int SA(int p) { return p == 0 ? 0 : p == 1 ? 0 : p == 2 ? 0 : p == 3 ? 1 : p == 4 ? 1 : 2; }
__host__ __device__ constexpr int SB(int p) { return p == 0 ? 0 : p == 1 ? 1 : p == 2 ? 2 : p == 3 ? 1 : p == 4 ? 2 : 2; }

// Derivative operators on a field pointer `p` at the zone (no 1/h factors).
template <int N, class C, class T>
__device__ __forceinline__ C fd1(const T* __restrict__ p, int s)
{
    C acc = 0;
#pragma unroll
    for (int k = 1; k <= N; ++k) acc += (C)Stencil<N>::D1[k] * ((C)p[k * s] - (C)p[-k * s]);
    return acc;
}

template <int N, class C, class T>
__device__ __forceinline__ C fd2(const T* __restrict__ p, int s)
{
    const C f0 = (C)p[0];
    C acc = 0;
#pragma unroll
    for (int k = 1; k <= N; ++k) acc += (C)Stencil<N>::D2[k] * (((C)p[k * s] - f0) + ((C)p[-k * s] - f0));
    return acc;
}

template <int N, class C, class T>
__device__ __forceinline__ C fdmix(const T* __restrict__ p, int sa, int sb)
{
    C acc = 0;
#pragma unroll
    for (int q = 1; q <= N; ++q) {
        C in = 0;
#pragma unroll
        for (int r = 1; r <= N; ++r) {
            C d = ((C)p[q * sa + r * sb] - (C)p[q * sa - r * sb]) -
                  ((C)p[-q * sa + r * sb] - (C)p[-q * sa - r * sb]);
            in += (C)Stencil<N>::D1[r] * d;
        }
        acc += (C)Stencil<N>::D1[q] * in;
    }
    return acc;
}

// division by chi is done in double whatever C is
template <class C> __device__ __forceinline__ C inv_chi(C chi, double floor_)
{
    double c = (double)chi;
    if (c < floor_) c = floor_;
    return (C)(1.0 / c);
}

// Christoffel symbols from d_a g~_p: Gl[k][ij] = G~_kij, Gu[k][ij] = G~^k_ij,
// and the contracted G~d^i = g~^jk G~^i_jk
template <class C>
__device__ __forceinline__ void christoffels(const C (&gu)[6], const C (&dg)[3][6], C (&Gl)[3][6],
                                             C (&Gu)[3][6], C (&Gd)[3])
{
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int p = 0; p < 6; ++p) {
            const int i = SA(p), j = SB(p);
            Gl[k][p] = (C)0.5 * (dg[i][S(j, k)] + dg[j][S(i, k)] - dg[k][p]);
        }
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int p = 0; p < 6; ++p)
            Gu[k][p] = gu[S(k, 0)] * Gl[0][p] + gu[S(k, 1)] * Gl[1][p] + gu[S(k, 2)] * Gl[2][p];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        C s = 0;
#pragma unroll
        for (int p = 0; p < 6; ++p) s += (C)SW(p) * gu[p] * Gu[i][p];
        Gd[i] = s;
    }
}

// Full Ricci tensor R_ij = R~_ij + R^chi_ij and scalar R = chi g~^ij R_ij.
// Rt holds on entry -1/2 g~^lm d_l d_m g~_ij + 1/2 (g~_ki d_j G~^k + g~_kj d_i G~^k).
template <class C>
__device__ __forceinline__ void ricci(const C (&gdn)[6], const C (&gu)[6], const C (&Gl)[3][6],
                                      const C (&Gu)[3][6], const C (&Gd)[3], C chi, C ic,
                                      const C (&dchi)[3], const C (&ddchi)[6], C (&Rt)[6],
                                      C (&Rij)[6], C& Rs)
{
    // the quadratic Christoffel terms
    //   g~^lm (G~^k_li G~_jkm + G~^k_lj G~_ikm + G~^k_im G~_klj)
    // contract as sum_kl (G~^k_li H_jk^l + G~^k_lj H_ik^l + G~^k_il H_kj^l)
    // with H_jk^l = g~^lm G~_jkm (27 values instead of a 3 x 3 x 3 sum per
    // (l, m) pair)
    C H[3][3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int l = 0; l < 3; ++l)
                H[j][k][l] = gu[S(l, 0)] * Gl[j][S(k, 0)] + gu[S(l, 1)] * Gl[j][S(k, 1)] + gu[S(l, 2)] * Gl[j][S(k, 2)];
#pragma unroll
    for (int p = 0; p < 6; ++p) {
        const int i = SA(p), j = SB(p);
        C s = 0;
#pragma unroll
        for (int k = 0; k < 3; ++k) s += Gd[k] * (C)0.5 * (Gl[i][S(j, k)] + Gl[j][S(i, k)]);
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int l = 0; l < 3; ++l)
                s += Gu[k][S(l, i)] * H[j][k][l] + Gu[k][S(l, j)] * H[i][k][l] + Gu[k][S(i, l)] * H[k][j][l];
        Rt[p] += s;
    }
    C Dchi[6], trD = 0, dc2 = 0;
#pragma unroll
    for (int p = 0; p < 6; ++p)
        Dchi[p] = ddchi[p] - (Gu[0][p] * dchi[0] + Gu[1][p] * dchi[1] + Gu[2][p] * dchi[2]);
#pragma unroll
    for (int p = 0; p < 6; ++p) {
        trD += (C)SW(p) * gu[p] * Dchi[p];
        dc2 += (C)SW(p) * gu[p] * dchi[SA(p)] * dchi[SB(p)];
    }
    Rs = 0;
#pragma unroll
    for (int p = 0; p < 6; ++p) {
        const int i = SA(p), j = SB(p);
        Rij[p] = Rt[p] + (C)0.5 * ic * Dchi[p] + (C)0.5 * ic * gdn[p] * trD -
                 (C)0.25 * ic * ic * dchi[i] * dchi[j] - (C)0.75 * ic * ic * gdn[p] * dc2;
        Rs += (C)SW(p) * gu[p] * Rij[p];
    }
    Rs *= chi;
}

// The algebraic part of the 22 right-hand sides (everything except the
// advection and dissipation terms) from centre values and derivatives:
//   dg[a][p] = d_a g~_p, dbe[a][i] = d_a beta^i, Lb[i] = g~^jk d_j d_k beta^i,
//   Bj[j] = d_j d_k beta^k, eK[j] = d_j (2 Khat + Theta), Rt as for ricci().
template <class C>
__device__ __forceinline__ void z4c_algebra(const ParamsDev& P, C chi, const C (&gdn)[6],
                                            const C (&gu)[6], C Kh, const C (&A)[6],
                                            const C (&Gam)[3], C Th, C al, const C (&be)[3],
                                            const C (&dg)[3][6], const C (&dchi)[3],
                                            const C (&ddchi)[6], const C (&dal)[3],
                                            const C (&ddal)[6], const C (&dbe)[3][3],
                                            const C (&Lb)[3], const C (&Bj)[3], const C (&eK)[3],
                                            C (&Rt)[6], C (&rhs)[NF])
{
    C Gl[3][6], Gu[3][6], Gd[3];
    christoffels<C>(gu, dg, Gl, Gu, Gd);
    const C ic = inv_chi<C>(chi, P.chi_floor);
    const C K = Kh + (C)2 * Th;
    C Rij[6], Rs;
    ricci<C>(gdn, gu, Gl, Gu, Gd, chi, ic, dchi, ddchi, Rt, Rij, Rs);

    // A~_ik g~^kl, A~^ij, A~_ij A~^ij
    C Am[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int l = 0; l < 3; ++l)
            Am[i][l] = A[S(i, 0)] * gu[S(0, l)] + A[S(i, 1)] * gu[S(1, l)] + A[S(i, 2)] * gu[S(2, l)];
    C Au[6];
#pragma unroll
    for (int p = 0; p < 6; ++p) {
        const int i = SA(p), j = SB(p);
        Au[p] = gu[S(i, 0)] * Am[0][j] + gu[S(i, 1)] * Am[1][j] + gu[S(i, 2)] * Am[2][j];
    }
    C AA = 0;
#pragma unroll
    for (int p = 0; p < 6; ++p) AA += (C)SW(p) * A[p] * Au[p];

    // D_i D_j alpha and its trace D^i D_i alpha
    C DDa[6], trDDa = 0, cda = 0;
#pragma unroll
    for (int p = 0; p < 6; ++p)
        cda += (C)SW(p) * gu[p] * (C)0.5 * (dchi[SA(p)] * dal[SB(p)] + dchi[SB(p)] * dal[SA(p)]);
#pragma unroll
    for (int p = 0; p < 6; ++p) {
        const int i = SA(p), j = SB(p);
        DDa[p] = ddal[p] - (Gu[0][p] * dal[0] + Gu[1][p] * dal[1] + Gu[2][p] * dal[2]) +
                 (C)0.5 * ic * (dchi[i] * dal[j] + dchi[j] * dal[i] - gdn[p] * cda);
        trDDa += (C)SW(p) * gu[p] * DDa[p];
    }
    trDDa *= chi;

    const C divb = dbe[0][0] + dbe[1][1] + dbe[2][2];
#pragma unroll
    for (int f = 0; f < NF; ++f) rhs[f] = 0;
    if (P.terms & 1u) {
        rhs[F_CHI] = (C)(2.0 / 3.0) * chi * (al * K - divb);
#pragma unroll
        for (int p = 0; p < 6; ++p) {
            const int i = SA(p), j = SB(p);
            C s = (C)-2 * al * A[p] - (C)(2.0 / 3.0) * gdn[p] * divb;
#pragma unroll
            for (int k = 0; k < 3; ++k) s += gdn[S(i, k)] * dbe[j][k] + gdn[S(j, k)] * dbe[i][k];
            rhs[F_GXX + p] = s;
        }
        rhs[F_KH] = -trDDa + al * (AA + K * K * (C)(1.0 / 3.0)) + (C)(P.kappa1 * (1.0 - P.kappa2)) * al * Th;
        C X[6], trX = 0;
#pragma unroll
        for (int p = 0; p < 6; ++p) {
            X[p] = -DDa[p] + al * Rij[p];
            trX += (C)SW(p) * gu[p] * X[p];
        }
#pragma unroll
        for (int p = 0; p < 6; ++p) {
            const int i = SA(p), j = SB(p);
            C s = chi * (X[p] - gdn[p] * trX * (C)(1.0 / 3.0));
            const C AgA = Am[i][0] * A[S(0, j)] + Am[i][1] * A[S(1, j)] + Am[i][2] * A[S(2, j)];
            s += al * (K * A[p] - (C)2 * AgA);
#pragma unroll
            for (int k = 0; k < 3; ++k) s += A[S(i, k)] * dbe[j][k] + A[S(j, k)] * dbe[i][k];
            s -= (C)(2.0 / 3.0) * A[p] * divb;
            rhs[F_AXX + p] = s;
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            C s = (C)(2.0 / 3.0) * Gd[i] * divb - (Gd[0] * dbe[0][i] + Gd[1] * dbe[1][i] + Gd[2] * dbe[2][i]);
            s += Lb[i] + (gu[S(i, 0)] * Bj[0] + gu[S(i, 1)] * Bj[1] + gu[S(i, 2)] * Bj[2]) * (C)(1.0 / 3.0);
            s -= (C)2 * (Au[S(i, 0)] * dal[0] + Au[S(i, 1)] * dal[1] + Au[S(i, 2)] * dal[2]);
            C t = 0;
#pragma unroll
            for (int p = 0; p < 6; ++p) t += (C)SW(p) * Gu[i][p] * Au[p];
            t -= (C)1.5 * ic * (Au[S(i, 0)] * dchi[0] + Au[S(i, 1)] * dchi[1] + Au[S(i, 2)] * dchi[2]);
            t -= (gu[S(i, 0)] * eK[0] + gu[S(i, 1)] * eK[1] + gu[S(i, 2)] * eK[2]) * (C)(1.0 / 3.0);
            s += (C)2 * al * t;
            s -= (C)2 * al * (C)P.kappa1 * (Gam[i] - Gd[i]);
            rhs[F_GAMX + i] = s;
        }
        rhs[F_TH] = (C)0.5 * al * (Rs - AA + (C)(2.0 / 3.0) * K * K) -
                    al * (C)(P.kappa1 * (2.0 + P.kappa2)) * Th;
    }
    if (P.terms & 2u) {
        rhs[F_ALPHA] = (C)-2 * al * Kh;
#pragma unroll
        for (int i = 0; i < 3; ++i) rhs[F_BETAX + i] = (C)P.mu_S * Gam[i] - (C)P.eta * be[i];
    }
}

// Constraint monitors of one zone (direct stencil reads, double):
// out = H, M^x, M^y, M^z, Theta, G^x, G^y, G^z with
//   H = R - A~_ij A~^ij + (2/3) K^2,
//   M^i = d_j A~^ij + G~^i_jk A~^jk - (2/3) g~^ij d_j K - (3/2) A~^ij d_j chi / chi,
//   G^i = G~^i - G~d^i.
template <int N, class T>
__device__ __forceinline__ void zone_constraints(const T* __restrict__ z, int64_t slab, int sy,
                                                 int sz, double ih, const ParamsDev& P,
                                                 double (&out)[8])
{
    using C = double;
    const int st[3] = {1, sy, sz};
    auto cen = [&](int f) { return (C)z[f * slab]; };
    const C chi = cen(F_CHI), Kh = cen(F_KH), Th = cen(F_TH);
    C gdn[6], A[6], Gam[3];
#pragma unroll
    for (int p = 0; p < 6; ++p) { gdn[p] = cen(F_GXX + p); A[p] = cen(F_AXX + p); }
#pragma unroll
    for (int i = 0; i < 3; ++i) Gam[i] = cen(F_GAMX + i);
    C gu[6];
    {
        const C c0 = gdn[3] * gdn[5] - gdn[4] * gdn[4];
        const C c1 = gdn[2] * gdn[4] - gdn[1] * gdn[5];
        const C c2 = gdn[1] * gdn[4] - gdn[2] * gdn[3];
        const C id = 1.0 / (gdn[0] * c0 + gdn[1] * c1 + gdn[2] * c2);
        gu[0] = c0 * id; gu[1] = c1 * id; gu[2] = c2 * id;
        gu[3] = (gdn[0] * gdn[5] - gdn[2] * gdn[2]) * id;
        gu[4] = (gdn[1] * gdn[2] - gdn[0] * gdn[4]) * id;
        gu[5] = (gdn[0] * gdn[3] - gdn[1] * gdn[1]) * id;
    }
    C dg[3][6], dchi[3], ddchi[6], dK[3], dA[3][6], Rt[6];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int p = 0; p < 6; ++p) {
            dg[a][p] = ih * fd1<N, C>(z + (F_GXX + p) * slab, st[a]);
            dA[a][p] = ih * fd1<N, C>(z + (F_AXX + p) * slab, st[a]);
        }
        dchi[a] = ih * fd1<N, C>(z + F_CHI * slab, st[a]);
        dK[a] = ih * (fd1<N, C>(z + F_KH * slab, st[a]) + 2.0 * fd1<N, C>(z + F_TH * slab, st[a]));
    }
    const C ih2 = ih * ih;
#pragma unroll
    for (int p = 0; p < 6; ++p) Rt[p] = 0;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const int a = SA(q), b = SB(q);
        const C wq = -0.5 * SW(q) * gu[q] * ih2;
#pragma unroll
        for (int p = 0; p < 6; ++p) {
            const T* pf = z + (F_GXX + p) * slab;
            Rt[p] += wq * ((a == b) ? fd2<N, C>(pf, st[a]) : fdmix<N, C>(pf, st[a], st[b]));
        }
        const T* pf = z + F_CHI * slab;
        ddchi[q] = ih2 * ((a == b) ? fd2<N, C>(pf, st[a]) : fdmix<N, C>(pf, st[a], st[b]));
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const C dG = ih * fd1<N, C>(z + (F_GAMX + k) * slab, st[a]);
#pragma unroll
            for (int p = 0; p < 6; ++p) {
                const int i = SA(p), j = SB(p);
                if (a == j) Rt[p] += 0.5 * gdn[S(k, i)] * dG;
                if (a == i) Rt[p] += 0.5 * gdn[S(k, j)] * dG;
            }
        }
    C Gl[3][6], Gu[3][6], Gd[3];
    christoffels<C>(gu, dg, Gl, Gu, Gd);
    const C ic = inv_chi<C>(chi, P.chi_floor);
    C Rij[6], Rs;
    ricci<C>(gdn, gu, Gl, Gu, Gd, chi, ic, dchi, ddchi, Rt, Rij, Rs);
    C Au[6], AA = 0;
#pragma unroll
    for (int p = 0; p < 6; ++p) {
        const int i = SA(p), j = SB(p);
        C s = 0;
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int l = 0; l < 3; ++l) s += gu[S(i, k)] * gu[S(j, l)] * A[S(k, l)];
        Au[p] = s;
    }
#pragma unroll
    for (int p = 0; p < 6; ++p) AA += SW(p) * A[p] * Au[p];
    const C K = Kh + 2.0 * Th;
    out[0] = Rs - AA + (2.0 / 3.0) * K * K;
    C dgu[3][6];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int p = 0; p < 6; ++p) {
            const int i = SA(p), j = SB(p);
            C s = 0;
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int d = 0; d < 3; ++d) s -= gu[S(i, c)] * gu[S(j, d)] * dg[a][S(c, d)];
            dgu[a][p] = s;
        }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        C s = 0;
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int l = 0; l < 3; ++l)
                    s += dgu[j][S(i, k)] * gu[S(j, l)] * A[S(k, l)] +
                         gu[S(i, k)] * dgu[j][S(j, l)] * A[S(k, l)] +
                         gu[S(i, k)] * gu[S(j, l)] * dA[j][S(k, l)];
#pragma unroll
        for (int p = 0; p < 6; ++p) s += SW(p) * Gu[i][p] * Au[p];
#pragma unroll
        for (int j = 0; j < 3; ++j) s -= (2.0 / 3.0) * gu[S(i, j)] * dK[j] + 1.5 * Au[S(i, j)] * dchi[j] * ic;
        out[1 + i] = s;
        out[5 + i] = Gam[i] - Gd[i];
    }
    out[4] = Th;
}

// Algebraic constraints and floors on one zone's state, in double.
__device__ __forceinline__ void enforce_zone(double* u, const ParamsDev& P)
{
    double g0 = u[F_GXX], g1 = u[F_GXY], g2 = u[F_GXZ], g3 = u[F_GYY], g4 = u[F_GYZ], g5 = u[F_GZZ];
    const double det = g0 * (g3 * g5 - g4 * g4) - g1 * (g1 * g5 - g4 * g2) + g2 * (g1 * g4 - g3 * g2);
    const double s = 1.0 / cbrt(det);
    g0 *= s; g1 *= s; g2 *= s; g3 *= s; g4 *= s; g5 *= s;
    const double c0 = g3 * g5 - g4 * g4, c1 = g2 * g4 - g1 * g5, c2 = g1 * g4 - g2 * g3;
    const double d = g0 * c0 + g1 * c1 + g2 * c2;
    const double id = 1.0 / d;
    const double gu0 = c0 * id, gu1 = c1 * id, gu2 = c2 * id, gu3 = (g0 * g5 - g2 * g2) * id,
                 gu4 = (g1 * g2 - g0 * g4) * id, gu5 = (g0 * g3 - g1 * g1) * id;
    const double tr = gu0 * u[F_AXX] + gu3 * u[F_AYY] + gu5 * u[F_AZZ] +
                      2.0 * (gu1 * u[F_AXY] + gu2 * u[F_AXZ] + gu4 * u[F_AYZ]);
    u[F_GXX] = g0; u[F_GXY] = g1; u[F_GXZ] = g2; u[F_GYY] = g3; u[F_GYZ] = g4; u[F_GZZ] = g5;
    u[F_AXX] -= g0 * tr * (1.0 / 3.0);
    u[F_AXY] -= g1 * tr * (1.0 / 3.0);
    u[F_AXZ] -= g2 * tr * (1.0 / 3.0);
    u[F_AYY] -= g3 * tr * (1.0 / 3.0);
    u[F_AYZ] -= g4 * tr * (1.0 / 3.0);
    u[F_AZZ] -= g5 * tr * (1.0 / 3.0);
    if (u[F_CHI] < P.chi_floor) u[F_CHI] = P.chi_floor;
    if (u[F_ALPHA] < P.alpha_floor) u[F_ALPHA] = P.alpha_floor;
}

}  // namespace z4c
