/*
 * Z4c reference oracle -- TEST INFRASTRUCTURE ONLY (see z4c_oracle.h).
 *
 * The discrete Z4c right-hand side at every active zone.
 *
 * Paper: Sec. 2 (Z4c formulation, Bona-Masso 1+log lapse, Gamma-driver
 * shift; the continuum equations are the standard published vacuum Z4c
 * system, which the paper adopts unchanged), Sec. 3 and its footnote on
 * centred differences of order 2(N_g-1), Sec. 4.3 (Kreiss-Oliger
 * dissipation 0.5, kappa1 = 0.02, kappa2 = 0, 6th-order differencing).
 *
 * Discretisation readings (the paper does not print them):
 *  - centred first and second derivatives of order 2N use the 2N+1 points
 *    -N..N; a mixed derivative is the product of two 1D first-derivative
 *    operators;
 *  - advection beta^d d_d f uses the order-2N lopsided stencil on the points
 *    -(N-1)..N+1 when beta^d > 0 and its mirror image when beta^d < 0;
 *  - Kreiss-Oliger: sigma (-1)^(r+1) 2^(-2r) h^-1 sum_d Delta_d^r f with
 *    r = N+1 and Delta the undivided second difference, on all 22 fields;
 *  - every 1D stencil is evaluated in difference form sum_k w_k (f_k - f_0),
 *    identical to sum_k w_k f_k because the weights of a derivative sum to 0.
 *  - chi is floored (chi_floor) wherever it divides.
 *  - the evolved Gamma^i is used where it is differentiated, in its damping
 *    term and in the shift equation; the metric-derived Gamma_d^i elsewhere.
 *  - 1+log lapse driven by Khat with mu_L = 2/alpha; integrated Gamma-driver
 *    d_t beta^i = mu_S Gamma^i - eta beta^i; both advected.
 */
#include "z4c_oracle.h"
#include <stdlib.h>
#include <string.h>
#include <math.h>

/* Fornberg (1988) recurrence for the weights of derivatives 0..deriv at 0
 * on the nodes pts[0..npts-1]; returns the weights of order `deriv`. */
int or_fd_weights(int deriv, int npts, const double *pts, double *w)
{
    if (npts < 1 || npts > 32 || deriv < 0 || deriv >= npts) return -1;
    double c[32][33];
    memset(c, 0, sizeof(c));
    double c1 = 1.0, c4 = pts[0];
    c[0][0] = 1.0;
    for (int i = 1; i < npts; ++i) {
        int mn = i < deriv ? i : deriv;
        double c2 = 1.0, c5 = c4;
        c4 = pts[i];
        for (int j = 0; j < i; ++j) {
            double c3 = pts[i] - pts[j];
            c2 *= c3;
            if (j == i - 1) {
                for (int k = mn; k >= 1; --k)
                    c[i][k] = c1 * (k * c[i - 1][k - 1] - c5 * c[i - 1][k]) / c2;
                c[i][0] = -c1 * c5 * c[i - 1][0] / c2;
            }
            for (int k = mn; k >= 1; --k) c[j][k] = (c4 * c[j][k] - k * c[j][k - 1]) / c3;
            c[j][0] = c4 * c[j][0] / c3;
        }
        c1 = c2;
    }
    for (int i = 0; i < npts; ++i) w[i] = c[i][deriv];
    return 0;
}

/* ----------------------------------------------------------- stencils */
typedef struct {
    int N;              /* half width: order 2N                               */
    double c1[17];      /* centred d/dx on -N..N, index k+N                   */
    double c2[17];      /* centred d2/dx2 on -N..N                            */
    double lp[17];      /* lopsided (+) on -(N-1)..N+1, index k+N+1           */
    double lm[17];      /* lopsided (-) on -(N+1)..N-1, index k+N+1           */
    double ko[17];      /* Delta^r on -r..r (r=N+1), index k+r, times the
                           factor (-1)^(r+1) 2^(-2r)                          */
} stencils_t;

static int make_stencils(int order, stencils_t *s)
{
    if (order != 4 && order != 6 && order != 8) return -1;
    memset(s, 0, sizeof(*s));
    int N = order / 2;
    s->N = N;
    double p[20];
    for (int k = -N; k <= N; ++k) p[k + N] = k;
    or_fd_weights(1, 2 * N + 1, p, s->c1);
    or_fd_weights(2, 2 * N + 1, p, s->c2);
    double w[20];
    for (int k = -(N - 1); k <= N + 1; ++k) p[k + N - 1] = k;
    or_fd_weights(1, 2 * N + 1, p, w);
    for (int k = -(N - 1); k <= N + 1; ++k) s->lp[k + N + 1] = w[k + N - 1];
    for (int k = -(N + 1); k <= N - 1; ++k) p[k + N + 1] = k;
    or_fd_weights(1, 2 * N + 1, p, w);
    for (int k = -(N + 1); k <= N - 1; ++k) s->lm[k + N + 1] = w[k + N + 1];
    int r = N + 1;
    double binom = 1.0; /* C(2r, r+k) built from k=-r upward */
    double fac = ((r + 1) % 2 == 0 ? 1.0 : -1.0) / ldexp(1.0, 2 * r);
    for (int k = -r; k <= r; ++k) {
        int q = k + r; /* C(2r, q) */
        if (q > 0) binom = binom * (2 * r - q + 1) / q;
        double sgn = ((k + r) % 2 == 0) ? 1.0 : -1.0;
        s->ko[q] = fac * sgn * binom;
    }
    return 0;
}

/* --------------------------------------------------------- zone access */
typedef struct {
    const double *u;    /* block base                                        */
    int64_t E, sf;      /* cells per axis, field stride                      */
    int64_t st[3];      /* strides x, y, z                                   */
} blk_t;

static inline double at(const blk_t *B, int f, int64_t c) { return B->u[f * B->sf + c]; }

/* centred first derivative along a at cell c */
static double d1(const blk_t *B, const stencils_t *S, int f, int64_t c, int a, double ih)
{
    double acc = 0.0, f0 = at(B, f, c);
    for (int k = -S->N; k <= S->N; ++k)
        if (k) acc += S->c1[k + S->N] * (at(B, f, c + k * B->st[a]) - f0);
    return acc * ih;
}

/* second derivative d_a d_b at cell c: centred 1D operator if a == b, else
 * the product of first-derivative operators along a and b */
static double d2(const blk_t *B, const stencils_t *S, int f, int64_t c, int a, int b, double ih)
{
    if (a == b) {
        double acc = 0.0, f0 = at(B, f, c);
        for (int k = -S->N; k <= S->N; ++k)
            if (k) acc += S->c2[k + S->N] * (at(B, f, c + k * B->st[a]) - f0);
        return acc * ih * ih;
    }
    double acc = 0.0, g0 = d1(B, S, f, c, b, ih);
    for (int k = -S->N; k <= S->N; ++k)
        if (k) acc += S->c1[k + S->N] * (d1(B, S, f, c + k * B->st[a], b, ih) - g0);
    return acc * ih;
}

/* lopsided first derivative along a, upwinded for the sign of v */
static double dlop(const blk_t *B, const stencils_t *S, int f, int64_t c, int a, double v, double ih)
{
    int N = S->N;
    double acc = 0.0, f0 = at(B, f, c);
    if (v > 0.0) {
        for (int k = -(N - 1); k <= N + 1; ++k)
            if (k) acc += S->lp[k + N + 1] * (at(B, f, c + k * B->st[a]) - f0);
    } else if (v < 0.0) {
        for (int k = -(N + 1); k <= N - 1; ++k)
            if (k) acc += S->lm[k + N + 1] * (at(B, f, c + k * B->st[a]) - f0);
    }
    return acc * ih;
}

/* Kreiss-Oliger operator summed over the three axes (without sigma/h) */
static double kodiss(const blk_t *B, const stencils_t *S, int f, int64_t c)
{
    int r = S->N + 1;
    double acc = 0.0, f0 = at(B, f, c);
    for (int a = 0; a < 3; ++a)
        for (int k = -r; k <= r; ++k)
            if (k) acc += S->ko[k + r] * (at(B, f, c + k * B->st[a]) - f0);
    return acc;
}

/* ------------------------------------------------------------ algebra */
static const int SYM[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};

static void inverse3(const double g[3][3], double gu[3][3], double *det)
{
    double d = g[0][0] * (g[1][1] * g[2][2] - g[1][2] * g[2][1]) -
               g[0][1] * (g[1][0] * g[2][2] - g[1][2] * g[2][0]) +
               g[0][2] * (g[1][0] * g[2][1] - g[1][1] * g[2][0]);
    double id = 1.0 / d;
    gu[0][0] = (g[1][1] * g[2][2] - g[1][2] * g[2][1]) * id;
    gu[0][1] = (g[0][2] * g[2][1] - g[0][1] * g[2][2]) * id;
    gu[0][2] = (g[0][1] * g[1][2] - g[0][2] * g[1][1]) * id;
    gu[1][0] = (g[1][2] * g[2][0] - g[1][0] * g[2][2]) * id;
    gu[1][1] = (g[0][0] * g[2][2] - g[0][2] * g[2][0]) * id;
    gu[1][2] = (g[0][2] * g[1][0] - g[0][0] * g[1][2]) * id;
    gu[2][0] = (g[1][0] * g[2][1] - g[1][1] * g[2][0]) * id;
    gu[2][1] = (g[0][1] * g[2][0] - g[0][0] * g[2][1]) * id;
    gu[2][2] = (g[0][0] * g[1][1] - g[0][1] * g[1][0]) * id;
    *det = d;
}

/* all the derivative data one zone needs */
typedef struct {
    double chi, g[3][3], Khat, A[3][3], Gam[3], Theta, alpha, beta[3];
    double dchi[3], dg[3][3][3], dKhat[3], dA[3][3][3], dGam[3][3], dTheta[3], dalpha[3],
        dbeta[3][3];
    double ddchi[3][3], ddg[3][3][3][3], ddalpha[3][3], ddbeta[3][3][3];
} zone_t;

static void load_zone(const blk_t *B, const stencils_t *S, int64_t c, double ih, zone_t *z,
                      int need_dA)
{
    z->chi = at(B, O_CHI, c);
    z->Khat = at(B, O_KHAT, c);
    z->Theta = at(B, O_THETA, c);
    z->alpha = at(B, O_ALPHA, c);
    for (int i = 0; i < 3; ++i) {
        z->Gam[i] = at(B, O_GAMX + i, c);
        z->beta[i] = at(B, O_BETAX + i, c);
        for (int j = 0; j < 3; ++j) {
            z->g[i][j] = at(B, O_GXX + SYM[i][j], c);
            z->A[i][j] = at(B, O_AXX + SYM[i][j], c);
        }
    }
    for (int k = 0; k < 3; ++k) {
        /* dX[k] = d_k X */
        z->dchi[k] = d1(B, S, O_CHI, c, k, ih);
        z->dKhat[k] = d1(B, S, O_KHAT, c, k, ih);
        z->dTheta[k] = d1(B, S, O_THETA, c, k, ih);
        z->dalpha[k] = d1(B, S, O_ALPHA, c, k, ih);
        for (int i = 0; i < 3; ++i) {
            z->dGam[k][i] = d1(B, S, O_GAMX + i, c, k, ih);
            z->dbeta[k][i] = d1(B, S, O_BETAX + i, c, k, ih);
            for (int j = 0; j < 3; ++j) {
                z->dg[k][i][j] = d1(B, S, O_GXX + SYM[i][j], c, k, ih);
                z->dA[k][i][j] = need_dA ? d1(B, S, O_AXX + SYM[i][j], c, k, ih) : 0.0;
            }
        }
        for (int l = 0; l < 3; ++l) {
            z->ddchi[k][l] = d2(B, S, O_CHI, c, k, l, ih);
            z->ddalpha[k][l] = d2(B, S, O_ALPHA, c, k, l, ih);
            for (int i = 0; i < 3; ++i) {
                z->ddbeta[k][l][i] = d2(B, S, O_BETAX + i, c, k, l, ih);
                for (int j = 0; j < 3; ++j)
                    z->ddg[k][l][i][j] = d2(B, S, O_GXX + SYM[i][j], c, k, l, ih);
            }
        }
    }
}

/* geometric quantities shared by the RHS and the constraints */
typedef struct {
    double gu[3][3], chib, K;
    double Gl[3][3][3];  /* Gamma~_{kij} = 1/2 (d_i g_jk + d_j g_ik - d_k g_ij) */
    double Gu[3][3][3];  /* Gamma~^k_{ij}                                      */
    double Gd[3];        /* Gamma~_d^i = g^jk Gamma~^i_jk                      */
    double Au[3][3];     /* A~^{ij}                                            */
    double AA;           /* A~_ij A~^ij                                        */
    double R[3][3];      /* R_ij = R~_ij + R^chi_ij                            */
    double Rs;           /* R = chi g~^ij R_ij                                 */
    double DDa[3][3];    /* D_i D_j alpha                                      */
    double trDDa;        /* D^i D_i alpha = chi g~^ij D_i D_j alpha            */
} geom_t;

static void geometry(const zone_t *z, const or_params *p, geom_t *G)
{
    double det;
    inverse3(z->g, G->gu, &det);
    G->chib = z->chi > p->chi_floor ? z->chi : p->chi_floor;
    G->K = z->Khat + 2.0 * z->Theta;
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                G->Gl[k][i][j] = 0.5 * (z->dg[i][j][k] + z->dg[j][i][k] - z->dg[k][i][j]);
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double s = 0.0;
                for (int l = 0; l < 3; ++l) s += G->gu[k][l] * G->Gl[l][i][j];
                G->Gu[k][i][j] = s;
            }
    for (int i = 0; i < 3; ++i) {
        double s = 0.0;
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) s += G->gu[j][k] * G->Gu[i][j][k];
        G->Gd[i] = s;
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) s += G->gu[i][k] * G->gu[j][l] * z->A[k][l];
            G->Au[i][j] = s;
        }
    G->AA = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) G->AA += z->A[i][j] * G->Au[i][j];

    /* conformal Ricci tensor R~_ij */
    double Rt[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int l = 0; l < 3; ++l)
                for (int m = 0; m < 3; ++m) s += -0.5 * G->gu[l][m] * z->ddg[l][m][i][j];
            for (int k = 0; k < 3; ++k)
                s += 0.5 * (z->g[k][i] * z->dGam[j][k] + z->g[k][j] * z->dGam[i][k]);
            for (int k = 0; k < 3; ++k)
                s += G->Gd[k] * 0.5 * (G->Gl[i][j][k] + G->Gl[j][i][k]);
            for (int l = 0; l < 3; ++l)
                for (int m = 0; m < 3; ++m)
                    for (int k = 0; k < 3; ++k)
                        s += G->gu[l][m] * (G->Gu[k][l][i] * G->Gl[j][k][m] +
                                            G->Gu[k][l][j] * G->Gl[i][k][m] +
                                            G->Gu[k][i][m] * G->Gl[k][l][j]);
            Rt[i][j] = s;
        }
    /* conformal-factor part R^chi_ij */
    double Dchi[3][3], trDchi = 0.0, dchi2 = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = z->ddchi[i][j];
            for (int k = 0; k < 3; ++k) s -= G->Gu[k][i][j] * z->dchi[k];
            Dchi[i][j] = s;
        }
    for (int l = 0; l < 3; ++l)
        for (int m = 0; m < 3; ++m) {
            trDchi += G->gu[l][m] * Dchi[l][m];
            dchi2 += G->gu[l][m] * z->dchi[l] * z->dchi[m];
        }
    double ic = 1.0 / G->chib;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double Rc = 0.5 * ic * Dchi[i][j] + 0.5 * ic * z->g[i][j] * trDchi -
                        0.25 * ic * ic * z->dchi[i] * z->dchi[j] -
                        0.75 * ic * ic * z->g[i][j] * dchi2;
            G->R[i][j] = Rt[i][j] + Rc;
        }
    G->Rs = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) G->Rs += z->chi * G->gu[i][j] * G->R[i][j];

    /* physical second covariant derivative of the lapse */
    double dchida = 0.0;
    for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) dchida += G->gu[k][l] * z->dchi[k] * z->dalpha[l];
    G->trDDa = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = z->ddalpha[i][j];
            for (int k = 0; k < 3; ++k) s -= G->Gu[k][i][j] * z->dalpha[k];
            s += 0.5 * ic *
                 (z->dchi[i] * z->dalpha[j] + z->dchi[j] * z->dalpha[i] - z->g[i][j] * dchida);
            G->DDa[i][j] = s;
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) G->trDDa += z->chi * G->gu[i][j] * G->DDa[i][j];
}

static void zone_rhs(const zone_t *z, const or_params *p, double rhs[ONF])
{
    geom_t G;
    geometry(z, p, &G);
    double divb = z->dbeta[0][0] + z->dbeta[1][1] + z->dbeta[2][2];
    for (int f = 0; f < ONF; ++f) rhs[f] = 0.0;
    if (p->terms & OT_PHYS) {
        double a = z->alpha, K = G.K, ic = 1.0 / G.chib;
        rhs[O_CHI] = (2.0 / 3.0) * z->chi * (a * K - divb);
        for (int i = 0; i < 3; ++i)
            for (int j = i; j < 3; ++j) {
                double s = -2.0 * a * z->A[i][j] - (2.0 / 3.0) * z->g[i][j] * divb;
                for (int k = 0; k < 3; ++k) s += z->g[i][k] * z->dbeta[j][k] + z->g[j][k] * z->dbeta[i][k];
                rhs[O_GXX + SYM[i][j]] = s;
            }
        rhs[O_KHAT] = -G.trDDa + a * (G.AA + K * K / 3.0) + p->kappa1 * (1.0 - p->kappa2) * a * z->Theta;
        /* trace-free part of X_ij = -D_i D_j alpha + alpha R_ij */
        double X[3][3], trX = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) X[i][j] = -G.DDa[i][j] + a * G.R[i][j];
        for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l) trX += G.gu[k][l] * X[k][l];
        for (int i = 0; i < 3; ++i)
            for (int j = i; j < 3; ++j) {
                double s = z->chi * (X[i][j] - z->g[i][j] * trX / 3.0);
                double AgA = 0.0;
                for (int k = 0; k < 3; ++k)
                    for (int l = 0; l < 3; ++l) AgA += z->A[i][k] * G.gu[k][l] * z->A[l][j];
                s += a * (K * z->A[i][j] - 2.0 * AgA);
                for (int k = 0; k < 3; ++k) s += z->A[i][k] * z->dbeta[j][k] + z->A[j][k] * z->dbeta[i][k];
                s -= (2.0 / 3.0) * z->A[i][j] * divb;
                rhs[O_AXX + SYM[i][j]] = s;
            }
        for (int i = 0; i < 3; ++i) {
            double s = (2.0 / 3.0) * G.Gd[i] * divb;
            for (int j = 0; j < 3; ++j) s -= G.Gd[j] * z->dbeta[j][i];
            for (int j = 0; j < 3; ++j)
                for (int k = 0; k < 3; ++k)
                    s += G.gu[j][k] * z->ddbeta[j][k][i] + G.gu[i][j] * z->ddbeta[j][k][k] / 3.0;
            for (int j = 0; j < 3; ++j) s -= 2.0 * G.Au[i][j] * z->dalpha[j];
            double t = 0.0;
            for (int j = 0; j < 3; ++j)
                for (int k = 0; k < 3; ++k) t += G.Gu[i][j][k] * G.Au[j][k];
            for (int j = 0; j < 3; ++j) t -= 1.5 * G.Au[i][j] * z->dchi[j] * ic;
            for (int j = 0; j < 3; ++j) t -= G.gu[i][j] * (2.0 * z->dKhat[j] + z->dTheta[j]) / 3.0;
            s += 2.0 * a * t;
            s -= 2.0 * a * p->kappa1 * (z->Gam[i] - G.Gd[i]);
            rhs[O_GAMX + i] = s;
        }
        rhs[O_THETA] = 0.5 * a * (G.Rs - G.AA + (2.0 / 3.0) * K * K) - a * p->kappa1 * (2.0 + p->kappa2) * z->Theta;
    }
    if (p->terms & OT_GAUGE) {
        rhs[O_ALPHA] = -2.0 * z->alpha * z->Khat;
        for (int i = 0; i < 3; ++i) rhs[O_BETAX + i] = p->mu_S * z->Gam[i] - p->eta * z->beta[i];
    }
}

int or_rhs(const or_mesh *m, const or_params *p, const double *u, double *rhs)
{
    return or_rhs_blocks(m, p, u, rhs, 0);
}

int or_rhs_blocks(const or_mesh *m, const or_params *p, const double *u, double *rhs,
                  const int8_t *only)
{
    stencils_t S;
    if (make_stencils(p->fd_order, &S)) return -1;
    int g = m->g;
    if (g < S.N + 1) return -1;
    int64_t roff = 0;
    for (int b = 0; b < m->nb; ++b) {
        int n = m->n[b];
        if (only && !only[b]) { roff += (int64_t)ONF * n * n * n; continue; }
        blk_t B;
        B.E = n + 2 * g;
        B.u = u + or_block_offset(m, b);
        B.sf = B.E * B.E * B.E;
        B.st[0] = 1; B.st[1] = B.E; B.st[2] = B.E * B.E;
        double h = m->dx0 / (double)(1 << m->level[b]), ih = 1.0 / h;
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    int64_t c = ((int64_t)(k + g) * B.E + (j + g)) * B.E + (i + g);
                    zone_t z;
                    load_zone(&B, &S, c, ih, &z, 0);
                    double r[ONF];
                    zone_rhs(&z, p, r);
                    for (int f = 0; f < ONF; ++f) {
                        /* advection of the lapse and shift belongs to the gauge */
                        int gauge_field = (f == O_ALPHA || f >= O_BETAX);
                        if ((p->terms & OT_ADVECT) && (!gauge_field || (p->terms & OT_GAUGE)))
                            for (int a = 0; a < 3; ++a)
                                r[f] += z.beta[a] * dlop(&B, &S, f, c, a, z.beta[a], ih);
                        if (p->terms & OT_DISSIP) r[f] += p->ko_sigma * ih * kodiss(&B, &S, f, c);
                    }
                    for (int f = 0; f < ONF; ++f)
                        rhs[roff + (((int64_t)f * n + k) * n + j) * n + i] = r[f];
                }
        roff += (int64_t)ONF * n * n * n;
    }
    return 0;
}

/* ------------------------------------------------------- constraints */
int or_constraints(const or_mesh *m, const or_params *p, const double *u, double *out, int nexc,
                   const double *exc, double r_exc, double *norms)
{
    stencils_t S;
    if (make_stencils(p->fd_order, &S)) return -1;
    int g = m->g;
    double sH2 = 0, sHi = 0, sM2 = 0, sMi = 0, sT2 = 0, sG2 = 0, vol = 0;
    int64_t coff = 0;
    for (int b = 0; b < m->nb; ++b) {
        int n = m->n[b];
        blk_t B;
        B.E = n + 2 * g;
        B.u = u + or_block_offset(m, b);
        B.sf = B.E * B.E * B.E;
        B.st[0] = 1; B.st[1] = B.E; B.st[2] = B.E * B.E;
        double h = m->dx0 / (double)(1 << m->level[b]), ih = 1.0 / h, dv = h * h * h;
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    int64_t c = ((int64_t)(k + g) * B.E + (j + g)) * B.E + (i + g);
                    zone_t z;
                    load_zone(&B, &S, c, ih, &z, 1);
                    geom_t G;
                    geometry(&z, p, &G);
                    double H = G.Rs - G.AA + (2.0 / 3.0) * G.K * G.K;
                    double M[3];
                    double dK[3];
                    for (int q = 0; q < 3; ++q) dK[q] = z.dKhat[q] + 2.0 * z.dTheta[q];
                    /* d_k g~^{ab} = -g~^ac g~^bd d_k g~_cd */
                    double dgu[3][3][3];
                    for (int k2 = 0; k2 < 3; ++k2)
                        for (int a = 0; a < 3; ++a)
                            for (int bb = 0; bb < 3; ++bb) {
                                double s = 0.0;
                                for (int cc = 0; cc < 3; ++cc)
                                    for (int d = 0; d < 3; ++d)
                                        s -= G.gu[a][cc] * G.gu[bb][d] * z.dg[k2][cc][d];
                                dgu[k2][a][bb] = s;
                            }
                    for (int ii = 0; ii < 3; ++ii) {
                        /* d_j A~^{ij} by the product rule */
                        double s = 0.0;
                        for (int jj = 0; jj < 3; ++jj)
                            for (int kk = 0; kk < 3; ++kk)
                                for (int ll = 0; ll < 3; ++ll)
                                    s += dgu[jj][ii][kk] * G.gu[jj][ll] * z.A[kk][ll] +
                                         G.gu[ii][kk] * dgu[jj][jj][ll] * z.A[kk][ll] +
                                         G.gu[ii][kk] * G.gu[jj][ll] * z.dA[jj][kk][ll];
                        for (int jj = 0; jj < 3; ++jj)
                            for (int kk = 0; kk < 3; ++kk) s += G.Gu[ii][jj][kk] * G.Au[jj][kk];
                        for (int jj = 0; jj < 3; ++jj) s -= (2.0 / 3.0) * G.gu[ii][jj] * dK[jj];
                        for (int jj = 0; jj < 3; ++jj) s -= 1.5 * G.Au[ii][jj] * z.dchi[jj] / G.chib;
                        M[ii] = s;
                    }
                    double Gc[3];
                    for (int q = 0; q < 3; ++q) Gc[q] = z.Gam[q] - G.Gd[q];
                    if (out) {
                        double vals[8] = {H, M[0], M[1], M[2], z.Theta, Gc[0], Gc[1], Gc[2]};
                        for (int q = 0; q < 8; ++q)
                            out[coff + (((int64_t)q * n + k) * n + j) * n + i] = vals[q];
                    }
                    /* norm region */
                    double x = m->lo[0] + (m->ilo[3 * b] + i + 0.5) * h;
                    double y = m->lo[1] + (m->ilo[3 * b + 1] + j + 0.5) * h;
                    double zz = m->lo[2] + (m->ilo[3 * b + 2] + k + 0.5) * h;
                    int keep = 1;
                    for (int e = 0; e < nexc; ++e) {
                        double dx_ = x - exc[3 * e], dy_ = y - exc[3 * e + 1], dz_ = zz - exc[3 * e + 2];
                        if (dx_ * dx_ + dy_ * dy_ + dz_ * dz_ < r_exc * r_exc) keep = 0;
                    }
                    if (!keep) continue;
                    double M2 = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
                    double G2 = Gc[0] * Gc[0] + Gc[1] * Gc[1] + Gc[2] * Gc[2];
                    sH2 += H * H * dv;
                    sM2 += M2 * dv;
                    sT2 += z.Theta * z.Theta * dv;
                    sG2 += G2 * dv;
                    vol += dv;
                    if (fabs(H) > sHi) sHi = fabs(H);
                    if (sqrt(M2) > sMi) sMi = sqrt(M2);
                }
        coff += (int64_t)8 * n * n * n;
    }
    if (norms) {
        norms[0] = vol > 0 ? sqrt(sH2 / vol) : 0.0;
        norms[1] = sHi;
        norms[2] = vol > 0 ? sqrt(sM2 / vol) : 0.0;
        norms[3] = sMi;
        norms[4] = vol > 0 ? sqrt(sT2 / vol) : 0.0;
        norms[5] = vol > 0 ? sqrt(sG2 / vol) : 0.0;
    }
    return 0;
}

/* ------------------------------------------------ refinement criteria */
/* Sec. 3.3: chi-min (refine if chi falls below a threshold), dchi-max
 * (refine if the gradient of chi exceeds a threshold), radius (keep blocks
 * within a radius of a point at or above a level).  Reductions run over
 * active zones; |d chi| is the Euclidean norm of the centred gradient.
 * Derefinement (not described in the paper): the refine test fails with a
 * hysteresis factor (chi_min > 1.5 chi_thr, max|d chi| < 0.5 dchi_thr). */
int or_refine_flags(const or_mesh *m, const or_params *p, const double *u, int criterion,
                    double chi_thr, double dchi_thr, int level_max, double radius,
                    const double *centre, int radius_level, int8_t *flags)
{
    stencils_t S;
    if (make_stencils(p->fd_order, &S)) return -1;
    int g = m->g;
    for (int b = 0; b < m->nb; ++b) {
        int n = m->n[b];
        blk_t B;
        B.E = n + 2 * g;
        B.u = u + or_block_offset(m, b);
        B.sf = B.E * B.E * B.E;
        B.st[0] = 1; B.st[1] = B.E; B.st[2] = B.E * B.E;
        double h = m->dx0 / (double)(1 << m->level[b]), ih = 1.0 / h;
        double chimin = INFINITY, gmax = 0.0, rmin = INFINITY;
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    int64_t c = ((int64_t)(k + g) * B.E + (j + g)) * B.E + (i + g);
                    double ch = at(&B, O_CHI, c);
                    if (ch < chimin) chimin = ch;
                    if (criterion == 1) {
                        double gx = d1(&B, &S, O_CHI, c, 0, ih), gy = d1(&B, &S, O_CHI, c, 1, ih),
                               gz = d1(&B, &S, O_CHI, c, 2, ih);
                        double gn = sqrt(gx * gx + gy * gy + gz * gz);
                        if (gn > gmax) gmax = gn;
                    }
                    if (criterion == 2) {
                        double x = m->lo[0] + (m->ilo[3 * b] + i + 0.5) * h - centre[0];
                        double y = m->lo[1] + (m->ilo[3 * b + 1] + j + 0.5) * h - centre[1];
                        double zz = m->lo[2] + (m->ilo[3 * b + 2] + k + 0.5) * h - centre[2];
                        double r = sqrt(x * x + y * y + zz * zz);
                        if (r < rmin) rmin = r;
                    }
                }
        int f = 0, lev = m->level[b];
        if (criterion == 0) {
            if (chimin < chi_thr) f = 1;
            else if (chimin > 1.5 * chi_thr) f = -1;
        } else if (criterion == 1) {
            if (gmax > dchi_thr) f = 1;
            else if (gmax < 0.5 * dchi_thr) f = -1;
        } else if (criterion == 2) {
            f = (rmin < radius && lev < radius_level) ? 1 : 0;
        } else return -1;
        if (f > 0 && lev >= level_max) f = 0;
        if (f < 0 && lev == 0) f = 0;
        flags[b] = (int8_t)f;
    }
    return 0;
}

/* --------------------------------------------------------------- Psi4 */
/* Outgoing Weyl scalar in a coordinate tetrad (Sec. 3.4 wave extraction).
 * Physical metric gamma_ij = g~_ij / chi and extrinsic curvature
 * K_ij = A~_ij / chi + gamma_ij K / 3 with K = Khat + 2 Theta; their
 * derivatives follow from the centred derivatives of the evolved fields by
 * the product rule.  Electric and magnetic parts of the Weyl tensor (vacuum):
 *   E_ij = R_ij - K_ik K^k_j + K K_ij   (K the trace of K_ij),
 *   B_ij = symmetric part of eps_i^kl D_k K_lj.
 * Tetrad: radial v = x - origin, u = (-v_y, v_x, 0), w^a = eps^a_bc u^b v^c,
 * Gram-Schmidt in the order v, w, u -> e_r, e_theta, e_phi;
 * m = (e_theta + i e_phi)/sqrt 2 and Psi4 = -(E_ij - i B_ij) mbar^i mbar^j,
 * which is  d2h+/dt2 - i d2hx/dt2  for an outgoing linear wave. */
static int levi(int a, int b, int c)
{
    if (a == b || b == c || a == c) return 0;
    return ((a == 0 && b == 1) || (a == 1 && b == 2) || (a == 2 && b == 0)) ? 1 : -1;
}

static void zone_psi4(const zone_t *z, const double x[3], double out[2])
{
    const double ic = 1.0 / z->chi;
    double gam[3][3], dgam[3][3][3], ddgam[3][3][3][3], Kij[3][3], dKij[3][3][3], dK[3];
    const double Kt = z->Khat + 2.0 * z->Theta;
    for (int k = 0; k < 3; ++k) dK[k] = z->dKhat[k] + 2.0 * z->dTheta[k];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) gam[i][j] = z->g[i][j] * ic;
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) dgam[k][i][j] = (z->dg[k][i][j] - gam[i][j] * z->dchi[k]) * ic;
    for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l)
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j)
                    ddgam[k][l][i][j] = (z->ddg[k][l][i][j] - dgam[k][i][j] * z->dchi[l] -
                                         dgam[l][i][j] * z->dchi[k] - gam[i][j] * z->ddchi[k][l]) * ic;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Kij[i][j] = z->A[i][j] * ic + gam[i][j] * Kt / 3.0;
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                dKij[k][i][j] = (z->dA[k][i][j] - z->A[i][j] * z->dchi[k] * ic) * ic +
                                dgam[k][i][j] * Kt / 3.0 + gam[i][j] * dK[k] / 3.0;
    double gu[3][3], det;
    inverse3(gam, gu, &det);
    const double sg = sqrt(det);
    /* Christoffel symbols Gamma^k_ij and their derivatives d_m Gamma^k_ij */
    double G[3][3][3], dG[3][3][3][3], dgu[3][3][3];
    for (int m = 0; m < 3; ++m)
        for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l) {
                double s = 0.0;
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) s -= gu[k][a] * gu[l][b] * dgam[m][a][b];
                dgu[m][k][l] = s;
            }
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double s = 0.0;
                for (int l = 0; l < 3; ++l)
                    s += gu[k][l] * (dgam[i][j][l] + dgam[j][i][l] - dgam[l][i][j]);
                G[k][i][j] = 0.5 * s;
            }
    for (int m = 0; m < 3; ++m)
        for (int k = 0; k < 3; ++k)
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    double s = 0.0;
                    for (int l = 0; l < 3; ++l)
                        s += dgu[m][k][l] * (dgam[i][j][l] + dgam[j][i][l] - dgam[l][i][j]) +
                             gu[k][l] * (ddgam[m][i][j][l] + ddgam[m][j][i][l] - ddgam[m][l][i][j]);
                    dG[m][k][i][j] = 0.5 * s;
                }
    /* Ricci tensor R_ij = d_k G^k_ij - d_j G^k_ik + G^k_kp G^p_ij - G^k_jp G^p_ik */
    double R[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) {
                s += dG[k][k][i][j] - dG[j][k][i][k];
                for (int p = 0; p < 3; ++p) s += G[k][k][p] * G[p][i][j] - G[k][j][p] * G[p][i][k];
            }
            R[i][j] = s;
        }
    double trK = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) trK += gu[i][j] * Kij[i][j];
    double E[3][3], Bm[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double kk = 0.0;
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) kk += Kij[i][k] * gu[k][l] * Kij[l][j];
            E[i][j] = R[i][j] - kk + trK * Kij[i][j];
        }
    /* D_k K_lj */
    double DK[3][3][3];
    for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l)
            for (int j = 0; j < 3; ++j) {
                double s = dKij[k][l][j];
                for (int m = 0; m < 3; ++m) s -= G[m][k][l] * Kij[m][j] + G[m][k][j] * Kij[l][m];
                DK[k][l][j] = s;
            }
    double Braw[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int m = 0; m < 3; ++m)
                for (int k = 0; k < 3; ++k)
                    for (int l = 0; l < 3; ++l) {
                        const int e = levi(m, k, l);
                        if (e) s += gam[i][m] * (e / sg) * DK[k][l][j];
                    }
            Braw[i][j] = s;
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Bm[i][j] = 0.5 * (Braw[i][j] + Braw[j][i]);
    /* tetrad */
    double v[3] = {x[0], x[1], x[2]}, u[3] = {-x[1], x[0], 0.0}, w[3];
    for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (int d = 0; d < 3; ++d)
            for (int b = 0; b < 3; ++b)
                for (int c = 0; c < 3; ++c) {
                    const int e = levi(d, b, c);
                    if (e) s += gu[a][d] * (e * sg) * u[b] * v[c];
                }
        w[a] = s;
    }
#define DOT(p, q) (gam[0][0]*p[0]*q[0] + gam[1][1]*p[1]*q[1] + gam[2][2]*p[2]*q[2] + \
                   gam[0][1]*(p[0]*q[1] + p[1]*q[0]) + gam[0][2]*(p[0]*q[2] + p[2]*q[0]) + \
                   gam[1][2]*(p[1]*q[2] + p[2]*q[1]))
    double uu = DOT(u, u), vv = DOT(v, v);
    if (!(uu > 1e-24 * vv) || !(vv > 0.0)) { out[0] = out[1] = 0.0; return; }
    double er[3], et[3], ep[3];
    for (int a = 0; a < 3; ++a) er[a] = v[a] / sqrt(vv);
    double wr = DOT(w, er);
    for (int a = 0; a < 3; ++a) et[a] = w[a] - wr * er[a];
    double tt = DOT(et, et);
    for (int a = 0; a < 3; ++a) et[a] /= sqrt(tt);
    double ur = DOT(u, er), ut = DOT(u, et);
    for (int a = 0; a < 3; ++a) ep[a] = u[a] - ur * er[a] - ut * et[a];
    double pp = DOT(ep, ep);
    for (int a = 0; a < 3; ++a) ep[a] /= sqrt(pp);
#undef DOT
    double EP = 0.0, EQ = 0.0, BP = 0.0, BQ = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const double P = 0.5 * (et[i] * et[j] - ep[i] * ep[j]);
            const double Q = 0.5 * (et[i] * ep[j] + ep[i] * et[j]);
            EP += E[i][j] * P; EQ += E[i][j] * Q;
            BP += Bm[i][j] * P; BQ += Bm[i][j] * Q;
        }
    out[0] = -EP + BQ;
    out[1] = EQ + BP;
}

int or_psi4(const or_mesh *m, const or_params *p, const double *u, const double *origin, double *out)
{
    stencils_t S;
    if (make_stencils(p->fd_order, &S)) return -1;
    int g = m->g;
    if (g < S.N + 1) return -1;
    int64_t roff = 0;
    for (int b = 0; b < m->nb; ++b) {
        int n = m->n[b];
        blk_t B;
        B.E = n + 2 * g;
        B.u = u + or_block_offset(m, b);
        B.sf = B.E * B.E * B.E;
        B.st[0] = 1; B.st[1] = B.E; B.st[2] = B.E * B.E;
        double h = m->dx0 / (double)(1 << m->level[b]), ih = 1.0 / h;
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    int64_t c = ((int64_t)(k + g) * B.E + (j + g)) * B.E + (i + g);
                    zone_t z;
                    load_zone(&B, &S, c, ih, &z, 1);
                    double x[3] = {m->lo[0] + (m->ilo[3 * b] + i + 0.5) * h - origin[0],
                                   m->lo[1] + (m->ilo[3 * b + 1] + j + 0.5) * h - origin[1],
                                   m->lo[2] + (m->ilo[3 * b + 2] + k + 0.5) * h - origin[2]};
                    double ps[2];
                    zone_psi4(&z, x, ps);
                    for (int q = 0; q < 2; ++q)
                        out[roff + (((int64_t)q * n + k) * n + j) * n + i] = ps[q];
                }
        roff += (int64_t)2 * n * n * n;
    }
    return 0;
}
