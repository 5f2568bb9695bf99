/*
 * Z4c reference oracle -- TEST INFRASTRUCTURE ONLY (see z4c_oracle.h).
 *
 * Per-MeshBlock features for the learned refinement indicator: cheap
 * reductions of the state over a block's active zones, the kind of
 * quantities the chi-based criteria of Sec. 3.3 use (chi itself, the
 * gradient of chi) widened to the other fields.  Sixteen raw features:
 *   0 max |d chi|        1 mean |d chi|      2 max |d alpha|   3 mean |d alpha|
 *   4 max |dd g~|        5 mean |dd g~|      6 min alpha       7 min chi
 *   8 max |Khat|         9 max |A~|         10 max |Theta|    11 max |Gamma~|
 *  12 max |beta|        13 max |dd chi|     14 max |d Khat|   15 log2 dx
 * |d f| is the Euclidean norm of the centred gradient; |dd g~| at a zone is
 * the largest |d_a d_b g~_ij| over all components; |A~| = sqrt(sum_ij A~_ij^2)
 * over all nine entries; vector norms are Euclidean.
 */
#include "z4c_oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* the oracle's own stencil helpers live in rhs.c; restated minimally here */
int or_fd_weights(int deriv, int npts, const double *pts, double *w);

static const int SY[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};

int or_block_features(const or_mesh *m, const or_params *p, const double *u, double *feat)
{
    int N = p->fd_order / 2;
    if (N < 2 || N > 4) return -1;
    double pts[9], c1[9], c2[9];
    for (int k = -N; k <= N; ++k) pts[k + N] = k;
    or_fd_weights(1, 2 * N + 1, pts, c1);
    or_fd_weights(2, 2 * N + 1, pts, c2);
    int g = m->g;
    for (int b = 0; b < m->nb; ++b) {
        int n = m->n[b];
        int64_t E = n + 2 * g, sf = E * E * E, st[3] = {1, E, E * E};
        const double *B = u + or_block_offset(m, b);
        double h = m->dx0 / (double)(1 << m->level[b]), ih = 1.0 / h;
        double f[16];
        for (int q = 0; q < 16; ++q) f[q] = 0.0;
        f[6] = INFINITY;
        f[7] = INFINITY;
        double cnt = 0.0;
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    int64_t c = ((int64_t)(k + g) * E + (j + g)) * E + (i + g);
                    double grad[3][3]; /* chi, alpha, Khat */
                    const int gf[3] = {O_CHI, O_ALPHA, O_KHAT};
                    for (int q = 0; q < 3; ++q)
                        for (int a = 0; a < 3; ++a) {
                            double s = 0.0, f0 = B[gf[q] * sf + c];
                            for (int kk = -N; kk <= N; ++kk)
                                if (kk) s += c1[kk + N] * (B[gf[q] * sf + c + kk * st[a]] - f0);
                            grad[q][a] = s * ih;
                        }
                    /* second derivatives: pure (centred) and mixed (product of d1) */
                    double ddg = 0.0, ddchi = 0.0;
                    for (int fi = 0; fi < 7; ++fi) {
                        int fld = fi == 6 ? O_CHI : O_GXX + fi;
                        for (int a = 0; a < 3; ++a)
                            for (int bb = a; bb < 3; ++bb) {
                                double s = 0.0;
                                if (a == bb) {
                                    double f0 = B[fld * sf + c];
                                    for (int kk = -N; kk <= N; ++kk)
                                        if (kk) s += c2[kk + N] * (B[fld * sf + c + kk * st[a]] - f0);
                                    s *= ih * ih;
                                } else {
                                    /* c1 is odd, so the sum over +-p1, +-p2 pairs is a
                                     * double difference (exactly 0 on constants) */
                                    const double *F = B + fld * sf + c;
                                    for (int p1 = 1; p1 <= N; ++p1)
                                        for (int p2 = 1; p2 <= N; ++p2)
                                            s += c1[p1 + N] * c1[p2 + N] *
                                                 ((F[p1 * st[a] + p2 * st[bb]] - F[p1 * st[a] - p2 * st[bb]]) -
                                                  (F[-p1 * st[a] + p2 * st[bb]] - F[-p1 * st[a] - p2 * st[bb]]));
                                    s *= ih * ih;
                                }
                                if (fi == 6) { if (fabs(s) > ddchi) ddchi = fabs(s); }
                                else if (fabs(s) > ddg) ddg = fabs(s);
                            }
                    }
                    double nchi = sqrt(grad[0][0] * grad[0][0] + grad[0][1] * grad[0][1] + grad[0][2] * grad[0][2]);
                    double nal = sqrt(grad[1][0] * grad[1][0] + grad[1][1] * grad[1][1] + grad[1][2] * grad[1][2]);
                    double nK = sqrt(grad[2][0] * grad[2][0] + grad[2][1] * grad[2][1] + grad[2][2] * grad[2][2]);
                    double A2 = 0.0;
                    for (int a = 0; a < 3; ++a)
                        for (int bb = 0; bb < 3; ++bb) {
                            double v = B[(O_AXX + SY[a][bb]) * sf + c];
                            A2 += v * v;
                        }
                    double G2 = 0.0, b2 = 0.0;
                    for (int a = 0; a < 3; ++a) {
                        double v = B[(O_GAMX + a) * sf + c], w = B[(O_BETAX + a) * sf + c];
                        G2 += v * v;
                        b2 += w * w;
                    }
                    double al = B[O_ALPHA * sf + c], ch = B[O_CHI * sf + c];
                    if (nchi > f[0]) f[0] = nchi;
                    f[1] += nchi;
                    if (nal > f[2]) f[2] = nal;
                    f[3] += nal;
                    if (ddg > f[4]) f[4] = ddg;
                    f[5] += ddg;
                    if (al < f[6]) f[6] = al;
                    if (ch < f[7]) f[7] = ch;
                    if (fabs(B[O_KHAT * sf + c]) > f[8]) f[8] = fabs(B[O_KHAT * sf + c]);
                    if (sqrt(A2) > f[9]) f[9] = sqrt(A2);
                    if (fabs(B[O_THETA * sf + c]) > f[10]) f[10] = fabs(B[O_THETA * sf + c]);
                    if (sqrt(G2) > f[11]) f[11] = sqrt(G2);
                    if (sqrt(b2) > f[12]) f[12] = sqrt(b2);
                    if (ddchi > f[13]) f[13] = ddchi;
                    if (nK > f[14]) f[14] = nK;
                    cnt += 1.0;
                }
        f[1] /= cnt;
        f[3] /= cnt;
        f[5] /= cnt;
        f[15] = log2(h);
        memcpy(feat + 16 * b, f, sizeof(f));
    }
    return 0;
}
