/*
 * Z4c reference oracle -- TEST INFRASTRUCTURE ONLY (see z4c_oracle.h).
 *
 * Classic four-stage Runge-Kutta (Sec. 3: an explicit RK family with the
 * ghosts filled at each stage; Sec. 4.3: RK4 in every test), on four
 * registers U, S1, S2 and an accumulator A:
 *   stage 1: k1 = F(U):   S1 = U + dt/2 k1,  A  = U + dt/6 k1
 *   stage 2: k2 = F(S1):  S2 = U + dt/2 k2,  A += dt/3 k2
 *   stage 3: k3 = F(S2):  S1 = U + dt   k3,  A += dt/3 k3
 *   stage 4: k4 = F(S1):  U  = A + dt/6 k4
 * which is U_{n+1} = U_n + dt (k1 + 2 k2 + 2 k3 + k4)/6.
 *
 * After each write of S1, S2 or U (active zones only), when enabled:
 * det(g~) = 1 is restored by g~ <- det(g~)^(-1/3) g~, A~ is made trace-free
 * with the new metric, then chi <- max(chi, chi_floor) and
 * alpha <- max(alpha, alpha_floor).  (The paper prints none of this; it is
 * the usual algebraic-constraint enforcement of the Z4c literature.)
 */
#include "z4c_oracle.h"
#include <stdlib.h>
#include <string.h>
#include <math.h>

static const int SYMI[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};

static void enforce_zone(const or_params *p, double *v /* [ONF] */)
{
    double g[3][3], A[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            g[i][j] = v[O_GXX + SYMI[i][j]];
            A[i][j] = v[O_AXX + SYMI[i][j]];
        }
    double det = g[0][0] * (g[1][1] * g[2][2] - g[1][2] * g[2][1]) -
                 g[0][1] * (g[1][0] * g[2][2] - g[1][2] * g[2][0]) +
                 g[0][2] * (g[1][0] * g[2][1] - g[1][1] * g[2][0]);
    double s = 1.0 / cbrt(det);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) g[i][j] *= s;
    /* inverse of the rescaled metric */
    double d = g[0][0] * (g[1][1] * g[2][2] - g[1][2] * g[2][1]) -
               g[0][1] * (g[1][0] * g[2][2] - g[1][2] * g[2][0]) +
               g[0][2] * (g[1][0] * g[2][1] - g[1][1] * g[2][0]);
    double gu[3][3];
    gu[0][0] = (g[1][1] * g[2][2] - g[1][2] * g[2][1]) / d;
    gu[0][1] = (g[0][2] * g[2][1] - g[0][1] * g[2][2]) / d;
    gu[0][2] = (g[0][1] * g[1][2] - g[0][2] * g[1][1]) / d;
    gu[1][0] = gu[0][1];
    gu[1][1] = (g[0][0] * g[2][2] - g[0][2] * g[2][0]) / d;
    gu[1][2] = (g[0][2] * g[1][0] - g[0][0] * g[1][2]) / d;
    gu[2][0] = gu[0][2];
    gu[2][1] = gu[1][2];
    gu[2][2] = (g[0][0] * g[1][1] - g[0][1] * g[1][0]) / d;
    double tr = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) tr += gu[i][j] * A[i][j];
    for (int i = 0; i < 3; ++i)
        for (int j = i; j < 3; ++j) {
            v[O_GXX + SYMI[i][j]] = g[i][j];
            v[O_AXX + SYMI[i][j]] = A[i][j] - g[i][j] * tr / 3.0;
        }
    if (v[O_CHI] < p->chi_floor) v[O_CHI] = p->chi_floor;
    if (v[O_ALPHA] < p->alpha_floor) v[O_ALPHA] = p->alpha_floor;
}

/* the register update of one stage from its right-hand side k (interior
 * layout), for the blocks with only[b] != 0 (all when only is NULL) */
int or_rk4_update(const or_mesh *m, const or_params *p, int stage, double dt, const double *k,
                  double *U, double *S1, double *S2, double *A, const int8_t *only)
{
    if (stage < 1 || stage > 4) return -1;
    int g = m->g;
    int64_t roff = 0;
    for (int b = 0; b < m->nb; ++b) {
        int n = m->n[b];
        int64_t E = n + 2 * g, off = or_block_offset(m, b), sf = E * E * E, sr = (int64_t)n * n * n;
        if (only && !only[b]) { roff += (int64_t)ONF * sr; continue; }
        for (int kk = 0; kk < n; ++kk)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    int64_t c = ((int64_t)(kk + g) * E + (j + g)) * E + (i + g);
                    int64_t ci = ((int64_t)kk * n + j) * n + i;
                    double out[ONF];
                    double *dst = stage == 1 ? S1 : stage == 2 ? S2 : stage == 3 ? S1 : U;
                    for (int f = 0; f < ONF; ++f) {
                        double kv = k[roff + f * sr + ci];
                        int64_t q = off + f * sf + c;
                        switch (stage) {
                        case 1: out[f] = U[q] + 0.5 * dt * kv; A[q] = U[q] + dt / 6.0 * kv; break;
                        case 2: out[f] = U[q] + 0.5 * dt * kv; A[q] += dt / 3.0 * kv; break;
                        case 3: out[f] = U[q] + dt * kv; A[q] += dt / 3.0 * kv; break;
                        default: out[f] = A[q] + dt / 6.0 * kv; break;
                        }
                    }
                    if (p->enforce) enforce_zone(p, out);
                    for (int f = 0; f < ONF; ++f) dst[off + f * sf + c] = out[f];
                }
        roff += (int64_t)ONF * sr;
    }
    return 0;
}

int or_rk4_stage(const or_mesh *m, const or_params *p, int stage, double dt, double *U,
                 double *S1, double *S2, double *A)
{
    if (stage < 1 || stage > 4) return -1;
    double *src = stage == 1 ? U : stage == 2 ? S1 : stage == 3 ? S2 : S1;
    int rc = or_fill_ghosts(m, src);
    if (rc) return rc;
    /* interior RHS */
    int64_t nint = 0;
    for (int b = 0; b < m->nb; ++b) nint += (int64_t)ONF * m->n[b] * m->n[b] * m->n[b];
    double *k = (double *)malloc(sizeof(double) * (nint > 0 ? nint : 1));
    if (!k) return -2;
    rc = or_rhs(m, p, src, k);
    if (!rc) rc = or_rk4_update(m, p, stage, dt, k, U, S1, S2, A, NULL);
    free(k);
    return rc;
}
