/*
 * Z4c reference oracle -- TEST INFRASTRUCTURE ONLY (see z4c_oracle.h).
 *
 * Mesh bookkeeping and the per-stage ghost fill (Sec. 3: "the ghost zones
 * are filled by either the active region of neighboring MeshBlocks or the
 * boundary conditions"), including the Lagrange restriction and
 * prolongation at refinement boundaries (Sec. 3.1, Eqs. 1-2).
 *
 * Readings (the paper describes the mechanism with coarse buffers; the
 * values it produces are defined here pointwise):
 *  - A ghost cell takes the value of the field at its cell centre, after the
 *    domain boundary condition is applied to its global index: periodic wrap,
 *    or outflow = clamp to the nearest active cell of the domain (a copy of
 *    the nearest active zone, applied to every axis that lies outside).
 *  - If a leaf of the same level covers the centre: copy of its active value.
 *  - If a finer leaf covers it: restriction = tensor-product Lagrange
 *    interpolation (Eqs. 1-2) through the n = g+1 fine centres per axis
 *    nearest the target, all inside the owning fine block's active region
 *    (window shifted inward at its edges, ties towards the block interior).
 *  - If a coarser leaf covers it: prolongation = Lagrange interpolation
 *    through the n = g+1 coarse centres nearest the target per axis; each
 *    coarse value is the active value of a coarse leaf or, where finer data
 *    cover that coarse cell, its restriction ("composite" coarse values, what
 *    the coarse-buffer exchange of Sec. 3.1 assembles).  A stencil that would
 *    need data two levels away is an error.
 *  - The interpolation order is n (n points, exact to degree n-1): the text's
 *    "order n+1" conflicts with its own 3rd/5th-order statements for n=3,5.
 */
#include "z4c_oracle.h"
#include <stdlib.h>
#include <string.h>
#include <math.h>

int64_t or_block_offset(const or_mesh *m, int b)
{
    int64_t off = 0;
    for (int c = 0; c < b; ++c) {
        int64_t E = m->n[c] + 2 * m->g;
        off += (int64_t)ONF * E * E * E;
    }
    return off;
}

int64_t or_total_size(const or_mesh *m) { return or_block_offset(m, m->nb); }

/* ---------------------------------------------------------------- lookup */

typedef struct {
    int unit;            /* gcd of all block sizes and corners            */
    int nlev;
    int64_t *off;        /* [nb] register offset of each block            */
    int64_t dim[32][3];  /* per level: map extent in units                */
    int32_t *map[32];    /* per level: block id covering the unit, or -1  */
} lookup_t;

static int gcd_i(int a, int b) { a = abs(a); b = abs(b); while (b) { int t = a % b; a = b; b = t; } return a; }

static int lookup_build(const or_mesh *m, lookup_t *L)
{
    memset(L, 0, sizeof(*L));
    int u = 0, lmax = 0;
    for (int b = 0; b < m->nb; ++b) {
        u = gcd_i(u, m->n[b]);
        for (int a = 0; a < 3; ++a) u = gcd_i(u, m->ilo[3 * b + a]);
        if (m->level[b] > lmax) lmax = m->level[b];
    }
    if (u <= 0 || lmax >= 30) return -1;
    L->off = (int64_t *)malloc(sizeof(int64_t) * (m->nb + 1));
    if (!L->off) return -1;
    L->off[0] = 0;
    for (int b = 0; b < m->nb; ++b) {
        int64_t E = m->n[b] + 2 * m->g;
        L->off[b + 1] = L->off[b] + (int64_t)ONF * E * E * E;
    }
    L->unit = u;
    L->nlev = lmax + 1;
    for (int l = 0; l < L->nlev; ++l) {
        int64_t tot = 1;
        for (int a = 0; a < 3; ++a) {
            int64_t N = (int64_t)m->nroot[a] << l;
            if (N % u) return -1;
            L->dim[l][a] = N / u;
            tot *= L->dim[l][a];
        }
        L->map[l] = (int32_t *)malloc(sizeof(int32_t) * tot);
        if (!L->map[l]) return -1;
        for (int64_t q = 0; q < tot; ++q) L->map[l][q] = -1;
    }
    for (int b = 0; b < m->nb; ++b) {
        int l = m->level[b], nu = m->n[b] / u;
        int64_t c0 = m->ilo[3 * b] / u, c1 = m->ilo[3 * b + 1] / u, c2 = m->ilo[3 * b + 2] / u;
        for (int z = 0; z < nu; ++z)
            for (int y = 0; y < nu; ++y)
                for (int x = 0; x < nu; ++x) {
                    int64_t X = c0 + x, Y = c1 + y, Z = c2 + z;
                    if (X < 0 || Y < 0 || Z < 0 || X >= L->dim[l][0] || Y >= L->dim[l][1] ||
                        Z >= L->dim[l][2])
                        return -1;
                    int64_t q = (Z * L->dim[l][1] + Y) * L->dim[l][0] + X;
                    if (L->map[l][q] != -1) return -1; /* overlap */
                    L->map[l][q] = b;
                }
    }
    return 0;
}

static void lookup_free(lookup_t *L)
{
    free(L->off);
    for (int l = 0; l < L->nlev; ++l) free(L->map[l]);
}

/* block of exactly level l containing global cell I (inside the domain) */
static int leaf_at(const lookup_t *L, int l, const int64_t I[3])
{
    if (l < 0 || l >= L->nlev) return -1;
    int64_t q[3];
    for (int a = 0; a < 3; ++a) {
        q[a] = I[a] / L->unit;
        if (I[a] < 0 || q[a] >= L->dim[l][a]) return -1;
    }
    return L->map[l][(q[2] * L->dim[l][1] + q[1]) * L->dim[l][0] + q[0]];
}

/* apply the domain boundary condition to a global index at level l;
 * returns 0 if the index is inside the domain after it */
static void apply_bc(const or_mesh *m, int l, int64_t I[3])
{
    for (int a = 0; a < 3; ++a) {
        int64_t N = (int64_t)m->nroot[a] << l;
        if (m->bc == 0) {
            I[a] %= N;
            if (I[a] < 0) I[a] += N;
        } else {
            if (I[a] < 0) I[a] = 0;
            if (I[a] >= N) I[a] = N - 1;
        }
    }
}

/* Lagrange weights (Eq. 1) of nodes x[0..n-1] at point t */
static void lagrange(int n, const double *x, double t, double *w)
{
    for (int i = 0; i < n; ++i) {
        double p = 1.0;
        for (int q = 0; q < n; ++q)
            if (q != i) p *= (t - x[q]) / (x[i] - x[q]);
        w[i] = p;
    }
}

static void interior_values(const or_mesh *m, const lookup_t *L, const double *u, int b,
                            const int64_t I[3], double out[ONF])
{
    int64_t E = m->n[b] + 2 * m->g;
    int64_t off = L->off[b];
    int64_t i = I[0] - m->ilo[3 * b] + m->g, j = I[1] - m->ilo[3 * b + 1] + m->g,
            k = I[2] - m->ilo[3 * b + 2] + m->g;
    for (int f = 0; f < ONF; ++f) out[f] = u[off + (((int64_t)f * E + k) * E + j) * E + i];
}

/* restriction to coarse cell J (level l) from fine leaf F (level l+1) */
static void restrict_values(const or_mesh *m, const lookup_t *L, const double *u, int F,
                            const int64_t J[3], double out[ONF])
{
    int nr = m->g + 1;
    int64_t lo[3];
    double x[16], w[3][16];
    for (int a = 0; a < 3; ++a) {
        int64_t c = 2 * J[a];           /* fine cells c, c+1; target at c+1 (a face) */
        int64_t s;
        if (nr % 2 == 0) s = c - nr / 2 + 1;
        else {
            /* odd: tie between c-(nr-1)/2 and c+1+(nr-1)/2; take the side of
             * the block interior */
            double mid = m->ilo[3 * F + a] + 0.5 * m->n[F];
            s = ((double)(c + 1) < mid) ? c - (nr - 1) / 2 + 1 : c - (nr - 1) / 2;
        }
        int64_t blo = m->ilo[3 * F + a], bhi = blo + m->n[F] - 1;
        if (s < blo) s = blo;
        if (s + nr - 1 > bhi) s = bhi - nr + 1;
        lo[a] = s;
        for (int q = 0; q < nr; ++q) x[q] = (double)(s + q) + 0.5; /* fine centres, fine units */
        lagrange(nr, x, (double)(c + 1), w[a]);
    }
    for (int f = 0; f < ONF; ++f) out[f] = 0.0;
    double v[ONF];
    for (int kc = 0; kc < nr; ++kc)
        for (int jc = 0; jc < nr; ++jc)
            for (int ic = 0; ic < nr; ++ic) {
                int64_t P[3] = {lo[0] + ic, lo[1] + jc, lo[2] + kc};
                double wt = w[0][ic] * w[1][jc] * w[2][kc];
                interior_values(m, L, u, F, P, v);
                for (int f = 0; f < ONF; ++f) out[f] += wt * v[f];
            }
}

/* memo of composite coarse values, keyed by (level, cell) */
typedef struct {
    int64_t cap, used;
    int64_t *key;
    double *val;
} memo_t;

static uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static int64_t memo_key(int l, const int64_t K[3])
{
    return ((((int64_t)l * 4096 + K[2]) * 65536 + K[1]) * 65536) + K[0];
}

static double *memo_find(memo_t *M, int64_t key, int *found)
{
    if (M->used * 2 >= M->cap) {
        int64_t ncap = M->cap ? 2 * M->cap : 1 << 16;
        int64_t *nk = (int64_t *)malloc(sizeof(int64_t) * ncap);
        double *nv = (double *)malloc(sizeof(double) * ONF * ncap);
        if (!nk || !nv) { free(nk); free(nv); *found = -1; return NULL; }
        for (int64_t q = 0; q < ncap; ++q) nk[q] = -1;
        for (int64_t q = 0; q < M->cap; ++q)
            if (M->key[q] >= 0) {
                uint64_t h = mix64((uint64_t)M->key[q]) % (uint64_t)ncap;
                while (nk[h] >= 0) h = (h + 1) % (uint64_t)ncap;
                nk[h] = M->key[q];
                memcpy(nv + ONF * h, M->val + ONF * q, sizeof(double) * ONF);
            }
        free(M->key); free(M->val);
        M->key = nk; M->val = nv; M->cap = ncap;
    }
    uint64_t h = mix64((uint64_t)key) % (uint64_t)M->cap;
    while (M->key[h] >= 0) {
        if (M->key[h] == key) { *found = 1; return M->val + ONF * h; }
        h = (h + 1) % (uint64_t)M->cap;
    }
    M->key[h] = key;
    M->used++;
    *found = 0;
    return M->val + ONF * h;
}

static int composite_values(const or_mesh *m, const lookup_t *L, const double *u, int l,
                            const int64_t Iin[3], int allow_prolong, memo_t *M, double out[ONF]);

/* prolongation to fine cell I (level l) from coarse data at level l-1 */
static int prolong_values(const or_mesh *m, const lookup_t *L, const double *u, int l,
                          const int64_t I[3], memo_t *M, double out[ONF])
{
    int np = m->g + 1;
    int64_t lo[3];
    double x[16], w[3][16];
    for (int a = 0; a < 3; ++a) {
        int64_t J = I[a] / 2;           /* I is inside the domain, so >= 0 */
        int odd = (int)(I[a] - 2 * J); /* 0: target at -1/4, 1: at +1/4 */
        int64_t s;
        if (np % 2) s = J - (np - 1) / 2;
        else s = odd ? J - np / 2 + 1 : J - np / 2;
        lo[a] = s;
        /* in coarse units, coarse centre q sits at q+1/2, the target at (I+1/2)/2 */
        for (int q = 0; q < np; ++q) x[q] = (double)(s + q) + 0.5;
        lagrange(np, x, 0.5 * ((double)I[a] + 0.5), w[a]);
    }
    for (int f = 0; f < ONF; ++f) out[f] = 0.0;
    for (int kc = 0; kc < np; ++kc)
        for (int jc = 0; jc < np; ++jc)
            for (int ic = 0; ic < np; ++ic) {
                int64_t K[3] = {lo[0] + ic, lo[1] + jc, lo[2] + kc};
                apply_bc(m, l - 1, K);
                int found;
                double *v = memo_find(M, memo_key(l - 1, K), &found);
                if (found < 0) return -2;
                if (!found && composite_values(m, L, u, l - 1, K, 0, M, v)) return -1;
                double wt = w[0][ic] * w[1][jc] * w[2][kc];
                for (int f = 0; f < ONF; ++f) out[f] += wt * v[f];
            }
    return 0;
}

static int composite_values(const or_mesh *m, const lookup_t *L, const double *u, int l,
                            const int64_t Iin[3], int allow_prolong, memo_t *M, double out[ONF])
{
    int64_t I[3] = {Iin[0], Iin[1], Iin[2]};
    apply_bc(m, l, I);
    int b = leaf_at(L, l, I);
    if (b >= 0) { interior_values(m, L, u, b, I, out); return 0; }
    int64_t C[3] = {2 * I[0], 2 * I[1], 2 * I[2]};
    int F = leaf_at(L, l + 1, C);
    if (F >= 0) { restrict_values(m, L, u, F, I, out); return 0; }
    if (!allow_prolong) return -1;
    int64_t P[3] = {I[0] / 2, I[1] / 2, I[2] / 2};
    if (leaf_at(L, l - 1, P) >= 0) return prolong_values(m, L, u, l, I, M, out);
    return -1;
}

int or_fill_ghosts_from(const or_mesh *m, const double *src, double *u, const int8_t *only)
{
    if (m->bc == 2) return 0;
    lookup_t L;
    if (lookup_build(m, &L)) { lookup_free(&L); return -1; }
    int rc = 0;
    int g = m->g;
    memo_t M = {0, 0, NULL, NULL};
    for (int b = 0; b < m->nb && !rc; ++b) {
        if (only && !only[b]) continue;
        int n = m->n[b], l = m->level[b];
        int64_t E = n + 2 * g, off = L.off[b];
        for (int k = 0; k < E && !rc; ++k)
            for (int j = 0; j < E && !rc; ++j)
                for (int i = 0; i < E; ++i) {
                    int ghost = (i < g || i >= g + n || j < g || j >= g + n || k < g || k >= g + n);
                    if (!ghost) continue;
                    int64_t I[3] = {m->ilo[3 * b] + i - g, m->ilo[3 * b + 1] + j - g,
                                    m->ilo[3 * b + 2] + k - g};
                    double v[ONF];
                    if (composite_values(m, &L, src, l, I, 1, &M, v)) { rc = -3; break; }
                    for (int f = 0; f < ONF; ++f) u[off + (((int64_t)f * E + k) * E + j) * E + i] = v[f];
                }
    }
    free(M.key);
    free(M.val);
    lookup_free(&L);
    return rc;
}

int or_fill_ghosts(const or_mesh *m, double *u)
{
    if (m->bc == 2) return 0;
    /* Values are computed from active zones only, so the result does not
     * depend on the order blocks are visited.  Compute from a copy so that
     * no ghost is read while being written. */
    int64_t tot = or_total_size(m);
    double *src = (double *)malloc(sizeof(double) * (tot > 0 ? tot : 1));
    if (!src) return -2;
    memcpy(src, u, sizeof(double) * tot);
    int rc = or_fill_ghosts_from(m, src, u, NULL);
    free(src);
    return rc;
}
