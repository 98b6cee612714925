/*
 * oracle/hier.c -- plain FP64 CPU oracle of the hierarchical method.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the bench's
 * CPU-baseline leg may load this library.  It shares no code, header, table or
 * helper with the GPU library.
 *
 * Fang, Huang, Huber, McCammon, Zhang, "Hierarchical Orthogonal Matrix
 * Generation and Matrix-Vector Multiplications in Rigid Body Simulations".
 * One rigid body with n beads at r_k.  Its Z-matrix (Eq. 1.2) is
 * Z = [I ... I; A_1 ... A_n] with A_k f = r_k x f.  Q~ is a (3n-6) x 3n matrix
 * with orthonormal rows spanning the orthogonal complement of Z's row space.
 * This file computes the paper's particular Q~:
 *
 *   tree      Section 2.1 and its binary-tree comment: nested cubical boxes,
 *             split at midpoints in z, then y, then x, empty halves pruned,
 *             until a box holds at most s beads (a leaf; s = 1 by default).
 *   Q_gen     Algorithm 1 with Eqs. 3.4-3.8: per internal node p with children
 *             x, y the 3 x k matrix K = [R22 | S22 | sqrt(n_x n/n_y) R21] is
 *             factored K = [T22 | 0] G with G orthogonal (a QR of K^T); the
 *             blocks of a leaf child are absent (Cases I and II).
 *   up        Algorithm 2, Eqs. 4.2-4.3 (Info-set M_p and Residue eps_p).
 *   down      Algorithm 3, Theorem 4.3 (Velocity-sets L_x, L_y from L_p).
 *   explicit  Algorithm 1's U and Residue Vectors formed as dense blocks.
 *
 * Readings of points the paper leaves open (all stated again where used):
 *   - root box: lower corner = per-axis minimum of the body's beads, side h =
 *     largest per-axis extent; each coordinate is quantised to 21 bits as
 *     q = min(floor(((x - lo) / h) * 2^21), 2^21 - 1) (q = 0 when h = 0).  The
 *     split bit of a box at a level is the next bit of q; bit 1 = upper half.
 *   - x = lower-half child, y = upper-half child; a box whose beads fall in
 *     one half is replaced by that half (single-child chains collapse).
 *   - beads that share all 63 code bits are split by the highest differing
 *     bit of their body-local sorted position (ties keep user order).  No
 *     passage fixes this split: parity unpinned beyond the basis-free pins
 *     (rows orthonormal and orthogonal to Z, the projector of LAPACK's QR).
 *   - one tree per body, coordinates relative to the body's lower corner.
 *   - QR by Householder reflections in LAPACK's convention:
 *     beta = -sign(alpha) * ||(alpha, x)|| with sign(alpha) = +1 for
 *     alpha >= 0, tau = (beta - alpha) / beta, v = [1; x / (alpha - beta)], and
 *     tau = 0 (identity) when x = 0.  T22 = R(1:3,1:3)^T, G = Q^T.
 *   - Q~ rows follow the block form Q~_p = [Residue_p; diag(Q~_x, Q~_y)]
 *     (Section 3): a node's residue rows, then its x subtree's rows, then its y
 *     subtree's rows (pre-order).
 *   - Q~v drops the root Info-set; Q~^T w starts from a zero root
 *     Velocity-set (Section 4.2).
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared -o liboracle_hier.so hier.c -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define QBITS 21
#define QMAX ((1u << QBITS) - 1u)

typedef struct {
    int64_t first, last;   /* range of sorted bead positions covered */
    int64_t x, y;          /* child: >= 0 internal node id, < 0 leaf -(sorted pos + 1) */
    int64_t n;             /* beads below */
    double c[3];           /* centroid, body-local coordinates */
    double T22[3][3];      /* lower triangular */
    int k;                 /* columns of K: 3 + 3[x internal] + 3[y internal] */
    int dim;               /* residue rows: k - 3 */
    double G[9][9];        /* k x k orthogonal */
    double sx, sy;         /* sqrt(n_x/n), sqrt(n_y/n) */
    int64_t off;           /* first residue row of this node in Q~ */
    double kappa;          /* sigma_1 / sigma_3 of T22 (k > 3 nodes, buckets of 3 or more) */
    int bucket;            /* 1: a leaf box of 2..s beads (no children) */
    double *hv;            /* bucket: the 6 Householder vectors, 3n x 6, column-major */
    double htau[6];        /* bucket: their taus */
} onode;

typedef struct or_body {
    int64_t n;
    int64_t s;             /* leaf size: boxes of at most s beads are leaves */
    double *r;             /* body-local positions, user order, n x 3 */
    uint64_t *code;        /* user order */
    int64_t *perm;         /* sorted position -> user index */
    uint64_t *scode;       /* codes in sorted order */
    int64_t nint;
    onode *nodes;          /* internal node 0 is the root */
} or_body;

/* ------------------------------------------------------------------------ */
/* tree: quantised coordinates and the nested-box bisection (Section 2.1)   */
/* ------------------------------------------------------------------------ */

static uint32_t quantise(double x, double lo, double h)
{
    if (!(h > 0.0)) return 0;
    double t = ((x - lo) / h) * 2097152.0;   /* 2^21 */
    double f = floor(t);
    if (f < 0.0) f = 0.0;
    if (f > (double)QMAX) f = (double)QMAX;
    return (uint32_t)f;
}

/* Bits of one box level, most significant first: z, then y, then x. */
static uint64_t interleave(uint32_t qx, uint32_t qy, uint32_t qz)
{
    uint64_t code = 0;
    for (int l = QBITS - 1; l >= 0; --l) {
        code = (code << 1) | ((qz >> l) & 1u);
        code = (code << 1) | ((qy >> l) & 1u);
        code = (code << 1) | ((qx >> l) & 1u);
    }
    return code;
}

void or_codes(const double *pos, int64_t n, uint64_t *codes)
{
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) { lo[d] = pos[d]; hi[d] = pos[d]; }
    for (int64_t i = 1; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            if (pos[3 * i + d] < lo[d]) lo[d] = pos[3 * i + d];
            if (pos[3 * i + d] > hi[d]) hi[d] = pos[3 * i + d];
        }
    double h = 0.0;
    for (int d = 0; d < 3; ++d)
        if (hi[d] - lo[d] > h) h = hi[d] - lo[d];
    for (int64_t i = 0; i < n; ++i)
        codes[i] = interleave(quantise(pos[3 * i + 0], lo[0], h),
                              quantise(pos[3 * i + 1], lo[1], h),
                              quantise(pos[3 * i + 2], lo[2], h));
}

static const uint64_t *g_sort_codes;

static int cmp_bead(const void *pa, const void *pb)
{
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    uint64_t ca = g_sort_codes[a], cb = g_sort_codes[b];
    if (ca != cb) return ca < cb ? -1 : 1;
    return a < b ? -1 : (a > b ? 1 : 0);
}

static int highest_bit(uint64_t v)
{
    int b = -1;
    while (v) { v >>= 1; ++b; }
    return b;
}

/* Last sorted position of the lower half of the box holding [lo, hi]. */
static int64_t split_of(const or_body *B, int64_t lo, int64_t hi)
{
    uint64_t a = B->scode[lo], z = B->scode[hi];
    if (a == z) {
        /* all 63 bits agree: split by the body-local sorted position */
        int b = highest_bit((uint64_t)(lo ^ hi));
        int64_t upper_start = (hi >> b) << b;
        return upper_start - 1;
    }
    /* the box splits at the first bit where the range's codes differ; bits
       above it are shared (empty halves above it were pruned) */
    int b = highest_bit(a ^ z);
    uint64_t m = 1ull << b;
    int64_t L = lo, H = hi;          /* first position with bit b set */
    while (L < H) {
        int64_t mid = L + (H - L) / 2;
        if (B->scode[mid] & m) H = mid; else L = mid + 1;
    }
    return L - 1;
}

static int64_t build_rec(or_body *B, int64_t lo, int64_t hi)
{
    if (lo == hi) return -(lo + 1);
    int64_t id = B->nint++;
    B->nodes[id].first = lo;
    B->nodes[id].last = hi;
    if (hi - lo + 1 <= B->s) {
        /* a box of 2..s beads is a leaf (a bucket) */
        B->nodes[id].bucket = 1;
        B->nodes[id].x = B->nodes[id].y = -1;
        return id;
    }
    int64_t s = split_of(B, lo, hi);
    int64_t x = build_rec(B, lo, s);
    int64_t y = build_rec(B, s + 1, hi);
    B->nodes[id].x = x;
    B->nodes[id].y = y;
    return id;
}

/* ------------------------------------------------------------------------ */
/* per-node factorisation (Section 3)                                       */
/* ------------------------------------------------------------------------ */

/* [u]x: the matrix of f -> u x f (the A_k of Eq. 1.2). */
static void cross_matrix(const double u[3], double A[3][3])
{
    A[0][0] = 0.0;   A[0][1] = -u[2]; A[0][2] = u[1];
    A[1][0] = u[2];  A[1][1] = 0.0;   A[1][2] = -u[0];
    A[2][0] = -u[1]; A[2][1] = u[0];  A[2][2] = 0.0;
}

/* Householder QR of the k x 3 matrix A (in place) with Q formed explicitly:
   A = Q R, Q k x k orthogonal, R upper triangular in A's top 3 rows. */
static void householder_qr(int k, double A[9][3], double Q[9][9])
{
    double V[3][9];
    double tau[3];
    for (int j = 0; j < 3; ++j) {
        double alpha = A[j][j];
        double xs = 0.0;
        for (int i = j + 1; i < k; ++i) xs += A[i][j] * A[i][j];
        double xnorm = sqrt(xs);
        for (int i = 0; i < 9; ++i) V[j][i] = 0.0;
        V[j][j] = 1.0;
        if (xnorm == 0.0) {
            tau[j] = 0.0;
            continue;
        }
        double nrm = sqrt(alpha * alpha + xnorm * xnorm);
        double beta = (alpha >= 0.0) ? -nrm : nrm;
        tau[j] = (beta - alpha) / beta;
        double scal = 1.0 / (alpha - beta);
        for (int i = j + 1; i < k; ++i) V[j][i] = A[i][j] * scal;
        A[j][j] = beta;
        for (int i = j + 1; i < k; ++i) A[i][j] = 0.0;
        for (int l = j + 1; l < 3; ++l) {
            double w = 0.0;
            for (int i = j; i < k; ++i) w += V[j][i] * A[i][l];
            for (int i = j; i < k; ++i) A[i][l] -= tau[j] * V[j][i] * w;
        }
    }
    /* Q = H_1 H_2 H_3 applied to the identity, rightmost factor first */
    for (int i = 0; i < k; ++i)
        for (int l = 0; l < k; ++l) Q[i][l] = (i == l) ? 1.0 : 0.0;
    for (int j = 2; j >= 0; --j) {
        if (tau[j] == 0.0) continue;
        for (int l = 0; l < k; ++l) {
            double w = 0.0;
            for (int i = 0; i < k; ++i) w += V[j][i] * Q[i][l];
            for (int i = 0; i < k; ++i) Q[i][l] -= tau[j] * V[j][i] * w;
        }
    }
}

/* sigma_1 / sigma_3 of a 3x3 matrix, from the eigenvalues of T^T T (cyclic
   Jacobi).  Used only to flag ill-conditioned nodes. */
static double cond3(double T[3][3])
{
    double S[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int l = 0; l < 3; ++l) s += T[l][i] * T[l][j];
            S[i][j] = s;
        }
    for (int sweep = 0; sweep < 50; ++sweep) {
        double off = fabs(S[0][1]) + fabs(S[0][2]) + fabs(S[1][2]);
        if (off == 0.0) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                if (S[p][q] == 0.0) continue;
                double theta = (S[q][q] - S[p][p]) / (2.0 * S[p][q]);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int l = 0; l < 3; ++l) {
                    double a = S[l][p], b = S[l][q];
                    S[l][p] = c * a - s * b;
                    S[l][q] = s * a + c * b;
                }
                for (int l = 0; l < 3; ++l) {
                    double a = S[p][l], b = S[q][l];
                    S[p][l] = c * a - s * b;
                    S[q][l] = s * a + c * b;
                }
            }
    }
    double e[3] = {S[0][0], S[1][1], S[2][2]};
    double mx = e[0], mn = e[0];
    for (int i = 1; i < 3; ++i) { if (e[i] > mx) mx = e[i]; if (e[i] < mn) mn = e[i]; }
    if (mn <= 0.0) return INFINITY;
    return sqrt(mx / mn);
}

/* A leaf box of n = 2..s beads (Section 2.1 allows leaves of more than one
   bead; the paper leaves their processing open).  Reading: the leaf's Z about
   its centroid c has the translation rows U_t = [I ... I] / sqrt(n) and the
   rotation rows Z_r = [A_1 ... A_n] with A_k = [r_k - c]x, orthogonal to U_t.
   A Householder QR (the convention above) of the 3n x 6 matrix
   X = [U_t^T | Z_r^T] gives X = Q [R; 0] with R(1:3,1:3) = -I (U_t^T has
   orthonormal columns, and each pivot is positive) and R(1:3,4:6) = 0.
   The leaf's orthogonal transform is G = diag(-1,-1,-1,1,...,1) Q^T: its rows
   1-3 are U_t, its rows 4-6 the rotation rows with Z_r = R(4:6,4:6)^T G(4:6,:),
   so T22 = R(4:6,4:6)^T (lower triangular) as for a node, and its rows 7..3n
   are the leaf's 3n - 6 residue rows.  A two-bead leaf has a rank-2 Z_r: its
   T22(3,3) is set to the exact 0 (as Eq. 3.9 for two beads). */
static void gen_bucket(or_body *B, onode *p)
{
    int64_t n = p->last - p->first + 1, m = 3 * n;
    p->n = n;
    for (int d = 0; d < 3; ++d) p->c[d] = 0.0;
    for (int64_t b = 0; b < n; ++b)
        for (int d = 0; d < 3; ++d) p->c[d] += B->r[3 * B->perm[p->first + b] + d];
    for (int d = 0; d < 3; ++d) p->c[d] /= (double)n;
    double *X = (double *)calloc((size_t)(m * 6), sizeof(double));   /* column-major m x 6 */
    double rs = 1.0 / sqrt((double)n);
    for (int64_t b = 0; b < n; ++b) {
        double u[3], A[3][3];
        for (int d = 0; d < 3; ++d) u[d] = B->r[3 * B->perm[p->first + b] + d] - p->c[d];
        cross_matrix(u, A);
        for (int d = 0; d < 3; ++d) {
            X[d * m + 3 * b + d] = rs;                            /* U_t^T */
            for (int e = 0; e < 3; ++e) X[(3 + e) * m + 3 * b + d] = A[e][d];   /* Z_r^T = A_b^T */
        }
    }
    for (int j = 0; j < 6; ++j) {
        double *col = X + j * m;
        double alpha = col[j], xs = 0.0;
        for (int64_t i = j + 1; i < m; ++i) xs += col[i] * col[i];
        double xnorm = sqrt(xs);
        if (xnorm == 0.0 || j >= m - 1) {
            p->htau[j] = 0.0;
            for (int64_t i = j + 1; i < m; ++i) col[i] = 0.0;
            continue;
        }
        const double nrm = sqrt(alpha * alpha + xnorm * xnorm);
        const double beta = (alpha >= 0.0) ? -nrm : nrm;
        p->htau[j] = (beta - alpha) / beta;
        double scal = 1.0 / (alpha - beta);
        for (int64_t i = j + 1; i < m; ++i) col[i] *= scal;   /* v = [1; x / (alpha - beta)] */
        col[j] = beta;
        for (int l = j + 1; l < 6; ++l) {
            double *cl = X + l * m, w = cl[j];
            for (int64_t i = j + 1; i < m; ++i) w += col[i] * cl[i];
            w *= p->htau[j];
            cl[j] -= w;
            for (int64_t i = j + 1; i < m; ++i) cl[i] -= w * col[i];
        }
    }
    /* T22 = R(4:6,4:6)^T */
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) p->T22[i][j] = (j <= i) ? X[(3 + i) * m + 3 + j] : 0.0;
    if (n == 2) p->T22[2][2] = 0.0;
    p->hv = X;
    p->k = 0;
    p->dim = (int)(m - 6);
    p->sx = p->sy = 0.0;
    p->kappa = (n >= 3) ? cond3(p->T22) : 0.0;
}

/* t <- Q^T t = H_6 ... H_1 t for a bucket (t: 3n values) */
static void bucket_qt(const onode *p, double *t)
{
    int64_t m = 3 * p->n;
    for (int j = 0; j < 6; ++j) {
        if (p->htau[j] == 0.0) continue;
        const double *v = p->hv + j * m;
        double w = t[j];
        for (int64_t i = j + 1; i < m; ++i) w += v[i] * t[i];
        w *= p->htau[j];
        t[j] -= w;
        for (int64_t i = j + 1; i < m; ++i) t[i] -= w * v[i];
    }
}

/* t <- Q t = H_1 ... H_6 t */
static void bucket_q(const onode *p, double *t)
{
    int64_t m = 3 * p->n;
    for (int j = 5; j >= 0; --j) {
        if (p->htau[j] == 0.0) continue;
        const double *v = p->hv + j * m;
        double w = t[j];
        for (int64_t i = j + 1; i < m; ++i) w += v[i] * t[i];
        w *= p->htau[j];
        t[j] -= w;
        for (int64_t i = j + 1; i < m; ++i) t[i] -= w * v[i];
    }
}

/* Algorithm 1 (generation part): post-order over the tree. */
static void gen_rec(or_body *B, int64_t id)
{
    onode *p = &B->nodes[id];
    if (p->bucket) {
        gen_bucket(B, p);
        return;
    }
    int64_t nx, ny;
    double cx[3], cy[3];
    int xin = p->x >= 0, yin = p->y >= 0;
    if (xin) {
        gen_rec(B, p->x);
        nx = B->nodes[p->x].n;
        memcpy(cx, B->nodes[p->x].c, sizeof cx);
    } else {
        nx = 1;
        memcpy(cx, &B->r[3 * B->perm[-(p->x + 1)]], sizeof cx);
    }
    if (yin) {
        gen_rec(B, p->y);
        ny = B->nodes[p->y].n;
        memcpy(cy, B->nodes[p->y].c, sizeof cy);
    } else {
        ny = 1;
        memcpy(cy, &B->r[3 * B->perm[-(p->y + 1)]], sizeof cy);
    }
    p = &B->nodes[id];
    double n = (double)(nx + ny);
    p->n = nx + ny;
    /* centroid of p from the children's centroids */
    for (int d = 0; d < 3; ++d) p->c[d] = ((double)nx * cx[d] + (double)ny * cy[d]) / n;
    /* R21 shifts x's moment from c_x to c_p (Eq. 3.4) */
    double dxp[3];
    for (int d = 0; d < 3; ++d) dxp[d] = cx[d] - p->c[d];
    double R21[3][3];
    cross_matrix(dxp, R21);
    double s3 = sqrt((double)nx * n / (double)ny);
    /* K = [R22 | S22 | sqrt(n_x n / n_y) R21] (Eq. 3.5); a leaf child has no
       R22 (or S22) block (Cases I and II) */
    double K[3][9];
    int k = 0;
    if (xin) { for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) K[i][k + j] = B->nodes[p->x].T22[i][j]; k += 3; }
    if (yin) { for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) K[i][k + j] = B->nodes[p->y].T22[i][j]; k += 3; }
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) K[i][k + j] = s3 * R21[i][j];
    k += 3;
    /* QR of K^T: K^T = Q R  =>  K = [R(1:3,:)^T | 0] Q^T, so T22 = R^T, G = Q^T */
    double A[9][3], Q[9][9];
    for (int i = 0; i < k; ++i) for (int j = 0; j < 3; ++j) A[i][j] = K[j][i];
    householder_qr(k, A, Q);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) p->T22[i][j] = (j <= i) ? A[j][i] : 0.0;
    /* Case I (two beads, Eq. 3.9): K has rank 2 and T22's third column is
       zero; the computed R(3,3) is rounding noise of either sign, which would
       otherwise become a pivot one level up, so it is set to its exact 0. */
    if (k == 3) p->T22[2][2] = 0.0;
    memset(p->G, 0, sizeof p->G);
    for (int i = 0; i < k; ++i) for (int j = 0; j < k; ++j) p->G[i][j] = Q[j][i];
    p->k = k;
    p->dim = k - 3;
    p->sx = sqrt((double)nx / n);
    p->sy = sqrt((double)ny / n);
    p->kappa = (k > 3) ? cond3(p->T22) : 0.0;
}

/* Pre-order residue row offsets: Q~_p = [Residue_p; diag(Q~_x, Q~_y)]. */
static int64_t offsets_rec(or_body *B, int64_t id, int64_t off)
{
    onode *p = &B->nodes[id];
    p->off = off;
    off += p->dim;
    if (p->bucket) return off;
    if (p->x >= 0) off = offsets_rec(B, p->x, off);
    if (p->y >= 0) off = offsets_rec(B, p->y, off);
    return off;
}

/* ------------------------------------------------------------------------ */
/* public: build / free / introspection                                     */
/* ------------------------------------------------------------------------ */

void or_free(or_body *B)
{
    if (!B) return;
    for (int64_t i = 0; i < B->nint; ++i) free(B->nodes[i].hv);
    free(B->r); free(B->code); free(B->perm); free(B->scode); free(B->nodes);
    free(B);
}

/* pos: n x 3 FP64 positions of one body in user order; leaves of at most s
   beads (s >= 1).  NULL when n < 2 or s < 1. */
or_body *or_build_s(const double *pos, int64_t n, int64_t s)
{
    if (n < 2 || s < 1) return NULL;
    or_body *B = (or_body *)calloc(1, sizeof *B);
    B->n = n;
    B->s = s;
    B->r = (double *)malloc(sizeof(double) * 3 * n);
    B->code = (uint64_t *)malloc(sizeof(uint64_t) * n);
    B->perm = (int64_t *)malloc(sizeof(int64_t) * n);
    B->scode = (uint64_t *)malloc(sizeof(uint64_t) * n);
    B->nodes = (onode *)calloc((size_t)(n - 1), sizeof(onode));
    or_codes(pos, n, B->code);
    double lo[3] = {pos[0], pos[1], pos[2]};
    for (int64_t i = 1; i < n; ++i)
        for (int d = 0; d < 3; ++d)
            if (pos[3 * i + d] < lo[d]) lo[d] = pos[3 * i + d];
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) B->r[3 * i + d] = pos[3 * i + d] - lo[d];
    for (int64_t i = 0; i < n; ++i) B->perm[i] = i;
    g_sort_codes = B->code;
    qsort(B->perm, (size_t)n, sizeof(int64_t), cmp_bead);
    for (int64_t i = 0; i < n; ++i) B->scode[i] = B->code[B->perm[i]];
    B->nint = 0;
    build_rec(B, 0, n - 1);
    gen_rec(B, 0);
    offsets_rec(B, 0, 0);
    return B;
}

or_body *or_build(const double *pos, int64_t n) { return or_build_s(pos, n, 1); }

int64_t or_n(const or_body *B) { return B->n; }
int64_t or_rows(const or_body *B) { return 3 * B->n - 6; }
int64_t or_num_internal(const or_body *B) { return B->nint; }

void or_perm(const or_body *B, int64_t *perm)
{
    memcpy(perm, B->perm, sizeof(int64_t) * B->n);
}

/* The tree as sorted-position ranges: for internal node id, its range
   [first, last] and the last sorted position of its x child (x covers
   [first, split], y covers [split + 1, last]).  A binary tree over sorted
   positions is fixed by these triples. */
void or_tree(const or_body *B, int64_t *first, int64_t *last, int64_t *split)
{
    for (int64_t i = 0; i < B->nint; ++i) {
        const onode *p = &B->nodes[i];
        first[i] = p->first;
        last[i] = p->last;
        split[i] = p->bucket ? -1 : ((p->x >= 0) ? B->nodes[p->x].last : -(p->x + 1));
    }
}

double or_max_kappa(const or_body *B)
{
    double m = 0.0;
    for (int64_t i = 0; i < B->nint; ++i)
        if (B->nodes[i].kappa > m) m = B->nodes[i].kappa;
    return m;
}

/* Per-node record for tests: ints = {first, last, x, y, n, k, dim, off, bucket},
   dbl = {c[3], T22[9] row-major, sx, sy, kappa, G[81] row-major (k x k in the
   top-left corner)} = 96 doubles. */
void or_node(const or_body *B, int64_t id, int64_t *ints, double *dbl)
{
    const onode *p = &B->nodes[id];
    ints[0] = p->first; ints[1] = p->last; ints[2] = p->x; ints[3] = p->y;
    ints[4] = p->n; ints[5] = p->k; ints[6] = p->dim; ints[7] = p->off; ints[8] = p->bucket;
    for (int d = 0; d < 3; ++d) dbl[d] = p->c[d];
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) dbl[3 + 3 * i + j] = p->T22[i][j];
    dbl[12] = p->sx; dbl[13] = p->sy; dbl[14] = p->kappa;
    for (int i = 0; i < 9; ++i) for (int j = 0; j < 9; ++j) dbl[15 + 9 * i + j] = p->G[i][j];
}

/* ------------------------------------------------------------------------ */
/* Algorithm 2: upward pass, Q v (Eqs. 4.2-4.3)                             */
/* ------------------------------------------------------------------------ */

/* Info-set of node id into M[6]; residues into out (one RHS, stride 1). */
static void up_rec(const or_body *B, int64_t id, const double *v, double *out,
                   double *Mall, double M[6])
{
    const onode *p = &B->nodes[id];
    if (p->bucket) {
        /* [M; eps] = G f with G = diag(-1,-1,-1,1,...) Q^T over the leaf's beads */
        int64_t m = 3 * p->n;
        double *t = (double *)malloc(sizeof(double) * (size_t)m);
        for (int64_t b = 0; b < p->n; ++b)
            for (int d = 0; d < 3; ++d) t[3 * b + d] = v[3 * B->perm[p->first + b] + d];
        bucket_qt(p, t);
        for (int d = 0; d < 3; ++d) { M[d] = -t[d]; M[3 + d] = t[3 + d]; }
        for (int64_t i = 0; i < p->dim; ++i) out[p->off + i] = t[6 + i];
        free(t);
        if (Mall) for (int d = 0; d < 6; ++d) Mall[6 * id + d] = M[d];
        return;
    }
    double Mx[6] = {0}, My[6] = {0};
    if (p->x >= 0) up_rec(B, p->x, v, out, Mall, Mx);
    else { int64_t u = B->perm[-(p->x + 1)]; for (int d = 0; d < 3; ++d) Mx[d] = v[3 * u + d]; }
    if (p->y >= 0) up_rec(B, p->y, v, out, Mall, My);
    else { int64_t u = B->perm[-(p->y + 1)]; for (int d = 0; d < 3; ++d) My[d] = v[3 * u + d]; }
    /* t = [M_x(4:6); M_y(4:6); sqrt(n_y/n) M_x(1:3) - sqrt(n_x/n) M_y(1:3)],
       leaf children contribute no (4:6) part */
    double t[9];
    int k = 0;
    if (p->x >= 0) { for (int d = 0; d < 3; ++d) t[k + d] = Mx[3 + d]; k += 3; }
    if (p->y >= 0) { for (int d = 0; d < 3; ++d) t[k + d] = My[3 + d]; k += 3; }
    for (int d = 0; d < 3; ++d) t[k + d] = p->sy * Mx[d] - p->sx * My[d];
    k += 3;
    for (int d = 0; d < 3; ++d) M[d] = p->sx * Mx[d] + p->sy * My[d];
    double u[9];
    for (int i = 0; i < k; ++i) {
        double s = 0.0;
        for (int j = 0; j < k; ++j) s += p->G[i][j] * t[j];
        u[i] = s;
    }
    for (int d = 0; d < 3; ++d) M[3 + d] = u[d];
    for (int i = 0; i < p->dim; ++i) out[p->off + i] = u[3 + i];
    if (Mall) for (int d = 0; d < 6; ++d) Mall[6 * id + d] = M[d];
}

/* ------------------------------------------------------------------------ */
/* Algorithm 3: downward pass, Q^T w (Theorem 4.3, Eqs. 4.6-4.7)             */
/* ------------------------------------------------------------------------ */

static void down_rec(const or_body *B, int64_t id, const double L[6], const double *w, double *out)
{
    const onode *p = &B->nodes[id];
    if (p->bucket) {
        /* f = G^T [L; w_p] = Q diag(-1,-1,-1,1,...) [L; w_p] */
        int64_t m = 3 * p->n;
        double *t = (double *)malloc(sizeof(double) * (size_t)m);
        for (int d = 0; d < 3; ++d) { t[d] = -L[d]; t[3 + d] = L[3 + d]; }
        for (int64_t i = 0; i < p->dim; ++i) t[6 + i] = w[p->off + i];
        bucket_q(p, t);
        for (int64_t b = 0; b < p->n; ++b)
            for (int d = 0; d < 3; ++d) out[3 * B->perm[p->first + b] + d] = t[3 * b + d];
        free(t);
        return;
    }
    int k = p->k;
    double in[9], s[9];
    for (int d = 0; d < 3; ++d) in[d] = L[3 + d];
    for (int i = 0; i < p->dim; ++i) in[3 + i] = w[p->off + i];
    /* s = G^T [L_p(4:6); w_p]; block j of s is sum_i Q_ji (.)_i in the
       paper's Q_ij notation, whose G block (i,j) is Q_ij^T */
    for (int i = 0; i < k; ++i) {
        double acc = 0.0;
        for (int j = 0; j < k; ++j) acc += p->G[j][i] * in[j];
        s[i] = acc;
    }
    double Lx[6] = {0}, Ly[6] = {0};
    int q = 0;
    if (p->x >= 0) { for (int d = 0; d < 3; ++d) Lx[3 + d] = s[q + d]; q += 3; }
    if (p->y >= 0) { for (int d = 0; d < 3; ++d) Ly[3 + d] = s[q + d]; q += 3; }
    for (int d = 0; d < 3; ++d) {
        Lx[d] = p->sx * L[d] + p->sy * s[q + d];
        Ly[d] = p->sy * L[d] - p->sx * s[q + d];
    }
    if (p->x >= 0) down_rec(B, p->x, Lx, w, out);
    else { int64_t u = B->perm[-(p->x + 1)]; for (int d = 0; d < 3; ++d) out[3 * u + d] = Lx[d]; }
    if (p->y >= 0) down_rec(B, p->y, Ly, w, out);
    else { int64_t u = B->perm[-(p->y + 1)]; for (int d = 0; d < 3; ++d) out[3 * u + d] = Ly[d]; }
}

/* v, out: row-major (rows x nrhs).  transpose = 0: v (3n x nrhs) -> out
   ((3n-6) x nrhs) = Q~ v.  transpose = 1: v ((3n-6) x nrhs) -> out (3n x nrhs)
   = Q~^T v.  With root != NULL (6 x nrhs) the full Q = [Q_Z; Q~] is applied:
   transpose = 0 also returns the root Info-set Q_Z v, transpose = 1 uses it as
   the root Velocity-set. */
void or_apply_full(const or_body *B, const double *v, double *out, int transpose,
                   int64_t nrhs, double *root)
{
    int64_t n3 = 3 * B->n, rows = 3 * B->n - 6;
    double *vi = (double *)malloc(sizeof(double) * (size_t)n3);
    double *oi = (double *)malloc(sizeof(double) * (size_t)n3);
    for (int64_t r = 0; r < nrhs; ++r) {
        if (!transpose) {
            for (int64_t i = 0; i < n3; ++i) vi[i] = v[i * nrhs + r];
            double M[6];
            up_rec(B, 0, vi, oi, NULL, M);
            for (int64_t i = 0; i < rows; ++i) out[i * nrhs + r] = oi[i];
            if (root) for (int d = 0; d < 6; ++d) root[d * nrhs + r] = M[d];
        } else {
            for (int64_t i = 0; i < rows; ++i) vi[i] = v[i * nrhs + r];
            double L[6] = {0, 0, 0, 0, 0, 0};
            if (root) for (int d = 0; d < 6; ++d) L[d] = root[d * nrhs + r];
            down_rec(B, 0, L, vi, oi);
            for (int64_t i = 0; i < n3; ++i) out[i * nrhs + r] = oi[i];
        }
    }
    free(vi);
    free(oi);
}

void or_apply(const or_body *B, const double *v, double *out, int transpose, int64_t nrhs)
{
    or_apply_full(B, v, out, transpose, nrhs, NULL);
}

/* Upward pass for one RHS that also records every internal node's Info-set
   (Mall: nint x 6). */
void or_up_infosets(const or_body *B, const double *v, double *out, double *Mall)
{
    double M[6];
    up_rec(B, 0, v, out, Mall, M);
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1: explicit rows (Eqs. 3.6-3.8 with the leaf cases)            */
/* ------------------------------------------------------------------------ */

/* U (3 x 3n_p, columns over p's sorted beads) of node id; residue rows are
   written into Qs ((3n-6) x 3n, sorted column order). */
static void expl_rec(const or_body *B, int64_t id, double *U, double *Qs)
{
    const onode *p = &B->nodes[id];
    int64_t np = p->n, ncol = 3 * np;
    if (p->bucket) {
        /* rows of G = diag(-1,-1,-1,1,...) Q^T: column c is Q^T e_c; rows
           4-6 are U, rows 7.. the residue rows */
        int64_t ncolQ = 3 * B->n;
        double *t = (double *)malloc(sizeof(double) * (size_t)ncol);
        for (int64_t c = 0; c < ncol; ++c) {
            for (int64_t i = 0; i < ncol; ++i) t[i] = (i == c) ? 1.0 : 0.0;
            bucket_qt(p, t);
            for (int i = 0; i < 3; ++i) U[i * ncol + c] = t[3 + i];
            for (int64_t i = 0; i < p->dim; ++i) Qs[(p->off + i) * ncolQ + 3 * p->first + c] = t[6 + i];
        }
        free(t);
        return;
    }
    int64_t nx = (p->x >= 0) ? B->nodes[p->x].n : 1;
    int64_t ny = np - nx;
    int k = p->k;
    double *J = (double *)calloc((size_t)(k * ncol), sizeof(double));
    int q = 0;
    if (p->x >= 0) {
        double *Ux = (double *)malloc(sizeof(double) * 3 * 3 * nx);
        expl_rec(B, p->x, Ux, Qs);
        for (int i = 0; i < 3; ++i)
            for (int64_t c = 0; c < 3 * nx; ++c) J[(q + i) * ncol + c] = Ux[i * 3 * nx + c];
        free(Ux);
        q += 3;
    }
    if (p->y >= 0) {
        double *Uy = (double *)malloc(sizeof(double) * 3 * 3 * ny);
        expl_rec(B, p->y, Uy, Qs);
        for (int i = 0; i < 3; ++i)
            for (int64_t c = 0; c < 3 * ny; ++c) J[(q + i) * ncol + 3 * nx + c] = Uy[i * 3 * ny + c];
        free(Uy);
        q += 3;
    }
    /* last block row: [sqrt(n_y/n) I_{n_x}, -sqrt(n_x/n) I_{n_y}] with
       I_m = m^{-1/2} [I ... I] (Theorem 3.2) */
    for (int64_t b = 0; b < nx; ++b)
        for (int d = 0; d < 3; ++d) J[(q + d) * ncol + 3 * b + d] = p->sy / sqrt((double)nx);
    for (int64_t b = 0; b < ny; ++b)
        for (int d = 0; d < 3; ++d) J[(q + d) * ncol + 3 * (nx + b) + d] = -p->sx / sqrt((double)ny);
    /* [U; Residue] = G J (Eqs. 3.7-3.8) */
    int64_t ncolQ = 3 * B->n;
    for (int i = 0; i < k; ++i)
        for (int64_t c = 0; c < ncol; ++c) {
            double s = 0.0;
            for (int j = 0; j < k; ++j) s += p->G[i][j] * J[j * ncol + c];
            if (i < 3) U[i * ncol + c] = s;
            else Qs[(p->off + i - 3) * ncolQ + 3 * p->first + c] = s;
        }
    free(J);
}

/* Dense Q~ ((3n-6) x 3n, row-major, user column order).  With Uroot != NULL
   (3 x 3n, user column order) also returns the root's U, so that
   Q_Z = [I_n; U_root] completes the full orthogonal Q. */
void or_explicit_full(const or_body *B, double *Q, double *Uroot)
{
    int64_t n = B->n, rows = 3 * n - 6, ncol = 3 * n;
    double *Qs = (double *)calloc((size_t)((rows > 0 ? rows : 0) * ncol + 1), sizeof(double));
    double *U = (double *)malloc(sizeof(double) * 3 * ncol);
    expl_rec(B, 0, U, Qs);
    for (int64_t i = 0; i < rows; ++i)
        for (int64_t s = 0; s < n; ++s)
            for (int d = 0; d < 3; ++d)
                Q[i * ncol + 3 * B->perm[s] + d] = Qs[i * ncol + 3 * s + d];
    if (Uroot)
        for (int i = 0; i < 3; ++i)
            for (int64_t s = 0; s < n; ++s)
                for (int d = 0; d < 3; ++d)
                    Uroot[i * ncol + 3 * B->perm[s] + d] = U[i * ncol + 3 * s + d];
    free(Qs);
    free(U);
}

void or_explicit(const or_body *B, double *Q)
{
    or_explicit_full(B, Q, NULL);
}
