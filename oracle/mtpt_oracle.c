/*
 * mtpt_oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * A plain, slow, obviously correct FP64 CPU implementation of one time step of
 * mass-transfer particle tracking (MTPT), following Schauer et al.,
 * "Parallelized domain decomposition for mass transfer particle tracking
 * simulations" (arXiv 2204.03756), Sec. 3.  It exists only to check the HIP
 * path: only the tests, the smoke check and the benchmark's CPU-baseline leg
 * load it.  It shares no source, header, table or helper with the HIP path.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (see build.py).
 * Contraction is off so that every "+", "-", "*" below is one IEEE operation.
 *
 * Layouts (all in original particle order, "pid" = index):
 *   positions  x[n][dim]   double (row-major)
 *   masses     m[S][n]     double (species-major)
 *   neighbours CSR row_ptr[n+1], col[nnz] int64, each row sorted ascending,
 *              the particle itself included.
 *
 * Functions and the passage each follows:
 *   or_philox4x32_10     Philox4x32-10 (Salmon et al., SC'11); the paper only
 *                        asks for standard-normal jumps (Sec. 3).
 *   or_log, or_sincos_2pi, or_normals
 *                        Box-Muller from two Philox uniforms, with log, sin and
 *                        cos evaluated from their series (no libm), so that any
 *                        other implementation of the same recipe can agree bit
 *                        for bit.
 *   or_metric_make, or_pair_dist2
 *                        the dispersion tensor of Sec. 2 in the kernel of Sec. 3,
 *                        Eq. (2): Cholesky factor for the jumps, Mahalanobis
 *                        distance and ellipsoidal cutoff (the identity tensor is
 *                        the isotropic method, bit for bit).
 *   or_rw_step           Sec. 3: random-walk update X += v dt + xi*sqrt(2 D_RW dt)
 *                        (xi replaced by L xi with a tensor) and zero-flux walls
 *                        as elastic reflection.
 *   or_neighbors         Sec. 3: neighbours within the search radius psi,
 *                        Eq. (1); K-D tree range search (Bentley) or brute force.
 *   or_mt_weights        Sec. 3: Gaussian kernel Eq. (2)/(3) without its
 *                        prefactor (it cancels), and the symmetric normalisation
 *                        W_ij = K_ij / (0.5 (sum_k K_ik + sum_k K_kj)).
 *   or_mt_step           Sec. 3, Eq. (4) and Eq. (5): M_i += sum_j beta (M_j - M_i) W_ij.
 *   or_react             A+B->C mass-based reaction; not in the paper (named there
 *                        as future work in Sec. 8): parity unpinned against the
 *                        paper, pinned only by invariants and a closed form.
 *   or_total             Neumaier-compensated FP64 sum of a mass array.
 *   or_run               the whole step loop.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, "Parallel random   */
/* numbers: as easy as 1, 2, 3").  Round function: two 32x32->64       */
/* multiplies by fixed multipliers, the high halves xored with the     */
/* other two words and the round key, words permuted; the key is       */
/* bumped by the Weyl constants between rounds.                         */
/* ------------------------------------------------------------------ */
void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform in (0,1) from 52 random bits: u = (2k+1) 2^-53, exact in FP64,
 * never 0 or 1.  k = high word (32 bits) then the top 20 bits of the low word. */
double or_uniform52(uint32_t lo_word, uint32_t hi_word)
{
    uint64_t k = ((uint64_t)hi_word << 20) | (uint64_t)(lo_word >> 12);
    return (double)(2u * k + 1u) * 0x1p-53;
}

/* Natural log of u in (0,1), from u = m 2^e with m in [sqrt(1/2), sqrt(2)]:
 *   log m = 2 atanh(s) = 2 (s + s^3/3 + s^5/5 + ...),  s = (m-1)/(m+1),
 * |s| <= 0.1716, truncated after s^23 (remainder < 1e-19 relative);
 *   log u = e ln2 + log m, with ln2 split into a 42-bit head (exact products)
 * and a tail.  Every multiply-add is one fused multiply-add (fma, rounded
 * once), every other operation is rounded on its own. */
static const double OR_LN2_HI = 0.6931471805598903;      /* 0x1.62e42fefa38p-1 */
static const double OR_LN2_LO = 5.497923018708371e-14;   /* ln2 - OR_LN2_HI   */
static const double OR_SQRT2 = 1.4142135623730951;

double or_log(double u)
{
    uint64_t bits;
    memcpy(&bits, &u, sizeof bits);
    int e = (int)((bits >> 52) & 0x7ffu) - 1023;
    uint64_t mbits = (bits & 0x000fffffffffffffull) | 0x3ff0000000000000ull;
    double m;
    memcpy(&m, &mbits, sizeof m);
    if (m > OR_SQRT2) {
        m = m * 0.5;
        e = e + 1;
    }
    double f = m - 1.0;
    double s = f / (2.0 + f);
    double z = s * s;
    /* Horner: t = 1/3 + z (1/5 + z (1/7 + ... + z (1/23))) */
    double t = 1.0 / 23.0;
    for (int k = 10; k >= 1; --k)
        t = fma(z, t, 1.0 / (double)(2 * k + 1));
    double ts = s + s;
    double lm = fma(ts, z * t, ts);
    double ed = (double)e;
    double r = fma(ed, OR_LN2_LO, lm);
    return fma(ed, OR_LN2_HI, r);
}

/* sin and cos of 2 pi u for u in (0,1).  4u = q + f (exact), q the quadrant;
 * the angle inside the quadrant is f pi/2, folded to y in [0, pi/4] by
 * sin(pi/2 - y) = cos y.  On [0, pi/4] the Taylor series through y^19 and
 * y^18, in z = y^2 by Horner with fused multiply-adds:
 *   sin y = y (1 - z/3! + z^2/5! - ... - z^9/19!),
 *   cos y =    1 - z/2! + z^2/4! - ... - z^9/18!.
 * The coefficients are +-1/n!, each n! exact in FP64 and divided once. */
static const double OR_HALF_PI = 1.5707963267948966;

static double or_inv_fact(int n)
{
    double f = 1.0;
    for (int k = 2; k <= n; ++k)
        f = f * (double)k;   /* exact up to 22! */
    return 1.0 / f;
}

void or_sincos_2pi(double u, double* s_out, double* c_out)
{
    double v = 4.0 * u;
    int q = (int)v;
    double f = v - (double)q;
    double y;
    int swap;
    if (f <= 0.5) {
        y = f * OR_HALF_PI;
        swap = 0;
    } else {
        y = (1.0 - f) * OR_HALF_PI;
        swap = 1;
    }
    double z = y * y;
    /* k = 9 down to 1: coefficient of z^k is (-1)^k / (2k+1)! (sin), (-1)^k / (2k)! (cos) */
    double ts = -or_inv_fact(19), tc = -or_inv_fact(18);
    for (int k = 8; k >= 1; --k) {
        double sg = (k & 1) ? -1.0 : 1.0;
        ts = fma(z, ts, sg * or_inv_fact(2 * k + 1));
        tc = fma(z, tc, sg * or_inv_fact(2 * k));
    }
    ts = fma(z, ts, 1.0);
    tc = fma(z, tc, 1.0);
    double sy = y * ts, cy = tc;
    double sp = swap ? cy : sy; /* sin of the in-quadrant angle */
    double cp = swap ? sy : cy; /* cos of the in-quadrant angle */
    double s, c;
    switch (q & 3) {
    case 0: s = sp;  c = cp;  break;
    case 1: s = cp;  c = -sp; break;
    case 2: s = -sp; c = -cp; break;
    default: s = -cp; c = sp; break;
    }
    *s_out = s;
    *c_out = c;
}

/* Two standard normals by Box-Muller from one Philox call.
 * key = (seed low word, seed high word); counter = (pid, call, step low word,
 * step high word).  u1 from words 0,1 and u2 from words 2,3;
 * z0 = sqrt(-2 log u1) cos(2 pi u2), z1 = sqrt(-2 log u1) sin(2 pi u2). */
void or_normal_pair(uint64_t seed, int64_t step, uint32_t pid, uint32_t call, double z[2])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {pid, call, (uint32_t)(uint64_t)step, (uint32_t)((uint64_t)step >> 32)};
    uint32_t w[4];
    or_philox4x32_10(ctr, key, w);
    double u1 = or_uniform52(w[0], w[1]);
    double u2 = or_uniform52(w[2], w[3]);
    double r = sqrt(-2.0 * or_log(u1));
    double sn, cs;
    or_sincos_2pi(u2, &sn, &cs);
    z[0] = r * cs;
    z[1] = r * sn;
}

/* The d standard-normal components of particle pid's jump at a step: call 0
 * gives dimensions 0 and 1, call 1 gives dimension 2 (its z0). */
void or_normals(uint64_t seed, int64_t step, int dim, int64_t n, double* xi /* [n][dim] */)
{
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; ++p) {
        double z[2];
        or_normal_pair(seed, step, (uint32_t)p, 0u, z);
        xi[p * dim + 0] = z[0];
        xi[p * dim + 1] = z[1];
        if (dim == 3) {
            or_normal_pair(seed, step, (uint32_t)p, 1u, z);
            xi[p * dim + 2] = z[0];
        }
    }
}

/* ------------------------------------------------------------------ */
/* Dispersion tensor.  The advection-dispersion equation of Sec. 2      */
/* carries a dispersion tensor D; the paper's runs take D = D I, and    */
/* the kernel of Sec. 3, Eq. (2), is written with the tensor D_MT.      */
/* Here both parts share one symmetric positive-definite shape tensor   */
/* T: D_RW = d_rw T and D_MT = d_mt T (T = I: the isotropic method).    */
/* With T = L L^T (Cholesky, L lower triangular) and M = L^-1:          */
/*   walk      X += v dt + sqrt(2 d_rw dt) L xi   (covariance 2 dt D_RW) */
/*   kernel    K_ij = exp(-beta q_ij / (4 d_mt dt)),                    */
/*             q_ij = dx^T T^-1 dx = |M dx|^2   (Mahalanobis distance)   */
/*   cutoff    q_ij <= psi^2 (an ellipsoid; psi as in Eq. (1)).          */
/* Eq. (2) prints D_MT in the exponent where its inverse belongs: only   */
/* D_MT^-1 makes the exponent dimensionless and matches the prefactor's  */
/* det(D_MT), the normal density of covariance (2 dt / beta) D_MT.      */
/* Every value below is formed in one fixed order, each operation       */
/* rounded once (contraction is off):                                    */
/*   L00 = sqrt(T00), L10 = T10 / L00, L11 = sqrt(T11 - L10*L10),        */
/*   L20 = T20 / L00, L21 = (T21 - L20*L10) / L11,                       */
/*   L22 = sqrt((T22 - L20*L20) - L21*L21);                              */
/*   M00 = 1/L00, M11 = 1/L11, M22 = 1/L22 (forward substitution of      */
/*   L M = I): M10 = -((L10*M00)*M11), M21 = -((L21*M11)*M22),           */
/*   M20 = -(((L20*M00) + (L21*M10))*M22);                               */
/*   u = L xi: u0 = L00*z0, u1 = L10*z0 + L11*z1,                        */
/*   u2 = (L20*z0 + L21*z1) + L22*z2;                                    */
/*   y = M dx likewise, q = (y0*y0 + y1*y1) + y2*y2.                     */
/* With T = I these reduce bit for bit to the isotropic forms (products  */
/* by 1 are exact, products by 0 add a signed zero), so T = I is the     */
/* isotropic method.                                                      */
/* ------------------------------------------------------------------ */
typedef struct {
    int tensor;        /* 0: Euclidean r2 and scalar jumps; 1: the tensor forms above */
    double l[6];       /* L00, L10, L11, L20, L21, L22 */
    double mi[6];      /* M00, M10, M11, M20, M21, M22 */
    double reach[3];   /* K-D tree pruning factor per axis (see or_query) */
} or_metric;

/* T: NULL (isotropic) or a symmetric [3][3] row-major tensor whose leading
 * dim x dim block is used.  Returns 0, or -1 when T is not symmetric
 * positive definite. */
static int or_metric_make(int dim, const double* T, or_metric* g)
{
    memset(g, 0, sizeof *g);
    g->reach[0] = g->reach[1] = g->reach[2] = 1.0;
    if (!T)
        return 0;
    for (int r = 0; r < dim; ++r)
        for (int c = 0; c < dim; ++c)
            if (!isfinite(T[r * 3 + c]) || T[r * 3 + c] != T[c * 3 + r])
                return -1;
    g->tensor = 1;
    double* l = g->l;
    double* m = g->mi;
    if (!(T[0] > 0.0))
        return -1;
    l[0] = sqrt(T[0]);
    l[1] = T[3] / l[0];
    double p1 = T[4] - l[1] * l[1];
    if (!(p1 > 0.0))
        return -1;
    l[2] = sqrt(p1);
    m[0] = 1.0 / l[0];
    m[2] = 1.0 / l[2];
    m[1] = -((l[1] * m[0]) * m[2]);
    if (dim == 3) {
        l[3] = T[6] / l[0];
        l[4] = (T[7] - l[3] * l[1]) / l[2];
        double p2 = (T[8] - l[3] * l[3]) - l[4] * l[4];
        if (!(p2 > 0.0))
            return -1;
        l[5] = sqrt(p2);
        m[5] = 1.0 / l[5];
        m[4] = -((l[4] * m[2]) * m[5]);
        m[3] = -(((l[3] * m[0]) + (l[4] * m[1])) * m[5]);
    }
    /* the ellipsoid q <= psi2 reaches |dx_a| <= psi sqrt(T_aa) along axis a */
    for (int a = 0; a < dim; ++a)
        g->reach[a] = T[a * 3 + a] * (1.0 + 1e-6);
    return 0;
}

/* Squared distance, one fixed operation order for every caller:
 * ((dx0*dx0) + (dx1*dx1)) + (dx2*dx2), dx = x_j - x_i; with a tensor the
 * Mahalanobis form |M dx|^2 in the order stated above. */
static double or_r2(int dim, const double* xi, const double* xj)
{
    double d0 = xj[0] - xi[0];
    double d1 = xj[1] - xi[1];
    double r2 = d0 * d0 + d1 * d1;
    if (dim == 3) {
        double d2 = xj[2] - xi[2];
        r2 = r2 + d2 * d2;
    }
    return r2;
}

static double or_dist2(const or_metric* g, int dim, const double* xi, const double* xj)
{
    if (!g->tensor)
        return or_r2(dim, xi, xj);
    const double* m = g->mi;
    double d0 = xj[0] - xi[0];
    double d1 = xj[1] - xi[1];
    double y0 = m[0] * d0;
    double y1 = m[1] * d0 + m[2] * d1;
    double q = y0 * y0 + y1 * y1;
    if (dim == 3) {
        double d2 = xj[2] - xi[2];
        double y2 = (m[3] * d0 + m[4] * d1) + m[5] * d2;
        q = q + y2 * y2;
    }
    return q;
}

/* exported for the tests: q of one pair under tensor T (NULL: isotropic) */
double or_pair_dist2(int dim, const double* T, const double* xi, const double* xj)
{
    or_metric g;
    if (or_metric_make(dim, T, &g) != 0)
        return -1.0;
    return or_dist2(&g, dim, xi, xj);
}

/* ------------------------------------------------------------------ */
/* Sec. 3: random walk X_i(t+dt) = X_i(t) + xi_i sqrt(2 D_RW dt), then  */
/* zero-flux walls as elastic reflection: a coordinate that left the    */
/* box is mirrored about the wall it crossed, repeatedly until inside.  */
/* With a drift velocity v (the advective term of the ADE, Sec. 2 and   */
/* Sec. 8) the displacement is v dt + xi sqrt(2 D_RW dt):               */
/* jump_k = z_k * sdev + vel_k * dt, each product and the sum rounded;  */
/* with a dispersion tensor z_k is replaced by u_k = (L z)_k.           */
/* fp32 != 0: the position state is FP32 (inputs already rounded); the  */
/* jump is formed in FP64 and rounded once, the add and the reflection  */
/* are done in float.                                                    */
/* ------------------------------------------------------------------ */
void or_rw_step(int dim, int64_t n, const double lo[3], const double hi[3], double d_rw,
                const double vel[3], double dt, uint64_t seed, int64_t step, int fp32,
                const double* tens, double* x /* [n][dim] */)
{
    or_metric g;
    if (or_metric_make(dim, tens, &g) != 0)
        return;
    double sdev = sqrt(2.0 * d_rw * dt);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; ++p) {
        double z[3], zz[2];
        or_normal_pair(seed, step, (uint32_t)p, 0u, zz);
        z[0] = zz[0];
        z[1] = zz[1];
        z[2] = 0.0;
        if (dim == 3) {
            or_normal_pair(seed, step, (uint32_t)p, 1u, zz);
            z[2] = zz[0];
        }
        if (g.tensor) {
            const double* l = g.l;
            double u0 = l[0] * z[0];
            double u1 = l[1] * z[0] + l[2] * z[1];
            double u2 = dim == 3 ? (l[3] * z[0] + l[4] * z[1]) + l[5] * z[2] : 0.0;
            z[0] = u0;
            z[1] = u1;
            z[2] = u2;
        }
        for (int k = 0; k < dim; ++k) {
            double jump = z[k] * sdev + vel[k] * dt;
            if (fp32) {
                float xf = (float)x[p * dim + k];
                float jf = (float)jump;
                float lf = (float)lo[k], hf = (float)hi[k];
                xf = xf + jf;
                while (xf < lf || xf > hf)
                    xf = (xf < lf) ? 2.0f * lf - xf : 2.0f * hf - xf;
                x[p * dim + k] = (double)xf;
            } else {
                double xd = x[p * dim + k] + jump;
                while (xd < lo[k] || xd > hi[k])
                    xd = (xd < lo[k]) ? 2.0 * lo[k] - xd : 2.0 * hi[k] - xd;
                x[p * dim + k] = xd;
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* K-D tree (Bentley 1975), as used by the paper for the range search   */
/* within psi (Sec. 3).  Median split cycling through the dimensions,   */
/* leaves of at most OR_LEAF points.                                     */
/* ------------------------------------------------------------------ */
#define OR_LEAF 12
#define OR_TASK_MIN 65536   /* subtrees at least this large are built as OpenMP tasks */

typedef struct {
    int dim;
    const double* x;
    int64_t* idx;    /* permutation of 0..n-1, reordered by the build */
    double* split;   /* splitting value per inner node, heap-numbered (root 1) */
} or_tree;

static double or_coord(const or_tree* t, int64_t k, int ax) { return t->x[t->idx[k] * t->dim + ax]; }

static void or_swap(int64_t* a, int64_t* b)
{
    int64_t tmp = *a;
    *a = *b;
    *b = tmp;
}

/* Quickselect: reorder idx[lo..hi) so that position k holds the element of
 * rank k-lo along axis ax, smaller-or-equal ones before it and
 * greater-or-equal ones after it. */
static void or_select(or_tree* t, int64_t lo, int64_t hi, int64_t k, int ax)
{
    while (hi - lo > 1) {
        int64_t mid = lo + (hi - lo) / 2;
        /* median of three as pivot */
        double a = or_coord(t, lo, ax), b = or_coord(t, mid, ax), c = or_coord(t, hi - 1, ax);
        int64_t piv = (a < b) ? ((b < c) ? mid : ((a < c) ? hi - 1 : lo))
                              : ((a < c) ? lo : ((b < c) ? hi - 1 : mid));
        double pv = or_coord(t, piv, ax);
        or_swap(&t->idx[piv], &t->idx[hi - 1]);
        int64_t store = lo;
        for (int64_t i = lo; i < hi - 1; ++i) {
            if (or_coord(t, i, ax) < pv) {
                or_swap(&t->idx[i], &t->idx[store]);
                ++store;
            }
        }
        or_swap(&t->idx[store], &t->idx[hi - 1]);
        if (store == k)
            return;
        if (k < store)
            hi = store;
        else
            lo = store + 1;
    }
}

/* The splitting value is recorded before the children are built, because
 * building the right child reorders the slot the median sits in.  The two
 * children cover disjoint index ranges and heap slots, so building them as
 * concurrent tasks gives the same tree as building them in turn. */
static void or_build(or_tree* t, int64_t node, int64_t lo, int64_t hi, int depth)
{
    if (hi - lo <= OR_LEAF)
        return;
    int ax = depth % t->dim;
    int64_t mid = lo + (hi - lo) / 2;
    or_select(t, lo, hi, mid, ax);
    t->split[node] = or_coord(t, mid, ax);
    if (hi - lo >= OR_TASK_MIN) {
#pragma omp task
        or_build(t, 2 * node, lo, mid, depth + 1);
        or_build(t, 2 * node + 1, mid, hi, depth + 1);
#pragma omp taskwait
    } else {
        or_build(t, 2 * node, lo, mid, depth + 1);
        or_build(t, 2 * node + 1, mid, hi, depth + 1);
    }
}

/* Number of heap slots the build can touch: sizes at depth d are at most
 * ceil(n / 2^d), and a node of at most OR_LEAF points is a leaf. */
static int64_t or_tree_slots(int64_t n)
{
    int64_t slots = 2, size = n;
    while (size > OR_LEAF) {
        size = (size + 1) / 2;
        slots *= 2;
    }
    return slots;
}

/* Range query: every point p with dist2(q, p) <= psi2.  A subtree is
 * skipped only when the squared distance to its splitting plane, computed
 * in FP64, exceeds psi2 times the reach of the cutoff along the axis (1 for
 * the sphere; T_aa (1 + 1e-6) for the ellipsoid, whose points beyond a
 * plane at distance h along axis a have q >= h^2 / T_aa): every point
 * beyond the plane then lies outside the cutoff too, so no pair the
 * brute-force search accepts is lost. */
static void or_query(const or_tree* t, const or_metric* g, int64_t node, int64_t lo, int64_t hi,
                     int depth, const double* q, double psi2, int64_t* out, int64_t* count, int64_t cap)
{
    if (hi - lo <= OR_LEAF) {
        for (int64_t k = lo; k < hi; ++k) {
            int64_t j = t->idx[k];
            if (or_dist2(g, t->dim, q, t->x + j * t->dim) <= psi2) {
                if (*count < cap)
                    out[*count] = j;
                ++*count;
            }
        }
        return;
    }
    int ax = depth % t->dim;
    int64_t mid = lo + (hi - lo) / 2;
    double split = t->split[node];
    double diff = split - q[ax];
    double lim = g->tensor ? psi2 * g->reach[ax] : psi2;
    if (q[ax] < split) {
        or_query(t, g, 2 * node, lo, mid, depth + 1, q, psi2, out, count, cap);
        if (diff * diff <= lim)
            or_query(t, g, 2 * node + 1, mid, hi, depth + 1, q, psi2, out, count, cap);
    } else {
        or_query(t, g, 2 * node + 1, mid, hi, depth + 1, q, psi2, out, count, cap);
        if (diff * diff <= lim)
            or_query(t, g, 2 * node, lo, mid, depth + 1, q, psi2, out, count, cap);
    }
}

static int or_cmp_i64(const void* a, const void* b)
{
    int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return (x > y) - (x < y);
}

/* Neighbour sets N(i) = { j : dist2_ij <= psi2 }, i included (Sec. 3),
 * from one search structure: counts into row_ptr[n+1], then the rows,
 * each sorted ascending, into *col_out (allocated here with malloc) when
 * col_out is given.  method 0: brute force over all pairs; 1: K-D tree.
 * Returns nnz, or -1 on allocation failure. */
static int64_t or_search(int dim, int64_t n, const double* x, double psi2, const or_metric* g,
                         int method, int64_t* row_ptr, int64_t** col_out)
{
    or_tree tree = {dim, x, NULL, NULL};
    if (method == 1) {
        tree.idx = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
        tree.split = (double*)malloc((size_t)or_tree_slots(n) * sizeof(double));
        if (!tree.idx || !tree.split) {
            free(tree.idx);
            free(tree.split);
            return -1;
        }
        for (int64_t i = 0; i < n; ++i)
            tree.idx[i] = i;
#pragma omp parallel
#pragma omp single
        or_build(&tree, 1, 0, n, 0);
    }
    int64_t* cnt = (int64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    if (!cnt) {
        free(tree.idx);
        free(tree.split);
        return -1;
    }
    /* pass 1: counts */
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = 0;
        if (method == 1) {
            or_query(&tree, g, 1, 0, n, 0, x + i * dim, psi2, NULL, &c, 0);
        } else {
            for (int64_t j = 0; j < n; ++j)
                if (or_dist2(g, dim, x + i * dim, x + j * dim) <= psi2)
                    ++c;
        }
        cnt[i] = c;
    }
    row_ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i)
        row_ptr[i + 1] = row_ptr[i] + cnt[i];
    int64_t nnz = row_ptr[n];
    if (col_out) {
        int64_t* col = (int64_t*)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int64_t));
        if (!col) {
            free(cnt);
            free(tree.idx);
            free(tree.split);
            return -1;
        }
        /* pass 2: fill, then sort each row ascending */
#pragma omp parallel for schedule(dynamic, 1024)
        for (int64_t i = 0; i < n; ++i) {
            int64_t* row = col + row_ptr[i];
            int64_t c = 0;
            if (method == 1) {
                or_query(&tree, g, 1, 0, n, 0, x + i * dim, psi2, row, &c, cnt[i]);
            } else {
                for (int64_t j = 0; j < n; ++j)
                    if (or_dist2(g, dim, x + i * dim, x + j * dim) <= psi2)
                        row[c++] = j;
            }
            qsort(row, (size_t)cnt[i], sizeof(int64_t), or_cmp_i64);
        }
        *col_out = col;
    }
    free(cnt);
    free(tree.idx);
    free(tree.split);
    return nnz;
}

/* Neighbour sets as CSR (see or_search).  tens: NULL or the shape tensor
 * (then dist2 is the Mahalanobis form).  Writes row_ptr[n+1] always and col
 * only if the total fits in cap.  Returns nnz, or -1 on allocation failure
 * or a tensor that is not positive definite. */
int64_t or_neighbors(int dim, int64_t n, const double* x, double psi2, const double* tens, int method,
                     int64_t* row_ptr, int64_t* col, int64_t cap)
{
    or_metric g;
    if (or_metric_make(dim, tens, &g) != 0)
        return -1;
    int64_t* c = NULL;
    int64_t nnz = or_search(dim, n, x, psi2, &g, method, row_ptr, col ? &c : NULL);
    if (nnz >= 0 && col && nnz <= cap && nnz > 0)
        memcpy(col, c, (size_t)nnz * sizeof(int64_t));
    free(c);
    return nnz;
}

/* ------------------------------------------------------------------ */
/* Sec. 3, Eq. (2)-(3): Gaussian mass-transfer kernel with the          */
/* bandwidth set by beta, K_ij = exp(-beta r2 / (4 D_MT dt)) (r2 the     */
/* Mahalanobis form with a tensor); the normalising prefactor is        */
/* dropped because it cancels in W.  Then the symmetric normalisation   */
/* by the mean of the row and column sums,                               */
/* W_ij = K_ij / (0.5 (s_i + s_j)),  s_i = sum_{k in N(i)} K_ik,        */
/* with the self term K_ii = 1 included (the sums run over all k).      */
/* K and W are written per CSR entry; W_ii is written as 0 (it never    */
/* moves mass).                                                          */
/* ------------------------------------------------------------------ */
static void or_weights(const or_metric* g, int dim, int64_t n, const double* x, double d_mt, double dt,
                       double beta, const int64_t* row_ptr, const int64_t* col, double* s, double* kv,
                       double* wv)
{
    double denom = 4.0 * d_mt * dt;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            int64_t j = col[e];
            double r2 = or_dist2(g, dim, x + i * dim, x + j * dim);
            double k = exp(-(beta * r2) / denom);
            if (kv)
                kv[e] = k;
            acc = acc + k;
        }
        s[i] = acc;
    }
    if (wv) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
                int64_t j = col[e];
                if (j == i) {
                    wv[e] = 0.0;
                    continue;
                }
                double r2 = or_dist2(g, dim, x + i * dim, x + j * dim);
                double k = exp(-(beta * r2) / denom);
                wv[e] = k / (0.5 * (s[i] + s[j]));
            }
        }
    }
}

void or_mt_weights(int dim, int64_t n, const double* x, double d_mt, double dt, double beta,
                   const double* tens, const int64_t* row_ptr, const int64_t* col, double* s /* [n] */,
                   double* kv /* [nnz] or NULL */, double* wv /* [nnz] or NULL */)
{
    or_metric g;
    if (or_metric_make(dim, tens, &g) != 0)
        return;
    or_weights(&g, dim, n, x, d_mt, dt, beta, row_ptr, col, s, kv, wv);
}

/* Sec. 3, Eq. (4)-(5): explicit update M_i(t+dt) = M_i(t) + delta_i with
 * delta_i = sum_j beta (M_j(t) - M_i(t)) W_ij, every delta from M(t) (the
 * right-hand side uses time t only), summed in ascending j.
 * m_in and m_out are [S][n] and must not alias.  Returns the number of
 * ordered pairs i != j within psi, or -1 on failure. */
int64_t or_mt_step(int dim, int64_t n, int n_species, const double* x, const double* m_in,
                   double* m_out, double d_mt, double dt, double beta, double psi, const double* tens,
                   int method)
{
    or_metric g;
    if (or_metric_make(dim, tens, &g) != 0)
        return -1;
    double psi2 = psi * psi;
    int64_t* row_ptr = (int64_t*)malloc((size_t)(n + 1) * sizeof(int64_t));
    if (!row_ptr)
        return -1;
    int64_t* col = NULL;
    int64_t nnz = or_search(dim, n, x, psi2, &g, method, row_ptr, &col);
    double* wv = (double*)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(double));
    double* s = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    if (nnz < 0 || !wv || !s) {
        free(row_ptr); free(col); free(wv); free(s);
        return -1;
    }
    or_weights(&g, dim, n, x, d_mt, dt, beta, row_ptr, col, s, NULL, wv);
    for (int c = 0; c < n_species; ++c) {
        const double* mi = m_in + (int64_t)c * n;
        double* mo = m_out + (int64_t)c * n;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double delta = 0.0;
            for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
                int64_t j = col[e];
                if (j == i)
                    continue;
                delta = delta + (mi[j] - mi[i]) * wv[e];
            }
            mo[i] = mi[i] + beta * delta;
        }
    }
    free(row_ptr); free(col); free(wv); free(s);
    return nnz - n;
}

/* ------------------------------------------------------------------ */
/* A + B -> C, well-mixed second order over dt inside each particle,    */
/* on concentrations c = N M / V (Sec. 3's mass-to-concentration map,   */
/* V the volume of the simulation box).  da/dt = db/dt = -k a b has     */
/* the exact solution with D = a - b >= 0 (swap otherwise):             */
/*   a' = a D / (D - b expm1(-k D dt))   (D > 0),  a' = a/(1 + k a dt)   */
/*   (D = 0),  b' = a' - D,  c' = c + (a - a').                          */
/* m is [3][n]: species A, B, C.                                         */
/* ------------------------------------------------------------------ */
void or_react(int64_t n, double* m, double k_react, double dt, double n_total, double volume)
{
    double to_c = n_total / volume;
    double to_m = volume / n_total;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double a = m[i] * to_c;
        double b = m[n + i] * to_c;
        int swapped = 0;
        if (b > a) {
            double tmp = a;
            a = b;
            b = tmp;
            swapped = 1;
        }
        double d = a - b;
        double a_new;
        if (d > 0.0)
            a_new = a * d / (d - b * expm1(-k_react * d * dt));
        else
            a_new = a / (1.0 + k_react * a * dt);
        double b_new = a_new - d;
        double reacted = a - a_new;
        if (swapped) {
            double tmp = a_new;
            a_new = b_new;
            b_new = tmp;
        }
        m[i] = a_new * to_m;
        m[n + i] = b_new * to_m;
        m[2 * n + i] = m[2 * n + i] + reacted * to_m;
    }
}

/* Neumaier-compensated FP64 sum (Neumaier 1974). */
double or_total(int64_t n, const double* v)
{
    double sum = 0.0, comp = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double t = sum + v[i];
        if (fabs(sum) >= fabs(v[i]))
            comp = comp + ((sum - t) + v[i]);
        else
            comp = comp + ((v[i] - t) + sum);
        sum = t;
    }
    return sum + comp;
}

/* ------------------------------------------------------------------ */
/* The step loop: for each step t = start_step .. start_step+steps-1,   */
/*   random walk (if d_rw > 0 or v != 0) -> neighbours within psi ->    */
/*   weights -> mass transfer -> reaction (3 species, k_react > 0) ->   */
/*   record.                                                            */
/* The box [lo, hi] is the simulation's own box (its volume maps masses */
/* to concentrations for the reaction); tens is NULL or the shape       */
/* tensor of the dispersion.                                            */
/* fp32 != 0 keeps the position state in FP32 (the caller passes        */
/* positions already rounded to float); the mass transfer itself is     */
/* always FP64.  pairs_out[steps] gets the ordered pairs i != j per step */
/* and totals_out[steps][S] the compensated mass totals after the step. */
/* Returns 0, or -1 on failure (allocation, or a tensor that is not     */
/* positive definite).                                                   */
/* ------------------------------------------------------------------ */
int or_run(int dim, int64_t n, int n_species, const double* lo, const double* hi, double d_rw,
           const double* vel, double d_mt, double dt, double beta, double psi, double k_react,
           uint64_t seed, int64_t start_step, int fp32, const double* tens, int method, int64_t steps,
           double* x, double* m, int64_t* pairs_out, double* totals_out, int n_threads)
{
#ifdef _OPENMP
    if (n_threads > 0)
        omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
    or_metric g;
    if (or_metric_make(dim, tens, &g) != 0)
        return -1;
    double* m2 = (double*)malloc((size_t)n_species * (size_t)(n > 0 ? n : 1) * sizeof(double));
    if (!m2)
        return -1;
    double volume = 1.0;
    for (int k = 0; k < dim; ++k)
        volume = volume * (hi[k] - lo[k]);
    for (int64_t s = 0; s < steps; ++s) {
        int64_t t = start_step + s;
        int moving = d_rw > 0.0;
        for (int k = 0; k < dim; ++k)
            moving = moving || vel[k] != 0.0;
        if (moving)
            or_rw_step(dim, n, lo, hi, d_rw, vel, dt, seed, t, fp32, tens, x);
        int64_t pairs = or_mt_step(dim, n, n_species, x, m, m2, d_mt, dt, beta, psi, tens, method);
        if (pairs < 0) {
            free(m2);
            return -1;
        }
        memcpy(m, m2, (size_t)n_species * (size_t)n * sizeof(double));
        if (n_species == 3 && k_react > 0.0)
            or_react(n, m, k_react, dt, (double)n, volume);
        if (pairs_out)
            pairs_out[s] = pairs;
        if (totals_out)
            for (int c = 0; c < n_species; ++c)
                totals_out[s * n_species + c] = or_total(n, m + (int64_t)c * n);
    }
    free(m2);
    return 0;
}

int or_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_threads(int n_threads)
{
#ifdef _OPENMP
    if (n_threads > 0)
        omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
}
