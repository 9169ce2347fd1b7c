/*
 * fmm_oracle.c -- FP64 CPU oracle for the 3-D Laplace fast multipole method.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or table with the GPU
 * library: the GPU path works in a spherical-harmonic basis, this oracle in
 * Cartesian Taylor monomials, and both truncate the same Taylor series, so
 * they agree up to rounding.
 *
 * What it computes (Yokota, Ibeid, Keyes, "Fast Multipole Method as a
 * Matrix-Free Hierarchical Low-Rank Approximation"):
 *   - Sec. 1 / Sec. 2.2: the direct N-body sum phi_i = sum_{j!=i} q_j/|x_i-x_j|
 *     (the dense "direct operator"), and its gradient;
 *   - Sec. 1: the FMM approximation of that sum, built on a hierarchical
 *     spatial decomposition with multipole and local expansions;
 *   - Sec. 2.2: interaction lists produced by a dual tree traversal with a
 *     multipole acceptance criterion (MAC); with theta = 1/2 the same-level
 *     lists are the classical "parent's neighbours' children that are not
 *     neighbours", at most 6^3-3^3 = 189 sources per box.
 * The paper prints no expansion formulas.  The ones used here are Taylor's
 * theorem applied to 1/|r| (the Cartesian form of the Greengard-Rokhlin
 * expansions): with T_g(r) = (1/g!) d^g (1/|r|),
 *   P2M  M_a   = sum_j q_j (x_j - c)^a                       |a| <= p
 *   M2M  M_a(c) = sum_{b<=a} C(a,b) (c'-c)^(a-b) M_b(c')
 *   M2L  L_b   = sum_a (-1)^|a| C(a+b,a) M_a T_(a+b)(c_A - c_B)  |a|,|b| <= p
 *   L2L  L_b(c') = sum_{g>=b} C(g,b) (c'-c)^(g-b) L_g(c)
 *   L2P  phi(x) = sum_b L_b (x - c)^b, grad = exact derivative of that polynomial
 * and T obeys (n = |g|, T_0 = 1/|r|)
 *   |r|^2 T_g = -(2 - 1/n) sum_i r_i T_(g-e_i) - (1 - 1/n) sum_i T_(g-2e_i).
 *
 * Readings where the paper is silent (root cube, keys, leaf rule, MAC form,
 * split rule) are the ones the GPU library also follows; they are restated
 * at each function below.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC (no -ffast-math: IEEE order matters
 * for the integer decisions of the tree and the lists).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_MAX_LEVEL 21

/* ------------------------------------------------------------------------ */
/* Threads                                                                   */
/* ------------------------------------------------------------------------ */
int oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Direct sum (Sec. 1: the O(N^2) problem the FMM approximates)              */
/* ------------------------------------------------------------------------ */
/* Neumaier's compensated summation: s + c carries the running sum. */
static inline void neumaier_add(double *s, double *c, double v) {
    double t = *s + v;
    if (fabs(*s) >= fabs(v)) *c += (*s - t) + v;
    else                     *c += (v - t) + *s;
    *s = t;
}

/*
 * phi_i  = sum_{j != i, x_j != x_i} q_j / |x_i - x_j|
 * grad_i = -sum_{j != i, x_j != x_i} q_j (x_i - x_j) / |x_i - x_j|^3
 * for every i in targ[0..nt) (or all i when targ == NULL; then nt is ignored).
 * pts is [n][3] (row-major), phi is [nt], grad is [nt][3] (may be NULL).
 */
void oracle_direct(int64_t n, const double *pts, const double *q,
                   int64_t nt, const int64_t *targ, double *phi, double *grad) {
    if (!targ) nt = n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t i = targ ? targ[t] : t;
        double xi = pts[3 * i], yi = pts[3 * i + 1], zi = pts[3 * i + 2];
        double s = 0, sc = 0, gx = 0, gxc = 0, gy = 0, gyc = 0, gz = 0, gzc = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = xi - pts[3 * j], dy = yi - pts[3 * j + 1], dz = zi - pts[3 * j + 2];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) continue;
            double r = sqrt(r2);
            double v = q[j] / r;
            double w = v / r2;
            neumaier_add(&s, &sc, v);
            neumaier_add(&gx, &gxc, -w * dx);
            neumaier_add(&gy, &gyc, -w * dy);
            neumaier_add(&gz, &gzc, -w * dz);
        }
        phi[t] = s + sc;
        if (grad) {
            grad[3 * t] = gx + gxc;
            grad[3 * t + 1] = gy + gyc;
            grad[3 * t + 2] = gz + gzc;
        }
    }
}

/*
 * Hessian of phi (second derivatives in x_i) at every target:
 *   H_i = sum_{j != i, x_j != x_i} q_j (3 d d^T / |d|^5 - I / |d|^3),  d = x_i - x_j
 * hess is [nt][6] in the order xx, yy, zz, xy, xz, yz.
 */
void oracle_direct_hessian(int64_t n, const double *pts, const double *q, int64_t nt, const int64_t *targ,
                           double *hess) {
    if (!targ) nt = n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t i = targ ? targ[t] : t;
        double h[6] = {0, 0, 0, 0, 0, 0}, hc[6] = {0, 0, 0, 0, 0, 0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3] = {pts[3 * i] - pts[3 * j], pts[3 * i + 1] - pts[3 * j + 1], pts[3 * i + 2] - pts[3 * j + 2]};
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 == 0.0) continue;
            double r = sqrt(r2), ir3 = q[j] / (r2 * r), ir5 = 3.0 * ir3 / r2;
            neumaier_add(&h[0], &hc[0], ir5 * d[0] * d[0] - ir3);
            neumaier_add(&h[1], &hc[1], ir5 * d[1] * d[1] - ir3);
            neumaier_add(&h[2], &hc[2], ir5 * d[2] * d[2] - ir3);
            neumaier_add(&h[3], &hc[3], ir5 * d[0] * d[1]);
            neumaier_add(&h[4], &hc[4], ir5 * d[0] * d[2]);
            neumaier_add(&h[5], &hc[5], ir5 * d[1] * d[2]);
        }
        for (int a = 0; a < 6; ++a) hess[6 * t + a] = h[a] + hc[a];
    }
}

/* ------------------------------------------------------------------------ */
/* Cartesian multi-indices                                                   */
/*
 * Charges and dipoles (Sec. 1 with source positions as variables: a dipole g_j at x_j is
 * the derivative of a unit charge's field along g_j when x_j moves):
 *   phi_i  = sum_{j != i, x_j != x_i} [ q_j / |d| + g_j . d / |d|^3 ],      d = x_i - x_j
 *   grad_i = sum_{j != i, x_j != x_i} [ -q_j d / |d|^3 + g_j / |d|^3 - 3 (g_j . d) d / |d|^5 ]
 * dip is [n][3]; targets, phi and grad as in oracle_direct.
 */
void oracle_direct_dip(int64_t n, const double *pts, const double *q, const double *dip,
                       int64_t nt, const int64_t *targ, double *phi, double *grad) {
    if (!targ) nt = n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t i = targ ? targ[t] : t;
        double xi = pts[3 * i], yi = pts[3 * i + 1], zi = pts[3 * i + 2];
        double s = 0, sc = 0, g[3] = {0, 0, 0}, gc[3] = {0, 0, 0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3] = {xi - pts[3 * j], yi - pts[3 * j + 1], zi - pts[3 * j + 2]};
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 == 0.0) continue;
            double r = sqrt(r2), r3 = r2 * r;
            const double *gj = dip + 3 * j;
            double gd = gj[0] * d[0] + gj[1] * d[1] + gj[2] * d[2];
            neumaier_add(&s, &sc, q[j] / r + gd / r3);
            for (int a = 0; a < 3; ++a)
                neumaier_add(&g[a], &gc[a], -q[j] * d[a] / r3 + gj[a] / r3 - 3.0 * gd * d[a] / (r3 * r2));
        }
        phi[t] = s + sc;
        if (grad)
            for (int a = 0; a < 3; ++a) grad[3 * t + a] = g[a] + gc[a];
    }
}

/* ------------------------------------------------------------------------ */
/* Multi-indices a = (a0,a1,a2) with |a| <= P, enumerated degree by degree.  */
typedef struct {
    int P;          /* highest total degree held */
    int n;          /* number of multi-indices, (P+1)(P+2)(P+3)/6 */
    int *a;         /* [n][3] components */
    int *deg;       /* [n] |a| */
    int *lookup;    /* [(P+1)^3] index of (a0,a1,a2), -1 outside */
} mindex;

static int mi_count(int P) { return (P + 1) * (P + 2) * (P + 3) / 6; }

static void mi_init(mindex *m, int P) {
    m->P = P;
    m->n = mi_count(P);
    m->a = (int *)malloc(sizeof(int) * 3 * m->n);
    m->deg = (int *)malloc(sizeof(int) * m->n);
    int L = P + 1;
    m->lookup = (int *)malloc(sizeof(int) * L * L * L);
    for (int i = 0; i < L * L * L; ++i) m->lookup[i] = -1;
    int k = 0;
    for (int d = 0; d <= P; ++d)
        for (int a0 = d; a0 >= 0; --a0)
            for (int a1 = d - a0; a1 >= 0; --a1) {
                int a2 = d - a0 - a1;
                m->a[3 * k] = a0; m->a[3 * k + 1] = a1; m->a[3 * k + 2] = a2;
                m->deg[k] = d;
                m->lookup[(a0 * L + a1) * L + a2] = k;
                ++k;
            }
}

static void mi_free(mindex *m) { free(m->a); free(m->deg); free(m->lookup); }

static inline int mi_idx(const mindex *m, int a0, int a1, int a2) {
    if (a0 < 0 || a1 < 0 || a2 < 0) return -1;
    int L = m->P + 1;
    if (a0 >= L || a1 >= L || a2 >= L) return -1;
    return m->lookup[(a0 * L + a1) * L + a2];
}

/* Binomial coefficients C(n,k) for n <= 2*16. */
static double binom_tab[64][64];
static int binom_ready = 0;
static void binom_init(void) {
    if (binom_ready) return;
    for (int n = 0; n < 64; ++n)
        for (int k = 0; k < 64; ++k) binom_tab[n][k] = 0.0;
    for (int n = 0; n < 64; ++n) {
        binom_tab[n][0] = 1.0;
        for (int k = 1; k <= n; ++k) binom_tab[n][k] = binom_tab[n - 1][k - 1] + (k <= n - 1 ? binom_tab[n - 1][k] : 0.0);
    }
    binom_ready = 1;
}

/* Everything the expansions of order p need. */
typedef struct {
    int p;
    mindex mp;    /* |a| <= p  : multipole / local coefficients */
    mindex m2p;   /* |g| <= 2p : T_g derivative tensors          */
    /* M2L contraction: for local b and multipole a, the coefficient
       (-1)^|a| C(a+b,a) and the index of a+b in m2p. */
    double *m2l_coef;   /* [n_p][n_p] */
    int *m2l_gidx;      /* [n_p][n_p] */
} expctx;

static void exp_init(expctx *e, int p) {
    binom_init();
    e->p = p;
    mi_init(&e->mp, p);
    mi_init(&e->m2p, 2 * p);
    int n = e->mp.n;
    e->m2l_coef = (double *)malloc(sizeof(double) * n * n);
    e->m2l_gidx = (int *)malloc(sizeof(int) * n * n);
    for (int b = 0; b < n; ++b) {
        const int *bb = e->mp.a + 3 * b;
        for (int a = 0; a < n; ++a) {
            const int *aa = e->mp.a + 3 * a;
            double c = binom_tab[aa[0] + bb[0]][aa[0]] * binom_tab[aa[1] + bb[1]][aa[1]] *
                       binom_tab[aa[2] + bb[2]][aa[2]];
            if (e->mp.deg[a] & 1) c = -c;
            e->m2l_coef[b * n + a] = c;
            e->m2l_gidx[b * n + a] = mi_idx(&e->m2p, aa[0] + bb[0], aa[1] + bb[1], aa[2] + bb[2]);
        }
    }
}

static void exp_free(expctx *e) {
    mi_free(&e->mp);
    mi_free(&e->m2p);
    free(e->m2l_coef);
    free(e->m2l_gidx);
}

/* T_g(r) = (1/g!) d^g (1/|r|) for all |g| <= m->P, by the recurrence above. */
static void taylor_T(const mindex *m, const double r[3], double *T) {
    double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    T[0] = 1.0 / sqrt(r2);
    for (int k = 1; k < m->n; ++k) {
        const int *g = m->a + 3 * k;
        int n = m->deg[k];
        double s1 = 0.0, s2 = 0.0;
        for (int i = 0; i < 3; ++i) {
            int g1[3] = {g[0], g[1], g[2]};
            g1[i] -= 1;
            int i1 = mi_idx(m, g1[0], g1[1], g1[2]);
            if (i1 >= 0) s1 += r[i] * T[i1];
            g1[i] -= 1;
            int i2 = mi_idx(m, g1[0], g1[1], g1[2]);
            if (i2 >= 0) s2 += T[i2];
        }
        T[k] = (-(2.0 - 1.0 / n) * s1 - (1.0 - 1.0 / n) * s2) / r2;
    }
}

/* powers v^0..v^P */
static void powers(double v, int P, double *out) {
    out[0] = 1.0;
    for (int i = 1; i <= P; ++i) out[i] = out[i - 1] * v;
}

/* P2M: M_a += sum_j q_j (x_j - c)^a */
static void p2m_acc(const expctx *e, int64_t n, const double *pts, const double *q, const double c[3], double *M) {
    int p = e->p;
    double px[32], py[32], pz[32];
    for (int64_t j = 0; j < n; ++j) {
        powers(pts[3 * j] - c[0], p, px);
        powers(pts[3 * j + 1] - c[1], p, py);
        powers(pts[3 * j + 2] - c[2], p, pz);
        for (int k = 0; k < e->mp.n; ++k) {
            const int *a = e->mp.a + 3 * k;
            M[k] += q[j] * px[a[0]] * py[a[1]] * pz[a[2]];
        }
    }
}

/* P2M of dipoles: the derivative of a charge's multipole along its dipole as the charge
   moves, M_a += sum_j sum_i g_ji a_i (x_j - c)^(a - e_i) */
static void p2m_dip_acc(const expctx *e, int64_t n, const double *pts, const double *dip, const double c[3],
                        double *M) {
    int p = e->p;
    double px[32], py[32], pz[32];
    for (int64_t j = 0; j < n; ++j) {
        powers(pts[3 * j] - c[0], p, px);
        powers(pts[3 * j + 1] - c[1], p, py);
        powers(pts[3 * j + 2] - c[2], p, pz);
        const double *g = dip + 3 * j;
        for (int k = 0; k < e->mp.n; ++k) {
            const int *a = e->mp.a + 3 * k;
            double v = 0.0;
            if (a[0] > 0) v += g[0] * a[0] * px[a[0] - 1] * py[a[1]] * pz[a[2]];
            if (a[1] > 0) v += g[1] * a[1] * px[a[0]] * py[a[1] - 1] * pz[a[2]];
            if (a[2] > 0) v += g[2] * a[2] * px[a[0]] * py[a[1]] * pz[a[2] - 1];
            M[k] += v;
        }
    }
}

/* M2M: M_a(c) += sum_{b<=a} C(a,b) d^(a-b) M_b(c'),  d = c' - c */
static void m2m_acc(const expctx *e, const double *Mc, const double d[3], double *Mp) {
    int p = e->p;
    double dx[32], dy[32], dz[32];
    powers(d[0], p, dx); powers(d[1], p, dy); powers(d[2], p, dz);
    for (int ia = 0; ia < e->mp.n; ++ia) {
        const int *a = e->mp.a + 3 * ia;
        double s = 0.0;
        for (int b0 = 0; b0 <= a[0]; ++b0)
            for (int b1 = 0; b1 <= a[1]; ++b1)
                for (int b2 = 0; b2 <= a[2]; ++b2) {
                    int ib = mi_idx(&e->mp, b0, b1, b2);
                    s += binom_tab[a[0]][b0] * binom_tab[a[1]][b1] * binom_tab[a[2]][b2] *
                         dx[a[0] - b0] * dy[a[1] - b1] * dz[a[2] - b2] * Mc[ib];
                }
        Mp[ia] += s;
    }
}

/* M2L: L_b(A) += sum_a (-1)^|a| C(a+b,a) M_a(B) T_(a+b)(c_A - c_B); Tbuf holds m2p.n doubles */
static void m2l_acc(const expctx *e, const double *M, const double D[3], double *L, double *Tbuf) {
    taylor_T(&e->m2p, D, Tbuf);
    int n = e->mp.n;
    for (int b = 0; b < n; ++b) {
        const double *cf = e->m2l_coef + (size_t)b * n;
        const int *gi = e->m2l_gidx + (size_t)b * n;
        double s = 0.0;
        for (int a = 0; a < n; ++a) s += cf[a] * M[a] * Tbuf[gi[a]];
        L[b] += s;
    }
}

/* L2L: L_b(c') += sum_{g>=b} C(g,b) d^(g-b) L_g(c),  d = c' - c */
static void l2l_acc(const expctx *e, const double *Lp, const double d[3], double *Lc) {
    int p = e->p;
    double dx[32], dy[32], dz[32];
    powers(d[0], p, dx); powers(d[1], p, dy); powers(d[2], p, dz);
    for (int ib = 0; ib < e->mp.n; ++ib) {
        const int *b = e->mp.a + 3 * ib;
        double s = 0.0;
        for (int ig = 0; ig < e->mp.n; ++ig) {
            const int *g = e->mp.a + 3 * ig;
            if (g[0] < b[0] || g[1] < b[1] || g[2] < b[2]) continue;
            s += binom_tab[g[0]][b[0]] * binom_tab[g[1]][b[1]] * binom_tab[g[2]][b[2]] *
                 dx[g[0] - b[0]] * dy[g[1] - b[1]] * dz[g[2] - b[2]] * Lp[ig];
        }
        Lc[ib] += s;
    }
}

/* L2P: phi += sum_b L_b t^b, grad and hess (xx, yy, zz, xy, xz, yz) += the first and
 * second derivatives of the same polynomial,  t = x - c */
static double dpow(const double *tp, int b, int k) {   /* d^k/dt^k of t^b */
    if (b < k) return 0.0;
    double f = 1.0;
    for (int i = 0; i < k; ++i) f *= (double)(b - i);
    return f * tp[b - k];
}
static void l2p_one_h(const expctx *e, const double *L, const double c[3], const double x[3],
                      double *phi, double *grad, double *hess) {
    int p = e->p;
    double tx[32], ty[32], tz[32];
    powers(x[0] - c[0], p, tx); powers(x[1] - c[1], p, ty); powers(x[2] - c[2], p, tz);
    double s = 0, gx = 0, gy = 0, gz = 0, h[6] = {0, 0, 0, 0, 0, 0};
    for (int k = 0; k < e->mp.n; ++k) {
        const int *b = e->mp.a + 3 * k;
        s += L[k] * tx[b[0]] * ty[b[1]] * tz[b[2]];
        if (b[0] > 0) gx += L[k] * b[0] * tx[b[0] - 1] * ty[b[1]] * tz[b[2]];
        if (b[1] > 0) gy += L[k] * b[1] * tx[b[0]] * ty[b[1] - 1] * tz[b[2]];
        if (b[2] > 0) gz += L[k] * b[2] * tx[b[0]] * ty[b[1]] * tz[b[2] - 1];
        if (hess) {
            h[0] += L[k] * dpow(tx, b[0], 2) * ty[b[1]] * tz[b[2]];
            h[1] += L[k] * tx[b[0]] * dpow(ty, b[1], 2) * tz[b[2]];
            h[2] += L[k] * tx[b[0]] * ty[b[1]] * dpow(tz, b[2], 2);
            h[3] += L[k] * dpow(tx, b[0], 1) * dpow(ty, b[1], 1) * tz[b[2]];
            h[4] += L[k] * dpow(tx, b[0], 1) * ty[b[1]] * dpow(tz, b[2], 1);
            h[5] += L[k] * tx[b[0]] * dpow(ty, b[1], 1) * dpow(tz, b[2], 1);
        }
    }
    *phi += s;
    if (grad) { grad[0] += gx; grad[1] += gy; grad[2] += gz; }
    if (hess) for (int a = 0; a < 6; ++a) hess[a] += h[a];
}
static void l2p_one(const expctx *e, const double *L, const double c[3], const double x[3],
                    double *phi, double *grad) {
    l2p_one_h(e, L, c, x, phi, grad, NULL);
}

/* ------------------------------------------------------------------------ */
/* Single-operator entry points (used by the tests that pin each step)       */
/* ------------------------------------------------------------------------ */
int oracle_num_coeffs(int p) { return mi_count(p); }

/* Multi-index table of order p: out[k][3] */
void oracle_multi_indices(int p, int *out) {
    mindex m; mi_init(&m, p);
    memcpy(out, m.a, sizeof(int) * 3 * m.n);
    mi_free(&m);
}

/* T_g(r) for |g| <= P, in the enumeration of oracle_multi_indices(P). */
void oracle_taylor_T(int P, const double r[3], double *T) {
    mindex m; mi_init(&m, P);
    taylor_T(&m, r, T);
    mi_free(&m);
}

void oracle_p2m(int p, int64_t n, const double *pts, const double *q, const double c[3], double *M) {
    expctx e; exp_init(&e, p);
    memset(M, 0, sizeof(double) * e.mp.n);
    p2m_acc(&e, n, pts, q, c, M);
    exp_free(&e);
}

void oracle_p2m_dip(int p, int64_t n, const double *pts, const double *dip, const double c[3], double *M) {
    expctx e;
    exp_init(&e, p);
    for (int k = 0; k < e.mp.n; ++k) M[k] = 0.0;
    p2m_dip_acc(&e, n, pts, dip, c, M);
    exp_free(&e);
}

void oracle_m2m(int p, const double *Mc, const double d[3], double *Mp) {
    expctx e; exp_init(&e, p);
    memset(Mp, 0, sizeof(double) * e.mp.n);
    m2m_acc(&e, Mc, d, Mp);
    exp_free(&e);
}

void oracle_m2l(int p, const double *M, const double D[3], double *L) {
    expctx e; exp_init(&e, p);
    double *T = (double *)malloc(sizeof(double) * e.m2p.n);
    memset(L, 0, sizeof(double) * e.mp.n);
    m2l_acc(&e, M, D, L, T);
    free(T);
    exp_free(&e);
}

void oracle_l2l(int p, const double *Lp, const double d[3], double *Lc) {
    expctx e; exp_init(&e, p);
    memset(Lc, 0, sizeof(double) * e.mp.n);
    l2l_acc(&e, Lp, d, Lc);
    exp_free(&e);
}

void oracle_l2p(int p, const double *L, const double c[3], int64_t n, const double *x, double *phi, double *grad) {
    expctx e; exp_init(&e, p);
    for (int64_t i = 0; i < n; ++i) {
        phi[i] = 0.0;
        if (grad) grad[3 * i] = grad[3 * i + 1] = grad[3 * i + 2] = 0.0;
        l2p_one(&e, L, c, x + 3 * i, phi + i, grad ? grad + 3 * i : NULL);
    }
    exp_free(&e);
}

/* Far field of a multipole about c evaluated directly: sum_a (-1)^|a| M_a T_a(x - c) */
void oracle_multipole_eval(int p, const double *M, const double c[3], int64_t n, const double *x, double *phi) {
    mindex m; mi_init(&m, p);
    double *T = (double *)malloc(sizeof(double) * m.n);
    for (int64_t i = 0; i < n; ++i) {
        double r[3] = {x[3 * i] - c[0], x[3 * i + 1] - c[1], x[3 * i + 2] - c[2]};
        taylor_T(&m, r, T);
        double s = 0.0;
        for (int k = 0; k < m.n; ++k) s += ((m.deg[k] & 1) ? -1.0 : 1.0) * M[k] * T[k];
        phi[i] = s;
    }
    free(T);
    mi_free(&m);
}

/* ------------------------------------------------------------------------ */
/* Tree (Sec. 1 hierarchical decomposition; Sec. 3.1 1-D Morton locality)    */
/* ------------------------------------------------------------------------ */
typedef struct {
    int level;
    uint64_t prefix;     /* key >> 3*(21-level) */
    int64_t start, count;/* range in the sorted order */
    int64_t parent;
    int64_t child[8];    /* -1 when the octant is empty; all -1 for a leaf */
    int nchild;
} ocell;

typedef struct {
    int64_t n;
    int ncrit;
    float theta;
    int lists;           /* 0: dual traversal (split both); 1: one cell at a time (level skip) */
    int k;               /* root side = 2^k */
    double x0[3];        /* root corner */
    double *pts;         /* [n][3] input order (copy) */
    uint64_t *key;       /* [n] input order */
    int64_t *order;      /* sorted position -> input index */
    ocell *cells;
    int64_t ncells, cap;
    /* lists */
    int64_t *m2l;        /* [nm2l][2] (target, source) */
    int64_t nm2l, m2l_cap;
    int64_t *p2p;        /* [np2p][2] (target leaf, source leaf) */
    int64_t np2p, p2p_cap;
} oplan;

/*
 * Root cube (reading of the silent paper): lo/hi are the per-axis extremes of
 * the inputs; the side is the smallest power of two 2^k with
 * hi_a - x0_a <= 2^k on every axis (the closed box), where x0_a is lo_a rounded
 * down to a multiple of 2^(k-22).  A point on the upper face is clamped into the
 * last cell, whose closure contains it.  All box centres and centre differences
 * are then dyadic and exact.
 */
static void root_cube(int64_t n, const double *pts, int *k_out, double x0[3]) {
    double lo[3], hi[3];
    for (int a = 0; a < 3; ++a) { lo[a] = pts[a]; hi[a] = pts[a]; }
    for (int64_t i = 1; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            double v = pts[3 * i + a];
            if (v < lo[a]) lo[a] = v;
            if (v > hi[a]) hi[a] = v;
        }
    double E = 0.0;
    for (int a = 0; a < 3; ++a) if (hi[a] - lo[a] > E) E = hi[a] - lo[a];
    int e = 0;
    frexp(E, &e);           /* 2^(e-1) <= E < 2^e  (e = 0 for E = 0) */
    int k = e - 1;          /* smallest k with 2^k >= E when E is a power of two; raised below if needed */
    for (;;) {
        double unit = ldexp(1.0, k - 22);
        int ok = 1;
        for (int a = 0; a < 3; ++a) {
            x0[a] = floor(lo[a] / unit) * unit;
            if (!(hi[a] - x0[a] <= ldexp(1.0, k))) ok = 0;
        }
        if (ok) break;
        ++k;
    }
    *k_out = k;
}

/* Per-axis integer coordinate at level 21: floor((x - x0) * 2^(21-k)), clamped. */
static inline uint64_t axis_coord(double x, double x0, int k) {
    double v = floor((x - x0) * ldexp(1.0, ORACLE_MAX_LEVEL - k));
    if (v < 0) v = 0;
    double top = (double)((1u << ORACLE_MAX_LEVEL) - 1);
    if (v > top) v = top;
    return (uint64_t)v;
}

/* 63-bit Morton key: bit b of ix -> 3b+2, of iy -> 3b+1, of iz -> 3b. */
static uint64_t morton(uint64_t ix, uint64_t iy, uint64_t iz) {
    uint64_t key = 0;
    for (int b = 0; b < ORACLE_MAX_LEVEL; ++b) {
        key |= ((ix >> b) & 1ull) << (3 * b + 2);
        key |= ((iy >> b) & 1ull) << (3 * b + 1);
        key |= ((iz >> b) & 1ull) << (3 * b);
    }
    return key;
}

static void prefix_coords(uint64_t prefix, int level, uint64_t c[3]) {
    c[0] = c[1] = c[2] = 0;
    for (int b = 0; b < level; ++b) {
        c[0] |= ((prefix >> (3 * b + 2)) & 1ull) << b;
        c[1] |= ((prefix >> (3 * b + 1)) & 1ull) << b;
        c[2] |= ((prefix >> (3 * b)) & 1ull) << b;
    }
}

static void cell_center(const oplan *P, const ocell *c, double ctr[3]) {
    uint64_t ic[3];
    prefix_coords(c->prefix, c->level, ic);
    double side = ldexp(1.0, P->k - c->level);
    for (int a = 0; a < 3; ++a) ctr[a] = P->x0[a] + ((double)ic[a] + 0.5) * side;
}

static const uint64_t *g_sort_keys;
static int cmp_key_index(const void *pa, const void *pb) {
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    uint64_t ka = g_sort_keys[a], kb = g_sort_keys[b];
    if (ka < kb) return -1;
    if (ka > kb) return 1;
    return (a < b) ? -1 : (a > b);
}

static int64_t new_cell(oplan *P) {
    if (P->ncells == P->cap) {
        P->cap = P->cap ? 2 * P->cap : 1024;
        P->cells = (ocell *)realloc(P->cells, sizeof(ocell) * P->cap);
    }
    return P->ncells++;
}

/* Leaf rule (reading): a cell splits iff it holds more than ncrit bodies and
   its level is below 21; children exist only for non-empty octants. */
static void build_cell(oplan *P, int64_t ci) {
    ocell c = P->cells[ci];
    for (int o = 0; o < 8; ++o) P->cells[ci].child[o] = -1;
    P->cells[ci].nchild = 0;
    if (!(c.count > P->ncrit && c.level < ORACLE_MAX_LEVEL)) return;
    int shift = 3 * (ORACLE_MAX_LEVEL - (c.level + 1));
    int64_t pos = c.start, end = c.start + c.count;
    for (int o = 0; o < 8; ++o) {
        uint64_t want = c.prefix * 8 + (uint64_t)o;
        int64_t s = pos;
        while (pos < end && (P->key[P->order[pos]] >> shift) == want) ++pos;
        if (pos > s) {
            int64_t ch = new_cell(P);
            ocell *cc = &P->cells[ch];
            cc->level = c.level + 1;
            cc->prefix = want;
            cc->start = s;
            cc->count = pos - s;
            cc->parent = ci;
            P->cells[ci].child[o] = ch;
            P->cells[ci].nchild++;
        }
    }
    for (int o = 0; o < 8; ++o) {
        int64_t ch = P->cells[ci].child[o];
        if (ch >= 0) build_cell(P, ch);
    }
}

static inline int is_leaf(const ocell *c) { return c->nchild == 0; }

static void push_pair(int64_t **arr, int64_t *n, int64_t *cap, int64_t a, int64_t b) {
    if (*n == *cap) {
        *cap = *cap ? 2 * *cap : 4096;
        *arr = (int64_t *)realloc(*arr, sizeof(int64_t) * 2 * *cap);
    }
    (*arr)[2 * *n] = a;
    (*arr)[2 * *n + 1] = b;
    ++*n;
}

/*
 * MAC (reading of Sec. 2.2's "multipole acceptance criterion"):
 *   accept A <- B  iff  A != B  and  theta * |c_A - c_B| >= R_A + R_B,
 * R = half the box side, evaluated exactly: centres and radii are integers in
 * units of the finer box's half side; theta^2 |dc|^2 >= (R_A+R_B)^2 is then
 * a comparison of an exact integer times the double theta*theta.
 */
static int mac_accept(const oplan *P, const ocell *A, const ocell *B, double theta2) {
    int lf = A->level > B->level ? A->level : B->level;
    uint64_t ia[3], ib[3];
    prefix_coords(A->prefix, A->level, ia);
    prefix_coords(B->prefix, B->level, ib);
    int64_t sa = (int64_t)1 << (lf - A->level), sb = (int64_t)1 << (lf - B->level);
    int64_t d2 = 0;
    for (int a = 0; a < 3; ++a) {
        int64_t ca = (2 * (int64_t)ia[a] + 1) * sa;
        int64_t cb = (2 * (int64_t)ib[a] + 1) * sb;
        d2 += (ca - cb) * (ca - cb);
    }
    int64_t s = sa + sb;
    return theta2 * (double)d2 >= (double)(s * s);
    (void)P;
}

/*
 * Dual tree traversal (Sec. 2.2, after Dehnen 2002).  From (root, root):
 *   1. A != B and the MAC holds          -> M2L(A <- B)
 *   2. else both leaves                  -> P2P(A <- B)   (includes A == B)
 *   3. else both non-leaves, same level  -> all child pairs (a, b)
 *   4. else split the coarser cell (lower level; on a tie the non-leaf one)
 *      if it is not a leaf, otherwise the other one.
 * The rules do not depend on the order of A and B, so the lists are symmetric.
 *
 * Level-skip variant (lists = 1; the paper's remark that distant members of an
 * interaction list can be served by their parent): rule 3 splits only one of the two
 * cells, the one with the smaller Morton prefix, so that a target's children can take
 * the other cell's multipole whole when the MAC allows it.  The choice depends on the
 * unordered pair only, so the lists stay symmetric.
 */
static void traverse(oplan *P) {
    double theta2 = (double)P->theta * (double)P->theta;
    int64_t cap = 1024, top = 0;
    int64_t *stack = (int64_t *)malloc(sizeof(int64_t) * 2 * cap);
    stack[0] = 0; stack[1] = 0; top = 1;
    while (top > 0) {
        --top;
        int64_t ai = stack[2 * top], bi = stack[2 * top + 1];
        const ocell *A = &P->cells[ai], *B = &P->cells[bi];
        if (ai != bi && mac_accept(P, A, B, theta2)) {
            push_pair(&P->m2l, &P->nm2l, &P->m2l_cap, ai, bi);
            continue;
        }
        int la = is_leaf(A), lb = is_leaf(B);
        if (la && lb) {
            push_pair(&P->p2p, &P->np2p, &P->p2p_cap, ai, bi);
            continue;
        }
        /* children pairs to push */
        int64_t ca[8], cb[8];
        int na = 0, nb = 0;
        if (!la && !lb && A->level == B->level && P->lists == 0) {
            for (int o = 0; o < 8; ++o) if (A->child[o] >= 0) ca[na++] = A->child[o];
            for (int o = 0; o < 8; ++o) if (B->child[o] >= 0) cb[nb++] = B->child[o];
        } else if (!la && !lb && A->level == B->level) {
            if (A->prefix <= B->prefix) {
                for (int o = 0; o < 8; ++o) if (A->child[o] >= 0) ca[na++] = A->child[o];
                cb[0] = bi; nb = 1;
            } else {
                ca[0] = ai; na = 1;
                for (int o = 0; o < 8; ++o) if (B->child[o] >= 0) cb[nb++] = B->child[o];
            }
        } else {
            int splitA;
            if (A->level < B->level) splitA = !la;
            else if (B->level < A->level) splitA = lb;     /* coarser is B: split B unless it is a leaf */
            else splitA = !la;                              /* same level, exactly one non-leaf */
            if (splitA) {
                for (int o = 0; o < 8; ++o) if (A->child[o] >= 0) ca[na++] = A->child[o];
                cb[0] = bi; nb = 1;
            } else {
                ca[0] = ai; na = 1;
                for (int o = 0; o < 8; ++o) if (B->child[o] >= 0) cb[nb++] = B->child[o];
            }
        }
        /* push in reverse so that pairs pop in (a, b) order (cosmetic only) */
        for (int x = na - 1; x >= 0; --x)
            for (int y = nb - 1; y >= 0; --y) {
                if (top == cap) {
                    cap *= 2;
                    stack = (int64_t *)realloc(stack, sizeof(int64_t) * 2 * cap);
                }
                stack[2 * top] = ca[x];
                stack[2 * top + 1] = cb[y];
                ++top;
            }
    }
    free(stack);
}

/* Returns NULL on invalid arguments. pts is [n][3] doubles (FP32 values). */
void *oracle_plan_create(int64_t n, const double *pts, int ncrit, float theta, int lists) {
    if (n < 1 || ncrit < 1 || !(theta > 0.0f) || lists < 0 || lists > 1) return NULL;
    oplan *P = (oplan *)calloc(1, sizeof(oplan));
    P->n = n;
    P->ncrit = ncrit;
    P->theta = theta;
    P->lists = lists;
    P->pts = (double *)malloc(sizeof(double) * 3 * n);
    memcpy(P->pts, pts, sizeof(double) * 3 * n);
    root_cube(n, P->pts, &P->k, P->x0);
    P->key = (uint64_t *)malloc(sizeof(uint64_t) * n);
    for (int64_t i = 0; i < n; ++i)
        P->key[i] = morton(axis_coord(P->pts[3 * i], P->x0[0], P->k),
                           axis_coord(P->pts[3 * i + 1], P->x0[1], P->k),
                           axis_coord(P->pts[3 * i + 2], P->x0[2], P->k));
    P->order = (int64_t *)malloc(sizeof(int64_t) * n);
    for (int64_t i = 0; i < n; ++i) P->order[i] = i;
    g_sort_keys = P->key;
    qsort(P->order, (size_t)n, sizeof(int64_t), cmp_key_index);   /* ties by input index */
    int64_t r = new_cell(P);
    P->cells[r].level = 0;
    P->cells[r].prefix = 0;
    P->cells[r].start = 0;
    P->cells[r].count = n;
    P->cells[r].parent = -1;
    build_cell(P, r);
    traverse(P);
    return P;
}

void oracle_plan_destroy(void *h) {
    oplan *P = (oplan *)h;
    if (!P) return;
    free(P->pts); free(P->key); free(P->order); free(P->cells);
    free(P->m2l); free(P->p2p);
    free(P);
}

/* counts[0..4] = ncells, nm2l, np2p, k, nleaves */
void oracle_plan_counts(void *h, int64_t *counts) {
    oplan *P = (oplan *)h;
    int64_t nl = 0;
    for (int64_t c = 0; c < P->ncells; ++c) nl += is_leaf(&P->cells[c]);
    counts[0] = P->ncells; counts[1] = P->nm2l; counts[2] = P->np2p; counts[3] = P->k; counts[4] = nl;
}

void oracle_plan_root(void *h, double x0[3]) {
    oplan *P = (oplan *)h;
    x0[0] = P->x0[0]; x0[1] = P->x0[1]; x0[2] = P->x0[2];
}

/* cells: level[nc], prefix[nc], start[nc], count[nc], parent[nc], leaf[nc] */
void oracle_plan_cells(void *h, int32_t *level, uint64_t *prefix, int64_t *start, int64_t *count,
                       int64_t *parent, int32_t *leaf) {
    oplan *P = (oplan *)h;
    for (int64_t c = 0; c < P->ncells; ++c) {
        level[c] = P->cells[c].level;
        prefix[c] = P->cells[c].prefix;
        start[c] = P->cells[c].start;
        count[c] = P->cells[c].count;
        parent[c] = P->cells[c].parent;
        leaf[c] = is_leaf(&P->cells[c]);
    }
}

void oracle_plan_pairs(void *h, int64_t *m2l, int64_t *p2p) {
    oplan *P = (oplan *)h;
    if (m2l) memcpy(m2l, P->m2l, sizeof(int64_t) * 2 * P->nm2l);
    if (p2p) memcpy(p2p, P->p2p, sizeof(int64_t) * 2 * P->np2p);
}

/* sorted position -> input index; keys in input order */
void oracle_plan_order(void *h, int64_t *order, uint64_t *keys) {
    oplan *P = (oplan *)h;
    if (order) memcpy(order, P->order, sizeof(int64_t) * P->n);
    if (keys) memcpy(keys, P->key, sizeof(uint64_t) * P->n);
}

/* ------------------------------------------------------------------------ */
/* FMM evaluation                                                            */
/* ------------------------------------------------------------------------ */
/* CSR of pairs grouped by target. */
static void group_by_target(int64_t ncell, const int64_t *pairs, int64_t np, int64_t **off_out, int64_t **src_out) {
    int64_t *off = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    for (int64_t i = 0; i < np; ++i) off[pairs[2 * i] + 1]++;
    for (int64_t c = 0; c < ncell; ++c) off[c + 1] += off[c];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (ncell + 1));
    memcpy(fill, off, sizeof(int64_t) * (ncell + 1));
    int64_t *src = (int64_t *)malloc(sizeof(int64_t) * (np ? np : 1));
    for (int64_t i = 0; i < np; ++i) src[fill[pairs[2 * i]]++] = pairs[2 * i + 1];
    free(fill);
    *off_out = off;
    *src_out = src;
}

/*
 * mode bit 0: near field (P2P), bit 1: far field (P2M..L2P).
 * nsample > 0: only targets sample[0..nsample) (input indices) are evaluated
 * (the far field is then computed only into the ancestors of their leaves);
 * phi / grad are [nsample] / [nsample][3].  nsample == 0: all targets, in
 * input order, phi [n], grad [n][3].  Charges q are in input order.
 * timing (nullable) receives seconds: [upward, m2l, downward+l2p, p2p].
 */
static void fmm_eval_impl(void *h, int p, const double *q, const double *dip, int mode, int64_t nsample,
                          const int64_t *sample, double *phi, double *grad, double *hess, double *timing) {
    oplan *P = (oplan *)h;
    int64_t nc = P->ncells, n = P->n;
    expctx e;
    exp_init(&e, p);
    int nk = e.mp.n;
    double t0 = 0, t1 = 0, t2 = 0, t3 = 0, t4 = 0;
#ifdef _OPENMP
    t0 = omp_get_wtime();
#endif
    /* leaf of every sorted position, and the sorted position of every input index */
    int64_t *leaf_of = (int64_t *)malloc(sizeof(int64_t) * n);
    int64_t *pos_of = (int64_t *)malloc(sizeof(int64_t) * n);
    for (int64_t c = 0; c < nc; ++c)
        if (is_leaf(&P->cells[c]))
            for (int64_t s = P->cells[c].start; s < P->cells[c].start + P->cells[c].count; ++s) leaf_of[s] = c;
    for (int64_t s = 0; s < n; ++s) pos_of[P->order[s]] = s;

    /* targets to evaluate: sorted positions */
    int64_t nt = nsample > 0 ? nsample : n;
    int64_t *tpos = (int64_t *)malloc(sizeof(int64_t) * nt);
    for (int64_t t = 0; t < nt; ++t) tpos[t] = nsample > 0 ? pos_of[sample[t]] : pos_of[t];

    /* cells whose local expansion is needed */
    char *need = (char *)calloc((size_t)nc, 1);
    for (int64_t t = 0; t < nt; ++t) {
        int64_t c = leaf_of[tpos[t]];
        while (c >= 0 && !need[c]) { need[c] = 1; c = P->cells[c].parent; }
    }

    /* bodies in sorted order */
    double *sp = (double *)malloc(sizeof(double) * 3 * n);
    double *sq = (double *)malloc(sizeof(double) * n);
    double *sd = dip ? (double *)malloc(sizeof(double) * 3 * n) : NULL;
    for (int64_t s = 0; s < n; ++s) {
        int64_t i = P->order[s];
        sp[3 * s] = P->pts[3 * i]; sp[3 * s + 1] = P->pts[3 * i + 1]; sp[3 * s + 2] = P->pts[3 * i + 2];
        sq[s] = q[i];
        if (sd) { sd[3 * s] = dip[3 * i]; sd[3 * s + 1] = dip[3 * i + 1]; sd[3 * s + 2] = dip[3 * i + 2]; }
    }
    double *ctr = (double *)malloc(sizeof(double) * 3 * nc);
    for (int64_t c = 0; c < nc; ++c) cell_center(P, &P->cells[c], ctr + 3 * c);

    double *ophi = (double *)calloc((size_t)nt, sizeof(double));
    double *ograd = (double *)calloc((size_t)nt * 3, sizeof(double));
    double *ohess = hess ? (double *)calloc((size_t)nt * 6, sizeof(double)) : NULL;

    int maxlev = 0;
    for (int64_t c = 0; c < nc; ++c) if (P->cells[c].level > maxlev) maxlev = P->cells[c].level;

    if (mode & 2) {
        double *M = (double *)calloc((size_t)nc * nk, sizeof(double));
        double *L = (double *)calloc((size_t)nc * nk, sizeof(double));
        /* upward pass: P2M at leaves, then M2M level by level, deepest first */
        for (int lev = maxlev; lev >= 0; --lev) {
#pragma omp parallel for schedule(dynamic, 4)
            for (int64_t c = 0; c < nc; ++c) {
                const ocell *C = &P->cells[c];
                if (C->level != lev) continue;
                if (is_leaf(C)) {
                    p2m_acc(&e, C->count, sp + 3 * C->start, sq + C->start, ctr + 3 * c, M + (size_t)c * nk);
                    if (sd) p2m_dip_acc(&e, C->count, sp + 3 * C->start, sd + 3 * C->start, ctr + 3 * c, M + (size_t)c * nk);
                } else {
                    for (int o = 0; o < 8; ++o) {
                        int64_t ch = C->child[o];
                        if (ch < 0) continue;
                        double d[3] = {ctr[3 * ch] - ctr[3 * c], ctr[3 * ch + 1] - ctr[3 * c + 1],
                                       ctr[3 * ch + 2] - ctr[3 * c + 2]};
                        m2m_acc(&e, M + (size_t)ch * nk, d, M + (size_t)c * nk);
                    }
                }
            }
        }
#ifdef _OPENMP
        t1 = omp_get_wtime();
#endif
        /* M2L into every needed target cell */
        int64_t *off, *src;
        group_by_target(nc, P->m2l, P->nm2l, &off, &src);
#pragma omp parallel
        {
            double *T = (double *)malloc(sizeof(double) * e.m2p.n);
#pragma omp for schedule(dynamic, 1)
            for (int64_t c = 0; c < nc; ++c) {
                if (!need[c]) continue;
                for (int64_t k = off[c]; k < off[c + 1]; ++k) {
                    int64_t b = src[k];
                    double D[3] = {ctr[3 * c] - ctr[3 * b], ctr[3 * c + 1] - ctr[3 * b + 1],
                                   ctr[3 * c + 2] - ctr[3 * b + 2]};
                    m2l_acc(&e, M + (size_t)b * nk, D, L + (size_t)c * nk, T);
                }
            }
            free(T);
        }
        free(off); free(src);
#ifdef _OPENMP
        t2 = omp_get_wtime();
#endif
        /* downward pass: L2L level by level from the root */
        for (int lev = 1; lev <= maxlev; ++lev) {
#pragma omp parallel for schedule(dynamic, 4)
            for (int64_t c = 0; c < nc; ++c) {
                const ocell *C = &P->cells[c];
                if (C->level != lev || !need[c]) continue;
                int64_t par = C->parent;
                double d[3] = {ctr[3 * c] - ctr[3 * par], ctr[3 * c + 1] - ctr[3 * par + 1],
                               ctr[3 * c + 2] - ctr[3 * par + 2]};
                l2l_acc(&e, L + (size_t)par * nk, d, L + (size_t)c * nk);
            }
        }
        /* L2P */
#pragma omp parallel for schedule(static)
        for (int64_t t = 0; t < nt; ++t) {
            int64_t s = tpos[t];
            int64_t c = leaf_of[s];
            l2p_one_h(&e, L + (size_t)c * nk, ctr + 3 * c, sp + 3 * s, ophi + t, ograd + 3 * t,
                      ohess ? ohess + 6 * t : NULL);
        }
        free(M); free(L);
#ifdef _OPENMP
        t3 = omp_get_wtime();
#endif
    } else {
        t1 = t2 = t3 = t0;
    }
    if (mode & 1) {
        int64_t *off, *src;
        group_by_target(nc, P->p2p, P->np2p, &off, &src);
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t t = 0; t < nt; ++t) {
            int64_t s = tpos[t];
            int64_t c = leaf_of[s];
            double xi = sp[3 * s], yi = sp[3 * s + 1], zi = sp[3 * s + 2];
            double f = 0, gx = 0, gy = 0, gz = 0, hh[6] = {0, 0, 0, 0, 0, 0};
            for (int64_t k = off[c]; k < off[c + 1]; ++k) {
                const ocell *B = &P->cells[src[k]];
                for (int64_t j = B->start; j < B->start + B->count; ++j) {
                    if (j == s) continue;
                    double dx = xi - sp[3 * j], dy = yi - sp[3 * j + 1], dz = zi - sp[3 * j + 2];
                    double r2 = dx * dx + dy * dy + dz * dz;
                    if (r2 == 0.0) continue;
                    double r = sqrt(r2);
                    double v = sq[j] / r, w = v / r2;
                    f += v; gx -= w * dx; gy -= w * dy; gz -= w * dz;
                    if (sd) {   /* dipole g_j: g.d / r^3, gradient g / r^3 - 3 (g.d) d / r^5 */
                        const double *g = sd + 3 * j;
                        double r3 = r2 * r, gd = g[0] * dx + g[1] * dy + g[2] * dz;
                        f += gd / r3;
                        gx += g[0] / r3 - 3.0 * gd * dx / (r3 * r2);
                        gy += g[1] / r3 - 3.0 * gd * dy / (r3 * r2);
                        gz += g[2] / r3 - 3.0 * gd * dz / (r3 * r2);
                    }
                    if (ohess) {
                        double w5 = 3.0 * w / r2;      /* 3 q / r^5 */
                        hh[0] += w5 * dx * dx - w; hh[1] += w5 * dy * dy - w; hh[2] += w5 * dz * dz - w;
                        hh[3] += w5 * dx * dy; hh[4] += w5 * dx * dz; hh[5] += w5 * dy * dz;
                    }
                }
            }
            ophi[t] += f; ograd[3 * t] += gx; ograd[3 * t + 1] += gy; ograd[3 * t + 2] += gz;
            if (ohess) for (int a = 0; a < 6; ++a) ohess[6 * t + a] += hh[a];
        }
        free(off); free(src);
    }
#ifdef _OPENMP
    t4 = omp_get_wtime();
#endif
    for (int64_t t = 0; t < nt; ++t) {
        phi[t] = ophi[t];
        if (grad) { grad[3 * t] = ograd[3 * t]; grad[3 * t + 1] = ograd[3 * t + 1]; grad[3 * t + 2] = ograd[3 * t + 2]; }
        if (hess) for (int a = 0; a < 6; ++a) hess[6 * t + a] = ohess[6 * t + a];
    }
    if (timing) {
        timing[0] = t1 - t0;
        timing[1] = t2 - t1;
        timing[2] = t3 - t2;
        timing[3] = t4 - t3;
    }
    free(ophi); free(ograd); free(ohess); free(ctr); free(sp); free(sq); free(sd); free(need); free(tpos); free(leaf_of);
    free(pos_of);
    exp_free(&e);
}

void oracle_fmm_eval(void *h, int p, const double *q, int mode, int64_t nsample, const int64_t *sample,
                     double *phi, double *grad, double *hess, double *timing) {
    fmm_eval_impl(h, p, q, NULL, mode, nsample, sample, phi, grad, hess, timing);
}

/* The same with dipoles dip [n][3] (input order) beside the charges: P2M adds each
   dipole's multipole (p2m_dip_acc), P2P its exact field; no Hessian. */
void oracle_fmm_eval_dip(void *h, int p, const double *q, const double *dip, int mode, int64_t nsample,
                         const int64_t *sample, double *phi, double *grad, double *timing) {
    fmm_eval_impl(h, p, q, dip, mode, nsample, sample, phi, grad, NULL, timing);
}
