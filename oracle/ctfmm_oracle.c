/*
 * ctfmm_oracle.c -- plain, slow FP64 CPU reference for the Cartesian
 * traceless fast multipole method of Coles & Bieri, "An Optimizing Symbolic
 * Algebra Approach for Generating Fast Multipole Method Operators"
 * (arXiv 1811.06332).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may use it.  It shares no code, header, table or
 * generator with the GPU path.
 *
 * Every tensor here is kept in FULL symmetric storage: all C(p+3,3)
 * multi-index components (nx,ny,nz), |n| <= p, are computed and stored,
 * dependent (trace-determined) components included.  No trace relation and
 * no reduced basis is used; the operators are the equations written out:
 *
 *   detracer T, D = T/(2n-1)!!          Appendix A, Eq. (Detracer)
 *   traceless gradient D_k(r)           Appendix A, Eq. (traceless grad),
 *                                       compact form Eq. (Detracer3)
 *   P2M  M'_n = sum_a q_a (-r_a)^n, M = D[M']        Sec. 2.1, Eq. (P2M)
 *   M2M  M'_n = sum_{k<=n} n!/(k!(n-k)!) (-d)^(n-k) M_k, then D
 *                                       Sec. 2.1, Eq. (M2M), (M2M part 2)
 *   M2L  L_n += sum_{|m|<=p-|n|} M_m D_{n+m}(r) / m!  Sec. 2.1, Eq. (M2L)
 *   L2L  L_n  = sum_{|k|<=p-|n|} d^k/k! L_{n+k}       Sec. 2.1, Eq. (L2L)
 *   L2P  grad^n Phi(x_b) ~ shifted L_n                 Sec. 2.1, Eq. (L2P)
 *   P2P  Phi_b = sum_a q_a/|x_b-x_a|                   Appendix B, Eq. (PhiAB)
 *
 * Readings taken where the text is ambiguous (all multi-index factorials
 * are componentwise, n! = nx! ny! nz!):
 *   - P2M's "-r_a^n" is (-r_a)^n, so a positive charge has a positive
 *     monopole and a positive potential (Sec. 2.1 says the potential is
 *     positive).
 *   - The M2M sum "|k| <= n" runs over k <= n componentwise (indices with
 *     negative components vanish, Appendix D).
 *   - M2L truncates at total degree |n|+|m| <= p.
 *   - Self pairs are excluded and coincident pairs contribute nothing.
 *
 * The tree is a uniform octree over a cube (the configurations name
 * octrees; the paper's binary median tree is not used), expansion centres
 * at geometric cell centres (Appendix C).  Interaction lists are the
 * ws=1 ("non-adjacent") rule: at each level l >= 2, a cell B receives M2L
 * from every same-level cell A whose parent is adjacent to or equal to
 * B's parent while A itself is not adjacent to or equal to B.  Adjacent
 * leaves (and the leaf itself) form the near field (Appendix C).
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC (no intrinsics, no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PMAX 16

/* ---------------------------------------------------------------- indices */

static int g_ready = 0;
static int g_nfull[OR_PMAX + 2];               /* C(p+3,3): components with rank <= p */
static int g_idx[OR_PMAX + 1][OR_PMAX + 1][OR_PMAX + 1];
static int g_ix[1000], g_iy[1000], g_iz[1000]; /* inverse map, C(19,3)=969 */
/* n! for 0 <= n <= 3*OR_PMAX+1, tabulated once (exact in FP64 below 23!) */
static double g_fact[3 * OR_PMAX + 2];
static double fact(int n) { return g_fact[n]; }
/* f_{n,m} of the detracer, tabulated once per (component of n, m) */
static double g_f[969][OR_PMAX / 2 + 1][OR_PMAX / 2 + 1][OR_PMAX / 2 + 1];
static double f_nm_eval(int n1, int n2, int n3, int m1, int m2, int m3);

static void init_tables(void)
{
    if (g_ready) return;
    g_fact[0] = 1.0;
    for (int i = 1; i <= 3 * OR_PMAX + 1; ++i) g_fact[i] = g_fact[i - 1] * (double)i;
    int c = 0;
    for (int n = 0; n <= OR_PMAX; ++n) {
        for (int a = n; a >= 0; --a)
            for (int b = n - a; b >= 0; --b) {
                int z = n - a - b;
                g_idx[a][b][z] = c;
                g_ix[c] = a; g_iy[c] = b; g_iz[c] = z;
                ++c;
            }
        g_nfull[n] = c;
    }
    for (int e = 0; e < c; ++e)
        for (int m1 = 0; 2 * m1 <= g_ix[e]; ++m1)
            for (int m2 = 0; 2 * m2 <= g_iy[e]; ++m2)
                for (int m3 = 0; 2 * m3 <= g_iz[e]; ++m3)
                    g_f[e][m1][m2][m3] = f_nm_eval(g_ix[e], g_iy[e], g_iz[e], m1, m2, m3);
    g_ready = 1;
}

/* number of full components of ranks 0..p (C(p+3,3)) */
int oracle_nfull(int p) { init_tables(); return (p < 0 || p > OR_PMAX) ? 0 : g_nfull[p]; }

/* linear position of (a,b,c) in full storage (rank-major, a then b descending) */
int oracle_full_index(int a, int b, int c)
{
    init_tables();
    if (a < 0 || b < 0 || c < 0 || a + b + c > OR_PMAX) return -1;
    return g_idx[a][b][c];
}

/* double factorial, with (-1)!! = 1 */
static double dfact(int n) { double f = 1.0; for (int i = n; i > 1; i -= 2) f *= i; return f; }

static double mfact(int a, int b, int c) { return fact(a) * fact(b) * fact(c); }

static double ipow(double x, int e) { double r = 1.0; for (int i = 0; i < e; ++i) r *= x; return r; }

/* ---------------------------------------------------------------- detracer */

/*
 * f_{n,m} = (-1)^m (2n-2m-1)!! n! / (2^m m! (n-2m)!)   (Appendix A)
 * with n = (n1,n2,n3), m = (m1,m2,m3), n = |n|, m = |m|, bold factorials.
 */
static double f_nm_eval(int n1, int n2, int n3, int m1, int m2, int m3)
{
    int n = n1 + n2 + n3, m = m1 + m2 + m3;
    double s = (m & 1) ? -1.0 : 1.0;
    return s * dfact(2 * n - 2 * m - 1) * mfact(n1, n2, n3)
           / (ipow(2.0, m) * mfact(m1, m2, m3) * mfact(n1 - 2 * m1, n2 - 2 * m2, n3 - 2 * m3));
}

static double f_nm(int n1, int n2, int n3, int m1, int m2, int m3)
{
    return g_f[g_idx[n1][n2][n3]][m1][m2][m3];
}

/*
 * T[A^(n)]_n = sum_{m <= floor(n/2)} f_{n,m} sum_{|k|=m} (m!/k!) A_{n-2m+2k}
 * (Appendix A, Eq. Detracer), applied to the rank-|n| part of A.
 */
static double detracer_T_component(const double *A, int n1, int n2, int n3)
{
    double t = 0.0;
    for (int m1 = 0; 2 * m1 <= n1; ++m1)
        for (int m2 = 0; 2 * m2 <= n2; ++m2)
            for (int m3 = 0; 2 * m3 <= n3; ++m3) {
                int m = m1 + m2 + m3;
                double inner = 0.0;
                for (int k1 = 0; k1 <= m; ++k1)
                    for (int k2 = 0; k2 <= m - k1; ++k2) {
                        int k3 = m - k1 - k2;
                        inner += fact(m) / mfact(k1, k2, k3)
                                 * A[g_idx[n1 - 2 * m1 + 2 * k1][n2 - 2 * m2 + 2 * k2][n3 - 2 * m3 + 2 * k3]];
                    }
                t += f_nm(n1, n2, n3, m1, m2, m3) * inner;
            }
    return t;
}

/* out = T[A] rank by rank (full storage, ranks 0..p) */
void oracle_detracer_T(int p, const double *A, double *out)
{
    init_tables();
    for (int c = 0; c < g_nfull[p]; ++c)
        out[c] = detracer_T_component(A, g_ix[c], g_iy[c], g_iz[c]);
}

/* out = D[A] = T[A]/(2n-1)!! rank by rank (Appendix A) */
void oracle_detracer_D(int p, const double *A, double *out)
{
    init_tables();
    for (int c = 0; c < g_nfull[p]; ++c) {
        int n = g_ix[c] + g_iy[c] + g_iz[c];
        out[c] = detracer_T_component(A, g_ix[c], g_iy[c], g_iz[c]) / dfact(2 * n - 1);
    }
}

/* ------------------------------------------------------ traceless gradient */

/*
 * D_k(r) = grad^k (1/|r|) = (-1)^k |r|^{-2k-1} T[r^k]_k   (Eq. traceless grad)
 * T[r^k]_k = sum_{m <= floor(k/2)} f_{k,m} |r|^{2m} r^{k-2m}  (Eq. Detracer3)
 */
void oracle_dtensor(int p, const double r[3], double *D)
{
    init_tables();
    double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double rn = sqrt(r2);
    for (int c = 0; c < g_nfull[p]; ++c) {
        int k1 = g_ix[c], k2 = g_iy[c], k3 = g_iz[c], k = k1 + k2 + k3;
        double t = 0.0;
        for (int m1 = 0; 2 * m1 <= k1; ++m1)
            for (int m2 = 0; 2 * m2 <= k2; ++m2)
                for (int m3 = 0; 2 * m3 <= k3; ++m3) {
                    int m = m1 + m2 + m3;
                    t += f_nm(k1, k2, k3, m1, m2, m3) * ipow(r2, m)
                         * ipow(r[0], k1 - 2 * m1) * ipow(r[1], k2 - 2 * m2) * ipow(r[2], k3 - 2 * m3);
                }
        double sgn = (k & 1) ? -1.0 : 1.0;
        D[c] = sgn * t / ipow(rn, 2 * k + 1);
    }
}

/* --------------------------------------------------------------- operators */

/* P2M (Eq. P2M): M = sum_a q_a D[(-r_a)^n], r_a = x_a - z.  M is ADDED to. */
void oracle_p2m(int p, const double z[3], int64_t n, const double *xyz, const double *q, double *M)
{
    init_tables();
    int nf = g_nfull[p];
    double *Mp = (double *)calloc((size_t)nf, sizeof(double));
    double *Mt = (double *)malloc((size_t)nf * sizeof(double));
    for (int64_t a = 0; a < n; ++a) {
        double rx = -(xyz[3 * a + 0] - z[0]);
        double ry = -(xyz[3 * a + 1] - z[1]);
        double rz = -(xyz[3 * a + 2] - z[2]);
        for (int c = 0; c < nf; ++c)
            Mp[c] += q[a] * ipow(rx, g_ix[c]) * ipow(ry, g_iy[c]) * ipow(rz, g_iz[c]);
    }
    oracle_detracer_D(p, Mp, Mt);
    for (int c = 0; c < nf; ++c) M[c] += Mt[c];
    free(Mp);
    free(Mt);
}

/*
 * P2M of point dipoles (Appendix B.1): each dipole p_a is a pure dipole at
 * its own position x_a -- rank-1 components M'_{e_i} = -p_{a,i} (so that
 * the expansion's potential is -p_a . grad (1/|x - x_a|)), every other
 * component zero -- moved to the centre z by Eq. M2M (d = x_a - z).  M is
 * ADDED to.
 */
void oracle_m2m(int p, const double d[3], const double *Min, double *Mout);

void oracle_p2m_dipole(int p, const double z[3], int64_t n, const double *xyz, const double *dip, double *M)
{
    init_tables();
    int nf = g_nfull[p];
    double *Md = (double *)calloc((size_t)nf, sizeof(double));
    for (int64_t a = 0; a < n; ++a) {
        memset(Md, 0, (size_t)nf * sizeof(double));
        if (p >= 1) {
            Md[g_idx[1][0][0]] = -dip[3 * a + 0];
            Md[g_idx[0][1][0]] = -dip[3 * a + 1];
            Md[g_idx[0][0][1]] = -dip[3 * a + 2];
        }
        double d[3] = {xyz[3 * a] - z[0], xyz[3 * a + 1] - z[1], xyz[3 * a + 2] - z[2]};
        oracle_m2m(p, d, Md, M);
    }
    free(Md);
}

/*
 * M2M (Eq. M2M, M2M part 2): move the expansion from centre z to z' = z - d,
 * i.e. d = z_child - z_parent.  M'_n = sum_{k<=n} n!/(k!(n-k)!) (-d)^(n-k) M_k,
 * then Mout += D[M'].
 */
void oracle_m2m(int p, const double d[3], const double *Min, double *Mout)
{
    init_tables();
    int nf = g_nfull[p];
    double *Mp = (double *)calloc((size_t)nf, sizeof(double));
    double *Mt = (double *)malloc((size_t)nf * sizeof(double));
    for (int c = 0; c < nf; ++c) {
        int n1 = g_ix[c], n2 = g_iy[c], n3 = g_iz[c];
        double s = 0.0;
        for (int k1 = 0; k1 <= n1; ++k1)
            for (int k2 = 0; k2 <= n2; ++k2)
                for (int k3 = 0; k3 <= n3; ++k3) {
                    double w = mfact(n1, n2, n3) / (mfact(k1, k2, k3) * mfact(n1 - k1, n2 - k2, n3 - k3));
                    s += w * ipow(-d[0], n1 - k1) * ipow(-d[1], n2 - k2) * ipow(-d[2], n3 - k3)
                         * Min[g_idx[k1][k2][k3]];
                }
        Mp[c] = s;
    }
    oracle_detracer_D(p, Mp, Mt);
    for (int c = 0; c < nf; ++c) Mout[c] += Mt[c];
    free(Mp);
    free(Mt);
}

/* M2L with a given derivative tensor D (full storage to rank p):
 * L_n += sum_{|m| <= p-|n|} M_m D_{n+m} / m!   (Eq. M2L) */
void oracle_m2l_with_D(int p, const double *M, const double *D, double *L)
{
    init_tables();
    for (int c = 0; c < g_nfull[p]; ++c) {
        int n1 = g_ix[c], n2 = g_iy[c], n3 = g_iz[c], n = n1 + n2 + n3;
        double s = 0.0;
        for (int e = 0; e < g_nfull[p - n]; ++e) {
            int m1 = g_ix[e], m2 = g_iy[e], m3 = g_iz[e];
            s += M[e] * D[g_idx[n1 + m1][n2 + m2][n3 + m3]] / mfact(m1, m2, m3);
        }
        L[c] += s;
    }
}

/* M2L (Eq. M2L) for r = z_B - z_A; L is ADDED to. */
void oracle_m2l(int p, const double r[3], const double *M, double *L)
{
    init_tables();
    double *D = (double *)malloc((size_t)g_nfull[p] * sizeof(double));
    oracle_dtensor(p, r, D);
    oracle_m2l_with_D(p, M, D, L);
    free(D);
}

/* L2L (Eq. L2L): L at z' = z + d from L at z; Lout is ADDED to. */
void oracle_l2l(int p, const double d[3], const double *Lin, double *Lout)
{
    init_tables();
    for (int c = 0; c < g_nfull[p]; ++c) {
        int n1 = g_ix[c], n2 = g_iy[c], n3 = g_iz[c], n = n1 + n2 + n3;
        double s = 0.0;
        for (int e = 0; e < g_nfull[p - n]; ++e) {
            int k1 = g_ix[e], k2 = g_iy[e], k3 = g_iz[e];
            s += ipow(d[0], k1) * ipow(d[1], k2) * ipow(d[2], k3) / mfact(k1, k2, k3)
                 * Lin[g_idx[n1 + k1][n2 + k2][n3 + k3]];
        }
        Lout[c] += s;
    }
}

/*
 * L2P (Eq. L2P): shift L to the particle offset rb = x_b - z_B and read the
 * rank-0 (potential) and rank-1 (gradient) components:
 *   Phi = sum_{|n|<=p} rb^n/n! L_n,  dPhi/dx_i = sum_{|n|<=p-1} rb^n/n! L_{n+e_i}.
 * Results are ADDED to phi[0] and grad[0..2].
 */
void oracle_l2p(int p, const double rb[3], const double *L, double *phi, double *grad)
{
    init_tables();
    double f = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    for (int c = 0; c < g_nfull[p]; ++c) {
        int n1 = g_ix[c], n2 = g_iy[c], n3 = g_iz[c], n = n1 + n2 + n3;
        double w = ipow(rb[0], n1) * ipow(rb[1], n2) * ipow(rb[2], n3) / mfact(n1, n2, n3);
        f += w * L[c];
        if (n <= p - 1) {
            gx += w * L[g_idx[n1 + 1][n2][n3]];
            gy += w * L[g_idx[n1][n2 + 1][n3]];
            gz += w * L[g_idx[n1][n2][n3 + 1]];
        }
    }
    phi[0] += f;
    grad[0] += gx;
    grad[1] += gy;
    grad[2] += gz;
}

/* one source on one target: q/|x_b-x_a| and its gradient w.r.t. x_b */
static void pair_kernel(const double *xb, const double *xa, double qa, double *phi, double *grad)
{
    double dx = xb[0] - xa[0], dy = xb[1] - xa[1], dz = xb[2] - xa[2];
    double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 == 0.0) return; /* coincident pair: contributes nothing */
    double r = sqrt(r2);
    double ir = 1.0 / r;
    phi[0] += qa * ir;
    double ir3 = qa * ir * ir * ir;
    grad[0] -= ir3 * dx;
    grad[1] -= ir3 * dy;
    grad[2] -= ir3 * dz;
}

/*
 * One point dipole p_a at x_a on a target at x_b (Appendix B.1: the limit of
 * charges +s at x_a + d/2 and -s at x_a - d/2 with s d = p_a): potential
 * p_a.(x_b - x_a)/|x_b - x_a|^3 and its gradient with respect to x_b,
 * p_a/|r|^3 - 3 (p_a.r) r/|r|^5.  Coincident: nothing.
 */
static void pair_kernel_dipole(const double *xb, const double *xa, const double *pa, double *phi, double *grad)
{
    double dx = xb[0] - xa[0], dy = xb[1] - xa[1], dz = xb[2] - xa[2];
    double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 == 0.0) return;
    double ir = 1.0 / sqrt(r2);
    double ir3 = ir * ir * ir, ir5 = ir3 * ir * ir;
    double pr = pa[0] * dx + pa[1] * dy + pa[2] * dz;
    phi[0] += pr * ir3;
    grad[0] += pa[0] * ir3 - 3.0 * pr * dx * ir5;
    grad[1] += pa[1] * ir3 - 3.0 * pr * dy * ir5;
    grad[2] += pa[2] * ir3 - 3.0 * pr * dz * ir5;
}

/* Direct sum over charges q and point dipoles dip ([n][3]) at the targets
 * tgt[0..nt) (NULL = all particles); self pairs skipped; overwritten. */
void oracle_direct_dipoles(int64_t n, const double *xyz, const double *q, const double *dip, int64_t nt,
                           const int64_t *tgt, double *phi, double *grad, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    if (!tgt) nt = n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t b = tgt ? tgt[t] : t;
        double f = 0.0, g[3] = {0.0, 0.0, 0.0};
        for (int64_t a = 0; a < n; ++a) {
            if (a == b) continue;
            pair_kernel(&xyz[3 * b], &xyz[3 * a], q[a], &f, g);
            pair_kernel_dipole(&xyz[3 * b], &xyz[3 * a], &dip[3 * a], &f, g);
        }
        phi[t] = f;
        grad[3 * t + 0] = g[0];
        grad[3 * t + 1] = g[1];
        grad[3 * t + 2] = g[2];
    }
}

/*
 * Direct O(N^2) sum (Eq. PhiAB) at the targets tgt[0..nt) (particle
 * indices; NULL = all particles).  Self pairs are skipped.
 * phi[nt], grad[3*nt] are overwritten.
 */
void oracle_direct(int64_t n, const double *xyz, const double *q, int64_t nt, const int64_t *tgt,
                   double *phi, double *grad, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    if (!tgt) nt = n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t b = tgt ? tgt[t] : t;
        double f = 0.0, g[3] = {0.0, 0.0, 0.0};
        for (int64_t a = 0; a < n; ++a) {
            if (a == b) continue;
            pair_kernel(&xyz[3 * b], &xyz[3 * a], q[a], &f, g);
        }
        phi[t] = f;
        grad[3 * t + 0] = g[0];
        grad[3 * t + 1] = g[1];
        grad[3 * t + 2] = g[2];
    }
}

/* ------------------------------------------------------------ uniform tree */

typedef struct {
    int p, depth, nf;
    double lo[3], side;
    int64_t n;
    const double *xyz, *q;
    const double *dip;  /* [n][3] point dipoles, or NULL */
    int64_t *leaf_of;   /* [n] linear leaf index (row-major, x fastest) */
    int64_t *start;     /* [nleaves+1] offsets into order */
    int64_t *order;     /* [n] particle indices grouped by leaf, input order within a leaf */
    double **M, **L;    /* per level l: (8^l) * nf, NULL for unused levels */
} otree;

static inline int64_t ncell1(int l) { return (int64_t)1 << l; }
static inline int64_t cell_id(int l, int64_t i, int64_t j, int64_t k) { return i + ncell1(l) * (j + ncell1(l) * k); }

static void cell_center(const otree *T, int l, int64_t i, int64_t j, int64_t k, double z[3])
{
    double h = T->side / (double)ncell1(l);
    z[0] = T->lo[0] + ((double)i + 0.5) * h;
    z[1] = T->lo[1] + ((double)j + 0.5) * h;
    z[2] = T->lo[2] + ((double)k + 0.5) * h;
}

/* leaf coordinate: floor((x - lo)/side * 2^d), clamped to [0, 2^d-1] */
static int64_t leaf_coord(double x, double lo, double side, int d)
{
    double s = floor((x - lo) / side * (double)ncell1(d));
    int64_t i = (int64_t)s;
    if (s < 0.0) i = 0;
    if (i > ncell1(d) - 1) i = ncell1(d) - 1;
    return i;
}

static int build_tree(otree *T)
{
    int d = T->depth;
    int64_t nl = ncell1(3 * d);
    T->leaf_of = (int64_t *)malloc((size_t)(T->n > 0 ? T->n : 1) * sizeof(int64_t));
    T->start = (int64_t *)calloc((size_t)nl + 1, sizeof(int64_t));
    T->order = (int64_t *)malloc((size_t)(T->n > 0 ? T->n : 1) * sizeof(int64_t));
    if (!T->leaf_of || !T->start || !T->order) return -1;
    for (int64_t a = 0; a < T->n; ++a) {
        int64_t i = leaf_coord(T->xyz[3 * a + 0], T->lo[0], T->side, d);
        int64_t j = leaf_coord(T->xyz[3 * a + 1], T->lo[1], T->side, d);
        int64_t k = leaf_coord(T->xyz[3 * a + 2], T->lo[2], T->side, d);
        T->leaf_of[a] = cell_id(d, i, j, k);
        T->start[T->leaf_of[a] + 1]++;
    }
    for (int64_t c = 0; c < nl; ++c) T->start[c + 1] += T->start[c];
    int64_t *fill = (int64_t *)malloc((size_t)nl * sizeof(int64_t));
    if (!fill) return -1;
    memcpy(fill, T->start, (size_t)nl * sizeof(int64_t));
    for (int64_t a = 0; a < T->n; ++a) T->order[fill[T->leaf_of[a]]++] = a;
    free(fill);
    return 0;
}

static void free_tree(otree *T)
{
    free(T->leaf_of);
    free(T->start);
    free(T->order);
    if (T->M) for (int l = 0; l <= T->depth; ++l) free(T->M[l]);
    if (T->L) for (int l = 0; l <= T->depth; ++l) free(T->L[l]);
    free(T->M);
    free(T->L);
}

/* upward pass: P2M at every leaf, then M2M from level depth to level 2 */
static int upward(otree *T)
{
    int d = T->depth, nf = T->nf, p = T->p;
    T->M = (double **)calloc((size_t)d + 1, sizeof(double *));
    if (!T->M) return -1;
    for (int l = 2; l <= d; ++l) {
        T->M[l] = (double *)calloc((size_t)ncell1(3 * l) * nf, sizeof(double));
        if (!T->M[l]) return -1;
    }
    int64_t nside = ncell1(d);
#pragma omp parallel
    {
#pragma omp for schedule(dynamic, 64)
        for (int64_t c = 0; c < ncell1(3 * d); ++c) {
            int64_t b = T->start[c], e = T->start[c + 1];
            if (e == b) continue;
            int64_t i = c % nside, j = (c / nside) % nside, k = c / (nside * nside);
            double z[3];
            cell_center(T, d, i, j, k, z);
            double *px = (double *)malloc((size_t)(e - b) * 3 * sizeof(double));
            double *pq = (double *)malloc((size_t)(e - b) * sizeof(double));
            for (int64_t s = b; s < e; ++s) {
                int64_t a = T->order[s];
                px[3 * (s - b) + 0] = T->xyz[3 * a + 0];
                px[3 * (s - b) + 1] = T->xyz[3 * a + 1];
                px[3 * (s - b) + 2] = T->xyz[3 * a + 2];
                pq[s - b] = T->q[a];
            }
            oracle_p2m(p, z, e - b, px, pq, &T->M[d][(size_t)c * nf]);
            if (T->dip) {
                double *pd = (double *)malloc((size_t)(e - b) * 3 * sizeof(double));
                for (int64_t s = b; s < e; ++s)
                    for (int x = 0; x < 3; ++x) pd[3 * (s - b) + x] = T->dip[3 * T->order[s] + x];
                oracle_p2m_dipole(p, z, e - b, px, pd, &T->M[d][(size_t)c * nf]);
                free(pd);
            }
            free(px);
            free(pq);
        }
    }
    for (int l = d; l >= 3; --l) {
        int64_t ns = ncell1(l - 1);
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t c = 0; c < ncell1(3 * (l - 1)); ++c) {
            int64_t I = c % ns, J = (c / ns) % ns, K = c / (ns * ns);
            double zp[3];
            cell_center(T, l - 1, I, J, K, zp);
            for (int o = 0; o < 8; ++o) {
                int64_t i = 2 * I + (o & 1), j = 2 * J + ((o >> 1) & 1), k = 2 * K + ((o >> 2) & 1);
                double zc[3], dd[3];
                cell_center(T, l, i, j, k, zc);
                dd[0] = zc[0] - zp[0]; dd[1] = zc[1] - zp[1]; dd[2] = zc[2] - zp[2];
                oracle_m2m(p, dd, &T->M[l][(size_t)cell_id(l, i, j, k) * nf], &T->M[l - 1][(size_t)c * nf]);
            }
        }
    }
    return 0;
}

static inline int64_t iabs64(int64_t x) { return x < 0 ? -x : x; }
static inline int64_t imax3(int64_t a, int64_t b, int64_t c) { int64_t m = a > b ? a : b; return m > c ? m : c; }

/* M2L into cell (i,j,k) at level l from its ws=1 interaction list */
static void m2l_cell(otree *T, int l, int64_t i, int64_t j, int64_t k, double *Lc)
{
    int nf = T->nf, p = T->p;
    int64_t ns = ncell1(l);
    int64_t I = i >> 1, J = j >> 1, K = k >> 1;
    double zb[3];
    cell_center(T, l, i, j, k, zb);
    for (int64_t a = 2 * (I - 1); a <= 2 * (I + 1) + 1; ++a)
        for (int64_t b = 2 * (J - 1); b <= 2 * (J + 1) + 1; ++b)
            for (int64_t c = 2 * (K - 1); c <= 2 * (K + 1) + 1; ++c) {
                if (a < 0 || b < 0 || c < 0 || a >= ns || b >= ns || c >= ns) continue;
                if (imax3(iabs64(a - i), iabs64(b - j), iabs64(c - k)) <= 1) continue;
                double za[3], r[3];
                cell_center(T, l, a, b, c, za);
                r[0] = zb[0] - za[0]; r[1] = zb[1] - za[1]; r[2] = zb[2] - za[2];
                oracle_m2l(p, r, &T->M[l][(size_t)cell_id(l, a, b, c) * nf], Lc);
            }
}

/*
 * Downward pass for the cells in `need` (per level, a 0/1 mask of the cells
 * whose L is needed).  L of a needed cell = M2L from its interaction list
 * + L2L from its parent (levels >= 3).
 */
static int downward(otree *T, unsigned char **need)
{
    int d = T->depth, nf = T->nf, p = T->p;
    T->L = (double **)calloc((size_t)d + 1, sizeof(double *));
    if (!T->L) return -1;
    for (int l = 2; l <= d; ++l) {
        T->L[l] = (double *)calloc((size_t)ncell1(3 * l) * nf, sizeof(double));
        if (!T->L[l]) return -1;
    }
    for (int l = 2; l <= d; ++l) {
        int64_t ns = ncell1(l);
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t c = 0; c < ncell1(3 * l); ++c) {
            if (need && !need[l][c]) continue;
            int64_t i = c % ns, j = (c / ns) % ns, k = c / (ns * ns);
            double *Lc = &T->L[l][(size_t)c * nf];
            if (l >= 3) {
                double zc[3], zp[3], dd[3];
                cell_center(T, l, i, j, k, zc);
                cell_center(T, l - 1, i >> 1, j >> 1, k >> 1, zp);
                dd[0] = zc[0] - zp[0]; dd[1] = zc[1] - zp[1]; dd[2] = zc[2] - zp[2];
                oracle_l2l(p, dd, &T->L[l - 1][(size_t)cell_id(l - 1, i >> 1, j >> 1, k >> 1) * nf], Lc);
            }
            m2l_cell(T, l, i, j, k, Lc);
        }
    }
    return 0;
}

/* far field (L2P) + near field (P2P over adjacent-or-equal leaves) for particle b */
static void evaluate_particle(const otree *T, int64_t b, double *phi, double *grad)
{
    int d = T->depth;
    int64_t ns = ncell1(d);
    int64_t c = T->leaf_of[b];
    int64_t i = c % ns, j = (c / ns) % ns, k = c / (ns * ns);
    double f = 0.0, g[3] = {0.0, 0.0, 0.0};
    if (d >= 2) {
        double z[3], rb[3];
        cell_center(T, d, i, j, k, z);
        rb[0] = T->xyz[3 * b + 0] - z[0];
        rb[1] = T->xyz[3 * b + 1] - z[1];
        rb[2] = T->xyz[3 * b + 2] - z[2];
        oracle_l2p(T->p, rb, &T->L[d][(size_t)c * T->nf], &f, g);
    }
    for (int64_t a1 = i - 1; a1 <= i + 1; ++a1)
        for (int64_t b1 = j - 1; b1 <= j + 1; ++b1)
            for (int64_t c1 = k - 1; c1 <= k + 1; ++c1) {
                if (a1 < 0 || b1 < 0 || c1 < 0 || a1 >= ns || b1 >= ns || c1 >= ns) continue;
                int64_t src = cell_id(d, a1, b1, c1);
                for (int64_t s = T->start[src]; s < T->start[src + 1]; ++s) {
                    int64_t a = T->order[s];
                    if (a == b) continue;
                    pair_kernel(&T->xyz[3 * b], &T->xyz[3 * a], T->q[a], &f, g);
                    if (T->dip) pair_kernel_dipole(&T->xyz[3 * b], &T->xyz[3 * a], &T->dip[3 * a], &f, g);
                }
            }
    phi[0] = f;
    grad[0] = g[0];
    grad[1] = g[1];
    grad[2] = g[2];
}

/*
 * Full FMM on a uniform octree of the given depth over the cube
 * [lo, lo+side)^3.  Targets: tgt[0..nt) particle indices, or all particles
 * (in input order) when tgt is NULL.  Only cells on the paths of the target
 * leaves get a downward pass, so a sample of targets costs the upward pass
 * plus work proportional to the sample.
 *
 * M_dump/L_dump (optional, may be NULL): full-storage expansions of every
 * cell of levels 0..depth, cells row-major (x fastest) within a level,
 * levels concatenated; levels below 2 (and unneeded cells) are zero.
 *
 * Returns 0 on success, -1 on bad arguments, -2 on allocation failure.
 */
static int fmm_uniform_impl(int64_t n, const double *xyz, const double *q, const double *dip, int p, int depth,
                            const double lo[3], double side, int64_t nt, const int64_t *tgt, double *phi,
                            double *grad, double *M_dump, double *L_dump, int nthreads);

int oracle_fmm_uniform(int64_t n, const double *xyz, const double *q, int p, int depth,
                       const double lo[3], double side, int64_t nt, const int64_t *tgt,
                       double *phi, double *grad, double *M_dump, double *L_dump, int nthreads)
{
    return fmm_uniform_impl(n, xyz, q, NULL, p, depth, lo, side, nt, tgt, phi, grad, M_dump, L_dump, nthreads);
}

/* The uniform FMM with point dipoles dip ([n][3]) beside the charges: P2M
 * adds oracle_p2m_dipole, the near field the dipole pair terms. */
int oracle_fmm_uniform_dipoles(int64_t n, const double *xyz, const double *q, const double *dip, int p, int depth,
                               const double lo[3], double side, int64_t nt, const int64_t *tgt, double *phi,
                               double *grad, int nthreads)
{
    if (!dip) return -1;
    return fmm_uniform_impl(n, xyz, q, dip, p, depth, lo, side, nt, tgt, phi, grad, NULL, NULL, nthreads);
}

static int fmm_uniform_impl(int64_t n, const double *xyz, const double *q, const double *dip, int p, int depth,
                            const double lo[3], double side, int64_t nt, const int64_t *tgt, double *phi,
                            double *grad, double *M_dump, double *L_dump, int nthreads)
{
    init_tables();
    if (p < 0 || p > OR_PMAX || depth < 0 || depth > 9 || n < 0 || side <= 0.0) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    otree T;
    memset(&T, 0, sizeof(T));
    T.p = p; T.depth = depth; T.nf = g_nfull[p];
    T.lo[0] = lo[0]; T.lo[1] = lo[1]; T.lo[2] = lo[2]; T.side = side;
    T.n = n; T.xyz = xyz; T.q = q; T.dip = dip;
    int rc = 0;
    unsigned char **need = NULL;
    if (build_tree(&T)) { rc = -2; goto done; }
    if (depth >= 2) {
        if (upward(&T)) { rc = -2; goto done; }
        if (tgt) {
            need = (unsigned char **)calloc((size_t)depth + 1, sizeof(unsigned char *));
            if (!need) { rc = -2; goto done; }
            for (int l = 0; l <= depth; ++l) {
                need[l] = (unsigned char *)calloc((size_t)ncell1(3 * l), 1);
                if (!need[l]) { rc = -2; goto done; }
            }
            int64_t ns = ncell1(depth);
            for (int64_t t = 0; t < nt; ++t) {
                int64_t c = T.leaf_of[tgt[t]];
                int64_t i = c % ns, j = (c / ns) % ns, k = c / (ns * ns);
                for (int l = depth; l >= 0; --l) {
                    need[l][cell_id(l, i, j, k)] = 1;
                    i >>= 1; j >>= 1; k >>= 1;
                }
            }
        }
        if (downward(&T, need)) { rc = -2; goto done; }
    }
    {
        int64_t cnt = tgt ? nt : n;
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t t = 0; t < cnt; ++t) {
            int64_t b = tgt ? tgt[t] : t;
            evaluate_particle(&T, b, &phi[t], &grad[3 * t]);
        }
    }
    if (M_dump || L_dump) {
        size_t off = 0;
        for (int l = 0; l <= depth; ++l) {
            size_t cnt = (size_t)ncell1(3 * l) * T.nf;
            if (M_dump) {
                if (l >= 2 && T.M) memcpy(M_dump + off, T.M[l], cnt * sizeof(double));
                else memset(M_dump + off, 0, cnt * sizeof(double));
            }
            if (L_dump) {
                if (l >= 2 && T.L) memcpy(L_dump + off, T.L[l], cnt * sizeof(double));
                else memset(L_dump + off, 0, cnt * sizeof(double));
            }
            off += cnt;
        }
    }
done:
    if (need) {
        for (int l = 0; l <= depth; ++l) free(need[l]);
        free(need);
    }
    free_tree(&T);
    return rc;
}

/* threads the OpenMP runtime will use for the next parallel region */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ========================================================== adaptive octree */
/*
 * Adaptive octree over a cube (Appendix C recommends splitting geometrically
 * at the cell centre for inhomogeneous distributions): a node holding more
 * than leaf_max particles is split into its non-empty octants, down to level
 * OA_DMAX.  Interactions follow the classic adaptive FMM lists, every one
 * evaluated with the paper's operators:
 *   V(B): children of the same-level neighbours of parent(B) that are not
 *         adjacent to B                          -> M2L (Eq. M2L)
 *   U(B), B a leaf: leaves adjacent to B (B too) -> P2P (Eq. PhiAB)
 *   W(B), B a leaf: descendants of B's same-level neighbours that are not
 *         adjacent to B while their parent is    -> multipole evaluated at
 *         B's particles: M2L to the particle, then its rank-0/1 components
 *   X(B): the leaves C with B in W(C)            -> local expansion of C's
 *         particles about B: M2L of a single-charge multipole
 * "Adjacent" means the closed cubes touch or overlap.  Expansion centres are
 * the geometric cell centres.
 */
#define OA_DMAX 21

typedef struct {
    int level;
    uint64_t pre;      /* Morton prefix of the node at its level */
    int64_t b, e;      /* sorted particle range */
    int parent;
    int child[8];      /* node index or -1 */
    int leaf;
    int64_t ix, iy, iz; /* integer coordinates at its level */
} oanode;

typedef struct {
    int *v;
    int n, cap;
} ivec;

static void ivec_push(ivec *a, int x)
{
    if (a->n == a->cap) {
        a->cap = a->cap ? 2 * a->cap : 8;
        a->v = (int *)realloc(a->v, (size_t)a->cap * sizeof(int));
    }
    a->v[a->n++] = x;
}

static uint64_t oa_spread(uint64_t v)
{
    uint64_t r = 0;
    for (int b = 0; b < OA_DMAX; ++b) r |= ((v >> b) & 1ull) << (3 * b);
    return r;
}

typedef struct {
    int p, leaf_max;
    double lo[3], side;
    int64_t n;
    const double *xyz, *q;
    int64_t *order;    /* particles sorted by key (ties by index) */
    uint64_t *key;     /* key of sorted position */
    oanode *nd;
    int nn, ncap;
    int maxlev;
    int *lev_start;    /* nodes grouped per level: indices lev_list[lev_start[l] .. lev_start[l+1]) */
    int *lev_list;
    int64_t *leaf_of;  /* particle -> leaf node */
    ivec *U, *V, *W, *X;
    double **M, **L;   /* per node, full storage */
    int nf;
} oatree;

static const oatree *g_sort_tree;
static int cmp_key(const void *a, const void *b)
{
    const int64_t ia = *(const int64_t *)a, ib = *(const int64_t *)b;
    uint64_t ka = g_sort_tree->key[ia], kb = g_sort_tree->key[ib];
    if (ka != kb) return ka < kb ? -1 : 1;
    return ia < ib ? -1 : (ia > ib);
}

static int oa_new_node(oatree *T, int level, uint64_t pre, int64_t b, int64_t e, int parent)
{
    if (T->nn == T->ncap) {
        T->ncap = T->ncap ? 2 * T->ncap : 1024;
        T->nd = (oanode *)realloc(T->nd, (size_t)T->ncap * sizeof(oanode));
    }
    oanode *x = &T->nd[T->nn];
    x->level = level; x->pre = pre; x->b = b; x->e = e; x->parent = parent; x->leaf = 1;
    for (int o = 0; o < 8; ++o) x->child[o] = -1;
    int64_t ix = 0, iy = 0, iz = 0;
    for (int l = 0; l < level; ++l) {
        ix |= (int64_t)((pre >> (3 * l)) & 1) << l;
        iy |= (int64_t)((pre >> (3 * l + 1)) & 1) << l;
        iz |= (int64_t)((pre >> (3 * l + 2)) & 1) << l;
    }
    x->ix = ix; x->iy = iy; x->iz = iz;
    if (level > T->maxlev) T->maxlev = level;
    return T->nn++;
}

static void oa_split(oatree *T, int node)
{
    oanode nd = T->nd[node];
    if (nd.e - nd.b <= T->leaf_max || nd.level >= OA_DMAX) return;
    T->nd[node].leaf = 0;
    int sh = 3 * (OA_DMAX - nd.level - 1);
    int64_t s = nd.b;
    for (int o = 0; o < 8; ++o) {
        uint64_t cpre = nd.pre * 8 + (uint64_t)o;
        int64_t e = s;
        while (e < nd.e && (T->key[e] >> sh) == cpre) ++e;
        if (e > s) {
            int c = oa_new_node(T, nd.level + 1, cpre, s, e, node);
            T->nd[node].child[o] = c;
            oa_split(T, c);
        }
        s = e;
    }
}

/* closed cubes of nodes A and B touch or overlap */
static int oa_adjacent(const oanode *A, const oanode *B)
{
    int sa = OA_DMAX - A->level, sb = OA_DMAX - B->level;
    int64_t ca[3] = {A->ix, A->iy, A->iz}, cb[3] = {B->ix, B->iy, B->iz};
    for (int d = 0; d < 3; ++d) {
        int64_t alo = ca[d] << sa, ahi = (ca[d] + 1) << sa;
        int64_t blo = cb[d] << sb, bhi = (cb[d] + 1) << sb;
        if (alo > bhi || blo > ahi) return 0;
    }
    return 1;
}

/* node at (level, ix, iy, iz) or -1 */
static int oa_find(const oatree *T, int level, int64_t ix, int64_t iy, int64_t iz)
{
    int64_t n1 = (int64_t)1 << level;
    if (ix < 0 || iy < 0 || iz < 0 || ix >= n1 || iy >= n1 || iz >= n1) return -1;
    int cur = 0;
    for (int l = 1; l <= level; ++l) {
        int sh = level - l;
        int o = (int)(((ix >> sh) & 1) | (((iy >> sh) & 1) << 1) | (((iz >> sh) & 1) << 2));
        cur = T->nd[cur].child[o];
        if (cur < 0) return -1;
    }
    return cur;
}

static void oa_collect_U(const oatree *T, int node, int B, ivec *out)
{
    if (!oa_adjacent(&T->nd[node], &T->nd[B])) return;
    if (T->nd[node].leaf) { ivec_push(out, node); return; }
    for (int o = 0; o < 8; ++o)
        if (T->nd[node].child[o] >= 0) oa_collect_U(T, T->nd[node].child[o], B, out);
}

static void oa_collect_W(const oatree *T, int node, int B, ivec *out)
{
    /* node is a descendant of a neighbour of B whose parent is adjacent to B */
    for (int o = 0; o < 8; ++o) {
        int c = T->nd[node].child[o];
        if (c < 0) continue;
        if (!oa_adjacent(&T->nd[c], &T->nd[B])) ivec_push(out, c);
        else if (!T->nd[c].leaf) oa_collect_W(T, c, B, out);
    }
}

static void oa_build_lists(oatree *T)
{
    int nn = T->nn > 0 ? T->nn : 1;
    T->U = (ivec *)calloc((size_t)nn, sizeof(ivec));
    T->V = (ivec *)calloc((size_t)nn, sizeof(ivec));
    T->W = (ivec *)calloc((size_t)nn, sizeof(ivec));
    T->X = (ivec *)calloc((size_t)nn, sizeof(ivec));
    nn = T->nn;
    for (int B = 0; B < nn; ++B) {
        const oanode *b = &T->nd[B];
        if (b->level >= 1) {
            const oanode *P = &T->nd[b->parent];
            for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        int Q = oa_find(T, P->level, P->ix + dx, P->iy + dy, P->iz + dz);
                        if (Q < 0) continue;
                        for (int o = 0; o < 8; ++o) {
                            int C = T->nd[Q].child[o];
                            if (C >= 0 && !oa_adjacent(&T->nd[C], b)) ivec_push(&T->V[B], C);
                        }
                    }
        }
        if (b->leaf) {
            oa_collect_U(T, 0, B, &T->U[B]);
            for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        if (!dx && !dy && !dz) continue;
                        int C = oa_find(T, b->level, b->ix + dx, b->iy + dy, b->iz + dz);
                        if (C >= 0 && !T->nd[C].leaf) oa_collect_W(T, C, B, &T->W[B]);
                    }
        }
    }
    for (int B = 0; B < nn; ++B)
        for (int i = 0; i < T->W[B].n; ++i) ivec_push(&T->X[T->W[B].v[i]], B);
}

static void oa_center(const oatree *T, const oanode *x, double z[3])
{
    double h = T->side / (double)((int64_t)1 << x->level);
    z[0] = T->lo[0] + ((double)x->ix + 0.5) * h;
    z[1] = T->lo[1] + ((double)x->iy + 0.5) * h;
    z[2] = T->lo[2] + ((double)x->iz + 0.5) * h;
}

/* automatic root cube: centred on the bounding box, side = largest extent * (1 + 2^-20) */
void oracle_auto_root(int64_t n, const double *xyz, double lo[3], double *side)
{
    double mn[3] = {0, 0, 0}, mx[3] = {0, 0, 0};
    for (int64_t a = 0; a < n; ++a)
        for (int d = 0; d < 3; ++d) {
            double v = xyz[3 * a + d];
            if (a == 0 || v < mn[d]) mn[d] = v;
            if (a == 0 || v > mx[d]) mx[d] = v;
        }
    double s = 0.0;
    for (int d = 0; d < 3; ++d)
        if (mx[d] - mn[d] > s) s = mx[d] - mn[d];
    if (!(s > 0.0)) s = 1.0;
    s = s * (1.0 + 1.0 / 1048576.0);
    for (int d = 0; d < 3; ++d) lo[d] = (mn[d] + mx[d]) * 0.5 - s * 0.5;
    *side = s;
}

static void oa_free(oatree *T)
{
    free(T->order); free(T->key); free(T->leaf_of);
    if (T->U) for (int i = 0; i < T->nn; ++i) { free(T->U[i].v); free(T->V[i].v); free(T->W[i].v); free(T->X[i].v); }
    free(T->U); free(T->V); free(T->W); free(T->X);
    if (T->M) for (int i = 0; i < T->nn; ++i) free(T->M[i]);
    if (T->L) for (int i = 0; i < T->nn; ++i) free(T->L[i]);
    free(T->M); free(T->L); free(T->nd);
}

/*
 * Full FMM on the adaptive octree.  side <= 0 selects the automatic root
 * cube.  Targets as in oracle_fmm_uniform (all particles when tgt is NULL).
 * stats (optional, 8 int64): nodes, leaves, max level, |V|, |U| (leaf pairs),
 * |W|, |X| totals, and the root box is written to root_out[4] (lo, side) if
 * given.  Returns 0, -1 (arguments) or -2 (allocation).
 */
static int fmm_adaptive_impl(int64_t n, const double *xyz, const double *q, int p, int leaf_max,
                             const double lo_in[3], double side_in, int64_t nt, const int64_t *tgt,
                             double *phi, double *grad, int64_t *stats, double *root_out, int nthreads,
                             const int *order_r2, const int8_t *vorder);

int oracle_fmm_adaptive(int64_t n, const double *xyz, const double *q, int p, int leaf_max,
                        const double lo_in[3], double side_in, int64_t nt, const int64_t *tgt,
                        double *phi, double *grad, int64_t *stats, double *root_out, int nthreads)
{
    return fmm_adaptive_impl(n, xyz, q, p, leaf_max, lo_in, side_in, nt, tgt, phi, grad, stats, root_out,
                             nthreads, NULL, NULL);
}

/*
 * The adaptive FMM with the M2L order of every V-list pair taken from a
 * table indexed by |v|^2, v the integer offset between the two same-level
 * cells (4 <= |v|^2 <= 27 for the ws=1 lists): M2L of that pair is Eq. M2L
 * truncated at |n| + |m| <= order_r2[|v|^2] (<= p), acting on the order-p
 * expansions.  Every other operator keeps order p.
 */
int oracle_fmm_adaptive_orders(int64_t n, const double *xyz, const double *q, int p, int leaf_max,
                               const double lo_in[3], double side_in, int64_t nt, const int64_t *tgt,
                               double *phi, double *grad, int64_t *stats, double *root_out, int nthreads,
                               const int *order_r2)
{
    if (!order_r2) return -1;
    for (int k = 4; k <= 27; ++k)
        if (order_r2[k] < 0 || order_r2[k] > p) return -1;
    return fmm_adaptive_impl(n, xyz, q, p, leaf_max, lo_in, side_in, nt, tgt, phi, grad, stats, root_out,
                             nthreads, order_r2, NULL);
}

/*
 * The adaptive FMM with the M2L order of every V-list pair given: entry k
 * of node i's V list (the order of oracle_adaptive_tree) is translated by
 * Eq. M2L truncated at |n| + |m| <= vorder[V_off[i] + k] (<= p), acting on
 * the order-p expansions.  Every other operator keeps order p.
 */
int oracle_fmm_adaptive_pair_orders(int64_t n, const double *xyz, const double *q, int p, int leaf_max,
                                    const double lo_in[3], double side_in, int64_t nt, const int64_t *tgt,
                                    double *phi, double *grad, int64_t *stats, double *root_out, int nthreads,
                                    const int8_t *vorder)
{
    if (!vorder) return -1;
    return fmm_adaptive_impl(n, xyz, q, p, leaf_max, lo_in, side_in, nt, tgt, phi, grad, stats, root_out,
                             nthreads, NULL, vorder);
}

/*
 * The adaptive tree of n particles and its U/V/W/X lists: root cube (given,
 * or the automatic cube), 63-bit keys, particles sorted by key (ties by
 * index), nodes split while they hold more than leaf_max particles, then the
 * lists by tree recursion.  Returns 0 or -2 (allocation).
 */
static int oa_make_tree(oatree *T, int64_t n, const double *xyz, const double *q, int p, int leaf_max,
                        const double lo_in[3], double side_in)
{
    memset(T, 0, sizeof(*T));
    T->p = p; T->leaf_max = leaf_max; T->n = n; T->xyz = xyz; T->q = q; T->nf = g_nfull[p];
    if (side_in > 0.0) {
        T->lo[0] = lo_in[0]; T->lo[1] = lo_in[1]; T->lo[2] = lo_in[2]; T->side = side_in;
    } else {
        oracle_auto_root(n, xyz, T->lo, &T->side);
    }
    T->order = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    T->key = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    uint64_t *pkey = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    T->leaf_of = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!T->order || !T->key || !pkey || !T->leaf_of) { free(pkey); return -2; }
    for (int64_t a = 0; a < n; ++a) {
        uint64_t c[3];
        for (int d = 0; d < 3; ++d) {
            double s = floor((xyz[3 * a + d] - T->lo[d]) / T->side * (double)((int64_t)1 << OA_DMAX));
            int64_t i = (int64_t)s;
            if (s < 0.0) i = 0;
            if (i > ((int64_t)1 << OA_DMAX) - 1) i = ((int64_t)1 << OA_DMAX) - 1;
            c[d] = (uint64_t)i;
        }
        pkey[a] = oa_spread(c[0]) | (oa_spread(c[1]) << 1) | (oa_spread(c[2]) << 2);
        T->order[a] = a;
    }
    memcpy(T->key, pkey, (size_t)n * sizeof(uint64_t));
    g_sort_tree = T;
    qsort(T->order, (size_t)n, sizeof(int64_t), cmp_key);
    for (int64_t s = 0; s < n; ++s) T->key[s] = pkey[T->order[s]];
    free(pkey);
    oa_new_node(T, 0, 0, 0, n, -1);
    oa_split(T, 0);
    for (int i = 0; i < T->nn; ++i)
        if (T->nd[i].leaf)
            for (int64_t s = T->nd[i].b; s < T->nd[i].e; ++s) T->leaf_of[T->order[s]] = i;
    oa_build_lists(T);
    return 0;
}

/*
 * The adaptive tree and lists of oracle_fmm_adaptive, for an element-by-element
 * comparison.  sizes[6] receives: nodes, particles, and the total lengths of
 * the U, V, W and X lists.  With the arrays given (each may be NULL), node i
 * (the oracle's numbering: depth-first creation order) gets its level, its
 * Morton prefix key (3*level bits, x in bit 0 of each triple), leaf flag,
 * parent (-1 for the root) and sorted particle range [pb, pe); order[s] is
 * the input index at sorted position s; list L of node i is
 * L_list[L_off[i] .. L_off[i+1]) (node indices, in the oracle's order).
 * Returns 0, -1 (arguments) or -2 (allocation).
 */
int oracle_adaptive_tree(int64_t n, const double *xyz, int leaf_max, const double lo_in[3], double side_in,
                         int64_t *sizes, int32_t *level, uint64_t *key, int32_t *leaf, int32_t *parent,
                         int64_t *pb, int64_t *pe, int64_t *order, int64_t *u_off, int32_t *u_list,
                         int64_t *v_off, int32_t *v_list, int64_t *w_off, int32_t *w_list, int64_t *x_off,
                         int32_t *x_list)
{
    init_tables();
    if (n < 1 || leaf_max < 1 || !sizes) return -1;
    oatree T;
    if (oa_make_tree(&T, n, xyz, NULL, 0, leaf_max, lo_in, side_in) != 0) { oa_free(&T); return -2; }
    ivec *lists[4] = {T.U, T.V, T.W, T.X};
    int64_t *offs[4] = {u_off, v_off, w_off, x_off};
    int32_t *vals[4] = {u_list, v_list, w_list, x_list};
    sizes[0] = T.nn;
    sizes[1] = n;
    for (int k = 0; k < 4; ++k) {
        int64_t tot = 0;
        for (int i = 0; i < T.nn; ++i) {
            if (offs[k]) offs[k][i] = tot;
            for (int j = 0; j < lists[k][i].n; ++j)
                if (vals[k]) vals[k][tot + j] = lists[k][i].v[j];
            tot += lists[k][i].n;
        }
        if (offs[k]) offs[k][T.nn] = tot;
        sizes[2 + k] = tot;
    }
    for (int i = 0; i < T.nn; ++i) {
        const oanode *x = &T.nd[i];
        if (level) level[i] = x->level;
        if (key) key[i] = x->pre;
        if (leaf) leaf[i] = x->leaf;
        if (parent) parent[i] = x->parent;
        if (pb) pb[i] = x->b;
        if (pe) pe[i] = x->e;
    }
    if (order) memcpy(order, T.order, (size_t)n * sizeof(int64_t));
    oa_free(&T);
    return 0;
}

static int fmm_adaptive_impl(int64_t n, const double *xyz, const double *q, int p, int leaf_max,
                             const double lo_in[3], double side_in, int64_t nt, const int64_t *tgt,
                             double *phi, double *grad, int64_t *stats, double *root_out, int nthreads,
                             const int *order_r2, const int8_t *vorder)
{
    init_tables();
    if (p < 0 || p > OR_PMAX || n < 1 || leaf_max < 1) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    oatree T;
    if (oa_make_tree(&T, n, xyz, q, p, leaf_max, lo_in, side_in) != 0) { oa_free(&T); return -2; }
    if (root_out) { root_out[0] = T.lo[0]; root_out[1] = T.lo[1]; root_out[2] = T.lo[2]; root_out[3] = T.side; }
    /* first entry of every node's V list in the V-list order of oracle_adaptive_tree */
    int64_t *voff = (int64_t *)calloc((size_t)T.nn + 1, sizeof(int64_t));
    if (!voff) { oa_free(&T); return -2; }
    for (int i = 0; i < T.nn; ++i) voff[i + 1] = voff[i] + T.V[i].n;
    if (vorder)
        for (int64_t k = 0; k < voff[T.nn]; ++k)
            if (vorder[k] < 0 || vorder[k] > p) { free(voff); oa_free(&T); return -1; }
    int nf = T.nf;
    size_t nnodes = T.nn > 0 ? (size_t)T.nn : 1;
    T.M = (double **)calloc(nnodes, sizeof(double *));
    T.L = (double **)calloc(nnodes, sizeof(double *));
    for (int i = 0; i < T.nn; ++i) {
        T.M[i] = (double *)calloc((size_t)nf, sizeof(double));
        T.L[i] = (double *)calloc((size_t)nf, sizeof(double));
    }
    /* upward: P2M at leaves, then M2M from the deepest level up */
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < T.nn; ++i) {
        if (!T.nd[i].leaf) continue;
        double z[3];
        oa_center(&T, &T.nd[i], z);
        int64_t cnt = T.nd[i].e - T.nd[i].b;
        double *px = (double *)malloc((size_t)cnt * 3 * sizeof(double));
        double *pq = (double *)malloc((size_t)cnt * sizeof(double));
        for (int64_t s = T.nd[i].b; s < T.nd[i].e; ++s) {
            int64_t a = T.order[s];
            for (int d = 0; d < 3; ++d) px[3 * (s - T.nd[i].b) + d] = xyz[3 * a + d];
            pq[s - T.nd[i].b] = q[a];
        }
        oracle_p2m(p, z, cnt, px, pq, T.M[i]);
        free(px);
        free(pq);
    }
    for (int l = T.maxlev; l >= 1; --l) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int i = 0; i < T.nn; ++i) {
            if (T.nd[i].level != l - 1 || T.nd[i].leaf) continue;
            double zp[3];
            oa_center(&T, &T.nd[i], zp);
            for (int o = 0; o < 8; ++o) {
                int c = T.nd[i].child[o];
                if (c < 0) continue;
                double zc[3], dd[3];
                oa_center(&T, &T.nd[c], zc);
                dd[0] = zc[0] - zp[0]; dd[1] = zc[1] - zp[1]; dd[2] = zc[2] - zp[2];
                oracle_m2m(p, dd, T.M[c], T.M[i]);
            }
        }
    }
    /* downward: per level, L2L from the parent, M2L from V, local expansions of X.
       With explicit targets only the paths from the root to their leaves are needed. */
    char *need = (char *)calloc(nnodes, 1);
    if (!need) { oa_free(&T); return -2; }
    if (tgt) {
        for (int64_t t = 0; t < nt; ++t)
            for (int i = (int)T.leaf_of[tgt[t]]; i >= 0 && !need[i]; i = T.nd[i].parent) need[i] = 1;
    } else {
        memset(need, 1, (size_t)T.nn);
    }
    for (int l = 1; l <= T.maxlev; ++l) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int i = 0; i < T.nn; ++i) {
            if (T.nd[i].level != l || !need[i]) continue;
            double zb[3];
            oa_center(&T, &T.nd[i], zb);
            int par = T.nd[i].parent;
            if (par >= 0 && T.nd[par].level >= 1) {
                double zp[3], dd[3];
                oa_center(&T, &T.nd[par], zp);
                dd[0] = zb[0] - zp[0]; dd[1] = zb[1] - zp[1]; dd[2] = zb[2] - zp[2];
                oracle_l2l(p, dd, T.L[par], T.L[i]);
            }
            for (int k = 0; k < T.V[i].n; ++k) {
                int C = T.V[i].v[k];
                double za[3], r[3];
                oa_center(&T, &T.nd[C], za);
                r[0] = zb[0] - za[0]; r[1] = zb[1] - za[1]; r[2] = zb[2] - za[2];
                int order = p;
                if (order_r2) {
                    int64_t dx = T.nd[i].ix - T.nd[C].ix, dy = T.nd[i].iy - T.nd[C].iy, dz = T.nd[i].iz - T.nd[C].iz;
                    order = order_r2[dx * dx + dy * dy + dz * dz];
                }
                if (vorder) order = vorder[voff[i] + k];
                oracle_m2l(order, r, T.M[C], T.L[i]);
            }
            for (int k = 0; k < T.X[i].n; ++k) {
                int C = T.X[i].v[k];
                for (int64_t s = T.nd[C].b; s < T.nd[C].e; ++s) {
                    int64_t a = T.order[s];
                    double Mq[1000], r[3], xa[3] = {xyz[3 * a], xyz[3 * a + 1], xyz[3 * a + 2]};
                    memset(Mq, 0, (size_t)nf * sizeof(double));
                    oracle_p2m(p, xa, 1, xa, &q[a], Mq);
                    r[0] = zb[0] - xa[0]; r[1] = zb[1] - xa[1]; r[2] = zb[2] - xa[2];
                    oracle_m2l(p, r, Mq, T.L[i]);
                }
            }
        }
    }
    free(need);
    free(voff);
    /* evaluation: L2P + W (M2L to the particle) + U (direct) */
    int64_t cnt = tgt ? nt : n;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < cnt; ++t) {
        int64_t b = tgt ? tgt[t] : t;
        int B = (int)T.leaf_of[b];
        const double *xb = &xyz[3 * b];
        double f = 0.0, g[3] = {0.0, 0.0, 0.0}, z[3], rb[3];
        oa_center(&T, &T.nd[B], z);
        rb[0] = xb[0] - z[0]; rb[1] = xb[1] - z[1]; rb[2] = xb[2] - z[2];
        oracle_l2p(p, rb, T.L[B], &f, g);
        double *Lp = (double *)malloc((size_t)nf * sizeof(double));
        for (int k = 0; k < T.W[B].n; ++k) {
            int C = T.W[B].v[k];
            double za[3], r[3], zero[3] = {0.0, 0.0, 0.0};
            oa_center(&T, &T.nd[C], za);
            r[0] = xb[0] - za[0]; r[1] = xb[1] - za[1]; r[2] = xb[2] - za[2];
            memset(Lp, 0, (size_t)nf * sizeof(double));
            oracle_m2l(p, r, T.M[C], Lp);
            oracle_l2p(p, zero, Lp, &f, g);
        }
        free(Lp);
        for (int k = 0; k < T.U[B].n; ++k) {
            int C = T.U[B].v[k];
            for (int64_t s = T.nd[C].b; s < T.nd[C].e; ++s) {
                int64_t a = T.order[s];
                if (a == b) continue;
                pair_kernel(xb, &xyz[3 * a], q[a], &f, g);
            }
        }
        phi[t] = f;
        grad[3 * t + 0] = g[0];
        grad[3 * t + 1] = g[1];
        grad[3 * t + 2] = g[2];
    }
    if (stats) {
        int64_t st[8] = {T.nn, 0, T.maxlev, 0, 0, 0, 0, 0};
        for (int i = 0; i < T.nn; ++i) {
            st[1] += T.nd[i].leaf;
            st[3] += T.V[i].n; st[4] += T.U[i].n; st[5] += T.W[i].n; st[6] += T.X[i].n;
        }
        memcpy(stats, st, sizeof(st));
    }
    oa_free(&T);
    return 0;
}

/* ================================================= dual-tree traversal (θ-MAC) */
/*
 * The FMM driver of Appendix C on the adaptive octree (geometric splits at
 * the cell centre, leaves of at most leaf_max particles):
 *   - expansion centre of every node: its geometric centre (centre = 0), or
 *     the charge-weighted mean of its particles (centre = 1, and the AP
 *     variant, centre = 2), the geometric centre where the node's total
 *     charge is not positive; enclosing radius r = the largest distance
 *     from the centre to a particle of the node;
 *   - P2M at the leaves, M2M to the parents (Eq. P2M, Eq. M2M);
 *   - dual-tree traversal from (root, root): a pair of distinct nodes
 *     (A, B) is accepted when theta |z_B - z_A| > r_A + r_B (the MAC, read
 *     with scalar radii) and then translated both ways by M2L (Eq. M2L);
 *     otherwise the larger node -- by enclosing radius, the first of the
 *     pair on a tie, and never a leaf -- is opened and each of its children
 *     is paired with the other node; two leaves that fail the MAC are
 *     summed directly both ways.  A node paired with itself is replaced by
 *     the pairs of its children (each child with itself, and each two
 *     children once, in octant order); a leaf with itself is summed
 *     directly;
 *   - L2L from every node to its children (Eq. L2L), L2P at the leaves
 *     (Eq. L2P), plus the direct part.
 * The AP variant (centre = 2) drops the rank-1 multipole (the dipole, which
 * vanishes about the centre of mass) from every M2L and gives the gradient
 * only (phi is not written and may be NULL); it needs positive charges.
 * theta = 0 accepts no pair: the result is the direct sum.
 */
typedef struct {
    oatree *T;
    double theta;
    double (*zr)[4];   /* centre and radius per node */
    ivec m2l;          /* accepted pairs (a, b), a != b, in traversal order */
    ivec *p2p;         /* per leaf: its direct partners (both ways, itself included) */
    int64_t n_p2p;     /* unordered direct pairs, self pairs included */
} oadual;

static void dual_pair(oadual *D, int a, int b)
{
    oatree *T = D->T;
    const oanode *A = &T->nd[a], *B = &T->nd[b];
    if (a == b) {
        if (A->leaf) {
            ivec_push(&D->p2p[a], a);
            D->n_p2p++;
            return;
        }
        for (int i = 0; i < 8; ++i) {
            int ci = A->child[i];
            if (ci < 0) continue;
            for (int j = i; j < 8; ++j) {
                int cj = A->child[j];
                if (cj >= 0) dual_pair(D, ci, cj);
            }
        }
        return;
    }
    double dx = D->zr[b][0] - D->zr[a][0], dy = D->zr[b][1] - D->zr[a][1], dz = D->zr[b][2] - D->zr[a][2];
    double dist = sqrt(dx * dx + dy * dy + dz * dz);
    if (D->theta * dist > D->zr[a][3] + D->zr[b][3]) {
        ivec_push(&D->m2l, a);
        ivec_push(&D->m2l, b);
        return;
    }
    if (A->leaf && B->leaf) {
        ivec_push(&D->p2p[a], b);
        ivec_push(&D->p2p[b], a);
        D->n_p2p++;
        return;
    }
    int open_a = !A->leaf && (B->leaf || D->zr[a][3] >= D->zr[b][3]);
    const oanode *O = open_a ? A : B;
    for (int i = 0; i < 8; ++i) {
        int c = O->child[i];
        if (c < 0) continue;
        if (open_a) dual_pair(D, c, b);
        else dual_pair(D, a, c);
    }
}

/* centres and radii (see above), then the traversal */
static int dual_setup(oadual *D, oatree *T, const double *xyz, const double *q, double theta, int centre)
{
    memset(D, 0, sizeof(*D));
    D->T = T;
    D->theta = theta;
    D->zr = (double (*)[4])calloc((size_t)T->nn, sizeof(double[4]));
    D->p2p = (ivec *)calloc((size_t)T->nn, sizeof(ivec));
    if (!D->zr || !D->p2p) return -2;
    for (int i = 0; i < T->nn; ++i) {
        const oanode *x = &T->nd[i];
        double z[3];
        oa_center(T, x, z);
        if (centre != 0) {
            double w = 0.0, s[3] = {0.0, 0.0, 0.0};
            for (int64_t k = x->b; k < x->e; ++k) {
                int64_t a = T->order[k];
                w += q[a];
                for (int d = 0; d < 3; ++d) s[d] += q[a] * xyz[3 * a + d];
            }
            if (w > 0.0)
                for (int d = 0; d < 3; ++d) z[d] = s[d] / w;
        }
        double r = 0.0;
        for (int64_t k = x->b; k < x->e; ++k) {
            int64_t a = T->order[k];
            double dx = xyz[3 * a] - z[0], dy = xyz[3 * a + 1] - z[1], dz = xyz[3 * a + 2] - z[2];
            double d = sqrt(dx * dx + dy * dy + dz * dz);
            if (d > r) r = d;
        }
        D->zr[i][0] = z[0]; D->zr[i][1] = z[1]; D->zr[i][2] = z[2]; D->zr[i][3] = r;
    }
    dual_pair(D, 0, 0);
    return 0;
}

static void dual_free(oadual *D)
{
    if (D->p2p)
        for (int i = 0; i < D->T->nn; ++i) free(D->p2p[i].v);
    free(D->p2p);
    free(D->m2l.v);
    free(D->zr);
}

static int dual_check(int64_t n, int leaf_max, double theta, int centre, const double *q)
{
    if (n < 1 || leaf_max < 1 || !(theta >= 0.0) || centre < 0 || centre > 2) return -1;
    if (centre == 2)
        for (int64_t a = 0; a < n; ++a)
            if (!(q[a] > 0.0)) return -1;
    return 0;
}

int oracle_fmm_dual(int64_t n, const double *xyz, const double *q, int p, int leaf_max, double theta, int centre,
                    const double lo_in[3], double side_in, int64_t nt, const int64_t *tgt, double *phi, double *grad,
                    int64_t *stats, double *root_out, int nthreads)
{
    init_tables();
    if (p < 0 || p > OR_PMAX || dual_check(n, leaf_max, theta, centre, q) != 0) return -1;
    if (centre != 2 && !phi) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    oatree T;
    if (oa_make_tree(&T, n, xyz, q, p, leaf_max, lo_in, side_in) != 0) { oa_free(&T); return -2; }
    if (root_out) { root_out[0] = T.lo[0]; root_out[1] = T.lo[1]; root_out[2] = T.lo[2]; root_out[3] = T.side; }
    int nn = T.nn, nf = T.nf;
    oadual D;
    T.M = (double **)calloc((size_t)nn, sizeof(double *));
    T.L = (double **)calloc((size_t)nn, sizeof(double *));
    if (!T.M || !T.L || dual_setup(&D, &T, xyz, q, theta, centre) != 0) { dual_free(&D); oa_free(&T); return -2; }
    for (int i = 0; i < nn; ++i) {
        T.M[i] = (double *)calloc((size_t)nf, sizeof(double));
        T.L[i] = (double *)calloc((size_t)nf, sizeof(double));
    }
    /* upward: P2M at the leaves, M2M from the deepest level up */
    for (int i = 0; i < nn; ++i) {
        if (!T.nd[i].leaf) continue;
        int64_t cnt = T.nd[i].e - T.nd[i].b;
        double *px = (double *)malloc((size_t)cnt * 3 * sizeof(double));
        double *pq = (double *)malloc((size_t)cnt * sizeof(double));
        for (int64_t s2 = T.nd[i].b; s2 < T.nd[i].e; ++s2) {
            int64_t a = T.order[s2];
            for (int d = 0; d < 3; ++d) px[3 * (s2 - T.nd[i].b) + d] = xyz[3 * a + d];
            pq[s2 - T.nd[i].b] = q[a];
        }
        oracle_p2m(p, D.zr[i], cnt, px, pq, T.M[i]);
        free(px);
        free(pq);
    }
    for (int l = T.maxlev; l >= 1; --l)
        for (int i = 0; i < nn; ++i) {
            if (T.nd[i].level != l - 1 || T.nd[i].leaf) continue;
            for (int o = 0; o < 8; ++o) {
                int c = T.nd[i].child[o];
                if (c < 0) continue;
                double dd[3] = {D.zr[c][0] - D.zr[i][0], D.zr[c][1] - D.zr[i][1], D.zr[c][2] - D.zr[i][2]};
                oracle_m2m(p, dd, T.M[c], T.M[i]);
            }
        }
    /* AP: the dipole about the centre of mass is dropped */
    if (centre == 2 && p >= 1)
        for (int i = 0; i < nn; ++i) {
            T.M[i][g_idx[1][0][0]] = 0.0;
            T.M[i][g_idx[0][1][0]] = 0.0;
            T.M[i][g_idx[0][0][1]] = 0.0;
        }
    /* the accepted pairs, both ways */
    for (int k = 0; k < D.m2l.n; k += 2) {
        int a = D.m2l.v[k], b = D.m2l.v[k + 1];
        double r[3] = {D.zr[b][0] - D.zr[a][0], D.zr[b][1] - D.zr[a][1], D.zr[b][2] - D.zr[a][2]};
        double rm[3] = {-r[0], -r[1], -r[2]};
        oracle_m2l(p, r, T.M[a], T.L[b]);   /* A -> B */
        oracle_m2l(p, rm, T.M[b], T.L[a]);  /* B -> A */
    }
    /* downward: L2L from the root down */
    for (int l = 1; l <= T.maxlev; ++l)
        for (int i = 0; i < nn; ++i) {
            if (T.nd[i].level != l) continue;
            int par = T.nd[i].parent;
            double dd[3] = {D.zr[i][0] - D.zr[par][0], D.zr[i][1] - D.zr[par][1], D.zr[i][2] - D.zr[par][2]};
            oracle_l2l(p, dd, T.L[par], T.L[i]);
        }
    /* evaluation: L2P at the particle's leaf + the direct partners */
    int64_t cnt = tgt ? nt : n;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < cnt; ++t) {
        int64_t b = tgt ? tgt[t] : t;
        int B = (int)T.leaf_of[b];
        const double *xb = &xyz[3 * b];
        double f = 0.0, g[3] = {0.0, 0.0, 0.0};
        double rb[3] = {xb[0] - D.zr[B][0], xb[1] - D.zr[B][1], xb[2] - D.zr[B][2]};
        oracle_l2p(p, rb, T.L[B], &f, g);
        for (int k = 0; k < D.p2p[B].n; ++k) {
            int C = D.p2p[B].v[k];
            for (int64_t s2 = T.nd[C].b; s2 < T.nd[C].e; ++s2) {
                int64_t a = T.order[s2];
                if (a == b) continue;
                pair_kernel(xb, &xyz[3 * a], q[a], &f, g);
            }
        }
        if (phi) phi[t] = centre == 2 ? 0.0 : f;
        grad[3 * t + 0] = g[0];
        grad[3 * t + 1] = g[1];
        grad[3 * t + 2] = g[2];
    }
    if (stats) {
        int64_t st[8] = {T.nn, 0, T.maxlev, D.m2l.n / 2, D.n_p2p, 0, 0, 0};
        for (int i = 0; i < T.nn; ++i) st[1] += T.nd[i].leaf;
        memcpy(stats, st, sizeof(st));
    }
    dual_free(&D);
    oa_free(&T);
    return 0;
}

/*
 * The integer result of the traversal, in the node order of
 * oracle_adaptive_tree: sizes = {nodes, accepted pairs, ordered direct leaf
 * pairs}; m2l[2k], m2l[2k+1] = the k-th accepted pair (a, b) in traversal
 * order; p2p = ordered direct pairs (leaf, partner), leaves in node order and
 * partners in traversal order (itself included); zr = centre and radius per
 * node.  Outputs may be NULL (sizes only); m2l and p2p must hold the sizes.
 */
int oracle_dual_pairs(int64_t n, const double *xyz, const double *q, int leaf_max, double theta, int centre,
                      const double lo_in[3], double side_in, int64_t *sizes, int32_t *m2l, int32_t *p2p, double *zr)
{
    init_tables();
    if (!sizes || dual_check(n, leaf_max, theta, centre, q) != 0) return -1;
    oatree T;
    if (oa_make_tree(&T, n, xyz, q, 0, leaf_max, lo_in, side_in) != 0) { oa_free(&T); return -2; }
    oadual D;
    if (dual_setup(&D, &T, xyz, q, theta, centre) != 0) { dual_free(&D); oa_free(&T); return -2; }
    int64_t np = 0;
    for (int i = 0; i < T.nn; ++i) np += D.p2p[i].n;
    sizes[0] = T.nn;
    sizes[1] = D.m2l.n / 2;
    sizes[2] = np;
    if (m2l) memcpy(m2l, D.m2l.v, (size_t)D.m2l.n * sizeof(int32_t));
    if (p2p) {
        int64_t k = 0;
        for (int i = 0; i < T.nn; ++i)
            for (int j = 0; j < D.p2p[i].n; ++j) {
                p2p[2 * k] = i;
                p2p[2 * k + 1] = D.p2p[i].v[j];
                ++k;
            }
    }
    if (zr) memcpy(zr, D.zr, (size_t)T.nn * sizeof(double[4]));
    dual_free(&D);
    oa_free(&T);
    return 0;
}
