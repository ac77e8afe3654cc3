/*
 * CPU FP64 oracle for the rigid-multiblob blob mobility (test infrastructure).
 *
 * This file is test infrastructure: only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark load it.  It shares no code with the
 * GPU library.  It is deliberately plain: one 3x3 block per blob pair, written
 * straight from the definitions, summed in source-index order with Kahan
 * compensation, no blocking and no reordering.
 *
 * Definitions followed:
 *   - Free-space blob-blob mobility: the Rotne-Prager-Yamakawa tensor with its
 *     overlap branch (Sec. 2.1.1, eq:RPYTensor); self block I/(6 pi eta a).
 *   - Single no-slip wall at z = 0 (Sec. 2.1.1 and Sec. 5): RPY plus the
 *     translation-translation Rotne-Prager-Blake correction.  The paper cites
 *     but does not print that correction; it is the double Faxen operator
 *     (eq:MobilityFaxen) applied to the image part of Blake's half-space
 *     Green's function.  Written out, for target i, source j at height h = z_j,
 *     R = r_i - (x_j, y_j, -z_j), L = |R|, e = R/L, ez = e_z, xi = a/L,
 *     hh = h/L:
 *        W = (6 pi eta a)^-1 [c1 I + c2 e e^T + c3 e z^T + c4 z e^T + c5 z z^T]
 *        c1 = xi/4 [-3 - 6 ez hh + 6 hh^2 + 2 xi^2 (3 ez^2 - 1) + 2 xi^4 (1 - 5 ez^2)]
 *        c2 = xi/4 [-3 + 18 ez hh - 18 hh^2 + 6 xi^2 (1 - 5 ez^2) + 10 xi^4 (7 ez^2 - 1)]
 *        c3 = xi [3/2 hh (1 - 6 ez^2 + 6 ez hh) + 3 ez xi^2 (5 ez^2 - 1) + 5 ez xi^4 (2 - 7 ez^2)]
 *        c4 = xi [3/2 hh - 5 ez xi^4]
 *        c5 = xi [-3 hh^2 - 3 ez^2 xi^2 + xi^4 (15 ez^2 - 2)]
 *     Rows are velocity components of blob i, columns force components on
 *     blob j.  The overlap (r_ij <= 2a) correction stays the free-space one,
 *     as the paper states for blobs that overlap each other but not the wall.
 *     Pinned by: a symbolic re-derivation from Blake's image system, the
 *     self-mobility limit, decay of the correction with height, and the
 *     paper's Appendix D sphere-near-wall fits.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (see build.py).
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define ORACLE_PI 3.14159265358979323846

/* Free-space RPY 3x3 block of the pair (i, j) with r = r_i - r_j (eq:RPYTensor),
 * without the 1/(6 pi eta a) prefactor. */
static void rpy_block(const double r[3], double a, double B[9])
{
    double d = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    double ciso, crr;
    if (d > 2.0 * a) {
        ciso = 3.0 * a / (4.0 * d) + a * a * a / (2.0 * d * d * d);
        crr = 3.0 * a / (4.0 * d) - 3.0 * a * a * a / (2.0 * d * d * d);
    } else {
        ciso = 1.0 - 9.0 * d / (32.0 * a);
        crr = 3.0 * d / (32.0 * a);
    }
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) {
            double outer = (d > 0.0) ? r[p] * r[q] / (d * d) : 0.0;
            B[3 * p + q] = (p == q ? ciso : 0.0) + crr * outer;
        }
}

/* Wall (image) correction block of target r_i, source r_j, without the
 * 1/(6 pi eta a) prefactor.  Requires z_j > 0 and z_i > -z_j. */
static void wall_block(const double ri[3], const double rj[3], double a, double B[9])
{
    double R[3] = {ri[0] - rj[0], ri[1] - rj[1], ri[2] + rj[2]};
    double L = sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
    double e[3] = {R[0] / L, R[1] / L, R[2] / L};
    double ez = e[2];
    double xi = a / L;
    double hh = rj[2] / L;
    double xi2 = xi * xi, xi4 = xi2 * xi2, ez2 = ez * ez;
    double c1 = xi / 4.0 * (-3.0 - 6.0 * ez * hh + 6.0 * hh * hh + 2.0 * xi2 * (3.0 * ez2 - 1.0)
                            + 2.0 * xi4 * (1.0 - 5.0 * ez2));
    double c2 = xi / 4.0 * (-3.0 + 18.0 * ez * hh - 18.0 * hh * hh + 6.0 * xi2 * (1.0 - 5.0 * ez2)
                            + 10.0 * xi4 * (7.0 * ez2 - 1.0));
    double c3 = xi * (1.5 * hh * (1.0 - 6.0 * ez2 + 6.0 * ez * hh) + 3.0 * ez * xi2 * (5.0 * ez2 - 1.0)
                      + 5.0 * ez * xi4 * (2.0 - 7.0 * ez2));
    double c4 = xi * (1.5 * hh - 5.0 * ez * xi4);
    double c5 = xi * (-3.0 * hh * hh - 3.0 * ez2 * xi2 + xi4 * (15.0 * ez2 - 2.0));
    const double zh[3] = {0.0, 0.0, 1.0};
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q)
            B[3 * p + q] = (p == q ? c1 : 0.0) + c2 * e[p] * e[q] + c3 * e[p] * zh[q]
                           + c4 * zh[p] * e[q] + c5 * zh[p] * zh[q];
}

/* Full 3x3 mobility block M_ij (with prefactor).  wall != 0 adds the wall
 * correction. */
void oracle_pair_block(const double *ri, const double *rj, double a, double eta, int wall,
                       double *out)
{
    double r[3] = {ri[0] - rj[0], ri[1] - rj[1], ri[2] - rj[2]};
    double B[9], W[9];
    double pref = 1.0 / (6.0 * ORACLE_PI * eta * a);
    rpy_block(r, a, B);
    if (wall) {
        wall_block(ri, rj, a, W);
        for (int k = 0; k < 9; ++k) B[k] += W[k];
    }
    for (int k = 0; k < 9; ++k) out[k] = pref * B[k];
}

/* The wall correction block alone (with prefactor), for pin tests. */
void oracle_wall_block(const double *ri, const double *rj, double a, double eta, double *out)
{
    double W[9];
    double pref = 1.0 / (6.0 * ORACLE_PI * eta * a);
    wall_block(ri, rj, a, W);
    for (int k = 0; k < 9; ++k) out[k] = pref * W[k];
}

/* v_i = sum_j M_ij lambda_j for targets i in [i0, i1) against all sources,
 * positions and vectors as [n][3] row-major.  The j-sum runs in index order
 * with Kahan compensation per component. */
void oracle_matvec_rows(int64_t n_src, const double *r_src, const double *lam,
                        int64_t i0, int64_t i1, const double *r_tgt, double a, double eta,
                        int wall, double *v)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = i0; i < i1; ++i) {
        double s[3] = {0.0, 0.0, 0.0}, c[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < n_src; ++j) {
            double M[9];
            oracle_pair_block(&r_tgt[3 * i], &r_src[3 * j], a, eta, wall, M);
            for (int p = 0; p < 3; ++p) {
                double t = M[3 * p + 0] * lam[3 * j + 0] + M[3 * p + 1] * lam[3 * j + 1]
                           + M[3 * p + 2] * lam[3 * j + 2];
                double y = t - c[p];
                double u = s[p] + y;
                c[p] = (u - s[p]) - y;
                s[p] = u;
            }
        }
        v[3 * i + 0] = s[0];
        v[3 * i + 1] = s[1];
        v[3 * i + 2] = s[2];
    }
}

/* Full square mobility product over one set of blobs. */
void oracle_matvec(int64_t n, const double *r, const double *lam, double a, double eta, int wall,
                   double *v)
{
    oracle_matvec_rows(n, r, lam, 0, n, r, a, eta, wall, v);
}

/* Dense (3n x 3n) row-major mobility matrix of n blobs. */
void oracle_assemble(int64_t n, const double *r, double a, double eta, int wall, double *M)
{
    int64_t ld = 3 * n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double B[9];
            oracle_pair_block(&r[3 * i], &r[3 * j], a, eta, wall, B);
            for (int p = 0; p < 3; ++p)
                for (int q = 0; q < 3; ++q) M[(3 * i + p) * ld + 3 * j + q] = B[3 * p + q];
        }
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
