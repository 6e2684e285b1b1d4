/*
 * Plain FP64 CPU oracle for the spatially mixed force evaluation of ML-MIX
 * (Birks et al., arXiv 2502.19081).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the correctness reference that the
 * tests, the smoke check and the benchmark's CPU baseline call. The product
 * path (the HIP library) never includes, links or calls it, and it shares no
 * code, header or table with the HIP library.
 *
 * It is deliberately slow and literal: plain loops over atoms, neighbours and
 * basis functions, no blocking or fusion, every floating-point expression
 * written in the order the definition gives (build with -ffp-contract=off).
 *
 * What it computes, and the passage each part follows:
 *  - minimum-image pair distances and the neighbour set (the neighbour lists
 *    the region-tracking fix reuses; Methods, "Region tracking");
 *  - the mixing weight lambda and masks (Algorithms 1 and 2, generalised to
 *    geometric core regions; lambda = max over regions as in Algorithm 2);
 *  - the buffer set (Algorithm 3 and the buffer-set equation of "Spatial
 *    potential mixing": atoms outside the lambda>0 set within the buffer
 *    radius of one inside it);
 *  - the expensive potential on the induced subsystem S only (Algorithm 4
 *    and Fig. 10: atoms outside S are removed from the neighbour list);
 *  - forces as minus the derivative of the sum of site energies (the
 *    force/site-energy equation of "Spatial potential mixing", read with a
 *    minus sign);
 *  - the cheap potential on every atom;
 *  - the blend F = lambda F_exp + (1 - lambda) F_cheap (Algorithm 4).
 * The two potentials are synthetic stand-ins the paper does not define (it
 * cites ACE and UF3): an ACE-style model (Chebyshev radial x real spherical
 * harmonic atomic basis, product basis up to correlation order 3, linear
 * readout) and a UF3-style model (clamped cubic B-spline 2-body and 3-body).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Box and pair displacement                                                  */
/* ------------------------------------------------------------------------ */

/* d = x_j - x_i, folded once into [-L/2, L/2] along periodic dimensions. */
static void mi_disp(const double *L, const int32_t *per, const double *xi,
                    const double *xj, double *d)
{
    for (int k = 0; k < 3; ++k) {
        double dx = xj[k] - xi[k];
        if (per[k]) {
            double h = 0.5 * L[k];
            if (dx > h)
                dx = dx - L[k];
            else if (dx < -h)
                dx = dx + L[k];
        }
        d[k] = dx;
    }
}

static double norm2(const double *d)
{
    double s = d[0] * d[0];
    s = s + d[1] * d[1];
    s = s + d[2] * d[2];
    return s;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the later parallel regions (timing of the baseline only). */
void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Neighbour set: N(i) = { j != i : |d_ij|^2 < r_list^2 }, rows ascending.   */
/* method 0 = all pairs, method 1 = cell bins of edge >= r_list.             */
/* ------------------------------------------------------------------------ */

typedef struct {
    int nc[3];
    double cs[3];
    int64_t *start; /* ncell + 1 */
    int32_t *atoms;
} bins_t;

static int bins_build(bins_t *b, int n, const double *pos, const double *L,
                      double r_list)
{
    for (int k = 0; k < 3; ++k) {
        int nc = (int)floor(L[k] / r_list);
        if (nc < 1)
            nc = 1;
        b->nc[k] = nc;
        b->cs[k] = L[k] / nc;
    }
    int64_t ncell = (int64_t)b->nc[0] * b->nc[1] * b->nc[2];
    b->start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    b->atoms = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *cid = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!b->start || !b->atoms || !cid)
        return -1;
    for (int i = 0; i < n; ++i) {
        int c[3];
        for (int k = 0; k < 3; ++k) {
            int q = (int)floor(pos[3 * i + k] / b->cs[k]);
            if (q < 0)
                q = 0;
            if (q >= b->nc[k])
                q = b->nc[k] - 1;
            c[k] = q;
        }
        cid[i] = (c[2] * b->nc[1] + c[1]) * b->nc[0] + c[0];
        b->start[cid[i] + 1] += 1;
    }
    for (int64_t c = 0; c < ncell; ++c)
        b->start[c + 1] += b->start[c];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncell);
    memcpy(fill, b->start, sizeof(int64_t) * (size_t)ncell);
    for (int i = 0; i < n; ++i)
        b->atoms[fill[cid[i]]++] = i;
    free(fill);
    free(cid);
    return 0;
}

static void bins_free(bins_t *b)
{
    free(b->start);
    free(b->atoms);
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Visit the candidate partners of atom i. For each dimension the cell offsets
 * -1, 0, +1 are reduced to a set of distinct cells (periodic wrap) or clipped
 * (non-periodic), so no cell is visited twice. */
static int row_of(int i, int n, const double *pos, const double *L,
                  const int32_t *per, double rl2, int method, const bins_t *b,
                  int32_t *out)
{
    int cnt = 0;
    double d[3];
    if (method == 0) {
        for (int j = 0; j < n; ++j) {
            if (j == i)
                continue;
            mi_disp(L, per, pos + 3 * i, pos + 3 * j, d);
            if (norm2(d) < rl2) {
                if (out)
                    out[cnt] = j;
                cnt++;
            }
        }
        return cnt;
    }
    int ci[3];
    for (int k = 0; k < 3; ++k) {
        int q = (int)floor(pos[3 * i + k] / b->cs[k]);
        if (q < 0)
            q = 0;
        if (q >= b->nc[k])
            q = b->nc[k] - 1;
        ci[k] = q;
    }
    int lst[3][3], nl[3];
    for (int k = 0; k < 3; ++k) {
        nl[k] = 0;
        for (int o = -1; o <= 1; ++o) {
            int q = ci[k] + o;
            if (per[k]) {
                q = ((q % b->nc[k]) + b->nc[k]) % b->nc[k];
            } else if (q < 0 || q >= b->nc[k]) {
                continue;
            }
            int dup = 0;
            for (int t = 0; t < nl[k]; ++t)
                if (lst[k][t] == q)
                    dup = 1;
            if (!dup)
                lst[k][nl[k]++] = q;
        }
    }
    for (int a = 0; a < nl[2]; ++a)
        for (int bb = 0; bb < nl[1]; ++bb)
            for (int c = 0; c < nl[0]; ++c) {
                int64_t cell = ((int64_t)lst[2][a] * b->nc[1] + lst[1][bb]) * b->nc[0] + lst[0][c];
                for (int64_t s = b->start[cell]; s < b->start[cell + 1]; ++s) {
                    int j = b->atoms[s];
                    if (j == i)
                        continue;
                    mi_disp(L, per, pos + 3 * i, pos + 3 * j, d);
                    if (norm2(d) < rl2) {
                        if (out)
                            out[cnt] = j;
                        cnt++;
                    }
                }
            }
    if (out)
        qsort(out, (size_t)cnt, sizeof(int32_t), cmp_i32);
    return cnt;
}

/* Two-pass CSR build: offs must hold n+1 entries; nbr is filled when not NULL
 * (then offs must already hold the prefix sums returned by the first pass). */
int or_neighbors(int n, const double *pos, const double *L, const int32_t *per,
                 double r_list, int method, int64_t *offs, int32_t *nbr)
{
    bins_t b;
    memset(&b, 0, sizeof b);
    if (method == 1 && bins_build(&b, n, pos, L, r_list) != 0)
        return -1;
    double rl2 = r_list * r_list;
    if (nbr == NULL) {
        int32_t *cnt = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
#pragma omp parallel for schedule(dynamic, 64)
        for (int i = 0; i < n; ++i)
            cnt[i] = row_of(i, n, pos, L, per, rl2, method, &b, NULL);
        offs[0] = 0;
        for (int i = 0; i < n; ++i)
            offs[i + 1] = offs[i] + cnt[i];
        free(cnt);
    } else {
#pragma omp parallel for schedule(dynamic, 64)
        for (int i = 0; i < n; ++i)
            row_of(i, n, pos, L, per, rl2, method, &b, nbr + offs[i]);
    }
    if (method == 1)
        bins_free(&b);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Mixing weight (Algorithms 1-2 with geometric core regions).               */
/* Region g: type 0 = sphere about c, type 1 = infinite cylinder about the   */
/* coordinate axis `axis` through c. follow >= 0 replaces c by that atom's    */
/* position. b(d) = 1 for d < r_core, 1 - (d - r_core)/r_blend inside the    */
/* blend shell, 0 beyond; lambda_i = max_g b_g(d_ig).                         */
/* flags bit0: lambda > 0, bit1: lambda == 1.                                 */
/* ------------------------------------------------------------------------ */

/* Blend value at t in [0, 1) (distance into the blend shell over its width):
 * linear 1 - t (Algorithm 2), or the cubic 1 - 3 t^2 + 2 t^3, which has zero
 * slope at both ends (the paper offers a cubic option without printing it;
 * this is the reading adopted). */
static double blend_value(double t, int cubic)
{
    return cubic ? 1.0 - t * t * (3.0 - 2.0 * t) : 1.0 - t;
}

void or_lambda(int n, const double *pos, const double *L, const int32_t *per,
               int nreg, const int32_t *type, const int32_t *axis,
               const int32_t *follow, const double *center,
               const double *r_core, const double *r_blend, const int32_t *blend,
               double *lam, uint8_t *flags)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        double best = 0.0;
        for (int g = 0; g < nreg; ++g) {
            if (type[g] == 2)
                continue; /* seeded regions: or_lambda_seeded */
            const double *c = center + 3 * g;
            if (follow[g] >= 0)
                c = pos + 3 * follow[g];
            double d[3];
            mi_disp(L, per, c, pos + 3 * i, d);
            if (type[g] == 1)
                d[axis[g]] = 0.0;
            double d2 = norm2(d);
            double rc = r_core[g];
            double rb = r_blend[g];
            double outer = rc + rb;
            double b;
            if (d2 < rc * rc) {
                b = 1.0;
            } else if (d2 < outer * outer) {
                double dist = sqrt(d2);
                double t = (dist - rc) / rb;
                b = blend_value(t, blend[g]);
            } else {
                b = 0.0;
            }
            if (b > best)
                best = b;
        }
        lam[i] = best;
        uint8_t f = 0;
        if (best > 0.0)
            f |= 1;
        if (best == 1.0)
            f |= 2;
        flags[i] = f;
    }
}

/* Seeded regions, as the paper's fix builds them (Algorithms 1 and 2), over
 * the neighbour list, raising lam where a seeded region gives more:
 *  Algorithm 1: every seed atom, and every neighbour j of a seed i with
 *    |x_i - x_j| < r_core, is a core atom (lambda 1);
 *  Algorithm 2: for every core atom i and neighbour j with
 *    |x_i - x_j| = r < r_blend, lambda_j = max(lambda_j, b(r / r_blend)).
 * Each seeded region g (type 2) has its own r_core, r_blend and blend
 * function; all share the seed set. Distances: FP64 minimum image, strict
 * comparisons on the squared distance, r = sqrt(d2). Flags are rewritten
 * from the final lambda (bit0 lambda > 0, bit1 lambda == 1). */
void or_lambda_seeded(int n, const double *pos, const double *L, const int32_t *per,
                      const int64_t *offs, const int32_t *nbr, const uint8_t *seed,
                      int nreg, const int32_t *type, const double *r_core,
                      const double *r_blend, const int32_t *blend, double *lam,
                      uint8_t *flags)
{
    uint8_t *core = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    for (int g = 0; g < nreg; ++g) {
        if (type[g] != 2)
            continue;
        const double rc2 = r_core[g] * r_core[g], rb = r_blend[g], rb2 = rb * rb;
        /* Algorithm 1: scatter from the seeds */
        for (int i = 0; i < n; ++i)
            core[i] = 0;
        for (int i = 0; i < n; ++i) {
            if (!seed[i])
                continue;
            core[i] = 1;
            for (int64_t s = offs[i]; s < offs[i + 1]; ++s) {
                const int j = nbr[s];
                double d[3];
                mi_disp(L, per, pos + 3 * i, pos + 3 * j, d);
                if (norm2(d) < rc2)
                    core[j] = 1;
            }
        }
        for (int i = 0; i < n; ++i)
            if (core[i])
                lam[i] = 1.0;
        /* Algorithm 2: scatter from the core atoms, keeping the maximum */
        for (int i = 0; i < n; ++i) {
            if (!core[i])
                continue;
            for (int64_t s = offs[i]; s < offs[i + 1]; ++s) {
                const int j = nbr[s];
                double d[3];
                mi_disp(L, per, pos + 3 * i, pos + 3 * j, d);
                const double d2 = norm2(d);
                if (d2 < rb2) {
                    const double v = blend_value(sqrt(d2) / rb, blend[g]);
                    if (v > lam[j])
                        lam[j] = v;
                }
            }
        }
    }
    free(core);
    for (int i = 0; i < n; ++i) {
        uint8_t f = 0;
        if (lam[i] > 0.0)
            f |= 1;
        if (lam[i] == 1.0)
            f |= 2;
        flags[i] = f;
    }
}

/* Buffer (Algorithm 3 and the buffer-set equation): an atom with lambda == 0
 * joins the buffer (flags bit2) when some neighbour j with lambda_j > 0 lies
 * strictly closer than r_buffer. Requires r_buffer <= the list radius. */
void or_buffer(int n, const double *pos, const double *L, const int32_t *per,
               const int64_t *offs, const int32_t *nbr, double r_buffer,
               const double *lam, uint8_t *flags)
{
    double rb2 = r_buffer * r_buffer;
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < n; ++i) {
        if (lam[i] > 0.0)
            continue;
        for (int64_t s = offs[i]; s < offs[i + 1]; ++s) {
            int j = nbr[s];
            if (!(lam[j] > 0.0))
                continue;
            double d[3];
            mi_disp(L, per, pos + 3 * i, pos + 3 * j, d);
            if (norm2(d) < rb2) {
                flags[i] |= 4;
                break;
            }
        }
    }
}

/* The cheap potential's own buffer when it is masked like the expensive one
 * (Algorithm 4 for potential 1, whose weight is 1 - lambda): an atom with
 * lambda == 1 joins it (flags bit3) when some neighbour j with lambda_j < 1
 * lies strictly closer than r_buffer. The cheap subsystem is then
 * {lambda < 1} plus these atoms. */
void or_cheap_buffer(int n, const double *pos, const double *L, const int32_t *per,
                     const int64_t *offs, const int32_t *nbr, double r_buffer,
                     const double *lam, uint8_t *flags)
{
    double rb2 = r_buffer * r_buffer;
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < n; ++i) {
        if (!(lam[i] == 1.0))
            continue;
        for (int64_t s = offs[i]; s < offs[i + 1]; ++s) {
            int j = nbr[s];
            if (lam[j] == 1.0)
                continue;
            double d[3];
            mi_disp(L, per, pos + 3 * i, pos + 3 * j, d);
            if (norm2(d) < rb2) {
                flags[i] |= 8;
                break;
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Special functions for the ACE-style model                                  */
/* ------------------------------------------------------------------------ */

static double fact(int k)
{
    double f = 1.0;
    for (int i = 2; i <= k; ++i)
        f *= (double)i;
    return f;
}

/* Q_l^m(z) = d^m P_l(z) / dz^m from the explicit expansion
 * P_l(z) = sum_k (-1)^k (2l-2k)! / (2^l k! (l-k)! (l-2k)!) z^(l-2k). */
static double legendre_dm(int l, int m, double z)
{
    if (m > l)
        return 0.0;
    double s = 0.0;
    for (int k = 0; 2 * k <= l - m; ++k) {
        double c = fact(2 * l - 2 * k) / (pow(2.0, l) * fact(k) * fact(l - k) * fact(l - 2 * k - m));
        if (k & 1)
            c = -c;
        s += c * pow(z, l - 2 * k - m);
    }
    return s;
}

/* Real orthonormal spherical harmonics of a unit vector u, no Condon-Shortley
 * phase: m > 0: sqrt2 N Q_l^m(u_z) Re (u_x + i u_y)^m; m = 0: N Q_l^0(u_z);
 * m < 0: sqrt2 N Q_l^|m|(u_z) Im (u_x + i u_y)^|m|; N = sqrt((2l+1)/(4pi)
 * (l-|m|)!/(l+|m|)!). Index lm = l^2 + l + m. gu (optional) is the gradient
 * of the polynomial extension with respect to (u_x, u_y, u_z). */
void or_ylm(int lmax, const double *u, double *Y, double *gu)
{
    double C[32], S[32];
    C[0] = 1.0;
    S[0] = 0.0;
    for (int m = 1; m <= lmax; ++m) {
        C[m] = C[m - 1] * u[0] - S[m - 1] * u[1];
        S[m] = S[m - 1] * u[0] + C[m - 1] * u[1];
    }
    for (int l = 0; l <= lmax; ++l) {
        for (int m = -l; m <= l; ++m) {
            int am = m < 0 ? -m : m;
            double N = sqrt((2.0 * l + 1.0) / (4.0 * OR_PI) * fact(l - am) / fact(l + am));
            double q = legendre_dm(l, am, u[2]);
            double dq = legendre_dm(l, am + 1, u[2]);
            double t, tx, ty;
            if (m > 0) {
                t = sqrt(2.0) * C[am];
                tx = sqrt(2.0) * am * C[am - 1];
                ty = -sqrt(2.0) * am * S[am - 1];
            } else if (m < 0) {
                t = sqrt(2.0) * S[am];
                tx = sqrt(2.0) * am * S[am - 1];
                ty = sqrt(2.0) * am * C[am - 1];
            } else {
                t = 1.0;
                tx = 0.0;
                ty = 0.0;
            }
            int lm = l * l + l + m;
            Y[lm] = N * q * t;
            if (gu) {
                gu[3 * lm + 0] = N * q * tx;
                gu[3 * lm + 1] = N * q * ty;
                gu[3 * lm + 2] = N * dq * t;
            }
        }
    }
}

/* Chebyshev radial basis with a (1 - (r/rc)^2)^2 envelope:
 * R_n(r) = T_n(2r/rc - 1) (1 - (r/rc)^2)^2 and dR_n/dr. */
void or_radial(int n_rad, double rc, double r, double *R, double *dR)
{
    double x = 2.0 * r / rc - 1.0;
    double s = r / rc;
    double w = 1.0 - s * s;
    double f = w * w;
    double df = 2.0 * w * (-2.0 * s / rc);
    double T[64], U[64];
    T[0] = 1.0;
    U[0] = 1.0;
    if (n_rad > 1) {
        T[1] = x;
        U[1] = 2.0 * x;
    }
    for (int n = 2; n < n_rad; ++n) {
        T[n] = 2.0 * x * T[n - 1] - T[n - 2];
        U[n] = 2.0 * x * U[n - 1] - U[n - 2];
    }
    for (int n = 0; n < n_rad; ++n) {
        double dT = (n == 0) ? 0.0 : n * U[n - 1]; /* T_n' = n U_{n-1} */
        R[n] = T[n] * f;
        dR[n] = dT * (2.0 / rc) * f + T[n] * df;
    }
}

/* Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration. */
static void gauss_legendre(int N, double *x, double *w)
{
    for (int i = 0; i < N; ++i) {
        double z = cos(OR_PI * (i + 0.75) / (N + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= N; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            double dp = N * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16)
                break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= N; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        double dp = N * (z * p1 - p0) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* Real Gaunt table G[lm1][lm2][lm3] = integral over the sphere of
 * Y_lm1 Y_lm2 Y_lm3, by Gauss-Legendre quadrature in cos(theta) times the
 * uniform rule in phi, both exact for the degrees involved. */
void or_gaunt_table(int lmax, double *G)
{
    int L2 = (lmax + 1) * (lmax + 1);
    int Nz = 2 * lmax + 2, Np = 4 * lmax + 4;
    double *zx = (double *)malloc(sizeof(double) * Nz);
    double *zw = (double *)malloc(sizeof(double) * Nz);
    double *Y = (double *)malloc(sizeof(double) * L2);
    gauss_legendre(Nz, zx, zw);
    memset(G, 0, sizeof(double) * (size_t)L2 * L2 * L2);
    for (int a = 0; a < Nz; ++a) {
        for (int b = 0; b < Np; ++b) {
            double phi = 2.0 * OR_PI * b / Np;
            double st = sqrt(1.0 - zx[a] * zx[a]);
            double u[3] = {st * cos(phi), st * sin(phi), zx[a]};
            or_ylm(lmax, u, Y, NULL);
            double w = zw[a] * 2.0 * OR_PI / Np;
            for (int i = 0; i < L2; ++i)
                for (int j = 0; j < L2; ++j)
                    for (int k = 0; k < L2; ++k)
                        G[((size_t)i * L2 + j) * L2 + k] += w * Y[i] * Y[j] * Y[k];
        }
    }
    free(zx);
    free(zw);
    free(Y);
}

/* ------------------------------------------------------------------------ */
/* ACE-style expensive potential on the induced subsystem                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t n_species, n_rad, lmax, order;
    double rcut;
    const double *c0; /* [ns] */
    const double *c1; /* [ns][nchan] */
    const double *c2; /* [ns][lmax+1][nchan][nchan], a <= b read */
    const double *c3; /* [ns][K][K][K], K = nchan*(lmax+1), p <= q <= r read */
} or_ace_model;

typedef struct {
    int l1, l2, l3, n;
    int *m1, *m2, *m3; /* lm indices */
    double *g;
} gaunt_list;

static gaunt_list *gaunt_lists(int lmax)
{
    int L1 = lmax + 1, L2 = L1 * L1;
    double *G = (double *)malloc(sizeof(double) * (size_t)L2 * L2 * L2);
    or_gaunt_table(lmax, G);
    gaunt_list *gl = (gaunt_list *)calloc((size_t)L1 * L1 * L1, sizeof(gaunt_list));
    for (int l1 = 0; l1 <= lmax; ++l1)
        for (int l2 = 0; l2 <= lmax; ++l2)
            for (int l3 = 0; l3 <= lmax; ++l3) {
                gaunt_list *e = &gl[(l1 * L1 + l2) * L1 + l3];
                e->l1 = l1;
                e->l2 = l2;
                e->l3 = l3;
                int cap = (2 * l1 + 1) * (2 * l2 + 1) * (2 * l3 + 1);
                e->m1 = (int *)malloc(sizeof(int) * cap);
                e->m2 = (int *)malloc(sizeof(int) * cap);
                e->m3 = (int *)malloc(sizeof(int) * cap);
                e->g = (double *)malloc(sizeof(double) * cap);
                e->n = 0;
                for (int a = l1 * l1; a < (l1 + 1) * (l1 + 1); ++a)
                    for (int b = l2 * l2; b < (l2 + 1) * (l2 + 1); ++b)
                        for (int c = l3 * l3; c < (l3 + 1) * (l3 + 1); ++c) {
                            double v = G[((size_t)a * L2 + b) * L2 + c];
                            if (fabs(v) > 1e-12) {
                                e->m1[e->n] = a;
                                e->m2[e->n] = b;
                                e->m3[e->n] = c;
                                e->g[e->n] = v;
                                e->n++;
                            }
                        }
            }
    free(G);
    return gl;
}

static void gaunt_lists_free(gaunt_list *gl, int lmax)
{
    int L1 = lmax + 1;
    for (int i = 0; i < L1 * L1 * L1; ++i) {
        free(gl[i].m1);
        free(gl[i].m2);
        free(gl[i].m3);
        free(gl[i].g);
    }
    free(gl);
}

/* Site energy E_i = c0 + sum_k c_k B_k and dE_i/dA by differentiating each
 * product basis function (product rule), for centre species z. A and dA are
 * [nchan][L2]. */
static double ace_site(const or_ace_model *m, const gaunt_list *gl, int z,
                       const double *A, double *dA)
{
    int nchan = m->n_species * m->n_rad;
    int L1 = m->lmax + 1, L2 = L1 * L1, K = nchan * L1;
    memset(dA, 0, sizeof(double) * (size_t)nchan * L2);
    double E = m->c0[z];
    if (m->order >= 1) {
        for (int a = 0; a < nchan; ++a) {
            double c = m->c1[(size_t)z * nchan + a];
            E += c * A[a * L2 + 0];
            dA[a * L2 + 0] += c;
        }
    }
    if (m->order >= 2) {
        for (int l = 0; l <= m->lmax; ++l)
            for (int a = 0; a < nchan; ++a)
                for (int b = a; b < nchan; ++b) {
                    double c = m->c2[(((size_t)z * L1 + l) * nchan + a) * nchan + b];
                    double s = 0.0;
                    for (int lm = l * l; lm < (l + 1) * (l + 1); ++lm)
                        s += A[a * L2 + lm] * A[b * L2 + lm];
                    E += c * s;
                    for (int lm = l * l; lm < (l + 1) * (l + 1); ++lm) {
                        dA[a * L2 + lm] += c * A[b * L2 + lm];
                        dA[b * L2 + lm] += c * A[a * L2 + lm];
                    }
                }
    }
    if (m->order >= 3) {
        for (int p = 0; p < K; ++p)
            for (int q = p; q < K; ++q)
                for (int r = q; r < K; ++r) {
                    int a = p / L1, l1 = p % L1;
                    int b = q / L1, l2 = q % L1;
                    int cc = r / L1, l3 = r % L1;
                    if ((l1 + l2 + l3) & 1)
                        continue;
                    if (l3 > l1 + l2 || l3 < abs(l1 - l2))
                        continue;
                    double c = m->c3[(((size_t)z * K + p) * K + q) * K + r];
                    const gaunt_list *e = &gl[(l1 * L1 + l2) * L1 + l3];
                    double s = 0.0;
                    for (int t = 0; t < e->n; ++t) {
                        double x1 = A[a * L2 + e->m1[t]];
                        double x2 = A[b * L2 + e->m2[t]];
                        double x3 = A[cc * L2 + e->m3[t]];
                        s += e->g[t] * x1 * x2 * x3;
                        dA[a * L2 + e->m1[t]] += c * e->g[t] * x2 * x3;
                        dA[b * L2 + e->m2[t]] += c * e->g[t] * x1 * x3;
                        dA[cc * L2 + e->m3[t]] += c * e->g[t] * x1 * x2;
                    }
                    E += c * s;
                }
    }
    return E;
}

/* Evaluate the ACE-style potential on the subsystem S (in_S[i] != 0; NULL =
 * every atom). Pairs are (i, j) with both in S and r_ij < rcut. Outputs:
 * e_out[i] = E_i for i in S (0 otherwise), f_out[3i+k] = -d(sum_i w_i E_i)/dx_ik
 * for i in S (0 otherwise), with w_i = weights[i] or 1 when weights is NULL.
 * target (optional): only forces of atoms with target[i] != 0 are required;
 * site energies are then formed for those atoms and their S-neighbours only,
 * and f_out/e_out are meaningful on target atoms only (others 0). */
int or_ace_eval(const or_ace_model *m, int n, const double *pos,
                const int32_t *species, const double *L, const int32_t *per,
                const int64_t *offs, const int32_t *nbr, const uint8_t *in_S,
                const uint8_t *target, const double *weights, double *e_out,
                double *f_out)
{
    int nchan = m->n_species * m->n_rad;
    int L1 = m->lmax + 1, L2 = L1 * L1;
    int KA = nchan * L2;
    double rc2 = m->rcut * m->rcut;
    gaunt_list *gl = gaunt_lists(m->lmax);
    uint8_t *need = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    for (int i = 0; i < n; ++i) {
        if (in_S && !in_S[i])
            continue;
        if (!target || target[i]) {
            need[i] = 1;
            if (target) {
                for (int64_t s = offs[i]; s < offs[i + 1]; ++s) {
                    int j = nbr[s];
                    if (in_S && !in_S[j])
                        continue;
                    double d[3];
                    mi_disp(L, per, pos + 3 * i, pos + 3 * j, d);
                    if (norm2(d) < rc2)
                        need[j] = 1;
                }
            }
        }
    }
    int64_t npair = offs[n];
    double *g = (double *)calloc((size_t)(npair > 0 ? npair : 1) * 3, sizeof(double));
    memset(e_out, 0, sizeof(double) * (size_t)n);
    memset(f_out, 0, sizeof(double) * 3 * (size_t)n);
#pragma omp parallel
    {
        double *A = (double *)malloc(sizeof(double) * KA);
        double *dA = (double *)malloc(sizeof(double) * KA);
        double R[64], dR[64];
        double *Y = (double *)malloc(sizeof(double) * L2);
        double *gu = (double *)malloc(sizeof(double) * 3 * L2);
#pragma omp for schedule(dynamic, 4)
        for (int i = 0; i < n; ++i) {
            if (!need[i])
                continue;
            memset(A, 0, sizeof(double) * KA);
            for (int64_t s = offs[i]; s < offs[i + 1]; ++s) {
                int j = nbr[s];
                if (in_S && !in_S[j])
                    continue;
                double d[3];
                mi_disp(L, per, pos + 3 * i, pos + 3 * j, d);
                double r2 = norm2(d);
                if (!(r2 < rc2))
                    continue;
                double r = sqrt(r2);
                double u[3] = {d[0] / r, d[1] / r, d[2] / r};
                or_radial(m->n_rad, m->rcut, r, R, dR);
                or_ylm(m->lmax, u, Y, NULL);
                int zj = species[j];
                for (int nn = 0; nn < m->n_rad; ++nn)
                    for (int lm = 0; lm < L2; ++lm)
                        A[(zj * m->n_rad + nn) * L2 + lm] += R[nn] * Y[lm];
            }
            double E = ace_site(m, gl, species[i], A, dA);
            double w = weights ? weights[i] : 1.0;
            e_out[i] = E;
            for (int64_t s = offs[i]; s < offs[i + 1]; ++s) {
                int j = nbr[s];
                if (in_S && !in_S[j])
                    continue;
                double d[3];
                mi_disp(L, per, pos + 3 * i, pos + 3 * j, d);
                double r2 = norm2(d);
                if (!(r2 < rc2))
                    continue;
                double r = sqrt(r2);
                double u[3] = {d[0] / r, d[1] / r, d[2] / r};
                or_radial(m->n_rad, m->rcut, r, R, dR);
                or_ylm(m->lmax, u, Y, gu);
                int zj = species[j];
                double gx = 0.0, gy = 0.0, gz = 0.0;
                for (int lm = 0; lm < L2; ++lm) {
                    /* gradient of Y(d/|d|) w.r.t. d: (I - u u^T) gu / r */
                    double ud = u[0] * gu[3 * lm] + u[1] * gu[3 * lm + 1] + u[2] * gu[3 * lm + 2];
                    double gY[3];
                    for (int k = 0; k < 3; ++k)
                        gY[k] = (gu[3 * lm + k] - u[k] * ud) / r;
                    for (int nn = 0; nn < m->n_rad; ++nn) {
                        double c = dA[(zj * m->n_rad + nn) * L2 + lm];
                        /* d/dd [R_n(r) Y(u)] = R_n' u Y + R_n grad Y */
                        gx += c * (dR[nn] * u[0] * Y[lm] + R[nn] * gY[0]);
                        gy += c * (dR[nn] * u[1] * Y[lm] + R[nn] * gY[1]);
                        gz += c * (dR[nn] * u[2] * Y[lm] + R[nn] * gY[2]);
                    }
                }
                g[3 * s + 0] = w * gx;
                g[3 * s + 1] = w * gy;
                g[3 * s + 2] = w * gz;
            }
        }
        free(A);
        free(dA);
        free(Y);
        free(gu);
    }
    /* g_ij = dE_i/d(x_j - x_i): F_i += g_ij, F_j -= g_ij. */
    for (int i = 0; i < n; ++i) {
        if (!need[i])
            continue;
        for (int64_t s = offs[i]; s < offs[i + 1]; ++s) {
            int j = nbr[s];
            for (int k = 0; k < 3; ++k) {
                f_out[3 * i + k] += g[3 * s + k];
                f_out[3 * j + k] -= g[3 * s + k];
            }
        }
    }
    if (target) {
        for (int i = 0; i < n; ++i)
            if (!target[i]) {
                e_out[i] = 0.0;
                f_out[3 * i] = f_out[3 * i + 1] = f_out[3 * i + 2] = 0.0;
            }
    }
    free(g);
    free(need);
    gaunt_lists_free(gl, m->lmax);
    return 0;
}

/* Site-energy derivative dE_i/dA for one given A vector (test hook). */
double or_ace_site(const or_ace_model *m, int z, const double *A, double *dA)
{
    gaunt_list *gl = gaunt_lists(m->lmax);
    double E = ace_site(m, gl, z, A, dA);
    gaunt_lists_free(gl, m->lmax);
    return E;
}

/* ------------------------------------------------------------------------ */
/* UF3-style cheap potential                                                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t n_species, n_knots2, n_knots3, pad;
    double rcut2, rcut3;
    const double *c2; /* [ns][ns][n_knots2+2] */
    const double *c3; /* [ns][nb3][nb3][nb3], nb3 = n_knots3+2 */
} or_uf3_model;

/* Clamped knot vector: n_pts uniform points on [0, top], end points repeated
 * so that each appears four times; length n_pts + 6. */
static void clamped_knots(int n_pts, double top, double *t)
{
    for (int i = 0; i < n_pts + 6; ++i) {
        int k = i - 3;
        if (k < 0)
            k = 0;
        if (k > n_pts - 1)
            k = n_pts - 1;
        t[i] = top * k / (n_pts - 1);
    }
}

/* All cubic B-spline basis functions and derivatives at x by the Cox-de Boor
 * recursion over the knot vector t of length nt (nt - 4 functions). */
void or_bspline(const double *t, int nt, double x, double *B, double *dB)
{
    double N[4][80];
    int nb0 = nt - 1;
    for (int i = 0; i < nb0; ++i)
        N[0][i] = (t[i] <= x && x < t[i + 1]) ? 1.0 : 0.0;
    for (int k = 1; k <= 3; ++k) {
        for (int i = 0; i < nt - 1 - k; ++i) {
            double a = 0.0, b = 0.0;
            double den1 = t[i + k] - t[i];
            double den2 = t[i + k + 1] - t[i + 1];
            if (den1 > 0.0)
                a = (x - t[i]) / den1 * N[k - 1][i];
            if (den2 > 0.0)
                b = (t[i + k + 1] - x) / den2 * N[k - 1][i + 1];
            N[k][i] = a + b;
        }
    }
    int nb = nt - 4;
    for (int i = 0; i < nb; ++i) {
        B[i] = N[3][i];
        double a = 0.0, b = 0.0;
        double den1 = t[i + 3] - t[i];
        double den2 = t[i + 4] - t[i + 1];
        if (den1 > 0.0)
            a = 3.0 / den1 * N[2][i];
        if (den2 > 0.0)
            b = 3.0 / den2 * N[2][i + 1];
        dB[i] = a - b;
    }
}

void or_clamped_knots(int n_pts, double top, double *t) { clamped_knots(n_pts, top, t); }

/* E_i = 1/2 sum_{j, r_ij < rc2} V2^{z_i z_j}(r_ij)
 *     + sum_{j < k; r_ij, r_ik < rc3} V3^{z_i}(r_ij, r_ik, r_jk),
 * V2 = sum_n c2[z_i][z_j][n] B_n(r), V3 = sum_pqs c3[z_i][p][q][s] B_p(r_ij)
 * B_q(r_ik) B_s(r_jk), r_jk = |d_ik - d_ij|; forces = -grad of sum_i E_i.
 * With in_S (NULL = every atom) the potential sees the induced subsystem
 * only, as Algorithm 4 removes the atoms of the other potential from the
 * neighbour list: atoms outside S are neither centres nor neighbours. */
int or_uf3_eval(const or_uf3_model *m, int n, const double *pos,
                const int32_t *species, const double *L, const int32_t *per,
                const int64_t *offs, const int32_t *nbr, const uint8_t *target,
                const uint8_t *in_S, double *e_out, double *f_out)
{
    int ns = m->n_species;
    int nb2 = m->n_knots2 + 2;
    int nb3 = m->n_knots3 > 0 ? m->n_knots3 + 2 : 0;
    double t2[80], t3a[80], t3c[80];
    clamped_knots(m->n_knots2, m->rcut2, t2);
    if (nb3) {
        clamped_knots(m->n_knots3, m->rcut3, t3a);
        clamped_knots(m->n_knots3, 2.0 * m->rcut3, t3c);
    }
    double rc2 = m->rcut2 * m->rcut2, rc3 = m->rcut3 * m->rcut3;
    uint8_t *need = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    double rmax = m->rcut2 > m->rcut3 ? m->rcut2 : m->rcut3;
    for (int i = 0; i < n; ++i) {
        if ((!target || target[i]) && (!in_S || in_S[i])) {
            need[i] = 1;
            if (target)
                for (int64_t s = offs[i]; s < offs[i + 1]; ++s) {
                    double d[3];
                    mi_disp(L, per, pos + 3 * i, pos + 3 * nbr[s], d);
                    if (norm2(d) < rmax * rmax && (!in_S || in_S[nbr[s]]))
                        need[nbr[s]] = 1;
                }
        }
    }
    int64_t npair = offs[n];
    double *h = (double *)calloc((size_t)(npair > 0 ? npair : 1) * 3, sizeof(double));
    memset(e_out, 0, sizeof(double) * (size_t)n);
    memset(f_out, 0, sizeof(double) * 3 * (size_t)n);
#pragma omp parallel
    {
        double B[80], dB[80], Bq[80], dBq[80], Bs[80], dBs[80];
#pragma omp for schedule(dynamic, 16)
        for (int i = 0; i < n; ++i) {
            if (!need[i])
                continue;
            int zi = species[i];
            double E = 0.0;
            int64_t s0 = offs[i], s1 = offs[i + 1];
            for (int64_t s = s0; s < s1; ++s) {
                int j = nbr[s];
                if (in_S && !in_S[j])
                    continue;
                double d[3];
                mi_disp(L, per, pos + 3 * i, pos + 3 * j, d);
                double r2 = norm2(d);
                if (!(r2 < rc2))
                    continue;
                double r = sqrt(r2);
                or_bspline(t2, m->n_knots2 + 6, r, B, dB);
                const double *c = m->c2 + ((size_t)zi * ns + species[j]) * nb2;
                double V = 0.0, dV = 0.0;
                for (int q = 0; q < nb2; ++q) {
                    V += c[q] * B[q];
                    dV += c[q] * dB[q];
                }
                E += 0.5 * V;
                for (int k = 0; k < 3; ++k)
                    h[3 * s + k] += 0.5 * dV * d[k] / r;
            }
            if (nb3) {
                const double *c3 = m->c3 + (size_t)zi * nb3 * nb3 * nb3;
                for (int64_t sj = s0; sj < s1; ++sj) {
                    if (in_S && !in_S[nbr[sj]])
                        continue;
                    double dj[3];
                    mi_disp(L, per, pos + 3 * i, pos + 3 * nbr[sj], dj);
                    double rj2 = norm2(dj);
                    if (!(rj2 < rc3))
                        continue;
                    for (int64_t sk = sj + 1; sk < s1; ++sk) {
                        if (in_S && !in_S[nbr[sk]])
                            continue;
                        double dk[3];
                        mi_disp(L, per, pos + 3 * i, pos + 3 * nbr[sk], dk);
                        double rk2 = norm2(dk);
                        if (!(rk2 < rc3))
                            continue;
                        double rj = sqrt(rj2), rk = sqrt(rk2);
                        double e[3] = {dk[0] - dj[0], dk[1] - dj[1], dk[2] - dj[2]};
                        double rjk = sqrt(norm2(e));
                        or_bspline(t3a, m->n_knots3 + 6, rj, B, dB);
                        or_bspline(t3a, m->n_knots3 + 6, rk, Bq, dBq);
                        or_bspline(t3c, m->n_knots3 + 6, rjk, Bs, dBs);
                        double V = 0.0, V1 = 0.0, V2 = 0.0, V3 = 0.0;
                        for (int p = 0; p < nb3; ++p)
                            for (int q = 0; q < nb3; ++q)
                                for (int t = 0; t < nb3; ++t) {
                                    double c = c3[((size_t)p * nb3 + q) * nb3 + t];
                                    V += c * B[p] * Bq[q] * Bs[t];
                                    V1 += c * dB[p] * Bq[q] * Bs[t];
                                    V2 += c * B[p] * dBq[q] * Bs[t];
                                    V3 += c * B[p] * Bq[q] * dBs[t];
                                }
                        E += V;
                        for (int k = 0; k < 3; ++k) {
                            /* d r_jk / d d_ij = -(d_ik - d_ij)/r_jk */
                            h[3 * sj + k] += V1 * dj[k] / rj - V3 * e[k] / rjk;
                            h[3 * sk + k] += V2 * dk[k] / rk + V3 * e[k] / rjk;
                        }
                    }
                }
            }
            e_out[i] = E;
        }
    }
    for (int i = 0; i < n; ++i) {
        if (!need[i])
            continue;
        for (int64_t s = offs[i]; s < offs[i + 1]; ++s) {
            int j = nbr[s];
            for (int k = 0; k < 3; ++k) {
                f_out[3 * i + k] += h[3 * s + k];
                f_out[3 * j + k] -= h[3 * s + k];
            }
        }
    }
    if (target)
        for (int i = 0; i < n; ++i)
            if (!target[i]) {
                e_out[i] = 0.0;
                f_out[3 * i] = f_out[3 * i + 1] = f_out[3 * i + 2] = 0.0;
            }
    free(h);
    free(need);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Blend (Algorithm 4) and compensated sums                                  */
/* ------------------------------------------------------------------------ */

void or_blend(int n, const double *lam, const double *fe, const double *fc,
              double *f)
{
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k)
            f[3 * i + k] = lam[i] * fe[3 * i + k] + (1.0 - lam[i]) * fc[3 * i + k];
}

/* Neumaier-compensated sum. */
double or_sum(int n, const double *x)
{
    double s = 0.0, c = 0.0;
    for (int i = 0; i < n; ++i) {
        double t = s + x[i];
        if (fabs(s) >= fabs(x[i]))
            c += (s - t) + x[i];
        else
            c += (x[i] - t) + s;
        s = t;
    }
    return s + c;
}
