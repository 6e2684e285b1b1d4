// Constrained linear fitting of the cheap potential on gfx950 (Methods,
// "Constrained potential fitting").
//
// The cheap potential is linear in its free spline coefficients u, so a
// configuration's energy and forces are A u for a design matrix A. Three
// kernels build and solve the fit:
//  - k_fit_design: one wavefront per atom i produces the derivatives of F_i
//    (three rows) and of the site energy E_i by every parameter. Lane t owns
//    parameter columns t and t + 64. Interactions are produced 64 at a time
//    (one per lane) as records in LDS and then consumed by every lane for its
//    own columns, so each output element is a sum in a fixed order (no
//    atomics). F_i collects the pairs of i, the triplets centred on i, and the
//    triplets centred on a neighbour j in which i is a leg.
//  - k_fit_gram_partial / k_fit_gram_reduce: G = A^T diag(w) A and
//    b = A^T diag(w) y. Each workgroup stages 32 rows at a time in LDS and
//    every thread accumulates 4 x 4 blocks of the upper triangle; partials of
//    fixed row chunks are summed in chunk order.
//  - k_fit_search: one workgroup runs the whole lambda search: the normal
//    equations (G_S + lam G_H + ridge I) c = b_S + lam b_H solved by a
//    Cholesky factorisation held packed in LDS, the hard residual
//    ||A_H c - y_H||^2 from the hard rows, decades of lam until the residual
//    is at most alpha, then interval bisection until it is within tol of
//    alpha. Every loop has a fixed bound.
// Everything is FP64 whatever the context's force precision.
#include "internal.h"

namespace mlmix {

constexpr int kFitWave = 64;
constexpr int kFitColsPerLane = 2;  // columns per lane: kFitMaxParams <= 128

// ---------------------------------------------------------------- B-splines

__device__ __forceinline__ double fit_knot(int i, int npts, double top)
{
    int k = i - 3;
    k = k < 0 ? 0 : (k > npts - 1 ? npts - 1 : k);
    return top * (double)k / (double)(npts - 1);
}

// The four non-zero clamped uniform cubic B-splines at x (0 <= x < top) and
// their derivatives, by the Cox-de Boor triangle on the span holding x; the
// functions are B_first .. B_first+3.
__device__ void fit_bspline(double x, int npts, double top, int &first, double N[4], double dN[4])
{
    const double h = top / (double)(npts - 1);
    int sp = (int)floor(x / h);
    sp = sp < 0 ? 0 : (sp > npts - 2 ? npts - 2 : sp);
    const int mu = sp + 3;
    double B[4] = {1.0, 0.0, 0.0, 0.0}, B2[3] = {0.0, 0.0, 0.0};
    double left[4], right[4];
    for (int j = 1; j <= 3; ++j) {
        left[j] = x - fit_knot(mu + 1 - j, npts, top);
        right[j] = fit_knot(mu + j, npts, top) - x;
        double saved = 0.0;
        for (int r = 0; r < j; ++r) {
            const double tmp = B[r] / (right[r + 1] + left[j - r]);
            B[r] = saved + right[r + 1] * tmp;
            saved = left[j - r] * tmp;
        }
        B[j] = saved;
        if (j == 2) {
            B2[0] = B[0];
            B2[1] = B[1];
            B2[2] = B[2];
        }
    }
    // derivative of B_k = 3 (B2_k / (t_k+3 - t_k) - B2_k+1 / (t_k+4 - t_k+1)),
    // with the degree-2 functions B2_{mu-2..mu} non-zero
    for (int r = 0; r < 4; ++r) {
        const int k = mu - 3 + r;
        const double a = r >= 1 ? B2[r - 1] / (fit_knot(k + 3, npts, top) - fit_knot(k, npts, top)) : 0.0;
        const double b = r <= 2 ? B2[r] / (fit_knot(k + 4, npts, top) - fit_knot(k + 1, npts, top)) : 0.0;
        N[r] = B[r];
        dN[r] = 3.0 * (a - b);
    }
    first = sp;
}

__device__ __forceinline__ double fit_win(const double *v, int first, int idx)
{
    const unsigned o = (unsigned)(idx - first);
    return o < 4u ? v[o] : 0.0;
}

__device__ __forceinline__ double fit_disp(const double *__restrict__ pos, int n, int i, int j,
                                           const Box &b, double d[3])
{
#pragma clang fp contract(off)
    for (int k = 0; k < 3; ++k) {
        double dx = pos[k * n + j] - pos[k * n + i];
        if (b.per[k]) {
            const double hh = 0.5 * b.L[k];
            dx = dx > hh ? dx - b.L[k] : (dx < -hh ? dx + b.L[k] : dx);
        }
        d[k] = dx;
    }
    double r2 = d[0] * d[0];
    r2 = r2 + d[1] * d[1];
    r2 = r2 + d[2] * d[2];
    return r2;
}

// ------------------------------------------------------------ design rows

struct FitShape {
    int ns, nk2, nk3, nd, n2cols;  // n2cols: 2-body columns (all species pairs)
    double rc2, rc3;
};

// Column k decoded: kind 2 (species pair za <= zb, spline n) or 3 (centre
// species z, legs p <= q, third side s); kind 0 = no column.
struct FitCol {
    int kind, a, b, p, q, s;
};

__device__ FitCol fit_decode(const FitShape &sh, int k)
{
    FitCol c{0, 0, 0, 0, 0, 0};
    if (k >= sh.nd)
        return c;
    const int nf2 = sh.nk2 - 1;  // nb2 - 3
    if (k < sh.n2cols) {
        int pair = k / nf2;
        c.kind = 2;
        c.p = k - pair * nf2;
        for (int za = 0; za < sh.ns; ++za) {
            const int row = sh.ns - za;
            if (pair < row) {
                c.a = za;
                c.b = za + pair;
                break;
            }
            pair -= row;
        }
        return c;
    }
    const int nb3 = sh.nk3 + 2, nf3 = sh.nk3 - 1;
    const int per_z = nf3 * (nf3 + 1) / 2 * nb3;
    int r = k - sh.n2cols;
    c.kind = 3;
    c.a = r / per_z;
    r -= c.a * per_z;
    int pq = r / nb3;
    c.s = r - pq * nb3;
    for (int p = 0; p < nf3; ++p) {
        const int row = nf3 - p;
        if (pq < row) {
            c.p = p;
            c.q = p + pq;
            break;
        }
        pq -= row;
    }
    return c;
}

// One record: a pair (kind 2) or a triplet (kind 3) as seen by atom i.
struct FitRec {
    int z;       // species of the centre (triplet) or of j (pair); -1 = empty
    int centre;  // triplet centred on i (its energy is part of E_i)
    int fa, fb, fs;
    double A[4], dA[4], Bv[4], dBv[4], C[4], dC[4];
    double v1[3], v2[3];
};

// Entry of the list of i's neighbours inside the 3-body cutoff.
struct FitLeg {
    int j, z, f;
    double u[3], r, B[4], dB[4], d[3];
};

__global__ void __launch_bounds__(kFitWave)
    k_fit_design(int n, int cap, const int *__restrict__ nbr, const int *__restrict__ cnt,
                 const double *__restrict__ pos, const int32_t *__restrict__ species, Box box,
                 FitShape sh, double *__restrict__ rows, int ld, double *__restrict__ erow,
                 int *__restrict__ hdr)
{
    __shared__ FitRec rec[kFitWave];
    __shared__ FitLeg leg[kMaxTriplet];
    __shared__ int legpre[kMaxTriplet + 1];
    __shared__ int nleg;
    const int i = blockIdx.x;
    const int lane = threadIdx.x;
    if (i >= n)
        return;
    const int zi = sp_clamp(species[i], sh.ns);
    FitCol col[kFitColsPerLane];
    double e[kFitColsPerLane], f[kFitColsPerLane][3];
    for (int m = 0; m < kFitColsPerLane; ++m) {
        col[m] = fit_decode(sh, lane + kFitWave * m);
        e[m] = 0.0;
        f[m][0] = f[m][1] = f[m][2] = 0.0;
    }
    const double rc2sq = sh.rc2 * sh.rc2, rc3sq = sh.rc3 * sh.rc3;
    const bool three = sh.nk3 > 0;
    const int ci = cnt[i] < cap ? cnt[i] : cap;
    if (lane == 0)
        nleg = 0;
    __syncthreads();

    // consume one batch: every lane adds the records to its own columns
    auto consume = [&](int nrec) {
        for (int t = 0; t < nrec; ++t) {
            const FitRec &R = rec[t];
            if (R.z < 0)
                continue;
            for (int m = 0; m < kFitColsPerLane; ++m) {
                const FitCol &c = col[m];
                if (c.kind == 2 && R.fs < 0) {
                    // pair: columns of the sorted species pair
                    const int lo = R.z < zi ? R.z : zi, hi = R.z < zi ? zi : R.z;
                    if (c.a != lo || c.b != hi)
                        continue;
                    const double bv = fit_win(R.A, R.fa, c.p), dv = fit_win(R.dA, R.fa, c.p);
                    e[m] += 0.5 * bv;
                    for (int k = 0; k < 3; ++k)
                        f[m][k] += dv * R.v1[k];
                } else if (c.kind == 3 && R.fs >= 0 && c.a == R.z) {
                    const double ap = fit_win(R.A, R.fa, c.p), aq = fit_win(R.A, R.fa, c.q);
                    const double bp = fit_win(R.Bv, R.fb, c.p), bq = fit_win(R.Bv, R.fb, c.q);
                    const double dap = fit_win(R.dA, R.fa, c.p), daq = fit_win(R.dA, R.fa, c.q);
                    const double dbp = fit_win(R.dBv, R.fb, c.p), dbq = fit_win(R.dBv, R.fb, c.q);
                    const double cs = fit_win(R.C, R.fs, c.s), dcs = fit_win(R.dC, R.fs, c.s);
                    const bool sym = c.p != c.q;
                    const double P = ap * bq + (sym ? aq * bp : 0.0);
                    const double Pa = dap * bq + (sym ? daq * bp : 0.0);
                    const double Pb = ap * dbq + (sym ? aq * dbp : 0.0);
                    const double X = Pa * cs;
                    const double Y = R.centre ? Pb * cs : P * dcs;
                    if (R.centre)
                        e[m] += P * cs;
                    for (int k = 0; k < 3; ++k)
                        f[m][k] += X * R.v1[k] + Y * R.v2[k];
                }
            }
        }
    };

    // 1. pairs of i, and the list of neighbours inside the 3-body cutoff
    for (int base = 0; base < ci; base += kFitWave) {
        const int slot = base + lane;
        FitRec &R = rec[lane];
        R.z = -1;
        R.fs = -1;
        bool in3 = false;
        double d[3] = {0.0, 0.0, 0.0}, r2 = 0.0;
        int j = -1;
        if (slot < ci) {
            j = nbr[(size_t)i * cap + slot];
            if (j >= 0 && j < n) {
                r2 = fit_disp(pos, n, i, j, box, d);
                const double r = sqrt(r2);
                if (r2 < rc2sq) {
                    R.z = sp_clamp(species[j], sh.ns);
                    fit_bspline(r, sh.nk2, sh.rc2, R.fa, R.A, R.dA);
                    for (int k = 0; k < 3; ++k)
                        R.v1[k] = d[k] / r;
                }
                in3 = three && r2 < rc3sq;
            }
        }
        // append the 3-body legs in row order
        const unsigned long long m3 = __ballot(in3);
        const int before = __popcll(m3 & ((1ull << lane) - 1ull));
        const int pos3 = nleg + before;
        if (in3) {
            if (pos3 < kMaxTriplet) {
                FitLeg &G = leg[pos3];
                const double r = sqrt(r2);
                G.j = j;
                G.z = sp_clamp(species[j], sh.ns);
                G.r = r;
                for (int k = 0; k < 3; ++k) {
                    G.d[k] = d[k];
                    G.u[k] = d[k] / r;
                }
                fit_bspline(r, sh.nk3, sh.rc3, G.f, G.B, G.dB);
            } else {
                atomicOr(&hdr[H_STATUS], MLMIX_STATUS_TRIPLET_OVERFLOW);
            }
        }
        __syncthreads();
        consume(ci - base < kFitWave ? ci - base : kFitWave);
        if (lane == 0) {
            const int tot = nleg + __popcll(m3);
            nleg = tot < kMaxTriplet ? tot : kMaxTriplet;
        }
        __syncthreads();
    }
    const int m = nleg;

    if (three && m > 0) {
        // 2. triplets centred on i: unordered leg pairs (a < b)
        const int npairs = m * (m - 1) / 2;
        for (int base = 0; base < npairs; base += kFitWave) {
            const int t = base + lane;
            FitRec &R = rec[lane];
            R.z = -1;
            if (t < npairs) {
                int a = 0, rem = t;
                while (rem >= m - 1 - a) {
                    rem -= m - 1 - a;
                    ++a;
                }
                const int b = a + 1 + rem;
                const FitLeg &Ga = leg[a], &Gb = leg[b];
                double dd[3];
                for (int k = 0; k < 3; ++k)
                    dd[k] = Gb.d[k] - Ga.d[k];
                const double rjk = sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
                R.z = zi;
                R.centre = 1;
                R.fa = Ga.f;
                R.fb = Gb.f;
                for (int q = 0; q < 4; ++q) {
                    R.A[q] = Ga.B[q];
                    R.dA[q] = Ga.dB[q];
                    R.Bv[q] = Gb.B[q];
                    R.dBv[q] = Gb.dB[q];
                }
                fit_bspline(rjk, sh.nk3, 2.0 * sh.rc3, R.fs, R.C, R.dC);
                for (int k = 0; k < 3; ++k) {
                    R.v1[k] = Ga.u[k];
                    R.v2[k] = Gb.u[k];
                }
            }
            __syncthreads();
            consume(npairs - base < kFitWave ? npairs - base : kFitWave);
            __syncthreads();
        }

        // 3. triplets centred on a 3-body neighbour j with i as one leg
        if (lane == 0) {
            int acc = 0;
            for (int a = 0; a < m; ++a) {
                legpre[a] = acc;
                const int cj = cnt[leg[a].j];
                acc += cj < cap ? cj : cap;
            }
            legpre[m] = acc;
        }
        __syncthreads();
        const int total = legpre[m];
        for (int base = 0; base < total; base += kFitWave) {
            const int t = base + lane;
            FitRec &R = rec[lane];
            R.z = -1;
            if (t < total) {
                int a = 0;
                while (legpre[a + 1] <= t)
                    ++a;
                const FitLeg &Ga = leg[a];
                const int j = Ga.j;
                const int k = nbr[(size_t)j * cap + (t - legpre[a])];
                if (k >= 0 && k < n && k != i) {
                    double djk[3];
                    const double r2jk = fit_disp(pos, n, j, k, box, djk);
                    if (r2jk < rc3sq) {
                        const double rjk = sqrt(r2jk);
                        double d3[3];
                        for (int q = 0; q < 3; ++q)
                            d3[q] = Ga.d[q] + djk[q];
                        const double r3 = sqrt(d3[0] * d3[0] + d3[1] * d3[1] + d3[2] * d3[2]);
                        R.z = Ga.z;
                        R.centre = 0;
                        R.fa = Ga.f;
                        for (int q = 0; q < 4; ++q) {
                            R.A[q] = Ga.B[q];
                            R.dA[q] = Ga.dB[q];
                        }
                        fit_bspline(rjk, sh.nk3, sh.rc3, R.fb, R.Bv, R.dBv);
                        fit_bspline(r3, sh.nk3, 2.0 * sh.rc3, R.fs, R.C, R.dC);
                        for (int q = 0; q < 3; ++q) {
                            R.v1[q] = Ga.u[q];
                            R.v2[q] = d3[q] / r3;
                        }
                    }
                }
            }
            __syncthreads();
            consume(total - base < kFitWave ? total - base : kFitWave);
            __syncthreads();
        }
    }

    for (int mm = 0; mm < kFitColsPerLane; ++mm) {
        const int k = lane + kFitWave * mm;
        if (k >= sh.nd)
            break;
        erow[(size_t)k * n + i] = e[mm];
        for (int q = 0; q < 3; ++q)
            rows[(size_t)(1 + (size_t)q * n + i) * ld + k] = f[mm][q];
    }
}

// rows[0][k] = sum_i erow[k][i], one workgroup per column, fixed order
__global__ void __launch_bounds__(256) k_fit_erow_sum(int n, const double *__restrict__ erow,
                                                      double *__restrict__ rows)
{
    __shared__ double sh[256];
    const int k = blockIdx.x;
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256)
        s += erow[(size_t)k * n + i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        rows[k] = sh[0];
}

void launch_fit_design(hipStream_t s, const Ctx &c, void *ws, const WsLayout &L, const Box &b,
                       const double *pos, const int32_t *species, double *rows, int ld,
                       double *erow, int nd)
{
    if (L.n == 0)
        return;
    FitShape sh;
    sh.ns = c.m.ns;
    sh.nk2 = c.d.uf3_n_knots2;
    sh.nk3 = c.d.uf3_n_knots3;
    sh.nd = nd;
    sh.n2cols = sh.ns * (sh.ns + 1) / 2 * (sh.nk2 - 1);
    sh.rc2 = c.d.uf3_rcut2;
    sh.rc3 = c.d.uf3_rcut3;
    k_fit_design<<<L.n, kFitWave, 0, s>>>(L.n, L.cap, at<int>(ws, L.nbr), at<int>(ws, L.cnt), pos,
                                          species, b, sh, rows, ld, erow, at<int>(ws, L.hdr));
    k_fit_erow_sum<<<nd, 256, 0, s>>>(L.n, erow, rows);
}

// ------------------------------------------------------------------ Gram

constexpr int kGramRows = 32;  // rows staged per LDS pass

__host__ __device__ inline int fit_nblk(int nd) { return (nd + 3) / 4; }

// Upper-triangle 4x4 block index t -> (bi, bj), bi <= bj, row by row.
__device__ __forceinline__ void fit_blk(int t, int nb, int &bi, int &bj)
{
    bi = 0;
    while (t >= nb - bi) {
        t -= nb - bi;
        ++bi;
    }
    bj = bi + t;
}

__global__ void __launch_bounds__(256)
    k_fit_gram_partial(long long nrows, int nd, int ld, const double *__restrict__ A,
                       const double *__restrict__ y, const double *__restrict__ w,
                       long long chunk, double *__restrict__ part)
{
    const int nb = fit_nblk(nd), nd4 = nb * 4;
    const int nblk = nb * (nb + 1) / 2;
    __shared__ double tile[kGramRows][kFitMaxParams + 4];
    __shared__ double wy[kGramRows][2];
    const long long r0 = (long long)blockIdx.x * chunk;
    long long r1 = r0 + chunk;
    if (r1 > nrows)
        r1 = nrows;
    constexpr int kPer = (kFitMaxParams / 4) * (kFitMaxParams / 4 + 1) / 2 / 256 + 1;
    double acc[kPer][16];
    int bis[kPer], bjs[kPer];
    for (int u = 0; u < kPer; ++u) {
        const int t = threadIdx.x + 256 * u;
        bis[u] = -1;
        if (t < nblk)
            fit_blk(t, nb, bis[u], bjs[u]);
        for (int e = 0; e < 16; ++e)
            acc[u][e] = 0.0;
    }
    double bacc[4] = {0.0, 0.0, 0.0, 0.0};
    for (long long rb = r0; rb < r1; rb += kGramRows) {
        const int nr = (int)(r1 - rb < kGramRows ? r1 - rb : kGramRows);
        for (int e = threadIdx.x; e < kGramRows * nd4; e += 256) {
            const int r = e / nd4, k = e - r * nd4;
            tile[r][k] = (r < nr && k < nd) ? A[(size_t)(rb + r) * ld + k] : 0.0;
        }
        if ((int)threadIdx.x < kGramRows) {
            const int r = threadIdx.x;
            wy[r][0] = r < nr ? (w ? w[rb + r] : 1.0) : 0.0;
            wy[r][1] = r < nr ? (y ? y[rb + r] : 0.0) : 0.0;
        }
        __syncthreads();
        for (int r = 0; r < nr; ++r) {
            const double wr = wy[r][0];
            for (int u = 0; u < kPer; ++u) {
                if (bis[u] < 0)
                    continue;
                double ai[4], aj[4];
                for (int q = 0; q < 4; ++q) {
                    ai[q] = wr * tile[r][4 * bis[u] + q];
                    aj[q] = tile[r][4 * bjs[u] + q];
                }
                for (int p = 0; p < 4; ++p)
                    for (int q = 0; q < 4; ++q)
                        acc[u][4 * p + q] += ai[p] * aj[q];
            }
            if ((int)threadIdx.x < nb) {
                const double wyr = wr * wy[r][1];
                for (int q = 0; q < 4; ++q)
                    bacc[q] += wyr * tile[r][4 * threadIdx.x + q];
            }
        }
        __syncthreads();
    }
    double *out = part + (size_t)blockIdx.x * ((size_t)nblk * 16 + nd4);
    for (int u = 0; u < kPer; ++u) {
        const int t = threadIdx.x + 256 * u;
        if (t < nblk)
            for (int e = 0; e < 16; ++e)
                out[(size_t)t * 16 + e] = acc[u][e];
    }
    if ((int)threadIdx.x < nb)
        for (int q = 0; q < 4; ++q)
            out[(size_t)nblk * 16 + 4 * threadIdx.x + q] = bacc[q];
}

// G[k][l] += sum over chunks (both triangles written), b[k] += likewise
__global__ void __launch_bounds__(256) k_fit_gram_reduce(int nd, int nparts,
                                                         const double *__restrict__ part,
                                                         double *__restrict__ G,
                                                         double *__restrict__ bvec)
{
    const int nb = fit_nblk(nd), nd4 = nb * 4;
    const int nblk = nb * (nb + 1) / 2;
    const size_t stride = (size_t)nblk * 16 + nd4;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= nblk * 16 + nd4)
        return;
    double s = 0.0;
    for (int p = 0; p < nparts; ++p)
        s += part[(size_t)p * stride + e];
    if (e < nblk * 16) {
        int bi, bj;
        fit_blk(e / 16, nb, bi, bj);
        const int k = 4 * bi + (e % 16) / 4, l = 4 * bj + (e % 4);
        if (k < nd && l < nd) {
            if (bi != bj || k <= l) {
                G[(size_t)k * nd + l] += s;
                if (k != l)
                    G[(size_t)l * nd + k] += s;
            }
        }
    } else {
        const int k = e - nblk * 16;
        if (k < nd)
            bvec[k] += s;
    }
}

size_t fit_gram_parts(long long nrows, long long &chunk)
{
    long long parts = (nrows + 255) / 256;
    parts = parts < 1 ? 1 : (parts > 512 ? 512 : parts);
    chunk = (nrows + parts - 1) / parts;
    chunk = (chunk + kGramRows - 1) / kGramRows * kGramRows;
    if (chunk < kGramRows)
        chunk = kGramRows;
    parts = (nrows + chunk - 1) / chunk;
    return (size_t)(parts < 1 ? 1 : parts);
}

size_t fit_gram_part_bytes(int nd, size_t parts)
{
    const int nb = fit_nblk(nd);
    return parts * ((size_t)nb * (nb + 1) / 2 * 16 + (size_t)nb * 4) * sizeof(double);
}

void launch_fit_gram(hipStream_t s, long long nrows, int nd, int ld, const double *A,
                     const double *y, const double *w, double *G, double *b, double *part)
{
    if (nrows <= 0)
        return;
    long long chunk = 0;
    const size_t parts = fit_gram_parts(nrows, chunk);
    k_fit_gram_partial<<<(unsigned)parts, 256, 0, s>>>(nrows, nd, ld, A, y, w, chunk, part);
    const int nb = fit_nblk(nd);
    const int ne = nb * (nb + 1) / 2 * 16 + nb * 4;
    k_fit_gram_reduce<<<(ne + 255) / 256, 256, 0, s>>>(nd, (int)parts, part, G, b);
}

// ---------------------------------------------------------------- search

struct FitSearchArgs {
    int nd, nh, ldh;
    const double *GS, *bS, *AH, *yH;
    double alpha, tol, lam0, ridge;
    int max_decades, max_bisect;
    double *GH, *bH;  // scratch nd*nd + nd
    double *c, *info;
};

// Block sum over 256 threads in a fixed order.
__device__ double fit_block_sum(double v, double *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double s = red[0];
    __syncthreads();
    return s;
}

__global__ void __launch_bounds__(256) k_fit_search(FitSearchArgs a)
{
    constexpr int kPacked = kFitMaxParams * (kFitMaxParams + 1) / 2;
    __shared__ double Lp[kPacked];
    __shared__ double z[kFitMaxParams], cur[kFitMaxParams], keep[kFitMaxParams];
    __shared__ double red[256];
    __shared__ int fail;
    const int nd = a.nd, tid = threadIdx.x;
    auto P = [](int r, int c2) { return r * (r + 1) / 2 + c2; };  // r >= c2

    // G_H = A_H^T A_H and b_H = A_H^T y_H
    for (int e = tid; e < nd * nd + nd; e += 256) {
        double s = 0.0;
        if (e < nd * nd) {
            const int k = e / nd, l = e - k * nd;
            for (int h = 0; h < a.nh; ++h)
                s += a.AH[(size_t)h * a.ldh + k] * a.AH[(size_t)h * a.ldh + l];
            a.GH[e] = s;
        } else {
            const int k = e - nd * nd;
            for (int h = 0; h < a.nh; ++h)
                s += a.AH[(size_t)h * a.ldh + k] * a.yH[h];
            a.bH[k] = s;
        }
    }
    __threadfence();
    __syncthreads();

    // one solve at lam: cur = c(lam); returns the hard residual (or -1 when
    // the factorisation meets a non-positive pivot)
    auto solve = [&](double lam) -> double {
        for (int e = tid; e < nd * (nd + 1) / 2; e += 256) {
            int r = (int)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
            while (r * (r + 1) / 2 > e)
                --r;
            while ((r + 1) * (r + 2) / 2 <= e)
                ++r;
            const int c2 = e - r * (r + 1) / 2;
            double v = a.GS[(size_t)r * nd + c2] + lam * a.GH[(size_t)r * nd + c2];
            if (r == c2)
                v += a.ridge;
            Lp[e] = v;
        }
        if (tid < nd)
            z[tid] = a.bS[tid] + lam * a.bH[tid];
        if (tid == 0)
            fail = 0;
        __syncthreads();
        // left-looking Cholesky, column by column
        for (int j = 0; j < nd; ++j) {
            double t = 0.0;
            const int i = j + tid;  // rows j .. nd-1; nd <= 256 threads
            if (i < nd) {
                t = Lp[P(i, j)];
                for (int k = 0; k < j; ++k)
                    t -= Lp[P(i, k)] * Lp[P(j, k)];
            }
            __syncthreads();
            if (i == j) {
                if (!(t > 0.0))
                    fail = 1;
                Lp[P(j, j)] = t > 0.0 ? sqrt(t) : 1.0;
            }
            __syncthreads();
            if (i > j && i < nd)
                Lp[P(i, j)] = t / Lp[P(j, j)];
            __syncthreads();
        }
        // L x = z, then L^T c = x (in place in z)
        for (int j = 0; j < nd; ++j) {
            if (tid == 0)
                z[j] = z[j] / Lp[P(j, j)];
            __syncthreads();
            const int i = j + 1 + tid;
            if (i < nd)
                z[i] -= Lp[P(i, j)] * z[j];
            __syncthreads();
        }
        for (int j = nd - 1; j >= 0; --j) {
            if (tid == 0)
                z[j] = z[j] / Lp[P(j, j)];
            __syncthreads();
            if (tid < j)
                z[tid] -= Lp[P(j, tid)] * z[j];
            __syncthreads();
        }
        if (tid < nd)
            cur[tid] = z[tid];
        __syncthreads();
        double part = 0.0;
        for (int h = tid; h < a.nh; h += 256) {
            double r = -a.yH[h];
            for (int k = 0; k < nd; ++k)
                r += a.AH[(size_t)h * a.ldh + k] * cur[k];
            part += r * r;
        }
        const double res = fit_block_sum(part, red);
        return fail ? -1.0 : res;
    };
    auto save = [&]() {
        if (tid < nd)
            keep[tid] = cur[tid];
        __syncthreads();
    };

    int nsolve = 0, status = 0, dec = 0;
    double lam = a.lam0;
    double res = solve(lam);
    ++nsolve;
    double best_res = res, best_lam = lam, lam_lo = lam, out_lam = lam, out_res = res;
    save();
    if (res < 0.0) {
        status = 3;
    } else if (res > a.alpha) {
        while (res > a.alpha && dec < a.max_decades && res >= 0.0) {
            lam_lo = lam;
            lam *= 10.0;
            ++dec;
            res = solve(lam);
            ++nsolve;
            if (res >= 0.0 && res < best_res) {
                best_res = res;
                best_lam = lam;
                save();
            }
        }
        if (res < 0.0) {
            status = 3;
            out_lam = best_lam;
            out_res = best_res;
        } else if (res > a.alpha) {
            status = 1;
            out_lam = best_lam;
            out_res = best_res;
        } else {
            // bisection: lo fails, hi passes (keep holds c(hi))
            double lo = lam_lo, hi = lam, r_hi = res;
            save();
            int it = 0;
            while (!(a.alpha - r_hi < a.tol)) {
                if (it == a.max_bisect) {
                    status = 2;
                    break;
                }
                const double mid = 0.5 * (lo + hi);
                const double rm = solve(mid);
                ++nsolve;
                if (rm < 0.0) {
                    status = 3;
                    break;
                }
                if (rm <= a.alpha) {
                    hi = mid;
                    r_hi = rm;
                    save();
                } else {
                    lo = mid;
                }
                ++it;
            }
            out_lam = hi;
            out_res = r_hi;
            lam_lo = lo;
        }
    }
    if (tid < nd)
        a.c[tid] = keep[tid];
    if (tid == 0) {
        a.info[0] = out_lam;
        a.info[1] = out_res;
        a.info[2] = (double)nsolve;
        a.info[3] = (double)status;
        a.info[4] = lam_lo;
        a.info[5] = (double)dec;
    }
}

void launch_fit_search(hipStream_t s, int nd, int nh, int ldh, const double *GS, const double *bS,
                       const double *AH, const double *yH, double alpha, double tol, double lam0,
                       double ridge, int max_decades, int max_bisect, double *c, double *info,
                       double *scratch)
{
    FitSearchArgs a{nd, nh, ldh, GS, bS, AH, yH, alpha, tol, lam0, ridge, max_decades, max_bisect,
                    scratch, scratch + (size_t)nd * nd, c, info};
    k_fit_search<<<1, 256, 0, s>>>(a);
}

}  // namespace mlmix
