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
//    triplets centred on a neighbour j in which i is a leg (the other leg
//    from j's 3-body list, built beforehand by k_fit_list3).
//  - k_fit_gram_partial / k_fit_gram_reduce: G = A^T diag(w) A and
//    b = A^T diag(w) y. Each workgroup stages 32 rows at a time in LDS and
//    every thread accumulates 4 x 4 blocks of the upper triangle; partials of
//    fixed row chunks are summed in chunk order.
//  - k_fit_search: one workgroup runs the whole lambda search (G_H and b_H
//    come from the Gram kernels just before): the normal
//    equations (G_S + lam G_H + ridge I) c = b_S + lam b_H solved by a
//    Cholesky factorisation held packed in LDS, the hard residual
//    sum_h w_h (A_H c - y_H)_h^2 from the hard rows, decades of lam until the residual
//    is at most alpha, then interval bisection until it is within tol of
//    alpha. Every loop has a fixed bound.
// Everything is FP64 whatever the context's force precision.
#include "internal.h"

namespace mlmix {

constexpr int kFitWave = 64;
constexpr int kFitColsPerLane = 2;  // columns per lane: kFitMaxParams <= 128

// ---------------------------------------------------------------- B-splines

// The four non-zero clamped uniform cubic B-splines at x (0 <= x < top) and
// their derivatives, by the Cox-de Boor triangle on the span holding x. The
// recursion runs in knot units u = x / h (B-splines do not change when x and
// the knots are scaled together), where every knot difference is a small
// integer, so no division is left; ih = 1/h = (npts - 1)/top. The functions
// are B_first .. B_first+3.
__device__ __forceinline__ int fit_k(int i, int npts)
{
    const int k = i - 3;
    return k < 0 ? 0 : (k > npts - 1 ? npts - 1 : k);
}

__device__ __forceinline__ double fit_inv_small(int m)
{
    // 1/m for the knot-difference counts 1..3 that occur (0 never divides)
    return m == 1 ? 1.0 : (m == 2 ? 0.5 : 1.0 / 3.0);
}

__device__ void fit_bspline(double x, int npts, double ih, int &first, double N[4], double dN[4])
{
    const double u = x * ih;
    int sp = (int)floor(u);
    sp = sp < 0 ? 0 : (sp > npts - 2 ? npts - 2 : sp);
    const int mu = sp + 3;
    double B[4] = {1.0, 0.0, 0.0, 0.0}, B2[3] = {0.0, 0.0, 0.0};
    double left[4], right[4];
#pragma unroll
    for (int j = 1; j <= 3; ++j) {
        left[j] = u - (double)fit_k(mu + 1 - j, npts);
        right[j] = (double)fit_k(mu + j, npts) - u;
        double saved = 0.0;
#pragma unroll
        for (int r = 0; r < j; ++r) {
            const int m = fit_k(mu + r + 1, npts) - fit_k(mu + 1 - j + r, npts);
            const double tmp = B[r] * fit_inv_small(m);
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
    // dB_k/du = 3 (B2_k / (K_k+3 - K_k) - B2_k+1 / (K_k+4 - K_k+1)), with the
    // degree-2 functions B2_{mu-2..mu} non-zero; d/dx = ih d/du
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int k = mu - 3 + r;
        const double a = r >= 1 ? B2[r - 1] * fit_inv_small(fit_k(k + 3, npts) - fit_k(k, npts)) : 0.0;
        const double b = r <= 2 ? B2[r] * fit_inv_small(fit_k(k + 4, npts) - fit_k(k + 1, npts)) : 0.0;
        N[r] = B[r];
        dN[r] = 3.0 * ih * (a - b);
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
    double ih2, ih3, ih3c;         // knots per A: 2-body, 3-body legs, third side
};

// Column k decoded: kind 2 (species pair a <= b, spline p) or 3 (centre
// species a, leg pair index p of (p1 <= p2), third side s); kind 0 = none.
struct FitCol {
    int kind, a, b, p, s;
};

__device__ FitCol fit_decode(const FitShape &sh, int k)
{
    FitCol c{0, 0, 0, 0, 0};
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
    c.p = r / nb3;
    c.s = r - c.p * nb3;
    return c;
}

// Entry of the list of i's neighbours inside the 3-body cutoff.
struct FitLeg {
    int j, z, f;
    double d[3], ir, B[4], dB[4];  // d = x_j - x_i, ir = 1/|d|
};

// One configuration of a batched design launch (everything per workspace).
struct FitCfgDev {
    int n, cap;
    const int *nbr, *cnt;
    const double *pos;
    const int32_t *species;
    double *rows, *erow;
    int *l3, *l3cnt, *hdr;
    Box box;
};
// Configurations of one launch, passed by value as kernel arguments; the
// workgroup of global atom b belongs to the configuration whose atom range
// [atom0[c], atom0[c+1]) holds b.
struct FitBatch {
    int ncfg, ld;
    int atom0[kFitBatch + 1];
    FitCfgDev c[kFitBatch];
};

static_assert(sizeof(FitBatch) + 64 <= 4096, "design launch arguments exceed 4 KB");

__device__ __forceinline__ int fit_cfg_of(const FitBatch &B, int b)
{
    int c = 0;
    while (c + 1 < B.ncfg && B.atom0[c + 1] <= b)
        ++c;
    return c;
}

constexpr int kFitRec = 16;   // records per batch
constexpr int kFitLegs = 32;  // 3-body neighbours per atom in the design kernel

// Dense records in dynamic LDS, record index fastest:
//   pairs:    B[nf2][R], dB[nf2][R] (the 2-body basis and its derivative)
//   triplets: P, Pa, Pb [npq][R] (leg products symmetrised over p1 <= p2 and
//             their derivatives by leg a and leg b), C, dC [nb3][R] (third side)
//   then v1, v2 [3][R] (force directions), z [R], centre [R] (ints).
__host__ __device__ inline int fit_dense(int nk2, int nk3)
{
    const int nf2 = nk2 - 1;
    const int nf3 = nk3 > 0 ? nk3 - 1 : 0;
    const int npq = nf3 * (nf3 + 1) / 2;
    const int t3 = nk3 > 0 ? 3 * npq + 2 * (nk3 + 2) : 0;
    return 2 * nf2 > t3 ? 2 * nf2 : t3;
}

size_t fit_design_lds(int nk2, int nk3)
{
    return (size_t)(fit_dense(nk2, nk3) + 6) * kFitRec * sizeof(double) + 2 * kFitRec * sizeof(int);
}

__global__ void __launch_bounds__(kFitWave) k_fit_design(FitBatch Bt, FitShape sh)
{
    extern __shared__ double smem[];
    __shared__ FitLeg leg[kFitLegs];
    __shared__ int legpre[kFitLegs + 1];
    __shared__ int nleg;
    const int cfg = fit_cfg_of(Bt, blockIdx.x);
    const FitCfgDev &Cf = Bt.c[cfg];
    const int n = Cf.n, cap = Cf.cap, ld = Bt.ld;
    const int *__restrict__ nbr = Cf.nbr;
    const int *__restrict__ cnt = Cf.cnt;
    const double *__restrict__ pos = Cf.pos;
    const int32_t *__restrict__ species = Cf.species;
    double *__restrict__ rows = Cf.rows;
    double *__restrict__ erow = Cf.erow;
    const int *__restrict__ l3 = Cf.l3;
    const int *__restrict__ l3cnt = Cf.l3cnt;
    int *__restrict__ hdr = Cf.hdr;
    const Box box = Cf.box;
    const int i = blockIdx.x - Bt.atom0[cfg];
    const int lane = threadIdx.x;
    if (i >= n)
        return;
    constexpr int R = kFitRec;
    const int nf2 = sh.nk2 - 1;
    const bool three = sh.nk3 > 1;
    const int nb3 = sh.nk3 + 2, nf3 = three ? sh.nk3 - 1 : 0;
    const int npq = nf3 * (nf3 + 1) / 2;
    const int dense = fit_dense(sh.nk2, sh.nk3);
    double *D = smem;
    double *V = smem + (size_t)dense * R;
    int *RZ = reinterpret_cast<int *>(V + 6 * R);
    int *RC = RZ + R;
    double *P = D, *Pa = D + npq * R, *Pb = D + 2 * npq * R;
    double *C = D + 3 * npq * R, *dC = C + nb3 * R;

    const int zi = sp_clamp(species[i], sh.ns);
    FitCol col[kFitColsPerLane];
    double e[kFitColsPerLane], f[kFitColsPerLane][3];
    for (int m = 0; m < kFitColsPerLane; ++m) {
        col[m] = fit_decode(sh, lane + kFitWave * m);
        e[m] = 0.0;
        f[m][0] = f[m][1] = f[m][2] = 0.0;
    }
    const double rc2sq = sh.rc2 * sh.rc2, rc3sq = sh.rc3 * sh.rc3;
    const int ci = cnt[i] < cap ? cnt[i] : cap;
    if (lane == 0)
        nleg = 0;
    __syncthreads();

    // 1. pairs of i (2-body columns), and the list of its 3-body legs
    for (int base = 0; base < ci; base += R) {
        const int slot = base + lane;
        bool in3 = false;
        double d[3] = {0.0, 0.0, 0.0}, r2 = 0.0;
        int j = -1;
        if (lane < R) {
            RZ[lane] = -1;
            if (slot < ci) {
                j = nbr[(size_t)i * cap + slot];
                if (j >= 0 && j < n) {
                    r2 = fit_disp(pos, n, i, j, box, d);
                    const double r = sqrt(r2);
                    if (r2 < rc2sq) {
                        int fb;
                        double Bw[4], dBw[4];
                        fit_bspline(r, sh.nk2, sh.ih2, fb, Bw, dBw);
                        RZ[lane] = sp_clamp(species[j], sh.ns);
                        for (int q = 0; q < nf2; ++q) {
                            const unsigned o = (unsigned)(q - fb);
                            D[q * R + lane] = o < 4u ? Bw[o] : 0.0;
                            D[(nf2 + q) * R + lane] = o < 4u ? dBw[o] : 0.0;
                        }
                        for (int k = 0; k < 3; ++k)
                            V[k * R + lane] = d[k] / r;
                    }
                    in3 = three && r2 < rc3sq;
                }
            }
        }
        const unsigned long long m3 = __ballot(in3);
        const int pos3 = nleg + __popcll(m3 & ((1ull << lane) - 1ull));
        if (in3) {
            if (pos3 < kFitLegs) {
                FitLeg &G = leg[pos3];
                const double r = sqrt(r2);
                G.j = j;
                G.z = sp_clamp(species[j], sh.ns);
                G.ir = 1.0 / r;
                for (int k = 0; k < 3; ++k)
                    G.d[k] = d[k];
                fit_bspline(r, sh.nk3, sh.ih3, G.f, G.B, G.dB);
            } else {
                atomicOr(&hdr[H_STATUS], MLMIX_STATUS_TRIPLET_OVERFLOW);
            }
        }
        __syncthreads();
        const int nrec = ci - base < R ? ci - base : R;
        for (int t = 0; t < nrec; ++t) {
            const int zj = RZ[t];
            if (zj < 0)
                continue;
            const int lo = zj < zi ? zj : zi, hi = zj < zi ? zi : zj;
            for (int m = 0; m < kFitColsPerLane; ++m) {
                const FitCol &c = col[m];
                if (c.kind != 2 || c.a != lo || c.b != hi)
                    continue;
                const double bv = D[c.p * R + t], dv = D[(nf2 + c.p) * R + t];
                e[m] += 0.5 * bv;
                for (int k = 0; k < 3; ++k)
                    f[m][k] += dv * V[k * R + t];
            }
        }
        if (lane == 0) {
            const int tot = nleg + __popcll(m3);
            nleg = tot < kFitLegs ? tot : kFitLegs;
        }
        __syncthreads();
    }
    const int m = nleg;

    // dense leg products of one triplet record (lane t < R): legs a and b
    // (windows fa/A/dA and fb/Bv/dBv), third side (fs/Cw/dCw)
    auto put = [&](int t, int fa, const double *A, const double *dA, int fb, const double *Bv,
                   const double *dBv, int fs, const double *Cw, const double *dCw, bool centre) {
        int idx = 0;
        for (int p1 = 0; p1 < nf3; ++p1) {
            const unsigned o1a = (unsigned)(p1 - fa), o1b = (unsigned)(p1 - fb);
            const double a1 = o1a < 4u ? A[o1a] : 0.0, da1 = o1a < 4u ? dA[o1a] : 0.0;
            const double b1 = o1b < 4u ? Bv[o1b] : 0.0, db1 = o1b < 4u ? dBv[o1b] : 0.0;
            for (int p2 = p1; p2 < nf3; ++p2, ++idx) {
                const unsigned o2a = (unsigned)(p2 - fa), o2b = (unsigned)(p2 - fb);
                const double a2 = o2a < 4u ? A[o2a] : 0.0, da2 = o2a < 4u ? dA[o2a] : 0.0;
                const double b2 = o2b < 4u ? Bv[o2b] : 0.0, db2 = o2b < 4u ? dBv[o2b] : 0.0;
                const bool sym = p1 != p2;
                P[idx * R + t] = a1 * b2 + (sym ? a2 * b1 : 0.0);
                Pa[idx * R + t] = da1 * b2 + (sym ? da2 * b1 : 0.0);
                if (centre)
                    Pb[idx * R + t] = a1 * db2 + (sym ? a2 * db1 : 0.0);
            }
        }
        for (int q = 0; q < nb3; ++q) {
            const unsigned o = (unsigned)(q - fs);
            C[q * R + t] = o < 4u ? Cw[o] : 0.0;
            dC[q * R + t] = o < 4u ? dCw[o] : 0.0;
        }
    };
    // every lane adds a batch of triplet records to its own columns
    auto consume3 = [&](int nrec) {
        for (int t = 0; t < nrec; ++t) {
            const int z = RZ[t];
            if (z < 0)
                continue;
            const bool centre = RC[t] != 0;
            const double v1[3] = {V[t], V[R + t], V[2 * R + t]};
            const double v2[3] = {V[3 * R + t], V[4 * R + t], V[5 * R + t]};
            for (int mm = 0; mm < kFitColsPerLane; ++mm) {
                const FitCol &c = col[mm];
                if (c.kind != 3 || c.a != z)
                    continue;
                const double u = P[c.p * R + t], ua = Pa[c.p * R + t];
                const double cs = C[c.s * R + t];
                const double X = ua * cs;
                double Y;
                if (centre) {
                    Y = Pb[c.p * R + t] * cs;
                    e[mm] += u * cs;
                } else {
                    Y = u * dC[c.s * R + t];
                }
                for (int k = 0; k < 3; ++k)
                    f[mm][k] += X * v1[k] + Y * v2[k];
            }
        }
    };

    if (three && m > 0) {
        // 2. triplets centred on i: unordered leg pairs (a < b)
        const int npairs = m * (m - 1) / 2;
        for (int base = 0; base < npairs; base += R) {
            const int t = base + lane;
            if (lane < R) {
                RZ[lane] = -1;
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
                    int fs;
                    double Cw[4], dCw[4];
                    fit_bspline(rjk, sh.nk3, sh.ih3c, fs, Cw, dCw);
                    put(lane, Ga.f, Ga.B, Ga.dB, Gb.f, Gb.B, Gb.dB, fs, Cw, dCw, true);
                    for (int k = 0; k < 3; ++k) {
                        V[k * R + lane] = Ga.d[k] * Ga.ir;
                        V[(3 + k) * R + lane] = Gb.d[k] * Gb.ir;
                    }
                    RZ[lane] = zi;
                    RC[lane] = 1;
                }
            }
            __syncthreads();
            consume3(npairs - base < R ? npairs - base : R);
            __syncthreads();
        }

        // 3. triplets centred on a 3-body neighbour j with i as one leg: the
        // other leg k runs over j's own 3-body list (k != i)
        if (lane == 0) {
            int acc = 0;
            for (int a = 0; a < m; ++a) {
                legpre[a] = acc;
                acc += l3cnt[leg[a].j];
            }
            legpre[m] = acc;
        }
        __syncthreads();
        const int total = legpre[m];
        for (int base = 0; base < total; base += R) {
            const int t = base + lane;
            if (lane < R) {
                RZ[lane] = -1;
                if (t < total) {
                    int a = 0;
                    while (legpre[a + 1] <= t)
                        ++a;
                    const FitLeg &Ga = leg[a];
                    const int j = Ga.j;
                    const int k = l3[(size_t)j * kMaxTriplet + (t - legpre[a])];
                    if (k >= 0 && k < n && k != i) {
                        double djk[3];
                        const double r2jk = fit_disp(pos, n, j, k, box, djk);
                        if (r2jk < rc3sq) {
                            const double rjk = sqrt(r2jk);
                            double d3[3];
                            for (int q = 0; q < 3; ++q)
                                d3[q] = Ga.d[q] + djk[q];
                            const double r3 = sqrt(d3[0] * d3[0] + d3[1] * d3[1] + d3[2] * d3[2]);
                            int fb, fs;
                            double Bw[4], dBw[4], Cw[4], dCw[4];
                            fit_bspline(rjk, sh.nk3, sh.ih3, fb, Bw, dBw);
                            fit_bspline(r3, sh.nk3, sh.ih3c, fs, Cw, dCw);
                            put(lane, Ga.f, Ga.B, Ga.dB, fb, Bw, dBw, fs, Cw, dCw, false);
                            for (int q = 0; q < 3; ++q) {
                                V[q * R + lane] = Ga.d[q] * Ga.ir;
                                V[(3 + q) * R + lane] = d3[q] / r3;
                            }
                            RZ[lane] = Ga.z;
                            RC[lane] = 0;
                        }
                    }
                }
            }
            __syncthreads();
            consume3(total - base < R ? total - base : R);
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

// Every atom's neighbours inside the 3-body cutoff, in row order (at most
// kMaxTriplet; more sets MLMIX_STATUS_TRIPLET_OVERFLOW).
__global__ void __launch_bounds__(kFitWave) k_fit_list3(FitBatch Bt, double rc3sq)
{
    const int cfg = fit_cfg_of(Bt, blockIdx.x);
    const FitCfgDev &Cf = Bt.c[cfg];
    const int n = Cf.n, cap = Cf.cap;
    const int *__restrict__ nbr = Cf.nbr;
    const int *__restrict__ cnt = Cf.cnt;
    const double *__restrict__ pos = Cf.pos;
    int *__restrict__ l3 = Cf.l3;
    int *__restrict__ l3cnt = Cf.l3cnt;
    int *__restrict__ hdr = Cf.hdr;
    const Box box = Cf.box;
    const int i = blockIdx.x - Bt.atom0[cfg];
    const int lane = threadIdx.x;
    if (i >= n)
        return;
    const int ci = cnt[i] < cap ? cnt[i] : cap;
    int m = 0;
    for (int base = 0; base < ci; base += kFitWave) {
        const int slot = base + lane;
        bool in3 = false;
        int j = -1;
        if (slot < ci) {
            j = nbr[(size_t)i * cap + slot];
            if (j >= 0 && j < n) {
                double d[3];
                in3 = fit_disp(pos, n, i, j, box, d) < rc3sq;
            }
        }
        const unsigned long long b = __ballot(in3);
        const int at3 = m + __popcll(b & ((1ull << lane) - 1ull));
        if (in3) {
            if (at3 < kMaxTriplet)
                l3[(size_t)i * kMaxTriplet + at3] = j;
            else
                atomicOr(&hdr[H_STATUS], MLMIX_STATUS_TRIPLET_OVERFLOW);
        }
        m += __popcll(b);
    }
    if (lane == 0)
        l3cnt[i] = m < kMaxTriplet ? m : kMaxTriplet;
}

// rows[0][k] = sum_i erow[k][i], one workgroup per (column, configuration),
// fixed order
__global__ void __launch_bounds__(256) k_fit_erow_sum(FitBatch Bt)
{
    __shared__ double sh[256];
    const int k = blockIdx.x;
    const FitCfgDev &Cf = Bt.c[blockIdx.y];
    const int n = Cf.n;
    const double *__restrict__ erow = Cf.erow;
    double *__restrict__ rows = Cf.rows;
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

void launch_fit_design(hipStream_t s, const Ctx &c, const FitCfgHost *cfg, int ncfg, int ld, int nd)
{
    FitShape sh;
    sh.ns = c.m.ns;
    sh.nk2 = c.d.uf3_n_knots2;
    sh.nk3 = c.d.uf3_n_knots3;
    sh.nd = nd;
    sh.n2cols = sh.ns * (sh.ns + 1) / 2 * (sh.nk2 - 1);
    sh.rc2 = c.d.uf3_rcut2;
    sh.rc3 = c.d.uf3_rcut3;
    sh.ih2 = (double)(sh.nk2 - 1) / sh.rc2;
    sh.ih3 = sh.nk3 > 1 ? (double)(sh.nk3 - 1) / sh.rc3 : 0.0;
    sh.ih3c = sh.nk3 > 1 ? (double)(sh.nk3 - 1) / (2.0 * sh.rc3) : 0.0;
    for (int c0 = 0; c0 < ncfg; c0 += kFitBatch) {
        FitBatch Bt{};
        Bt.ld = ld;
        int atoms = 0;
        for (int q = 0; q < kFitBatch && c0 + q < ncfg; ++q) {
            const FitCfgHost &h = cfg[c0 + q];
            const WsLayout &L = h.L;
            if (L.n == 0)
                continue;
            FitCfgDev &d = Bt.c[Bt.ncfg];
            d.n = L.n;
            d.cap = L.cap;
            d.nbr = at<int>(h.ws, L.nbr);
            d.cnt = at<int>(h.ws, L.cnt);
            d.pos = h.pos;
            d.species = h.species;
            d.rows = h.rows;
            d.erow = at<double>(h.ws, L.g);
            d.l3 = reinterpret_cast<int *>(d.erow + (size_t)nd * L.n);
            d.l3cnt = d.l3 + (size_t)kMaxTriplet * L.n;
            d.hdr = at<int>(h.ws, L.hdr);
            d.box = h.box;
            Bt.atom0[Bt.ncfg] = atoms;
            atoms += L.n;
            ++Bt.ncfg;
        }
        if (Bt.ncfg == 0)
            continue;
        Bt.atom0[Bt.ncfg] = atoms;
        if (sh.nk3 > 1)
            k_fit_list3<<<atoms, kFitWave, 0, s>>>(Bt, sh.rc3 * sh.rc3);
        k_fit_design<<<atoms, kFitWave, fit_design_lds(sh.nk2, sh.nk3), s>>>(Bt, sh);
        k_fit_erow_sum<<<dim3(nd, Bt.ncfg), 256, 0, s>>>(Bt);
    }
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
    // eight running sums (partial p goes to sum p mod 8) keep eight loads in
    // flight; they are combined in a fixed order
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int p = 0;
    for (; p + 8 <= nparts; p += 8)
        for (int q = 0; q < 8; ++q)
            acc[q] += part[(size_t)(p + q) * stride + e];
    for (int q = 0; p < nparts; ++p, ++q)
        acc[q] += part[(size_t)p * stride + e];
    const double s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
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
    const double *GS, *bS, *AH, *yH, *wH;
    double alpha, tol, lam0, ridge;
    int max_decades, max_bisect;
    const double *GH, *bH;  // A_H^T W A_H and A_H^T W y_H (built before the search)
    double *c, *info;
};

__device__ __forceinline__ double fit_wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o);
    return v;
}

// Orders one wavefront's LDS writes before its later LDS reads.
__device__ __forceinline__ void fit_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

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
    // packed lower triangle of M plus the right-hand side as an extra row nd
    // (factorising that row performs the forward substitution)
    constexpr int kPacked = (kFitMaxParams + 1) * (kFitMaxParams + 2) / 2;
    __shared__ double Lp[kPacked];
    __shared__ double cur[kFitMaxParams], keep[kFitMaxParams], rdg[kFitMaxParams];
    __shared__ double red[256];
    __shared__ int fail;
    const int nd = a.nd, tid = threadIdx.x;
    auto P = [](int r, int c2) { return r * (r + 1) / 2 + c2; };  // r >= c2


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
            Lp[P(nd, tid)] = a.bS[tid] + lam * a.bH[tid];
        if (tid == 0)
            fail = 0;
        __syncthreads();
        // left-looking Cholesky, column by column. The unnormalised column
        // is written first; every thread then scales its own entry by
        // 1/sqrt(t_jj) (kept in rdg), so a column needs two barriers. The
        // diagonal of Lp keeps t_jj; the substitutions use rdg.
        for (int j = 0; j < nd; ++j) {
            const int i = j + tid;  // rows j .. nd (nd = right-hand side); nd < 256
            double t = 0.0;
            if (i <= nd) {
                // four partial sums so that the LDS loads of later terms are
                // in flight while earlier ones accumulate
                const double *li = Lp + P(i, 0), *lj = Lp + P(j, 0);
                double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
                int k = 0;
                for (; k + 4 <= j; k += 4) {
                    t0 += li[k] * lj[k];
                    t1 += li[k + 1] * lj[k + 1];
                    t2 += li[k + 2] * lj[k + 2];
                    t3 += li[k + 3] * lj[k + 3];
                }
                for (; k < j; ++k)
                    t0 += li[k] * lj[k];
                t = Lp[P(i, j)] - ((t0 + t1) + (t2 + t3));
                Lp[P(i, j)] = t;
            }
            __syncthreads();
            const double tj = Lp[P(j, j)];
            const double r = tj > 0.0 ? 1.0 / sqrt(tj) : 1.0;
            if (i > j && i <= nd)
                Lp[P(i, j)] = t * r;
            if (tid == 0) {
                if (!(tj > 0.0))
                    fail = 1;
                rdg[j] = r;
            }
            __syncthreads();
        }
        // row nd now holds x with L x = b; L^T c = x by wavefront 0, column
        // by column (c_j = x_j / L_jj, then x_k -= L_jk c_j for k < j)
        if (tid < 64) {
            for (int k = tid; k < nd; k += 64)
                cur[k] = Lp[P(nd, k)];
            fit_wave_sync();
            for (int j = nd - 1; j >= 0; --j) {
                if (tid == 0)
                    cur[j] = cur[j] * rdg[j];
                fit_wave_sync();
                const double cj = cur[j];
                for (int k = tid; k < j; k += 64)
                    cur[k] -= Lp[P(j, k)] * cj;
                fit_wave_sync();
            }
        }
        __syncthreads();
        // hard residual: each wavefront takes four rows at a time, lanes
        // over the parameters
        double part = 0.0;
        const int wv = tid >> 6, ln = tid & 63;
        for (int h0 = 4 * wv; h0 < a.nh; h0 += 16) {
            double r[4] = {0.0, 0.0, 0.0, 0.0};
            for (int k = ln; k < nd; k += 64) {
                const double ck = cur[k];
                for (int q = 0; q < 4; ++q)
                    if (h0 + q < a.nh)
                        r[q] += a.AH[(size_t)(h0 + q) * a.ldh + k] * ck;
            }
            for (int q = 0; q < 4; ++q) {
                const double rq = fit_wave_sum(r[q]);
                if (ln == 0 && h0 + q < a.nh) {
                    const double d = rq - a.yH[h0 + q];
                    part += (a.wH ? a.wH[h0 + q] : 1.0) * d * d;
                }
            }
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
                       const double *AH, const double *yH, const double *wH, double alpha,
                       double tol, double lam0, double ridge, int max_decades, int max_bisect,
                       double *c, double *info, double *scratch)
{
    // G_H, b_H by the Gram kernels (zeroed by a fill kernel first), then the
    // search in one workgroup
    double *GH = scratch, *bH = scratch + (size_t)nd * nd, *part = bH + nd;
    launch_fill_f64(s, GH, 0.0, (size_t)nd * nd + nd);
    launch_fit_gram(s, nh, nd, ldh, AH, yH, wH, GH, bH, part);
    FitSearchArgs a{nd, nh, ldh, GS, bS, AH, yH, wH, alpha, tol, lam0, ridge, max_decades, max_bisect,
                    GH, bH, c, info};
    k_fit_search<<<1, 256, 0, s>>>(a);
}

}  // namespace mlmix
