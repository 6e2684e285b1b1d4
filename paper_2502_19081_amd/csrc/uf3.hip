// Cheap UF3-style 2+3-body potential on every atom, on gfx950.
//
// One wavefront per centre atom i. Pair terms: lanes own neighbour slots,
// E_i += V2(r)/2 and h_ij = dE_i/dd_ij = V2'(r) u/2. Three-body terms: the
// neighbours inside the 3-body cutoff are compacted into LDS in row order
// with their B-spline bases; lane t owns leg j = t and loops over the other
// legs k. Because the coefficients are symmetric in the two leg indices,
// E_i3 = sum_{j<k} V3 = 1/2 sum_j sum_{k!=j} V3(r_ij, r_ik, r_jk) and
// dE_i3/dd_ij = sum_{k!=j} [dV3/dr_1 u_ij - dV3/dr_3 (d_ik - d_ij)/r_jk],
// so every lane writes only its own slot (no atomics, fixed summation
// order). Forces follow in the gather kernel: F_i = sum_j (h_ij - h_ji).
#include "internal.h"

namespace mlmix {

template <typename T>
struct Uf3Args {
    int ns, nk2, nk3, nb2, nb3;
    double rc2sq, rc3sq;
    T h2, ih2, h3, ih3, h3c, ih3c;
    const T *c2, *c3;
    const T *p2, *p3;  // per-span B-spline polynomial coefficients [npts - 1][4][4]
};

// The four non-zero clamped uniform cubic B-splines at x and their
// derivatives from the per-span cubic coefficients (Horner, no division):
// span sp = clamp(floor(x / h), 0, npts - 2), t = x / h - sp, basis r of the
// span = sum_e poly[16 sp + 4 r + e] t^e, derivative / h.
template <typename T>
__device__ __forceinline__ void bspline4p(T x, T ih, int npts, const T *__restrict__ poly, int &first,
                                          T N[4], T dN[4])
{
    const T u = x * ih;
    int sp = (int)floor(u);
    sp = sp < 0 ? 0 : (sp > npts - 2 ? npts - 2 : sp);
    const T t = u - T(sp);
    const T *c = poly + 16 * sp;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const T a0 = c[4 * r], a1 = c[4 * r + 1], a2 = c[4 * r + 2], a3 = c[4 * r + 3];
        N[r] = ((a3 * t + a2) * t + a1) * t + a0;
        dN[r] = ((T(3) * a3 * t + T(2) * a2) * t + a1) * ih;
    }
    first = sp;
}

// d = x_j - x_i folded once along periodic dimensions; returns |d|^2 (FP64,
// no FMA contraction, so the cutoff decisions match the neighbour search).
__device__ __forceinline__ double pair_disp_u(const double *__restrict__ pos, int n, int i, int j,
                                              const Box &b, double d[3])
{
#pragma clang fp contract(off)
    const double xj[3] = {pos[j], pos[n + j], pos[2 * n + j]};
    const double xi[3] = {pos[i], pos[n + i], pos[2 * n + i]};
    for (int k = 0; k < 3; ++k) {
        double dx = xj[k] - xi[k];
        if (b.per[k]) {
            double hh = 0.5 * b.L[k];
            dx = dx > hh ? dx - b.L[k] : (dx < -hh ? dx + b.L[k] : dx);
        }
        d[k] = dx;
    }
    double r2 = d[0] * d[0];
    r2 = r2 + d[1] * d[1];
    r2 = r2 + d[2] * d[2];
    return r2;
}

template <typename T>
__device__ __forceinline__ T wave_sum_t(T v)
{
#pragma unroll
    for (int d = 32; d > 0; d >>= 1)
        v += __shfl_xor(v, d);
    return v;
}

// Per-wave LDS slice of the cheap kernel, in elements of T (ints stored in
// T-sized slots are avoided: the integer arrays follow the T arrays).
struct Uf3Slice {
    int hs, d3, r3, B3, dB3, c3s, nT;  // offsets of the T arrays and their total
};

__host__ __device__ inline Uf3Slice uf3_slice(int cap, int nb3c)
{
    Uf3Slice l;
    l.hs = 0;
    l.d3 = l.hs + 3 * cap;
    l.r3 = l.d3 + 3 * kMaxTriplet;
    l.B3 = l.r3 + kMaxTriplet;
    l.dB3 = l.B3 + 4 * kMaxTriplet;
    l.c3s = l.dB3 + 4 * kMaxTriplet;
    l.nT = l.c3s + nb3c;
    return l;
}

// Four centre atoms per 256-thread block, one wavefront each. The loops run
// to the block's maximum row length so that the four waves meet at every
// barrier; each wave works in its own LDS slice.
template <typename T>
__global__ void __launch_bounds__(256)
    k_uf3(const double *__restrict__ pos, int n, Box b, const int32_t *__restrict__ species,
          int cap, const int *__restrict__ nbr, const int *__restrict__ cnt, Uf3Args<T> a,
          T *__restrict__ hout, double *__restrict__ e_cheap, int *hdr)
{
    const int nb3c = a.nb3 > 0 ? a.nb3 * a.nb3 * a.nb3 : 0;
    const Uf3Slice sl = uf3_slice(cap, nb3c);
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + w;
    const bool valid = i < n;
    extern __shared__ __align__(16) char smem_raw[];
    T *base = reinterpret_cast<T *>(smem_raw) + (size_t)w * sl.nT;
    T *hs = base + sl.hs;
    T *d3 = base + sl.d3;
    T *r3 = base + sl.r3;
    T *B3 = base + sl.B3;
    T *dB3 = base + sl.dB3;
    T *c3s = base + sl.c3s;
    int *ibase = reinterpret_cast<int *>(reinterpret_cast<T *>(smem_raw) + 4 * (size_t)sl.nT);
    int *f3 = ibase + w * 2 * kMaxTriplet;
    int *sl3 = f3 + kMaxTriplet;
    // per-span B-spline polynomials, shared by the block
    T *pp2 = reinterpret_cast<T *>(ibase + 4 * 2 * kMaxTriplet);
    T *pp3 = pp2 + 16 * (a.nk2 - 1);
    for (int e = threadIdx.x; e < 16 * (a.nk2 - 1); e += blockDim.x)
        pp2[e] = a.p2[e];
    if (a.nb3 > 0)
        for (int e = threadIdx.x; e < 16 * (a.nk3 - 1); e += blockDim.x)
            pp3[e] = a.p3[e];
    __shared__ int count3[4];
    __shared__ int cmax_s[4];
    const int zi = valid ? sp_clamp(species[i], a.ns) : 0;
    const int c = valid ? cnt[i] : 0;
    const int *row = nbr + (size_t)(valid ? i : 0) * cap;
    if (lane == 0) {
        count3[w] = 0;
        cmax_s[w] = c;
    }
    for (int e = lane; e < nb3c; e += 64)
        c3s[e] = a.c3[(size_t)zi * nb3c + e];
    for (int e = lane; e < 3 * c; e += 64)
        hs[e] = T(0);
    __syncthreads();
    const int cmax = max(max(cmax_s[0], cmax_s[1]), max(cmax_s[2], cmax_s[3]));
    T Ep = T(0);
    for (int base0 = 0; base0 < cmax; base0 += 64) {
        int slot = base0 + lane;
        bool in3 = false;
        double d[3] = {0.0, 0.0, 0.0};
        double r2 = 0.0;
        if (slot < c) {
            int j = row[slot];
            r2 = pair_disp_u(pos, n, i, j, b, d);
            if (r2 < a.rc2sq) {
                double rd = sqrt(r2);
                T r = T(rd);
                int f;
                T N[4], dN[4];
                bspline4p<T>(r, a.ih2, a.nk2, pp2, f, N, dN);
                const T *cc = a.c2 + ((size_t)zi * a.ns + sp_clamp(species[j], a.ns)) * a.nb2 + f;
                T V = T(0), dV = T(0);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    V += cc[q] * N[q];
                    dV += cc[q] * dN[q];
                }
                Ep += T(0.5) * V;
                T sc = T(0.5) * dV / r;
                hs[slot * 3 + 0] = sc * T(d[0]);
                hs[slot * 3 + 1] = sc * T(d[1]);
                hs[slot * 3 + 2] = sc * T(d[2]);
            }
            in3 = a.nb3 > 0 && r2 < a.rc3sq;
        }
        unsigned long long mask = __ballot(in3);
        int before = __popcll(mask & ((1ull << lane) - 1ull));
        int p = count3[w] + before;
        if (in3 && p < kMaxTriplet) {
            double rd = sqrt(r2);
            d3[p * 3 + 0] = T(d[0]);
            d3[p * 3 + 1] = T(d[1]);
            d3[p * 3 + 2] = T(d[2]);
            r3[p] = T(rd);
            sl3[p] = slot;
            int f;
            T N[4], dN[4];
            bspline4p<T>(T(rd), a.ih3, a.nk3, pp3, f, N, dN);
            f3[p] = f;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                B3[p * 4 + q] = N[q];
                dB3[p * 4 + q] = dN[q];
            }
        }
        __syncthreads();
        if (lane == 0)
            count3[w] += __popcll(mask);
        __syncthreads();
    }
    int n3 = count3[w];
    if (n3 > kMaxTriplet) {
        if (lane == 0)
            atomicOr(&hdr[H_STATUS], MLMIX_STATUS_TRIPLET_OVERFLOW);
        n3 = kMaxTriplet;
    }
    if (a.nb3 > 0) {
        // lane = leg j (low four bits) + k residue class kc (high two bits):
        // lane (j, kc) sums the triplets (j, k) with k = kc (mod 4), then the
        // four partial sums of leg j meet in a fixed shuffle order.
        const int jl = lane & 15, kc = lane >> 4;
        const int nb = a.nb3;
        for (int jb = 0; jb < n3; jb += 16) {
            const int t = jb + jl;
            T hx = T(0), hy = T(0), hz = T(0);
            if (t < n3) {
                T dj0 = d3[t * 3], dj1 = d3[t * 3 + 1], dj2 = d3[t * 3 + 2];
                T rj = r3[t];
                int fj = f3[t];
                T Bj[4], dBj[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    Bj[q] = B3[t * 4 + q];
                    dBj[q] = dB3[t * 4 + q];
                }
                for (int k = kc; k < n3; k += 4) {
                    if (k == t)
                        continue;
                    T e0 = d3[k * 3] - dj0, e1 = d3[k * 3 + 1] - dj1, e2 = d3[k * 3 + 2] - dj2;
                    T rjk = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
                    int fs;
                    T Ns[4], dNs[4];
                    bspline4p<T>(rjk, a.ih3c, a.nk3, pp3, fs, Ns, dNs);
                    int fk = f3[k];
                    T V = T(0), V1 = T(0), V3 = T(0);
#pragma unroll
                    for (int pp = 0; pp < 4; ++pp) {
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const T *cr = c3s + ((fj + pp) * nb + (fk + q)) * nb + fs;
                            T bk = B3[k * 4 + q];
                            T s0 = T(0), s1 = T(0);
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                s0 += cr[u] * Ns[u];
                                s1 += cr[u] * dNs[u];
                            }
                            V += Bj[pp] * bk * s0;
                            V1 += dBj[pp] * bk * s0;
                            V3 += Bj[pp] * bk * s1;
                        }
                    }
                    Ep += T(0.5) * V;
                    T a1 = V1 / rj;
                    T a3 = V3 / rjk;
                    hx += a1 * dj0 - a3 * e0;
                    hy += a1 * dj1 - a3 * e1;
                    hz += a1 * dj2 - a3 * e2;
                }
            }
            hx += __shfl_xor(hx, 16);
            hy += __shfl_xor(hy, 16);
            hz += __shfl_xor(hz, 16);
            hx += __shfl_xor(hx, 32);
            hy += __shfl_xor(hy, 32);
            hz += __shfl_xor(hz, 32);
            if (kc == 0 && t < n3) {
                int slt = sl3[t];
                hs[slt * 3 + 0] += hx;
                hs[slt * 3 + 1] += hy;
                hs[slt * 3 + 2] += hz;
            }
        }
    }
    __syncthreads();
    if (!valid)
        return;
    T *ho = hout + (size_t)i * cap * 3;
    for (int e = lane; e < 3 * c; e += 64)
        ho[e] = hs[e];
    T E = wave_sum_t(Ep);
    if (lane == 0)
        e_cheap[i] = (double)E;
}

template <typename T>
static void uf3_t(hipStream_t s, const Ctx &c, void *ws, const WsLayout &L, const Box &b,
                  const double *pos, const int32_t *species, double *e_cheap)
{
    const DevModel &m = c.m;
    Uf3Args<T> a;
    a.ns = m.ns;
    a.nk2 = m.nk2;
    a.nk3 = m.nk3;
    a.nb2 = m.nb2;
    a.nb3 = m.nb3;
    a.rc2sq = m.rc2 * m.rc2;
    a.rc3sq = m.nb3 > 0 ? m.rc3 * m.rc3 : -1.0;
    double h2 = m.rc2 / (m.nk2 - 1);
    a.h2 = T(h2);
    a.ih2 = T(1.0 / h2);
    double h3 = m.nb3 > 0 ? m.rc3 / (m.nk3 - 1) : 1.0;
    a.h3 = T(h3);
    a.ih3 = T(1.0 / h3);
    a.h3c = T(2.0 * h3);
    a.ih3c = T(0.5 / h3);
    char *base = static_cast<char *>(m.base);
    a.c2 = reinterpret_cast<const T *>(base + m.u2);
    a.c3 = reinterpret_cast<const T *>(base + m.u3);
    a.p2 = reinterpret_cast<const T *>(base + m.up2);
    a.p3 = reinterpret_cast<const T *>(base + m.up3);
    int nb3c = m.nb3 > 0 ? m.nb3 * m.nb3 * m.nb3 : 0;
    Uf3Slice sl = uf3_slice(L.cap, nb3c);
    size_t sm = 4 * ((size_t)sl.nT * sizeof(T) + 2 * kMaxTriplet * sizeof(int)) +
                16 * ((size_t)(m.nk2 - 1) + (m.nb3 > 0 ? m.nk3 - 1 : 0)) * sizeof(T) + 16;
    k_uf3<T><<<(L.n + 3) / 4, 256, sm, s>>>(pos, L.n, b, species, L.cap, at<int>(ws, L.nbr),
                                 at<int>(ws, L.cnt), a, at<T>(ws, L.h), e_cheap,
                                 at<int>(ws, L.hdr));
}

void launch_uf3(hipStream_t s, const Ctx &c, void *ws, const WsLayout &L, const Box &b,
                const double *pos, const int32_t *species, double *e_cheap)
{
    if (L.n == 0)
        return;
    if (c.prec == MLMIX_FP64)
        uf3_t<double>(s, c, ws, L, b, pos, species, e_cheap);
    else
        uf3_t<float>(s, c, ws, L, b, pos, species, e_cheap);
}

}  // namespace mlmix
