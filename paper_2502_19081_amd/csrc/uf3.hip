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
};

// The four non-zero clamped uniform cubic B-splines at x (first index
// `first`) and their derivatives; knots t(i) = h * clamp(i - 3, 0, npts - 1).
template <typename T>
__device__ __forceinline__ void bspline4(T x, T h, T ih, int npts, int &first, T N[4], T dN[4])
{
    int sp = (int)floor(x * ih);
    if (sp < 0)
        sp = 0;
    if (sp > npts - 2)
        sp = npts - 2;
    int k = sp + 3;
    auto t = [&](int q) -> T {
        int v = q - 3;
        v = v < 0 ? 0 : (v > npts - 1 ? npts - 1 : v);
        return h * T(v);
    };
    T left[4], right[4], Nn[4], N2[3];
    Nn[0] = T(1);
#pragma unroll
    for (int j = 1; j <= 3; ++j) {
        left[j] = x - t(k + 1 - j);
        right[j] = t(k + j) - x;
        T saved = T(0);
#pragma unroll
        for (int r = 0; r < j; ++r) {
            T temp = Nn[r] / (right[r + 1] + left[j - r]);
            Nn[r] = saved + right[r + 1] * temp;
            saved = left[j - r] * temp;
        }
        Nn[j] = saved;
        if (j == 2) {
            N2[0] = Nn[0];
            N2[1] = Nn[1];
            N2[2] = Nn[2];
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        N[r] = Nn[r];
        T a = (r >= 1) ? N2[r - 1] / (t(k + r) - t(k + r - 3)) : T(0);
        T b = (r <= 2) ? N2[r] / (t(k + r + 1) - t(k + r - 2)) : T(0);
        dN[r] = T(3) * (a - b);
    }
    first = k - 3;
}

// d = x_j - x_i folded once along periodic dimensions; returns |d|^2 (FP64,
// no FMA contraction, so the cutoff decisions match the neighbour search).
__device__ __forceinline__ double pair_disp_u(const double *__restrict__ pos, int n, int i, int j,
                                              const Box &b, double d[3])
{
#pragma clang fp contract(off)
    for (int k = 0; k < 3; ++k) {
        double dx = pos[k * n + j] - pos[k * n + i];
        if (b.per[k]) {
            double hh = 0.5 * b.L[k];
            if (dx > hh)
                dx = dx - b.L[k];
            else if (dx < -hh)
                dx = dx + b.L[k];
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

template <typename T>
__global__ void __launch_bounds__(64)
    k_uf3(const double *__restrict__ pos, int n, Box b, const int32_t *__restrict__ species,
          int cap, const int *__restrict__ nbr, const int *__restrict__ cnt, Uf3Args<T> a,
          T *__restrict__ hout, double *__restrict__ e_cheap, int *hdr)
{
    extern __shared__ char smem_raw[];
    T *hs = reinterpret_cast<T *>(smem_raw);          // [cap][3]
    T *d3 = hs + 3 * cap;                             // [64][3]
    T *r3 = d3 + 3 * kMaxTriplet;                     // [64]
    T *B3 = r3 + kMaxTriplet;                         // [64][4]
    T *dB3 = B3 + 4 * kMaxTriplet;                    // [64][4]
    T *c3s = dB3 + 4 * kMaxTriplet;                   // [nb3^3]
    int *f3 = reinterpret_cast<int *>(c3s + (a.nb3 > 0 ? a.nb3 * a.nb3 * a.nb3 : 0));  // [64]
    int *sl3 = f3 + kMaxTriplet;                      // [64]
    __shared__ int count3;
    int i = blockIdx.x;
    int lane = threadIdx.x;
    int zi = sp_clamp(species[i], a.ns);
    int c = cnt[i];
    const int *row = nbr + (size_t)i * cap;
    if (lane == 0)
        count3 = 0;
    const int nb3c = a.nb3 * a.nb3 * a.nb3;
    for (int e = lane; e < nb3c; e += 64)
        c3s[e] = a.c3[(size_t)zi * nb3c + e];
    for (int e = lane; e < 3 * c; e += 64)
        hs[e] = T(0);
    __syncthreads();
    T Ep = T(0);
    for (int base = 0; base < c; base += 64) {
        int slot = base + lane;
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
                bspline4<T>(r, a.h2, a.ih2, a.nk2, f, N, dN);
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
        int p = count3 + before;
        if (in3 && p < kMaxTriplet) {
            double rd = sqrt(r2);
            d3[p * 3 + 0] = T(d[0]);
            d3[p * 3 + 1] = T(d[1]);
            d3[p * 3 + 2] = T(d[2]);
            r3[p] = T(rd);
            sl3[p] = slot;
            int f;
            T N[4], dN[4];
            bspline4<T>(T(rd), a.h3, a.ih3, a.nk3, f, N, dN);
            f3[p] = f;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                B3[p * 4 + q] = N[q];
                dB3[p * 4 + q] = dN[q];
            }
        }
        __syncthreads();
        if (lane == 0)
            count3 += __popcll(mask);
        __syncthreads();
    }
    int n3 = count3;
    if (n3 > kMaxTriplet) {
        if (lane == 0)
            atomicOr(&hdr[H_STATUS], MLMIX_STATUS_TRIPLET_OVERFLOW);
        n3 = kMaxTriplet;
    }
    if (a.nb3 > 0 && lane < n3) {
        const int t = lane;
        T dj0 = d3[t * 3], dj1 = d3[t * 3 + 1], dj2 = d3[t * 3 + 2];
        T rj = r3[t];
        int fj = f3[t];
        T Bj[4], dBj[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            Bj[q] = B3[t * 4 + q];
            dBj[q] = dB3[t * 4 + q];
        }
        T hx = T(0), hy = T(0), hz = T(0);
        const int nb = a.nb3;
        for (int k = 0; k < n3; ++k) {
            if (k == t)
                continue;
            T e0 = d3[k * 3] - dj0, e1 = d3[k * 3 + 1] - dj1, e2 = d3[k * 3 + 2] - dj2;
            T rjk = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
            int fs;
            T Ns[4], dNs[4];
            bspline4<T>(rjk, a.h3c, a.ih3c, a.nk3, fs, Ns, dNs);
            int fk = f3[k];
            T V = T(0), V1 = T(0), V3 = T(0);
#pragma unroll
            for (int p = 0; p < 4; ++p) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const T *cr = c3s + ((fj + p) * nb + (fk + q)) * nb + fs;
                    T bk = B3[k * 4 + q];
                    T s0 = T(0), s1 = T(0);
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        s0 += cr[u] * Ns[u];
                        s1 += cr[u] * dNs[u];
                    }
                    V += Bj[p] * bk * s0;
                    V1 += dBj[p] * bk * s0;
                    V3 += Bj[p] * bk * s1;
                }
            }
            Ep += T(0.5) * V;
            T a1 = V1 / rj;
            T a3 = V3 / rjk;
            hx += a1 * dj0 - a3 * e0;
            hy += a1 * dj1 - a3 * e1;
            hz += a1 * dj2 - a3 * e2;
        }
        int sl = sl3[t];
        hs[sl * 3 + 0] += hx;
        hs[sl * 3 + 1] += hy;
        hs[sl * 3 + 2] += hz;
    }
    __syncthreads();
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
    int nb3c = m.nb3 > 0 ? m.nb3 * m.nb3 * m.nb3 : 0;
    size_t sm = (size_t)(3 * L.cap + 3 * kMaxTriplet + kMaxTriplet + 8 * kMaxTriplet + nb3c) * sizeof(T) +
                2 * kMaxTriplet * sizeof(int) + 16;
    k_uf3<T><<<L.n, 64, sm, s>>>(pos, L.n, b, species, L.cap, at<int>(ws, L.nbr),
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
