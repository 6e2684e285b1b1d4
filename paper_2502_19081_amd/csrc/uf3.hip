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

// Four consecutive coefficients (16-byte aligned for float, two 16-byte
// loads for double).
__device__ __forceinline__ void load4(const float *p, float v[4])
{
    const float4 q = *reinterpret_cast<const float4 *>(p);
    v[0] = q.x;
    v[1] = q.y;
    v[2] = q.z;
    v[3] = q.w;
}

__device__ __forceinline__ void load4(const double *p, double v[4])
{
    const double2 q0 = *reinterpret_cast<const double2 *>(p);
    const double2 q1 = *reinterpret_cast<const double2 *>(p + 2);
    v[0] = q0.x;
    v[1] = q0.y;
    v[2] = q1.x;
    v[3] = q1.y;
}

// Square root and reciprocal of the 3-body leg-pair distance: the hardware
// instructions (1 ulp) in FP32, the correctly rounded ones in FP64.
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fast_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fast_rcp(double x) { return 1.0 / x; }

// Length of a pair and its inverse from the FP64 squared length (whose
// cutoff tests stay in FP64): the hardware instructions on the FP32 value in
// FP32, the correctly rounded FP64 ones in FP64.
__device__ __forceinline__ void pair_len(double r2, float &r, float &ir)
{
    r = __builtin_amdgcn_sqrtf((float)r2);
    ir = __builtin_amdgcn_rcpf(r);
}
__device__ __forceinline__ void pair_len(double r2, double &r, double &ir)
{
    r = sqrt(r2);
    ir = 1.0 / r;
}

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
        T cr[4];
        load4(c + 4 * r, cr);  // 16-byte aligned (spans of 16 values)
        const T a0 = cr[0], a1 = cr[1], a2 = cr[2], a3 = cr[3];
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

__device__ __forceinline__ void wave_sync_lds_u()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Per-wave LDS arrays of the cheap kernel, in elements of T: leg vectors d3
// (3 x 64), inverse lengths (64), bases and derivatives (2 x 4 x 64) and the
// per-round pair contributions (6 x 64; afterwards the leg sums, 3 x 64).
constexpr int kUf3WaveT = 3 * kMaxTriplet + kMaxTriplet + 8 * kMaxTriplet + 6 * kMaxTriplet;

__host__ __device__ inline int uf3_c3_elems(int ns, int nb3)
{
    return nb3 > 0 ? ns * nb3 * nb3 * (nb3 - 3) * 4 : 0;
}

// Four centre atoms per block, one wavefront each (grid-stride over groups
// of atoms when the grid is capped); the spline and coefficient tables are
// staged once per block (the only block barrier), everything after it is
// wave-local.
//
// Pair terms: lane l owns row slots l + 64 u (u < U); all row entries and
// partner positions are loaded before any arithmetic, E_i += V2(r)/2 and
// h_ij = V2'(r) u / 2. Three-body terms: the legs inside the 3-body cutoff
// are compacted by ballot into LDS in row order with their B-spline bases;
// every unordered leg pair {j, k} is evaluated once (the coefficients are
// symmetric in the two leg indices), E_i3 = sum_{j<k} V3(r_ij, r_ik, r_jk).
// The pairs are enumerated cyclically, p = (o - 1) n3 + j with partner
// k = (j + o) mod n3 for o = 1..n3/2 (for even n3 the last offset only for
// j < n3/2), 64 pairs per round. Each pair leaves
// dV3/dd_ij = V_1 u_ij - V_3 e / r_jk and dV3/dd_ik = V_2 u_ik + V_3 e / r_jk
// (e = d_ik - d_ij) in LDS, and the lane of each leg adds the entries of its
// pairs in a fixed order: no atomics, the same bits on every run.
template <typename T, int U, bool LOOP, bool SEG>
__global__ void __launch_bounds__(256)
    k_uf3(const double *__restrict__ pos, int n, Box b, const int32_t *__restrict__ species,
          int cap, const int *__restrict__ nbr, const int *__restrict__ cnt, Uf3Args<T> a,
          T *__restrict__ hout, double *__restrict__ e_cheap, int *hdr,
          const uint8_t *__restrict__ mflags, Seg sg)
{
    const int nb = a.nb3;
    const int c3n = uf3_c3_elems(a.ns, nb);
    constexpr int nT = kUf3WaveT;
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    extern __shared__ __align__(16) char smem_raw[];
    T *c3x = reinterpret_cast<T *>(smem_raw);
    T *d3 = c3x + c3n + (size_t)w * nT;
    T *ir3 = d3 + 3 * kMaxTriplet;
    T *B3 = ir3 + kMaxTriplet;
    T *dB3 = B3 + 4 * kMaxTriplet;
    T *rb = dB3 + 4 * kMaxTriplet;
    constexpr int wpb = 4;  // waves (atoms in flight) per block
    int *f3 = reinterpret_cast<int *>(c3x + c3n + wpb * (size_t)nT) + w * kMaxTriplet;
    T *pp2 = reinterpret_cast<T *>(reinterpret_cast<int *>(c3x + c3n + wpb * (size_t)nT) +
                                   wpb * kMaxTriplet);
    T *pp3 = pp2 + 16 * (a.nk2 - 1);
    T *c2s = pp3 + (nb > 0 ? 16 * (a.nk3 - 1) : 0);
    const int c2n = a.ns * a.ns * a.nb2;
    for (int e = threadIdx.x; e < 16 * (a.nk2 - 1); e += blockDim.x)
        pp2[e] = a.p2[e];
    for (int e = threadIdx.x; e < c2n; e += blockDim.x)
        c2s[e] = a.c2[e];
    if (nb > 0) {
        for (int e = threadIdx.x; e < 16 * (a.nk3 - 1); e += blockDim.x)
            pp3[e] = a.p3[e];
        for (int e = threadIdx.x; e < c3n; e += blockDim.x)
            c3x[e] = a.c3[e];
    }
    __syncthreads();
    // one atom per wave: one group of atoms per block, or a grid-stride loop
    // over groups (capped grids); no block barrier below
    auto atom = [&](const int i) {
        wave_sync_lds_u();
        const Box bi = seg_box<SEG, true>(b, sg, i);  // box of the atom's system
        const int zi = sp_clamp(species[i], a.ns);
        const int c = cnt[i];
        const int *row = nbr + (size_t)i * cap;
        // masked (S_c = {lambda < 1} plus the cheap buffer): a centre outside
        // S_c has no cheap energy or gradients, partners outside are absent
        auto in_sc = [&](int k) { return !(mflags[k] & 2) || (mflags[k] & 8); };
        const bool centre = !mflags || in_sc(i);
        int jj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int slot = lane + 64 * u;
            jj[u] = slot < c ? row[slot] : -1;
            if (jj[u] >= 0 && (!centre || (mflags && !in_sc(jj[u]))))
                jj[u] = -1;  // the slot's gradient is written as zero
        }
        double dd[U][3], rr2[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            rr2[u] = 1.0e300;
            dd[u][0] = dd[u][1] = dd[u][2] = 0.0;
            if (jj[u] >= 0)
                rr2[u] = pair_disp_u(pos, n, i, jj[u], bi, dd[u]);
        }
        int zj[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            zj[u] = (a.ns > 1 && jj[u] >= 0) ? sp_clamp(species[jj[u]], a.ns) : 0;
        T Ep = T(0);
        int n3 = 0;
        T hx[U], hy[U], hz[U];  // dE_i/dd_ij of the lane's slots
        int leg[U];             // 3-body leg index of the slot, or -1
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int slot = lane + 64 * u;
            const double r2 = rr2[u];
            hx[u] = hy[u] = hz[u] = T(0);
            leg[u] = -1;
            T r = T(1), ir = T(1);
            if (r2 < a.rc2sq || (nb > 0 && r2 < a.rc3sq))
                pair_len(r2, r, ir);
            if (r2 < a.rc2sq) {
                int f;
                T N[4], dN[4];
                bspline4p<T>(r, a.ih2, a.nk2, pp2, f, N, dN);
                const T *cc = c2s + (zi * a.ns + zj[u]) * a.nb2 + f;
                T V = T(0), dV = T(0);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    V += cc[q] * N[q];
                    dV += cc[q] * dN[q];
                }
                Ep += T(0.5) * V;
                const T sc = T(0.5) * dV * ir;
                hx[u] = sc * T(dd[u][0]);
                hy[u] = sc * T(dd[u][1]);
                hz[u] = sc * T(dd[u][2]);
            }
            const bool in3 = nb > 0 && r2 < a.rc3sq;
            const unsigned long long mask = __ballot(in3);
            const int p = n3 + __popcll(mask & ((1ull << lane) - 1ull));
            if (in3 && p < kMaxTriplet) {
                d3[p * 3 + 0] = T(dd[u][0]);
                d3[p * 3 + 1] = T(dd[u][1]);
                d3[p * 3 + 2] = T(dd[u][2]);
                ir3[p] = ir;
                leg[u] = p;
                int f;
                T N[4], dN[4];
                bspline4p<T>(r, a.ih3, a.nk3, pp3, f, N, dN);
                f3[p] = f;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    B3[p * 4 + q] = N[q];
                    dB3[p * 4 + q] = dN[q];
                }
            }
            n3 += __popcll(mask);
        }
        wave_sync_lds_u();
        if (n3 > kMaxTriplet) {
            if (lane == 0)
                seg_status_or<SEG>(&hdr[H_STATUS], sg, i, MLMIX_STATUS_TRIPLET_OVERFLOW);
            n3 = kMaxTriplet;
        }
        if (nb > 0) {
            const T *cz = c3x + (size_t)zi * nb * nb * (nb - 3) * 4;
            const int hh = n3 >> 1;
            const float rn3 = 1.0f / (float)(n3 > 0 ? n3 : 1);
            const bool even = (n3 & 1) == 0;
            // V3 of the leg pair (j, k) added to the energy; dV3/dd_ij and
            // dV3/dd_ik returned in cj, ck
            auto leg_pair = [&](const int j, const int k, T cj[3], T ck[3]) {
                const T dj0 = d3[j * 3], dj1 = d3[j * 3 + 1], dj2 = d3[j * 3 + 2];
                const T dk0 = d3[k * 3], dk1 = d3[k * 3 + 1], dk2 = d3[k * 3 + 2];
                const int fj = f3[j], fk = f3[k];
                T Bj[4], dBj[4], Bk[4], dBk[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    Bj[q] = B3[j * 4 + q];
                    dBj[q] = dB3[j * 4 + q];
                    Bk[q] = B3[k * 4 + q];
                    dBk[q] = dB3[k * 4 + q];
                }
                const T e0 = dk0 - dj0, e1 = dk1 - dj1, e2 = dk2 - dj2;
                const T rjk = fast_sqrt(e0 * e0 + e1 * e1 + e2 * e2);
                int fs;
                T Ns[4], dNs[4];
                bspline4p<T>(rjk, a.ih3c, a.nk3, pp3, fs, Ns, dNs);
                // contract the r_jk basis first, then leg k, then leg j
                T V = T(0), V1 = T(0), V2 = T(0), V3 = T(0);
#pragma unroll
                for (int pa = 0; pa < 4; ++pa) {
                    T u0 = T(0), uk = T(0), u1 = T(0);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        T cr[4];
                        load4(cz + ((((fj + pa) * nb + (fk + q)) * (nb - 3) + fs) << 2), cr);
                        const T s0 = ((cr[0] * Ns[0] + cr[1] * Ns[1]) + cr[2] * Ns[2]) + cr[3] * Ns[3];
                        const T s1 = ((cr[0] * dNs[0] + cr[1] * dNs[1]) + cr[2] * dNs[2]) + cr[3] * dNs[3];
                        u0 += s0 * Bk[q];
                        uk += s0 * dBk[q];
                        u1 += s1 * Bk[q];
                    }
                    V += Bj[pa] * u0;
                    V1 += dBj[pa] * u0;
                    V2 += Bj[pa] * uk;
                    V3 += Bj[pa] * u1;
                }
                Ep += V;
                const T irjk = fast_rcp(rjk);
                const T aj = V1 * ir3[j], ak = V2 * ir3[k], ajk = V3 * irjk;
                cj[0] = aj * dj0 - ajk * e0;
                cj[1] = aj * dj1 - ajk * e1;
                cj[2] = aj * dj2 - ajk * e2;
                ck[0] = ak * dk0 + ajk * e0;
                ck[1] = ak * dk1 + ajk * e1;
                ck[2] = ak * dk2 + ajk * e2;
            };
            T gx = T(0), gy = T(0), gz = T(0);  // lane x < n3: leg x
            // Two layouts of the unordered pairs {x, x + o} (o = 1..n3/2) on
            // the lanes, whichever takes fewer rounds of 64:
            //  blocks: lane x + n3 s (s < S = 64 / n3) takes offsets
            //   o = s + 1 + r S in round r; in a round the lanes of one block
            //   have distinct second legs, so lane x + n3 s keeps the
            //   first-leg term of its pair and receives the second-leg term
            //   of the pair (x - o, x) of its block through one LDS slot
            //   (no search); the S partial sums of a leg are added at the end;
            //  cyclic: pair p = (o - 1) n3 + j on lane p mod 64 of round
            //   p / 64; each leg lane collects its terms from the round's
            //   slots by offset.
            const int S = n3 > 0 ? 64 / n3 : 1;
            const int ngrid = n3 * hh;
            const bool blocks = n3 > 0 && (hh + S - 1) / S <= (ngrid + 63) / 64;
            if (blocks) {
                const int sb = (int)(((float)lane + 0.5f) * rn3);  // lane / n3
                const int x = lane - sb * n3;
                const bool lane_in = sb < S;
                const int nr = (hh + S - 1) / S;
                for (int r = 0; r < nr; ++r) {
                    const int o = sb + 1 + r * S;
                    // second leg (x + o) mod n3; a block past the last offset
                    // has no pairs and maps every lane to its own slot
                    int k = x + (o <= hh ? o : 0);
                    if (k >= n3)
                        k -= n3;
                    T cj[3] = {T(0), T(0), T(0)}, ck[3] = {T(0), T(0), T(0)};
                    if (lane_in && o <= hh && !(even && o == hh && x >= hh))
                        leg_pair(x, k, cj, ck);
                    if (lane_in) {
                        gx += cj[0];
                        gy += cj[1];
                        gz += cj[2];
                        rb[(k + sb * n3) * 3 + 0] = ck[0];
                        rb[(k + sb * n3) * 3 + 1] = ck[1];
                        rb[(k + sb * n3) * 3 + 2] = ck[2];
                    }
                    wave_sync_lds_u();
                    if (lane_in) {
                        gx += rb[lane * 3 + 0];
                        gy += rb[lane * 3 + 1];
                        gz += rb[lane * 3 + 2];
                    }
                    wave_sync_lds_u();
                }
                // partial sums of leg x from the blocks s = 1..S-1
                if (lane_in) {
                    rb[lane * 3 + 0] = gx;
                    rb[lane * 3 + 1] = gy;
                    rb[lane * 3 + 2] = gz;
                }
                wave_sync_lds_u();
                if (lane < n3)
                    for (int s2 = 1; s2 < S; ++s2) {
                        gx += rb[(lane + s2 * n3) * 3 + 0];
                        gy += rb[(lane + s2 * n3) * 3 + 1];
                        gz += rb[(lane + s2 * n3) * 3 + 2];
                    }
                wave_sync_lds_u();
            } else {
                for (int t0 = 0; t0 < ngrid; t0 += 64) {
                    const int p = t0 + lane;
                    T cj[3] = {T(0), T(0), T(0)}, ck[3] = {T(0), T(0), T(0)};
                    if (p < ngrid) {
                        // o = p / n3 + 1 without an integer division (the float
                        // quotient of p + 1/2 sits at least 1/(2 n3) from an integer)
                        const int o = (int)(((float)p + 0.5f) * rn3) + 1;
                        const int j = p - (o - 1) * n3;
                        if (!(even && o == hh && j >= hh)) {
                            int k = j + o;
                            if (k >= n3)
                                k -= n3;
                            leg_pair(j, k, cj, ck);
                        }
                    }
                    rb[lane * 6 + 0] = cj[0];
                    rb[lane * 6 + 1] = cj[1];
                    rb[lane * 6 + 2] = cj[2];
                    rb[lane * 6 + 3] = ck[0];
                    rb[lane * 6 + 4] = ck[1];
                    rb[lane * 6 + 5] = ck[2];
                    wave_sync_lds_u();
                    if (lane < n3) {
                        const int x = lane;
                        for (int o = 1; o <= hh; ++o) {
                            // pair (x, x + o): x is the first leg
                            const int q1 = (o - 1) * n3 + x - t0;
                            if (!(even && o == hh && x >= hh) && q1 >= 0 && q1 < 64) {
                                gx += rb[q1 * 6 + 0];
                                gy += rb[q1 * 6 + 1];
                                gz += rb[q1 * 6 + 2];
                            }
                            // pair (x - o, x): x is the second leg
                            int jp = x - o;
                            if (jp < 0)
                                jp += n3;
                            const int q2 = (o - 1) * n3 + jp - t0;
                            if (!(even && o == hh && jp >= hh) && q2 >= 0 && q2 < 64) {
                                gx += rb[q2 * 6 + 3];
                                gy += rb[q2 * 6 + 4];
                                gz += rb[q2 * 6 + 5];
                            }
                        }
                    }
                    wave_sync_lds_u();
                }
            }
            // leg sums back to the lanes that own the legs' slots
            if (lane < n3) {
                rb[lane * 3 + 0] = gx;
                rb[lane * 3 + 1] = gy;
                rb[lane * 3 + 2] = gz;
            }
            wave_sync_lds_u();
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (leg[u] >= 0) {
                    hx[u] += rb[leg[u] * 3 + 0];
                    hy[u] += rb[leg[u] * 3 + 1];
                    hz[u] += rb[leg[u] * 3 + 2];
                }
        }
        T *ho = hout + (size_t)i * cap * 3;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int slot = lane + 64 * u;
            if (slot < c) {
                ho[slot * 3 + 0] = hx[u];
                ho[slot * 3 + 1] = hy[u];
                ho[slot * 3 + 2] = hz[u];
            }
        }
        T E = wave_sum_t(Ep);
        if (lane == 0)
            e_cheap[i] = (double)E;
    };
    if constexpr (!LOOP) {
        const int i = blockIdx.x * wpb + w;
        if (i < n)
            atom(i);
    } else {
        for (int grp = blockIdx.x; grp < (n + wpb - 1) / wpb; grp += gridDim.x) {
            const int i = grp * wpb + w;
            if (i < n)
                atom(i);
        }
    }
}

template <typename T>
static void uf3_t(hipStream_t s, const Ctx &c, void *ws, const WsLayout &L, const Box &b,
                  const double *pos, const int32_t *species, double *e_cheap, int side_blocks,
                  const uint8_t *mask_flags)
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
    const int c3n = uf3_c3_elems(m.ns, m.nb3);
    const size_t nT = kUf3WaveT;
    // eight waves per block on capped grids measured slower overall (the
    // kernel then crowds the expensive chain: 159-166 us against 152 us)
    const int wpb = 4;
    size_t sm = ((size_t)c3n + wpb * nT) * sizeof(T) + wpb * kMaxTriplet * sizeof(int) +
                (16 * ((size_t)(m.nk2 - 1) + (m.nb3 > 0 ? m.nk3 - 1 : 0)) +
                 (size_t)m.ns * m.ns * m.nb2) * sizeof(T) + 16;
    unsigned nblk = (L.n + wpb - 1) / wpb;
    if (side_blocks > 0 && nblk > (unsigned)side_blocks)
        nblk = side_blocks;
#define MLMIX_UF3_W(U, LOOP)                                                                     \
    (L.nseg > 0 ? k_uf3<T, U, LOOP, true> : k_uf3<T, U, LOOP, false>)<<<nblk, 256, sm, s>>>(     \
        pos, L.n, b, species, L.cap, at<int>(ws, L.nbr), at<int>(ws, L.cnt), a, at<T>(ws, L.h),    \
        e_cheap, at<int>(ws, L.hdr), mask_flags, seg_args(ws, L))
#define MLMIX_UF3(U)                                                                             \
    if (nblk < (unsigned)((L.n + wpb - 1) / wpb))                                                 \
        MLMIX_UF3_W(U, true);                                                                     \
    else                                                                                          \
        MLMIX_UF3_W(U, false)
    switch ((L.cap + 63) / 64) {
    case 1: MLMIX_UF3(1); break;
    case 2: MLMIX_UF3(2); break;
    case 3: MLMIX_UF3(3); break;
    default: MLMIX_UF3(4); break;
    }
#undef MLMIX_UF3
#undef MLMIX_UF3_W
}

void launch_uf3(hipStream_t s, const Ctx &c, void *ws, const WsLayout &L, const Box &b,
                const double *pos, const int32_t *species, double *e_cheap, int side_blocks,
                const uint8_t *mask_flags)
{
    if (L.n == 0)
        return;
    if (c.prec == MLMIX_FP64)
        uf3_t<double>(s, c, ws, L, b, pos, species, e_cheap, side_blocks, mask_flags);
    else
        uf3_t<float>(s, c, ws, L, b, pos, species, e_cheap, side_blocks, mask_flags);
}

}  // namespace mlmix
