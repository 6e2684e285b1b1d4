// Expensive ACE-style potential on the induced subsystem S (Algorithm 4 and
// Fig. 10: atoms outside S are removed from every neighbour list), on gfx950.
//
//  k_ace_basis    atomic basis A_i[a][lm] = sum_{j in S, r<rc} R_n(r) Y_lm(u)
//                 (one wavefront per S atom; per-neighbour R, Y staged in LDS;
//                 lanes own (channel, lm) accumulators, summed in row order)
//  k_ace_contract site energy and its adjoint dE/dA in one pass. The order-3
//                 readout is a symmetric cubic form E3 = sum_p A_p D_p with
//                 D_{c,l3,m3} = sum_{l1<=l2} sum_{ab} W[ab][c] P_{ab,m3},
//                 P_{ab,m3} = sum_{m1 m2} G A_{a l1 m1} A_{b l2 m2} (sparse
//                 Gaunt stage, LDS) and W the symmetrised coefficients (dense
//                 stage); dE3/dA = 3 D. Order 2 likewise: dE2/dA = 2 D2.
//  k_ace_pairgrad hand-written adjoint of the atomic basis: per pair,
//                 g_ij = dE_i/dd_ij = sum_{n,lm} dE/dA (R_n' u Y + R_n grad Y),
//                 recomputing R, Y and grad Y instead of storing them.
// Forces follow from g in the gather kernel: F_i = sum_j (g_ij - g_ji).
#include "internal.h"
#include "basis.h"

namespace mlmix {

template <typename T>
struct AceArgs {
    int ns, nrad, lmax, order, nchan, KA, L2, L1;
    T rc;
    double rc2;
    const T *K, *c0, *c1, *c2s, *W, *gval;
    const PBlock *pb;
    const int *gm3, *gidx;
    int pb_lo[kMaxLmax + 1], pb_hi[kMaxLmax + 1];
    int w_per_species;
};

__device__ __forceinline__ void pair_disp_d(const double *__restrict__ pos, int n, int i, int j,
                                            const Box &b, double d[3])
{
#pragma clang fp contract(off)
    for (int k = 0; k < 3; ++k) {
        double dx = pos[k * n + j] - pos[k * n + i];
        if (b.per[k]) {
            double h = 0.5 * b.L[k];
            if (dx > h)
                dx = dx - b.L[k];
            else if (dx < -h)
                dx = dx + b.L[k];
        }
        d[k] = dx;
    }
}

__device__ __forceinline__ double norm2_d(const double d[3])
{
#pragma clang fp contract(off)
    double s = d[0] * d[0];
    s = s + d[1] * d[1];
    s = s + d[2] * d[2];
    return s;
}

constexpr int kMaxOwn = 16;  // (channel, lm) entries per lane: KA <= 1024

template <typename T>
__global__ void __launch_bounds__(64)
    k_ace_basis(const double *__restrict__ pos, int n, Box b, const int32_t *__restrict__ species,
                int cap, const int *__restrict__ nbr, const int *__restrict__ cnt,
                const int *__restrict__ S_idx, const int *__restrict__ S_local,
                const int *__restrict__ hdr, AceArgs<T> a, T *__restrict__ A)
{
    int s = blockIdx.x;
    if (s >= hdr[H_NS])
        return;
    extern __shared__ char smem_raw[];
    T *Rt = reinterpret_cast<T *>(smem_raw);
    T *Yt = Rt + 64 * a.nrad;
    int *zt = reinterpret_cast<int *>(Yt + 64 * a.L2);
    int lane = threadIdx.x;
    int i = S_idx[s];
    int c = cnt[i];
    const int *row = nbr + (size_t)i * cap;
    T acc[kMaxOwn];
    int own_z[kMaxOwn], own_n[kMaxOwn], own_lm[kMaxOwn];
#pragma unroll
    for (int k = 0; k < kMaxOwn; ++k) {
        acc[k] = T(0);
        int e = lane + 64 * k;
        int ch = e / a.L2;
        own_lm[k] = e - ch * a.L2;
        own_z[k] = (e < a.KA) ? ch / a.nrad : -2;
        own_n[k] = ch % a.nrad;
    }
    for (int base = 0; base < c; base += 64) {
        int slot = base + lane;
        int zj = -1;
        if (slot < c) {
            int j = row[slot];
            if (S_local[j] >= 0) {
                double d[3];
                pair_disp_d(pos, n, i, j, b, d);
                double r2 = norm2_d(d);
                if (r2 < a.rc2) {
                    double rd = sqrt(r2);
                    T r = T(rd);
                    T ux = T(d[0] / rd), uy = T(d[1] / rd), uz = T(d[2] / rd);
                    T R[kMaxNrad], dR[kMaxNrad];
                    radial<T>(a.nrad, r, a.rc, R, dR);
#pragma unroll
                    for (int k = 0; k < kMaxNrad; ++k)
                        if (k < a.nrad)
                            Rt[lane * a.nrad + k] = R[k];
                    T *Yrow = Yt + lane * a.L2;
                    ylm_stream<T>(a.lmax, ux, uy, uz, a.K,
                                  [&](int lm, T Y, T, T, T) { Yrow[lm] = Y; });
                    zj = sp_clamp(species[j], a.ns);
                }
            }
        }
        zt[lane] = zj;
        __syncthreads();
        int m = c - base < 64 ? c - base : 64;
        for (int t = 0; t < m; ++t) {
            int z = zt[t];
            if (z < 0)
                continue;
#pragma unroll
            for (int k = 0; k < kMaxOwn; ++k)
                if (own_z[k] == z)
                    acc[k] += Rt[t * a.nrad + own_n[k]] * Yt[t * a.L2 + own_lm[k]];
        }
        __syncthreads();
    }
    T *As = A + (size_t)s * a.KA;
#pragma unroll
    for (int k = 0; k < kMaxOwn; ++k) {
        int e = lane + 64 * k;
        if (e < a.KA)
            As[e] = acc[k];
    }
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int d = 32; d > 0; d >>= 1)
        v += __shfl_xor(v, d);
    return v;
}

constexpr int kMaxOut = 8;  // order-3 outputs (c, m3) per lane

template <typename T>
__global__ void __launch_bounds__(64)
    k_ace_contract(const int32_t *__restrict__ species, const int *__restrict__ S_idx,
                   const int *__restrict__ hdr, AceArgs<T> a, const T *__restrict__ A,
                   T *__restrict__ dEdA, double *__restrict__ e_exp)
{
    int s = blockIdx.x;
    if (s >= hdr[H_NS])
        return;
    extern __shared__ char smem_raw[];
    T *As = reinterpret_cast<T *>(smem_raw);
    T *dAs = As + a.KA;
    T *Ps = dAs + a.KA;
    int lane = threadIdx.x;
    int i = S_idx[s];
    int z = sp_clamp(species[i], a.ns);
    const int nch = a.nchan, L2 = a.L2;
    for (int e = lane; e < a.KA; e += 64) {
        As[e] = A[(size_t)s * a.KA + e];
        dAs[e] = T(0);
    }
    __syncthreads();
    T Ep = T(0);
    // order 1: E1 = sum_a c1_a A_{a,00}
    for (int ch = lane; ch < nch; ch += 64) {
        T c = a.c1[z * nch + ch];
        dAs[ch * L2] += c;
        Ep += c * As[ch * L2];
    }
    __syncthreads();
    // order 2: D2_{a,lm} = sum_b C2_{ab,l} A_{b,lm}; E2 = A.D2; dE2/dA = 2 D2
    if (a.order >= 2) {
        for (int e = lane; e < a.KA; e += 64) {
            int ch = e / L2, lm = e - ch * L2;
            int l = 0;
            while ((l + 1) * (l + 1) <= lm)
                ++l;
            const T *C = a.c2s + (((size_t)z * a.L1 + l) * nch + ch) * nch;
            T D = T(0);
            for (int bb = 0; bb < nch; ++bb)
                D += C[bb] * As[bb * L2 + lm];
            dAs[e] += T(2) * D;
            Ep += As[e] * D;
        }
    }
    __syncthreads();
    if (a.order >= 3) {
        const T *Wz = a.W + (size_t)z * a.w_per_species;
        const int nab = nch * nch;
        for (int l3 = 0; l3 <= a.lmax; ++l3) {
            if (a.pb_lo[l3] >= a.pb_hi[l3])
                continue;
            const int d3 = 2 * l3 + 1;
            const int nout = nch * d3;
            T acc[kMaxOut];
#pragma unroll
            for (int k = 0; k < kMaxOut; ++k)
                acc[k] = T(0);
            for (int p = a.pb_lo[l3]; p < a.pb_hi[l3]; ++p) {
                const PBlock pb = a.pb[p];
                const int o1 = pb.l1 * pb.l1, o2 = pb.l2 * pb.l2;
                // sparse Gaunt stage: P_{ab,m3}
                for (int ab = lane; ab < nab; ab += 64) {
                    int aa = ab / nch, bb = ab - aa * nch;
                    const T *Aa = As + aa * L2 + o1;
                    const T *Ab = As + bb * L2 + o2;
                    for (int m3 = 0; m3 < d3; ++m3) {
                        int e0 = a.gm3[pb.gm3_off + m3], e1 = a.gm3[pb.gm3_off + m3 + 1];
                        T pv = T(0);
                        for (int e = e0; e < e1; ++e) {
                            int mm = a.gidx[e];
                            pv += a.gval[e] * Aa[mm & 0xff] * Ab[mm >> 8];
                        }
                        Ps[ab * d3 + m3] = pv;
                    }
                }
                __syncthreads();
                // dense stage: D_{c,m3} += sum_ab W[ab][c] P_{ab,m3}
                const T *Wb = Wz + pb.w_off;
#pragma unroll
                for (int k = 0; k < kMaxOut; ++k) {
                    int o = lane + 64 * k;
                    if (o < nout) {
                        int cc = o / d3, m3 = o - cc * d3;
                        T sacc = acc[k];
                        for (int ab = 0; ab < nab; ++ab)
                            sacc += Wb[(size_t)ab * nch + cc] * Ps[ab * d3 + m3];
                        acc[k] = sacc;
                    }
                }
                __syncthreads();
            }
#pragma unroll
            for (int k = 0; k < kMaxOut; ++k) {
                int o = lane + 64 * k;
                if (o < nout) {
                    int cc = o / d3, m3 = o - cc * d3;
                    int idx = cc * L2 + l3 * l3 + m3;
                    dAs[idx] += T(3) * acc[k];
                    Ep += As[idx] * acc[k];
                }
            }
            __syncthreads();
        }
    }
    T E = wave_sum(Ep);
    if (lane == 0)
        e_exp[i] = (double)a.c0[z] + (double)E;
    for (int e = lane; e < a.KA; e += 64)
        dEdA[(size_t)s * a.KA + e] = dAs[e];
}

template <typename T>
__global__ void __launch_bounds__(64)
    k_ace_pairgrad(const double *__restrict__ pos, int n, Box b, const int32_t *__restrict__ species,
                   int cap, const int *__restrict__ nbr, const int *__restrict__ cnt,
                   const int *__restrict__ S_idx, const int *__restrict__ S_local,
                   const int *__restrict__ hdr, AceArgs<T> a, const T *__restrict__ dEdA,
                   const double *__restrict__ weights, T *__restrict__ g)
{
    int s = blockIdx.x;
    if (s >= hdr[H_NS])
        return;
    extern __shared__ char smem_raw[];
    T *dAs = reinterpret_cast<T *>(smem_raw);
    int lane = threadIdx.x;
    int i = S_idx[s];
    T w = weights ? T(weights[i]) : T(1);
    for (int e = lane; e < a.KA; e += 64)
        dAs[e] = dEdA[(size_t)s * a.KA + e] * w;
    __syncthreads();
    int c = cnt[i];
    const int *row = nbr + (size_t)i * cap;
    T *gs = g + (size_t)s * cap * 3;
    for (int base = 0; base < c; base += 64) {
        int slot = base + lane;
        if (slot >= c)
            continue;
        int j = row[slot];
        T gx = T(0), gy = T(0), gz = T(0);
        if (S_local[j] >= 0) {
            double d[3];
            pair_disp_d(pos, n, i, j, b, d);
            double r2 = norm2_d(d);
            if (r2 < a.rc2) {
                double rd = sqrt(r2);
                T r = T(rd);
                T ux = T(d[0] / rd), uy = T(d[1] / rd), uz = T(d[2] / rd);
                T R[kMaxNrad], dR[kMaxNrad];
                radial<T>(a.nrad, r, a.rc, R, dR);
                const T *col = dAs + sp_clamp(species[j], a.ns) * a.nrad * a.L2;
                T rad = T(0), vx = T(0), vy = T(0), vz = T(0);
                const int L2 = a.L2, nrad = a.nrad;
                ylm_stream<T>(a.lmax, ux, uy, uz, a.K, [&](int lm, T Y, T yx, T yy, T yz) {
                    T sR = T(0), sD = T(0);
#pragma unroll
                    for (int k = 0; k < kMaxNrad; ++k)
                        if (k < nrad) {
                            T v = col[k * L2 + lm];
                            sR += v * R[k];
                            sD += v * dR[k];
                        }
                    rad += sD * Y;
                    vx += sR * yx;
                    vy += sR * yy;
                    vz += sR * yz;
                });
                // grad of Y(d/|d|) w.r.t. d is (I - u u^T) grad_u Y / r
                T ud = ux * vx + uy * vy + uz * vz;
                T ir = T(1) / r;
                gx = rad * ux + (vx - ux * ud) * ir;
                gy = rad * uy + (vy - uy * ud) * ir;
                gz = rad * uz + (vz - uz * ud) * ir;
            }
        }
        gs[slot * 3 + 0] = gx;
        gs[slot * 3 + 1] = gy;
        gs[slot * 3 + 2] = gz;
    }
}

template <typename T>
static AceArgs<T> make_args(const Ctx &c)
{
    const DevModel &m = c.m;
    AceArgs<T> a;
    a.ns = m.ns;
    a.nrad = m.nrad;
    a.lmax = m.lmax;
    a.order = m.order;
    a.nchan = m.nchan;
    a.KA = m.KA;
    a.L2 = m.L2;
    a.L1 = m.lmax + 1;
    a.rc = T(m.rc_exp);
    a.rc2 = m.rc_exp * m.rc_exp;
    char *base = static_cast<char *>(m.base);
    a.K = reinterpret_cast<const T *>(base + m.ylmK);
    a.c0 = reinterpret_cast<const T *>(base + m.c0);
    a.c1 = reinterpret_cast<const T *>(base + m.c1);
    a.c2s = reinterpret_cast<const T *>(base + m.c2s);
    a.W = reinterpret_cast<const T *>(base + m.W);
    a.gval = reinterpret_cast<const T *>(base + m.gval);
    a.pb = reinterpret_cast<const PBlock *>(base + m.pb);
    a.gm3 = reinterpret_cast<const int *>(base + m.gm3);
    a.gidx = reinterpret_cast<const int *>(base + m.gidx);
    a.w_per_species = m.w_per_species;
    return a;
}

// pb_lo / pb_hi are filled by the host from the block list (sorted by l3).
extern void pb_ranges(const Ctx &c, int *lo, int *hi);

template <typename T>
static void forward_t(hipStream_t s, const Ctx &c, void *ws, const WsLayout &L, const Box &b,
                      const double *pos, const int32_t *species, double *e_exp)
{
    AceArgs<T> a = make_args<T>(c);
    pb_ranges(c, a.pb_lo, a.pb_hi);
    int n = L.n;
    const int *hdr = at<int>(ws, L.hdr);
    size_t sm_basis = (size_t)64 * (a.nrad + a.L2) * sizeof(T) + 64 * sizeof(int);
    k_ace_basis<T><<<n, 64, sm_basis, s>>>(pos, n, b, species, L.cap, at<int>(ws, L.nbr),
                                           at<int>(ws, L.cnt), at<int>(ws, L.S_idx),
                                           at<int>(ws, L.S_local), hdr, a, at<T>(ws, L.A));
    size_t sm_c = (size_t)(2 * a.KA + a.nchan * a.nchan * (2 * a.lmax + 1)) * sizeof(T);
    k_ace_contract<T><<<n, 64, sm_c, s>>>(species, at<int>(ws, L.S_idx), hdr, a, at<T>(ws, L.A),
                                          at<T>(ws, L.dEdA), e_exp);
}

template <typename T>
static void pairgrad_t(hipStream_t s, const Ctx &c, void *ws, const WsLayout &L, const Box &b,
                       const double *pos, const int32_t *species, const double *weights)
{
    AceArgs<T> a = make_args<T>(c);
    int n = L.n;
    size_t sm = (size_t)a.KA * sizeof(T);
    k_ace_pairgrad<T><<<n, 64, sm, s>>>(pos, n, b, species, L.cap, at<int>(ws, L.nbr),
                                        at<int>(ws, L.cnt), at<int>(ws, L.S_idx),
                                        at<int>(ws, L.S_local), at<int>(ws, L.hdr), a,
                                        at<T>(ws, L.dEdA), weights, at<T>(ws, L.g));
}

void launch_ace_forward(hipStream_t s, const Ctx &c, void *ws, const WsLayout &L, const Box &b,
                        const double *pos, const int32_t *species, double *e_exp)
{
    if (L.n == 0)
        return;
    if (c.prec == MLMIX_FP64)
        forward_t<double>(s, c, ws, L, b, pos, species, e_exp);
    else
        forward_t<float>(s, c, ws, L, b, pos, species, e_exp);
}

void launch_ace_pairgrad(hipStream_t s, const Ctx &c, void *ws, const WsLayout &L, const Box &b,
                         const double *pos, const int32_t *species, const double *weights)
{
    if (L.n == 0)
        return;
    if (c.prec == MLMIX_FP64)
        pairgrad_t<double>(s, c, ws, L, b, pos, species, weights);
    else
        pairgrad_t<float>(s, c, ws, L, b, pos, species, weights);
}

}  // namespace mlmix
