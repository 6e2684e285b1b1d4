// Force gather + blend (Algorithm 4), FP64 energy sums and the FP64
// velocity-Verlet kernels, on gfx950.
//
// Gather: with g_ij = dE_i/dd_ij stored per (centre, row slot), the force is
// F_i = sum_j (g_ij - g_ji), where g_ji sits in j's row at the reverse slot.
// Sixteen lanes per atom (a DPP row: lanes over row slots, then a fixed-order
// sum within the row), four atoms per wavefront: no atomics, so repeated
// runs and replicas evaluated alone or in a batch give the same bits. The
// blend F = lambda F_exp + (1 - lambda) F_cheap is fused into the same pass.
#include <hip/hip_ext.h>

#include "internal.h"
#include "reduce.h"

namespace mlmix {

template <typename T>
struct TypeTag {
    using type = T;
};

// 64-bit value moved by a DPP lane pattern (two 32-bit moves)
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over the 16 lanes of a DPP row in a fixed order (pairs, quads, halves,
// rows); every lane of the row receives the same bits.
__device__ __forceinline__ double row16_sum_d(double v)
{
    v += dpp_d<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_d<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_d<0x141>(v);  // row_half_mirror
    v += dpp_d<0x140>(v);  // row_mirror
    return v;
}

template <typename T, bool KICK, bool SEG>
__global__ void __launch_bounds__(256)
    k_gather_blend(int n, int cap, const int *__restrict__ nbr, const int *__restrict__ cnt,
                   const int *__restrict__ rev, const int *__restrict__ S_local,
                   const T *__restrict__ g, const T *__restrict__ h, int use_exp, int use_cheap,
                   const double *__restrict__ lambda, double *__restrict__ forces,
                   double *__restrict__ e_exp, double *__restrict__ f_exp,
                   double *__restrict__ f_cheap, double sign, KickArgs ka, LangevinArgs la,
                   Seg sg)
{
    // workgroup vb takes atoms 16 vb ...; the workgroups are numbered XCD by
    // XCD (the grid is padded to a multiple of 8), so each XCD takes a
    // contiguous range of atoms and the partner rows around it stay in its
    // L2
    const int nbk = (n + kGatherAtoms - 1) / kGatherAtoms;
    const int vb = xcd_major(blockIdx.x, gridDim.x);
    if (vb >= nbk)
        return;  // uniform across the workgroup (padding)
    const int ga = threadIdx.x >> 4;  // atom of the workgroup
    const int i = vb * kGatherAtoms + ga;
    const int lane = threadIdx.x & 15;  // slot lane within the atom's row
    double ee = 0.0, ec = 0.0, ke = 0.0;  // energy terms of atom i (lane 0, KICK)
    if (i < n) {
        int c = cnt[i];
        int si = S_local[i];
        double fe0 = 0.0, fe1 = 0.0, fe2 = 0.0, fc0 = 0.0, fc1 = 0.0, fc2 = 0.0;
        const size_t rowo = (size_t)i * cap;
        for (int slot = lane; slot < c; slot += 16) {
            int j = nbr[rowo + slot];
            int r = rev[rowo + slot];
            if (r < 0)
                continue;
            if (use_exp && si >= 0) {
                int sj = S_local[j];
                if (sj >= 0) {
                    const T *a = g + ((size_t)si * cap + slot) * 3;
                    const T *bb = g + ((size_t)sj * cap + r) * 3;
                    fe0 += (double)a[0] - (double)bb[0];
                    fe1 += (double)a[1] - (double)bb[1];
                    fe2 += (double)a[2] - (double)bb[2];
                }
            }
            if (use_cheap) {
                const T *a = h + (rowo + slot) * 3;
                const T *bb = h + ((size_t)j * cap + r) * 3;
                fc0 += (double)a[0] - (double)bb[0];
                fc1 += (double)a[1] - (double)bb[1];
                fc2 += (double)a[2] - (double)bb[2];
            }
        }
        fe0 = row16_sum_d(fe0);
        fe1 = row16_sum_d(fe1);
        fe2 = row16_sum_d(fe2);
        fc0 = row16_sum_d(fc0);
        fc1 = row16_sum_d(fc1);
        fc2 = row16_sum_d(fc2);
        if (lane == 0) {
            double lam = lambda ? lambda[i] : 1.0;
            double om = 1.0 - lam;
            double F[3] = {sign * (lam * fe0 + om * fc0), sign * (lam * fe1 + om * fc1),
                           sign * (lam * fe2 + om * fc2)};
            if (la.xi && lam == 0.0) {
                // Langevin friction and noise on the cheap region
                const double m = la.mass[i];
                const double g = -m * la.c_fric, sg = sqrt(m * la.c_rand);
                for (int q = 0; q < 3; ++q)
                    F[q] = F[q] + (g * la.vel[q * n + i] + sg * la.xi[q * n + i]);
            }
            if (forces) {
                forces[i] = F[0];
                forces[n + i] = F[1];
                forces[2 * n + i] = F[2];
            }
            if (f_exp) {
                f_exp[i] = fe0;
                f_exp[n + i] = fe1;
                f_exp[2 * n + i] = fe2;
            }
            if (f_cheap) {
                f_cheap[i] = fc0;
                f_cheap[n + i] = fc1;
                f_cheap[2 * n + i] = fc2;
            }
            if (e_exp && si < 0)
                e_exp[i] = 0.0;
            if (KICK) {
                const double m = ka.mass[i];
                const double cf = 0.5 * ka.dt * kKappa / m;
                double v2 = 0.0;
                double xn[3];
                // (per lane: a wavefront holds four atoms, maybe of two systems)
                const Box bx = seg_box<SEG>(ka.box, sg, i);
                for (int q = 0; q < 3; ++q) {
                    // kicks and drifts as explicit fused multiply-adds, the same
                    // in every kernel that applies them (so fused and separate
                    // steps give the same bits)
                    const double v = fma(cf, F[q], ka.vel[q * n + i]);
                    v2 += v * v;
                    if (ka.next) {
                        // the next step's opening half kick and drift, as
                        // k_vv computes them
                        const double vn = fma(cf, F[q], v);
                        ka.vel[q * n + i] = vn;
                        double x = fma(ka.dt, vn, ka.pos[q * n + i]);
                        if (bx.per[q]) {
                            x = x - bx.L[q] * floor(x / bx.L[q]);
                            if (x >= bx.L[q])
                                x -= bx.L[q];
                        }
                        ka.pos[q * n + i] = x;
                        xn[q] = x;
                    } else {
                        ka.vel[q * n + i] = v;
                    }
                }
                if (ka.next && ka.chk.hdr)
                    disp_check<SEG>(ka.chk, xn, n, i, bx);
                ke = 0.5 * m * v2;
                ee = si < 0 ? 0.0 : e_exp[i];
                ec = ka.e_cheap[i];
                if (ka.ke_atom)
                    ka.ke_atom[i] = ke;
            }
        }
    }
    if (KICK && ka.part) {
        // block partial; k_reduce_final sums the partials in a fixed order
        // (a last-block-done reduction in this kernel measured 61 us against
        // 12 + 4 us on 8,193 atoms: the per-block device-scope fences)
        __shared__ double sh[3][kGatherAtoms];
        if (lane == 0) {
            sh[0][ga] = ee;
            sh[1][ga] = ec;
            sh[2][ga] = ke;
        }
        __syncthreads();
        if (threadIdx.x < 3) {
            const int q = threadIdx.x;
            double v[kGatherAtoms];
            for (int k = 0; k < kGatherAtoms; ++k)
                v[k] = sh[q][k];
            for (int w = kGatherAtoms / 2; w > 0; w >>= 1)  // pairwise, fixed order
                for (int k = 0; k < w; ++k)
                    v[k] = v[k] + v[k + w];
            ka.part[vb * 3 + q] = v[0];
        }
    }
}

__global__ void __launch_bounds__(256) k_reduce_final(const double *__restrict__ part, int nb,
                                                      double *__restrict__ out);

void launch_gather_blend(hipStream_t s, const Ctx &c, void *ws, const WsLayout &L, int use_exp,
                         int use_cheap, const double *lambda, double *forces, double *e_exp,
                         double *f_exp, double *f_cheap, double sign, const KickArgs *kick,
                         const LangevinArgs *lang, hipEvent_t ev0, hipEvent_t ev1)
{
    int n = L.n;
    if (n == 0)
        return;
    unsigned nb = (n + kGatherAtoms - 1) / kGatherAtoms;
    const unsigned grid = (nb + 7) / 8 * 8;
    LangevinArgs la{};
    if (lang)
        la = *lang;
    KickArgs ka{};
    if (kick) {
        ka = *kick;
        // a batch sums its energies per system in k_seg_sums instead
        ka.part = L.nseg == 0 ? at<double>(ws, L.red) : nullptr;
    }
    // ev0 / ev1: the kernel's own start and end (stage timing)
    auto go = [&](auto kern, auto tc) {
        using T = typename decltype(tc)::type;
        if (ev0)
            hipExtLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, s, ev0, ev1, 0u, n, L.cap,
                                  at<int>(ws, L.nbr), at<int>(ws, L.cnt), at<int>(ws, L.rev),
                                  at<int>(ws, L.S_local), at<T>(ws, L.g), at<T>(ws, L.h), use_exp,
                                  use_cheap, lambda, forces, e_exp, f_exp, f_cheap, sign, ka, la,
                                  seg_args(ws, L));
        else
            kern<<<grid, 256, 0, s>>>(n, L.cap, at<int>(ws, L.nbr), at<int>(ws, L.cnt),
                                    at<int>(ws, L.rev), at<int>(ws, L.S_local), at<T>(ws, L.g),
                                    at<T>(ws, L.h), use_exp, use_cheap, lambda, forces, e_exp,
                                    f_exp, f_cheap, sign, ka, la, seg_args(ws, L));
    };
    auto by_kick = [&](auto tc) {
        using T = typename decltype(tc)::type;
        if (kick)
            go(L.nseg > 0 ? k_gather_blend<T, true, true> : k_gather_blend<T, true, false>, tc);
        else
            go(L.nseg > 0 ? k_gather_blend<T, false, true> : k_gather_blend<T, false, false>, tc);
    };
    if (c.prec == MLMIX_FP64)
        by_kick(TypeTag<double>());
    else
        by_kick(TypeTag<float>());
    if (kick && !ka.defer && ka.part)
        k_reduce_final<<<1, 256, 0, s>>>(ka.part, (int)nb, ka.energies);
}

__global__ void __launch_bounds__(256) k_fill_f64(double *p, double v, size_t n)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = v;
}

void launch_fill_f64(hipStream_t s, double *p, double v, size_t n)
{
    if (n == 0)
        return;
    k_fill_f64<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, v, n);
}

__global__ void __launch_bounds__(256) k_copy_i32(int32_t *dst, const int32_t *src, size_t n)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        dst[i] = src[i];
}

void launch_copy_i32(hipStream_t s, int32_t *dst, const int32_t *src, size_t n)
{
    if (n == 0)
        return;
    k_copy_i32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(dst, src, n);
}

// ------------------------------------------------------------ reductions

__global__ void __launch_bounds__(256)
    k_reduce_partial(int n, const double *__restrict__ e_exp, const double *__restrict__ e_cheap,
                     const double *__restrict__ vel, const double *__restrict__ mass,
                     double *__restrict__ part)
{
    __shared__ double sh[3][4];
    double a = 0.0, bsum = 0.0, k = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        if (e_exp)
            a += e_exp[i];
        if (e_cheap)
            bsum += e_cheap[i];
        if (vel && mass) {
            double v2 = vel[i] * vel[i] + vel[n + i] * vel[n + i] + vel[2 * n + i] * vel[2 * n + i];
            k += 0.5 * mass[i] * v2;
        }
    }
    a = wave_sum_d(a);
    bsum = wave_sum_d(bsum);
    k = wave_sum_d(k);
    int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[0][w] = a;
        sh[1][w] = bsum;
        sh[2][w] = k;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 0; q < 3; ++q)
            part[blockIdx.x * 3 + q] = (sh[q][0] + sh[q][1]) + (sh[q][2] + sh[q][3]);
    }
}

__global__ void __launch_bounds__(256) k_reduce_final(const double *__restrict__ part, int nb,
                                                      double *__restrict__ out)
{
    reduce_parts(part, nb, out);
}

void launch_reduce(hipStream_t s, void *ws, const WsLayout &L, const double *e_exp,
                   const double *e_cheap, const double *vel, const double *mass, double *out)
{
    double *part = at<double>(ws, L.red);
    int nb = (L.n + 255) / 256;
    if (nb > kReduceBlocks)
        nb = kReduceBlocks;
    if (nb < 1)
        nb = 1;
    k_reduce_partial<<<nb, 256, 0, s>>>(L.n, e_exp, e_cheap, vel, mass, part);
    k_reduce_final<<<1, 256, 0, s>>>(part, nb, out);
}

// -------------------------------------------------------- velocity Verlet

template <bool SEG>
__global__ void __launch_bounds__(256) k_vv(int n, Box b0, double *__restrict__ pos,
                                            double *__restrict__ vel,
                                            const double *__restrict__ mass,
                                            const double *__restrict__ f, double dt, int drift,
                                            Seg sg, DispCheck chk)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const Box b = seg_box<SEG>(b0, sg, i);
    double c = 0.5 * dt * kKappa / mass[i];
    double xn[3];
    for (int k = 0; k < 3; ++k) {
        double v = fma(c, f[k * n + i], vel[k * n + i]);
        vel[k * n + i] = v;
        if (drift) {
            double x = fma(dt, v, pos[k * n + i]);
            if (b.per[k]) {
                x = x - b.L[k] * floor(x / b.L[k]);
                if (x >= b.L[k])
                    x -= b.L[k];
            }
            pos[k * n + i] = x;
            xn[k] = x;
        }
    }
    if (drift && chk.hdr)
        disp_check<SEG>(chk, xn, n, i, b);
}

// Closing half kick of a step fused with the per-block energy partials
// (same grid-stride partition and block reduction as k_reduce_partial; the
// kinetic energy uses the kicked velocities).
__global__ void __launch_bounds__(256) k_vv_kick_sums(int n, double *__restrict__ vel,
                                                      const double *__restrict__ mass,
                                                      const double *__restrict__ f, double dt,
                                                      const double *__restrict__ e_exp,
                                                      const double *__restrict__ e_cheap,
                                                      double *__restrict__ part)
{
    __shared__ double sh[3][4];
    double a = 0.0, bsum = 0.0, k = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double c = 0.5 * dt * kKappa / mass[i];
        double v2 = 0.0;
        for (int q = 0; q < 3; ++q) {
            const double v = fma(c, f[q * n + i], vel[q * n + i]);
            vel[q * n + i] = v;
            v2 += v * v;
        }
        a += e_exp[i];
        bsum += e_cheap[i];
        k += 0.5 * mass[i] * v2;
    }
    a = wave_sum_d(a);
    bsum = wave_sum_d(bsum);
    k = wave_sum_d(k);
    int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[0][w] = a;
        sh[1][w] = bsum;
        sh[2][w] = k;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 0; q < 3; ++q)
            part[blockIdx.x * 3 + q] = (sh[q][0] + sh[q][1]) + (sh[q][2] + sh[q][3]);
    }
}

void launch_vv_kick_sums(hipStream_t s, void *ws, const WsLayout &L, double *vel,
                         const double *mass, const double *forces, double dt, const double *e_exp,
                         const double *e_cheap, double *out)
{
    if (L.n == 0) {
        launch_reduce(s, ws, L, e_exp, e_cheap, vel, mass, out);
        return;
    }
    double *part = at<double>(ws, L.red);
    int nb = (L.n + 255) / 256;
    if (nb > kReduceBlocks)
        nb = kReduceBlocks;
    k_vv_kick_sums<<<nb, 256, 0, s>>>(L.n, vel, mass, forces, dt, e_exp, e_cheap, part);
    k_reduce_final<<<1, 256, 0, s>>>(part, nb, out);
}

void launch_vv_kick_drift(hipStream_t s, void *ws, const WsLayout &L, const Box &b, double *pos,
                          double *vel, const double *mass, const double *forces, double dt,
                          int drift, const DispCheck *chk)
{
    if (L.n == 0)
        return;
    const DispCheck dc = chk ? *chk : DispCheck{nullptr, 0.0, nullptr, nullptr, nullptr};
    (L.nseg > 0 ? k_vv<true> : k_vv<false>)<<<(L.n + 255) / 256, 256, 0, s>>>(
        L.n, b, pos, vel, mass, forces, dt, drift, seg_args(ws, L), dc);
}

// ------------------------------------------------------ batched systems

// Segment index of every atom of a batch: one workgroup per segment.
__global__ void __launch_bounds__(256) k_seg_fill(const SegGeo *__restrict__ geo,
                                                  int *__restrict__ seg_of)
{
    const SegGeo G = geo[blockIdx.x];
    for (int t = threadIdx.x; t < G.n; t += blockDim.x)
        seg_of[G.off + t] = (int)blockIdx.x;
}

void launch_seg_fill(hipStream_t s, void *ws, const WsLayout &L)
{
    if (L.nseg > 0)
        k_seg_fill<<<L.nseg, 256, 0, s>>>(at<SegGeo>(ws, L.segs), at<int>(ws, L.seg_of));
}

// List state of the systems a new batch keeps from an old one: one
// workgroup per new segment, skipped for a segment new to the batch. A kept
// system's rows hold its atoms' batch indices, which move by the difference
// of its offsets; padding (-1) stays.
__global__ void __launch_bounds__(256) k_carry_lists(
    const SegGeo *__restrict__ geo_n, const int *__restrict__ map, int n_new, int cap,
    int *__restrict__ nbr_n, int *__restrict__ cnt_n, int *__restrict__ rev_n,
    double *__restrict__ ref_n, int *__restrict__ flag_n, const SegGeo *__restrict__ geo_o,
    int n_old, const int *__restrict__ nbr_o, const int *__restrict__ cnt_o,
    const int *__restrict__ rev_o, const double *__restrict__ ref_o,
    const int *__restrict__ flag_o)
{
    const int k = blockIdx.x;
    const int ko = map[k];
    if (ko < 0)
        return;  // uniform: a system new to the batch builds its list
    const SegGeo Gn = geo_n[k], Go = geo_o[ko];
    const int shift = Gn.off - Go.off;
    const size_t rows = (size_t)Gn.n * cap;
    for (size_t t = threadIdx.x; t < rows; t += blockDim.x) {
        const int v = nbr_o[(size_t)Go.off * cap + t];
        nbr_n[(size_t)Gn.off * cap + t] = v >= 0 ? v + shift : v;
        rev_n[(size_t)Gn.off * cap + t] = rev_o[(size_t)Go.off * cap + t];
    }
    for (int t = threadIdx.x; t < Gn.n; t += blockDim.x) {
        cnt_n[Gn.off + t] = cnt_o[Go.off + t];
        for (int q = 0; q < 3; ++q)
            ref_n[(size_t)q * n_new + Gn.off + t] = ref_o[(size_t)q * n_old + Go.off + t];
    }
    if (threadIdx.x == 0) {
        flag_n[4 * k + kSegMoved] = flag_o[4 * ko + kSegMoved];
        flag_n[4 * k + kSegBuilt] = flag_o[4 * ko + kSegBuilt];
    }
}

void launch_carry_lists(hipStream_t s, void *ws_new, const WsLayout &Ln, const void *ws_old,
                        const WsLayout &Lo)
{
    if (Ln.nseg == 0)
        return;
    void *wo = const_cast<void *>(ws_old);
    k_carry_lists<<<Ln.nseg, 256, 0, s>>>(
        at<SegGeo>(ws_new, Ln.segs), at<int>(ws_new, Ln.seg_map), Ln.n, Ln.cap,
        at<int>(ws_new, Ln.nbr), at<int>(ws_new, Ln.cnt), at<int>(ws_new, Ln.rev),
        at<double>(ws_new, Ln.ref_pos), at<int>(ws_new, Ln.seg_flag), at<SegGeo>(wo, Lo.segs), Lo.n,
        at<int>(wo, Lo.nbr), at<int>(wo, Lo.cnt), at<int>(wo, Lo.rev), at<double>(wo, Lo.ref_pos),
        at<int>(wo, Lo.seg_flag));
}

// Energy sums and set sizes of every system of a batch: one workgroup per
// segment; thread t sums the segment's atoms t, t + 256, ... (counted from
// the segment's first atom), then the wave butterfly and the four waves in
// a fixed order, so a system's sums have the same bits wherever it sits in
// whichever batch. out[3 k + q] = (sum e_exp, sum e_cheap, kinetic in eV) of
// segment k (kinetic from the per-atom 0.5 m v^2 the force gather left in
// ke, or 0 without it); counts[2 k] = (|S|, |{lambda > 0}|) from the flags.
__global__ void __launch_bounds__(256) k_seg_sums(const SegGeo *__restrict__ geo,
                                                  const double *__restrict__ e_exp,
                                                  const double *__restrict__ e_cheap,
                                                  const double *__restrict__ ke,
                                                  const uint8_t *__restrict__ flags,
                                                  double *__restrict__ out,
                                                  int32_t *__restrict__ counts)
{
    __shared__ double sh[3][4];
    __shared__ int shc[2][4];
    const SegGeo G = geo[blockIdx.x];
    double a = 0.0, b = 0.0, k = 0.0;
    int cs = 0, cm = 0;
    for (int t = threadIdx.x; t < G.n; t += blockDim.x) {
        const int i = G.off + t;
        a += e_exp[i];
        b += e_cheap[i];
        if (ke)
            k += ke[i];
        const uint8_t f = flags[i];
        cs += (f & 5) ? 1 : 0;
        cm += (f & 1) ? 1 : 0;
    }
    a = wave_sum_d(a);
    b = wave_sum_d(b);
    k = wave_sum_d(k);
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        cs += __shfl_xor(cs, d);
        cm += __shfl_xor(cm, d);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[0][w] = a;
        sh[1][w] = b;
        sh[2][w] = k;
        shc[0][w] = cs;
        shc[1][w] = cm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (out) {
            for (int q = 0; q < 3; ++q)
                out[3 * blockIdx.x + q] = (sh[q][0] + sh[q][1]) + (sh[q][2] + sh[q][3]);
            out[3 * blockIdx.x + 2] /= kKappa;
        }
        if (counts) {
            counts[2 * blockIdx.x] = (shc[0][0] + shc[0][1]) + (shc[0][2] + shc[0][3]);
            counts[2 * blockIdx.x + 1] = (shc[1][0] + shc[1][1]) + (shc[1][2] + shc[1][3]);
        }
    }
}

void launch_seg_sums(hipStream_t s, void *ws, const WsLayout &L, const double *e_exp,
                     const double *e_cheap, const double *ke, const uint8_t *flags, double *out,
                     int32_t *counts)
{
    if (L.nseg > 0)
        k_seg_sums<<<L.nseg, 256, 0, s>>>(at<SegGeo>(ws, L.segs), e_exp, e_cheap, ke, flags, out,
                                          counts);
}

// ------------------------------------------------------------ peak probe

// Matrix-core FP32 throughput: every wave runs `iters` rounds of eight
// independent 16x16x4 MFMA chains on register operands (no memory traffic)
// and stores one value so that the work is kept.
__global__ void __launch_bounds__(256) k_probe_mfma_f32(int iters, float *sink)
{
    typedef float f4 __attribute__((ext_vector_type(4)));
    const int lane = threadIdx.x & 63;
    const float a = 1.0f + 1e-7f * (float)lane, b = 1.0f - 1e-7f * (float)threadIdx.x;
    f4 c[8];
    for (int k = 0; k < 8; ++k)
        c[k] = (f4){0.f, 0.f, 0.f, 0.f};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 8; ++k)
            c[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c[k], 0, 0, 0);
    }
    float s = 0.f;
    for (int k = 0; k < 8; ++k)
        s += c[k][0] + c[k][1] + c[k][2] + c[k][3];
    if (s == -1.0f)  // never true; keeps the chains
        sink[blockIdx.x] = s;
}

void launch_probe_mfma_f32(hipStream_t s, int blocks, int iters, float *sink)
{
    k_probe_mfma_f32<<<blocks, 256, 0, s>>>(iters, sink);
}

}  // namespace mlmix
