// Expensive ACE-style potential on the induced subsystem S (Algorithm 4 and
// Fig. 10: atoms outside S are removed from every neighbour list), on gfx950.
//
// Per-atom arrays A and dE/dA are stored channel-fastest: X[s][lm][c] with
// c < nchp (channels padded to a multiple of four, padding zero).
//
//  k_ace_basis    atomic basis A_i[lm][a] = sum_{j in S, r<rc} R_n(r) Y_lm(u)
//                 (one wavefront per S atom; per-neighbour R, Y staged in LDS;
//                 lanes own (lm, channel) accumulators, summed in row order)
//  k_ace_blocks   order-3 readout as a symmetric cubic form, per block
//                 (l1 <= l2, l3): P_{ab,m3} = sum_{m1 m2} G A_{a l1 m1} A_{b l2 m2}
//                 (sparse Gaunt stage, VALU/LDS) and D_{c,l3 m3} = sum_ab
//                 P_{ab,m3} W_{ab,c} (dense stage on MFMA for single-species
//                 models; W holds the symmetrised coefficients)
//  k_ace_finalize D3 = sum of the l3 blocks, D2 for order 2, then
//                 dE/dA = c1 + 2 D2 + 3 D3 and E = c0 + sum A (c1 + D2 + D3)
//  k_ace_pairgrad hand-written adjoint of the atomic basis: per pair,
//                 g_ij = dE_i/dd_ij = sum_{n,lm} dE/dA (R_n' u Y + R_n grad Y),
//                 recomputing R, Y and grad Y instead of storing them.
// Forces follow from g in the gather kernel: F_i = sum_j (g_ij - g_ji).
#include "internal.h"
#include "basis.h"

namespace mlmix {

template <typename T>
struct AceArgs {
    int ns, nrad, lmax, order, nchan, nchp, KAt, L2, L1;
    T rc;
    double rc2;
    const T *K, *c0, *c1, *c2s, *W, *gval;
    const PBlock *pb;
    const int *gm3, *gofs;
    int pb_lo[kMaxLmax + 1], pb_hi[kMaxLmax + 1];
    int w_per_species;
};


__device__ __forceinline__ void pair_disp_d(const double *__restrict__ pos, int n, int i, int j,
                                            const Box &b, double d[3])
{
#pragma clang fp contract(off)
    // issue the six loads before any folding so that they overlap
    const double xj[3] = {pos[j], pos[n + j], pos[2 * n + j]};
    const double xi[3] = {pos[i], pos[n + i], pos[2 * n + i]};
    for (int k = 0; k < 3; ++k) {
        double dx = xj[k] - xi[k];
        if (b.per[k]) {
            double h = 0.5 * b.L[k];
            dx = dx > h ? dx - b.L[k] : (dx < -h ? dx + b.L[k] : dx);
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

constexpr int kMaxOwn = 16;  // (lm, channel) entries per lane: L2 * nchp <= 1024

// wpb atoms per block (one wavefront each). The neighbour-chunk loop runs to
// the block's longest row so that the waves meet at every barrier.
template <typename T, bool SEG>
__global__ void __launch_bounds__(256)
    k_ace_basis(const double *__restrict__ pos, int n, Box b0, const int32_t *__restrict__ species,
                int cap, const int *__restrict__ nbr, const int *__restrict__ cnt,
                const int *__restrict__ S_idx, const int *__restrict__ S_local,
                const int *__restrict__ hdr, AceArgs<T> a, int wpb, T *__restrict__ A, Seg sg)
{
    const int nS = hdr[H_NS];
    if (blockIdx.x * wpb >= nS)
        return;  // uniform across the block
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int s = blockIdx.x * wpb + w;
    const bool valid = s < nS;
    extern __shared__ __align__(16) char smem_raw[];
    const size_t slice = (size_t)64 * (a.nrad + a.L2);
    T *Rt = reinterpret_cast<T *>(smem_raw) + (size_t)w * slice;
    T *Yt = Rt + 64 * a.nrad;
    int *zt = reinterpret_cast<int *>(reinterpret_cast<T *>(smem_raw) + (size_t)wpb * slice) + w * 64;
    __shared__ int cm[4];
    const int i = valid ? S_idx[s] : 0;
    const Box b = seg_box<SEG, true>(b0, sg, i);
    const int c = valid ? cnt[i] : 0;
    if (lane == 0)
        cm[w] = c;
    const int *row = nbr + (size_t)i * cap;
    // lane owns entries e = lane + 64 k of the layout [lm][nchp]
    T acc[kMaxOwn];
    int own_z[kMaxOwn], own_n[kMaxOwn], own_lm[kMaxOwn];
#pragma unroll
    for (int k = 0; k < kMaxOwn; ++k) {
        acc[k] = T(0);
        int e = lane + 64 * k;
        int lm = e / a.nchp;
        int ch = e - lm * a.nchp;
        own_lm[k] = lm < a.L2 ? lm : 0;
        own_z[k] = (lm < a.L2 && ch < a.nchan) ? ch / a.nrad : -2;
        own_n[k] = ch % a.nrad;
    }
    __syncthreads();
    int cmax = 0;
    for (int q = 0; q < wpb; ++q)
        cmax = max(cmax, cm[q]);
    const int nown = (a.KAt + 63) >> 6;
    for (int base = 0; base < cmax; base += 64) {
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
                    double ird = 1.0 / rd;
                    T r = T(rd);
                    T ux = T(d[0] * ird), uy = T(d[1] * ird), uz = T(d[2] * ird);
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
            const T *Rr = Rt + t * a.nrad;
            const T *Yr = Yt + t * a.L2;
#pragma unroll
            for (int k = 0; k < kMaxOwn; ++k) {
                if (k >= nown)
                    break;
                if (own_z[k] == z)
                    acc[k] += Rr[own_n[k]] * Yr[own_lm[k]];
            }
        }
        __syncthreads();
    }
    if (!valid)
        return;
    T *As = A + (size_t)s * a.KAt;
#pragma unroll
    for (int k = 0; k < kMaxOwn; ++k) {
        int e = lane + 64 * k;
        if (e < a.KAt)
            As[e] = acc[k];  // padded channels stay zero
    }
}

template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 op(float x, float y, v4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, c, 0, 0, 0);
    }
};

// Rows of the P tile (atoms x m3, padded to 16) and its row stride (odd, so
// that 16 consecutive rows fall into distinct LDS banks).
__host__ __device__ inline int blocks_rows(int ta, int lmax) { return ((ta * (2 * lmax + 1) + 15) / 16) * 16; }
__host__ __device__ inline int blocks_kstride(int nch, int nchp) { return nch * nchp + 1; }

// Order-3 contraction. A persistent grid walks the work items (tile of TA
// atoms of S, block (l1 <= l2, l3)); consecutive items share the tile.
// Sparse Gaunt stage: items (atom, m3, a, four b) accumulate
// sum G A_{a,l1 m1} A_{b..b+3,l2 m2} over the block's entries into the P
// tile [row = atom*d3 + m3][k = a*nchp + b]. Dense stage: D[row][c] =
// sum_k P[row][k] W[k][c] as 16x16 MFMA tiles (weights staged in LDS,
// single-species models) or VALU groups of four channels (weights read
// through the cache, indexed by each atom's species). The block's D goes
// to Dpart; k_ace_finalize sums the blocks of one l3 in a fixed order.
template <typename T>
__global__ void __launch_bounds__(256)
    k_ace_blocks(const int32_t *__restrict__ species, const int *__restrict__ S_idx,
                 const int *__restrict__ hdr, AceArgs<T> a, int TA, int n_pb, int max_ent,
                 int use_mfma, int stage_w, const int *__restrict__ dp_off, int dp_stride,
                 const T *__restrict__ A, T *__restrict__ Dpart)
{
    const int nS = hdr[H_NS];
    const int ntile = (nS + TA - 1) / TA;
    const int nitems = ntile * n_pb;
    if ((int)blockIdx.x >= nitems)
        return;  // uniform across the block (the chunking below leaves
                 // workgroups with blockIdx.x >= nitems without work)
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int nch = a.nchan, nchp = a.nchp, KAt = a.KAt;
    const int Kp = nch * nchp;
    const int Ks = blocks_kstride(nch, nchp);
    const int rowsp = blocks_rows(TA, a.lmax);
    extern __shared__ __align__(16) char smem_raw[];
    T *At = reinterpret_cast<T *>(smem_raw);  // [TA][L2][nchp]
    T *P = At + (size_t)TA * KAt;              // [rowsp][Ks]
    T *Ws = P + (size_t)rowsp * Ks;            // [Kp][nchp] when staged
    T *gv = Ws + (stage_w ? (size_t)Kp * nchp : 0);
    int *gi = reinterpret_cast<int *>(gv + max_ent);
    int *g3 = gi + max_ent;
    __shared__ int zt[16];
    int cur_tile = -1;
    // contiguous chunk of items per workgroup: consecutive items share a tile
    const int per = (nitems + gridDim.x - 1) / gridDim.x;
    const int i_lo = blockIdx.x * per;
    const int i_hi = min(nitems, i_lo + per);
    for (int item = i_lo; item < i_hi; ++item) {
        const int tile = item / n_pb, p = item - tile * n_pb;
        const int s0 = tile * TA;
        const int na = (nS - s0) < TA ? (nS - s0) : TA;
        const PBlock pb = a.pb[p];
        const int d3 = 2 * pb.l3 + 1;
        const int nrows = na * d3;
        __syncthreads();  // the previous item's readers are done with LDS
        if (tile != cur_tile) {
            if (tid < na)
                zt[tid] = sp_clamp(species[S_idx[s0 + tid]], a.ns);
            const T *src = A + (size_t)s0 * KAt;
            for (int e = tid; e < na * KAt; e += 256)
                At[e] = src[e];
            cur_tile = tile;
        }
        const int e_lo = a.gm3[pb.gm3_off];
        const int e_hi = a.gm3[pb.gm3_off + d3];
        for (int e = tid; e < e_hi - e_lo; e += 256) {
            gv[e] = a.gval[e_lo + e];
            gi[e] = a.gofs[e_lo + e];
        }
        for (int e = tid; e <= d3; e += 256)
            g3[e] = a.gm3[pb.gm3_off + e] - e_lo;
        const T *Wb = a.W + pb.w_off;  // single-species weights of the block
        if (stage_w) {
            for (int e = tid; e < Kp * nchp; e += 256)
                Ws[e] = Wb[e];
            Wb = Ws;
        }
        __syncthreads();
        const int ncb = nchp >> 2;
        // the matrix-core stages exist for FP32 only (FP64 keeps the VALU)
        bool done = false;
        if constexpr (sizeof(T) == 4) {
        if (use_mfma) {
            done = true;
            // sparse Gaunt stage on MFMA: for each row (atom t, m3),
            // P[a][b] = sum_e (g_e A[o1_e][a]) A[o2_e][b], i.e. a 16x16 product
            // with K = the m3 group's Gaunt entries, four per instruction.
            const int nat = (nch + 15) >> 4;
            const int kk = lane >> 4;
            for (int rr = wv; rr < nrows; rr += 4) {
                const int t = rr / d3, m3 = rr - t * d3;
                const T *Att = At + (size_t)t * KAt;
                const int e0 = g3[m3], e1 = g3[m3 + 1];
                for (int at_ = 0; at_ < nat; ++at_)
                    for (int bt = 0; bt < nat; ++bt) {
                        const int ar = at_ * 16 + (lane & 15);
                        const int bc = bt * 16 + (lane & 15);
                        typename Mfma<T>::v4 acc = {T(0), T(0), T(0), T(0)};
                        for (int k0 = e0; k0 < e1; k0 += 4) {
                            const int e = k0 + kk;
                            T av = T(0), bv = T(0);
                            if (e < e1) {
                                const int of = gi[e];
                                if (ar < nch)
                                    av = gv[e] * Att[(of & 0xffff) + ar];
                                if (bc < nch)
                                    bv = Att[(of >> 16) + bc];
                            }
                            acc = Mfma<T>::op(av, bv, acc);
                        }
                        // lane holds P[a = at_*16 + 4 kk + v][b = bc]; padded
                        // columns nch <= b < nchp are written as zeros
                        if (bc < nchp) {
                            T *Pr = P + (size_t)rr * Ks + bc;
#pragma unroll
                            for (int v = 0; v < 4; ++v) {
                                const int a2 = at_ * 16 + 4 * kk + v;
                                if (a2 < nch)
                                    Pr[a2 * nchp] = bc < nch ? acc[v] : T(0);
                            }
                        }
                    }
            }
        }
        }
        if (!done) {
        // sparse Gaunt stage on VALU. Thread -> (a, four b) once; rows advance
        // by a fixed stride, so no per-item integer division is needed.
        const int Q = nch * ncb;
        const int rstep = Q <= 256 ? 256 / Q : 1;
        for (int q = (Q <= 256 ? (tid < rstep * Q ? tid % Q : Q) : tid); q < Q; q += 256) {
            const int aa = q / ncb, bq = q - aa * ncb;
            int r = Q <= 256 ? tid / Q : 0;
            int t = r / d3, m3 = r - t * d3;
            for (; r < nrows; r += rstep) {
                const T *Att = At + (size_t)t * KAt;
                T p0 = T(0), p1 = T(0), p2 = T(0), p3 = T(0);
                const int e1 = g3[m3 + 1];
                for (int e = g3[m3]; e < e1; ++e) {
                    int of = gi[e];
                    T ga = gv[e] * Att[(of & 0xffff) + aa];
                    const T *Bb = Att + (of >> 16) + bq * 4;
                    p0 += ga * Bb[0];
                    p1 += ga * Bb[1];
                    p2 += ga * Bb[2];
                    p3 += ga * Bb[3];
                }
                T *Pr = P + (size_t)r * Ks + aa * nchp + bq * 4;
                Pr[0] = p0;
                Pr[1] = p1;
                Pr[2] = p2;
                Pr[3] = p3;
                m3 += rstep;
                while (m3 >= d3) {
                    m3 -= d3;
                    ++t;
                }
            }
        }
        }
        __syncthreads();
        T *Dbase = Dpart + dp_off[p];
        done = false;
        if constexpr (sizeof(T) == 4) {
        if (use_mfma) {
            done = true;
            // D[row][c] = sum_k P[row][k] Ws[k][c]: 16x16 tiles over 4 waves
            const int nrt = (nrows + 15) >> 4, nct = (nch + 15) >> 4;
            for (int tt = wv; tt < nrt * nct; tt += 4) {
                const int rt = tt / nct, ct = tt - rt * nct;
                const int row = rt * 16 + (lane & 15);
                const int col = ct * 16 + (lane & 15);
                const int kk = lane >> 4;
                const bool rv = row < nrows, cv = col < nch;
                const T *Pr = P + (size_t)row * Ks;
                typename Mfma<T>::v4 acc = {T(0), T(0), T(0), T(0)};
                for (int k0 = 0; k0 < Kp; k0 += 4) {
                    int k = k0 + kk;
                    T av = rv ? Pr[k] : T(0);
                    T bv = cv ? Wb[k * nchp + col] : T(0);
                    acc = Mfma<T>::op(av, bv, acc);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    int r = rt * 16 + 4 * kk + v;
                    if (r < nrows && cv) {
                        int t = r / d3, m3 = r - t * d3;
                        Dbase[(size_t)(s0 + t) * dp_stride + m3 * nch + col] = acc[v];
                    }
                }
            }
        }
        }
        if (!done) {
            // VALU: groups (row, four channels); weights per atom species
            for (int g = tid; g < nrows * ncb; g += 256) {
                int r = g / ncb, cb = g - r * ncb;
                int t = r / d3, m3 = r - t * d3;
                const T *Pr = P + (size_t)r * Ks;
                const T *Wc = a.W + (size_t)zt[t] * a.w_per_species + pb.w_off + cb * 4;
                T s0v = T(0), s1v = T(0), s2v = T(0), s3v = T(0);
                for (int k = 0; k < Kp; ++k) {
                    T pv = Pr[k];
                    const T *w = Wc + (size_t)k * nchp;
                    s0v += pv * w[0];
                    s1v += pv * w[1];
                    s2v += pv * w[2];
                    s3v += pv * w[3];
                }
                T vals[4] = {s0v, s1v, s2v, s3v};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    int c = cb * 4 + q;
                    if (c < nch)
                        Dbase[(size_t)(s0 + t) * dp_stride + m3 * nch + c] = vals[q];
                }
            }
        }
    }
}

// APB S atoms per 256-thread workgroup (1: threads over the atomic-basis
// entries, for small S where latency rules; 4: a wave per atom, lanes over
// the entries, for large S where the staged tables are shared by four atoms):
// D3 = sum of the partial-D columns of the (l3, m3) in the listed order (the
// column set of the contraction that wrote them), D2 from the order-2
// coefficients, dE/dA = c1 + 2 D2 + 3 D3 and E = c0 + sum A (c1 + D2 + D3).
// The atom's A row, the column set and (when they fit, stage_c2) the
// order-2 coefficients transposed to [z][l][b][c] are staged in LDS, so that
// a lane's loads are independent LDS reads plus coalesced reads of the
// partial D.
template <typename T, int APB>
__global__ void __launch_bounds__(256)
    k_ace_finalize(const int32_t *__restrict__ species, const int *__restrict__ S_idx,
                   const int *__restrict__ hdr, AceArgs<T> a, DSumSel ds, int stage_c2,
                   int stage_d, int dp_stride, const T *__restrict__ A,
                   const T *__restrict__ Dpart, T *__restrict__ dEdA, double *__restrict__ e_exp)
{
    constexpr int TPA = 256 / APB;  // threads per atom
    const int nS = hdr[H_NS];
    if ((int)blockIdx.x * APB >= nS)
        return;  // uniform across the block
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const int sub = tid / TPA, st = tid - sub * TPA;  // atom of the block, thread within it
    const int s = blockIdx.x * APB + sub;
    const int nch = a.nchan, nchp = a.nchp, L1 = a.L1, KAt = a.KAt;
    extern __shared__ __align__(16) char smem_raw[];
    T *As = reinterpret_cast<T *>(smem_raw) + (size_t)sub * KAt;           // [APB][KAt]
    T *Ct = reinterpret_cast<T *>(smem_raw) + (size_t)APB * KAt;           // [ns][L1][b][c]
    const size_t nC = stage_c2 ? (size_t)a.ns * L1 * nch * nch : 0;
    const int L2 = L1 * L1;
    __shared__ double esum[4];
    // the column set: the split the vector-sparse contraction chose for this
    // |S| (it chooses it the same way), else the per-(block, m3) set
    int lg = 0;
    {
        const int ntile = (nS + kO3Atoms - 1) / kO3Atoms;
        int G = 1;
        while (G < ds.max_split && ntile * G < ds.grid) {
            G <<= 1;
            ++lg;
        }
    }
    const int *dset = ds.tab + ds.off[lg];
    const int ntab = L2 + 1 + ds.ncol[lg];
    const int nD = stage_d ? ds.span[lg] * nch : 0;  // staged prefix of a partial-D row
    T *Dl = Ct + nC + (size_t)sub * nD;                // [APB][nD]
    int *tbl = reinterpret_cast<int *>(Ct + nC + (size_t)APB * nD);  // [L2 + 1] run offsets, then the columns
    const int *dcols = tbl + L2 + 1;
    // staging: eight loads in flight per thread before their LDS stores
    constexpr int UN = 8;
    if (a.order >= 2)
        for (int e0 = tid; e0 < (int)nC; e0 += UN * 256) {
            T v[UN];
#pragma unroll
            for (int u = 0; u < UN; ++u) {
                const int e = min(e0 + u * 256, (int)nC - 1);
                const int c = e % nch, r = e / nch;
                const int b = r % nch, zl = r / nch;
                v[u] = a.c2s[((size_t)zl * nch + c) * nch + b];
            }
#pragma unroll
            for (int u = 0; u < UN; ++u)
                if (e0 + u * 256 < (int)nC)
                    Ct[e0 + u * 256] = v[u];
        }
    for (int e0 = tid; e0 < ntab; e0 += UN * 256) {
        int v[UN];
#pragma unroll
        for (int u = 0; u < UN; ++u)
            v[u] = dset[min(e0 + u * 256, ntab - 1)];
#pragma unroll
        for (int u = 0; u < UN; ++u)
            if (e0 + u * 256 < ntab)
                tbl[e0 + u * 256] = v[u];
    }
    if (s < nS) {
        for (int e0 = st; e0 < KAt; e0 += UN * TPA) {
            T v[UN];
#pragma unroll
            for (int u = 0; u < UN; ++u)
                v[u] = A[(size_t)s * KAt + min(e0 + u * TPA, KAt - 1)];
#pragma unroll
            for (int u = 0; u < UN; ++u)
                if (e0 + u * TPA < KAt)
                    As[e0 + u * TPA] = v[u];
        }
        for (int e0 = st; e0 < nD; e0 += UN * TPA) {
            T v[UN];
#pragma unroll
            for (int u = 0; u < UN; ++u)
                v[u] = Dpart[(size_t)s * dp_stride + min(e0 + u * TPA, nD - 1)];
#pragma unroll
            for (int u = 0; u < UN; ++u)
                if (e0 + u * TPA < nD)
                    Dl[e0 + u * TPA] = v[u];
        }
    }
    __syncthreads();
    if (s >= nS)
        return;  // after the only block barrier (APB = 4; APB = 1 returned above)
    const int i = S_idx[s];
    const int z = sp_clamp(species[i], a.ns);
    const T *Ds = stage_d ? Dl : Dpart + (size_t)s * dp_stride;
    const T *Cz = stage_c2 ? Ct + (size_t)z * L1 * nch * nch : nullptr;
    double es = 0.0;
    for (int e = st; e < KAt; e += TPA) {
        const int lm = e / nchp, c = e - lm * nchp;
        if (c >= nch) {
            dEdA[(size_t)s * KAt + e] = T(0);
            continue;
        }
        int l = (int)sqrtf((float)lm);
        l -= (l * l > lm);
        l += ((l + 1) * (l + 1) <= lm);
        const int m3 = lm - l * l;
        T c1t = (l == 0) ? a.c1[z * nch + c] : T(0);
        T D2 = T(0);
        if (a.order >= 2) {
            const T *Al = As + lm * nchp;
            if (Cz) {
                const T *C = Cz + (size_t)l * nch * nch + c;
                for (int bb = 0; bb < nch; ++bb)
                    D2 += C[bb * nch] * Al[bb];
            } else {
                const T *C = a.c2s + (((size_t)z * L1 + l) * nch + c) * nch;
                for (int bb = 0; bb < nch; ++bb)
                    D2 += C[bb] * Al[bb];
            }
        }
        T D3 = T(0);
        if (a.order >= 3) {
            // all block loads first (independent), then the sum in block order
            constexpr int kPre = 16;
            const int k0 = tbl[lm], nk = tbl[lm + 1] - k0;
            const int *cl = dcols + k0;
            T v[kPre];
#pragma unroll
            for (int k = 0; k < kPre; ++k)
                v[k] = k < nk ? Ds[cl[k] + c] : T(0);
#pragma unroll
            for (int k = 0; k < kPre; ++k)
                D3 += v[k];
            for (int k = kPre; k < nk; ++k)
                D3 += Ds[cl[k] + c];
        }
        const T Av = As[e];
        dEdA[(size_t)s * KAt + e] = c1t + T(2) * D2 + T(3) * D3;
        es += (double)(Av * (c1t + D2 + D3));
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1)
        es += __shfl_xor(es, d);
    if constexpr (APB == 4) {
        if (lane == 0)
            e_exp[i] = (double)a.c0[z] + es;
    } else {
        if (lane == 0)
            esum[wv] = es;
        __syncthreads();
        if (tid == 0)
            e_exp[i] = (double)a.c0[z] + ((esum[0] + esum[1]) + (esum[2] + esum[3]));
    }
}

template <typename T, bool SEG>
__global__ void __launch_bounds__(256)
    k_ace_pairgrad(const double *__restrict__ pos, int n, Box b0, const int32_t *__restrict__ species,
                   int cap, const int *__restrict__ nbr, const int *__restrict__ cnt,
                   const int *__restrict__ S_idx, const int *__restrict__ S_local,
                   const int *__restrict__ hdr, AceArgs<T> a, int wpb, const T *__restrict__ dEdA,
                   const double *__restrict__ weights, T *__restrict__ g, Seg sg)
{
    const int nS = hdr[H_NS];
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int s = blockIdx.x * wpb + w;
    if (s >= nS)
        return;  // no barrier in this kernel
    extern __shared__ __align__(16) char smem_raw[];
    T *dAs = reinterpret_cast<T *>(smem_raw) + (size_t)w * a.KAt;
    const int i = S_idx[s];
    const Box b = seg_box<SEG, true>(b0, sg, i);
    T wgt = weights ? T(weights[i]) : T(1);
    for (int e = lane; e < a.KAt; e += 64)
        dAs[e] = dEdA[(size_t)s * a.KAt + e] * wgt;
    // the wave reads back only its own slice: order the LDS writes before
    // the reads of other lanes of the same wave
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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
                double ird = 1.0 / rd;
                T r = T(rd);
                T ux = T(d[0] * ird), uy = T(d[1] * ird), uz = T(d[2] * ird);
                T R[kMaxNrad], dR[kMaxNrad];
                radial<T>(a.nrad, r, a.rc, R, dR);
                const T *col = dAs + sp_clamp(species[j], a.ns) * a.nrad;
                T rad = T(0), vx = T(0), vy = T(0), vz = T(0);
                const int nchp = a.nchp, nrad = a.nrad;
                ylm_stream<T>(a.lmax, ux, uy, uz, a.K, [&](int lm, T Y, T yx, T yy, T yz) {
                    T sR = T(0), sD = T(0);
                    const T *cl = col + lm * nchp;
#pragma unroll
                    for (int k = 0; k < kMaxNrad; ++k)
                        if (k < nrad) {
                            T v = cl[k];
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
                T ir = T(ird);
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

// The same pair adjoint in FP32 with two S atoms per wave (32 lanes each) for
// large systems: each half first lists its row's valid pairs (partner in S,
// inside the cutoff) in LDS by ballot, then its 32 lanes take the listed
// pairs 32 at a time, recomputing the geometry; invalid slots get a zero
// gradient from their owner lane. At lmax 5 and 26 pairs in a row of 64 slots
// this keeps about 80 % of the lanes on the harmonic work instead of 40 %.
template <bool SEG>
__global__ void __launch_bounds__(256)
    k_ace_pairgrad_h(const double *__restrict__ pos, int n, Box b0,
                     const int32_t *__restrict__ species, int cap, const int *__restrict__ nbr,
                     const int *__restrict__ cnt, const int *__restrict__ S_idx,
                     const int *__restrict__ S_local, const int *__restrict__ hdr,
                     AceArgs<float> a, const float *__restrict__ dEdA,
                     const double *__restrict__ weights, float *__restrict__ g, Seg sg)
{
    const int nS = hdr[H_NS];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int half = lane >> 5, hl = lane & 31;
    const int s0 = (blockIdx.x * 4 + w) * 2;
    if (s0 >= nS)
        return;  // uniform across the wave; no block barrier in this kernel
    const int s = s0 + half;
    const bool live = s < nS;
    extern __shared__ __align__(16) char smem_raw[];
    // per wave: dE/dA rows of its two atoms, then the two pair lists
    float *dAs = reinterpret_cast<float *>(smem_raw) + (size_t)w * (2 * a.KAt + 2 * cap);
    int *lst = reinterpret_cast<int *>(dAs + 2 * a.KAt);
    float *dA = dAs + half * a.KAt;
    int *pl = lst + half * cap;
    const int i = live ? S_idx[s] : 0;
    const Box b = seg_box<SEG, false>(b0, sg, i);
    const float wgt = (weights && live) ? float(weights[i]) : 1.0f;
    if (live)
        for (int e = hl; e < a.KAt; e += 32)
            dA[e] = dEdA[(size_t)s * a.KAt + e] * wgt;
    const int c = live ? cnt[i] : 0;
    const int cmax = max(c, __shfl_xor(c, 32));
    const int *row = nbr + (size_t)i * cap;
    float *gs = g + (size_t)s * cap * 3;
    // 1. the valid pairs of each half's row, listed in slot order
    int nv = 0;
    for (int base = 0; base < cmax; base += 32) {
        const int slot = base + hl;
        bool ok = false;
        if (slot < c) {
            const int j = row[slot];
            if (S_local[j] >= 0) {
                double d[3];
                pair_disp_d(pos, n, i, j, b, d);
                ok = norm2_d(d) < a.rc2;
            }
            if (!ok) {
                gs[slot * 3 + 0] = 0.f;
                gs[slot * 3 + 1] = 0.f;
                gs[slot * 3 + 2] = 0.f;
            }
        }
        const unsigned long long m = __ballot(ok);
        const unsigned hm = (unsigned)(m >> (32 * half));
        if (ok)
            pl[nv + __popc(hm & ((1u << hl) - 1u))] = slot;
        nv += __popc(hm);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // 2. the listed pairs, 32 per round in each half
    const int nvmax = max(nv, __shfl_xor(nv, 32));
    for (int base = 0; base < nvmax; base += 32) {
        const int k = base + hl;
        if (k >= nv)
            continue;
        const int slot = pl[k];
        const int j = row[slot];
        double d[3];
        pair_disp_d(pos, n, i, j, b, d);
        const double rd = sqrt(norm2_d(d));
        const double ird = 1.0 / rd;
        const float r = float(rd);
        const float ux = float(d[0] * ird), uy = float(d[1] * ird), uz = float(d[2] * ird);
        float R[kMaxNrad], dR[kMaxNrad];
        radial<float>(a.nrad, r, a.rc, R, dR);
        const float *col = dA + sp_clamp(species[j], a.ns) * a.nrad;
        float rad = 0.f, vx = 0.f, vy = 0.f, vz = 0.f;
        const int nchp = a.nchp, nrad = a.nrad;
        ylm_stream<float>(a.lmax, ux, uy, uz, a.K, [&](int lm, float Y, float yx, float yy, float yz) {
            float sR = 0.f, sD = 0.f;
            const float *cl = col + lm * nchp;
#pragma unroll
            for (int q = 0; q < kMaxNrad; ++q)
                if (q < nrad) {
                    const float v = cl[q];
                    sR += v * R[q];
                    sD += v * dR[q];
                }
            rad += sD * Y;
            vx += sR * yx;
            vy += sR * yy;
            vz += sR * yz;
        });
        const float ud = ux * vx + uy * vy + uz * vz;
        const float ir = float(ird);
        gs[slot * 3 + 0] = rad * ux + (vx - ux * ud) * ir;
        gs[slot * 3 + 1] = rad * uy + (vy - uy * ud) * ir;
        gs[slot * 3 + 2] = rad * uz + (vz - uz * ud) * ir;
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
    a.nchp = m.nchp;
    a.KAt = m.KAt;
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
    a.gofs = reinterpret_cast<const int *>(base + m.gofs);
    a.w_per_species = m.w_per_species;
    return a;
}

// pb_lo / pb_hi are filled by the host from the block list (sorted by l3).
extern void pb_ranges(const Ctx &c, int *lo, int *hi);

typedef float f4v_t __attribute__((ext_vector_type(4)));

// Geometry of one valid expensive pair, in the compacted order of the row.
struct PairGeo {
    float r, ux, uy, uz, ir;
    int zj, slot, pad;
};
static_assert(sizeof(PairGeo) == 32, "PairGeo is eight 4-byte words");

// Valid pairs of centre i (partner in S, inside the cutoff) over the whole
// row: lane l tests slots l + 64 u, u < 4 (rows hold at most 256 slots); the
// ballots give each valid pair its index in row order (pp[u], -1 if not
// valid) and the function returns their number. Pairs whose index lies in
// [64 rnd, 64 rnd + 64) leave their geometry in geo[index - 64 rnd].
__device__ __forceinline__ int compact_pairs(const double *__restrict__ pos, int n, const Box &b,
                                             const int32_t *__restrict__ species, int ns,
                                             const int *__restrict__ row, int c,
                                             const int *__restrict__ S_local, int i, double rc2,
                                             int lane, int rnd, PairGeo *geo, int (&pp)[4])
{
    int nv = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        pp[u] = -1;
        if (64 * u >= c)
            continue;  // uniform
        const int slot = lane + 64 * u;
        bool ok = false;
        double d[3] = {0.0, 0.0, 0.0}, r2 = 0.0;
        int j = 0;
        if (slot < c) {
            j = row[slot];
            if (S_local[j] >= 0) {
                pair_disp_d(pos, n, i, j, b, d);
                r2 = norm2_d(d);
                ok = r2 < rc2;
            }
        }
        const unsigned long long mask = __ballot(ok);
        const int p = nv + __popcll(mask & ((1ull << lane) - 1ull));
        if (ok) {
            pp[u] = p;
            if (p >= 64 * rnd && p < 64 * rnd + 64) {
                const double rd = sqrt(r2), ird = 1.0 / rd;
                PairGeo gq;
                gq.r = float(rd);
                gq.ux = float(d[0] * ird);
                gq.uy = float(d[1] * ird);
                gq.uz = float(d[2] * ird);
                gq.ir = float(ird);
                gq.zj = sp_clamp(species[j], ns);
                gq.slot = slot;
                gq.pad = 0;
                geo[p - 64 * rnd] = gq;
            }
        }
        nv += __popcll(mask);
    }
    return nv;
}

// Geometry of the pairs with compacted index in [64 rnd, 64 rnd + 64) for a
// later round (rows with more than 64 valid pairs): recomputed from the
// positions with the same operations.
__device__ __forceinline__ void pairs_round(const double *__restrict__ pos, int n, const Box &b,
                                            const int32_t *__restrict__ species, int ns,
                                            const int *__restrict__ row, int i, int lane, int rnd,
                                            const int (&pp)[4], PairGeo *geo)
{
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int p = pp[u];
        if (p >= 64 * rnd && p < 64 * rnd + 64) {
            const int slot = lane + 64 * u;
            const int j = row[slot];
            double d[3];
            pair_disp_d(pos, n, i, j, b, d);
            const double r2 = norm2_d(d);
            const double rd = sqrt(r2), ird = 1.0 / rd;
            PairGeo gq;
            gq.r = float(rd);
            gq.ux = float(d[0] * ird);
            gq.uy = float(d[1] * ird);
            gq.uz = float(d[2] * ird);
            gq.ir = float(ird);
            gq.zj = sp_clamp(species[j], ns);
            gq.slot = slot;
            gq.pad = 0;
            geo[p - 64 * rnd] = gq;
        }
    }
}

__device__ __forceinline__ void wave_sync_ace()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The same atomic basis in passes over 64 list slots (each lane evaluates
// its own slot's pair; valid pairs compacted per pass): measured faster on
// large systems (1M atoms, lmax 5: 10.58 against 10.82 ms per step), where
// the whole-row form below is slower; small systems take the whole-row form
// (8,193 atoms: 132.7 against 135.4 us per step).
template <int MT, int NT, bool SEG>
__global__ void __launch_bounds__(256)
    k_ace_basis_mfma_chunks(const double *__restrict__ pos, int n, Box b0,
                     const int32_t *__restrict__ species, int cap, const int *__restrict__ nbr,
                     const int *__restrict__ cnt, const int *__restrict__ S_idx,
                     const int *__restrict__ S_local, const int *__restrict__ hdr,
                     AceArgs<float> a, int wpb, float *__restrict__ A, Seg sg)
{
    constexpr int RW = 16 * MT + 1, YW = 16 * NT + 1;
    const int nS = hdr[H_NS];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int s = blockIdx.x * wpb + w;
    if (s >= nS)
        return;  // no barriers in this kernel
    extern __shared__ __align__(16) char smem_raw[];
    float *Rz = reinterpret_cast<float *>(smem_raw) + (size_t)w * 64 * (RW + YW);
    float *Yt = Rz + 64 * RW;
    const int m16 = lane & 15, kg = lane >> 4;
    const int i = S_idx[s];
    const Box b = seg_box<SEG, true>(b0, sg, i);
    const int c = cnt[i];
    const int *row = nbr + (size_t)i * cap;
    const int nrad = a.nrad, nch = a.nchan, L2 = a.L2;
    f4v_t acc[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
            acc[mt][nt] = (f4v_t){0.f, 0.f, 0.f, 0.f};
    for (int base = 0; base < c; base += 64) {
        const int slot = base + lane;
        bool ok = false;
        float R[kMaxNrad], dR[kMaxNrad];
        float ux = 0.f, uy = 0.f, uz = 0.f;
        int zj = 0;
        if (slot < c) {
            const int j = row[slot];
            if (S_local[j] >= 0) {
                double d[3];
                pair_disp_d(pos, n, i, j, b, d);
                const double r2 = norm2_d(d);
                if (r2 < a.rc2) {
                    const double rd = sqrt(r2), ird = 1.0 / rd;
                    radial<float>(nrad, float(rd), a.rc, R, dR);
                    ux = float(d[0] * ird);
                    uy = float(d[1] * ird);
                    uz = float(d[2] * ird);
                    zj = sp_clamp(species[j], a.ns);
                    ok = true;
                }
            }
        }
        const unsigned long long mask = __ballot(ok);
        const int nv = __popcll(mask);
        const int nv4 = (nv + 3) & ~3;
        const int p = __popcll(mask & ((1ull << lane) - 1ull));
        if (ok) {
            float *rr = Rz + p * RW;
            for (int ch = 0; ch < 16 * MT; ++ch)
                rr[ch] = 0.f;
#pragma unroll
            for (int k = 0; k < kMaxNrad; ++k)
                if (k < nrad)
                    rr[zj * nrad + k] = R[k];
            float *yr = Yt + p * YW;
            ylm_stream<float>(a.lmax, ux, uy, uz, a.K,
                              [&](int lm, float Y, float, float, float) { yr[lm] = Y; });
            for (int lm = L2; lm < 16 * NT; ++lm)
                yr[lm] = 0.f;
        }
        if (lane >= nv && lane < nv4) {
            // zero the rows that pad K to a multiple of four (rows nv.. are
            // not written by the compaction, whichever lanes hold pairs)
            for (int ch = 0; ch < 16 * MT; ++ch)
                Rz[lane * RW + ch] = 0.f;
            for (int lm = 0; lm < 16 * NT; ++lm)
                Yt[lane * YW + lm] = 0.f;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int k0 = 0; k0 < nv4; k0 += 4) {
            const int kr = k0 + kg;
            float xa[MT], yb[NT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                xa[mt] = Rz[kr * RW + mt * 16 + m16];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                yb[nt] = Yt[kr * YW + nt * 16 + m16];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[mt], yb[nt], acc[mt][nt], 0, 0, 0);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // lane holds A[ch = 16 mt + 4 kg + v][lm = 16 nt + m16]: four consecutive
    // channels of one lm, stored as one 16-byte write (padded channels are 0)
    float *As = A + (size_t)s * a.KAt;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int lm = nt * 16 + m16, ch0 = mt * 16 + 4 * kg;
            if (lm < L2 && ch0 < a.nchp)
                *reinterpret_cast<f4v_t *>(As + lm * a.nchp + ch0) = acc[mt][nt];
        }
}

// Atomic basis on the matrix cores (FP32 potentials): one wave per S atom.
// The valid pairs of the whole row (partner in S, inside the cutoff) are
// compacted by ballot first, their geometry left in LDS; lane q then
// evaluates the radial functions and harmonics of compacted pair q into
// wave-private LDS rows (radial row masked by the partner's species, so that
// channel (z, n) holds R_n only for z = z_j; rows padded with zeros to a
// multiple of four), and A[(z, n)][lm] = sum_j R_zn,j Y_lm,j accumulates as
// 16x16x4 MFMA tiles (MT channel tiles x NT lm tiles, K = the compacted
// pairs, 64 per round; rows hold about 40 valid pairs, so one round). Row
// strides are odd so that the row writes of the 64 lanes and the tile reads
// are free of bank conflicts.
template <int MT, int NT, bool SEG>
__global__ void __launch_bounds__(256)
    k_ace_basis_mfma(const double *__restrict__ pos, int n, Box b0,
                     const int32_t *__restrict__ species, int cap, const int *__restrict__ nbr,
                     const int *__restrict__ cnt, const int *__restrict__ S_idx,
                     const int *__restrict__ S_local, const int *__restrict__ hdr,
                     AceArgs<float> a, int wpb, float *__restrict__ A, Seg sg)
{
    constexpr int RW = 16 * MT + 1, YW = 16 * NT + 1;
    const int nS = hdr[H_NS];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int s = blockIdx.x * wpb + w;
    if (s >= nS)
        return;  // no barriers in this kernel
    extern __shared__ __align__(16) char smem_raw[];
    // per wave: R rows [64][RW], Y rows [64][YW], then 64 PairGeo (8 floats each)
    float *Rz = reinterpret_cast<float *>(smem_raw) + (size_t)w * (64 * (RW + YW) + 64 * 8);
    float *Yt = Rz + 64 * RW;
    const int m16 = lane & 15, kg = lane >> 4;
    const int i = S_idx[s];
    const Box b = seg_box<SEG, true>(b0, sg, i);
    const int c = cnt[i];
    const int *row = nbr + (size_t)i * cap;
    const int nrad = a.nrad, nch = a.nchan, L2 = a.L2;
    f4v_t acc[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
            acc[mt][nt] = (f4v_t){0.f, 0.f, 0.f, 0.f};
    PairGeo *geo = reinterpret_cast<PairGeo *>(Yt + 64 * YW);  // [64]
    int pp[4];
    const int nv_all = compact_pairs(pos, n, b, species, a.ns, row, c, S_local, i, a.rc2, lane, 0,
                                     geo, pp);
    for (int rnd = 0; 64 * rnd < nv_all; ++rnd) {
        if (rnd > 0)
            pairs_round(pos, n, b, species, a.ns, row, i, lane, rnd, pp, geo);
        wave_sync_ace();
        const int nv = min(64, nv_all - 64 * rnd);
        const int nv4 = (nv + 3) & ~3;
        // lane q builds the rows of compacted pair q (rows nv..nv4-1 zero)
        if (lane < nv) {
            const PairGeo gq = geo[lane];
            float R[kMaxNrad], dR[kMaxNrad];
            radial<float>(nrad, gq.r, a.rc, R, dR);
            float *rr = Rz + lane * RW;
            for (int ch = 0; ch < 16 * MT; ++ch)
                rr[ch] = 0.f;
#pragma unroll
            for (int k = 0; k < kMaxNrad; ++k)
                if (k < nrad)
                    rr[gq.zj * nrad + k] = R[k];
            float *yr = Yt + lane * YW;
            ylm_stream<float>(a.lmax, gq.ux, gq.uy, gq.uz, a.K,
                              [&](int lm, float Y, float, float, float) { yr[lm] = Y; });
            for (int lm = L2; lm < 16 * NT; ++lm)
                yr[lm] = 0.f;
        } else if (lane < nv4) {
            for (int ch = 0; ch < 16 * MT; ++ch)
                Rz[lane * RW + ch] = 0.f;
            for (int lm = 0; lm < 16 * NT; ++lm)
                Yt[lane * YW + lm] = 0.f;
        }
        wave_sync_ace();
        for (int k0 = 0; k0 < nv4; k0 += 4) {
            const int kr = k0 + kg;
            float xa[MT], yb[NT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                xa[mt] = Rz[kr * RW + mt * 16 + m16];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                yb[nt] = Yt[kr * YW + nt * 16 + m16];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[mt], yb[nt], acc[mt][nt], 0, 0, 0);
        }
        wave_sync_ace();
    }
    // lane holds A[ch = 16 mt + 4 kg + v][lm = 16 nt + m16]: four consecutive
    // channels of one lm, stored as one 16-byte write (padded channels are 0)
    float *As = A + (size_t)s * a.KAt;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int lm = nt * 16 + m16, ch0 = mt * 16 + 4 * kg;
            if (lm < L2 && ch0 < a.nchp)
                *reinterpret_cast<f4v_t *>(As + lm * a.nchp + ch0) = acc[mt][nt];
        }
}

// The finalisation inside the pair adjoint (k_ace_pairgrad_wg): the
// workgroup computes its atom's dE/dA from the partial D as the finalisation
// kernel does (same terms, same order of the sums) instead of reading it back.
struct FinArgs {
    const float *A;      // [S][KAt] atomic basis
    const float *Dpart;  // [S][dp_stride] partial D
    int dp_stride;
    DSumSel ds;          // the column set of the contraction that wrote it
    double *e_exp;       // site energies (NULL: gradient only)
};

// Pair adjoint on the matrix cores (FP32 potentials): one wave per S atom.
// G = dE/dA of the atom (times its weight) is staged transposed, [(z, n)][lm].
// The valid pairs of the whole row (partner in S, inside the cutoff) are
// compacted by ballot first (geometry in LDS), 64 per round, and lane q
// builds the species-masked rows R and dR of compacted pair q;
// S_R = R G and S_D = dR G (pairs x lm) are 16x16x4 MFMA tiles (K =
// channels); each pair's lane then contracts its rows with the harmonics and
// their gradients, g = rad u + (v - u (u.v)) / r with rad = sum S_D Y and
// v = sum S_R grad_u Y, and writes g to its list slot (0 for other slots).
template <int MT, int NT, bool SEG>
__global__ void __launch_bounds__(256)
    k_ace_pairgrad_mfma(const double *__restrict__ pos, int n, Box b0,
                        const int32_t *__restrict__ species, int cap, const int *__restrict__ nbr,
                        const int *__restrict__ cnt, const int *__restrict__ S_idx,
                        const int *__restrict__ S_local, const int *__restrict__ hdr,
                        AceArgs<float> a, int wpb, const float *__restrict__ dEdA,
                        const double *__restrict__ weights, float *__restrict__ g, Seg sg)
{
    constexpr int RW = 16 * MT + 1, YW = 16 * NT + 1;
    constexpr int PAIR = 64 * RW * 2 > 64 * YW * 2 ? 64 * RW * 2 : 64 * YW * 2;
    const int nS = hdr[H_NS];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int s = blockIdx.x * wpb + w;
    if (s >= nS)
        return;  // no barriers in this kernel
    extern __shared__ __align__(16) char smem_raw[];
    float *base = reinterpret_cast<float *>(smem_raw) + (size_t)w * (PAIR + 16 * MT * YW + 64 * 8);
    float *Rr = base, *Dr = base + 64 * RW;           // [64][RW] each
    float *SR = base, *SD = base + 64 * YW;           // [64][YW] each (after the MFMAs)
    float *Gt = base + PAIR;                          // [16 MT][YW]
    PairGeo *geo = reinterpret_cast<PairGeo *>(Gt + 16 * MT * YW);  // [64]
    const int m16 = lane & 15, kg = lane >> 4;
    const int i = S_idx[s];
    const Box b = seg_box<SEG, true>(b0, sg, i);
    const float wgt = weights ? float(weights[i]) : 1.0f;
    const int nrad = a.nrad, nch = a.nchan, L2 = a.L2, nchp = a.nchp;
    for (int e = lane; e < 16 * MT * 16 * NT; e += 64) {
        const int ch = e / (16 * NT), lm = e - ch * (16 * NT);
        Gt[ch * YW + lm] = (ch < nch && lm < L2) ? dEdA[(size_t)s * a.KAt + lm * nchp + ch] * wgt : 0.f;
    }
    const int c = cnt[i];
    const int *row = nbr + (size_t)i * cap;
    float *gs = g + (size_t)s * cap * 3;
    int pp[4];
    const int nv_all = compact_pairs(pos, n, b, species, a.ns, row, c, S_local, i, a.rc2, lane, 0,
                                     geo, pp);
    // slots without a valid pair get a zero gradient from their owner lane
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int slot = lane + 64 * u;
        if (slot < c && pp[u] < 0) {
            gs[slot * 3 + 0] = 0.f;
            gs[slot * 3 + 1] = 0.f;
            gs[slot * 3 + 2] = 0.f;
        }
    }
    for (int rnd = 0; 64 * rnd < nv_all; ++rnd) {
        if (rnd > 0)
            pairs_round(pos, n, b, species, a.ns, row, i, lane, rnd, pp, geo);
        wave_sync_ace();
        const int nv = min(64, nv_all - 64 * rnd);
        const int nrt = (nv + 15) >> 4;
        // lane q builds the radial rows of compacted pair q; rows up to the
        // next multiple of 16 (one MFMA row tile) are zero
        if (lane < nv) {
            const PairGeo gq = geo[lane];
            float R[kMaxNrad], dR[kMaxNrad];
            radial<float>(nrad, gq.r, a.rc, R, dR);
            float *rr = Rr + lane * RW, *dr = Dr + lane * RW;
            for (int ch = 0; ch < 16 * MT; ++ch) {
                rr[ch] = 0.f;
                dr[ch] = 0.f;
            }
#pragma unroll
            for (int k = 0; k < kMaxNrad; ++k)
                if (k < nrad) {
                    rr[gq.zj * nrad + k] = R[k];
                    dr[gq.zj * nrad + k] = dR[k];
                }
        } else if (lane < 16 * nrt) {
            float *rr = Rr + lane * RW, *dr = Dr + lane * RW;
            for (int ch = 0; ch < 16 * MT; ++ch) {
                rr[ch] = 0.f;
                dr[ch] = 0.f;
            }
        }
        wave_sync_ace();
        // S tiles: rows = compacted pairs (nrt tiles of 16), cols = lm, K = channels
        f4v_t sr[4][NT], sd[4][NT];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                sr[rt][nt] = (f4v_t){0.f, 0.f, 0.f, 0.f};
                sd[rt][nt] = (f4v_t){0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
        for (int k0 = 0; k0 < 16 * MT; k0 += 4) {
            const int kc = k0 + kg;
            float gb[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                gb[nt] = Gt[kc * YW + nt * 16 + m16];
#pragma unroll
            for (int rt = 0; rt < 4; ++rt)
                if (rt < nrt) {
                    const float xr = Rr[(rt * 16 + m16) * RW + kc];
                    const float xd = Dr[(rt * 16 + m16) * RW + kc];
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) {
                        sr[rt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(xr, gb[nt], sr[rt][nt], 0, 0, 0);
                        sd[rt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(xd, gb[nt], sd[rt][nt], 0, 0, 0);
                    }
                }
        }
        wave_sync_ace();
        // lane holds S[pair row = 16 rt + 4 kg + v][lm = 16 nt + m16]
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
            if (rt < nrt) {
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int sl = rt * 16 + 4 * kg + v, lm = nt * 16 + m16;
                        SR[sl * YW + lm] = sr[rt][nt][v];
                        SD[sl * YW + lm] = sd[rt][nt][v];
                    }
            }
        wave_sync_ace();
        if (lane < nv) {
            const PairGeo gq = geo[lane];
            const float *srow = SR + lane * YW, *drow = SD + lane * YW;
            float rad = 0.f, vx = 0.f, vy = 0.f, vz = 0.f;
            ylm_stream<float>(a.lmax, gq.ux, gq.uy, gq.uz, a.K, [&](int lm, float Y, float yx, float yy, float yz) {
                const float sR = srow[lm], sD = drow[lm];
                rad += sD * Y;
                vx += sR * yx;
                vy += sR * yy;
                vz += sR * yz;
            });
            const float ud = gq.ux * vx + gq.uy * vy + gq.uz * vz;
            gs[gq.slot * 3 + 0] = rad * gq.ux + (vx - gq.ux * ud) * gq.ir;
            gs[gq.slot * 3 + 1] = rad * gq.uy + (vy - gq.uy * ud) * gq.ir;
            gs[gq.slot * 3 + 2] = rad * gq.uz + (vz - gq.uz * ud) * gq.ir;
        }
        wave_sync_ace();
    }
}

// Pair adjoint with the finalisation, one workgroup of four waves per S atom
// (single-precision modes). The work of one atom is spread over the
// waves instead of resting on one wave's latency:
//  1. every thread stages a share of the finalisation's tables into LDS (the
//     A row, the species' order-2 matrices, the used prefix of the partial-D
//     row, the column set), all loads in flight together; wave 0 meanwhile
//     compacts the row's valid pairs (partner in S, inside the cutoff) by
//     ballot into geo;
//  2. G = dE/dA (times the atom's weight in a backward call), [(z, n)][lm],
//     and the site energy from the staged tables, two to four elements per
//     thread (dE/dA = c1 + 2 D2 + 3 D3; the same terms and sums as the
//     finalisation kernel);
//  3. per round of 64 compacted pairs: wave w builds the species-masked rows
//     R and dR of pairs 16 w .. 16 w + 15 and their 16-row MFMA tiles S_R =
//     R G and S_D = dR G (pairs x lm, K = channels) into the shared S rows;
//  4. wave w contracts all 64 pairs' S rows with the harmonics of its share
//     of the orders |m| ({0}, {1}, {2}, {3..lmax}: one share per wave, so
//     the stream is uniform within a wave), leaving partial sums rad =
//     sum S_D Y and v = sum S_R grad_u Y per pair; the four partials are
//     added in wave order and g = rad u + (v - u (u.v)) / r goes to the
//     pair's list slot (0 for slots without a valid pair).
template <int MT, int NT, bool SEG>
struct PairWgLds {
    static constexpr int RW = 16 * MT + 1, YW = 16 * NT + 1;
    static constexpr int S_ROWS = 64 * YW * 2;  // S_R, S_D of 64 pairs
    static constexpr int P_ROWS = 64 * RW * 2;  // R, dR of 64 pairs (then the partial sums)
    static constexpr int U = S_ROWS + P_ROWS;   // also the staging space of step 1
    static constexpr int GT = 16 * MT * YW;
    static constexpr int TBL = ((16 * NT + 1 + 256) + 63) / 64 * 64;  // column table (ints)
    static constexpr int FLOATS = U + GT + 64 * 8 + TBL + 16;
    static_assert(4 * 64 * 4 <= P_ROWS, "partial sums fit the R rows");
};

template <int MT, int NT, bool SEG>
__global__ void __launch_bounds__(256)
    k_ace_pairgrad_wg(const double *__restrict__ pos, int n, Box b0,
                      const int32_t *__restrict__ species, int cap, const int *__restrict__ nbr,
                      const int *__restrict__ cnt, const int *__restrict__ S_idx,
                      const int *__restrict__ S_local, const int *__restrict__ hdr,
                      AceArgs<float> a, const double *__restrict__ weights,
                      float *__restrict__ g, Seg sg, FinArgs fa)
{
    using LY = PairWgLds<MT, NT, SEG>;
    constexpr int RW = LY::RW, YW = LY::YW;
    const int nS = hdr[H_NS];
    const int s = blockIdx.x;
    if (s >= nS)
        return;  // uniform across the workgroup
    extern __shared__ __align__(16) char smem_raw[];
    float *U = reinterpret_cast<float *>(smem_raw);
    float *SR = U, *SD = U + 64 * YW;                      // [64][YW] each
    float *Rr = U + LY::S_ROWS, *Dr = Rr + 64 * RW;        // [64][RW] each
    float *part = Rr;                                      // [4 waves][64 pairs][4] after the MFMAs
    float *Gt = U + LY::U;                                 // [16 MT][YW]
    PairGeo *geo = reinterpret_cast<PairGeo *>(Gt + LY::GT);  // [64]
    int *tbl = reinterpret_cast<int *>(Gt + LY::GT + 64 * 8);  // [TBL]
    double *red = reinterpret_cast<double *>(tbl + LY::TBL);   // [4] energy partials
    int *nvs = reinterpret_cast<int *>(red + 4);               // valid pairs of the row
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int m16 = lane & 15, kg = lane >> 4;
    const int i = S_idx[s];
    const Box b = seg_box<SEG, true>(b0, sg, i);
    const int nrad = a.nrad, nch = a.nchan, L2 = a.L2, nchp = a.nchp;
    const int z = sp_clamp(species[i], a.ns);
    const int c = cnt[i];
    const int *row = nbr + (size_t)i * cap;
    float *gs = g + (size_t)s * cap * 3;
    const float wgt = weights ? float(weights[i]) : 1.0f;  // backward: dL/dE_i

    // ---- 1. staging (all threads) and the pair compaction (wave 0)
    int lg = 0;
    {
        const int ntile = (nS + kO3Atoms - 1) / kO3Atoms;
        int G = 1;
        while (G < fa.ds.max_split && ntile * G < fa.ds.grid) {
            G <<= 1;
            ++lg;
        }
    }
    const int *dset = fa.ds.tab + fa.ds.off[lg];
    const int nA = a.KAt;
    const int nC = a.order >= 2 ? a.L1 * nch * nch : 0;
    const int nD = a.order >= 3 ? fa.ds.span[lg] * nch : 0;
    const int ntab = L2 + 1 + fa.ds.ncol[lg];
    const int tot = nA + nC + nD;  // <= LY::U (host check)
    float *As = U, *Cs = U + nA, *Dl = U + nA + nC;
    {
        const float *srcA = fa.A + (size_t)s * a.KAt;
        const float *srcC = a.c2s + (size_t)z * a.L1 * nch * nch;
        const float *srcD = fa.Dpart + (size_t)s * fa.dp_stride;
        constexpr int SPL = (LY::U + 255) / 256;
        float v[SPL];
#pragma unroll
        for (int k = 0; k < SPL; ++k) {
            const int e = min(tid + 256 * k, tot - 1);  // clamped: every load is in bounds
            const float *src =
                e < nA ? srcA + e : (e < nA + nC ? srcC + (e - nA) : srcD + (e - nA - nC));
            v[k] = *src;
        }
        constexpr int TPT = LY::TBL / 256 > 0 ? (LY::TBL + 255) / 256 : 1;
        int tv[TPT];
#pragma unroll
        for (int k = 0; k < TPT; ++k)
            tv[k] = dset[min(tid + 256 * k, ntab - 1)];
#pragma unroll
        for (int k = 0; k < SPL; ++k)
            if (tid + 256 * k < LY::U)
                U[tid + 256 * k] = v[k];
#pragma unroll
        for (int k = 0; k < TPT; ++k)
            if (tid + 256 * k < LY::TBL)
                tbl[tid + 256 * k] = tv[k];
    }
    int pp[4] = {-1, -1, -1, -1};
    if (w == 0) {
        const int nv_all = compact_pairs(pos, n, b, species, a.ns, row, c, S_local, i, a.rc2,
                                         lane, 0, geo, pp);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int slot = lane + 64 * u;
            if (slot < c && pp[u] < 0) {
                gs[slot * 3 + 0] = 0.f;
                gs[slot * 3 + 1] = 0.f;
                gs[slot * 3 + 2] = 0.f;
            }
        }
        if (lane == 0)
            *nvs = nv_all;
    }
    __syncthreads();

    // ---- 2. G = dE/dA and the site energy
    {
        const int *dcols = tbl + L2 + 1;
        double es = 0.0;
        static_assert((16 * MT * 16 * NT) % 256 == 0, "whole elements per thread");
#pragma unroll
        for (int it = 0; it < 16 * MT * 16 * NT / 256; ++it) {
            const int e = tid + 256 * it;
            const int ch = e / (16 * NT), lm = e - ch * (16 * NT);
            float val = 0.f;
            if (ch < nch && lm < L2) {
                int l = (int)sqrtf((float)lm);
                l -= (l * l > lm);
                l += ((l + 1) * (l + 1) <= lm);
                const float c1t = (l == 0) ? a.c1[z * nch + ch] : 0.f;
                float D2 = 0.f, D3 = 0.f;
                if (a.order >= 2) {
                    const float *C = Cs + ((size_t)l * nch + ch) * nch;
                    const float *Al = As + lm * nchp;
                    for (int bb = 0; bb < nch; ++bb)
                        D2 += C[bb] * Al[bb];
                }
                if (a.order >= 3) {
                    constexpr int kPre = 8;
                    const int k0 = tbl[lm], nk = tbl[lm + 1] - k0;
                    const int *cl = dcols + k0;
                    float pv[kPre];
#pragma unroll
                    for (int k = 0; k < kPre; ++k)
                        pv[k] = k < nk ? Dl[cl[k] + ch] : 0.f;
#pragma unroll
                    for (int k = 0; k < kPre; ++k)
                        D3 += pv[k];
                    for (int k = kPre; k < nk; ++k)
                        D3 += Dl[cl[k] + ch];
                }
                val = c1t + 2.f * D2 + 3.f * D3;
                es += (double)(As[lm * nchp + ch] * (c1t + D2 + D3));
            }
            Gt[ch * YW + lm] = val * wgt;
        }
        if (fa.e_exp) {
#pragma unroll
            for (int d = 32; d > 0; d >>= 1)
                es += __shfl_xor(es, d);
            if (lane == 0)
                red[w] = es;
        }
    }
    __syncthreads();  // G ready; the staged tables are free for the pair rows
    if (fa.e_exp && tid == 0)
        fa.e_exp[i] = (double)a.c0[z] + (((red[0] + red[1]) + red[2]) + red[3]);
    const int nv_all = *nvs;

    // this wave's share of the orders |m|
    const int m_lo = w, m_hi = w < 3 ? w : a.lmax;
    for (int rnd = 0; 64 * rnd < nv_all; ++rnd) {
        if (rnd > 0) {
            __syncthreads();  // every wave is done with the last round's geo and S rows
            if (w == 0)
                pairs_round(pos, n, b, species, a.ns, row, i, lane, rnd, pp, geo);
            __syncthreads();
        }
        const int nv = min(64, nv_all - 64 * rnd);
        const int p0 = 16 * w;              // this wave's row tile
        const int nvw = min(16, nv - p0);   // its valid pairs (may be <= 0)
        // ---- 3. rows and the S tile of pairs p0 .. p0 + 15
        if (nvw > 0) {
            if (lane < 16) {
                float *rr = Rr + (p0 + lane) * RW, *dr = Dr + (p0 + lane) * RW;
                for (int ch = 0; ch < 16 * MT; ++ch) {
                    rr[ch] = 0.f;
                    dr[ch] = 0.f;
                }
                if (lane < nvw) {
                    const PairGeo gq = geo[p0 + lane];
                    float R[kMaxNrad], dR[kMaxNrad];
                    radial<float>(nrad, gq.r, a.rc, R, dR);
#pragma unroll
                    for (int k = 0; k < kMaxNrad; ++k)
                        if (k < nrad) {
                            rr[gq.zj * nrad + k] = R[k];
                            dr[gq.zj * nrad + k] = dR[k];
                        }
                }
            }
            wave_sync_ace();
            f4v_t sr[NT], sd[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                sr[nt] = (f4v_t){0.f, 0.f, 0.f, 0.f};
                sd[nt] = (f4v_t){0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
            for (int k0 = 0; k0 < 16 * MT; k0 += 4) {
                const int kc = k0 + kg;
                const float xr = Rr[(p0 + m16) * RW + kc];
                const float xd = Dr[(p0 + m16) * RW + kc];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    const float gb = Gt[kc * YW + nt * 16 + m16];
                    sr[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(xr, gb, sr[nt], 0, 0, 0);
                    sd[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(xd, gb, sd[nt], 0, 0, 0);
                }
            }
            // lane holds S[pair row = p0 + 4 kg + v][lm = 16 nt + m16]
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int sl = p0 + 4 * kg + v, lm = nt * 16 + m16;
                    SR[sl * YW + lm] = sr[nt][v];
                    SD[sl * YW + lm] = sd[nt][v];
                }
        }
        __syncthreads();  // every S row written; the R rows are free for the partial sums
        // ---- 4. this wave's orders for every pair of the round (lane = pair)
        {
            float rad = 0.f, vx = 0.f, vy = 0.f, vz = 0.f;
            if (lane < nv && m_lo <= a.lmax) {
                const PairGeo gq = geo[lane];
                const float *srow = SR + lane * YW, *drow = SD + lane * YW;
                ylm_stream<float>(
                    a.lmax, gq.ux, gq.uy, gq.uz, a.K,
                    [&](int lm, float Y, float yx, float yy, float yz) {
                        const float sR = srow[lm], sD = drow[lm];
                        rad += sD * Y;
                        vx += sR * yx;
                        vy += sR * yy;
                        vz += sR * yz;
                    },
                    m_lo, m_hi);
            }
            float *pw = part + ((size_t)w * 64 + lane) * 4;
            pw[0] = rad;
            pw[1] = vx;
            pw[2] = vy;
            pw[3] = vz;
        }
        __syncthreads();
        // ---- the four partials in wave order, g to the pair's slot (wave w:
        // pairs p0 .. p0 + 15 of the round)
        if (lane < 16 && p0 + lane < nv) {
            const int q = p0 + lane;
            float acc[4];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                acc[k] = part[(size_t)q * 4 + k];
#pragma unroll
            for (int ww = 1; ww < 4; ++ww)
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    acc[k] += part[((size_t)ww * 64 + q) * 4 + k];
            const PairGeo gq = geo[q];
            const float rad = acc[0], vx = acc[1], vy = acc[2], vz = acc[3];
            const float ud = gq.ux * vx + gq.uy * vy + gq.uz * vz;
            gs[gq.slot * 3 + 0] = rad * gq.ux + (vx - gq.ux * ud) * gq.ir;
            gs[gq.slot * 3 + 1] = rad * gq.uy + (vy - gq.uy * ud) * gq.ir;
            gs[gq.slot * 3 + 2] = rad * gq.uz + (vz - gq.uz * ud) * gq.ir;
        }
    }
}

template <int MT, int NT>
static size_t basis_mfma_lds()
{
    return (size_t)64 * (16 * MT + 1 + 16 * NT + 1) * sizeof(float) + 64 * sizeof(PairGeo);
}
template <int MT, int NT>
static size_t pairgrad_mfma_lds()
{
    constexpr int RW = 16 * MT + 1, YW = 16 * NT + 1;
    constexpr int PAIR = 64 * RW * 2 > 64 * YW * 2 ? 64 * RW * 2 : 64 * YW * 2;
    return (size_t)(PAIR + 16 * MT * YW + 64 * 8) * sizeof(float);
}

// Waves per workgroup that keep a workgroup's LDS within 64 KiB.
static int mfma_wpb(size_t per_wave)
{
    int wpb = 4;
    while (wpb > 1 && per_wave * wpb > 64 * 1024)
        wpb >>= 1;
    return wpb;
}

template <int MT, int NT>
static void basis_mfma_launch(hipStream_t s, const Ctx &c, void *ws, const WsLayout &L, const Box &b,
                              const double *pos, const int32_t *species, const AceArgs<float> &a)
{
    // a batched call keeps the whole-row form whatever its total size: the
    // two forms group the pairs differently (different rounding), and a
    // system must give the same bits alone and in any batch
    if (c.basis_chunks > 0 || (c.basis_chunks < 0 && L.n > 65536 && L.nseg == 0)) {
        const size_t per = (size_t)64 * (16 * MT + 1 + 16 * NT + 1) * sizeof(float);
        const int wpb = mfma_wpb(per);
        auto kern = L.nseg > 0 ? k_ace_basis_mfma_chunks<MT, NT, true>
                               : k_ace_basis_mfma_chunks<MT, NT, false>;
        kern<<<(L.n + wpb - 1) / wpb, 64 * wpb, per * wpb, s>>>(
            pos, L.n, b, species, L.cap, at<int>(ws, L.nbr), at<int>(ws, L.cnt),
            at<int>(ws, L.S_idx), at<int>(ws, L.S_local), at<int>(ws, L.hdr), a, wpb,
            at<float>(ws, L.A), seg_args(ws, L));
        return;
    }
    const size_t per = basis_mfma_lds<MT, NT>();
    const int wpb = mfma_wpb(per);
    auto kern = L.nseg > 0 ? k_ace_basis_mfma<MT, NT, true> : k_ace_basis_mfma<MT, NT, false>;
    kern<<<(L.n + wpb - 1) / wpb, 64 * wpb, per * wpb, s>>>(
        pos, L.n, b, species, L.cap, at<int>(ws, L.nbr), at<int>(ws, L.cnt), at<int>(ws, L.S_idx),
        at<int>(ws, L.S_local), at<int>(ws, L.hdr), a, wpb, at<float>(ws, L.A), seg_args(ws, L));
}

template <int MT, int NT>
static void pairgrad_mfma_launch(hipStream_t s, const Ctx &c, void *ws, const WsLayout &L,
                                 const Box &b, const double *pos, const int32_t *species,
                                 const double *weights, const AceArgs<float> &a)
{
    const size_t per = pairgrad_mfma_lds<MT, NT>();
    const int wpb = mfma_wpb(per);
    auto kern = L.nseg > 0 ? k_ace_pairgrad_mfma<MT, NT, true> : k_ace_pairgrad_mfma<MT, NT, false>;
    kern<<<(L.n + wpb - 1) / wpb, 64 * wpb, per * wpb, s>>>(
        pos, L.n, b, species, L.cap, at<int>(ws, L.nbr), at<int>(ws, L.cnt), at<int>(ws, L.S_idx),
        at<int>(ws, L.S_local), at<int>(ws, L.hdr), a, wpb, at<float>(ws, L.dEdA), weights,
        at<float>(ws, L.g), seg_args(ws, L));
}

// The workgroup pair adjoint with the folded finalisation: (channel tiles,
// lm tiles) within its instantiated range and every table within its LDS.
static bool pair_wg_tiles(const Ctx &c, int &mt, int &nt)
{
    mt = (c.m.nchan + 15) / 16;
    nt = (c.m.L2 + 15) / 16;
    if (!(mt >= 1 && mt <= 2 && nt >= 1 && nt <= 3))
        return false;
    int span = 0, ncol = 0;
    for (int k = 0; k < kDSumSets; ++k) {
        span = std::max(span, c.m.dsum_span[k]);
        ncol = std::max(ncol, c.m.dsum_ncol[k]);
    }
    const int nch = c.m.nchan;
    const int tot = c.m.KAt + (c.m.order >= 2 ? (c.m.lmax + 1) * nch * nch : 0) +
                    (c.m.order >= 3 ? span * nch : 0);
    const int u = 64 * (16 * nt + 1) * 2 + 64 * (16 * mt + 1) * 2;
    const int tblcap = ((16 * nt + 1 + 256) + 63) / 64 * 64;
    return tot >= 1 && tot <= u && c.m.L2 + 1 + ncol <= tblcap;
}

template <int MT, int NT>
static void pairgrad_wg_launch(hipStream_t s, const WsLayout &L, const Box &b, const double *pos,
                               const int32_t *species, void *ws, const AceArgs<float> &a,
                               const double *weights, const FinArgs &fin)
{
    const size_t lds = (size_t)PairWgLds<MT, NT, false>::FLOATS * sizeof(float);
    auto kern = L.nseg > 0 ? k_ace_pairgrad_wg<MT, NT, true> : k_ace_pairgrad_wg<MT, NT, false>;
    kern<<<L.n, 256, lds, s>>>(pos, L.n, b, species, L.cap, at<int>(ws, L.nbr), at<int>(ws, L.cnt),
                               at<int>(ws, L.S_idx), at<int>(ws, L.S_local), at<int>(ws, L.hdr), a,
                               weights, at<float>(ws, L.g), seg_args(ws, L), fin);
}

// (channel tiles, lm tiles) of the matrix-core basis / adjoint kernels: 0 if
// the model is outside the instantiated range (then the VALU kernels run).
// The adjoint's S rows take 64 x (16 nt + 1) floats per wave twice: from
// three lm tiles on (lmax >= 5) one wave fits a SIMD and the VALU kernel
// (2.3 KB per wave at lmax 5) measured faster (0.70 vs 1.49 ms on the
// 1,023,800-atom cell).
static int mfma_tiles(const Ctx &c, bool pair, int &mt, int &nt)
{
    mt = (c.m.nchan + 15) / 16;
    nt = (c.m.L2 + 15) / 16;
    if (pair && nt > 2)
        return 0;
    return mt >= 1 && mt <= 2 && nt >= 1 && nt <= 4;
}

// The pair adjoint computes dE/dA itself (the finalisation folded in) in
// the single-precision modes, where the workgroup pair adjoint takes the
// model, for systems whose few S atoms leave the GPU latency-bound (8,193
// atoms: 15.0 against 23.2 us for the one-wave form); large systems keep the
// finalisation kernel and the one-wave adjoint (1,023,800 atoms: 0.69 + 0.43
// against 2.08 ms). A batched call takes the workgroup form whatever its
// size, so that a system gives the same bits alone and in any batch.
bool ace_fin_fused(const Ctx &c, const WsLayout &L)
{
    int mt, nt;
    return c.prec != MLMIX_FP64 && c.basis_mfma && c.fuse_fin && pair_wg_tiles(c, mt, nt) &&
           (L.nseg > 0 || L.n <= 65536);
}

static DSumSel dsum_sel(const Ctx &c, const WsLayout &L, bool fp32)
{
    DSumSel ds;
    ds.tab = reinterpret_cast<const int *>(static_cast<char *>(c.m.base) + c.m.dsum);
    const bool vsets = c.m.order >= 3 && c.m.n_pb > 0 && c.o3 == 1 && c.o3v && fp32;
    for (int k = 0; k < kDSumBlocks; ++k) {
        ds.off[k] = c.m.dsum_off[vsets ? k : kDSumBlocks];
        ds.span[k] = c.m.dsum_span[vsets ? k : kDSumBlocks];
        ds.ncol[k] = c.m.dsum_ncol[vsets ? k : kDSumBlocks];
    }
    ds.grid = vsets ? o3v_grid(c, L.n) : 1;
    ds.max_split = c.o3_max_split;
    return ds;
}

// Dispatch over (channel tiles, lm tiles); false if the model is outside the
// instantiated range (then the VALU kernels run).
template <bool PAIR>
static bool mfma_dispatch(hipStream_t s, const Ctx &c, void *ws, const WsLayout &L, const Box &b,
                          const double *pos, const int32_t *species, const double *weights)
{
    AceArgs<float> a = make_args<float>(c);
    int mt, nt;
    if (!mfma_tiles(c, PAIR, mt, nt))
        return false;
#define O3_GO(M, N)                                                                    \
    if (mt == M && nt == N) {                                                          \
        if (PAIR)                                                                      \
            pairgrad_mfma_launch<M, N>(s, c, ws, L, b, pos, species, weights, a);      \
        else                                                                           \
            basis_mfma_launch<M, N>(s, c, ws, L, b, pos, species, a);                  \
        return true;                                                                   \
    }
    O3_GO(1, 1) O3_GO(1, 2) O3_GO(1, 3) O3_GO(1, 4)
    O3_GO(2, 1) O3_GO(2, 2) O3_GO(2, 3) O3_GO(2, 4)
#undef O3_GO
    return false;
}

template <typename T>
static void basis_t(hipStream_t s, const Ctx &c, void *ws, const WsLayout &L, const Box &b,
                    const double *pos, const int32_t *species)
{
    AceArgs<T> a = make_args<T>(c);
    int n = L.n;
    int wpb = 4;
    while (wpb > 1 && (size_t)wpb * 64 * ((a.nrad + a.L2) * sizeof(T) + sizeof(int)) > 48 * 1024)
        wpb >>= 1;
    size_t sm = (size_t)wpb * 64 * ((a.nrad + a.L2) * sizeof(T) + sizeof(int)) + 16;
    auto kern = L.nseg > 0 ? k_ace_basis<T, true> : k_ace_basis<T, false>;
    kern<<<(n + wpb - 1) / wpb, 64 * wpb, sm, s>>>(
        pos, n, b, species, L.cap, at<int>(ws, L.nbr), at<int>(ws, L.cnt), at<int>(ws, L.S_idx),
        at<int>(ws, L.S_local), at<int>(ws, L.hdr), a, wpb, at<T>(ws, L.A), seg_args(ws, L));
}

// LDS bytes of one order-3 block workgroup of ta atoms.
static size_t blocks_lds(const Ctx &c, int ta, size_t tsz, int stage_w)
{
    const DevModel &m = c.m;
    size_t b = (size_t)ta * m.KAt * tsz;
    b += (size_t)blocks_rows(ta, m.lmax) * blocks_kstride(m.nchan, m.nchp) * tsz;
    if (stage_w)
        b += (size_t)m.nchan * m.nchp * m.nchp * tsz;
    b += (size_t)c.max_ent_pb * (tsz + sizeof(int)) + (2 * m.lmax + 2) * sizeof(int) + 32;
    return b;
}

// Launch shape of the order-3 blocks: MFMA stages for single-species FP32
// models (FP64, the verification precision, and multi-species models keep
// the VALU stages); tile of c.ace_tile atoms (default 4) with the block's
// weights staged in LDS (c.ace_stage_w, default on) — the best of a sweep
// over 1-8 atoms with and without staging on the 8,193-atom workload; the
// tile shrinks until the LDS tile fits 64 KiB.
static void blocks_shape(const Ctx &c, size_t tsz, int &ta, int &mfma, int &stage)
{
    const DevModel &m = c.m;
    mfma = (m.ns == 1 && tsz == 4) ? 1 : 0;
    stage = mfma ? c.ace_stage_w : 0;
    for (ta = c.ace_tile; ta > 1; ta >>= 1)
        if (blocks_lds(c, ta, tsz, stage) <= 64 * 1024)
            break;
    if (blocks_lds(c, ta, tsz, stage) > 64 * 1024)
        stage = 0;
}

template <typename T>
static void contract_t(hipStream_t s, const Ctx &c, void *ws, const WsLayout &L,
                       const int32_t *species)
{
    AceArgs<T> a = make_args<T>(c);
    pb_ranges(c, a.pb_lo, a.pb_hi);
    const int *dp_off = reinterpret_cast<const int *>(static_cast<char *>(c.m.base) + c.m.dpoff);
    T *Dpart = at<T>(ws, L.dpart);
    if (a.order >= 3 && c.m.n_pb > 0 && c.o3 && sizeof(T) == 4) {
        if (c.o3 == 2)
            launch_ace_o3w(s, c, ws, L, species);
        else
            launch_ace_o3(s, c, ws, L);
    } else if (a.order >= 3 && c.m.n_pb > 0) {
        int TA, mf, stage;
        blocks_shape(c, sizeof(T), TA, mf, stage);
        size_t sm = blocks_lds(c, TA, sizeof(T), stage);
        long items = (long)((L.n + TA - 1) / TA) * c.m.n_pb;
        int grid = (int)(items < 8192 ? items : 8192);
        k_ace_blocks<T><<<grid, 256, sm, s>>>(species, at<int>(ws, L.S_idx), at<int>(ws, L.hdr), a,
                                              TA, c.m.n_pb, c.max_ent_pb, mf, stage, dp_off,
                                              c.m.dp_stride, at<T>(ws, L.A), Dpart);
    }
}

template <typename T>
static void finalize_t(hipStream_t s, const Ctx &c, void *ws, const WsLayout &L,
                       const int32_t *species, double *e_exp)
{
    AceArgs<T> a = make_args<T>(c);
    T *Dpart = at<T>(ws, L.dpart);
    const size_t nC = (size_t)c.m.ns * (c.m.lmax + 1) * c.m.nchan * c.m.nchan;
    // the column set of the contraction that wrote the partial D
    const DSumSel ds = dsum_sel(c, L, sizeof(T) == 4);
    // small systems: one atom per workgroup (8,193 atoms: 10.5 against 14.5 us);
    // large: four (1M atoms: 0.55 against 0.99 ms, the staged tables shared)
    // (a batched call keeps one atom per wave whatever its size, so that a
    // system's site energies do not depend on the batch it runs in)
    const int apb = (L.n <= 65536 && L.nseg == 0) ? 1 : 4;
    size_t sm = (size_t)apb * c.m.KAt * sizeof(T) + (size_t)c.m.dsum_len * sizeof(int) + 16;
    int stage_c2 = 0;
    if (sm + nC * sizeof(T) <= 48 * 1024) {
        stage_c2 = 1;
        sm += nC * sizeof(T);
    }
    // the partial-D rows too (their used prefix; the largest of any split),
    // when they fit: every load of the kernel is then issued before its LDS
    // work (1M atoms: 0.43 -> 0.27 ms)
    int span = 0;
    for (int k = 0; k < kDSumBlocks; ++k)
        span = std::max(span, ds.span[k]);
    const size_t dbytes = (size_t)apb * span * c.m.nchan * sizeof(T);
    int stage_d = 0;
    if (c.m.order >= 3 && sm + dbytes <= 48 * 1024) {
        stage_d = 1;
        sm += dbytes;
    }
    if (apb == 1)
        k_ace_finalize<T, 1><<<L.n, 256, sm, s>>>(species, at<int>(ws, L.S_idx), at<int>(ws, L.hdr),
                                                  a, ds, stage_c2, stage_d, c.m.dp_stride,
                                                  at<T>(ws, L.A), Dpart, at<T>(ws, L.dEdA), e_exp);
    else
        k_ace_finalize<T, 4><<<(L.n + 3) / 4, 256, sm, s>>>(
            species, at<int>(ws, L.S_idx), at<int>(ws, L.hdr), a, ds, stage_c2, stage_d,
            c.m.dp_stride, at<T>(ws, L.A), Dpart, at<T>(ws, L.dEdA), e_exp);
}

template <typename T>
static void pairgrad_t(hipStream_t s, const Ctx &c, void *ws, const WsLayout &L, const Box &b,
                       const double *pos, const int32_t *species, const double *weights)
{
    AceArgs<T> a = make_args<T>(c);
    int n = L.n;
    if constexpr (sizeof(T) == 4) {
        if (c.pair_half) {
            // two atoms per wave, four waves per workgroup
            const size_t sm = (size_t)4 * (2 * a.KAt + 2 * L.cap) * sizeof(float);
            auto kern = L.nseg > 0 ? k_ace_pairgrad_h<true> : k_ace_pairgrad_h<false>;
            kern<<<(n + 7) / 8, 256, sm, s>>>(
                pos, n, b, species, L.cap, at<int>(ws, L.nbr), at<int>(ws, L.cnt),
                at<int>(ws, L.S_idx), at<int>(ws, L.S_local), at<int>(ws, L.hdr), a,
                at<float>(ws, L.dEdA), weights, at<float>(ws, L.g), seg_args(ws, L));
            return;
        }
    }
    const int wpb = 4;
    size_t sm = (size_t)wpb * a.KAt * sizeof(T) + 16;
    auto kern = L.nseg > 0 ? k_ace_pairgrad<T, true> : k_ace_pairgrad<T, false>;
    kern<<<(n + wpb - 1) / wpb, 64 * wpb, sm, s>>>(
        pos, n, b, species, L.cap, at<int>(ws, L.nbr), at<int>(ws, L.cnt), at<int>(ws, L.S_idx),
        at<int>(ws, L.S_local), at<int>(ws, L.hdr), a, wpb, at<T>(ws, L.dEdA), weights,
        at<T>(ws, L.g), seg_args(ws, L));
}

void launch_ace_basis(hipStream_t s, const Ctx &c, void *ws, const WsLayout &L, const Box &b,
                      const double *pos, const int32_t *species)
{
    if (L.n == 0)
        return;
    if (c.prec == MLMIX_FP64)
        basis_t<double>(s, c, ws, L, b, pos, species);
    else if (!(c.basis_mfma && mfma_dispatch<false>(s, c, ws, L, b, pos, species, nullptr)))
        basis_t<float>(s, c, ws, L, b, pos, species);
}

void launch_ace_contract(hipStream_t s, const Ctx &c, void *ws, const WsLayout &L,
                         const int32_t *species, hipEvent_t ev0, hipEvent_t ev1)
{
    if (L.n == 0) {
        if (ev0) {  // keep the stage's event pair complete
            (void)hipEventRecord(ev0, s);
            (void)hipEventRecord(ev1, s);
        }
        return;
    }
    if (c.prec != MLMIX_FP64 && c.o3) {
        if (c.o3 == 2)
            launch_ace_o3w(s, c, ws, L, species, ev0, ev1);
        else
            launch_ace_o3(s, c, ws, L, ev0, ev1);
        return;
    }
    if (c.prec == MLMIX_FP64)
        contract_t<double>(s, c, ws, L, species);
    else
        contract_t<float>(s, c, ws, L, species);
}

void launch_ace_finalize(hipStream_t s, const Ctx &c, void *ws, const WsLayout &L,
                         const int32_t *species, double *e_exp)
{
    if (L.n == 0)
        return;
    if (c.prec == MLMIX_FP64)
        finalize_t<double>(s, c, ws, L, species, e_exp);
    else
        finalize_t<float>(s, c, ws, L, species, e_exp);
}

void launch_ace_pairgrad(hipStream_t s, const Ctx &c, void *ws, const WsLayout &L, const Box &b,
                         const double *pos, const int32_t *species, const double *weights,
                         double *e_exp)
{
    if (L.n == 0)
        return;
    if (ace_fin_fused(c, L)) {
        FinArgs fa;
        fa.A = at<float>(ws, L.A);
        fa.Dpart = at<float>(ws, L.dpart);
        fa.dp_stride = c.m.dp_stride;
        fa.ds = dsum_sel(c, L, true);
        fa.e_exp = e_exp;
        const AceArgs<float> a = make_args<float>(c);
        int mt, nt;
        pair_wg_tiles(c, mt, nt);
#define WG_GO(M, N)                                                        \
    if (mt == M && nt == N)                                                \
        pairgrad_wg_launch<M, N>(s, L, b, pos, species, ws, a, weights, fa);
        WG_GO(1, 1) WG_GO(1, 2) WG_GO(1, 3) WG_GO(2, 1) WG_GO(2, 2) WG_GO(2, 3)
#undef WG_GO
    } else if (c.prec == MLMIX_FP64)
        pairgrad_t<double>(s, c, ws, L, b, pos, species, weights);
    else if (!(c.basis_mfma && mfma_dispatch<true>(s, c, ws, L, b, pos, species, weights)))
        pairgrad_t<float>(s, c, ws, L, b, pos, species, weights);
}

}  // namespace mlmix
