// Order-3 product-basis contraction on the matrix cores, for single-species
// models of at most 16 radial channels (ACE-style model; the order-3 term of
// the site energy written as a symmetric cubic form in the atomic basis A,
// block by block over (l1 <= l2, l3) with real Gaunt coefficients).
//
// A workgroup owns a tile of 16 atoms of S and stages their A rows in LDS
// ([atom][lm][16 channels], zero padded). Each of its four waves owns a fixed
// list of work items (m3 row ranges of blocks, balanced on the host) and, for
// every block and m3, one 16-row tile whose rows are the 16 atoms:
//
//  sparse stage  P_t[a][b] = sum_e g_e A_t[l1 m1_e][a] A_t[l2 m2_e][b] for
//                each atom t, as a 16x16 MFMA product whose K runs over the
//                (m1, m2) entries of the row (four per step; padded entries
//                have g = 0). The wave writes P_t into its own LDS rows:
//                with BF16 / FP8 operands in the layout [b / 4][a][b % 4]
//                (a stride: the channels rounded up to a multiple of four),
//                which makes the lanes' writes and the dense stage's reads
//                free of bank conflicts; with FP32 operands (kept in
//                registers first) eight channels a at a time as [a][b].
//  dense stage   D[t][c] = sum_{a,b} P_t[a][b] W[a][b][c] as 16x16 MFMA
//                steps with the block's weights held in registers (one
//                fragment per lane, loaded once per block); with FP32
//                operands the K steps run over exactly the nch^2 pairs
//                (a, b) (lane q holds b = (nch / 4) q + j).
//
// When S holds few tiles, the block lists of one tile are split over G = 2,
// 4 or 8 workgroups (chosen on the device from the size of S, so that the
// grid stays busy); each workgroup stages the tile and runs its bins.
//
// Operand formats: FP32 (16x16x4 steps), BF16 (P and W rounded to nearest
// even, 16x16x32 steps) or FP8 E4M3 (16x16x32 steps; P scaled per row, i.e.
// per (atom, block, m3), by the bound sum|g| max|A_l1| max|A_l2| / 240 on
// |P|, with the maxima over the atom's channels and m; W per (block, c) by
// max|W| / 240). Accumulation is FP32 in every format. The tile's D goes to the
// per-block partial buffer [atom][block offset + m3 * nch + c]; the
// finalize kernel adds the blocks of one l3 in a fixed order, so results do
// not depend on the launch shape.
#include <hip/hip_ext.h>

#include <type_traits>

#include "internal.h"

namespace mlmix {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef __bf16 bf4v __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
typedef int i4v __attribute__((ext_vector_type(4)));

struct O3Args {
    const int *e;         // entries: (packed A-row offsets, coefficient bits) pairs
    const int *mt;        // (first entry, groups of four) per (block, m3)
    const int *mtv;       // (first entry, exact entry count) per (block, m3)
    const int *rowv;      // bins as flat row lists: (first entry, count, block | m3 << 16, D column)
    const int *rbeg;      // per split G: 4 G + 1 offsets (in rows) into rowv
    float *sink;          // 64 floats past the partial-D buffer (masked lanes' stores)
    const float *wr;      // reduced-precision fragments of the vector-sparse form
    const int *base;      // first (block, m3) row of each block
    const float *w;       // weight fragments [block][NC][64][4]
    const float *sw;      // FP8 weight scales [block][16]
    const int *order;     // per split G = 1, 2, 4, 8: the items of bin 0, bin 1, ...
                          // (block | first m3 << 16 | end m3 << 24)
    const int *wbeg;      // per split G: 4 G + 1 bin offsets into order
    const float *gs;      // sum of |g| per (block, m3) (FP8 row-scale bound)
    const int *dp_off;    // per-block offset in the partial buffer
    const PBlock *pb;
    int n_pb, nch, L1, L2, KAt, dp_stride;
    int max_split;  // largest G the kernel may choose (1, 2, 4 or 8)
};

constexpr int kO3MaxGroups = 8;  // entries of one (block, m3) row: at most 4 x 8

// bytes of one P row per format (16-byte pad keeps rows 4 banks apart); the
// FP32 rows hold eight channels a at a time, each with its nc values of b
__host__ __device__ constexpr int o3_row_bytes(int qm, int nc)
{
    return qm == 0 ? 4 * (nc < 8 ? nc : 8) * nc + 16 : 4 * nc * 4 * (qm == 1 ? 2 : 1) + 16;
}

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// this lane's (offsets, coefficient) of the four-entry groups of one row;
// all eight groups are read (the table is padded past its end), so the loads
// stay in flight while the previous row is computed
__device__ __forceinline__ void o3_load_row(const int *__restrict__ e, int e0, int q,
                                            int2 (&ent)[kO3MaxGroups])
{
    const int2 *src = reinterpret_cast<const int2 *>(e) + e0 + q;
#pragma unroll
    for (int k = 0; k < kO3MaxGroups; ++k)
        ent[k] = src[4 * k];
}

// FP32 sparse stage of one row: the 16 atoms' 16x16 tiles P_t[a = m][b =
// 4 q + v] stay in registers (cc[t]); the dense stage then stages them half a
// channel range at a time.
template <int NG>
__device__ __forceinline__ void o3_sparse_regs(const float *__restrict__ At, int L2, int m,
                                               const int2 (&ent)[kO3MaxGroups], f4v (&cc)[kO3Atoms])
{
#pragma unroll
    for (int t = 0; t < kO3Atoms; t += 4) {
        const float *A0 = At + (size_t)t * L2 * 16 + m;
#pragma unroll
        for (int u = 0; u < 4; ++u)
            cc[t + u] = (f4v){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < NG; ++k) {
            const int o1 = ent[k].x & 0xffff, o2 = ent[k].x >> 16;
            const float g = __int_as_float(ent[k].y);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float *Au = A0 + u * L2 * 16;
                cc[t + u] = __builtin_amdgcn_mfma_f32_16x16x4f32(Au[o2], g * Au[o1], cc[t + u], 0, 0, 0);
            }
        }
    }
}

// Sparse stage of one row for the 16 atoms with NG entry groups (unrolled):
// P_t[a = m][b = 4 q + v] accumulates on the matrix cores and is written to
// the wave's P rows in the operand format.
template <int QM, int NC, int NG>
__device__ __forceinline__ void o3_sparse(const float *__restrict__ At, int L2, int L1, int m,
                                          int q, int lane, const int2 (&ent)[kO3MaxGroups],
                                          char *Pw, float *sP, const float *amax, int l1, int l2,
                                          float gsum)
{
    constexpr int rowb = o3_row_bytes(QM, NC);
    for (int t = 0; t < kO3Atoms; t += 4) {
        const float *A0 = At + (size_t)t * L2 * 16 + m;
        f4v c[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            c[u] = (f4v){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < NG; ++k) {
            const int o1 = ent[k].x & 0xffff, o2 = ent[k].x >> 16;
            const float g = __int_as_float(ent[k].y);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float *Au = A0 + u * L2 * 16;
                c[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(Au[o2], g * Au[o1], c[u], 0, 0, 0);
            }
        }
        // lane holds P[a = m][b = 4 q + v]; chunk (b / 4 = q, a = m)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const f4v cv = c[u];
            char *dst = Pw + (size_t)(t + u) * rowb;
            if constexpr (QM == 0) {
                if (m < NC)
                    *reinterpret_cast<f4v *>(dst + (q * NC + m) * 16) = cv;
            } else if constexpr (QM == 1) {
                const bf2v p0 = __builtin_convertvector((f2v){cv[0], cv[1]}, bf2v);
                const bf2v p1 = __builtin_convertvector((f2v){cv[2], cv[3]}, bf2v);
                if (m < NC)
                    *reinterpret_cast<bf4v *>(dst + (q * NC + m) * 8) = (bf4v){p0[0], p0[1], p1[0], p1[1]};
            } else {
                const float *am = amax + (t + u) * L1;
                const float sc = gsum * am[l1] * am[l2];  // >= max|P| / 240
                const float inv = sc > 0.0f ? 1.0f / sc : 0.0f;
                int pk = __builtin_amdgcn_cvt_pk_fp8_f32(cv[0] * inv, cv[1] * inv, 0, false);
                pk = __builtin_amdgcn_cvt_pk_fp8_f32(cv[2] * inv, cv[3] * inv, pk, true);
                if (m < NC)
                    *reinterpret_cast<int *>(dst + (q * NC + m) * 4) = pk;
                if (lane == 0)
                    sP[t + u] = sc;
            }
        }
    }
}

template <int QM, int NC, int NW>  // NW waves per workgroup (4 or 8)
__global__ void __launch_bounds__(64 * NW, NW == 4 ? 2 : 1)
    k_ace_o3(const int *__restrict__ hdr, O3Args a, const float *__restrict__ A,
             float *__restrict__ Dpart)
{
    constexpr int NTH = 64 * NW;
    const int nS = hdr[H_NS];
    const int ntile = (nS + kO3Atoms - 1) / kO3Atoms;
    int G = 1, lg = 0;
    while (G < a.max_split && ntile * G < (int)gridDim.x) {
        G <<= 1;
        ++lg;
    }
    const int nitem = ntile * G;
    if ((int)blockIdx.x >= nitem)
        return;  // uniform across the workgroup
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int m = lane & 15, q = lane >> 4;
    const int nch = a.nch, L2 = a.L2, L1 = a.L1;
    constexpr int rowb = o3_row_bytes(QM, NC);
    extern __shared__ __align__(16) char smem_raw[];
    float *At = reinterpret_cast<float *>(smem_raw);  // [16][L2][16]
    char *Pw = smem_raw + (size_t)kO3Atoms * L2 * 16 * sizeof(float) + (size_t)wv * kO3Atoms * rowb;
    float *sPall = reinterpret_cast<float *>(smem_raw + (size_t)kO3Atoms * L2 * 16 * sizeof(float) +
                                             (size_t)NW * kO3Atoms * rowb);
    float *sP = sPall + wv * kO3Atoms;
    float *amax = sPall + NW * kO3Atoms;  // [16][L1]: max |A| per atom and l (FP8)
    const int *order = a.order;
    // bin offsets of the split G: the tables of G' = 1, 2, .. G / 2 come first
    const int *wbeg = a.wbeg + NW * (G - 1) + lg;

    for (int item = blockIdx.x; item < nitem; item += gridDim.x) {
        const int tile = item >> lg, bin = (item & (G - 1)) * NW + wv;
        const int w_lo = wbeg[bin], w_hi = wbeg[bin + 1];
        const int s0 = tile * kO3Atoms;
        const int na = min(kO3Atoms, nS - s0);
        __syncthreads();  // every wave is done with the previous tile's A
        // stage the tile's A rows (NC channels in HBM, 16 in LDS, zero padded)
        for (int r = tid; r < kO3Atoms * L2; r += NTH) {
            const int t = r / L2, lm = r - t * L2;
            f4v *dst = reinterpret_cast<f4v *>(At + (size_t)r * 16);
            const f4v *src = reinterpret_cast<const f4v *>(A + (size_t)(s0 + t) * a.KAt + lm * NC);
#pragma unroll
            for (int c4 = 0; c4 < 4; ++c4)
                dst[c4] = (c4 < NC / 4 && t < na) ? src[c4] : (f4v){0.f, 0.f, 0.f, 0.f};
        }
        __syncthreads();
        if constexpr (QM == 2) {
            if (tid < kO3Atoms * L1) {
                const int t = tid / L1, l = tid - t * L1;
                const f4v *row = reinterpret_cast<const f4v *>(At + ((size_t)t * L2 + l * l) * 16);
                float mx = 0.0f;
                for (int k = 0; k < (2 * l + 1) * 4; ++k) {
                    const f4v v = row[k];
                    mx = fmaxf(mx, fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fmaxf(fabsf(v[2]), fabsf(v[3]))));
                }
                amax[t * L1 + l] = mx;
            }
            __syncthreads();
        }

        for (int wi = w_lo; wi < w_hi; ++wi) {
            const int code = order[wi];
            const int p = code & 0xffff, m3lo = (code >> 16) & 0xff, m3hi = (code >> 24) & 0xff;
            const PBlock pbk = a.pb[p];
            const int rbase = a.base[p];
            // weight fragments of this lane: element 4 i + j <-> (a = i, b = 4 q + j, c = m)
            f4v wf[NC];
            const f4v *wsrc = reinterpret_cast<const f4v *>(a.w) + (size_t)p * NC * 64 + lane;
#pragma unroll
            for (int i = 0; i < NC; ++i)
                wf[i] = wsrc[i * 64];
            bf8v wb[NC / 2];
            long w8[NC / 2];
            if constexpr (QM == 1) {
#pragma unroll
                for (int i = 0; i < NC / 2; ++i) {
                    const f4v x = wf[2 * i], y = wf[2 * i + 1];
                    const bf2v p0 = __builtin_convertvector((f2v){x[0], x[1]}, bf2v);
                    const bf2v p1 = __builtin_convertvector((f2v){x[2], x[3]}, bf2v);
                    const bf2v p2 = __builtin_convertvector((f2v){y[0], y[1]}, bf2v);
                    const bf2v p3 = __builtin_convertvector((f2v){y[2], y[3]}, bf2v);
                    wb[i] = (bf8v){p0[0], p0[1], p1[0], p1[1], p2[0], p2[1], p3[0], p3[1]};
                }
            } else if constexpr (QM == 2) {
#pragma unroll
                for (int i = 0; i < NC / 2; ++i) {
                    const f4v x = wf[2 * i], y = wf[2 * i + 1];
                    int lo = __builtin_amdgcn_cvt_pk_fp8_f32(x[0], x[1], 0, false);
                    lo = __builtin_amdgcn_cvt_pk_fp8_f32(x[2], x[3], lo, true);
                    int hi = __builtin_amdgcn_cvt_pk_fp8_f32(y[0], y[1], 0, false);
                    hi = __builtin_amdgcn_cvt_pk_fp8_f32(y[2], y[3], hi, true);
                    w8[i] = (long)(((unsigned long)(unsigned)hi << 32) | (unsigned)lo);
                }
            }
            const float swc = QM == 2 ? a.sw[p * 16 + m] : 1.0f;
            float *Dblk = Dpart + a.dp_off[p];

            // entries of the first row; each row prefetches the next one's
            int2 ent[kO3MaxGroups], ent_n[kO3MaxGroups];
            int e0 = a.mt[2 * (rbase + m3lo)], ng = a.mt[2 * (rbase + m3lo) + 1];
            o3_load_row(a.e, e0, q, ent);
            for (int m3 = m3lo; m3 < m3hi; ++m3) {
                const int row = rbase + m3;
                int ngn = 0;
                if (m3 + 1 < m3hi) {
                    ngn = a.mt[2 * row + 3];
                    o3_load_row(a.e, a.mt[2 * row + 2], q, ent_n);
                }
                f4v acc = {0.f, 0.f, 0.f, 0.f};
                const char *Prow = Pw + (size_t)m * rowb;
                if constexpr (QM == 0) {
                    // ---- sparse stage into registers, then the dense stage
                    // in passes of HW = min(NC, 8) channels a
                    f4v cc[kO3Atoms];
#define O3_SPARSE(NGV) o3_sparse_regs<NGV>(At, L2, m, ent, cc)
                    switch (ng) {
                    case 0: O3_SPARSE(0); break;
                    case 1: O3_SPARSE(1); break;
                    case 2: O3_SPARSE(2); break;
                    case 3: O3_SPARSE(3); break;
                    case 4: O3_SPARSE(4); break;
                    case 5: O3_SPARSE(5); break;
                    case 6: O3_SPARSE(6); break;
                    case 7: O3_SPARSE(7); break;
                    default: O3_SPARSE(8); break;
                    }
#undef O3_SPARSE
                    // dense stage, eight channels a at a time: P rows
                    // [a - a0][b] (b contiguous); lane (atom m, q) takes the
                    // NJ = NC / 4 values b = NJ q + j, so K runs over exactly
                    // NC^2 values (a, b), against weights W[a][NJ q + j][c = m]
                    constexpr int NJ = NC / 4;
#pragma unroll
                    for (int a0 = 0; a0 < NC; a0 += 8) {
                        constexpr int HW = NC < 8 ? NC : 8;
                        const int hw = NC - a0 < HW ? NC - a0 : HW;
                        if (m >= a0 && m < a0 + hw && 4 * q < NC)
#pragma unroll
                            for (int t = 0; t < kO3Atoms; ++t)
                                *reinterpret_cast<f4v *>(Pw + (size_t)t * rowb +
                                                         ((m - a0) * NC + 4 * q) * 4) = cc[t];
                        wave_sync_lds();
#pragma unroll
                        for (int i = 0; i < HW; ++i)
                            if (i < hw) {
                                const float *pr =
                                    reinterpret_cast<const float *>(Prow) + i * NC + NJ * q;
                                float pv[NJ];
#pragma unroll
                                for (int j = 0; j < NJ; ++j)
                                    pv[j] = pr[j];
#pragma unroll
                                for (int j = 0; j < NJ; ++j)
                                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(pv[j], wf[a0 + i][j],
                                                                               acc, 0, 0, 0);
                            }
                        wave_sync_lds();  // the next pass overwrites the rows
                    }
                } else {
                    const float gsum = QM == 2 ? a.gs[row] * (1.0f / 240.0f) : 0.0f;
                    // ---- sparse stage: P_t for the 16 atoms, four at a time
#define O3_SPARSE(NGV)                                                                        \
    o3_sparse<QM, NC, NGV>(At, L2, L1, m, q, lane, ent, Pw, sP, amax, pbk.l1, pbk.l2, gsum)
                    switch (ng) {
                    case 0: O3_SPARSE(0); break;
                    case 1: O3_SPARSE(1); break;
                    case 2: O3_SPARSE(2); break;
                    case 3: O3_SPARSE(3); break;
                    case 4: O3_SPARSE(4); break;
                    case 5: O3_SPARSE(5); break;
                    case 6: O3_SPARSE(6); break;
                    case 7: O3_SPARSE(7); break;
                    default: O3_SPARSE(8); break;
                    }
#undef O3_SPARSE
                    wave_sync_lds();
                    // ---- dense stage: D[atom m-row][c] over the 16 atoms
                    if constexpr (QM == 1) {
#pragma unroll
                        for (int i = 0; i < NC / 2; ++i) {
                            const bf8v pv = *reinterpret_cast<const bf8v *>(Prow + (q * NC + 2 * i) * 8);
                            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pv, wb[i], acc, 0, 0, 0);
                        }
                    } else {
#pragma unroll
                        for (int i = 0; i < NC / 2; ++i) {
                            const long pv = *reinterpret_cast<const long *>(Prow + (q * NC + 2 * i) * 4);
                            acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(pv, w8[i], acc, 0, 0, 0);
                        }
                    }
                }
                // lane holds D[atom = 4 q + v][c = m]
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int t = 4 * q + v;
                    float dv = acc[v];
                    if constexpr (QM == 2)
                        dv *= sP[t] * swc;
                    if (t < na && m < nch)
                        Dblk[(size_t)(s0 + t) * a.dp_stride + m3 * nch + m] = dv;
                }
                wave_sync_lds();  // P rows and scales are rewritten by the next m3
#pragma unroll
                for (int k = 0; k < kO3MaxGroups; ++k)
                    ent[k] = ent_n[k];
                ng = ngn;
            }
        }
    }
}

// ------------------------------------------------------ VALU sparse form
//
// The single-species contraction used by default (every operand format): the same
// tiles of 16 atoms and the same partial-D output, the work of a tile split
// into per-wave bins of rows (block, m3) listed flat by the host, and the
// sparse stage on the vector ALUs, leaving P directly in the registers the
// dense stage reads (no P round trip through LDS, no wave barrier):
//
//  lane (t = atom, q):  P_t[a][NJ q + j] for every channel a and j < NJ =
//                       nchp / 4 (NJ * nchp accumulators), summed over the
//                       row's Gaunt entries e as g_e A_t[l1 m1_e][a]
//                       A_t[l2 m2_e][NJ q + j]; the entries are
//                       wave-uniform (one vector load per row, a row ahead,
//                       read back lane by lane) and the A values of entry
//                       e + 1 are read from LDS while entry e is accumulated;
//  dense stage:         D[t][c] = sum_{a, j} P_t[a][NJ q + j]
//                       W[a][NJ q + j][c], two accumulators in a fixed
//                       alternation: FP32 as nchp * NJ 16x16x4 MFMA steps
//                       (K over exactly nchp^2 pairs); BF16 / FP8 as
//                       nchp / A_PER 16x16x32 steps, step s taking the
//                       channels a = A_PER s .. A_PER (s + 1) - 1 (A_PER =
//                       min(8 / NJ, nchp)): lane (t, q) packs its values
//                       P_t[a][NJ q + j] of those channels (zero padded to
//                       eight), rounded to nearest even; FP8 E4M3 divides
//                       them by the atom's scale max |P_t| / 240 over the
//                       row (the four lanes of the atom compare theirs) and
//                       the weights by the per-(block, c) scale max |W| / 240,
//                       and multiplies both back into D.
//
// Two or three waves per SIMD: the vector sparse stage of one runs beside
// the matrix-core dense stage of another. (Interleaving the dense steps of a
// row with the next row's vector work inside one wave needs P and the
// weights twice in registers: one wave per SIMD at 16 channels, measured
// slower, 4.4 against 3.3 ms on 102,858 atoms in S, and no faster at 12.)
template <int QM, int NC, int NW, int BPW>  // BPW bins of the eight-wave table per wave
__global__ void __launch_bounds__(64 * NW, NC <= 12 ? 3 : 2)
    k_ace_o3v(const int *__restrict__ hdr, O3Args a, const float *__restrict__ A,
              float *__restrict__ Dpart)
{
#pragma clang fp contract(off)
    constexpr int NTH = 64 * NW, NJ = NC / 4;
    constexpr int APER = 8 / NJ < NC ? 8 / NJ : NC;  // channels a per 32-deep step
    constexpr int NST = NC / APER;                   // 32-deep steps (BF16 / FP8)
    const int nS = hdr[H_NS];
    const int ntile = (nS + kO3Atoms - 1) / kO3Atoms;
    int G = 1, lg = 0;
    while (G < a.max_split && ntile * G < (int)gridDim.x) {
        G <<= 1;
        ++lg;
    }
    const int nitem = ntile * G;
    // the splits of one tile on one XCD: its A rows come from that XCD's L2
    // after the first fetch
    const int vb = xcd_major(blockIdx.x, gridDim.x);
    if (vb >= nitem)
        return;  // uniform across the workgroup
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int m = lane & 15, q = lane >> 4;
    const int nch = a.nch, L2 = a.L2;
    const int astr = L2 * 16 + 4;  // LDS floats per atom
    extern __shared__ __align__(16) char smem_raw[];
    float *At = reinterpret_cast<float *>(smem_raw);  // [16][astr]
    const float *At_t = At + (size_t)m * astr;       // this lane's atom (t = m)
    const int *rbeg = a.rbeg + NW * BPW * (G - 1) + lg;  // the table's bins: NW BPW per split
    const int2 *etab = reinterpret_cast<const int2 *>(a.e);
    const int4 *rows = reinterpret_cast<const int4 *>(a.rowv);

    float P[NC][NJ];
    float wf[QM == 0 ? NC : 1][NJ];  // FP32 weight fragments
    bf8v wb[QM == 1 ? NST : 1];      // BF16 weight fragments
    long w8[QM == 2 ? NST : 1];      // FP8 weight fragments
    float swc = 1.0f;                // FP8 weight scale of column c = m
    f4v acc0, acc1;
    f4v a1[2][NC / 4];
    float a2[2][NJ];

    for (int item = vb; item < nitem; item += gridDim.x)
    for (int bb = 0; bb < BPW; ++bb) {  // the wave's bins of this item, in order
        const int tile = item >> lg, bin = ((item & (G - 1)) * NW + wv) * BPW + bb;
        const int r_lo = rbeg[bin], nr = rbeg[bin + 1] - r_lo;  // nr <= 128 (host check)
        const int s0 = tile * kO3Atoms;
        const int na = min(kO3Atoms, nS - s0);
        // the bin's row records, two per lane (rows lane and 64 + lane)
        int4 rec0 = make_int4(0, 0, 0, 0), rec1 = make_int4(0, 0, 0, 0);
        if (lane < nr)
            rec0 = rows[r_lo + lane];
        if (64 + lane < nr)
            rec1 = rows[r_lo + 64 + lane];
        // field f of row k's record (wave-uniform)
        auto field = [&](int k, int f) -> int {
            const int4 &rc = k < 64 ? rec0 : rec1;
            const int v = f == 0 ? rc.x : (f == 1 ? rc.y : (f == 2 ? rc.z : rc.w));
            return __builtin_amdgcn_readlane(v, k & 63);
        };
        // a row's entries, one per lane: every lane loads (the table is padded
        // by 32 entries past its end); lanes at or past the count are zeroed
        // where the row starts (not here: that would wait for the load)
        auto entries = [&](int k, int &ne) -> int2 {
            ne = field(k, 1);
            return etab[field(k, 0) + min(lane, 31)];
        };
        int pcur = -1;
        // weight fragments of block p: lane (c = m, q) holds W[a = i][NJ q + j][c]
        // (FP32), or the eight values of each 32-deep step (BF16 / FP8)
        auto weights = [&](int p) {
            if constexpr (QM == 0) {
                const float *wsrc = a.w + ((size_t)p * NC * 64 + lane) * 4;
#pragma unroll
                for (int i = 0; i < NC; ++i)
#pragma unroll
                    for (int j = 0; j < NJ; ++j)
                        wf[i][j] = wsrc[i * 256 + j];
            } else {
                const f4v *wsrc = reinterpret_cast<const f4v *>(a.wr) + ((size_t)p * NST * 64 + lane) * 2;
#pragma unroll
                for (int st = 0; st < NST; ++st) {
                    const f4v x = wsrc[st * 128], y = wsrc[st * 128 + 1];
                    if constexpr (QM == 1) {
                        const bf2v p0 = __builtin_convertvector((f2v){x[0], x[1]}, bf2v);
                        const bf2v p1 = __builtin_convertvector((f2v){x[2], x[3]}, bf2v);
                        const bf2v p2 = __builtin_convertvector((f2v){y[0], y[1]}, bf2v);
                        const bf2v p3 = __builtin_convertvector((f2v){y[2], y[3]}, bf2v);
                        wb[st] = (bf8v){p0[0], p0[1], p1[0], p1[1], p2[0], p2[1], p3[0], p3[1]};
                    } else {
                        int lo = __builtin_amdgcn_cvt_pk_fp8_f32(x[0], x[1], 0, false);
                        lo = __builtin_amdgcn_cvt_pk_fp8_f32(x[2], x[3], lo, true);
                        int hi = __builtin_amdgcn_cvt_pk_fp8_f32(y[0], y[1], 0, false);
                        hi = __builtin_amdgcn_cvt_pk_fp8_f32(y[2], y[3], hi, true);
                        w8[st] = (long)(((unsigned long)(unsigned)hi << 32) | (unsigned)lo);
                    }
                }
                if constexpr (QM == 2)
                    swc = a.sw[p * 16 + m];
            }
            pcur = p;
        };
        // entries of the current and the next row alternate between two
        // register sets by row parity (a copy of a loaded register would make
        // the wave wait for the load where it is issued); the first row's
        // entries and weights are read while the tile's A rows are staged
        int neE[2] = {0, 0};
        int2 entE[2];
        if (nr > 0) {
            weights(field(0, 2) & 0xffff);
            entE[0] = entries(0, neE[0]);
        }
        if (bb == 0) {  // the tile's A rows, once per item (bb is uniform)
            __syncthreads();  // every wave is done with the previous tile's A
            for (int r = tid; r < kO3Atoms * L2; r += NTH) {
                const int t = r / L2, lm = r - t * L2;
                f4v *dst = reinterpret_cast<f4v *>(At + (size_t)t * astr + lm * 16);
                const f4v *src = reinterpret_cast<const f4v *>(A + (size_t)(s0 + t) * a.KAt + lm * NC);
#pragma unroll
                for (int c4 = 0; c4 < NC / 4; ++c4)
                    dst[c4] = t < na ? src[c4] : (f4v){0.f, 0.f, 0.f, 0.f};
            }
            __syncthreads();
        }

        // D of the last row: lane holds D[atom = 4 q + v][c = m]; lanes
        // outside the tile or the channels (and every lane before the first
        // row) write to a sink past the buffer's end, so that the stores need
        // no branch
        int dcol = 0;
        float psc = 1.0f;  // FP8: this lane's atom scale of the last row
        auto store_d = [&](bool real) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int t = 4 * q + v;
                float d = acc0[v] + acc1[v];
                if constexpr (QM == 2)
                    d = d * (__shfl(psc, t) * swc);  // atom t's scale sits in lane t
                float *dst = (real && t < na && m < nch)
                                 ? Dpart + (size_t)(s0 + t) * a.dp_stride + dcol + m
                                 : a.sink + lane;
                *dst = d;
            }
        };
        acc0 = (f4v){0.f, 0.f, 0.f, 0.f};
        acc1 = (f4v){0.f, 0.f, 0.f, 0.f};

        // row k (entries in set H): its P on the vector ALUs, its D on the
        // matrix cores (stored at the start of the next row, after that
        // row's wait for its entries, so that the wait does not also wait
        // for the stores)
        auto row = [&](int k, auto hc) {
            constexpr int H = decltype(hc)::value;
            const int ne = neE[H];
            const int2 ent = lane < ne ? entE[H] : make_int2(0, 0);
            const int ox0 = __builtin_amdgcn_readlane(ent.x, 0);
            __builtin_amdgcn_sched_barrier(0);
            // a row whose column differs from the last row's opens a run: the
            // last run's D is stored and the accumulators start from zero
            // (FP8: every row is its own run, each with its own scale)
            const int col = field(k, 3);
            const bool fresh = QM == 2 || k == 0 || col != dcol;
            if (fresh)
                store_d(k > 0);
            const int p = field(k, 2) & 0xffff;
            dcol = col;
            // the block's weights (read while the sparse stage runs), then the
            // next row's entries (a valid row past the end is read and not
            // used)
            if (p != pcur)
                weights(p);
            entE[H ^ 1] = entries(min(k + 1, nr - 1), neE[H ^ 1]);

            // A values of entry e into register set h (entry lanes past the
            // count hold zero offsets: in-bounds reads whose values are not
            // used)
            auto load = [&](int e, int h) {
                const int ox = e == 0 ? ox0 : __builtin_amdgcn_readlane(ent.x, e);
                const f4v *r1 = reinterpret_cast<const f4v *>(At_t + (ox & 0xffff));
                const float *r2 = At_t + (ox >> 16) + NJ * q;
#pragma unroll
                for (int k4 = 0; k4 < NC / 4; ++k4)
                    a1[h][k4] = r1[k4];
                if constexpr (NJ == 4) {
                    const f4v v = *reinterpret_cast<const f4v *>(r2);
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        a2[h][j] = v[j];
                } else {
#pragma unroll
                    for (int j = 0; j < NJ; ++j)
                        a2[h][j] = r2[j];
                }
            };
            auto accumulate = [&](int e, int h, bool first) {
                const float g = __int_as_float(__builtin_amdgcn_readlane(ent.y, e));
                float b[NJ];
#pragma unroll
                for (int j = 0; j < NJ; ++j)
                    b[j] = g * a2[h][j];
#pragma unroll
                for (int i = 0; i < NC; ++i)
#pragma unroll
                    for (int j = 0; j < NJ; ++j)
                        P[i][j] = first ? a1[h][i / 4][i % 4] * b[j]
                                        : fmaf(a1[h][i / 4][i % 4], b[j], P[i][j]);
            };
            // ---- sparse stage: two register sets, each load one entry ahead
            // (scheduling barriers keep it ahead of the other set's
            // arithmetic: the scheduler would sink it to its use). Every row
            // has at least one entry (host check).
            load(0, 0);
            load(1, 1);
            __builtin_amdgcn_sched_barrier(0);
            accumulate(0, 0, true);
            for (int e = 1; e < ne; e += 2) {
                load(e + 1, 0);
                __builtin_amdgcn_sched_barrier(0);
                accumulate(e, 1, false);
                if (e + 1 >= ne)
                    break;
                load(e + 2, 1);
                __builtin_amdgcn_sched_barrier(0);
                accumulate(e + 1, 0, false);
            }
            // ---- dense stage (matrix cores): lane (t = m, q) supplies
            // P_t[i][NJ q + j], lane (c = m, q) the weight W[i][NJ q + j][c]
            if (fresh) {
                acc0 = (f4v){0.f, 0.f, 0.f, 0.f};
                acc1 = (f4v){0.f, 0.f, 0.f, 0.f};
            }
            if constexpr (QM == 0) {
#pragma unroll
                for (int i = 0; i < NC; ++i)
#pragma unroll
                    for (int j = 0; j < NJ; ++j) {
                        if (((i * NJ + j) & 1) == 0)
                            acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(P[i][j], wf[i][j], acc0, 0, 0, 0);
                        else
                            acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(P[i][j], wf[i][j], acc1, 0, 0, 0);
                    }
            } else {
                // eight values of step st: u < APER NJ -> P[APER st + u / NJ][u % NJ]
                auto val = [&](int st, int u, float sc) -> float {
                    return u < APER * NJ ? P[APER * st + u / NJ][u % NJ] * sc : 0.0f;
                };
                float inv = 1.0f;
                if constexpr (QM == 2) {
                    // the atom's scale: max |P_t| over its four lanes
                    float mx = 0.0f;
#pragma unroll
                    for (int i = 0; i < NC; ++i)
#pragma unroll
                        for (int j = 0; j < NJ; ++j)
                            mx = fmaxf(mx, fabsf(P[i][j]));
                    mx = fmaxf(mx, __shfl_xor(mx, 16));
                    mx = fmaxf(mx, __shfl_xor(mx, 32));
                    psc = mx * (1.0f / 240.0f);
                    inv = psc > 0.0f ? 1.0f / psc : 0.0f;
                }
#pragma unroll
                for (int st = 0; st < NST; ++st) {
                    f4v r;
                    if constexpr (QM == 1) {
                        const bf2v p0 = __builtin_convertvector((f2v){val(st, 0, 1.f), val(st, 1, 1.f)}, bf2v);
                        const bf2v p1 = __builtin_convertvector((f2v){val(st, 2, 1.f), val(st, 3, 1.f)}, bf2v);
                        const bf2v p2 = __builtin_convertvector((f2v){val(st, 4, 1.f), val(st, 5, 1.f)}, bf2v);
                        const bf2v p3 = __builtin_convertvector((f2v){val(st, 6, 1.f), val(st, 7, 1.f)}, bf2v);
                        const bf8v pv = {p0[0], p0[1], p1[0], p1[1], p2[0], p2[1], p3[0], p3[1]};
                        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pv, wb[st], (st & 1) ? acc1 : acc0, 0, 0, 0);
                    } else {
                        int lo = __builtin_amdgcn_cvt_pk_fp8_f32(val(st, 0, inv), val(st, 1, inv), 0, false);
                        lo = __builtin_amdgcn_cvt_pk_fp8_f32(val(st, 2, inv), val(st, 3, inv), lo, true);
                        int hi = __builtin_amdgcn_cvt_pk_fp8_f32(val(st, 4, inv), val(st, 5, inv), 0, false);
                        hi = __builtin_amdgcn_cvt_pk_fp8_f32(val(st, 6, inv), val(st, 7, inv), hi, true);
                        const long pv = (long)(((unsigned long)(unsigned)hi << 32) | (unsigned)lo);
                        r = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(pv, w8[st], (st & 1) ? acc1 : acc0, 0, 0, 0);
                    }
                    if (st & 1)
                        acc1 = r;
                    else
                        acc0 = r;
                }
            }
        };
        for (int k = 0; k < nr; k += 2) {
            row(k, std::integral_constant<int, 0>());
            if (k + 1 >= nr)
                break;
            row(k + 1, std::integral_constant<int, 1>());
        }
        if (nr > 0)
            store_d(true);
    }
}

// grid of the vector-sparse contraction over a capacity of n S atoms: as
// many resident workgroups as the registers allow (waves per SIMD: three up
// to 12 channels, else two), at most one per (tile, split) item
// waves per workgroup of the vector-sparse contraction for a capacity of n
// S atoms: eight by default; large systems run four-wave workgroups that
// take the eight-wave table's bins two per wave (more, smaller workgroups
// balance the many tiles better)
int o3v_waves(const Ctx &c, int n)
{
    return c.o3_waves == 8 && n > kO3FourWaveMin ? 4 : c.o3_waves;
}

int o3v_grid(const Ctx &c, int n)
{
    const long items = (((long)n + kO3Atoms - 1) / kO3Atoms) * kO3MaxSplit;
    const int nw = o3v_waves(c, n) == 8 ? 8 : 4;
    const int per_cu = std::max(1, 4 * (c.m.nchp <= 12 ? 3 : 2) / nw);
    return (int)std::min<long>(std::max<long>(items, 1), 256L * per_cu);
}

size_t o3v_lds_bytes(const Ctx &c)
{
    return (size_t)kO3Atoms * (c.m.L2 * 16 + 4) * sizeof(float);
}

// ------------------------------------------------------------- wide form
//
// The same contraction for FP32 models of any number of species and at most
// 32 channels (channels a = species of the neighbour x radial function):
// the same tiles of 16 atoms, work items, bins and per-block partial D; the
// channel dimensions take NT = ceil(channels / 16) tiles of 16.
//
//  sparse stage  for each channel tile ta of a, every tile tb of b:
//                P_t[a][b] as 16x16 MFMA products over the row's Gaunt
//                entries (the atoms' A rows in LDS 16 NT channels apart,
//                zero padded), all 16 atoms' tiles in registers;
//  dense stage   eight channels a at a time through LDS: lane (atom m, q)
//                reads P_m[a][NJ q + j], j < NJ = nchp / 4, so the MFMA K
//                runs over exactly nchp^2 values (a, b), against weight
//                fragments W_z[a][NJ q + j][16 ct + m] read through the cache
//                (one set per centre species z and channel tile ct of c).
//                A tile whose atoms are of several species runs the dense
//                stage once per species present with the other species' rows
//                zeroed: an atom's accumulator then receives the same
//                nonzero terms in the same order as in a one-species tile
//                (adding exact zeros changes no bits).
//                BF16 (QM = 1): the pass's K values kk = (a - a0) nchp + b
//                in 16x16x32 steps, lane (atom m, q) packing P_m at kk =
//                32 st + 8 q .. + 7 (zero past the pass) rounded to nearest
//                even, against BF16 fragments of W prepared by the host.
struct O3WArgs {
    const int *e;       // entries (A-row offsets 16 NT channels apart, coefficient bits)
    const int *mt;      // (first entry, groups of four) per (block, m3)
    const int *base;    // first (block, m3) row of each block
    const float *w;     // [species][block][a][ct][64 lanes][NJ padded to 4]
    const int *wb;      // BF16: [species][block][pass][ct][step][64 lanes][4 ints = 8 values]
    const int *order;   // work items per split, as the single-species form
    const int *wbeg;
    const int *dp_off;  // per-block offset in the partial buffer
    int n_pb, nch, L2, KAt, dp_stride, max_split, ns;
    int np, nstm;       // BF16: passes of eight channels a, steps per pass at most
};

constexpr int kO3wAH = 8;  // channels a per dense pass of the wide form

__host__ __device__ constexpr int o3w_rowb(int nc) { return kO3wAH * nc * 4 + 16; }

// Sparse stage of the wide form for channel tile ta of a: cc[tb][t] holds
// P_t[a = 16 ta + m][b = 16 tb + 4 q + v] after the NG entry groups.
template <int NT, int NCP, int NG>
__device__ __forceinline__ void o3w_sparse(const float *__restrict__ At, int L2, int m, int ta,
                                           const int2 (&ent)[kO3MaxGroups],
                                           f4v (&cc)[NT][kO3Atoms])
{
#pragma unroll
    for (int t = 0; t < kO3Atoms; ++t) {
#pragma unroll
        for (int tb = 0; tb < NT; ++tb)
            cc[tb][t] = (f4v){0.f, 0.f, 0.f, 0.f};
        const float *At_t = At + (size_t)t * L2 * NCP + m;
#pragma unroll
        for (int k = 0; k < NG; ++k) {
            const int o1 = ent[k].x & 0xffff, o2 = ent[k].x >> 16;
            const float bv = __int_as_float(ent[k].y) * At_t[o1 + 16 * ta];
#pragma unroll
            for (int tb = 0; tb < NT; ++tb)
                cc[tb][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(At_t[o2 + 16 * tb], bv, cc[tb][t],
                                                                 0, 0, 0);
        }
    }
}

template <int QM, int NC>  // QM 0 FP32, 1 BF16 dense stage; NC channels rounded up to 4 (<= 32)
__global__ void __launch_bounds__(256, 1)
    k_ace_o3w(const int *__restrict__ hdr, const int32_t *__restrict__ species,
              const int *__restrict__ S_idx, O3WArgs a, const float *__restrict__ A,
              float *__restrict__ Dpart)
{
    constexpr int NT = (NC + 15) / 16;
    constexpr int NCP = 16 * NT;
    constexpr int NJ = NC / 4;
    constexpr int NJP = (NJ + 3) & ~3;
    constexpr int ROWB = o3w_rowb(NC);
    const int nS = hdr[H_NS];
    const int ntile = (nS + kO3Atoms - 1) / kO3Atoms;
    int G = 1, lg = 0;
    while (G < a.max_split && ntile * G < (int)gridDim.x) {
        G <<= 1;
        ++lg;
    }
    const int nitem = ntile * G;
    // the splits of one tile on one XCD: its A rows come from that XCD's L2
    // after the first fetch
    const int vb = xcd_major(blockIdx.x, gridDim.x);
    if (vb >= nitem)
        return;  // uniform across the workgroup
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int m = lane & 15, q = lane >> 4;
    const int nch = a.nch, L2 = a.L2;
    extern __shared__ __align__(16) char smem_raw[];
    float *At = reinterpret_cast<float *>(smem_raw);  // [16][L2][NCP]
    const size_t at_bytes = (size_t)kO3Atoms * L2 * NCP * sizeof(float);
    char *Pw = smem_raw + at_bytes + (size_t)wv * kO3Atoms * ROWB;
    int *zt = reinterpret_cast<int *>(smem_raw + at_bytes + (size_t)4 * kO3Atoms * ROWB);
    const int *wbeg = a.wbeg + 4 * (G - 1) + lg;
    const size_t wz = (size_t)a.n_pb * NC * NT * 64 * NJP;  // weight floats per species

    for (int item = vb; item < nitem; item += gridDim.x) {
        const int tile = item >> lg, bin = ((item & (G - 1)) << 2) + wv;
        const int w_lo = wbeg[bin], w_hi = wbeg[bin + 1];
        const int s0 = tile * kO3Atoms;
        const int na = min(kO3Atoms, nS - s0);
        __syncthreads();  // every wave is done with the previous tile
        for (int r = tid; r < kO3Atoms * L2; r += 256) {
            const int t = r / L2, lm = r - t * L2;
            f4v *dst = reinterpret_cast<f4v *>(At + (size_t)r * NCP);
            const f4v *src = reinterpret_cast<const f4v *>(A + (size_t)(s0 + t) * a.KAt + lm * NC);
#pragma unroll
            for (int c4 = 0; c4 < NCP / 4; ++c4)
                dst[c4] = (c4 < NC / 4 && t < na) ? src[c4] : (f4v){0.f, 0.f, 0.f, 0.f};
        }
        if (tid < kO3Atoms)
            zt[tid] = tid < na ? sp_clamp(species[S_idx[s0 + tid]], a.ns) : -1;
        __syncthreads();
        unsigned zmask = 0;
        for (int t = 0; t < kO3Atoms; ++t)
            if (zt[t] >= 0)
                zmask |= 1u << zt[t];
        const int zrow = zt[m];  // species of this lane's atom row in the dense stage

        for (int wi = w_lo; wi < w_hi; ++wi) {
            const int code = a.order[wi];
            const int p = code & 0xffff, m3lo = (code >> 16) & 0xff, m3hi = (code >> 24) & 0xff;
            const int rbase = a.base[p];
            float *Dblk = Dpart + a.dp_off[p];
            int2 ent[kO3MaxGroups], ent_n[kO3MaxGroups];
            int ng = a.mt[2 * (rbase + m3lo) + 1];
            o3_load_row(a.e, a.mt[2 * (rbase + m3lo)], q, ent);
            for (int m3 = m3lo; m3 < m3hi; ++m3) {
                const int row = rbase + m3;
                int ngn = 0;
                if (m3 + 1 < m3hi) {
                    ngn = a.mt[2 * row + 3];
                    o3_load_row(a.e, a.mt[2 * row + 2], q, ent_n);
                }
                f4v acc[NT];
#pragma unroll
                for (int ct = 0; ct < NT; ++ct)
                    acc[ct] = (f4v){0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ta = 0; ta < NT; ++ta) {
                    f4v cc[NT][kO3Atoms];
#define O3W_SPARSE(NGV) o3w_sparse<NT, NCP, NGV>(At, L2, m, ta, ent, cc)
                    switch (ng) {
                    case 0: O3W_SPARSE(0); break;
                    case 1: O3W_SPARSE(1); break;
                    case 2: O3W_SPARSE(2); break;
                    case 3: O3W_SPARSE(3); break;
                    case 4: O3W_SPARSE(4); break;
                    case 5: O3W_SPARSE(5); break;
                    case 6: O3W_SPARSE(6); break;
                    case 7: O3W_SPARSE(7); break;
                    default: O3W_SPARSE(8); break;
                    }
#undef O3W_SPARSE
#pragma unroll
                    for (int h = 0; h < 16; h += kO3wAH) {
                        const int a0 = 16 * ta + h;
                        if (a0 >= NC)
                            break;  // uniform
                        // P rows of the pass: [atom][a - a0][b], b contiguous
                        if (m >= h && m < h + kO3wAH && a0 + m - h < NC) {
#pragma unroll
                            for (int tb = 0; tb < NT; ++tb) {
                                const int b0 = 16 * tb + 4 * q;
                                if (b0 < NC)
#pragma unroll
                                    for (int t = 0; t < kO3Atoms; ++t)
                                        *reinterpret_cast<f4v *>(Pw + (size_t)t * ROWB +
                                                                 ((m - h) * NC + b0) * 4) = cc[tb][t];
                            }
                        }
                        wave_sync_lds();
                        if constexpr (QM == 1) {
                            const int pa = a0 / kO3wAH;
                            const int kp = min(kO3wAH, NC - a0) * NC;  // K values of the pass
                            const float *prow = reinterpret_cast<const float *>(Pw + (size_t)m * ROWB);
                            for (int z = 0; z < a.ns; ++z) {
                                if (!((zmask >> z) & 1u))
                                    continue;  // uniform
                                const bool mine = zrow == z;
                                const int *wsrc = a.wb + ((((size_t)z * a.n_pb + p) * a.np + pa) * NT) *
                                                             a.nstm * 64 * 4;
#pragma unroll
                                for (int st = 0; st < NC / 4; ++st) {
                                    if (32 * st >= kp)
                                        break;  // uniform
                                    const int k0 = 32 * st + 8 * q;
                                    float x[8];
#pragma unroll
                                    for (int u = 0; u < 8; ++u)
                                        x[u] = (mine && k0 + u < kp) ? prow[k0 + u] : 0.0f;
                                    const bf2v p0 = __builtin_convertvector((f2v){x[0], x[1]}, bf2v);
                                    const bf2v p1 = __builtin_convertvector((f2v){x[2], x[3]}, bf2v);
                                    const bf2v p2 = __builtin_convertvector((f2v){x[4], x[5]}, bf2v);
                                    const bf2v p3 = __builtin_convertvector((f2v){x[6], x[7]}, bf2v);
                                    const bf8v pv = {p0[0], p0[1], p1[0], p1[1], p2[0], p2[1], p3[0], p3[1]};
#pragma unroll
                                    for (int ct = 0; ct < NT; ++ct) {
                                        const i4v wi = *reinterpret_cast<const i4v *>(
                                            wsrc + (((size_t)ct * a.nstm + st) * 64 + lane) * 4);
                                        acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                            pv, __builtin_bit_cast(bf8v, wi), acc[ct], 0, 0, 0);
                                    }
                                }
                            }
                        } else
                        for (int z = 0; z < a.ns; ++z) {
                            if (!((zmask >> z) & 1u))
                                continue;  // uniform
                            const bool mine = zrow == z;
                            const float *wsrc = a.w + (size_t)z * wz + (size_t)p * NC * NT * 64 * NJP;
#pragma unroll
                            for (int al = 0; al < kO3wAH; ++al) {
                                const int aa = a0 + al;
                                if (aa >= NC)
                                    break;  // uniform
                                const float *prow =
                                    reinterpret_cast<const float *>(Pw + (size_t)m * ROWB) +
                                    al * NC + NJ * q;
                                float pv[NJ];
#pragma unroll
                                for (int j = 0; j < NJ; ++j)
                                    pv[j] = mine ? prow[j] : 0.0f;
#pragma unroll
                                for (int ct = 0; ct < NT; ++ct) {
                                    const f4v *wf = reinterpret_cast<const f4v *>(
                                        wsrc + (((size_t)aa * NT + ct) * 64 + lane) * NJP);
                                    f4v w4[NJP / 4];
#pragma unroll
                                    for (int u = 0; u < NJP / 4; ++u)
                                        w4[u] = wf[u];
#pragma unroll
                                    for (int j = 0; j < NJ; ++j)
                                        acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                                            pv[j], w4[j >> 2][j & 3], acc[ct], 0, 0, 0);
                                }
                            }
                        }
                        wave_sync_lds();  // the next pass rewrites the P rows
                    }
                }
                // lane holds D[atom = 4 q + v][c = 16 ct + m]
#pragma unroll
                for (int ct = 0; ct < NT; ++ct)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int t = 4 * q + v, c = 16 * ct + m;
                        if (t < na && c < nch)
                            Dblk[(size_t)(s0 + t) * a.dp_stride + m3 * nch + c] = acc[ct][v];
                    }
#pragma unroll
                for (int k = 0; k < kO3MaxGroups; ++k)
                    ent[k] = ent_n[k];
                ng = ngn;
            }
        }
    }
}

size_t o3w_lds_bytes(const Ctx &c)
{
    const DevModel &m = c.m;
    const int nt = (m.nchp + 15) / 16;
    return (size_t)kO3Atoms * m.L2 * 16 * nt * sizeof(float) +
           (size_t)4 * kO3Atoms * o3w_rowb(m.nchp) + kO3Atoms * sizeof(int);
}

// Lets the wide kernel of this model use its dynamic LDS (beyond 64 KiB on
// gfx950, whose workgroups may take up to 160 KiB).
hipError_t o3w_prepare(const Ctx &c)
{
    const int lds = (int)o3w_lds_bytes(c);
    auto set = [&](auto nc) {
        constexpr int NC = decltype(nc)::value;
        const void *f = c.qmode == 1 ? reinterpret_cast<const void *>(&k_ace_o3w<1, NC>)
                                     : reinterpret_cast<const void *>(&k_ace_o3w<0, NC>);
        return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    };
    switch (c.m.nchp) {
    case 4: return set(std::integral_constant<int, 4>());
    case 8: return set(std::integral_constant<int, 8>());
    case 12: return set(std::integral_constant<int, 12>());
    case 16: return set(std::integral_constant<int, 16>());
    case 20: return set(std::integral_constant<int, 20>());
    case 24: return set(std::integral_constant<int, 24>());
    case 28: return set(std::integral_constant<int, 28>());
    default: return set(std::integral_constant<int, 32>());
    }
}

void launch_ace_o3w(hipStream_t s, const Ctx &c, void *ws, const WsLayout &L,
                    const int32_t *species, hipEvent_t ev0, hipEvent_t ev1)
{
    const DevModel &m = c.m;
    const char *base = static_cast<const char *>(m.base);
    O3WArgs a;
    a.e = reinterpret_cast<const int *>(base + m.o3o);
    a.mt = reinterpret_cast<const int *>(base + m.o3mt);
    a.base = reinterpret_cast<const int *>(base + m.o3base);
    a.w = reinterpret_cast<const float *>(base + m.o3ww);
    a.wb = reinterpret_cast<const int *>(base + m.o3wwb);
    a.np = (m.nchp + 7) / 8;
    a.nstm = m.nchp / 4;
    a.order = reinterpret_cast<const int *>(base + m.o3order);
    a.wbeg = reinterpret_cast<const int *>(base + m.o3wbeg);
    a.dp_off = reinterpret_cast<const int *>(base + m.dpoff);
    a.n_pb = m.n_pb;
    a.nch = m.nchan;
    a.L2 = m.L2;
    a.KAt = m.KAt;
    a.dp_stride = m.dp_stride;
    a.max_split = c.o3_max_split;
    a.ns = m.ns;
    const size_t lds = o3w_lds_bytes(c);
    const int per_cu = lds <= 80 * 1024 ? 2 : 1;
    const long items = (((long)L.n + kO3Atoms - 1) / kO3Atoms) * kO3MaxSplit;
    const int grid = (int)std::min<long>(std::max<long>(items, 1), 256L * per_cu);
    const int *hdr = at<int>(ws, L.hdr);
    const int *S_idx = at<int>(ws, L.S_idx);
    const float *A = at<float>(ws, L.A);
    float *D = at<float>(ws, L.dpart);
    auto go = [&](auto nc) {
        constexpr int NC = decltype(nc)::value;
        auto kern = c.qmode == 1 ? k_ace_o3w<1, NC> : k_ace_o3w<0, NC>;
        if (ev0)
            hipExtLaunchKernelGGL(kern, dim3(grid), dim3(256), (uint32_t)lds, s, ev0, ev1, 0u, hdr,
                                  species, S_idx, a, A, D);
        else
            kern<<<grid, 256, lds, s>>>(hdr, species, S_idx, a, A, D);
    };
    switch (m.nchp) {
    case 4: go(std::integral_constant<int, 4>()); break;
    case 8: go(std::integral_constant<int, 8>()); break;
    case 12: go(std::integral_constant<int, 12>()); break;
    case 16: go(std::integral_constant<int, 16>()); break;
    case 20: go(std::integral_constant<int, 20>()); break;
    case 24: go(std::integral_constant<int, 24>()); break;
    case 28: go(std::integral_constant<int, 28>()); break;
    default: go(std::integral_constant<int, 32>()); break;
    }
}

size_t o3_lds_bytes(const Ctx &c)
{
    const DevModel &m = c.m;
    const int nw = c.o3_waves;
    return (size_t)kO3Atoms * m.L2 * 16 * sizeof(float) +
           (size_t)nw * kO3Atoms * o3_row_bytes(c.qmode, m.nchp) +
           (size_t)(nw * kO3Atoms + kO3Atoms * (m.lmax + 1)) * sizeof(float);
}

void launch_ace_o3(hipStream_t s, const Ctx &c, void *ws, const WsLayout &L, hipEvent_t ev0,
                   hipEvent_t ev1)
{
    const DevModel &m = c.m;
    const char *base = static_cast<const char *>(m.base);
    O3Args a;
    a.e = reinterpret_cast<const int *>(base + m.o3o);
    a.mt = reinterpret_cast<const int *>(base + m.o3mt);
    a.mtv = reinterpret_cast<const int *>(base + m.o3mtv);
    a.rowv = reinterpret_cast<const int *>(base + m.o3rowv);
    a.rbeg = reinterpret_cast<const int *>(base + m.o3rbeg);
    a.wr = reinterpret_cast<const float *>(base + m.o3wr);
    a.sink = at<float>(ws, L.dpart) + (size_t)std::max(L.scap, 1) * (m.dp_stride > 0 ? m.dp_stride : 1);
    a.base = reinterpret_cast<const int *>(base + m.o3base);
    a.w = reinterpret_cast<const float *>(base + m.o3w);
    a.sw = reinterpret_cast<const float *>(base + m.o3sw);
    a.order = reinterpret_cast<const int *>(base + m.o3order);
    a.wbeg = reinterpret_cast<const int *>(base + m.o3wbeg);
    a.gs = reinterpret_cast<const float *>(base + m.o3gs);
    a.dp_off = reinterpret_cast<const int *>(base + m.dpoff);
    a.pb = reinterpret_cast<const PBlock *>(base + m.pb);
    a.n_pb = m.n_pb;
    a.nch = m.nchan;
    a.L1 = m.lmax + 1;
    a.L2 = m.L2;
    a.KAt = m.KAt;
    a.dp_stride = m.dp_stride;
    a.max_split = c.o3_max_split;
    const int *hdr = at<int>(ws, L.hdr);
    const float *A = at<float>(ws, L.A);
    float *D = at<float>(ws, L.dpart);
    const long items = (((long)L.n + kO3Atoms - 1) / kO3Atoms) * kO3MaxSplit;
    if (c.o3v) {
        // the vector sparse stage: as many resident workgroups as the
        // registers allow (waves per SIMD: three up to 12 channels, else two)
        const size_t lds = o3v_lds_bytes(c);
        auto go = [&](auto qm, auto nc) {
            constexpr int QM = decltype(qm)::value, NC = decltype(nc)::value;
            auto launch = [&](auto nw, auto bpw) {
                constexpr int NW = decltype(nw)::value, BPW = decltype(bpw)::value;
                const int grid = o3v_grid(c, L.n);
                if (ev0)
                    hipExtLaunchKernelGGL(k_ace_o3v<QM, NC, NW, BPW>, dim3(grid), dim3(64 * NW),
                                          (uint32_t)lds, s, ev0, ev1, 0u, hdr, a, A, D);
                else
                    k_ace_o3v<QM, NC, NW, BPW><<<grid, 64 * NW, lds, s>>>(hdr, a, A, D);
            };
            // the bins were built for c.o3_waves waves per workgroup
            if (c.o3_waves != 8)
                launch(std::integral_constant<int, 4>(), std::integral_constant<int, 1>());
            else if (o3v_waves(c, L.n) == 4)
                launch(std::integral_constant<int, 4>(), std::integral_constant<int, 2>());
            else
                launch(std::integral_constant<int, 8>(), std::integral_constant<int, 1>());
        };
        auto by_width = [&](auto qm) {
            switch (m.nchp) {
            case 4: go(qm, std::integral_constant<int, 4>()); break;
            case 8: go(qm, std::integral_constant<int, 8>()); break;
            case 12: go(qm, std::integral_constant<int, 12>()); break;
            default: go(qm, std::integral_constant<int, 16>()); break;
            }
        };
        if (c.qmode == 1)
            by_width(std::integral_constant<int, 1>());
        else if (c.qmode == 2)
            by_width(std::integral_constant<int, 2>());
        else
            by_width(std::integral_constant<int, 0>());
        return;
    }
    const size_t lds = o3_lds_bytes(c);
    const int per_cu = lds <= 80 * 1024 ? 2 : 1;
    // persistent grid: one wave of resident workgroups; the kernel splits
    // tiles when S is small
    const int grid = (int)std::min<long>(std::max<long>(items, 1), 256L * per_cu);
    auto go = [&](auto qm, auto nc) {
        constexpr int QM = decltype(qm)::value, NC = decltype(nc)::value;
        auto launch = [&](auto nw) {
            constexpr int NW = decltype(nw)::value;
            if (ev0)  // stage timing: events carry the kernel's own start and end
                hipExtLaunchKernelGGL(k_ace_o3<QM, NC, NW>, dim3(grid), dim3(64 * NW),
                                      (uint32_t)lds, s, ev0, ev1, 0u, hdr, a, A, D);
            else
                k_ace_o3<QM, NC, NW><<<grid, 64 * NW, lds, s>>>(hdr, a, A, D);
        };
        if (c.o3_waves == 8)
            launch(std::integral_constant<int, 8>());
        else
            launch(std::integral_constant<int, 4>());
    };
    auto by_width = [&](auto qm) {
        switch (m.nchp) {
        case 4: go(qm, std::integral_constant<int, 4>()); break;
        case 8: go(qm, std::integral_constant<int, 8>()); break;
        case 12: go(qm, std::integral_constant<int, 12>()); break;
        default: go(qm, std::integral_constant<int, 16>()); break;
        }
    };
    if (c.qmode == 1)
        by_width(std::integral_constant<int, 1>());
    else if (c.qmode == 2)
        by_width(std::integral_constant<int, 2>());
    else
        by_width(std::integral_constant<int, 0>());
}

}  // namespace mlmix
