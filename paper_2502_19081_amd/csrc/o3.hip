// Order-3 product-basis contraction on the matrix cores, for single-species
// models of at most 16 radial channels (ACE-style model; the order-3 term of
// the site energy written as a symmetric cubic form in the atomic basis A,
// block by block over (l1 <= l2, l3) with real Gaunt coefficients).
//
// A workgroup owns a tile of 16 atoms of S and stages their A rows in LDS
// ([atom][lm][16 channels], zero padded). Each of its four waves owns a fixed
// list of blocks (balanced on the host) and, for every block and m3, one
// 16-row tile whose rows are the 16 atoms:
//
//  sparse stage  P_t[a][b] = sum_e g_e A_t[l1 m1_e][a] A_t[l2 m2_e][b] for
//                each atom t, as a 16x16 MFMA product whose K runs over the
//                (m1, m2) entries of the row (four per step; padded entries
//                have g = 0). The wave writes P_t into its own LDS rows in
//                the layout [b / 4][a][b % 4] (a stride nch2), which makes
//                the lanes' 16-byte writes and the dense stage's reads free
//                of bank conflicts.
//  dense stage   D[t][c] = sum_{a,b} P_t[a][b] W[a][b][c] as 16x16 MFMA
//                steps with the block's weights held in registers (one
//                fragment per lane, loaded once per block).
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
#include "internal.h"

namespace mlmix {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef __bf16 bf4v __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf2v __attribute__((ext_vector_type(2)));

struct O3Args {
    const float *g;       // entry coefficients
    const int *o;         // packed A-row offsets of the entries
    const int *mt;        // (start, groups) per (block, m3)
    const int *base;      // first (block, m3) row of each block
    const float *w;       // weight fragments [block][nch2][64][4]
    const float *sw;      // FP8 weight scales [block][16]
    const int *order;     // per split G = 1, 2, 4, 8: the blocks of bin 0, bin 1, ...
    const int *wbeg;      // per split G: 4 G + 1 bin offsets into its order
    const float *gs;      // sum of |g| per (block, m3) (FP8 row-scale bound)
    const int *dp_off;    // per-block offset in the partial buffer
    const PBlock *pb;
    int n_pb, nch, nch2, L1, L2, KAt, nchp, dp_stride;
};

constexpr int kO3Atoms = 16;

// bytes of one P row per format (16-byte pad keeps rows 4 banks apart)
__host__ __device__ inline int o3_row_bytes(int qm, int nch2)
{
    const int es = qm == 0 ? 4 : (qm == 1 ? 2 : 1);
    return 4 * nch2 * 4 * es + 16;
}

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int QM>
__global__ void __launch_bounds__(256, 1)
    k_ace_o3(const int *__restrict__ hdr, O3Args a, const float *__restrict__ A,
             float *__restrict__ Dpart)
{
    const int nS = hdr[H_NS];
    const int ntile = (nS + kO3Atoms - 1) / kO3Atoms;
    int G = 1, lg = 0;
    while (G < kO3MaxSplit && ntile * G < (int)gridDim.x) {
        G <<= 1;
        ++lg;
    }
    const int nitem = ntile * G;
    if ((int)blockIdx.x >= nitem)
        return;  // uniform across the workgroup
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = lane & 15, q = lane >> 4;
    const int nch = a.nch, nch2 = a.nch2, L2 = a.L2;
    const int rowb = o3_row_bytes(QM, nch2);
    extern __shared__ __align__(16) char smem_raw[];
    float *At = reinterpret_cast<float *>(smem_raw);  // [16][L2][16]
    char *Pw = smem_raw + (size_t)kO3Atoms * L2 * 16 * sizeof(float) + (size_t)wv * kO3Atoms * rowb;
    float *sPall = reinterpret_cast<float *>(smem_raw + (size_t)kO3Atoms * L2 * 16 * sizeof(float) +
                                             (size_t)4 * kO3Atoms * rowb);
    float *sP = sPall + wv * kO3Atoms;
    float *amax = sPall + 4 * kO3Atoms;  // [16][L1]: max |A| per atom and l (FP8)
    const int *order = a.order + lg * a.n_pb;
    const int *wbeg = a.wbeg + 4 * (G - 1) + lg;

    for (int item = blockIdx.x; item < nitem; item += gridDim.x) {
        const int tile = item >> lg, bin = ((item & (G - 1)) << 2) + wv;
        const int w_lo = wbeg[bin], w_hi = wbeg[bin + 1];
        const int s0 = tile * kO3Atoms;
        const int na = min(kO3Atoms, nS - s0);
        __syncthreads();  // every wave is done with the previous tile's A
        for (int e = tid; e < kO3Atoms * L2 * 16; e += 256) {
            const int t = e / (L2 * 16), r = e - t * (L2 * 16);
            const int lm = r >> 4, c = r & 15;
            At[e] = (t < na && c < nch) ? A[(size_t)(s0 + t) * a.KAt + lm * a.nchp + c] : 0.0f;
        }
        __syncthreads();
        if constexpr (QM == 2) {
            if (tid < kO3Atoms * a.L1) {
                const int t = tid / a.L1, l = tid - t * a.L1;
                const f4v *row = reinterpret_cast<const f4v *>(At + ((size_t)t * L2 + l * l) * 16);
                float mx = 0.0f;
                for (int k = 0; k < (2 * l + 1) * 4; ++k) {
                    const f4v v = row[k];
                    mx = fmaxf(mx, fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fmaxf(fabsf(v[2]), fabsf(v[3]))));
                }
                amax[t * a.L1 + l] = mx;
            }
            __syncthreads();
        }

        for (int wi = w_lo; wi < w_hi; ++wi) {
            const int p = order[wi];
            const PBlock pbk = a.pb[p];
            const int d3 = 2 * pbk.l3 + 1;
            // weight fragments of this lane: element 4 i + j <-> (a = i, b = 4 q + j, c = m)
            f4v wf[16];
            const f4v *wsrc = reinterpret_cast<const f4v *>(a.w) + (size_t)p * nch2 * 64 + lane;
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (i < nch2)
                    wf[i] = wsrc[i * 64];
            bf8v wb[8];
            long w8[8];
            if constexpr (QM == 1) {
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    if (2 * i < nch2) {
                        f4v x = wf[2 * i], y = wf[2 * i + 1];
                        bf2v p0 = __builtin_convertvector((f2v){x[0], x[1]}, bf2v);
                        bf2v p1 = __builtin_convertvector((f2v){x[2], x[3]}, bf2v);
                        bf2v p2 = __builtin_convertvector((f2v){y[0], y[1]}, bf2v);
                        bf2v p3 = __builtin_convertvector((f2v){y[2], y[3]}, bf2v);
                        wb[i] = (bf8v){p0[0], p0[1], p1[0], p1[1], p2[0], p2[1], p3[0], p3[1]};
                    }
            } else if constexpr (QM == 2) {
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    if (2 * i < nch2) {
                        f4v x = wf[2 * i], y = wf[2 * i + 1];
                        int lo = __builtin_amdgcn_cvt_pk_fp8_f32(x[0], x[1], 0, false);
                        lo = __builtin_amdgcn_cvt_pk_fp8_f32(x[2], x[3], lo, true);
                        int hi = __builtin_amdgcn_cvt_pk_fp8_f32(y[0], y[1], 0, false);
                        hi = __builtin_amdgcn_cvt_pk_fp8_f32(y[2], y[3], hi, true);
                        w8[i] = (long)(((unsigned long)(unsigned)hi << 32) | (unsigned)lo);
                    }
            }
            const float swc = QM == 2 ? a.sw[p * 16 + m] : 1.0f;
            float *Dblk = Dpart + a.dp_off[p];

            for (int m3 = 0; m3 < d3; ++m3) {
                const int row = a.base[p] + m3;
                const int e0 = a.mt[2 * row], ng = a.mt[2 * row + 1];
                const float gsum = QM == 2 ? a.gs[row] * (1.0f / 240.0f) : 0.0f;
                float ge[8];
                int oe[8];
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    if (k < ng) {
                        ge[k] = a.g[e0 + 4 * k + q];
                        oe[k] = a.o[e0 + 4 * k + q];
                    }
                // ---- sparse stage: P_t for the 16 atoms, two at a time
                for (int t = 0; t < kO3Atoms; t += 2) {
                    const float *A0 = At + (size_t)t * L2 * 16 + m;
                    const float *A1 = A0 + L2 * 16;
                    f4v c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int k = 0; k < 8; ++k)
                        if (k < ng) {
                            const int o1 = oe[k] & 0xffff, o2 = oe[k] >> 16;
                            c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(A0[o2], ge[k] * A0[o1], c0, 0, 0, 0);
                            c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(A1[o2], ge[k] * A1[o1], c1, 0, 0, 0);
                        }
                    // lane holds P[a = m][b = 4 q + v]; chunk (b / 4 = q, a = m)
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const f4v cv = h ? c1 : c0;
                        char *dst = Pw + (size_t)(t + h) * rowb;
                        if constexpr (QM == 0) {
                            if (m < nch2)
                                *reinterpret_cast<f4v *>(dst + (q * nch2 + m) * 16) = cv;
                        } else if constexpr (QM == 1) {
                            bf2v p0 = __builtin_convertvector((f2v){cv[0], cv[1]}, bf2v);
                            bf2v p1 = __builtin_convertvector((f2v){cv[2], cv[3]}, bf2v);
                            if (m < nch2)
                                *reinterpret_cast<bf4v *>(dst + (q * nch2 + m) * 8) =
                                    (bf4v){p0[0], p0[1], p1[0], p1[1]};
                        } else {
                            const float *am = amax + (t + h) * a.L1;
                            const float sc = gsum * am[pbk.l1] * am[pbk.l2];  // >= max|P| / 240
                            const float inv = sc > 0.0f ? 1.0f / sc : 0.0f;
                            int pk = __builtin_amdgcn_cvt_pk_fp8_f32(cv[0] * inv, cv[1] * inv, 0, false);
                            pk = __builtin_amdgcn_cvt_pk_fp8_f32(cv[2] * inv, cv[3] * inv, pk, true);
                            if (m < nch2)
                                *reinterpret_cast<int *>(dst + (q * nch2 + m) * 4) = pk;
                            if (lane == 0)
                                sP[t + h] = sc;
                        }
                    }
                }
                wave_sync_lds();
                // ---- dense stage: D[atom m-row][c] over the 16 atoms
                f4v acc = {0.f, 0.f, 0.f, 0.f};
                const char *Prow = Pw + (size_t)m * rowb;
                if constexpr (QM == 0) {
#pragma unroll
                    for (int i = 0; i < 16; ++i)
                        if (i < nch2) {
                            const f4v pv = *reinterpret_cast<const f4v *>(Prow + (q * nch2 + i) * 16);
                            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(pv[0], wf[i][0], acc, 0, 0, 0);
                            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(pv[1], wf[i][1], acc, 0, 0, 0);
                            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(pv[2], wf[i][2], acc, 0, 0, 0);
                            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(pv[3], wf[i][3], acc, 0, 0, 0);
                        }
                } else if constexpr (QM == 1) {
#pragma unroll
                    for (int i = 0; i < 8; ++i)
                        if (2 * i < nch2) {
                            const bf8v pv = *reinterpret_cast<const bf8v *>(Prow + (q * nch2 + 2 * i) * 8);
                            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pv, wb[i], acc, 0, 0, 0);
                        }
                } else {
#pragma unroll
                    for (int i = 0; i < 8; ++i)
                        if (2 * i < nch2) {
                            const long pv = *reinterpret_cast<const long *>(Prow + (q * nch2 + 2 * i) * 4);
                            acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(pv, w8[i], acc, 0, 0, 0);
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
            }
        }
    }
}

size_t o3_lds_bytes(const Ctx &c)
{
    const DevModel &m = c.m;
    return (size_t)kO3Atoms * m.L2 * 16 * sizeof(float) +
           (size_t)4 * kO3Atoms * o3_row_bytes(c.qmode, c.o3_nch2) +
           (size_t)(4 * kO3Atoms + kO3Atoms * (m.lmax + 1)) * sizeof(float);
}

void launch_ace_o3(hipStream_t s, const Ctx &c, void *ws, const WsLayout &L)
{
    const DevModel &m = c.m;
    const char *base = static_cast<const char *>(m.base);
    O3Args a;
    a.g = reinterpret_cast<const float *>(base + m.o3g);
    a.o = reinterpret_cast<const int *>(base + m.o3o);
    a.mt = reinterpret_cast<const int *>(base + m.o3mt);
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
    a.nch2 = c.o3_nch2;
    a.L2 = m.L2;
    a.KAt = m.KAt;
    a.nchp = m.nchp;
    a.dp_stride = m.dp_stride;
    const size_t lds = o3_lds_bytes(c);
    const int per_cu = lds <= 80 * 1024 ? 2 : 1;
    // persistent grid: one wave of resident workgroups; the kernel splits
    // tiles when S is small
    const long items = (((long)L.n + kO3Atoms - 1) / kO3Atoms) * kO3MaxSplit;
    const int grid = (int)std::min<long>(std::max<long>(items, 1), 256L * per_cu);
    const int *hdr = at<int>(ws, L.hdr);
    const float *A = at<float>(ws, L.A);
    float *D = at<float>(ws, L.dpart);
    if (c.qmode == 1)
        k_ace_o3<1><<<grid, 256, lds, s>>>(hdr, a, A, D);
    else if (c.qmode == 2)
        k_ace_o3<2><<<grid, 256, lds, s>>>(hdr, a, A, D);
    else
        k_ace_o3<0><<<grid, 256, lds, s>>>(hdr, a, A, D);
}

}  // namespace mlmix
