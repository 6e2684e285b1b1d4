// C ABI of the library: model tables, workspace layout, argument checks and
// the launch sequence of one mixed force evaluation (see include/mlmix.h).
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <memory>
#include <new>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

#include "basis.h"
#include "internal.h"

using namespace mlmix;

struct PendingEvent {
    int stage;
    hipEvent_t a, b;
};

// Second stream of a workspace: the reverse slots and the cheap potential run
// on it beside the expensive path (fork and join through events on the
// caller's stream, so the step stays capturable in a HIP graph).
struct SideStream {
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};

// Langevin thermostat of one workspace (off when tau <= 0).
struct LangevinSet {
    double temperature = 0.0, tau = 0.0;
    const double *xi = nullptr;
};

struct mlmix_ctx {
    Ctx c;
    std::mutex mu;
    std::unordered_map<void *, WsLayout> ws;
    std::unordered_map<void *, LangevinSet> lang;
    std::unordered_map<void *, SideStream> side;
    std::unordered_map<void *, std::vector<mlmix_segment>> batch;  // segments of batch workspaces
    uint32_t prof_mask = 0;
    double flops[7] = {0, 0, 0, 0, 0, 0, 0};
    std::vector<PendingEvent> pending;
    std::vector<hipEvent_t> pool;
};

static const char *kStageNames[MLMIX_N_STAGES] = {
    "neighbours", "regions", "compaction", "ace_basis", "ace_contract", "ace_finalize",
    "ace_pairgrad", "uf3", "gather_blend", "integrator", "energy_sums", "reverse_slots"};

enum {
    ST_NBR, ST_REG, ST_CMP, ST_BASIS, ST_CONTRACT, ST_FIN, ST_PAIR, ST_UF3, ST_GATHER, ST_VV, ST_RED,
    ST_REV
};

static hipEvent_t take_event(mlmix_ctx *ctx)
{
    if (!ctx->pool.empty()) {
        hipEvent_t e = ctx->pool.back();
        ctx->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess)
        return nullptr;
    return e;
}

// Set for the duration of an allocation-free call: stage brackets take
// events, which such a call must not create.
static thread_local bool tl_no_timers = false;

// Brackets one stage with events when its bit is set in the profile mask.
// Times a stage with two events on its stream. With kernel_events the stage
// is one kernel whose launcher passes k0/k1 to hipExtLaunchKernel, so the
// events carry the kernel's own start and end (no bracket overhead).
struct StageTimer {
    mlmix_ctx *ctx;
    hipStream_t s;
    int stage;
    hipEvent_t a = nullptr;
    hipEvent_t k0 = nullptr, k1 = nullptr;
    StageTimer(mlmix_ctx *c, hipStream_t st, int stg, bool kernel_events = false)
        : ctx(c), s(st), stage(stg)
    {
        if (!tl_no_timers && (ctx->prof_mask & (1u << stage))) {
            if (kernel_events) {
                k0 = take_event(ctx);
                k1 = take_event(ctx);
                if (!k0 || !k1) {
                    if (k0)
                        ctx->pool.push_back(k0);
                    if (k1)
                        ctx->pool.push_back(k1);
                    k0 = k1 = nullptr;
                }
            } else {
                a = take_event(ctx);
                if (a)
                    (void)hipEventRecord(a, s);
            }
        }
    }
    ~StageTimer()
    {
        // a destructor must not throw: a bracket that cannot be queued is
        // dropped (its events are released)
        try {
            if (k0) {
                ctx->pending.push_back({stage, k0, k1});
            } else if (a) {
                hipEvent_t b = take_event(ctx);
                if (b) {
                    (void)hipEventRecord(b, s);
                    ctx->pending.push_back({stage, a, b});
                } else {
                    ctx->pool.push_back(a);
                }
            }
        } catch (...) {
            (void)hipEventDestroy(k0 ? k0 : a);
            if (k1)
                (void)hipEventDestroy(k1);
        }
    }
};

// Message of the last failing call on this thread (a fixed buffer: reporting
// an error allocates nothing).
static thread_local char g_err[512];

static int fail(int code, const char *msg)
{
    std::snprintf(g_err, sizeof g_err, "%s", msg);
    return code;
}

static int fail_hip(const char *what, hipError_t e)
{
    std::snprintf(g_err, sizeof g_err, "%s: %s", what, hipGetErrorString(e));
    return MLMIX_E_HIP;
}

// Handler of every entry point's function-try-block: no C++ exception
// crosses the C ABI (the host tables and bookkeeping use the standard
// containers, which report exhausted host memory by throwing).
static int host_exception() noexcept
{
    try {
        throw;
    } catch (const std::bad_alloc &) {
        return fail(MLMIX_E_HOST, "host memory exhausted");
    } catch (const std::exception &ex) {
        return fail(MLMIX_E_HOST, ex.what());
    } catch (...) {
        return fail(MLMIX_E_HOST, "unexpected host exception");
    }
}

extern "C" const char *mlmix_last_error(void) { return g_err; }

#define HIP_OK(expr)                        \
    do {                                    \
        hipError_t e_ = (expr);             \
        if (e_ != hipSuccess)               \
            return fail_hip(#expr, e_);     \
    } while (0)

// ------------------------------------------- workspace of the allocation-free call
// mlmix_compute_noalloc keeps its workspace in this file-scope device array
// (one copy per GPU the library runs on, held until the process ends). Host
// code never passes the array's name to a kernel or a copy: the device
// address of each GPU's copy is looked up once per device, at mlmix_create
// with that device current, and kept in g_scratch_dev.
static __device__ __align__(256) unsigned char scratch[MLMIX_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_dev[kMaxDevices] = {};

static int scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return fail(MLMIX_E_ARG, "device index beyond the library's table of 64 devices");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (g_scratch_dev[device])
        return MLMIX_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess)
        return fail_hip("hipGetSymbolAddress(scratch)", e);
    if (!p)
        return fail(MLMIX_E_HIP, "hipGetSymbolAddress(scratch) returned no address");
    g_scratch_dev[device] = p;
    return MLMIX_OK;
}

static void *scratch_ptr(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return nullptr;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    return g_scratch_dev[device];
}

namespace mlmix {

// ------------------------------------------------------------ tabulation

static std::vector<double> ylm_norm(int lmax)
{
    int L2 = (lmax + 1) * (lmax + 1);
    std::vector<double> K(L2);
    for (int l = 0; l <= lmax; ++l)
        for (int m = -l; m <= l; ++m) {
            int am = m < 0 ? -m : m;
            double r = 1.0;  // (l-|m|)!/(l+|m|)!
            for (int q = l - am + 1; q <= l + am; ++q)
                r /= q;
            double N = std::sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * r);
            K[l * l + l + m] = (m == 0) ? N : std::sqrt(2.0) * N;
        }
    return K;
}

// Wigner 3j symbol by Racah's single-sum formula (factorials up to
// (3 kMaxLmax + 1)! are exact enough in double for the cancellations of the
// alternating sum at l <= 6).
static double wigner3j(int j1, int j2, int j3, int m1, int m2, int m3)
{
    if (m1 + m2 + m3 != 0 || j3 > j1 + j2 || j3 < std::abs(j1 - j2))
        return 0.0;
    if (std::abs(m1) > j1 || std::abs(m2) > j2 || std::abs(m3) > j3)
        return 0.0;
    double f[3 * kMaxLmax + 2];
    f[0] = 1.0;
    for (int k = 1; k < 3 * kMaxLmax + 2; ++k)
        f[k] = f[k - 1] * k;
    const double tri = f[j1 + j2 - j3] * f[j1 - j2 + j3] * f[-j1 + j2 + j3] / f[j1 + j2 + j3 + 1];
    const double pre = std::sqrt(tri * f[j1 + m1] * f[j1 - m1] * f[j2 + m2] * f[j2 - m2] *
                                 f[j3 + m3] * f[j3 - m3]);
    double sum = 0.0;
    for (int k = 0; k <= j1 + j2 + j3; ++k) {
        const int a[6] = {k, j3 - j2 + k + m1, j3 - j1 + k - m2, j1 + j2 - j3 - k, j1 - k - m1,
                          j2 - k + m2};
        if (*std::min_element(a, a + 6) < 0)
            continue;
        const double den = f[a[0]] * f[a[1]] * f[a[2]] * f[a[3]] * f[a[4]] * f[a[5]];
        sum += ((k & 1) ? -1.0 : 1.0) / den;
    }
    return (((j1 - j2 - m3) & 1) ? -1.0 : 1.0) * pre * sum;
}

// Real Gaunt coefficients G[lm1][lm2][lm3] = integral of the product of three
// real harmonics over the sphere, from the closed form of the complex ones,
//   int Y_l1^m1 Y_l2^m2 Y_l3^m3 = sqrt((2l1+1)(2l2+1)(2l3+1)/(4 pi))
//                                 (l1 l2 l3; 0 0 0) (l1 l2 l3; m1 m2 m3),
// and the change of basis to the real harmonics that ylm_stream evaluates
// (no Condon-Shortley phase; index l^2 + l + m, cosine type for m > 0, sine
// type for m < 0): with Y_l^m the complex harmonics (Condon-Shortley phase),
//   Y_{l,m>0}  = ((-1)^m Y_l^m + Y_l^-m) / sqrt(2),
//   Y_{l,-m<0} = ((-1)^m Y_l^m - Y_l^-m) / (i sqrt(2)),   Y_{l,0} = Y_l^0.
// Each real harmonic has at most two complex components, so each real
// coefficient is a sum of at most eight complex ones (its imaginary part is
// zero).
static std::vector<double> gaunt(int lmax)
{
    typedef std::complex<double> cd;
    const int L2 = (lmax + 1) * (lmax + 1);
    // complex components (m, coefficient) of every real harmonic
    std::vector<int> nc(L2), cm((size_t)2 * L2);
    std::vector<cd> cc((size_t)2 * L2);
    const double r2 = 1.0 / std::sqrt(2.0);
    for (int l = 0; l <= lmax; ++l)
        for (int m = -l; m <= l; ++m) {
            const int q = l * l + l + m, mu = std::abs(m);
            const double sg = (mu & 1) ? -1.0 : 1.0;
            if (m == 0) {
                nc[q] = 1;
                cm[2 * q] = 0;
                cc[2 * q] = cd(1.0, 0.0);
            } else if (m > 0) {
                nc[q] = 2;
                cm[2 * q] = mu;
                cc[2 * q] = cd(sg * r2, 0.0);
                cm[2 * q + 1] = -mu;
                cc[2 * q + 1] = cd(r2, 0.0);
            } else {  // 1 / i = -i
                nc[q] = 2;
                cm[2 * q] = mu;
                cc[2 * q] = cd(0.0, -sg * r2);
                cm[2 * q + 1] = -mu;
                cc[2 * q + 1] = cd(0.0, r2);
            }
        }
    std::vector<double> G((size_t)L2 * L2 * L2, 0.0);
    for (int l1 = 0; l1 <= lmax; ++l1)
        for (int l2 = 0; l2 <= lmax; ++l2)
            for (int l3 = 0; l3 <= lmax; ++l3) {
                if ((l1 + l2 + l3) & 1 || l3 > l1 + l2 || l3 < std::abs(l1 - l2))
                    continue;
                const double pre =
                    std::sqrt((2.0 * l1 + 1.0) * (2.0 * l2 + 1.0) * (2.0 * l3 + 1.0) / (4.0 * M_PI)) *
                    wigner3j(l1, l2, l3, 0, 0, 0);
                for (int q1 = l1 * l1; q1 < (l1 + 1) * (l1 + 1); ++q1)
                    for (int q2 = l2 * l2; q2 < (l2 + 1) * (l2 + 1); ++q2)
                        for (int q3 = l3 * l3; q3 < (l3 + 1) * (l3 + 1); ++q3) {
                            cd v(0.0, 0.0);
                            for (int a = 0; a < nc[q1]; ++a)
                                for (int b = 0; b < nc[q2]; ++b)
                                    for (int c = 0; c < nc[q3]; ++c) {
                                        const int m1 = cm[2 * q1 + a], m2 = cm[2 * q2 + b],
                                                  m3 = cm[2 * q3 + c];
                                        if (m1 + m2 + m3 != 0)
                                            continue;
                                        v += cc[2 * q1 + a] * cc[2 * q2 + b] * cc[2 * q3 + c] *
                                             (pre * wigner3j(l1, l2, l3, m1, m2, m3));
                                    }
                            G[((size_t)q1 * L2 + q2) * L2 + q3] = v.real();
                        }
            }
    return G;
}

struct HostTables {
    std::vector<double> K, c0, c1, c2s, W, gval, u2, u3, up2, up3, wsc;
    std::vector<PBlock> pb;
    std::vector<int> gm3, gidx, gofs, dpoff;
    int w_per_species = 0;
    int dp_stride = 0;
    // matrix-core order-3 kernel
    bool o3 = false;
    int o3_kind = 0;  // 1 single-species narrow form, 2 wide form
    bool o3_wide_ready = false;  // wide-form weight fragments built
    std::vector<double> o3ww;
    std::vector<int32_t> o3wwb;  // BF16 wide-form fragments, two values per int
    int o3_nch2 = 0;
    std::vector<double> o3g, o3w, o3sw, o3gs;
    std::vector<int> o3o, o3mt, o3mtv, o3base, o3order, o3wbeg;
    std::vector<int> o3rowv, o3rbeg;  // bins as flat row lists (vector-sparse form)
    std::vector<double> o3wr;         // its reduced-precision weight fragments
    int o3rows_max = 0;               // longest such list
    bool o3rows_empty = false;        // some (block, m3) has no Gaunt entry
    // per split G of the vector-sparse form with summed runs: per (l3, m3)
    // the partial-D columns its rows write (empty: one column per row)
    std::vector<std::vector<std::vector<int>>> o3vsets;
    std::vector<int> dsum;  // the column sets of every form (DevModel::dsum)
    int dsum_off[kDSumSets] = {};
    int dsum_span[kDSumSets] = {};  // per set: 1 + its largest column / nchan
    int dsum_ncol[kDSumSets] = {};  // per set: the number of columns it lists
    int dsum_len = 0;
};

// Tables of the per-wave matrix-core order-3 kernel (single-species models
// of at most 16 channels in a single-precision mode):
//  - Gaunt entries of each (block, m3), padded with zero entries to a
//    multiple of four (one MFMA K step), as pairs (packed offsets
//    (l1 m1)*16 | (l2 m2)*16 << 16 of the two A rows in the kernel's
//    16-channel LDS layout, FP32 bits of the coefficient); (first entry,
//    groups) per (block, m3), and (first entry, exact count) for the FP32
//    form whose sparse stage runs on the vector ALUs;
//  - the block weights as per-lane MFMA fragments: for lane (c = l % 16,
//    q = l / 16) element f = 4 i + j holds W[a = i][b = 4 q + j][c], stored
//    [block][i][lane][4] so that a wave loads them as 16-byte rows; in the
//    FP8 mode divided by the per-(block, c) scale max|W| / 240;
//  - longest-processing-time assignments of the blocks to 4 G bins (four
//    waves of each of G workgroups sharing a tile), G = 1, 2, 4, 8;
//  - per (block, m3) the sum of |g|, for the FP8 row-scale bound.
//
// The wide form (FP32, more than one species or 17-32 channels) uses the same
// entry lists with A rows 16 NT channels apart in LDS (NT = channel tiles of
// 16), its own cost model, and weight fragments for its dense stage, per
// species: for lane (c = l % 16, q = l / 16), channel tile ct and a, the
// NJ = nchp / 4 values W[a][b = NJ q + j][c = 16 ct + c], j < NJ, padded to a
// multiple of four, stored [species][block][a][ct][lane][NJ padded].
// Bins of the vector-sparse form as flat row lists grouped by output: an
// item is a run of the rows (p, m3) of one (l3, m3) over a range of the
// blocks p of that l3, and a wave sums a run's products in its matrix
// accumulators and stores one partial-D column for the run. The partial
// buffer then holds one column per item where the other forms write one per
// (block, m3), and the finalisation sums fewer of them. Items above a cut
// (a fraction of a bin's even share of the cost) are split into block
// ranges of near-even size, and go longest first onto the least loaded bin;
// of the cuts tried, the one whose longest bin is shortest is kept. Each bin
// runs its items in (l3, m3, first block) order. Columns are numbered in that order over the
// whole tile, so that the columns of one (l3, m3) lie side by side. Per
// split G = 1 .. 16: 4 G bins (waves x G workgroups), the offsets of the
// bins' rows in o3rbeg, and the columns of each (l3, m3) in o3vsets.
static void build_o3v_runs(HostTables &t, int lmax, int nch, int waves, long total,
                           const std::vector<std::vector<int>> &rcost)
{
    const int P = (int)t.pb.size(), L2 = (lmax + 1) * (lmax + 1);
    std::vector<int> plo(lmax + 1, 0), phi(lmax + 1, 0);  // blocks of each l3
    for (int p = P - 1; p >= 0; --p)
        plo[t.pb[p].l3] = p;
    for (int p = 0; p < P; ++p)
        phi[t.pb[p].l3] = p + 1;
    t.o3rowv.clear();
    t.o3rbeg.clear();
    t.o3rows_max = 0;
    struct Item {
        long cost;
        int l3, m3, lo, hi;
    };
    for (int G = 1; G <= kO3MaxSplit; G <<= 1) {
        const int nb = waves * G;
        // items cut at 1/2, 1/3, ... 1/8 of a bin's even share: the cut whose
        // assignment has the least loaded longest bin (a run's store counts
        // 2 nch), the coarser cut on ties
        std::vector<Item> items;  // in (l3, m3, first block) order
        std::vector<std::vector<int>> lists;
        long best = -1;
        for (int div : {2, 3, 4, 6, 8}) {
            const long cap = std::max<long>(1, total / nb / div);
            std::vector<Item> its;
            for (int l3 = 0; l3 <= lmax; ++l3)
                for (int m3 = 0; m3 < 2 * l3 + 1; ++m3) {
                    long gc = 0;
                    for (int p = plo[l3]; p < phi[l3]; ++p)
                        gc += rcost[p][m3];
                    const int k = (int)std::max<long>(
                        1, std::min<long>(phi[l3] - plo[l3], (gc + cap - 1) / cap));
                    int lo = plo[l3];
                    for (int part = 0; part < k; ++part) {
                        const int hi = lo + (phi[l3] - lo) / (k - part);
                        long cst = 2 * nch;
                        for (int p = lo; p < hi; ++p)
                            cst += rcost[p][m3];
                        its.push_back({cst, l3, m3, lo, hi});
                        lo = hi;
                    }
                }
            std::vector<int> idx(its.size());
            for (size_t i = 0; i < its.size(); ++i)
                idx[i] = (int)i;
            std::stable_sort(idx.begin(), idx.end(),
                             [&](int x, int y) { return its[x].cost > its[y].cost; });
            std::vector<std::vector<int>> ls(nb);
            std::vector<long> load(nb, 0);
            for (int i : idx) {
                int w = 0;
                for (int k = 1; k < nb; ++k)
                    if (load[k] < load[w])
                        w = k;
                ls[w].push_back(i);
                load[w] += its[i].cost;
            }
            const long mx = *std::max_element(load.begin(), load.end());
            if (best < 0 || mx < best) {
                best = mx;
                items.swap(its);
                lists.swap(ls);
            }
        }
        std::vector<std::vector<int>> cols(L2);
        for (size_t i = 0; i < items.size(); ++i)
            cols[items[i].l3 * items[i].l3 + items[i].m3].push_back((int)i * nch);
        t.o3vsets.push_back(cols);
        for (int w = 0; w < nb; ++w) {
            t.o3rbeg.push_back((int)t.o3rowv.size() / 4);
            std::sort(lists[w].begin(), lists[w].end());
            int nrow = 0;
            for (int i : lists[w]) {
                const Item &it = items[i];
                for (int p = it.lo; p < it.hi; ++p, ++nrow) {
                    const int row = t.o3base[p] + it.m3;
                    t.o3rowv.push_back(t.o3mtv[2 * row]);
                    t.o3rowv.push_back(t.o3mtv[2 * row + 1]);
                    t.o3rowv.push_back(p | (it.m3 << 16));
                    t.o3rowv.push_back(i * nch);
                }
            }
            t.o3rows_max = std::max(t.o3rows_max, nrow);
        }
        t.o3rbeg.push_back((int)t.o3rowv.size() / 4);
    }
}

// Partial-D column sets for the finalisation, which sums into each (l3, m3)
// the columns of its set in the listed order: one set per split G of the
// vector-sparse form (its run columns, or the per-row columns when it keeps
// one per row), then the per-(block, m3) set of the other forms (the blocks
// of l3 in block order).
static void build_dsum(const mlmix_model_desc &d, HostTables &t)
{
    const int lmax = d.ace_lmax, L2 = (lmax + 1) * (lmax + 1), nch = d.n_species * d.ace_n_rad;
    t.dsum.clear();
    t.dsum_len = 0;
    int span = 0, ncol = 0;
    auto put = [&](const std::vector<std::vector<int>> &cols) -> int {
        const int off = (int)t.dsum.size();
        int k = 0;
        span = 0;
        for (int lm = 0; lm < L2; ++lm) {
            t.dsum.push_back(k);
            k += (int)cols[lm].size();
            for (int col : cols[lm])
                span = std::max(span, col / nch + 1);
        }
        t.dsum.push_back(k);
        for (int lm = 0; lm < L2; ++lm)
            t.dsum.insert(t.dsum.end(), cols[lm].begin(), cols[lm].end());
        t.dsum_len = std::max(t.dsum_len, L2 + 1 + k);
        ncol = k;
        return off;
    };
    std::vector<std::vector<int>> blocks(L2);
    if (d.ace_order >= 3)
        for (size_t p = 0; p < t.pb.size(); ++p)
            for (int m3 = 0; m3 < 2 * t.pb[p].l3 + 1; ++m3)
                blocks[t.pb[p].l3 * t.pb[p].l3 + m3].push_back(t.dpoff[p] + m3 * nch);
    const int per_block = put(blocks);
    const int per_block_span = span, per_block_ncol = ncol;
    for (int k = 0; k < kDSumBlocks; ++k) {
        t.dsum_off[k] = k < (int)t.o3vsets.size() ? put(t.o3vsets[k]) : per_block;
        t.dsum_span[k] = k < (int)t.o3vsets.size() ? span : per_block_span;
        t.dsum_ncol[k] = k < (int)t.o3vsets.size() ? ncol : per_block_ncol;
    }
    t.dsum_off[kDSumBlocks] = per_block;
    t.dsum_span[kDSumBlocks] = per_block_span;
    t.dsum_ncol[kDSumBlocks] = per_block_ncol;
}

// BF16 bits of a float, rounded to nearest with ties to even (the rounding
// the device's conversion applies to the products it packs).
static uint32_t bf16_bits(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, sizeof(u));
    if ((u & 0x7fffffffu) > 0x7f800000u)
        return (u >> 16) | 0x40u;  // NaN stays NaN
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

static void build_o3(const mlmix_model_desc &d, HostTables &t, int waves)
{
    const int nch = d.n_species * d.ace_n_rad, lmax = d.ace_lmax;
    const int nchp = (nch + 3) & ~3;
    const bool reduced = d.precision == MLMIX_BF16_CONTRACT || d.precision == MLMIX_FP8_CONTRACT;
    t.o3 = false;
    t.o3_kind = 0;
    if (d.ace_order < 3 || t.pb.empty() || d.precision == MLMIX_FP64)
        return;
    const bool narrow_ok = d.n_species == 1 && nch <= 16;
    const bool wide_ok = !narrow_ok && nch <= 32 &&
                         (d.precision == MLMIX_FP32 || d.precision == MLMIX_BF16_CONTRACT);
    if (!narrow_ok && !wide_ok)
        return;
    const int kind = narrow_ok ? 1 : 2;
    const int NT = kind == 1 ? 1 : (nchp + 15) / 16;  // channel tiles of the wide form
    const int NCP = 16 * NT;                          // LDS channel stride of the A rows
    const int NJ = nchp / 4, NJP = (NJ + 3) & ~3;
    const int nch2 = nchp;  // row width of the kernel: channels rounded up to 4
    std::vector<int> cost(t.pb.size(), 0);
    std::vector<std::vector<int>> rcost(t.pb.size());  // per (block, m3) row
    for (size_t p = 0; p < t.pb.size(); ++p) {
        const PBlock &b = t.pb[p];
        t.o3base.push_back((int)t.o3mt.size() / 2);
        for (int m3 = 0; m3 < 2 * b.l3 + 1; ++m3) {
            int e0 = t.gm3[b.gm3_off + m3], e1 = t.gm3[b.gm3_off + m3 + 1];
            int n_e = e1 - e0, ng = (n_e + 3) / 4;
            if (ng > 8)
                return;  // more than 32 entries in one row: keep the general kernel
            t.o3mt.push_back((int)t.o3g.size());  // entry index (pairs in o3o)
            t.o3mt.push_back(ng);
            t.o3mtv.push_back((int)t.o3g.size());
            t.o3mtv.push_back(n_e);
            if (n_e == 0)
                t.o3rows_empty = true;
            for (int e = e0; e < e0 + 4 * ng; ++e) {
                int o = 0;
                float g = 0.0f;
                if (e < e1) {
                    int m1 = t.gidx[e] & 0xff, m2 = t.gidx[e] >> 8;
                    int o1 = (b.l1 * b.l1 + m1) * NCP, o2 = (b.l2 * b.l2 + m2) * NCP;
                    o = o1 | (o2 << 16);
                    g = (float)t.gval[e];
                }
                int gbits;
                std::memcpy(&gbits, &g, sizeof(int));
                t.o3o.push_back(o);
                t.o3o.push_back(gbits);
                t.o3g.push_back(g);
            }
            // MFMA steps per row tile: sparse 16 rows x groups (x NT^2 tiles
            // in the wide form), dense in units of a 16x16x4 FP32 step
            // (reduced operands are 8x cheaper)
            const int rc = kind == 2 ? 16 * NT * NT * ng + nch2 * NT * NJ + 4
                                     : 16 * ng + (reduced ? std::max(1, nch2 / 8) : 4 * nch2) + 4;
            cost[p] += rc;
            rcost[p].push_back(rc);
        }
    }
    (void)lmax;
    // the kernel reads eight groups of every row: pad past the end
    for (int e = 0; e < 32; ++e) {
        t.o3o.push_back(0);
        t.o3o.push_back(0);
    }
    const size_t P = t.pb.size();
    // wide-form fragments: for the wide form, and for a single-species FP32
    // model too (the wide form can then be selected for comparisons)
    if (kind == 2 || d.precision == MLMIX_FP32) {
        const int ns = d.n_species;
        t.o3ww.assign((size_t)ns * P * nch2 * NT * 64 * NJP, 0.0);
        for (int z = 0; z < ns; ++z)
            for (size_t p = 0; p < P; ++p)
                for (int a = 0; a < nch; ++a)
                    for (int ct = 0; ct < NT; ++ct)
                        for (int l = 0; l < 64; ++l)
                            for (int j = 0; j < NJ; ++j) {
                                const int c = 16 * ct + (l & 15), b = NJ * (l >> 4) + j;
                                double v = 0.0;
                                if (b < nch && c < nch)
                                    v = t.W[(size_t)z * t.w_per_species + t.pb[p].w_off +
                                            ((size_t)a * nchp + b) * nchp + c];
                                t.o3ww[((((((size_t)z * P + p) * nch2 + a) * NT + ct) * 64 + l) *
                                        NJP) + j] = v;
                            }
        t.o3_wide_ready = true;
    }
    if (kind == 2 && d.precision == MLMIX_BF16_CONTRACT) {
        // BF16 fragments of the wide form's dense stage: per pass of eight
        // channels a (a0 = 8 pa), the pass's K values kk = (a - a0) nchp + b
        // in 32-deep steps; lane (c = 16 ct + l % 16, q = l / 16) holds
        // W[a][b][c] of kk = 32 st + 8 q + u, u < 8, rounded to nearest even
        const int ns = d.n_species, np = (nchp + 7) / 8, nstm = nchp / 4;
        t.o3wwb.assign((size_t)ns * P * np * NT * nstm * 64 * 4, 0);
        for (int z = 0; z < ns; ++z)
            for (size_t p = 0; p < P; ++p)
                for (int pa = 0; pa < np; ++pa) {
                    const int a0 = 8 * pa, kp = std::min(8, nchp - a0) * nchp;
                    for (int ct = 0; ct < NT; ++ct)
                        for (int st = 0; st < nstm; ++st)
                            for (int l = 0; l < 64; ++l) {
                                const int c = 16 * ct + (l & 15), q = l >> 4;
                                uint32_t bits[8];
                                for (int u = 0; u < 8; ++u) {
                                    const int kk = 32 * st + 8 * q + u;
                                    double v = 0.0;
                                    const int a = a0 + kk / nchp, b = kk % nchp;
                                    if (kk < kp && a < nch && b < nch && c < nch)
                                        v = t.W[(size_t)z * t.w_per_species + t.pb[p].w_off +
                                                ((size_t)a * nchp + b) * nchp + c];
                                    bits[u] = bf16_bits((float)v);
                                }
                                int32_t *dst = &t.o3wwb[(((((((size_t)z * P + p) * np + pa) * NT + ct) *
                                                            nstm + st) * 64 + l) * 4)];
                                for (int k = 0; k < 4; ++k)
                                    dst[k] = (int32_t)(bits[2 * k] | (bits[2 * k + 1] << 16));
                            }
                }
    }
    if (kind == 2) {
        t.o3sw.assign(P * 16, 1.0);
    } else {
    // weight fragments (and FP8 column scales)
    t.o3sw.assign(P * 16, 1.0);
    if (d.precision == MLMIX_FP8_CONTRACT)
        for (size_t p = 0; p < P; ++p)
            for (int c = 0; c < 16; ++c)
                t.o3sw[p * 16 + c] = c < nch ? t.wsc[p * nchp + c] : 0.0;
    t.o3w.assign(P * nch2 * 64 * 4, 0.0);
    for (size_t p = 0; p < P; ++p)
        for (int i = 0; i < nch2; ++i)
            for (int l = 0; l < 64; ++l)
                for (int j = 0; j < 4; ++j) {
                    // FP32: lane q holds b = (nch2 / 4) q + j, j < nch2 / 4
                    // (K over exactly the nch2^2 pairs); BF16 / FP8 (32-deep
                    // K steps): b = 4 q + j
                    const int c = l & 15, q = l >> 4, a = i;
                    const int njk = reduced ? 4 : nch2 / 4;
                    const int b = j < njk ? njk * q + j : nch2;  // j >= njk: zero
                    double v = 0.0;
                    if (a < nch && b < nch && c < nch) {
                        v = t.W[t.pb[p].w_off + ((size_t)a * nchp + b) * nchp + c];
                        if (d.precision == MLMIX_FP8_CONTRACT) {
                            double sw = t.o3sw[p * 16 + c];
                            v = sw > 0.0 ? v / sw : 0.0;
                        }
                    }
                    t.o3w[(((p * nch2) + i) * 64 + l) * 4 + j] = v;
                }
    }
    // reduced-precision fragments of the vector-sparse form (32-deep K steps):
    // step s covers channels a = A_PER s .. A_PER s + A_PER - 1 (A_PER =
    // min(8 / NJ, nch2)); for lane (c = l % 16, q = l / 16) value u < 8 is
    // W[a = A_PER s + u / NJ][b = NJ q + u % NJ][c] for u < A_PER NJ, else
    // zero; in the FP8 mode divided by the per-(block, c) scale.
    // Stored [block][s][lane][8].
    if (kind == 1) {
        const int njv = nch2 / 4, aper = std::min(8 / njv, nch2), nst = nch2 / aper;
        t.o3wr.assign(P * nst * 64 * 8, 0.0);
        for (size_t p = 0; p < P; ++p)
            for (int st = 0; st < nst; ++st)
                for (int l = 0; l < 64; ++l)
                    for (int u = 0; u < aper * njv; ++u) {
                        const int c = l & 15, q = l >> 4;
                        const int a = aper * st + u / njv, b = njv * q + u % njv;
                        if (a >= nch || b >= nch || c >= nch)
                            continue;
                        double v = t.W[t.pb[p].w_off + ((size_t)a * nchp + b) * nchp + c];
                        if (d.precision == MLMIX_FP8_CONTRACT) {
                            const double sw = t.o3sw[p * 16 + c];
                            v = sw > 0.0 ? v / sw : 0.0;
                        }
                        t.o3wr[(((p * nst) + st) * 64 + l) * 8 + u] = v;
                    }
    }
    // work items to waves, for a tile's block list split over G = 1, 2, 4, 8
    // workgroups (4 G bins). An item is a range of m3 rows of one block: for
    // G > 1, a block costing more than half of a bin's even share is cut into
    // row ranges of about that cost, so that no single block sets the time of
    // its wave. Items go longest first onto the least loaded bin; each bin
    // runs its items in (block, first row) order. Item code: block | first
    // row << 16 | end row << 24.
    long total = 0;
    for (size_t p = 0; p < P; ++p)
        total += cost[p];
    // the vector-sparse FP32 and BF16 forms sum runs of rows on chip (below);
    // the FP8 form scales each row's products by the row's own bound and
    // keeps one partial-D column per (block, m3)
    bool runs = kind == 1 && d.precision != MLMIX_FP8_CONTRACT;
    if (const char *e = std::getenv("MLMIX_O3_RUNS"))
        runs = runs && std::atoi(e) != 0;  // 0: one column per row (comparisons)
    t.o3vsets.clear();
    t.o3order.clear();
    t.o3wbeg.clear();
    t.o3rowv.clear();
    t.o3rbeg.clear();
    t.o3rows_max = 0;
    for (int G = 1; G <= kO3MaxSplit; G <<= 1) {
        // bins: the waves of the G workgroups sharing a tile (the wide form
        // always has four waves per workgroup)
        const int nb = (kind == 1 ? waves : 4) * G;
        // one workgroup per tile (large S): whole blocks (measured faster)
        const long cap = G == 1 ? total : std::max<long>(1, total / nb / 2);
        std::vector<std::pair<long, int>> items;  // (cost, code)
        for (size_t p = 0; p < P; ++p) {
            const int d3 = (int)rcost[p].size();
            const int k = (int)std::min<long>(d3, (cost[p] + cap - 1) / cap);
            int lo = 0;
            for (int part = 0; part < k; ++part) {
                const int hi = lo + (d3 - lo) / (k - part);  // near-even row counts
                long cst = 0;
                for (int r = lo; r < hi; ++r)
                    cst += rcost[p][r];
                items.push_back({cst, (int)p | (lo << 16) | (hi << 24)});
                lo = hi;
            }
        }
        std::stable_sort(items.begin(), items.end(),
                         [](const std::pair<long, int> &x, const std::pair<long, int> &y) {
                             return x.first > y.first;
                         });
        std::vector<std::vector<int>> lists(nb);
        std::vector<long> load(nb, 0);
        for (const auto &it : items) {
            int w = 0;
            for (int k = 1; k < nb; ++k)
                if (load[k] < load[w])
                    w = k;
            lists[w].push_back(it.second);
            load[w] += it.first;
        }
        for (int w = 0; w < nb; ++w) {
            t.o3wbeg.push_back((int)t.o3order.size());  // absolute offsets
            t.o3rbeg.push_back((int)t.o3rowv.size() / 4);
            std::sort(lists[w].begin(), lists[w].end(), [](int x, int y) {
                const int px = x & 0xffff, py = y & 0xffff;
                return px != py ? px < py : ((x >> 16) & 0xff) < ((y >> 16) & 0xff);
            });
            t.o3order.insert(t.o3order.end(), lists[w].begin(), lists[w].end());
            if (runs)
                continue;
            // the same bin as a flat list of rows (first entry, exact count,
            // block | m3 << 16, partial-D column of the row)
            int nrow = 0;
            for (int code : lists[w]) {
                const int p = code & 0xffff, lo = (code >> 16) & 0xff, hi = (code >> 24) & 0xff;
                for (int m3 = lo; m3 < hi; ++m3, ++nrow) {
                    const int row = t.o3base[p] + m3;
                    t.o3rowv.push_back(t.o3mtv[2 * row]);
                    t.o3rowv.push_back(t.o3mtv[2 * row + 1]);
                    t.o3rowv.push_back(p | (m3 << 16));
                    t.o3rowv.push_back(t.dpoff[p] + m3 * nch);
                }
            }
            t.o3rows_max = std::max(t.o3rows_max, nrow);
        }
        t.o3wbeg.push_back((int)t.o3order.size());
        if (!runs)
            t.o3rbeg.push_back((int)t.o3rowv.size() / 4);
    }
    if (runs)
        build_o3v_runs(t, lmax, nch, waves, total, rcost);
    // FP8 row-scale bound: sum of |g| over the row's entries
    t.o3gs.clear();
    for (size_t r = 0; r < t.o3mt.size() / 2; ++r) {
        double gs = 0.0;
        for (int e = t.o3mt[2 * r]; e < t.o3mt[2 * r] + 4 * t.o3mt[2 * r + 1]; ++e)
            gs += std::fabs(t.o3g[e]);
        t.o3gs.push_back(gs);
    }
    t.o3_nch2 = nch2;
    t.o3 = true;
    t.o3_kind = kind;
}

// Clamped uniform cubic B-splines on knots t(i) = clamp(i - 3, 0, npts - 1)
// (unit spacing): the four non-zero basis values at x by the Cox-de Boor
// recursion (host only: fits the per-span polynomials below).
static void host_bspline4(double x, int npts, int &first, double N[4])
{
    int sp = (int)std::floor(x);
    sp = sp < 0 ? 0 : (sp > npts - 2 ? npts - 2 : sp);
    const int k = sp + 3;
    auto t = [&](int q) -> double {
        int v = q - 3;
        v = v < 0 ? 0 : (v > npts - 1 ? npts - 1 : v);
        return double(v);
    };
    double left[4], right[4], Nn[4];
    Nn[0] = 1.0;
    for (int j = 1; j <= 3; ++j) {
        left[j] = x - t(k + 1 - j);
        right[j] = t(k + j) - x;
        double saved = 0.0;
        for (int r = 0; r < j; ++r) {
            double temp = Nn[r] / (right[r + 1] + left[j - r]);
            Nn[r] = saved + right[r + 1] * temp;
            saved = left[j - r] * temp;
        }
        Nn[j] = saved;
    }
    for (int r = 0; r < 4; ++r)
        N[r] = Nn[r];
    first = sp;
}

// Per-span cubic coefficients of the four basis functions in the local
// coordinate t = x/h - span (knot spacing h drops out): values at four
// interior points of each span, solved as a 4x4 Vandermonde system.
static std::vector<double> bspline_span_poly(int npts)
{
    std::vector<double> out((size_t)std::max(0, npts - 1) * 16, 0.0);
    const double tm[4] = {0.125, 0.375, 0.625, 0.875};
    for (int sp = 0; sp + 1 < npts; ++sp) {
        double Nv[4][4];  // [point][basis]
        for (int q = 0; q < 4; ++q) {
            int f;
            host_bspline4(sp + tm[q], npts, f, Nv[q]);
        }
        for (int r = 0; r < 4; ++r) {
            double A[4][5];
            for (int q = 0; q < 4; ++q) {
                double p = 1.0;
                for (int e = 0; e < 4; ++e) {
                    A[q][e] = p;
                    p *= tm[q];
                }
                A[q][4] = Nv[q][r];
            }
            for (int c = 0; c < 4; ++c) {  // Gaussian elimination, partial pivoting
                int piv = c;
                for (int q = c + 1; q < 4; ++q)
                    if (std::fabs(A[q][c]) > std::fabs(A[piv][c]))
                        piv = q;
                for (int e = 0; e < 5; ++e)
                    std::swap(A[c][e], A[piv][e]);
                for (int q = 0; q < 4; ++q)
                    if (q != c) {
                        double fct = A[q][c] / A[c][c];
                        for (int e = c; e < 5; ++e)
                            A[q][e] -= fct * A[c][e];
                    }
            }
            for (int e = 0; e < 4; ++e)
                out[(size_t)sp * 16 + r * 4 + e] = A[e][4] / A[e][e];
        }
    }
    return out;
}

static int build_tables(const mlmix_model_desc &d, HostTables &t, int o3_waves)
{
    const int ns = d.n_species, nr = d.ace_n_rad, lmax = d.ace_lmax;
    const int L1 = lmax + 1, L2 = L1 * L1, nch = ns * nr, K3 = nch * L1;
    const int nchp = (nch + 3) & ~3;  // W columns padded to a multiple of four
    t.K = ylm_norm(lmax);
    t.c0.assign(d.ace_c0, d.ace_c0 + ns);
    t.c1.assign(d.ace_c1, d.ace_c1 + (size_t)ns * nch);
    t.c2s.assign((size_t)ns * L1 * nch * nch, 0.0);
    if (d.ace_order >= 2) {
        for (int z = 0; z < ns; ++z)
            for (int l = 0; l < L1; ++l)
                for (int a = 0; a < nch; ++a)
                    for (int b = 0; b < nch; ++b) {
                        int lo = std::min(a, b), hi = std::max(a, b);
                        double v = d.ace_c2[(((size_t)z * L1 + l) * nch + lo) * nch + hi];
                        t.c2s[(((size_t)z * L1 + l) * nch + a) * nch + b] = (a == b) ? v : 0.5 * v;
                    }
    }
    if (d.ace_order >= 3) {
        std::vector<double> G = gaunt(lmax);
        for (int l3 = 0; l3 <= lmax; ++l3)
            for (int l1 = 0; l1 <= lmax; ++l1)
                for (int l2 = l1; l2 <= lmax; ++l2) {
                    if ((l1 + l2 + l3) & 1)
                        continue;
                    if (l3 > l1 + l2 || l3 < l2 - l1)
                        continue;
                    PBlock p{};
                    p.l1 = l1;
                    p.l2 = l2;
                    p.l3 = l3;
                    p.w_off = t.w_per_species;
                    p.gm3_off = (int)t.gm3.size();
                    for (int m3 = 0; m3 < 2 * l3 + 1; ++m3) {
                        t.gm3.push_back((int)t.gidx.size());
                        for (int m1 = 0; m1 < 2 * l1 + 1; ++m1)
                            for (int m2 = 0; m2 < 2 * l2 + 1; ++m2) {
                                double v = G[((size_t)(l1 * l1 + m1) * L2 + (l2 * l2 + m2)) * L2 +
                                             (l3 * l3 + m3)];
                                if (std::fabs(v) > 1e-12) {
                                    t.gidx.push_back(m1 | (m2 << 8));
                                    // LDS offsets of A_{., l1 m1} and A_{., l2 m2} in the
                                    // channel-fastest layout [lm][nchp]
                                    t.gofs.push_back(((l1 * l1 + m1) * nchp) |
                                                     (((l2 * l2 + m2) * nchp) << 16));
                                    t.gval.push_back(v);
                                }
                            }
                    }
                    t.gm3.push_back((int)t.gidx.size());
                    t.dpoff.push_back(t.dp_stride);
                    t.dp_stride += nch * (2 * l3 + 1);
                    t.pb.push_back(p);
                    t.w_per_species += nch * nchp * nchp;
                }
        // W[z][block][ab][c]: the symmetric coefficient C_{alpha beta gamma} =
        // c3[sorted] / (number of distinct orderings), doubled for l1 < l2 (the
        // (l2, l1) ordering gives the same contribution).
        t.W.assign((size_t)ns * t.w_per_species, 0.0);
        for (int z = 0; z < ns; ++z)
            for (const PBlock &p : t.pb)
                for (int a = 0; a < nch; ++a)
                    for (int b = 0; b < nch; ++b)
                        for (int c = 0; c < nch; ++c) {
                            int al = a * L1 + p.l1, be = b * L1 + p.l2, ga = c * L1 + p.l3;
                            int s[3] = {al, be, ga};
                            std::sort(s, s + 3);
                            int mult = (s[0] == s[2]) ? 1 : ((s[0] == s[1] || s[1] == s[2]) ? 3 : 6);
                            double v = d.ace_c3[(((size_t)z * K3 + s[0]) * K3 + s[1]) * K3 + s[2]] / mult;
                            if (p.l1 < p.l2)
                                v *= 2.0;
                            t.W[(size_t)z * t.w_per_species + p.w_off + ((size_t)a * nchp + b) * nchp + c] = v;
                        }
    }
    // FP8 weight scales: max |W| over K per (block, output channel), first
    // species (the reduced-precision contraction is for single-species models)
    t.wsc.assign(std::max<size_t>(1, t.pb.size() * (size_t)nchp), 1.0);
    for (size_t p = 0; p < t.pb.size(); ++p)
        for (int c = 0; c < nchp; ++c) {
            double mx = 0.0;
            for (int k = 0; k < nch * nchp; ++k)
                mx = std::max(mx, std::fabs(t.W[t.pb[p].w_off + (size_t)k * nchp + c]));
            t.wsc[p * nchp + c] = mx > 0.0 ? mx / 240.0 : 0.0;
        }
    build_o3(d, t, o3_waves);
    build_dsum(d, t);
    // cheap model
    int nb2 = d.uf3_n_knots2 + 2;
    t.up2 = bspline_span_poly(d.uf3_n_knots2);
    t.up3 = bspline_span_poly(d.uf3_n_knots3 > 0 ? d.uf3_n_knots3 : 2);
    t.u2.assign(d.uf3_c2, d.uf3_c2 + (size_t)ns * ns * nb2);
    for (int a = 0; a < ns; ++a)
        for (int b = 0; b < ns; ++b)
            for (int q = 0; q < nb2; ++q)
                if (t.u2[((size_t)a * ns + b) * nb2 + q] != t.u2[((size_t)b * ns + a) * nb2 + q])
                    return fail(MLMIX_E_ARG, "uf3_c2 is not symmetric in the species pair");
    if (d.uf3_n_knots3 > 0) {
        int nb3 = d.uf3_n_knots3 + 2;
        t.u3.assign(d.uf3_c3, d.uf3_c3 + (size_t)ns * nb3 * nb3 * nb3);
        for (int z = 0; z < ns; ++z)
            for (int p = 0; p < nb3; ++p)
                for (int q = 0; q < nb3; ++q)
                    for (int s = 0; s < nb3; ++s)
                        if (t.u3[(((size_t)z * nb3 + p) * nb3 + q) * nb3 + s] !=
                            t.u3[(((size_t)z * nb3 + q) * nb3 + p) * nb3 + s])
                            return fail(MLMIX_E_ARG, "uf3_c3 is not symmetric in its first two indices");
        // device layout: for every (z, a, b) and every first index c0 of a
        // span of the third (r_jk) basis, the four coefficients c0..c0+3
        // side by side, so that one span is one 4-wide load
        const int nsp = nb3 - 3;
        std::vector<double> x((size_t)ns * nb3 * nb3 * nsp * 4);
        for (int z = 0; z < ns; ++z)
            for (int a = 0; a < nb3; ++a)
                for (int b = 0; b < nb3; ++b)
                    for (int c0 = 0; c0 < nsp; ++c0)
                        for (int u = 0; u < 4; ++u)
                            x[((((size_t)z * nb3 + a) * nb3 + b) * nsp + c0) * 4 + u] =
                                t.u3[(((size_t)z * nb3 + a) * nb3 + b) * nb3 + c0 + u];
        t.u3.swap(x);
    }
    return MLMIX_OK;
}

template <typename T>
static void append(std::vector<char> &blob, size_t &off, const std::vector<double> &v)
{
    off = (blob.size() + 255) & ~(size_t)255;
    blob.resize(off + v.size() * sizeof(T) + 16);
    T *p = reinterpret_cast<T *>(blob.data() + off);
    for (size_t i = 0; i < v.size(); ++i)
        p[i] = T(v[i]);
}

template <typename I>
static void append_raw(std::vector<char> &blob, size_t &off, const std::vector<I> &v)
{
    off = (blob.size() + 255) & ~(size_t)255;
    blob.resize(off + v.size() * sizeof(I) + 16);
    if (!v.empty())
        std::memcpy(blob.data() + off, v.data(), v.size() * sizeof(I));
}

template <typename T>
static std::vector<char> pack(const HostTables &t, DevModel &m)
{
    std::vector<char> blob;
    append<T>(blob, m.ylmK, t.K);
    append<T>(blob, m.c0, t.c0);
    append<double>(blob, m.c0d, t.c0);
    append<T>(blob, m.c1, t.c1);
    append<T>(blob, m.c2s, t.c2s);
    append<T>(blob, m.W, t.W);
    append<T>(blob, m.gval, t.gval);
    append_raw(blob, m.pb, t.pb);
    append_raw(blob, m.gm3, t.gm3);
    append_raw(blob, m.gidx, t.gidx);
    append_raw(blob, m.gofs, t.gofs);
    append<T>(blob, m.u2, t.u2);
    append<T>(blob, m.u3, t.u3);
    append<T>(blob, m.up2, t.up2);
    append<T>(blob, m.up3, t.up3);
    append_raw(blob, m.dpoff, t.dpoff);
    append<float>(blob, m.wsc, t.wsc);
    append_raw(blob, m.o3o, t.o3o);
    append_raw(blob, m.o3mt, t.o3mt);
    append_raw(blob, m.o3mtv, t.o3mtv);
    append_raw(blob, m.o3rowv, t.o3rowv);
    append_raw(blob, m.o3rbeg, t.o3rbeg);
    append<float>(blob, m.o3wr, t.o3wr);
    append_raw(blob, m.o3base, t.o3base);
    append<float>(blob, m.o3w, t.o3w);
    append<float>(blob, m.o3ww, t.o3ww);
    append_raw(blob, m.o3wwb, t.o3wwb);
    append<float>(blob, m.o3sw, t.o3sw);
    append_raw(blob, m.o3order, t.o3order);
    append_raw(blob, m.o3wbeg, t.o3wbeg);
    append<float>(blob, m.o3gs, t.o3gs);
    append_raw(blob, m.dsum, t.dsum);
    return blob;
}

void pb_ranges(const Ctx &c, int *lo, int *hi)
{
    for (int l = 0; l <= kMaxLmax; ++l) {
        lo[l] = 0;
        hi[l] = 0;
    }
    // blocks are ordered by l3; the per-l3 ranges are stored at creation
    for (int l = 0; l <= c.m.lmax; ++l) {
        lo[l] = c.m_pb_lo[l];
        hi[l] = c.m_pb_hi[l];
    }
}

Grid make_grid(const Ctx &c, const Box &b)
{
    Grid g;
    g.bucket = 0;  // set with the workspace layout
    double half = 0.5 * c.r_list;
    g.ncell = 1;
    for (int k = 0; k < 3; ++k) {
        int nc = (int)std::floor(b.L[k] / half);
        if (nc < 1)
            nc = 1;
        g.nc[k] = nc;
        g.cs[k] = b.L[k] / nc;
        g.ncell *= nc;
    }
    return g;
}

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Records per cell bucket: four times the mean occupancy plus 8, at least 16.
static int bucket_size(int n, int ncell)
{
    const double mean = (double)n / (double)ncell;
    int bk = (int)std::ceil(4.0 * mean + 8.0);
    bk = (bk + 3) & ~3;
    return bk < 16 ? 16 : bk;
}

// Offsets of every workspace array for n atoms (all systems of a batch),
// ncell cell counts and nrec bucket records; nseg > 0 adds the segment
// tables of a batch.
static void layout_arrays(const Ctx &c, WsLayout &L, size_t ncell, size_t nrec, int nseg)
{
    const int n = L.n, cap = L.cap;
    int P = 1;
    while (P < cap)
        P <<= 1;
    L.P = P;
    L.nseg = nseg;
    size_t tsz = c.prec == MLMIX_FP64 ? 8 : 4;
    size_t off = 0;
    auto take = [&](size_t &field, size_t bytes) {
        field = off;
        off = align_up(off + bytes);
    };
    size_t nn = (size_t)(n > 0 ? n : 1);
    int nba = (n + kScanTile - 1) / kScanTile;
    int nsp = 2 * nba + 2;  // compaction block totals
    take(L.hdr, H_COUNT * sizeof(int));
    take(L.cell_count, ncell * sizeof(int));
    take(L.cell_atoms, nrec * sizeof(CellAtom));
    take(L.seedcore, nn);
    take(L.scan_part, (size_t)nsp * sizeof(int));
    take(L.nbr, nn * cap * sizeof(int));
    take(L.rev, nn * cap * sizeof(int));
    take(L.cnt, nn * sizeof(int));
    take(L.ref_pos, 3 * nn * sizeof(double));
    take(L.S_idx, nn * sizeof(int));
    take(L.M_idx, nn * sizeof(int));
    take(L.S_local, nn * sizeof(int));
    take(L.cand, nn);
    // superblocks of about 8 A (at most 32 per dimension) for the region lists
    if (nseg == 0) {
        size_t nsb = 1;
        for (int k = 0; k < 3; ++k) {
            const double len = L.grid.cs[k] * L.grid.nc[k];
            L.rgn[k] = std::max(1, std::min(32, (int)std::floor(len / 8.0)));
            nsb *= (size_t)L.rgn[k];
        }
        take(L.rgrid, nsb * (kRegionGridCap + 1) * sizeof(int));
    } else {
        L.rgn[0] = L.rgn[1] = L.rgn[2] = 0;
        take(L.rgrid, sizeof(int));
    }
    const size_t ns = (size_t)(L.scap > 0 ? L.scap : 1);
    take(L.A, ns * c.m.KAt * tsz);
    take(L.dEdA, ns * c.m.KAt * tsz);
    take(L.g, ns * cap * 3 * tsz);
    take(L.h, nn * cap * 3 * tsz);
    take(L.red, (size_t)std::max(kReduceBlocks, n <= kGatherKickMax ? (n + kGatherAtoms - 1) / kGatherAtoms : 0) * 3 *
                    sizeof(double));
    // (64 floats past the end: the sink of the contraction's masked lanes)
    take(L.dpart, (ns * (size_t)(c.m.dp_stride > 0 ? c.m.dp_stride : 1) + 64) * tsz);
    if (nseg > 0) {
        take(L.seg_of, nn * sizeof(int));
        take(L.segs, (size_t)nseg * sizeof(SegGeo));
        take(L.seg_status, (size_t)nseg * sizeof(int));
        take(L.seg_flag, (size_t)nseg * 4 * sizeof(int));
        take(L.seg_map, (size_t)nseg * sizeof(int));
        take(L.seg_red, nn * sizeof(double));  // per-atom kinetic energy of the step
    }
    L.total = off;
}

WsLayout make_layout(const Ctx &c, int n, int cap, const Box &b, int scap)
{
    WsLayout L{};
    L.n = n;
    L.cap = cap;
    L.scap = (scap <= 0 || scap > n) ? n : scap;
    L.grid = make_grid(c, b);
    L.grid.bucket = bucket_size(n, L.grid.ncell);
    layout_arrays(c, L, (size_t)L.grid.ncell, (size_t)L.grid.ncell * L.grid.bucket, 0);
    return L;
}

// Layout of a batch workspace: every system's own grid and buckets, their
// cells and records side by side (geo receives the device segment table).
static WsLayout make_batch_layout(const Ctx &c, const std::vector<SegGeo> &in, int cap, int scap,
                                  std::vector<SegGeo> &geo)
{
    WsLayout L{};
    long long n = 0, ncell = 0, nrec = 0;
    geo = in;
    for (SegGeo &G : geo) {
        G.grid = make_grid(c, G.box);
        G.grid.bucket = bucket_size(G.n, G.grid.ncell);
        G.cell0 = (int)ncell;
        G.rec0 = nrec;
        ncell += G.grid.ncell;
        nrec += (long long)G.grid.ncell * G.grid.bucket;
        n += G.n;
    }
    L.n = (int)n;
    L.cap = cap;
    L.scap = (scap <= 0 || scap > L.n) ? L.n : scap;
    L.grid = Grid{};
    L.grid.ncell = (int)ncell;
    L.grid.bucket = 0;  // per segment
    layout_arrays(c, L, (size_t)ncell, (size_t)nrec, (int)geo.size());
    return L;
}

__global__ void k_zero_i32(int *p, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = 0;
}

}  // namespace mlmix

// ------------------------------------------------------------------ ABI

static int check_box(const mlmix_ctx *ctx, const mlmix_box *box, Box &b)
{
    if (!box)
        return fail(MLMIX_E_ARG, "box is NULL");
    for (int k = 0; k < 3; ++k) {
        if (!(box->L[k] > 0.0) || !std::isfinite(box->L[k]))
            return fail(MLMIX_E_BOX, "box length must be positive and finite");
        if (box->periodic[k] && box->L[k] < 2.0 * ctx->c.r_list)
            return fail(MLMIX_E_BOX, "periodic box length below twice the list radius");
        b.L[k] = box->L[k];
        b.per[k] = box->periodic[k] ? 1 : 0;
    }
    return MLMIX_OK;
}

extern "C" int mlmix_create(const mlmix_model_desc *desc, mlmix_ctx **out)
try {
    if (!desc || !out)
        return fail(MLMIX_E_ARG, "NULL argument");
    *out = nullptr;
    const mlmix_model_desc &d = *desc;
    if (d.n_species < 1 || d.n_species > 8)
        return fail(MLMIX_E_ARG, "n_species must be 1..8");
    if (d.precision != MLMIX_FP64 && d.precision != MLMIX_FP32 &&
        d.precision != MLMIX_BF16_CONTRACT && d.precision != MLMIX_FP8_CONTRACT)
        return fail(MLMIX_E_ARG, "precision must be MLMIX_FP64, MLMIX_FP32, MLMIX_BF16_CONTRACT or "
                                 "MLMIX_FP8_CONTRACT");
    if (d.precision == MLMIX_FP8_CONTRACT && d.n_species != 1)
        return fail(MLMIX_E_ARG, "the FP8 contraction mode supports one species");
    if (d.ace_n_rad < 1 || d.ace_n_rad > kMaxNrad || d.ace_lmax < 0 || d.ace_lmax > kMaxLmax ||
        d.ace_order < 1 || d.ace_order > 3 || !(d.ace_rcut > 0.0))
        return fail(MLMIX_E_ARG, "ACE sizes out of range (n_rad 1..16, lmax 0..6, order 1..3)");
    if (!d.ace_c0 || !d.ace_c1 || (d.ace_order >= 2 && !d.ace_c2) || (d.ace_order >= 3 && !d.ace_c3))
        return fail(MLMIX_E_ARG, "missing ACE coefficient array");
    if (d.uf3_n_knots2 < 4 || d.uf3_n_knots2 > 64 || !(d.uf3_rcut2 > 0.0) || !d.uf3_c2)
        return fail(MLMIX_E_ARG, "UF3 2-body needs 4..64 knots, rcut2 > 0 and coefficients");
    if (d.uf3_n_knots3 != 0 && (d.uf3_n_knots3 < 4 || d.uf3_n_knots3 > 16 || !(d.uf3_rcut3 > 0.0) ||
                                !d.uf3_c3))
        return fail(MLMIX_E_ARG, "UF3 3-body needs 4..16 knots, rcut3 > 0 and coefficients");
    if (!(d.skin >= 0.0))
        return fail(MLMIX_E_ARG, "skin must be >= 0");
    int nch = d.n_species * d.ace_n_rad;
    int L2 = (d.ace_lmax + 1) * (d.ace_lmax + 1);
    if (((nch + 3) & ~3) * L2 > 1024)
        return fail(MLMIX_E_ARG, "atomic basis larger than 1024 entries (channels padded to 4)");
    if (nch * (2 * d.ace_lmax + 1) > 8 * 64)
        return fail(MLMIX_E_ARG, "order-3 output block larger than 512 entries");

    // owned here until every step succeeded (early returns release it)
    std::unique_ptr<mlmix_ctx> holder(new mlmix_ctx());
    mlmix_ctx *ctx = holder.get();
    Ctx &c = ctx->c;
    c.d = d;
    c.prec = d.precision == MLMIX_FP64 ? MLMIX_FP64 : MLMIX_FP32;
    c.qmode = d.precision == MLMIX_BF16_CONTRACT ? 1 : (d.precision == MLMIX_FP8_CONTRACT ? 2 : 0);
    // tuning overrides of the order-3 launch shape (benchmark sweeps)
    if (const char *e = std::getenv("MLMIX_ACE_TILE")) {
        int v = std::atoi(e);
        if (v == 1 || v == 2 || v == 4 || v == 8 || v == 16)
            c.ace_tile = v;
    }
    if (const char *e = std::getenv("MLMIX_ACE_STAGE_W"))
        c.ace_stage_w = std::atoi(e) ? 1 : 0;
    double rmax = std::max(d.ace_rcut, d.uf3_rcut2);
    if (d.uf3_n_knots3 > 0)
        rmax = std::max(rmax, d.uf3_rcut3);
    c.r_list = rmax + d.skin;
    HIP_OK(hipGetDevice(&c.device));
    {
        // device address of this GPU's copy of the allocation-free call's
        // workspace (once per device)
        const int rc_s = scratch_setup(c.device);
        if (rc_s != MLMIX_OK)
            return rc_s;
    }
    HostTables t;
    // waves per workgroup of the single-species order-3 kernel (tuning)
    if (const char *e = std::getenv("MLMIX_O3_WAVES"))
        c.o3_waves = std::atoi(e) == 8 ? 8 : 4;
    int rc = build_tables(d, t, c.o3_waves);
    if (rc != MLMIX_OK)
        return rc;
    DevModel &m = c.m;
    m.ns = d.n_species;
    m.nrad = d.ace_n_rad;
    m.lmax = d.ace_lmax;
    m.order = d.ace_order;
    m.nchan = nch;
    m.L2 = L2;
    m.KA = nch * L2;
    m.nchp = (nch + 3) & ~3;
    m.KAt = L2 * m.nchp;
    m.rc_exp = d.ace_rcut;
    m.rc2 = d.uf3_rcut2;
    m.rc3 = d.uf3_rcut3;
    m.nk2 = d.uf3_n_knots2;
    m.nk3 = d.uf3_n_knots3;
    m.nb2 = d.uf3_n_knots2 + 2;
    m.nb3 = d.uf3_n_knots3 > 0 ? d.uf3_n_knots3 + 2 : 0;
    m.n_pb = (int)t.pb.size();
    m.w_per_species = t.w_per_species;
    for (int l = 0; l <= kMaxLmax; ++l) {
        c.m_pb_lo[l] = 0;
        c.m_pb_hi[l] = 0;
    }
    for (int p = 0; p < (int)t.pb.size(); ++p) {
        int l3 = t.pb[p].l3;
        if (c.m_pb_hi[l3] == 0)
            c.m_pb_lo[l3] = p;
        c.m_pb_hi[l3] = p + 1;
    }
    {
        // Operation counts of the kernels as written (a multiply-add counts
        // two, a division or square root one).
        double KA = m.KA, nr = m.nrad, L2d = L2;
        // order-3 contraction per S atom: sparse stage 2 per (entry, a, b)
        // plus the coefficient product per (entry, a); dense stage 2 per
        // (a, b, c, m3)
        double con = 0.0, dense = 0.0;
        if (d.ace_order >= 3) {
            double nab = (double)nch * nch;
            for (const PBlock &p : t.pb) {
                int nnz = t.gm3[p.gm3_off + 2 * p.l3 + 1] - t.gm3[p.gm3_off];
                con += 2.0 * nab * nnz + (double)nch * nnz + 2.0 * nab * nch * (2 * p.l3 + 1);
                dense += 2.0 * nab * nch * (2 * p.l3 + 1);
            }
        }
        ctx->flops[0] = con;                                  // order-3 contraction, per S atom
        ctx->flops[1] = 16.0 + 6.0 * nr + 8.0 * L2d + 2.0 * nr * L2d;   // atomic basis, per pair
        ctx->flops[2] = 31.0 + 10.0 * nr + L2d * (4.0 * nr + 24.0);     // pair adjoint, per pair
        ctx->flops[3] = 96.0;                                 // cheap 2-body, per pair
        ctx->flops[4] = 444.0;  // cheap 3-body, per unordered leg pair (r_jk spline, 4x4x4
                                // contraction with the three derivatives, two leg forces)
        ctx->flops[5] = dense;                                // dense order-3 stage, per S atom
        // finalisation per S atom: per (channel, lm) the order-2 product
        // (2 per channel), dE/dA = c1 + 2 D2 + 3 D3, the energy term and the
        // weight (9), plus one add per listed partial-D column and channel
        ctx->flops[6] = (double)nch * L2d * ((d.ace_order >= 2 ? 2.0 * nch : 0.0) + 9.0) +
                        (d.ace_order >= 3 ? (double)t.dsum_ncol[0] * nch : 0.0);
    }
    c.max_ent = 0;
    c.max_gm3 = 0;
    c.max_ent_pb = 0;
    m.dp_stride = t.dp_stride;
    for (int k = 0; k < kDSumSets; ++k) {
        m.dsum_off[k] = t.dsum_off[k];
        m.dsum_span[k] = t.dsum_span[k];
        m.dsum_ncol[k] = t.dsum_ncol[k];
    }
    m.dsum_len = t.dsum_len;
    for (const PBlock &p : t.pb)
        c.max_ent_pb = std::max(c.max_ent_pb, t.gm3[p.gm3_off + 2 * p.l3 + 1] - t.gm3[p.gm3_off]);
    for (int l = 0; l <= d.ace_lmax; ++l) {
        if (c.m_pb_hi[l] <= c.m_pb_lo[l])
            continue;
        const PBlock &f = t.pb[c.m_pb_lo[l]], &la = t.pb[c.m_pb_hi[l] - 1];
        int g_lo = f.gm3_off, g_hi = la.gm3_off + 2 * l + 2;
        c.max_gm3 = std::max(c.max_gm3, g_hi - g_lo);
        c.max_ent = std::max(c.max_ent, t.gm3[g_hi - 1] - t.gm3[g_lo]);
    }
    c.o3 = t.o3 ? t.o3_kind : 0;
    c.o3_nch2 = t.o3_nch2;
    if (const char *e = std::getenv("MLMIX_FORK_AT"))
        c.fork_at = std::max(0, std::min(2, std::atoi(e)));
    if (const char *e = std::getenv("MLMIX_SIDE_BLOCKS"))
        c.side_blocks = std::max(-1, std::atoi(e));
    if (const char *e = std::getenv("MLMIX_REV_BLOCKS"))
        c.rev_blocks = std::max(1, std::atoi(e));
    if (const char *e = std::getenv("MLMIX_O3_MAX_SPLIT")) {
        int v = std::atoi(e);
        if (v == 1 || v == 2 || v == 4 || v == 8 || v == 16)
            c.o3_max_split = v;
    }
    if (const char *e = std::getenv("MLMIX_FUSE_FIN"))
        c.fuse_fin = std::atoi(e) ? 1 : 0;  // 0: the finalisation as its own kernel (comparisons)
    if (const char *e = std::getenv("MLMIX_O3_VALU"))
        c.o3v = std::atoi(e) ? 1 : 0;  // 0: matrix-core sparse stage (comparisons)
    if (t.o3rows_max > kO3VMaxRows || t.o3rows_empty)
        c.o3v = 0;  // a bin longer than the kernel's row registers hold, or an empty row
    if (const char *e = std::getenv("MLMIX_BASIS_CHUNKS"))
        c.basis_chunks = std::max(-1, std::min(1, std::atoi(e)));
    if (const char *e = std::getenv("MLMIX_PAIR_HALF"))
        c.pair_half = std::atoi(e) ? 1 : 0;  // 0: one atom per wave (comparisons)
    if (const char *e = std::getenv("MLMIX_BASIS_MFMA"))
        c.basis_mfma = std::atoi(e) ? 1 : 0;  // VALU kernels (comparisons)
    if (const char *e = std::getenv("MLMIX_ACE_O3")) {
        const int v = std::atoi(e);
        if (!v)
            c.o3 = 0;  // general block kernel (comparisons)
        else if (v == 2 && c.o3 == 1 && c.qmode == 0 && t.o3_wide_ready)
            c.o3 = 2;  // the wide form for a single-species model (comparisons)
    }
    {
        int lim = 0;
        if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, c.device) ==
                hipSuccess &&
            lim > 0)
            c.max_lds = lim;
    }
    if (c.o3 == 2 && (o3w_lds_bytes(c) > (size_t)c.max_lds || o3w_prepare(c) != hipSuccess)) {
        (void)hipGetLastError();
        c.o3 = 0;  // the wide form does not fit this device: VALU blocks
    }
    if ((c.qmode == 2 && c.o3 != 1) || (c.qmode == 1 && c.o3 == 0)) {
        return fail(MLMIX_E_ARG, "the FP8 contraction mode needs a single-species model with at "
                                 "most 16 channels, the BF16 mode a model of at most 32 channels "
                                 "(species x radial functions), both correlation order 3");
    }
    std::vector<char> blob = c.prec == MLMIX_FP64 ? pack<double>(t, m) : pack<float>(t, m);
    m.bytes = blob.size();
    hipError_t e = hipMalloc(&m.base, m.bytes);
    if (e != hipSuccess)
        return fail_hip("hipMalloc(model)", e);
    e = hipMemcpy(m.base, blob.data(), m.bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(m.base);
        return fail_hip("hipMemcpy(model)", e);
    }
    *out = holder.release();
    return MLMIX_OK;
} catch (...) {
    return host_exception();
}

extern "C" int mlmix_destroy(mlmix_ctx *ctx)
try {
    if (!ctx)
        return MLMIX_OK;
    for (PendingEvent &p : ctx->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (hipEvent_t e : ctx->pool)
        (void)hipEventDestroy(e);
    for (auto &kv : ctx->side) {
        if (kv.second.s)
            (void)hipStreamDestroy(kv.second.s);
        if (kv.second.fork)
            (void)hipEventDestroy(kv.second.fork);
        if (kv.second.join)
            (void)hipEventDestroy(kv.second.join);
    }
    if (ctx->c.m.base)
        (void)hipFree(ctx->c.m.base);
    delete ctx;
    return MLMIX_OK;
} catch (...) {
    return host_exception();
}

extern "C" double mlmix_list_radius(const mlmix_ctx *ctx) { return ctx ? ctx->c.r_list : 0.0; }

extern "C" int mlmix_workspace_size(const mlmix_ctx *ctx, int32_t n_atoms, int32_t nbr_cap,
                                    int32_t s_cap, const mlmix_box *box, size_t *bytes)
try {
    if (!ctx || !bytes)
        return fail(MLMIX_E_ARG, "NULL argument");
    if (n_atoms < 0 || nbr_cap < 1 || nbr_cap > kMaxCap)
        return fail(MLMIX_E_ARG, "n_atoms >= 0 and 1 <= nbr_cap <= 256 required");
    Box b;
    int rc = check_box(ctx, box, b);
    if (rc)
        return rc;
    WsLayout L = make_layout(ctx->c, n_atoms, nbr_cap, b, s_cap);
    if ((double)L.grid.ncell * L.grid.bucket >= 2147483647.0)
        return fail(MLMIX_E_ARG, "box too large for the cell grid (2^31 bucket records)");
    *bytes = L.total;
    return MLMIX_OK;
} catch (...) {
    return host_exception();
}

extern "C" int mlmix_workspace_init(mlmix_ctx *ctx, void *stream, void *ws, size_t ws_bytes,
                                    int32_t n_atoms, int32_t nbr_cap, int32_t s_cap,
                                    const mlmix_box *box)
try {
    if (!ctx || !ws)
        return fail(MLMIX_E_ARG, "NULL argument");
    if (n_atoms < 0 || nbr_cap < 1 || nbr_cap > kMaxCap)
        return fail(MLMIX_E_ARG, "n_atoms >= 0 and 1 <= nbr_cap <= 256 required");
    Box b;
    int rc = check_box(ctx, box, b);
    if (rc)
        return rc;
    WsLayout L = make_layout(ctx->c, n_atoms, nbr_cap, b, s_cap);
    if ((double)L.grid.ncell * L.grid.bucket >= 2147483647.0)
        return fail(MLMIX_E_ARG, "box too large for the cell grid (2^31 bucket records)");
    if (ws_bytes < L.total)
        return fail(MLMIX_E_WORKSPACE, "workspace smaller than mlmix_workspace_size()");
    hipStream_t s = static_cast<hipStream_t>(stream);
    k_zero_i32<<<1, H_COUNT, 0, s>>>(at<int>(ws, L.hdr), H_COUNT);
    // cell counts start at zero; afterwards the reverse-slot pass of every
    // rebuild clears them
    k_zero_i32<<<(L.grid.ncell + 255) / 256, 256, 0, s>>>(at<int>(ws, L.cell_count), L.grid.ncell);
    HIP_OK(hipGetLastError());
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->batch.erase(ws);  // a single system now
    auto prev = ctx->ws.find(ws);
    if (prev == ctx->ws.end() || prev->second.n != L.n)
        ctx->lang.erase(ws);  // the noise buffer was sized for another system
    ctx->ws[ws] = L;
    return MLMIX_OK;
} catch (...) {
    return host_exception();
}

static int lookup(mlmix_ctx *ctx, void *ws, int n, const mlmix_box *box, WsLayout &L, Box &b)
{
    int rc = check_box(ctx, box, b);
    if (rc)
        return rc;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        auto it = ctx->ws.find(ws);
        if (it == ctx->ws.end())
            return fail(MLMIX_E_STATE, "workspace was not initialised with mlmix_workspace_init");
        L = it->second;
    }
    if (L.nseg > 0)
        return fail(MLMIX_E_ARG, "a batch workspace (mlmix_batch_init) needs the mlmix_batch_* calls");
    if (L.n != n)
        return fail(MLMIX_E_ARG, "n_atoms differs from the workspace's");
    Grid g = make_grid(ctx->c, b);
    if (g.nc[0] != L.grid.nc[0] || g.nc[1] != L.grid.nc[1] || g.nc[2] != L.grid.nc[2])
        return fail(MLMIX_E_ARG, "box grid changed: call mlmix_workspace_init again");
    g.bucket = L.grid.bucket;
    L.grid = g;
    return MLMIX_OK;
}

static int compute_impl(mlmix_ctx *ctx, hipStream_t s, void *ws, const WsLayout &L, const Box &b,
                        const double *pos, const int32_t *species, const mlmix_region *regions,
                        int32_t n_regions, double r_buffer, uint32_t mode, double *forces,
                        double *e_exp, double *e_cheap, double *lambda, uint8_t *flags,
                        int32_t *n_expensive, double *f_exp, double *f_cheap,
                        const KickArgs *kick = nullptr, const LangevinArgs *lang = nullptr,
                        double *red_out = nullptr, bool disp_checked = false)
{
    const Ctx &c = ctx->c;
    int m = (int)(mode & 0xff);
    bool energy_only = (mode & MLMIX_ENERGY_ONLY) != 0;
    // the second stream only beside the expensive chain of a mixed step: in
    // the all-cheap and all-expensive modes there is nothing for its kernels
    // to overlap with, and the fork and join events cost more than they save
    bool fork = (mode & MLMIX_SINGLE_STREAM) == 0 && m == MLMIX_MODE_MIXED;
    const bool masked = (mode & MLMIX_CHEAP_MASKED) != 0 && m == MLMIX_MODE_MIXED;
    SideStream sd;
    if (fork) {
        // the workspace's second stream is created by its first forked
        // evaluation outside a graph capture; a capture before that runs on
        // the caller's stream alone
        hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
        HIP_OK(hipStreamIsCapturing(s, &cst));
        std::lock_guard<std::mutex> g(ctx->mu);
        SideStream &e = ctx->side[ws];
        if (!e.s && cst == hipStreamCaptureStatusNone) {
            HIP_OK(hipStreamCreateWithFlags(&e.s, hipStreamNonBlocking));
            HIP_OK(hipEventCreateWithFlags(&e.fork, hipEventDisableTiming));
            HIP_OK(hipEventCreateWithFlags(&e.join, hipEventDisableTiming));
        }
        sd = e;
        fork = sd.s != nullptr;
    }
    hipStream_t s2 = fork ? sd.s : s;  // stream of the reverse slots and the cheap potential
    // workgroup cap of those two kernels when they run beside the expensive
    // chain (MLMIX_SIDE_BLOCKS; none by default: with the workgroup pair
    // adjoint the expensive chain of an 8,193-atom step is short enough that
    // the cheap potential needs the whole GPU beside it, 95.7 against
    // 100.9 us per step with one workgroup per compute unit)
    const int rev_blocks = c.rev_blocks;
    const int side_blocks = (!fork || m == MLMIX_MODE_ALL_CHEAP)
                                ? 0
                                : (c.side_blocks >= 0 ? c.side_blocks : 0);
    {
        StageTimer t(ctx, s, ST_NBR);
        RegionArgs ra{m, species, c.m.ns, regions, n_regions, r_buffer, lambda, flags, nullptr,
                      (mode & MLMIX_SEEDED) ? 1 : 0, nullptr};
        if (red_out) {  // the previous step's energy partials (multi-step call)
            ra.red_part = at<double>(ws, L.red);
            ra.red_nb = (L.n + kGatherAtoms - 1) / kGatherAtoms;
            ra.red_out = red_out;
        }
        launch_neighbors(s, ws, L, b, c.r_list, pos, (mode & MLMIX_FORCE_REBUILD) ? 1 : 0,
                         c.d.skin, ra, disp_checked);
    }
    // fork: reverse slots and the cheap potential need only the list; they are
    // started after the neighbour rows (fork_at 0) or after the atomic basis
    // (fork_at 1, beside the matrix-core contraction)
    bool fork_recorded = false;
    auto record_fork = [&]() -> int {
        if (fork && !fork_recorded) {
            HIP_OK(hipEventRecord(sd.fork, s));
            fork_recorded = true;
        }
        return MLMIX_OK;
    };
    auto fork_side = [&]() -> int {
        if (fork) {
            int rc = record_fork();
            if (rc)
                return rc;
            HIP_OK(hipStreamWaitEvent(sd.s, sd.fork, 0));
        }
        {
            StageTimer t(ctx, s2, ST_REV);
            launch_reverse(s2, ws, L, side_blocks > 0 ? rev_blocks : 0);
        }
        if (!energy_only) {
            if (m != MLMIX_MODE_ALL_EXPENSIVE) {
                StageTimer t(ctx, s2, ST_UF3);
                launch_uf3(s2, c, ws, L, b, pos, species, e_cheap, side_blocks,
                           masked ? flags : nullptr);
            } else {
                launch_fill_f64(s2, e_cheap, 0.0, (size_t)L.n);
            }
        }
        if (fork)
            HIP_OK(hipEventRecord(sd.join, sd.s));
        return MLMIX_OK;
    };
    // fork_at 0: side kernels issued right after the rows; 2: fork point
    // recorded after the rows, side kernels issued after the compaction (so
    // that a captured graph keeps the expensive chain on the first queue);
    // 1: both after the atomic basis
    // With the cheap potential masked its kernel needs the final masks: the
    // fork point then follows the region stage.
    const bool late = c.fork_at == 1 && m != MLMIX_MODE_ALL_CHEAP && !masked;
    if (c.fork_at == 2 && !masked) {
        int rc = record_fork();
        if (rc)
            return rc;
    } else if (!late && !masked) {
        int rc = fork_side();
        if (rc)
            return rc;
    }
    {
        StageTimer t(ctx, s, ST_REG);
        RegionArgs ra{m, species, c.m.ns, regions, n_regions, r_buffer, lambda, flags, nullptr,
                      (mode & MLMIX_SEEDED) ? 1 : 0, nullptr};
        launch_regions(s, ws, L, b, m, pos, r_buffer, flags, (mode & MLMIX_FORCE_REBUILD) ? 1 : 0,
                       ra);
        if (masked)
            launch_cheap_buffer(s, ws, L, b, pos, r_buffer, flags);
    }
    if (masked) {
        int rc = record_fork();
        if (rc)
            return rc;
    }
    {
        StageTimer t(ctx, s, ST_CMP);
        launch_compact(s, ws, L, flags, n_expensive);
    }
    if (c.fork_at == 2 || masked) {
        int rc = fork_side();
        if (rc)
            return rc;
    }
    if (m != MLMIX_MODE_ALL_CHEAP) {
        {
            StageTimer t(ctx, s, ST_BASIS);
            launch_ace_basis(s, c, ws, L, b, pos, species);
        }
        if (late) {
            int rc = fork_side();
            if (rc)
                return rc;
        }
        {
            // the matrix-core contraction is one kernel: timed by its own events
            StageTimer t(ctx, s, ST_CONTRACT, c.o3 && c.prec != MLMIX_FP64);
            launch_ace_contract(s, c, ws, L, species, t.k0, t.k1);
        }
        // the finalisation runs inside the pair adjoint where that kernel
        // can take it (the energy-only call keeps its own kernel)
        const bool fused = !energy_only && ace_fin_fused(c, L);
        if (!fused) {
            StageTimer t(ctx, s, ST_FIN);
            launch_ace_finalize(s, c, ws, L, species, e_exp);
        }
        if (!energy_only) {
            StageTimer t(ctx, s, ST_PAIR);
            launch_ace_pairgrad(s, c, ws, L, b, pos, species, nullptr, fused ? e_exp : nullptr);
        }
    }
    // join
    if (fork)
        HIP_OK(hipStreamWaitEvent(s, sd.join, 0));
    if (energy_only) {
        launch_gather_blend(s, c, ws, L, 0, 0, lambda, nullptr, e_exp, nullptr, nullptr, 1.0);
        HIP_OK(hipGetLastError());
        return MLMIX_OK;
    }
    {
        // timed by the kernel's own events (a bracket on the stream would also
        // hold the wait for the second stream's join)
        StageTimer t(ctx, s, ST_GATHER, true);
        launch_gather_blend(s, c, ws, L, m != MLMIX_MODE_ALL_CHEAP, m != MLMIX_MODE_ALL_EXPENSIVE,
                            lambda, forces, e_exp, f_exp, f_cheap, 1.0, kick, lang, t.k0, t.k1);
    }
    HIP_OK(hipGetLastError());
    return MLMIX_OK;
}

static int check_compute_args(mlmix_ctx *ctx, const double *pos, const int32_t *species,
                              const mlmix_region *regions, int32_t n_regions, double r_buffer,
                              uint32_t mode, double *forces, double *e_exp, double *e_cheap,
                              double *lambda, uint8_t *flags, int32_t n_atoms)
{
    int m = (int)(mode & 0xff);
    if (m != MLMIX_MODE_MIXED && m != MLMIX_MODE_ALL_EXPENSIVE && m != MLMIX_MODE_ALL_CHEAP)
        return fail(MLMIX_E_ARG, "unknown mode");
    if (mode & ~(0xffu | MLMIX_FORCE_REBUILD | MLMIX_ENERGY_ONLY | MLMIX_SINGLE_STREAM |
                 MLMIX_SEEDED | MLMIX_CHEAP_MASKED))
        return fail(MLMIX_E_ARG, "unknown mode flag");
    // per-atom arrays may be NULL for an empty system (nothing is read or written)
    if (n_atoms > 0 && (!pos || !species || !e_exp || !lambda || !flags))
        return fail(MLMIX_E_ARG, "NULL array argument");
    if (n_atoms > 0 && !(mode & MLMIX_ENERGY_ONLY) && (!forces || !e_cheap))
        return fail(MLMIX_E_ARG, "forces and e_cheap are required unless MLMIX_ENERGY_ONLY");
    if (m == MLMIX_MODE_MIXED) {
        if (n_regions < 0 || (n_regions > 0 && !regions))
            return fail(MLMIX_E_ARG, "bad region array");
        if (!(r_buffer >= 0.0) || r_buffer > ctx->c.r_list)
            return fail(MLMIX_E_ARG, "r_buffer must lie in [0, list radius]");
    }
    return MLMIX_OK;
}

// An empty system: the counts and energy sums are zero, nothing else is touched.
static int empty_outputs(hipStream_t s, int32_t *n_expensive, double *energies, int n_energies)
{
    if (n_expensive)
        k_zero_i32<<<1, 64, 0, s>>>(n_expensive, 2);
    if (energies)
        launch_fill_f64(s, energies, 0.0, (size_t)3 * n_energies);
    HIP_OK(hipGetLastError());
    return MLMIX_OK;
}

extern "C" int mlmix_compute(mlmix_ctx *ctx, void *stream, void *ws, int32_t n_atoms,
                             const double *pos, const int32_t *species, const mlmix_box *box,
                             const mlmix_region *regions, int32_t n_regions, double r_buffer,
                             uint32_t mode, double *forces, double *e_exp, double *e_cheap,
                             double *lambda, uint8_t *flags, int32_t *n_expensive,
                             double *f_exp, double *f_cheap)
try {
    if (!ctx || !ws)
        return fail(MLMIX_E_ARG, "NULL context or workspace");
    WsLayout L;
    Box b;
    int rc = lookup(ctx, ws, n_atoms, box, L, b);
    if (rc)
        return rc;
    rc = check_compute_args(ctx, pos, species, regions, n_regions, r_buffer, mode, forces, e_exp,
                            e_cheap, lambda, flags, n_atoms);
    if (rc)
        return rc;
    if (L.n == 0)
        return empty_outputs(static_cast<hipStream_t>(stream), n_expensive, nullptr, 0);
    return compute_impl(ctx, static_cast<hipStream_t>(stream), ws, L, b, pos, species, regions,
                        n_regions, r_buffer, mode, forces, e_exp, e_cheap, lambda, flags,
                        n_expensive, f_exp, f_cheap);
} catch (...) {
    return host_exception();
}

extern "C" int mlmix_compute_noalloc(mlmix_ctx *ctx, void *stream, int32_t n_atoms,
                                     int32_t nbr_cap, int32_t s_cap, const double *pos,
                                     const int32_t *species, const mlmix_box *box,
                                     const mlmix_region *regions, int32_t n_regions,
                                     double r_buffer, uint32_t mode, double *forces,
                                     double *e_exp, double *e_cheap, double *lambda,
                                     uint8_t *flags, int32_t *n_expensive, int32_t *status,
                                     size_t *bytes_used)
try {
    if (!ctx)
        return fail(MLMIX_E_ARG, "NULL context");
    if (n_atoms < 0 || nbr_cap < 1 || nbr_cap > kMaxCap)
        return fail(MLMIX_E_ARG, "n_atoms >= 0 and 1 <= nbr_cap <= 256 required");
    if (mode & ~(0xffu | MLMIX_FORCE_REBUILD | MLMIX_SINGLE_STREAM | MLMIX_SEEDED |
                 MLMIX_CHEAP_MASKED))
        return fail(MLMIX_E_ARG, "unknown or unsupported mode flag (MLMIX_ENERGY_ONLY is not "
                                 "available here)");
    Box b;
    int rc = check_box(ctx, box, b);
    if (rc)
        return rc;
    rc = check_compute_args(ctx, pos, species, regions, n_regions, r_buffer, mode, forces, e_exp,
                            e_cheap, lambda, flags, n_atoms);
    if (rc)
        return rc;
    const WsLayout L = make_layout(ctx->c, n_atoms, nbr_cap, b, s_cap);
    if (bytes_used)
        *bytes_used = L.total;
    if ((double)L.grid.ncell * L.grid.bucket >= 2147483647.0)
        return fail(MLMIX_E_ARG, "box too large for the cell grid (2^31 bucket records)");
    if (L.total > (size_t)MLMIX_NOALLOC_SCRATCH_BYTES)
        return fail(MLMIX_E_WORKSPACE, "this system needs more workspace than the library's "
                                       "static scratch (MLMIX_NOALLOC_SCRATCH_BYTES; *bytes_used "
                                       "holds the need): lower s_cap or nbr_cap, or use "
                                       "mlmix_compute with a workspace");
    void *ws = scratch_ptr(ctx->c.device);
    if (!ws)
        return fail(MLMIX_E_STATE, "the static scratch of this device was not set up "
                                   "(mlmix_create on this device failed or was not called)");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (L.n == 0) {
        if (status)
            k_zero_i32<<<1, 64, 0, s>>>(status, 2);
        return empty_outputs(s, n_expensive, nullptr, 0);
    }
    // the scratch keeps whatever the last call on this GPU left: clear the
    // header and the cell counts with fill kernels (no memset nodes, so the
    // call may be captured), then build the list afresh
    k_zero_i32<<<1, H_COUNT, 0, s>>>(at<int>(ws, L.hdr), H_COUNT);
    k_zero_i32<<<(L.grid.ncell + 255) / 256, 256, 0, s>>>(at<int>(ws, L.cell_count),
                                                           L.grid.ncell);
    HIP_OK(hipGetLastError());
    struct NoTimers {
        NoTimers() { tl_no_timers = true; }
        ~NoTimers() { tl_no_timers = false; }
    } no_timers;
    rc = compute_impl(ctx, s, ws, L, b, pos, species, regions, n_regions, r_buffer,
                      mode | MLMIX_FORCE_REBUILD | MLMIX_SINGLE_STREAM, forces, e_exp, e_cheap,
                      lambda, flags, n_expensive, nullptr, nullptr);
    if (rc)
        return rc;
    if (status) {  // the status word and the largest row count of this call
        static_assert(H_REQCAP == H_STATUS + 1, "status words are adjacent");
        launch_copy_i32(s, status, at<int>(ws, L.hdr) + H_STATUS, 2);
        HIP_OK(hipGetLastError());
    }
    return MLMIX_OK;
} catch (...) {
    return host_exception();
}

extern "C" int mlmix_backward(mlmix_ctx *ctx, void *stream, void *ws, int32_t n_atoms,
                              const double *pos, const int32_t *species, const mlmix_box *box,
                              const double *grad_e, double *grad_pos)
try {
    if (!ctx || !ws || !pos || !species || !grad_e || !grad_pos)
        return fail(MLMIX_E_ARG, "NULL argument");
    WsLayout L;
    Box b;
    int rc = lookup(ctx, ws, n_atoms, box, L, b);
    if (rc)
        return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    launch_ace_pairgrad(s, ctx->c, ws, L, b, pos, species, grad_e, nullptr);
    launch_gather_blend(s, ctx->c, ws, L, 1, 0, nullptr, grad_pos, nullptr, nullptr, nullptr, -1.0);
    HIP_OK(hipGetLastError());
    return MLMIX_OK;
} catch (...) {
    return host_exception();
}

extern "C" int mlmix_energy_reduce(mlmix_ctx *ctx, void *stream, void *ws, int32_t n_atoms,
                                   const double *e_exp, const double *e_cheap, const double *vel,
                                   const double *mass, double *energies)
try {
    if (!ctx || !ws || !energies)
        return fail(MLMIX_E_ARG, "NULL argument");
    WsLayout L;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        auto it = ctx->ws.find(ws);
        if (it == ctx->ws.end())
            return fail(MLMIX_E_STATE, "workspace was not initialised");
        L = it->second;
    }
    if (L.n != n_atoms)
        return fail(MLMIX_E_ARG, "n_atoms differs from the workspace's");
    launch_reduce(static_cast<hipStream_t>(stream), ws, L, e_exp, e_cheap, vel, mass, energies);
    HIP_OK(hipGetLastError());
    return MLMIX_OK;
} catch (...) {
    return host_exception();
}

extern "C" int mlmix_set_langevin(mlmix_ctx *ctx, void *ws, int32_t n_atoms,
                                  double temperature_K, double damping_fs, const double *xi)
try {
    if (!ctx || !ws)
        return fail(MLMIX_E_ARG, "NULL argument");
    if (!(temperature_K >= 0.0) || !std::isfinite(temperature_K) || !std::isfinite(damping_fs))
        return fail(MLMIX_E_ARG, "temperature must be finite and non-negative, damping finite");
    if (damping_fs > 0.0 && !xi)
        return fail(MLMIX_E_ARG, "a thermostat needs the noise buffer");
    std::lock_guard<std::mutex> g(ctx->mu);
    auto it = ctx->ws.find(ws);
    if (it == ctx->ws.end())
        return fail(MLMIX_E_STATE, "workspace was not initialised with mlmix_workspace_init");
    if (it->second.n != n_atoms)
        return fail(MLMIX_E_ARG, "n_atoms differs from the workspace's");
    if (damping_fs > 0.0)
        ctx->lang[ws] = LangevinSet{temperature_K, damping_fs, xi};
    else
        ctx->lang.erase(ws);
    return MLMIX_OK;
} catch (...) {
    return host_exception();
}

extern "C" int mlmix_vv_step(mlmix_ctx *ctx, void *stream, void *ws, int32_t n_atoms, double *pos,
                             double *vel, const double *mass, const int32_t *species, double dt,
                             const mlmix_box *box, const mlmix_region *regions, int32_t n_regions,
                             double r_buffer, uint32_t mode, double *forces, double *e_exp,
                             double *e_cheap, double *lambda, uint8_t *flags,
                             int32_t *n_expensive, double *energies)
try {
    if (!ctx || !ws || (n_atoms > 0 && (!vel || !mass)))
        return fail(MLMIX_E_ARG, "NULL argument");
    if (mode & MLMIX_ENERGY_ONLY)
        return fail(MLMIX_E_ARG, "MLMIX_ENERGY_ONLY is not valid for an MD step");
    if (!(dt > 0.0))
        return fail(MLMIX_E_ARG, "dt must be positive");
    WsLayout L;
    Box b;
    int rc = lookup(ctx, ws, n_atoms, box, L, b);
    if (rc)
        return rc;
    rc = check_compute_args(ctx, pos, species, regions, n_regions, r_buffer, mode, forces, e_exp,
                            e_cheap, lambda, flags, n_atoms);
    if (rc)
        return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (L.n == 0)
        return empty_outputs(s, n_expensive, energies, 1);
    // the drift also does the skin check of the new positions
    const DispCheck dc = disp_check_args(ws, L, ctx->c.d.skin);
    {
        StageTimer t(ctx, s, ST_VV);
        launch_vv_kick_drift(s, ws, L, b, pos, vel, mass, forces, dt, 1, &dc);
    }
    // small systems: closing half kick and energy partials inside the gather
    const bool fused = energies && L.n > 0 && L.n <= kGatherKickMax;
    KickArgs ka{vel, mass, dt, e_cheap, nullptr, energies};
    LangevinSet ls;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        auto it = ctx->lang.find(ws);
        if (it != ctx->lang.end())
            ls = it->second;
    }
    // friction and noise use the half-step velocity the opening kick just made
    LangevinArgs la{vel, mass, ls.xi, 0.0, 0.0};
    if (ls.tau > 0.0) {
        la.c_fric = 1.0 / (kKappa * ls.tau);
        la.c_rand = 2.0 * kBoltzmann * ls.temperature / (kKappa * ls.tau * dt);
    }
    rc = compute_impl(ctx, s, ws, L, b, pos, species, regions, n_regions, r_buffer, mode, forces,
                      e_exp, e_cheap, lambda, flags, n_expensive, nullptr, nullptr,
                      fused ? &ka : nullptr, ls.tau > 0.0 ? &la : nullptr, nullptr, true);
    if (rc)
        return rc;
    if (!fused && energies) {
        // closing half kick fused with the energy partial sums
        StageTimer t(ctx, s, ST_RED);
        launch_vv_kick_sums(s, ws, L, vel, mass, forces, dt, e_exp, e_cheap, energies);
    } else if (!fused) {
        StageTimer t(ctx, s, ST_VV);
        launch_vv_kick_drift(s, ws, L, b, pos, vel, mass, forces, dt, 0);
    }
    HIP_OK(hipGetLastError());
    return MLMIX_OK;
} catch (...) {
    return host_exception();
}

extern "C" int mlmix_vv_steps(mlmix_ctx *ctx, void *stream, void *ws, int32_t n_atoms,
                              double *pos, double *vel, const double *mass,
                              const int32_t *species, double dt, int32_t n_steps,
                              const mlmix_box *box, const mlmix_region *regions,
                              int32_t n_regions, double r_buffer, uint32_t mode, double *forces,
                              double *e_exp, double *e_cheap, double *lambda, uint8_t *flags,
                              int32_t *n_expensive, double *energies)
try {
    if (!ctx || !ws || !energies || (n_atoms > 0 && (!vel || !mass)))
        return fail(MLMIX_E_ARG, "NULL argument");
    if (n_steps < 1)
        return fail(MLMIX_E_ARG, "n_steps must be at least 1");
    if (mode & MLMIX_ENERGY_ONLY)
        return fail(MLMIX_E_ARG, "MLMIX_ENERGY_ONLY is not valid for an MD step");
    if (!(dt > 0.0))
        return fail(MLMIX_E_ARG, "dt must be positive");
    bool thermo = false;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        thermo = ctx->lang.find(ws) != ctx->lang.end();
    }
    if (thermo && n_steps > 1)
        return fail(MLMIX_E_STATE, "with a thermostat each step needs fresh normals: one step per call");
    WsLayout L;
    Box b;
    int rc = lookup(ctx, ws, n_atoms, box, L, b);
    if (rc)
        return rc;
    rc = check_compute_args(ctx, pos, species, regions, n_regions, r_buffer, mode, forces, e_exp,
                            e_cheap, lambda, flags, n_atoms);
    if (rc)
        return rc;
    if (n_steps == 1 || L.n == 0 || L.n > kGatherKickMax) {
        for (int k = 0; k < n_steps; ++k) {
            rc = mlmix_vv_step(ctx, stream, ws, n_atoms, pos, vel, mass, species, dt, box, regions,
                               n_regions, r_buffer, mode, forces, e_exp, e_cheap, lambda, flags,
                               n_expensive, energies + 3 * (size_t)k);
            if (rc)
                return rc;
        }
        return MLMIX_OK;
    }
    // fused steps: the gather of step k also applies step k+1's opening half
    // kick and drift, and step k+1's binning kernel sums step k's energies
    hipStream_t s = static_cast<hipStream_t>(stream);
    // every drift (the opening kernel's, then the gathers') does the skin check
    const DispCheck dc = disp_check_args(ws, L, ctx->c.d.skin);
    {
        StageTimer t(ctx, s, ST_VV);
        launch_vv_kick_drift(s, ws, L, b, pos, vel, mass, forces, dt, 1, &dc);
    }
    for (int k = 0; k < n_steps; ++k) {
        const bool last = k + 1 == n_steps;
        KickArgs ka{vel, mass, dt, e_cheap, nullptr, energies + 3 * (size_t)k,
                    last ? 0 : 1, last ? 0 : 1, pos, b, nullptr, dc};
        rc = compute_impl(ctx, s, ws, L, b, pos, species, regions, n_regions, r_buffer, mode,
                          forces, e_exp, e_cheap, lambda, flags, n_expensive, nullptr, nullptr,
                          &ka, nullptr, k > 0 ? energies + 3 * (size_t)(k - 1) : nullptr, true);
        if (rc)
            return rc;
    }
    HIP_OK(hipGetLastError());
    return MLMIX_OK;
} catch (...) {
    return host_exception();
}

// ------------------------------------------------------ batched systems

static int check_segments(const mlmix_ctx *ctx, int32_t n_segments, const mlmix_segment *segs,
                          std::vector<SegGeo> &out)
{
    if (n_segments < 1 || n_segments > (1 << 20) || !segs)
        return fail(MLMIX_E_ARG, "1 <= n_segments <= 2^20 and a segment table required");
    out.clear();
    out.reserve((size_t)n_segments);
    long long next = 0;
    for (int k = 0; k < n_segments; ++k) {
        const mlmix_segment &q = segs[k];
        if (q.offset != next)
            return fail(MLMIX_E_ARG, "segments must tile the batch arrays in order (offset of "
                                     "each = sum of the n_atoms before it)");
        if (q.n_atoms < 1)
            return fail(MLMIX_E_ARG, "every segment needs at least one atom");
        if (q.region_offset < 0 || q.n_regions < 0)
            return fail(MLMIX_E_ARG, "negative region range in a segment");
        Box b;
        int rc = check_box(ctx, &q.box, b);
        if (rc)
            return rc;
        SegGeo G{};
        G.box = b;
        G.off = q.offset;
        G.n = q.n_atoms;
        G.reg0 = q.region_offset;
        G.nreg = q.n_regions;
        out.push_back(G);
        next += q.n_atoms;
        if (next > 2147483647LL)
            return fail(MLMIX_E_ARG, "more than 2^31 - 1 atoms in a batch");
    }
    return MLMIX_OK;
}

static int batch_layout(const mlmix_ctx *ctx, int32_t n_segments, const mlmix_segment *segs,
                        int32_t nbr_cap, int32_t s_cap, WsLayout &L, std::vector<SegGeo> &geo)
{
    if (nbr_cap < 1 || nbr_cap > kMaxCap)
        return fail(MLMIX_E_ARG, "1 <= nbr_cap <= 256 required");
    std::vector<SegGeo> in;
    int rc = check_segments(ctx, n_segments, segs, in);
    if (rc)
        return rc;
    L = make_batch_layout(ctx->c, in, nbr_cap, s_cap, geo);
    for (const SegGeo &G : geo)
        if ((double)G.grid.ncell * G.grid.bucket >= 2147483647.0)
            return fail(MLMIX_E_ARG, "box too large for the cell grid (2^31 bucket records)");
    return MLMIX_OK;
}

extern "C" int mlmix_batch_workspace_size(const mlmix_ctx *ctx, int32_t n_segments,
                                          const mlmix_segment *segs, int32_t nbr_cap,
                                          int32_t s_cap, size_t *bytes)
try {
    if (!ctx || !bytes)
        return fail(MLMIX_E_ARG, "NULL argument");
    WsLayout L;
    std::vector<SegGeo> geo;
    int rc = batch_layout(ctx, n_segments, segs, nbr_cap, s_cap, L, geo);
    if (rc)
        return rc;
    *bytes = L.total;
    return MLMIX_OK;
} catch (...) {
    return host_exception();
}

extern "C" int mlmix_batch_init(mlmix_ctx *ctx, void *stream, void *ws, size_t ws_bytes,
                                int32_t n_segments, const mlmix_segment *segs, int32_t nbr_cap,
                                int32_t s_cap)
try {
    if (!ctx || !ws)
        return fail(MLMIX_E_ARG, "NULL argument");
    WsLayout L;
    std::vector<SegGeo> geo;
    int rc = batch_layout(ctx, n_segments, segs, nbr_cap, s_cap, L, geo);
    if (rc)
        return rc;
    if (ws_bytes < L.total)
        return fail(MLMIX_E_WORKSPACE, "workspace smaller than mlmix_batch_workspace_size()");
    hipStream_t s = static_cast<hipStream_t>(stream);
    k_zero_i32<<<1, H_COUNT, 0, s>>>(at<int>(ws, L.hdr), H_COUNT);
    k_zero_i32<<<(L.grid.ncell + 255) / 256, 256, 0, s>>>(at<int>(ws, L.cell_count), L.grid.ncell);
    k_zero_i32<<<(L.nseg + 255) / 256, 256, 0, s>>>(at<int>(ws, L.seg_status), L.nseg);
    k_zero_i32<<<(4 * L.nseg + 255) / 256, 256, 0, s>>>(at<int>(ws, L.seg_flag), 4 * L.nseg);
    HIP_OK(hipGetLastError());
    // the segment table (the host copy is released when this call returns)
    HIP_OK(hipMemcpyAsync(at<SegGeo>(ws, L.segs), geo.data(), geo.size() * sizeof(SegGeo),
                          hipMemcpyHostToDevice, s));
    HIP_OK(hipStreamSynchronize(s));
    launch_seg_fill(s, ws, L);
    HIP_OK(hipGetLastError());
    std::vector<mlmix_segment> keep(segs, segs + n_segments);
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->lang.erase(ws);
    ctx->ws[ws] = L;
    ctx->batch[ws].swap(keep);
    return MLMIX_OK;
} catch (...) {
    return host_exception();
}

static int batch_lookup(mlmix_ctx *ctx, void *ws, int32_t n_atoms, int32_t n_regions,
                        WsLayout &L)
{
    if (!ctx || !ws)
        return fail(MLMIX_E_ARG, "NULL context or workspace");
    std::lock_guard<std::mutex> g(ctx->mu);
    auto it = ctx->ws.find(ws);
    auto bt = ctx->batch.find(ws);
    if (it == ctx->ws.end() || bt == ctx->batch.end() || it->second.nseg == 0)
        return fail(MLMIX_E_STATE, "workspace was not initialised with mlmix_batch_init");
    L = it->second;
    if (L.n != n_atoms)
        return fail(MLMIX_E_ARG, "n_atoms differs from the batch's (sum over its segments)");
    for (const mlmix_segment &q : bt->second)
        if ((long long)q.region_offset + q.n_regions > (long long)n_regions)
            return fail(MLMIX_E_ARG, "a segment's regions reach past n_regions");
    return MLMIX_OK;
}

extern "C" int mlmix_batch_carry_lists(mlmix_ctx *ctx, void *stream, void *ws_new,
                                       const void *ws_old, const int32_t *seg_map)
try {
    if (!ctx || !ws_new || !ws_old || !seg_map)
        return fail(MLMIX_E_ARG, "NULL argument");
    WsLayout Ln, Lo;
    std::vector<mlmix_segment> sn, so;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        auto in = ctx->ws.find(ws_new), io = ctx->ws.find(const_cast<void *>(ws_old));
        auto bn = ctx->batch.find(ws_new), bo = ctx->batch.find(const_cast<void *>(ws_old));
        if (in == ctx->ws.end() || io == ctx->ws.end() || bn == ctx->batch.end() ||
            bo == ctx->batch.end() || in->second.nseg == 0 || io->second.nseg == 0)
            return fail(MLMIX_E_STATE, "both workspaces must be initialised with mlmix_batch_init");
        Ln = in->second;
        Lo = io->second;
        sn = bn->second;
        so = bo->second;
    }
    if (ws_new == ws_old)
        return fail(MLMIX_E_ARG, "the two workspaces must differ");
    if (Ln.cap != Lo.cap)
        return fail(MLMIX_E_ARG, "the two workspaces have different row capacities");
    std::vector<int> used(so.size(), 0);
    for (size_t k = 0; k < sn.size(); ++k) {
        const int ko = seg_map[k];
        if (ko < -1 || ko >= (int)so.size())
            return fail(MLMIX_E_ARG, "seg_map entry out of range");
        if (ko < 0)
            continue;
        if (used[ko]++)
            return fail(MLMIX_E_ARG, "an old segment mapped twice");
        if (so[ko].n_atoms != sn[k].n_atoms)
            return fail(MLMIX_E_ARG, "a kept system changed its atom count");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_OK(hipMemcpyAsync(at<int>(ws_new, Ln.seg_map), seg_map, sn.size() * sizeof(int),
                          hipMemcpyHostToDevice, s));
    launch_carry_lists(s, ws_new, Ln, ws_old, Lo);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(s));  // the host map is the caller's
    return MLMIX_OK;
} catch (...) {
    return host_exception();
}

static int check_batch_mode(uint32_t mode)
{
    if (mode & (MLMIX_SEEDED | MLMIX_ENERGY_ONLY))
        return fail(MLMIX_E_ARG, "batched calls take neither seeded regions nor "
                                 "MLMIX_ENERGY_ONLY");
    return MLMIX_OK;
}

extern "C" int mlmix_batch_compute(mlmix_ctx *ctx, void *stream, void *ws, int32_t n_atoms,
                                   const double *pos, const int32_t *species,
                                   const mlmix_region *regions, int32_t n_regions,
                                   double r_buffer, uint32_t mode, double *forces, double *e_exp,
                                   double *e_cheap, double *lambda, uint8_t *flags,
                                   int32_t *n_expensive, double *energies)
try {
    WsLayout L;
    int rc = batch_lookup(ctx, ws, n_atoms, n_regions, L);
    if (rc)
        return rc;
    rc = check_batch_mode(mode);
    if (rc)
        return rc;
    rc = check_compute_args(ctx, pos, species, regions, n_regions, r_buffer, mode, forces, e_exp,
                            e_cheap, lambda, flags, n_atoms);
    if (rc)
        return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Box unused{};  // every kernel takes its atom's box from the segment table
    rc = compute_impl(ctx, s, ws, L, unused, pos, species, regions, n_regions, r_buffer, mode,
                      forces, e_exp, e_cheap, lambda, flags, nullptr, nullptr, nullptr);
    if (rc)
        return rc;
    if (n_expensive || energies) {
        launch_seg_sums(s, ws, L, e_exp, e_cheap, nullptr, flags, energies, n_expensive);
        HIP_OK(hipGetLastError());
    }
    return MLMIX_OK;
} catch (...) {
    return host_exception();
}

extern "C" int mlmix_batch_vv_steps(mlmix_ctx *ctx, void *stream, void *ws, int32_t n_atoms,
                                    double *pos, double *vel, const double *mass,
                                    const int32_t *species, double dt, int32_t n_steps,
                                    const mlmix_region *regions, int32_t n_regions,
                                    double r_buffer, uint32_t mode, double *forces,
                                    double *e_exp, double *e_cheap, double *lambda,
                                    uint8_t *flags, int32_t *n_expensive, double *energies)
try {
    WsLayout L;
    int rc = batch_lookup(ctx, ws, n_atoms, n_regions, L);
    if (rc)
        return rc;
    rc = check_batch_mode(mode);
    if (rc)
        return rc;
    if (!vel || !mass || !energies)
        return fail(MLMIX_E_ARG, "NULL argument");
    if (n_steps < 1)
        return fail(MLMIX_E_ARG, "n_steps must be at least 1");
    if (!(dt > 0.0))
        return fail(MLMIX_E_ARG, "dt must be positive");
    rc = check_compute_args(ctx, pos, species, regions, n_regions, r_buffer, mode, forces, e_exp,
                            e_cheap, lambda, flags, n_atoms);
    if (rc)
        return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Box unused{};
    double *ke = at<double>(ws, L.seg_red);
    const DispCheck dc = disp_check_args(ws, L, ctx->c.d.skin);
    {
        StageTimer t(ctx, s, ST_VV);
        launch_vv_kick_drift(s, ws, L, unused, pos, vel, mass, forces, dt, 1, &dc);
    }
    for (int k = 0; k < n_steps; ++k) {
        const bool last = k + 1 == n_steps;
        // the gather closes the step (half kick, per-atom kinetic energy) and,
        // before the next step, applies its opening half kick and drift
        KickArgs ka{vel, mass, dt, e_cheap, nullptr, nullptr, last ? 0 : 1, 0, pos, unused, ke, dc};
        rc = compute_impl(ctx, s, ws, L, unused, pos, species, regions, n_regions, r_buffer, mode,
                          forces, e_exp, e_cheap, lambda, flags, nullptr, nullptr, nullptr, &ka,
                          nullptr, nullptr, true);
        if (rc)
            return rc;
        StageTimer t(ctx, s, ST_RED);
        launch_seg_sums(s, ws, L, e_exp, e_cheap, ke, flags,
                        energies + (size_t)k * L.nseg * 3, last ? n_expensive : nullptr);
    }
    HIP_OK(hipGetLastError());
    return MLMIX_OK;
} catch (...) {
    return host_exception();
}

extern "C" int mlmix_batch_status(mlmix_ctx *ctx, void *stream, void *ws, int32_t *segment_bits,
                                  int32_t *required_cap)
try {
    if (!ctx || !ws)
        return fail(MLMIX_E_ARG, "NULL argument");
    WsLayout L;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        auto it = ctx->ws.find(ws);
        if (it == ctx->ws.end() || it->second.nseg == 0)
            return fail(MLMIX_E_STATE, "workspace was not initialised with mlmix_batch_init");
        L = it->second;
    }
    if (segment_bits) {
        HIP_OK(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
        HIP_OK(hipMemcpy(segment_bits, at<int>(ws, L.seg_status), (size_t)L.nseg * sizeof(int),
                         hipMemcpyDeviceToHost));
    }
    return mlmix_status(ctx, stream, ws, nullptr, required_cap);
} catch (...) {
    return host_exception();
}

extern "C" int mlmix_status(mlmix_ctx *ctx, void *stream, void *ws, int32_t *status_bits,
                            int32_t *required_cap)
try {
    if (!ctx || !ws)
        return fail(MLMIX_E_ARG, "NULL argument");
    WsLayout L;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        auto it = ctx->ws.find(ws);
        if (it == ctx->ws.end())
            return fail(MLMIX_E_STATE, "workspace was not initialised");
        L = it->second;
    }
    HIP_OK(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    int hdr[H_COUNT];
    HIP_OK(hipMemcpy(hdr, at<int>(ws, L.hdr), sizeof hdr, hipMemcpyDeviceToHost));
    if (status_bits)
        *status_bits = hdr[H_STATUS];
    if (required_cap)
        *required_cap = hdr[H_REQCAP];
    int st = hdr[H_STATUS];
    if (st & (MLMIX_STATUS_NEIGH_OVERFLOW | MLMIX_STATUS_TRIPLET_OVERFLOW))
        return fail(MLMIX_E_NEIGH_OVERFLOW, "neighbour row capacity exceeded");
    if (st & MLMIX_STATUS_SEEDED_REGIONS)
        return fail(MLMIX_E_ARG, "more than 8 seeded regions");
    if (st & MLMIX_STATUS_S_OVERFLOW)
        return fail(MLMIX_E_WORKSPACE, "|S| exceeded the workspace's S capacity (n_expensive[0] "
                                       "holds the required value)");
    if (st & MLMIX_STATUS_CELL_OVERFLOW)
        return fail(MLMIX_E_NEIGH_OVERFLOW, "cell bucket capacity exceeded (local density far "
                                            "above the mean)");
    if (st & MLMIX_STATUS_NONFINITE)
        return fail(MLMIX_E_NONFINITE, "non-finite position");
    if (st & MLMIX_STATUS_BAD_SPECIES)
        return fail(MLMIX_E_ARG, "species index outside [0, n_species)");
    if (st & MLMIX_STATUS_OUT_OF_BOX)
        return fail(MLMIX_E_BOX, "atom outside a non-periodic box dimension");
    return MLMIX_OK;
} catch (...) {
    return host_exception();
}

extern "C" int mlmix_list_builds(mlmix_ctx *ctx, void *stream, void *ws, int32_t *builds)
try {
    if (!ctx || !ws || !builds)
        return fail(MLMIX_E_ARG, "NULL argument");
    WsLayout L;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        auto it = ctx->ws.find(ws);
        if (it == ctx->ws.end())
            return fail(MLMIX_E_STATE, "workspace was not initialised");
        L = it->second;
    }
    HIP_OK(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    HIP_OK(hipMemcpy(builds, at<int>(ws, L.hdr) + H_NBUILD, sizeof(int32_t),
                     hipMemcpyDeviceToHost));
    return MLMIX_OK;
} catch (...) {
    return host_exception();
}

extern "C" int mlmix_get_neighbors(mlmix_ctx *ctx, void *stream, void *ws, int32_t n_atoms,
                                   int32_t *nbr_out, int32_t *cnt_out)
try {
    if (!ctx || !ws || !nbr_out || !cnt_out)
        return fail(MLMIX_E_ARG, "NULL argument");
    WsLayout L;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        auto it = ctx->ws.find(ws);
        if (it == ctx->ws.end())
            return fail(MLMIX_E_STATE, "workspace was not initialised");
        L = it->second;
    }
    if (L.n != n_atoms)
        return fail(MLMIX_E_ARG, "n_atoms differs from the workspace's");
    hipStream_t s = static_cast<hipStream_t>(stream);
    launch_copy_i32(s, nbr_out, at<int>(ws, L.nbr), (size_t)L.n * L.cap);
    launch_copy_i32(s, cnt_out, at<int>(ws, L.cnt), (size_t)L.n);
    HIP_OK(hipGetLastError());
    return MLMIX_OK;
} catch (...) {
    return host_exception();
}

extern "C" int mlmix_get_index_sets(mlmix_ctx *ctx, void *stream, void *ws, int32_t n_atoms,
                                    int32_t *S_out, int32_t *M_out)
try {
    if (!ctx || !ws || !S_out || !M_out)
        return fail(MLMIX_E_ARG, "NULL argument");
    WsLayout L;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        auto it = ctx->ws.find(ws);
        if (it == ctx->ws.end())
            return fail(MLMIX_E_STATE, "workspace was not initialised");
        L = it->second;
    }
    if (L.n != n_atoms)
        return fail(MLMIX_E_ARG, "n_atoms differs from the workspace's");
    hipStream_t s = static_cast<hipStream_t>(stream);
    launch_copy_i32(s, S_out, at<int>(ws, L.S_idx), (size_t)L.n);
    launch_copy_i32(s, M_out, at<int>(ws, L.M_idx), (size_t)L.n);
    HIP_OK(hipGetLastError());
    return MLMIX_OK;
} catch (...) {
    return host_exception();
}

// ------------------------------------------- constrained fit of the cheap potential

static int fit_params(const Ctx &c)
{
    const int ns = c.d.n_species, nk2 = c.d.uf3_n_knots2, nk3 = c.d.uf3_n_knots3;
    int nd = ns * (ns + 1) / 2 * (nk2 - 1);
    if (nk3 > 0)
        nd += ns * ((nk3 - 1) * nk3 / 2) * (nk3 + 2);
    return nd;
}

extern "C" int mlmix_fit_n_params(mlmix_ctx *ctx, int32_t *n_params)
try {
    if (!ctx || !n_params)
        return fail(MLMIX_E_ARG, "NULL argument");
    *n_params = fit_params(ctx->c);
    return MLMIX_OK;
} catch (...) {
    return host_exception();
}

static int fit_config(mlmix_ctx *ctx, int nd, void *ws, int32_t n_atoms, const double *pos,
                      const int32_t *species, const mlmix_box *box, double *rows, FitCfgHost &h)
{
    if (!ws || !pos || !species || !rows)
        return fail(MLMIX_E_ARG, "NULL argument");
    int rc = lookup(ctx, ws, n_atoms, box, h.L, h.box);
    if (rc)
        return rc;
    // per-atom energy rows and 3-body lists live in the pair-gradient
    // scratch of the workspace
    const size_t avail = h.L.red - h.L.g;  // the expensive and cheap gradient buffers
    if ((size_t)h.L.n * (nd * sizeof(double) + (kMaxTriplet + 1) * sizeof(int)) > avail)
        return fail(MLMIX_E_WORKSPACE, "workspace too small for the design rows (raise nbr_cap)");
    h.ws = ws;
    h.pos = pos;
    h.species = species;
    h.rows = rows;
    return MLMIX_OK;
}

static int fit_nd_check(mlmix_ctx *ctx, int32_t ld, int &nd)
{
    nd = fit_params(ctx->c);
    if (nd < 1 || nd > kFitMaxParams)
        return fail(MLMIX_E_ARG, "the cheap potential has more free parameters than the fit supports");
    if (ld < nd)
        return fail(MLMIX_E_ARG, "ld is smaller than the number of parameters");
    return MLMIX_OK;
}

extern "C" int mlmix_fit_design(mlmix_ctx *ctx, void *stream, void *ws, int32_t n_atoms,
                                const double *pos, const int32_t *species, const mlmix_box *box,
                                double *rows, int32_t ld)
try {
    if (!ctx)
        return fail(MLMIX_E_ARG, "NULL argument");
    int nd = 0;
    int rc = fit_nd_check(ctx, ld, nd);
    if (rc)
        return rc;
    FitCfgHost h;
    rc = fit_config(ctx, nd, ws, n_atoms, pos, species, box, rows, h);
    if (rc)
        return rc;
    launch_fit_design(static_cast<hipStream_t>(stream), ctx->c, &h, 1, ld, nd);
    HIP_OK(hipGetLastError());
    return MLMIX_OK;
} catch (...) {
    return host_exception();
}

extern "C" int mlmix_fit_design_batch(mlmix_ctx *ctx, void *stream, int32_t n_configs,
                                      const mlmix_fit_config *configs, int32_t ld)
try {
    if (!ctx || (n_configs > 0 && !configs) || n_configs < 0)
        return fail(MLMIX_E_ARG, "NULL argument or negative count");
    int nd = 0;
    int rc = fit_nd_check(ctx, ld, nd);
    if (rc)
        return rc;
    std::vector<FitCfgHost> h((size_t)n_configs);
    for (int q = 0; q < n_configs; ++q) {
        const mlmix_fit_config &c = configs[q];
        rc = fit_config(ctx, nd, c.ws, c.n_atoms, c.pos, c.species, &c.box, c.rows, h[q]);
        if (rc)
            return rc;
    }
    launch_fit_design(static_cast<hipStream_t>(stream), ctx->c, h.data(), n_configs, ld, nd);
    HIP_OK(hipGetLastError());
    return MLMIX_OK;
} catch (...) {
    return host_exception();
}

extern "C" int mlmix_fit_work_size(int64_t n_rows, int32_t n_params, size_t *bytes)
try {
    if (!bytes || n_rows < 0 || n_params < 1 || n_params > kFitMaxParams)
        return fail(MLMIX_E_ARG, "bad sizes");
    long long chunk = 0;
    const size_t parts = fit_gram_parts(n_rows > 0 ? n_rows : 1, chunk);
    // Gram partials of n_rows rows, after G_H and b_H of the search
    *bytes = ((size_t)n_params * n_params + n_params) * sizeof(double) +
             fit_gram_part_bytes(n_params, parts);
    return MLMIX_OK;
} catch (...) {
    return host_exception();
}

extern "C" int mlmix_fit_gram(mlmix_ctx *ctx, void *stream, const double *rows, int64_t n_rows,
                              int32_t n_params, int32_t ld, const double *y, const double *w,
                              double *G, double *b, void *work, size_t work_bytes)
try {
    if (!ctx || !G || !b || (n_rows > 0 && (!rows || !work)))
        return fail(MLMIX_E_ARG, "NULL argument");
    if (n_rows < 0 || n_params < 1 || n_params > kFitMaxParams || ld < n_params)
        return fail(MLMIX_E_ARG, "bad sizes");
    size_t need = 0;
    int rc = mlmix_fit_work_size(n_rows, n_params, &need);
    if (rc)
        return rc;
    if (work_bytes < need)
        return fail(MLMIX_E_WORKSPACE, "work buffer smaller than mlmix_fit_work_size");
    launch_fit_gram(static_cast<hipStream_t>(stream), n_rows, n_params, ld, rows, y, w, G, b,
                    static_cast<double *>(work) + (size_t)n_params * n_params + n_params);
    HIP_OK(hipGetLastError());
    return MLMIX_OK;
} catch (...) {
    return host_exception();
}

extern "C" int mlmix_fit_constrained(mlmix_ctx *ctx, void *stream, int32_t n_params,
                                     const double *GS, const double *bS, const double *AH,
                                     int32_t ld_h, int32_t n_hard, const double *yH,
                                     const double *wH, double alpha,
                                     double tol, double lambda0, double ridge,
                                     int32_t max_decades, int32_t max_bisect, double *c,
                                     double *info, void *work, size_t work_bytes)
try {
    if (!ctx || !GS || !bS || !c || !info || !work || (n_hard > 0 && (!AH || !yH)))
        return fail(MLMIX_E_ARG, "NULL argument");
    if (n_params < 1 || n_params > kFitMaxParams || n_hard < 0 || (n_hard > 0 && ld_h < n_params))
        return fail(MLMIX_E_ARG, "bad sizes");
    if (!(alpha > 0.0) || !(tol > 0.0) || !(lambda0 > 0.0) || !(ridge >= 0.0) ||
        !std::isfinite(alpha) || !std::isfinite(tol) || !std::isfinite(lambda0) ||
        !std::isfinite(ridge))
        return fail(MLMIX_E_ARG, "alpha, tol and lambda0 must be positive, ridge non-negative");
    if (max_decades < 0 || max_decades > 64 || max_bisect < 0 || max_bisect > 1000)
        return fail(MLMIX_E_ARG, "iteration limits out of range");
    size_t need = 0;
    int rc = mlmix_fit_work_size(n_hard, n_params, &need);
    if (rc)
        return rc;
    if (work_bytes < need)
        return fail(MLMIX_E_WORKSPACE, "work buffer smaller than mlmix_fit_work_size(n_hard)");
    launch_fit_search(static_cast<hipStream_t>(stream), n_params, n_hard, ld_h, GS, bS, AH, yH, wH,
                      alpha, tol, lambda0, ridge, max_decades, max_bisect, c, info,
                      static_cast<double *>(work));
    HIP_OK(hipGetLastError());
    return MLMIX_OK;
} catch (...) {
    return host_exception();
}

extern "C" int mlmix_profile_enable(mlmix_ctx *ctx, uint32_t stage_mask)
try {
    if (!ctx)
        return fail(MLMIX_E_ARG, "NULL context");
    ctx->prof_mask = stage_mask & ((1u << MLMIX_N_STAGES) - 1u);
    return MLMIX_OK;
} catch (...) {
    return host_exception();
}

extern "C" int mlmix_profile_replay(mlmix_ctx *ctx, void *stream, void *ws, int32_t n_atoms,
                                    const double *pos, const int32_t *species,
                                    const mlmix_box *box, double *e_out, int32_t stage,
                                    int32_t reps)
try {
    if (!ctx || !ws || !species || reps < 0)
        return fail(MLMIX_E_ARG, "NULL argument or negative count");
    if (stage != ST_CONTRACT && stage != ST_PAIR && stage != ST_UF3)
        return fail(MLMIX_E_ARG, "only the order-3 contraction (stage 4), the pair adjoint "
                                 "(stage 6) and the cheap potential (stage 7) can be replayed");
    if ((stage == ST_UF3 || stage == ST_PAIR) && (!pos || !box || !e_out))
        return fail(MLMIX_E_ARG, "the pair adjoint and the cheap potential need pos, box and e_out");
    if (stage == ST_PAIR && ctx->c.prec == MLMIX_FP64)
        return fail(MLMIX_E_ARG, "the pair adjoint replays in the single-precision modes only");
    WsLayout L;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        auto it = ctx->ws.find(ws);
        if (it == ctx->ws.end())
            return fail(MLMIX_E_STATE, "workspace was not initialised");
        L = it->second;
    }
    if (L.n != n_atoms)
        return fail(MLMIX_E_ARG, "n_atoms differs from the workspace's");
    if (L.nseg > 0)
        return fail(MLMIX_E_ARG, "replays take a single-system workspace");
    Box b{};
    if (stage != ST_CONTRACT) {
        int rc = check_box(ctx, box, b);
        if (rc)
            return rc;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int r = 0; r < reps; ++r) {
        if (stage == ST_CONTRACT)
            launch_ace_contract(s, ctx->c, ws, L, species);
        else if (stage == ST_PAIR)  // with the finalisation where a step folds it in
            launch_ace_pairgrad(s, ctx->c, ws, L, b, pos, species, nullptr,
                                ace_fin_fused(ctx->c, L) ? e_out : nullptr);
        else  // uncapped, as on one stream
            launch_uf3(s, ctx->c, ws, L, b, pos, species, e_out, 0);
    }
    HIP_OK(hipGetLastError());
    return MLMIX_OK;
} catch (...) {
    return host_exception();
}

extern "C" int mlmix_probe_mfma_f32(void *stream, int32_t blocks, int32_t iters, float *sink,
                                    double *flops)
try {
    if (!sink || !flops || blocks < 1 || iters < 1)
        return fail(MLMIX_E_ARG, "NULL argument or non-positive size");
    launch_probe_mfma_f32(static_cast<hipStream_t>(stream), blocks, iters, sink);
    HIP_OK(hipGetLastError());
    // 4 waves per block, 8 chains per round, 2 * 16 * 16 * 4 flops per MFMA
    *flops = (double)blocks * 4.0 * (double)iters * 8.0 * 2048.0;
    return MLMIX_OK;
} catch (...) {
    return host_exception();
}

extern "C" int mlmix_profile_read(mlmix_ctx *ctx, double *ms, int64_t *count)
try {
    if (!ctx || !ms || !count)
        return fail(MLMIX_E_ARG, "NULL argument");
    for (int i = 0; i < MLMIX_N_STAGES; ++i) {
        ms[i] = 0.0;
        count[i] = 0;
    }
    int rc = MLMIX_OK;
    for (PendingEvent &p : ctx->pending) {
        float t = 0.0f;
        hipError_t e = hipEventSynchronize(p.b);
        if (e == hipSuccess)
            e = hipEventElapsedTime(&t, p.a, p.b);
        if (e != hipSuccess)
            rc = fail_hip("profile events", e);
        ms[p.stage] += t;
        count[p.stage] += 1;
        ctx->pool.push_back(p.a);
        ctx->pool.push_back(p.b);
    }
    ctx->pending.clear();
    return rc;
} catch (...) {
    return host_exception();
}

extern "C" const char *mlmix_profile_stage_name(int32_t stage)
{
    if (stage < 0 || stage >= MLMIX_N_STAGES)
        return "";
    return kStageNames[stage];
}

extern "C" int mlmix_model_flops(const mlmix_ctx *ctx, double *out)
try {
    if (!ctx || !out)
        return fail(MLMIX_E_ARG, "NULL argument");
    for (int i = 0; i < 7; ++i)
        out[i] = ctx->flops[i];
    return MLMIX_OK;
} catch (...) {
    return host_exception();
}

extern "C" int mlmix_gaunt_table(int32_t lmax, double *out)
try {
    if (!out || lmax < 0 || lmax > kMaxLmax)
        return fail(MLMIX_E_ARG, "0 <= lmax <= 6 and an output array required");
    const std::vector<double> G = gaunt(lmax);
    std::memcpy(out, G.data(), G.size() * sizeof(double));
    return MLMIX_OK;
} catch (...) {
    return host_exception();
}
