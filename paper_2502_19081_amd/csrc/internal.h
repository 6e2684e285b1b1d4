// Internal declarations of the HIP library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "mlmix.h"

namespace mlmix {

constexpr int kWave = 64;
constexpr int kMaxLmax = 6;
constexpr int kMaxL2 = (kMaxLmax + 1) * (kMaxLmax + 1);
constexpr int kMaxNrad = 16;
constexpr int kMaxCap = 256;
constexpr int kMaxTriplet = 64;   // neighbours inside the 3-body cutoff per centre
constexpr int kScanTile = 2048;   // elements per block in the device scans
constexpr int kReduceBlocks = 256;
constexpr int kO3VMaxRows = 128;  // rows of one bin of the vector-sparse FP32 contraction
constexpr int kO3Atoms = 16;      // S atoms per tile of the order-3 kernels
constexpr int kO3MaxSplit = 16;   // workgroups sharing one 16-atom tile of the order-3 kernel
// partial-D column sets of the order-3 sums: one per split G = 1 .. 16 of the
// vector-sparse contraction, then the per-(block, m3) set of the other forms
constexpr int kDSumSets = 6;
constexpr int kDSumBlocks = 5;  // index of the per-(block, m3) set

// Header words at the start of every workspace (int32 unless noted).
enum HeaderWord {
    H_BUILT = 0,      // a neighbour list exists
    H_REBUILD = 1,    // rebuild requested for the current call
    H_STATUS = 2,     // MLMIX_STATUS_* bits
    H_REQCAP = 3,     // largest neighbour count seen
    H_NS = 4,         // |S|
    H_NM = 5,         // |{lambda > 0}|
    H_FWD = 6,        // a forward pass with dE/dA exists
    H_MOVED = 7,      // an atom moved more than half the skin since the last build
    H_NBUILD = 8,     // neighbour-list builds since the workspace was initialised
    H_COUNT = 64
};

// Cell-ordered copy of an atom written during binning: the neighbour search
// reads one 32-byte record per candidate.
struct CellAtom {
    double x, y, z;
    int j, pad;
};

struct Box {
    double L[3];
    int per[3];
};

// Cell grid of edge >= list radius / 2 (a +-2 cell stencil covers the radius).
struct Grid {
    int nc[3];
    double cs[3];
    int ncell;
    int bucket;  // records per cell bucket
};

// One system of a batched call: atoms [off, off + n) of the batch arrays, its
// box and cell grid (cells [cell0, cell0 + grid.ncell) of the batch's cell
// counts, bucket records from rec0) and its regions [reg0, reg0 + nreg).
struct SegGeo {
    Box box;
    Grid grid;
    int off, n;
    int cell0, reg0, nreg, pad;
    long long rec0;
};

// Segment lookup of a batched call; all null for a single system. of[i] is
// the segment of atom i, geo the segment table, status per-segment
// MLMIX_STATUS_* words (the workspace header keeps their union).
struct Seg {
    const int *of;
    const SegGeo *geo;
    int *status;
    // per-segment list state [nseg][4]: 0 an atom moved more than half the
    // skin since the segment's last build, 1 built, 2 rebuild in this call:
    // every system of a batch keeps or rebuilds its list by its own atoms
    int *flag;
};
constexpr int kSegMoved = 0, kSegBuilt = 1, kSegRebuild = 2;

// Kernels that need an atom's box or grid take a template flag SEG: false
// for a single system (no segment code at all, the box stays a kernel
// argument), true for a batch.

// Box of atom i (and of every partner in its rows). WAVE: i is the same on
// every lane of the wave, so the segment index is read once (scalar).
template <bool SEG, bool WAVE = false>
__device__ __forceinline__ Box seg_box(const Box &b, const Seg &sg, int i)
{
    if constexpr (SEG) {
        int k = sg.of[i];
        if constexpr (WAVE)
            k = __builtin_amdgcn_readfirstlane(k);
        return sg.geo[k].box;
    } else {
        return b;
    }
}

// Status bits of atom i's system: the workspace header, and in a batched
// call also the atom's segment word.
template <bool SEG>
__device__ __forceinline__ void seg_status_or(int *hdr_status, const Seg &sg, int i, int bits)
{
    atomicOr(hdr_status, bits);
    if constexpr (SEG)
        atomicOr(&sg.status[sg.of[i]], bits);
}

struct WsLayout {
    int n, cap, P;  // atoms, row capacity, capacity rounded up to a power of two
    int scap;       // capacity of S (rows of the per-S buffers A, dE/dA, g, partial D)
    Grid grid;      // single system: its grid; batch: ncell = cells of all segments
    int n_scan_blk;  // blocks of the atom-sized scans
    int nseg;        // segments of a batch workspace (0: one system)
    size_t hdr, cell_count, cell_atoms, scan_part, seedcore;
    size_t nbr, cnt, rev, ref_pos, S_idx, M_idx, S_local, cand;
    size_t A, dEdA, g, h, red, dpart;
    size_t seg_of, segs, seg_status, seg_red, seg_flag, seg_map;  // batch workspaces only
    // region lists per superblock of the box (single systems): rgn[k]
    // superblocks along dimension k, each (count or -1, kRegionGridCap ids)
    size_t rgrid;
    int rgn[3];
    size_t total;
};

template <typename T>
inline T *at(void *ws, size_t off) { return reinterpret_cast<T *>(static_cast<char *>(ws) + off); }

inline Seg seg_args(void *ws, const WsLayout &L)
{
    if (L.nseg == 0)
        return Seg{nullptr, nullptr, nullptr, nullptr};
    return Seg{at<int>(ws, L.seg_of), at<SegGeo>(ws, L.segs), at<int>(ws, L.seg_status),
               at<int>(ws, L.seg_flag)};
}

// Model tables on the device, in the arithmetic type of the context.
struct DevModel {
    int ns, nrad, lmax, order, nchan, KA, L2;
    int nchp, KAt;  // channels padded to a multiple of 4; per-atom entries L2 * nchp
    double rc_exp, rc2, rc3;
    int nb2, nb3, nk2, nk3;
    int n_pb;  // (l1 <= l2, l3) blocks of the order-3 contraction
    void *base;
    size_t bytes;
    // offsets (bytes) into base
    size_t ylmK, c0, c0d, c1, c2s, W, pb, gm3, gidx, gofs, gval, u2, u3, up2, up3, dpoff, wsc;
    // tables of the matrix-core order-3 kernel (single species, <= 16 channels)
    size_t o3o, o3mt, o3mtv, o3rowv, o3rbeg, o3wr, o3base, o3w, o3sw, o3order, o3wbeg, o3gs;
    size_t o3ww;   // weight fragments of the wide form
    size_t o3wwb;  // its BF16 fragments (BF16 mode: eight values per lane and 32-deep step)
    int dp_stride;  // partial-D entries per S atom (sum over blocks of nchan*(2 l3 + 1))
    // partial-D column lists: set k at dsum + dsum_off[k] holds L2 + 1 run
    // offsets, then the columns (atom-relative, channel 0) summed into each
    // (l3, m3) in that order; dsum_len = the longest set in ints; the
    // columns of set k lie in the first dsum_span[k] * nchan entries of a row
    size_t dsum;
    int dsum_off[kDSumSets], dsum_span[kDSumSets], dsum_ncol[kDSumSets], dsum_len;
    int w_per_species;  // entries of W per centre species
    int gm3_total, g_total;
};

// Which partial-D column set the finalisation sums: set off[lg] of tab for
// the split G = 2^lg that the vector-sparse contraction chooses from |S|,
// its grid and its split limit (every off[] the same set for the other forms).
struct DSumSel {
    const int *tab;
    int off[kDSumBlocks];
    int span[kDSumBlocks];  // the set's columns lie in [0, span * nchan) of a row
    int ncol[kDSumBlocks];  // columns listed in the set (its table: L2 + 1 + ncol ints)
    int grid, max_split;
};

// One (l1 <= l2, l3) block of the order-3 contraction.
struct PBlock {
    int l1, l2, l3;
    int w_off;   // offset of the block's W[nchan*nchan][nchan] inside one species' W
    int gm3_off; // offset into gm3: 2*l3+2 entry offsets (entries grouped by m3)
    int pad[3];
};

struct Ctx {
    mlmix_model_desc d;  // pointers inside are not kept
    int prec;            // MLMIX_FP64 or a single-precision mode (FP32, BF16/FP8 contraction)
    int qmode;           // order-3 dense operands: 0 native, 1 BF16, 2 FP8
    double r_list;
    DevModel m;
    int m_pb_lo[kMaxLmax + 1], m_pb_hi[kMaxLmax + 1];  // order-3 blocks per l3
    int max_ent, max_gm3;  // Gaunt entries / m3 offsets of the largest l3 group
    int max_ent_pb;        // Gaunt entries of the largest single block
    // order-3 contraction on the matrix cores: 0 no (VALU blocks), 1 the
    // single-species form (<= 16 channels, FP32/BF16/FP8 operands), 2 the wide
    // form (FP32, any species count, <= 32 channels)
    int o3 = 0;
    int max_lds = 65536;   // dynamic LDS a workgroup may use on this device
    int basis_mfma = 1;    // atomic basis and pair adjoint on the matrix cores (FP32)
    int basis_chunks = -1; // basis in 64-slot passes: -1 above 65,536 atoms, 0 never, 1 always
    int pair_half = 1;     // FP32 vector pair adjoint with two atoms per wave (0: one)
    // second-stream fork after the rows (0), after the basis (1), or recorded
    // after the rows and issued after the compaction (2). Measured per mixed
    // step on 8,193 atoms with the workgroup pair adjoint and the cheap
    // potential uncapped: 95.5 / 95.8 / 95.7 us at 2 against 101.0 / 101.5 /
    // 101.8 us at 0 (alternating runs; the one-wave adjoint's longer chain
    // preferred 0)
    int fork_at = 2;
    // workgroup cap of the cheap-potential kernel on the second stream
    // (grid-stride loop): -1 automatic, 0 uncapped. The best cap follows the
    // length of the expensive chain beside it. With the one-wave pair adjoint,
    // per mixed step on 8,193 atoms: 160 / 129 / 111 / 123 / 120 / 120 / 126
    // us at 128 / 192 / 256 / 384 / 512 / 1024 workgroups / uncapped; with
    // the shorter chain of the workgroup pair adjoint (fork point 2): 95.7 /
    // 96.1 us uncapped / 768 against 100.9 us at 256. On 1,023,800 atoms caps
    // of 1024 and 2048 measured no better than none (11.6 / 11.2 / 11.3 ms).
    // Automatic: uncapped.
    int side_blocks = -1;
    int rev_blocks = 1024;  // cap of the reverse-slot kernel when capped (256 / 1024 measured 153.0 / 152.4 us)
    int o3_nch2 = 0;       // row width of that kernel (channels rounded up to 4)
    // largest tile split of the single-species forms and their waves per
    // workgroup: for the FP32 vector-sparse form on the 8,193-atom cell (910
    // atoms in S) 19.2 / 17.6 / 19.4 us at splits 4 / 8 / 16 with four waves,
    // 16.7 / 18.3 / 18.2 us with eight; on 102,858 atoms in S 3.32 ms with
    // four waves and 3.42 with eight
    int o3_max_split = 4;
    int o3_waves = 8;      // waves per workgroup of the single-species form (4 or 8)
    int o3v = 1;           // FP32 single-species form with the vector sparse stage
    int fuse_fin = 1;      // the matrix-core pair adjoint does the finalisation
    int ace_tile = 4;      // atoms per order-3 block workgroup (tuning)
    int ace_stage_w = 1;   // stage the block's weights in LDS (tuning)
    int device;
};

WsLayout make_layout(const Ctx &c, int n, int cap, const Box &b, int scap);
Grid make_grid(const Ctx &c, const Box &b);

// Species index clamped into the model's range (invalid input is reported by
// a status bit; clamping keeps every table read in bounds).
__host__ __device__ inline int sp_clamp(int z, int ns) { return z < 0 ? 0 : (z >= ns ? ns - 1 : z); }

// Inputs and outputs of the per-atom mixing weight pass (lambda, masks and
// buffer candidates), which runs inside the binning kernel.
// Regions per superblock list, and the region count from which the mixing
// weights use the lists (below it every atom tests every region)
constexpr int kRegionGridCap = 31;
constexpr int kRegionGridMin = 8;

struct RegionArgs {
    int mode;
    const int32_t *species;
    int ns;
    const mlmix_region *reg;
    int nreg;
    double r_buffer;
    double *lam;
    uint8_t *flags;
    uint8_t *cand;
    int seeded;         // MLMIX_SEEDED: seeded regions, seed bits in flags
    uint8_t *seedcore;  // per atom: bit k = core atom of the k-th seeded region
    // energy partials of the previous step of a multi-step call, summed by
    // the first workgroup of the binning kernel into red_out (none if NULL)
    const double *red_part;
    int red_nb;
    double *red_out;
    const int *rgrid = nullptr;  // region lists per superblock (nullptr: every region)
    int rgn[3] = {0, 0, 0};       // superblocks per dimension
};
constexpr int kMaxSeeded = 8;  // seeded regions per evaluation

// ---- launchers (geom.hip) ----
// checked: the integrator kernel that last moved the atoms did the skin check
void launch_neighbors(hipStream_t s, void *ws, const WsLayout &L, const Box &b, double r_list,
                      const double *pos, int force_rebuild, double skin, const RegionArgs &ra,
                      bool checked = false);
void launch_reverse(hipStream_t s, void *ws, const WsLayout &L, int side_blocks);
void launch_regions(hipStream_t s, void *ws, const WsLayout &L, const Box &b, int mode,
                    const double *pos, double r_buffer, uint8_t *flags, int force_rebuild,
                    const RegionArgs &ra);
void launch_compact(hipStream_t s, void *ws, const WsLayout &L, uint8_t *flags, int32_t *n_expensive);
void launch_cheap_buffer(hipStream_t s, void *ws, const WsLayout &L, const Box &b,
                         const double *pos, double r_buffer, uint8_t *flags);

// ---- ace.hip ----
void launch_ace_basis(hipStream_t s, const Ctx &c, void *ws, const WsLayout &L, const Box &b,
                      const double *pos, const int32_t *species);
// ev0/ev1 (may be null): start and end events of the matrix-core contraction
// kernel (hipExtLaunchKernel), for stage timing
void launch_ace_contract(hipStream_t s, const Ctx &c, void *ws, const WsLayout &L,
                         const int32_t *species, hipEvent_t ev0 = nullptr,
                         hipEvent_t ev1 = nullptr);
void launch_ace_finalize(hipStream_t s, const Ctx &c, void *ws, const WsLayout &L,
                         const int32_t *species, double *e_exp);
// e_exp: where the pair adjoint writes the site energies when it does the
// finalisation itself (ace_fin_fused; NULL: the gradient only)
void launch_ace_pairgrad(hipStream_t s, const Ctx &c, void *ws, const WsLayout &L, const Box &b,
                         const double *pos, const int32_t *species, const double *weights,
                         double *e_exp);
bool ace_fin_fused(const Ctx &c, const WsLayout &L);

// ---- o3.hip ----
void launch_ace_o3(hipStream_t s, const Ctx &c, void *ws, const WsLayout &L,
                   hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
size_t o3_lds_bytes(const Ctx &c);
size_t o3v_lds_bytes(const Ctx &c);
int o3v_waves(const Ctx &c, int n);
int o3v_grid(const Ctx &c, int n);
void launch_ace_o3w(hipStream_t s, const Ctx &c, void *ws, const WsLayout &L,
                    const int32_t *species, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
size_t o3w_lds_bytes(const Ctx &c);
hipError_t o3w_prepare(const Ctx &c);

// ---- uf3.hip ----
// mask_flags: NULL, or the flags array (MLMIX_CHEAP_MASKED): the cheap
// potential then sees S_c = {lambda < 1} plus its buffer only
void launch_uf3(hipStream_t s, const Ctx &c, void *ws, const WsLayout &L, const Box &b,
                const double *pos, const int32_t *species, double *e_cheap, int side_blocks,
                const uint8_t *mask_flags = nullptr);

// ---- tail.hip ----
// Closing half kick of a velocity-Verlet step and per-block energy partials,
// fused into the force gather for systems up to kGatherKickMax atoms (one
// partial per kGatherAtoms atoms, summed by one workgroup).
// The skin check of the positions an integrator kernel has just drifted:
// an atom that moved more than half the skin since the last list build
// (minimum image, so a face crossing is no motion) raises H_MOVED, and the
// next evaluation needs no check of its own. hdr == nullptr: no check.
struct DispCheck {
    const double *ref;  // positions at the last build (SoA)
    double thr2;        // (skin / 2)^2
    int *hdr;
    const int *seg_of;  // batch: the atom's segment, whose moved flag is raised too
    int *seg_flag;
};

template <bool SEG>
__device__ __forceinline__ void disp_check(const DispCheck &dc, const double x[3], int n, int i,
                                           const Box &b)
{
#pragma clang fp contract(off)
    double d2 = 0.0;
    for (int k = 0; k < 3; ++k) {
        double d = x[k] - dc.ref[k * n + i];
        if (b.per[k]) {
            const double h = 0.5 * b.L[k];
            d = d > h ? d - b.L[k] : (d < -h ? d + b.L[k] : d);
        }
        d2 = d2 + d * d;
    }
    if (!(d2 <= dc.thr2)) {
        dc.hdr[H_MOVED] = 1;
        if constexpr (SEG)
            dc.seg_flag[4 * dc.seg_of[i] + kSegMoved] = 1;
    }
}

DispCheck disp_check_args(void *ws, const WsLayout &L, double skin);

struct KickArgs {
    double *vel;
    const double *mass;
    double dt;
    const double *e_cheap;
    double *part;      // [blocks][3]: expensive, cheap, kinetic (set by the launcher)
    double *energies;  // final sums
    int next;          // also apply the next step's opening half kick and drift
    int defer;         // leave the final sum to the next step's binning kernel
    double *pos;       // positions (drift of the next step)
    Box box;
    double *ke_atom;   // per-atom kinetic energy 0.5 m v^2 of the full step (batches)
    DispCheck chk;     // skin check of the next step's drifted positions (next != 0)
};
constexpr int kGatherKickMax = 65536;
// S capacities above this run the vector-sparse contraction in four-wave
// workgroups (two bins of the eight-wave table per wave)
constexpr int kO3FourWaveMin = 65536;
constexpr int kGatherAtoms = 16;  // atoms per workgroup of the force gather (16 lanes each)
// Workgroup b of a grid of gd runs on XCD b mod 8 (round-robin dispatch);
// numbering the workgroups XCD by XCD (a bijection when gd is a multiple of
// 8) gives each XCD a contiguous range of work items.
__device__ __forceinline__ int xcd_major(int b, int gd)
{
    return (gd & 7) ? b : (b & 7) * (gd >> 3) + (b >> 3);
}

constexpr double kKappa = 9.648533212e-3;     // eV/A/amu in A/fs^2
constexpr double kBoltzmann = 8.617333262e-5;  // eV/K

// Langevin terms added to the blended force of atoms with lambda == 0 inside
// an MD step: F += -(m c_fric) v + sqrt(m c_rand) xi.
struct LangevinArgs {
    const double *vel;   // velocities at the force call (after the opening half kick)
    const double *mass;
    const double *xi;    // [3][n] standard normals, refilled by the caller per step
    double c_fric;       // 1 / (kappa tau)
    double c_rand;       // 2 kB T / (kappa tau dt)
};
void launch_gather_blend(hipStream_t s, const Ctx &c, void *ws, const WsLayout &L, int use_exp,
                         int use_cheap, const double *lambda, double *forces, double *e_exp,
                         double *f_exp, double *f_cheap, double sign,
                         const KickArgs *kick = nullptr, const LangevinArgs *lang = nullptr,
                         hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
void launch_fill_f64(hipStream_t s, double *p, double v, size_t n);
void launch_vv_kick_sums(hipStream_t s, void *ws, const WsLayout &L, double *vel,
                         const double *mass, const double *forces, double dt, const double *e_exp,
                         const double *e_cheap, double *out);
void launch_reduce(hipStream_t s, void *ws, const WsLayout &L, const double *e_exp,
                   const double *e_cheap, const double *vel, const double *mass, double *out);
void launch_vv_kick_drift(hipStream_t s, void *ws, const WsLayout &L, const Box &b, double *pos,
                          double *vel, const double *mass, const double *forces, double dt,
                          int drift, const DispCheck *chk = nullptr);
void launch_copy_i32(hipStream_t s, int32_t *dst, const int32_t *src, size_t n);
void launch_seg_fill(hipStream_t s, void *ws, const WsLayout &L);
// Neighbour-list state of the systems a new batch keeps from an old one
// (rows with their atom indices moved to the new offsets, counts, reverse
// slots, reference positions, per-system built and moved flags); seg_map of
// the new workspace holds each new segment's old index or -1.
void launch_carry_lists(hipStream_t s, void *ws_new, const WsLayout &Ln, const void *ws_old,
                        const WsLayout &Lo);
void launch_seg_sums(hipStream_t s, void *ws, const WsLayout &L, const double *e_exp,
                     const double *e_cheap, const double *ke, const uint8_t *flags, double *out,
                     int32_t *counts);
void launch_probe_mfma_f32(hipStream_t s, int blocks, int iters, float *sink);

// ---- fit.hip (constrained linear fitting of the cheap potential) ----
constexpr int kFitMaxParams = 120;  // packed Cholesky factor of the search in LDS
constexpr int kFitBatch = 24;       // configurations per design launch (kernel-argument size)
// One configuration of a design call: its workspace (whose pair-gradient
// scratch holds the per-atom energy rows and 3-body lists), positions,
// species, box and output rows.
struct FitCfgHost {
    void *ws;
    WsLayout L;
    Box box;
    const double *pos;
    const int32_t *species;
    double *rows;
};
void launch_fit_design(hipStream_t s, const Ctx &c, const FitCfgHost *cfg, int ncfg, int ld, int nd);
size_t fit_gram_parts(long long nrows, long long &chunk);
size_t fit_gram_part_bytes(int nd, size_t parts);
void launch_fit_gram(hipStream_t s, long long nrows, int nd, int ld, const double *A,
                     const double *y, const double *w, double *G, double *b, double *part);
void launch_fit_search(hipStream_t s, int nd, int nh, int ldh, const double *GS, const double *bS,
                       const double *AH, const double *yH, const double *wH, double alpha,
                       double tol, double lam0, double ridge, int max_decades, int max_bisect,
                       double *c, double *info, double *scratch);

}  // namespace mlmix
