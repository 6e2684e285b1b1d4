// Geometry stage of the mixed force evaluation on gfx950:
// neighbour-list rebuild decision, cell binning, neighbour rows, reverse
// slots, the mixing weight lambda and masks (Algorithms 1-2 with geometric
// core regions), the buffer set (Algorithm 3 / buffer-set equation) and the
// ordered stream compaction of S = {lambda > 0} + buffer.
//
// Every geometric decision (pair inside a radius, lambda, membership) is made
// in FP64 without FMA contraction so that it reproduces the CPU reference
// bit for bit.
#include "internal.h"
#include "reduce.h"

namespace mlmix {

#pragma clang fp contract(off)

__device__ __forceinline__ void pair_disp(const double *__restrict__ pos, int n, int i, int j,
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

__device__ __forceinline__ double norm2(const double d[3])
{
#pragma clang fp contract(off)
    double s = d[0] * d[0];
    s = s + d[1] * d[1];
    s = s + d[2] * d[2];
    return s;
}

__device__ __forceinline__ int cell_coord(double x, const Grid &g, int k)
{
    int q = (int)floor(x / g.cs[k]);
    if (q < 0)
        q = 0;
    if (q >= g.nc[k])
        q = g.nc[k] - 1;
    return q;
}

// ---------------------------------------------------------------- scans

__device__ __forceinline__ int wave_incl_scan(int x)
{
    int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int t = __shfl_up(x, d);
        if (lane >= d)
            x += t;
    }
    return x;
}

// Exclusive scan across a 256-thread block.
__device__ __forceinline__ int block_excl_scan(int v, int *sh, int &total)
{
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int x = wave_incl_scan(v);
    if (lane == 63)
        sh[w] = x;
    __syncthreads();
    int off = 0;
    total = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int s = sh[k];
        if (k < w)
            off += s;
        total += s;
    }
    __syncthreads();
    return off + x - v;
}

constexpr int kPer = kScanTile / 256;

// ------------------------------------------------------ rebuild decision
//
// Without a forced rebuild, k_displacement raises H_MOVED when an atom moved
// more than half the skin since the last build; the binning kernel (every
// workgroup, from words no kernel writes meanwhile) decides rebuild = forced
// or never built or moved, and its first workgroup publishes the decision in
// H_REBUILD for the later kernels; the row kernel's first workgroup clears
// H_MOVED for the next call and marks the list built.

template <bool SEG>
__global__ void __launch_bounds__(256) k_displacement(const double *__restrict__ pos,
                                                      const double *__restrict__ ref, int n,
                                                      Box b0, double thr2, int *hdr, Seg sg)
{
#pragma clang fp contract(off)
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    // positions in periodic dimensions wrap when an atom crosses a face: the
    // difference is folded to the minimum image (a crossing is no motion;
    // the rows hold atom indices, and every pair distance is folded anyway)
    const Box b = seg_box<SEG>(b0, sg, i);
    double d2 = 0.0;
    for (int k = 0; k < 3; ++k) {
        double d = pos[k * n + i] - ref[k * n + i];
        if (b.per[k]) {
            const double h = 0.5 * b.L[k];
            d = d > h ? d - b.L[k] : (d < -h ? d + b.L[k] : d);
        }
        d2 = d2 + d * d;
    }
    if (!(d2 <= thr2)) {
        hdr[H_MOVED] = 1;
        if constexpr (SEG)
            sg.flag[4 * sg.of[i] + kSegMoved] = 1;
    }
}

// ------------------------------------------------ lambda, cell lists

// Mixing weight of atom i: the largest linear blend over the regions
// (Algorithms 1-2), its masks (bit 0: lambda > 0, bit 1: lambda == 1) and
// whether it may join the buffer (lambda == 0 but near some region).
// Blend value at t in [0, 1): linear 1 - t (Algorithm 2) or cubic
// 1 - 3 t^2 + 2 t^3 (zero slope at both ends).
__device__ __forceinline__ double blend_value(double t, int cubic)
{
#pragma clang fp contract(off)
    return cubic ? 1.0 - t * t * (3.0 - 2.0 * t) : 1.0 - t;
}

// Mixing weight of atom i from the geometric regions (Algorithms 1-2 with
// core shapes): the largest blend value over the regions, its masks (bit 0:
// lambda > 0, bit 1: lambda == 1) and whether it may join the buffer
// (lambda == 0 but near some region). Seeded regions are applied by later
// passes over the neighbour rows; here seed atoms (with any seeded region
// present) are core atoms of all of them, and the seed bit of flags is kept.
template <bool SEG>
__device__ __forceinline__ void atom_lambda(const double *__restrict__ pos, int n, const Box &b,
                                            int i, const RegionArgs &ra, int *hdr, const Seg &sg)
{
#pragma clang fp contract(off)
    int z = ra.species[i];
    if (z < 0 || z >= ra.ns)
        seg_status_or<SEG>(&hdr[H_STATUS], sg, i, MLMIX_STATUS_BAD_SPECIES);
    const uint8_t keep = ra.seeded ? (uint8_t)(ra.flags[i] & MLMIX_FLAG_SEED) : (uint8_t)0;
    if (ra.mode == MLMIX_MODE_ALL_EXPENSIVE) {
        ra.lam[i] = 1.0;
        ra.flags[i] = (uint8_t)(3 | keep);
        ra.cand[i] = 0;
        return;
    }
    if (ra.mode == MLMIX_MODE_ALL_CHEAP) {
        ra.lam[i] = 0.0;
        ra.flags[i] = keep;
        ra.cand[i] = 0;
        return;
    }
    double best = 0.0;
    bool near = false;
    int n_seeded = 0;
    double xi[3] = {pos[i], pos[n + i], pos[2 * n + i]};
    // a batched call: the atom's own system's regions, atom indices local to it
    int g0 = 0, g1 = ra.nreg, a0 = 0, na = n;
    if constexpr (SEG) {
        const SegGeo &G = sg.geo[sg.of[i]];
        g0 = G.reg0;
        g1 = G.reg0 + G.nreg;
        a0 = G.off;
        na = G.n;
    }
    // single systems with many regions: only the regions listed for the
    // atom's superblock (every region within the buffer prefilter distance
    // of it); the largest blend value and the prefilter bit do not depend on
    // the order in which regions are visited
    const int *list = nullptr;
    int nlist = -1;
    if constexpr (!SEG) {
        if (ra.rgrid) {
            int sb = 0;
            for (int k = 2; k >= 0; --k) {
                double x = xi[k];
                if (b.per[k])
                    x = x - b.L[k] * floor(x / b.L[k]);
                int q = (int)(x * ra.rgn[k] / b.L[k]);
                q = q < 0 ? 0 : (q >= ra.rgn[k] ? ra.rgn[k] - 1 : q);
                sb = sb * ra.rgn[k] + q;
            }
            list = ra.rgrid + (size_t)sb * (kRegionGridCap + 1);
            nlist = list[0];  // -1: the list overflowed, every region
        }
    }
    const int nvisit = nlist >= 0 ? nlist : g1 - g0;
    for (int iv = 0; iv < nvisit; ++iv) {
        const int g = nlist >= 0 ? list[1 + iv] : g0 + iv;
        mlmix_region r = ra.reg[g];
        if (r.type == MLMIX_REGION_SEEDED) {
            ++n_seeded;
            continue;
        }
        double c[3] = {r.center[0], r.center[1], r.center[2]};
        if (r.follow_atom >= 0 && r.follow_atom < na) {
            const int fa = a0 + r.follow_atom;
            c[0] = pos[fa];
            c[1] = pos[n + fa];
            c[2] = pos[2 * n + fa];
        }
        double d[3];
        for (int k = 0; k < 3; ++k) {
            double dx = xi[k] - c[k];
            if (b.per[k]) {
                double h = 0.5 * b.L[k];
                if (dx > h)
                    dx = dx - b.L[k];
                else if (dx < -h)
                    dx = dx + b.L[k];
            }
            d[k] = dx;
        }
        if (r.type == 1 && r.axis >= 0 && r.axis < 3)
            d[r.axis] = 0.0;
        double d2 = norm2(d);
        double rc = r.r_core, rb = r.r_blend;
        double outer = rc + rb;
        double v;
        if (d2 < rc * rc) {
            v = 1.0;
        } else if (d2 < outer * outer) {
            double dist = sqrt(d2);
            double t = (dist - rc) / rb;
            v = blend_value(t, r.blend);
        } else {
            v = 0.0;
        }
        if (v > best)
            best = v;
        // buffer prefilter: a buffer atom lies within r_buffer of an atom
        // with lambda > 0, hence (triangle inequality) within
        // r_core + r_blend + r_buffer of some region; a margin keeps the
        // test conservative under rounding
        double far = outer + ra.r_buffer + 1.0e-6;
        if (d2 < far * far)
            near = true;
    }
    if (ra.seeded) {
        const bool is_seed = keep != 0 && n_seeded > 0;
        if (is_seed)
            best = 1.0;
        ra.seedcore[i] = is_seed ? (uint8_t)0xff : (uint8_t)0;
        if (n_seeded > kMaxSeeded && i == 0)
            atomicOr(&hdr[H_STATUS], MLMIX_STATUS_SEEDED_REGIONS);
    }
    ra.lam[i] = best;
    uint8_t f = keep;
    if (best > 0.0)
        f |= 1;
    if (best == 1.0)
        f |= 2;
    ra.flags[i] = f;
    ra.cand[i] = (best == 0.0 && near) ? 1 : 0;
}


// Region lists per superblock (single systems with many geometric regions):
// one thread per superblock of the box lists every region whose buffer
// prefilter sphere (r_core + r_blend + r_buffer, plus a margin for rounding)
// reaches the superblock's box (minimum image along periodic dimensions; an
// axis region ignores its axis). A list longer than kRegionGridCap is marked
// -1 and its atoms test every region.
__global__ void __launch_bounds__(256) k_region_grid(const double *__restrict__ pos, int n, Box b,
                                                     const mlmix_region *__restrict__ reg, int nreg,
                                                     double r_buffer, int g0, int g1, int g2,
                                                     int *__restrict__ lists)
{
#pragma clang fp contract(off)
    const int sb = blockIdx.x * blockDim.x + threadIdx.x;
    if (sb >= g0 * g1 * g2)
        return;
    const int q[3] = {sb % g0, (sb / g0) % g1, sb / (g0 * g1)};
    const int gn[3] = {g0, g1, g2};
    int *out = lists + (size_t)sb * (kRegionGridCap + 1);
    int cnt = 0;
    for (int g = 0; g < nreg; ++g) {
        const mlmix_region r = reg[g];
        double c[3] = {r.center[0], r.center[1], r.center[2]};
        if (r.follow_atom >= 0 && r.follow_atom < n) {
            c[0] = pos[r.follow_atom];
            c[1] = pos[n + r.follow_atom];
            c[2] = pos[2 * n + r.follow_atom];
        }
        double d2 = 0.0;
        for (int k = 0; k < 3; ++k) {
            if (r.type == 1 && r.axis == k)
                continue;
            const double w = b.L[k] / gn[k];
            const double mid = (q[k] + 0.5) * w;
            double d = c[k] - mid;
            if (b.per[k]) {
                const double h = 0.5 * b.L[k];
                d = d - b.L[k] * floor((d + h) / b.L[k]);  // into [-L/2, L/2)
            }
            d = fabs(d) - 0.5 * w;
            if (d > 0.0)
                d2 = d2 + d * d;
        }
        const double far = r.r_core + r.r_blend + r_buffer + 1.0e-3;
        if (d2 < far * far) {
            if (cnt < kRegionGridCap)
                out[1 + cnt] = g;
            ++cnt;
        }
    }
    out[0] = cnt <= kRegionGridCap ? cnt : -1;
}

// One thread per atom: the mixing weight pass (every call), then, when the
// list is rebuilt, cell binning into fixed-capacity buckets (g.bucket
// records per cell): cell index, one device atomic for the slot, one 32-byte
// record. Counts
// must be zero on entry (cleared by the reverse-slot pass of the previous
// rebuild and at workspace set-up). A full bucket drops the atom and raises
// MLMIX_STATUS_CELL_OVERFLOW. On a forced rebuild it also raises the rebuild
// flag (otherwise the flag comes from the displacement check before it) and,
// whenever the list is rebuilt, marks the workspace as built. Order inside a
// bucket follows the atomics; the rows are sorted afterwards.
template <bool SEG>
__global__ void __launch_bounds__(256) k_bin_bucket(const double *__restrict__ pos, int n, Box b0,
                                                    Grid g0, int force, int *hdr,
                                                    int *__restrict__ count,
                                                    CellAtom *__restrict__ atoms, RegionArgs ra,
                                                    Seg sg)
{
    // the previous step's energy sums (multi-step calls), by the whole of
    // workgroup 0 before anything else
    if (ra.red_part && blockIdx.x == 0)
        reduce_parts(ra.red_part, ra.red_nb, ra.red_out);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    // the atom's system: its box, grid and first cell / bucket record
    Box b = b0;
    Grid g = g0;
    int cell0 = 0;
    size_t rec0 = 0;
    if constexpr (SEG) {
        if (i < n) {
            const SegGeo &G = sg.geo[sg.of[i]];
            b = G.box;
            g = G.grid;
            cell0 = G.cell0;
            rec0 = (size_t)G.rec0;
        }
    }
    if (i < n)
        atom_lambda<SEG>(pos, n, b, i, ra, hdr, sg);
    int rebuild = (force || hdr[H_BUILT] == 0 || hdr[H_MOVED] != 0) ? 1 : 0;
    if (blockIdx.x == 0 && threadIdx.x == 0)
        hdr[H_REBUILD] = rebuild;  // some list is rebuilt (in a batch: some system's)
    if constexpr (SEG) {
        // a batch: every system keeps or rebuilds its own list, so that its
        // bits do not depend on the systems beside it; the system's first
        // atom publishes the decision for the row and reverse-slot kernels
        rebuild = 0;
        if (i < n) {
            const int k = sg.of[i];
            const int *f = sg.flag + 4 * k;
            rebuild = (force || f[kSegBuilt] == 0 || f[kSegMoved] != 0) ? 1 : 0;
            if (i == sg.geo[k].off)
                sg.flag[4 * k + kSegRebuild] = rebuild;
        }
    }
    if (!rebuild)
        return;  // uniform for a single system
    if (i >= n)
        return;
    double x[3];
    int c[3];
    bool bad = false, out = false;
    for (int k = 0; k < 3; ++k) {
        x[k] = pos[k * n + i];
        if (!(x[k] == x[k]) || x[k] < -1.0e300 || x[k] > 1.0e300)
            bad = true;
        if (!b.per[k] && (x[k] < 0.0 || x[k] >= b.L[k]))
            out = true;
        c[k] = cell_coord(x[k], g, k);
    }
    if (bad)
        seg_status_or<SEG>(&hdr[H_STATUS], sg, i, MLMIX_STATUS_NONFINITE);
    if (out)
        seg_status_or<SEG>(&hdr[H_STATUS], sg, i, MLMIX_STATUS_OUT_OF_BOX);
    const int cell = (c[2] * g.nc[1] + c[1]) * g.nc[0] + c[0];
    const int slot = atomicAdd(&count[cell0 + cell], 1);
    if (slot < g.bucket) {
        CellAtom r;
        r.x = x[0];
        r.y = x[1];
        r.z = x[2];
        r.j = i;
        r.pad = 0;
        atoms[rec0 + (size_t)cell * g.bucket + slot] = r;
    } else {
        seg_status_or<SEG>(&hdr[H_STATUS], sg, i, MLMIX_STATUS_CELL_OVERFLOW);
    }
}

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Ascending bitonic sort of 64 V keys held V per lane (key e = V lane + v):
// in-lane stages swap registers, cross-lane stages exchange with the lane
// lane ^ (j / V) and keep the minimum or the maximum.
template <int V>
__device__ __forceinline__ void wave_bitonic_sort(int (&x)[V])
{
    const int lane = threadIdx.x & 63;
    constexpr int N = 64 * V;
#pragma unroll
    for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j < V) {
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const int u = v ^ j;
                    if (u > v) {
                        const bool up = ((lane * V + v) & k) == 0;
                        const int a = x[v], b = x[u];
                        if ((a > b) == up) {
                            x[v] = b;
                            x[u] = a;
                        }
                    }
                }
            } else {
                const int pl = j / V;
                const bool lower = (lane & pl) == 0;
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const int other = __shfl_xor(x[v], pl);
                    const bool up = ((lane * V + v) & k) == 0;
                    x[v] = (lower == up) ? min(x[v], other) : max(x[v], other);
                }
            }
        }
    }
}

template <int V>
__device__ __forceinline__ void row_sort_store(const int *row, int lane, int keep, int cap,
                                               int *__restrict__ out)
{
    int x[V];
#pragma unroll
    for (int v = 0; v < V; ++v)
        x[v] = row[lane * V + v];
    wave_bitonic_sort<V>(x);
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int sl = lane * V + v;
        if (sl < cap)
            out[sl] = sl < keep ? x[v] : -1;
    }
}

// Candidate records listed per wave (at most this many; more fall back to
// the per-cell walk).
constexpr int kNbrList = 512;

// One wavefront per atom, four atoms per 256-thread block, no block-level
// barriers (each wave works in its own LDS slice). Each lane owns up to two
// cells of the (up to) 5x5x5 stencil of half-radius cells; a wave scan of
// their bucket sizes places the candidates' record indices side by side in
// LDS, and the lanes then test two 32-byte records per round (loads issued
// first). Partners closer than the list radius are kept by ballot
// compaction, and the row is finally sorted ascending in registers (bitonic
// over 64, 128 or 256 keys).
template <bool SEG>
__global__ void __launch_bounds__(256) k_neighbors(const double *__restrict__ pos, int n, Box b0,
                                                   Grid g0, const int *__restrict__ count0,
                                                   const CellAtom *__restrict__ atoms0, double rl2,
                                                   int cap, int P, int *__restrict__ nbr,
                                                   int *__restrict__ cnt,
                                                   double *__restrict__ ref, int *hdr,
                                                   double rb2, uint8_t *__restrict__ flags,
                                                   const uint8_t *__restrict__ cand, Seg sg)
{
#pragma clang fp contract(off)
    int rebuild = hdr[H_REBUILD];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        hdr[H_MOVED] = 0;  // for the next call's displacement check
        if (rebuild) {
            hdr[H_BUILT] = 1;
            hdr[H_NBUILD] += 1;
        }
    }
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + w;
    if constexpr (SEG) {
        // the decision of the atom's own system (published by the binning
        // kernel); the wave of its first atom clears the system's moved flag
        // and marks its list built
        if (i < n) {
            const int k = __builtin_amdgcn_readfirstlane(sg.of[i]);
            rebuild = sg.flag[4 * k + kSegRebuild];
            if (i == sg.geo[k].off && lane == 0) {
                sg.flag[4 * k + kSegMoved] = 0;
                if (rebuild)
                    sg.flag[4 * k + kSegBuilt] = 1;
            }
        }
    }
    if (rebuild == 0) {
        // kept list: this call's buffer test over the kept row (the same
        // test as the rebuild path below): a candidate joins the buffer when
        // a partner with lambda > 0 lies strictly inside r_buffer
        if (rb2 >= 0.0 && i < n && cand[i]) {
            const Box bb = seg_box<SEG, true>(b0, sg, i);
            const int c = cnt[i];
            const int *row = nbr + (size_t)i * cap;
            bool hit = false;
            for (int sl = lane; sl < c; sl += 64) {
                const int j = row[sl];
                if (flags[j] & 1) {
                    double d[3];
                    pair_disp(pos, n, i, j, bb, d);
                    if (norm2(d) < rb2)
                        hit = true;
                }
            }
            if (__ballot(hit) != 0ull && lane == 0)
                flags[i] = (uint8_t)(flags[i] | 4);
        }
        return;
    }
    __shared__ int rows[4][kMaxCap];
    __shared__ int lists[4][kNbrList];
    if (i >= n)
        return;
    // the atom's system: its box, grid, cell counts and bucket records
    Box b = b0;
    Grid g = g0;
    const int *count = count0;
    const CellAtom *atoms = atoms0;
    if constexpr (SEG) {
        const SegGeo &G = sg.geo[__builtin_amdgcn_readfirstlane(sg.of[i])];
        b = G.box;
        g = G.grid;
        count = count0 + G.cell0;
        atoms = atoms0 + G.rec0;
    }
    const int Pe = P < 64 ? 64 : P;  // keys sorted (64 V)
    int *row = rows[w];
    for (int t = lane; t < Pe; t += 64)
        row[t] = 0x7fffffff;
    int nst[3];
    for (int k = 0; k < 3; ++k)
        nst[k] = (b.per[k] && g.nc[k] < 5) ? g.nc[k] : 5;
    const int total = nst[0] * nst[1] * nst[2];  // <= 125
    double xi[3];
    int ci[3];
    for (int k = 0; k < 3; ++k) {
        xi[k] = pos[k * n + i];
        ci[k] = cell_coord(xi[k], g, k);
    }
    // stencil cells t = lane and t = lane + 64: first slot and size
    int sz[2];
    size_t bg[2];
    for (int h = 0; h < 2; ++h) {
        int t = lane + 64 * h;
        sz[h] = 0;
        bg[h] = 0;
        if (t < total) {
            int o[3] = {t % nst[0] - 2, (t / nst[0]) % nst[1] - 2, t / (nst[0] * nst[1]) - 2};
            int q[3];
            bool ok = true;
            for (int k = 0; k < 3; ++k) {
                int v = ci[k] + o[k];
                if (b.per[k]) {
                    v %= g.nc[k];
                    if (v < 0)
                        v += g.nc[k];
                } else if (v < 0 || v >= g.nc[k]) {
                    ok = false;
                }
                q[k] = v;
            }
            if (ok) {
                int cell = (q[2] * g.nc[1] + q[1]) * g.nc[0] + q[0];
                bg[h] = (size_t)cell * g.bucket;
                sz[h] = min(count[cell], g.bucket);
            }
        }
    }
    // partner test of one record: inside the list radius (FP64, minimum
    // image, no contraction) and not the atom itself; hits are compacted by
    // ballot into the row (c counts every hit, also those past P). A buffer
    // candidate (rb2 >= 0) also looks for a partner with lambda > 0 strictly
    // inside the buffer radius (the same distance as the buffer pass).
    int c = 0;
    const bool want_buf = rb2 >= 0.0 && cand[i];
    bool in_buf = false;
    auto test = [&](bool valid, const CellAtom &r) {
        bool hit = false;
        if (valid) {
            double d[3] = {r.x - xi[0], r.y - xi[1], r.z - xi[2]};
            for (int k = 0; k < 3; ++k) {
                if (b.per[k]) {
                    double hh = 0.5 * b.L[k];
                    double dx = d[k];
                    dx = dx > hh ? dx - b.L[k] : (dx < -hh ? dx + b.L[k] : dx);
                    d[k] = dx;
                }
            }
            const double d2 = norm2(d);
            hit = (r.j != i) && d2 < rl2;
            if (want_buf && hit && d2 < rb2 && (flags[r.j] & 1))
                in_buf = true;
        }
        unsigned long long m = __ballot(hit);
        int p = c + __popcll(m & ((1ull << lane) - 1ull));
        if (hit && p < P)
            row[p] = r.j;
        c += __popcll(m);
    };
    // candidates in stencil-cell order: offsets by a wave scan of the sizes
    const int inc0 = wave_incl_scan(sz[0]);
    const int tot0 = __shfl(inc0, 63);
    const int inc1 = wave_incl_scan(sz[1]);
    const int ncand = tot0 + __shfl(inc1, 63);
    if (ncand <= kNbrList) {
        // dense list of the candidates' record indices; every lane then takes
        // two records per round, loads first
        int *lst = lists[w];
        const int o0 = inc0 - sz[0], o1 = tot0 + inc1 - sz[1];
        for (int k = 0; k < sz[0]; ++k)
            lst[o0 + k] = (int)bg[0] + k;
        for (int k = 0; k < sz[1]; ++k)
            lst[o1 + k] = (int)bg[1] + k;
        wave_sync_lds();
        for (int f0 = 0; f0 < ncand; f0 += 128) {
            const int fa = f0 + lane, fb = f0 + 64 + lane;
            CellAtom ra{}, rb{};
            if (fa < ncand)
                ra = atoms[lst[fa]];
            if (fb < ncand)
                rb = atoms[lst[fb]];
            test(fa < ncand, ra);
            test(fb < ncand, rb);
        }
    } else {
        // dense cells: every lane walks its own stencil cells (t and t + 64),
        // kB records of each at a time with their loads issued first
        int szmax = max(sz[0], sz[1]);
#pragma unroll
        for (int d = 32; d > 0; d >>= 1)
            szmax = max(szmax, __shfl_xor(szmax, d));
        constexpr int kB = 2;
        for (int k0 = 0; k0 < szmax; k0 += kB) {
            CellAtom rec[2][kB];
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int u = 0; u < kB; ++u)
                    if (k0 + u < sz[h])
                        rec[h][u] = atoms[bg[h] + k0 + u];
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int u = 0; u < kB; ++u)
                    test(k0 + u < sz[h], rec[h][u]);
        }
    }
    wave_sync_lds();
    const int keep = c < cap ? c : cap;
    int *out = nbr + (size_t)i * cap;
    if (Pe == 64)
        row_sort_store<1>(row, lane, keep, cap, out);
    else if (Pe == 128)
        row_sort_store<2>(row, lane, keep, cap, out);
    else
        row_sort_store<4>(row, lane, keep, cap, out);
    if (__ballot(in_buf) != 0ull && lane == 0)
        flags[i] = (uint8_t)(flags[i] | 4);
    if (lane == 0) {
        cnt[i] = keep;
        // same-address device atomics serialise across the whole grid: only
        // an overflowing row records its length
        if (c > cap) {
            seg_status_or<SEG>(&hdr[H_STATUS], sg, i, MLMIX_STATUS_NEIGH_OVERFLOW);
            atomicMax(&hdr[H_REQCAP], c);
        }
    }
    if (lane < 3)
        ref[lane * n + i] = pos[lane * n + i];
}

// rev[i][s] = slot of i in the row of j = nbr[i][s] (rows are ascending).
// One wavefront per atom i (grid-stride), lane l owns slots l + 64 u; the U
// searches of a lane advance together, each a branch-free binary search of
// log2(P) steps (P = row capacity rounded up to a power of two). The bucket
// counts of the rebuild are no longer needed: they are cleared here for the
// next one.
template <int U>
__global__ void __launch_bounds__(256) k_reverse(int n, int cap, int P, const int *__restrict__ nbr,
                                                 const int *__restrict__ cnt,
                                                 int *__restrict__ rev, int *__restrict__ count,
                                                 int ncell, int *hdr, const int *__restrict__ seg_of,
                                                 const int *__restrict__ seg_flag)
{
    if (hdr[H_REBUILD] == 0)
        return;
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    for (int c = tid; c < ncell; c += gridDim.x * blockDim.x)
        count[c] = 0;
    const int lane = threadIdx.x & 63;
    for (int i = blockIdx.x * 4 + (threadIdx.x >> 6); i < n; i += gridDim.x * 4) {
        if (seg_of && seg_flag[4 * seg_of[i] + kSegRebuild] == 0)
            continue;  // a batch system that kept its list keeps its slots (uniform)
        const int ci = cnt[i];
        const int *rowi = nbr + (size_t)i * cap;
        int j[U], cj[U], pos[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int sl = lane + 64 * u;
            j[u] = sl < ci ? rowi[sl] : -1;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            cj[u] = j[u] >= 0 ? cnt[j[u]] : 0;
            pos[u] = 0;
        }
        // pos = number of entries of row j smaller than i
        for (int step = P >> 1; step > 0; step >>= 1) {
            int v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = pos[u] + step - 1;
                v[u] = (j[u] >= 0 && k < cj[u]) ? nbr[(size_t)j[u] * cap + k] : 0x7fffffff;
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (v[u] < i)
                    pos[u] += step;
        }
        if (P == 1) {
#pragma unroll
            for (int u = 0; u < U; ++u)
                pos[u] = (j[u] >= 0 && cj[u] > 0 && nbr[(size_t)j[u] * cap] < i) ? 1 : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int sl = lane + 64 * u;
            if (sl < cap) {
                int r = -1;
                if (j[u] >= 0 && pos[u] < cj[u] && nbr[(size_t)j[u] * cap + pos[u]] == i)
                    r = pos[u];
                rev[(size_t)i * cap + sl] = r;
            }
        }
    }
}

DispCheck disp_check_args(void *ws, const WsLayout &L, double skin)
{
    const double thr = 0.5 * skin;
    if (L.nseg > 0)
        return DispCheck{at<double>(ws, L.ref_pos), thr * thr, at<int>(ws, L.hdr),
                         at<int>(ws, L.seg_of), at<int>(ws, L.seg_flag)};
    return DispCheck{at<double>(ws, L.ref_pos), thr * thr, at<int>(ws, L.hdr), nullptr, nullptr};
}

void launch_neighbors(hipStream_t s, void *ws, const WsLayout &L, const Box &b, double r_list,
                      const double *pos, int force_rebuild, double skin, const RegionArgs &ra,
                      bool checked)
{
    // the row kernel also finds the buffer atoms (mixed mode) whenever it runs
    int *hdr = at<int>(ws, L.hdr);
    const Grid &g = L.grid;
    const int n = L.n;
    if (n == 0)
        return;
    if (!force_rebuild && !checked) {
        double thr = 0.5 * skin;
        if (L.nseg > 0)
            k_displacement<true><<<(n + 255) / 256, 256, 0, s>>>(
                pos, at<double>(ws, L.ref_pos), n, b, thr * thr, hdr, seg_args(ws, L));
        else
            k_displacement<false><<<(n + 255) / 256, 256, 0, s>>>(
                pos, at<double>(ws, L.ref_pos), n, b, thr * thr, hdr, seg_args(ws, L));
    }
    int *count = at<int>(ws, L.cell_count);
    RegionArgs r = ra;
    r.cand = at<uint8_t>(ws, L.cand);
    r.seedcore = at<uint8_t>(ws, L.seedcore);
    if (L.nseg == 0 && ra.mode == MLMIX_MODE_MIXED && !ra.seeded && ra.nreg >= kRegionGridMin) {
        const int nsb = L.rgn[0] * L.rgn[1] * L.rgn[2];
        int *lists = at<int>(ws, L.rgrid);
        k_region_grid<<<(nsb + 255) / 256, 256, 0, s>>>(pos, n, b, ra.reg, ra.nreg, ra.r_buffer,
                                                         L.rgn[0], L.rgn[1], L.rgn[2], lists);
        r.rgrid = lists;
        for (int k = 0; k < 3; ++k)
            r.rgn[k] = L.rgn[k];
    }
    const Seg sg = seg_args(ws, L);
    if (L.nseg > 0)
        k_bin_bucket<true><<<(n + 255) / 256, 256, 0, s>>>(pos, n, b, g, force_rebuild, hdr, count,
                                                           at<CellAtom>(ws, L.cell_atoms), r, sg);
    else
        k_bin_bucket<false><<<(n + 255) / 256, 256, 0, s>>>(pos, n, b, g, force_rebuild, hdr, count,
                                                            at<CellAtom>(ws, L.cell_atoms), r, sg);
    // (with seeded regions lambda is not final yet: the buffer pass follows them)
    const double rb2 =
        ra.mode == MLMIX_MODE_MIXED && !ra.seeded ? ra.r_buffer * ra.r_buffer : -1.0;
    if (L.nseg > 0)
        k_neighbors<true><<<(n + 3) / 4, 256, 0, s>>>(pos, n, b, g, count, at<CellAtom>(ws, L.cell_atoms),
                                                r_list * r_list, L.cap, L.P, at<int>(ws, L.nbr),
                                                at<int>(ws, L.cnt), at<double>(ws, L.ref_pos), hdr,
                                                rb2, ra.flags, r.cand, sg);
    else
        k_neighbors<false><<<(n + 3) / 4, 256, 0, s>>>(pos, n, b, g, count, at<CellAtom>(ws, L.cell_atoms),
                                                r_list * r_list, L.cap, L.P, at<int>(ws, L.nbr),
                                                at<int>(ws, L.cnt), at<double>(ws, L.ref_pos), hdr,
                                                rb2, ra.flags, r.cand, sg);
}

// Reverse slots of a rebuilt list (skipped on the device when the list was
// kept); needed by the force gather only, so it may run beside the potentials.
// Uncapped form: one thread per (i, s), early-exit binary search in row j,
// over a grid of at most kRevFlatBlocks workgroups that strides over the
// slots (a kept list then costs a few microseconds instead of the dispatch of
// one workgroup per 256 slots: 1M atoms x 128 slots are 512k workgroups).
constexpr unsigned kRevFlatBlocks = 16384;
__global__ void __launch_bounds__(256) k_reverse_flat(int n, int cap, const int *__restrict__ nbr,
                                                      const int *__restrict__ cnt,
                                                      int *__restrict__ rev,
                                                      int *__restrict__ count, int ncell, int *hdr,
                                                      const int *__restrict__ seg_of,
                                                      const int *__restrict__ seg_flag)
{
    if (hdr[H_REBUILD] == 0)
        return;
    const size_t nslot = (size_t)n * cap;
    const size_t tot = nslot > (size_t)ncell ? nslot : (size_t)ncell;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += stride) {
        if (t < (size_t)ncell)
            count[t] = 0;
        if (t >= nslot)
            continue;
        // 32-bit division whenever the index fits (64-bit division is slow)
        const int i = t < 0xffffffffull ? (int)((unsigned)t / (unsigned)cap) : (int)(t / cap);
        if (seg_of && seg_flag[4 * seg_of[i] + kSegRebuild] == 0)
            continue;  // a batch system that kept its list keeps its slots
        const int sl = (int)(t - (size_t)i * cap);
        int r = -1;
        if (sl < cnt[i]) {
            const int j = nbr[t];
            const int *rowj = nbr + (size_t)j * cap;
            int lo = 0, hi = cnt[j] - 1;
            while (lo <= hi) {
                const int mid = (lo + hi) >> 1;
                const int v = rowj[mid];
                if (v == i) {
                    r = mid;
                    break;
                }
                if (v < i)
                    lo = mid + 1;
                else
                    hi = mid - 1;
            }
        }
        rev[t] = r;
    }
}

void launch_reverse(hipStream_t s, void *ws, const WsLayout &L, int side_blocks)
{
    const int n = L.n;
    if (n == 0)
        return;
    const Seg sg = seg_args(ws, L);  // batch: per-system decisions
    // uncapped: one thread per slot (measured faster on 1M atoms); capped
    // beside the expensive chain: a wave per atom, grid-stride
    const size_t tot = std::max((size_t)n * L.cap, (size_t)L.grid.ncell);
    if (side_blocks <= 0 || (tot + 255) / 256 <= (size_t)side_blocks) {
        k_reverse_flat<<<(unsigned)std::min<size_t>((tot + 255) / 256, kRevFlatBlocks), 256, 0, s>>>(
            n, L.cap, at<int>(ws, L.nbr), at<int>(ws, L.cnt), at<int>(ws, L.rev),
            at<int>(ws, L.cell_count), L.grid.ncell, at<int>(ws, L.hdr), sg.of, sg.flag);
        return;
    }
    unsigned nblk = (unsigned)((n + 3) / 4);
    if (nblk > (unsigned)side_blocks)
        nblk = side_blocks;
#define MLMIX_REV(U)                                                                              \
    k_reverse<U><<<nblk, 256, 0, s>>>(n, L.cap, L.P, at<int>(ws, L.nbr), at<int>(ws, L.cnt),       \
                                      at<int>(ws, L.rev), at<int>(ws, L.cell_count), L.grid.ncell, \
                                      at<int>(ws, L.hdr), sg.of, sg.flag)
    switch ((L.cap + 63) / 64) {
    case 1: MLMIX_REV(1); break;
    case 2: MLMIX_REV(2); break;
    case 3: MLMIX_REV(3); break;
    default: MLMIX_REV(4); break;
    }
#undef MLMIX_REV
}

// --------------------------------------------------------- lambda / masks

// One wavefront per atom (lanes over row slots): an atom with lambda == 0
// near a region joins the buffer when any neighbour with lambda > 0 lies
// strictly inside r_buffer.
template <bool SEG>
__global__ void __launch_bounds__(256) k_buffer(const double *__restrict__ pos, int n, Box b0,
                                                int cap, const int *__restrict__ nbr,
                                                const int *__restrict__ cnt, double rb2,
                                                uint8_t *__restrict__ flags,
                                                const uint8_t *__restrict__ cand, Seg sg)
{
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= n || !cand[i])
        return;
    const Box b = seg_box<SEG, true>(b0, sg, i);
    const int c = cnt[i];
    const int *row = nbr + (size_t)i * cap;
    bool hit = false;
    for (int s = lane; s < c; s += 64) {
        int j = row[s];
        if (flags[j] & 1) {
            double d[3];
            pair_disp(pos, n, i, j, b, d);
            if (norm2(d) < rb2)
                hit = true;
        }
    }
    if (__ballot(hit) != 0ull && lane == 0)
        flags[i] = (uint8_t)(flags[i] | 4);
}

// Seeded regions, pass 1 (Algorithm 1 as a gather over the symmetric rows):
// atom j (not a seed) is a core atom of seeded region k when a seed lies in
// its row strictly closer than that region's r_core. One wavefront per atom.
__global__ void __launch_bounds__(256) k_seed_core(const double *__restrict__ pos, int n, Box b,
                                                   int cap, const int *__restrict__ nbr,
                                                   const int *__restrict__ cnt,
                                                   const mlmix_region *__restrict__ reg, int nreg,
                                                   double *__restrict__ lam,
                                                   uint8_t *__restrict__ flags,
                                                   uint8_t *__restrict__ seedcore)
{
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (j >= n || (flags[j] & MLMIX_FLAG_SEED))
        return;
    const int c = cnt[j];
    const int *row = nbr + (size_t)j * cap;
    unsigned bits = 0;
    for (int sl = lane; sl < c; sl += 64) {
        const int i = row[sl];
        if (!(flags[i] & MLMIX_FLAG_SEED))
            continue;
        double d[3];
        pair_disp(pos, n, j, i, b, d);
        const double d2 = norm2(d);
        int k = 0;
        for (int g = 0; g < nreg && k < kMaxSeeded; ++g) {
            if (reg[g].type != MLMIX_REGION_SEEDED)
                continue;
            if (d2 < reg[g].r_core * reg[g].r_core)
                bits |= 1u << k;
            ++k;
        }
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1)
        bits |= __shfl_xor(bits, d);
    if (lane == 0) {
        seedcore[j] = (uint8_t)bits;
        if (bits) {
            lam[j] = 1.0;
            flags[j] = (uint8_t)(flags[j] | 3);
        }
    }
}

// Seeded regions, pass 2 (Algorithm 2 as a gather): an atom j with
// lambda < 1 takes the largest b(r / r_blend) over the core atoms i of each
// seeded region in its row with r < r_blend (a maximum: the order of the
// lanes does not matter). Atoms left at lambda == 0 become buffer candidates.
__global__ void __launch_bounds__(256) k_seed_blend(const double *__restrict__ pos, int n, Box b,
                                                    int cap, const int *__restrict__ nbr,
                                                    const int *__restrict__ cnt,
                                                    const mlmix_region *__restrict__ reg,
                                                    int nreg, double *__restrict__ lam,
                                                    uint8_t *__restrict__ flags,
                                                    const uint8_t *__restrict__ seedcore,
                                                    uint8_t *__restrict__ cand)
{
#pragma clang fp contract(off)
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (j >= n)
        return;
    const double lj = lam[j];
    double best = 0.0;
    if (lj < 1.0) {
        const int c = cnt[j];
        const int *row = nbr + (size_t)j * cap;
        for (int sl = lane; sl < c; sl += 64) {
            const int i = row[sl];
            const unsigned core = seedcore[i];
            if (!core)
                continue;
            double d[3];
            pair_disp(pos, n, j, i, b, d);
            const double d2 = norm2(d);
            int k = 0;
            for (int g = 0; g < nreg && k < kMaxSeeded; ++g) {
                if (reg[g].type != MLMIX_REGION_SEEDED)
                    continue;
                const double rb = reg[g].r_blend;
                if ((core & (1u << k)) && d2 < rb * rb) {
                    const double v = blend_value(sqrt(d2) / rb, reg[g].blend);
                    best = v > best ? v : best;
                }
                ++k;
            }
        }
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) {
            const double o = __shfl_xor(best, d);
            best = o > best ? o : best;
        }
    }
    if (lane == 0) {
        double l = lj;
        if (best > l) {
            l = best;
            lam[j] = l;
            flags[j] = (uint8_t)(flags[j] | 1);
        }
        cand[j] = l == 0.0 ? 1 : 0;
    }
}

// The cheap potential's buffer (MLMIX_CHEAP_MASKED): an atom with
// lambda == 1 joins it (flags bit3) when a row partner with lambda < 1 lies
// strictly inside r_buffer. One wavefront per atom; others return at once.
template <bool SEG>
__global__ void __launch_bounds__(256) k_cheap_buffer(const double *__restrict__ pos, int n, Box b0,
                                                      int cap, const int *__restrict__ nbr,
                                                      const int *__restrict__ cnt, double rb2,
                                                      uint8_t *__restrict__ flags, Seg sg)
{
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= n || !(flags[i] & 2))
        return;
    const Box b = seg_box<SEG, true>(b0, sg, i);
    const int c = cnt[i];
    const int *row = nbr + (size_t)i * cap;
    bool hit = false;
    for (int sl = lane; sl < c; sl += 64) {
        const int j = row[sl];
        if (flags[j] & 2)
            continue;
        double d[3];
        pair_disp(pos, n, i, j, b, d);
        if (norm2(d) < rb2)
            hit = true;
    }
    if (__ballot(hit) != 0ull && lane == 0)
        flags[i] = (uint8_t)(flags[i] | 8);
}

void launch_cheap_buffer(hipStream_t s, void *ws, const WsLayout &L, const Box &b,
                         const double *pos, double r_buffer, uint8_t *flags)
{
    if (L.n == 0)
        return;
    if (L.nseg > 0)
        k_cheap_buffer<true><<<(L.n + 3) / 4, 256, 0, s>>>(pos, L.n, b, L.cap, at<int>(ws, L.nbr),
                                                           at<int>(ws, L.cnt), r_buffer * r_buffer,
                                                           flags, seg_args(ws, L));
    else
        k_cheap_buffer<false><<<(L.n + 3) / 4, 256, 0, s>>>(pos, L.n, b, L.cap, at<int>(ws, L.nbr),
                                                            at<int>(ws, L.cnt), r_buffer * r_buffer,
                                                            flags, seg_args(ws, L));
}

// Region stage after the rows, for seeded regions only: the seeded passes
// (MLMIX_SEEDED), then the buffer pass (lambda is final only now). Lambda and
// the masks of the geometric regions come from the binning kernel of the
// neighbour stage, and without seeded regions the row kernel does the buffer
// test on every call (on the rows it builds, or on the kept rows).
void launch_regions(hipStream_t s, void *ws, const WsLayout &L, const Box &b, int mode,
                    const double *pos, double r_buffer, uint8_t *flags, int force_rebuild,
                    const RegionArgs &ra)
{
    int n = L.n;
    const bool seeded = ra.seeded && mode == MLMIX_MODE_MIXED;
    if (n > 0 && seeded) {
        uint8_t *core = at<uint8_t>(ws, L.seedcore);
        k_seed_core<<<(n + 3) / 4, 256, 0, s>>>(pos, n, b, L.cap, at<int>(ws, L.nbr),
                                                at<int>(ws, L.cnt), ra.reg, ra.nreg, ra.lam,
                                                flags, core);
        k_seed_blend<<<(n + 3) / 4, 256, 0, s>>>(pos, n, b, L.cap, at<int>(ws, L.nbr),
                                                 at<int>(ws, L.cnt), ra.reg, ra.nreg, ra.lam,
                                                 flags, core, at<uint8_t>(ws, L.cand));
    }
    // without seeded regions the row kernel has done the buffer test on
    // every call (rebuilt rows or kept ones)
    if (n == 0 || !seeded)
        return;
    uint8_t *cand = at<uint8_t>(ws, L.cand);
    if (mode == MLMIX_MODE_MIXED) {
        if (L.nseg > 0)
            k_buffer<true><<<(n + 3) / 4, 256, 0, s>>>(pos, n, b, L.cap, at<int>(ws, L.nbr),
                                                       at<int>(ws, L.cnt), r_buffer * r_buffer,
                                                       flags, cand, seg_args(ws, L));
        else
            k_buffer<false><<<(n + 3) / 4, 256, 0, s>>>(pos, n, b, L.cap, at<int>(ws, L.nbr),
                                                        at<int>(ws, L.cnt), r_buffer * r_buffer,
                                                        flags, cand, seg_args(ws, L));
    }
}

// ------------------------------------------------------------ compaction

// Systems of at most this many scan tiles (2048 atoms each) compact in one
// pass.
constexpr int kCmpDirect = 32;

__global__ void __launch_bounds__(256) k_cmp_blocksum(const uint8_t *__restrict__ flags, int n,
                                                      int *__restrict__ partS,
                                                      int *__restrict__ partM)
{
    __shared__ int sh[4];
    int base = blockIdx.x * kScanTile + threadIdx.x * kPer;
    int s = 0, m = 0;
    for (int k = 0; k < kPer; ++k)
        if (base + k < n) {
            uint8_t f = flags[base + k];
            s += (f & 5) ? 1 : 0;
            m += (f & 1) ? 1 : 0;
        }
    int ts, tm;
    block_excl_scan(s, sh, ts);
    block_excl_scan(m, sh, tm);
    if (threadIdx.x == 0) {
        partS[blockIdx.x] = ts;
        partM[blockIdx.x] = tm;
    }
}

// Second pass: each block adds the block totals before it (a fixed-order
// reduction, so no third launch is needed) and writes its part of S and M;
// the last block also publishes |S| and |M|.
__global__ void __launch_bounds__(256) k_cmp_apply(const uint8_t *__restrict__ flags, int n,
                                                   const int *__restrict__ partS,
                                                   const int *__restrict__ partM, int *hdr,
                                                   int32_t *n_expensive, int *__restrict__ S_idx,
                                                   int *__restrict__ M_idx,
                                                   int *__restrict__ S_local, int direct,
                                                   int scap)
{
    __shared__ int sh[4];
    __shared__ int offs[2];
    // offsets of this block: sums of partS/partM over the blocks before it,
    // or (small systems, no first pass) counts of their flags
    int os = 0, om = 0;
    if (direct) {
        const int lim = (int)blockIdx.x * kScanTile;  // a multiple of 2048
        if ((reinterpret_cast<uintptr_t>(flags) & 3) == 0) {
            // four flags per load, eight loads in flight per thread
            const uint32_t *fw = reinterpret_cast<const uint32_t *>(flags);
            for (int w0 = 0; w0 < lim / 4; w0 += 8 * 256) {
                uint32_t v[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int e = w0 + k * 256 + (int)threadIdx.x;
                    v[k] = e < lim / 4 ? fw[e] : 0u;
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const uint32_t f = (v[k] >> (8 * q)) & 0xffu;
                        os += (f & 5u) ? 1 : 0;
                        om += (f & 1u) ? 1 : 0;
                    }
                }
            }
        } else {
            for (int e0 = 0; e0 < lim; e0 += 8 * 256) {
                uint8_t v[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int e = e0 + k * 256 + (int)threadIdx.x;
                    v[k] = e < lim ? flags[e] : (uint8_t)0;
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    os += (v[k] & 5) ? 1 : 0;
                    om += (v[k] & 1) ? 1 : 0;
                }
            }
        }
    } else {
        for (int b = threadIdx.x; b < (int)blockIdx.x; b += 256) {
            os += partS[b];
            om += partM[b];
        }
    }
    int ts, tm;
    block_excl_scan(os, sh, ts);
    block_excl_scan(om, sh, tm);
    if (threadIdx.x == 0) {
        offs[0] = ts;
        offs[1] = tm;
    }
    __syncthreads();
    int base = blockIdx.x * kScanTile + threadIdx.x * kPer;
    uint8_t f[kPer];
    int s = 0, m = 0;
    for (int k = 0; k < kPer; ++k) {
        f[k] = (base + k < n) ? flags[base + k] : 0;
        s += (f[k] & 5) ? 1 : 0;
        m += (f[k] & 1) ? 1 : 0;
    }
    int bs, bm;
    int es = block_excl_scan(s, sh, bs) + offs[0];
    int em = block_excl_scan(m, sh, bm) + offs[1];
    for (int k = 0; k < kPer; ++k) {
        int i = base + k;
        if (i >= n)
            break;
        if (f[k] & 5) {
            // atoms past the S capacity get no rows of the per-S buffers: the
            // evaluation is then incomplete, which the status bit reports
            S_idx[es] = i;
            S_local[i] = es < scap ? es : -1;
            es++;
        } else {
            S_local[i] = -1;
        }
        if (f[k] & 1) {
            M_idx[em] = i;
            em++;
        }
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        const int nS = offs[0] + bs;
        hdr[H_NS] = nS < scap ? nS : scap;
        if (nS > scap)
            atomicOr(&hdr[H_STATUS], MLMIX_STATUS_S_OVERFLOW);
        hdr[H_NM] = offs[1] + bm;
        if (n_expensive) {
            n_expensive[0] = offs[0] + bs;
            n_expensive[1] = offs[1] + bm;
        }
    }
}

// Small systems (at most kCmpSmallBlocks blocks of 256 atoms): one atom per
// thread and one launch with one round of loads. Each block counts the flags
// before it (at most 16 words of four flags per thread, all issued at once)
// and ranks its own atoms by wave ballots; the same S, M and counts as the
// tiled passes.
constexpr int kCmpSmallBlocks = 64;

__global__ void __launch_bounds__(256) k_cmp_small(const uint8_t *__restrict__ flags, int n,
                                                   int *hdr, int32_t *n_expensive,
                                                   int *__restrict__ S_idx,
                                                   int *__restrict__ M_idx,
                                                   int *__restrict__ S_local, int scap)
{
    __shared__ int cS[4], cM[4], bS[4], bM[4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int i = (int)blockIdx.x * 256 + tid;
    const uint8_t f = i < n ? flags[i] : (uint8_t)0;
    const int lim = (int)blockIdx.x * 256;  // flags before this block
    int os = 0, om = 0;
    if ((reinterpret_cast<uintptr_t>(flags) & 3) == 0) {
        const uint32_t *fw = reinterpret_cast<const uint32_t *>(flags);
        uint32_t v[kCmpSmallBlocks / 4];
#pragma unroll
        for (int k = 0; k < kCmpSmallBlocks / 4; ++k) {
            const int e = k * 256 + tid;
            v[k] = e < lim / 4 ? fw[e] : 0u;
        }
#pragma unroll
        for (int k = 0; k < kCmpSmallBlocks / 4; ++k)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t b = (v[k] >> (8 * q)) & 0xffu;
                os += (b & 5u) ? 1 : 0;
                om += (b & 1u) ? 1 : 0;
            }
    } else {
        for (int e = tid; e < lim; e += 256) {
            const uint8_t b = flags[e];
            os += (b & 5) ? 1 : 0;
            om += (b & 1) ? 1 : 0;
        }
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        os += __shfl_xor(os, d);
        om += __shfl_xor(om, d);
    }
    const bool inS = (f & 5) != 0, inM = (f & 1) != 0;
    const unsigned long long mS = __ballot(inS), mM = __ballot(inM);
    const unsigned long long lt = (1ull << lane) - 1ull;
    if (lane == 0) {
        cS[w] = __popcll(mS);
        cM[w] = __popcll(mM);
        bS[w] = os;
        bM[w] = om;
    }
    __syncthreads();
    int es = __popcll(mS & lt), em = __popcll(mM & lt), tS = 0, tM = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        es += bS[k] + (k < w ? cS[k] : 0);
        em += bM[k] + (k < w ? cM[k] : 0);
        tS += bS[k] + cS[k];
        tM += bM[k] + cM[k];
    }
    if (i < n) {
        if (inS) {
            S_idx[es] = i;
            S_local[i] = es < scap ? es : -1;
        } else {
            S_local[i] = -1;
        }
        if (inM)
            M_idx[em] = i;
    }
    if (blockIdx.x == gridDim.x - 1 && tid == 0) {
        hdr[H_NS] = tS < scap ? tS : scap;
        if (tS > scap)
            atomicOr(&hdr[H_STATUS], MLMIX_STATUS_S_OVERFLOW);
        hdr[H_NM] = tM;
        if (n_expensive) {
            n_expensive[0] = tS;
            n_expensive[1] = tM;
        }
    }
}

void launch_compact(hipStream_t s, void *ws, const WsLayout &L, uint8_t *flags,
                    int32_t *n_expensive)
{
    int n = L.n;
    if (n <= kCmpSmallBlocks * 256) {
        const int nb = n > 0 ? (n + 255) / 256 : 1;
        k_cmp_small<<<nb, 256, 0, s>>>(flags, n, at<int>(ws, L.hdr), n_expensive,
                                       at<int>(ws, L.S_idx), at<int>(ws, L.M_idx),
                                       at<int>(ws, L.S_local), L.scap);
        return;
    }
    int nb = (n + kScanTile - 1) / kScanTile;
    if (nb < 1)
        nb = 1;
    int *partS = at<int>(ws, L.scan_part);
    int *partM = partS + nb;
    // up to kCmpDirect tiles: one pass, each block counts the flags before it
    const int direct = nb <= kCmpDirect ? 1 : 0;
    if (!direct)
        k_cmp_blocksum<<<nb, 256, 0, s>>>(flags, n, partS, partM);
    k_cmp_apply<<<nb, 256, 0, s>>>(flags, n, partS, partM, at<int>(ws, L.hdr), n_expensive,
                                   at<int>(ws, L.S_idx), at<int>(ws, L.M_idx),
                                   at<int>(ws, L.S_local), direct, L.scap);
}

}  // namespace mlmix
