/*
 * mlmix.h — C ABI of the MI355X (gfx950) library for the spatially mixed
 * force evaluation of ML-MIX (Birks et al., arXiv 2502.19081).
 *
 * One call evaluates, on one HIP stream and without a host synchronisation:
 *   cell-list neighbour search (the neighbour lists the paper's region fix
 *   reuses; Methods, "Region tracking"),
 *   the mixing weight lambda_i and masks (Algorithms 1-2, with geometric
 *   core regions; lambda = max over regions as in Algorithm 2),
 *   the buffer set (Algorithm 3 and the buffer-set equation of "Spatial
 *   potential mixing"), stream compaction of S = {lambda > 0} + buffer,
 *   the expensive ACE-style potential on the induced subsystem S only
 *   (Algorithm 4 and Fig. 10) with its hand-written adjoint forces
 *   (forces = minus the derivative of the summed site energies, the
 *   force/site-energy equation of "Spatial potential mixing"),
 *   the cheap UF3-style 2+3-body potential on every atom, and the blend
 *   F_i = lambda_i F_exp,i + (1 - lambda_i) F_cheap,i (Algorithm 4).
 *
 * Conventions shared by every entry point
 *  - Units: Angstrom, eV, amu, fs.
 *  - Device pointers: every array argument marked [dev] is device memory
 *    owned by the caller; the library reads inputs and writes outputs and
 *    keeps no reference after the call returns (work is enqueued on
 *    `stream`, so the arrays must stay alive until the stream reaches it).
 *  - Layout: per-atom 3-vectors are SoA, 3 x n doubles: x[0..n), y[0..n),
 *    z[0..n).
 *  - stream: a hipStream_t cast to void* (NULL = the null stream).
 *  - Workspace: caller-owned device memory of at least
 *    mlmix_workspace_size() bytes, cleared once by mlmix_workspace_init().
 *    It holds the neighbour list and every intermediate; one workspace per
 *    independent system (replica). The library allocates no device memory
 *    except the model tables at mlmix_create().
 *  - Return value: MLMIX_OK or a negative MLMIX_E_* code for errors detected
 *    on the host (argument checks). Conditions found on the device
 *    (neighbour overflow, atom outside a non-periodic box, non-finite
 *    input) are recorded in the workspace and reported by mlmix_status().
 *    Nothing aborts or throws across the ABI; mlmix_last_error() gives a
 *    thread-local message for the last failing call.
 */
#ifndef MLMIX_H
#define MLMIX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MLMIX_OK 0
#define MLMIX_E_ARG (-1)
#define MLMIX_E_HIP (-2)
#define MLMIX_E_WORKSPACE (-3)
#define MLMIX_E_NEIGH_OVERFLOW (-4)
#define MLMIX_E_BOX (-5)
#define MLMIX_E_NONFINITE (-6)
#define MLMIX_E_STATE (-7)
#define MLMIX_E_HOST (-8) /* host-side failure inside the library (host memory exhausted) */

/* Arithmetic of the two potentials. Positions, lambda, the blend, energy
 * sums and the integrator are FP64 in every mode. The two reduced-precision
 * modes compute in FP32 except the dense stage of the order-3 product-basis
 * contraction (the coupled products P of two atomic-basis blocks against the
 * weights), whose operands are rounded to BF16 or scaled to FP8 with FP32
 * accumulation on the matrix cores. FP8 is OCP E4M3 with two kinds of
 * scale, neither shared across atoms: each row of P (one atom, one
 * (l1, l2, l3) block, one m3) is divided by its own largest magnitude / 240
 * (by the bound sum|Gaunt| x max_m1|A_l1| x max_m2|A_l2| / 240 in the
 * matrix-core sparse form, used when a model's rows do not fit the default
 * vector form), and each output channel c of a block's weights by
 * max|W(., c)| / 240; each row's product is multiplied back by both scales
 * in FP32 after its accumulation, before it joins the FP32 sum over the
 * rows that share an output (l3, m3). The BF16 mode takes models of at most
 * 32 channels (species x radial functions) of correlation order 3, the FP8
 * mode single-species models of at most 16; mlmix_create returns MLMIX_E_ARG
 * for other models in these modes. */
#define MLMIX_FP64 0
#define MLMIX_FP32 1
#define MLMIX_BF16_CONTRACT 2
#define MLMIX_FP8_CONTRACT 3

/* Evaluation modes (low byte) and flags. */
#define MLMIX_MODE_MIXED 0          /* lambda from regions, S = {lambda>0} + buffer */
#define MLMIX_MODE_ALL_EXPENSIVE 1  /* lambda = 1, S = every atom, cheap skipped */
#define MLMIX_MODE_ALL_CHEAP 2      /* lambda = 0, S empty, expensive skipped */
#define MLMIX_FORCE_REBUILD 0x100u  /* rebuild the neighbour list now */
#define MLMIX_ENERGY_ONLY 0x200u    /* stop after the expensive site energies */
/* Run every stage on the caller's stream (no fork onto the workspace's
 * second stream). For callers that already overlap several evaluations on
 * streams of their own, in particular inside a graph capture whose streams
 * are themselves forked off the capture's origin stream: such a capture
 * with the library's fork nested inside ended in a crash of the runtime's
 * capture end, so this path keeps such captures one level deep. */
#define MLMIX_SINGLE_STREAM 0x400u
/* The regions may include seeded regions (MLMIX_REGION_SEEDED); `flags` is
 * then also an input: seed atoms carry MLMIX_FLAG_SEED, which every
 * evaluation leaves set. The buffer then comes from its own pass after the
 * seeded core and blend passes (two more neighbour-row kernels). */
#define MLMIX_SEEDED 0x800u
#define MLMIX_FLAG_SEED 0x80u
/* Mask the cheap potential as Algorithm 4 masks each potential in turn: it
 * sees only its own subsystem S_c = {lambda < 1} plus its buffer (atoms with
 * lambda == 1 strictly closer than r_buffer to an atom with lambda < 1;
 * flags bit3). Atoms outside S_c are neither centres nor neighbours of the
 * cheap potential (e_cheap and f_cheap are 0 there). Without this flag the
 * cheap potential runs on every atom with the full lists. MIXED mode only. */
#define MLMIX_CHEAP_MASKED 0x1000u

/* Device status bits reported by mlmix_status(). */
#define MLMIX_STATUS_NEIGH_OVERFLOW 1
#define MLMIX_STATUS_OUT_OF_BOX 2
#define MLMIX_STATUS_NONFINITE 4
#define MLMIX_STATUS_TRIPLET_OVERFLOW 8
#define MLMIX_STATUS_BAD_SPECIES 16
#define MLMIX_STATUS_SEEDED_REGIONS 64 /* more than 8 seeded regions */
#define MLMIX_STATUS_CELL_OVERFLOW 32 /* a cell held more atoms than its bucket
                                         (4 x the mean occupancy + 8) */
#define MLMIX_STATUS_S_OVERFLOW 128   /* |S| exceeded the workspace's S capacity */

/* Model description (host memory; copied by mlmix_create).
 *
 * Expensive ACE-style model (a synthetic stand-in: the paper cites ACE but
 * does not define it). For a centre atom i of species z_i and neighbours j
 * in S closer than ace_rcut:
 *   R_n(r) = T_n(2r/rc - 1) (1 - (r/rc)^2)^2, n < ace_n_rad (Chebyshev T_n)
 *   A_{a,l,m} = sum_j R_n(r_ij) Y_lm(r_ij/|r_ij|), a = z_j*n_rad + n,
 *   Y_lm real orthonormal spherical harmonics, l <= ace_lmax;
 *   E_i = c0[z] + sum_a c1[z][a] A_{a00}
 *       + sum_{l, a<=b} c2[z][l][a][b] sum_m A_{alm} A_{blm}            (order>=2)
 *       + sum_{p<=q<=r} c3[z][p][q][r] sum_m G A_{p,m1} A_{q,m2} A_{r,m3} (order 3)
 *   with p = a*(lmax+1)+l, G the real Gaunt coefficients, and only l-triples
 *   of even sum that satisfy the triangle rule.
 *   Arrays (row-major doubles): c0[ns], c1[ns][nchan], c2[ns][lmax+1][nchan]
 *   [nchan], c3[ns][K][K][K] with nchan = ns*n_rad, K = nchan*(lmax+1);
 *   entries outside a<=b resp. p<=q<=r are ignored; c3 may be NULL when
 *   order < 3.
 * Cheap UF3-style model: clamped uniform cubic B-splines, n_knots points on
 *   [0, rcut] (n_knots + 2 basis functions).
 *   E_i = 1/2 sum_j V2^{z_i z_j}(r_ij) + sum_{j<k} V3^{z_i}(r_ij, r_ik, r_jk),
 *   c2[ns][ns][n_knots2+2] (must be symmetric in the species pair),
 *   c3[ns][nb][nb][nb] (nb = n_knots3+2; the r_jk axis spans [0, 2 rcut3];
 *   must be symmetric in its first two basis indices); n_knots3 = 0 turns
 *   the 3-body term off (c3 may then be NULL). */
typedef struct {
    int32_t n_species;
    int32_t precision; /* MLMIX_FP64, MLMIX_FP32, MLMIX_BF16_CONTRACT, MLMIX_FP8_CONTRACT */
    double skin;       /* neighbour-list skin; list radius = max cutoff + skin */
    int32_t ace_n_rad, ace_lmax, ace_order, ace_pad;
    double ace_rcut;
    const double *ace_c0, *ace_c1, *ace_c2, *ace_c3;
    int32_t uf3_n_knots2, uf3_n_knots3;
    double uf3_rcut2, uf3_rcut3;
    const double *uf3_c2, *uf3_c3;
} mlmix_model_desc;

/* Orthorhombic box [0, L) per dimension. Periodic dimensions need
 * L >= 2 * list radius; positions must already be wrapped into [0, L)
 * there. Along non-periodic dimensions atoms must stay inside [0, L). */
typedef struct {
    double L[3];
    int32_t periodic[3];
    int32_t pad;
} mlmix_box;

/* Core region (device array of these, 56 bytes each).
 * type 0 (MLMIX_REGION_SPHERE): sphere about `center`; type 1
 * (MLMIX_REGION_CYLINDER): infinite cylinder along coordinate axis `axis`
 * through `center`. follow_atom >= 0 replaces the centre by that atom's
 * current position. lambda = 1 for d < r_core, b(t) with
 * t = (d - r_core)/r_blend for r_core <= d < r_core + r_blend, else 0.
 * type 2 (MLMIX_REGION_SEEDED, needs MLMIX_SEEDED): the paper's region fix
 * (Algorithms 1-2) over the neighbour list: seed atoms (flag bit
 * MLMIX_FLAG_SEED set on input) and their neighbours closer than r_core are
 * core atoms (lambda 1); a neighbour j of a core atom i at distance
 * r < r_blend gets lambda_j = max(lambda_j, b(r / r_blend)). center, axis and
 * follow_atom are ignored; at most 8 seeded regions, all sharing the seeds;
 * r_core and r_blend should not exceed the list radius.
 * blend: MLMIX_BLEND_LINEAR b(t) = 1 - t (Algorithm 2) or MLMIX_BLEND_CUBIC
 * b(t) = 1 - 3t^2 + 2t^3 (zero slope at both ends).
 * The atom's lambda is the maximum over regions. */
typedef struct {
    int32_t type;
    int32_t axis;
    int32_t follow_atom;
    int32_t blend;
    double center[3];
    double r_core;
    double r_blend;
} mlmix_region;

#define MLMIX_REGION_SPHERE 0
#define MLMIX_REGION_CYLINDER 1
#define MLMIX_REGION_SEEDED 2
#define MLMIX_BLEND_LINEAR 0
#define MLMIX_BLEND_CUBIC 1

typedef struct mlmix_ctx mlmix_ctx;

/* Builds the model tables on the current HIP device. Returns MLMIX_E_ARG for
 * inconsistent sizes (n_rad 1..16, lmax 0..6, order 1..3, knots >= 4) or
 * non-symmetric cheap coefficients. */
int mlmix_create(const mlmix_model_desc *desc, mlmix_ctx **out);
int mlmix_destroy(mlmix_ctx *ctx);

/* List radius (max cutoff + skin) of the model. */
double mlmix_list_radius(const mlmix_ctx *ctx);

/* Bytes of workspace for n_atoms atoms, a neighbour-row capacity of nbr_cap
 * (1..256), an S capacity s_cap and the given box (the cell grid depends on
 * it). s_cap bounds |S| (the expensive atoms plus their buffer): the
 * buffers of the expensive potential (atomic basis, dE/dA, pair gradients,
 * the order-3 partial sums: about 4 nbr_cap x 3 + 20 K bytes per S row in
 * FP32 for the workloads here) are sized for s_cap rows instead of n_atoms.
 * s_cap <= 0 or > n_atoms means n_atoms (required for MLMIX_MODE_ALL_EXPENSIVE,
 * where S is every atom). An evaluation whose S exceeds s_cap leaves the
 * atoms past the capacity out of S and raises MLMIX_STATUS_S_OVERFLOW
 * (mlmix_status returns MLMIX_E_WORKSPACE; n_expensive[0] holds the |S| that
 * was needed). */
int mlmix_workspace_size(const mlmix_ctx *ctx, int32_t n_atoms, int32_t nbr_cap, int32_t s_cap,
                         const mlmix_box *box, size_t *bytes);

/* Clears the workspace header (status, neighbour-list state) on `stream`.
 * Must be called once before the first mlmix_compute on a workspace and
 * again whenever n_atoms, nbr_cap, s_cap or the box size changes (the same
 * n_atoms, nbr_cap, s_cap and box as mlmix_workspace_size).
 * Second stream: an evaluation without MLMIX_SINGLE_STREAM forks the reverse
 * slots and the cheap potential onto the workspace's second stream and joins
 * back on the caller's stream before returning, so calls stay ordered on
 * `stream` and capturable in a HIP graph. The first such evaluation outside
 * a graph capture creates that stream (default priority, owned by the
 * context, destroyed by mlmix_destroy); until then evaluations run on the
 * caller's stream alone. Calls on one workspace must not overlap. */
int mlmix_workspace_init(mlmix_ctx *ctx, void *stream, void *ws, size_t ws_bytes,
                         int32_t n_atoms, int32_t nbr_cap, int32_t s_cap, const mlmix_box *box);

/* The mixed force evaluation.
 *  pos [dev] 3 x n double (SoA), species [dev] int32[n] in [0, n_species),
 *  regions [dev] mlmix_region[n_regions] (ignored unless mode is MIXED),
 *  r_buffer: buffer radius (Algorithm 3), 0 <= r_buffer <= list radius.
 * Outputs [dev]: forces 3 x n double (blended; may be NULL with
 *  MLMIX_ENERGY_ONLY), e_exp[n] (expensive site energies on S, 0 elsewhere),
 *  e_cheap[n] (cheap site energies, 0 in ALL_EXPENSIVE mode), lambda[n],
 *  flags[n] (bit0 lambda>0, bit1 lambda==1, bit2 buffer, bit3 cheap buffer
 *  with MLMIX_CHEAP_MASKED, bit7 seed as passed in), n_expensive
 *  int32[2] (|S|, |{lambda>0}|). f_exp and f_cheap (3 x n double) are
 *  optional (NULL) copies of the two unblended force fields.
 * The neighbour list is rebuilt when MLMIX_FORCE_REBUILD is set, on the first
 * call after mlmix_workspace_init, or when an atom moved more than skin/2
 * since the last rebuild (decided on the device). An empty system (n_atoms
 * = 0) may pass NULL per-atom arrays; only n_expensive is written (zeros),
 * and mlmix_vv_step / mlmix_vv_steps write zero energy sums. */
int mlmix_compute(mlmix_ctx *ctx, void *stream, void *ws, int32_t n_atoms,
                  const double *pos, const int32_t *species, const mlmix_box *box,
                  const mlmix_region *regions, int32_t n_regions, double r_buffer,
                  uint32_t mode, double *forces, double *e_exp, double *e_cheap,
                  double *lambda, uint8_t *flags, int32_t *n_expensive,
                  double *f_exp, double *f_cheap);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the mixed
 * force evaluation of mlmix_compute without a caller workspace. Its
 * workspace is a static device array of the library,
 * MLMIX_NOALLOC_SCRATCH_BYTES per GPU (each GPU the library runs on holds
 * its copy until the process ends; the device address is looked up by
 * mlmix_create on that device). The call allocates nothing (no hipMalloc,
 * no stream or event creation): every stage runs on `stream`, the neighbour
 * list is rebuilt on each call (the scratch keeps the last call's contents,
 * so the header and cell counts are cleared first by fill kernels), and no
 * stage timing is recorded. nbr_cap and s_cap as for mlmix_workspace_size;
 * status [dev] int32[2] (may be NULL) receives this call's MLMIX_STATUS_*
 * bits and largest neighbour count (as mlmix_status reports them for a
 * workspace; read it after the stream reaches the call); *bytes_used [host]
 * (may be NULL) receives the scratch bytes this system needs. Arguments and
 * outputs otherwise as mlmix_compute (without f_exp / f_cheap;
 * MLMIX_ENERGY_ONLY is refused). The results equal mlmix_compute's with
 * MLMIX_FORCE_REBUILD on a workspace of the same nbr_cap and s_cap bit for
 * bit. Calls that overlap on one GPU (other streams, other threads, other
 * contexts) share the scratch and race: the caller serialises them.
 * Errors: those of mlmix_compute, and MLMIX_E_WORKSPACE when the system
 * needs more than MLMIX_NOALLOC_SCRATCH_BYTES (lower s_cap or nbr_cap). */
#define MLMIX_NOALLOC_SCRATCH_BYTES (64u << 20)
int mlmix_compute_noalloc(mlmix_ctx *ctx, void *stream, int32_t n_atoms, int32_t nbr_cap,
                          int32_t s_cap, const double *pos, const int32_t *species,
                          const mlmix_box *box, const mlmix_region *regions, int32_t n_regions,
                          double r_buffer, uint32_t mode, double *forces, double *e_exp,
                          double *e_cheap, double *lambda, uint8_t *flags,
                          int32_t *n_expensive, int32_t *status, size_t *bytes_used);

/* Adjoint of the expensive site energies: grad_pos = d(sum_i w_i E_i)/dx
 * (3 x n double [dev]) for weights w = grad_e [dev] double[n], using S, the
 * neighbour list and dE/dA from the last mlmix_compute on this workspace
 * (the per-neighbour basis is recomputed, not stored). */
int mlmix_backward(mlmix_ctx *ctx, void *stream, void *ws, int32_t n_atoms,
                   const double *pos, const int32_t *species, const mlmix_box *box,
                   const double *grad_e, double *grad_pos);

/* One velocity-Verlet step (FP64): v += dt/2 kappa F/m; x += dt v; wrap;
 * F = mlmix_compute(x); v += dt/2 kappa F/m. `forces` must hold F(x) on
 * entry and holds the new forces on return. mass [dev] double[n] (amu),
 * dt in fs, kappa = 9.648533212e-3 A fs^-2 per eV A^-1 amu^-1.
 * energies [dev] double[3] receives (sum e_exp, sum e_cheap, kinetic) of
 * the new state (may be NULL). Other arguments as in mlmix_compute. */
int mlmix_vv_step(mlmix_ctx *ctx, void *stream, void *ws, int32_t n_atoms, double *pos,
                  double *vel, const double *mass, const int32_t *species, double dt,
                  const mlmix_box *box, const mlmix_region *regions, int32_t n_regions,
                  double r_buffer, uint32_t mode, double *forces, double *e_exp,
                  double *e_cheap, double *lambda, uint8_t *flags, int32_t *n_expensive,
                  double *energies);

/* n_steps velocity-Verlet steps in one call, each exactly as mlmix_vv_step
 * (same results bit for bit); energies [dev] double[n_steps][3] receives the
 * sums of every step (required). Up to 65,536 atoms the steps are fused: the
 * force gather of a step also applies the next step's opening half kick and
 * drift, and the next step's binning kernel sums the previous step's
 * energies, so a step launches two kernels fewer. With a thermostat set
 * (mlmix_set_langevin) only n_steps = 1 is accepted (each step needs fresh
 * normals): MLMIX_E_STATE otherwise. Other errors as for mlmix_vv_step. */
int mlmix_vv_steps(mlmix_ctx *ctx, void *stream, void *ws, int32_t n_atoms, double *pos,
                   double *vel, const double *mass, const int32_t *species, double dt,
                   int32_t n_steps, const mlmix_box *box, const mlmix_region *regions,
                   int32_t n_regions, double r_buffer, uint32_t mode, double *forces,
                   double *e_exp, double *e_cheap, double *lambda, uint8_t *flags,
                   int32_t *n_expensive, double *energies);

/* Langevin thermostat on the cheap region for mlmix_vv_step on workspace ws
 * (Methods, "Si stretched bond" and "Diffusion coefficients": a weak
 * thermostat, time constant 2 ps, acting only where the cheap potential
 * alone gives the force, to hold the temperature against the drift that
 * force mixing causes, Discussion). Every atom with lambda == 0 at the step's
 * force call gets, added to its blended force,
 *     F_L = -m v / (kappa tau) + sqrt(2 m kB T / (kappa tau dt)) xi,
 * with v its half-step velocity (after the opening half kick), kB =
 * 8.617333262e-5 eV/K, kappa as below, and xi the three standard normals of
 * that atom in xi [dev] double[3][n] (caller-owned; the step reads it, so the
 * caller refills it before each step, also under graph capture). F_L is part
 * of `forces` on return, and the closing half kick and the next step's
 * opening kick use it. temperature_K >= 0; damping_fs = tau in fs, <= 0
 * turns the thermostat off (xi may then be NULL). The setting lives with the
 * workspace until changed; mlmix_workspace_init with another n_atoms drops
 * it. mlmix_compute ignores it. Errors: MLMIX_E_ARG (NULL ctx/ws, xi NULL
 * with tau > 0, negative or non-finite T, n_atoms not the workspace's),
 * MLMIX_E_STATE (workspace not initialised). */
int mlmix_set_langevin(mlmix_ctx *ctx, void *ws, int32_t n_atoms, double temperature_K,
                       double damping_fs, const double *xi);

/* FP64 sums (sum e_exp, sum e_cheap, kinetic energy from vel and mass; vel
 * and mass may be NULL, kinetic is then 0) into energies [dev] double[3]. */
int mlmix_energy_reduce(mlmix_ctx *ctx, void *stream, void *ws, int32_t n_atoms,
                        const double *e_exp, const double *e_cheap, const double *vel,
                        const double *mass, double *energies);

/* ---------------------------------------------------------------------
 * Batched systems: several independent systems (MD replicas) sharing one
 * model, evaluated and integrated together, one launch per kernel for the
 * whole batch (the serving workload). The systems' atoms sit side by side
 * in the batch arrays (SoA over all n_atoms of the batch: x of every atom,
 * then y, then z); a segment table gives each system its range, box and
 * regions. Every kernel takes its atom's box, cell grid and regions from the
 * table, neighbour rows never cross systems, and each system's results are
 * the same bits alone and in any batch (launch shapes that change the
 * rounding do not depend on the batch's size or composition). Each system
 * keeps or rebuilds its own neighbour list (its list is rebuilt when one of
 * its atoms moved more than skin/2 since its last build, or on a forced
 * rebuild, which applies to all); the systems share dt, r_buffer and the
 * mode; seeded regions and MLMIX_ENERGY_ONLY are not available. */
typedef struct {
    int32_t offset;        /* first atom of the system in the batch arrays (the
                              segments tile [0, n_atoms) in order) */
    int32_t n_atoms;       /* >= 1 */
    mlmix_box box;         /* the system's box, as for a single system */
    int32_t region_offset; /* its regions are regions[region_offset ..
                              region_offset + n_regions) of the call's array;
                              follow_atom counts from the system's first atom */
    int32_t n_regions;
} mlmix_segment;

/* Bytes of a batch workspace for the segment table segs [host] (n_segments
 * entries), a neighbour-row capacity nbr_cap and an S capacity s_cap for
 * the whole batch (as for mlmix_workspace_size; 0 = every atom). */
int mlmix_batch_workspace_size(const mlmix_ctx *ctx, int32_t n_segments,
                               const mlmix_segment *segs, int32_t nbr_cap, int32_t s_cap,
                               size_t *bytes);

/* Prepares a batch workspace for the segment table segs [host]: clears its
 * header, copies the table to the device (waits for `stream` once: call it
 * outside graph capture) and tags every atom with its segment. Call it again
 * whenever the set of systems changes; the next call rebuilds every list.
 * Errors: MLMIX_E_ARG (segments not tiling [0, n) in order, an empty
 * segment, sizes), MLMIX_E_BOX, MLMIX_E_WORKSPACE. */
int mlmix_batch_init(mlmix_ctx *ctx, void *stream, void *ws, size_t ws_bytes, int32_t n_segments,
                     const mlmix_segment *segs, int32_t nbr_cap, int32_t s_cap);

/* The mixed force evaluation of every system of the batch, as mlmix_compute
 * per system: n_atoms = the batch's total, per-atom arrays over the batch,
 * regions [dev] mlmix_region[n_regions] holding every segment's range.
 * n_expensive [dev] int32[n_segments][2] (may be NULL) receives each
 * system's |S| and |{lambda > 0}|; energies [dev] double[n_segments][3] (may
 * be NULL) each system's (sum e_exp, sum e_cheap, 0). */
int mlmix_batch_compute(mlmix_ctx *ctx, void *stream, void *ws, int32_t n_atoms,
                        const double *pos, const int32_t *species, const mlmix_region *regions,
                        int32_t n_regions, double r_buffer, uint32_t mode, double *forces,
                        double *e_exp, double *e_cheap, double *lambda, uint8_t *flags,
                        int32_t *n_expensive, double *energies);

/* n_steps velocity-Verlet steps of every system of the batch, each step as
 * mlmix_vv_step per system (the same bits as that system's own
 * mlmix_vv_steps up to the energy sums' summation order, which here is per
 * system and fixed): one launch per kernel per step for the whole batch.
 * energies [dev] double[n_steps][n_segments][3] receives each system's
 * (sum e_exp, sum e_cheap, kinetic) after every step; n_expensive [dev]
 * int32[n_segments][2] (may be NULL) the set sizes of the last step. A
 * thermostat set with mlmix_set_langevin does not apply here. */
int mlmix_batch_vv_steps(mlmix_ctx *ctx, void *stream, void *ws, int32_t n_atoms, double *pos,
                         double *vel, const double *mass, const int32_t *species, double dt,
                         int32_t n_steps, const mlmix_region *regions, int32_t n_regions,
                         double r_buffer, uint32_t mode, double *forces, double *e_exp,
                         double *e_cheap, double *lambda, uint8_t *flags, int32_t *n_expensive,
                         double *energies);

/* After mlmix_batch_init of a new batch: takes over, from the old batch
 * workspace ws_old, the neighbour-list state of the systems the new batch
 * keeps, so that each keeps or rebuilds its list as it would have in the old
 * batch (its bits then do not depend on the batch being rebuilt around it).
 * seg_map [host] int32[n_segments of ws_new]: the old segment index of each
 * new segment, or -1 for a system new to the batch (its list is built by the
 * next call). Rows, counts, reverse slots and reference positions are copied
 * (row indices moved to the new offsets) with the systems' built and moved
 * flags. Waits for `stream` (call it outside graph capture). Errors:
 * MLMIX_E_ARG (NULL, the same workspace twice, different row capacities, a
 * map entry out of range or used twice, a kept system whose atom count
 * changed), MLMIX_E_STATE (a workspace not initialised as a batch). */
int mlmix_batch_carry_lists(mlmix_ctx *ctx, void *stream, void *ws_new, const void *ws_old,
                            const int32_t *seg_map);

/* As mlmix_status for a batch workspace, and segment_bits [host]
 * int32[n_segments] (may be NULL) receives each system's own MLMIX_STATUS_*
 * bits (so that a failing replica can be evicted alone). */
int mlmix_batch_status(mlmix_ctx *ctx, void *stream, void *ws, int32_t *segment_bits,
                       int32_t *required_cap);

/* Waits for `stream`, then reads the device status word of the workspace:
 * *status_bits receives MLMIX_STATUS_* bits, *required_cap the largest
 * neighbour count of an overflowing row (0 without overflow; for regrowing
 * nbr_cap). Returns MLMIX_OK when no
 * bit is set, else the matching negative code (overflow first). */
int mlmix_status(mlmix_ctx *ctx, void *stream, void *ws, int32_t *status_bits,
                 int32_t *required_cap);

/* Waits for `stream`, then *builds [host] receives the number of neighbour-
 * list builds on the workspace since mlmix_workspace_init / mlmix_batch_init
 * (forced or triggered by the skin check; for a batch, the calls in which
 * some system's list was rebuilt). */
int mlmix_list_builds(mlmix_ctx *ctx, void *stream, void *ws, int32_t *builds);

/* Test hooks (device -> device copies, enqueued on stream): the neighbour
 * rows (int32[n][nbr_cap], ascending j, unused slots -1) and counts, and
 * the compacted index sets S and M (ascending, int32[n] each, valid up to
 * the counts written to n_expensive by mlmix_compute). */
int mlmix_get_neighbors(mlmix_ctx *ctx, void *stream, void *ws, int32_t n_atoms,
                        int32_t *nbr_out, int32_t *cnt_out);
int mlmix_get_index_sets(mlmix_ctx *ctx, void *stream, void *ws, int32_t n_atoms,
                         int32_t *S_out, int32_t *M_out);

/* Test hook, host only (no device call): the real Gaunt coefficients the
 * order-3 contraction uses, G[lm1][lm2][lm3] = integral over the unit sphere
 * of Y_lm1 Y_lm2 Y_lm3 (real orthonormal harmonics without the
 * Condon-Shortley phase, index l^2 + l + m, cosine type for m > 0), from
 * the Wigner-3j closed form. out [host] double[L2^3], L2 = (lmax + 1)^2,
 * 0 <= lmax <= 6. Errors: MLMIX_E_ARG. */
int mlmix_gaunt_table(int32_t lmax, double *out);

/* ---------------------------------------------------------------------
 * Constrained linear fitting of the cheap potential (Methods, "Constrained
 * potential fitting"). The cheap potential is linear in its free spline
 * coefficients u, so the energies and forces of a configuration are A u.
 * Free parameters, in column order: for each species pair za <= zb the
 * 2-body coefficients n < n_knots2 - 1 (the last three of n_knots2 + 2
 * vanish at the cutoff); then for each centre species z, legs p <= q <
 * n_knots3 - 1 and third side s < n_knots3 + 2 the 3-body coefficient
 * c3[z][p][q][s] = c3[z][q][p][s]. The fit is FP64 in every precision mode.
 * Soft data is matched in the least-squares sense while the hard data must
 * satisfy ||A_H u - y_H||^2 <= alpha; at a fixed multiplier lam the augmented
 * Lagrangian's minimiser solves (G_S + lam G_H + ridge I) u = b_S + lam b_H
 * with G = A^T W A, b = A^T W y (W = diag(w); G_H, b_H with unit weights). */

/* Number of free parameters of the context's cheap potential. */
int mlmix_fit_n_params(mlmix_ctx *ctx, int32_t *n_params);

/* Design rows of one configuration: rows [dev] double[(1 + 3 n) x ld],
 * row-major; row 0 = d(total energy)/du, row 1 + q n + i = d(F_i,q)/du.
 * Reads the neighbour rows of the last mlmix_compute / mlmix_vv_step on ws,
 * which must have been given these positions (the call builds no list), and
 * uses the workspace's pair-gradient scratch for per-atom energy rows and
 * 3-body neighbour lists (so call mlmix_compute again before
 * mlmix_backward). Errors: MLMIX_E_ARG (NULL, ld < n_params, more than 120
 * parameters, n_atoms not the workspace's), MLMIX_E_WORKSPACE (nbr_cap too
 * small for n x (8 n_params + 260) bytes in that scratch), MLMIX_E_BOX.
 * More than 32 neighbours inside the 3-body cutoff of one atom sets
 * MLMIX_STATUS_TRIPLET_OVERFLOW (read with mlmix_status). */
int mlmix_fit_design(mlmix_ctx *ctx, void *stream, void *ws, int32_t n_atoms, const double *pos,
                     const int32_t *species, const mlmix_box *box, double *rows, int32_t ld);

/* Several configurations in one call (one set of launches over all their
 * atoms, 24 configurations per launch), each as for mlmix_fit_design; the
 * array is read on the host during the call. Each workspace may appear once.
 * Errors as for mlmix_fit_design, for the first configuration that fails
 * (nothing is launched then). */
typedef struct {
    void *ws;
    int32_t n_atoms;
    int32_t pad;
    const double *pos;      /* [dev] 3 x n_atoms */
    const int32_t *species; /* [dev] n_atoms */
    mlmix_box box;
    double *rows;           /* [dev] (1 + 3 n_atoms) x ld */
} mlmix_fit_config;
int mlmix_fit_design_batch(mlmix_ctx *ctx, void *stream, int32_t n_configs,
                           const mlmix_fit_config *configs, int32_t ld);

/* Bytes of device scratch that mlmix_fit_gram needs for n_rows rows, and
 * that mlmix_fit_constrained needs with n_rows = n_hard. */
int mlmix_fit_work_size(int64_t n_rows, int32_t n_params, size_t *bytes);

/* G += A^T diag(w) A and b += A^T diag(w) y for rows [dev] double[n_rows x
 * ld] (row-major), y, w [dev] double[n_rows] (w NULL = unit weights, y NULL
 * = zero). G [dev] double[n_params x n_params] (both triangles written) and
 * b [dev] double[n_params] are accumulated, so the caller zeroes them first
 * and may stream the rows in several calls. work [dev] holds at least
 * mlmix_fit_work_size(n_rows, n_params) bytes. Fixed summation order. */
int mlmix_fit_gram(mlmix_ctx *ctx, void *stream, const double *rows, int64_t n_rows,
                   int32_t n_params, int32_t ld, const double *y, const double *w, double *G,
                   double *b, void *work, size_t work_bytes);

/* The lambda search, all on the device: solve at lambda0, 10 lambda0, ...
 * (at most max_decades increases) until the hard residual
 * sum_h wH_h (A_H u - y_H)_h^2 <= alpha, then
 * bisect between the last failing and the first passing lambda (at most
 * max_bisect solves) until the passing end's residual lies within tol of
 * alpha (the paper's default tol is alpha / 10). GS, bS from
 * mlmix_fit_gram of the soft rows; AH [dev] double[n_hard x ld_h], yH and
 * wH [dev] double[n_hard] are the hard rows and their weights (wH NULL =
 * unit weights; 1/n^2 on total-energy rows gives per-atom errors). Outputs u [dev] double[n_params]
 * (the passing end's solution) and info [dev] double[6] = {lambda, hard
 * residual, number of solves, status, last failing lambda, decades}; status
 * 0 = converged (also when lambda0 already passes), 1 = alpha not reached
 * (the solution with the smallest residual seen is returned), 2 = bisection
 * limit, 3 = non-positive pivot in the factorisation. work holds at least
 * mlmix_fit_work_size(n_hard, n_params) bytes. Errors: MLMIX_E_ARG (NULL, sizes, alpha/tol/lambda0 not
 * positive, ridge negative, limits beyond 64 decades / 1000 solves). */
int mlmix_fit_constrained(mlmix_ctx *ctx, void *stream, int32_t n_params, const double *GS,
                          const double *bS, const double *AH, int32_t ld_h, int32_t n_hard,
                          const double *yH, const double *wH, double alpha, double tol,
                          double lambda0,
                          double ridge, int32_t max_decades, int32_t max_bisect, double *u,
                          double *info, void *work, size_t work_bytes);

/* Stage timing for benchmarks. Stages (bit i of the mask, name from
 * mlmix_profile_stage_name(i)): 0 neighbours (lambda and masks, cells,
 * rows), 1 regions (buffer), 2 compaction, 3 expensive atomic basis,
 * 4 expensive order-3 contraction, 5 expensive site energy and dE/dA
 * (orders 1-2, sum of the order-3 blocks), 6 expensive pair adjoint, 7 cheap
 * potential, 8 gather + blend, 9 integrator, 10 energy sums, 11 reverse
 * slots of a rebuilt list. Stages 7 and 11 run on the workspace's second
 * stream, beside stages 1-6.
 * mlmix_profile_enable(ctx, mask) brackets each selected stage of later
 * calls with HIP events recorded on the caller's stream (no host wait);
 * mlmix_profile_read() waits for those events and returns, per stage, the
 * summed milliseconds and the number of bracketed launches since the last
 * read (arrays of MLMIX_N_STAGES entries). */
#define MLMIX_N_STAGES 12
int mlmix_profile_enable(mlmix_ctx *ctx, uint32_t stage_mask);
int mlmix_profile_read(mlmix_ctx *ctx, double *ms, int64_t *count);
const char *mlmix_profile_stage_name(int32_t stage);

/* Benchmark hook: launches the kernels of one stage reps times, back to back
 * on `stream`, on the data the last evaluation left in ws (every replay does
 * the same work). Stage 4 (the expensive order-3 contraction) reads and
 * writes workspace arrays only (pos, box and e_out may be NULL); stage 6
 * (the expensive pair adjoint, FP32/BF16/FP8 models; with the finalisation
 * folded in where a step folds it in) also reads pos [dev] and box and
 * writes the expensive site energies of S to e_out [dev] double[n]; stage 7
 * (the cheap potential, uncapped as on one stream) reads pos and box and
 * writes the cheap site energies to e_out [dev] double[n]. Species as in
 * mlmix_compute. Timing these launches with two events gives the kernel's
 * own duration without the dispatch gap in front of it. Errors: MLMIX_E_ARG
 * (NULL, negative reps, another stage, stage 6 of an FP64 model, n_atoms not
 * the workspace's, a batch workspace), MLMIX_E_STATE (workspace not
 * initialised). */
int mlmix_profile_replay(mlmix_ctx *ctx, void *stream, void *ws, int32_t n_atoms,
                         const double *pos, const int32_t *species, const mlmix_box *box,
                         double *e_out, int32_t stage, int32_t reps);

/* Achievable-peak probe: launches `blocks` workgroups of four waves, each
 * running `iters` rounds of eight independent FP32 16x16x4 matrix-core
 * chains on register operands; *flops receives the launch's flop count (the
 * caller times the launch with events on `stream`). sink [dev] float[blocks]
 * is never written in practice (it keeps the work). */
int mlmix_probe_mfma_f32(void *stream, int32_t blocks, int32_t iters, float *sink, double *flops);

/* Operation counts of the kernels as written, for roofline reporting
 * (out[7]): [0] expensive order-3 contraction per S atom, [1] atomic basis
 * per expensive pair, [2] pair adjoint per expensive pair, [3] cheap 2-body
 * per pair, [4] cheap 3-body per unordered pair of legs, [5] the part of [0]
 * spent in the dense order-3 stage (the stage whose operands the BF16/FP8
 * modes narrow), [6] finalisation (dE/dA and site energy from A and the
 * partial D) per S atom. */
int mlmix_model_flops(const mlmix_ctx *ctx, double *out);

/* Thread-local description of the last error. */
const char *mlmix_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MLMIX_H */
