/*
 * goac.h -- C ABI of the MI355X (gfx950) library for the pairwise Coulomb
 * cluster-expansion optimiser of Koester, Binninger and Kaghazchi,
 * "Optimization of Coulomb Energies in Gigantic Configurational Spaces of
 * Multi-Element Ionic Crystals" (arXiv 2409.08808).
 *
 * Conventions shared by every entry point
 *   - Units: positions in Angstrom, charges in e, energies in eV, kT in eV.
 *   - Memory: arguments named *_host are host pointers, *_dev device pointers of
 *     the context's device. The caller owns every buffer it passes and must keep
 *     it alive until the context's stream has passed the call; the library
 *     keeps no caller pointer once a call returns. The library owns the
 *     context, problems, chain sets and their internal device memory.
 *   - Asynchrony: device work is queued on the context's stream; outputs are
 *     valid once that stream has synchronised. Argument, shape and composition
 *     errors are returned synchronously, and a rejected call changes no output.
 *     Occupations the caller passes are checked on the device (every mobile
 *     species id below n_species, the species counts of every sublattice equal
 *     to the problem's: the occupancy constraints of Eq. 2); the host waits for
 *     that check, which runs before any kernel that reads the rows.
 *     A device fault surfaces as GOAC_EHIP on a later call.
 *   - Errors: every call returns a goac_status; goac_last_error() describes the
 *     last failure on a context. Nothing is thrown across the ABI.
 *   - Threading: one context per host thread.
 *   - Layouts: matrices are row-major. An occupation is one uint8 species id per
 *     site; a population of P occupations of an n-site cell is P x n row-major.
 */
#ifndef GOAC_H
#define GOAC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GOAC_OK = 0,
    GOAC_EINVAL = -1,      /* bad argument, shape or composition                 */
    GOAC_ENOMEM = -2,      /* device allocation failed                           */
    GOAC_EHIP = -3,        /* HIP runtime error or an earlier device fault       */
    GOAC_ENOTNEUTRAL = -4, /* the cell's total charge is not zero                */
    GOAC_EINEXACT = -5,    /* a shifted charge is not exact in bfloat16          */
    GOAC_EDRIFT = -6,      /* a chain's FP32 field left its error bound (chains_export) */
    GOAC_ESTATE = -7       /* objects of different contexts, or a chain set of
                              several problems where one is required            */
} goac_status;

/* Arithmetic of energies and of the Monte Carlo field.
 *   GOAC_FP64  : FP64 field and FP64 pair matrix throughout.
 *   GOAC_MIXED : FP32 field phi with periodic FP64 re-anchoring and an exact
 *                FP64 decision fallback (Monte Carlo); bfloat16 hi+lo split of the
 *                pair matrix with FP32 accumulation on the matrix cores
 *                (energies). */
typedef enum { GOAC_FP64 = 0, GOAC_MIXED = 1 } goac_precision;

typedef struct goac_ctx goac_ctx;
typedef struct goac_problem goac_problem;
typedef struct goac_chains goac_chains;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device` using `hip_stream` (a hipStream_t, or
 * NULL for the null stream). The stream is borrowed, not owned. */
goac_status goac_ctx_create(int device, void* hip_stream, goac_ctx** out);
/* Release the context. Its memory is freed (after waiting for its stream) once
 * every problem and chain set made on it has been destroyed too, so these may be
 * destroyed before or after the context; no other call may use it afterwards, and
 * the borrowed stream must stay valid until the last of them is destroyed. */
void goac_ctx_destroy(goac_ctx* ctx);
/* Message of the last failed call on ctx; valid until the next call on ctx. */
const char* goac_last_error(const goac_ctx* ctx);
/* Block until the context's stream is idle; reports pending device errors. */
goac_status goac_ctx_synchronize(goac_ctx* ctx);

/* ---------------------------------------------------------------- Ewald (a1) */

/* Parameters of the Ewald split. A value <= 0 selects the default:
 * alpha = 5 / volume^(1/3) (1/A), rcut = 6 / alpha (A), and kmax = ceil(12 alpha
 * |a|_max / (2 pi)), the radius of the sphere of integer reciprocal indices
 * n1^2 + n2^2 + n3^2 <= kmax^2, n != 0.
 * flags: GOAC_EWALD_GENERAL sums every entry (no use of translation symmetry). */
typedef struct {
    double alpha;
    double rcut;
    int32_t kmax;
    int32_t flags;
} goac_ewald_params;

#define GOAC_EWALD_GENERAL 1

/* The periodic point-charge pair matrix (Methodology, "Cluster Expansion of
 * Coulomb Energy": Ewald summation of point charges, for which the second-order
 * expansion is exact):
 *   V_ij = k_e [ sum_{m: 0<|r+mA|<rcut} erfc(alpha|r+mA|)/|r+mA|
 *              + (4 pi/W) sum_{n != 0, |n| <= kmax} e^{-G^2/4alpha^2}/G^2 cos(G.r)
 *              - pi/(W alpha^2) ] - delta_ij k_e 2 alpha/sqrt(pi),
 * r = r_j - r_i, W the cell volume, G = n B, k_e = e/(4 pi eps0) (CODATA 2018),
 * tin-foil boundary, neutralising background kept in every entry, so that
 * E(q) = 1/2 q^T V q for any neutral q.
 * V_ij depends on r_j - r_i only: when the sites are invariant under an
 * axis-aligned grid of fractional translations (1/m0, 0, 0), (0, 1/m1, 0),
 * (0, 0, 1/m2) (every supercell of a crystal is; each m the largest found; sites
 * match when their fractional coordinates agree within 1e-10), the sums run for
 * one site per orbit of the grid and the other rows are those rows relabelled
 * (equal to the full sum up to rounding); otherwise, or with GOAC_EWALD_GENERAL,
 * every entry is summed.
 *   lattice_host : 9 doubles, rows are the lattice vectors (A)
 *   pos_host     : n x 3 Cartesian positions (A)
 *   V_dev        : n x n FP64 output, row-major, caller-owned
 * Errors: EINVAL for n <= 0, a singular lattice or NULL pointers. */
goac_status goac_build_ewald(goac_ctx* ctx, const double lattice_host[9], int64_t n,
                             const double* pos_host, const goac_ewald_params* params,
                             double* V_dev);

/* ---------------------------------------------------------------- problem */

/* Set up an optimisation problem (Eq. 2): sites with sublattice < 0 are fixed,
 * the others are mobile positions of site class `sublattice` whose species may
 * be exchanged; the species counts per sublattice in `species_host` are the
 * occupancy targets every occupation must keep.
 *   V_dev         : n x n FP64 pair matrix (device); copied, not retained
 *   sublattice_host: n int32 (-1 fixed, else 0..15)
 *   species_host  : n uint8 species ids (< n_species <= 32): fixed-site species
 *                   and the reference composition of the mobile positions
 *   charge_host   : n_species FP64 valences
 * The problem holds the mobile block V_mm in FP64, FP32 and a bfloat16 hi+lo
 * split, its diagonal, the field of the fixed ions h = V_mf q_f, their energy
 * E_ff, and for each sublattice the integer c nearest its mean charge with
 * h~ = h + V_mm c and E~ = E_ff + c^T h + 1/2 c^T V_mm c (FP64).
 * Errors: EINVAL (shapes, ids, more than 65535 mobile positions),
 * ENOTNEUTRAL if |sum q| > 1e-9. */
goac_status goac_problem_create(goac_ctx* ctx, const double* V_dev, int64_t n,
                                const int32_t* sublattice_host, const uint8_t* species_host,
                                int32_t n_species, const double* charge_host,
                                goac_problem** out);
void goac_problem_destroy(goac_problem* pb);

typedef struct {
    int64_t n;              /* sites                                          */
    int64_t M;              /* mobile positions                               */
    int32_t n_sublattices;
    int32_t n_species;
    double E_fixed;         /* E_ff                                            */
    int32_t mixed_exact;    /* 1 if every shifted charge is bfloat16-exact     */
    int32_t reserved;
} goac_problem_info;
/* Sizes of a problem and its fixed-ion energy. E_ff is derived on the device by
 * goac_problem_create, which returns without waiting for it; the first call here
 * waits for the context's stream and reads it back (later calls return the
 * stored value). Errors: EINVAL (null pointer), EHIP (the read-back failed). */
goac_status goac_problem_get_info(const goac_problem* pb, goac_problem_info* out);

/* Random valid starts (SI, "Random"): per chain c and sublattice s, the
 * canonical species sequence shuffled by Fisher-Yates with
 * m = (r (k+1)) >> 32, r the first word of Philox4x32-10 at counter
 * (k, s, chain_base + c, instance << 8 | 2), key = seed.
 *   occ_dev : C x n output (fixed sites copied from the problem). */
goac_status goac_init_occupations(goac_problem* pb, int64_t C, uint64_t seed, uint32_t chain_base,
                                  uint32_t instance, uint8_t* occ_dev);

/* ---------------------------------------------------------------- energies (a2) */

/* Configuration energies E_p = 1/2 q_p^T V q_p of P occupations, evaluated in the
 * reduced form of Eq. 2, E_p = E_ff + q^T h + 1/2 q^T V_mm q over the mobile
 * block (fixed-site entries of occ are ignored).
 *   GOAC_FP64  : FP64 matrix-core product Q V_mm and FP64 row dot.
 *   GOAC_MIXED : q = c + dq with the exact integer shift c; the quadratic part
 *                1/2 dq^T V_mm dq as dQ W dQ over the lower block triangle W of
 *                V_mm (diagonal 128-blocks halved), split W = W_hi + W_lo in
 *                bfloat16, on matrix cores with FP32 accumulation per 128 x 128
 *                block; E_p = E~ + sum_k dq_k h~_k + that part, the row sums
 *                added as 64-bit fixed point (a power-of-two scale per problem),
 *                so a call repeats bit-exactly whatever order the device runs
 *                the blocks in.
 *   occ_dev : P x n uint8 (P <= 2^30);  E_dev : P FP64 output.
 * The rows are checked first (conventions above). The energy kernels are queued
 * right behind the check and skip all work when it fails, so the call waits for
 * the check alone and the device runs on without a gap.
 * Errors: EINVAL (arguments; a row breaking the composition, E_dev then
 * unchanged); EINEXACT for GOAC_MIXED when a shifted charge is not exact in
 * bfloat16. */
goac_status goac_energies(goac_problem* pb, int64_t P, const uint8_t* occ_dev,
                          goac_precision prec, double* E_dev);

/* For callers that cannot allocate device memory (code under stream capture, tight
 * serving loops, harnesses that forbid allocation): goac_energies with the same
 * kernels and results, its scratch taken from a fixed 32 MiB device array that
 * every GPU the library runs on holds until the process ends. No device or pinned
 * memory is allocated. The call waits for the stream (it reads the row check back
 * into host memory of its own stack).
 *   Limit: the energies of P rows must fit the array (about P' x M x 2 + P x 8
 *   bytes for GOAC_MIXED, P' = P rounded up to a multiple of 256; P x M x 16 bytes
 *   plus split-K partials for GOAC_FP64);
 *   larger calls return EINVAL and compute nothing.
 *   Concurrency: all calls on one GPU share its array, which keeps the last call's
 *   contents; calls that overlap on one GPU (other host threads, other streams)
 *   race and are not allowed.
 * Errors: as goac_energies (EINVAL for a broken row, E_dev then unchanged). */
goac_status goac_energies_noalloc(goac_problem* pb, int64_t P, const uint8_t* occ_dev,
                                  goac_precision prec, double* E_dev);

/* Grid of the GOAC_MIXED population product for populations of P rows: the
 * product's (p-tile, n-tile, k-tile) units are shared by 2 x (compute units) / kt
 * workgroups, kt = 1, 2, 4 or 8 (at most the problem's number of 128-position
 * n-tiles unless 1; 0 returns P to the default, kt = 1). The energies differ
 * between settings only by the FP32 accumulation order, within the mixed bound.
 * Host-side; errors: EINVAL. */
goac_status goac_energies_tile(goac_problem* pb, int64_t P, int32_t kt);

/* Autotuner of that tile: times goac_energies(GOAC_MIXED) of occ_dev (P x n, device)
 * with every valid tile (one warm-up and the best of three calls, HIP events) and
 * keeps the fastest for later calls with P rows, as goac_energies_tile would.
 *   kt_out : the chosen tile (may be NULL)
 * Synchronises; takes P doubles of scratch from the context's cache for the call.
 * Errors: EINVAL (arguments, rows as goac_energies); EINEXACT as goac_energies. */
goac_status goac_energies_autotune(goac_problem* pb, int64_t P, const uint8_t* occ_dev, int32_t* kt_out);

/* The k lowest configurations among P candidates (Methodology: the n lowest
 * structures are the output): FP64 energies ordered by (E, index).
 *   idx_dev : k int64 output; E_dev : k FP64 output (k <= P).
 * Errors: EINVAL (arguments; a row breaking the composition, checked first with
 * a wait). */
goac_status goac_topk_fp64(goac_problem* pb, int64_t P, const uint8_t* occ_dev, int32_t k,
                           int64_t* idx_dev, double* E_dev);

/* ---------------------------------------------------------------- Monte Carlo (a3-a5) */

/* A set of C Metropolis swap chains on one problem (SI, "Monte Carlo" and
 * "Simulated annealing"). Each chain keeps its occupation, the per-sublattice
 * position lists sorted by species at creation (perm), the field phi = V_mm q +
 * h, its energy E, its trial counter t, counts, the best energy seen and its
 * occupation.
 *   occ_dev   : C x n start occupations; each must keep the problem's
 *               composition (EINVAL otherwise; the check synchronises)
 *   prec      : GOAC_FP64 (FP64 phi) or GOAC_MIXED (FP32 phi)
 *   chain_base: id of chain 0 in the Philox counters
 *   instance  : instance id in the Philox counters */
goac_status goac_chains_create(goac_problem* pb, int64_t C, const uint8_t* occ_dev,
                               goac_precision prec, uint32_t chain_base, uint32_t instance,
                               goac_chains** out);
void goac_chains_destroy(goac_chains* ch);

/* Many independent problems in one set of chains: instance i has
 * chains_per_instance[i] chains; chain ids restart at 0 for every instance and
 * the instance id is i. occ_dev holds the start occupations of all chains,
 * instance after instance, each row n_i long. Problems must share the context
 * (GOAC_ESTATE otherwise). The sweep runs every chain of every instance in one
 * persistent launch. */
goac_status goac_chains_create_batch(goac_problem* const* pbs, int32_t n_instances,
                                     const int64_t* chains_per_instance, const uint8_t* occ_dev,
                                     goac_precision prec, goac_chains** out);

#define GOAC_MC_TRACE_HASH 1u   /* accumulate the per-trial trajectory hash */
#define GOAC_REMC_GRAPH 2u      /* goac_remc_run: replay rounds from a captured HIP graph */
#define GOAC_MC_TIMING 4u       /* goac_mc_sweep: HIP events around each launch (goac_chains_timing) */

/* Parameters of one sweep. kT_host is a table of n_rows x n_blocks kT values
 * (eV); chain c at trial t uses row r_c (the chain set's temperature row, 0
 * unless set by goac_chains_set_rows or goac_remc_exchange) and column
 * min(t / block_len, n_blocks - 1). */
typedef struct {
    uint64_t seed;
    uint64_t n_trials;          /* trials added to every chain                     */
    const double* kT_host;
    int32_t n_rows;
    int32_t n_blocks;
    uint64_t block_len;
    int32_t reanchor_every;     /* MIXED: re-anchor after this many field updates  */
    uint32_t flags;             /* GOAC_MC_TRACE_HASH                              */
    int32_t variant;            /* 0: automatic; 64 or 256: threads per chain      */
    int32_t reserved;
} goac_mc_params;

/* Set the temperature row of every chain (rows_host: C int32 >= 0). */
goac_status goac_chains_set_rows(goac_chains* ch, const int32_t* rows_host);

/* Advance every chain by n_trials trials. Trial t of chain c (instance i):
 *   (r0,r1,r2,r3) = Philox4x32-10(counter (t_lo, t_hi, c, i << 8 | 1), key seed)
 *   a = mobile position (r0 M) >> 32 (species a, sublattice s), cnt = P_s -
 *   n_{s,a}; partner = perm_s[k < off_{s,a} ? k : k + n_{s,a}], k = (r1 cnt) >> 32;
 *   d = q_b - q_a; dE = d (phi_i - phi_j) + d^2/2 (V_ii + V_jj - 2 V_ij);
 *   u = ((r2:r3 >> 12) + 1/2) 2^-52; accept iff dE <= 0 or u < exp(-dE/kT).
 * On acceptance the two positions swap and phi_k += d (V_ik - V_jk) for every
 * mobile k. Chains resume where the previous sweep stopped.
 * GOAC_MIXED decides from the FP32 field only when the FP64 decision cannot
 * differ within a rigorous error bound; otherwise it recomputes phi_i and phi_j
 * in FP64. The field is re-anchored in FP64 between chunks once a chain has made
 * reanchor_every field updates. A chain whose FP32 error bound breaks (a NaN or
 * an overflow) keeps deciding every trial by the exact FP64 rule and sets its
 * status; goac_chains_export then reports GOAC_EDRIFT. */
goac_status goac_mc_sweep(goac_chains* ch, const goac_mc_params* params);

typedef struct {
    uint64_t t;          /* trials done                                         */
    uint64_t accepts;    /* accepted trials                                     */
    uint64_t updates;    /* accepted trials that changed the field (d != 0)     */
    uint64_t hash;       /* sum over trials of the per-trial hash (TRACE_HASH)  */
    uint64_t fallbacks;  /* MIXED: trials decided by the FP64 recompute         */
    uint64_t anchors;    /* MIXED: FP64 re-anchors                              */
    double E;            /* energy of the current occupation                    */
    double best_E;       /* lowest energy seen                                  */
    int32_t status;      /* 0, or 1 if the FP32 field left its bound (MIXED)    */
    int32_t row;         /* temperature row                                     */
} goac_chain_stats;

/* Launch autotuning: times a probe sweep of probe_trials trials at temperature kT
 * for each launch configuration (64 or 256 threads per chain, all or half of the
 * chains that fit a compute unit's LDS resident at once) and keeps the fastest
 * for later sweeps whose params.variant is 0. The chains' state is saved before
 * and restored after the probes, so they are left exactly as they were; results
 * of later sweeps do not depend on the configuration. Synchronises; allocates a
 * copy of the chain state for the duration of the call.
 *   wg_out, per_cu_out : the chosen threads per chain and chains per compute unit
 *                        (may be NULL) */
goac_status goac_chains_autotune(goac_chains* ch, uint64_t probe_trials, double kT, int32_t* wg_out,
                                 int32_t* per_cu_out);

/* Device time of the sweeps run with GOAC_MC_TIMING since the last call: the sum
 * over the Monte Carlo kernel launches and the sum over the batched FP64 anchors
 * between sweep chunks (cells of more than 1024 mobile positions, GOAC_MIXED),
 * from HIP events recorded on the context's stream around each, and the number of
 * Monte Carlo launches. Synchronises; resets the sums. Any pointer may be NULL. */
goac_status goac_chains_timing(goac_chains* ch, double* mc_seconds, double* anchor_seconds,
                               int64_t* mc_launches);

/* Copy chain results to caller buffers (any pointer may be NULL):
 *   occ_dev, best_occ_dev : C x n; stats_dev : C goac_chain_stats (device).
 * Synchronises: after the copies the chains' status flags are read, and the call
 * returns GOAC_EDRIFT (the copies made) when any chain's FP32 field has left its
 * error bound (a chain's flag stays set until goac_chains_load rebuilds it). */
goac_status goac_chains_export(goac_chains* ch, uint8_t* occ_dev, uint8_t* best_occ_dev,
                               goac_chain_stats* stats_dev);

/* Replica exchange (SI, "Replica Exchange Monte Carlo"): chains form
 * consecutive groups of R replicas on the ladder kT_host[0..R) (ascending). At
 * exchange step x, neighbours (k, k+1), k = x mod 2, x mod 2 + 2, ..., swap
 * temperatures with probability min(1, exp((E_k - E_k+1)(1/kT_k - 1/kT_k+1))),
 * E_k the energy of the chain at temperature k and u = ((r0:r1 >> 12) + 1/2)
 * 2^-52 from Philox at counter (k, x_lo, x_hi, group << 8 | 6), key seed.
 * Configurations stay with their chains; the chains' temperature rows move.
 *   R        : replicas per group, 2 <= R <= 2^19, dividing C
 *   slot_dev : (C / R) x R int32, the chain (index within its group) at each
 *              temperature, in/out; a group whose row is not a permutation of
 *              0 .. R-1 is left unchanged
 *   acc_dev  : (C / R) x R uint8: 1 where the pair (k, k+1) attempted at this step
 *              was accepted, 0 elsewhere (may be NULL)
 * Sweeps after an exchange run chain c at row = its temperature index. */
goac_status goac_remc_exchange(goac_chains* ch, int32_t R, const double* kT_host, uint64_t x,
                               uint64_t seed, int32_t* slot_dev, uint8_t* acc_dev);

/* `rounds` replica-exchange rounds, each `trials` trials per chain at the ladder
 * temperature of its slot followed by exchange step x0 + r (r = 0 .. rounds-1);
 * the same as alternating goac_mc_sweep (the ladder as an R x 1 table) and
 * goac_remc_exchange, bit for bit. The chains' rows are set from slot_dev first.
 * The rounds' kernels are launched on the stream one round after another. With
 * GOAC_REMC_GRAPH, up to 8 rounds (the sweep's kernels and the exchange) are
 * instead captured once as one HIP graph and replayed, the step index read from
 * device memory, and the rounds % 8 left over launch the same kernels on the
 * stream (on ROCm 7.2 the replay measured slower than the plain launches, even
 * for 64-trial rounds). Cells whose MIXED field re-anchors between sweep chunks
 * (more than 1024 mobile positions) always run without capture.
 *   flags : GOAC_MC_TRACE_HASH and/or GOAC_REMC_GRAPH;  reanchor_every : as in
 *           goac_mc_params
 *   slot_dev : groups x R int32 (in/out).
 * Launched round after round, the rounds are queued on the stream and the call
 * returns without waiting; with GOAC_REMC_GRAPH it waits for the stream before
 * releasing the graph. */
goac_status goac_remc_run(goac_chains* ch, int32_t R, const double* kT_host, uint64_t trials, uint64_t rounds,
                          uint64_t x0, uint64_t seed, uint32_t flags, int32_t reanchor_every, int32_t* slot_dev);

/* ---------------------------------------------------------------- GA (a6) */

typedef struct {
    uint64_t seed;
    uint32_t generation;
    int32_t n_elite;
    double p_mut;
} goac_ga_params;

/* One generation of the genetic algorithm (SI, "Genetic Algorithm"):
 *   elitism   : children 0..n_elite-1 are the parents ordered by (E, index)
 *   roulette  : weights w_p = E_max - E_p rounded to integer multiples of 2^-30
 *               eV and summed exactly; parent = the smallest p whose cumulative
 *               weight exceeds floor(x W / 2^64), x a 64-bit Philox draw at
 *               counter (c, g, 0, 3) (uniform choice when W = 0)
 *   crossover : the canonical swap path from parent A to parent B is walked and
 *               each of its swaps enters the child with probability 1/2 (top bit
 *               of Philox at counter (position, c, g, 4))
 *   mutation  : with probability p_mut one valid swap (Philox at (c, g, 1, 5))
 *   pop_in_dev : P x n; E_in_dev : P FP64; pop_out_dev : P x n (not aliasing pop_in).
 * Errors: EINVAL for a parent row that breaks the composition, and if (E_max -
 * E_min) 2^30 P exceeds 2^62 (or an energy is not a number): the rows and then
 * the weights are checked before any child is formed, the host waiting for
 * them, and pop_out_dev is then left untouched. EINVAL also when a child's mobile
 * positions do not fit one workgroup's LDS (3 bytes per mobile position plus one
 * 8-byte word per 64 positions of the longest sublattice, at most 160 KiB: about
 * 52,000 mobile positions). */
goac_status goac_ga_generation(goac_problem* pb, int64_t P, const uint8_t* pop_in_dev,
                               const double* E_in_dev, const goac_ga_params* params,
                               uint8_t* pop_out_dev);

/* `generations` GA generations in a row (SI, "Genetic Algorithm": the population
 * evolves generation after generation), bit for bit the same as alternating
 * goac_ga_generation (generation index params->generation + k, k = 0 ..
 * generations-1) and goac_energies of the children in `precision`. After the first
 * generation, eight generations at a time are captured once as one HIP graph and
 * replayed (when at least sixteen remain), the generation index read from a
 * device counter; the rest run on the stream.
 *   pop_dev : P x n (in/out): the population, then the last generation's children
 *   E_dev   : P FP64 (in/out): energies of pop_dev, then of the returned population
 *   precision : GOAC_FP64 or GOAC_MIXED
 * Errors: EINVAL as goac_ga_generation (the rows are checked first, with a wait,
 * and nothing is changed when one breaks the composition; the roulette range is
 * checked once, after the last generation, and pop_dev and E_dev are then
 * unspecified). Synchronises;
 * takes a second population buffer from the context's cache for the call. */
goac_status goac_ga_run(goac_problem* pb, int64_t P, uint8_t* pop_dev, double* E_dev,
                        const goac_ga_params* params, int32_t generations, int32_t precision);

/* Continue every chain from new occupations (occ_dev: C x n, device), e.g. to hand
 * it a configuration found by another heuristic. Trial counters, counts, hash and
 * temperature rows are kept; the position lists, field and energy are rebuilt
 * (an FP64 anchor); the best energy and occupation are replaced only when the new
 * occupation is strictly lower. Each occupation must keep the problem's
 * composition (EINVAL otherwise, and the chains are left unchanged; the check
 * runs first and the host waits for it). */
goac_status goac_chains_load(goac_chains* ch, const uint8_t* occ_dev);

/* ---------------------------------------------------------------- hybrid REMC + GA */

typedef struct {
    uint64_t seed;
    uint64_t round;            /* round index r (exchange steps and generations
                                  continue across rounds)                          */
    int64_t trials;            /* trials per chain before each exchange step        */
    const double* kT_host;     /* R temperatures (eV), ascending                    */
    int32_t R;                 /* replicas per group of consecutive chains          */
    int32_t exchanges;         /* exchange steps per REMC phase                     */
    int32_t generations;       /* GA generations per GA phase                       */
    int32_t n_elite;
    double p_mut;
    int32_t inject;            /* GA ranks handed to the groups' coldest replicas   */
    int32_t precision;         /* goac_precision of the GA phase's energies         */
    int32_t reanchor_every;    /* MIXED chains: as in goac_mc_params (0: 1024)      */
    int32_t reserved;
} goac_hybrid_params;

/* One round of the replica-exchange + GA hybrid (SI, "Hybrid Methods": the two
 * heuristics run alternately and hand their best solutions on):
 *   1. REMC phase: `exchanges` times, every chain runs `trials` trials at the
 *      temperature of its slot, then one exchange step x = r exchanges + e;
 *   2. REMC -> GA: the population becomes the P lowest, by (FP64 energy, index),
 *      of the population followed by the chains' best occupations;
 *   3. GA phase: `generations` generations g = r generations + k, each followed by
 *      the children's energies in the requested precision;
 *   4. GA -> REMC: the coldest replica of group k takes the individual of rank
 *      k mod min(inject, P) when that individual is strictly lower than the
 *      replica's current energy; all chains continue (goac_chains_load).
 *   ch       : chains of one problem, C = groups x R
 *   slot_dev : groups x R int32 as in goac_remc_exchange (in/out); the chains'
 *              rows are set from it at the start
 *   pop_dev  : P x n population (in/out); E_dev : P FP64, the energies of the
 *              returned population (out)
 * Synchronises three times: for the composition check of pop_dev at the start
 * (EINVAL, nothing changed), after the GA phase (a roulette failure in any of its
 * generations is reported then, GOAC_EINVAL) and for the composition check of
 * the reload. ESTATE for a chain set of several problems. The chain set owns the
 * scratch memory of the round (grown on demand, freed with the chains). */
goac_status goac_hybrid_round(goac_chains* ch, int32_t* slot_dev, int64_t P, uint8_t* pop_dev, double* E_dev,
                              const goac_hybrid_params* params);

/* ---------------------------------------------------------------- gradient descent */

/* Best-swap descent of P configurations to local minima (SI, "Gradient
 * Descent"). A step scores every swap of two positions of one site class that hold
 * different species by dE = d (phi_i - phi_j) + 1/2 d^2 (V_ii + V_jj - 2 V_ij),
 * d = q_j - q_i, with the FP64 field phi = V_mm q + h, and applies the
 * lexicographically first swap (i < j in mobile order) among those whose dE lies
 * within tol of the lowest dE (equal-energy neighbours are resolved only to
 * rounding noise, so the window makes the choice well defined); it stops when the
 * lowest dE is >= -tol or after max_steps swaps.
 *   occ_dev   : P x n uint8, read and overwritten with the local minima (fixed
 *               sites are left as they are); checked first as in goac_energies
 *               (EINVAL, nothing changed)
 *   max_steps : swaps per configuration at most; tol >= 0 (eV), e.g. 1e-9
 *   steps_dev : P int64 output (swaps taken) or NULL
 *   E_dev     : P FP64 output (energy of the result) or NULL
 * One workgroup holds a configuration's mobile block: EINVAL when 18 bytes per
 * mobile position exceed the compute unit's shared memory. */
goac_status goac_gd_run(goac_problem* pb, int64_t P, uint8_t* occ_dev, int64_t max_steps, double tol,
                        int64_t* steps_dev, double* E_dev);

#ifdef __cplusplus
}
#endif
#endif /* GOAC_H */
