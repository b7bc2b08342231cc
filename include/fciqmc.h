/*
 * fciqmc.h -- C ABI of the MI355X FCIQMC library (libfciqmc.so).
 *
 * The library runs the FCIQMC iteration of Booth, Smart & Alavi,
 * "Linear-scaling and parallelizable algorithms for stochastic quantum
 * chemistry" (arXiv:1305.6981), on one AMD Instinct MI355X (gfx950), with the
 * whole signed-walker list resident in device memory:
 *   - spawning: one attempt per walker, a random single or double excitation
 *     with its generation probability (Sec. 5, Eq. p_sing and the double
 *     excitation formula), the Slater-Condon element, and acceptance with
 *     probability tau |H_ij| / P_gen, the integer part deterministic
 *     (Sec. 2, Eq. pspawn);
 *   - death/cloning of all walkers on a determinant at once (Eq. pdeath);
 *   - annihilation of the spawned walkers against the main list with the
 *     initiator rule applied to spawns onto unoccupied determinants, and the
 *     diagonal element computed when a determinant becomes occupied (Sec. 4.2);
 *   - the projected energy (Eq. ProjE) and the population-control shift
 *     (Sec. 2), with blocking error bars (Sec. 7).
 *
 * Conventions
 *   - spin orbital p = 2*s + sigma (s spatial orbital, sigma 0 = alpha,
 *     1 = beta); a determinant has bit p set when p is occupied (the
 *     bit-string representation of Sec. 3) and takes as many 64-bit words as
 *     its spin orbitals need, low word first: W = 1 up to 64 spin orbitals,
 *     W = 2 up to 128 (2*n_orb <= 128; fciqmc_det_words; W = 2 can be forced
 *     for fewer with fciqmc_params.det_words). Every determinant argument and
 *     array below holds W words per determinant, and all systems of a handle
 *     share one W (the first system's).
 *   - all pointers in this header are HOST pointers; the library copies what
 *     it needs at the call and never keeps a caller's pointer.
 *   - return value: 0 on success, a negative FCIQMC_E* code on failure; the
 *     message of the last failure on the calling thread is returned by
 *     fciqmc_last_error(). No C++ exception crosses this boundary.
 *   - a handle is used by one host thread at a time; its device work runs on
 *     the HIP stream given at creation (NULL: the library's own stream).
 *   - results do not depend on memory layout, table sizes, launch shapes or
 *     on which other systems share a batch: every random decision is drawn
 *     from a Philox4x32-10 stream keyed by (seed, iteration, determinant,
 *     walker ordinal), and every merge is an integer sum.
 */
#ifndef FCIQMC_H
#define FCIQMC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FCIQMC_OK            0
#define FCIQMC_EINVAL       -1   /* bad argument: sizes, tau <= 0, 2*n_orb > 128, ... */
#define FCIQMC_ENOMEM       -2   /* device or host allocation failed / does not fit */
#define FCIQMC_EDEVICE      -3   /* a HIP call failed (message kept) */
#define FCIQMC_ECAPACITY    -4   /* a table could not be grown */
#define FCIQMC_EOVERFLOW    -5   /* a population left the int32 range, or died out */
#define FCIQMC_ESTATE       -6   /* call not valid for this handle or slot */

typedef struct fciqmc_t fciqmc_t;   /* opaque; owned by the library */

/* The Hamiltonian in an M-orbital determinant basis with N = n_alpha + n_beta
 * electrons (Sec. 2). */
typedef struct {
    int32_t n_orb;              /* M spatial orbitals, 1 <= M <= 64 */
    int32_t n_alpha, n_beta;    /* electrons per spin */
    int32_t reserved0;
    double e_core;              /* constant energy */
    const double *h1;           /* M*M row-major one-electron integrals, symmetric */
    const double *eri;          /* eight-fold packed (pq|rs): pair ij = i(i+1)/2 + j (i >= j),
                                   element IJ(IJ+1)/2 + KL (IJ >= KL); M(M+1)/2*(M(M+1)/2+1)/2 doubles */
    const uint8_t *orb_irrep;   /* NULL: no point group; else an abelian irrep label 0..7 per
                                   spatial orbital, direct product = XOR (Sec. 5) */
    double p_double;            /* >= 0: probability of drawing a double excitation; < 0: the
                                   ratio of double to all symmetry-allowed excitations of the
                                   reference (Sec. 5) */
    const uint64_t *ref_det;    /* NULL: aufbau (lowest n_alpha / n_beta orbitals by h_pp);
                                   else W words */
} fciqmc_hamiltonian;

/* Run parameters. */
typedef struct {
    double tau;                 /* time step, > 0 */
    double shift_damping;       /* zeta in S <- S - zeta/(A tau) ln(N_w/N_prev) */
    double initial_shift;       /* S before the target is reached, relative to E0 = H_00 */
    int32_t shift_update_every; /* A >= 1: the target test and the shift update happen when
                                   the number of completed iterations is a multiple of A */
    int32_t initiator_threshold;/* n_a: a determinant is an initiator when |C| > n_a (the
                                   reference always is); 0 gives plain FCIQMC */
    int64_t target_walkers;     /* the shift starts to vary once N_w >= target */
    int64_t initial_walkers;    /* walkers placed on the reference at start (0: 10) */
    int64_t det_capacity;       /* initial main-list capacity in entries (0: automatic; rounded
                                   up to whole chunks of 1024); the list is re-bucketed as it
                                   grows, and results do not depend on it */
    int64_t spawn_capacity;     /* initial capacity of the handle's spawn-record buffer in
                                   records (0: automatic); it grows by itself (an iteration
                                   that overflows it is re-run bit-exactly) */
    uint64_t seed;              /* Philox key */
    int32_t avg_start;          /* iterations after the shift starts varying before samples
                                   enter the averages */
    /* Restricted space (Sec. 5 and its note on truncated and active-space
     * calculations): a child outside the space is a null excitation, so the run
     * samples the ground state of H within the space. space = 0: the full space;
     * else a bitwise OR of FCIQMC_SPACE_*; the reference must lie in the space
     * (EINVAL otherwise). */
    int32_t space;
    int32_t max_excitation;     /* FCIQMC_SPACE_EXCITATION: at most this many electrons
                                   outside the reference's orbitals (2: CISD) */
    int32_t max_seniority;      /* FCIQMC_SPACE_SENIORITY: at most this many singly
                                   occupied spatial orbitals */
    uint64_t frozen_occupied;   /* FCIQMC_SPACE_FROZEN: spin orbitals (0-63) occupied in
                                   every determinant (a CAS core) */
    uint64_t frozen_empty;      /* FCIQMC_SPACE_FROZEN: spin orbitals (0-63) empty in every
                                   determinant (CAS virtuals) */
    /* Spin-coupled functions (Sec. 5.3, Eqs. EqualCoeffs and SpinCoup): 0 samples
     * determinants; +1 / -1 samples the pairs {D, D~} (alpha and beta exchanged)
     * symmetric under the exchange with the sign of even / odd total spin S.
     * Needs n_alpha = n_beta and no restricted space (EINVAL otherwise). A function
     * is held as the smaller determinant of its pair (walker lists in and out);
     * excitations are drawn from that determinant, the target's generation
     * probability sums over its two determinants. Closed pairs (every orbital
     * empty or doubly occupied) exist for even S only. */
    int32_t hphf;
    int32_t reserved1;
    uint64_t frozen_occupied_hi;/* as frozen_occupied, for spin orbitals 64-127 */
    uint64_t frozen_empty_hi;   /* as frozen_empty, for spin orbitals 64-127 */
    int32_t det_words;          /* 64-bit words per determinant: 0 as the spin orbitals need
                                   (Sec. 3); 2 forces two words for at most 64 (EINVAL: other
                                   values, or 1 for more than 64 spin orbitals) */
    int32_t reserved2;
} fciqmc_params;

#define FCIQMC_SPACE_EXCITATION 1
#define FCIQMC_SPACE_SENIORITY  2
#define FCIQMC_SPACE_FROZEN     4

/* Estimators and counters of one system. Counts refer to the last completed
 * iteration unless marked total. */
typedef struct {
    int64_t iteration;          /* completed iterations */
    int64_t n_walkers;          /* N_w = sum |C| */
    int64_t n_dets;             /* occupied determinants */
    int64_t ref_pop;            /* C_0 */
    int64_t attempts;           /* spawn attempts (= N_w at the start of the iteration) */
    int64_t spawns;             /* accepted spawning events (records entering annihilation) */
    int64_t merged;             /* distinct determinants receiving a nonzero spawned sum */
    int64_t aborted;            /* walkers discarded by the initiator rule */
    int64_t total_attempts, total_spawns;
    int64_t n_samples;          /* iterations in the averages */
    int64_t n_var;              /* iteration at which the shift started to vary */
    int64_t n_prev;             /* N_w at the last shift update */
    int64_t table_slots;        /* main-list capacity in entries: buckets x 256 (layout only) */
    int64_t table_used;         /* main-list entries after the last iteration: the occupied
                                   determinants and the reference (layout only; the list is
                                   re-bucketed before the mean bucket passes 5/8 full) */
    double shift;               /* S, relative to E0 */
    double e_ref;               /* E0 = H_00 */
    double p_double;
    double proj_num;            /* sum over D != D0 of <D|H|D0> C_D */
    double e_proj_inst;         /* E0 + proj_num / C_0 (NaN when C_0 = 0) */
    double e_proj_mean, e_proj_err;   /* E0 + <num>/<C_0> and its blocking error */
    double shift_mean, shift_err;     /* E0 + <S> and its blocking error */
    double ms_last_call;        /* wall time of the last fciqmc_iterate on this handle */
    int32_t shift_varying;
    int32_t status;             /* 0, or the FCIQMC_E* code that stopped this system */
    int64_t redos;              /* total: iterations re-run after the spawn-record buffer
                                   overflowed (each re-run is bit-identical to an
                                   uninterrupted one) */
    int64_t spills;             /* total: iterations whose new determinants overflowed
                                   their bucket (completed through the spill list, then
                                   re-bucketed; results unaffected) */
    /* Device time (ms) of the phases of one iteration of the handle: the last
     * iteration of the last fciqmc_iterate call runs as direct launches bracketed
     * by events (the others run in graphs). Spawning includes the attempt mapping
     * (chunk scans); death runs inside the annihilation pass, so ms_death is 0 and
     * its time is part of ms_annihilate; the estimators include the shift. */
    double ms_spawn, ms_death, ms_annihilate, ms_estimators;
    int64_t born;               /* determinants that entered the main list: unoccupied
                                   after death, with an initiator among the parents of
                                   their merged spawns (Sec. 4.2) */
} fciqmc_estimates;

/* One iteration's record (the last 256 iterations of each slot are kept). */
typedef struct {
    int64_t iteration;          /* completed iterations after this one */
    int64_t n_walkers, n_dets, ref_pop;
    int64_t attempts, spawns, merged, aborted, born;
    int64_t entries;            /* main-list entries after the iteration (the occupied
                                   determinants and the reference) */
    double proj_num, shift;
    int32_t shift_varying, status;
} fciqmc_iteration;

/* Create a handle holding one system and place initial_walkers on the
 * reference D0, whose diagonal element E0 = H_00 is the energy origin of the
 * shift (Sec. 2). The integrals are copied to the device with the pair and
 * single-excitation term tables derived from them (Sec. 5).
 * hip_stream: a hipStream_t (e.g. torch.cuda.current_stream().cuda_stream),
 * or NULL. Errors: EINVAL, ENOMEM, EDEVICE. */
int fciqmc_init(const fciqmc_hamiltonian *ham, const fciqmc_params *prm, void *hip_stream,
                fciqmc_t **out);

/* Advance every active system of the handle by n_iterations (>= 0) full
 * iterations: spawning from every walker with an excitation drawn by the
 * generator of Sec. 5 and accepted with probability tau |H_ij| / P_gen
 * (Sec. 2, Eq. pspawn); death/cloning of every determinant (Eq. pdeath);
 * merging of the spawned walkers per child (Sec. 4.1) and annihilation against
 * the main list with the initiator rule for unoccupied children (Sec. 4.2);
 * the estimators (Eq. ProjE) and the shift update (Sec. 2). Iterations run in
 * graph-captured launches of up to 64; the main list is re-bucketed as it
 * grows, and an iteration that overflows the spawn-record buffer is re-run
 * bit-exactly after the buffer grows.
 * Errors: EINVAL, EDEVICE, ECAPACITY, EOVERFLOW. */
int fciqmc_iterate(fciqmc_t *h, int32_t n_iterations);

/* Estimators of system 0 of the handle: N_w, N_d, C_0 and the projected-energy
 * numerator of the last iteration (Eq. ProjE), the shift and its update state
 * (Sec. 2), and the averages of E_proj and of the shift with blocking error
 * bars kept online (the blocking of correlated ratios cited in Sec. 7). */
int fciqmc_estimators(fciqmc_t *h, fciqmc_estimates *out);

/* Release everything. NULL-safe. */
int fciqmc_free(fciqmc_t *h);

/* Copy the main list of system 0 (Sec. 4.2) -- its occupied determinants as
 * bit strings (Sec. 3; W words each, det has room for cap * W words), sorted
 * as unsigned integers, with their signed populations -- into the caller's
 * host arrays (each of length cap; any may be NULL). flags[i] is 1
 * when the determinant is an initiator for the next iteration (|C| > n_a, or
 * the reference; Sec. 4.2). Returns the number of occupied determinants
 * (which may exceed cap: then only cap are written), or a negative error code. */
int64_t fciqmc_walkers(fciqmc_t *h, uint64_t *det, int32_t *pop, uint32_t *flags, int64_t cap);

/* Replace the main list of system 0 (Sec. 4.2; determinants as bit strings of
 * W words each, Sec. 3) for a checkpoint restart. Entries with
 * pop == 0 are ignored; the reference is kept in the list even when absent.
 * iteration is the number of completed iterations, shift is S relative to E0,
 * varying / n_var / n_prev restore the shift-update state. The averages are
 * cleared. Errors: EINVAL (duplicates, electron-count mismatch), ENOMEM. */
int fciqmc_load_walkers(fciqmc_t *h, const uint64_t *det, const int32_t *pop, int64_t n,
                        int64_t iteration, double shift, int64_t n_prev, int32_t varying,
                        int64_t n_var);

/* 64-bit words per determinant of the handle's systems (Sec. 3): 1 or 2, or a
 * negative error code. */
int32_t fciqmc_det_words(const fciqmc_t *h);

/* Set the shift S of system 0 (Sec. 2; relative to E0) and start (varying = 1)
 * or stop its variation; when started, N_prev is set to the current N_w and
 * n_var to the current iteration. Used to end a growth stage run at a raised
 * shift. */
int fciqmc_set_shift(fciqmc_t *h, double shift, int32_t varying);

/* Re-bucket the main list (Sec. 4.2) of every active system into at least
 * `slots` entries of capacity (rounded up to a multiple of 4096) now, rather
 * than when its buckets fill. A list already that large is left alone.
 * Results never depend on the capacity. Errors: EINVAL (slots < 0),
 * ECAPACITY (the device cannot hold the larger list; the old one stays). */
int fciqmc_reserve(fciqmc_t *h, int64_t slots);

/* Thread-local message of the last failure ("" when none). */
const char *fciqmc_last_error(void);

/* ---- batching and serving: many independent systems in one handle -------
 * Not in the paper (its parallelism is one system over many processes); these
 * calls run many independent systems at once. The systems of a batch advance
 * together: every iteration of every system is one pass of the same kernels
 * over a descriptor table, so one launch serves all of them, and each
 * system's walker list is bit-identical to the list it would have alone.
 * Slots are numbered 0 .. max_slots-1. */

/* Create a handle with room for max_slots systems and admit n of them
 * (hams[i], prms[i] -> slot i). Errors: EINVAL, ENOMEM, EDEVICE. */
int fciqmc_batch_create(int32_t max_slots, int32_t n, const fciqmc_hamiltonian *hams,
                        const fciqmc_params *prms, void *hip_stream, fciqmc_t **out);

/* Advance every active system by n_iterations (same as fciqmc_iterate). */
int fciqmc_batch_iterate(fciqmc_t *h, int32_t n_iterations);

/* Advance each active slot i by n_iter[i] iterations (n_iter has max_slots
 * entries; inactive slots are ignored). Systems that reach their count idle
 * while the others run. */
int fciqmc_batch_iterate_each(fciqmc_t *h, const int32_t *n_iter);

/* Admit one system into a free slot while others may be mid-run. Fails with
 * ENOMEM when its footprint (fciqmc_footprint_bytes: a main list of twice the
 * walker target in entries of 20 B -- key 8, population 4, diagonal element 8
 * -- plus 4 B per bucket of 256 entries, and its integral tables) does not
 * fit in the free device memory left after the reserve, with ESTATE when no
 * slot is free. */
int fciqmc_batch_admit(fciqmc_t *h, const fciqmc_hamiltonian *ham, const fciqmc_params *prm,
                       int32_t *slot);

/* Retire a slot and free its device memory. */
int fciqmc_batch_retire(fciqmc_t *h, int32_t slot);

/* fciqmc_estimators and fciqmc_walkers for the system in `slot`. */
int fciqmc_batch_slot_estimators(fciqmc_t *h, int32_t slot, fciqmc_estimates *out);
int64_t fciqmc_batch_slot_walkers(fciqmc_t *h, int32_t slot, uint64_t *det, int32_t *pop,
                                  uint32_t *flags, int64_t cap);

/* Device bytes a system with the given walker target would reserve, and the
 * number of active slots. */
int64_t fciqmc_footprint_bytes(const fciqmc_hamiltonian *ham, const fciqmc_params *prm);
int32_t fciqmc_batch_active(fciqmc_t *h);

/* ---- instrumentation -------------------------------------------------------
 * Per-kernel-group device time (ms) accumulated since the last reset, measured
 * with HIP events on the handle's stream around each group of non-graph
 * launches (enable with fciqmc_set_profiling(h, 1); graph launches are then
 * disabled). Groups: 0 chunk sums of |C| (first iteration of a launch),
 * 1 attempt mapping (chunk scans), 2 spawning (Sec. 2, 5: records of the
 * accepted spawns), 3 annihilation (the records sorted by bucket, then death,
 * merge and annihilation per bucket: Eq. pdeath, Sec. 4.1, 4.2),
 * 4 statistics reduction / shift (Eq. ProjE, Sec. 2). counts[k] is the number
 * of launches measured. */
int fciqmc_set_profiling(fciqmc_t *h, int32_t on);
int fciqmc_kernel_times(fciqmc_t *h, double ms[5], int64_t counts[5]);

/* Records of iterations first .. first + n - 1 of a slot (each must be among the
 * slot's last 256 iterations) into out[0 .. n). Returns n, or EINVAL / ESTATE. */
int64_t fciqmc_history(fciqmc_t *h, int32_t slot, int64_t first, int64_t n, fciqmc_iteration *out);

/* ---- launch shape ----------------------------------------------------------
 * spawn_grid: workgroups of the spawning kernel; tile: consecutive attempts a
 * workgroup takes at a time (a power of two, 256 .. 2^20; a tile never spans
 * two chunks of the table); post_grid: workgroups of the
 * death/annihilation kernel. Results never depend on these (every random
 * number is keyed by determinant and walker ordinal, every merge is an
 * integer sum). fciqmc_autotune saves every active system (walker list,
 * dynamics, statistics, iteration log), runs iters_per_trial iterations of all
 * of them for each candidate shape (spawn grid 2/4/8/16 x CUs with tile
 * 1024/2048/4096, then post grid 2/3/4/6/8 x CUs), keeps the shape with the
 * lowest spawning time per attempt and annihilation time per iteration, and
 * restores the systems: their walker lists continue exactly as if no trial
 * had run (the projected-energy numerator may differ in its last bits, since
 * its partial sums follow the table layout and the launch shape). */
int fciqmc_set_launch(fciqmc_t *h, int32_t spawn_grid, int32_t tile, int32_t post_grid);
int fciqmc_get_launch(fciqmc_t *h, int32_t *spawn_grid, int32_t *tile, int32_t *post_grid);
int fciqmc_autotune(fciqmc_t *h, int32_t iters_per_trial);

/* ---- export without allocation ------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as fciqmc_walkers (system 0, sorted by determinant, flags as there),
 * staged on the device in a fixed area that the library holds on each GPU
 * until the process ends (32 MiB + 256 B: at most 2^21 = 2097152 occupied
 * determinants), so the call allocates nothing. Every call on one GPU shares
 * that GPU's area: calls that overlap in time on one GPU (from several host
 * threads or handles) race and must be serialised by the caller. Returns the
 * number of occupied determinants (only min(n, cap) entries are written), or
 * ECAPACITY when the list exceeds 2^21 determinants (nothing written),
 * EINVAL, ESTATE (also for two-word determinants, which the area does not
 * hold), EDEVICE. */
int64_t fciqmc_walkers_noalloc(fciqmc_t *h, uint64_t *det, int32_t *pop, uint32_t *flags,
                               int64_t cap);

/* ---- error bars -------------------------------------------------------------
 * The blocking analysis behind e_proj_err / shift_err, for a caller's own
 * series (host only, no device work): blocks of 2^l consecutive samples are
 * averaged level by level, kept online in O(log n) memory, and the error of
 * <num>/<den> (den NULL: of <num>) is read at the first level with >= 16 blocks
 * whose error the next two levels do not exceed by more than its relative
 * uncertainty 1/sqrt(2(n-1)) -- the blocking of correlated ratios cited in the
 * paper's Sec. 7. *err is NaN when no level has 16 blocks. Errors: EINVAL. */
int fciqmc_blocking(const double *num, const double *den, int64_t n, double *mean, double *err);

/* ---- test knobs -------------------------------------------------------------
 * planner = 0: do not size the buckets or the spawn-record buffer before each
 * launch, so that overflows are met inside an iteration: an overflowing record
 * buffer abandons the iteration, grows and re-runs it (fciqmc_estimates.redos),
 * an overflowing bucket completes the iteration through the spill list and is
 * re-bucketed (fciqmc_estimates.spills). record_capacity > 0 replaces the record
 * buffer by one of that many records now (0: leave it). tile_map_limit >= 0 caps
 * the map from spawn tiles to chunks at that many entries (0: no map), so tile
 * grabs beyond it search the chunk offsets instead; -1 restores the default.
 * Results do not depend on any of these. Errors: EINVAL, ENOMEM. */
int fciqmc_set_test_options(fciqmc_t *h, int32_t planner, int64_t tile_map_limit,
                            int64_t record_capacity);

#ifdef __cplusplus
}
#endif
#endif
