/*
 * CPU oracle for the FCIQMC iteration of Booth, Smart & Alavi,
 * "Linear-scaling and parallelizable algorithms for stochastic quantum
 * chemistry" (arXiv:1305.6981).
 *
 * TEST INFRASTRUCTURE ONLY. This is a plain, slow reference implementation
 * (single-threaded unless the virtual processes are spread over host threads)
 * used by the test-suite, the smoke check and the CPU baseline leg of the
 * benchmark. The product library never links, loads or calls it,
 * and it shares no source with the HIP path.
 *
 * Conventions (shared only as a *data format* with the product ABI):
 *   spin orbital p = 2*s + sigma (s spatial, sigma 0 = alpha, 1 = beta);
 *   a determinant has bit p set when p is occupied and is passed as W 64-bit
 *   words, low word first (Sec. 3: as many words as the spin orbitals need):
 *   W = 1 up to 64 spin orbitals, W = 2 up to 128 (orc_det_words; W = 2 can
 *   also be forced for fewer with orc_params.det_words). Arrays of
 *   determinants hold W words per entry;
 *   h1 is M*M row-major; eri is the eight-fold packed (pq|rs) array with pair
 *   index ij = i(i+1)/2 + j (i >= j) and element IJ(IJ+1)/2 + KL (IJ >= KL).
 */
#ifndef FCIQMC_ORACLE_H
#define FCIQMC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t n_orb, n_alpha, n_beta, pad0;
    double e_core;
    const double *h1;
    const double *eri;
    const uint8_t *orb_irrep;   /* NULL: every orbital in the totally symmetric irrep */
    double p_double;            /* < 0: ratio of double to all excitations from D0 */
    const uint64_t *ref_det;    /* NULL: aufbau by h_pp; else W words */
} orc_ham;

typedef struct {
    double tau, zeta, shift0;
    int32_t shift_every, n_a;
    int64_t target, n_init;
    uint64_t seed;
    int32_t avg_start, pad0;
    uint64_t hash_seed;         /* seeds the random orbital map of Algorithm 1 */
    int64_t hash_range;         /* initial size of the main-list hash table; 0 = auto */
    /* Virtual processes (Sec. 4.1): 0 or 1 = one list. */
    int32_t n_procs;
    int32_t ref_own_proc;       /* 1: the reference alone on process 0 (needs n_procs >= 2) */
    uint64_t proc_seed;         /* seeds the random map of the process hash; 0 = default */
    int32_t n_threads;          /* host threads over which the processes run; 0 = 1 */
    /* Restricted space (Sec. 5: children outside it are null excitations): a bitwise OR
     * of ORC_SPACE_* selects the conditions a determinant of the space meets. */
    int32_t space;
    int32_t max_excitation;     /* ORC_SPACE_EXCITATION: at most this many electrons moved
                                   away from the reference */
    int32_t max_seniority;      /* ORC_SPACE_SENIORITY: at most this many singly occupied
                                   spatial orbitals */
    int32_t hphf;               /* 0: determinants; +1 / -1: spin-coupled functions
                                   (Sec. 5.3) of even / odd total spin S (needs
                                   n_alpha = n_beta; no restricted space) */
    uint64_t frozen_occupied;   /* ORC_SPACE_FROZEN: spin orbitals occupied in every determinant */
    uint64_t frozen_empty;      /* ORC_SPACE_FROZEN: spin orbitals empty in every determinant */
    uint64_t frozen_occupied_hi, frozen_empty_hi;   /* the same for spin orbitals 64..127 */
    int32_t det_words;          /* 0: as the spin orbitals need; 2: two words even for <= 64 */
    int32_t pad1;
} orc_params;

#define ORC_SPACE_EXCITATION 1
#define ORC_SPACE_SENIORITY  2
#define ORC_SPACE_FROZEN     4

typedef struct {
    int64_t iteration, n_walkers, n_dets, ref_pop;
    int64_t attempts, spawns, merged, aborted;
    int64_t total_attempts, total_spawns, n_samples, n_var;
    double shift, e_ref, p_double, proj_num, e_proj_inst;
    double e_proj_mean, e_proj_err, shift_mean, shift_err;
    int32_t shift_varying, pad0;
    int64_t n_prev;
    int64_t born;               /* determinants entering the main list (Sec. 4.2) */
} orc_est;

typedef struct orc_state orc_state;

/* Whole-run interface (same meaning as the product's fciqmc_* calls). */
int     orc_create(const orc_ham *ham, const orc_params *prm, orc_state **out);
int     orc_iterate(orc_state *st, int32_t n_iter);
int     orc_estimates(orc_state *st, orc_est *out);
int64_t orc_walkers(orc_state *st, uint64_t *det, int32_t *pop, uint32_t *flags, int64_t cap);
int     orc_load_walkers(orc_state *st, const uint64_t *det, const int32_t *pop, int64_t n,
                         int64_t iteration, double shift, int64_t n_prev, int32_t varying,
                         int64_t n_var);
void    orc_free(orc_state *st);
int64_t orc_proc_dets(orc_state *st, int32_t p);           /* main-list entries on process p */
int32_t orc_owner(const orc_state *st, const uint64_t *det);   /* process that owns det */
int32_t orc_det_words(const orc_state *st);                     /* W */
const char *orc_last_error(void);

/* Unit-level entry points used by the pins. */
void    orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* (Determinant arguments below: W words each, W = orc_det_words of the state.) */
int     orc_decode(const uint64_t *det, int32_t words, int32_t *occ);   /* byte-table decode */
int64_t orc_hash(const orc_state *st, const uint64_t *det, int64_t range);   /* Algorithm 1 */
double  orc_hel(const orc_state *st, const uint64_t *bra, const uint64_t *ket);   /* <bra|H|ket> */
double  orc_hdiag(const orc_state *st, const uint64_t *det);
double  orc_pgen(const orc_state *st, const uint64_t *det, const uint64_t *target);
/* Elements between the stored functions of the run (determinants, or spin-coupled
 * functions held as their smaller determinant): <bra|H|ket> with ket the source,
 * and the diagonal element. */
double  orc_fn_hel(const orc_state *st, const uint64_t *bra, const uint64_t *ket);
double  orc_fn_diag(const orc_state *st, const uint64_t *fn);
double  orc_proj_num(const orc_state *st, const uint64_t *det, const double *c, int64_t n);
int     orc_sample_excitations(const orc_state *st, const uint64_t *det, int64_t iteration,
                               int64_t n_samples, uint64_t *out_det, double *out_pgen,
                               double *out_hel);
double  orc_log(double x);                              /* shift-update logarithm */
int     orc_blocking(const double *num, const double *den, int64_t n,
                     double *mean_ratio, double *err, int32_t *level);

#ifdef __cplusplus
}
#endif
#endif
