// Internal layout shared by the kernels and the host engine of libfciqmc.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fq {

constexpr int BQ = 256;              // entries per bucket of the main list (a wavefront's unit
                                     // in annihilation: four per lane)
constexpr int CHUNK = 1024;          // four consecutive buckets: the unit of attempt mapping and
                                     // spawn staging, and one workgroup's unit in annihilation
constexpr int BPC = CHUNK / BQ;      // buckets per chunk
constexpr int BUCKET_FILL = 128;     // planned mean entries per bucket (half full)
constexpr int NCLASS = 16;           // symmetry classes: 2 spins x up to 8 abelian irreps
constexpr int REC_CAP = 256;         // per-system ring of per-iteration records
constexpr int MAX_GRAPH_ITERS = 64;  // iterations captured in one graph launch
constexpr int SCAN_G = 2048;         // workgroups of the chunk-sum and scan-down kernels; each
                                     // takes one contiguous range of chunks
constexpr int FIN_BLOCKS = 64;       // workgroups per system reducing the chunk statistics

// Status bits set on the device.
constexpr uint32_t ST_TABLE_FULL = 1u;     // the spawn-record buffer overflowed: the iteration
                                           // is abandoned, the buffer grown, the iteration redone
constexpr uint32_t ST_POP_OVERFLOW = 2u;   // a population left int32
constexpr uint32_t ST_DIED = 4u;           // N_w reached zero
constexpr uint32_t ST_SPAWN_OVERFLOW = 8u; // one spawning event would create > 2^30 walkers
constexpr uint32_t ST_SPILLED = 16u;       // new determinants did not fit their bucket: the
                                           // iteration completed with them in the spill list,
                                           // the system pauses until the host re-buckets
constexpr uint32_t ST_SPILL_FULL = 32u;    // the spill list itself overflowed (fatal)


struct IterRecord {
    int64_t iter;      // completed iterations after this one
    int64_t nw, nd, c0, attempts, spawns, merged, aborted;
    int64_t born;      // determinants that entered the main list
    int64_t used;      // entries in the buckets after the iteration (occupied + the reference)
    int64_t n_var, n_prev;
    double num, shift;
    int32_t varying, status;
};

// Statistics of one bucket of an iteration (one share per wavefront of a chunk).
// counts packs three numbers below 2^21: entries | merged spawn targets << 21 |
// occupied << 42.
struct ChunkStat {
    int64_t nw, aborted;
    uint64_t counts;
    double num;
    int64_t born;
};
constexpr int CNT_SHIFT_MERGED = 21, CNT_SHIFT_ND = 42;
constexpr int POST_WAVES = BPC;   // wavefronts of a k_post workgroup: one bucket and one
                                   // ChunkStat share each
constexpr uint64_t CNT_FIELD = (1ull << 21) - 1;

// One workgroup's share of a system's iteration statistics.
struct FinPart {
    int64_t nw, nd, merged, aborted, used, attempts, born;
    double num;
};

// Per-system descriptor, resident in device memory. The first block is
// written by the host at admission / growth; the second block is updated by
// the finalize kernel every iteration.
struct SysDesc {
    // --- set by the host
    int32_t active, M, N, n_so;
    int32_t A, n_a, n_class, pad1;  // n_class: 2 x (largest irrep label + 1)
    double tau, zeta, e0, e_core, p_double, p_single;
    double inv_p_double, inv_p_single;   // 1/P_double, 1/P_single (0 when the type is impossible)
    // With no point group (two classes, the spins) every determinant has n_emp[s]
    // empty orbitals of spin s, and a double excitation's pgen is pgen_c1[s] (both
    // electrons of spin s) or pgen_c1[2 + s] (unlike spins, first hole of spin s);
    // 0 where the case cannot occur.
    double pgen_c1[4];
    int32_t n_emp[2];
    int64_t target;
    uint64_t seed, d0, valid;
    uint64_t cmask[NCLASS];
    uint64_t irr_packed[2];          // 4 bits per spatial orbital
    const double *h1, *eri;
    const double *jk;                // [n_so][64]: (pp|qq) - (pq|qp) for p < q, spin orbitals
    const double *t3;                // [n_so][64][64]: (pa|qq) - d(s_p,s_q)(pq|qa), same-spin p, a
    // Main list: nb buckets of BQ entries (structure of arrays); a determinant lives
    // in bucket floor(mix64(D) nb / 2^64), the entries of bucket b are the first
    // bcnt[b] of [b BQ, (b+1) BQ), every one occupied (the reference may sit at 0).
    uint64_t *key;                   // determinant
    int32_t *pop;                    // signed walker count
    double *hdiag;                   // stored H_DD
    int32_t *bcnt;                   // entries per bucket
    uint64_t cap;                    // nb * BQ
    int64_t nbuckets;                // nb
    int64_t nchunks, gchunk0;        // chunks (nb / BPC) of this system and the first global one
    int64_t stop_at;                 // iterate while iter < stop_at
    // Restricted space (FCIQMC_SPACE_* bits; children outside it are null excitations).
    int32_t space, max_ex, max_sen, pad2;
    uint64_t frz_occ, frz_emp;
    // Spin-coupled functions (Sec. 5.3): hphf = 0 (determinants), +1 / -1 (even / odd
    // total spin); lam = hphf (-1)^{N/2}, the relative sign of a pair's determinants.
    int32_t hphf, lam;
    // --- updated on the device
    int64_t iter;
    double shift;
    int32_t varying, pad3;
    int64_t n_prev, n_var;
    // --- set by the host: determinants of more than 64 spin orbitals (two words,
    // Sec. 3): the high words of d0, valid, cmask, frz_occ and frz_emp, and the irreps
    // of spatial orbitals 32-63 (4 bits each); det_words = 1 or 2 selects the width.
    uint64_t d0_hi, valid_hi;
    uint64_t cmask_hi[NCLASS];
    uint64_t irr_packed_hi[2];
    uint64_t frz_occ_hi, frz_emp_hi;
    int32_t det_words, pad5;
};

// A spawn record (16 B, written and read with one vector access): child
// determinant, signed walkers, and a tag word whose meaning depends on the buffer.
struct __attribute__((aligned(16))) SpawnRec {
    uint64_t det;
    int32_t w;
    uint32_t tag;
};

struct EngineArgs {
    SysDesc *desc;
    int32_t max_sys;
    int32_t tile;                    // attempts per spawn-kernel tile
    unsigned int *work;              // [0] next spawn tile, [1] next post chunk (reset per iteration)
    uint32_t *status;                // per system: ST_* bits (kept apart from the read-only
    unsigned long long *spawns;      // descriptors) and spawning events of the iteration
    const int32_t *chunk_sys;        // system of each global chunk (-1: unused)
    const int32_t *chunk_local;      // chunk index inside its system's table
    unsigned long long *chunk_nw;    // [2][chunk_cap] sum |C| per chunk: this iteration's
                                     // attempts in half (step & 1), the next one's in the other
    int64_t chunk_cap;
    unsigned long long *step;        // iterations run by this handle (selects the halves)
    unsigned long long *chunk_off;   // exclusive scan of chunk_nw
    unsigned long long *chunk_toff;  // exclusive scan of the spawn tiles of each chunk
    ChunkStat *chunk_stat;           // [chunks][POST_WAVES]
    unsigned long long *blk;         // [2][4][SCAN_G]: per chunk range sum |C|, tiles, and
                                     // their exclusive scans, halves selected like chunk_nw
    FinPart *fin_part;               // [max_sys][FIN_BLOCKS]
    int64_t *c0;                     // [max_sys] population on the reference after the iteration
    unsigned long long *total;       // [0] total attempts, [1] total spawn tiles
    const int64_t *nchunks;          // global chunks in use
    IterRecord *rec;                 // [max_sys][REC_CAP]
    uint32_t *tile_chunk;            // [tile_cap] chunk of each spawn tile (k_scan_down); tiles
    int64_t tile_cap;                // beyond the capacity are found by search
    // Spawn records of the iteration (the per-destination blocks of Sec. 4.1, with the
    // bucket as destination): appended by k_spawn with their rank among the bucket's
    // records, grouped by bucket by k_scatter.
    SpawnRec *recs;                  // [rec_cap] tag: global bucket | initiator flag << 31, or
                                     // the system | REC_UNRANKED for k_fix to place
    uint32_t *rec_rank;              // [rec_cap] rank among its bucket's records
    SpawnRec *srt;                   // [rec_cap] the records grouped by bucket; tag: bit 0
                                     // initiator flag, bits 1-2 k_post's round marks
    unsigned long long *rec_count;   // records appended this iteration
    int64_t rec_cap;
    uint32_t *bhist;                 // [BPC chunk_cap] records per bucket (zeroed by k_bscan_down)
    uint32_t *boff;                  // [BPC chunk_cap + 1] first sorted record of each bucket,
                                     // and the end of the last one
    long long *d0acc;                // [max_sys] walkers spawned onto the reference (kept out of
                                     // the records: the reference is the hot spot of Sec. 4.1)
    unsigned long long *boff_rg;     // [2 SCAN_G] records per range of buckets, their scan
    // New determinants that did not fit their bucket (completed, then re-bucketed by the host).
    uint64_t *sp_det;
    int32_t *sp_pop, *sp_sys;
    double *sp_hd;
    unsigned long long *sp_count;
    int64_t sp_cap;
    uint32_t *spilled;               // [max_sys] set by k_post when a bucket spilled
    // Every system of the launch draws plain determinants with no point group and no
    // restricted space: the spawning kernel is then launched in its variant that
    // leaves those cases out.
    int32_t plain;
};

// Staging area of the export that allocates nothing (fciqmc_walkers_noalloc): a
// 64-bit counter, then keys, populations and initiator flags of up to
// NOALLOC_MAX_DETS entries (32 MiB + 256 B).
constexpr int64_t NOALLOC_MAX_DETS = (int64_t)1 << 21;
constexpr size_t NOALLOC_KEYS_OFF = 256;
constexpr size_t NOALLOC_VALS_OFF = NOALLOC_KEYS_OFF + 8 * (size_t)NOALLOC_MAX_DETS;
constexpr size_t NOALLOC_FLAGS_OFF = NOALLOC_VALS_OFF + 4 * (size_t)NOALLOC_MAX_DETS;
constexpr size_t NOALLOC_BYTES = NOALLOC_FLAGS_OFF + 4 * (size_t)NOALLOC_MAX_DETS;

// Kernel launchers (kernels.hip, compiled once per determinant width: one word in fq,
// two words in fq::w2). Determinant arrays hold the width's words per entry.
constexpr int NKERN = 5;   // profiled kernel groups: chunk sums, scans, spawn, annihilation
                           // (record sort + death/annihilation pass), statistics/shift
#define FQ_WIDTH_LAUNCHERS                                                                     \
    /* first: the chunk sums are taken from the tables (the first iteration of a launch,     \
       after any host-side change); later iterations use the sums the previous iteration's   \
       k_post wrote. */                                                                       \
    void launch_iteration(const EngineArgs &a, int post_grid, int spawn_grid, bool first,      \
                          hipStream_t s, hipEvent_t *ev /* NKERN + 1 events or nullptr */);     \
    hipError_t launch_load(SysDesc *d_desc, int32_t sys, const uint64_t *det,                 \
                           const int32_t *pop, int64_t n, uint32_t *d_err, hipStream_t s);      \
    /* Move every entry of the buckets (src_*, src_nb buckets, counts src_cnt) and the spill  \
       entries of system sys into the descriptor's (empty) buckets. */                        \
    hipError_t launch_rebucket(SysDesc *d_desc, int32_t sys, const uint64_t *src_key,         \
                               const int32_t *src_pop, const double *src_hd,                  \
                               const int32_t *src_cnt, int64_t src_nb, const uint64_t *sp_det, \
                               const int32_t *sp_pop, const double *sp_hd,                    \
                               const int32_t *sp_sys, int64_t n_sp, uint32_t *d_err,          \
                               hipStream_t s);                                                 \
    hipError_t launch_compact(const uint64_t *key, const int32_t *pop, const int32_t *cnt,    \
                              int64_t nb, uint64_t *out_det, int32_t *out_pop,                \
                              unsigned long long *count, hipStream_t s);                      \
    /* H_DD (or the function's diagonal) of one determinant, words lo and hi. */              \
    hipError_t launch_e0(const SysDesc *desc, int32_t sys, uint64_t lo, uint64_t hi,          \
                         double *out, hipStream_t s);
FQ_WIDTH_LAUNCHERS
namespace w2 {
FQ_WIDTH_LAUNCHERS
}  // namespace w2
// Export into the staging area `stage` (NOALLOC layout): compaction of the occupied
// slots (entries past NOALLOC_MAX_DETS are counted, not written), then a bitonic
// sort by determinant of the first n entries padded to a power of two.
hipError_t launch_stage_compact(const uint64_t *key, const int32_t *pop, const int32_t *cnt,
                                int64_t nb, void *stage, hipStream_t s);
hipError_t launch_stage_sort(void *stage, int64_t n, hipStream_t s);
// Initiator flag of each of the n sorted entries: |pop| > n_a, or the reference.
hipError_t launch_stage_flags(void *stage, int64_t n, int32_t n_a, uint64_t d0, hipStream_t s);
int spawn_grid_size();
int post_grid_size();

}  // namespace fq
