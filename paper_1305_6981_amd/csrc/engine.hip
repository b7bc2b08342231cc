// Host engine of libfciqmc: the C ABI declared in include/fciqmc.h.
//
// A handle holds up to max_slots independent systems. Each system owns a main
// list in device memory, hash-partitioned into buckets of at most 1024 packed
// entries (structure of arrays: determinant, population, stored diagonal
// element, plus a count per bucket), its integrals, and a row of the device
// descriptor table. One iteration of every system is one pass of the kernels
// over the descriptor table; up to 64 iterations are captured in one HIP graph.
// Between launches the host reads the per-iteration records, feeds the
// estimator averages, and re-buckets a list whose buckets would fill up, or
// grows the spawn-record buffer. An iteration whose records overflowed the
// buffer is abandoned and re-run after growth (the counter-based random
// numbers make the re-run identical); new determinants that did not fit their
// bucket complete the iteration in a spill list and are re-bucketed before the
// system continues.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/fciqmc.h"
#include "engine.h"

using namespace fq;

// Determinants on the host: one 128-bit integer (bit p: spin orbital p occupied).
// The API and the device hold W = 1 or 2 64-bit words per determinant, low word
// first (Sec. 3: as many words as the spin orbitals need).
typedef unsigned __int128 hdet_t;
static inline int hpopc(hdet_t x) {
    return __builtin_popcountll((uint64_t)x) + __builtin_popcountll((uint64_t)(x >> 64));
}
static inline hdet_t hbit(int p) { return (hdet_t)1 << p; }
static inline uint64_t hlo(hdet_t x) { return (uint64_t)x; }
static inline uint64_t hhi(hdet_t x) { return (uint64_t)(x >> 64); }
static inline hdet_t hdet_in(const uint64_t *w, int W) {
    return W > 1 ? (((hdet_t)w[1] << 64) | (hdet_t)w[0]) : (hdet_t)w[0];
}
static inline void hdet_out(hdet_t d, uint64_t *w, int W) {
    w[0] = hlo(d);
    if (W > 1) w[1] = hhi(d);
}
static const hdet_t HEVEN = ((hdet_t)0x5555555555555555ull << 64) | (hdet_t)0x5555555555555555ull;
// Words per determinant for a system of n_orb spatial orbitals (det_words: 0 as needed,
// 2 forced).
static inline int words_for(int n_orb, int det_words) {
    return (2 * n_orb > 64 || det_words == 2) ? 2 : 1;
}
// The kernels' launchers of the handle's width.
#define FQ_LAUNCH(W, fn, ...) ((W) == 2 ? fq::w2::fn(__VA_ARGS__) : fq::fn(__VA_ARGS__))

// Device staging area of fciqmc_walkers_noalloc (every call on a GPU shares
// that GPU's copy). Host code never uses this name as an address: the address
// of each device's copy is taken once per device with hipGetSymbolAddress when
// the first handle on that device is created, and passed to the kernels.
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {

thread_local std::string g_err;

int set_err(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return set_err(FCIQMC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Main-list capacities: a multiple of 4 buckets, at least 4 buckets.
int64_t round_cap(int64_t x) {
    const int64_t q = 4 * CHUNK;
    return std::max<int64_t>(q, (x + q - 1) / q * q);
}

// Main-list capacity for `entries` entries at the planned mean bucket fill.
int64_t cap_for_entries(int64_t entries) {
    return round_cap((std::max<int64_t>(entries, 1) + BUCKET_FILL - 1) / BUCKET_FILL * BQ);
}

int64_t next_pow2(int64_t x) {
    int64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

// ---------------------------------------------------------------------------
// Error bars of correlated averages by blocking (Flyvbjerg & Petersen, the
// analysis of correlated ratios the paper's conclusions cite), kept online in
// O(log n) memory. Level 0 receives every sample (x, y); each completed pair at
// level l is averaged and passed to level l + 1, so level l sees the first
// floor(n / 2^l) block means. Per level the accumulators hold sums of the
// deviations from the level's first value (dx = x - x_first, ...): dx, dy,
// dx^2, dy^2 and dx dy, from which the level's means, variances of the mean and
// covariance follow. The error of the ratio <x>/<y> is the standard error of the
// linearised ratio estimator, sqrt(var(xbar - r ybar)) / ybar with r = xbar/ybar;
// a plain mean is the case y = 1. The level reported is the first one with at
// least 16 blocks whose error the next two levels (with >= 16 blocks) do not
// exceed by more than the error's own relative uncertainty 1/sqrt(2(n - 1));
// when none qualifies, the deepest level with >= 16 blocks.
// ---------------------------------------------------------------------------
class Blocker {
  public:
    void clear() { *this = Blocker(); }
    int64_t count() const { return lev_[0].n; }

    void add(double x, double y) {
        for (int l = 0; l < kLevels; ++l) {
            Level &L = lev_[l];
            if (L.n == 0) {
                L.x0 = x;
                L.y0 = y;
            }
            const double dx = x - L.x0, dy = y - L.y0;
            L.sx += dx;
            L.sy += dy;
            L.sxx += dx * dx;
            L.syy += dy * dy;
            L.sxy += dx * dy;
            L.n += 1;
            if (!L.pending) {
                L.pending = true;
                L.px = x;
                L.py = y;
                return;
            }
            L.pending = false;
            x = (L.px + x) * 0.5;
            y = (L.py + y) * 0.5;
        }
    }

    // Mean of x / mean of y over all samples, and its error bar (NaN when no
    // level has 16 blocks).
    void result(double &mean, double &err) const {
        mean = NAN;
        err = NAN;
        const Level &L0 = lev_[0];
        if (L0.n == 0) return;
        mean = (L0.x0 + L0.sx / (double)L0.n) / (L0.y0 + L0.sy / (double)L0.n);
        double e[kLevels];
        int top = 0;   // levels with >= 16 blocks: 0 .. top-1
        while (top < kLevels && lev_[top].n >= 16) {
            e[top] = level_error(lev_[top]);
            ++top;
        }
        if (top == 0) return;
        int pick = top - 1;
        for (int l = 0; l < top; ++l) {
            const double allow = e[l] * (1.0 + 1.0 / std::sqrt(2.0 * (double)(lev_[l].n - 1)));
            const bool next_ok = l + 1 >= top || e[l + 1] <= allow;
            const bool next2_ok = l + 2 >= top || e[l + 2] <= allow;
            if (next_ok && next2_ok) {
                pick = l;
                break;
            }
        }
        err = e[pick];
    }

  private:
    static constexpr int kLevels = 64;
    struct Level {
        int64_t n = 0;
        double x0 = 0, y0 = 0, sx = 0, sy = 0, sxx = 0, syy = 0, sxy = 0;
        bool pending = false;
        double px = 0, py = 0;
    };
    static double level_error(const Level &L) {
        const double n = (double)L.n;
        const double norm = n * (n - 1.0);
        const double vx = (L.sxx - L.sx * L.sx / n) / norm;
        const double vy = (L.syy - L.sy * L.sy / n) / norm;
        const double cxy = (L.sxy - L.sx * L.sy / n) / norm;
        const double xbar = L.x0 + L.sx / n, ybar = L.y0 + L.sy / n;
        const double r = xbar / ybar;
        const double v = (vx - 2.0 * r * cxy + r * r * vy) / (ybar * ybar);
        return std::sqrt(v > 0.0 ? v : 0.0);
    }
    Level lev_[kLevels];
};

struct SysHost {
    bool active = false;
    fciqmc_params prm{};
    int M = 0, N = 0, na = 0, nb = 0;
    std::vector<double> h1, eri;
    std::vector<uint8_t> irrep;
    double e_core = 0.0, p_double = 0.0, e0 = 0.0;
    hdet_t d0 = 0;
    int W = 1;                 // 64-bit words per determinant
    int64_t cap = 0;           // main-list capacity: buckets * BQ
    void *block = nullptr;     // one device allocation for the main list + integrals
    uint64_t *key = nullptr;   // W words per entry
    int32_t *pop = nullptr;
    double *hd = nullptr;
    int32_t *bcnt = nullptr;
    double *d_h1 = nullptr, *d_eri = nullptr, *d_jk = nullptr;
    std::vector<double> jk;    // [n_so][64 W] pair table
    std::vector<double> t3;    // [n_so][64 W][64 W] single-excitation term table
    double *d_t3 = nullptr;
    int64_t growth = 0;        // expected per-iteration increase of the entries
    int64_t spawn_peak = 0;    // most spawn records of one iteration in the last launch
    double spawn_rate = 1.0;   // largest ratio of consecutive iterations' records
    int64_t reserve_bytes = 0; // admission accounting (target footprint)
    // mirrored dynamics and statistics
    IterRecord last{};
    int64_t tot_att = 0, tot_sp = 0;
    int64_t redos = 0;         // iterations re-run after the record buffer overflowed
    int64_t spills = 0;        // iterations whose new determinants overflowed a bucket
    Blocker e_blk, s_blk;      // (num, C_0) and (S, 1) samples of the averaging window
    int fatal = 0;
};

}  // namespace

struct fciqmc_t {
    int dev = 0;
    int W = 1;                              // words per determinant of every system here
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int max_sys = 0;
    std::vector<SysHost> sys;
    std::vector<SysDesc> hdesc;
    SysDesc *d_desc = nullptr;
    IterRecord *d_rec = nullptr;            // per-iteration records: pinned host memory that
    IterRecord *h_rec = nullptr;            // k_finalize writes through d_rec, read as h_rec
    uint32_t *d_status = nullptr;           // per system ST_* bits (device)
    unsigned int *d_work = nullptr;         // dynamic work counters
    unsigned long long *d_spawns = nullptr; // per system spawn counter (device)
    std::vector<uint32_t> hstatus;          // host mirror of d_status
    std::vector<IterRecord> hrec;
    // global chunk layout
    int64_t chunk_alloc = 0, n_chunks = 0;
    int32_t *d_chunk_sys = nullptr, *d_chunk_local = nullptr;
    unsigned long long *d_chunk_nw = nullptr, *d_chunk_off = nullptr, *d_total = nullptr;
    unsigned long long *d_chunk_toff = nullptr;
    ChunkStat *d_chunk_stat = nullptr;
    uint32_t *d_tile_chunk = nullptr;       // chunk of each spawn tile
    bool tile_map_off = false;              // its allocation failed once: search instead
    void *d_stage = nullptr;                // this device's staging area (not owned)
    // spawn records (see EngineArgs) and the spill list
    void *d_recs = nullptr;
    int64_t rec_cap = 0;
    unsigned long long *d_rec_count = nullptr;
    uint32_t *d_bhist = nullptr, *d_boff = nullptr;
    long long *d_d0acc = nullptr;
    unsigned long long *d_boff_rg = nullptr;
    void *d_spill = nullptr;
    int64_t sp_cap = 0;
    unsigned long long *d_sp_count = nullptr;
    uint32_t *d_spilled = nullptr;
    int64_t tile_cap = 0;
    unsigned long long *d_blk = nullptr;    // [2][4][SCAN_G] range sums and scans
    unsigned long long *d_step = nullptr;   // iterations run (selects the halves of the sums)
    FinPart *d_fin = nullptr;               // [max_sys][FIN_BLOCKS]
    int64_t *d_c0 = nullptr;                // [max_sys]
    int64_t *d_nchunks = nullptr;
    uint32_t *d_err = nullptr;
    int spawn_grid = 2048;
    int post_grid = 1024;
    int tile = 2048;
    std::map<int, hipGraphExec_t> graphs;   // by 2 L + plain (L iterations, kernel variant)
    bool use_graph = true;
    bool profiling = false;
    hipEvent_t ev[NKERN + 1] = {};
    double kms[NKERN] = {};
    int64_t kcount[NKERN] = {};
    double phase_ms[NKERN] = {};            // kernel groups of the last sampled iteration
    double ms_last = 0.0;
    bool planner = true;                    // size tables before each launch (test knob)
    int64_t tile_map_limit = -1;            // cap on the tile map (test knob; -1: none)
};

namespace {

void drop_graphs(fciqmc_t *h) {
    for (auto &kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
    h->graphs.clear();
}

EngineArgs make_args(fciqmc_t *h) {
    EngineArgs a{};
    a.desc = h->d_desc;
    a.max_sys = h->max_sys;
    a.chunk_sys = h->d_chunk_sys;
    a.chunk_local = h->d_chunk_local;
    a.chunk_nw = h->d_chunk_nw;
    a.chunk_cap = h->chunk_alloc;
    a.step = h->d_step;
    a.chunk_off = h->d_chunk_off;
    a.chunk_toff = h->d_chunk_toff;
    a.chunk_stat = h->d_chunk_stat;
    a.blk = h->d_blk;
    a.fin_part = h->d_fin;
    a.c0 = h->d_c0;
    a.total = h->d_total;
    a.nchunks = h->d_nchunks;
    a.rec = h->d_rec;
    a.tile = h->tile;
    a.status = h->d_status;
    a.spawns = h->d_spawns;
    a.work = h->d_work;
    a.tile_chunk = h->d_tile_chunk;
    a.tile_cap = h->tile_cap;
    char *r = (char *)h->d_recs;
    const size_t rc = (size_t)h->rec_cap;
    const size_t rb = 16 * (size_t)h->W;     // bytes per record
    a.recs = (SpawnRec *)r;
    a.srt = (SpawnRec *)(r + rb * rc);
    a.rec_rank = (uint32_t *)(r + 2 * rb * rc);
    a.rec_count = h->d_rec_count;
    a.rec_cap = h->rec_cap;
    a.bhist = h->d_bhist;
    a.d0acc = h->d_d0acc;
    a.boff = h->d_boff;
    a.boff_rg = h->d_boff_rg;
    char *q = (char *)h->d_spill;
    const size_t sc = (size_t)h->sp_cap;
    const size_t kb = 8 * (size_t)h->W;      // bytes per determinant
    a.sp_det = (uint64_t *)q;
    a.sp_hd = (double *)(q + kb * sc);
    a.sp_pop = (int32_t *)(q + (kb + 8) * sc);
    a.sp_sys = (int32_t *)(q + (kb + 12) * sc);
    a.sp_count = h->d_sp_count;
    a.sp_cap = h->sp_cap;
    a.spilled = h->d_spilled;
    a.plain = 1;
    for (int s = 0; s < h->max_sys; ++s) {
        const SysDesc &d = h->hdesc[s];
        if (h->sys[s].active && (d.n_class != 2 || d.hphf || d.space)) a.plain = 0;
    }
    return a;
}

// The spawn-record buffer for `cap` records (32 W + 4 B each: unsorted, sorted, rank).
int ensure_records(fciqmc_t *h, int64_t cap) {
    if (cap <= h->rec_cap) return 0;
    HIP_TRY(hipStreamSynchronize(h->stream));
    hipFree(h->d_recs);
    h->d_recs = nullptr;
    h->rec_cap = 0;
    drop_graphs(h);
    if (hipMalloc(&h->d_recs, (size_t)cap * (32 * h->W + 4)) != hipSuccess) {
        (void)hipGetLastError();
        return set_err(FCIQMC_ENOMEM, "spawn-record buffer of " + std::to_string(cap) +
                                          " records does not fit in device memory");
    }
    h->rec_cap = cap;
    return 0;
}

int upload_desc(fciqmc_t *h) {
    HIP_TRY(hipMemcpyAsync(h->d_desc, h->hdesc.data(), sizeof(SysDesc) * h->max_sys,
                           hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipMemcpyAsync(h->d_status, h->hstatus.data(), sizeof(uint32_t) * h->max_sys,
                           hipMemcpyHostToDevice, h->stream));
    return 0;
}

int download_desc(fciqmc_t *h) {
    HIP_TRY(hipMemcpyAsync(h->hdesc.data(), h->d_desc, sizeof(SysDesc) * h->max_sys,
                           hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipMemcpyAsync(h->hstatus.data(), h->d_status, sizeof(uint32_t) * h->max_sys,
                           hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return 0;
}

// Clear what spawning accumulates for system s outside the records (its event
// count and its walkers onto the reference): after an abandoned iteration or a load.
int reset_spawns(fciqmc_t *h, int s) {
    HIP_TRY(hipMemsetAsync(h->d_spawns + s, 0, sizeof(unsigned long long), h->stream));
    HIP_TRY(hipMemsetAsync(h->d_d0acc + s, 0, sizeof(long long), h->stream));
    return 0;
}

// Lay the chunks of all active systems out contiguously.
int relayout(fciqmc_t *h) {
    int64_t total = 0;
    for (int s = 0; s < h->max_sys; ++s)
        if (h->sys[s].active) total += h->sys[s].cap / CHUNK;
    if (total > h->chunk_alloc) {
        int64_t na = next_pow2(std::max<int64_t>(total, 64));
        hipFree(h->d_chunk_sys);
        hipFree(h->d_chunk_local);
        hipFree(h->d_chunk_nw);
        hipFree(h->d_chunk_off);
        hipFree(h->d_chunk_toff);
        hipFree(h->d_chunk_stat);
        hipFree(h->d_bhist);
        hipFree(h->d_boff);
        h->d_chunk_sys = nullptr;
        h->chunk_alloc = 0;
        HIP_TRY(hipMalloc(&h->d_chunk_sys, na * sizeof(int32_t)));
        HIP_TRY(hipMalloc(&h->d_chunk_local, na * sizeof(int32_t)));
        HIP_TRY(hipMalloc(&h->d_chunk_nw, 2 * na * sizeof(unsigned long long)));
        HIP_TRY(hipMalloc(&h->d_chunk_off, na * sizeof(unsigned long long)));
        HIP_TRY(hipMalloc(&h->d_chunk_toff, na * sizeof(unsigned long long)));
        HIP_TRY(hipMalloc(&h->d_chunk_stat, na * POST_WAVES * sizeof(ChunkStat)));
        HIP_TRY(hipMalloc(&h->d_bhist, BPC * na * sizeof(uint32_t)));
        HIP_TRY(hipMalloc(&h->d_boff, (BPC * na + 1) * sizeof(uint32_t)));
        h->chunk_alloc = na;
        drop_graphs(h);
    }
    // record counts start at zero (the record scan keeps them so after every iteration)
    HIP_TRY(hipMemsetAsync(h->d_bhist, 0, BPC * h->chunk_alloc * sizeof(uint32_t), h->stream));
    std::vector<int32_t> cs(total), cl(total);
    int64_t g = 0;
    for (int s = 0; s < h->max_sys; ++s) {
        SysDesc &d = h->hdesc[s];
        if (!h->sys[s].active) {
            d.gchunk0 = 0;
            d.nchunks = 0;
            d.nbuckets = 0;
            continue;
        }
        const int64_t nc = h->sys[s].cap / CHUNK;
        d.gchunk0 = g;
        d.nchunks = nc;
        d.nbuckets = h->sys[s].cap / BQ;
        for (int64_t c = 0; c < nc; ++c) {
            cs[g + c] = s;
            cl[g + c] = (int32_t)c;
        }
        g += nc;
    }
    h->n_chunks = total;
    if (total > 0) {
        HIP_TRY(hipMemcpyAsync(h->d_chunk_sys, cs.data(), total * sizeof(int32_t),
                               hipMemcpyHostToDevice, h->stream));
        HIP_TRY(hipMemcpyAsync(h->d_chunk_local, cl.data(), total * sizeof(int32_t),
                               hipMemcpyHostToDevice, h->stream));
    }
    HIP_TRY(hipMemcpyAsync(h->d_nchunks, &h->n_chunks, sizeof(int64_t), hipMemcpyHostToDevice,
                           h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return 0;
}

// The tile -> chunk map: room for every chunk's first tile and for twice the
// walkers of the last iteration in whole tiles, grown by doubling (a graph holds
// the pointer, so growing drops the graphs). Tiles beyond it are found by search.
int ensure_tile_map(fciqmc_t *h) {
    int64_t walkers = 0;
    for (int s = 0; s < h->max_sys; ++s)
        if (h->sys[s].active) walkers += std::max<int64_t>(h->sys[s].last.nw, 0);
    int64_t want = h->n_chunks + 2 * walkers / std::max(h->tile, 1) + 65536;
    if (h->tile_map_limit >= 0) want = std::min<int64_t>(want, h->tile_map_limit);
    if (want <= h->tile_cap || h->tile_map_off) return 0;
    int64_t cap = std::max<int64_t>(want, 2 * h->tile_cap);
    if (h->tile_map_limit >= 0) cap = std::min<int64_t>(cap, h->tile_map_limit);
    HIP_TRY(hipStreamSynchronize(h->stream));
    hipFree(h->d_tile_chunk);
    h->d_tile_chunk = nullptr;
    h->tile_cap = 0;
    drop_graphs(h);
    if (hipMalloc(&h->d_tile_chunk, cap * sizeof(uint32_t)) != hipSuccess) {
        (void)hipGetLastError();   // no room: every tile grab searches instead
        h->d_tile_chunk = nullptr;
        h->tile_map_off = true;
        return 0;
    }
    h->tile_cap = cap;
    return 0;
}

// Device bytes of a main list of cap entries: determinant (W words), population,
// H_DD per entry, and one count per bucket.
int64_t table_bytes(int64_t cap, int W) {
    return cap * (int64_t)(8 * W + sizeof(int32_t) + sizeof(double)) +
           (cap / BQ) * (int64_t)sizeof(int32_t) + 256;
}

// h1, the packed ERI, the pair table and the single-excitation term table, with
// rows of 64 W spin orbitals.
int64_t integral_doubles(int M, int W) {
    const int64_t np = (int64_t)M * (M + 1) / 2, ns = 64 * (int64_t)W;
    return (int64_t)M * M + np * (np + 1) / 2 + ns * ns + (int64_t)2 * M * ns * ns;
}

int64_t integral_bytes(int M, int W) { return integral_doubles(M, W) * 8 + 256; }

void carve(SysHost &S, void *blk, int64_t cap) {
    char *p = (char *)blk;
    S.key = (uint64_t *)p;
    p += cap * 8 * S.W;
    S.hd = (double *)p;
    p += cap * sizeof(double);
    S.pop = (int32_t *)p;
    p += cap * sizeof(int32_t);
    S.bcnt = (int32_t *)p;
    p += (cap / BQ) * sizeof(int32_t);
    p = (char *)(((uintptr_t)p + 255) & ~(uintptr_t)255);
    S.d_h1 = (double *)p;
    p += (size_t)S.M * S.M * sizeof(double);
    S.d_eri = (double *)p;
    p += (size_t)S.eri.size() * sizeof(double);
    S.d_jk = (double *)p;
    p += (size_t)64 * S.W * 64 * S.W * sizeof(double);
    S.d_t3 = (double *)p;
    S.block = blk;
    S.cap = cap;
}

// Allocate the main list of a system with cap entries (every bucket empty) and
// room for its integrals. Old storage is released by the caller.
int alloc_tables(fciqmc_t *h, SysHost &S, int64_t cap, void **block_out) {
    const int64_t tb = table_bytes(cap, S.W), ib = integral_bytes(S.M, S.W);
    void *blk = nullptr;
    hipError_t e = hipMalloc(&blk, (size_t)(tb + ib));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_err(FCIQMC_ENOMEM, "device allocation of " + std::to_string(tb + ib) +
                                          " bytes failed: " + hipGetErrorString(e));
    }
    SysHost T = S;
    carve(T, blk, cap);
    HIP_TRY(hipMemsetAsync(T.bcnt, 0, (size_t)(cap / BQ) * sizeof(int32_t), h->stream));
    *block_out = blk;
    return 0;
}

int upload_integrals(fciqmc_t *h, SysHost &S) {
    HIP_TRY(hipMemcpyAsync(S.d_h1, S.h1.data(), S.h1.size() * 8, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipMemcpyAsync(S.d_eri, S.eri.data(), S.eri.size() * 8, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipMemcpyAsync(S.d_jk, S.jk.data(), S.jk.size() * 8, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipMemcpyAsync(S.d_t3, S.t3.data(), S.t3.size() * 8, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return 0;
}

void fill_desc_tables(fciqmc_t *h, int s) {
    SysHost &S = h->sys[s];
    SysDesc &d = h->hdesc[s];
    d.key = S.key;
    d.pop = S.pop;
    d.hdiag = S.hd;
    d.bcnt = S.bcnt;
    d.h1 = S.d_h1;
    d.eri = S.d_eri;
    d.jk = S.d_jk;
    d.t3 = S.d_t3;
    d.cap = (uint64_t)S.cap;
    d.nbuckets = S.cap / BQ;
}

// Move the main list of system s (and any of its entries waiting in the spill
// list) into new_cap entries' worth of buckets, in a new allocation.
int rebucket_system(fciqmc_t *h, int s, int64_t new_cap, int64_t n_spill) {
    SysHost &S = h->sys[s];
    for (int attempt = 0;; ++attempt) {
        void *blk = nullptr;
        int rc = alloc_tables(h, S, new_cap, &blk);
        if (rc) return rc == FCIQMC_ENOMEM ? FCIQMC_ECAPACITY : rc;
        SysHost T = S;
        carve(T, blk, new_cap);
        // the integrals (same layout after the list) move device to device
        const size_t ib = (size_t)((const char *)(S.d_t3 + S.t3.size()) - (const char *)S.d_h1);
        HIP_TRY(hipMemcpyAsync(T.d_h1, S.d_h1, ib, hipMemcpyDeviceToDevice, h->stream));
        // the kernel reads the destination from the descriptor
        SysDesc keep = h->hdesc[s];
        SysHost S_old = S;
        carve(S, blk, new_cap);
        fill_desc_tables(h, s);
        h->hdesc[s].nchunks = new_cap / CHUNK;
        h->hdesc[s].nbuckets = new_cap / BQ;
        rc = upload_desc(h);
        if (rc) return rc;
        HIP_TRY(hipMemsetAsync(h->d_err, 0, sizeof(uint32_t), h->stream));
        const EngineArgs a = make_args(h);
        HIP_TRY(FQ_LAUNCH(h->W, launch_rebucket, h->d_desc, s, S_old.key, S_old.pop, S_old.hd,
                          S_old.bcnt, S_old.cap / BQ, a.sp_det, a.sp_pop, a.sp_hd, a.sp_sys,
                          n_spill, h->d_err, h->stream));
        uint32_t err = 0;
        HIP_TRY(hipMemcpyAsync(&err, h->d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        if (!err) {
            HIP_TRY(hipFree(S_old.block));
            S.last.used = std::max<int64_t>(S.last.used, S.last.nd + 1);
            rc = relayout(h);
            if (rc) return rc;
            return upload_desc(h);
        }
        // a bucket overflowed (far beyond the planned fill): back out, try twice the buckets
        HIP_TRY(hipFree(blk));
        S = S_old;
        h->hdesc[s] = keep;
        fill_desc_tables(h, s);
        rc = upload_desc(h);
        if (rc) return rc;
        if (attempt >= 4) return set_err(FCIQMC_ECAPACITY, "re-bucketing the main list failed");
        new_cap *= 2;
    }
}

hdet_t aufbau(const std::vector<double> &h1, int M, int na, int nb) {
    std::vector<int> order(M);
    for (int i = 0; i < M; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return h1[a * M + a] < h1[b * M + b]; });
    hdet_t d = 0;
    for (int i = 0; i < na; ++i) d |= hbit(2 * order[i]);
    for (int i = 0; i < nb; ++i) d |= hbit(2 * order[i] + 1);
    return d;
}

// Numbers of symmetry-allowed singles and doubles from det, counted per class.
void excitation_counts(const SysHost &S, hdet_t det, int64_t &ns, int64_t &nd) {
    const int nso = 2 * S.M;
    int n_occ[NCLASS] = {0}, n_emp[NCLASS] = {0};
    auto cls = [&](int p) { return 2 * (int)S.irrep[p >> 1] + (p & 1); };
    for (int p = 0; p < nso; ++p) ((det >> p) & 1 ? n_occ : n_emp)[cls(p)]++;
    ns = 0;
    for (int c = 0; c < NCLASS; ++c) ns += (int64_t)n_occ[c] * n_emp[c];
    nd = 0;
    std::vector<int> occ;
    for (int p = 0; p < nso; ++p)
        if ((det >> p) & 1) occ.push_back(p);
    for (size_t i = 0; i < occ.size(); ++i)
        for (size_t j = i + 1; j < occ.size(); ++j) {
            const int p = occ[i], q = occ[j];
            const int g = S.irrep[p >> 1] ^ S.irrep[q >> 1];
            if ((p & 1) == (q & 1)) {
                const int sp = p & 1;
                for (int ga = 0; ga < 8; ++ga) {
                    const int gb = ga ^ g;
                    if (gb < ga) continue;
                    const int na_ = n_emp[2 * ga + sp], nb_ = n_emp[2 * gb + sp];
                    nd += (ga == gb) ? (int64_t)na_ * (na_ - 1) / 2 : (int64_t)na_ * nb_;
                }
            } else {
                for (int ga = 0; ga < 8; ++ga)
                    nd += (int64_t)n_emp[2 * ga + 0] * n_emp[2 * (ga ^ g) + 1];
            }
        }
}

int validate(const fciqmc_hamiltonian *ham, const fciqmc_params *prm) {
    if (!ham || !prm) return set_err(FCIQMC_EINVAL, "null hamiltonian or params");
    if (ham->n_orb < 1 || ham->n_orb > 64)
        return set_err(FCIQMC_EINVAL, "n_orb must be in 1..64 (2*n_orb <= 128)");
    if (prm->det_words < 0 || prm->det_words > 2 || (prm->det_words == 1 && 2 * ham->n_orb > 64))
        return set_err(FCIQMC_EINVAL, "det_words must be 0, 1 (at most 64 spin orbitals) or 2");
    if (ham->n_alpha < 0 || ham->n_beta < 0 || ham->n_alpha > ham->n_orb ||
        ham->n_beta > ham->n_orb || ham->n_alpha + ham->n_beta == 0)
        return set_err(FCIQMC_EINVAL, "bad electron counts");
    if (!ham->h1 || !ham->eri) return set_err(FCIQMC_EINVAL, "missing integrals");
    if (!(prm->tau > 0.0)) return set_err(FCIQMC_EINVAL, "tau must be positive");
    if (prm->shift_update_every < 1) return set_err(FCIQMC_EINVAL, "shift_update_every must be >= 1");
    if (ham->p_double > 1.0) return set_err(FCIQMC_EINVAL, "p_double > 1");
    if (prm->initial_walkers < 0 || prm->initial_walkers > 2147483647)
        return set_err(FCIQMC_EINVAL, "initial_walkers out of range");
    if (ham->orb_irrep)
        for (int i = 0; i < ham->n_orb; ++i)
            if (ham->orb_irrep[i] > 7) return set_err(FCIQMC_EINVAL, "irrep labels must be 0..7");
    if (prm->space & ~(FCIQMC_SPACE_EXCITATION | FCIQMC_SPACE_SENIORITY | FCIQMC_SPACE_FROZEN))
        return set_err(FCIQMC_EINVAL, "unknown space restriction");
    if (((prm->space & FCIQMC_SPACE_EXCITATION) && prm->max_excitation < 0) ||
        ((prm->space & FCIQMC_SPACE_SENIORITY) && prm->max_seniority < 0) ||
        ((prm->space & FCIQMC_SPACE_FROZEN) &&
         ((prm->frozen_occupied & prm->frozen_empty) ||
          (prm->frozen_occupied_hi & prm->frozen_empty_hi))))
        return set_err(FCIQMC_EINVAL, "inconsistent space restriction");
    if (prm->hphf != 0 && prm->hphf != 1 && prm->hphf != -1)
        return set_err(FCIQMC_EINVAL, "hphf must be 0, 1 or -1");
    if (prm->hphf && ham->n_alpha != ham->n_beta)
        return set_err(FCIQMC_EINVAL, "spin-coupled functions need n_alpha = n_beta");
    if (prm->hphf && prm->space)
        return set_err(FCIQMC_EINVAL, "spin-coupled functions with a restricted space are not supported");
    return 0;
}

hdet_t host_spin_flip(hdet_t D) { return ((D & HEVEN) << 1) | ((D >> 1) & HEVEN); }

// Whether det lies in the run's restricted space (host check of the reference).
bool host_in_space(const fciqmc_params *prm, hdet_t d0, hdet_t det) {
    if ((prm->space & FCIQMC_SPACE_EXCITATION) && hpopc(det & ~d0) > prm->max_excitation)
        return false;
    if ((prm->space & FCIQMC_SPACE_SENIORITY) && hpopc((det ^ (det >> 1)) & HEVEN) > prm->max_seniority)
        return false;
    const hdet_t fo = ((hdet_t)prm->frozen_occupied_hi << 64) | (hdet_t)prm->frozen_occupied;
    const hdet_t fe = ((hdet_t)prm->frozen_empty_hi << 64) | (hdet_t)prm->frozen_empty;
    if ((prm->space & FCIQMC_SPACE_FROZEN) && ((det & fo) != fo || (det & fe))) return false;
    return true;
}

int64_t initial_capacity(const fciqmc_params *prm) {
    return prm->det_capacity > 0 ? round_cap(prm->det_capacity)
                                 : cap_for_entries(4 * std::max<int64_t>(prm->initial_walkers, 1024));
}

// Device bytes reserved for a system at its walker target: a main list of twice
// the target in entries, and its integrals.
int64_t target_footprint(const fciqmc_hamiltonian *ham, const fciqmc_params *prm) {
    const int64_t cap = round_cap(2 * std::max<int64_t>(prm->target_walkers, 1));
    const int W = words_for(ham->n_orb, prm->det_words);
    return table_bytes(cap, W) + integral_bytes(ham->n_orb, W);
}

int load_list(fciqmc_t *h, int s, const std::vector<hdet_t> &det, const std::vector<int32_t> &pop);

// Admit a system into slot s (slot must be free).
int admit(fciqmc_t *h, int s, const fciqmc_hamiltonian *ham, const fciqmc_params *prm) {
    int rc = validate(ham, prm);
    if (rc) return rc;
    SysHost &S = h->sys[s];
    S = SysHost();
    S.prm = *prm;
    S.M = ham->n_orb;
    S.na = ham->n_alpha;
    S.nb = ham->n_beta;
    S.N = S.na + S.nb;
    S.e_core = ham->e_core;
    S.h1.assign(ham->h1, ham->h1 + (size_t)S.M * S.M);
    const int64_t np = (int64_t)S.M * (S.M + 1) / 2;
    S.eri.assign(ham->eri, ham->eri + np * (np + 1) / 2);
    S.irrep.assign(S.M, 0);
    if (ham->orb_irrep) S.irrep.assign(ham->orb_irrep, ham->orb_irrep + S.M);
    const int nso = 2 * S.M;
    S.W = words_for(S.M, prm->det_words);
    if (S.W != h->W)
        return set_err(FCIQMC_EINVAL, "a batch holds determinants of one width: this system takes " +
                                          std::to_string(S.W) + " 64-bit words, the batch " +
                                          std::to_string(h->W));
    const hdet_t valid = nso == 128 ? ~(hdet_t)0 : (hbit(nso) - 1);
    if (ham->ref_det) {
        S.d0 = hdet_in(ham->ref_det, S.W);
        int a = 0, b = 0;
        for (int p = 0; p < 128; ++p)
            if ((S.d0 >> p) & 1) (p & 1 ? b : a)++;
        if ((S.d0 & ~valid) || a != S.na || b != S.nb)
            return set_err(FCIQMC_EINVAL, "reference determinant does not match the electron counts");
    } else {
        S.d0 = aufbau(S.h1, S.M, S.na, S.nb);
    }
    if (!host_in_space(prm, S.d0, S.d0))
        return set_err(FCIQMC_EINVAL, "the reference lies outside the restricted space");
    if (ham->p_double >= 0.0) {
        S.p_double = ham->p_double;
    } else {
        int64_t ns, nd;
        excitation_counts(S, S.d0, ns, nd);
        S.p_double = (ns + nd) > 0 ? (double)nd / (double)(ns + nd) : 0.0;
    }
    if (prm->hphf) {   // the reference function, stored as the smaller determinant of its pair
        const hdet_t f = host_spin_flip(S.d0);
        if (f == S.d0 && prm->hphf < 0)
            return set_err(FCIQMC_EINVAL, "a closed-shell reference has no odd-spin function");
        S.d0 = std::min(S.d0, f);
    }
    S.reserve_bytes = target_footprint(ham, prm);
    // free-memory admission
    size_t fr = 0, tot = 0;
    HIP_TRY(hipMemGetInfo(&fr, &tot));
    int64_t reserved = 0;
    for (int t = 0; t < h->max_sys; ++t)
        if (t != s && h->sys[t].active)
            reserved += std::max<int64_t>(0, h->sys[t].reserve_bytes - table_bytes(h->sys[t].cap, h->W));
    const int64_t need = S.reserve_bytes;
    if ((int64_t)fr - reserved < need + (int64_t)(1ull << 30))
        return set_err(FCIQMC_ENOMEM, "system footprint " + std::to_string(need) +
                                          " B does not fit in free device memory");
    // Pair table for the diagonal elements: (pp|qq) - (pq|qp) over spin orbitals p < q,
    // rows of ns = 64 W entries.
    const int ns = 64 * S.W;
    S.jk.assign((size_t)ns * ns, 0.0);
    auto eri_sp = [&](int i, int j, int k, int l) {
        auto tri = [](int x, int y) { return x >= y ? (int64_t)x * (x + 1) / 2 + y : (int64_t)y * (y + 1) / 2 + x; };
        const int64_t a = tri(i, j), b = tri(k, l);
        return S.eri[a >= b ? a * (a + 1) / 2 + b : b * (b + 1) / 2 + a];
    };
    for (int p = 0; p < nso; ++p)
        for (int q = p + 1; q < nso; ++q) {
            const double coul = eri_sp(p >> 1, p >> 1, q >> 1, q >> 1);
            const double exch = ((p ^ q) & 1) ? 0.0 : eri_sp(p >> 1, q >> 1, q >> 1, p >> 1);
            S.jk[(size_t)p * ns + q] = coul - exch;
        }
    // Single-excitation terms: for p -> a (same spin) and each spectator q,
    // (pa|qq) - [same spin](pq|qa), the difference the Slater-Condon sum adds.
    S.t3.assign((size_t)nso * ns * ns, 0.0);
    for (int p = 0; p < nso; ++p)
        for (int a = 0; a < nso; ++a) {
            if ((p ^ a) & 1) continue;
            for (int q = 0; q < nso; ++q) {
                const double coul = eri_sp(p >> 1, a >> 1, q >> 1, q >> 1);
                const double exch = ((p ^ q) & 1) ? 0.0 : eri_sp(p >> 1, q >> 1, q >> 1, a >> 1);
                S.t3[((size_t)p * ns + a) * ns + q] = coul - exch;
            }
        }
    const int64_t cap = initial_capacity(prm);
    void *blk = nullptr;
    rc = alloc_tables(h, S, cap, &blk);
    if (rc) return rc;
    carve(S, blk, cap);
    rc = upload_integrals(h, S);
    if (rc) return rc;
    S.growth = cap / 16;
    S.active = true;
    SysDesc &d = h->hdesc[s];
    std::memset(&d, 0, sizeof d);
    d.active = 1;
    d.M = S.M;
    d.N = S.N;
    d.n_so = nso;
    {
        int mx = 0;
        for (int i = 0; i < S.M; ++i) mx = std::max<int>(mx, S.irrep[i]);
        d.n_class = 2 * (mx + 1);
    }
    d.A = prm->shift_update_every;
    d.n_a = prm->initiator_threshold;
    d.tau = prm->tau;
    d.zeta = prm->shift_damping;
    d.e_core = S.e_core;
    d.p_double = S.p_double;
    d.p_single = 1.0 - S.p_double;
    d.inv_p_double = d.p_double > 0.0 ? 1.0 / d.p_double : 0.0;
    d.inv_p_single = d.p_single > 0.0 ? 1.0 / d.p_single : 0.0;
    {
        // pgen of a double excitation without a point group, by the same operations
        // as the general branch of the kernels' excitation generator
        const int ne[2] = {S.M - hpopc(S.d0 & HEVEN), S.M - hpopc(S.d0 & (HEVEN << 1))};
        d.n_emp[0] = ne[0];
        d.n_emp[1] = ne[1];
        auto pg = [&](int nba, int nbb, int nal) {
            return (2.0 * d.p_double * (1.0 / (double)nba + 1.0 / (double)nbb)) /
                   (double)((int64_t)S.N * (int64_t)(S.N - 1) * (int64_t)nal);
        };
        const int nal_u = (ne[1] > 0 ? ne[0] : 0) + (ne[0] > 0 ? ne[1] : 0);
        for (int sp = 0; sp < 2; ++sp) {
            d.pgen_c1[sp] = ne[sp] >= 2 && S.N >= 2 ? pg(ne[sp] - 1, ne[sp] - 1, ne[sp]) : 0.0;
            d.pgen_c1[2 + sp] =
                ne[sp] > 0 && ne[1 - sp] > 0 && S.N >= 2 ? pg(ne[1 - sp], ne[sp], nal_u) : 0.0;
        }
    }
    d.target = prm->target_walkers;
    d.seed = prm->seed;
    d.d0 = hlo(S.d0);
    d.d0_hi = hhi(S.d0);
    d.det_words = S.W;
    d.space = prm->space;
    d.max_ex = prm->max_excitation;
    d.max_sen = prm->max_seniority;
    d.frz_occ = prm->frozen_occupied;
    d.frz_emp = prm->frozen_empty;
    d.frz_occ_hi = prm->frozen_occupied_hi;
    d.frz_emp_hi = prm->frozen_empty_hi;
    d.hphf = prm->hphf;
    d.lam = ((S.N / 2) & 1) ? -prm->hphf : prm->hphf;
    d.valid = hlo(valid);
    d.valid_hi = hhi(valid);
    for (int p = 0; p < nso; ++p) {
        const int c = 2 * S.irrep[p >> 1] + (p & 1);
        if (p < 64)
            d.cmask[c] |= 1ull << p;
        else
            d.cmask_hi[c] |= 1ull << (p - 64);
    }
    for (int i = 0; i < S.M; ++i) {
        uint64_t *w = i < 32 ? d.irr_packed : d.irr_packed_hi;
        w[(i >> 4) & 1] |= (uint64_t)S.irrep[i] << (4 * (i & 15));
    }
    d.shift = prm->initial_shift;
    fill_desc_tables(h, s);
    rc = relayout(h);
    if (rc) return rc;
    const int64_t n0 = prm->initial_walkers > 0 ? prm->initial_walkers : 10;
    rc = load_list(h, s, {S.d0}, {(int32_t)n0});
    if (rc) return rc;
    S.last.shift = prm->initial_shift;
    return 0;
}

// Replace the list of system s by (det, pop).
int load_list(fciqmc_t *h, int s, const std::vector<hdet_t> &det, const std::vector<int32_t> &pop) {
    SysHost &S = h->sys[s];
    const int64_t n = (int64_t)det.size();
    std::vector<uint64_t> words((size_t)n * S.W);
    for (int64_t i = 0; i < n; ++i) hdet_out(det[i], &words[(size_t)i * S.W], S.W);
    uint64_t *dd = nullptr;
    int32_t *dp = nullptr;
    HIP_TRY(hipMalloc(&dd, std::max<int64_t>(n, 1) * 8 * S.W));
    HIP_TRY(hipMalloc(&dp, std::max<int64_t>(n, 1) * 4));
    HIP_TRY(hipMemcpyAsync(dd, words.data(), n * 8 * S.W, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipMemcpyAsync(dp, pop.data(), n * 4, hipMemcpyHostToDevice, h->stream));
    int64_t need = std::max<int64_t>(S.cap, cap_for_entries(n));
    int rc = 0;
    for (int attempt = 0; rc == 0; ++attempt) {
        if (need > S.cap) {
            void *blk = nullptr;
            rc = alloc_tables(h, S, need, &blk);
            if (rc) break;
            SysHost T = S;
            carve(T, blk, need);
            rc = upload_integrals(h, T);
            if (rc) break;
            HIP_TRY(hipFree(S.block));
            carve(S, blk, need);
            fill_desc_tables(h, s);
            rc = relayout(h);
            if (rc) break;
        } else {
            HIP_TRY(hipMemsetAsync(S.bcnt, 0, (size_t)(S.cap / BQ) * sizeof(int32_t), h->stream));
        }
        h->hstatus[s] = 0;
        rc = reset_spawns(h, s);
        if (rc) break;
        rc = upload_desc(h);
        if (rc) break;
        HIP_TRY(hipMemsetAsync(h->d_err, 0, sizeof(uint32_t), h->stream));
        HIP_TRY(FQ_LAUNCH(h->W, launch_load, h->d_desc, s, dd, dp, n, h->d_err, h->stream));
        uint32_t err = 0;
        HIP_TRY(hipMemcpyAsync(&err, h->d_err, 4, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        if (!err) break;
        // a bucket overflowed: twice the buckets
        if (attempt >= 4) rc = set_err(FCIQMC_ECAPACITY, "walker list does not fit the buckets");
        need = 2 * S.cap;
    }
    hipFree(dd);
    hipFree(dp);
    if (rc) return rc;
    S.growth = std::max<int64_t>(256, n / 8);
    S.spawn_peak = 0;
    S.spawn_rate = 1.0;
    return 0;
}

int compute_e0(fciqmc_t *h, int s);

struct Walkers {
    std::vector<hdet_t> det;
    std::vector<int32_t> pop;
};

int export_walkers(fciqmc_t *h, int s, Walkers &w) {
    SysHost &S = h->sys[s];
    uint64_t *od = nullptr;
    int32_t *op = nullptr;
    unsigned long long *cnt = nullptr;
    HIP_TRY(hipMalloc(&od, S.cap * 8 * S.W));
    HIP_TRY(hipMalloc(&op, S.cap * 4));
    HIP_TRY(hipMalloc(&cnt, 8));
    HIP_TRY(hipMemsetAsync(cnt, 0, 8, h->stream));
    HIP_TRY(FQ_LAUNCH(h->W, launch_compact, S.key, S.pop, S.bcnt, S.cap / BQ, od, op, cnt, h->stream));
    unsigned long long n = 0;
    HIP_TRY(hipMemcpyAsync(&n, cnt, 8, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    std::vector<uint64_t> words(n * S.W);
    std::vector<hdet_t> dv(n);
    std::vector<int32_t> pv(n);
    if (n) {
        HIP_TRY(hipMemcpyAsync(words.data(), od, n * 8 * S.W, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipMemcpyAsync(pv.data(), op, n * 4, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
    }
    hipFree(od);
    hipFree(op);
    hipFree(cnt);
    for (size_t i = 0; i < n; ++i) dv[i] = hdet_in(&words[i * S.W], S.W);
    std::vector<size_t> idx(n);
    for (size_t i = 0; i < n; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return dv[a] < dv[b]; });
    w.det.resize(n);
    w.pop.resize(n);
    for (size_t i = 0; i < n; ++i) {
        w.det[i] = dv[idx[i]];
        w.pop[i] = pv[idx[i]];
    }
    return 0;
}

int fill_estimates(fciqmc_t *h, int s, fciqmc_estimates *o) {
    SysHost &S = h->sys[s];
    if (!S.active) return set_err(FCIQMC_ESTATE, "slot is not active");
    const IterRecord &r = S.last;
    std::memset(o, 0, sizeof *o);
    o->iteration = h->hdesc[s].iter;
    o->n_walkers = r.nw;
    o->n_dets = r.nd;
    o->ref_pop = r.c0;
    o->attempts = r.attempts;
    o->spawns = r.spawns;
    o->merged = r.merged;
    o->aborted = r.aborted;
    o->born = r.born;
    o->total_attempts = S.tot_att;
    o->total_spawns = S.tot_sp;
    o->n_samples = S.e_blk.count();
    o->n_var = h->hdesc[s].n_var;
    o->n_prev = h->hdesc[s].n_prev;
    o->table_slots = S.cap;
    o->table_used = std::max<int64_t>(r.used, r.nd);
    o->shift = h->hdesc[s].shift;
    o->e_ref = S.e0;
    o->p_double = S.p_double;
    o->proj_num = r.num;
    o->e_proj_inst = r.c0 != 0 ? S.e0 + r.num / (double)r.c0 : NAN;
    double m, e;
    S.e_blk.result(m, e);
    o->e_proj_mean = S.e0 + m;
    o->e_proj_err = e;
    S.s_blk.result(m, e);
    o->shift_mean = S.e0 + m;
    o->shift_err = e;
    o->ms_last_call = h->ms_last;
    o->redos = S.redos;
    o->spills = S.spills;
    o->ms_spawn = h->phase_ms[0] + h->phase_ms[1] + h->phase_ms[2];
    o->ms_death = 0.0;   // death runs inside the annihilation pass
    o->ms_annihilate = h->phase_ms[3];
    o->ms_estimators = h->phase_ms[4];
    o->shift_varying = h->hdesc[s].varying;
    o->status = S.fatal;
    return 0;
}

// Statistics of the list as loaded (before any iteration): N_w, N_d, C_0, num.
int refresh_stats_after_load(fciqmc_t *h, int s, const std::vector<hdet_t> &det,
                             const std::vector<int32_t> &pop, double num) {
    SysHost &S = h->sys[s];
    IterRecord r{};
    for (size_t i = 0; i < det.size(); ++i) {
        if (det[i] == S.d0) r.c0 = pop[i];
        if (pop[i] == 0) continue;
        r.nw += pop[i] < 0 ? -(int64_t)pop[i] : pop[i];
        r.nd++;
    }
    r.num = num;
    r.shift = h->hdesc[s].shift;
    S.last = r;
    return 0;
}

int run_iterations(fciqmc_t *h, int L, bool sample);

int capture_or_get(fciqmc_t *h, int L, hipGraphExec_t *out) {
    // a graph holds the spawning kernel's variant: one graph per length and variant
    EngineArgs a = make_args(h);
    const int key = 2 * L + a.plain;
    auto it = h->graphs.find(key);
    if (it != h->graphs.end()) {
        *out = it->second;
        return 0;
    }
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(h->stream, hipStreamCaptureModeRelaxed));
    for (int i = 0; i < L; ++i)
        FQ_LAUNCH(h->W, launch_iteration, a, h->post_grid, h->spawn_grid, i == 0, h->stream, nullptr);
    HIP_TRY(hipStreamEndCapture(h->stream, &g));
    hipGraphExec_t ex = nullptr;
    HIP_TRY(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
    HIP_TRY(hipGraphDestroy(g));
    h->graphs[key] = ex;
    *out = ex;
    return 0;
}

// Before a launch of up to L iterations: re-bucket any main list whose buckets
// would pass 5/8 full on average during the launch (each iteration adds at most
// `growth` entries, the largest increase seen, with slack), size the spawn-record
// buffer for the launch (the largest record count of the last launch growing at
// the largest rate seen), and return how many iterations that headroom allows.
// Whatever the estimates miss is caught on the device: an overflowing record
// buffer abandons the iteration for a re-run, an overflowing bucket spills.
int plan_launch(fciqmc_t *h, int L, int *L_out) {
    int allowed = L;
    int64_t rec_need = 0;
    double rate = 1.0;
    for (int s = 0; s < h->max_sys; ++s) {
        SysHost &S = h->sys[s];
        if (!S.active || S.fatal) continue;
        const SysDesc &d = h->hdesc[s];
        if (d.iter >= d.stop_at) continue;
        // records of one iteration: at most one per attempt before anything is known
        rec_need += S.spawn_peak > 0 ? S.spawn_peak : std::max<int64_t>(S.last.nw, 1);
        rate = std::max(rate, S.spawn_rate);
        if (!h->planner) continue;   // overflows are left to the redo and spill paths
        const int64_t g = std::max<int64_t>(S.growth, 256);
        int64_t used = std::max<int64_t>(S.last.used, S.last.nd + 1);
        if (used + 4 * g > S.cap * 5 / 8) {
            const int64_t nc = std::max<int64_t>(cap_for_entries(used + 8 * g),
                                                 round_cap(S.cap + S.cap / 2));
            const int rc = rebucket_system(h, s, nc, 0);
            if (rc) return rc;
        }
        const int64_t room = (S.cap * 5 / 8 - used) / g;
        allowed = (int)std::max<int64_t>(1, std::min<int64_t>(allowed, room));
    }
    if (h->planner && rec_need > 0) {
        const int lg = std::min(allowed, 8);
        const double grow = std::pow(rate, (double)lg);
        const int64_t want = (int64_t)(1.5 * (double)rec_need * grow) + 65536;
        if (want > h->rec_cap) {
            const int rc = ensure_records(h, std::max<int64_t>(want, h->rec_cap + h->rec_cap / 2));
            if (rc) return rc;
        }
        if (rate > 1.0) {
            const double fit = std::log((double)h->rec_cap / (1.25 * (double)rec_need)) / std::log(rate);
            allowed = (int)std::max<double>(1.0, std::min<double>((double)allowed, std::floor(fit)));
        }
    }
    *L_out = allowed;
    return 0;
}

// Spawn records of iteration `it` of system s (from the host ring of records).
int64_t rr_spawns(const fciqmc_t *h, int s, int64_t it) {
    return h->h_rec[(int64_t)s * REC_CAP + it % REC_CAP].spawns;
}

// Launch L iterations (graph or direct), then read records and statuses. With
// `sample` the last iteration runs as direct launches bracketed by events, which
// gives the per-phase device times of one iteration on the graph path too.
int run_iterations(fciqmc_t *h, int L, bool sample) {
    bool grow_records = false;
    std::vector<int> spilled;
    std::vector<int64_t> before(h->max_sys);
    for (int s = 0; s < h->max_sys; ++s) before[s] = h->hdesc[s].iter;
    int rc = ensure_tile_map(h);
    if (rc) return rc;
    rc = upload_desc(h);
    if (rc) return rc;
    EngineArgs a = make_args(h);
    if (h->profiling) {
        for (int i = 0; i < L; ++i) {
            FQ_LAUNCH(h->W, launch_iteration, a, h->post_grid, h->spawn_grid, i == 0, h->stream, h->ev);
            HIP_TRY(hipEventSynchronize(h->ev[NKERN]));
            for (int k = 0; k < NKERN; ++k) {
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, h->ev[k], h->ev[k + 1]));
                h->kms[k] += ms;
                h->kcount[k]++;
            }
        }
        HIP_TRY(hipGetLastError());
    } else if (h->use_graph) {
        const int Lg = sample ? L - 1 : L;
        if (Lg > 0) {
            hipGraphExec_t ex = nullptr;
            rc = capture_or_get(h, Lg, &ex);
            if (rc) return rc;
            HIP_TRY(hipGraphLaunch(ex, h->stream));
        }
        if (sample) {
            FQ_LAUNCH(h->W, launch_iteration, a, h->post_grid, h->spawn_grid, true, h->stream, h->ev);
            HIP_TRY(hipGetLastError());
            HIP_TRY(hipEventSynchronize(h->ev[NKERN]));
            for (int k = 0; k < NKERN; ++k) {
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, h->ev[k], h->ev[k + 1]));
                h->phase_ms[k] = ms;
            }
        }
    } else {
        for (int i = 0; i < L; ++i)
        FQ_LAUNCH(h->W, launch_iteration, a, h->post_grid, h->spawn_grid, i == 0, h->stream, nullptr);
        HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipStreamSynchronize(h->stream));
    rc = download_desc(h);
    if (rc) return rc;
    for (int s = 0; s < h->max_sys; ++s) {
        SysHost &S = h->sys[s];
        if (!S.active) continue;
        SysDesc &d = h->hdesc[s];
        const int64_t n_new = d.iter - before[s];
        if (n_new > 0) {
            // the stream has been synchronised: the records are in host memory
            const IterRecord *rr = h->h_rec + (int64_t)s * REC_CAP;
            int64_t prev_used = S.last.used, seen = 0;
            for (int64_t it = before[s] + 1; it <= d.iter; ++it) {
                const IterRecord &r = rr[it % REC_CAP];
                seen = std::max<int64_t>(seen, r.used - prev_used);
                prev_used = r.used;
                S.tot_att += r.attempts;
                S.tot_sp += r.spawns;
                if (r.varying && r.iter - r.n_var >= S.prm.avg_start) {
                    S.e_blk.add(r.num, (double)r.c0);
                    S.s_blk.add(r.shift, 1.0);
                }
                S.last = r;
            }
            // headroom estimates for the next launch: the largest growth of the entries
            // and the largest record count of this one, with 25 % slack, and the largest
            // ratio of consecutive record counts
            S.growth = std::max<int64_t>(256, seen + seen / 4);
            int64_t peak = 0, prev = 0;
            double rt = 1.0;
            for (int64_t it = before[s] + 1; it <= d.iter; ++it) {
                const int64_t sp = rr_spawns(h, s, it);
                peak = std::max(peak, sp);
                if (prev > 0) rt = std::max(rt, (double)sp / (double)prev);
                prev = sp;
            }
            S.spawn_peak = peak + peak / 4;
            S.spawn_rate = std::min(rt, 4.0);
        }
        uint32_t &st = h->hstatus[s];
        if (st & ST_TABLE_FULL) {
            // the record buffer overflowed: this iteration was abandoned and runs again
            st &= ~ST_TABLE_FULL;
            S.redos += 1;
            rc = reset_spawns(h, s);
            if (rc) return rc;
            grow_records = true;
        }
        if (st & ST_SPILLED) {
            st &= ~ST_SPILLED;
            S.spills += 1;
            spilled.push_back(s);
        }
        if (st) {
            S.fatal = (st & ST_SPILL_FULL) ? FCIQMC_ECAPACITY : FCIQMC_EOVERFLOW;
            return set_err(S.fatal,
                           "system " + std::to_string(s) + ": status " + std::to_string(st) +
                               ((st & ST_DIED) ? " (walkers died out)"
                                : (st & ST_SPILL_FULL) ? " (more new determinants than the spill list holds)"
                                                       : " (population overflow)"));
        }
    }
    if (grow_records) {
        rc = ensure_records(h, 2 * h->rec_cap);
        if (rc) return rc;
    }
    if (!spilled.empty()) {
        unsigned long long n_sp = 0;
        HIP_TRY(hipMemcpyAsync(&n_sp, h->d_sp_count, sizeof n_sp, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        const int64_t n_take = std::min<int64_t>((int64_t)n_sp, h->sp_cap);
        for (int s : spilled) {
            SysHost &S = h->sys[s];
            const int64_t used = std::max<int64_t>(S.last.used, S.last.nd + 1) + n_take;
            const int64_t nc = std::max<int64_t>(cap_for_entries(used + 8 * S.growth),
                                                 round_cap(2 * S.cap));
            rc = rebucket_system(h, s, nc, n_take);
            if (rc) return rc;
        }
        HIP_TRY(hipMemsetAsync(h->d_sp_count, 0, sizeof(unsigned long long), h->stream));
    }
    return 0;
}

int iterate_each(fciqmc_t *h, const std::vector<int64_t> &n) {
    hipEvent_t t0, t1;
    HIP_TRY(hipEventCreate(&t0));
    HIP_TRY(hipEventCreate(&t1));
    HIP_TRY(hipEventRecord(t0, h->stream));
    for (int s = 0; s < h->max_sys; ++s)
        if (h->sys[s].active) h->hdesc[s].stop_at = h->hdesc[s].iter + std::max<int64_t>(n[s], 0);
    for (;;) {
        int64_t rem = 0;
        for (int s = 0; s < h->max_sys; ++s)
            if (h->sys[s].active && !h->sys[s].fatal)
                rem = std::max<int64_t>(rem, h->hdesc[s].stop_at - h->hdesc[s].iter);
        if (rem <= 0) break;
        int L = 0;
        int rc = plan_launch(h, (int)std::min<int64_t>(rem, MAX_GRAPH_ITERS), &L);
        if (rc) return rc;
        // the launch that ends the call samples the per-phase times of its last iteration
        rc = run_iterations(h, L, L >= rem);
        if (rc) return rc;
    }
    HIP_TRY(hipEventRecord(t1, h->stream));
    HIP_TRY(hipEventSynchronize(t1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, t0, t1));
    h->ms_last = ms;
    hipEventDestroy(t0);
    hipEventDestroy(t1);
    return 0;
}

// Entries of the spill list (new determinants that did not fit their bucket).
constexpr int64_t SPILL_CAP = (int64_t)1 << 16;

// Address of the staging area on each device (resolved once per device, with
// that device current).
constexpr int MAX_DEVICES = 64;
std::mutex g_stage_mu;
void *g_stage_ptr[MAX_DEVICES] = {};

int resolve_stage(int dev, void **out) {
    if (dev < 0 || dev >= MAX_DEVICES) return set_err(FCIQMC_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_stage_mu);
    if (!g_stage_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return set_err(FCIQMC_EDEVICE, "staging area has no device address");
        g_stage_ptr[dev] = p;
    }
    *out = g_stage_ptr[dev];
    return 0;
}

int create_handle(int max_slots, void *stream, int W, fciqmc_t **out) {
    fciqmc_t *h = new (std::nothrow) fciqmc_t();
    if (!h) return set_err(FCIQMC_ENOMEM, "host allocation failed");
    h->W = W;
    HIP_TRY(hipGetDevice(&h->dev));
    {
        const int rc = resolve_stage(h->dev, &h->d_stage);
        if (rc) {
            delete h;
            return rc;
        }
    }
    if (stream) {
        h->stream = (hipStream_t)stream;
    } else {
        HIP_TRY(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
        h->own_stream = true;
    }
    h->max_sys = max_slots;
    h->sys.resize(max_slots);
    h->hdesc.assign(max_slots, SysDesc{});
    h->hstatus.assign(max_slots, 0u);
    HIP_TRY(hipMalloc(&h->d_desc, sizeof(SysDesc) * max_slots));
    HIP_TRY(hipMalloc(&h->d_status, sizeof(uint32_t) * max_slots));
    HIP_TRY(hipMalloc(&h->d_work, sizeof(unsigned int) * 4));
    HIP_TRY(hipMemsetAsync(h->d_work, 0, sizeof(unsigned int) * 4, h->stream));
    HIP_TRY(hipMalloc(&h->d_spawns, sizeof(unsigned long long) * max_slots));
    HIP_TRY(hipMemsetAsync(h->d_spawns, 0, sizeof(unsigned long long) * max_slots, h->stream));
    HIP_TRY(hipHostMalloc((void **)&h->h_rec, sizeof(IterRecord) * REC_CAP * max_slots,
                          hipHostMallocDefault));
    std::memset(h->h_rec, 0, sizeof(IterRecord) * REC_CAP * max_slots);
    HIP_TRY(hipHostGetDevicePointer((void **)&h->d_rec, h->h_rec, 0));
    HIP_TRY(hipMalloc(&h->d_total, 2 * sizeof(unsigned long long)));
    HIP_TRY(hipMalloc(&h->d_nchunks, sizeof(int64_t)));
    HIP_TRY(hipMalloc(&h->d_blk, 2 * 4 * SCAN_G * sizeof(unsigned long long)));
    HIP_TRY(hipMalloc(&h->d_step, sizeof(unsigned long long)));
    HIP_TRY(hipMemsetAsync(h->d_step, 0, sizeof(unsigned long long), h->stream));
    HIP_TRY(hipMalloc(&h->d_fin, sizeof(FinPart) * FIN_BLOCKS * max_slots));
    HIP_TRY(hipMalloc(&h->d_c0, sizeof(int64_t) * max_slots));
    HIP_TRY(hipMalloc(&h->d_err, sizeof(uint32_t)));
    HIP_TRY(hipMalloc(&h->d_rec_count, sizeof(unsigned long long)));
    HIP_TRY(hipMalloc(&h->d_boff_rg, 2 * SCAN_G * sizeof(unsigned long long)));
    HIP_TRY(hipMalloc(&h->d_d0acc, sizeof(long long) * max_slots));
    HIP_TRY(hipMemsetAsync(h->d_d0acc, 0, sizeof(long long) * max_slots, h->stream));
    HIP_TRY(hipMemsetAsync(h->d_rec_count, 0, sizeof(unsigned long long), h->stream));
    {
        const int rc = ensure_records(h, 65536);
        if (rc) return rc;
    }
    h->sp_cap = SPILL_CAP;
    HIP_TRY(hipMalloc(&h->d_spill, (size_t)h->sp_cap * (16 + 8 * h->W)));
    HIP_TRY(hipMalloc(&h->d_sp_count, sizeof(unsigned long long)));
    HIP_TRY(hipMemsetAsync(h->d_sp_count, 0, sizeof(unsigned long long), h->stream));
    HIP_TRY(hipMalloc(&h->d_spilled, sizeof(uint32_t) * max_slots));
    HIP_TRY(hipMemsetAsync(h->d_spilled, 0, sizeof(uint32_t) * max_slots, h->stream));
    for (int k = 0; k <= NKERN; ++k) HIP_TRY(hipEventCreate(&h->ev[k]));
    h->spawn_grid = spawn_grid_size();
    h->post_grid = post_grid_size();
    int rc = upload_desc(h);
    if (rc) return rc;
    rc = relayout(h);
    if (rc) return rc;
    *out = h;
    return 0;
}

}  // namespace

namespace {
int compute_e0(fciqmc_t *h, int s) {
    double *d_out = nullptr;
    HIP_TRY(hipMalloc(&d_out, 8));
    int rc = upload_desc(h);
    if (rc) return rc;
    HIP_TRY(FQ_LAUNCH(h->W, launch_e0, h->d_desc, s, hlo(h->sys[s].d0), hhi(h->sys[s].d0), d_out,
                      h->stream));
    double e0 = 0;
    HIP_TRY(hipMemcpyAsync(&e0, d_out, 8, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    hipFree(d_out);
    h->sys[s].e0 = e0;
    h->hdesc[s].e0 = e0;
    return 0;
}

int admit_full(fciqmc_t *h, int s, const fciqmc_hamiltonian *ham, const fciqmc_params *prm) {
    int rc = admit(h, s, ham, prm);
    if (rc) {
        SysHost &S = h->sys[s];
        if (S.block) hipFree(S.block);
        S = SysHost();
        h->hdesc[s] = SysDesc{};
        relayout(h);
        upload_desc(h);
        return rc;
    }
    rc = compute_e0(h, s);
    if (rc) return rc;
    const int64_t n0 = prm->initial_walkers > 0 ? prm->initial_walkers : 10;
    h->sys[s].last = IterRecord{};
    h->sys[s].last.nw = n0;
    h->sys[s].last.nd = 1;
    h->sys[s].last.c0 = n0;
    h->sys[s].last.shift = prm->initial_shift;
    if (prm->spawn_capacity > 0) {   // the record buffer is shared by the handle's systems
        rc = ensure_records(h, prm->spawn_capacity);
        if (rc) return rc;
    }
    return upload_desc(h);
}

void release(fciqmc_t *h) {
    if (!h) return;
    hipStreamSynchronize(h->stream);
    drop_graphs(h);
    for (auto &S : h->sys)
        if (S.block) hipFree(S.block);
    hipFree(h->d_desc);
    if (h->h_rec) hipHostFree(h->h_rec);
    hipFree(h->d_status);
    hipFree(h->d_work);
    hipFree(h->d_spawns);
    hipFree(h->d_total);
    hipFree(h->d_nchunks);
    hipFree(h->d_blk);
    hipFree(h->d_step);
    hipFree(h->d_fin);
    hipFree(h->d_c0);
    hipFree(h->d_err);
    hipFree(h->d_chunk_sys);
    hipFree(h->d_chunk_local);
    hipFree(h->d_chunk_nw);
    hipFree(h->d_chunk_off);
    hipFree(h->d_chunk_toff);
    hipFree(h->d_chunk_stat);
    hipFree(h->d_tile_chunk);
    hipFree(h->d_recs);
    hipFree(h->d_rec_count);
    hipFree(h->d_bhist);
    hipFree(h->d_boff);
    hipFree(h->d_boff_rg);
    hipFree(h->d_d0acc);
    hipFree(h->d_spill);
    hipFree(h->d_sp_count);
    hipFree(h->d_spilled);
    for (auto &e : h->ev)
        if (e) hipEventDestroy(e);
    if (h->own_stream) hipStreamDestroy(h->stream);
    delete h;
}

int64_t walkers_out(fciqmc_t *h, int s, uint64_t *det, int32_t *pop, uint32_t *flags, int64_t cap) {
    if (!h || s < 0 || s >= h->max_sys || !h->sys[s].active)
        return set_err(FCIQMC_ESTATE, "slot is not active");
    Walkers w;
    int rc = export_walkers(h, s, w);
    if (rc) return rc;
    const SysHost &S = h->sys[s];
    const int64_t n = (int64_t)w.det.size();
    for (int64_t i = 0; i < n && i < cap; ++i) {
        if (det) hdet_out(w.det[i], det + i * S.W, S.W);
        if (pop) pop[i] = w.pop[i];
        if (flags) {
            const int64_t a = w.pop[i] < 0 ? -(int64_t)w.pop[i] : w.pop[i];
            flags[i] = (a > S.prm.initiator_threshold || w.det[i] == S.d0) ? 1u : 0u;
        }
    }
    return n;
}
}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *fciqmc_last_error(void) { return g_err.c_str(); }

int fciqmc_batch_create(int32_t max_slots, int32_t n, const fciqmc_hamiltonian *hams,
                        const fciqmc_params *prms, void *hip_stream, fciqmc_t **out) {
    if (!out) return set_err(FCIQMC_EINVAL, "null output handle");
    *out = nullptr;
    if (max_slots < 1 || n < 0 || n > max_slots) return set_err(FCIQMC_EINVAL, "bad slot counts");
    if (n > 0 && (!hams || !prms)) return set_err(FCIQMC_EINVAL, "null hamiltonians or params");
    for (int i = 0; i < n; ++i) {
        int rc = validate(&hams[i], &prms[i]);
        if (rc) return rc;
    }
    // one determinant width for the batch: the first system's (one word when empty)
    const int W = n > 0 ? words_for(hams[0].n_orb, prms[0].det_words) : 1;
    for (int i = 1; i < n; ++i)
        if (words_for(hams[i].n_orb, prms[i].det_words) != W)
            return set_err(FCIQMC_EINVAL, "a batch holds determinants of one width (64-bit words)");
    fciqmc_t *h = nullptr;
    int rc = create_handle(max_slots, hip_stream, W, &h);
    if (rc) {
        release(h);
        return rc;
    }
    for (int i = 0; i < n; ++i) {
        rc = admit_full(h, i, &hams[i], &prms[i]);
        if (rc) {
            std::string keep = g_err;
            release(h);
            g_err = keep;
            return rc;
        }
    }
    *out = h;
    return 0;
}

int fciqmc_init(const fciqmc_hamiltonian *ham, const fciqmc_params *prm, void *hip_stream,
                fciqmc_t **out) {
    return fciqmc_batch_create(1, 1, ham, prm, hip_stream, out);
}

int fciqmc_free(fciqmc_t *h) {
    release(h);
    return 0;
}

int fciqmc_iterate(fciqmc_t *h, int32_t n_iterations) {
    if (!h) return set_err(FCIQMC_EINVAL, "null handle");
    if (n_iterations < 0) return set_err(FCIQMC_EINVAL, "negative iteration count");
    std::vector<int64_t> n(h->max_sys, n_iterations);
    return iterate_each(h, n);
}

int fciqmc_batch_iterate(fciqmc_t *h, int32_t n_iterations) { return fciqmc_iterate(h, n_iterations); }

int fciqmc_batch_iterate_each(fciqmc_t *h, const int32_t *n_iter) {
    if (!h || !n_iter) return set_err(FCIQMC_EINVAL, "null argument");
    std::vector<int64_t> n(h->max_sys);
    for (int s = 0; s < h->max_sys; ++s) n[s] = n_iter[s];
    return iterate_each(h, n);
}

int fciqmc_estimators(fciqmc_t *h, fciqmc_estimates *out) {
    if (!h || !out) return set_err(FCIQMC_EINVAL, "null argument");
    return fill_estimates(h, 0, out);
}

int fciqmc_batch_slot_estimators(fciqmc_t *h, int32_t slot, fciqmc_estimates *out) {
    if (!h || !out || slot < 0 || slot >= h->max_sys) return set_err(FCIQMC_EINVAL, "bad argument");
    return fill_estimates(h, slot, out);
}

int32_t fciqmc_det_words(const fciqmc_t *h) {
    if (!h) return set_err(FCIQMC_EINVAL, "null handle");
    return h->W;
}

int64_t fciqmc_walkers(fciqmc_t *h, uint64_t *det, int32_t *pop, uint32_t *flags, int64_t cap) {
    if (!h) return set_err(FCIQMC_EINVAL, "null handle");
    return walkers_out(h, 0, det, pop, flags, cap);
}

int64_t fciqmc_batch_slot_walkers(fciqmc_t *h, int32_t slot, uint64_t *det, int32_t *pop,
                                  uint32_t *flags, int64_t cap) {
    if (!h) return set_err(FCIQMC_EINVAL, "null handle");
    return walkers_out(h, slot, det, pop, flags, cap);
}

int fciqmc_load_walkers(fciqmc_t *h, const uint64_t *det, const int32_t *pop, int64_t n,
                        int64_t iteration, double shift, int64_t n_prev, int32_t varying,
                        int64_t n_var) {
    if (!h) return set_err(FCIQMC_EINVAL, "null handle");
    if (n < 0 || (n > 0 && (!det || !pop)) || iteration < 0)
        return set_err(FCIQMC_EINVAL, "bad walker list");
    const int s = 0;
    SysHost &S = h->sys[s];
    if (!S.active) return set_err(FCIQMC_ESTATE, "slot is not active");
    const hdet_t valid = 2 * S.M == 128 ? ~(hdet_t)0 : (hbit(2 * S.M) - 1);
    std::vector<std::pair<hdet_t, int32_t>> v;
    v.reserve(n + 1);
    bool have_ref = false;
    for (int64_t i = 0; i < n; ++i) {
        if (pop[i] == 0) continue;
        const hdet_t d = hdet_in(det + i * S.W, S.W);
        int a = 0, b = 0;
        for (int p = 0; p < 128; ++p)
            if ((d >> p) & 1) (p & 1 ? b : a)++;
        if ((d & ~valid) || a != S.na || b != S.nb)
            return set_err(FCIQMC_EINVAL, "determinant with wrong electron counts in walker list");
        if (pop[i] == INT32_MIN) return set_err(FCIQMC_EINVAL, "population out of range");
        if (!host_in_space(&S.prm, S.d0, d))
            return set_err(FCIQMC_EINVAL, "determinant outside the restricted space in walker list");
        if (S.prm.hphf && (host_spin_flip(d) < d || (host_spin_flip(d) == d && S.prm.hphf < 0)))
            return set_err(FCIQMC_EINVAL, "a list of spin-coupled functions holds each as the "
                                          "smaller determinant of its pair");
        if (d == S.d0) have_ref = true;
        v.emplace_back(d, pop[i]);
    }
    if (!have_ref) v.emplace_back(S.d0, 0);
    std::sort(v.begin(), v.end());
    for (size_t i = 1; i < v.size(); ++i)
        if (v[i].first == v[i - 1].first)
            return set_err(FCIQMC_EINVAL, "duplicate determinant in walker list");
    std::vector<hdet_t> dv(v.size());
    std::vector<int32_t> pv(v.size());
    for (size_t i = 0; i < v.size(); ++i) {
        dv[i] = v[i].first;
        pv[i] = v[i].second;
    }
    SysDesc &d = h->hdesc[s];
    d.iter = iteration;
    d.shift = shift;
    d.n_prev = n_prev;
    d.varying = varying ? 1 : 0;
    d.n_var = n_var;
    int rc = load_list(h, s, dv, pv);
    if (rc) return rc;
    S.e_blk.clear();
    S.s_blk.clear();
    S.fatal = 0;
    refresh_stats_after_load(h, s, dv, pv, NAN);
    return upload_desc(h);
}

int fciqmc_set_shift(fciqmc_t *h, double shift, int32_t varying) {
    if (!h || !h->sys[0].active) return set_err(FCIQMC_EINVAL, "null handle");
    SysDesc &d = h->hdesc[0];
    d.shift = shift;
    d.varying = varying ? 1 : 0;
    if (varying) {
        d.n_prev = h->sys[0].last.nw;
        d.n_var = d.iter;
    }
    h->sys[0].e_blk.clear();
    h->sys[0].s_blk.clear();
    return upload_desc(h);
}

int fciqmc_reserve(fciqmc_t *h, int64_t slots) {
    if (!h) return set_err(FCIQMC_EINVAL, "null handle");
    if (slots < 0) return set_err(FCIQMC_EINVAL, "slots must be >= 0");
    const int64_t want = round_cap(slots);
    for (int s = 0; s < h->max_sys; ++s) {
        SysHost &S = h->sys[s];
        if (!S.active || S.fatal || S.cap >= want) continue;
        const int rc = rebucket_system(h, s, want, 0);
        if (rc) return rc;
    }
    return 0;
}

int fciqmc_batch_admit(fciqmc_t *h, const fciqmc_hamiltonian *ham, const fciqmc_params *prm,
                       int32_t *slot) {
    if (!h || !slot) return set_err(FCIQMC_EINVAL, "null argument");
    int s = -1;
    for (int i = 0; i < h->max_sys; ++i)
        if (!h->sys[i].active) {
            s = i;
            break;
        }
    if (s < 0) return set_err(FCIQMC_ESTATE, "no free slot");
    int rc = admit_full(h, s, ham, prm);
    if (rc) return rc;
    *slot = s;
    return 0;
}

int fciqmc_batch_retire(fciqmc_t *h, int32_t slot) {
    if (!h || slot < 0 || slot >= h->max_sys || !h->sys[slot].active)
        return set_err(FCIQMC_ESTATE, "slot is not active");
    HIP_TRY(hipStreamSynchronize(h->stream));
    SysHost &S = h->sys[slot];
    if (S.block) HIP_TRY(hipFree(S.block));
    S = SysHost();
    h->hdesc[slot] = SysDesc{};
    h->hstatus[slot] = 0;
    int rc = relayout(h);
    if (rc) return rc;
    return upload_desc(h);
}

int32_t fciqmc_batch_active(fciqmc_t *h) {
    if (!h) return 0;
    int32_t n = 0;
    for (auto &S : h->sys) n += S.active ? 1 : 0;
    return n;
}

int64_t fciqmc_footprint_bytes(const fciqmc_hamiltonian *ham, const fciqmc_params *prm) {
    if (!ham || !prm) return set_err(FCIQMC_EINVAL, "null argument");
    return target_footprint(ham, prm);
}

int fciqmc_set_profiling(fciqmc_t *h, int32_t on) {
    if (!h) return set_err(FCIQMC_EINVAL, "null handle");
    h->profiling = on != 0;
    for (int k = 0; k < NKERN; ++k) {
        h->kms[k] = 0.0;
        h->kcount[k] = 0;
    }
    return 0;
}

int fciqmc_set_launch(fciqmc_t *h, int32_t spawn_grid, int32_t tile, int32_t post_grid) {
    if (!h) return set_err(FCIQMC_EINVAL, "null handle");
    if (spawn_grid < 1 || post_grid < 1 || tile < 256 || tile > (1 << 20) || (tile & (tile - 1)))
        return set_err(FCIQMC_EINVAL, "launch shape out of range (tile: a power of two, 256..2^20)");
    h->spawn_grid = spawn_grid;
    h->post_grid = post_grid;
    h->tile = tile;
    drop_graphs(h);
    return 0;
}

int fciqmc_get_launch(fciqmc_t *h, int32_t *spawn_grid, int32_t *tile, int32_t *post_grid) {
    if (!h || !spawn_grid || !tile || !post_grid) return set_err(FCIQMC_EINVAL, "null argument");
    *spawn_grid = h->spawn_grid;
    *tile = h->tile;
    *post_grid = h->post_grid;
    return 0;
}

// What an autotuning trial advances of one system, restored after the trials: the
// walker list, the dynamics, the statistics and the per-iteration records.
struct SysSnapshot {
    int s = 0;
    std::vector<hdet_t> det;
    std::vector<int32_t> pop;
    SysDesc desc{};
    IterRecord last{};
    int64_t tot_att = 0, tot_sp = 0, redos = 0, spills = 0, growth = 0, spawn_peak = 0;
    double spawn_rate = 1.0;
    Blocker e_blk, s_blk;
    std::vector<IterRecord> ring;
};

int take_snapshot(fciqmc_t *h, int s, SysSnapshot &o) {
    SysHost &S = h->sys[s];
    Walkers w;
    const int rc = export_walkers(h, s, w);
    if (rc) return rc;
    o.s = s;
    o.det = std::move(w.det);
    o.pop = std::move(w.pop);
    if (!std::binary_search(o.det.begin(), o.det.end(), S.d0)) {   // the reference at 0
        const size_t at = std::lower_bound(o.det.begin(), o.det.end(), S.d0) - o.det.begin();
        o.det.insert(o.det.begin() + at, S.d0);
        o.pop.insert(o.pop.begin() + at, 0);
    }
    o.desc = h->hdesc[s];
    o.last = S.last;
    o.tot_att = S.tot_att;
    o.tot_sp = S.tot_sp;
    o.redos = S.redos;
    o.spills = S.spills;
    o.growth = S.growth;
    o.spawn_peak = S.spawn_peak;
    o.spawn_rate = S.spawn_rate;
    o.e_blk = S.e_blk;
    o.s_blk = S.s_blk;
    o.ring.assign(h->h_rec + (int64_t)s * REC_CAP, h->h_rec + (int64_t)(s + 1) * REC_CAP);
    return 0;
}

int restore_snapshot(fciqmc_t *h, const SysSnapshot &o) {
    const int s = o.s;
    SysHost &S = h->sys[s];
    SysDesc &d = h->hdesc[s];
    d.iter = o.desc.iter;
    d.stop_at = o.desc.iter;
    d.shift = o.desc.shift;
    d.varying = o.desc.varying;
    d.n_prev = o.desc.n_prev;
    d.n_var = o.desc.n_var;
    const int rc = load_list(h, s, o.det, o.pop);
    if (rc) return rc;
    S.last = o.last;
    S.tot_att = o.tot_att;
    S.tot_sp = o.tot_sp;
    S.redos = o.redos;
    S.spills = o.spills;
    S.growth = o.growth;
    S.spawn_peak = o.spawn_peak;
    S.spawn_rate = o.spawn_rate;
    S.e_blk = o.e_blk;
    S.s_blk = o.s_blk;
    S.fatal = 0;
    std::copy(o.ring.begin(), o.ring.end(), h->h_rec + (int64_t)s * REC_CAP);
    return upload_desc(h);
}

int fciqmc_autotune(fciqmc_t *h, int32_t iters_per_trial) {
    if (!h || iters_per_trial < 1) return set_err(FCIQMC_EINVAL, "bad argument");
    int cus = fq::post_grid_size() / 4;   // (four post workgroups per CU)
    // The trials run on the live systems; their state is saved first and restored
    // afterwards, so tuning leaves every trajectory where it was.
    std::vector<SysSnapshot> snaps;
    for (int s = 0; s < h->max_sys; ++s) {
        if (!h->sys[s].active || h->sys[s].fatal) continue;
        snaps.emplace_back();
        const int rc = take_snapshot(h, s, snaps.back());
        if (rc) return rc;
    }
    const bool was = h->profiling;
    h->profiling = true;
    auto trial = [&](int sg, int tl, int pg, double &spawn_ns, double &post_ns) -> int {
        h->spawn_grid = sg;
        h->tile = tl;
        h->post_grid = pg;
        for (int k = 0; k < NKERN; ++k) {
            h->kms[k] = 0.0;
            h->kcount[k] = 0;
        }
        int64_t a0 = 0;
        for (auto &S : h->sys) a0 += S.active ? S.tot_att : 0;
        std::vector<int64_t> n(h->max_sys, iters_per_trial);
        int rc = iterate_each(h, n);
        if (rc) return rc;
        int64_t a1 = 0;
        for (auto &S : h->sys) a1 += S.active ? S.tot_att : 0;
        spawn_ns = h->kms[2] * 1e6 / (double)std::max<int64_t>(a1 - a0, 1);
        post_ns = h->kms[3] * 1e6 / (double)iters_per_trial;   // per iteration
        return 0;
    };
    int best_sg = h->spawn_grid, best_tl = h->tile, best_pg = h->post_grid;
    double best_s = 1e300, best_p = 1e300;
    // (k_post is compiled for four resident workgroups per CU)
    const int sgs[4] = {2, 4, 8, 16}, tls[3] = {1024, 2048, 4096}, pgs[5] = {2, 3, 4, 6, 8};
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 3; ++j) {
            double sn, pn;
            int rc = trial(sgs[i] * cus, tls[j], best_pg, sn, pn);
            if (rc) {
                h->profiling = was;
                return rc;
            }
            if (sn < best_s) {
                best_s = sn;
                best_sg = sgs[i] * cus;
                best_tl = tls[j];
            }
        }
    for (int i = 0; i < 5; ++i) {
        double sn, pn;
        int rc = trial(best_sg, best_tl, pgs[i] * cus, sn, pn);
        if (rc) {
            h->profiling = was;
            return rc;
        }
        if (pn < best_p) {
            best_p = pn;
            best_pg = pgs[i] * cus;
        }
    }
    h->spawn_grid = best_sg;
    h->tile = best_tl;
    h->post_grid = best_pg;
    h->profiling = was;
    for (int k = 0; k < NKERN; ++k) {
        h->kms[k] = 0.0;
        h->kcount[k] = 0;
    }
    drop_graphs(h);
    for (const SysSnapshot &o : snaps) {
        const int rc = restore_snapshot(h, o);
        if (rc) return rc;
    }
    return 0;
}

int64_t fciqmc_history(fciqmc_t *h, int32_t slot, int64_t first, int64_t n, fciqmc_iteration *out) {
    if (!h || slot < 0 || slot >= h->max_sys || n < 0 || (n > 0 && !out))
        return set_err(FCIQMC_EINVAL, "bad argument");
    if (!h->sys[slot].active) return set_err(FCIQMC_ESTATE, "slot is not active");
    const int64_t cur = h->hdesc[slot].iter;
    const int64_t lo = std::max<int64_t>(1, cur - REC_CAP + 1);
    if (first < lo || first + n - 1 > cur) return set_err(FCIQMC_EINVAL, "iterations not in the log");
    for (int64_t i = 0; i < n; ++i) {
        const IterRecord &r = h->h_rec[(int64_t)slot * REC_CAP + (first + i) % REC_CAP];
        fciqmc_iteration &o = out[i];
        o.iteration = r.iter;
        o.n_walkers = r.nw;
        o.n_dets = r.nd;
        o.ref_pop = r.c0;
        o.attempts = r.attempts;
        o.spawns = r.spawns;
        o.merged = r.merged;
        o.aborted = r.aborted;
        o.born = r.born;
        o.entries = r.used;
        o.proj_num = r.num;
        o.shift = r.shift;
        o.shift_varying = r.varying;
        o.status = r.status;
    }
    return n;
}

int fciqmc_blocking(const double *num, const double *den, int64_t n, double *mean, double *err) {
    if (n < 0 || (n > 0 && !num) || !mean || !err) return set_err(FCIQMC_EINVAL, "bad argument");
    Blocker b;
    for (int64_t t = 0; t < n; ++t) b.add(num[t], den ? den[t] : 1.0);
    b.result(*mean, *err);
    return 0;
}

int fciqmc_set_test_options(fciqmc_t *h, int32_t planner, int64_t tile_map_limit,
                            int64_t record_capacity) {
    if (!h) return set_err(FCIQMC_EINVAL, "null handle");
    if (tile_map_limit < -1) return set_err(FCIQMC_EINVAL, "tile_map_limit must be >= -1");
    if (record_capacity < 0) return set_err(FCIQMC_EINVAL, "record_capacity must be >= 0");
    h->planner = planner != 0;
    if (record_capacity > 0) {
        HIP_TRY(hipStreamSynchronize(h->stream));
        hipFree(h->d_recs);
        h->d_recs = nullptr;
        h->rec_cap = 0;
        const int rc = ensure_records(h, record_capacity);
        if (rc) return rc;
    }
    if (tile_map_limit != h->tile_map_limit) {
        HIP_TRY(hipStreamSynchronize(h->stream));
        hipFree(h->d_tile_chunk);
        h->d_tile_chunk = nullptr;
        h->tile_cap = 0;
        h->tile_map_off = false;
        h->tile_map_limit = tile_map_limit;
        drop_graphs(h);
    }
    return 0;
}

int64_t fciqmc_walkers_noalloc(fciqmc_t *h, uint64_t *det, int32_t *pop, uint32_t *flags,
                               int64_t cap) {
    if (!h) return set_err(FCIQMC_EINVAL, "null handle");
    if (cap < 0) return set_err(FCIQMC_EINVAL, "cap must be >= 0");
    const int s = 0;
    const SysHost &S = h->sys[s];
    if (!S.active) return set_err(FCIQMC_ESTATE, "slot is not active");
    if (h->W != 1)
        return set_err(FCIQMC_ESTATE, "the staging export holds one-word determinants only");
    HIP_TRY(launch_stage_compact(S.key, S.pop, S.bcnt, S.cap / BQ, h->d_stage, h->stream));
    unsigned long long n = 0;
    HIP_TRY(hipMemcpyAsync(&n, h->d_stage, sizeof n, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    if ((int64_t)n > NOALLOC_MAX_DETS)
        return set_err(FCIQMC_ECAPACITY, "walker list of " + std::to_string(n) +
                                             " determinants exceeds the staging limit of " +
                                             std::to_string(NOALLOC_MAX_DETS));
    const int64_t m = std::min<int64_t>((int64_t)n, cap);
    if (m > 0 && (det || pop || flags)) {
        HIP_TRY(launch_stage_sort(h->d_stage, (int64_t)n, h->stream));
        if (flags)
            HIP_TRY(launch_stage_flags(h->d_stage, m, S.prm.initiator_threshold, hlo(S.d0), h->stream));
        const char *p = (const char *)h->d_stage;
        if (det)
            HIP_TRY(hipMemcpyAsync(det, p + NOALLOC_KEYS_OFF, (size_t)m * 8, hipMemcpyDeviceToHost,
                                   h->stream));
        if (pop)
            HIP_TRY(hipMemcpyAsync(pop, p + NOALLOC_VALS_OFF, (size_t)m * 4, hipMemcpyDeviceToHost,
                                   h->stream));
        if (flags)
            HIP_TRY(hipMemcpyAsync(flags, p + NOALLOC_FLAGS_OFF, (size_t)m * 4,
                                   hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
    }
    return (int64_t)n;
}

int fciqmc_kernel_times(fciqmc_t *h, double ms[5], int64_t counts[5]) {
    if (!h || !ms || !counts) return set_err(FCIQMC_EINVAL, "null argument");
    for (int k = 0; k < NKERN; ++k) {
        ms[k] = h->kms[k];
        counts[k] = h->kcount[k];
    }
    return 0;
}

}  // extern "C"
