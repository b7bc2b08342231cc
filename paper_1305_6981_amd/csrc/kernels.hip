// HIP kernels of the FCIQMC iteration (Booth, Smart & Alavi, arXiv:1305.6981)
// for gfx950.
//
// The main list of a system is hash-partitioned into buckets of at most 256
// densely packed entries (determinant, population, stored H_DD): the paper's
// distribution of determinants over processes by a hash (Sec. 4.1), with a
// wavefront in the role of a process. Four consecutive buckets form a chunk,
// the unit of attempt mapping. One iteration of every active system is
// eleven launches (twelve in the first iteration of a launch sequence):
//
//   k_chunk_sum   sum |C| over each bucket and over fixed contiguous ranges of
//                 buckets (first iteration of a launch sequence only;
//                 afterwards k_post provides the sums)
//   k_scan        exclusive scan of the range sums (one workgroup)
//   k_scan_down   per bucket: global attempt offset and spawn-tile offset
//   k_spawn       one spawning attempt per walker (Sec. 2, Eq. pspawn): random
//                 excitation with its pgen (Sec. 5), Slater-Condon element,
//                 acceptance; each accepted spawn becomes a record (child,
//                 signed walkers, initiator flag) addressed to the child's
//                 bucket -- the per-destination blocks of Sec. 4.1
//   k_fix         bucket and rank of records left unranked by k_spawn (rare)
//   k_bscan_*     exclusive scan of the records per bucket (range totals, their
//                 scan, then the scan inside each range)
//   k_scatter     the records grouped by bucket (a counting sort)
//   k_post        per bucket, by one wavefront: the records merged per child in
//                 an LDS hash (the sort and compress of Sec. 4.1); death/cloning
//                 of every entry (Eq. pdeath); annihilation with the initiator
//                 test for children that are unoccupied after death (Sec. 4.2);
//                 new determinants placed into the holes left by emptied
//                 entries, the bucket re-packed, H_DD of new determinants from a
//                 pair table staged in LDS; estimator partial sums (Eq. ProjE);
//                 the next iteration's bucket and range sums of |C|
//   k_reduce      per system, 64 workgroups: fixed-order reduction of the
//                 bucket statistics over fixed ranges of buckets
//   k_finalize    per system, one wavefront: sum of the 64 shares, the shift
//                 update, the per-iteration record
//
// All floating-point decisions follow the same operation order as the CPU
// oracle and are compiled with -ffp-contract=off.
#include "engine.h"

#ifndef FQ_DET_WORDS
#define FQ_DET_WORDS 1
#endif

namespace fq {
#if FQ_DET_WORDS == 2
namespace w2 {
#endif

// ---------------------------------------------------------------------------
// Determinants (Sec. 3): bit p set when spin orbital p is occupied, in as many
// 64-bit words as the spin orbitals need. This file is compiled once per width:
// one word (up to 64 spin orbitals, det_t = uint64_t) into namespace fq, two
// words (up to 128, det_t = a 128-bit integer with the operations used here)
// into fq::w2.
// ---------------------------------------------------------------------------
#if FQ_DET_WORDS == 1
typedef uint64_t det_t;
__device__ __forceinline__ uint64_t lo64(det_t x) { return x; }
__device__ __forceinline__ uint64_t hi64(det_t) { return 0ull; }
__device__ __forceinline__ det_t make_det(uint64_t lo, uint64_t) { return lo; }
__device__ __forceinline__ int dpopc(det_t x) { return __popcll(x); }
__device__ __forceinline__ int dctz(det_t x) { return __builtin_ctzll(x); }      // lowest set bit
__device__ __forceinline__ int dhib(det_t x) { return 63 - __builtin_clzll(x); } // highest set bit
#else
struct det_t {
    unsigned __int128 v;
    det_t() = default;
    __device__ constexpr explicit det_t(unsigned long long x) : v(x) {}
    __device__ explicit operator bool() const { return v != 0; }
};
__device__ __forceinline__ det_t det_raw(unsigned __int128 v) {
    det_t r;
    r.v = v;
    return r;
}
__device__ __forceinline__ det_t operator&(det_t a, det_t b) { return det_raw(a.v & b.v); }
__device__ __forceinline__ det_t operator|(det_t a, det_t b) { return det_raw(a.v | b.v); }
__device__ __forceinline__ det_t operator^(det_t a, det_t b) { return det_raw(a.v ^ b.v); }
__device__ __forceinline__ det_t operator~(det_t a) { return det_raw(~a.v); }
__device__ __forceinline__ det_t operator<<(det_t a, int k) { return det_raw(a.v << k); }
__device__ __forceinline__ det_t operator>>(det_t a, int k) { return det_raw(a.v >> k); }
__device__ __forceinline__ det_t operator-(det_t a, unsigned long long b) { return det_raw(a.v - b); }
__device__ __forceinline__ det_t &operator&=(det_t &a, det_t b) { a.v &= b.v; return a; }
__device__ __forceinline__ det_t &operator|=(det_t &a, det_t b) { a.v |= b.v; return a; }
__device__ __forceinline__ det_t &operator^=(det_t &a, det_t b) { a.v ^= b.v; return a; }
__device__ __forceinline__ bool operator==(det_t a, det_t b) { return a.v == b.v; }
__device__ __forceinline__ bool operator!=(det_t a, det_t b) { return a.v != b.v; }
__device__ __forceinline__ bool operator<(det_t a, det_t b) { return a.v < b.v; }
__device__ __forceinline__ uint64_t lo64(det_t x) { return (uint64_t)x.v; }
__device__ __forceinline__ uint64_t hi64(det_t x) { return (uint64_t)(x.v >> 64); }
__device__ __forceinline__ det_t make_det(uint64_t lo, uint64_t hi) {
    return det_raw(((unsigned __int128)hi << 64) | (unsigned __int128)lo);
}
__device__ __forceinline__ int dpopc(det_t x) { return __popcll(lo64(x)) + __popcll(hi64(x)); }
__device__ __forceinline__ int dctz(det_t x) {
    const uint64_t l = lo64(x);
    return l ? __builtin_ctzll(l) : 64 + __builtin_ctzll(hi64(x));
}
__device__ __forceinline__ int dhib(det_t x) {
    const uint64_t h = hi64(x);
    return h ? 127 - __builtin_clzll(h) : 63 - __builtin_clzll(lo64(x));
}
#endif
constexpr int NSO_MAX = 64 * FQ_DET_WORDS;   // spin orbitals a determinant holds
#define DBIT(p) (det_t(1ull) << (p))
__device__ __forceinline__ det_t even_bits() {
    return make_det(0x5555555555555555ull, 0x5555555555555555ull);
}
__device__ __forceinline__ det_t odd_bits() {
    return make_det(0xAAAAAAAAAAAAAAAAull, 0xAAAAAAAAAAAAAAAAull);
}
// The determinant-valued fields of a system's descriptor.
__device__ __forceinline__ det_t ref_of(const SysDesc &d) { return make_det(d.d0, d.d0_hi); }
__device__ __forceinline__ det_t valid_of(const SysDesc &d) { return make_det(d.valid, d.valid_hi); }
__device__ __forceinline__ det_t cmask_of(const SysDesc &d, int c) {
    return make_det(d.cmask[c], d.cmask_hi[c]);
}
__device__ __forceinline__ det_t *keys_of(const SysDesc &d) { return (det_t *)d.key; }

// ---------------------------------------------------------------------------
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11).
// Counter (bits 0-31 of D, bits 32-63 of D, k, ((iter mod 2^24) << 8) | block),
// key = seed XOR (bits 64-127 of D), i.e. the seed up to 64 spin orbitals.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32->64 product per multiplier gives both halves
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c.z;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        // three-input XORs (0x96 is the truth table of a ^ b ^ c)
        c = make_uint4(__builtin_amdgcn_bitop3_b32(hi1, c.y, k0, 0x96), lo1,
                       __builtin_amdgcn_bitop3_b32(hi0, c.w, k1, 0x96), lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__device__ __forceinline__ void draw2(uint64_t seed, det_t det, uint32_t k, int64_t iter,
                                      uint32_t block, uint64_t &x0, uint64_t &x1) {
    const uint64_t lo = lo64(det), key = seed ^ hi64(det);
    const uint4 ctr = make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), k,
                                 ((uint32_t)((uint64_t)iter & 0xFFFFFFu) << 8) | block);
    const uint4 w = philox10(ctr, (uint32_t)key, (uint32_t)(key >> 32));
    x0 = ((uint64_t)w.y << 32) | (uint64_t)w.x;
    x1 = ((uint64_t)w.w << 32) | (uint64_t)w.z;
}

__device__ __forceinline__ double u01(uint64_t x) {
    return (double)(x >> 11) * (1.0 / 9007199254740992.0);
}

// The four words of one Philox block of a spawning attempt: word 0 picks the
// type and, rescaled within the chosen type's interval, is the acceptance
// uniform; words 1-3 pick the orbitals.
__device__ __forceinline__ uint4 draw_words(uint64_t seed, det_t det, uint32_t k, int64_t iter,
                                            uint32_t block) {
    const uint64_t lo = lo64(det), key = seed ^ hi64(det);
    const uint4 ctr = make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), k,
                                 ((uint32_t)((uint64_t)iter & 0xFFFFFFu) << 8) | block);
    return philox10(ctr, (uint32_t)key, (uint32_t)(key >> 32));
}

// w / 2^32, exact in double.
__device__ __forceinline__ double u01_32(uint32_t w) {
    return (double)w * (1.0 / 4294967296.0);
}

// floor(w n / 2^32): an index in [0, n).
__device__ __forceinline__ uint32_t pick(uint32_t w, uint32_t n) { return __umulhi(w, n); }

// Positions of the set bits of each byte value: the k-th (0-based) set bit of
// byte b sits at bits [3k, 3k + 3) of sel8_entry(b).
__device__ __forceinline__ uint32_t sel8_entry(uint32_t b) {
    uint32_t e = 0, n = 0;
    for (uint32_t i = 0; i < 8; ++i)
        if (b & (1u << i)) {
            e |= i << (3 * n);
            ++n;
        }
    return e;
}

// j (j - 1) / 2 for j < 2^12 (0 for j = 0): the index of the first pair (i, j).
__device__ __forceinline__ uint32_t pair_base(uint32_t j) {
    return (uint32_t)__umul24(j, j - 1u) >> 1;
}

// Position of the k-th (0-based) set bit of x (k < popcount(x)): halving with
// popcounts down to one byte, then that byte's entry of the table sel8 (the
// sel8_entry values, staged in LDS).
__device__ __forceinline__ int select_bit(uint64_t x, uint32_t k, const uint32_t *sel8) {
    int pos = 0;
    uint32_t c = (uint32_t)__popc((uint32_t)x);
    if (k >= c) {
        k -= c;
        x >>= 32;
        pos = 32;
    }
    uint32_t w = (uint32_t)x;
    c = (uint32_t)__popc(w & 0xFFFFu);
    if (k >= c) { k -= c; w >>= 16; pos += 16; }
    c = (uint32_t)__popc(w & 0xFFu);
    if (k >= c) { k -= c; w >>= 8; pos += 8; }
    return pos + (int)((sel8[w & 0xFFu] >> (3u * k)) & 7u);
}
#if FQ_DET_WORDS == 2
__device__ __forceinline__ int select_bit(det_t x, uint32_t k, const uint32_t *sel8) {
    const uint32_t c = (uint32_t)__popcll(lo64(x));
    return k < c ? select_bit(lo64(x), k, sel8) : 64 + select_bit(hi64(x), k - c, sel8);
}
#endif

// 64-bit finaliser of MurmurHash3 (public domain): table placement only.
__device__ __forceinline__ uint64_t mix64(uint64_t h) {
    h ^= h >> 33;
    h *= 0xff51afd7ed558ccdull;
    h ^= h >> 33;
    h *= 0xc4ceb9fe1a85ec53ull;
    h ^= h >> 33;
    return h;
}

// Bucket of a determinant among nb buckets: the high word of mix64(D) * nb, i.e.
// the hash scaled onto [0, nb) (the placement of Sec. 4.1's process hash; the
// paper's Algorithm 1 is kept in the CPU oracle, results do not depend on it).
__device__ __forceinline__ uint32_t bucket_of(det_t D, uint64_t nb) {
#if FQ_DET_WORDS == 1
    return (uint32_t)__umul64hi(mix64(D), nb);
#else
    return (uint32_t)__umul64hi(mix64(lo64(D) ^ mix64(hi64(D) ^ 0x9E3779B97F4A7C15ull)), nb);
#endif
}

// ---------------------------------------------------------------------------
// Hamiltonian (spin orbital p = 2 s + sigma).
// ---------------------------------------------------------------------------
// Packed-pair index; operands stay below 2^24, so 24-bit multiplies are exact.
__device__ __forceinline__ int tri(int i, int j) {
    const int hi = i >= j ? i : j, lo = i >= j ? j : i;
    return (int)(__umul24((unsigned)hi, (unsigned)(hi + 1)) >> 1) + lo;
}

// The integral tables live in global memory; saying so lets the compiler use
// global (not flat) loads, which do not hold up the LDS wait counter.
typedef __attribute__((address_space(1))) const double gdouble;
__device__ __forceinline__ const gdouble *gptr(const double *p) { return (const gdouble *)p; }
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gp(T *p) {
    return (__attribute__((address_space(1))) T *)p;
}
// A load through the constant address space: for a uniform address the compiler
// issues a scalar load (scalar cache, scalar registers). Only for values this kernel
// reads before (or never) writing them.
template <typename T>
__device__ __forceinline__ T ld_uniform(const T *p) {
    return *(const __attribute__((address_space(4))) T *)p;
}

// 16-byte global loads and stores through plain vector types.
typedef int v4i32 __attribute__((ext_vector_type(4)));
typedef unsigned long long v2u64 __attribute__((ext_vector_type(2)));
typedef double v2f64 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ int4 gload_i4(const int32_t *p) {
    const v4i32 v = *gp(reinterpret_cast<const v4i32 *>(p));
    return make_int4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ ulonglong2 gload_u2(const uint64_t *p) {
    const v2u64 v = *gp(reinterpret_cast<const v2u64 *>(p));
    return make_ulonglong2(v.x, v.y);
}
__device__ __forceinline__ double2 gload_d2(const double *p) {
    const v2f64 v = *gp(reinterpret_cast<const v2f64 *>(p));
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ void gstore_i4(void *p, int x, int y, int z, int w) {
    v4i32 v;
    v.x = x;
    v.y = y;
    v.z = z;
    v.w = w;
    *gp(reinterpret_cast<v4i32 *>(p)) = v;
}

// Main-list keys in global memory (one 16-byte access for two words).
#if FQ_DET_WORDS == 1
__device__ __forceinline__ det_t ldk(const det_t *p) { return *gp(p); }
__device__ __forceinline__ void stk(det_t *p, det_t v) { *gp(p) = v; }
#else
__device__ __forceinline__ det_t ldk(const det_t *p) {
    const ulonglong2 w = gload_u2((const uint64_t *)p);
    return make_det(w.x, w.y);
}
__device__ __forceinline__ void stk(det_t *p, det_t v) {
    v2u64 w;
    w.x = lo64(v);
    w.y = hi64(v);
    *gp(reinterpret_cast<v2u64 *>(p)) = w;
}
#endif

// Spawn records: one 16-byte access each (two for two-word determinants, whose
// records take 32 bytes).
#if FQ_DET_WORDS == 1
typedef SpawnRec rec_t;
__device__ __forceinline__ void put_rec(rec_t *p, det_t D, int32_t w, uint32_t tag) {
    gstore_i4(p, (int)(uint32_t)D, (int)(uint32_t)(D >> 32), w, (int)tag);
}
__device__ __forceinline__ rec_t get_rec(const rec_t *p) {
    const int4 x = gload_i4((const int32_t *)p);
    rec_t r;
    r.det = (uint64_t)(uint32_t)x.x | ((uint64_t)(uint32_t)x.y << 32);
    r.w = x.z;
    r.tag = (uint32_t)x.w;
    return r;
}
#else
struct __attribute__((aligned(16))) rec_t {
    det_t det;
    int32_t w;
    uint32_t tag;
    uint64_t pad;
};
static_assert(sizeof(rec_t) == 32, "two-word spawn records take 32 bytes");
__device__ __forceinline__ void put_rec(rec_t *p, det_t D, int32_t w, uint32_t tag) {
    const uint64_t lo = lo64(D), hi = hi64(D);
    gstore_i4(p, (int)(uint32_t)lo, (int)(uint32_t)(lo >> 32), (int)(uint32_t)hi,
              (int)(uint32_t)(hi >> 32));
    gstore_i4((char *)p + 16, w, (int)tag, 0, 0);
}
__device__ __forceinline__ rec_t get_rec(const rec_t *p) {
    const int4 x = gload_i4((const int32_t *)p);
    const int4 y = gload_i4((const int32_t *)p + 4);
    rec_t r;
    r.det = make_det((uint64_t)(uint32_t)x.x | ((uint64_t)(uint32_t)x.y << 32),
                     (uint64_t)(uint32_t)x.z | ((uint64_t)(uint32_t)x.w << 32));
    r.w = y.x;
    r.tag = (uint32_t)y.y;
    return r;
}
#endif
static_assert(sizeof(rec_t) == 16 * FQ_DET_WORDS, "record size");
__device__ __forceinline__ rec_t *recs_of(const EngineArgs &a) { return (rec_t *)a.recs; }
__device__ __forceinline__ rec_t *srt_of(const EngineArgs &a) { return (rec_t *)a.srt; }
__device__ __forceinline__ det_t *spill_dets(const EngineArgs &a) { return (det_t *)a.sp_det; }

__device__ __forceinline__ double eri_so(const SysDesc &d, int p, int q, int r, int s) {
    if (((p ^ q) | (r ^ s)) & 1) return 0.0;
    return gptr(d.eri)[tri(tri(p >> 1, q >> 1), tri(r >> 1, s >> 1))];
}

__device__ __forceinline__ double h_so(const SysDesc &d, int p, int q) {
    if ((p ^ q) & 1) return 0.0;
    return gptr(d.h1)[(p >> 1) * d.M + (q >> 1)];
}

// Both words are read at uniform addresses (scalar loads); the lane's label is
// then picked out with ALU operations only.
__device__ __forceinline__ int irrep_of(const SysDesc &d, int s) {
#if FQ_DET_WORDS == 1
    const uint64_t w0 = d.irr_packed[0], w1 = d.irr_packed[1];
#else
    const uint64_t w0 = (s & 32) ? d.irr_packed_hi[0] : d.irr_packed[0];
    const uint64_t w1 = (s & 32) ? d.irr_packed_hi[1] : d.irr_packed[1];
#endif
    return (int)((((s & 16) ? w1 : w0) >> (4 * (s & 15))) & 0xFull);
}

__device__ __forceinline__ int class_of(const SysDesc &d, int p) {
    return 2 * irrep_of(d, p >> 1) + (p & 1);
}

// The orbitals strictly between p and a, and the parity of the occupied ones.
__device__ __forceinline__ det_t between_mask(int p, int a) {
    const int lo = p < a ? p : a, hi = p < a ? a : p;
    return (DBIT(hi) - 1ull) & ~((det_t(2ull) << lo) - 1ull);
}
__device__ __forceinline__ int between_parity(det_t det, int p, int a) {
    return dpopc(det & between_mask(p, a)) & 1;
}

__device__ double hdiag_of(const SysDesc &d, det_t det) {
    double acc = d.e_core;
    for (det_t m = det; m; m &= m - 1ull) {
        const int p = dctz(m);
        acc = acc + h_so(d, p, p);
    }
    for (det_t m1 = det; m1; m1 &= m1 - 1ull) {
        const int p = dctz(m1);
        for (det_t m2 = m1 & (m1 - 1ull); m2; m2 &= m2 - 1ull) {
            const int q = dctz(m2);
            acc = acc + (eri_so(d, p, p, q, q) - eri_so(d, p, q, q, p));
        }
    }
    return acc;
}

// Single excitation p -> a: h_pa + sum over occupied q != p (ascending) of
// (pa|qq) - [same spin](pq|qa), each term read from the precomputed row
// t3[p][a][*]; four loads are issued before they are added, in order.
__device__ double hel_single(const SysDesc &d, det_t det, int p, int a) {
    double acc = h_so(d, p, a);
    const gdouble *row = gptr(d.t3) + ((p * NSO_MAX + a) * NSO_MAX);
    det_t m = det & ~DBIT(p);
    while (m) {
        const int q0 = dctz(m);
        m &= m - 1ull;
        const int q1 = m ? dctz(m) : q0;
        m &= m - 1ull;
        const int q2 = m ? dctz(m) : q0;
        m &= m - 1ull;
        const int q3 = m ? dctz(m) : q0;
        const int n = 1 + (q1 != q0) + (q2 != q0) + (q3 != q0);
        m &= m - 1ull;
        const double v0 = row[q0], v1 = row[q1], v2 = row[q2], v3 = row[q3];
        acc = acc + v0;
        if (n > 1) acc = acc + v1;
        if (n > 2) acc = acc + v2;
        if (n > 3) acc = acc + v3;
    }
    return between_parity(det, p, a) ? -acc : acc;
}

// p < q occupied, a, b empty. Pairing: unlike spins -> a' carries p's spin;
// like spins -> a' = min(a, b). Sign: q -> b' on det, then p -> a'.
__device__ double hel_double(const SysDesc &d, det_t det, int p, int q, int a, int b) {
    int ap, bp;
    if ((p ^ q) & 1) {
        const bool a_with_p = ((a ^ p) & 1) == 0;
        ap = a_with_p ? a : b;
        bp = a_with_p ? b : a;
    } else {
        ap = a < b ? a : b;
        bp = a < b ? b : a;
    }
    // the two parities at once: parity(x) ^ parity(y) = parity(x ^ y)
    const det_t d1 = (det & ~DBIT(q)) | DBIT(bp);
    const int par = dpopc((det & between_mask(q, bp)) ^ (d1 & between_mask(p, ap))) & 1;
    const double v = eri_so(d, p, ap, q, bp) - eri_so(d, p, bp, q, ap);
    return par ? -v : v;
}

// Whether a child lies in the system's restricted space (Sec. 5: outside it the
// excitation is null). Excitation level: electrons outside the reference's
// orbitals; seniority: spatial orbitals holding exactly one electron.
__device__ __forceinline__ bool in_space(const SysDesc &d, det_t det) {
    const int sp = d.space;
    if ((sp & 1) && dpopc(det & ~ref_of(d)) > d.max_ex) return false;
    if ((sp & 2) && dpopc((det ^ (det >> 1)) & even_bits()) > d.max_sen) return false;
    const det_t fo = make_det(d.frz_occ, d.frz_occ_hi), fe = make_det(d.frz_emp, d.frz_emp_hi);
    if ((sp & 4) && ((det & fo) != fo || (det & fe))) return false;
    return true;
}

// <det|H|d0> for det != d0 within two excitations of d0 (d0 is the source).
__device__ double hel_to_ref(const SysDesc &d, det_t det) {
    const det_t d0 = ref_of(d);
    const det_t from = d0 & ~det, to = det & ~d0;
    const int nd = dpopc(from);
    if (nd == 1) return hel_single(d, d0, dctz(from), dctz(to));
    const int p = dctz(from), q = dhib(from);
    const int a = dctz(to), b = dhib(to);
    return hel_double(d, d0, p, q, a, b);
}

// ---------------------------------------------------------------------------
// Excitation generation (Sec. 5). Symmetry classes are (irrep, spin) with
// class id 2*irrep + spin; cmask[c] holds the spin orbitals of class c.
// Returns false for a null excitation.
// ---------------------------------------------------------------------------
struct Excit {
    det_t det;
    double pgen;
    double hel;
    int p, a;
};


// Symmetry classes seen from the excitation generator. With no point group
// (every orbital in irrep 0, two classes: the spins) everything is bit
// arithmetic; otherwise the class masks are read from an LDS copy, since the
// class index differs between lanes.
template <bool C1>
struct ClassView {
    det_t valid;
    const det_t *cm;      // LDS copy of SysDesc::cmask (unused when C1)
    __device__ __forceinline__ det_t mask(int c) const {
        if (C1) return valid & ((c & 1) ? odd_bits() : even_bits());
        return cm[c];
    }
    __device__ __forceinline__ int irrep(const SysDesc &d, int s) const {
        return C1 ? 0 : irrep_of(d, s);
    }
    __device__ __forceinline__ int cls(const SysDesc &d, int p) const {
        return C1 ? (p & 1) : class_of(d, p);
    }
};

// Single excitation (Sec. 5.1) from the electron word w1 and the hole word w2:
// renormalised over the electrons that have an allowed target. Returns false
// for a null excitation; otherwise the child, pgen and the orbitals p -> a.
template <bool C1>
__device__ __forceinline__ bool excite_single(const SysDesc &d, const ClassView<C1> &cv,
                                              det_t det, uint32_t w1, uint32_t w2,
                                              const uint32_t *sel8, Excit &ex) {
    const det_t emp = ~det & valid_of(d);
    const int n_class = C1 ? 2 : d.n_class;
    det_t movable = det_t(0ull);
    for (int c = 0; c < n_class; ++c) {
        const det_t cm = C1 ? cv.mask(c) : cmask_of(d, c);
        if (emp & cm) movable |= det & cm;
    }
    const uint32_t nmov = (uint32_t)dpopc(movable);
    if (nmov == 0) return false;
    const int p = select_bit(movable, pick(w1, nmov), sel8);
    const det_t tg = emp & cv.mask(cv.cls(d, p));
    const uint32_t nal = (uint32_t)dpopc(tg);
    const int a = select_bit(tg, pick(w2, nal), sel8);
    ex.det = det ^ DBIT(p) ^ DBIT(a);
    ex.pgen = d.p_single / (double)((int64_t)nal * (int64_t)nmov);
    ex.p = p;
    ex.a = a;
    return true;
}

constexpr int EX_NULL = 0, EX_OK = 1, EX_SINGLE_DEFERRED = 2;

// One excitation from the words of one Philox block: w.x (type), w.y
// (electron or pair), w.z, w.w (holes). recip[k] = 1.0 / k, filled by IEEE
// division (same bits as dividing in place). With defer_single a single
// excitation is only recognised (EX_SINGLE_DEFERRED): the caller queues its
// words and generates it later, so the rare singles do not make whole
// wavefronts run the single path.
template <bool C1>
__device__ __forceinline__ int excite(const SysDesc &d, const ClassView<C1> &cv, det_t det,
                                      uint4 w, const double *recip, const uint32_t *sel8,
                                      bool defer_single, Excit &ex) {
    const det_t emp = ~det & valid_of(d);
    const int N = d.N;
    const int n_class = C1 ? 2 : d.n_class;
    if (!(u01_32(w.x) < d.p_double)) {
        if (defer_single) return EX_SINGLE_DEFERRED;
        if (!excite_single(d, cv, det, w.y, w.z, sel8, ex)) return EX_NULL;
        ex.hel = hel_single(d, det, ex.p, ex.a);
        return EX_OK;
    }
    // Double (Sec. 5.2): a unique pair by inverse triangular indexing.
    if (N < 2) return EX_NULL;
    const uint32_t npairs = (uint32_t)(N * (N - 1) / 2);
    const uint32_t K = pick(w.y, npairs);   // < 2016
    // The estimate from the hardware square root is within one of j (the largest
    // j with j (j - 1) / 2 <= K); one exact integer correction each way.
    // (float)(8 K + 1), exact below 2^23, by the mantissa trick
    const float x = __int_as_float((int)(0x4B000000u | (8u * K + 1u))) - 8388608.0f;
    uint32_t j = (uint32_t)((1.0f + __builtin_amdgcn_sqrtf(x)) * 0.5f);
    j -= pair_base(j) > K ? 1u : 0u;
    j += pair_base(j + 1) <= K ? 1u : 0u;
    const uint32_t i = K - pair_base(j);
    const int p = select_bit(det, i, sel8), q = select_bit(det, j, sel8);
    const bool same = ((p ^ q) & 1) == 0;
    int a, b;
    if (C1) {
        // No point group: every determinant has the same number of empty orbitals of
        // each spin (d.n_emp), so the allowed sets and their sizes follow from the
        // spins alone, and pgen is one of four per-system values (the general branch
        // below gives the same sets, counts and pgen).
        const int sp = p & 1;
        const det_t e0 = emp & even_bits(), e1 = emp & odd_bits();
        const uint32_t n0 = (uint32_t)d.n_emp[0], n1 = (uint32_t)d.n_emp[1];
        det_t allowed;
        uint32_t nal;
        if (same) {
            allowed = sp ? e1 : e0;
            const uint32_t ne = sp ? n1 : n0;
            nal = ne >= 2 ? ne : 0;
        } else {
            allowed = (n1 > 0 ? e0 : det_t(0ull)) | (n0 > 0 ? e1 : det_t(0ull));
            nal = (n1 > 0 ? n0 : 0u) + (n0 > 0 ? n1 : 0u);
        }
        if (nal == 0) return EX_NULL;
        a = select_bit(allowed, pick(w.z, nal), sel8);
        const int sa = a & 1;
        const det_t bset = same ? (allowed & ~DBIT(a)) : (sa ? e0 : e1);
        const uint32_t nba = same ? nal - 1 : (sa ? n0 : n1);
        b = select_bit(bset, pick(w.w, nba), sel8);
        ex.pgen = same ? (sp ? d.pgen_c1[1] : d.pgen_c1[0]) : (sa ? d.pgen_c1[3] : d.pgen_c1[2]);
    } else {
        const det_t A = same ? (emp & ((p & 1) ? odd_bits() : even_bits())) : emp;
        const int gpq = cv.irrep(d, p >> 1) ^ cv.irrep(d, q >> 1);
        // a orbitals whose partner class (Eq. sym1 plus spin) has an empty orbital besides a.
        det_t allowed = det_t(0ull);
        for (int c = 0; c < n_class; ++c) {
            const det_t memb = A & cmask_of(d, c);
            if (!memb) continue;
            const int sb = same ? (p & 1) : 1 - (c & 1);
            const int pc = 2 * (gpq ^ (c >> 1)) + sb;
            const int nb = dpopc(emp & cv.mask(pc)) - (pc == c ? 1 : 0);
            if (nb > 0) allowed |= memb;
        }
        const uint32_t nal = (uint32_t)dpopc(allowed);
        if (nal == 0) return EX_NULL;
        a = select_bit(allowed, pick(w.z, nal), sel8);
        const int ca = cv.cls(d, a);
        const int pca = 2 * (gpq ^ (ca >> 1)) + (same ? (p & 1) : 1 - (ca & 1));
        const det_t bset = emp & cv.mask(pca) & ~DBIT(a);
        const uint32_t nba = (uint32_t)dpopc(bset);
        b = select_bit(bset, pick(w.w, nba), sel8);
        const int cb = cv.cls(d, b);
        const int pcb = 2 * (gpq ^ (cb >> 1)) + (same ? (p & 1) : 1 - (cb & 1));
        const int nbb = dpopc(emp & cv.mask(pcb)) - (pcb == cb ? 1 : 0);
        ex.pgen = (2.0 * d.p_double * (recip[nba] + recip[nbb])) /
                  (double)((int64_t)N * (int64_t)(N - 1) * (int64_t)nal);
    }
    ex.det = det ^ DBIT(p) ^ DBIT(q) ^ DBIT(a) ^ DBIT(b);
    ex.hel = hel_double(d, det, p, q, a, b);
    return EX_OK;
}

// ---------------------------------------------------------------------------
// Spin-coupled functions (Sec. 5.3, Eqs. EqualCoeffs and SpinCoup). With spin
// orbitals interleaved, exchanging alpha and beta in every spatial orbital maps
// |D> to (-1)^{n2(D)} |D~> (n2: doubly occupied orbitals); the function of the
// pair {D, D~} is (|D> + lam (-1)^{n2(D)} |D~>)/sqrt2, lam = (-1)^S (-1)^{N/2}
// (SysDesc::lam), or |D> for a closed pair D = D~ (even S only). A function is
// stored as min(D, D~); excitations are drawn from that determinant only.
// ---------------------------------------------------------------------------
__device__ __forceinline__ det_t spin_flip(det_t D) {
    return ((D & even_bits()) << 1) | ((D >> 1) & even_bits());
}
__device__ __forceinline__ det_t fn_rep(det_t D) {
    const det_t f = spin_flip(D);
    return f < D ? f : D;
}
__device__ __forceinline__ int pair_sign(const SysDesc &d, det_t D) {
    return (dpopc(D & (D >> 1) & even_bits()) & 1) ? -d.lam : d.lam;
}

// <bra|H|ket> for a single or double excitation with ket the source (0 beyond).
__device__ double hel_between(const SysDesc &d, det_t bra, det_t ket) {
    const det_t from = ket & ~bra, to = bra & ~ket;
    const int n = dpopc(from);
    if (n == 1) return hel_single(d, ket, dctz(from), dctz(to));
    if (n == 2) return hel_double(d, ket, dctz(from), dhib(from), dctz(to), dhib(to));
    return 0.0;
}

// <Phi_j|H|Phi_i> for the stored functions Dj != Di, Di the source: both open,
// <Dj|H|Di> + lam (-1)^{n2(Dj)} <Dj~|H|Di>; one closed, sqrt2 <Dj|H|Di>; both
// closed, <Dj|H|Di>.
__device__ double fn_hel(const SysDesc &d, det_t Di, det_t Dj) {
    const det_t fi = spin_flip(Di), fj = spin_flip(Dj);
    const double h = hel_between(d, Dj, Di);
    if (fi != Di && fj != Dj) return h + (double)pair_sign(d, Dj) * hel_between(d, fj, Di);
    if (fi != Di || fj != Dj) return 1.4142135623730951 * h;
    return h;
}

// Diagonal element of a stored function from its determinant's diagonal hd.
__device__ __forceinline__ double fn_diag_from(const SysDesc &d, det_t D, double hd) {
    if (!d.hphf) return hd;
    const det_t f = spin_flip(D);
    if (f == D) return hd;
    return hd + (double)pair_sign(d, D) * hel_between(d, f, D);
}
__device__ double fn_diag(const SysDesc &d, det_t D) { return fn_diag_from(d, D, hdiag_of(d, D)); }

// Projected-energy element <Phi_0|H|Phi_D> (Eq. ProjE) and whether it can be
// nonzero (D within a double excitation of the reference, or its partner).
__device__ __forceinline__ bool near_ref(const SysDesc &d, det_t D) {
    return dpopc(D ^ ref_of(d)) <= 4 || (d.hphf && dpopc(spin_flip(D) ^ ref_of(d)) <= 4);
}
__device__ double ref_hel(const SysDesc &d, det_t D) {
    return d.hphf ? fn_hel(d, ref_of(d), D) : hel_to_ref(d, D);
}

// The probability that excite() draws T from det (Secs. 5.1, 5.2) by the same
// operations as the draw, 0 when it cannot draw T. recip[k] = 1/k.
__device__ double pgen_target(const SysDesc &d, const det_t *cm, const double *recip,
                              det_t det, det_t T) {
    const det_t from = det & ~T, to = T & ~det;
    const int nf = dpopc(from);
    if (nf != dpopc(to)) return 0.0;
    const det_t emp = ~det & valid_of(d);
    const bool c1 = d.n_class == 2;
    auto mask = [&](int c) -> det_t {
        return c1 ? (valid_of(d) & ((c & 1) ? odd_bits() : even_bits())) : cm[c];
    };
    auto cls = [&](int p) -> int { return c1 ? (p & 1) : class_of(d, p); };
    if (nf == 1) {
        const int p = dctz(from), a = dctz(to);
        if (cls(a) != cls(p)) return 0.0;
        det_t movable = det_t(0ull);
        for (int c = 0; c < (c1 ? 2 : d.n_class); ++c) {
            const det_t m = mask(c);
            if (emp & m) movable |= det & m;
        }
        const uint32_t nmov = (uint32_t)dpopc(movable);
        const uint32_t nal = (uint32_t)dpopc(emp & mask(cls(p)));
        return d.p_single / (double)((int64_t)nal * (int64_t)nmov);
    }
    if (nf != 2) return 0.0;
    const int p = dctz(from), q = dhib(from);
    const int a = dctz(to), b = dhib(to);
    const bool same = ((p ^ q) & 1) == 0;
    if (same ? (((a ^ p) & 1) || ((b ^ p) & 1)) : (((a ^ b) & 1) == 0)) return 0.0;
    if (c1) return same ? d.pgen_c1[p & 1] : d.pgen_c1[2 + (a & 1)];
    const int gpq = irrep_of(d, p >> 1) ^ irrep_of(d, q >> 1);
    const int ca = class_of(d, a), cb = class_of(d, b);
    const int pca = 2 * (gpq ^ (ca >> 1)) + (same ? (p & 1) : 1 - (ca & 1));
    if (cb != pca) return 0.0;
    const det_t A = same ? (emp & ((p & 1) ? odd_bits() : even_bits())) : emp;
    det_t allowed = det_t(0ull);
    for (int c = 0; c < d.n_class; ++c) {
        const det_t memb = A & cm[c];
        if (!memb) continue;
        const int sb = same ? (p & 1) : 1 - (c & 1);
        const int pc = 2 * (gpq ^ (c >> 1)) + sb;
        const int nb = dpopc(emp & cm[pc]) - (pc == c ? 1 : 0);
        if (nb > 0) allowed |= memb;
    }
    const uint32_t nal = (uint32_t)dpopc(allowed);
    const int pcb = 2 * (gpq ^ (cb >> 1)) + (same ? (p & 1) : 1 - (cb & 1));
    const uint32_t nba = (uint32_t)dpopc(emp & cm[pca] & ~DBIT(a));
    const int nbb = dpopc(emp & cm[pcb]) - (pcb == cb ? 1 : 0);
    return (2.0 * d.p_double * (recip[nba] + recip[nbb])) /
           (double)((int64_t)d.N * (int64_t)(d.N - 1) * (int64_t)nal);
}

// A drawn excitation as a spawn between stored functions: the target is the
// function holding the child, reached through the child or its partner (their
// probabilities add); the pair of the source itself is diagonal (null), and so is a
// closed pair in an odd-spin run. Returns false for a null excitation.
__device__ bool to_function(const SysDesc &d, const det_t *cm, const double *recip,
                            det_t D, Excit &ex) {
    const det_t Dj = fn_rep(ex.det), fx = spin_flip(ex.det);
    if (Dj == D || (d.hphf < 0 && spin_flip(Dj) == Dj)) return false;
    if (fx != ex.det) ex.pgen = ex.pgen + pgen_target(d, cm, recip, D, fx);
    ex.hel = fn_hel(d, D, Dj);
    ex.det = Dj;
    return true;
}

// Natural log for the shift update: x = m 2^e with m in (1/sqrt2, sqrt2],
// ln x = e ln2 + 2 atanh((m-1)/(m+1)), the atanh series summed by Horner's
// rule through the z^25 term. Fixed operation order (no contraction), so any
// IEEE-double implementation of the same method returns the same bits.
__device__ double shift_log(double x) {
    const uint64_t bits = (uint64_t)__double_as_longlong(x);
    int e = (int)((bits >> 52) & 0x7FFull) - 1023;
    double m = __longlong_as_double((long long)((bits & 0x000FFFFFFFFFFFFFull) |
                                                0x3FF0000000000000ull));
    if (m > 1.4142135623730951) {
        m = m * 0.5;
        e = e + 1;
    }
    const double z = (m - 1.0) / (m + 1.0);
    const double z2 = z * z;
    double sum = 1.0 / 27.0;
    for (int k = 25; k >= 1; k -= 2) sum = sum * z2 + 1.0 / (double)k;
    return (double)e * 0.6931471805599453 + 2.0 * z * sum;
}

__device__ __forceinline__ bool participating(const SysDesc &d, uint32_t status) {
    return d.active && status == 0 && d.iter < d.stop_at;
}

// ---------------------------------------------------------------------------
// Block reductions (256 threads, fixed order -> deterministic).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T block_sum(T v, T *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = (int)blockDim.x / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] = sh[t] + sh[t + s];
        __syncthreads();
    }
    const T r = sh[0];
    __syncthreads();
    return r;
}

// Sum over the 64 lanes of a wavefront with a fixed butterfly (deterministic).
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    for (int o = 32; o > 0; o >>= 1) v = v + __shfl_xor(v, o, 64);
    return v;
}

// Inclusive prefix sum over the 64 lanes of a wavefront by data-parallel primitives
// (DPP): shifts within rows of 16 lanes, then row broadcasts (no LDS traffic).
template <int CTRL>
__device__ __forceinline__ unsigned long long dpp_move(unsigned long long v) {
    const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)v, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(v >> 32), CTRL, 0xF, 0xF, false);
    return (unsigned long long)(uint32_t)lo | ((unsigned long long)(uint32_t)hi << 32);
}
__device__ __forceinline__ unsigned long long wave_incl_scan(unsigned long long x) {
    const int lane = threadIdx.x & 63, r = lane & 15;
    unsigned long long y = dpp_move<0x111>(x);   // row_shr:1
    if (r >= 1) x += y;
    y = dpp_move<0x112>(x);                      // row_shr:2
    if (r >= 2) x += y;
    y = dpp_move<0x114>(x);                      // row_shr:4
    if (r >= 4) x += y;
    y = dpp_move<0x118>(x);                      // row_shr:8
    if (r >= 8) x += y;
    y = dpp_move<0x142>(x);                      // row_bcast:15 (last lane of the row below)
    if (lane & 16) x += y;
    y = dpp_move<0x143>(x);                      // row_bcast:31 (lane 31, to the upper half)
    if (lane >= 32) x += y;
    return x;
}

// Halves of the chunk sums and range sums: this iteration's in (step & 1).
__device__ __forceinline__ unsigned cur_half(const EngineArgs &a) { return (unsigned)(*a.step & 1ull); }
__device__ __forceinline__ unsigned long long *sums(const EngineArgs &a, unsigned h) {
    return a.chunk_nw + (h ? a.chunk_cap : 0);
}
__device__ __forceinline__ unsigned long long *ranges(const EngineArgs &a, unsigned h) {
    return a.blk + (h ? 4 * SCAN_G : 0);
}

// ---------------------------------------------------------------------------
// K1: chunk sums of |C| on the current tables. Workgroup g takes the chunks
// [g per, (g+1) per) (per = ceil(chunks / SCAN_G)), four at a time, writes
// each chunk's sum and the range's total attempts and spawn tiles.
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long abs_sum4(int4 v) {
    return (unsigned long long)(abs(v.x)) + (unsigned long long)(abs(v.y)) +
           (unsigned long long)(abs(v.z)) + (unsigned long long)(abs(v.w));
}

__global__ __launch_bounds__(256) void k_chunk_sum(EngineArgs a,
                                                   const SysDesc *__restrict__ desc) {
    __shared__ unsigned long long sh[4][4];
    const int64_t nch = *a.nchunks;
    const int64_t per = (nch + SCAN_G - 1) / SCAN_G;
    const int64_t c0 = (int64_t)blockIdx.x * per;
    const int64_t c1 = c0 + per < nch ? c0 + per : nch;
    const int tsh = __builtin_ctzll((unsigned long long)a.tile);
    const unsigned long long tm = (unsigned long long)a.tile - 1ull;
    const int t = threadIdx.x;
    unsigned long long *const nws = sums(a, cur_half(a));
    unsigned long long *const rg = ranges(a, cur_half(a));
    unsigned long long bs = 0, bt = 0;    // range totals, kept by thread 0
    for (int64_t c = c0; c < c1; c += 4) {
        unsigned long long v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = 0;
            const int64_t cc = c + k;
            if (cc < c1) {
                const int sy = a.chunk_sys[cc];
                if (sy >= 0) {
                    // the chunk's four buckets, one per wavefront, four entries per lane
                    const SysDesc &d = desc[sy];
                    const int64_t lb = (int64_t)a.chunk_local[cc] * BPC + (t >> 6);
                    const int e = 4 * (t & 63);
                    const int n = d.bcnt[lb];
                    if (participating(d, a.status[sy]) && e < n) {
                        int4 q = *reinterpret_cast<const int4 *>(d.pop + lb * BQ + e);
                        if (e + 1 >= n) q.y = 0;
                        if (e + 2 >= n) q.z = 0;
                        if (e + 3 >= n) q.w = 0;
                        v[k] = abs_sum4(q);
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const unsigned long long w = wave_sum(v[k]);
            if ((t & 63) == 0) sh[k][t >> 6] = w;
        }
        __syncthreads();
        if (t == 0) {
            for (int k = 0; k < 4 && c + k < c1; ++k) {
                const unsigned long long x = sh[k][0] + sh[k][1] + sh[k][2] + sh[k][3];
                nws[c + k] = x;
                bs += x;
                bt += (x + tm) >> tsh;
            }
        }
        __syncthreads();
    }
    if (t == 0) {
        rg[blockIdx.x] = bs;
        rg[SCAN_G + blockIdx.x] = bt;
    }
}

// ---------------------------------------------------------------------------
// K2a: exclusive scan of the SCAN_G range totals (one workgroup, two per
// thread); also resets the dynamic work counters of the spawn and post kernels
// and the range sums that k_post accumulates for the next iteration.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_scan(EngineArgs a) {
    __shared__ unsigned long long part[1024], tpart[1024];
    const int t = threadIdx.x;
    unsigned long long *const rg = ranges(a, cur_half(a));
    unsigned long long *const rn = ranges(a, cur_half(a) ^ 1u);
    rn[2 * t] = 0ull;
    rn[2 * t + 1] = 0ull;
    rn[SCAN_G + 2 * t] = 0ull;
    rn[SCAN_G + 2 * t + 1] = 0ull;
    const unsigned long long s0 = rg[2 * t], s1 = rg[2 * t + 1];
    const unsigned long long t0 = rg[SCAN_G + 2 * t], t1 = rg[SCAN_G + 2 * t + 1];
    part[t] = s0 + s1;
    tpart[t] = t0 + t1;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const unsigned long long v = t >= off ? part[t - off] : 0ull;
        const unsigned long long vt = t >= off ? tpart[t - off] : 0ull;
        __syncthreads();
        part[t] += v;
        tpart[t] += vt;
        __syncthreads();
    }
    const unsigned long long run = part[t] - (s0 + s1), trun = tpart[t] - (t0 + t1);
    rg[2 * SCAN_G + 2 * t] = run;
    rg[2 * SCAN_G + 2 * t + 1] = run + s0;
    rg[3 * SCAN_G + 2 * t] = trun;
    rg[3 * SCAN_G + 2 * t + 1] = trun + t0;
    if (t == 1023) {
        a.total[0] = part[1023];
        a.total[1] = tpart[1023];
        a.work[0] = 0u;
        a.work[1] = 0u;
    }
}

// ---------------------------------------------------------------------------
// K2b: per chunk, the exclusive scans of |C| sums (attempt offsets) and of
// spawn tiles, inside each range from the range's offset.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_scan_down(EngineArgs a) {
    __shared__ unsigned long long ws[4], wt[4];
    const int64_t nch = *a.nchunks;
    const int64_t per = (nch + SCAN_G - 1) / SCAN_G;
    const int64_t c0 = (int64_t)blockIdx.x * per;
    const int64_t c1 = c0 + per < nch ? c0 + per : nch;
    const int tsh = __builtin_ctzll((unsigned long long)a.tile);
    const unsigned long long tm = (unsigned long long)a.tile - 1ull;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const unsigned long long *const nws = sums(a, cur_half(a));
    const unsigned long long *const rg = ranges(a, cur_half(a));
    unsigned long long base = rg[2 * SCAN_G + blockIdx.x];
    unsigned long long tbase = rg[3 * SCAN_G + blockIdx.x];
    for (int64_t c = c0; c < c1; c += 256) {
        const int64_t i = c + t;
        const unsigned long long v = i < c1 ? nws[i] : 0ull;
        const unsigned long long vt = (v + tm) >> tsh;
        // inclusive scans inside the wavefront
        unsigned long long x = v, xt = vt;
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned long long y = __shfl_up(x, o, 64);
            const unsigned long long yt = __shfl_up(xt, o, 64);
            if (lane >= o) {
                x += y;
                xt += yt;
            }
        }
        if (lane == 63) {
            ws[w] = x;
            wt[w] = xt;
        }
        __syncthreads();
        unsigned long long pre = 0, pret = 0;
        for (int k = 0; k < w; ++k) {
            pre += ws[k];
            pret += wt[k];
        }
        // The chunk of each of its tiles, for k_spawn's tile grabs: up to eight by the
        // chunk's thread, the rest (the reference determinant's chunk has thousands)
        // by the whole wavefront.
        const unsigned long long to = tbase + pret + xt - vt;
        const unsigned long long cap = (unsigned long long)a.tile_cap;
        if (i < c1) {
            a.chunk_off[i] = base + pre + x - v;
            a.chunk_toff[i] = to;
            const unsigned long long te = to + (vt < 8ull ? vt : 8ull);
            for (unsigned long long k = to; k < te && k < cap; ++k) a.tile_chunk[k] = (uint32_t)i;
        }
        for (uint64_t big = __ballot(i < c1 && vt > 8ull); big; big &= big - 1) {
            const int l = __builtin_ctzll(big);
            const unsigned long long tl = __shfl(to, l, 64), vl = __shfl(vt, l, 64);
            const unsigned long long te = tl + vl < cap ? tl + vl : cap;
            for (unsigned long long k = tl + 8ull + (unsigned long long)lane; k < te; k += 64ull)
                a.tile_chunk[k] = (uint32_t)(c + 64 * w + l);
        }
        base += ws[0] + ws[1] + ws[2] + ws[3];
        tbase += wt[0] + wt[1] + wt[2] + wt[3];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// K3: spawning. Attempts are numbered globally; a workgroup takes a tile of
// consecutive attempts, stages the keys and populations of the chunk(s)
// covering it in LDS with a prefix sum of |C|, and each thread walks a run of
// consecutive attempts: (slot, walker ordinal k) by one binary search, then
// k+1 / next occupied slot.
// ---------------------------------------------------------------------------

// Spawn records. A record is (child, signed walkers, child's global bucket |
// initiator flag << 31, rank among that bucket's records), appended to the
// iteration's record buffer; the rank comes from the bucket's record counter. A
// record that would land past the buffer's capacity is dropped and the system
// marked: the iteration is then abandoned and re-run after the buffer grows.
// Walkers spawned onto the reference go to a per-system sum instead (every
// iteration sends it many: the reference is the hot spot of Sec. 4.1).
constexpr uint32_t REC_UNRANKED = 0x40000000u;
__device__ __forceinline__ void put_record(const EngineArgs &a, const SysDesc &d, int s,
                                           unsigned long long j, det_t D, int32_t v, bool init,
                                           uint32_t *status) {
    if (j >= (unsigned long long)a.rec_cap) {
        atomicOr(status, ST_TABLE_FULL);
        return;
    }
    const uint32_t gb = (uint32_t)(d.gchunk0 * BPC) + bucket_of(D, (uint64_t)d.nbuckets);
    a.rec_rank[j] = __hip_atomic_fetch_add(&a.bhist[gb], 1u, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
    put_rec(recs_of(a) + j, D, v, gb | (init ? 0x80000000u : 0u));
}

// One record per active lane, with one buffer reservation for the wavefront
// (callable from divergent code). Its bucket and rank are left to k_fix, which
// keeps this path short in the spawning loop.
__device__ __forceinline__ void put_record_wave(const EngineArgs &a, int s, det_t D, int32_t v,
                                                bool init, uint32_t *status) {
    const uint64_t m = __ballot(1);
    const int lane = threadIdx.x & 63;
    const int leader = __builtin_ctzll(m);
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(a.rec_count, (unsigned long long)__popcll(m));
    base = __shfl(base, leader, 64);
    const unsigned long long j = base + (unsigned long long)__popcll(m & ((1ull << lane) - 1ull));
    if (j >= (unsigned long long)a.rec_cap) {
        atomicOr(status, ST_TABLE_FULL);
        return;
    }
    put_rec(recs_of(a) + j, D, v, (uint32_t)s | REC_UNRANKED | (init ? 0x80000000u : 0u));
}

// Work queued in LDS by the attempt loop and drained by the whole workgroup:
// single excitations (their matrix element is an O(N) gather loop that would
// stall a wavefront for one lane) and accepted spawns (their merge into the
// table is a chain of HBM round trips, overlapped with the other workgroups'
// spawning).
struct SingleItem {
    det_t D;             // source determinant
    uint32_t w0, w1, w2; // type/acceptance, electron and hole words
    int32_t C;           // source population (sign)
    uint32_t init;       // initiator flag of the source
    uint32_t pad;
};

constexpr int SPAWN_GRAB = 8;    // spawn tiles per dynamic grab at most (one counter serves the chip)
constexpr int SGL_QUEUE = 128 / FQ_DET_WORDS;   // (two words: the spawn kernel's LDS in 40 KB)
constexpr int SPW_QUEUE = 256;
constexpr int SGL_DRAIN = 48;     // drain the queues once they hold this many items
constexpr int SPW_DRAIN = 192;     // (a tile adds about 30 spawns; a fuller queue is merged inline)

// The acceptance uniform: the type word's uniform rescaled within the chosen
// type's interval [0, P_double) or [P_double, 1); given the type it is uniform
// on [0, 1) and independent of the orbital words.
__device__ __forceinline__ double accept_uniform(const SysDesc &d, uint32_t w0) {
    const double u = u01_32(w0);
    return u < d.p_double ? u * d.inv_p_double : (u - d.p_double) * d.inv_p_single;
}

__device__ __forceinline__ int32_t accept(const SysDesc &d, double hel, double pgen, double ua,
                                          int32_t C, uint32_t *status) {
    const double pr = (d.tau * fabs(hel)) / pgen;
    const double fl = floor(pr);
    if (fl > 1073741824.0) {
        atomicOr(status, ST_SPAWN_OVERFLOW);
        return 0;
    }
    const int32_t m = (int32_t)fl + (ua < pr - fl ? 1 : 0);
    return ((C > 0) == (hel > 0.0)) ? -m : m;
}

struct SpawnQueues {
    SingleItem sgl[SGL_QUEUE];
    det_t spd[SPW_QUEUE];
    int2 spv[SPW_QUEUE];   // (signed walkers, initiator flag)
    int nsgl, nspw, sys;
    unsigned long long base;   // first record of a drain
    uint32_t dead;             // the drained system's status, as seen by thread 0
};

// Add the wavefront's spawning events of system s to its counter and reset the
// per-thread tallies. The counter is one address for the whole chip, so it is
// touched once per wavefront per system, not per tile.
__device__ __forceinline__ void flush_spawn_count(unsigned long long *counter,
                                                  unsigned long long &spawned) {
    const unsigned long long ws = wave_sum(spawned);
    if ((threadIdx.x & 63) == 0 && ws) atomicAdd(counter, ws);
    spawned = 0;
}

// Drain both queues of system s with the whole workgroup (call uniformly).
// cm_lds: the LDS copy of the system's class masks (the descriptor's own copy is
// read instead for one-word determinants). PLAIN: as for k_spawn.
template <bool PLAIN>
__device__ void drain_queues(SpawnQueues &Q, const EngineArgs &a, const SysDesc &d, int s,
                             const uint32_t *sel8, const double *recip, const det_t *cm_lds,
                             unsigned long long &spawned) {
    const int t = threadIdx.x;
#if FQ_DET_WORDS == 1
    const det_t *const cmk = d.cmask;
#else
    const det_t *const cmk = cm_lds;
#endif
    uint32_t *status = &a.status[s];
    // a system whose record buffer overflowed re-runs the iteration: drop its queued work
    // (decided once for the workgroup: other workgroups may set the status meanwhile)
    if (t == 0) Q.dead = *(volatile uint32_t *)status;
    __syncthreads();
    const bool dead = Q.dead != 0;
    const int nsgl = dead ? 0 : (Q.nsgl < SGL_QUEUE ? Q.nsgl : SGL_QUEUE);
    for (int j = t; j < nsgl; j += blockDim.x) {
        const SingleItem it = Q.sgl[j];
        Excit ex;
        const bool ok = PLAIN || d.n_class == 2
                            ? excite_single(d, ClassView<true>{valid_of(d), nullptr}, it.D, it.w1, it.w2, sel8, ex)
                            : excite_single(d, ClassView<false>{valid_of(d), cmk}, it.D, it.w1, it.w2, sel8, ex);
        if (!ok || (!PLAIN && d.space && !in_space(d, ex.det))) continue;
        if (!PLAIN && d.hphf) {
            if (!to_function(d, cmk, recip, it.D, ex)) continue;
        } else {
            ex.hel = hel_single(d, it.D, ex.p, ex.a);
        }
        const double hel = ex.hel;
        if (hel == 0.0) continue;
        const int32_t v = accept(d, hel, ex.pgen, accept_uniform(d, it.w0), it.C, status);
        if (v == 0) continue;
        ++spawned;
        const det_t Dn = ex.det;
        const bool init = it.init != 0;
        if (Dn == ref_of(d)) {
            __hip_atomic_fetch_add(&a.d0acc[s], (long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            continue;
        }
        const int qq = atomicAdd(&Q.nspw, 1);
        if (qq < SPW_QUEUE) {
            Q.spd[qq] = Dn;
            Q.spv[qq] = make_int2(v, init ? 1 : 0);
        } else {
            put_record_wave(a, s, Dn, v, init, status);
        }
    }
    __syncthreads();
    // the queued records: one buffer reservation for the workgroup
    const int nspw = dead ? 0 : (Q.nspw < SPW_QUEUE ? Q.nspw : SPW_QUEUE);
    if (t == 0 && nspw > 0) Q.base = atomicAdd(a.rec_count, (unsigned long long)nspw);
    __syncthreads();
    for (int j = t; j < nspw; j += blockDim.x) {
        const int2 v = Q.spv[j];
        put_record(a, d, s, Q.base + (unsigned long long)j, Q.spd[j], v.x, v.y != 0, status);
    }
    __syncthreads();
    if (t == 0) {
        Q.nsgl = 0;
        Q.nspw = 0;
    }
    __syncthreads();
}

// Last index i < n with v[i] <= x, for v non-decreasing with v[0] <= x, by a
// whole wavefront: 64 samples per round, so 2^17 entries take three dependent
// loads instead of seventeen. Call with all 64 lanes active.
__device__ __forceinline__ int64_t last_le(const unsigned long long *v, int64_t n,
                                           unsigned long long x, int lane) {
    int64_t lo = 0, hi = n;
    while (hi - lo > 64) {
        const int64_t step = (hi - lo + 63) >> 6;
        const int64_t i = lo + (int64_t)lane * step;
        const bool le = i < hi && v[i] <= x;
        const int k = __popcll(__ballot(le)) - 1;   // samples <= x form a prefix of lanes
        lo = lo + (int64_t)k * step;
        hi = lo + step < hi ? lo + step : hi;
    }
    const int64_t i = lo + lane;
    const bool le = i < hi && v[i] <= x;
    return lo + __popcll(__ballot(le)) - 1;
}

// At most 80 VGPRs: six wavefronts per SIMD (the LDS use allows six workgroups per CU);
// four with two-word determinants (more registers and LDS per attempt).
// PLAIN: every system of the launch has no point group, no restricted space and plain
// determinants (EngineArgs::plain), so those branches are compiled out.
template <bool PLAIN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FQ_DET_WORDS == 1 ? 6 : 4, FQ_DET_WORDS == 1 ? 6 : 4)))
void k_spawn(EngineArgs a, const SysDesc *__restrict__ desc) {
    // inclusive sums of |C| over the staged entries, relative to the tile's first attempt
    // and clamped to 32 bits (the entries a thread can start in stay exact: a tile has at
    // most 2^20 attempts and |C| < 2^31)
    __shared__ int32_t s_rel[CHUNK];
    __shared__ det_t s_det[CHUNK];
    __shared__ int32_t s_pop[CHUNK];
    __shared__ unsigned long long s_wsum[4];   // per wavefront: walkers | entries << 48
    __shared__ long long s_c;
    __shared__ unsigned int s_tile;
    __shared__ double s_recip[65];
    __shared__ uint32_t s_sel8[256];
    __shared__ det_t s_cm[NCLASS];
    __shared__ SpawnQueues Q;
    const unsigned long long n_tiles = a.total[1];
    const int64_t nch = *a.nchunks;
    const unsigned long long tile = (unsigned long long)a.tile;
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    if (t > 0 && t <= 64) s_recip[t] = 1.0 / (double)t;
    s_sel8[t] = sel8_entry((uint32_t)t);
    if (t == 0) {
        s_recip[0] = 0.0;
        Q.nsgl = 0;
        Q.nspw = 0;
        Q.sys = -1;
    }
    __syncthreads();
    unsigned int next_tile = 0, grab_end = 0;   // wavefront 0's current grab of tiles
    // tiles per grab: SPAWN_GRAB when every workgroup gets many, fewer for small launches
    // (so that the tiles still spread over the workgroups)
    const unsigned long long per_wg = n_tiles / (4ull * gridDim.x);
    const unsigned int grab = per_wg >= (unsigned long long)SPAWN_GRAB ? (unsigned int)SPAWN_GRAB
                              : per_wg > 0ull ? (unsigned int)per_wg : 1u;
    unsigned long long spawned = 0;             // this thread's spawning events of system Q.sys
    for (;;) {
        // Tiles never cross a chunk: chunk c owns ceil(N_c / tile) consecutive tiles.
        // They are handed out dynamically, so no workgroup waits for a second round.
        if (wid == 0) {
            if (next_tile >= grab_end) {
                unsigned int g = 0;
                if (lane == 0) g = atomicAdd(&a.work[0], grab);
                next_tile = __shfl(g, 0, 64);
                grab_end = next_tile + grab;
            }
            const unsigned int tix = next_tile++;
            if (lane == 0) s_tile = tix;
            if (tix < n_tiles) {
                const int64_t cc = tix < (unsigned long long)a.tile_cap
                                       ? (int64_t)a.tile_chunk[tix]
                                       : last_le(a.chunk_toff, nch, tix, lane);
                if (lane == 0) s_c = cc;
            }
        }
        __syncthreads();
        const unsigned long long tix = s_tile;
        const int64_t c = s_c;
        __syncthreads();
        if (tix >= n_tiles) break;
        const unsigned long long off_c = a.chunk_off[c];
        const unsigned long long nw_c = sums(a, cur_half(a))[c];
        const unsigned long long j = tix - a.chunk_toff[c];
        const int s = __builtin_amdgcn_readfirstlane(a.chunk_sys[c]);
        const SysDesc &d = desc[s];
        uint32_t *status = &a.status[s];
        if (Q.sys != s) {
            // queued work and tallies belong to another system: finish them first
            if (Q.sys >= 0) {
                const int qs = __builtin_amdgcn_readfirstlane(Q.sys);
                if (Q.nsgl > 0 || Q.nspw > 0) drain_queues<PLAIN>(Q, a, desc[qs], qs, s_sel8, s_recip, s_cm, spawned);
                flush_spawn_count(&a.spawns[qs], spawned);
            }
            __syncthreads();
            if (t == 0) Q.sys = s;
            // the class masks of the new system (not read by the plain variant), ordered
            // before use by the barrier below
            if (!PLAIN && t < NCLASS) s_cm[t] = cmask_of(d, t);
        }
        // Stage the chunk's entries that hold walkers (its four buckets, one per
        // wavefront, four entries per lane), compacted, with the inclusive prefix sum
        // of |C|. Only the lanes over a bucket's entries read (the entries are packed
        // at the front of the bucket).
        const int64_t lb = (int64_t)a.chunk_local[c] * BPC + wid;
        const int64_t base = lb * BQ + 4 * lane;
        const int n_b = d.bcnt[lb] - 4 * lane;
        int4 pv = make_int4(0, 0, 0, 0);
#if FQ_DET_WORDS == 1
        ulonglong2 k01 = make_ulonglong2(0ull, 0ull), k23 = make_ulonglong2(0ull, 0ull);
        if (n_b > 0) {
            pv = gload_i4(d.pop + base);
            k01 = gload_u2(d.key + base);
            k23 = gload_u2(d.key + base + 2);
        }
#else
        det_t kk[4] = {det_t(0ull), det_t(0ull), det_t(0ull), det_t(0ull)};
        if (n_b > 0) {
            pv = gload_i4(d.pop + base);
            for (int u = 0; u < 4; ++u) kk[u] = ldk(keys_of(d) + base + u);
        }
#endif
        const int32_t pa[4] = {0 < n_b ? pv.x : 0, 1 < n_b ? pv.y : 0, 2 < n_b ? pv.z : 0,
                               3 < n_b ? pv.w : 0};
#if FQ_DET_WORDS == 1
        const uint64_t ka[4] = {k01.x, k01.y, k23.x, k23.y};
#else
        const det_t ka[4] = {kk[0], kk[1], kk[2], kk[3]};
#endif
        const int nocc = (pa[0] != 0) + (pa[1] != 0) + (pa[2] != 0) + (pa[3] != 0);
        unsigned long long run = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u)
            run += (unsigned long long)(pa[u] < 0 ? -(int64_t)pa[u] : (int64_t)pa[u]);
        // one scan of both: a lane's walkers (< 2^33) with its entry count (<= 4) above
        // bit 48; over the workgroup the sums stay below 2^41 and 2^10
        const unsigned long long mine = run | ((unsigned long long)nocc << 48);
        const unsigned long long xs = wave_incl_scan(mine);
        if (lane == 63) s_wsum[wid] = xs;
        __syncthreads();
        unsigned long long before = xs - mine;
        for (int w = 0; w < wid; ++w) before += s_wsum[w];
        unsigned long long wbefore = before & ((1ull << 48) - 1ull);
        int pos = (int)(before >> 48);
        const int n_occ = (int)((s_wsum[0] + s_wsum[1] + s_wsum[2] + s_wsum[3]) >> 48);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (pa[u] == 0) continue;
            wbefore += (unsigned long long)(pa[u] < 0 ? -(int64_t)pa[u] : (int64_t)pa[u]);
            s_pop[pos] = pa[u];
            s_det[pos] = ka[u];
            const long long rel = (long long)wbefore - (long long)(j * tile);
            s_rel[pos] = (int32_t)(rel < INT32_MIN ? INT32_MIN : rel > INT32_MAX ? INT32_MAX : rel);
            ++pos;
        }
        __syncthreads();
        // This tile's attempts, split into 256 consecutive runs whose lengths differ by
        // at most one (the longer runs first), so no wavefront idles lanes at the end.
        const unsigned long long lo_t = off_c + j * tile;
        const unsigned long long hi_t = (lo_t + tile < off_c + nw_c) ? lo_t + tile : off_c + nw_c;
        const unsigned long long n_t = hi_t - lo_t;   // <= tile <= 2^20
        const unsigned long long q_t = n_t >> 8, r_t = n_t & 255ull;
        const unsigned long long tt = (unsigned long long)t;
        unsigned long long at = lo_t + tt * q_t + (tt < r_t ? tt : r_t);
        const unsigned long long at_end = at + q_t + (tt < r_t ? 1ull : 0ull);
        // no attempts for a system that has stopped this iteration (its record buffer overflowed)
        const bool stopped = __builtin_amdgcn_readfirstlane(*(volatile uint32_t *)status) != 0;
        const bool defer = d.p_double >= 0.5;   // singles are rare: queue them
        const bool c1 = PLAIN || d.n_class == 2;           // no point group: classes are the spins
        const bool restricted = !PLAIN && d.space != 0;    // children outside the space are null
        const bool coupled = !PLAIN && d.hphf != 0;        // walkers on spin-coupled functions
        ClassView<true> cv1{valid_of(d), nullptr};
        ClassView<false> cvg{valid_of(d), s_cm};
        if (at < at_end && !stopped) {
            const int32_t xr = (int32_t)(at - lo_t);   // this thread's first attempt in the tile
            int sl = 0, hi = n_occ - 1;  // first occupied entry with inclusive sum past it
            while (sl < hi) {
                const int mid = (sl + hi) >> 1;
                if (s_rel[mid] > xr) hi = mid;
                else sl = mid + 1;
            }
            uint32_t k = sl ? (uint32_t)(xr - s_rel[sl - 1]) : (uint32_t)(at - off_c);
            for (;;) {
                const int32_t C = s_pop[sl];
                const det_t D = s_det[sl];
                const int64_t absC = C < 0 ? -(int64_t)C : (int64_t)C;
                const bool init = absC > d.n_a || D == ref_of(d);
                const uint4 w = draw_words(d.seed, D, k, d.iter, 0u);
                Excit ex;
                int r = c1 ? excite(d, cv1, D, w, s_recip, s_sel8, defer, ex)
                           : excite(d, cvg, D, w, s_recip, s_sel8, defer, ex);
                if (r == EX_SINGLE_DEFERRED) {
                    const int q = atomicAdd(&Q.nsgl, 1);
                    if (q < SGL_QUEUE) {
                        Q.sgl[q] = SingleItem{D, w.x, w.y, w.z, C, init ? 1u : 0u, 0u};
                        r = EX_NULL;
                    } else {
                        // queue full: generate it here
                        const bool ok = c1 ? excite_single(d, cv1, D, w.y, w.z, s_sel8, ex)
                                           : excite_single(d, cvg, D, w.y, w.z, s_sel8, ex);
                        r = ok ? EX_OK : EX_NULL;
                        if (ok) ex.hel = hel_single(d, D, ex.p, ex.a);
                    }
                }
                if (r == EX_OK && restricted && !in_space(d, ex.det)) r = EX_NULL;
                if (r == EX_OK && coupled && !to_function(d, s_cm, s_recip, D, ex)) r = EX_NULL;
                if (r == EX_OK) {
                    if (ex.hel != 0.0) {
                        const int32_t v = accept(d, ex.hel, ex.pgen, accept_uniform(d, w.x), C, status);
                        if (v != 0 && ex.det == ref_of(d)) {
                            ++spawned;
                            __hip_atomic_fetch_add(&a.d0acc[s], (long long)v, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                        } else if (v != 0) {
                            ++spawned;
                            const int q = atomicAdd(&Q.nspw, 1);
                            if (q < SPW_QUEUE) {
                                Q.spd[q] = ex.det;
                                Q.spv[q] = make_int2(v, init ? 1 : 0);
                            } else {
                                put_record_wave(a, s, ex.det, v, init, status);
                            }
                        }
                    }
                }
                if (++at >= at_end) break;
                if ((int64_t)(++k) >= absC) {
                    k = 0;
                    ++sl;
                }
            }
        }
        __syncthreads();
        if (Q.nsgl >= SGL_DRAIN || Q.nspw >= SPW_DRAIN) drain_queues<PLAIN>(Q, a, d, s, s_sel8, s_recip, s_cm, spawned);
    }
    __syncthreads();
    if (Q.sys >= 0) {
        const int qs = __builtin_amdgcn_readfirstlane(Q.sys);
        if (Q.nsgl > 0 || Q.nspw > 0) drain_queues<PLAIN>(Q, a, desc[qs], qs, s_sel8, s_recip, s_cm, spawned);
        flush_spawn_count(&a.spawns[qs], spawned);
    }
}

// ---------------------------------------------------------------------------
// K4a: bucket and rank of the records the spawning loop left unranked (those
// written while its queue was full; usually none).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fix(EngineArgs a, const SysDesc *__restrict__ desc) {
    const unsigned long long cnt = *a.rec_count;
    const int64_t n = cnt < (unsigned long long)a.rec_cap ? (int64_t)cnt : a.rec_cap;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t gf = recs_of(a)[i].tag;
        if (!(gf & REC_UNRANKED)) continue;
        const SysDesc &d = desc[gf & 0x3FFFFFFFu];
        const uint32_t gb = (uint32_t)(d.gchunk0 * BPC) + bucket_of(recs_of(a)[i].det, (uint64_t)d.nbuckets);
        a.rec_rank[i] = __hip_atomic_fetch_add(&a.bhist[gb], 1u, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
        recs_of(a)[i].tag = gb | (gf & 0x80000000u);
    }
}

// ---------------------------------------------------------------------------
// K4b: exclusive scan of the records per bucket (one workgroup; each thread
// takes a contiguous range of buckets).
// ---------------------------------------------------------------------------
// Bucket b's range of the record scan: SCAN_G ranges of ceil(buckets / SCAN_G).
__device__ __forceinline__ void bscan_range(int64_t nch, int g, int64_t &lo, int64_t &hi) {
    const int64_t per = (nch + SCAN_G - 1) / SCAN_G;
    lo = (int64_t)g * per;
    hi = lo + per < nch ? lo + per : nch;
    if (lo > nch) lo = nch;
}

// Records per range of buckets (coalesced: the workgroup reads its range in
// consecutive blocks of 256).
__global__ __launch_bounds__(256) void k_bscan_up(EngineArgs a) {
    __shared__ unsigned long long ws[4];
    int64_t lo, hi;
    bscan_range(*a.nchunks * BPC, blockIdx.x, lo, hi);
    unsigned long long v = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) v += a.bhist[i];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) a.boff_rg[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

// Exclusive scan of the SCAN_G range totals (one workgroup, two per thread).
__global__ __launch_bounds__(1024) void k_bscan_top(EngineArgs a) {
    __shared__ unsigned long long part[1024];
    const int t = threadIdx.x;
    const unsigned long long s0 = a.boff_rg[2 * t], s1 = a.boff_rg[2 * t + 1];
    part[t] = s0 + s1;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const unsigned long long x = t >= off ? part[t - off] : 0ull;
        __syncthreads();
        part[t] += x;
        __syncthreads();
    }
    const unsigned long long run = part[t] - (s0 + s1);
    a.boff_rg[SCAN_G + 2 * t] = run;
    a.boff_rg[SCAN_G + 2 * t + 1] = run + s0;
}

// First sorted record of each bucket: the range's offset plus a scan inside the range.
__global__ __launch_bounds__(256) void k_bscan_down(EngineArgs a) {
    __shared__ unsigned long long ws[4];
    int64_t lo, hi;
    bscan_range(*a.nchunks * BPC, blockIdx.x, lo, hi);
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    unsigned long long base = a.boff_rg[SCAN_G + blockIdx.x];
    for (int64_t c = lo; c < hi; c += 256) {
        const int64_t i = c + t;
        const unsigned long long v = i < hi ? a.bhist[i] : 0ull;
        unsigned long long x = v;
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned long long y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) ws[w] = x;
        __syncthreads();
        unsigned long long pre = 0;
        for (int k = 0; k < w; ++k) pre += ws[k];
        if (i < hi) {
            a.boff[i] = (uint32_t)(base + pre + x - v);
            a.bhist[i] = 0u;   // counted afresh next iteration
        }
        base += ws[0] + ws[1] + ws[2] + ws[3];
        __syncthreads();
    }
    // the end of the last bucket's records
    if (threadIdx.x == 0 && hi == *a.nchunks * BPC && lo < hi) a.boff[hi] = (uint32_t)base;
}

// ---------------------------------------------------------------------------
// K4c: the records grouped by bucket (order inside a bucket is immaterial:
// every merge is an integer sum).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_scatter(EngineArgs a) {
    const unsigned long long cnt = *a.rec_count;
    const int64_t n = cnt < (unsigned long long)a.rec_cap ? (int64_t)cnt : a.rec_cap;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const rec_t r = get_rec(recs_of(a) + i);
        const uint32_t gb = r.tag & 0x7FFFFFFFu;
        const uint32_t pos = a.boff[gb] + a.rec_rank[i];
        put_rec(srt_of(a) + pos, r.det, r.w, r.tag >> 31);
    }
}

// ---------------------------------------------------------------------------
// K4d: annihilation. A workgroup takes windows of consecutive chunks from a shared
// counter and, in each chunk, every wavefront one bucket, with no workgroup barrier
// inside a bucket:
//   - the bucket's records are merged per child in the wavefront's LDS hash
//     (the sort and compress of Sec. 4.1, by hashing);
//   - every entry dies first (Eq. pdeath); then the walkers that arrived for it
//     are added if it is still occupied, and otherwise survive only if an
//     initiator sent some of them (Sec. 4.2);
//   - children outside the bucket with an initiator parent become new entries
//     (emptied positions first); the other children are discarded;
//   - the bucket is re-packed; the estimator partials and the next iteration's
//     sum of |C| are written.
// A bucket with more than NREC records (rare at the planned sizes) merges them in
// rounds of at most NREC distinct children, staging its new determinants in the
// unsorted record buffer, which k_scatter has consumed by then.
// ---------------------------------------------------------------------------
constexpr int NREC = 64;                // distinct children per round in a wavefront's hash
constexpr int WHASH = 128;              // hash slots per wavefront (load <= 0.5)
constexpr int POST_QUEUE = 1024;        // new determinants whose H_DD is still to be computed
constexpr int POST_MAX_SYS = 256;       // systems whose status k_post snapshots in LDS
constexpr int POST_WIN = 32;            // chunks per window of bucket metadata in LDS
// the window's POST_WIN BPC + 1 record offsets are loaded by one thread each
static_assert(POST_WIN * BPC + 1 <= 256, "one k_post thread per record offset of a window");
constexpr uint32_t F_INIT = 1u;         // from an initiator parent (records and hash slots)
constexpr uint32_t F_MATCHED = 2u;      // hash slot: the child is an entry of the bucket
constexpr uint32_t F_MAYBE = 2u;        // record: found the hash full in this round,
constexpr uint32_t F_DEFER = 4u;        // record: left for a later round

// Orders the LDS accesses of a wavefront's lanes around it (LDS operations of one
// wavefront complete in issue order, so no wait is needed, only no code motion).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Home slot: a multiplicative hash of the folded words (the determinants of one
// bucket agree in the bits of mix64 that chose the bucket, not in these).
static_assert(WHASH == 128, "wh_home takes the top 7 bits of the product");
__device__ __forceinline__ uint32_t wh_home(det_t D) {
    const uint64_t f = lo64(D) ^ hi64(D);
    return (((uint32_t)f ^ (uint32_t)(f >> 32)) * 0x9E3779B1u) >> 25;
}

// A wavefront's working set in k_post: its merge hash (children, walkers arrived,
// flags) and the positions emptied in its bucket. One-word children mark an empty
// slot by 0 and are claimed by a 64-bit compare-and-swap; two-word children have no
// such atomic, so a 32-bit owner word (0: empty, else the claiming lane + 1) is
// claimed and the owner then writes the child.
struct WaveLds {
    det_t key[WHASH];          // child (one word: 0 when empty)
    long long acc[WHASH];      // walkers arrived for it
    uint32_t flg[WHASH];       // F_INIT | F_MATCHED
#if FQ_DET_WORDS == 2
    uint32_t own[WHASH];       // 0: empty; else the lane that entered the child, + 1
#endif
    uint16_t free_[BQ];        // positions emptied this iteration, ascending
};

#if FQ_DET_WORDS == 1
// Slot of D in a wavefront's hash (-1: absent). Call when no lane inserts.
__device__ __forceinline__ int wh_find(uint64_t D, const uint64_t *hk) {
    uint32_t h = wh_home(D);
    for (int k = 0; k < WHASH; ++k) {
        const uint64_t x = hk[h];
        if (x == D) return (int)h;
        if (x == 0ull) return -1;
        h = (h + 1u) & (uint32_t)(WHASH - 1);
    }
    return -1;
}

// Slot of D, claimed when absent. Lanes that race for an empty slot with the same D
// agree on it; with different D the losers probe on. For at most WHASH - 1
// distinct children (no limit needed). *own: this lane entered D (one lane per D).
__device__ __forceinline__ int wh_claim(uint64_t D, uint64_t *hk, bool *own) {
    uint32_t h = wh_home(D);
    *own = false;
    for (;;) {
        const uint64_t x = hk[h];
        if (x == D) return (int)h;
        if (x == 0ull) {
            const unsigned long long old =
                atomicCAS((unsigned long long *)&hk[h], 0ull, (unsigned long long)D);
            *own = old == 0ull;
            if (old == 0ull || old == D) return (int)h;
        }
        h = (h + 1u) & (uint32_t)(WHASH - 1);
    }
}

// As wh_claim, with at most NREC claims per round: *ncl counts claims made and
// claims in flight. -1 when D is absent and no claim is left (D may have been
// entered meanwhile by another lane, which a lookup afterwards settles).
__device__ __forceinline__ int wh_claim_limited(uint64_t D, uint64_t *hk, int *ncl) {
    uint32_t h = wh_home(D);
    for (int k = 0; k < WHASH; ++k) {
        const uint64_t x = hk[h];
        if (x == D) return (int)h;
        if (x == 0ull) {
            if (atomicAdd(ncl, 1) >= NREC) {
                atomicSub(ncl, 1);
                return -1;
            }
            const unsigned long long old =
                atomicCAS((unsigned long long *)&hk[h], 0ull, (unsigned long long)D);
            if (old == 0ull) return (int)h;
            atomicSub(ncl, 1);   // the slot went to another lane's claim
            if (old == D) return (int)h;
        }
        h = (h + 1u) & (uint32_t)(WHASH - 1);
    }
    return -1;
}

__device__ __forceinline__ int wl_find(det_t D, const WaveLds &W) { return wh_find(D, W.key); }
__device__ __forceinline__ int wl_claim(det_t D, WaveLds &W, bool *own, int) {
    return wh_claim(D, W.key, own);
}
__device__ __forceinline__ int wl_claim_limited(det_t D, WaveLds &W, int *ncl, int) {
    return wh_claim_limited(D, W.key, ncl);
}
__device__ __forceinline__ bool wl_used(const WaveLds &W, int h) { return W.key[h] != 0ull; }
__device__ __forceinline__ void wl_clear(WaveLds &W, int h) { W.key[h] = 0ull; }
#else
__device__ __forceinline__ bool wl_used(const WaveLds &W, int h) { return W.own[h] != 0u; }
__device__ __forceinline__ void wl_clear(WaveLds &W, int h) { W.own[h] = 0u; }
__device__ __forceinline__ int wl_find(det_t D, const WaveLds &W) {
    uint32_t h = wh_home(D);
    for (int k = 0; k < WHASH; ++k) {
        if (W.own[h] == 0u) return -1;
        if (W.key[h] == D) return (int)h;
        h = (h + 1u) & (uint32_t)(WHASH - 1);
    }
    return -1;
}
// Claim of a slot: lanes that find it empty race for its owner word; the winner
// writes the child, and after the wave-level ordering point every lane still
// probing compares the (now written) child with its own. A lane whose probe ends
// early leaves the loop masked off; the others stay in step.
__device__ __forceinline__ int wl_claim(det_t D, WaveLds &W, bool *own, int lane) {
    uint32_t h = wh_home(D);
    *own = false;
    for (;;) {
        bool won = false;
        if (W.own[h] == 0u) won = atomicCAS(&W.own[h], 0u, (uint32_t)lane + 1u) == 0u;
        if (won) W.key[h] = D;
        wave_sync();
        if (won) {
            *own = true;
            return (int)h;
        }
        if (W.key[h] == D) return (int)h;
        h = (h + 1u) & (uint32_t)(WHASH - 1);
    }
}
__device__ __forceinline__ int wl_claim_limited(det_t D, WaveLds &W, int *ncl, int lane) {
    uint32_t h = wh_home(D);
    for (int k = 0; k < WHASH; ++k) {
        bool won = false, full = false;
        if (W.own[h] == 0u) {
            if (atomicAdd(ncl, 1) >= NREC) {
                atomicSub(ncl, 1);
                full = true;
            } else {
                won = atomicCAS(&W.own[h], 0u, (uint32_t)lane + 1u) == 0u;
                if (!won) atomicSub(ncl, 1);   // the slot went to another lane's claim
            }
        }
        if (won) W.key[h] = D;
        wave_sync();
        if (won) return (int)h;
        if (full) return -1;
        if (W.key[h] == D) return (int)h;
        h = (h + 1u) & (uint32_t)(WHASH - 1);
    }
    return -1;
}
#endif

// H_DD = E_core + sum_p h_pp + sum_{p<q} [(pp|qq) - (pq|qp)], accumulated in
// ascending (p, q) order from the LDS copies of h_pp and of the pair table (its
// upper triangle, row after row: entry (p, q) at pair_row(p, n) + q), for two
// determinants with the same number of electrons at once: the two sums are
// independent chains that hide each other's add latency, and each keeps the
// order of a single sum.
__device__ __forceinline__ int pair_row(int p, int n) { return p * (2 * n - p - 3) / 2 - 1; }

__device__ __forceinline__ void hdiag_lds2(double e_core, det_t da, det_t db,
                                           const double *hpp, const double *jk, int n,
                                           double &ra, double &rb) {
    double xa = e_core, xb = e_core;
    for (det_t ma = da, mb = db; ma; ma &= ma - 1ull, mb &= mb - 1ull) {
        xa = xa + hpp[dctz(ma)];
        xb = xb + hpp[dctz(mb)];
    }
    for (det_t m1a = da, m1b = db; m1a; m1a &= m1a - 1ull, m1b &= m1b - 1ull) {
        const int ba = pair_row(dctz(m1a), n);
        const int bb = pair_row(dctz(m1b), n);
        for (det_t m2a = m1a & (m1a - 1ull), m2b = m1b & (m1b - 1ull); m2a;
             m2a &= m2a - 1ull, m2b &= m2b - 1ull) {
            xa = xa + jk[ba + dctz(m2a)];
            xb = xb + jk[bb + dctz(m2b)];
        }
    }
    ra = xa;
    rb = xb;
}

#if FQ_DET_WORDS == 2
// As hdiag_lds2, with the pair table read from global memory ([n_so][NSO_MAX],
// entry (p, q) at p NSO_MAX + q): for more than 64 spin orbitals, whose upper
// triangle would take 65 KB of LDS.
__device__ __forceinline__ void hdiag_glb2(double e_core, det_t da, det_t db, const double *hpp,
                                           const double *jk, double &ra, double &rb) {
    double xa = e_core, xb = e_core;
    for (det_t ma = da, mb = db; ma; ma &= ma - 1ull, mb &= mb - 1ull) {
        xa = xa + hpp[dctz(ma)];
        xb = xb + hpp[dctz(mb)];
    }
    const gdouble *t = gptr(jk);
    for (det_t m1a = da, m1b = db; m1a; m1a &= m1a - 1ull, m1b &= m1b - 1ull) {
        const gdouble *ra_ = t + dctz(m1a) * NSO_MAX, *rb_ = t + dctz(m1b) * NSO_MAX;
        for (det_t m2a = m1a & (m1a - 1ull), m2b = m1b & (m1b - 1ull); m2a;
             m2a &= m2a - 1ull, m2b &= m2b - 1ull) {
            xa = xa + ra_[dctz(m2a)];
            xb = xb + rb_[dctz(m2b)];
        }
    }
    ra = xa;
    rb = xb;
}
#endif

// Diagonal elements of the queued new determinants (positions in the system's
// arrays, all of one system, so all with the same electron count), two per
// thread at a time; the pair table from LDS (jk), or from global memory when jk is
// null (two-word determinants of more than 64 spin orbitals).
__device__ __forceinline__ void flush_new_dets(const SysDesc &d, const uint32_t *queue, int n,
                                               const double *hpp, const double *jk) {
    const int step = 2 * (int)blockDim.x;
    for (int j = threadIdx.x; j < n; j += step) {
        const uint32_t i0 = queue[j];
        const bool two = j + (int)blockDim.x < n;
        const uint32_t i1 = two ? queue[j + blockDim.x] : i0;
        double h0, h1;
        const det_t k0 = ldk(keys_of(d) + i0), k1 = ldk(keys_of(d) + i1);
#if FQ_DET_WORDS == 1
        hdiag_lds2(d.e_core, k0, k1, hpp, jk, d.n_so, h0, h1);
#else
        if (jk)
            hdiag_lds2(d.e_core, k0, k1, hpp, jk, d.n_so, h0, h1);
        else
            hdiag_glb2(d.e_core, k0, k1, hpp, d.jk, h0, h1);
#endif
        *gp(d.hdiag + i0) = fn_diag_from(d, k0, h0);
        if (two) *gp(d.hdiag + i1) = fn_diag_from(d, k1, h1);
    }
}

__device__ __forceinline__ uint64_t lanes_below(int lane) { return (1ull << lane) - 1ull; }

// Sum over the wavefront's lanes of a per-lane count v < 8, from ballots of its bits.
__device__ __forceinline__ int wave_total8(int v) {
    return __popcll(__ballot(v & 1)) + 2 * __popcll(__ballot(v & 2)) + 4 * __popcll(__ballot(v & 4));
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4)))
void k_post(EngineArgs a, const SysDesc *__restrict__ desc) {
    // Each wavefront's working set, and (between chunks only) the pair table from
    // which the diagonal elements of new determinants are computed.
    struct PairTable {
        double jk[64 * 63 / 2];   // (up to 64 spin orbitals)
        double hpp[NSO_MAX];
    };
#if FQ_DET_WORDS == 1
    // side by side: the staged pair table stays valid while the wavefronts use theirs
    struct PostLds {
        WaveLds w[POST_WAVES];
        PairTable tab;
    };
#else
    union PostLds {   // (two words: no room for both at four workgroups per CU)
        WaveLds w[POST_WAVES];
        PairTable tab;
    };
#endif
    __shared__ PostLds L;
    __shared__ uint32_t s_queue[POST_QUEUE];
    __shared__ uint32_t s_stat[POST_MAX_SYS];   // the systems' status at the kernel's start
    // Metadata of a window of POST_WIN chunks, read once for all its buckets.
    __shared__ int s_csys[POST_WIN];                 // system of the chunk (-1: not taking part)
    __shared__ int s_cloc[POST_WIN];                 // chunk index inside its system's table
    __shared__ uint8_t s_cnext[POST_WIN];            // its walkers spawn next iteration
    __shared__ int16_t s_bn[POST_WIN * BPC];         // entries per bucket
    __shared__ uint32_t s_boff[POST_WIN * BPC + 1];  // first sorted record per bucket, and the end
    __shared__ unsigned long long s_cnws[POST_WIN];  // the chunk's sum of |C| after the iteration
    __shared__ int s_cdone[POST_WIN];                // wavefronts done with the chunk
    __shared__ int s_qn, s_qsys;
    __shared__ int s_tabsys;                         // system whose pair table is staged (-1: none)
    __shared__ int s_ncl[POST_WAVES];
    __shared__ int64_t s_win;                        // first chunk of the window taken
    const int64_t nch = *a.nchunks;
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    WaveLds &W = L.w[wid];
    if (blockIdx.x == 0 && t == 0) *a.rec_count = 0ull;   // k_scatter has consumed the records
    unsigned long long *const nws_next = sums(a, cur_half(a) ^ 1u);
    unsigned long long *const rg_next = ranges(a, cur_half(a) ^ 1u);
    const int64_t per_range = (nch + SCAN_G - 1) / SCAN_G;
    const int tsh = __builtin_ctzll((unsigned long long)a.tile);
    const unsigned long long tm = (unsigned long long)a.tile - 1ull;
    // Which systems take part is decided from the status at the start: bits set while
    // this kernel runs (population overflow) are fatal to their system anyway.
    for (int i = t; i < a.max_sys && i < POST_MAX_SYS; i += 256) s_stat[i] = a.status[i];
    if (t == 0) {
        s_qn = 0;
        s_qsys = -1;
        s_tabsys = -1;
    }
    auto flush = [&]() {   // (uniform) H_DD of the queued new determinants
        const SysDesc &dq = desc[s_qsys];
        const bool in_lds = dq.n_so <= 64;   // the pair table's upper triangle fits in LDS
        if (FQ_DET_WORDS == 2 || s_tabsys != s_qsys) {   // (uniform) stage the system's tables
            if (in_lds)
                for (int i = t; i < dq.n_so * 64; i += 256) {
                    const int p = i >> 6, q = i & 63;
                    if (q > p && q < dq.n_so)
                        L.tab.jk[pair_row(p, dq.n_so) + q] = gptr(dq.jk)[p * NSO_MAX + q];
                }
            for (int i = t; i < dq.n_so; i += 256) L.tab.hpp[i] = h_so(dq, i, i);
            __syncthreads();
            if (t == 0) s_tabsys = s_qsys;   // (read again only after the barrier below)
        }
        flush_new_dets(dq, s_queue, s_qn < POST_QUEUE ? s_qn : POST_QUEUE, L.tab.hpp,
                       in_lds ? L.tab.jk : nullptr);
        __syncthreads();
    };
    // The workgroups take windows of consecutive chunks from a shared counter (so the
    // faster ones take more): POST_WIN chunks when every workgroup gets many, fewer for
    // small launches; inside a window the wavefronts run through the chunks
    // independently, and the last one done with a chunk writes the chunk's sum for the
    // next iteration.
    const int64_t per_wg = nch / (4 * (int64_t)gridDim.x);
    const int gwin = per_wg >= POST_WIN ? POST_WIN : per_wg > 0 ? (int)per_wg : 1;
    for (;;) {
        __syncthreads();   // the previous window is done
        if (s_qn > 0) {    // (uniform)
            flush();
            if (t == 0) {
                s_qn = 0;
                s_qsys = -1;
            }
        }
        if (t == 0) s_win = (int64_t)atomicAdd(&a.work[1], 1u) * gwin;
        __syncthreads();
        const int64_t c0 = s_win;
        if (c0 >= nch) break;
        const int nwin = (int)(nch - c0 < gwin ? nch - c0 : gwin);
        if (t < nwin) {
            const int sc = a.chunk_sys[c0 + t];
            bool live = false, next = false;
            if (sc >= 0) {
                const SysDesc &dc = desc[sc];
                live = participating(dc, sc < POST_MAX_SYS ? s_stat[sc] : a.status[sc]);
                next = live && dc.iter + 1 < dc.stop_at;
            }
            s_csys[t] = live ? sc : -1;
            s_cloc[t] = a.chunk_local[c0 + t];
            s_cnext[t] = next ? 1 : 0;
            s_cnws[t] = 0ull;
            s_cdone[t] = 0;
        }
        if (t <= nwin * BPC) s_boff[t] = a.boff[c0 * BPC + t];
        __syncthreads();
        if (t < nwin * BPC) {
            const int sc = s_csys[t / BPC];
            s_bn[t] = sc >= 0 ? (int16_t)desc[sc].bcnt[(int64_t)s_cloc[t / BPC] * BPC + t % BPC] : 0;
        }
        __syncthreads();
        // this wavefront's statistics over consecutive buckets of one system (per lane;
        // reduced when the system changes and at the end of the window)
        int64_t a_nw = 0, a_ab = 0, a_born = 0;
        uint64_t a_cnt = 0;
        double a_num = 0.0;
        for (int ci = 0; ci < nwin; ++ci) {
            const int64_t c = c0 + ci;
            const int s = s_csys[ci];
            const bool live = s >= 0;
            int64_t nw = 0, aborted = 0;
            uint64_t cnt = 0;                 // entries | merged targets << 21 | occupied << 42
            double num = 0.0;
            unsigned long long nwb = 0;       // sum |C| over the bucket's entries after the iteration
            int64_t born = 0;                 // new determinants (uniform)
            if (live) {
                const SysDesc &d = desc[s];
                uint32_t *status = &a.status[s];
                const int64_t lb = (int64_t)s_cloc[ci] * BPC + wid;
                const int64_t base = lb * BQ;
                const int n = s_bn[ci * BPC + wid];
                const uint32_t r0 = s_boff[ci * BPC + wid];
                const uint32_t nr = s_boff[ci * BPC + wid + 1] - r0;
                // the H_DD queue serves one system at a time: the first to use it in a window
                if (lane == 0 && s_qsys < 0) atomicCAS(&s_qsys, -1, s);
                // entry u * 64 + lane is this lane's u-th; R rounds cover the n entries
                const int R = (n + 63) >> 6;
                det_t kin[4] = {det_t(0ull), det_t(0ull), det_t(0ull), det_t(0ull)};
                int32_t pin[4] = {0, 0, 0, 0};
                double hin[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (u >= R) break;
                    if ((u << 6) + lane < n) {
                        kin[u] = ldk(keys_of(d) + base + (u << 6) + lane);
                        pin[u] = *gp(d.pop + base + (u << 6) + lane);
                        hin[u] = *gp(d.hdiag + base + (u << 6) + lane);
                    }
                }
                det_t rd = det_t(0ull);   // this lane's record (fast path), its hash slot, and
                int32_t rw = 0;       // whether this lane entered the child there
                uint32_t rf = 0u;
                int rh = 0;
                bool rown = false;
                if ((uint32_t)lane < nr && nr <= (uint32_t)NREC) {
                    const rec_t r = get_rec(srt_of(a) + r0 + lane);
                    rd = r.det;
                    rw = r.w;
                    rf = r.tag;
                }
                wl_clear(W, lane);
                wl_clear(W, lane + 64);
                W.acc[lane] = 0ll;
                W.acc[lane + 64] = 0ll;
                W.flg[lane] = 0u;
                W.flg[lane + 64] = 0u;
                // death of every entry (Eq. pdeath, one stochastic rounding for the whole
                // determinant); it depends on nothing that arrives
                // (branch-free over the lanes: p = 0 past the bucket's entries gives pd = 0)
                int32_t pdv[4] = {0, 0, 0, 0};
                bool ovf = false;   // a population left int32 (reported once for the bucket)
    #pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (u >= R) break;
                    const int32_t p = pin[u];
                    uint64_t xd, xu;
                    draw2(d.seed, kin[u], 0xFFFFFFFFu, d.iter, 0x80u, xd, xu);
                    const uint32_t absC = (uint32_t)(p < 0 ? -p : p);   // |p| <= 2^31 - 1
                    const double dv = ((hin[u] - d.e0) - d.shift) * d.tau * (double)absC;
                    const double ad = fabs(dv);
                    const double fl = floor(ad);
                    const bool big = fl > 1073741824.0;   // the entry is left as it is
                    // m <= 2^30 + 1; C - sign(C) sign(d) m
                    const int32_t m = (int32_t)(big ? 0.0 : fl) + (u01(xd) < ad - fl ? 1 : 0);
                    const int64_t pm = (int64_t)p + (((p > 0) == (dv > 0.0)) ? -(int64_t)m : (int64_t)m);
                    const bool range = pm > 2147483647ll || pm < -2147483647ll;
                    ovf |= p != 0 && (big || range);
                    pdv[u] = p == 0 ? 0 : big ? p : range ? 0 : (int32_t)pm;
                }
                wave_sync();
                long long spv[4] = {0ll, 0ll, 0ll, 0ll};   // walkers arrived per entry
                uint32_t flv = 0u;                         // bit u: an initiator sent some
                int kc = 0;                                // slow path: staged children (uniform)
                if (nr <= (uint32_t)NREC) {
                    // Fast path: at most NREC records, so at most NREC distinct children.
                    if ((uint32_t)lane < nr) {
                        rh = wl_claim(rd, W, &rown, lane);
                        atomicAdd((unsigned long long *)&W.acc[rh], (unsigned long long)(long long)rw);
                        if (rf & F_INIT) atomicOr(&W.flg[rh], F_INIT);
                    }
                    wave_sync();
                    if (nr > 0) {
    #pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            if (u >= R) break;
                            if ((u << 6) + lane >= n) continue;
                            const int h = wl_find(kin[u], W);
                            if (h < 0) continue;
                            spv[u] = W.acc[h];
                            flv |= (W.flg[h] & F_INIT) << u;
                            W.flg[h] |= F_MATCHED;   // a child matches at most one entry
                        }
                    }
                    wave_sync();
                } else {
                    // Slow path: rounds of at most NREC distinct children. A child whose
                    // records found the hash full is left whole for a later round; the
                    // children outside the bucket are staged, merged, in the bucket's range
                    // of the unsorted record buffer.
                    for (int round = 0;; ++round) {
                        if (round > 0) {
                            wl_clear(W, lane);
                            wl_clear(W, lane + 64);
                            W.acc[lane] = 0ll;
                            W.acc[lane + 64] = 0ll;
                            W.flg[lane] = 0u;
                            W.flg[lane + 64] = 0u;
                        }
                        if (lane == 0) s_ncl[wid] = 0;
                        wave_sync();
                        bool maybe = false;
                        for (uint32_t j = lane; j < nr; j += 64) {   // (a record stays with its lane)
                            rec_t *const srt = srt_of(a);
                            const uint32_t f = srt[r0 + j].tag;
                            if (round > 0 && !(f & F_DEFER)) continue;
                            const det_t D = srt[r0 + j].det;
                            const int h = wl_claim_limited(D, W, &s_ncl[wid], lane);
                            if (h < 0) {
                                srt[r0 + j].tag = (f & F_INIT) | F_MAYBE;
                                maybe = true;
                                continue;
                            }
                            if (f & F_DEFER) srt[r0 + j].tag = f & F_INIT;
                            atomicAdd((unsigned long long *)&W.acc[h],
                                      (unsigned long long)(long long)srt[r0 + j].w);
                            if (f & F_INIT) atomicOr(&W.flg[h], F_INIT);
                        }
                        wave_sync();
                        bool defer = false;
                        if (__ballot(maybe)) {
                            for (uint32_t j = lane; j < nr; j += 64) {
                                rec_t *const srt = srt_of(a);
                                const uint32_t f = srt[r0 + j].tag;
                                if (!(f & F_MAYBE)) continue;
                                const int h = wl_find(srt[r0 + j].det, W);
                                if (h < 0) {
                                    srt[r0 + j].tag = (f & F_INIT) | F_DEFER;
                                    defer = true;
                                    continue;
                                }
                                srt[r0 + j].tag = f & F_INIT;
                                atomicAdd((unsigned long long *)&W.acc[h],
                                          (unsigned long long)(long long)srt[r0 + j].w);
                                if (f & F_INIT) atomicOr(&W.flg[h], F_INIT);
                            }
                            wave_sync();
                        }
    #pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            if (u >= R) break;
                            if ((u << 6) + lane >= n) continue;
                            const int h = wl_find(kin[u], W);
                            if (h < 0) continue;
                            spv[u] += W.acc[h];
                            flv |= (W.flg[h] & F_INIT) << u;
                            W.flg[h] |= F_MATCHED;
                        }
                        wave_sync();
                        // stage this round's children outside the bucket (one per slot)
                        for (int h = lane; h < WHASH; h += 64) {
                            const det_t D = W.key[h];
                            const bool cand = wl_used(W, h) && !(W.flg[h] & F_MATCHED);
                            const uint64_t m = __ballot(cand);
                            if (cand) {
                                const uint32_t j = r0 + (uint32_t)kc + (uint32_t)__popcll(m & lanes_below(lane));
                                long long sp = W.acc[h];
                                if (sp > 2147483647ll || sp < -2147483647ll) {
                                    atomicOr(status, ST_POP_OVERFLOW);
                                    sp = 0;
                                }
                                put_rec(recs_of(a) + j, D, (int32_t)sp, W.flg[h] & F_INIT);
                            }
                            kc += __popcll(m);
                        }
                        wave_sync();
                        if (!__ballot(defer)) break;
                    }
                    __threadfence();   // the staged children, read back below by other lanes
                }
                // Annihilation (Sec. 4.2) of the bucket's own entries.
                int32_t npv[4] = {0, 0, 0, 0};
                uint32_t keepm = 0u;
                uint32_t nearm = 0u;   // bit u: entry u contributes to the projected energy
                int reborn = 0;        // entries emptied by death and re-entered by initiator
                                       // spawns (new determinants kept in place)
                // (branch-free over the lanes: past the bucket's entries D = 0, and nothing
                // arrives, so np = 0 and nothing is counted)
    #pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (u >= R) break;
                    const det_t D = kin[u];
                    const bool is_ref = D == ref_of(d);
                    const int64_t pd = pdv[u];
                    // (walkers spawned onto the reference arrive in their own sum)
                    long long sp = spv[u];
                    if (is_ref) sp += a.d0acc[s];
                    const bool alive = pd != 0 || is_ref;
                    const bool reb = !alive && sp != 0 && ((flv >> u) & 1u);
                    const long long asp = sp < 0 ? -sp : sp;
                    int64_t np = alive ? pd + sp : (reb ? sp : 0ll);
                    reborn += reb ? 1 : 0;
                    aborted += (!alive && !reb) ? asp : 0ll;
                    cnt += sp != 0 ? 1ull << CNT_SHIFT_MERGED : 0ull;
                    const bool range = np > 2147483647ll || np < -2147483647ll;
                    ovf |= range;
                    np = range ? 0ll : np;
                    npv[u] = (int32_t)np;
                    if (is_ref) {
                        a.c0[s] = np;
                        a.d0acc[s] = 0ll;   // consumed
                    }
                    const int64_t an = np < 0 ? -np : np;
                    nw += an;
                    nwb += (unsigned long long)an;
                    cnt += np != 0 ? 1ull << CNT_SHIFT_ND : 0ull;
                    nearm |= (np != 0 && !is_ref && near_ref(d, D)) ? 1u << u : 0u;
                    keepm |= (np != 0 || is_ref) ? 1u << u : 0u;   // the reference keeps its entry at 0
                }
                if (ovf) atomicOr(status, ST_POP_OVERFLOW);
                // positions emptied this iteration, ascending (round by round, lanes in order)
                int H = 0;
    #pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (u >= R) break;
                    const bool hole = (u << 6) + lane < n && !((keepm >> u) & 1u);
                    const uint64_t m = __ballot(hole);
                    if (hole) W.free_[H + __popcll(m & lanes_below(lane))] = (uint16_t)((u << 6) + lane);
                    H += __popcll(m);
                }
                const int Lk = n - H;
                wave_sync();
                // New determinants: children outside the bucket with an initiator parent go
                // to the emptied positions first, then past the end; the others are discarded.
                int K = 0;
                int calls = 0;
                uint32_t nearn = 0u;   // fast path: bit 0, this lane's new determinant
                                       // contributes to the projected energy
                auto place = [&](det_t D, long long sp, bool init) {   // (all lanes; D = 0: none)
                    const bool real = D != det_t(0ull) && sp != 0;
                    if (real) cnt += 1ull << CNT_SHIFT_MERGED;
                    if (real && !init) aborted += sp < 0 ? -sp : sp;
                    const bool nd = real && init;
                    const uint64_t m = __ballot(nd);
                    const int k = K + __popcll(m & lanes_below(lane));
                    K += __popcll(m);
                    const int call = calls++;
                    if (!nd) return;
                    const int64_t an = sp < 0 ? -sp : sp;
                    nw += an;
                    cnt += 1ull << CNT_SHIFT_ND;
                    if (call < 32 && near_ref(d, D)) nearn |= 1u << call;
                    const int pos = k < H ? (int)W.free_[k] : n + (k - H);
                    if (pos < BQ) {
                        nwb += (unsigned long long)an;
                        stk(keys_of(d) + base + pos, D);
                        *gp(d.pop + base + pos) = (int32_t)sp;
                        const int q = s_qsys == s ? atomicAdd(&s_qn, 1) : POST_QUEUE;
                        if (q < POST_QUEUE) {
                            s_queue[q] = (uint32_t)(base + pos);
                        } else {   // (another system's window, or many new determinants)
                            *gp(d.hdiag + base + pos) = fn_diag(d, D);
                        }
                    } else {
                        // the bucket is full: completed in the spill list, re-bucketed by the host
                        const unsigned long long j = atomicAdd(a.sp_count, 1ull);
                        if (j < (unsigned long long)a.sp_cap) {
                            spill_dets(a)[j] = D;
                            a.sp_pop[j] = (int32_t)sp;
                            a.sp_hd[j] = fn_diag(d, D);
                            a.sp_sys[j] = s;
                            a.spilled[s] = 1u;
                        } else {
                            atomicOr(status, ST_SPILL_FULL);
                        }
                    }
                };
                long long rsp = 0ll;   // fast path: walkers that arrived for this lane's child
                if (nr <= (uint32_t)NREC) {
                    // one lane per distinct child: the lane that entered it into the hash
                    const uint32_t f = rown ? W.flg[rh] : F_MATCHED;
                    const bool cand = !(f & F_MATCHED);
                    rsp = cand ? W.acc[rh] : 0ll;
                    if (rsp > 2147483647ll || rsp < -2147483647ll) {
                        atomicOr(status, ST_POP_OVERFLOW);
                        rsp = 0ll;
                        place(det_t(0ull), 0ll, false);
                    } else {
                        place(cand ? rd : det_t(0ull), rsp, (f & F_INIT) != 0u);
                    }
                } else {
                    for (int i0 = 0; i0 < kc; i0 += 64) {
                        const int i = i0 + lane;
                        const bool in = i < kc;
                        const rec_t *const st = recs_of(a);
                        place(in ? st[r0 + i].det : det_t(0ull), in ? (long long)st[r0 + i].w : 0ll,
                              in && (st[r0 + i].tag & F_INIT));
                    }
                }
                // Re-pack: n' = (kept entries) + (new determinants); when fewer new
                // determinants than emptied positions arrived, the kept entries past n' move
                // into the emptied positions that remain below n'.
                const int np_ = Lk + K < BQ ? Lk + K : BQ;
                uint32_t movedm = 0u;
                if (K < H) {   // uniform
                    int r = K;
    #pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        if (u >= R) break;
                        const bool mv = ((keepm >> u) & 1u) && (u << 6) + lane >= np_;
                        const uint64_t m = __ballot(mv);
                        if (mv) {
                            const int64_t dst = base + W.free_[r + __popcll(m & lanes_below(lane))];
                            stk(keys_of(d) + dst, kin[u]);
                            *gp(d.pop + dst) = npv[u];
                            *gp(d.hdiag + dst) = hin[u];
                            movedm |= 1u << u;
                        }
                        r += __popcll(m);
                    }
                }
    #pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (((keepm & ~movedm) >> u) & 1u && npv[u] != pin[u])
                        *gp(d.pop + base + (u << 6) + lane) = npv[u];
                if (lane == 0) {
                    d.bcnt[lb] = np_;
                    cnt += (uint64_t)np_;
                }
                born = K + wave_total8(reborn);
                // Projected-energy numerator (Eq. ProjE): the occupied determinants within a
                // double excitation of the reference, taken last, when few values are live.
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if ((nearm >> u) & 1u) num = num + ref_hel(d, kin[u]) * (double)npv[u];
                if (nr <= (uint32_t)NREC) {
                    if (nearn & 1u) num = num + ref_hel(d, rd) * (double)rsp;
                } else {
                    for (int i = lane; i < kc; i += 64) {
                        const rec_t *const st = recs_of(a);
                        const det_t D = st[r0 + i].det;
                        const int32_t sp = st[r0 + i].w;
                        if (sp != 0 && (st[r0 + i].tag & F_INIT) && near_ref(d, D))
                            num = num + ref_hel(d, D) * (double)sp;
                    }
                }
            }
            a_nw += nw;
            a_ab += aborted;
            a_cnt += cnt;
            a_num = a_num + num;
            a_born += born;
            // the statistics share of this wavefront: its accumulated buckets when the
            // system changes after this chunk or the window ends (fixed-order reduction),
            // nothing otherwise
            const bool last = ci + 1 == nwin || s_csys[ci + 1] != s;
            ChunkStat cs{0, 0, 0ull, 0.0, 0};
            if (last) {
                cs = ChunkStat{(int64_t)wave_sum((long long)a_nw), (int64_t)wave_sum((long long)a_ab),
                               (uint64_t)wave_sum((unsigned long long)a_cnt), wave_sum(a_num), a_born};
                a_nw = a_ab = a_born = 0;
                a_cnt = 0ull;
                a_num = 0.0;
            }
            {   // the wavefront's total, by DPP (all lanes active here)
                const unsigned long long x = wave_incl_scan(nwb);
                nwb = (unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, 63) |
                      ((unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), 63) << 32);
            }
            if (lane == 0) {
                a.chunk_stat[c * POST_WAVES + wid] = cs;
                // walkers that spawn next iteration: none if the system stops after this one
                if (s_cnext[ci] && nwb) atomicAdd(&s_cnws[ci], nwb);
                if (atomicAdd(&s_cdone[ci], 1) == POST_WAVES - 1) {
                    const unsigned long long x = atomicAdd(&s_cnws[ci], 0ull);
                    nws_next[c] = x;
                    if (x) {
                        atomicAdd(&rg_next[c / per_range], x);
                        atomicAdd(&rg_next[SCAN_G + c / per_range], (x + tm) >> tsh);
                    }
                }
            }
        }
    }
    __syncthreads();
    if (s_qn > 0) flush();   // uniform
}

// ---------------------------------------------------------------------------
// K5a: per system, FIN_BLOCKS workgroups each reduce one contiguous range of
// the system's chunk statistics (fixed ranges and trees: deterministic).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_reduce(EngineArgs a) {
    __shared__ long long shi[256];
    __shared__ double shd[256];
    const int s = blockIdx.y;
    const SysDesc &d = a.desc[s];
    if (!participating(d, a.status[s])) return;   // uniform across the workgroup
    const int t = threadIdx.x;
    const int64_t per = (d.nchunks + FIN_BLOCKS - 1) / FIN_BLOCKS;
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = lo + per < d.nchunks ? lo + per : d.nchunks;
    int64_t nw = 0, nd = 0, merged = 0, aborted = 0, att = 0, used = 0, born = 0;
    double num = 0.0;
    for (int64_t i = lo + t; i < hi; i += 256) {
        for (int w = 0; w < POST_WAVES; ++w) {
            const ChunkStat cs = a.chunk_stat[(d.gchunk0 + i) * POST_WAVES + w];
            used += (int64_t)(cs.counts & CNT_FIELD);
            merged += (int64_t)((cs.counts >> CNT_SHIFT_MERGED) & CNT_FIELD);
            nd += (int64_t)(cs.counts >> CNT_SHIFT_ND);
            nw += cs.nw;
            aborted += cs.aborted;
            born += cs.born;
            num = num + cs.num;
        }
        att += (int64_t)sums(a, cur_half(a))[d.gchunk0 + i];
    }
    FinPart p;
    p.nw = block_sum((long long)nw, shi);
    p.nd = block_sum((long long)nd, shi);
    p.merged = block_sum((long long)merged, shi);
    p.aborted = block_sum((long long)aborted, shi);
    p.attempts = block_sum((long long)att, shi);
    p.used = block_sum((long long)used, shi);
    p.born = block_sum((long long)born, shi);
    p.num = block_sum(num, shd);
    if (t == 0) a.fin_part[(int64_t)s * FIN_BLOCKS + blockIdx.x] = p;
}

// ---------------------------------------------------------------------------
// K5b: per system (one wavefront): sum of the FIN_BLOCKS shares by a fixed
// butterfly, the shift update, the per-iteration record.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_finalize(EngineArgs a) {
    const int s = blockIdx.x;
    if (s == 0 && threadIdx.x == 0) *a.step += 1ull;   // every kernel of this iteration has read it
    SysDesc &d = a.desc[s];
    if (!participating(d, a.status[s])) return;   // uniform across the wavefront
    const int t = threadIdx.x;
    const FinPart p = a.fin_part[(int64_t)s * FIN_BLOCKS + t];
    const int64_t nw = wave_sum((long long)p.nw);
    const int64_t nd = wave_sum((long long)p.nd);
    const int64_t c0 = a.c0[s];
    const int64_t merged = wave_sum((long long)p.merged);
    const int64_t aborted = wave_sum((long long)p.aborted);
    const int64_t att = wave_sum((long long)p.attempts);
    const int64_t used = wave_sum((long long)p.used);
    const int64_t born = wave_sum((long long)p.born);
    const double num = wave_sum(p.num);
    if (t == 0) {
        const int64_t done = d.iter + 1;
        {
            if (done % d.A == 0) {
                if (!d.varying) {
                    if (nw >= d.target) {
                        d.varying = 1;
                        d.n_prev = nw;
                        d.n_var = done;
                    }
                } else {
                    d.shift = d.shift - (d.zeta / ((double)d.A * d.tau)) *
                                            shift_log((double)nw / (double)d.n_prev);
                    d.n_prev = nw;
                }
            }
            if (nw == 0) a.status[s] |= ST_DIED;
        }
        IterRecord r;
        r.iter = done;
        r.nw = nw;
        r.nd = nd;
        r.c0 = c0;
        r.attempts = att;
        r.spawns = (int64_t)a.spawns[s];
        r.merged = merged;
        r.aborted = aborted;
        r.born = born;
        r.used = used;
        r.n_var = d.n_var;
        r.n_prev = d.n_prev;
        r.num = num;
        r.shift = d.shift;
        r.varying = d.varying;
        r.status = (int32_t)a.status[s];
        if (a.spilled[s]) {
            // new determinants wait in the spill list: pause until the host re-buckets
            a.status[s] |= ST_SPILLED;
            r.status = (int32_t)a.status[s];
            a.spilled[s] = 0u;
        }
        a.rec[(int64_t)s * REC_CAP + (done % REC_CAP)] = r;
        a.spawns[s] = 0ull;
        d.iter = done;
    }
}

static_assert(FIN_BLOCKS == 64, "k_finalize sums one share per lane of a wavefront");
static_assert(SCAN_G == 2048, "k_scan takes two range totals per thread of 1024");
static_assert(POST_WAVES * 64 == 256, "one ChunkStat share per wavefront of a k_post workgroup");

void launch_iteration(const EngineArgs &a, int post_grid, int spawn_grid, bool first,
                      hipStream_t s, hipEvent_t *ev) {
    if (ev) (void)hipEventRecord(ev[0], s);
    if (first)
        hipLaunchKernelGGL(k_chunk_sum, dim3(SCAN_G), dim3(256), 0, s, a, (const SysDesc *)a.desc);
    if (ev) (void)hipEventRecord(ev[1], s);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(k_scan_down, dim3(SCAN_G), dim3(256), 0, s, a);
    if (ev) (void)hipEventRecord(ev[2], s);
    if (a.plain)
        hipLaunchKernelGGL(k_spawn<true>, dim3((unsigned)spawn_grid), dim3(256), 0, s, a,
                           (const SysDesc *)a.desc);
    else
        hipLaunchKernelGGL(k_spawn<false>, dim3((unsigned)spawn_grid), dim3(256), 0, s, a,
                           (const SysDesc *)a.desc);
    if (ev) (void)hipEventRecord(ev[3], s);
    hipLaunchKernelGGL(k_fix, dim3((unsigned)spawn_grid), dim3(256), 0, s, a,
                       (const SysDesc *)a.desc);
    hipLaunchKernelGGL(k_bscan_up, dim3(SCAN_G), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_bscan_top, dim3(1), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(k_bscan_down, dim3(SCAN_G), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)spawn_grid), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_post, dim3((unsigned)post_grid), dim3(256), 0, s, a,
                       (const SysDesc *)a.desc);
    if (ev) (void)hipEventRecord(ev[4], s);
    hipLaunchKernelGGL(k_reduce, dim3(FIN_BLOCKS, (unsigned)a.max_sys), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)a.max_sys), dim3(64), 0, s, a);
    if (ev) (void)hipEventRecord(ev[5], s);
}

// ---------------------------------------------------------------------------
// Loading a walker list, re-bucketing into more (or fewer) buckets, exporting.
// ---------------------------------------------------------------------------
// Append determinant D (population p, diagonal element hd) to its bucket.
__device__ __forceinline__ bool bucket_put(const SysDesc &d, det_t D, int32_t p, double hd) {
    const uint32_t b = bucket_of(D, (uint64_t)d.nbuckets);
    const int pos = atomicAdd(&d.bcnt[b], 1);
    if (pos >= BQ) return false;
    const int64_t j = (int64_t)b * BQ + pos;
    keys_of(d)[j] = D;
    d.pop[j] = p;
    d.hdiag[j] = hd;
    return true;
}

__global__ void k_load(SysDesc *desc, int32_t sys, const det_t *det, const int32_t *pop,
                       int64_t n, uint32_t *err) {
    const SysDesc &d = desc[sys];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const det_t D = det[i];
        if (!bucket_put(d, D, pop[i], fn_diag(d, D))) atomicOr(err, 1u);
    }
}

__global__ void k_rebucket(SysDesc *desc, int32_t sys, const det_t *skey, const int32_t *spop,
                           const double *shd, const int32_t *scnt, int64_t snb,
                           const det_t *xdet, const int32_t *xpop, const double *xhd,
                           const int32_t *xsys, int64_t nx, uint32_t *err) {
    const SysDesc &d = desc[sys];
    const int64_t ns = snb * BQ;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ns + nx;
         i += (int64_t)gridDim.x * blockDim.x) {
        det_t D;
        int32_t p;
        double hd;
        if (i < ns) {
            if ((int)(i % BQ) >= scnt[i / BQ]) continue;
            D = skey[i];
            p = spop[i];
            hd = shd[i];
        } else {
            const int64_t k = i - ns;
            if (xsys[k] != sys) continue;
            D = xdet[k];
            p = xpop[k];
            hd = xhd[k];
        }
        if (p == 0 && D != ref_of(d)) continue;
        if (!bucket_put(d, D, p, hd)) atomicOr(err, 1u);
    }
}

// Occupied entries (population != 0) of nb buckets, in any order, into odet/opop
// (at most `limit` written; *count gets the total). One counter atomic per wavefront.
__global__ __launch_bounds__(256) void k_compact(const det_t *kv, const int32_t *pop,
                                                 const int32_t *cnt, int64_t nb, det_t *odet,
                                                 int32_t *opop, unsigned long long *count,
                                                 int64_t limit) {
    const int lane = threadIdx.x & 63;
    const int64_t ns = nb * BQ;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < ns;
         base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = base + threadIdx.x;
        bool take = false;
        det_t D = det_t(0ull);
        int32_t p = 0;
        if (i < ns && (int)(i % BQ) < cnt[i / BQ]) {
            D = kv[i];
            p = pop[i];
            take = p != 0;
        }
        const uint64_t m = __ballot(take);
        if (!m) continue;
        unsigned long long b = 0;
        const int first = __builtin_ctzll(m);
        if (lane == first) b = atomicAdd(count, (unsigned long long)__popcll(m));
        b = __shfl(b, first, 64);
        if (take) {
            const unsigned long long j = b + (unsigned long long)__popcll(m & ((1ull << lane) - 1ull));
            if (j < (unsigned long long)limit) {
                odet[j] = D;
                opop[j] = p;
            }
        }
    }
}

hipError_t launch_load(SysDesc *d_desc, int32_t sys, const uint64_t *det, const int32_t *pop,
                       int64_t n, uint32_t *d_err, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t g = (n + 255) / 256;
    hipLaunchKernelGGL(k_load, dim3((unsigned)(g < 65536 ? g : 65536)), dim3(256), 0, s, d_desc,
                       sys, (const det_t *)det, pop, n, d_err);
    return hipGetLastError();
}

hipError_t launch_rebucket(SysDesc *d_desc, int32_t sys, const uint64_t *src_key,
                           const int32_t *src_pop, const double *src_hd, const int32_t *src_cnt,
                           int64_t src_nb, const uint64_t *sp_det, const int32_t *sp_pop,
                           const double *sp_hd, const int32_t *sp_sys, int64_t n_sp,
                           uint32_t *d_err, hipStream_t s) {
    const int64_t g = (src_nb * BQ + n_sp + 255) / 256;
    if (g == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rebucket, dim3((unsigned)(g < 65536 ? g : 65536)), dim3(256), 0, s,
                       d_desc, sys, (const det_t *)src_key, src_pop, src_hd, src_cnt, src_nb,
                       (const det_t *)sp_det, sp_pop, sp_hd, sp_sys, n_sp, d_err);
    return hipGetLastError();
}

hipError_t launch_compact(const uint64_t *key, const int32_t *pop, const int32_t *cnt, int64_t nb,
                          uint64_t *out_det, int32_t *out_pop, unsigned long long *count,
                          hipStream_t s) {
    const int64_t g = (nb * BQ + 255) / 256;
    hipLaunchKernelGGL(k_compact, dim3((unsigned)(g < 65536 ? g : 65536)), dim3(256), 0, s,
                       (const det_t *)key, pop, cnt, nb, (det_t *)out_det, out_pop, count, nb * BQ);
    return hipGetLastError();
}

#if FQ_DET_WORDS == 1
// ---------------------------------------------------------------------------
// Export through a fixed staging area (no allocation): the counter is cleared by
// a kernel (no memset node), the occupied slots are compacted with one counter
// atomic per wavefront, and the keys are sorted by a bitonic network over the
// next power of two (padding keys ~0 sort last).
// ---------------------------------------------------------------------------
__global__ void k_stage_clear(unsigned long long *count) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *count = 0ull;
}

__global__ void k_stage_pad(uint64_t *key, int64_t n, int64_t P) {
    for (int64_t i = n + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < P;
         i += (int64_t)gridDim.x * blockDim.x)
        key[i] = ~0ull;
}

__global__ void k_stage_bitonic(uint64_t *key, int32_t *val, int64_t P, int64_t j, int64_t k) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < P;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t l = i ^ j;
        if (l <= i) continue;
        const bool up = (i & k) == 0;
        const uint64_t a = key[i], b = key[l];
        if ((a > b) == up) {
            key[i] = b;
            key[l] = a;
            const int32_t t = val[i];
            val[i] = val[l];
            val[l] = t;
        }
    }
}

__global__ void k_stage_flags(const uint64_t *key, const int32_t *val, int64_t n, int32_t n_a,
                              uint64_t d0, uint32_t *flags) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = val[i] < 0 ? -(int64_t)val[i] : (int64_t)val[i];
        flags[i] = (a > (int64_t)n_a || key[i] == d0) ? 1u : 0u;
    }
}

hipError_t launch_stage_flags(void *stage, int64_t n, int32_t n_a, uint64_t d0, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    char *p = (char *)stage;
    const int64_t g = (n + 255) / 256;
    hipLaunchKernelGGL(k_stage_flags, dim3((unsigned)(g < 8192 ? g : 8192)), dim3(256), 0, s,
                       (const uint64_t *)(p + NOALLOC_KEYS_OFF), (const int32_t *)(p + NOALLOC_VALS_OFF),
                       n, n_a, d0, (uint32_t *)(p + NOALLOC_FLAGS_OFF));
    return hipGetLastError();
}

hipError_t launch_stage_compact(const uint64_t *key, const int32_t *pop, const int32_t *cnt,
                                int64_t nb, void *stage, hipStream_t s) {
    char *p = (char *)stage;
    unsigned long long *count = (unsigned long long *)p;
    hipLaunchKernelGGL(k_stage_clear, dim3(1), dim3(64), 0, s, count);
    const int64_t g = (nb * BQ + 255) / 256;
    hipLaunchKernelGGL(k_compact, dim3((unsigned)(g < 65536 ? g : 65536)), dim3(256), 0, s, key,
                       pop, cnt, nb, (uint64_t *)(p + NOALLOC_KEYS_OFF),
                       (int32_t *)(p + NOALLOC_VALS_OFF), count, (int64_t)NOALLOC_MAX_DETS);
    return hipGetLastError();
}

hipError_t launch_stage_sort(void *stage, int64_t n, hipStream_t s) {
    if (n > NOALLOC_MAX_DETS) return hipErrorInvalidValue;
    char *p = (char *)stage;
    uint64_t *key = (uint64_t *)(p + NOALLOC_KEYS_OFF);
    int32_t *val = (int32_t *)(p + NOALLOC_VALS_OFF);
    int64_t P = 1;
    while (P < n) P <<= 1;
    if (P < 2) return hipSuccess;
    const int64_t g = (P + 255) / 256;
    const unsigned grid = (unsigned)(g < 8192 ? g : 8192);
    hipLaunchKernelGGL(k_stage_pad, dim3(grid), dim3(256), 0, s, key, n, P);
    for (int64_t k = 2; k <= P; k <<= 1)
        for (int64_t j = k >> 1; j > 0; j >>= 1)
            hipLaunchKernelGGL(k_stage_bitonic, dim3(grid), dim3(256), 0, s, key, val, P, j, k);
    return hipGetLastError();
}

#endif   // the staging export (one-word determinants only)

__global__ void k_e0(const SysDesc *desc, int32_t sys, uint64_t lo, uint64_t hi, double *out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *out = fn_diag(desc[sys], make_det(lo, hi));
}

hipError_t launch_e0(const SysDesc *desc, int32_t sys, uint64_t lo, uint64_t hi, double *out,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_e0, dim3(1), dim3(64), 0, s, desc, sys, lo, hi, out);
    return hipGetLastError();
}

#if FQ_DET_WORDS == 1

static int cu_count() {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
            cus = prop.multiProcessorCount;
    }
    return cus;
}
int post_grid_size() { return cu_count() * 4; }    // four workgroups per CU
int spawn_grid_size() { return cu_count() * 6; }   // six resident workgroups per CU
#endif

#if FQ_DET_WORDS == 2
}  // namespace w2
#endif
}  // namespace fq
