/*
 * CPU oracle: a plain FCIQMC iteration written from Booth, Smart & Alavi,
 * arXiv:1305.6981.
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the benchmark's
 * CPU-baseline leg. The product library neither links nor calls it, and the
 * two share no source.
 *
 * What is followed, and where:
 *   - walker dynamics: spawning, death/cloning, same-iteration isolation
 *     (Sec. 2, Eqs. master, pspawn, pdeath);
 *   - determinant representation and byte-table decoding (Sec. 3, 3.1);
 *   - Algorithm 1 hash with a random orbital map, a main-list hash table with
 *     chaining and a circular list of vacant slots (Sec. 4, 4.2);
 *   - sorting and compression of the spawned list (Sec. 4.1, footnote on
 *     sorting), annihilation and the initiator test at that stage (Sec. 4.2);
 *   - excitation generation with renormalisation over electrons/orbitals that
 *     have no allowed partner, and the generation probabilities of Eq. p_sing
 *     and of the double-excitation formula (Sec. 5, 5.1, 5.2);
 *   - Slater-Condon matrix elements ("standard rules", Sec. 2);
 *   - projected energy (Eq. ProjE) and the shift (Sec. 2);
 *   - blocking analysis of the correlated ratio (Sec. 7, Flyvbjerg-Petersen);
 *   - optionally, the distribution of determinants over P virtual processes
 *     (Sec. 4.1): each determinant lives on the process picked by a second
 *     Algorithm-1 hash (own random map, range P), every process spawns from
 *     its own list into one block per destination, the blocks are transposed
 *     (the all-to-all exchange), and each process compresses and annihilates
 *     what it received against its own list. Optionally the reference gets a
 *     process of its own and the rest are hashed over the other P-1. The
 *     processes may run on host threads; results do not depend on P or on
 *     the thread count (integer merges, determinant-keyed random numbers),
 *     except the rounding order of the projected-energy numerator sum.
 *
 * Readings where the paper is silent:
 *   RNG = Philox4x32-10 (Salmon et al., SC'11) keyed by the seed (XOR the
 *   determinant's second word beyond 64 spin orbitals), with a counter built
 *   from (determinant, walker ordinal, iteration, block); a
 *   spawning attempt uses one block: word 0 picks the type and, rescaled
 *   within the chosen type's probability interval, is the acceptance uniform;
 *   words 1-3 pick the orbitals (index = floor(w n / 2^32));
 *   the a/b orbitals are picked by enumerating the allowed set (the paper's
 *   stated alternative to drawing with rejection; same pgen); initiator =
 *   |C| > n_a or the reference; the merged spawn flag is the OR of parents'
 *   flags; occupancy for the initiator test is judged after death; the shift
 *   is S <- S - zeta/(A tau) ln(N_w/N_prev), tested every A iterations; death
 *   is one stochastic rounding per determinant.
 *
 * Built with -ffp-contract=off: every floating-point decision uses the
 * operation order written here.
 */
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* Per host thread, so that worker threads of the virtual-process mode keep
 * their own message until the caller collects it. */
static _Thread_local char g_err[512];

static int fail(const char *msg)
{
    snprintf(g_err, sizeof g_err, "%s", msg);
    return -1;
}

const char *orc_last_error(void) { return g_err; }

/* ------------------------------------------------------------------------ */
/* Determinants (Sec. 3): bit p set when spin orbital p is occupied, in as   */
/* many 64-bit words as the spin orbitals need (one up to 64, two up to 128). */
/* Held here as one 128-bit integer; in the API as 1 or 2 words, low first.  */
/* ------------------------------------------------------------------------ */
typedef unsigned __int128 det_t;
#define MAX_SO 128
#define MAX_ORB 64
#define DBIT(p) ((det_t)1 << (p))

static uint64_t det_lo(det_t d) { return (uint64_t)d; }
static uint64_t det_hi(det_t d) { return (uint64_t)(d >> 64); }
static det_t det_make(uint64_t lo, uint64_t hi) { return ((det_t)hi << 64) | (det_t)lo; }

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11).                       */
/* Each round: two 32x32->64 products of counter words 0 and 2 with the      */
/* round multipliers; the new counter is (hi1^c1^k0, lo1, hi0^c3^k1, lo0).   */
/* The two key words are bumped by the Weyl constants between rounds.        */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* Random-number contract (a reading: the paper uses a Mersenne Twister).
 * key = (lo32(K), hi32(K)) with K = seed XOR (bits 64..127 of D);
 * counter = (bits 0..31 of D, bits 32..63 of D, k, ((n mod 2^24) << 8) | block).
 * (For determinants of at most 64 spin orbitals K is the seed.)
 * Spawn attempt k on D at iteration n:
 *   block 0 -> x0 (excitation type), x1 (electron or electron pair)
 *   block 1 -> x2 (orbital a), x3 (orbital b)
 *   block 2 -> x4 (acceptance)
 * Death on D: k = 0xFFFFFFFF, block 0x80 -> x0.
 * A 64-bit draw is (w[2j+1] << 32) | w[2j]. */
static void draw_block(uint64_t seed, det_t det, uint32_t k, int64_t iter, uint32_t block,
                       uint64_t x[2])
{
    uint32_t ctr[4], key[2], w[4];
    const uint64_t lo = det_lo(det), kk = seed ^ det_hi(det);
    ctr[0] = (uint32_t)lo;
    ctr[1] = (uint32_t)(lo >> 32);
    ctr[2] = k;
    ctr[3] = ((uint32_t)((uint64_t)iter & 0xFFFFFFu) << 8) | block;
    key[0] = (uint32_t)kk;
    key[1] = (uint32_t)(kk >> 32);
    orc_philox4x32_10(ctr, key, w);
    x[0] = ((uint64_t)w[1] << 32) | (uint64_t)w[0];
    x[1] = ((uint64_t)w[3] << 32) | (uint64_t)w[2];
}

/* Uniform double in [0, 1) from the top 53 bits. */
static double unit_uniform(uint64_t x)
{
    return (double)(x >> 11) * (1.0 / 9007199254740992.0);
}

/* The four 32-bit words of one Philox block, for a spawning attempt: word 0
 * decides the type (and, rescaled, the acceptance), words 1-3 the orbitals. */
static void draw_words(uint64_t seed, det_t det, uint32_t k, int64_t iter, uint32_t block,
                       uint32_t w[4])
{
    uint32_t ctr[4], key[2];
    const uint64_t lo = det_lo(det), kk = seed ^ det_hi(det);
    ctr[0] = (uint32_t)lo;
    ctr[1] = (uint32_t)(lo >> 32);
    ctr[2] = k;
    ctr[3] = ((uint32_t)((uint64_t)iter & 0xFFFFFFu) << 8) | block;
    key[0] = (uint32_t)kk;
    key[1] = (uint32_t)(kk >> 32);
    orc_philox4x32_10(ctr, key, w);
}

/* w / 2^32, exact in double. */
static double unit_uniform32(uint32_t w) { return (double)w * (1.0 / 4294967296.0); }

/* Natural logarithm used by the shift update. Method: write x = m 2^e with
 * m in (1/sqrt2, sqrt2], then ln x = e ln2 + 2 atanh(z), z = (m-1)/(m+1),
 * with the odd series of atanh summed by Horner's rule up to z^25
 * (|z| <= 0.1716, so the first omitted term is below 1e-20). The operation
 * order is fixed so that the same method gives the same bits on any IEEE
 * double machine without fused multiply-adds. */
double orc_log(double x)
{
    uint64_t bits;
    memcpy(&bits, &x, sizeof bits);
    int e = (int)((bits >> 52) & 0x7FFu) - 1023;
    uint64_t mb = (bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull;
    double m;
    memcpy(&m, &mb, sizeof m);
    if (m > 1.4142135623730951) {
        m = m * 0.5;
        e = e + 1;
    }
    double z = (m - 1.0) / (m + 1.0);
    double z2 = z * z;
    double sum = 1.0 / 27.0;
    for (int k = 25; k >= 1; k -= 2)
        sum = sum * z2 + 1.0 / (double)k;
    return (double)e * 0.6931471805599453 + 2.0 * z * sum;
}

/* Uniform index in [0, n): floor(x * n / 2^64). */
/* floor(w n / 2^32): an index in [0, n) (bias below n / 2^32). */
static uint64_t uniform_index32(uint32_t w, uint64_t n)
{
    return ((uint64_t)w * n) >> 32;
}

/* ------------------------------------------------------------------------ */
/* Decoding through a 256-entry byte table (Sec. 3.1): each entry holds the  */
/* number of set bits of the byte and their positions.                      */
/* ------------------------------------------------------------------------ */
static int g_lut_ready;
static uint8_t g_lut_count[256];
static uint8_t g_lut_orb[256][8];

static void build_lut(void)
{
    if (g_lut_ready)
        return;
    for (int v = 0; v < 256; v++) {
        int c = 0;
        for (int b = 0; b < 8; b++)
            if (v & (1 << b))
                g_lut_orb[v][c++] = (uint8_t)b;
        g_lut_count[v] = (uint8_t)c;
    }
    g_lut_ready = 1;
}

static int decode_det(det_t det, int32_t *occ)
{
    build_lut();
    int n = 0;
    for (int byte = 0; byte < 16; byte++) {
        unsigned v = (unsigned)((det >> (8 * byte)) & 0xFFu);
        if (!v)
            continue;
        for (int j = 0; j < g_lut_count[v]; j++)
            occ[n++] = 8 * byte + g_lut_orb[v][j];
    }
    return n;
}

int orc_decode(const uint64_t *det, int32_t words, int32_t *occ)
{
    return decode_det(det_make(det[0], words > 1 ? det[1] : 0), occ);
}

static int popcount64(det_t x)
{
    int c = 0;
    while (x) {
        x &= x - 1;
        c++;
    }
    return c;
}

/* ------------------------------------------------------------------------ */
/* Hamiltonian.                                                              */
/* ------------------------------------------------------------------------ */
typedef struct {
    int M, N, n_alpha, n_beta, n_so;
    double e_core;
    double *h1, *eri;
    int irrep[MAX_ORB];
    int n_class;
    int class_of[MAX_SO];
    double p_double, p_single;
    double inv_p_double, inv_p_single;   /* 1/P_double, 1/P_single (0 when the type is impossible) */
    det_t d0;
    double e0;
    int hphf;                 /* 0, or the spin parity (+1 even S, -1 odd S) of the
                                 spin-coupled functions (Sec. 5.3) */
    int lam;                  /* their relative sign (-1)^S (-1)^{N/2} (see hphf_rep) */
} sys_t;

static int64_t pair_index(int i, int j)
{
    if (i < j) {
        int t = i;
        i = j;
        j = t;
    }
    return (int64_t)i * (i + 1) / 2 + j;
}

static double eri_spatial(const sys_t *s, int i, int j, int k, int l)
{
    int64_t a = pair_index(i, j), b = pair_index(k, l);
    if (a < b) {
        int64_t t = a;
        a = b;
        b = t;
    }
    return s->eri[a * (a + 1) / 2 + b];
}

/* (pq|rs) over spin orbitals: zero unless p,q share a spin and r,s share a spin. */
static double eri_so(const sys_t *s, int p, int q, int r, int t)
{
    if ((p & 1) != (q & 1) || (r & 1) != (t & 1))
        return 0.0;
    return eri_spatial(s, p >> 1, q >> 1, r >> 1, t >> 1);
}

static double h_so(const sys_t *s, int p, int q)
{
    if ((p & 1) != (q & 1))
        return 0.0;
    return s->h1[(p >> 1) * s->M + (q >> 1)];
}

/* Number of occupied orbitals strictly between p and a. */
static int n_between(det_t det, int p, int a)
{
    int lo = p < a ? p : a, hi = p < a ? a : p;
    int c = 0;
    for (int r = lo + 1; r < hi; r++)
        if ((det >> r) & 1u)
            c++;
    return c;
}

/* Diagonal element: E_core + sum_p h_pp + sum_{p<q} [(pp|qq) - (pq|qp)]. */
static double hdiag_of(const sys_t *s, det_t det)
{
    int32_t occ[MAX_SO];
    int n = decode_det(det, occ);
    double acc = s->e_core;
    for (int i = 0; i < n; i++)
        acc = acc + h_so(s, occ[i], occ[i]);
    for (int i = 0; i < n; i++)
        for (int j = i + 1; j < n; j++)
            acc = acc + (eri_so(s, occ[i], occ[i], occ[j], occ[j]) -
                         eri_so(s, occ[i], occ[j], occ[j], occ[i]));
    return acc;
}

/* Single excitation p -> a from det: sign * (h_pa + sum_{q occ, q != p} [(pa|qq) - (pq|qa)]). */
static double hel_single(const sys_t *s, det_t det, int p, int a)
{
    int32_t occ[MAX_SO];
    int n = decode_det(det, occ);
    double acc = h_so(s, p, a);
    for (int i = 0; i < n; i++) {
        int q = occ[i];
        if (q == p)
            continue;
        acc = acc + (eri_so(s, p, a, q, q) - eri_so(s, p, q, q, a));
    }
    if (n_between(det, p, a) & 1)
        acc = -acc;
    return acc;
}

/* Double excitation p,q -> a,b (p<q occupied; a,b empty).
 * Pairing: for unlike spins a' carries the spin of p; for like spins a' = min(a, b).
 * Sign: parity of q -> b' on det, times parity of p -> a' on the result. */
static double hel_double(const sys_t *s, det_t det, int p, int q, int a, int b)
{
    int ap, bp;
    if ((p & 1) != (q & 1)) {
        if ((a & 1) == (p & 1)) {
            ap = a;
            bp = b;
        } else {
            ap = b;
            bp = a;
        }
    } else {
        ap = a < b ? a : b;
        bp = a < b ? b : a;
    }
    int nsw = n_between(det, q, bp);
    det_t d1 = (det & ~DBIT(q)) | DBIT(bp);
    nsw += n_between(d1, p, ap);
    double v = eri_so(s, p, ap, q, bp) - eri_so(s, p, bp, q, ap);
    return (nsw & 1) ? -v : v;
}

/* <bra|H|ket>, ket taken as the source of the excitation. */
static double hel_general(const sys_t *s, det_t bra, det_t ket)
{
    if (popcount64(bra) != popcount64(ket))
        return 0.0;
    det_t diff = bra ^ ket;
    int nd = popcount64(diff);
    if (nd == 0)
        return hdiag_of(s, ket);
    int from[2], to[2], nf = 0, nt = 0;
    if (nd > 4)
        return 0.0;
    for (int r = 0; r < s->n_so; r++) {
        if (!((diff >> r) & 1u))
            continue;
        if ((ket >> r) & 1u)
            from[nf++] = r;
        else
            to[nt++] = r;
    }
    if (nd == 2)
        return hel_single(s, ket, from[0], to[0]);
    return hel_double(s, ket, from[0], from[1], to[0], to[1]);
}

/* ------------------------------------------------------------------------ */
/* Excitation generation (Sec. 5).                                           */
/* Symmetry classes: (irrep, spin); class id = 2*irrep + spin.               */
/* ------------------------------------------------------------------------ */
typedef struct {
    det_t det;
    int n;
    int32_t occ[MAX_SO];
    int n_unocc[16];
} detinfo_t;

static void det_setup(const sys_t *s, det_t det, detinfo_t *di)
{
    di->det = det;
    di->n = decode_det(det, di->occ);
    for (int c = 0; c < 16; c++)
        di->n_unocc[c] = 0;
    for (int r = 0; r < s->n_so; r++)
        if (!((det >> r) & 1u))
            di->n_unocc[s->class_of[r]]++;
}

static int class_id(int irrep, int spin) { return 2 * irrep + spin; }

/* Number of empty orbitals that can pair with x as the second orbital of a
 * double excitation from the pair (p, q) (Eq. sym1 plus spin), excluding x. */
static int n_partner(const sys_t *s, const detinfo_t *di, int p, int q, int x)
{
    int spin_b = ((p & 1) == (q & 1)) ? (p & 1) : 1 - (x & 1);
    int irrep_b = s->irrep[p >> 1] ^ s->irrep[q >> 1] ^ s->irrep[x >> 1];
    int cb = class_id(irrep_b, spin_b);
    int n = di->n_unocc[cb];
    if (cb == s->class_of[x])
        n -= 1;
    return n;
}

static int partner_ok(const sys_t *s, int p, int q, int x, int y)
{
    int spin_b = ((p & 1) == (q & 1)) ? (p & 1) : 1 - (x & 1);
    int irrep_b = s->irrep[p >> 1] ^ s->irrep[q >> 1] ^ s->irrep[x >> 1];
    return s->class_of[y] == class_id(irrep_b, spin_b) && y != x;
}

typedef struct {
    det_t det;      /* 0 = null excitation */
    double pgen;
    double hel;
} excit_t;

/* One excitation from the type word w[0] and the choice words w[1..3]. */
static void gen_excit(const sys_t *s, const detinfo_t *di, const uint32_t w[4], excit_t *out)
{
    const int N = di->n;
    const det_t det = di->det;
    out->det = 0;
    out->pgen = 0.0;
    out->hel = 0.0;
    int is_double = unit_uniform32(w[0]) < s->p_double;
    if (!is_double) {
        /* Sec. 5.1: renormalise over the electrons that have an allowed a. */
        int n_allow[MAX_SO], delta_s = 0;
        for (int e = 0; e < N; e++) {
            n_allow[e] = di->n_unocc[s->class_of[di->occ[e]]];
            if (n_allow[e] == 0)
                delta_s++;
        }
        if (N - delta_s == 0)
            return;
        uint64_t ke = uniform_index32(w[1], (uint64_t)(N - delta_s));
        int esel = -1;
        for (int e = 0; e < N; e++) {
            if (n_allow[e] == 0)
                continue;
            if (ke == 0) {
                esel = e;
                break;
            }
            ke--;
        }
        int p = di->occ[esel];
        int cls = s->class_of[p];
        uint64_t ka = uniform_index32(w[2], (uint64_t)n_allow[esel]);
        int a = -1;
        for (int r = 0; r < s->n_so; r++) {
            if (((det >> r) & 1u) || s->class_of[r] != cls)
                continue;
            if (ka == 0) {
                a = r;
                break;
            }
            ka--;
        }
        out->det = det ^ DBIT(p) ^ DBIT(a);
        out->pgen = s->p_single / (double)((int64_t)n_allow[esel] * (int64_t)(N - delta_s));
        out->hel = hel_single(s, det, p, a);
        return;
    }
    /* Sec. 5.2: a unique pair by inverse triangular indexing. */
    if (N < 2)
        return;
    int64_t n_pairs = (int64_t)N * (N - 1) / 2;
    int64_t K = (int64_t)uniform_index32(w[1], (uint64_t)n_pairs);
    int j = 1;
    while ((int64_t)(j + 1) * j / 2 <= K)
        j++;
    int i = (int)(K - (int64_t)j * (j - 1) / 2);
    int p = di->occ[i], q = di->occ[j];
    int same = (p & 1) == (q & 1);
    /* Count the allowed a orbitals and those with no partner b (delta_d). */
    int n_a_set = 0, delta_d = 0;
    for (int r = 0; r < s->n_so; r++) {
        if ((det >> r) & 1u)
            continue;
        if (same && (r & 1) != (p & 1))
            continue;
        n_a_set++;
        if (n_partner(s, di, p, q, r) == 0)
            delta_d++;
    }
    if (n_a_set - delta_d == 0)
        return;
    uint64_t ka = uniform_index32(w[2], (uint64_t)(n_a_set - delta_d));
    int a = -1;
    for (int r = 0; r < s->n_so; r++) {
        if ((det >> r) & 1u)
            continue;
        if (same && (r & 1) != (p & 1))
            continue;
        if (n_partner(s, di, p, q, r) == 0)
            continue;
        if (ka == 0) {
            a = r;
            break;
        }
        ka--;
    }
    int nba = n_partner(s, di, p, q, a);
    uint64_t kb = uniform_index32(w[3], (uint64_t)nba);
    int b = -1;
    for (int r = 0; r < s->n_so; r++) {
        if ((det >> r) & 1u)
            continue;
        if (!partner_ok(s, p, q, a, r))
            continue;
        if (kb == 0) {
            b = r;
            break;
        }
        kb--;
    }
    int nbb = n_partner(s, di, p, q, b);
    out->det = det ^ DBIT(p) ^ DBIT(q) ^ DBIT(a) ^ DBIT(b);
    out->pgen = (2.0 * s->p_double * (1.0 / (double)nba + 1.0 / (double)nbb)) /
                (double)((int64_t)N * (N - 1) * (int64_t)(n_a_set - delta_d));
    out->hel = hel_double(s, det, p, q, a, b);
}

/* The probability that gen_excit produces T from the determinant of di: the
 * single-excitation probability of Sec. 5.1 or the double-excitation formula of
 * Sec. 5.2 for the excitation that turns the determinant into T, 0 when T is not
 * a single or double excitation the generator can draw. */
static double pgen_of(const sys_t *s, const detinfo_t *di, det_t T)
{
    const det_t det = di->det;
    const int N = di->n;
    if (popcount64(T) != popcount64(det))
        return 0.0;
    const det_t from = det & ~T, to = T & ~det;
    const int nf = popcount64(from);
    int f[2], t[2], k = 0, m = 0;
    for (int r = 0; r < s->n_so; r++) {
        if ((from >> r) & 1u && k < 2)
            f[k++] = r;
        if ((to >> r) & 1u && m < 2)
            t[m++] = r;
    }
    if (nf == 1) {
        const int p = f[0], a = t[0];
        if (s->class_of[a] != s->class_of[p])
            return 0.0;
        int delta_s = 0;
        for (int e = 0; e < N; e++)
            if (di->n_unocc[s->class_of[di->occ[e]]] == 0)
                delta_s++;
        const int nal = di->n_unocc[s->class_of[p]];
        return s->p_single / (double)((int64_t)nal * (int64_t)(N - delta_s));
    }
    if (nf != 2)
        return 0.0;
    const int p = f[0], q = f[1], a = t[0], b = t[1];
    const int same = (p & 1) == (q & 1);
    if (same && ((a & 1) != (p & 1) || (b & 1) != (p & 1)))
        return 0.0;
    if (!partner_ok(s, p, q, a, b))
        return 0.0;
    int n_a_set = 0, delta_d = 0;
    for (int r = 0; r < s->n_so; r++) {
        if ((det >> r) & 1u)
            continue;
        if (same && (r & 1) != (p & 1))
            continue;
        n_a_set++;
        if (n_partner(s, di, p, q, r) == 0)
            delta_d++;
    }
    const int nba = n_partner(s, di, p, q, a), nbb = n_partner(s, di, p, q, b);
    return (2.0 * s->p_double * (1.0 / (double)nba + 1.0 / (double)nbb)) /
           (double)((int64_t)N * (N - 1) * (int64_t)(n_a_set - delta_d));
}

/* ------------------------------------------------------------------------ */
/* Spin-coupled functions (Sec. 5.3, Eqs. EqualCoeffs and SpinCoup). With the */
/* spin orbitals interleaved (p = 2s + sigma), exchanging the alpha and beta  */
/* occupations of every spatial orbital maps |D> to (-1)^{n2(D)} |D~>, n2 the */
/* number of doubly occupied orbitals (each such pair of creation operators   */
/* swaps order) and D~ the exchanged bit string. The function of the pair    */
/* {D, D~} with spin parity (-1)^S is (|D> + lam (-1)^{n2(D)} |D~>) / sqrt 2, */
/* lam = (-1)^S (-1)^{N/2}; a closed pair (D = D~: every orbital empty or      */
/* doubly occupied) is |D> itself and belongs to even S only. A function is    */
/* stored as min(D, D~).                                                        */
/* ------------------------------------------------------------------------ */
#define EVEN_BITS det_make(0x5555555555555555ull, 0x5555555555555555ull)

static det_t spin_flip(det_t D) { return ((D & EVEN_BITS) << 1) | ((D >> 1) & EVEN_BITS); }

static int n_doubly(det_t D) { return popcount64(D & (D >> 1) & EVEN_BITS); }

static det_t hphf_rep(det_t D)
{
    det_t f = spin_flip(D);
    return f < D ? f : D;
}

/* <Phi_j|H|Phi_i> for the functions stored as Dj and Di (Di the source of the
 * excitation, Dj != Di). Both open: <Dj|H|Di> + lam (-1)^{n2(Dj)} <Dj~|H|Di>; one
 * closed: sqrt2 <Dj|H|Di> (the other term equals the first); both closed:
 * <Dj|H|Di>. Every element is evaluated with Di as the source. */
static double hphf_hel(const sys_t *s, det_t Di, det_t Dj)
{
    const det_t fi = spin_flip(Di), fj = spin_flip(Dj);
    const double h = hel_general(s, Dj, Di);
    if (fi != Di && fj != Dj) {
        const int sg = (n_doubly(Dj) & 1) ? -s->lam : s->lam;
        return h + (double)sg * hel_general(s, fj, Di);
    }
    if (fi != Di || fj != Dj)
        return 1.4142135623730951 * h;
    return h;
}

/* Diagonal element of the stored function D (of the determinant D without
 * spin-coupled functions). */
static double fdiag(const sys_t *s, det_t D)
{
    const double h = hdiag_of(s, D);
    if (!s->hphf)
        return h;
    const det_t f = spin_flip(D);
    if (f == D)
        return h;
    const int sg = (n_doubly(D) & 1) ? -s->lam : s->lam;
    return h + (double)sg * hel_general(s, f, D);
}

/* <Phi_0|H|Phi_D> for the projected energy, 0 beyond double excitations. */
static double ref_hel(const sys_t *s, det_t D)
{
    if (!s->hphf)
        return popcount64(D ^ s->d0) <= 4 ? hel_general(s, D, s->d0) : 0.0;
    if (popcount64(D ^ s->d0) > 4 && popcount64(spin_flip(D) ^ s->d0) > 4)
        return 0.0;
    return hphf_hel(s, s->d0, D);
}

/* Counts of symmetry-allowed single and double excitations from a determinant,
 * by enumeration (used to fix P_double from the reference, Sec. 5). */
static void count_excitations(const sys_t *s, det_t det, int64_t *n_single, int64_t *n_double)
{
    int32_t occ[MAX_SO];
    int n = decode_det(det, occ);
    int64_t ns = 0, nd = 0;
    for (int e = 0; e < n; e++)
        for (int r = 0; r < s->n_so; r++)
            if (!((det >> r) & 1u) && s->class_of[r] == s->class_of[occ[e]])
                ns++;
    for (int i = 0; i < n; i++)
        for (int j = i + 1; j < n; j++) {
            int p = occ[i], q = occ[j];
            int sym = s->irrep[p >> 1] ^ s->irrep[q >> 1];
            for (int a = 0; a < s->n_so; a++) {
                if ((det >> a) & 1u)
                    continue;
                for (int b = a + 1; b < s->n_so; b++) {
                    if ((det >> b) & 1u)
                        continue;
                    if ((a & 1) + (b & 1) != (p & 1) + (q & 1))
                        continue;
                    if ((s->irrep[a >> 1] ^ s->irrep[b >> 1]) != sym)
                        continue;
                    nd++;
                }
            }
        }
    *n_single = ns;
    *n_double = nd;
}

/* ------------------------------------------------------------------------ */
/* Main walker list: hash table with chaining + circular list of vacancies   */
/* (Sec. 4.2), hashed with Algorithm 1.                                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t cap, high;        /* storage size; one past the highest slot ever used */
    det_t *det;               /* 0 = vacant */
    int32_t *pop;
    double *hdiag;
    int64_t *next;            /* chain link */
    int64_t *head;            /* hash table: first slot of each chain, -1 if none */
    int64_t range;            /* hash-table size */
    int64_t *ring;            /* circular list of vacant slots */
    int64_t ring_head, ring_count;
    int64_t n_entries;
    int64_t map[MAX_SO];      /* Algorithm 1 random orbital map */
} mainlist_t;

static int64_t hash_alg1(const int64_t *map, const int32_t *occ, int n, int64_t range)
{
    uint64_t h = 0;
    for (int i = 1; i <= n; i++)
        h = 1099511628211ull * h + (uint64_t)map[occ[i - 1]] * (uint64_t)i;
    int64_t r = (int64_t)h % range;
    return r < 0 ? -r : r;
}

static int64_t ml_hash(const mainlist_t *ml, det_t det)
{
    int32_t occ[MAX_SO];
    int n = decode_det(det, occ);
    return hash_alg1(ml->map, occ, n, ml->range);
}

static uint64_t splitmix64(uint64_t *state)
{
    uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* A 1-to-1 map from spin orbitals to distinct random integers (Algorithm 1). */
static void make_map(int64_t map[MAX_SO], uint64_t seed)
{
    uint64_t st = seed;
    for (int r = 0; r < MAX_SO; r++) {
        for (;;) {
            int64_t v = (int64_t)(splitmix64(&st) >> 2);
            int dup = 0;
            for (int t = 0; t < r; t++)
                if (map[t] == v)
                    dup = 1;
            if (!dup && v != 0) {
                map[r] = v;
                break;
            }
        }
    }
}

static int ml_init(mainlist_t *ml, int64_t cap, int64_t range, uint64_t hash_seed)
{
    memset(ml, 0, sizeof *ml);
    ml->cap = cap;
    ml->range = range;
    ml->det = calloc((size_t)cap, sizeof(det_t));
    ml->pop = calloc((size_t)cap, sizeof(int32_t));
    ml->hdiag = calloc((size_t)cap, sizeof(double));
    ml->next = malloc((size_t)cap * sizeof(int64_t));
    ml->ring = malloc((size_t)cap * sizeof(int64_t));
    ml->head = malloc((size_t)range * sizeof(int64_t));
    if (!ml->det || !ml->pop || !ml->hdiag || !ml->next || !ml->ring || !ml->head)
        return fail("oracle: out of host memory");
    for (int64_t i = 0; i < range; i++)
        ml->head[i] = -1;
    make_map(ml->map, hash_seed);
    return 0;
}

static void ml_free(mainlist_t *ml)
{
    free(ml->det);
    free(ml->pop);
    free(ml->hdiag);
    free(ml->next);
    free(ml->ring);
    free(ml->head);
    memset(ml, 0, sizeof *ml);
}

static int64_t ml_find(const mainlist_t *ml, det_t det)
{
    int64_t h = ml_hash(ml, det);
    for (int64_t i = ml->head[h]; i >= 0; i = ml->next[i])
        if (ml->det[i] == det)
            return i;
    return -1;
}

static void ml_link(mainlist_t *ml, int64_t slot)
{
    int64_t h = ml_hash(ml, ml->det[slot]);
    ml->next[slot] = ml->head[h];
    ml->head[h] = slot;
}

static int ml_rehash(mainlist_t *ml, int64_t new_range)
{
    int64_t *nh = malloc((size_t)new_range * sizeof(int64_t));
    if (!nh)
        return fail("oracle: out of host memory");
    free(ml->head);
    ml->head = nh;
    ml->range = new_range;
    for (int64_t i = 0; i < new_range; i++)
        nh[i] = -1;
    for (int64_t i = 0; i < ml->high; i++)
        if (ml->det[i])
            ml_link(ml, i);
    return 0;
}

static int ml_grow(mainlist_t *ml)
{
    int64_t nc = ml->cap * 2;
    det_t *d = realloc(ml->det, (size_t)nc * sizeof(det_t));
    if (!d)
        return fail("oracle: out of host memory");
    ml->det = d;
    int32_t *p = realloc(ml->pop, (size_t)nc * sizeof(int32_t));
    if (!p)
        return fail("oracle: out of host memory");
    ml->pop = p;
    double *h = realloc(ml->hdiag, (size_t)nc * sizeof(double));
    if (!h)
        return fail("oracle: out of host memory");
    ml->hdiag = h;
    int64_t *n = realloc(ml->next, (size_t)nc * sizeof(int64_t));
    if (!n)
        return fail("oracle: out of host memory");
    ml->next = n;
    /* The ring is rebuilt in the larger buffer, keeping its order. */
    int64_t *r = malloc((size_t)nc * sizeof(int64_t));
    if (!r)
        return fail("oracle: out of host memory");
    for (int64_t i = 0; i < ml->ring_count; i++)
        r[i] = ml->ring[(ml->ring_head + i) % ml->cap];
    free(ml->ring);
    ml->ring = r;
    ml->ring_head = 0;
    for (int64_t i = ml->cap; i < nc; i++) {
        ml->det[i] = 0;
        ml->pop[i] = 0;
        ml->hdiag[i] = 0.0;
    }
    ml->cap = nc;
    return 0;
}

/* Insert into the earliest vacancy recorded in the circular list, else past the end. */
static int64_t ml_insert(mainlist_t *ml, det_t det, int32_t pop, double hd)
{
    int64_t slot;
    if (ml->ring_count > 0) {
        slot = ml->ring[ml->ring_head];
        ml->ring_head = (ml->ring_head + 1) % ml->cap;
        ml->ring_count--;
    } else {
        if (ml->high == ml->cap && ml_grow(ml) != 0)
            return -1;
        slot = ml->high++;
    }
    ml->det[slot] = det;
    ml->pop[slot] = pop;
    ml->hdiag[slot] = hd;
    ml_link(ml, slot);
    ml->n_entries++;
    if (ml->n_entries > 2 * ml->range && ml_rehash(ml, ml->range * 2) != 0)
        return -1;
    return slot;
}

static void ml_remove(mainlist_t *ml, int64_t slot)
{
    int64_t h = ml_hash(ml, ml->det[slot]);
    int64_t *link = &ml->head[h];
    while (*link != slot)
        link = &ml->next[*link];
    *link = ml->next[slot];
    ml->det[slot] = 0;
    ml->pop[slot] = 0;
    ml->ring[(ml->ring_head + ml->ring_count) % ml->cap] = slot;
    ml->ring_count++;
    ml->n_entries--;
}

/* ------------------------------------------------------------------------ */
/* Whole state.                                                              */
/* ------------------------------------------------------------------------ */
typedef struct {
    det_t det;
    int64_t pop;
    uint32_t flag;
} spawn_t;

/* One virtual process (Sec. 4.1): its part of the main list, the spawned
 * records it created, bucketed by destination process, and the records it
 * received in the exchange. */
typedef struct {
    mainlist_t ml;
    spawn_t **out;            /* out[q]: records created here for process q */
    int64_t *n_out, *cap_out;
    spawn_t *in;              /* records received from every process, sender order */
    int64_t n_in, cap_in;
    /* this process's share of the last iteration's statistics */
    int64_t attempts, merged, aborted, born, nw, nd, c0;
    double num;
    /* entries of a walker list being loaded that this process owns */
    int64_t *load_idx;
    int64_t n_load;
    char err[512];
} proc_t;

struct orc_state {
    sys_t sys;
    orc_params prm;
    int32_t n_procs, n_threads;
    proc_t *proc;
    const uint64_t *load_det;     /* walker list being loaded (during orc_load_walkers) */
    const int32_t *load_pop;
    int64_t pmap[MAX_SO];     /* Algorithm 1 map of the process hash */
    int W;                    /* 64-bit words per determinant in the API (1 or 2) */
    /* dynamics */
    int64_t iter;
    double shift;
    int varying;
    int64_t n_prev, n_var;
    /* last iteration's statistics */
    int64_t nw, nd, c0, attempts, spawns, merged, aborted, born, tot_attempts, tot_spawns;
    double num;
    /* series for the averages */
    double *s_num, *s_den, *s_shift;
    int64_t n_series, cap_series;
};

/* A determinant given in the API's W words (low word first), and back. */
static det_t det_in(const orc_state *st, const uint64_t *w)
{
    return det_make(w[0], st->W > 1 ? w[1] : 0);
}
static void det_out(const orc_state *st, det_t d, uint64_t *w)
{
    w[0] = det_lo(d);
    if (st->W > 1)
        w[1] = det_hi(d);
}
static det_t load_det_at(const orc_state *st, int64_t t)
{
    return det_in(st, st->load_det + t * st->W);
}

static int cmp_spawn(const void *a, const void *b)
{
    det_t x = ((const spawn_t *)a)->det, y = ((const spawn_t *)b)->det;
    return x < y ? -1 : (x > y ? 1 : 0);
}

static int push_rec(spawn_t **buf, int64_t *n, int64_t *cap, det_t det, int64_t pop,
                    uint32_t flag)
{
    if (*n == *cap) {
        int64_t nc = *cap ? *cap * 2 : 1024;
        spawn_t *p = realloc(*buf, (size_t)nc * sizeof(spawn_t));
        if (!p)
            return fail("oracle: out of host memory");
        *buf = p;
        *cap = nc;
    }
    (*buf)[*n].det = det;
    (*buf)[*n].pop = pop;
    (*buf)[*n].flag = flag;
    (*n)++;
    return 0;
}

/* Owning process of a determinant: the process hash of Sec. 4.1 (Algorithm 1
 * with its own map, over the range of processes); with a dedicated reference
 * process, the reference sits on process 0 and the rest hash over 1..P-1. */
static int owner_of(const orc_state *st, det_t det)
{
    if (st->n_procs == 1)
        return 0;
    int lo = 0;
    if (st->prm.ref_own_proc) {
        if (det == st->sys.d0)
            return 0;
        lo = 1;
    }
    int32_t occ[MAX_SO];
    int n = decode_det(det, occ);
    return lo + (int)hash_alg1(st->pmap, occ, n, st->n_procs - lo);
}

static int push_series(orc_state *st, double num, double den, double shift)
{
    if (st->n_series == st->cap_series) {
        int64_t nc = st->cap_series ? st->cap_series * 2 : 1024;
        double *a = realloc(st->s_num, (size_t)nc * sizeof(double));
        double *b = a ? realloc(st->s_den, (size_t)nc * sizeof(double)) : NULL;
        double *c = b ? realloc(st->s_shift, (size_t)nc * sizeof(double)) : NULL;
        if (a)
            st->s_num = a;
        if (b)
            st->s_den = b;
        if (c)
            st->s_shift = c;
        if (!a || !b || !c)
            return fail("oracle: out of host memory");
        st->cap_series = nc;
    }
    st->s_num[st->n_series] = num;
    st->s_den[st->n_series] = den;
    st->s_shift[st->n_series] = shift;
    st->n_series++;
    return 0;
}

static int sys_init(sys_t *s, const orc_ham *h)
{
    memset(s, 0, sizeof *s);
    if (h->n_orb <= 0 || 2 * h->n_orb > MAX_SO)
        return fail("oracle: need 1 <= n_orb <= 64");
    if (h->n_alpha < 0 || h->n_beta < 0 || h->n_alpha > h->n_orb || h->n_beta > h->n_orb ||
        h->n_alpha + h->n_beta == 0)
        return fail("oracle: bad electron counts");
    if (!h->h1 || !h->eri)
        return fail("oracle: missing integrals");
    s->M = h->n_orb;
    s->n_alpha = h->n_alpha;
    s->n_beta = h->n_beta;
    s->N = h->n_alpha + h->n_beta;
    s->n_so = 2 * h->n_orb;
    s->e_core = h->e_core;
    int64_t np = (int64_t)s->M * (s->M + 1) / 2;
    int64_t ne = np * (np + 1) / 2;
    s->h1 = malloc((size_t)s->M * s->M * sizeof(double));
    s->eri = malloc((size_t)ne * sizeof(double));
    if (!s->h1 || !s->eri)
        return fail("oracle: out of host memory");
    memcpy(s->h1, h->h1, (size_t)s->M * s->M * sizeof(double));
    memcpy(s->eri, h->eri, (size_t)ne * sizeof(double));
    int max_irrep = 0;
    for (int r = 0; r < s->M; r++) {
        s->irrep[r] = h->orb_irrep ? h->orb_irrep[r] : 0;
        if (s->irrep[r] > 7)
            return fail("oracle: irrep labels must be 0..7");
        if (s->irrep[r] > max_irrep)
            max_irrep = s->irrep[r];
    }
    s->n_class = 2 * (max_irrep + 1);
    for (int r = 0; r < s->n_so; r++)
        s->class_of[r] = class_id(s->irrep[r >> 1], r & 1);
    /* Reference determinant. */
    if (h->ref_det) {
        s->d0 = det_make(h->ref_det[0], s->n_so > 64 ? h->ref_det[1] : 0);
        uint64_t a = 0, b = 0;
        for (int r = 0; r < s->n_so; r++)
            if ((s->d0 >> r) & 1u) {
                if (r & 1)
                    b++;
                else
                    a++;
            }
        if ((s->n_so < MAX_SO && (s->d0 >> s->n_so) != 0) || (int)a != s->n_alpha ||
            (int)b != s->n_beta)
            return fail("oracle: reference determinant does not match the electron counts");
    } else {
        int order[MAX_ORB];
        for (int r = 0; r < s->M; r++)
            order[r] = r;
        for (int r = 1; r < s->M; r++) {          /* insertion sort by (h_pp, index) */
            int v = order[r], t = r;
            while (t > 0 && s->h1[order[t - 1] * s->M + order[t - 1]] > s->h1[v * s->M + v]) {
                order[t] = order[t - 1];
                t--;
            }
            order[t] = v;
        }
        s->d0 = 0;
        for (int r = 0; r < s->n_alpha; r++)
            s->d0 |= DBIT(2 * order[r]);
        for (int r = 0; r < s->n_beta; r++)
            s->d0 |= DBIT(2 * order[r] + 1);
    }
    s->e0 = hdiag_of(s, s->d0);
    if (h->p_double >= 0.0) {
        if (h->p_double > 1.0)
            return fail("oracle: p_double > 1");
        s->p_double = h->p_double;
    } else {
        int64_t ns, nd;
        count_excitations(s, s->d0, &ns, &nd);
        s->p_double = (ns + nd) > 0 ? (double)nd / (double)(ns + nd) : 0.0;
    }
    s->p_single = 1.0 - s->p_double;
    s->inv_p_double = s->p_double > 0.0 ? 1.0 / s->p_double : 0.0;
    s->inv_p_single = s->p_single > 0.0 ? 1.0 / s->p_single : 0.0;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Blocking analysis (Flyvbjerg & Petersen) of <num>/<den>, or of <num> when */
/* den is NULL. At each level neighbouring samples are averaged in pairs (a  */
/* trailing odd sample is dropped). The reported level is the first one     */
/* (with at least 16 blocks) whose error is not exceeded by the next two     */
/* levels by more than its own statistical uncertainty e/sqrt(2(n-1)).       */
/* ------------------------------------------------------------------------ */
int orc_blocking(const double *num, const double *den, int64_t n, double *mean_ratio,
                 double *err, int32_t *level)
{
    *mean_ratio = NAN;
    *err = NAN;
    *level = -1;
    if (n < 1)
        return 0;
    double sx = 0.0, sy = 0.0;
    for (int64_t t = 0; t < n; t++) {
        sx = sx + num[t];
        sy = sy + (den ? den[t] : 1.0);
    }
    *mean_ratio = den ? (sx / (double)n) / (sy / (double)n) : sx / (double)n;
    double *x = malloc((size_t)n * sizeof(double));
    double *y = malloc((size_t)n * sizeof(double));
    if (!x || !y) {
        free(x);
        free(y);
        return fail("oracle: out of host memory");
    }
    for (int64_t t = 0; t < n; t++) {
        x[t] = num[t];
        y[t] = den ? den[t] : 1.0;
    }
    double e_lv[64];
    int64_t n_lv[64];
    int nlev = 0;
    int64_t m = n;
    while (m >= 2 && nlev < 64) {
        double xm = 0.0, ym = 0.0;
        for (int64_t t = 0; t < m; t++) {
            xm = xm + x[t];
            ym = ym + y[t];
        }
        xm = xm / (double)m;
        ym = ym / (double)m;
        double vx = 0.0, vy = 0.0, cxy = 0.0;
        for (int64_t t = 0; t < m; t++) {
            vx = vx + (x[t] - xm) * (x[t] - xm);
            vy = vy + (y[t] - ym) * (y[t] - ym);
            cxy = cxy + (x[t] - xm) * (y[t] - ym);
        }
        double norm = (double)m * (double)(m - 1);
        vx = vx / norm;
        vy = vy / norm;
        cxy = cxy / norm;
        double var;
        if (den) {
            double r = xm / ym;
            var = r * r * (vx / (xm * xm) + vy / (ym * ym) - 2.0 * cxy / (xm * ym));
        } else {
            var = vx;
        }
        e_lv[nlev] = sqrt(var > 0.0 ? var : 0.0);
        n_lv[nlev] = m;
        nlev++;
        int64_t h = m / 2;
        for (int64_t t = 0; t < h; t++) {
            x[t] = (x[2 * t] + x[2 * t + 1]) * 0.5;
            y[t] = (y[2 * t] + y[2 * t + 1]) * 0.5;
        }
        m = h;
    }
    free(x);
    free(y);
    int chosen = -1, last_ok = -1;
    for (int l = 0; l < nlev; l++) {
        if (n_lv[l] < 16)
            break;
        last_ok = l;
        double tol = e_lv[l] + e_lv[l] / sqrt(2.0 * (double)(n_lv[l] - 1));
        int ok = 1;
        for (int k = 1; k <= 2; k++)
            if (l + k < nlev && n_lv[l + k] >= 16 && e_lv[l + k] > tol)
                ok = 0;
        if (ok) {
            chosen = l;
            break;
        }
    }
    if (chosen < 0)
        chosen = last_ok;
    if (chosen >= 0) {
        *err = e_lv[chosen];
        *level = chosen;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Run interface.                                                            */
/* ------------------------------------------------------------------------ */
static void procs_free(orc_state *st)
{
    if (!st->proc)
        return;
    for (int p = 0; p < st->n_procs; p++) {
        proc_t *pr = &st->proc[p];
        ml_free(&pr->ml);
        if (pr->out)
            for (int q = 0; q < st->n_procs; q++)
                free(pr->out[q]);
        free(pr->out);
        free(pr->n_out);
        free(pr->cap_out);
        free(pr->in);
        free(pr->load_idx);
    }
    free(st->proc);
    st->proc = NULL;
}

/* Empty main lists on every process, hashed over `range` buckets each. */
static int procs_init(orc_state *st, int64_t range)
{
    const int P = st->n_procs;
    uint64_t hs = st->prm.hash_seed ? st->prm.hash_seed : 0x5EED5EEDull;
    st->proc = calloc((size_t)P, sizeof(proc_t));
    if (!st->proc)
        return fail("oracle: out of host memory");
    for (int p = 0; p < P; p++) {
        proc_t *pr = &st->proc[p];
        pr->out = calloc((size_t)P, sizeof(spawn_t *));
        pr->n_out = calloc((size_t)P, sizeof(int64_t));
        pr->cap_out = calloc((size_t)P, sizeof(int64_t));
        if (!pr->out || !pr->n_out || !pr->cap_out)
            return fail("oracle: out of host memory");
        if (ml_init(&pr->ml, 1024, range, hs) != 0)
            return -1;
    }
    return 0;
}

/* Whether D lies in the restricted space of the run (Sec. 5: a child outside it is
 * treated as a null excitation). The excitation level counts the electrons of D
 * outside the reference's orbitals; the seniority counts the spatial orbitals that
 * hold exactly one electron. */
static det_t frozen_occ(const orc_params *prm)
{
    return det_make(prm->frozen_occupied, prm->frozen_occupied_hi);
}
static det_t frozen_emp(const orc_params *prm)
{
    return det_make(prm->frozen_empty, prm->frozen_empty_hi);
}

static int in_space(const orc_params *prm, det_t d0, det_t D)
{
    if ((prm->space & ORC_SPACE_EXCITATION) && popcount64(D & ~d0) > prm->max_excitation)
        return 0;
    if (prm->space & ORC_SPACE_SENIORITY) {
        int single = 0;
        for (int s = 0; s < MAX_ORB; s++)
            single += (int)(((D >> (2 * s)) & 1u) != ((D >> (2 * s + 1)) & 1u));
        if (single > prm->max_seniority)
            return 0;
    }
    if ((prm->space & ORC_SPACE_FROZEN) &&
        ((D & frozen_occ(prm)) != frozen_occ(prm) || (D & frozen_emp(prm))))
        return 0;
    return 1;
}

int orc_create(const orc_ham *ham, const orc_params *prm, orc_state **out)
{
    *out = NULL;
    if (!ham || !prm)
        return fail("oracle: null argument");
    if (!(prm->tau > 0.0))
        return fail("oracle: tau must be positive");
    if (prm->shift_every <= 0)
        return fail("oracle: shift_every must be positive");
    if (prm->n_procs < 0 || prm->n_procs > 4096 || prm->n_threads < 0)
        return fail("oracle: n_procs must be in 0..4096 and n_threads >= 0");
    if (prm->ref_own_proc && prm->n_procs < 2)
        return fail("oracle: a dedicated reference process needs n_procs >= 2");
    if (prm->space & ~(ORC_SPACE_EXCITATION | ORC_SPACE_SENIORITY | ORC_SPACE_FROZEN))
        return fail("oracle: unknown space restriction");
    if (((prm->space & ORC_SPACE_EXCITATION) && prm->max_excitation < 0) ||
        ((prm->space & ORC_SPACE_SENIORITY) && prm->max_seniority < 0) ||
        ((prm->space & ORC_SPACE_FROZEN) && (frozen_occ(prm) & frozen_emp(prm))))
        return fail("oracle: inconsistent space restriction");
    orc_state *st = calloc(1, sizeof *st);
    if (!st)
        return fail("oracle: out of host memory");
    if (sys_init(&st->sys, ham) != 0) {
        free(st->sys.h1);
        free(st->sys.eri);
        free(st);
        return -1;
    }
    st->prm = *prm;
    const char *why = NULL;
    st->W = st->sys.n_so > 64 ? 2 : 1;
    if (prm->det_words == 2)
        st->W = 2;
    else if (prm->det_words != 0 && !(prm->det_words == 1 && st->W == 1))
        why = "oracle: det_words must be 0, 1 (at most 64 spin orbitals) or 2";
    if (!in_space(prm, st->sys.d0, st->sys.d0))
        why = "oracle: the reference is outside the restricted space";
    if (prm->hphf) {
        /* spin-coupled functions of spin parity hphf (Sec. 5.3) */
        sys_t *s = &st->sys;
        if (prm->hphf != 1 && prm->hphf != -1)
            why = "oracle: hphf must be 0, 1 or -1";
        else if (s->n_alpha != s->n_beta)
            why = "oracle: spin-coupled functions need n_alpha = n_beta";
        else if (prm->space)
            why = "oracle: spin-coupled functions with a restricted space are not supported";
        s->hphf = prm->hphf;
        s->lam = ((s->N / 2) & 1) ? -prm->hphf : prm->hphf;
        s->d0 = hphf_rep(s->d0);
        if (!why && spin_flip(s->d0) == s->d0 && prm->hphf < 0)
            why = "oracle: a closed-shell reference has no odd-spin function";
        s->e0 = fdiag(s, s->d0);
    }
    if (why) {
        free(st->sys.h1);
        free(st->sys.eri);
        free(st);
        return fail(why);
    }
    st->n_procs = prm->n_procs > 0 ? prm->n_procs : 1;
    st->n_threads = prm->n_threads > 0 ? prm->n_threads : 1;
    make_map(st->pmap, prm->proc_seed ? prm->proc_seed : 0xD15781B7ull);
    int64_t range = prm->hash_range > 0 ? prm->hash_range : 1024;
    if (procs_init(st, range) != 0) {
        orc_free(st);
        return -1;
    }
    int64_t n0 = prm->n_init > 0 ? prm->n_init : 10;
    if (n0 > 2147483647) {
        orc_free(st);
        return fail("oracle: initial population exceeds int32");
    }
    ml_insert(&st->proc[owner_of(st, st->sys.d0)].ml, st->sys.d0, (int32_t)n0, st->sys.e0);
    st->shift = prm->shift0;
    st->nw = n0;
    st->nd = 1;
    st->c0 = n0;
    *out = st;
    return 0;
}

void orc_free(orc_state *st)
{
    if (!st)
        return;
    procs_free(st);
    free(st->sys.h1);
    free(st->sys.eri);
    free(st->s_num);
    free(st->s_den);
    free(st->s_shift);
    free(st);
}

static int is_initiator(const orc_state *st, det_t det, int32_t pop)
{
    int64_t a = pop < 0 ? -(int64_t)pop : pop;
    return a > st->prm.n_a || det == st->sys.d0;
}

/* First half of an iteration on process p: spawning from every walker of its
 * list and death on each of its determinants (Sec. 2). Spawned records go to
 * the block of the process that owns the child (Sec. 4.1). */
static int proc_spawn_death(orc_state *st, int p)
{
    const sys_t *s = &st->sys;
    const double tau = st->prm.tau;
    const int64_t it = st->iter;
    proc_t *pr = &st->proc[p];
    mainlist_t *ml = &pr->ml;
    for (int q = 0; q < st->n_procs; q++)
        pr->n_out[q] = 0;
    int64_t attempts = 0;
    detinfo_t di;

    int64_t high = ml->high;
    for (int64_t slot = 0; slot < high; slot++) {
        det_t D = ml->det[slot];
        if (!D)
            continue;
        int32_t C = ml->pop[slot];
        int64_t absC = C < 0 ? -(int64_t)C : C;
        if (absC == 0)
            continue;          /* only the reference can sit at zero */
        uint32_t flag = (uint32_t)is_initiator(st, D, C);
        det_setup(s, D, &di);
        for (int64_t k = 0; k < absC; k++) {
            uint32_t w[4];
            draw_words(st->prm.seed, D, (uint32_t)k, it, 0, w);
            excit_t ex;
            gen_excit(s, &di, w, &ex);
            attempts++;
            if (s->hphf && ex.det) {
                /* The target is the function holding the child (Sec. 5.3): generated
                 * from D only, it is reached through the child or through its
                 * spin-exchanged partner, so its generation probability is the sum
                 * of the two. The pair of D itself is part of the diagonal. */
                const det_t Dj = hphf_rep(ex.det), fx = spin_flip(ex.det);
                if (Dj == D || (spin_flip(Dj) == Dj && s->hphf < 0)) {
                    ex.det = 0;
                } else {
                    if (fx != ex.det)
                        ex.pgen = ex.pgen + pgen_of(s, &di, fx);
                    ex.hel = hphf_hel(s, D, Dj);
                    ex.det = Dj;
                }
            }
            if (!ex.det || ex.hel == 0.0 || !in_space(&st->prm, s->d0, ex.det))
                continue;
            /* The acceptance uniform is the type word's uniform rescaled within the
             * chosen type's interval: given the type it is uniform on [0, 1) and
             * independent of the orbital words. */
            double u = unit_uniform32(w[0]);
            double ua = u < s->p_double ? u * s->inv_p_double : (u - s->p_double) * s->inv_p_single;
            /* Eq. pspawn: integer part created deterministically, fraction stochastically. */
            double ps = (tau * fabs(ex.hel)) / ex.pgen;
            double fl = floor(ps);
            if (fl > 1073741824.0)
                return fail("oracle: spawn count overflow");
            int64_t m = (int64_t)fl + (ua < ps - fl ? 1 : 0);
            if (m == 0)
                continue;
            int64_t sgn = ((C > 0) ? 1 : -1) * (ex.hel > 0.0 ? 1 : -1);
            int q = owner_of(st, ex.det);
            if (push_rec(&pr->out[q], &pr->n_out[q], &pr->cap_out[q], ex.det, -sgn * m, flag) != 0)
                return -1;
        }
        /* Eq. pdeath, all walkers on the determinant at once. */
        uint64_t xd[2];
        draw_block(st->prm.seed, D, 0xFFFFFFFFu, it, 0x80, xd);
        double d = ((ml->hdiag[slot] - s->e0) - st->shift) * tau * (double)absC;
        double ad = fabs(d);
        double fl = floor(ad);
        if (fl > 1073741824.0)
            return fail("oracle: death count overflow");
        int64_t m = (int64_t)fl + (unit_uniform(xd[0]) < ad - fl ? 1 : 0);
        int64_t cnew = (int64_t)C - (C > 0 ? 1 : -1) * (d > 0.0 ? 1 : -1) * m;
        if (cnew > 2147483647 || cnew < -2147483647)
            return fail("oracle: population overflow");
        if (cnew == 0 && D != s->d0)
            ml_remove(ml, slot);
        else
            ml->pop[slot] = (int32_t)cnew;
    }
    pr->attempts = attempts;
    return 0;
}

/* This process's share of N_w, N_d, C_0 and the numerator of Eq. ProjE. */
static void proc_stats(orc_state *st, int q)
{
    const sys_t *s = &st->sys;
    proc_t *pr = &st->proc[q];
    const mainlist_t *ml = &pr->ml;
    int64_t nw = 0, nd = 0, c0 = 0;
    double num = 0.0;
    for (int64_t slot = 0; slot < ml->high; slot++) {
        det_t D = ml->det[slot];
        if (!D)
            continue;
        int32_t C = ml->pop[slot];
        if (D == s->d0)
            c0 = C;
        if (C == 0)
            continue;
        nw += C < 0 ? -(int64_t)C : C;
        nd++;
        if (D != s->d0)
            num = num + ref_hel(s, D) * (double)C;
    }
    pr->nw = nw;
    pr->nd = nd;
    pr->c0 = c0;
    pr->num = num;
}

/* Sum of the per-process shares, in process order. */
static void gather_stats(orc_state *st)
{
    st->nw = st->nd = st->c0 = 0;
    st->num = 0.0;
    for (int p = 0; p < st->n_procs; p++) {
        st->nw += st->proc[p].nw;
        st->nd += st->proc[p].nd;
        st->c0 += st->proc[p].c0;
        st->num = st->num + st->proc[p].num;
    }
}

/* Second half on process q: receive the blocks addressed to it (the
 * exchange of Sec. 4.1, a transpose of the per-destination blocks), sort and
 * compress them, annihilate against the local list with the initiator test
 * (Sec. 4.2), then this process's share of the estimators (Eq. ProjE). */
static int proc_annihilate(orc_state *st, int q)
{
    const sys_t *s = &st->sys;
    proc_t *pr = &st->proc[q];
    mainlist_t *ml = &pr->ml;
    pr->n_in = 0;
    for (int p = 0; p < st->n_procs; p++) {
        const proc_t *src = &st->proc[p];
        for (int64_t t = 0; t < src->n_out[q]; t++)
            if (push_rec(&pr->in, &pr->n_in, &pr->cap_in, src->out[q][t].det,
                         src->out[q][t].pop, src->out[q][t].flag) != 0)
                return -1;
    }

    /* Sort and compress (Sec. 4.1): sum signed walkers on each determinant,
     * OR the initiator flags, drop entries that cancel to zero. */
    qsort(pr->in, (size_t)pr->n_in, sizeof(spawn_t), cmp_spawn);
    int64_t merged = 0, aborted = 0, born = 0;
    int64_t i = 0;
    while (i < pr->n_in) {
        det_t D = pr->in[i].det;
        int64_t c = 0;
        uint32_t f = 0;
        while (i < pr->n_in && pr->in[i].det == D) {
            c += pr->in[i].pop;
            f |= pr->in[i].flag;
            i++;
        }
        if (c == 0)
            continue;
        merged++;
        /* Annihilation against the main list (Sec. 4.2). */
        int64_t slot = ml_find(ml, D);
        if (slot >= 0) {
            int64_t nv = (int64_t)ml->pop[slot] + c;
            if (nv > 2147483647 || nv < -2147483647)
                return fail("oracle: population overflow");
            if (nv == 0 && D != s->d0)
                ml_remove(ml, slot);
            else
                ml->pop[slot] = (int32_t)nv;
        } else if (f) {
            if (c > 2147483647 || c < -2147483647)
                return fail("oracle: population overflow");
            if (ml_insert(ml, D, (int32_t)c, fdiag(s, D)) < 0)
                return -1;
            born++;
        } else {
            aborted += c < 0 ? -c : c;
        }
    }
    pr->merged = merged;
    pr->aborted = aborted;
    pr->born = born;
    proc_stats(st, q);
    return 0;
}

typedef struct {
    orc_state *st;
    int phase, first, stride;
    int bad;                  /* lowest failing process, or -1 */
} job_t;

/* Insert the loaded entries this process owns, in input order, each with its
 * diagonal element; then this process's share of the statistics. */
static int proc_load(orc_state *st, int q)
{
    proc_t *pr = &st->proc[q];
    mainlist_t *ml = &pr->ml;
    for (int64_t u = 0; u < pr->n_load; u++) {
        const int64_t t = pr->load_idx[u];
        const det_t D = load_det_at(st, t);
        if (ml_find(ml, D) >= 0)
            return fail("oracle: duplicate determinant in walker list");
        if (ml_insert(ml, D, st->load_pop[t], fdiag(&st->sys, D)) < 0)
            return -1;
    }
    proc_stats(st, q);
    return 0;
}

static void *run_job(void *arg)
{
    job_t *j = arg;
    j->bad = -1;
    for (int p = j->first; p < j->st->n_procs; p += j->stride) {
        int rc = j->phase == 0   ? proc_spawn_death(j->st, p)
                 : j->phase == 1 ? proc_annihilate(j->st, p)
                                 : proc_load(j->st, p);
        if (rc != 0) {
            snprintf(j->st->proc[p].err, sizeof j->st->proc[p].err, "%s", g_err);
            j->bad = p;
            break;
        }
    }
    return NULL;
}

/* Run one phase on every process, spread round-robin over the host threads;
 * a failure is reported for the lowest failing process. */
static int run_phase(orc_state *st, int phase)
{
    int T = st->n_threads < st->n_procs ? st->n_threads : st->n_procs;
    job_t jobs[256];
    pthread_t th[256];
    if (T > 256)
        T = 256;
    int started = 1;
    for (int t = 0; t < T; t++) {
        jobs[t].st = st;
        jobs[t].phase = phase;
        jobs[t].first = t;
        jobs[t].stride = T;
        jobs[t].bad = -1;
    }
    for (int t = 1; t < T; t++) {
        if (pthread_create(&th[t], NULL, run_job, &jobs[t]) != 0)
            break;
        started++;
    }
    if (started < T) {
        /* Not enough threads: do the rest on this one. */
        for (int t = started; t < T; t++)
            run_job(&jobs[t]);
    }
    run_job(&jobs[0]);
    for (int t = 1; t < started; t++)
        pthread_join(th[t], NULL);
    int bad = -1;
    for (int t = 0; t < T; t++)
        if (jobs[t].bad >= 0 && (bad < 0 || jobs[t].bad < bad))
            bad = jobs[t].bad;
    if (bad >= 0)
        return fail(st->proc[bad].err);
    return 0;
}

/* One iteration in the paper's order: spawning from every walker, death on
 * each determinant, then the exchange, compression and annihilation of the
 * spawned list against the main list with the initiator test, then the
 * estimators and the shift. */
static int one_iteration(orc_state *st)
{
    const double tau = st->prm.tau;
    const int P = st->n_procs;
    if (run_phase(st, 0) != 0 || run_phase(st, 1) != 0)
        return -1;

    /* Statistics aggregation over processes, in process order. */
    int64_t attempts = 0, spawns = 0, merged = 0, aborted = 0, born = 0;
    for (int p = 0; p < P; p++) {
        const proc_t *pr = &st->proc[p];
        attempts += pr->attempts;
        for (int q = 0; q < P; q++)
            spawns += pr->n_out[q];
        merged += pr->merged;
        aborted += pr->aborted;
        born += pr->born;
    }
    gather_stats(st);
    const int64_t nw = st->nw, c0 = st->c0;
    const double num = st->num;
    st->attempts = attempts;
    st->spawns = spawns;
    st->merged = merged;
    st->aborted = aborted;
    st->born = born;
    st->tot_attempts += attempts;
    st->tot_spawns += spawns;
    st->iter++;

    /* Shift: held until the walker target is reached, then
     * S <- S - zeta/(A tau) ln(N_w / N_prev), both tested every A iterations. */
    const int A = st->prm.shift_every;
    if (st->iter % A == 0) {
        if (!st->varying) {
            if (nw >= st->prm.target) {
                st->varying = 1;
                st->n_prev = nw;
                st->n_var = st->iter;
            }
        } else {
            st->shift = st->shift - (st->prm.zeta / ((double)A * tau)) *
                                        orc_log((double)nw / (double)st->n_prev);
            st->n_prev = nw;
        }
    }
    if (st->varying && st->iter - st->n_var >= st->prm.avg_start)
        if (push_series(st, num, (double)c0, st->shift) != 0)
            return -1;
    return 0;
}

int orc_iterate(orc_state *st, int32_t n_iter)
{
    if (!st)
        return fail("oracle: null state");
    for (int32_t t = 0; t < n_iter; t++)
        if (one_iteration(st) != 0)
            return -1;
    return 0;
}

int orc_estimates(orc_state *st, orc_est *out)
{
    if (!st || !out)
        return fail("oracle: null argument");
    memset(out, 0, sizeof *out);
    out->iteration = st->iter;
    out->n_walkers = st->nw;
    out->n_dets = st->nd;
    out->ref_pop = st->c0;
    out->attempts = st->attempts;
    out->spawns = st->spawns;
    out->merged = st->merged;
    out->aborted = st->aborted;
    out->born = st->born;
    out->total_attempts = st->tot_attempts;
    out->total_spawns = st->tot_spawns;
    out->n_samples = st->n_series;
    out->n_var = st->n_var;
    out->n_prev = st->n_prev;
    out->shift = st->shift;
    out->e_ref = st->sys.e0;
    out->p_double = st->sys.p_double;
    out->proj_num = st->num;
    out->e_proj_inst = st->c0 != 0 ? st->sys.e0 + st->num / (double)st->c0 : NAN;
    out->shift_varying = st->varying;
    int32_t lvl;
    double r, e;
    orc_blocking(st->s_num, st->s_den, st->n_series, &r, &e, &lvl);
    out->e_proj_mean = st->sys.e0 + r;
    out->e_proj_err = e;
    orc_blocking(st->s_shift, NULL, st->n_series, &r, &e, &lvl);
    out->shift_mean = st->sys.e0 + r;
    out->shift_err = e;
    return 0;
}

int32_t orc_det_words(const orc_state *st) { return st ? st->W : -1; }

int64_t orc_walkers(orc_state *st, uint64_t *det, int32_t *pop, uint32_t *flags, int64_t cap)
{
    if (!st)
        return fail("oracle: null state");
    int64_t n = 0;
    for (int p = 0; p < st->n_procs; p++) {
        const mainlist_t *ml = &st->proc[p].ml;
        for (int64_t slot = 0; slot < ml->high; slot++)
            if (ml->det[slot] && ml->pop[slot] != 0)
                n++;
    }
    if (!det)
        return n;
    spawn_t *tmp = malloc((size_t)(n ? n : 1) * sizeof(spawn_t));
    if (!tmp)
        return fail("oracle: out of host memory");
    int64_t k = 0;
    for (int p = 0; p < st->n_procs; p++) {
        const mainlist_t *ml = &st->proc[p].ml;
        for (int64_t slot = 0; slot < ml->high; slot++)
            if (ml->det[slot] && ml->pop[slot] != 0) {
                tmp[k].det = ml->det[slot];
                tmp[k].pop = ml->pop[slot];
                tmp[k].flag = (uint32_t)is_initiator(st, ml->det[slot], ml->pop[slot]);
                k++;
            }
    }
    qsort(tmp, (size_t)n, sizeof(spawn_t), cmp_spawn);
    for (int64_t t = 0; t < n && t < cap; t++) {
        det_out(st, tmp[t].det, det + t * st->W);
        if (pop)
            pop[t] = (int32_t)tmp[t].pop;
        if (flags)
            flags[t] = tmp[t].flag;
    }
    free(tmp);
    return n;
}

int64_t orc_proc_dets(orc_state *st, int32_t p)
{
    if (!st || p < 0 || p >= st->n_procs)
        return fail("oracle: bad process index");
    return st->proc[p].ml.n_entries;
}

int32_t orc_owner(const orc_state *st, const uint64_t *det) { return owner_of(st, det_in(st, det)); }

int orc_load_walkers(orc_state *st, const uint64_t *det, const int32_t *pop, int64_t n,
                     int64_t iteration, double shift, int64_t n_prev, int32_t varying,
                     int64_t n_var)
{
    if (!st)
        return fail("oracle: null state");
    if (st->sys.hphf)
        for (int64_t t = 0; t < n; t++) {
            const det_t D = det_in(st, det + t * st->W);
            if (pop[t] != 0 && (hphf_rep(D) != D || (spin_flip(D) == D && st->sys.hphf < 0)))
                return fail("oracle: a walker list of spin-coupled functions holds each "
                            "function as the smaller determinant of its pair");
        }
    int64_t range = st->proc[0].ml.range;
    procs_free(st);
    if (procs_init(st, range) != 0)
        return -1;
    /* Bucket the entries by owning process (input order kept), then let every
     * process insert its own bucket. */
    const int P = st->n_procs;
    int have_ref = 0;
    int32_t *own = malloc((size_t)(n ? n : 1) * sizeof(int32_t));
    if (!own)
        return fail("oracle: out of host memory");
    for (int64_t t = 0; t < n; t++) {
        own[t] = -1;
        if (pop[t] == 0)
            continue;
        const det_t D = det_in(st, det + t * st->W);
        if (D == st->sys.d0)
            have_ref = 1;
        own[t] = owner_of(st, D);
        st->proc[own[t]].n_load++;
    }
    int rc = 0;
    for (int p = 0; p < P && rc == 0; p++) {
        st->proc[p].load_idx = malloc((size_t)(st->proc[p].n_load ? st->proc[p].n_load : 1) *
                                      sizeof(int64_t));
        if (!st->proc[p].load_idx)
            rc = fail("oracle: out of host memory");
        st->proc[p].n_load = 0;
    }
    if (rc == 0) {
        for (int64_t t = 0; t < n; t++)
            if (own[t] >= 0) {
                proc_t *pr = &st->proc[own[t]];
                pr->load_idx[pr->n_load++] = t;
            }
        if (!have_ref)
            rc = ml_insert(&st->proc[owner_of(st, st->sys.d0)].ml, st->sys.d0, 0, st->sys.e0) < 0
                     ? -1
                     : 0;
    }
    free(own);
    st->load_det = det;
    st->load_pop = pop;
    if (rc == 0)
        rc = run_phase(st, 2);
    st->load_det = NULL;
    st->load_pop = NULL;
    for (int p = 0; p < P; p++) {
        free(st->proc[p].load_idx);
        st->proc[p].load_idx = NULL;
        st->proc[p].n_load = 0;
    }
    if (rc != 0)
        return -1;
    st->iter = iteration;
    st->shift = shift;
    st->n_prev = n_prev;
    st->varying = varying;
    st->n_var = n_var;
    st->n_series = 0;
    gather_stats(st);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Unit-level entry points.                                                  */
/* ------------------------------------------------------------------------ */
int64_t orc_hash(const orc_state *st, const uint64_t *det, int64_t range)
{
    int32_t occ[MAX_SO];
    int n = decode_det(det_in(st, det), occ);
    return hash_alg1(st->proc[0].ml.map, occ, n, range);
}

double orc_hel(const orc_state *st, const uint64_t *bra, const uint64_t *ket)
{
    return hel_general(&st->sys, det_in(st, bra), det_in(st, ket));
}

double orc_hdiag(const orc_state *st, const uint64_t *det)
{
    return hdiag_of(&st->sys, det_in(st, det));
}

double orc_fn_hel(const orc_state *st, const uint64_t *bra_w, const uint64_t *ket_w)
{
    const det_t bra = det_in(st, bra_w), ket = det_in(st, ket_w);
    if (bra == ket)
        return fdiag(&st->sys, ket);
    return st->sys.hphf ? hphf_hel(&st->sys, ket, bra) : hel_general(&st->sys, bra, ket);
}

double orc_fn_diag(const orc_state *st, const uint64_t *fn)
{
    return fdiag(&st->sys, det_in(st, fn));
}

double orc_pgen(const orc_state *st, const uint64_t *det, const uint64_t *target)
{
    detinfo_t di;
    det_setup(&st->sys, det_in(st, det), &di);
    return pgen_of(&st->sys, &di, det_in(st, target));
}

double orc_proj_num(const orc_state *st, const uint64_t *det, const double *c, int64_t n)
{
    double num = 0.0;
    for (int64_t t = 0; t < n; t++) {
        const det_t D = det_in(st, det + t * st->W);
        if (D != st->sys.d0)
            num = num + ref_hel(&st->sys, D) * c[t];
    }
    return num;
}

int orc_sample_excitations(const orc_state *st, const uint64_t *det_w, int64_t iteration,
                           int64_t n_samples, uint64_t *out_det, double *out_pgen,
                           double *out_hel)
{
    detinfo_t di;
    const det_t det = det_in(st, det_w);
    det_setup(&st->sys, det, &di);
    for (int64_t k = 0; k < n_samples; k++) {
        uint32_t w[4];
        draw_words(st->prm.seed, det, (uint32_t)k, iteration, 0, w);
        excit_t ex;
        gen_excit(&st->sys, &di, w, &ex);
        det_out(st, ex.det, out_det + k * st->W);
        out_pgen[k] = ex.pgen;
        out_hel[k] = ex.hel;
    }
    return 0;
}
