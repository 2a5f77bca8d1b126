/*
 * Plain, sequential CPU oracle for the static two-level (FKS) hash map.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code with the HIP path: every
 * formula below is written out again here, from the paper and from the
 * published methods it names, so that the two can be compared.
 *
 * What it computes, and where each piece comes from:
 *   - Section 2.2 (the construction): g k = hash(const) k mod n, shape =
 *     squared level-one bucket sizes, offsets = exclusive prefix sum of the
 *     shape, h k = offsets[g k] + hash(consts[g k]) k mod shape[g k]; the
 *     well-formed and collision-free properties; the table arr of size s with
 *     every key at h k and the empty cells filled with a key of K; the value
 *     array indexed like arr; the membership test arr[h a] = a.
 *   - Section 2.3 (functional construction): make_1 draws the level-one
 *     constants, hashes every key mod n, takes the histogram of bucket sizes
 *     and maps make_2 over the keys grouped by bucket; make_2 draws constants
 *     until the bucket's hashes mod m^2 are collision free (histogram over
 *     m^2 cells, any count above one is a collision).
 *   - Figure 1 vocabulary: random, hash, hist, presum, groupby.
 *   - Section 3.1: a string key is a slice of a byte context; the map keeps a
 *     copy of the context of its own keys, the needle brings its own.
 *
 * Fixed readings where the paper leaves a choice open (each one is written
 * down in the design notes; the HIP path implements the same ones):
 *   R1 random: SplitMix64 (Steele, Lea, Flood 2014), counter based:
 *      out_sigma(i) = fin(sigma + (i+1)*gamma).  Attempt r of level one owns
 *      the 772 stream entries starting at r*772: (a0,a1,b) of level one at
 *      +0..+2, the string base at +3, level-two triple t at +4+3t..+6+3t.
 *      Every bucket uses the same level-two triple for its t-th trial.
 *   R2 hash: Thorup's vector multiply-shift with 32-bit input words and a
 *      64-bit accumulator: H(x) = ((a0*lo32(x) + a1*hi32(x) + b) mod 2^64)
 *      >> 32, a 32-bit value; "mod" is exact unsigned remainder.
 *   R3 presum is the exclusive prefix sum.
 *   R4 an attempt of level one is rejected when a bucket holds more than 15
 *      keys or when sum(s^2) > c*n; make_2 gives up after T trials; a bucket
 *      that gives up and holds two equal keys makes the build fail with the
 *      duplicate-key error, otherwise the level-one attempt is rejected.
 *      When every attempt is rejected the build fails with the duplicate-key
 *      error if two of its keys are equal (the precondition of
 *      from_array_nodup, Section 3.2: equal keys share every bucket and no
 *      trial separates them), else with the rejected-build error.
 *   R5 an empty cell copies the lowest occupied cell of its own bucket.
 *   R6 strings are fingerprinted by a Horner polynomial over 32-bit
 *      little-endian words modulo the Mersenne prime 2^61-1, seeded with the
 *      byte length; the FKS construction runs on the fingerprints and a hit
 *      is confirmed by comparing the bytes.
 *   R7 table layout: 16-byte header per group of eight buckets
 *      {u32 slot base of the group, u32 sizes (4 bits per bucket), u8 t[8]}
 *      and 16-byte cells {u64 key, u32 value, u32 aux}.
 *   R8 a bucket of one key always takes trial 0 (one key cannot collide), so
 *      its trial byte holds a tag of that key instead: the top 8 bits of its
 *      trial-0 level-two hash.  A lookup may answer "absent" when a needle's
 *      tag differs, without reading the cell; the membership test itself is
 *      unchanged.  Empty buckets keep 0.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_GAMMA 0x9E3779B97F4A7C15ULL
#define OR_STRIDE 772u          /* stream entries per level-one attempt */
#define OR_TMAX 256u
#define OR_SMAX 15u
#define OR_P61 ((1ULL << 61) - 1ULL)

enum { OR_OK = 0, OR_EINVAL = -1, OR_ENOMEM = -2, OR_EDUPKEY = -3, OR_EBUILD = -4 };
enum { OR_KIND_U64 = 0, OR_KIND_BYTES = 1, OR_KIND_U64V64 = 2 };

/* ---- R1: SplitMix64 ---------------------------------------------------- */

static uint64_t or_fin(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t oracle_splitmix(uint64_t sigma, uint64_t i)
{
    return or_fin(sigma + (i + 1ULL) * OR_GAMMA);
}

/* ---- R2: multiply-shift hash ------------------------------------------- */

uint32_t oracle_hash(uint64_t a0, uint64_t a1, uint64_t b, uint64_t x)
{
    uint64_t lo = x & 0xFFFFFFFFULL;
    uint64_t hi = x >> 32;
    uint64_t acc = a0 * lo + a1 * hi + b;       /* wraps mod 2^64 */
    return (uint32_t)(acc >> 32);
}

/* The constants of level-one attempt r: out[0..2] = (a0,a1,b), out[3] = beta. */
void oracle_level1_consts(uint64_t sigma, uint32_t r, uint64_t out[4])
{
    uint64_t base = (uint64_t)r * OR_STRIDE;
    out[0] = oracle_splitmix(sigma, base + 0);
    out[1] = oracle_splitmix(sigma, base + 1);
    out[2] = oracle_splitmix(sigma, base + 2);
    out[3] = 1ULL + oracle_splitmix(sigma, base + 3) % (OR_P61 - 1ULL);
}

/* Level-two triple number t of attempt r. */
void oracle_level2_consts(uint64_t sigma, uint32_t r, uint32_t t, uint64_t out[3])
{
    uint64_t base = (uint64_t)r * OR_STRIDE + 4ULL + 3ULL * t;
    out[0] = oracle_splitmix(sigma, base + 0);
    out[1] = oracle_splitmix(sigma, base + 1);
    out[2] = oracle_splitmix(sigma, base + 2);
}

/* ---- R8: tag of a one-key bucket ------------------------------------------ */

/* The top 8 bits of the key's trial-0 level-two hash (C points at the attempt's triples). */
static uint8_t or_tag(const uint64_t* C, uint64_t x)
{
    return (uint8_t)(oracle_hash(C[0], C[1], C[2], x) >> 24);
}

/* ---- R6: string fingerprint -------------------------------------------- */

uint64_t oracle_fingerprint(const uint8_t* s, uint64_t len, uint64_t beta)
{
    unsigned __int128 p = OR_P61;
    uint64_t acc = len % OR_P61;
    uint64_t nwords = (len + 3) / 4;
    for (uint64_t k = 0; k < nwords; ++k) {
        uint64_t w = 0;
        for (uint64_t q = 0; q < 4; ++q) {
            uint64_t at = 4 * k + q;
            if (at < len) w |= (uint64_t)s[at] << (8 * q);
        }
        unsigned __int128 t = (unsigned __int128)acc * beta + w;
        acc = (uint64_t)(t % p);
    }
    return acc;
}

/* ---- the map ------------------------------------------------------------ */

typedef struct {
    int kind;
    uint64_t n, S, sigma;
    uint32_t r, c, T, R;
    uint64_t a[3];            /* level-one triple of the accepted attempt */
    uint64_t beta;
    uint64_t* C;              /* T level-two triples, 3*T words */
    uint8_t* header;          /* 16 * ceil(n/8) bytes */
    uint8_t* slots;           /* 16 * S bytes */
    /* bytes maps keep a copy of their context (Section 3.1) */
    int64_t* ctx_off;         /* n+1 */
    uint8_t* ctx_bytes;
    uint64_t ctx_nbytes;
    /* statistics of the build, for tests */
    uint32_t attempts_rejected_size, attempts_rejected_space, attempts_rejected_exhausted;
    uint64_t level2_trials;   /* sum over buckets with s>=2 of (t+1) */
} oracle_map;

static void or_put_u32(uint8_t* p, uint32_t v) { memcpy(p, &v, 4); }
static void or_put_u64(uint8_t* p, uint64_t v) { memcpy(p, &v, 8); }
static uint32_t or_get_u32(const uint8_t* p) { uint32_t v; memcpy(&v, p, 4); return v; }
static uint64_t or_get_u64(const uint8_t* p) { uint64_t v; memcpy(&v, p, 8); return v; }

static int or_bytes_equal(const oracle_map* M, const int64_t* off, const uint8_t* bytes,
                          uint64_t i, uint64_t j)
{
    (void)M;
    int64_t li = off[i + 1] - off[i], lj = off[j + 1] - off[j];
    if (li != lj) return 0;
    return memcmp(bytes + off[i], bytes + off[j], (size_t)li) == 0;
}

/*
 * One run of make_1 for level-one attempt r.  Returns OR_OK when accepted,
 * 1 when the attempt is rejected, or an error code.
 *   keyv[i]: the integer the construction hashes (the key itself, or the
 *            string fingerprint under this attempt's beta).
 */
static int or_attempt(oracle_map* M, const uint64_t* keyv, const uint32_t* vals, const uint32_t* vals_hi,
                      const int64_t* off, const uint8_t* bytes, uint32_t r)
{
    uint64_t n = M->n;
    uint64_t c1[4];
    oracle_level1_consts(M->sigma, r, c1);

    /* hashes = map ((mod n) . hash const) keys */
    uint32_t* g = malloc(sizeof(uint32_t) * n);
    /* shape = hist n hashes (rep n 1) -- bucket sizes, squared below */
    uint64_t* shape = calloc(n, sizeof(uint64_t));
    if (!g || !shape) { free(g); free(shape); return OR_ENOMEM; }
    #pragma omp parallel for schedule(static)
    for (uint64_t i = 0; i < n; ++i)
        g[i] = oracle_hash(c1[0], c1[1], c1[2], keyv[i]) % (uint32_t)n;
    for (uint64_t i = 0; i < n; ++i) shape[g[i]] += 1;
    for (uint64_t j = 0; j < n; ++j) {
        if (shape[j] > OR_SMAX) {
            free(g); free(shape);
            M->attempts_rejected_size++;
            return 1;
        }
    }
    /* offsets = presum (map (^2) shape), exclusive */
    uint64_t* offsets = malloc(sizeof(uint64_t) * (n + 1));
    if (!offsets) { free(g); free(shape); return OR_ENOMEM; }
    uint64_t S = 0;
    for (uint64_t j = 0; j < n; ++j) { offsets[j] = S; S += shape[j] * shape[j]; }
    offsets[n] = S;
    if (S > (uint64_t)M->c * n) {
        free(g); free(shape); free(offsets);
        M->attempts_rejected_space++;
        return 1;
    }

    /* groupby n hashes keys: key indices of every bucket, in input order */
    uint64_t* gstart = malloc(sizeof(uint64_t) * (n + 1));
    uint64_t* gfill = malloc(sizeof(uint64_t) * n);
    uint64_t* members = malloc(sizeof(uint64_t) * n);
    if (!gstart || !gfill || !members) {
        free(g); free(shape); free(offsets); free(gstart); free(gfill); free(members);
        return OR_ENOMEM;
    }
    uint64_t acc = 0;
    for (uint64_t j = 0; j < n; ++j) { gstart[j] = acc; gfill[j] = acc; acc += shape[j]; }
    gstart[n] = acc;
    for (uint64_t i = 0; i < n; ++i) members[gfill[g[i]]++] = i;

    /* level-two constants of this attempt, shared by all buckets */
    uint64_t* C = malloc(sizeof(uint64_t) * 3 * M->T);
    uint8_t* tvals = calloc(n, 1);
    if (!C || !tvals) {
        free(g); free(shape); free(offsets); free(gstart); free(gfill); free(members);
        free(C); free(tvals);
        return OR_ENOMEM;
    }
    for (uint32_t t = 0; t < M->T; ++t) oracle_level2_consts(M->sigma, r, t, C + 3 * t);

    /* consts = map make_2 (groupby ...): smallest t whose hashes mod s^2
       have no collision (hist over s^2 cells, no count above one) */
    int exhausted = 0, dup = 0;
    uint64_t trials = 0;
    #pragma omp parallel for schedule(dynamic, 4096) reduction(|: exhausted, dup) reduction(+: trials)
    for (uint64_t j = 0; j < n; ++j) {
        uint64_t s = shape[j];
        if (s <= 1) { tvals[j] = 0; continue; }
        uint32_t m2 = (uint32_t)(s * s);
        uint8_t seen[OR_SMAX * OR_SMAX];
        int found = 0;
        for (uint32_t t = 0; t < M->T; ++t) {
            memset(seen, 0, m2);
            int collision = 0;
            for (uint64_t q = gstart[j]; q < gstart[j + 1]; ++q) {
                uint32_t h = oracle_hash(C[3 * t], C[3 * t + 1], C[3 * t + 2], keyv[members[q]]) % m2;
                if (seen[h]) collision = 1;
                seen[h] = 1;
            }
            if (!collision) { tvals[j] = (uint8_t)t; found = 1; trials += t + 1; break; }
        }
        if (!found) {
            exhausted = 1;
            /* does the bucket hold two equal keys? */
            for (uint64_t q1 = gstart[j]; q1 < gstart[j + 1]; ++q1)
                for (uint64_t q2 = q1 + 1; q2 < gstart[j + 1]; ++q2) {
                    uint64_t i1 = members[q1], i2 = members[q2];
                    if (M->kind != OR_KIND_BYTES) {
                        if (keyv[i1] == keyv[i2]) dup = 1;
                    } else if (or_bytes_equal(M, off, bytes, i1, i2)) {
                        dup = 1;
                    }
                }
        }
    }
    if (exhausted) {
        free(g); free(shape); free(offsets); free(gstart); free(gfill); free(members);
        free(C); free(tvals);
        if (dup) return OR_EDUPKEY;
        M->attempts_rejected_exhausted++;
        return 1;
    }

    /* accepted: materialise header and cells */
    uint64_t ngroups = (n + 7) / 8;
    uint8_t* header = calloc(ngroups ? ngroups : 1, 16);
    uint8_t* slots = calloc(S ? S : 1, 16);
    uint8_t* occupied = calloc(S ? S : 1, 1);
    if (!header || !slots || !occupied) {
        free(g); free(shape); free(offsets); free(gstart); free(gfill); free(members);
        free(C); free(tvals); free(header); free(slots); free(occupied);
        return OR_ENOMEM;
    }
    #pragma omp parallel for schedule(static)
    for (uint64_t gi = 0; gi < ngroups; ++gi) {
        uint32_t sizes = 0;
        for (uint32_t k = 0; k < 8; ++k) {
            uint64_t j = 8 * gi + k;
            if (j < n) {
                sizes |= (uint32_t)shape[j] << (4 * k);
                /* R8: a bucket of one key stores its key's tag where the trial would be */
                header[16 * gi + 8 + k] = shape[j] == 1 ? or_tag(C, keyv[members[gstart[j]]]) : tvals[j];
            }
        }
        or_put_u32(header + 16 * gi, (uint32_t)offsets[8 * gi]);
        or_put_u32(header + 16 * gi + 4, sizes);
    }
    /* every key at h k (each key has its own cell: the table is collision free) */
    #pragma omp parallel for schedule(static)
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t j = g[i];
        uint64_t s = shape[j];
        uint32_t t = tvals[j];
        uint32_t m2 = (uint32_t)(s * s);
        uint64_t p = offsets[j] + oracle_hash(C[3 * t], C[3 * t + 1], C[3 * t + 2], keyv[i]) % m2;
        uint8_t* cell = slots + 16 * p;
        or_put_u64(cell, keyv[i]);
        or_put_u32(cell + 8, vals[i]);
        /* aux: the key index of a string key, the high half of a 64-bit value */
        or_put_u32(cell + 12, M->kind == OR_KIND_BYTES ? (uint32_t)i : (vals_hi ? vals_hi[i] : 0u));
        occupied[p] = 1;
    }
    /* empty cells copy the lowest occupied cell of the same bucket */
    #pragma omp parallel for schedule(static)
    for (uint64_t j = 0; j < n; ++j) {
        if (shape[j] == 0) continue;
        uint64_t lo = offsets[j], hi = offsets[j + 1], first = hi;
        for (uint64_t p = lo; p < hi; ++p) if (occupied[p]) { first = p; break; }
        for (uint64_t p = lo; p < hi; ++p)
            if (!occupied[p]) memcpy(slots + 16 * p, slots + 16 * first, 16);
    }

    M->S = S;
    M->r = r;
    M->a[0] = c1[0]; M->a[1] = c1[1]; M->a[2] = c1[2];
    M->beta = c1[3];
    M->C = C;
    M->header = header;
    M->slots = slots;
    M->level2_trials = trials;
    free(g); free(shape); free(offsets); free(gstart); free(gfill); free(members);
    free(tvals); free(occupied);
    return OR_OK;
}

static int or_check_params(uint64_t n, uint32_t c, uint32_t T, uint32_t R)
{
    if (n >= (1ULL << 30)) return OR_EINVAL;
    if (c < 1 || c > 16 || T < 1 || T > OR_TMAX || R < 1 || R > 1024) return OR_EINVAL;
    if ((uint64_t)c * n >= (1ULL << 32)) return OR_EINVAL;
    return OR_OK;
}

/* ---- equal keys: the precondition of from_array_nodup (Section 3.2) -----
 * Plain definition: sort a copy and compare neighbours.  Strings are ordered
 * by length, then bytes. */

static int or_cmp_u64(const void* a, const void* b)
{
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

static int or_has_equal_u64(const uint64_t* keys, uint64_t n)
{
    uint64_t* k = malloc(sizeof(uint64_t) * (n ? n : 1));
    if (!k) return OR_ENOMEM;
    memcpy(k, keys, sizeof(uint64_t) * n);
    qsort(k, n, sizeof(uint64_t), or_cmp_u64);
    int eq = 0;
    for (uint64_t i = 1; i < n && !eq; ++i) eq = k[i] == k[i - 1];
    free(k);
    return eq;
}

static const int64_t* or_str_off;
static const uint8_t* or_str_bytes;

static int or_cmp_str(const void* a, const void* b)
{
    uint64_t i = *(const uint64_t*)a, j = *(const uint64_t*)b;
    int64_t li = or_str_off[i + 1] - or_str_off[i], lj = or_str_off[j + 1] - or_str_off[j];
    if (li != lj) return li < lj ? -1 : 1;
    return memcmp(or_str_bytes + or_str_off[i], or_str_bytes + or_str_off[j], (size_t)li);
}

static int or_has_equal_bytes(const int64_t* off, const uint8_t* bytes, uint64_t n)
{
    uint64_t* idx = malloc(sizeof(uint64_t) * (n ? n : 1));
    if (!idx) return OR_ENOMEM;
    for (uint64_t i = 0; i < n; ++i) idx[i] = i;
    or_str_off = off;
    or_str_bytes = bytes;
    qsort(idx, n, sizeof(uint64_t), or_cmp_str);
    int eq = 0;
    for (uint64_t k = 1; k < n && !eq; ++k) eq = or_cmp_str(&idx[k], &idx[k - 1]) == 0;
    free(idx);
    return eq;
}

/* the error of a build whose every attempt was rejected */
static int or_rejected(int equal)
{
    return equal < 0 ? equal : (equal ? OR_EDUPKEY : OR_EBUILD);
}

static oracle_map* or_new(int kind, uint64_t n, uint64_t sigma, uint32_t c, uint32_t T, uint32_t R)
{
    oracle_map* M = calloc(1, sizeof(oracle_map));
    if (!M) return NULL;
    M->kind = kind; M->n = n; M->sigma = sigma; M->c = c; M->T = T; M->R = R;
    return M;
}

void oracle_free(oracle_map* M)
{
    if (!M) return;
    free(M->C); free(M->header); free(M->slots); free(M->ctx_off); free(M->ctx_bytes);
    free(M);
}

static int or_empty_map(oracle_map* M)
{
    /* n = 0: no buckets, no cells; every lookup is absent */
    uint64_t c1[4];
    oracle_level1_consts(M->sigma, 0, c1);
    M->S = 0; M->r = 0;
    M->a[0] = c1[0]; M->a[1] = c1[1]; M->a[2] = c1[2]; M->beta = c1[3];
    M->C = calloc(3 * (size_t)M->T, sizeof(uint64_t));
    if (!M->C) return OR_ENOMEM;
    for (uint32_t t = 0; t < M->T; ++t) oracle_level2_consts(M->sigma, 0, t, M->C + 3 * t);
    return OR_OK;
}

int oracle_build_u64(const uint64_t* keys, const uint32_t* vals, uint64_t n, uint64_t sigma,
                     uint32_t c, uint32_t T, uint32_t R, oracle_map** out)
{
    int rc = or_check_params(n, c, T, R);
    if (rc) return rc;
    oracle_map* M = or_new(OR_KIND_U64, n, sigma, c, T, R);
    if (!M) return OR_ENOMEM;
    if (n == 0) {
        rc = or_empty_map(M);
        if (rc) { oracle_free(M); return rc; }
        *out = M;
        return OR_OK;
    }
    for (uint32_t r = 0; r < R; ++r) {
        rc = or_attempt(M, keys, vals, NULL, NULL, NULL, r);
        if (rc == OR_OK) { *out = M; return OR_OK; }
        if (rc < 0) { oracle_free(M); return rc; }
    }
    oracle_free(M);
    return or_rejected(or_has_equal_u64(keys, n));
}

/* 64-bit values (the paper's value type is polymorphic, Figure 2): the same
 * construction over the keys; a cell holds the value's low half where a 32-bit
 * map holds its value and the high half in its aux word. */
int oracle_build_u64_v64(const uint64_t* keys, const uint64_t* vals, uint64_t n, uint64_t sigma,
                         uint32_t c, uint32_t T, uint32_t R, oracle_map** out)
{
    int rc = or_check_params(n, c, T, R);
    if (rc) return rc;
    oracle_map* M = or_new(OR_KIND_U64V64, n, sigma, c, T, R);
    if (!M) return OR_ENOMEM;
    if (n == 0) {
        rc = or_empty_map(M);
        if (rc) { oracle_free(M); return rc; }
        *out = M;
        return OR_OK;
    }
    uint32_t* lo = malloc(sizeof(uint32_t) * n);
    uint32_t* hi = malloc(sizeof(uint32_t) * n);
    if (!lo || !hi) { free(lo); free(hi); oracle_free(M); return OR_ENOMEM; }
    for (uint64_t i = 0; i < n; ++i) {
        lo[i] = (uint32_t)vals[i];
        hi[i] = (uint32_t)(vals[i] >> 32);
    }
    for (uint32_t r = 0; r < R; ++r) {
        rc = or_attempt(M, keys, lo, hi, NULL, NULL, r);
        if (rc == OR_OK) break;
        if (rc < 0) break;
    }
    free(lo); free(hi);
    if (rc == OR_OK) { *out = M; return OR_OK; }
    oracle_free(M);
    return rc < 0 ? rc : or_rejected(or_has_equal_u64(keys, n));
}

int oracle_build_bytes(const int64_t* offsets, const uint8_t* bytes, const uint32_t* vals,
                       uint64_t n, uint64_t sigma, uint32_t c, uint32_t T, uint32_t R,
                       oracle_map** out)
{
    int rc = or_check_params(n, c, T, R);
    if (rc) return rc;
    if (offsets[0] < 0) return OR_EINVAL;
    for (uint64_t i = 0; i < n; ++i)
        if (offsets[i + 1] < offsets[i]) return OR_EINVAL;
    oracle_map* M = or_new(OR_KIND_BYTES, n, sigma, c, T, R);
    if (!M) return OR_ENOMEM;
    /* the map owns a copy of its context, rebased to start at 0 */
    uint64_t nbytes = (uint64_t)(offsets[n] - offsets[0]);
    M->ctx_off = malloc(sizeof(int64_t) * (n + 1));
    M->ctx_bytes = malloc(nbytes ? nbytes : 1);
    if (!M->ctx_off || !M->ctx_bytes) { oracle_free(M); return OR_ENOMEM; }
    for (uint64_t i = 0; i <= n; ++i) M->ctx_off[i] = offsets[i] - offsets[0];
    memcpy(M->ctx_bytes, bytes + offsets[0], nbytes);
    M->ctx_nbytes = nbytes;
    if (n == 0) {
        rc = or_empty_map(M);
        if (rc) { oracle_free(M); return rc; }
        *out = M;
        return OR_OK;
    }
    uint64_t* y = malloc(sizeof(uint64_t) * n);
    if (!y) { oracle_free(M); return OR_ENOMEM; }
    for (uint32_t r = 0; r < R; ++r) {
        uint64_t c1[4];
        oracle_level1_consts(sigma, r, c1);
        for (uint64_t i = 0; i < n; ++i)
            y[i] = oracle_fingerprint(M->ctx_bytes + M->ctx_off[i],
                                      (uint64_t)(M->ctx_off[i + 1] - M->ctx_off[i]), c1[3]);
        rc = or_attempt(M, y, vals, NULL, M->ctx_off, M->ctx_bytes, r);
        if (rc == OR_OK) { free(y); *out = M; return OR_OK; }
        if (rc < 0) { free(y); oracle_free(M); return rc; }
    }
    free(y);
    rc = or_rejected(or_has_equal_bytes(M->ctx_off, M->ctx_bytes, n));
    oracle_free(M);
    return rc;
}

/* ---- from_array: the constructor that tolerates duplicate keys ---------
 * Figure 2 gives from_array beside from_array_nodup without fixing which
 * value a repeated key keeps; reading: the value of its first occurrence
 * (lowest input index).  The distinct keys then go through from_array_nodup;
 * the table does not depend on their order. */

static const uint64_t* or_sort_keys;

static int or_cmp_key_index(const void* a, const void* b)
{
    uint64_t i = *(const uint64_t*)a, j = *(const uint64_t*)b;
    uint64_t ki = or_sort_keys[i], kj = or_sort_keys[j];
    if (ki != kj) return ki < kj ? -1 : 1;
    return i < j ? -1 : (i > j ? 1 : 0);
}

int oracle_build_u64_dedup(const uint64_t* keys, const uint32_t* vals, uint64_t u, uint64_t sigma,
                           uint32_t c, uint32_t T, uint32_t R, oracle_map** out)
{
    if (u >= (1ULL << 32)) return OR_EINVAL;
    uint64_t* idx = malloc(sizeof(uint64_t) * (u ? u : 1));
    uint64_t* dk = malloc(sizeof(uint64_t) * (u ? u : 1));
    uint32_t* dv = malloc(sizeof(uint32_t) * (u ? u : 1));
    if (!idx || !dk || !dv) { free(idx); free(dk); free(dv); return OR_ENOMEM; }
    for (uint64_t i = 0; i < u; ++i) idx[i] = i;
    or_sort_keys = keys;
    qsort(idx, u, sizeof(uint64_t), or_cmp_key_index);
    uint64_t n = 0;
    for (uint64_t k = 0; k < u; ++k) {
        if (k == 0 || keys[idx[k]] != keys[idx[k - 1]]) {
            dk[n] = keys[idx[k]];
            dv[n] = vals[idx[k]];
            ++n;
        }
    }
    int rc = oracle_build_u64(dk, dv, n, sigma, c, T, R, out);
    free(idx); free(dk); free(dv);
    return rc;
}

/* ---- lookup: the membership test of Section 2.2 over the built table ---- */

static int64_t or_probe(const oracle_map* M, uint64_t x)
{
    if (M->n == 0) return -1;
    uint32_t j = oracle_hash(M->a[0], M->a[1], M->a[2], x) % (uint32_t)M->n;
    const uint8_t* h = M->header + 16 * (uint64_t)(j / 8);
    uint32_t k = j % 8;
    uint32_t base = or_get_u32(h), sizes = or_get_u32(h + 4);
    uint32_t s = (sizes >> (4 * k)) & 15u;
    if (s == 0) return -1;
    uint64_t off = base;
    for (uint32_t i = 0; i < k; ++i) {
        uint32_t si = (sizes >> (4 * i)) & 15u;
        off += (uint64_t)si * si;
    }
    uint32_t t = s == 1 ? 0 : h[8 + k];   /* R8: a one-key bucket's byte is its tag; its trial is 0 */
    const uint64_t* C = M->C + 3 * (uint64_t)t;
    return (int64_t)(off + oracle_hash(C[0], C[1], C[2], x) % (s * s));
}

int oracle_lookup_u64(const oracle_map* M, const uint64_t* q, uint64_t m,
                      uint32_t* vals, uint8_t* found, uint32_t missing)
{
    if (M->kind != OR_KIND_U64) return OR_EINVAL;
    #pragma omp parallel for schedule(static)
    for (uint64_t i = 0; i < m; ++i) {
        int64_t p = or_probe(M, q[i]);
        int hit = p >= 0 && or_get_u64(M->slots + 16 * (uint64_t)p) == q[i];
        found[i] = (uint8_t)hit;
        vals[i] = hit ? or_get_u32(M->slots + 16 * (uint64_t)p + 8) : missing;
    }
    return OR_OK;
}

int oracle_lookup_u64_v64(const oracle_map* M, const uint64_t* q, uint64_t m,
                          uint64_t* vals, uint8_t* found, uint64_t missing)
{
    if (M->kind != OR_KIND_U64V64) return OR_EINVAL;
    #pragma omp parallel for schedule(static)
    for (uint64_t i = 0; i < m; ++i) {
        int64_t p = or_probe(M, q[i]);
        const uint8_t* cell = M->slots + 16 * (uint64_t)(p >= 0 ? p : 0);
        int hit = p >= 0 && or_get_u64(cell) == q[i];
        found[i] = (uint8_t)hit;
        vals[i] = hit ? ((uint64_t)or_get_u32(cell + 12) << 32) | or_get_u32(cell + 8) : missing;
    }
    return OR_OK;
}

int oracle_lookup_bytes(const oracle_map* M, const int64_t* qoff, const uint8_t* qbytes,
                        uint64_t m, uint32_t* vals, uint8_t* found, uint32_t missing)
{
    if (M->kind != OR_KIND_BYTES) return OR_EINVAL;
    #pragma omp parallel for schedule(static)
    for (uint64_t i = 0; i < m; ++i) {
        uint64_t len = (uint64_t)(qoff[i + 1] - qoff[i]);
        const uint8_t* s = qbytes + qoff[i];
        int hit = 0;
        uint32_t v = missing;
        if (M->n) {
            uint64_t y = oracle_fingerprint(s, len, M->beta);
            int64_t p = or_probe(M, y);
            if (p >= 0 && or_get_u64(M->slots + 16 * (uint64_t)p) == y) {
                uint32_t idx = or_get_u32(M->slots + 16 * (uint64_t)p + 12);
                uint64_t l2 = (uint64_t)(M->ctx_off[idx + 1] - M->ctx_off[idx]);
                if (l2 == len && memcmp(M->ctx_bytes + M->ctx_off[idx], s, len) == 0) {
                    hit = 1;
                    v = or_get_u32(M->slots + 16 * (uint64_t)p + 8);
                }
            }
        }
        found[i] = (uint8_t)hit;
        vals[i] = v;
    }
    return OR_OK;
}

/* ---- introspection ------------------------------------------------------ */

/* Threads the loops marked "omp parallel for" run on: this file built with OpenMP
   (the all-cores leg of the CPU baseline) runs those independent loops -- one key,
   one bucket, one group or one query per iteration, each writing only its own
   entries -- on every host core; the plain build runs every loop in order.  Both
   give the same bytes. */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* info[0..]: n, S, r, T, c, kind, beta, a0, a1, a2, rejected(size),
   rejected(space), rejected(exhausted), level-two trials */
void oracle_info(const oracle_map* M, uint64_t info[14])
{
    info[0] = M->n; info[1] = M->S; info[2] = M->r; info[3] = M->T; info[4] = M->c;
    info[5] = (uint64_t)M->kind; info[6] = M->beta;
    info[7] = M->a[0]; info[8] = M->a[1]; info[9] = M->a[2];
    info[10] = M->attempts_rejected_size; info[11] = M->attempts_rejected_space;
    info[12] = M->attempts_rejected_exhausted; info[13] = M->level2_trials;
}

void oracle_export(const oracle_map* M, uint8_t* header, uint8_t* slots)
{
    uint64_t ng = (M->n + 7) / 8;
    if (header && ng) memcpy(header, M->header, 16 * ng);
    if (slots && M->S) memcpy(slots, M->slots, 16 * M->S);
}

/* ---- batched build: independent maps, seed of map m = out_sigma(m) ----- */

uint64_t oracle_batch_seed(uint64_t batch_sigma, uint64_t m)
{
    return oracle_splitmix(batch_sigma, m);
}
