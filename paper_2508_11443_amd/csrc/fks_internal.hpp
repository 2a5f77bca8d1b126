// Internal definitions of the FKS library: device arithmetic, table records,
// the map object and small host helpers.  Everything here is written for
// gfx950 (CDNA4): wave64, 64 KiB-per-workgroup LDS budget, 32-bit multiply
// pieces for 64-bit products.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fks.h"

namespace fks {

// ---- fixed readings of the construction -----------------------------------
// Stream entries reserved per level-one attempt: (a0, a1, b), the string base,
// and 256 level-two triples.
constexpr uint32_t kStride = 772;
constexpr uint32_t kTMax = 256;
constexpr uint32_t kSMax = 15;            // largest accepted bucket (4-bit size field)
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kP61 = (1ull << 61) - 1;

struct Triple {
    uint64_t a0, a1, b;
};

// 16-byte header record of a group of 8 buckets.
struct alignas(16) Group {
    uint32_t base;    // first cell of the group
    uint32_t sizes;   // 4 bits per bucket
    uint32_t t_lo;    // trial index of buckets 0..3 (one byte each; a one-key bucket's byte is its key's tag)
    uint32_t t_hi;    // the same for buckets 4..7
};

// 16-byte cell.
// four dwords: the unit of the 16-byte streaming loads and stores of cells and group records
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

struct alignas(16) Cell {
    uint64_t key;
    uint32_t val;
    uint32_t aux;
};

// A cell touched once by a kernel (a lookup's probe, a pass over the table): a streaming
// (non-temporal) access, which leaves the caches to data that is read again.
__device__ __forceinline__ Cell load_cell_once(const Cell* p) {
    const u32x4 w = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
    return Cell{(uint64_t)w.x | ((uint64_t)w.y << 32), w.z, w.w};
}
__device__ __forceinline__ void store_cell_once(Cell* p, const Cell& c) {
    const u32x4 w = {(uint32_t)c.key, (uint32_t)(c.key >> 32), c.val, c.aux};
    __builtin_nontemporal_store(w, reinterpret_cast<u32x4*>(p));
}

// ---- SplitMix64 (Steele, Lea & Flood 2014), counter based --------------------
__host__ __device__ inline uint64_t sm_fin(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__host__ __device__ inline uint64_t sm_out(uint64_t sigma, uint64_t i) {
    return sm_fin(sigma + (i + 1) * kGamma);
}
__host__ __device__ inline Triple level1_triple(uint64_t sigma, uint32_t r) {
    uint64_t b = (uint64_t)r * kStride;
    return Triple{sm_out(sigma, b), sm_out(sigma, b + 1), sm_out(sigma, b + 2)};
}
__host__ __device__ inline uint64_t level1_beta(uint64_t sigma, uint32_t r) {
    return 1 + sm_out(sigma, (uint64_t)r * kStride + 3) % (kP61 - 1);
}
__host__ __device__ inline Triple level2_triple(uint64_t sigma, uint32_t r, uint32_t t) {
    uint64_t b = (uint64_t)r * kStride + 4 + 3ull * t;
    return Triple{sm_out(sigma, b), sm_out(sigma, b + 1), sm_out(sigma, b + 2)};
}

// ---- Thorup's vector multiply-shift, w = 32, 64-bit accumulator -------------
// ((a0*lo + a1*hi + b) mod 2^64) >> 32, written as two 32x32+64 multiply-adds
// and two 32-bit low multiplies for the upper halves of a0 and a1.
__host__ __device__ inline uint32_t mshash(uint64_t a0, uint64_t a1, uint64_t b, uint64_t x) {
    uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    uint64_t t = (uint64_t)(uint32_t)a0 * lo + b;
    t = (uint64_t)(uint32_t)a1 * hi + t;
    return (uint32_t)(t >> 32) + (uint32_t)(a0 >> 32) * lo + (uint32_t)(a1 >> 32) * hi;
}
__host__ __device__ inline uint32_t mshash(const Triple& c, uint64_t x) {
    return mshash(c.a0, c.a1, c.b, x);
}

// ---- exact 32-bit remainder by a runtime divisor ------------------------------
// Lemire, Kaser & Kurz, "Faster remainder by direct computation" (2019):
// with M = floor((2^64-1)/d) + 1, a mod d = ((M*a mod 2^64) * d) >> 64 for every
// 32-bit a and d >= 1.
__host__ __device__ inline uint64_t fastmod_magic(uint32_t d) {
    return 0xFFFFFFFFFFFFFFFFull / d + 1;
}
__host__ __device__ inline uint32_t fastmod(uint32_t a, uint64_t M, uint32_t d) {
    uint64_t low = (uint64_t)(uint32_t)M * a;
    low += (uint64_t)((uint32_t)(M >> 32) * a) << 32;
    // high 64 bits of the 96-bit product low * d
    uint64_t mid = (uint64_t)(uint32_t)(low >> 32) * d + (uint32_t)(((uint64_t)(uint32_t)low * d) >> 32);
    return (uint32_t)(mid >> 32);
}

// ---- string fingerprint: Horner over 32-bit words mod 2^61-1 ----------------
__host__ __device__ inline uint64_t mulmod61(uint64_t a, uint64_t b) {
    // a, b < 2^61: the 122-bit product folded twice (2^61 == 1 mod p)
#if defined(__HIP_DEVICE_COMPILE__)
    uint64_t lo = a * b;
    uint64_t hi = __umul64hi(a, b);
#else
    unsigned __int128 p = (unsigned __int128)a * b;
    uint64_t lo = (uint64_t)p, hi = (uint64_t)(p >> 64);
#endif
    uint64_t r = (lo & kP61) + ((lo >> 61) | (hi << 3));
    r = (r & kP61) + (r >> 61);
    return r >= kP61 ? r - kP61 : r;
}
__host__ __device__ inline uint64_t addmod61(uint64_t a, uint64_t w) {
    uint64_t r = a + w;            // a < 2^61, w < 2^32: no overflow
    r = (r & kP61) + (r >> 61);
    return r >= kP61 ? r - kP61 : r;
}

// Bytes s[0..len), len <= 4*W, as W little-endian 32-bit words, zero past len.  They are
// read as the aligned dwords that cover the range and shifted into place (v_alignbyte):
// one round of independent loads instead of one load per byte.  Every dword read holds
// at least one byte of the range, so no read touches a page the range does not touch.
template <int W>
__device__ __forceinline__ void load_words(const uint8_t* s, uint32_t len, uint32_t (&w)[W]) {
    const uintptr_t at = (uintptr_t)s;
    const uint32_t* p = (const uint32_t*)(at & ~(uintptr_t)3);
    const uint32_t sh = (uint32_t)(at & 3);
    const uint32_t nraw = len ? (sh + len + 3) >> 2 : 0;
    uint32_t raw[W + 1];
#pragma unroll
    for (int k = 0; k <= W; ++k) raw[k] = (uint32_t)k < nraw ? p[k] : 0u;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const uint32_t v = __builtin_amdgcn_alignbyte(raw[k + 1], raw[k], sh);
        const int rem = (int)len - 4 * k;   // bytes of the range in word k
        w[k] = rem >= 4 ? v : rem <= 0 ? 0u : v & ((1u << (8 * rem)) - 1u);
    }
}

constexpr int kChunkWords = 16;   // strings are read 64 bytes at a time

// Horner step over the words of one chunk of c bytes (c <= 64)
__device__ __forceinline__ uint64_t horner_words(uint64_t acc, const uint32_t (&w)[kChunkWords], uint32_t c,
                                                 uint64_t beta) {
    const uint32_t nw = (c + 3) >> 2;
#pragma unroll
    for (int k = 0; k < kChunkWords; ++k)
        if ((uint32_t)k < nw) acc = addmod61(mulmod61(acc, beta), w[k]);
    return acc;
}

// Fingerprint of s[0..len): len mod p, then one Horner step per 32-bit word (the last one
// zero-padded).  For len <= 64, w holds the string's words on return.
__device__ __forceinline__ uint64_t fingerprint_words(const uint8_t* s, uint64_t len, uint64_t beta,
                                                      uint32_t (&w)[kChunkWords]) {
    uint64_t acc = len % kP61;
    for (uint64_t done = 0; done < len; done += 4 * kChunkWords) {
        const uint32_t c = (uint32_t)(len - done < 4 * kChunkWords ? len - done : 4 * kChunkWords);
        load_words<kChunkWords>(s + done, c, w);
        acc = horner_words(acc, w, c, beta);
    }
    if (len == 0) {
#pragma unroll
        for (int k = 0; k < kChunkWords; ++k) w[k] = 0u;
    }
    return acc;
}

// a[0..len) == b[0..len), 64 bytes at a time
__device__ __forceinline__ bool bytes_equal(const uint8_t* a, const uint8_t* b, uint64_t len) {
    bool eq = true;
    for (uint64_t done = 0; done < len && eq; done += 4 * kChunkWords) {
        const uint32_t c = (uint32_t)(len - done < 4 * kChunkWords ? len - done : 4 * kChunkWords);
        uint32_t u[kChunkWords], v[kChunkWords];
        load_words<kChunkWords>(a + done, c, u);
        load_words<kChunkWords>(b + done, c, v);
        uint32_t diff = 0;
#pragma unroll
        for (int k = 0; k < kChunkWords; ++k) diff |= u[k] ^ v[k];
        eq = diff == 0;
    }
    return eq;
}

// ---- header helpers ---------------------------------------------------------
__host__ __device__ inline uint32_t nib(uint32_t sizes, uint32_t k) {
    return (sizes >> (4 * k)) & 15u;
}
// sum of squared sizes of buckets 0..k-1 of a group
__host__ __device__ inline uint32_t prefix_sq(uint32_t sizes, uint32_t k) {
    const uint32_t v = sizes & ((k == 0) ? 0u : (0xFFFFFFFFu >> (32 - 4 * k)));
#if defined(__HIP_DEVICE_COMPILE__)
    // the even and the odd nibbles, one per byte, each squared and summed by a
    // 4-way byte dot product
    const uint32_t e = v & 0x0F0F0F0Fu, o = (v >> 4) & 0x0F0F0F0Fu;
    return __builtin_amdgcn_udot4(e, e, __builtin_amdgcn_udot4(o, o, 0u, false), false);
#else
    uint32_t acc = 0;
    for (uint32_t i = 0; i < 8; ++i) acc += nib(v, i) * nib(v, i);
    return acc;
#endif
}
__host__ __device__ inline uint32_t prefix_cnt(uint32_t sizes, uint32_t k) {
    // keep the nibbles below bucket k, then add them up pairwise
    uint32_t m = (k == 0) ? 0u : (0xFFFFFFFFu >> (32 - 4 * k));
    uint32_t v = sizes & m;
    v = (v & 0x0F0F0F0Fu) + ((v >> 4) & 0x0F0F0F0Fu);
    v = v + (v >> 8);
    v = v + (v >> 16);
    return v & 0xFFu;
}
__host__ __device__ inline uint32_t group_t(const Group& g, uint32_t k) {
    uint32_t w = k < 4 ? g.t_lo : g.t_hi;
    return (w >> (8 * (k & 3))) & 0xFFu;
}

// A bucket of one key always takes trial 0, so its trial byte holds a tag of that key
// instead: the top 8 bits of the key's trial-0 level-two hash (c0 = the first triple).
__host__ __device__ inline uint32_t tag_of(uint32_t h0) { return h0 >> 24; }   // h0: the trial-0 hash
__host__ __device__ inline uint32_t key_tag(const Triple& c0, uint64_t x) { return tag_of(mshash(c0, x)); }

// The cell needle x would occupy in bucket k of group record h, with the level-two
// triples C of the map.  False when x cannot be in the bucket: the bucket is empty, or it
// holds one key whose tag differs from x's (no cell is read then).  A true result still
// needs the key comparison of the membership test.
__host__ __device__ inline bool cell_of(const Group& h, uint32_t k, const Triple* C, uint64_t x, uint32_t& cell) {
    const uint32_t s = nib(h.sizes, k);
    if (s == 0) return false;
    const uint32_t tb = group_t(h, k);
    const uint32_t hv = mshash(C[s == 1 ? 0u : tb], x);
    if (s == 1 && (hv >> 24) != tb) return false;
    cell = h.base + prefix_sq(h.sizes, k) + (s == 1 ? 0u : hv % (s * s));
    return true;
}

}  // namespace fks

// ---- the map object (host side) ---------------------------------------------
struct fks_map {
    uint32_t kind;        // 0 u64, 1 bytes
    int device;
    uint64_t n, S, seed;
    uint32_t r, c, T, R, max_t;
    fks::Triple A;        // level-one triple of the accepted attempt
    uint64_t beta;        // string base of the accepted attempt
    uint64_t magic_n;     // fastmod magic of n
    fks::Group* header;   // ceil(n/8)
    fks::Cell* slots;     // S
    fks::Triple* C;       // T level-two triples (device)
    int64_t* ctx_off;     // bytes maps: copy of the offsets (n+1)
    uint8_t* ctx_bytes;   // bytes maps: copy of the context
    uint64_t ctx_nbytes;
    uint64_t device_bytes;
    fks_allocator alloc;  // where the map's memory came from (has_alloc == 0: the default pool)
    int has_alloc;
};

namespace fks {

// error bookkeeping
void set_hip_error(hipError_t e);
int hip_fail(hipError_t e);

// Device memory.  dev_alloc / dev_free go to the allocator of the innermost
// AllocScope on the calling thread: a caller's fks_allocator, or (none, or NULL)
// stream-ordered allocations from the device's default pool, which keeps freed
// blocks cached for the next build.  Every entry point that allocates opens a
// scope with the caller's allocator (or, to release an object, the allocator
// the object was built with), so all of a call's memory comes from one place.
void* dev_alloc(size_t bytes, hipStream_t s);
void dev_free(void* p, hipStream_t s);
// the current call allocates from the device's default pool (hipMallocAsync / hipFreeAsync),
// whose stream-ordered release may be issued while queued work still uses the memory
bool dev_pool_default();
class AllocScope {
  public:
    explicit AllocScope(const fks_allocator* a);
    ~AllocScope();
    AllocScope(const AllocScope&) = delete;
    AllocScope& operator=(const AllocScope&) = delete;

  private:
    const fks_allocator* prev_;
};
// a caller's allocator is usable: NULL, or both functions set
inline bool allocator_ok(const fks_allocator* a) { return !a || (a->alloc && a->free); }
// keep a copy of the caller's allocator in a built object
inline void keep_allocator(const fks_allocator* a, fks_allocator& dst, int& has) {
    has = a ? 1 : 0;
    dst = a ? *a : fks_allocator{nullptr, nullptr, nullptr};
}

// hist[s] = buckets of size s among the first n buckets of the G group records at
// `header` (the sizes of make_1); synchronous on the null stream
int size_histogram(const Group* header, uint64_t n, uint64_t hist[16]);

// *equal = whether keys[0..n) hold two equal entries; for string keys, `keys` are the
// strings' fingerprints under one base and off/bytes the strings (else both nullptr).
// Asked only when every level-one attempt of a build was rejected.  Synchronises `st`.
int has_equal_keys(const uint64_t* keys, uint64_t n, const int64_t* off, const uint8_t* bytes, hipStream_t st,
                   bool* equal);

// pinned host staging for the small readbacks of a build
struct Readback {
    uint64_t S;          // sum of squared sizes of the attempt
    uint32_t oversize;   // some bucket holds more than 15 keys
    uint32_t bad_input;  // string offsets not monotone / out of range
    uint32_t exhausted;  // some bucket ran out of level-two trials
    uint32_t dup;        // an exhausted bucket holds two equal keys
    uint32_t max_t;
    uint32_t stalled;    // the fused final pass could not resolve a partition's first cell
    uint32_t overflow;   // a fixed-capacity region of the cursor passes overflowed
    uint32_t pad;
};

}  // namespace fks

#define FKS_HIP(call)                                   \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return fks::hip_fail(e_); \
    } while (0)
