// Partitioned level-one attempt (partition.hip): plan, buffers, entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fks_internal.hpp"

namespace fks {

constexpr uint32_t kPartBits = 10;                   // 1024 buckets per partition
constexpr uint32_t kPartBuckets = 1u << kPartBits;

// A map of a batch built by the partition passes instead of a single workgroup
// ("wide" map, at most 65536 keys, so at most kSegParts partitions).  Global
// partition index = segment * kSegParts + partition within the map.
constexpr uint32_t kSegParts = 64;
struct WideSeg {
    Triple A;            // level-one triple of attempt 0
    uint64_t magic;      // remainder magic of n
    uint64_t in_lo, in_hi;   // the map's keys in the batch input
    uint64_t hdr_off;    // first group record of the map in the header pool
    uint64_t slot_off;   // first cell of the map in the cell pool
    uint32_t n, G;       // keys, groups of eight buckets
    uint32_t map;        // index of the map in the batch
    uint32_t c;          // space factor: the attempt fails when the map's cells exceed c*n
};

// Radix passes over the partition index q (bits_q bits), at most 8 bits (256 bins) each:
// one pass up to 2^8 partitions, two up to 2^16, three beyond (n < 2^30 gives q < 2^20).
struct PartPlan {
    uint32_t Q;        // partitions
    uint32_t bits_q;   // ceil(log2 Q)
    uint32_t passes;   // scatter passes: 0, 1, 2 or 3
    uint32_t shiftA;   // first-level bin = q >> shiftA
    uint32_t binsA;    // first-level bins
    uint32_t bitsB;    // two passes: second-level bin = q & (2^bitsB - 1); three: (q >> bitsC) & 255
    uint32_t binsAB;   // three passes: bins after the second pass (q >> bitsC)
    uint32_t bitsC;    // three passes: third-level bin = q & (2^bitsC - 1)
    uint32_t W1, W2, W3;   // workers of the first pass / per bin of the second and third passes
    uint64_t matrix;   // entries of the largest count matrix
    // two passes with cursors: capacity of a first-level bin's region and of a partition's
    uint64_t cap1, capQ;
};

// Inputs, scratch and outputs of one attempt (device pointers).
struct PartArgs {
    uint64_t n, G;
    bool aux;                   // an aux word travels with every key
    bool str;                   // keys are string fingerprints
    const uint32_t* aux_in;     // the input's aux words, or nullptr for the key index
    Triple A;
    uint64_t magic;
    const uint64_t* keys;       // the integers the construction hashes
    const uint32_t* vals;
    // scratch
    uint64_t *k1, *k2;          // partitioned keys after pass 1 / pass 2
    uint32_t *v1, *v2;          // values
    uint32_t *a1, *a2;          // string indices (string maps)
    uint32_t* cnt;              // per-worker bin counts (plan.matrix entries)
    uint32_t* off;              // their exclusive scan
    uint32_t* tsum;             // scan tile sums
    uint64_t* tpre;             // scanned tile sums
    uint64_t* offA;             // 257 first-level bin offsets
    uint64_t* offAB;            // three passes: binsAB+1 second-level bin offsets
    uint64_t* offQ;             // Q+1 partition offsets
    uint32_t* sqQ;              // Q sums of squared sizes
    uint64_t* cbase;            // Q+1 cell bases
    uint32_t* sizes;            // G size words (the headers' second word)
    uint64_t* S_dev;            // total cells
    uint32_t* oversize;         // a bucket above 15 keys
    uint32_t* stalled;          // fused final pass: a look-back gave up
    bool fused;                 // the final pass sizes the partitions itself (no size pass and scan)
    // two passes without count passes: each tile reserves its runs on per-bin cursors in
    // fixed-capacity regions (k1/v1/a1 hold binsA * cap1 records, k2/v2/a2 Q * capQ)
    bool cursor;
    unsigned long long* cur1;   // binsA first-level cursors
    unsigned long long* cur2;   // Q partition cursors: each partition's end
    uint64_t* begA;             // binsA region starts
    uint64_t* begQ;             // Q partition starts
    uint32_t* overflow;         // a region overflowed: the attempt is redone with counts
};

struct PartOut {
    PartPlan plan;
    const uint64_t* keys;       // records in partition order
    const uint32_t* vals;
    const uint32_t* aux;
    int aux_is_pos;
    const uint64_t* qbeg;       // partition q's records are [qbeg[q], min(qend[q], qbeg[q] + qcap))
    const uint64_t* qend;
    uint64_t qcap;              // 0: no cap (counted passes)
    bool prezeroed;             // the fused pass's look-back words and ticket are already zero
};

// Exclusive prefix sum of N u32 counts whose total is below 2^32 (three launches):
// tsum holds exscan_tiles(N) words and tpre exscan_tiles(N) + 1 words of scratch.
uint64_t exscan_tiles(uint64_t N);
void exscan_u32(const uint32_t* in, uint64_t N, uint32_t* tsum, uint64_t* tpre, uint32_t* out, hipStream_t st);

PartPlan part_plan(uint64_t n);

// The partition passes over the wide maps of a batch (attempt 0 of each).  Inputs:
// d_keys/d_vals (the batch input), segs (nseg device descriptors), Cpool (the maps'
// level-two triples, T per map, at index map*T), pools.  Scratch: as allocated by the
// caller (see wide_scratch_bytes).  Per-map outcome words flags[4*seg + 0..3]: nonzero
// word 0 = attempt rejected (a bucket over 15 keys, or more than c*n cells), word 1 =
// a bucket exhausted its trials, word 2 = that bucket holds equal keys, word 3 = max trial.
// cbase[seg*(kSegParts+1) + j] receives the partition cell offsets within the map, and
// entry kSegParts the map's cell count S.
size_t wide_scratch_bytes(uint64_t nkeys, uint32_t nseg, uint32_t W);
int wide_build(const uint64_t* d_keys, const uint32_t* d_vals, const WideSeg* segs, uint32_t nseg, uint64_t nkeys,
               uint32_t W, const Triple* Cpool, uint32_t T, Group* hdr_pool, Cell* slot_pool, uint32_t* flags,
               uint64_t* cbase, void* scratch, hipStream_t st);
uint64_t part_scan_tiles(const PartPlan& P);
int part_prepare(const PartArgs& a, hipStream_t st, PartOut& o);
// given_t: trial index of every bucket decided elsewhere (n bytes), or nullptr to search.
// reject: two device words (a bucket above 15 keys, bad string offsets); when either is set
// the pass writes nothing (nullptr: never).  cap: cells allocated at slots; a partition
// whose cells would end beyond them writes nothing (the caller compares S with cap).
// The fused pass uses up o's cleared look-back words (o.prezeroed is reset).
int part_finish(const PartArgs& a, PartOut& o, const Triple* C, uint32_t T, Group* header, Cell* slots,
                uint32_t* flags, const int64_t* ctx_off, const uint8_t* ctx_bytes, const uint8_t* given_t,
                const uint32_t* reject, uint64_t cap, hipStream_t st);

}  // namespace fks
