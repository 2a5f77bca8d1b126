// Partitioned level-one attempt (partition.hip): plan, buffers, entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fks_internal.hpp"

namespace fks {

constexpr uint32_t kPartBits = 10;                   // 1024 buckets per partition
constexpr uint32_t kPartBuckets = 1u << kPartBits;

struct PartPlan {
    uint32_t Q;        // partitions
    uint32_t bits_q;   // ceil(log2 Q)
    uint32_t passes;   // scatter passes: 0, 1 or 2
    uint32_t shiftA;   // first-level bin = q >> shiftA
    uint32_t binsA;    // first-level bins
    uint32_t bitsB;    // second-level bin = q & (2^bitsB - 1)
    uint32_t W1, W2;   // workers of the first pass / per first-level bin in the second pass
    uint64_t matrix;   // entries of the largest count matrix
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
    uint64_t* offQ;             // Q+1 partition offsets
    uint32_t* sqQ;              // Q sums of squared sizes
    uint64_t* cbase;            // Q+1 cell bases
    uint32_t* sizes;            // G size words (the headers' second word)
    uint64_t* S_dev;            // total cells
    uint32_t* oversize;         // a bucket above 15 keys
};

struct PartOut {
    PartPlan plan;
    const uint64_t* keys;       // records in partition order
    const uint32_t* vals;
    const uint32_t* aux;
    int aux_is_pos;
};

// Exclusive prefix sum of N u32 counts whose total is below 2^32 (three launches):
// tsum holds exscan_tiles(N) words and tpre exscan_tiles(N) + 1 words of scratch.
uint64_t exscan_tiles(uint64_t N);
void exscan_u32(const uint32_t* in, uint64_t N, uint32_t* tsum, uint64_t* tpre, uint32_t* out, hipStream_t st);

PartPlan part_plan(uint64_t n);
uint64_t part_scan_tiles(const PartPlan& P);
int part_prepare(const PartArgs& a, hipStream_t st, PartOut& o);
// given_t: trial index of every bucket decided elsewhere (n bytes), or nullptr to search
int part_finish(const PartArgs& a, const PartOut& o, const Triple* C, uint32_t T, Group* header, Cell* slots,
                uint32_t* flags, const int64_t* ctx_off, const uint8_t* ctx_bytes, const uint8_t* given_t,
                hipStream_t st);

}  // namespace fks
