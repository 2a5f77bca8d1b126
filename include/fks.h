/*
 * fks.h -- C ABI of a static two-level (Fredman-Komlos-Szemeredi) hash map
 * built and queried on an AMD Instinct MI355X (gfx950).
 *
 * The operations are the map interface of Section 3.2 (Figure 2):
 *   from_array_nodup : ctx -> [n](key, v) -> map      (fks_build_*)
 *   lookup           : ctx -> key -> map -> opt v      (fks_lookup_*)
 * with membership testing as a lookup that returns only the "found" flag
 * (Section 4, the third benchmarked operation).  The map is the hash set
 * construction of Section 2.2 extended to a map by storing each value beside
 * its key: g k = hash(const) k mod n picks a bucket, the bucket's own level-two
 * function places the key in its private block of s^2 cells, the blocks lie at
 * the exclusive prefix sum of the squared bucket sizes, and a key is found iff
 * the cell it hashes to holds it.  Keys are 64-bit integers or byte strings;
 * a string key is a slice of a byte context (Section 3.1): the map keeps its
 * own copy of the context of its keys, and every needle batch brings its own.
 *
 * Conventions for every entry point:
 *   - Pointers named d_* are device pointers (HBM of the current device);
 *     pointers named h_* are host pointers.  Inputs are borrowed for the call
 *     only; the library never keeps them.
 *   - `stream` is a hipStream_t passed as void*; NULL is the default stream.
 *     Builds are ordered on the stream and synchronise the host with it
 *     once per level-one attempt, to read its outcome (twice when the table
 *     needs more cells than the bound the build allocates first, or under
 *     params.schedule = 1, which reads the table size before its search).
 *     Lookups are fully asynchronous.
 *   - Return value 0 (FKS_OK) is success; negative values are the FKS_E*
 *     codes below.  Out-parameters are written only on success.
 *   - Maps are immutable after their build and may be read by any number of
 *     concurrent lookups, on any streams of the device they were built on.
 *   - Layout of a built table (what fks_export returns, and what the oracle
 *     reproduces byte for byte):
 *       header: ceil(n/8) records of 16 bytes, one per group of 8 buckets:
 *               u32 slot base of the group, u32 sizes (4 bits per bucket,
 *               bucket 8g+k in bits 4k..4k+3), u8 t[8]: the trial index of
 *               a bucket of two or more keys; for a bucket of one key (whose
 *               trial is always 0) the top 8 bits of that key's trial-0
 *               level-two hash, a tag that lets a lookup answer "absent"
 *               without reading the cell; 0 for an empty bucket;
 *       cells : S records of 16 bytes: u64 key, u32 value, u32 aux
 *               (aux = 0 for integer keys, the key's index for string keys;
 *               the key word of a string map is the string's fingerprint).
 */
#ifndef FKS_H
#define FKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes -------------------------------------------------------- */
#define FKS_OK        0
#define FKS_EINVAL   (-1)  /* bad argument: NULL pointer, n >= 2^30, c*n >= 2^32,
                              parameter out of range, offsets not monotone,
                              wrong key kind for the map */
#define FKS_ENOMEM   (-2)  /* device allocation failed */
#define FKS_EDUPKEY  (-3)  /* the no-duplicates contract of from_array_nodup was
                              broken: a bucket that no level-two trial could
                              separate holds two equal keys, or every level-one
                              attempt was rejected and two keys are equal */
#define FKS_EBUILD   (-4)  /* every level-one attempt was rejected and the keys
                              are distinct */
#define FKS_EHIP     (-5)  /* a HIP runtime call failed; see fks_last_hip_error */

/* ---- parameters ---------------------------------------------------------
 * c : space budget; a level-one attempt is kept only if the table has at
 *     most c*n cells (default 4, range 1..16; Section 2.3 analysis: the
 *     expected size is about 2n).
 * T : level-two trials per bucket before the level-one attempt is rejected
 *     (default 64, range 1..256; make_2 of Section 2.3 retries without bound,
 *     expected at most 2 trials).
 * R : level-one attempts before FKS_EBUILD (default 16, range 1..1024).
 * schedule : how single-map builds search level two (the table is the same):
 *     0 = every bucket searched by one lane over its keys in LDS (default);
 *     1 = the paper's flattened rounds (Section 2.5): round t tries triple t
 *         on every unfinished bucket with a histogram over the flat cells.
 * Attempts also reject any bucket of more than 15 keys.                     */
typedef struct fks_params {
    uint32_t c;
    uint32_t T;
    uint32_t R;
    uint32_t schedule;
} fks_params;

typedef struct fks_map fks_map;       /* opaque; owns all of its device memory */

/* ---- device memory ---------------------------------------------------------
 * Where a build takes its device memory.  The map of Figure 2 owns its arrays
 * (Section 3.1: it keeps even its own copy of the key context); the caller
 * decides where they live.
 *   alloc : returns `bytes` of device memory of the current device, usable in
 *           stream order on `stream`, or NULL when it cannot.
 *   free  : releases a pointer that alloc returned, in stream order on
 *           `stream` (the stream it is called with may differ from the one
 *           the memory was allocated on only in fks_destroy and the other
 *           release calls, which pass NULL after the map's last use).
 *   user  : passed back unchanged.
 * Every build entry point takes a `const fks_allocator*`: the map (or batch,
 * or sorted array) and all of the call's scratch come from it, and a failed
 * alloc makes the call release everything it took and return FKS_ENOMEM
 * without writing its out-parameter.  The built object keeps a copy of the
 * struct and returns its memory through it when it is released, so `user`
 * must stay valid until then.  NULL selects hipMallocAsync / hipFreeAsync on
 * the device's default memory pool.  Both function pointers must be set
 * (FKS_EINVAL otherwise).  The library calls them from the thread that made
 * the entry-point call.                                                       */
typedef struct fks_allocator {
    void* (*alloc)(uint64_t bytes, void* stream, void* user);
    void (*free)(void* ptr, void* stream, void* user);
    void* user;
} fks_allocator;

typedef struct fks_map_info {
    uint64_t n;           /* number of keys */
    uint64_t S;           /* number of cells */
    uint64_t header_bytes;/* 16 * ceil(n/8) */
    uint64_t slot_bytes;  /* 16 * S */
    uint64_t ctx_bytes;   /* bytes of the copied string context (0 for integer keys) */
    uint64_t seed;        /* sigma */
    uint32_t r;           /* accepted level-one attempt */
    uint32_t kind;        /* 0 = uint64 keys, 1 = byte-string keys, 2 = uint64 keys with uint64 values */
    uint32_t c, T, R;
    uint32_t max_t;       /* largest trial index used by any bucket */
    uint64_t device_bytes;/* device memory the map holds */
    uint64_t size_hist[16];/* size_hist[s] = buckets holding s keys (the histogram
                              of make_1, Section 2.3); sum(s * size_hist[s]) = n,
                              sum(s^2 * size_hist[s]) = S */
} fks_map_info;

/* Fill *p with the defaults {4, 64, 16, 0}. */
void fks_params_default(fks_params* p);

/*
 * from_array_nodup for 64-bit keys (Section 2.2 construction, Section 2.3
 * make_1/make_2, built data-parallel as in Sections 2.4-2.5).
 *   d_keys : n distinct uint64 keys (device).
 *   d_vals : n uint32 values (device); value i belongs to key i.
 *   n      : 0 <= n < 2^30; n = 0 builds the empty map.
 *   seed   : sigma, the seed of the map's random stream (the `random` of
 *            Figure 1); the table is a pure function of (keys as a set,
 *            values, seed, params).
 *   params : NULL for defaults.
 *   alloc  : where the map and the call's scratch live (see fks_allocator);
 *            NULL for the device's default stream-ordered pool.
 *   out    : receives the new map (release with fks_destroy).
 * Errors: FKS_EINVAL, FKS_ENOMEM, FKS_EDUPKEY, FKS_EBUILD, FKS_EHIP.
 */
int fks_build_u64(const uint64_t* d_keys, const uint32_t* d_vals, uint64_t n, uint64_t seed,
                  const fks_params* params, const fks_allocator* alloc, void* stream, fks_map** out);

/*
 * from_array (Figure 2) for 64-bit keys: like fks_build_u64, but the u input
 * pairs may repeat a key.  The paper leaves open which value a repeated key
 * keeps; here it is the value of its first occurrence (lowest input index).
 * The map holds the distinct keys (fks_info reports their number as n) and
 * its table equals fks_build_u64 over those keys with their kept values.
 * Errors: as fks_build_u64 (never FKS_EDUPKEY); u < 2^30.
 */
int fks_build_u64_from_array(const uint64_t* d_keys, const uint32_t* d_vals, uint64_t u, uint64_t seed,
                             const fks_params* params, const fks_allocator* alloc, void* stream, fks_map** out);

/*
 * from_array_nodup for 64-bit keys with 64-bit values (the value type of
 * Figure 2 is polymorphic).  The construction and the header are those of
 * fks_build_u64 over the same keys; a cell keeps the value's low half where a
 * 32-bit map keeps its value and the high half in its aux word, so the table
 * takes no more memory.  d_vals: n uint64 values (device).  Answer lookups
 * with fks_lookup_u64_v64 (fks_contains_u64 also works; fks_lookup_u64 returns
 * FKS_EINVAL).  Errors: as fks_build_u64.
 */
int fks_build_u64_v64(const uint64_t* d_keys, const uint64_t* d_vals, uint64_t n, uint64_t seed,
                      const fks_params* params, const fks_allocator* alloc, void* stream, fks_map** out);

/*
 * from_array_nodup for byte-string keys (Section 3.1 contexts, Section 3.3.1
 * slices).  Key i is bytes [d_offsets[i], d_offsets[i+1]) of d_bytes (CSR;
 * a string may be empty).  Offsets must be non-decreasing, d_offsets[0] >= 0
 * and d_offsets[n] <= nbytes.  The map copies d_offsets (n+1 int64) and the
 * first nbytes of d_bytes.  Each level-one attempt fingerprints every string
 * (Horner over 32-bit little-endian words mod 2^61-1, seeded with the byte
 * length) and runs the integer construction on the fingerprints; distinct
 * strings with equal fingerprints force a new attempt with a new base.
 * Errors: as fks_build_u64; FKS_EDUPKEY when two keys are equal strings.
 */
int fks_build_bytes(const int64_t* d_offsets, const uint8_t* d_bytes, uint64_t nbytes,
                    const uint32_t* d_vals, uint64_t n, uint64_t seed,
                    const fks_params* params, const fks_allocator* alloc, void* stream, fks_map** out);

/*
 * lookup (Figure 2) for m integer needles: d_vals_out[i] = value of
 * d_queries[i] and d_found_out[i] = 1 if the key is in the map, else
 * d_vals_out[i] = missing and d_found_out[i] = 0.  At most two dependent
 * table reads per needle.  Either output may be NULL to skip it; a given
 * output holds m entries (the call cannot check its size).
 * Errors: FKS_EINVAL (NULL map/queries with m > 0, string map), FKS_EHIP.
 */
int fks_lookup_u64(const fks_map* map, const uint64_t* d_queries, uint64_t m,
                   uint32_t* d_vals_out, uint8_t* d_found_out, uint32_t missing, void* stream);

/* Membership only (Section 4): d_found_out[i] = 1 iff d_queries[i] is a key
   (maps of kind 0 or 2). */
int fks_contains_u64(const fks_map* map, const uint64_t* d_queries, uint64_t m,
                     uint8_t* d_found_out, void* stream);

/* lookup on a map built by fks_build_u64_v64: d_vals_out (required) receives
   the 64-bit value or `missing`; d_found_out may be NULL.  Errors: FKS_EINVAL
   (other map kinds, NULL arguments with m > 0), FKS_EHIP. */
int fks_lookup_u64_v64(const fks_map* map, const uint64_t* d_queries, uint64_t m, uint64_t* d_vals_out,
                       uint8_t* d_found_out, uint64_t missing, void* stream);

/*
 * lookup for m string needles given in their own context (Section 3.1: the
 * needle's context differs from the map's): needle i is bytes
 * [d_q_offsets[i], d_q_offsets[i+1]) of d_q_bytes, which holds q_nbytes
 * bytes.  A hit needs equal fingerprints and then equal bytes (a third read,
 * of the stored string).  A needle whose pair of offsets is not a range
 * inside d_q_bytes (a negative start, an end before its start, or an end
 * past q_nbytes) reads nothing and is answered absent.  Either output may be
 * NULL.  Errors: FKS_EINVAL (NULL map or needle arrays with m > 0, a map that
 * is not a string map), FKS_EHIP.
 */
int fks_lookup_bytes(const fks_map* map, const int64_t* d_q_offsets, const uint8_t* d_q_bytes,
                     uint64_t q_nbytes, uint64_t m, uint32_t* d_vals_out, uint8_t* d_found_out,
                     uint32_t missing, void* stream);

/* Membership only for string needles, under the same contract. */
int fks_contains_bytes(const fks_map* map, const int64_t* d_q_offsets, const uint8_t* d_q_bytes,
                       uint64_t q_nbytes, uint64_t m, uint8_t* d_found_out, void* stream);

/* ---- map and reduce over values -------------------------------------------
 * Section 1 names the operations a hash map shares with an array: mapping a
 * function over its values, and reducing its values to one value.
 *
 * fks_map_values: a new map (release with fks_destroy) with the keys of `map`
 * and the value op(v) for each key's value v.  The header, the level-two
 * triples and a string map's context are copied unchanged and every cell's
 * value is rewritten, so the new table is byte for byte the one that building
 * the pairs (k, op(v)) with the same seed and parameters writes.  Arithmetic is
 * modulo 2^32 for maps with 32-bit values (a and b are taken modulo 2^32) and
 * modulo 2^64 for maps of fks_build_u64_v64.  FKS_VOP_GATHER reads
 * d_table[v] (table_len device entries of the value width: uint32, or uint64
 * for fks_build_u64_v64 maps); a value v >= table_len fails the call with
 * FKS_EINVAL and no map.  `map` is not modified.  Synchronises the stream
 * once.  Errors: FKS_EINVAL (NULL map/out, unknown op, NULL table with
 * table_len > 0, a value outside the table), FKS_ENOMEM, FKS_EHIP.
 *
 * fks_reduce_values: *d_out (one uint64 on the device) = the fold of op over
 * the values of the map's n keys, each key counted once (the fill copies of a
 * bucket's lowest key are not values of the map).  FKS_VRED_SUM is the sum
 * modulo 2^64; on an empty map the result is the operation's identity (0 for
 * SUM, MAX and XOR; all ones of the value width for MIN).  Asynchronous on
 * `stream`.  Errors: FKS_EINVAL (NULL map/d_out, unknown op), FKS_ENOMEM,
 * FKS_EHIP.                                                                  */
#define FKS_VOP_ADD    0u   /* v + a */
#define FKS_VOP_MUL    1u   /* v * a */
#define FKS_VOP_XOR    2u   /* v ^ a */
#define FKS_VOP_AFFINE 3u   /* v * a + b */
#define FKS_VOP_GATHER 4u   /* d_table[v] */
#define FKS_VRED_SUM   0u
#define FKS_VRED_MIN   1u
#define FKS_VRED_MAX   2u
#define FKS_VRED_XOR   3u

int fks_map_values(const fks_map* map, uint32_t op, uint64_t a, uint64_t b, const void* d_table,
                   uint64_t table_len, const fks_allocator* alloc, void* stream, fks_map** out);
int fks_reduce_values(const fks_map* map, uint32_t op, uint64_t* d_out, void* stream);

/* fks_reduce_values_noalloc: fks_reduce_values for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, result and errors; it
 * calls no allocator.  The partial folds of its first pass live in a static
 * device array of 4096 uint64 (32 KiB) that each device keeps from its first
 * call until the process ends; the first pass never has more workgroups than
 * that, for every map size, so no map is refused for size.  Nothing in the
 * array needs to start at zero: every partial is written before it is read.
 * Every call on one device shares the array, so two calls whose kernels
 * overlap on that device (on different streams, or from different host
 * threads without ordering between their streams) race and may return wrong
 * folds; calls ordered on one stream do not.  The first call on a device looks
 * up the array's address (hipGetSymbolAddress) and can fail with FKS_EHIP.  */
int fks_reduce_values_noalloc(const fks_map* map, uint32_t op, uint64_t* d_out, void* stream);


/* Sizes and build outcome of a map.  The bucket-size histogram is counted by
   one small kernel over the group headers, on the null stream, which the call
   waits for.  Errors: FKS_EINVAL, FKS_EHIP. */
int fks_info(const fks_map* map, fks_map_info* info);

/*
 * Copy the table to host memory: h_header (info.header_bytes), h_slots
 * (info.slot_bytes), optionally h_consts (3*T uint64: the level-two triples
 * of the accepted attempt).  Any pointer may be NULL.  Synchronous.
 */
int fks_export(const fks_map* map, void* h_header, void* h_slots, uint64_t* h_consts);

/* Release a map and its device memory.  NULL is ignored.  The caller must
   make sure no lookup on the map is still running. */
void fks_destroy(fks_map* map);

/* Text of an error code. */
const char* fks_strerror(int code);

/* The last HIP error code seen by the calling thread (hipError_t as int). */
int fks_last_hip_error(void);

/* Library version, major*10000 + minor*100 + patch. */
int fks_version(void);

/* ---- batches of maps ----------------------------------------------------
 * One more level of flattening above Section 2.4's buckets: M independent
 * maps (Section 3.2 notes that maps cannot be array elements, since that
 * would make arrays irregular) built in one persistent launch.  Map m holds
 * keys [h_map_offsets[m], h_map_offsets[m+1]) of d_keys / d_vals and is built
 * exactly as fks_build_u64 would build it with seed = entry m of the
 * SplitMix64 stream of batch_seed, so its table bytes equal the single-map
 * build's.  Limits: each map holds at most 65536 keys; c * total keys < 2^40.
 * Every map owns c * n cells of the batch's cell pool.  A map whose build
 * fails (FKS_EDUPKEY / FKS_EBUILD, see fks_batch_status) answers every
 * lookup with "absent"; the call itself still succeeds.
 *   h_map_offsets : host array of M+1 non-decreasing offsets, first one 0.
 *   schedule      : 0 = the tuned (or default) schedule for this batch size
 *                   class; otherwise one of fks_batch_schedules().
 */
typedef struct fks_batch fks_batch;

int fks_build_batch_u64(const uint64_t* d_keys, const uint32_t* d_vals, const uint64_t* h_map_offsets,
                        uint32_t M, uint64_t batch_seed, const fks_params* params, uint32_t schedule,
                        const fks_allocator* alloc, void* stream, fks_batch** out);

/* Needle i asks map d_map_ids[i] for key d_queries[i]; map ids >= M are
   answered "absent".  Asynchronous; outputs as fks_lookup_u64. */
int fks_lookup_batch_u64(const fks_batch* batch, const uint32_t* d_map_ids, const uint64_t* d_queries,
                         uint64_t m, uint32_t* d_vals_out, uint8_t* d_found_out, uint32_t missing,
                         void* stream);

/* Per-map outcome (host arrays of M entries; any may be NULL): status
   (FKS_OK or an error code), accepted attempt r, cell count S. */
int fks_batch_status(const fks_batch* batch, int32_t* h_status, uint32_t* h_r, uint32_t* h_S);

/* Sizes of map `index` (returns its status), as fks_info reports them; the
   histogram is counted only for a map that was built (FKS_OK). */
int fks_batch_info(const fks_batch* batch, uint32_t index, fks_map_info* info);

/* Table of map `index`, laid out as fks_export lays out a single map. */
int fks_batch_export(const fks_batch* batch, uint32_t index, void* h_header, void* h_slots,
                     uint64_t* h_consts);

void fks_batch_destroy(fks_batch* batch);

/* Schedules of the batched build: bits 0-1 select 256/512/1024 threads per
   workgroup, bits 4-7 the workgroups per CU; bit 8 set builds the maps of at
   least 8192 keys together through the partitioned passes first (attempt 0 of
   each; a map they reject continues in the per-workgroup kernel), and the
   tables are the same either way.  fks_batch_schedules lists the
   valid ones (returns their count; out may be NULL).  fks_batch_set_schedule
   records the schedule that schedule = 0 uses for batches of the same size
   class (log2 of M and of the mean map size) in this process. */
int fks_batch_schedules(uint32_t* out, int max_entries);
int fks_batch_set_schedule(uint32_t M, uint64_t total_keys, uint32_t schedule);

/* ---- serving --------------------------------------------------------------
 * A request loop over resident maps (not in the paper; it turns the map of
 * Sections 2-3 into a service).  Builds are admitted against a device-memory
 * budget (an estimate of c*n cells per pending build; idle maps are evicted
 * least recently used first when the budget would be exceeded) and run on three
 * build workers, each with its own stream, so three builds can be in flight (a
 * build waits for admission while another worker's build still holds its
 * reservation).  Lookup requests of any size that are
 * queued while other work runs are coalesced into one multi-request launch on
 * the lookup stream, replayed from a HIP graph captured per (ring slot, grid
 * size); so lookups overlap builds on the device.  Results do not depend on
 * what else is in flight: each request's outputs are those of the same call
 * made alone.
 *   Device buffers passed to submit calls must stay valid until the request
 *   completes (fks_server_poll / fks_server_wait_all).  Lookups against a map
 *   that failed to build, or was evicted, complete with that error status.
 *   flags: bit 0 disables graph replay (plain launches).
 *   Device memory: fks_server_create reserves one slab (the budget, plus room
 *   for the running builds' scratch: 32 bytes for each key the budget admits)
 *   and every map and build scratch of the server is carved from it, so no
 *   request waits on the driver's allocator; fks_server_create fails with
 *   FKS_ENOMEM when the slab cannot be reserved.
 */
typedef struct fks_server fks_server;

typedef struct fks_server_stats {
    uint64_t requests, completed;
    uint64_t lookup_launches;     /* multi-request launches */
    uint64_t graph_replays;       /* launches replayed from a captured graph */
    uint64_t graphs_captured;
    uint64_t coalesced_requests;  /* lookup requests carried by those launches */
    uint64_t evictions;
    uint64_t resident_bytes;
    uint64_t queries_done, keys_built;
    double span_ms;               /* first submission to last completion */
    uint32_t resident_maps, pad;
} fks_server_stats_t;

int fks_server_create(uint64_t budget_bytes, const fks_params* params, uint32_t flags, fks_server** out);
/* Queue a build; *map_id names the future map at once (lookups may be queued
   against it before it is built).  Ordering: the request's device work starts
   only after everything queued on `stream` (the submitter's stream, a
   hipStream_t as void*; NULL = the default stream) before this call, so the
   inputs may still be in flight there; the call records an event on `stream`
   and the server's stream waits for it.  A build whose reservation (header +
   c*n cells + triples) exceeds the whole budget completes at once with
   FKS_ENOMEM and evicts nothing; otherwise idle maps are evicted, least
   recently used first, only when that makes room, else the build waits for
   lookups pinning resident maps to drain. */
int fks_server_submit_build(fks_server* srv, const uint64_t* d_keys, const uint32_t* d_vals, uint64_t n,
                            uint64_t seed, void* stream, uint64_t* req_id, uint32_t* map_id);
/* Queue a lookup of m needles against map_id, ordered after `stream` as
   fks_server_submit_build is.  The outputs are written by the time
   fks_server_poll reports the request done. */
int fks_server_submit_lookup(fks_server* srv, uint32_t map_id, const uint64_t* d_queries, uint64_t m,
                             uint32_t* d_vals_out, uint8_t* d_found_out, uint32_t missing, void* stream,
                             uint64_t* req_id);
/* *done = 1 once finished; *latency_ms = completion - submission (host clock). */
int fks_server_poll(fks_server* srv, uint64_t req_id, int* done, int* status, double* latency_ms);
int fks_server_wait_all(fks_server* srv);
/* Per-request submission and completion times (ms, host steady clock), kind
   (0 build, 1 lookup) and status, for requests 0..max_entries-1; returns the
   count written.  Any array may be NULL. */
int fks_server_latencies(fks_server* srv, double* h_submit_ms, double* h_done_ms, int32_t* h_kind,
                         int32_t* h_status, uint64_t max_entries);
int fks_server_stats(fks_server* srv, fks_server_stats_t* stats);
/* The resident map behind map_id, or NULL (not built yet, failed, evicted). */
const fks_map* fks_server_map(fks_server* srv, uint32_t map_id);
/* Waits for every submitted request, then releases the server and its maps. */
void fks_server_destroy(fks_server* srv);

/* ---- device random-access ceiling ----------------------------------------
 * Times `probes` independent random reads of width_bytes (16, 32, 64 or 128)
 * from a buffer of about buffer_bytes (allocated and released inside), after
 * one warm-up pass; *ms_out receives the time of the second pass.  The rate
 * probes / time is the ceiling that one- and two-probe lookups run against.
 * Synchronous.  Errors: FKS_EINVAL (ms_out NULL, probes 0, another width),
 * FKS_ENOMEM, FKS_EHIP; the buffers are released on every path. */
int fks_probe_random_reads(uint64_t buffer_bytes, uint64_t probes, uint32_t width_bytes, void* stream,
                           double* ms_out);

/* ---- comparison maps: sorted array and Eytzinger order (Section 4) --------
 * The search structures the paper measures its hash maps against: the pairs
 * sorted by key and found by binary search, or the same sorted pairs stored in
 * the level order of the complete binary search tree (Eytzinger layout) and
 * found by a root-to-leaf descent.  Same contract as fks_build_u64: keys
 * distinct (FKS_EDUPKEY otherwise), lookups return the value of the equal key
 * or `missing`.                                                              */
typedef struct fks_sorted fks_sorted;
#define FKS_LAYOUT_SORTED 0u      /* ascending keys, binary search */
#define FKS_LAYOUT_EYTZINGER 1u   /* level order of the complete search tree */

/* d_keys, d_vals: n device records, read only during the call; n < 2^32.
   The structure owns 12 bytes of device memory per key.  Synchronizes the
   stream once (duplicate check).  Errors: FKS_EINVAL, FKS_ENOMEM, FKS_EDUPKEY,
   FKS_EHIP. */
int fks_sorted_build_u64(const uint64_t* d_keys, const uint32_t* d_vals, uint64_t n, uint32_t layout,
                         const fks_allocator* alloc, void* stream, fks_sorted** out);
/* As fks_lookup_u64: d_vals_out may be NULL (membership only); asynchronous. */
int fks_sorted_lookup_u64(const fks_sorted* s, const uint64_t* d_queries, uint64_t m, uint32_t* d_vals_out,
                          uint8_t* d_found_out, uint32_t missing_value, void* stream);
/* Copies the n keys and values in layout order to host arrays. */
int fks_sorted_export(const fks_sorted* s, uint64_t* h_keys, uint32_t* h_vals);
int fks_sorted_info(const fks_sorted* s, uint64_t* n, uint32_t* layout);
void fks_sorted_destroy(fks_sorted* s);

/* ---- kernel timing ------------------------------------------------------
 * When enabled, every kernel the library launches is bracketed by two HIP
 * events recorded on the stream it runs on; fks_prof_read folds the finished
 * ones into per-kernel totals (it waits for pending events).  Process-wide,
 * thread-safe; off by default.                                              */
typedef struct fks_prof_entry {
    char name[40];        /* kernel name */
    uint64_t launches;    /* timed launches since the last reset */
    double total_ms;      /* summed event time of those launches */
} fks_prof_entry;

int fks_prof_enable(int on);
void fks_prof_reset(void);
/* Writes up to max_entries entries and returns how many it wrote; with
   out == NULL returns the number of kernels with totals. */
int fks_prof_read(fks_prof_entry* out, int max_entries);

#ifdef __cplusplus
}
#endif

#endif /* FKS_H */
