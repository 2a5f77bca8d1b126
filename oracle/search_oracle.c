/*
 * Plain, sequential CPU oracle for the comparison maps of Section 4: a sorted
 * array searched by binary search, and the same keys in Eytzinger (BFS) order.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite and the benchmark's CPU-baseline leg
 * do.  It shares no code with the HIP path.
 *
 * What it computes:
 *   - sorted layout: the (key, value) pairs ordered by key (qsort); equal keys
 *     are a precondition violation (the nodup contract of from_array_nodup,
 *     Figure 2) and make the build fail with the duplicate-key error.
 *   - Eytzinger layout: the complete binary search tree on the sorted keys,
 *     stored level by level (node i has children 2i and 2i+1, 1-based), filled
 *     by the textbook recursive in-order walk: visit the left child, take the
 *     next sorted pair, visit the right child.
 *   - lookup: for every needle, the value of the equal key or "absent"
 *     (the dictionary semantics the hash maps of Section 2.2 also have);
 *     binary search over the sorted array, or the tree descent over the
 *     Eytzinger array.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { SO_OK = 0, SO_EINVAL = -1, SO_ENOMEM = -2, SO_EDUPKEY = -3 };

typedef struct {
    uint64_t key;
    uint32_t val;
} so_pair;

static int so_cmp(const void* a, const void* b)
{
    const uint64_t x = ((const so_pair*)a)->key, y = ((const so_pair*)b)->key;
    return x < y ? -1 : x > y ? 1 : 0;
}

/* recursive in-order fill of the BFS-numbered tree rooted at node i (1-based) */
static void so_fill(const so_pair* sorted, uint64_t n, uint64_t i, uint64_t* next,
                    uint64_t* out_keys, uint32_t* out_vals)
{
    if (i > n) return;
    so_fill(sorted, n, 2 * i, next, out_keys, out_vals);
    out_keys[i - 1] = sorted[*next].key;
    out_vals[i - 1] = sorted[*next].val;
    ++*next;
    so_fill(sorted, n, 2 * i + 1, next, out_keys, out_vals);
}

/* layout 0: sorted array; layout 1: Eytzinger order.  out arrays hold n entries. */
int oracle_search_build(const uint64_t* keys, const uint32_t* vals, uint64_t n, uint32_t layout,
                        uint64_t* out_keys, uint32_t* out_vals)
{
    if (layout > 1 || (n && (!keys || !vals || !out_keys || !out_vals))) return SO_EINVAL;
    if (n == 0) return SO_OK;
    so_pair* p = (so_pair*)malloc(sizeof(so_pair) * n);
    if (!p) return SO_ENOMEM;
    for (uint64_t i = 0; i < n; ++i) {
        p[i].key = keys[i];
        p[i].val = vals[i];
    }
    qsort(p, n, sizeof(so_pair), so_cmp);
    for (uint64_t i = 1; i < n; ++i)
        if (p[i].key == p[i - 1].key) {
            free(p);
            return SO_EDUPKEY;
        }
    if (layout == 0) {
        for (uint64_t i = 0; i < n; ++i) {
            out_keys[i] = p[i].key;
            out_vals[i] = p[i].val;
        }
    } else {
        uint64_t next = 0;
        so_fill(p, n, 1, &next, out_keys, out_vals);
    }
    free(p);
    return SO_OK;
}

/* lookups against a built layout (the arrays oracle_search_build wrote) */
int oracle_search_lookup(const uint64_t* lkeys, const uint32_t* lvals, uint64_t n, uint32_t layout,
                         const uint64_t* q, uint64_t m, uint32_t* out_vals, uint8_t* out_found,
                         uint32_t missing)
{
    if (layout > 1) return SO_EINVAL;
    for (uint64_t j = 0; j < m; ++j) {
        const uint64_t x = q[j];
        int64_t hit = -1;
        if (layout == 0) {
            uint64_t lo = 0, hi = n; /* first index with key >= x */
            while (lo < hi) {
                const uint64_t mid = lo + (hi - lo) / 2;
                if (lkeys[mid] < x) lo = mid + 1;
                else hi = mid;
            }
            if (lo < n && lkeys[lo] == x) hit = (int64_t)lo;
        } else {
            uint64_t i = 1;
            while (i <= n) {
                if (lkeys[i - 1] == x) {
                    hit = (int64_t)(i - 1);
                    break;
                }
                i = lkeys[i - 1] < x ? 2 * i + 1 : 2 * i;
            }
        }
        if (out_found) out_found[j] = hit >= 0;
        if (out_vals) out_vals[j] = hit >= 0 ? lvals[hit] : missing;
    }
    return SO_OK;
}
