/*
 * DialSort CPU ORACLE -- test infrastructure only.
 *
 * A plain, sequential, obviously-correct statement of what the DialSort hot
 * path computes.  Only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark may load this library; the product path never does.  It shares
 * no source, header or table with the HIP library.
 *
 * What it follows (DialSort, Sec. 3.3 "Mathematical Formulation, Correctness,
 * and Ordered Projection"):
 *   - H is initialised to zero, then every key x adds one to H[x]
 *     (ingestion, Eq. (1) "eq:ingestion");
 *   - the ordered projection sweeps k = 0, 1, ..., U-1 and emits k exactly H[k]
 *     times (Eq. (2) "eq:projection");
 *   - Theorem "thm:correct": the emitted sequence is nondecreasing, equals the
 *     input as a multiset and has length n = sum_k H[k].
 * The output is written in place when out == keys, as the paper's CPU
 * implementation does (Sec. 9.2, Table "tab:struct_cost").
 *
 * Readings where the paper is silent (each one is listed in the design notes):
 *   - a key x >= U is an error (Sec. 16: the method applies only to keys in
 *     [0, U-1]); the return code is ERANGE and outputs are unspecified;
 *   - counters are 32-bit unsigned (Sec. 7, Table "tab:wse3" gives 4 bytes per
 *     histogram cell), so n must be <= 2^32 - 1 (EOVERFLOW otherwise);
 *   - U must lie in [1, 2^32] (EINVAL otherwise);
 *   - the stand-alone projection writes min(sum H, out_cap) elements and returns
 *     EOVERFLOW when sum H > out_cap.
 *
 * Status numbers: 0 OK, 1 EINVAL, 2 ERANGE, 3 EOVERFLOW (the same numbering as
 * the product's public header, restated here on purpose).
 */
#include <stdint.h>
#include <stddef.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL 1
#define ORACLE_ERANGE 2
#define ORACLE_EOVERFLOW 3

/* Eq. (1): H := 0; for every key x: H[x] := H[x] + 1. */
int oracle_histogram(const uint32_t *keys, uint64_t n, uint64_t U, uint32_t *H) {
    uint64_t i, k;
    if (U == 0 || U > ((uint64_t)1 << 32) || H == NULL) return ORACLE_EINVAL;
    if (n > 0 && keys == NULL) return ORACLE_EINVAL;
    if (n > (uint64_t)0xFFFFFFFFu) return ORACLE_EOVERFLOW;
    for (k = 0; k < U; ++k) H[k] = 0;
    for (i = 0; i < n; ++i) {
        uint64_t x = keys[i];
        if (x >= U) return ORACLE_ERANGE;
        H[x] = H[x] + 1;
    }
    return ORACLE_OK;
}

/* Eq. (2): for k = 0 .. U-1, emit k exactly H[k] times.  Writes at most
 * out_cap elements; *written receives the number written. */
int oracle_reconstruct(const uint32_t *H, uint64_t U, uint32_t *out, uint64_t out_cap,
                       uint64_t *written) {
    uint64_t k, r, pos = 0, total = 0;
    if (U == 0 || U > ((uint64_t)1 << 32) || H == NULL) return ORACLE_EINVAL;
    if (out_cap > 0 && out == NULL) return ORACLE_EINVAL;
    for (k = 0; k < U; ++k) {
        total += H[k];
        for (r = 0; r < H[k]; ++r) {
            if (pos < out_cap) {
                out[pos] = (uint32_t)k;
                pos = pos + 1;
            }
        }
    }
    if (written) *written = pos;
    return total > out_cap ? ORACLE_EOVERFLOW : ORACLE_OK;
}

/* Ingestion followed by the ordered projection into out (out may equal keys). */
int oracle_sort(const uint32_t *keys, uint64_t n, uint64_t U, uint32_t *H, uint32_t *out) {
    uint64_t written = 0;
    int st = oracle_histogram(keys, n, U, H);
    if (st != ORACLE_OK) return st;
    if (n > 0 && out == NULL) return ORACLE_EINVAL;
    st = oracle_reconstruct(H, U, out, n, &written);
    if (st != ORACLE_OK) return st;
    /* Theorem "thm:correct", item 3: the projection has exactly n elements. */
    return written == n ? ORACLE_OK : ORACLE_EOVERFLOW;
}

/* ---- Queries on H (Sec. 3.3, the paragraph on the canonical ordered state):
 * answered from H alone, without the ordered projection. */

/* frequency(k) = H[k]; a key outside [0, U) occurs 0 times. */
void oracle_frequency(const uint32_t *H, uint64_t U, const uint32_t *q, uint64_t nq, uint32_t *out) {
    uint64_t i;
    for (i = 0; i < nq; ++i) out[i] = (uint64_t)q[i] < U ? H[q[i]] : 0;
}

/* presence(k) = 1 when k occurs in the input, i.e. H[k] > 0. */
void oracle_presence(const uint32_t *H, uint64_t U, const uint32_t *q, uint64_t nq, uint8_t *out) {
    uint64_t i;
    for (i = 0; i < nq; ++i) out[i] = ((uint64_t)q[i] < U && H[q[i]] > 0) ? 1 : 0;
}

/* range-count(a, b): the keys in [a, b), summed bin by bin as the paper states
 * it (O(b - a)); bounds past U are cut at U, and a >= b counts nothing. */
void oracle_range_count(const uint32_t *H, uint64_t U, const uint64_t *a, const uint64_t *b, uint64_t nq,
                        uint64_t *out) {
    uint64_t i, k;
    for (i = 0; i < nq; ++i) {
        uint64_t lo = a[i] < U ? a[i] : U, hi = b[i] < U ? b[i] : U, s = 0;
        for (k = lo; k < hi; ++k) s += H[k];
        out[i] = s;
    }
}

/* P[k] = H[0] + ... + H[k-1] for k = 0 .. U (U + 1 entries). */
void oracle_prefix(const uint32_t *H, uint64_t U, uint64_t *P) {
    uint64_t k, s = 0;
    for (k = 0; k < U; ++k) {
        P[k] = s;
        s += H[k];
    }
    P[U] = s;
}

/* select(r): the element at position r of the ordered projection (Eq. (2)),
 * found by walking the bins in ascending order; 0xFFFFFFFF when r >= sum H. */
void oracle_select(const uint32_t *H, uint64_t U, const uint64_t *r, uint64_t nq, uint32_t *out) {
    uint64_t i, k;
    for (i = 0; i < nq; ++i) {
        uint64_t acc = 0;
        out[i] = 0xFFFFFFFFu;
        for (k = 0; k < U; ++k) {
            acc += H[k];
            if (acc > r[i]) {
                out[i] = (uint32_t)k;
                break;
            }
        }
    }
}

/* Eq. (1) over one more piece of a key stream: H[x] := H[x] + 1 for every key
 * x of the piece, H not cleared.  A count passing 2^32 - 1 is EOVERFLOW. */
int oracle_histogram_accumulate(const uint32_t *keys, uint64_t n, uint64_t U, uint32_t *H) {
    uint64_t i;
    if (U == 0 || U > ((uint64_t)1 << 32) || H == NULL) return ORACLE_EINVAL;
    if (n > 0 && keys == NULL) return ORACLE_EINVAL;
    for (i = 0; i < n; ++i) {
        uint64_t x = keys[i];
        if (x >= U) return ORACLE_ERANGE;
        if (H[x] == 0xFFFFFFFFu) return ORACLE_EOVERFLOW;
        H[x] = H[x] + 1;
    }
    return ORACLE_OK;
}

/* The General Self-Indexing Principle (Sec. 3.4) with phi(x) = x - lo (mod
 * 2^32), an order-isomorphism from [lo, lo + U) onto [0, U): Eq. (1) over
 * phi(x), then Eq. (2) emitting phi^-1(k) = lo + k, H[k] times. */
int oracle_sort_offset(const uint32_t *keys, uint64_t n, uint32_t lo, uint64_t U, uint32_t *H, uint32_t *out) {
    uint64_t i, k, r, pos = 0;
    if (U == 0 || U > ((uint64_t)1 << 32) || H == NULL) return ORACLE_EINVAL;
    if (n > 0 && (keys == NULL || out == NULL)) return ORACLE_EINVAL;
    if (n > (uint64_t)0xFFFFFFFFu) return ORACLE_EOVERFLOW;
    for (k = 0; k < U; ++k) H[k] = 0;
    for (i = 0; i < n; ++i) {
        uint64_t x = (uint32_t)(keys[i] - lo);
        if (x >= U) return ORACLE_ERANGE;
        H[x] = H[x] + 1;
    }
    for (k = 0; k < U; ++k)
        for (r = 0; r < H[k]; ++r) out[pos++] = (uint32_t)(lo + k);
    return pos == n ? ORACLE_OK : ORACLE_EOVERFLOW;
}

/* The General Self-Indexing Principle (Sec. 3.4) for a domain given by its
 * index map: keys are the indices phi(s) in [0, U), and phi^-1 is the table
 * lut (U entries).  Eq. (1) over the indices, then Eq. (2) emitting lut[k],
 * H[k] times, for k ascending. */
int oracle_sort_lut(const uint32_t *keys, uint64_t n, uint64_t U, const uint32_t *lut, uint32_t *H, uint32_t *out) {
    uint64_t i, k, r, pos = 0;
    if (U == 0 || U > ((uint64_t)1 << 32) || H == NULL || lut == NULL) return ORACLE_EINVAL;
    if (n > 0 && (keys == NULL || out == NULL)) return ORACLE_EINVAL;
    if (n > (uint64_t)0xFFFFFFFFu) return ORACLE_EOVERFLOW;
    for (k = 0; k < U; ++k) H[k] = 0;
    for (i = 0; i < n; ++i) {
        if (keys[i] >= U) return ORACLE_ERANGE;
        H[keys[i]] = H[keys[i]] + 1;
    }
    for (k = 0; k < U; ++k)
        for (r = 0; r < H[k]; ++r) out[pos++] = lut[k];
    return ORACLE_OK;
}

/* The smallest and largest key, one comparison of each key against each
 * running bound, as int32 when is_signed: they fix the smallest offset map
 * phi(x) = x - min of Sec. 3.4 that holds the keys.  n == 0 leaves
 * (UINT32_MAX, 0), or (INT32_MAX, INT32_MIN) when signed. */
int oracle_key_range(const uint32_t *keys, uint64_t n, int is_signed, uint32_t *minmax) {
    uint64_t i;
    if (minmax == NULL || (n > 0 && keys == NULL)) return ORACLE_EINVAL;
    if (is_signed) {
        int32_t lo = INT32_MAX, hi = INT32_MIN;
        for (i = 0; i < n; ++i) {
            int32_t x = (int32_t)keys[i];
            if (x < lo) lo = x;
            if (x > hi) hi = x;
        }
        minmax[0] = (uint32_t)lo;
        minmax[1] = (uint32_t)hi;
    } else {
        uint32_t lo = 0xFFFFFFFFu, hi = 0;
        for (i = 0; i < n; ++i) {
            if (keys[i] < lo) lo = keys[i];
            if (keys[i] > hi) hi = keys[i];
        }
        minmax[0] = lo;
        minmax[1] = hi;
    }
    return ORACLE_OK;
}

/* DialSort-Radix (Sec. 8, "Full int32 range"): LSD, base 256, 4 passes, no
 * order comparison.  Each pass is DialSort on one 8-bit digit: Eq. (1) counts
 * the digits into H[0, 256), the running count of H gives where each digit's
 * run starts, and the keys are placed in input order within their digit's run
 * (stable), so the passes compose.  Signed keys go through phi(x) = x with its
 * sign bit flipped (Sec. 3.4), which maps int32 order onto uint32 order, and
 * come back through the same flip.  tmp holds n keys. */
int oracle_sort_radix(const uint32_t *keys, uint64_t n, int is_signed, uint32_t *out, uint32_t *tmp) {
    uint64_t i;
    int pass, d;
    const uint32_t flip = is_signed ? 0x80000000u : 0u;
    uint32_t *src = tmp, *dst = out;
    if (n > 0 && (keys == NULL || out == NULL || tmp == NULL)) return ORACLE_EINVAL;
    for (i = 0; i < n; ++i) tmp[i] = keys[i] ^ flip;
    for (pass = 0; pass < 4; ++pass) {
        uint64_t H[256], start[256], run = 0;
        const int shift = 8 * pass;
        for (d = 0; d < 256; ++d) H[d] = 0;
        for (i = 0; i < n; ++i) H[(src[i] >> shift) & 255u] += 1;
        for (d = 0; d < 256; ++d) {
            start[d] = run;
            run += H[d];
        }
        for (i = 0; i < n; ++i) {
            const uint32_t x = src[i];
            const uint32_t dg = (x >> shift) & 255u;
            dst[start[dg]] = x;
            start[dg] += 1;
        }
        /* the next pass reads what this one wrote */
        src = dst;
        dst = (dst == out) ? tmp : out;
    }
    /* four passes: the last one wrote into tmp */
    for (i = 0; i < n; ++i) out[i] = src[i] ^ flip;
    return ORACLE_OK;
}
