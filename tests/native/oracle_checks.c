/*
 * oracle_checks.c -- the oracle (oracle/fnr_oracle.c) built with gcc under the
 * address and undefined-behaviour sanitizers (tests/test_native_cpu.py), run
 * over the inputs of its pins: random tiny frames below and above the window
 * size with small alphabets (ties), both pixel types, windows 3..31, one to
 * three passes, pitches with padding, and introsort on adversarial orders and
 * with a zero depth bound.  Each result is compared with a brute-force
 * statement written here: the window gathered with clamped coordinates and
 * fully sorted by insertion, its middle element taken where the centre equals
 * the window's minimum or maximum.  Prints "ok" and returns 0 when every case
 * agrees and the sanitizers report nothing.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint64_t scans, sorts, partitions, heapsorts, insertions;
} sort_stats;

int oracle_fnr(const void *src, size_t src_pitch, void *dst, size_t dst_pitch, int W, int H, int bytes, int k,
               int passes, uint64_t *counts, sort_stats *st);
int oracle_median(const void *src, size_t src_pitch, const uint8_t *mask, size_t mask_pitch, void *dst,
                  size_t dst_pitch, int W, int H, int bytes, int k, uint64_t *sorts, sort_stats *st);
int oracle_detect(const void *src, size_t src_pitch, uint8_t *mask, size_t mask_pitch, int W, int H, int bytes,
                  int k, uint64_t *count);
int oracle_detect_directional(const void *src, size_t src_pitch, uint8_t *mask, size_t mask_pitch, int W, int H,
                              int bytes, uint64_t *count);
void oracle_introsort(uint32_t *a, int n, sort_stats *st);
void oracle_introsort_depth(uint32_t *a, int n, int depth_limit, sort_stats *st);

static uint64_t rng_state = 12013972u;
static uint32_t next_u32(void) { /* xorshift64* */
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return (uint32_t)((rng_state * 2685821657736338717ull) >> 32);
}

static int failures = 0;

static uint32_t get(const uint8_t *f, size_t pitch, int bytes, int x, int y) {
    return bytes == 1 ? f[(size_t)y * pitch + x] : ((const uint16_t *)(f + (size_t)y * pitch))[x];
}

static void put(uint8_t *f, size_t pitch, int bytes, int x, int y, uint32_t v) {
    if (bytes == 1)
        f[(size_t)y * pitch + x] = (uint8_t)v;
    else
        ((uint16_t *)(f + (size_t)y * pitch))[x] = (uint16_t)v;
}

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* one brute-force FNR pass from a to b (packed, pitch W * bytes) */
static uint64_t brute_pass(const uint8_t *a, uint8_t *b, int W, int H, int bytes, int k) {
    const int r = k / 2, n = k * k;
    uint32_t *S = malloc(sizeof(uint32_t) * n);
    uint64_t flagged = 0;
    const size_t pitch = (size_t)W * bytes;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int m = 0;
            for (int j = -r; j <= r; ++j)
                for (int i = -r; i <= r; ++i)
                    S[m++] = get(a, pitch, bytes, clampi(x + i, 0, W - 1), clampi(y + j, 0, H - 1));
            for (int p = 1; p < n; ++p) /* insertion sort */
                for (int q = p; q > 0 && S[q - 1] > S[q]; --q) {
                    const uint32_t t = S[q];
                    S[q] = S[q - 1];
                    S[q - 1] = t;
                }
            const uint32_t c = get(a, pitch, bytes, x, y);
            const int noisy = c == S[0] || c == S[n - 1];
            flagged += noisy;
            put(b, pitch, bytes, x, y, noisy ? S[(n - 1) / 2] : c);
        }
    free(S);
    return flagged;
}

static void check_fnr_case(int W, int H, int bytes, int k, int passes, int alphabet, int pad) {
    const size_t pitch = (size_t)W * bytes + (size_t)pad * bytes, packed = (size_t)W * bytes;
    uint8_t *src = malloc(pitch * H), *dst = malloc(pitch * H);
    uint8_t *a = malloc(packed * H), *b = malloc(packed * H);
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W + pad; ++x) {
            const uint32_t v = alphabet ? next_u32() % alphabet : next_u32() & (bytes == 1 ? 0xff : 0xffff);
            if (x < W) {
                put(src, pitch, bytes, x, y, v);
                put(a, packed, bytes, x, y, v);
            } else {
                put(src, pitch, bytes, x, y, v); /* padding is never read */
            }
        }
    memset(dst, 0xab, pitch * H);
    uint64_t counts[3] = {0, 0, 0}, want[3] = {0, 0, 0};
    if (oracle_fnr(src, pitch, dst, pitch, W, H, bytes, k, passes, counts, NULL) != 0) {
        fprintf(stderr, "oracle_fnr rejected %dx%d k=%d\n", W, H, k);
        ++failures;
    }
    for (int p = 0; p < passes; ++p) {
        want[p] = brute_pass(a, b, W, H, bytes, k);
        uint8_t *t = a;
        a = b;
        b = t;
    }
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W + pad; ++x) {
            const uint32_t g = get(dst, pitch, bytes, x, y);
            const uint32_t w = x < W ? get(a, packed, bytes, x, y) : (bytes == 1 ? 0xab : 0xabab);
            if (g != w) {
                fprintf(stderr, "fnr %dx%d b=%d k=%d p=%d: (%d,%d) %u != %u\n", W, H, bytes, k, passes, x, y, g, w);
                ++failures;
                goto out;
            }
        }
    for (int p = 0; p < passes; ++p)
        if (counts[p] != want[p]) {
            fprintf(stderr, "fnr %dx%d k=%d pass %d count %llu != %llu\n", W, H, k, p, (unsigned long long)counts[p],
                    (unsigned long long)want[p]);
            ++failures;
        }
out:
    free(src);
    free(dst);
    free(a);
    free(b);
}

static void check_mask_paths(void) {
    /* detect, masked median, plain median and the directional detector on one
       frame each: results within range, no sanitizer report */
    const int W = 37, H = 23;
    uint8_t f[37 * 23], m[37 * 23], d[37 * 23];
    for (int i = 0; i < W * H; ++i) f[i] = (uint8_t)(next_u32() % 4);
    uint64_t c = 0, s = 0;
    if (oracle_detect(f, W, m, W, W, H, 1, 5, &c) != 0 || c > (uint64_t)(W * H)) ++failures;
    if (oracle_median(f, W, m, W, d, W, W, H, 1, 5, &s, NULL) != 0 || s != c) ++failures;
    if (oracle_median(f, W, NULL, 0, d, W, W, H, 1, 9, &s, NULL) != 0 || s != (uint64_t)(W * H)) ++failures;
    if (oracle_detect_directional(f, W, m, W, W, H, 1, &c) != 0 || c > (uint64_t)(W * H)) ++failures;
}

static int sorted(const uint32_t *v, int n) {
    for (int i = 1; i < n; ++i)
        if (v[i - 1] > v[i]) return 0;
    return 1;
}

static void check_introsort(void) {
    enum { N = 961 };
    static uint32_t v[N];
    for (int kind = 0; kind < 6; ++kind)
        for (int n = 1; n <= N; n += (n < 40 ? 1 : 37)) {
            for (int i = 0; i < n; ++i) {
                switch (kind) {
                    case 0: v[i] = next_u32(); break;              /* random */
                    case 1: v[i] = (uint32_t)i; break;             /* sorted */
                    case 2: v[i] = (uint32_t)(n - i); break;       /* reversed */
                    case 3: v[i] = (uint32_t)(i < n / 2 ? i : n - i); break; /* organ pipe */
                    case 4: v[i] = 7; break;                       /* constant */
                    default: v[i] = next_u32() % 3; break;         /* few values */
                }
            }
            sort_stats st = {0, 0, 0, 0, 0};
            if (kind % 2)
                oracle_introsort_depth(v, n, 0, &st); /* heapsort branch alone */
            else
                oracle_introsort(v, n, &st);
            if (!sorted(v, n)) {
                fprintf(stderr, "introsort kind %d n %d not sorted\n", kind, n);
                ++failures;
            }
        }
}

int main(void) {
    for (int t = 0; t < 60; ++t) {
        const int W = 1 + (int)(next_u32() % 12), H = 1 + (int)(next_u32() % 12);
        const int k = 3 + 2 * (int)(next_u32() % 4);
        const int bytes = 1 + (int)(next_u32() % 2);
        const int passes = 1 + (int)(next_u32() % 3);
        const int alphabet = (int)(next_u32() % 3) == 0 ? 0 : 2 + (int)(next_u32() % 4);
        check_fnr_case(W, H, bytes, k, passes, alphabet, (int)(next_u32() % 3));
    }
    check_fnr_case(40, 33, 2, 17, 1, 0, 1);
    check_fnr_case(35, 31, 1, 31, 1, 5, 0);
    check_fnr_case(31, 31, 2, 25, 2, 0, 2);
    check_mask_paths();
    check_introsort();
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("ok\n");
    return 0;
}
