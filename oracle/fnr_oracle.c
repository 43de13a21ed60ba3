/*
 * fnr_oracle.c -- CPU oracle of the Fast Noise Reduction (FNR) filter.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file: it exists so that tests, the smoke check and the CPU timing leg of
 * the benchmark can compare the GPU kernels against a plain, slow, obviously
 * correct statement of the method.  It shares no code, header, table or helper
 * with the GPU library.
 *
 * What it computes (Gupta, Beg, Niranjan, "A Novel Approach to Fast Image
 * Filtering Algorithm of Infrared Images based on Intro Sort Algorithm"):
 *
 *   Section 3.3  S_xy is the k x k set of grey levels around (x, y), centre
 *                included; x is the horizontal and y the vertical coordinate.
 *   Eq. 3a/3b    g_max and g_min are the largest and smallest grey level in S_xy.
 *   Step 2       p(x, y) is noisy when g(x, y) equals g_min or g_max, and a
 *                signal pixel otherwise.
 *   Section 3.4  a noisy pixel is replaced by the median grey level g_m of S_xy;
 *                signal pixels are left alone.  The median is found by sorting
 *                S_xy with introsort (Eq. 4: quicksort that switches to heapsort
 *                once the recursion depth passes a bound that grows with the
 *                number of elements).
 *   Section 4    the filter may be applied to the whole image more than once
 *                (Fig. 5-6 use two passes); Table 1 counts one window scan for
 *                every pixel of the frame, borders included.
 *
 * Readings where the paper is silent (each listed in the design notes):
 *   - border: window coordinates are clamped to the frame (replicate edge);
 *   - passes: every pass reads an unchanged copy of the previous pass' output;
 *   - "Arg max / Arg min" in Eq. 3a/3b are read as the max / min values;
 *   - ties count: equality with either extreme flags the pixel;
 *   - k is odd, n = k*k, and g_m is element (n-1)/2 of S_xy sorted ascending;
 *   - introsort parameters (unstated): median-of-three pivot, depth bound
 *     2*floor(log2 n), insertion sort for ranges of at most 16 elements;
 *   - u16 frames are compared as full 16-bit values, whatever range they hold.
 *
 * Pixels are read into uint32_t working arrays so one code path serves both
 * pixel types; results are written back in the frame's own type.
 */

#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef uint32_t px_t;

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-2)

/* Counters a test can read back to see which branches of introsort ran. */
typedef struct {
    uint64_t scans;       /* windows scanned for g_min / g_max (Eq. 3a/3b) */
    uint64_t sorts;       /* introsort calls */
    uint64_t partitions;  /* quicksort partition steps */
    uint64_t heapsorts;   /* ranges handed to heapsort (depth bound reached) */
    uint64_t insertions;  /* ranges finished by insertion sort */
} oracle_sort_stats;

/* ------------------------------------------------------------------------- */
/* Introsort (Section 3.4, Eq. 4).                                           */
/* ------------------------------------------------------------------------- */

#define INSERTION_RANGE 16

static void swap_px(px_t *a, px_t *b) { px_t t = *a; *a = *b; *b = t; }

static void insertion_sort(px_t *a, int n) {
    for (int i = 1; i < n; ++i) {
        px_t v = a[i];
        int j = i - 1;
        while (j >= 0 && a[j] > v) {
            a[j + 1] = a[j];
            --j;
        }
        a[j + 1] = v;
    }
}

/* Max-heap on a[0..n): restore the heap property below `root`. */
static void sift_down(px_t *a, int root, int n) {
    for (;;) {
        int child = 2 * root + 1;
        if (child >= n) return;
        if (child + 1 < n && a[child + 1] > a[child]) child = child + 1;
        if (a[root] >= a[child]) return;
        swap_px(&a[root], &a[child]);
        root = child;
    }
}

static void heap_sort(px_t *a, int n) {
    for (int i = n / 2 - 1; i >= 0; --i) sift_down(a, i, n);
    for (int end = n - 1; end > 0; --end) {
        swap_px(&a[0], &a[end]); /* largest remaining goes to the back */
        sift_down(a, 0, end);
    }
}

static px_t median_of_three(px_t a, px_t b, px_t c) {
    if (a < b) {
        if (b < c) return b;
        return a < c ? c : a;
    }
    if (a < c) return a;
    return b < c ? c : b;
}

/*
 * Hoare partition of a[0..n) around a pivot value taken from the range.
 * Returns `cut` with every a[i] <= pivot for i < cut and every a[i] >= pivot for
 * i >= cut.  Both scans are bounds-checked: speed is not the point here.
 */
static int partition(px_t *a, int n, px_t pivot) {
    int i = 0, j = n - 1;
    for (;;) {
        while (i < n && a[i] < pivot) ++i;
        while (j >= 0 && a[j] > pivot) --j;
        if (i >= j) return i;
        swap_px(&a[i], &a[j]);
        ++i;
        --j;
    }
}

static int floor_log2(int n) {
    int l = 0;
    while (n > 1) {
        n >>= 1;
        ++l;
    }
    return l;
}

static void introsort_range(px_t *a, int n, int depth, oracle_sort_stats *st) {
    while (n > INSERTION_RANGE) {
        if (depth == 0) {
            /* recursion too deep for this many elements: heapsort the rest */
            if (st) st->heapsorts++;
            heap_sort(a, n);
            return;
        }
        --depth;
        px_t pivot = median_of_three(a[0], a[n / 2], a[n - 1]);
        int cut = partition(a, n, pivot);
        if (st) st->partitions++;
        if (cut <= 0 || cut >= n) {
            /* Cannot happen with a pivot drawn from the range; fall back to a
               sort that needs no pivot rather than loop forever. */
            heap_sort(a, n);
            return;
        }
        introsort_range(a + cut, n - cut, depth, st); /* upper part */
        n = cut;                                      /* loop on the lower part */
    }
    if (st) st->insertions++;
    insertion_sort(a, n);
}

/* Sort a[0..n) ascending with an explicit depth bound (tests force 0 to
   exercise the heapsort branch alone). */
void oracle_introsort_depth(px_t *a, int n, int depth_limit, oracle_sort_stats *st) {
    if (st) st->sorts++;
    if (n > 1) introsort_range(a, n, depth_limit, st);
}

/* Introsort with the depth bound 2*floor(log2 n). */
void oracle_introsort(px_t *a, int n, oracle_sort_stats *st) {
    oracle_introsort_depth(a, n, n > 1 ? 2 * floor_log2(n) : 0, st);
}

/* ------------------------------------------------------------------------- */
/* Frames, windows and the two steps of the method.                          */
/* ------------------------------------------------------------------------- */

static int clamp_int(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

static int check_frame(const void *p, size_t pitch, int W, int H, int bytes) {
    if (!p) return ORACLE_EINVAL;
    if (W < 1 || H < 1) return ORACLE_EINVAL;
    if (bytes != 1 && bytes != 2) return ORACLE_EINVAL;
    if (pitch < (size_t)W * (size_t)bytes) return ORACLE_EINVAL;
    return ORACLE_OK;
}

static int check_window(int k) { return (k >= 1 && (k & 1)) ? ORACLE_OK : ORACLE_EINVAL; }

static void read_frame(const void *src, size_t pitch, int W, int H, int bytes, px_t *A) {
    const unsigned char *base = (const unsigned char *)src;
    for (int y = 0; y < H; ++y) {
        const unsigned char *row = base + (size_t)y * pitch;
        for (int x = 0; x < W; ++x) {
            if (bytes == 1) {
                A[(size_t)y * W + x] = row[x];
            } else {
                uint16_t v;
                memcpy(&v, row + 2 * (size_t)x, 2);
                A[(size_t)y * W + x] = v;
            }
        }
    }
}

static void write_frame(const px_t *A, int W, int H, int bytes, void *dst, size_t pitch) {
    unsigned char *base = (unsigned char *)dst;
    for (int y = 0; y < H; ++y) {
        unsigned char *row = base + (size_t)y * pitch;
        for (int x = 0; x < W; ++x) {
            px_t v = A[(size_t)y * W + x];
            if (bytes == 1) {
                row[x] = (unsigned char)v;
            } else {
                uint16_t s = (uint16_t)v;
                memcpy(row + 2 * (size_t)x, &s, 2);
            }
        }
    }
}

/*
 * S_xy of Section 3.3, listed row by row (y-r .. y+r) and, inside a row, from
 * x-r to x+r -- the order of the paper's 3x3 example.  Positions outside the
 * frame take the value of the nearest edge pixel.
 */
static void gather_window(const px_t *A, int W, int H, int x, int y, int k, px_t *S) {
    int r = (k - 1) / 2, m = 0;
    for (int j = -r; j <= r; ++j) {
        int yy = clamp_int(y + j, 0, H - 1);
        for (int i = -r; i <= r; ++i) {
            int xx = clamp_int(x + i, 0, W - 1);
            S[m++] = A[(size_t)yy * W + xx];
        }
    }
}

/* Eq. 3a/3b then Step 2: is the centre grey level one of the window's extremes? */
static int is_noisy(const px_t *S, int n, px_t centre) {
    px_t gmax = S[0], gmin = S[0];
    for (int i = 1; i < n; ++i) {
        if (S[i] > gmax) gmax = S[i];
        if (S[i] < gmin) gmin = S[i];
    }
    return centre == gmin || centre == gmax;
}

/* Section 3.4: g_m, the middle element of S_xy after sorting it. */
static px_t window_median(px_t *S, int n, oracle_sort_stats *st) {
    oracle_introsort(S, n, st);
    return S[(n - 1) / 2];
}

enum { MODE_DETECT = 0, MODE_MEDIAN = 1, MODE_FNR = 2 };

/*
 * One whole-frame pass.  Every pixel, borders included, reads its window from
 * A; results go to B, so no pixel of this pass sees another's output.
 *   MODE_DETECT: mask_out[y][x] = 1 for a noisy pixel, 0 otherwise.
 *   MODE_MEDIAN: B = g_m where mask_in is non-zero (everywhere if mask_in is
 *                NULL, the standard median filter of Section 2), else A.
 *   MODE_FNR:    B = g_m at noisy pixels, A elsewhere.
 * Returns the number of windows sorted (noisy pixels in MODE_DETECT).
 */
static uint64_t frame_pass(const px_t *A, px_t *B, int W, int H, int k, int mode,
                           const uint8_t *mask_in, size_t mask_in_pitch,
                           uint8_t *mask_out, size_t mask_out_pitch,
                           px_t *S, oracle_sort_stats *st) {
    int n = k * k;
    uint64_t count = 0;
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            px_t c = A[(size_t)y * W + x];
            gather_window(A, W, H, x, y, k, S);
            int replace;
            if (mode == MODE_MEDIAN)
                replace = mask_in ? (mask_in[(size_t)y * mask_in_pitch + x] != 0) : 1;
            else {
                replace = is_noisy(S, n, c);
                if (st) st->scans++;
            }
            if (mode == MODE_DETECT) {
                mask_out[(size_t)y * mask_out_pitch + x] = (uint8_t)replace;
                count += (uint64_t)replace;
                continue;
            }
            if (replace) {
                B[(size_t)y * W + x] = window_median(S, n, st);
                count++;
            } else {
                B[(size_t)y * W + x] = c;
            }
        }
    }
    return count;
}

/* ------------------------------------------------------------------------- */
/* Entry points for the test harness (host buffers; pitch in bytes;          */
/* bytes = 1 for uint8 frames, 2 for uint16 frames).                         */
/* ------------------------------------------------------------------------- */

/* Writes S_xy of pixel (x, y) into S (k*k values, paper order). */
int oracle_window(const void *src, size_t pitch, int W, int H, int bytes, int k, int x, int y,
                  uint32_t *S) {
    if (check_frame(src, pitch, W, H, bytes) || check_window(k) || !S) return ORACLE_EINVAL;
    if (x < 0 || x >= W || y < 0 || y >= H) return ORACLE_EINVAL;
    px_t *A = (px_t *)malloc(sizeof(px_t) * (size_t)W * H);
    if (!A) return ORACLE_ENOMEM;
    read_frame(src, pitch, W, H, bytes, A);
    gather_window(A, W, H, x, y, k, S);
    free(A);
    return ORACLE_OK;
}

/* Noise detection (Section 3.3) of every pixel: mask 1 = noisy, 0 = signal. */
int oracle_detect(const void *src, size_t src_pitch, uint8_t *mask, size_t mask_pitch, int W,
                  int H, int bytes, int k, uint64_t *count) {
    if (check_frame(src, src_pitch, W, H, bytes) || check_window(k)) return ORACLE_EINVAL;
    if (!mask || mask_pitch < (size_t)W) return ORACLE_EINVAL;
    px_t *A = (px_t *)malloc(sizeof(px_t) * (size_t)W * H);
    px_t *S = (px_t *)malloc(sizeof(px_t) * (size_t)k * k);
    if (!A || !S) {
        free(A);
        free(S);
        return ORACLE_ENOMEM;
    }
    read_frame(src, src_pitch, W, H, bytes, A);
    uint64_t c = frame_pass(A, NULL, W, H, k, MODE_DETECT, NULL, 0, mask, mask_pitch, S, NULL);
    if (count) *count = c;
    free(A);
    free(S);
    return ORACLE_OK;
}

/* Median replacement (Section 3.4) where mask != 0, or at every pixel when
   mask is NULL (the standard median filter).  Pixels outside the mask are
   copied.  `sorts` (nullable) receives the number of windows sorted. */
int oracle_median(const void *src, size_t src_pitch, const uint8_t *mask, size_t mask_pitch,
                  void *dst, size_t dst_pitch, int W, int H, int bytes, int k, uint64_t *sorts,
                  oracle_sort_stats *st) {
    if (check_frame(src, src_pitch, W, H, bytes) || check_frame(dst, dst_pitch, W, H, bytes) ||
        check_window(k))
        return ORACLE_EINVAL;
    if (mask && mask_pitch < (size_t)W) return ORACLE_EINVAL;
    px_t *A = (px_t *)malloc(sizeof(px_t) * (size_t)W * H);
    px_t *B = (px_t *)malloc(sizeof(px_t) * (size_t)W * H);
    px_t *S = (px_t *)malloc(sizeof(px_t) * (size_t)k * k);
    if (!A || !B || !S) {
        free(A);
        free(B);
        free(S);
        return ORACLE_ENOMEM;
    }
    read_frame(src, src_pitch, W, H, bytes, A);
    uint64_t c = frame_pass(A, B, W, H, k, MODE_MEDIAN, mask, mask_pitch, NULL, 0, S, st);
    write_frame(B, W, H, bytes, dst, dst_pitch);
    if (sorts) *sorts = c;
    free(A);
    free(B);
    free(S);
    return ORACLE_OK;
}

/* The whole FNR method, `passes` times over the frame.  counts (nullable)
   receives the number of noisy pixels found in each pass. */
int oracle_fnr(const void *src, size_t src_pitch, void *dst, size_t dst_pitch, int W, int H,
               int bytes, int k, int passes, uint64_t *counts, oracle_sort_stats *st) {
    if (check_frame(src, src_pitch, W, H, bytes) || check_frame(dst, dst_pitch, W, H, bytes) ||
        check_window(k) || passes < 1)
        return ORACLE_EINVAL;
    px_t *A = (px_t *)malloc(sizeof(px_t) * (size_t)W * H);
    px_t *B = (px_t *)malloc(sizeof(px_t) * (size_t)W * H);
    px_t *S = (px_t *)malloc(sizeof(px_t) * (size_t)k * k);
    if (!A || !B || !S) {
        free(A);
        free(B);
        free(S);
        return ORACLE_ENOMEM;
    }
    read_frame(src, src_pitch, W, H, bytes, A);
    for (int p = 0; p < passes; ++p) {
        uint64_t c = frame_pass(A, B, W, H, k, MODE_FNR, NULL, 0, NULL, 0, S, st);
        if (counts) counts[p] = c;
        px_t *t = A; /* the output of this pass is the snapshot the next one reads */
        A = B;
        B = t;
    }
    write_frame(A, W, H, bytes, dst, dst_pitch);
    free(A);
    free(B);
    free(S);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------- */
/* Directional detector (opt-in; a reading of Fig. 1's caption).             */
/* ------------------------------------------------------------------------- */
/*
 * Section 3 argues that the grey level of a signal pixel varies monotonically
 * along the object's surface while an impulse cannot, and the caption of
 * Fig. 1 (the figure itself is missing) compares the central pixel with its two
 * neighbours in the 3 x 3 window.  Reading taken here: the four lines through
 * the centre of the 3 x 3 S_xy are the row, the column and the two diagonals;
 * the centre is monotone along a line when its grey level lies between the two
 * neighbours on that line (min <= g(x, y) <= max, ties included), and the pixel
 * is noisy when it is monotone along none of the four.  Neighbours outside the
 * frame are clamped as everywhere else.  The paper does not fix this rule: only
 * the min/max detector above is the paper's.
 */
static int between(px_t c, px_t a, px_t b) {
    px_t lo = a < b ? a : b, hi = a < b ? b : a;
    return lo <= c && c <= hi;
}

int oracle_detect_directional(const void *src, size_t src_pitch, uint8_t *mask, size_t mask_pitch,
                              int W, int H, int bytes, uint64_t *count) {
    if (check_frame(src, src_pitch, W, H, bytes)) return ORACLE_EINVAL;
    if (!mask || mask_pitch < (size_t)W) return ORACLE_EINVAL;
    px_t *A = (px_t *)malloc(sizeof(px_t) * (size_t)W * H);
    if (!A) return ORACLE_ENOMEM;
    read_frame(src, src_pitch, W, H, bytes, A);
    px_t S[9]; /* S_xy of the 3 x 3 window in the paper's listing order */
    uint64_t c = 0;
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            gather_window(A, W, H, x, y, 3, S);
            const px_t g = S[4];
            /* row (S[3], S[5]), column (S[1], S[7]), diagonal (S[0], S[8]),
               anti-diagonal (S[2], S[6]) */
            const int monotone = between(g, S[3], S[5]) || between(g, S[1], S[7]) ||
                                 between(g, S[0], S[8]) || between(g, S[2], S[6]);
            mask[(size_t)y * mask_pitch + x] = monotone ? 0 : 1;
            c += monotone ? 0 : 1;
        }
    }
    if (count) *count = c;
    free(A);
    return ORACLE_OK;
}
