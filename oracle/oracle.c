/*
 * oracle.c -- plain, slow, obviously correct CPU reference for maximal all-ones square
 * detection.  TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
 * baseline may call it; the product path never does.  It shares no code with the HIP
 * library (its own cell readers, its own packer/unpacker, its own loops).
 *
 * What it computes (paper, Section 1 and Section 2.1 eq. (1)):
 *   dp[i][j] = 0                                              if A[i][j] = 0
 *   dp[i][j] = 1 + min(dp[i-1][j], dp[i][j-1], dp[i-1][j-1])  if A[i][j] = 1
 * with dp = 0 outside the matrix (the paper leaves the zero case and the border implicit;
 * this is the reading that makes dp[i][j] "the side of the largest square ending at that
 * cell", Section 1).  S = max dp (0 for an empty or all-zero matrix, Algorithm 1's early
 * return), and the reported square is the first cell in row-major order with dp == S,
 * i.e. its bottom-right corner; (-1, -1) when S == 0.  The area is S * S (Algorithm 1's
 * return value).
 *
 * Two evaluation modes (Section 2.1): the full O(mn) table, and the space-optimised one
 * that keeps only the previous row (O(n) memory), used for very large matrices and for
 * streaming rows out chunk by chunk.
 *
 * Also here, as a second witness: the paper's frequency-based method (Section 3), written
 * from its description, with a record of where the best side was last raised.
 *
 * And the largest all-ones rectangle (the extension of Section 6's future work, in the
 * histogram form of Section 2.3), by its plain definition; see max_rect below.  And the largest
 * all-ones cube of a binary volume (Section 6's higher dimensions); see oracle_max_cube_packed.
 *
 * Inputs: uint8 row-major (a cell is 1 iff its byte is non-zero), or packed uint64 rows where
 * column j is bit (j & 63) of word (j >> 6), padding bits ignored.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL 1
#define ORACLE_ENOMEM 3

/* ---- cell readers (the oracle's own) ---- */
static int cell_u8(const uint8_t *a, int64_t ld, int64_t i, int64_t j) {
    return a[i * ld + j] != 0;
}

static int cell_packed(const uint64_t *bits, int64_t ldw, int64_t i, int64_t j) {
    uint64_t word = bits[i * ldw + j / 64];
    return (int)((word >> (j % 64)) & 1u);
}

typedef struct {
    const uint8_t *u8;
    const uint64_t *packed;
    int64_t ld;
} reader;

static int cell(const reader *r, int64_t i, int64_t j) {
    return r->u8 ? cell_u8(r->u8, r->ld, i, j) : cell_packed(r->packed, r->ld, i, j);
}

static int32_t min3(int32_t a, int32_t b, int32_t c) {
    int32_t m = a < b ? a : b;
    return m < c ? m : c;
}

/* One dp row from the previous one: the recurrence of Section 2.1, eq. (1). */
static void dp_row(const reader *r, int64_t i, int64_t n, const int32_t *prev, int32_t *cur) {
    for (int64_t j = 0; j < n; ++j) {
        if (!cell(r, i, j)) {
            cur[j] = 0;
            continue;
        }
        int32_t up = (i > 0) ? prev[j] : 0;
        int32_t left = (j > 0) ? cur[j - 1] : 0;
        int32_t diag = (i > 0 && j > 0) ? prev[j - 1] : 0;
        cur[j] = 1 + min3(up, left, diag);
    }
}

/* Keep the first row-major maximum: update only on a strict increase. */
static void track(const int32_t *row, int64_t i, int64_t n, int64_t res[3]) {
    for (int64_t j = 0; j < n; ++j) {
        if (row[j] > res[0]) {
            res[0] = row[j];
            res[1] = i;
            res[2] = j;
        }
    }
}

static int check_dims(int64_t m, int64_t n, int64_t ld, int64_t min_ld, const void *p) {
    if (m < 0 || n < 0) return ORACLE_EINVAL;
    if (m > 0 && n > 0 && (p == NULL || ld < min_ld)) return ORACLE_EINVAL;
    return ORACLE_OK;
}

/* Space-optimised evaluation (two rolling rows).  res = {S, row, col}. */
static int max_square(const reader *r, int64_t m, int64_t n, int64_t res[3]) {
    res[0] = 0;
    res[1] = -1;
    res[2] = -1;
    if (m == 0 || n == 0) return ORACLE_OK;
    int32_t *prev = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    int32_t *cur = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    if (!prev || !cur) {
        free(prev);
        free(cur);
        return ORACLE_ENOMEM;
    }
    for (int64_t i = 0; i < m; ++i) {
        dp_row(r, i, n, prev, cur);
        track(cur, i, n, res);
        int32_t *t = prev;
        prev = cur;
        cur = t;
    }
    free(prev);
    free(cur);
    return ORACLE_OK;
}

int oracle_max_square_u8(const uint8_t *a, int64_t m, int64_t n, int64_t ld, int64_t res[3]) {
    int e = check_dims(m, n, ld, n, a);
    if (e) return e;
    reader r = {a, NULL, ld};
    return max_square(&r, m, n, res);
}

int oracle_max_square_packed(const uint64_t *bits, int64_t m, int64_t n, int64_t ld_words,
                             int64_t res[3]) {
    int e = check_dims(m, n, ld_words, (n + 63) / 64, bits);
    if (e) return e;
    reader r = {NULL, bits, ld_words};
    return max_square(&r, m, n, res);
}

/* Full table: writes every dp row into dp (row stride ld_dp) and returns {S, row, col}. */
static int square_map(const reader *r, int64_t m, int64_t n, int32_t *dp, int64_t ld_dp,
                      int64_t res[3]) {
    res[0] = 0;
    res[1] = -1;
    res[2] = -1;
    if (m == 0 || n == 0) return ORACLE_OK;
    if (dp == NULL || ld_dp < n) return ORACLE_EINVAL;
    int32_t *zero = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    if (!zero) return ORACLE_ENOMEM;
    for (int64_t i = 0; i < m; ++i) {
        const int32_t *prev = (i > 0) ? dp + (i - 1) * ld_dp : zero;
        dp_row(r, i, n, prev, dp + i * ld_dp);
        track(dp + i * ld_dp, i, n, res);
    }
    free(zero);
    return ORACLE_OK;
}

int oracle_square_map_u8(const uint8_t *a, int64_t m, int64_t n, int64_t ld, int32_t *dp,
                         int64_t ld_dp, int64_t res[3]) {
    int e = check_dims(m, n, ld, n, a);
    if (e) return e;
    reader r = {a, NULL, ld};
    return square_map(&r, m, n, dp, ld_dp, res);
}

int oracle_square_map_packed(const uint64_t *bits, int64_t m, int64_t n, int64_t ld_words,
                             int32_t *dp, int64_t ld_dp, int64_t res[3]) {
    int e = check_dims(m, n, ld_words, (n + 63) / 64, bits);
    if (e) return e;
    reader r = {NULL, bits, ld_words};
    return square_map(&r, m, n, dp, ld_dp, res);
}

/* ---- streaming mode: hand out dp rows chunk by chunk, O(n) state ---- */
typedef struct {
    reader r;
    int64_t m, n, next_row;
    int32_t *prev;
    int64_t res[3];
} oracle_stream;

oracle_stream *oracle_stream_open_packed(const uint64_t *bits, int64_t m, int64_t n,
                                         int64_t ld_words) {
    if (check_dims(m, n, ld_words, (n + 63) / 64, bits)) return NULL;
    oracle_stream *s = (oracle_stream *)calloc(1, sizeof(oracle_stream));
    if (!s) return NULL;
    s->r.u8 = NULL;
    s->r.packed = bits;
    s->r.ld = ld_words;
    s->m = m;
    s->n = n;
    s->next_row = 0;
    s->prev = (int32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    s->res[0] = 0;
    s->res[1] = -1;
    s->res[2] = -1;
    if (!s->prev) {
        free(s);
        return NULL;
    }
    return s;
}

/* Compute the next `rows` dp rows into out (row stride ld_out); returns rows produced. */
int64_t oracle_stream_next(oracle_stream *s, int64_t rows, int32_t *out, int64_t ld_out) {
    int64_t done = 0;
    while (done < rows && s->next_row < s->m) {
        int32_t *cur = out + done * ld_out;
        dp_row(&s->r, s->next_row, s->n, s->prev, cur);
        track(cur, s->next_row, s->n, s->res);
        memcpy(s->prev, cur, (size_t)s->n * sizeof(int32_t));
        ++s->next_row;
        ++done;
    }
    return done;
}

void oracle_stream_result(const oracle_stream *s, int64_t res[3]) {
    res[0] = s->res[0];
    res[1] = s->res[1];
    res[2] = s->res[2];
}

void oracle_stream_close(oracle_stream *s) {
    if (s) {
        free(s->prev);
        free(s);
    }
}

/* ---- the oracle's own packer and unpacker (encoding above) ---- */
int oracle_pack_u8(const uint8_t *a, int64_t m, int64_t n, int64_t ld, uint64_t *bits,
                   int64_t ld_words) {
    int e = check_dims(m, n, ld, n, a);
    if (e) return e;
    if (m > 0 && n > 0 && (bits == NULL || ld_words < (n + 63) / 64)) return ORACLE_EINVAL;
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t w = 0; w < (n + 63) / 64; ++w) bits[i * ld_words + w] = 0;
        for (int64_t j = 0; j < n; ++j)
            if (cell_u8(a, ld, i, j)) bits[i * ld_words + j / 64] |= (uint64_t)1 << (j % 64);
    }
    return ORACLE_OK;
}

int oracle_unpack(const uint64_t *bits, int64_t m, int64_t n, int64_t ld_words, uint8_t *a,
                  int64_t ld) {
    int e = check_dims(m, n, ld_words, (n + 63) / 64, bits);
    if (e) return e;
    if (m > 0 && n > 0 && (a == NULL || ld < n)) return ORACLE_EINVAL;
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) a[i * ld + j] = (uint8_t)cell_packed(bits, ld_words, i, j);
    return ORACLE_OK;
}

/*
 * ---- second witness: the frequency-based method of Section 3 ----
 * Written from the method's description, in this file's own structure.  h[j] is the
 * frequency array: the number of consecutive ones ending at the current row in column j.
 * `best` is the largest side confirmed so far, and the only side worth looking for in the
 * next row is k = best + 1 (the method's dynamic threshold): a square of side k ending in
 * row i needs k consecutive columns whose heights all reach k.  Each row is handled in two
 * sweeps: the heights of the whole row are brought up to date first, then the row is walked
 * once, counting the run of consecutive columns with h >= k; the first column where that
 * run reaches k confirms side k there.  No second confirmation can happen in the same row,
 * since a side can grow by at most one per row (dp[i][j] <= dp[i-1][j-1] + 1), so the walk
 * stops at the first one.  Test additions: res = {best, row, col} with (row, col) the cell
 * where best was last raised, and row_trace[i] (nullable) = best after row i.  Returns the
 * side, not the area.
 */
int oracle_freq_alg1_u8(const uint8_t *a, int64_t m, int64_t n, int64_t ld, int64_t res[3],
                        int64_t *row_trace) {
    res[0] = 0;
    res[1] = -1;
    res[2] = -1;
    int e = check_dims(m, n, ld, n, a);
    if (e) return e;
    if (m == 0 || n == 0) return ORACLE_OK;
    int64_t *h = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    if (!h) return ORACLE_ENOMEM;
    int64_t best = 0;
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = 0; j < n; ++j) h[j] = cell_u8(a, ld, i, j) ? h[j] + 1 : 0;
        const int64_t k = best + 1;
        int64_t run = 0;
        for (int64_t j = 0; j < n; ++j) {
            run = h[j] >= k ? run + 1 : 0;
            if (run == k) {
                best = k;
                res[1] = i;
                res[2] = j;
                break;
            }
        }
        if (row_trace) row_trace[i] = best;
    }
    res[0] = best;
    free(h);
    return ORACLE_OK;
}

/*
 * ---- every m x n matrix at once (tiny shapes) ----
 * Matrix number `mask` has A[i][j] = bit (i*n + j) of mask.  For each mask the full dp of
 * Section 2.1 eq. (1) is evaluated and S and the row-major-first corner (as i*n + j, or -1)
 * are recorded.  m*n <= 26.
 */
int oracle_all_masks(int m, int n, int64_t *side, int64_t *corner) {
    if (m <= 0 || n <= 0 || m * n > 26) return ORACLE_EINVAL;
    int32_t dp[26];
    uint64_t count = (uint64_t)1 << (m * n);
    for (uint64_t mask = 0; mask < count; ++mask) {
        int64_t best = 0, at = -1;
        for (int i = 0; i < m; ++i) {
            for (int j = 0; j < n; ++j) {
                int k = i * n + j;
                if (!((mask >> k) & 1u)) {
                    dp[k] = 0;
                    continue;
                }
                int32_t up = i > 0 ? dp[k - n] : 0;
                int32_t left = j > 0 ? dp[k - 1] : 0;
                int32_t diag = (i > 0 && j > 0) ? dp[k - n - 1] : 0;
                dp[k] = 1 + min3(up, left, diag);
                if (dp[k] > best) {
                    best = dp[k];
                    at = k;
                }
            }
        }
        side[mask] = best;
        corner[mask] = at;
    }
    return ORACLE_OK;
}

/*
 * ---- largest all-ones rectangle ----
 * The extension the paper lists in its future work (Section 6), in the formulation its related
 * work describes (Section 2.3): each row becomes a histogram of the heights of the runs of ones
 * ending in it, H[i][j] = A[i][j] ? H[i-1][j] + 1 : 0.
 *
 * Plain definition.  A rectangle is rows i-h+1..i and columns j-w+1..j, all ones; its area is
 * h * w.  For bottom-right corner (i, j) and height h the widest such rectangle has
 * w = W_h(i, j), the number of consecutive columns ending at j whose height in row i is at least
 * h; so the largest area is the maximum of h * W_h(i, j) over every cell (i, j) and every
 * 1 <= h <= H[i][j].  Reported: that area; among the rectangles reaching it, the bottom-right
 * corner first in row-major order, then the smallest height.  res = {area, row, col, height,
 * width}; an empty or all-zero matrix gives {0, -1, -1, 0, 0}.
 *
 * Evaluation: rows top to bottom; per row, columns left to right, keeping W_h for every h up to
 * the row's tallest height; candidates are visited in (row, col, height) order and only a
 * strictly larger area replaces the best, which yields the tie-break above.
 */
static int max_rect(const reader *r, int64_t m, int64_t n, int64_t res[5]) {
    res[0] = 0;
    res[1] = -1;
    res[2] = -1;
    res[3] = 0;
    res[4] = 0;
    if (m == 0 || n == 0) return ORACLE_OK;
    int64_t *H = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    int64_t *W = (int64_t *)calloc((size_t)m + 1, sizeof(int64_t)); /* W[h], h = 1..m */
    if (!H || !W) {
        free(H);
        free(W);
        return ORACLE_ENOMEM;
    }
    for (int64_t i = 0; i < m; ++i) {
        int64_t hmax = 0;
        for (int64_t j = 0; j < n; ++j) {
            H[j] = cell(r, i, j) ? H[j] + 1 : 0;
            if (H[j] > hmax) hmax = H[j];
        }
        for (int64_t h = 1; h <= hmax; ++h) W[h] = 0;
        for (int64_t j = 0; j < n; ++j) {
            for (int64_t h = 1; h <= hmax; ++h) {
                W[h] = H[j] >= h ? W[h] + 1 : 0;
                if (h <= H[j] && h * W[h] > res[0]) {
                    res[0] = h * W[h];
                    res[1] = i;
                    res[2] = j;
                    res[3] = h;
                    res[4] = W[h];
                }
            }
        }
    }
    free(H);
    free(W);
    return ORACLE_OK;
}

int oracle_max_rect_u8(const uint8_t *a, int64_t m, int64_t n, int64_t ld, int64_t res[5]) {
    int rc = check_dims(m, n, ld, n, a);
    if (rc) return rc;
    reader r = {a, NULL, ld};
    return max_rect(&r, m, n, res);
}

int oracle_max_rect_packed(const uint64_t *bits, int64_t m, int64_t n, int64_t ld_words,
                           int64_t res[5]) {
    int rc = check_dims(m, n, ld_words, (n + 63) / 64, bits);
    if (rc) return rc;
    reader r = {NULL, bits, ld_words};
    return max_rect(&r, m, n, res);
}

/*
 * ---- largest all-ones cube (the higher-dimensional generalization of Section 6) ----
 * A binary volume A[z][y][x] of D planes of M rows of N columns.  The side map generalizes the
 * recurrence of Section 2.1 eq. (1) from the three neighbours of a cell in the plane to the
 * seven neighbours of a voxel that precede it along at least one axis:
 *     c[z][y][x] = 0                                        if A[z][y][x] = 0
 *     c[z][y][x] = 1 + min over (a, b, d) in {0,1}^3 \ {0} of c[z-a][y-b][x-d]   otherwise,
 * with c = 0 outside the volume; c is the side of the largest all-ones cube whose far corner
 * (largest z, y and x) is that voxel.  Reported: S = max c and the first far corner with c = S in
 * (z, y, x) lexicographic order; (0, -1, -1, -1) when S = 0.  Two rolling planes of c.
 * Input: packed planes, each M rows of ld_words words (column x = bit x & 63 of word x >> 6),
 * plane z starting at word z * M * ld_words.
 */
int oracle_max_cube_packed(const uint64_t *bits, int64_t D, int64_t M, int64_t N,
                           int64_t ld_words, int64_t res[4]) {
    res[0] = 0;
    res[1] = -1;
    res[2] = -1;
    res[3] = -1;
    if (D < 0 || M < 0 || N < 0) return ORACLE_EINVAL;
    if (D == 0 || M == 0 || N == 0) return ORACLE_OK;
    if (!bits || ld_words < (N + 63) / 64) return ORACLE_EINVAL;
    int32_t *prev = (int32_t *)calloc((size_t)(M * N), sizeof(int32_t));
    int32_t *cur = (int32_t *)calloc((size_t)(M * N), sizeof(int32_t));
    if (!prev || !cur) {
        free(prev);
        free(cur);
        return ORACLE_ENOMEM;
    }
    for (int64_t z = 0; z < D; ++z) {
        const uint64_t *plane = bits + z * M * ld_words;
        for (int64_t y = 0; y < M; ++y) {
            for (int64_t x = 0; x < N; ++x) {
                int32_t v = 0;
                if (cell_packed(plane, ld_words, y, x)) {
                    int32_t m = INT32_MAX;
                    for (int a = 0; a <= 1; ++a)
                        for (int b = 0; b <= 1; ++b)
                            for (int d = 0; d <= 1; ++d) {
                                if (a == 0 && b == 0 && d == 0) continue;
                                int32_t c = 0;
                                if (z - a >= 0 && y - b >= 0 && x - d >= 0)
                                    c = (a ? prev : cur)[(y - b) * N + (x - d)];
                                if (c < m) m = c;
                            }
                    v = 1 + m;
                }
                cur[y * N + x] = v;
                if (v > res[0]) {
                    res[0] = v;
                    res[1] = z;
                    res[2] = y;
                    res[3] = x;
                }
            }
        }
        int32_t *t = prev;
        prev = cur;
        cur = t;
    }
    free(prev);
    free(cur);
    return ORACLE_OK;
}
