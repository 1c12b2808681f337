/*
 * Every entry point of oracle.c under AddressSanitizer, UndefinedBehaviorSanitizer and
 * LeakSanitizer: random matrices of ragged shapes (0 to 200 rows, 0 to 200 columns, word
 * boundaries included) and densities, through the full table, the rolling rows, the
 * chunked stream, the packer and unpacker, the frequency method, every tiny matrix, the
 * largest rectangle and the largest cube, plus invalid arguments; and the outputs must agree
 * with one another.  Exit status: the number of disagreements (a sanitizer report aborts).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct oracle_stream oracle_stream;
int oracle_max_square_u8(const uint8_t *, int64_t, int64_t, int64_t, int64_t[3]);
int oracle_max_square_packed(const uint64_t *, int64_t, int64_t, int64_t, int64_t[3]);
int oracle_square_map_u8(const uint8_t *, int64_t, int64_t, int64_t, int32_t *, int64_t,
                         int64_t[3]);
int oracle_square_map_packed(const uint64_t *, int64_t, int64_t, int64_t, int32_t *, int64_t,
                             int64_t[3]);
oracle_stream *oracle_stream_open_packed(const uint64_t *, int64_t, int64_t, int64_t);
int64_t oracle_stream_next(oracle_stream *, int64_t, int32_t *, int64_t);
void oracle_stream_result(const oracle_stream *, int64_t[3]);
void oracle_stream_close(oracle_stream *);
int oracle_pack_u8(const uint8_t *, int64_t, int64_t, int64_t, uint64_t *, int64_t);
int oracle_unpack(const uint64_t *, int64_t, int64_t, int64_t, uint8_t *, int64_t);
int oracle_freq_alg1_u8(const uint8_t *, int64_t, int64_t, int64_t, int64_t[3], int64_t *);
int oracle_all_masks(int, int, int64_t *, int64_t *);
int oracle_max_rect_u8(const uint8_t *, int64_t, int64_t, int64_t, int64_t[5]);
int oracle_max_rect_packed(const uint64_t *, int64_t, int64_t, int64_t, int64_t[5]);
int oracle_max_cube_packed(const uint64_t *, int64_t, int64_t, int64_t, int64_t, int64_t[4]);

static uint64_t state = 0x9e3779b97f4a7c15ull;
static uint32_t rnd(void) {  /* xorshift64* */
    state ^= state >> 12;
    state ^= state << 25;
    state ^= state >> 27;
    return (uint32_t)((state * 0x2545f4914f6cdd1dull) >> 32);
}

static int failures = 0;
#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            fprintf(stderr, "line %d: %s\n", __LINE__, #c);             \
            ++failures;                                                 \
        }                                                               \
    } while (0)

static void one_matrix(int64_t m, int64_t n, uint32_t p_permille) {
    const int64_t ld = n + (rnd() % 3), ldw = (n + 63) / 64 + (rnd() % 2);
    uint8_t *a = malloc((size_t)(m * ld + 1));
    uint64_t *bits = malloc((size_t)(m * ldw + 1) * 8);
    uint8_t *back = malloc((size_t)(m * n + 1));
    int32_t *dp = malloc((size_t)(m * n + 1) * 4);
    int32_t *rows = malloc((size_t)(7 * n + 1) * 4);
    for (int64_t k = 0; k < m * ld; ++k) a[k] = (rnd() % 1000) < p_permille ? (uint8_t)(1 + rnd() % 255) : 0;
    int64_t r1[3], r2[3], r3[3], r4[3], r5[3], rect1[5], rect2[5];
    CHECK(oracle_max_square_u8(a, m, n, ld, r1) == 0);
    CHECK(oracle_square_map_u8(a, m, n, ld, dp, n, r2) == 0);
    CHECK(oracle_pack_u8(a, m, n, ld, bits, ldw) == 0);
    CHECK(oracle_unpack(bits, m, n, ldw, back, n) == 0);
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) CHECK(back[i * n + j] == (a[i * ld + j] != 0));
    CHECK(oracle_max_square_packed(bits, m, n, ldw, r3) == 0);
    int64_t *trace = malloc((size_t)(m + 1) * 8);
    CHECK(oracle_freq_alg1_u8(a, m, n, ld, r4, trace) == 0);
    CHECK(memcmp(r1, r2, sizeof r1) == 0 && memcmp(r1, r3, sizeof r1) == 0);
    CHECK(memcmp(r1, r4, sizeof r1) == 0);
    /* the stream hands out the same rows, 7 at a time */
    oracle_stream *s = oracle_stream_open_packed(bits, m, n, ldw);
    CHECK(s != NULL);
    if (s) {
        int64_t done = 0, got;
        while ((got = oracle_stream_next(s, 7, rows, n > 0 ? n : 1)) > 0) {
            for (int64_t r = 0; r < got; ++r)
                for (int64_t j = 0; j < n; ++j) CHECK(rows[r * n + j] == dp[(done + r) * n + j]);
            done += got;
        }
        CHECK(done == m || n == 0);
        oracle_stream_result(s, r5);
        CHECK(memcmp(r1, r5, sizeof r1) == 0);
        oracle_stream_close(s);
    }
    CHECK(oracle_max_rect_u8(a, m, n, ld, rect1) == 0);
    CHECK(oracle_max_rect_packed(bits, m, n, ldw, rect2) == 0);
    CHECK(memcmp(rect1, rect2, sizeof rect1) == 0);
    CHECK(rect1[0] >= r1[0] * r1[0]);
    free(a);
    free(bits);
    free(back);
    free(dp);
    free(rows);
    free(trace);
}

int main(void) {
    static const int64_t sides[] = {0, 1, 2, 3, 63, 64, 65, 127, 128, 129, 200};
    const int ns = (int)(sizeof sides / sizeof sides[0]);
    for (int x = 0; x < ns; ++x)
        for (int y = 0; y < ns; ++y)
            one_matrix(sides[x], sides[y], 100 + (uint32_t)(rnd() % 900));
    for (int k = 0; k < 60; ++k) one_matrix(rnd() % 150, rnd() % 150, 500 + rnd() % 500);

    /* every 3 x 4 matrix */
    int64_t side[4096], corner[4096];
    CHECK(oracle_all_masks(3, 4, side, corner) == 0);
    CHECK(side[4095] == 3 && side[0] == 0 && corner[0] == -1);

    /* cubes: ragged volumes, checked against a plane stacked on itself */
    for (int k = 0; k < 20; ++k) {
        const int64_t D = 1 + rnd() % 9, M = 1 + rnd() % 20, N = 1 + rnd() % 140;
        const int64_t ldw = (N + 63) / 64;
        uint64_t *vol = calloc((size_t)(D * M * ldw), 8);
        for (int64_t v = 0; v < D * M * ldw; ++v)
            vol[v] = ((uint64_t)rnd() << 32 | rnd()) | ((uint64_t)rnd() << 32 | rnd());
        int64_t res[4];
        CHECK(oracle_max_cube_packed(vol, D, M, N, ldw, res) == 0);
        CHECK(res[0] >= 0 && res[0] <= D && res[0] <= M && res[0] <= N);
        free(vol);
    }

    /* invalid arguments are refused, not dereferenced */
    int64_t r[3], r5v[5];
    CHECK(oracle_max_square_u8(NULL, 3, 3, 3, r) != 0);
    CHECK(oracle_max_square_u8(NULL, -1, 3, 3, r) != 0);
    CHECK(oracle_max_rect_u8(NULL, 3, 3, 2, r5v) != 0);
    CHECK(oracle_all_masks(6, 6, side, corner) != 0);
    CHECK(oracle_stream_open_packed(NULL, 3, 3, 1) == NULL);

    if (failures) fprintf(stderr, "%d disagreements\n", failures);
    else printf("oracle_check: every entry point consistent\n");
    return failures;
}
