/*
 * Host-side argument validation of the C ABI under AddressSanitizer and
 * UndefinedBehaviorSanitizer: every call below must be answered on the host, before any HIP
 * call, with the documented status (invalid arguments, sizes beyond the result key's fields,
 * workspace sizes of valid descriptors, tuning candidates).  No GPU is needed or touched.
 * Exit status: the number of calls that returned something unexpected.
 */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "../../include/maxsq.h"

static int failures = 0;

static void expect(const char *what, ms_status got, ms_status want) {
    if (got != want) {
        fprintf(stderr, "%s: status %d, expected %d\n", what, (int)got, (int)want);
        ++failures;
    }
}

int main(void) {
    uint64_t word = 0;
    const uint64_t *B = &word;  /* never dereferenced by these calls */
    ms_square sq;
    int32_t dp1 = 0;
    uint8_t byte = 0;
    const int64_t BIG = INT64_MAX, HUGE_SIDE = (int64_t)1 << 20;
    size_t bytes = 0;

    for (int s = 0; s <= 6; ++s) {
        const char *t = ms_status_string((ms_status)s);
        if (!t || !t[0]) ++failures;
    }
    if (strcmp(ms_status_string((ms_status)99), "unknown status") != 0) ++failures;

    /* ms_max_square / noalloc / map: sizes, strides, pointers, overflow, the 20-bit side */
    expect("max m<0", ms_max_square(NULL, B, -1, 5, 1, &sq, NULL), MS_ERR_INVALID_ARGUMENT);
    expect("max n<0", ms_max_square(NULL, B, 5, -1, 1, &sq, NULL), MS_ERR_INVALID_ARGUMENT);
    expect("max null bits", ms_max_square(NULL, NULL, 5, 5, 1, &sq, NULL),
           MS_ERR_INVALID_ARGUMENT);
    expect("max short ld", ms_max_square(NULL, B, 5, 130, 2, &sq, NULL),
           MS_ERR_INVALID_ARGUMENT);
    expect("max null out", ms_max_square(NULL, B, 5, 5, 1, NULL, NULL),
           MS_ERR_INVALID_ARGUMENT);
    expect("max m*n overflow", ms_max_square(NULL, B, BIG, BIG, BIG, &sq, NULL),
           MS_ERR_INVALID_ARGUMENT);
    expect("max m*n >= 2^44", ms_max_square(NULL, B, (int64_t)1 << 22, (int64_t)1 << 22,
                                            (int64_t)1 << 16, &sq, NULL),
           MS_ERR_INVALID_ARGUMENT);
    expect("max m*ld overflow", ms_max_square(NULL, B, (int64_t)1 << 40, 2, BIG, &sq, NULL),
           MS_ERR_INVALID_ARGUMENT);
    expect("max side field", ms_max_square(NULL, B, HUGE_SIDE, HUGE_SIDE, HUGE_SIDE / 64, &sq,
                                           NULL),
           MS_ERR_UNSUPPORTED);
    expect("noalloc null ctx", ms_max_square_noalloc(NULL, B, 5, 5, 1, &sq, NULL),
           MS_ERR_INVALID_ARGUMENT);
    expect("noalloc m<0", ms_max_square_noalloc(NULL, B, -5, 5, 1, &sq, NULL),
           MS_ERR_INVALID_ARGUMENT);
    expect("map null dp", ms_square_map(NULL, B, 5, 5, 1, NULL, 5, &sq, NULL),
           MS_ERR_INVALID_ARGUMENT);
    expect("map short ld_dp", ms_square_map(NULL, B, 5, 5, 1, &dp1, 4, &sq, NULL),
           MS_ERR_INVALID_ARGUMENT);
    expect("map m*ld_dp overflow", ms_square_map(NULL, B, (int64_t)1 << 40, 2, 1, &dp1, BIG,
                                                 &sq, NULL),
           MS_ERR_INVALID_ARGUMENT);
    expect("from_max null max", ms_square_map_from_max(NULL, B, 5, 5, 1, NULL, &dp1, 5, NULL),
           MS_ERR_INVALID_ARGUMENT);
    expect("from_max neg ld_dp", ms_square_map_from_max(NULL, B, 5, 5, 1, &sq, &dp1, -1, NULL),
           MS_ERR_INVALID_ARGUMENT);

    /* ms_pack_u8 */
    expect("pack null in", ms_pack_u8(NULL, NULL, 5, 5, 5, &word, 1, NULL),
           MS_ERR_INVALID_ARGUMENT);
    expect("pack short ld_bytes", ms_pack_u8(NULL, &byte, 5, 5, 4, &word, 1, NULL),
           MS_ERR_INVALID_ARGUMENT);
    expect("pack overflow", ms_pack_u8(NULL, &byte, BIG, BIG, BIG, &word, BIG, NULL),
           MS_ERR_INVALID_ARGUMENT);

    /* batched: the workspace query over valid descriptors, and invalid ones */
    ms_matrix mats[4] = {{B, 100, 200, 4}, {B, 0, 7, 1}, {B, 4096, 4096, 64}, {B, 1, 1, 1}};
    expect("batched ws", ms_batched_workspace_size(NULL, mats, 4, &bytes), MS_OK);
    if (bytes == 0) ++failures;
    expect("batched ws count<0", ms_batched_workspace_size(NULL, mats, -1, &bytes),
           MS_ERR_INVALID_ARGUMENT);
    ms_matrix bad[2] = {{B, 10, 10, 1}, {B, 10, 130, 2}};
    expect("batched ws bad desc", ms_batched_workspace_size(NULL, bad, 2, &bytes),
           MS_ERR_INVALID_ARGUMENT);
    ms_matrix wide[1] = {{B, HUGE_SIDE, HUGE_SIDE, HUGE_SIDE / 64}};
    expect("batched ws side field", ms_batched_workspace_size(NULL, wide, 1, &bytes),
           MS_ERR_UNSUPPORTED);
    expect("batched null out", ms_max_square_batched(NULL, mats, mats, 4, NULL, &word, 8, NULL),
           MS_ERR_INVALID_ARGUMENT);
    expect("batched count 0", ms_max_square_batched(NULL, NULL, NULL, 0, NULL, NULL, 0, NULL),
           MS_OK);

    /* all maximal squares, rectangle, cube */
    expect("allmax ws", ms_all_max_squares_workspace_size(NULL, 1000, 3000, &bytes), MS_OK);
    expect("allmax ws overflow", ms_all_max_squares_workspace_size(NULL, BIG, BIG, &bytes),
           MS_ERR_INVALID_ARGUMENT);
    int64_t count = 0;
    expect("allmax neg cap", ms_all_max_squares(NULL, B, 5, 5, 1, &sq, NULL, -1, &count, &word,
                                                8, NULL),
           MS_ERR_INVALID_ARGUMENT);
    ms_rect rect;
    expect("rect too wide", ms_max_rectangle(NULL, B, 2, 40000, 626, &rect, NULL),
           MS_ERR_UNSUPPORTED);
    expect("cube ws", ms_max_cube_workspace_size(NULL, 64, 64, 100, &bytes), MS_OK);
    expect("cube ws overflow", ms_max_cube_workspace_size(NULL, BIG, BIG, BIG, &bytes),
           MS_ERR_INVALID_ARGUMENT);
    ms_cube cube;
    expect("cube short ld", ms_max_cube(NULL, B, 4, 4, 130, 2, &cube, &word, 8, NULL),
           MS_ERR_INVALID_ARGUMENT);

    /* tuning candidates */
    const int nc = ms_num_candidates();
    for (int i = 0; i < nc; ++i) {
        ms_config c;
        expect("candidate", ms_candidate(i, &c), MS_OK);
    }
    ms_config c;
    expect("candidate past end", ms_candidate(nc, &c), MS_ERR_INVALID_ARGUMENT);
    expect("candidate null", ms_candidate(0, NULL), MS_ERR_INVALID_ARGUMENT);
    expect("graph mode -1", ms_set_batched_graphs(NULL, -1), MS_ERR_INVALID_ARGUMENT);
    expect("graph mode 3", ms_set_batched_graphs(NULL, 3), MS_ERR_INVALID_ARGUMENT);
    expect("autotune save null", ms_autotune_save(NULL, "x"), MS_ERR_INVALID_ARGUMENT);
    expect("destroy null", ms_destroy(NULL), MS_ERR_INVALID_ARGUMENT);

    if (failures) fprintf(stderr, "%d unexpected statuses\n", failures);
    else printf("abi_check: all statuses as documented\n");
    return failures;
}
