/*
 * maxsq.h -- C ABI of libmaxsq: maximal all-ones square detection in binary matrices on
 * AMD Instinct MI355X (gfx950).
 *
 * Problem (Bhandari, "An Efficient Frequency-Based Approach for Maximal Square Detection in
 * Binary Matrices", Section 1): find the largest contiguous square submatrix made only of
 * ones.  The per-cell quantity is the side of the largest all-ones square whose
 * bottom-right corner is that cell, i.e. the dp table of Section 2.1 eq. (1):
 *     dp[i][j] = A[i][j] ? 1 + min(dp[i-1][j], dp[i][j-1], dp[i-1][j-1]) : 0,
 * with dp = 0 outside the matrix.  S = max dp; the area Algorithm 1 returns is S * S.
 * Among the cells with dp == S this library reports the first one in row-major order.
 * An empty matrix (m == 0 or n == 0) or an all-zero one gives S = 0 (Algorithm 1's early
 * return) and the corner (-1, -1).
 *
 * Data layout
 *   uint8 input  : row-major, row stride ld_bytes >= n; a cell is 1 iff its byte != 0.
 *   packed input : row-major uint64 words, row stride ld_words >= ceil(n / 64); column j is
 *                  bit (j & 63) of word (j >> 6), least significant bit first.  Padding bits
 *                  (columns >= n) and padding words are ignored; they may hold anything.
 *   dp map       : int32, row-major, row stride ld_dp >= n (elements).
 *
 * Ownership and memory: every buffer argument is caller-owned device memory (a result may
 * also be pinned host memory from hipHostMalloc).  The library never frees or keeps a caller
 * pointer after the enqueued work completes.  A context owns only its device scratch (sized
 * to the largest matrix it has seen) and its tuning table.  For matrices with min(m, n) > 1024
 * the scratch includes the boundary words of the strip sweep (the pass for squares too wide
 * for the windowed ones): 16 bytes per 128 columns and row, as much as the packed matrix.  If
 * they cannot be allocated, such squares are finished by one wave instead (slower, same
 * result).
 *
 * Streams: every call enqueues its kernels on `stream` (a hipStream_t; NULL = the null
 * stream) and returns without waiting; results are valid once that stream has reached the
 * call.  A context's scratch is reused by every call on it, so calls on one context must be
 * ordered on one stream (or externally serialised); use one context per concurrent stream.
 *
 * Errors: arguments are validated before any HIP call, so MS_ERR_INVALID_ARGUMENT is
 * returned without touching the device.  A failed launch or allocation returns MS_ERR_HIP or
 * MS_ERR_OUT_OF_MEMORY.  No call aborts or throws across the ABI.
 *
 * Context: `ctx` may be NULL in every call below except ms_max_square_noalloc; the library
 * then uses a default context for the current HIP device, created on first use.
 */
#ifndef MAXSQ_H
#define MAXSQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ms_ctx ms_ctx;

typedef enum {
    MS_OK = 0,
    MS_ERR_INVALID_ARGUMENT = 1,
    MS_ERR_WORKSPACE_TOO_SMALL = 2,
    MS_ERR_OUT_OF_MEMORY = 3,
    MS_ERR_HIP = 4,
    MS_ERR_UNSUPPORTED = 5
} ms_status;

/* Result: side S and the row-major-first bottom-right corner (row, col) among the cells whose
 * dp equals S; row = col = -1 when S == 0.  The top-left corner is (row - S + 1, col - S + 1). */
typedef struct {
    int64_t side, row, col;
} ms_square;

/* One matrix of a batch: packed bits in device memory, m x n, row stride ld_words. */
typedef struct {
    const uint64_t *bits;
    int64_t m, n, ld_words;
} ms_matrix;

/* Tunable launch shapes of one context (see ms_candidate / ms_set_config).
 *   probe_variant : register tile of the erosion search: 0 = 16 rows per lane, sides up to 16
 *                   certified per tile; 1 = 32 rows, 16; 2 = 32 rows, 32; 3 = 32 rows, 64
 *                   (fewer owned rows per tile, for images whose squares mostly exceed 32)
 *   map_cols      : columns per lane of the dp-map pass (4 or 8)
 *   map_band_rows : minimum row-band height of the dp-map pass (the band is also >= 4 S)
 * All candidates compute identical results; they differ only in speed. */
typedef struct {
    int32_t probe_variant;
    int32_t map_cols;
    int32_t map_band_rows;
} ms_config;

/* Create / destroy a context bound to HIP device `hip_device` (-1 = the current device). */
ms_status ms_create(ms_ctx **ctx, int hip_device);
ms_status ms_destroy(ms_ctx *ctx);
const char *ms_status_string(ms_status s);

/*
 * Bit-pack a uint8 matrix (the input encoding step of the hot path): d_bits[i][j >> 6] bit
 * (j & 63) = (d_a[i * ld_bytes + j] != 0).  Writes words 0 .. ceil(n/64) - 1 of every row,
 * with zero padding bits; words beyond that are left untouched.
 * Invalid: m or n < 0; d_a or d_bits NULL with m * n > 0; ld_bytes < n;
 * ld_words < ceil(n/64); m * n overflowing int64.
 */
ms_status ms_pack_u8(ms_ctx *ctx, const uint8_t *d_a, int64_t m, int64_t n, int64_t ld_bytes,
                     uint64_t *d_bits, int64_t ld_words, void *stream);

/*
 * Largest all-ones square of a packed matrix (Section 1's problem; the quantity that the
 * paper's Algorithm 1 computes, as the side rather than the area).  Writes one ms_square to
 * d_out (device or pinned host memory).
 * Invalid: m or n < 0; d_bits NULL with m * n > 0; d_out NULL; ld_words < ceil(n/64);
 * m * n >= 2^44.  MS_ERR_UNSUPPORTED when min(m, n) >= 2^20: the side and the corner travel
 * through the device as one 64-bit key (20 bits of side, 44 of position), so sides must stay
 * below 2^20.  The same limits apply to every call below that takes a packed matrix (each
 * descriptor of a batch included).
 */
ms_status ms_max_square(ms_ctx *ctx, const uint64_t *d_bits, int64_t m, int64_t n,
                        int64_t ld_words, ms_square *d_out, void *stream);

/*
 * ms_max_square for callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): the same search and the same result, but the call
 * allocates nothing, neither device nor host memory.  Its scratch is one fixed array of the
 * library per GPU (4 MiB + 256 bytes), held from the library's load until the process ends;
 * ms_create, the set-up call, finds that array's address on the context's device.
 *   ctx      : required (not NULL), from ms_create; its device and tuning table are used.
 *   sizes    : n <= 262144 (4096 words per row) and at most 2^21 probe tiles (about 1e11
 *              cells at the default tiles); larger matrices return MS_ERR_WORKSPACE_TOO_SMALL
 *              before any HIP call.
 * Every call on one GPU shares that GPU's array: calls that overlap on the device (different
 * streams, or different contexts on the same GPU) race and must be serialised by the caller.
 * The array keeps the last call's state; the search returns its header to zero at the end of
 * every call, and the first call on a device, or a call after a failed launch, clears it with
 * a small kernel first.
 * Invalid: as ms_max_square, plus ctx NULL.
 */
ms_status ms_max_square_noalloc(ms_ctx *ctx, const uint64_t *d_bits, int64_t m, int64_t n,
                                int64_t ld_words, ms_square *d_out, void *stream);

/*
 * Full dp map of Section 2.1 eq. (1) into d_dp (int32, row stride ld_dp elements), plus the
 * largest square into d_out when d_out is not NULL.  Every cell of the m x n map is written;
 * elements between n and ld_dp are left untouched.
 * Invalid: as ms_max_square, plus d_dp NULL with m * n > 0, ld_dp < n, m * ld_dp overflow.
 */
ms_status ms_square_map(ms_ctx *ctx, const uint64_t *d_bits, int64_t m, int64_t n,
                        int64_t ld_words, int32_t *d_dp, int64_t ld_dp, ms_square *d_out,
                        void *stream);

/*
 * The same dp map when the largest square of this matrix is already on the device: d_max
 * (device or pinned host memory) must hold the ms_square that ms_max_square wrote for the same
 * d_bits, m, n; only its side is read, and it sets the bands' and windows' head start, so a
 * smaller side than the true one gives a wrong map.  Saves the search when both are wanted.
 * When d_max is the very result buffer of the last search run on this context (ms_max_square
 * or ms_square_map, same d_bits, m, n, ld_words, no other search on the context since), that
 * search's per-tile bounds are still in the context and the map sizes its halos by region, as
 * ms_square_map does; otherwise every band and window starts S rows / columns early.
 * Invalid: as ms_square_map, plus d_max NULL.
 */
ms_status ms_square_map_from_max(ms_ctx *ctx, const uint64_t *d_bits, int64_t m, int64_t n,
                                 int64_t ld_words, const ms_square *d_max, int32_t *d_dp,
                                 int64_t ld_dp, void *stream);

/*
 * Many matrices in one go.  h_mats is a host copy of the `count` descriptors whose device
 * copy is d_mats; results go to d_out[0 .. count-1] in the same order.  The tiles of all
 * matrices are spread over one probe launch.  The tile total and a fingerprint of every
 * descriptor's (index, m, n, ld_words) are computed on the host from h_mats and checked on the
 * device against d_mats; when the two copies disagree, every result is side -1 instead of a
 * search (the Python binding raises).
 * Submission: the first call with a given (d_mats, count, d_out, d_workspace, shapes, probe
 * variant) enqueues its launches one by one; a repeat of it is captured once into a HIP graph
 * (at most 8 kept per context) and replayed from then on, one submission per call.  A stream
 * under capture by the caller always gets the launches themselves.  See ms_set_batched_graphs
 * (and the MAXSQ_GRAPH environment variable) to turn the graphs off or capture at once.
 * The caller provides the workspace (size from ms_batched_workspace_size with the same
 * descriptors; that size fits every probe variant); the library keeps no pointer to it after
 * the work completes.
 * Invalid: count < 0; any descriptor invalid as in ms_max_square; NULL pointers with
 * count > 0.  MS_ERR_WORKSPACE_TOO_SMALL if workspace_bytes is below the required size.
 */
ms_status ms_batched_workspace_size(ms_ctx *ctx, const ms_matrix *h_mats, int64_t count,
                                    size_t *bytes);
ms_status ms_max_square_batched(ms_ctx *ctx, const ms_matrix *h_mats, const ms_matrix *d_mats,
                                int64_t count, ms_square *d_out, void *d_workspace,
                                size_t workspace_bytes, void *stream);

/*
 * All maximal squares (the paper's conclusion: the method identifies every maximal square, not
 * only its side).  d_max is the device result of ms_max_square on the same bits (side S).
 * Writes the positions i * n + j of every cell whose side-map value equals S -- the bottom-right
 * corners of all S x S all-ones squares -- in row-major order: the first min(count, capacity) of
 * them to d_pos (int64), and the full count to *d_count (device int64).  S = 0 (or an empty
 * matrix) gives count 0; a square wider than 3008 columns gives count -1 (not supported).
 * d_workspace of ms_all_max_squares_workspace_size(m, n) bytes is caller-owned scratch.
 * Invalid: as ms_max_square, plus capacity < 0, d_pos NULL with capacity > 0, d_count or (for
 * m * n > 0) d_max NULL.
 */
ms_status ms_all_max_squares_workspace_size(ms_ctx *ctx, int64_t m, int64_t n, size_t *bytes);
ms_status ms_all_max_squares(ms_ctx *ctx, const uint64_t *d_bits, int64_t m, int64_t n,
                             int64_t ld_words, const ms_square *d_max, int64_t *d_pos,
                             int64_t capacity, int64_t *d_count, void *d_workspace,
                             size_t workspace_bytes, void *stream);

/*
 * Largest all-ones rectangle: the extension to maximal rectangles that the paper proposes as
 * future work (Section 6), in the histogram form of its related work (Section 2.3): with
 * H[i][j] the height of the run of ones ending at (i, j), the widest rectangle of height h
 * whose bottom row is i spans the longest run of columns with H[i][j] >= h.
 * Writes one ms_rect to d_out (device or pinned host memory): the largest area; among the
 * rectangles reaching it, the bottom-right corner (row, col) first in row-major order, then
 * the smallest height; height x width = area.  An empty or all-zero matrix gives
 * {0, -1, -1, 0, 0}.  Rows up to 32768 columns (ceil(n / 64) <= 512 words); wider rows give
 * MS_ERR_UNSUPPORTED.  Uses the context's scratch (one header and a record per wave, allocated
 * on first use).
 * Invalid: as ms_max_square.
 */
typedef struct {
    int64_t area, row, col, height, width;
} ms_rect;
ms_status ms_max_rectangle(ms_ctx *ctx, const uint64_t *d_bits, int64_t m, int64_t n,
                           int64_t ld_words, ms_rect *d_out, void *stream);

/*
 * Largest all-ones cube of a binary volume: the generalization to higher dimensions that the
 * paper proposes as future work (Section 6).  The volume is D planes of M rows of N columns,
 * packed like a matrix: row y of plane z is ld_words words starting at word
 * (z * M + y) * ld_words (column x = bit x & 63 of word x >> 6).  The side map generalizes
 * eq. (1) of Section 2.1 to seven neighbours: c = A ? 1 + min over the voxels that precede
 * (z, y, x) by 0 or 1 along each axis (not all 0) : 0.
 * Writes one ms_cube to d_out (device or pinned host memory): S = max c and the far corner
 * (largest z, y, x) of a largest cube, the first in (z, y, x) order; {0, -1, -1, -1} when there
 * is none.  d_workspace of ms_max_cube_workspace_size(D, M, N) bytes is caller-owned (three
 * packed volumes and a control block).  This call BLOCKS: the search over the side is steered
 * on the device (a kernel after each probe picks the next one), and the host synchronises
 * `stream` once per round of eight probes (about 2 log2 S probes in all) to learn whether it
 * is done; d_out is written on the device.
 * Invalid: negative sizes, ld_words < ceil(N / 64), NULL bits (with cells), NULL d_out, NULL
 * workspace (with cells), D * M * N >= 2^44.  MS_ERR_WORKSPACE_TOO_SMALL as usual;
 * MS_ERR_UNSUPPORTED when D * M * ceil(N / 64) >= 2^32.
 */
typedef struct {
    int64_t side, z, y, x;
} ms_cube;
ms_status ms_max_cube_workspace_size(ms_ctx *ctx, int64_t D, int64_t M, int64_t N,
                                     size_t *bytes);
ms_status ms_max_cube(ms_ctx *ctx, const uint64_t *d_bits, int64_t D, int64_t M, int64_t N,
                      int64_t ld_words, ms_cube *d_out, void *d_workspace,
                      size_t workspace_bytes, void *stream);

/* Autotuning.  ms_num_candidates / ms_candidate enumerate the launch shapes the library can
 * run; ms_set_config forces one (NULL restores tuned/default choices); ms_get_config reports
 * the shape that would be used for an m x n matrix.  ms_autotune times every candidate on the
 * caller's packed matrix (blocking: it synchronises `stream`) and records the fastest for
 * that matrix's shape bucket; ms_autotune_save / ms_autotune_load persist the table as text.
 */
int ms_num_candidates(void);
ms_status ms_candidate(int index, ms_config *cfg);
ms_status ms_set_config(ms_ctx *ctx, const ms_config *cfg);
ms_status ms_get_config(ms_ctx *ctx, int64_t m, int64_t n, ms_config *cfg);
ms_status ms_autotune(ms_ctx *ctx, const uint64_t *d_bits, int64_t m, int64_t n,
                      int64_t ld_words, int32_t *d_dp_scratch, int64_t ld_dp, void *stream);
/* ms_autotune_batched times every probe variant on the caller's batch (same arguments as
 * ms_max_square_batched, whose results it leaves in d_out; blocking) and records the fastest
 * for later batched calls on this context. */
ms_status ms_autotune_batched(ms_ctx *ctx, const ms_matrix *h_mats, const ms_matrix *d_mats,
                              int64_t count, ms_square *d_out, void *d_workspace,
                              size_t workspace_bytes, void *stream);
ms_status ms_autotune_save(ms_ctx *ctx, const char *path);
ms_status ms_autotune_load(ms_ctx *ctx, const char *path);

/* How ms_max_square_batched submits its launches on this context: MS_GRAPHS_ON_REPEAT (the
 * default: a repeated batch is captured once into a HIP graph and replayed), MS_GRAPHS_OFF
 * (launches enqueued one by one: a serving loop whose batches rarely repeat, where a capture
 * or a graph eviction would land in a request's latency) or MS_GRAPHS_ALWAYS (captured on the
 * first call).  The environment variable MAXSQ_GRAPH, when set to 0 or 1, overrides it.
 * Invalid: a mode outside these three. */
enum { MS_GRAPHS_OFF = 0, MS_GRAPHS_ON_REPEAT = 1, MS_GRAPHS_ALWAYS = 2 };
ms_status ms_set_batched_graphs(ms_ctx *ctx, int mode);

#ifdef __cplusplus
}
#endif

#endif /* MAXSQ_H */
