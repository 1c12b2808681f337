// launch.hpp -- host-side launchers of the libmaxsq kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/maxsq.h"

namespace mshost {

// Device scratch of a context (single-matrix calls).  The key and flag return to zero at the
// end of every call, so the scratch needs clearing only once, when it is allocated.
struct ScratchHeader {
    unsigned long long key;     // running best (side, position) key
    uint32_t serial_flag;       // a square was too wide for the resolve pass
    uint32_t nsat;              // saturated tiles found by the probe
    ms_square result;           // last result (read by the map pass)
    // epoch << 32 | waves of the resolve pass that have finished.  The epoch counts searches and
    // sweeping maps and tags the strip words; sharing the word, every wave's completion count
    // returns it with no read of its own.
    unsigned long long done_epoch;
    // Bounding box of the probe tiles whose largest side may exceed the narrow map's region
    // halo (bound above REGION_SMALL, or saturated), as {2^30 - first tile row, last tile row
    // + 1, 2^30 - first tile column, last tile column + 1}, all zero when there is none: each
    // probe block stores the box of its tiles (BOX_RECORD_WORDS words), and the wave that
    // writes the result folds those records into big_box for the map.
    uint32_t big_box[4];
    uint64_t pad1[8];
    // Second 128-byte line: the strip sweep (squares too wide for the windowed passes; see
    // strip_words_needed), apart from the words above that every wave of a search hits with
    // atomics (a per-wave read of the epoch in that line measured 25 % slower searches).
    unsigned long long skey;    // the sweep's best (side, position) key
    unsigned long long tick;    // strip tickets: epoch << 32 | tickets taken in that launch
    uint32_t pad4;
    uint32_t fin;               // search: the last arrival and the last strip, each counted once
    uint32_t sdone;             // search: strips finished
    uint32_t timeout;           // epoch + 1 of a launch whose strip wait gave up (a search
                                // then reports failure)
    // Where the strip words are (0: none) and how many, and a forced batch height (0: the
    // kernels choose).  Written by the host's set-up kernel whenever the words or the header are
    // (re)initialised, so the search reads them from here rather than from its arguments.
    unsigned long long strips_ptr;
    int64_t strip_cap;
    int32_t strip_rows_forced;
    int32_t pad2;
    uint64_t pad3[9];
};
static_assert(sizeof(ScratchHeader) == 256, "header layout: two 128-byte lines");
static_assert(offsetof(ScratchHeader, skey) == 128, "strip fields start the second line");

// Erosion tile variants compiled into the library.
struct ProbeVariant {
    int rpl;  // rows per lane
    int kc;   // largest side certified by the tile's halo
};
constexpr int NUM_PROBE_VARIANTS = 4;
extern const ProbeVariant PROBE_VARIANTS[NUM_PROBE_VARIANTS];

int64_t probe_tile_rows(int variant);           // owned rows per tile
constexpr int64_t PROBE_TILE_WORDS = 15;        // owned words per tile

struct LaunchEnv {
    int num_cus;
    hipStream_t stream;
};

hipError_t launch_pack_u8(const LaunchEnv &env, const uint8_t *a, int64_t m, int64_t n,
                          int64_t ldb, uint64_t *bits, int64_t ldw);

// Per-block records of the probe's large-tile box: BOX_RECORD_WORDS uint32 per block (16-byte
// aligned), for at most max_probe_blocks(num_cus) blocks.
constexpr int BOX_RECORD_WORDS = 4;
int64_t max_probe_blocks(int num_cus);

// Largest square of one matrix; result into hdr->result and, if non-null, *out.  `sat` holds
// one byte per probe tile (max_probe_tiles(m, n) bytes cover every variant); `bounds` one int32
// per tile and `box_rec` the per-block box records, both filled for a map in the same call.
hipError_t launch_max_square(const LaunchEnv &env, int variant, const uint64_t *bits, int64_t m,
                             int64_t n, int64_t ldw, ScratchHeader *hdr, int32_t *serial_state,
                             uint8_t *sat, int32_t *bounds, uint32_t *box_rec, ms_square *out);
int64_t max_probe_tiles(int64_t m, int64_t n);

// Strip sweep: the recurrence over the whole matrix by many waves, for a square too wide for
// the windowed passes (map: S above 1984; search: a saturated tile's window beyond one word per
// lane).  Strips of STRIP_WORDS words; per (strip, row) two 64-bit boundary words, zeroed when
// allocated (the header's epoch tags them, so the header and the words are zeroed together).
// Needed only when min(m, n) > STRIP_MIN_SIDE; bnd == nullptr keeps the one-wave sweep.
constexpr int STRIP_WORDS = 2;
constexpr int64_t STRIP_MIN_SIDE = 1024;
// Rows per strip batch: 0 lets the kernels choose; 1..64 forces it (MAXSQ_STRIP_ROWS).
int strip_rows_setting();
int64_t strip_words_needed(int64_t m, int64_t n);
hipError_t launch_zero_u64(const LaunchEnv &env, uint64_t *p, int64_t count);
// Record the strip words (may be null) and the forced batch height in the header.
hipError_t launch_set_strips(const LaunchEnv &env, ScratchHeader *hdr, uint64_t *words,
                             int64_t count, int forced_rows);
// The map's narrow pass shortens its row bands (and narrows its window) until it has at least
// this many items per SIMD (4 SIMDs per CU), or reaches its shortest band.
constexpr int MAP_ITEMS_PER_SIMD = 2;

// Per-tile bounds of the search that ran in the same call, for a map split by tile class.
struct MapRegions {
    const int32_t *bounds;     // one per probe tile: an upper bound on its largest side, or -1
    int64_t tile_rows;         // the probe variant's owned rows per tile
    int64_t tile_ntx;          // tiles per tile row
    const uint32_t *big_box;   // ScratchHeader::big_box of that search
};

// dp map of one matrix; reads S from *maxsq on the device (a largest-square result).  With
// `regions`, the halos follow the per-tile bounds (see k_dpmap).
hipError_t launch_square_map(const LaunchEnv &env, int map_cols, int band_rows,
                             const uint64_t *bits, int64_t m, int64_t n, int64_t ldw, int32_t *dp,
                             int64_t ld_dp, const ms_square *maxsq, int32_t *serial_state,
                             const MapRegions *regions = nullptr, ScratchHeader *hdr = nullptr,
                             uint64_t *bnd = nullptr, int strip_rows = 0);

// Write a constant result (empty matrices).
// Zero a context header of `bytes` (a multiple of 4, at most 256) on env.stream.
hipError_t launch_zero_header(const LaunchEnv &env, void *p, size_t bytes);
hipError_t launch_write_result(const LaunchEnv &env, ms_square *out, ScratchHeader *hdr,
                               int64_t count);

// Largest square without any allocation: the scratch is a fixed device array of the library
// (one copy per GPU), laid out as a 256-byte header region | serial-pass state for
// NOALLOC_MAX_WORDS words per row | NOALLOC_MAX_TILES saturation bytes.
constexpr int64_t NOALLOC_MAX_WORDS = 4096;                   // n <= 262144
constexpr int64_t NOALLOC_MAX_TILES = int64_t(1) << 21;       // max_probe_tiles(m, n) bound
constexpr int64_t NOALLOC_STATE_BYTES = NOALLOC_MAX_WORDS * 64 * 2 * 4;
constexpr int64_t NOALLOC_SCRATCH_BYTES = 256 + NOALLOC_STATE_BYTES + NOALLOC_MAX_TILES;
constexpr int NOALLOC_MAX_DEVICES = 64;
// Once per device, with that device current: find the device address of the array.
hipError_t noalloc_setup(int device);
// Enqueue the search on the array of `device` (set up before); clears the header first when
// an earlier call on that device may have left it dirty.
hipError_t launch_max_square_noalloc(const LaunchEnv &env, int device, int variant,
                                     const uint64_t *bits, int64_t m, int64_t n, int64_t ldw,
                                     ms_square *out);

// Batched: workspace layout and launches.
struct BatchLayout {
    // byte offsets in the workspace: per-matrix keys, tile starts within an init block, flags;
    // per-init-block totals and starts; counters, serial-pass state, saturation bytes; the size
    size_t keys, local, parts, offsets, counters, serial_state, flags, sat, total;
    int64_t nblk;  // init blocks (at least one)
    uint64_t total_tiles;
    int64_t max_nwords;
    uint64_t shape_mix;  // fingerprint of every (i, m, n, ld_words), checked on the device
    int narrow_q;        // tile-width weight (see msk::narrow_tiles); -1 for a size bound
};
// Tile-width weights the batched autotuner tries (the first is the default).
constexpr int NUM_NARROW_WEIGHTS = 4;
extern const int NARROW_WEIGHTS[NUM_NARROW_WEIGHTS];
bool narrow_weight_valid(int q);
// Layout for probe variant `variant` and tile-width weight q; with q = -1 the sizes bound every
// variant and weight (the workspace size of the batched entry point).
BatchLayout batch_layout(int variant, int q, const ms_matrix *h_mats, int64_t count);
hipError_t launch_batched(const LaunchEnv &env, int variant, const ms_matrix *d_mats,
                          int64_t count, ms_square *out, void *ws, const BatchLayout &L);

// All maximal squares: workspace layout and launches.
struct AllMaxLayout {
    int64_t nux, entries;
    size_t counts, offsets, chunks, total;  // byte offsets in the workspace, and its size
};
AllMaxLayout all_max_layout(int64_t m, int64_t n);
hipError_t launch_all_max(const LaunchEnv &env, const uint64_t *bits, int64_t m, int64_t n,
                          int64_t ldw, const ms_square *maxsq, int64_t *pos, int64_t capacity,
                          int64_t *count, void *ws);


// Largest all-ones rectangle (rect.hip).  The scratch is a header followed by one record per
// block of the launch (rect_max_blocks records); the header returns to zero at the end of every
// call, so it needs clearing only when allocated.
struct RectScratch {
    unsigned long long best_area;  // largest area any finished row has reached (pruning bound)
    uint64_t pad[7];
};
static_assert(sizeof(RectScratch) == 64, "rect header layout");
struct RectRecord {
    int64_t area, pos, height;     // a block's best: area, i * n + col of its corner, height
};
constexpr int RECT_BLOCKS_PER_CU = 8;
constexpr int64_t RECT_MAX_WORDS = 512;  // widest row: 64 lanes x 8 words (32768 columns)
int64_t rect_max_blocks(int num_cus);
hipError_t launch_max_rect(const LaunchEnv &env, const uint64_t *bits, int64_t m, int64_t n,
                           int64_t ldw, RectScratch *rs, ms_rect *out);


// Largest all-ones cube (cube.hip).  The workspace holds a 256-byte control block and three
// volumes of D x M x ceil(n / 64) words; cube_volume(ws, .., k) is volume k (k < 3).
// The search state lives on the device: a one-thread control kernel after each probe reads the
// probe's first set voxel and decides the next shift (gallop, then bisection), so the host only
// reads the phase once per round of probes.
enum { CUBE_INIT = 0, CUBE_GALLOP = 1, CUBE_BISECT = 2, CUBE_DONE = 3 };
struct CubeControl {
    unsigned long long first;  // smallest z * M * n + y * n + x of a set voxel (~0: empty)
    unsigned long long fa;     // the same for E_a, the largest non-empty E so far
    int64_t a, b;              // E_a is in volume cur; the probe in flight builds E_{a+b} in nxt
    int64_t failed, limit, bstep, smax;  // bisection: the side is in [a, limit]
    int32_t phase, cur, nxt, pad;
};
static_assert(sizeof(CubeControl) <= 256, "cube control block");
size_t cube_workspace_bytes(int64_t D, int64_t M, int64_t n);
uint64_t *cube_volume(void *ws, int64_t D, int64_t M, int64_t n, int k);
// E_1: the input (row stride lds words) copied into dst (row stride ceil(n / 64)) with its padding
// cleared; lowers ctl->first to its first set voxel (cube_begin cleared it).
hipError_t launch_cube_copy(const LaunchEnv &env, const uint64_t *src, int64_t lds,
                            uint64_t *dst, int64_t D, int64_t M, int64_t n, CubeControl *ctl);
// The search on the device: cube_begin sets the state up (before the copy pass of the input
// into volume 0), cube_control advances it after a pass and writes *out once it is done, and
// cube_probe runs the next probe (E_{a+b} from E_a, volumes from the state) unless it is done.
hipError_t launch_cube_begin(const LaunchEnv &env, CubeControl *ctl, int64_t smax);
hipError_t launch_cube_control(const LaunchEnv &env, CubeControl *ctl, ms_cube *out, int64_t M,
                               int64_t n);
hipError_t launch_cube_probe(const LaunchEnv &env, uint64_t *const V[3], int64_t D, int64_t M,
                             int64_t n, CubeControl *ctl);

} // namespace mshost
