// api.cpp -- the C ABI of libmaxsq: argument validation (before any HIP call), contexts and
// their device scratch, launch-shape selection and autotuning, and the batched graph cache.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/maxsq.h"
#include "launch.hpp"

namespace {

constexpr int64_t POS_LIMIT = int64_t(1) << 44;  // cells addressable by the result key
// Sides the result key holds: 64 - 44 = 20 bits.  A side is at most min(m, n), so matrices with
// min(m, n) below this limit always fit.
constexpr int64_t SIDE_LIMIT = int64_t(1) << 20;

// ceil(a / b) for a >= 0, b > 0, without forming a + b - 1 (a may be near INT64_MAX when an
// argument is being validated)
int64_t cdiv(int64_t a, int64_t b) { return a / b + (a % b != 0); }

bool mul_overflows(int64_t a, int64_t b) {
    return a > 0 && b > 0 && a > INT64_MAX / b;
}

const ms_config DEFAULT_CONFIG = {1, 4, 64};

// A captured batched launch sequence.  Its launch arguments (tile total, workspace layout)
// depend on the shapes, so the entry is keyed on a hash of every (m, n, ld_words) as well as
// on the buffers; the matrix pointers are read from the device descriptors at run time.
struct GraphEntry {
    const void *mats;
    int64_t count;
    const void *out;
    const void *ws;
    int variant;
    int narrow;  // tile-width weight
    uint64_t shape_hash;
    hipGraphExec_t exec;
};

// Identity of a batch's shapes for the graph cache: four independent multiply-xor lanes over
// (m, n, ld_words) words (a byte-wise hash costs a dependent multiply per byte, about 0.3 ms per
// 10000 descriptors, as long as the device needs for the whole search).
uint64_t shape_hash(const ms_matrix *h_mats, int64_t count) {
    uint64_t h[4] = {0x9E3779B97F4A7C15ull, 0xC2B2AE3D27D4EB4Full, 0x165667B19E3779F9ull,
                     0xD6E8FEB86659FD93ull};
    for (int64_t i = 0; i < count; ++i) {
        uint64_t &a = h[i & 3];
        a = (a ^ (uint64_t)h_mats[i].m) * 0xBF58476D1CE4E5B9ull;
        a = (a ^ (uint64_t)h_mats[i].n) * 0x94D049BB133111EBull;
        a = (a ^ (uint64_t)h_mats[i].ld_words) * 0xBF58476D1CE4E5B9ull;
    }
    uint64_t r = (uint64_t)count;
    for (int k = 0; k < 4; ++k) r = (r ^ h[k] ^ (h[k] >> 29)) * 0x94D049BB133111EBull;
    return r ^ (r >> 32);
}

}  // namespace

struct ms_ctx {
    int device = 0;
    int num_cus = 256;
    // single-matrix scratch: header | serial-pass state | one saturation byte per probe tile
    void *scratch = nullptr;
    int64_t state_words = 0;
    int64_t sat_bytes = 0;
    void *strips = nullptr;   // boundary words of the strip sweep (zeroed with the header)
    int64_t strip_words = 0;
    bool dirty = false;
    bool has_forced = false;
    ms_config forced{};
    int batched_variant = -1;  // from ms_autotune_batched (or a loaded table); -1: default
    int batched_narrow = -1;   // its tile-width weight; -1: the default weight
    int graph_mode = MS_GRAPHS_ON_REPEAT;  // ms_set_batched_graphs
    std::map<int, ms_config> tuned;
    std::vector<GraphEntry> graphs;
    std::vector<GraphEntry> seen;  // batches run once eagerly (exec unused): a repeat is captured
    hipStream_t capture_stream = nullptr;
    // largest-rectangle scratch: header | one record per block of the launch
    void *rect_scratch = nullptr;
    // pinned host words through which the cube search reads its device flags
    uint64_t *pinned = nullptr;
    bool rect_dirty = false;
    // The last search run on this context's scratch: its per-tile bounds and large-tile box
    // stay there until the next search, so a map of the same matrix that is handed this
    // search's result can size its halos by region (see ms_square_map_from_max).
    struct {
        const uint64_t *bits = nullptr;
        int64_t m = -1, n = -1, ldw = -1;
        const ms_square *out = nullptr;
        int variant = -1;
    } last;
    std::mutex mu;
};

namespace {

std::mutex g_default_mu;
std::map<int, ms_ctx *> g_default;

ms_status hip_status(hipError_t e) {
    if (e == hipSuccess) return MS_OK;
    if (e == hipErrorOutOfMemory) return MS_ERR_OUT_OF_MEMORY;
    return MS_ERR_HIP;
}

ms_status init_ctx(ms_ctx *c, int dev) {
    if (dev < 0) {
        if (hipGetDevice(&dev) != hipSuccess) return MS_ERR_HIP;
    }
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || dev >= count) return MS_ERR_HIP;
    c->device = dev;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return MS_ERR_HIP;
    c->num_cus = cus > 0 ? cus : 256;
    // set-up of the allocation-free search on this device (once per device), with the device
    // current; the caller's current device is restored
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return MS_ERR_HIP;
    if (prev != dev && hipSetDevice(dev) != hipSuccess) return MS_ERR_HIP;
    const hipError_t se = mshost::noalloc_setup(dev);
    if (prev != dev && hipSetDevice(prev) != hipSuccess) return MS_ERR_HIP;
    if (se != hipSuccess) return MS_ERR_HIP;
    return MS_OK;
}

ms_status resolve(ms_ctx *ctx, ms_ctx **out) {
    if (ctx) {
        *out = ctx;
        return MS_OK;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MS_ERR_HIP;
    std::lock_guard<std::mutex> lk(g_default_mu);
    auto it = g_default.find(dev);
    if (it != g_default.end()) {
        *out = it->second;
        return MS_OK;
    }
    ms_ctx *c = new (std::nothrow) ms_ctx();
    if (!c) return MS_ERR_OUT_OF_MEMORY;
    ms_status s = init_ctx(c, dev);
    if (s != MS_OK) {
        delete c;
        return s;
    }
    g_default[dev] = c;
    *out = c;
    return MS_OK;
}

int bucket_of(int64_t m, int64_t n) {
    auto lg = [](int64_t v) {
        int r = 0;
        while (v > 1 && r < 62) {
            v >>= 1;
            ++r;
        }
        return r;
    };
    return lg(m) * 64 + lg(n);
}

// Untuned matrices of at least LARGE_CELLS cells take the probe tile certifying side 32: on the
// large matrices more tiles then finish in the probe and fewer go to the resolve pass (a 16384^2
// blob image: 441 instead of 543 us; a 32768^2 Bernoulli(0.9) matrix: 124 instead of 119 us).
// Below SMALL_CELLS the search is latency-bound (a 4000^2 matrix fills a tenth of the device's
// waves with 113-row tiles), and the 49-row tile, twice the tiles for half the chain each, is
// faster (1000^2: 10.1 instead of 12.5 us; 4000^2: 13.5 instead of 14.0 us).  The map keeps 4
// columns per lane: 8 (one entering-run computation per 8 cells) is faster for one map alone
// (2000^2: 11.2 instead of 12.5 us) but its 32-byte lane strides make each store instruction
// touch twice the cache lines, and with maps of several streams in flight the grid step drops
// (567 against 588 Gcells/s with four streams, each on its own hardware queue).
constexpr int64_t LARGE_CELLS = int64_t(1) << 26;
constexpr int64_t SMALL_CELLS = int64_t(1) << 24;

ms_config default_config(int64_t m, int64_t n) {
    ms_config c = DEFAULT_CONFIG;
    if (m > 0 && n > 0 && m >= LARGE_CELLS / n) c.probe_variant = 2;
    if (m > 0 && n > 0 && m < SMALL_CELLS / n) c.probe_variant = 0;
    return c;
}

// Untuned batched calls take the 49-row tile when the batch's matrices average under 2^20
// cells, the 113-row tile otherwise: the 10000-matrix batch (0.5 Mcells a matrix) 0.426 against
// 0.447 ms, the 45-matrix grid (11 Mcells) 187 against 90 us, 16 served requests (2.4 Mcells)
// 146 against 122 us.
int default_batched_variant(const ms_matrix *h_mats, int64_t count) {
    double cells = 0;
    for (int64_t i = 0; i < count; ++i) cells += (double)h_mats[i].m * (double)h_mats[i].n;
    return cells < (double)count * (double)(int64_t(1) << 20) ? 0 : DEFAULT_CONFIG.probe_variant;
}

ms_config config_for(ms_ctx *c, int64_t m, int64_t n) {
    if (c->has_forced) return c->forced;
    auto it = c->tuned.find(bucket_of(m, n));
    return it != c->tuned.end() ? it->second : default_config(m, n);
}

bool config_valid(const ms_config &cfg) {
    return cfg.probe_variant >= 0 && cfg.probe_variant < mshost::NUM_PROBE_VARIANTS &&
           (cfg.map_cols == 4 || cfg.map_cols == 8) && cfg.map_band_rows >= 1 &&
           cfg.map_band_rows <= (1 << 20);
}

// Make sure the context scratch holds the serial-pass state and the probe's saturation bytes
// for an m x n matrix.
// The strip sweep's boundary words, in an allocation of their own (grown apart from the
// scratch).  They are tagged with the header's epoch, so whenever the header is zeroed they are
// zeroed too (on the caller's stream, behind the header).
mshost::ScratchHeader *hdr_of(ms_ctx *c);

ms_status ensure_strips(ms_ctx *c, int64_t need, bool header_zeroed, hipStream_t stream) {
    const mshost::LaunchEnv env{c->num_cus, stream};
    if (need > c->strip_words) {
        if (c->strips) {
            if (hipDeviceSynchronize() != hipSuccess) return MS_ERR_HIP;
            (void)hipFree(c->strips);
            c->strips = nullptr;
            c->strip_words = 0;
        }
        void *p = nullptr;
        if (hipMalloc(&p, (size_t)need * sizeof(uint64_t)) != hipSuccess) {
            (void)hipGetLastError();  // without the words the kernels keep the one-wave sweep
            return mshost::launch_set_strips(env, hdr_of(c), nullptr, 0, 0) == hipSuccess
                       ? MS_OK
                       : MS_ERR_HIP;
        }
        c->strips = p;
        c->strip_words = need;
        header_zeroed = true;  // fresh memory: clear it
    }
    if (!header_zeroed) return MS_OK;
    uint64_t *w = static_cast<uint64_t *>(c->strips);
    if ((w && mshost::launch_zero_u64(env, w, c->strip_words) != hipSuccess) ||
        mshost::launch_set_strips(env, hdr_of(c), w, c->strip_words,
                                  mshost::strip_rows_setting()) != hipSuccess)
        return MS_ERR_HIP;
    return MS_OK;
}

// Make sure the context scratch holds the serial-pass state and the probe's saturation bytes
// for an m x n matrix, and the strip words that shape may need.
ms_status ensure_scratch(ms_ctx *c, int64_t m, int64_t n, hipStream_t stream) {
    const int64_t nwords = std::max<int64_t>(1, cdiv(n, 64));
    const int64_t tiles = mshost::max_probe_tiles(m, n);
    const int64_t strips = mshost::strip_words_needed(m, n);
    const mshost::LaunchEnv env{c->num_cus, stream};
    if (c->scratch && c->state_words >= nwords && c->sat_bytes >= tiles) {
        const bool zero = c->dirty;
        if (zero) {
            if (mshost::launch_zero_header(env, c->scratch, sizeof(mshost::ScratchHeader)) !=
                hipSuccess)
                return MS_ERR_HIP;
            c->dirty = false;
        }
        return ensure_strips(c, strips, zero, stream);
    }
    const int64_t words = std::max<int64_t>(nwords, c->state_words);
    const int64_t sat = std::max<int64_t>(tiles, c->sat_bytes);
    // header | serial state | saturation bytes | per-tile bounds (int32) | probe box records
    const size_t bytes = sizeof(mshost::ScratchHeader) + (size_t)words * 64 * 2 * sizeof(int32_t) +
                         (((size_t)sat + 255) & ~(size_t)255) +
                         (((size_t)sat * sizeof(int32_t) + 255) & ~(size_t)255) +
                         (size_t)mshost::max_probe_blocks(c->num_cus) *
                             mshost::BOX_RECORD_WORDS * sizeof(uint32_t);
    if (c->scratch) {
        if (hipDeviceSynchronize() != hipSuccess) return MS_ERR_HIP;
        (void)hipFree(c->scratch);
        c->scratch = nullptr;
        c->last.out = nullptr;  // the bounds went with the old scratch
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return hip_status(e);
    // the header is zeroed on the caller's stream, ahead of the search launched there next (a
    // memset on the null stream may still be pending when a non-blocking stream runs the probe,
    // and would then erase keys it pushed)
    if (mshost::launch_zero_header(env, p, sizeof(mshost::ScratchHeader)) != hipSuccess) {
        (void)hipFree(p);
        return MS_ERR_HIP;
    }
    c->scratch = p;
    c->state_words = words;
    c->sat_bytes = sat;
    c->dirty = false;
    return ensure_strips(c, strips, true, stream);
}

mshost::ScratchHeader *hdr_of(ms_ctx *c) { return static_cast<mshost::ScratchHeader *>(c->scratch); }
uint8_t *sat_of(ms_ctx *c) {
    return static_cast<uint8_t *>(c->scratch) + sizeof(mshost::ScratchHeader) +
           (size_t)c->state_words * 64 * 2 * sizeof(int32_t);
}
int32_t *bounds_of(ms_ctx *c) {
    return reinterpret_cast<int32_t *>(sat_of(c) + (((size_t)c->sat_bytes + 255) & ~(size_t)255));
}
uint32_t *box_records_of(ms_ctx *c) {
    return reinterpret_cast<uint32_t *>(
        reinterpret_cast<char *>(bounds_of(c)) +
        (((size_t)c->sat_bytes * sizeof(int32_t) + 255) & ~(size_t)255));
}
// The strip words for an m x n call, or nullptr (the kernels then keep the one-wave sweep)
// when the scratch holds too few of them for that shape.
uint64_t *strips_for(ms_ctx *c, int64_t m, int64_t n) {
    const int64_t need = cdiv(cdiv(std::max<int64_t>(n, 1), 64), (int64_t)mshost::STRIP_WORDS) *
                         std::max<int64_t>(m, 1) * 2;
    return c->strip_words >= need ? static_cast<uint64_t *>(c->strips) : nullptr;
}
int32_t *state_of(ms_ctx *c) {
    return reinterpret_cast<int32_t *>(static_cast<char *>(c->scratch) +
                                       sizeof(mshost::ScratchHeader));
}

ms_status validate_packed(const uint64_t *bits, int64_t m, int64_t n, int64_t ldw) {
    if (m < 0 || n < 0 || ldw < 0) return MS_ERR_INVALID_ARGUMENT;
    if (m == 0 || n == 0) return MS_OK;
    if (!bits) return MS_ERR_INVALID_ARGUMENT;
    if (ldw < cdiv(n, 64)) return MS_ERR_INVALID_ARGUMENT;
    if (mul_overflows(m, n) || m * n >= POS_LIMIT) return MS_ERR_INVALID_ARGUMENT;
    if (mul_overflows(m, ldw)) return MS_ERR_INVALID_ARGUMENT;
    if (std::min(m, n) >= SIDE_LIMIT) return MS_ERR_UNSUPPORTED;
    return MS_OK;
}

// Runs the two launches of the largest-square search; result lands in the scratch header.
ms_status run_max_square(ms_ctx *c, const ms_config &cfg, const uint64_t *bits, int64_t m,
                         int64_t n, int64_t ldw, ms_square *out, hipStream_t stream) {
    if (hipSetDevice(c->device) != hipSuccess) return MS_ERR_HIP;
    ms_status s = ensure_scratch(c, m, n, stream);
    if (s != MS_OK) return s;
    mshost::LaunchEnv env{c->num_cus, stream};
    hipError_t e;
    c->last.out = nullptr;
    if (m == 0 || n == 0) {
        e = mshost::launch_write_result(env, out, hdr_of(c), out ? 1 : 0);
    } else {
        e = mshost::launch_max_square(env, cfg.probe_variant, bits, m, n, ldw, hdr_of(c),
                                      state_of(c), sat_of(c), bounds_of(c), box_records_of(c),
                                      out);
    }
    if (e != hipSuccess) {
        c->dirty = true;
        return hip_status(e);
    }
    if (m > 0 && n > 0) {
        c->last.bits = bits;
        c->last.m = m;
        c->last.n = n;
        c->last.ldw = ldw;
        c->last.out = out;
        c->last.variant = cfg.probe_variant;
    }
    return MS_OK;
}

}  // namespace

extern "C" {

const char *ms_status_string(ms_status s) {
    // a C caller may pass any int: read it as one, not as the enum (whose range is 0..7 in C++)
    int v = 0;
    std::memcpy(&v, &s, sizeof v);
    switch (v) {
    case MS_OK: return "ok";
    case MS_ERR_INVALID_ARGUMENT: return "invalid argument";
    case MS_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case MS_ERR_OUT_OF_MEMORY: return "out of memory";
    case MS_ERR_HIP: return "HIP runtime error";
    case MS_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

ms_status ms_create(ms_ctx **ctx, int hip_device) {
    if (!ctx || hip_device < -1) return MS_ERR_INVALID_ARGUMENT;
    *ctx = nullptr;
    ms_ctx *c = new (std::nothrow) ms_ctx();
    if (!c) return MS_ERR_OUT_OF_MEMORY;
    ms_status s = init_ctx(c, hip_device);
    if (s != MS_OK) {
        delete c;
        return s;
    }
    *ctx = c;
    return MS_OK;
}

ms_status ms_destroy(ms_ctx *ctx) {
    if (!ctx) return MS_ERR_INVALID_ARGUMENT;
    {
        std::lock_guard<std::mutex> lk(g_default_mu);
        for (auto &kv : g_default)
            if (kv.second == ctx) return MS_ERR_INVALID_ARGUMENT;  // default contexts live on
    }
    if (ctx->scratch || ctx->rect_scratch || ctx->pinned || !ctx->graphs.empty()) {
        (void)hipSetDevice(ctx->device);
        (void)hipDeviceSynchronize();
    }
    for (auto &g : ctx->graphs) (void)hipGraphExecDestroy(g.exec);
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    if (ctx->strips) (void)hipFree(ctx->strips);
    if (ctx->rect_scratch) (void)hipFree(ctx->rect_scratch);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    delete ctx;
    return MS_OK;
}

ms_status ms_pack_u8(ms_ctx *ctx, const uint8_t *d_a, int64_t m, int64_t n, int64_t ld_bytes,
                     uint64_t *d_bits, int64_t ld_words, void *stream) {
    if (m < 0 || n < 0 || ld_bytes < 0 || ld_words < 0) return MS_ERR_INVALID_ARGUMENT;
    if (m > 0 && n > 0) {
        if (!d_a || !d_bits || ld_bytes < n || ld_words < cdiv(n, 64))
            return MS_ERR_INVALID_ARGUMENT;
        if (mul_overflows(m, n) || mul_overflows(m, ld_bytes) || mul_overflows(m, ld_words))
            return MS_ERR_INVALID_ARGUMENT;
    }
    ms_ctx *c = nullptr;
    ms_status s = resolve(ctx, &c);
    if (s != MS_OK) return s;
    if (m == 0 || n == 0) return MS_OK;
    std::lock_guard<std::mutex> lk(c->mu);
    if (hipSetDevice(c->device) != hipSuccess) return MS_ERR_HIP;
    mshost::LaunchEnv env{c->num_cus, (hipStream_t)stream};
    return hip_status(mshost::launch_pack_u8(env, d_a, m, n, ld_bytes, d_bits, ld_words));
}

ms_status ms_max_square(ms_ctx *ctx, const uint64_t *d_bits, int64_t m, int64_t n,
                        int64_t ld_words, ms_square *d_out, void *stream) {
    ms_status s = validate_packed(d_bits, m, n, ld_words);
    if (s != MS_OK) return s;
    if (!d_out) return MS_ERR_INVALID_ARGUMENT;
    ms_ctx *c = nullptr;
    s = resolve(ctx, &c);
    if (s != MS_OK) return s;
    std::lock_guard<std::mutex> lk(c->mu);
    return run_max_square(c, config_for(c, m, n), d_bits, m, n, ld_words, d_out,
                          (hipStream_t)stream);
}

ms_status ms_max_square_noalloc(ms_ctx *ctx, const uint64_t *d_bits, int64_t m, int64_t n,
                                int64_t ld_words, ms_square *d_out, void *stream) {
    ms_status s = validate_packed(d_bits, m, n, ld_words);
    if (s != MS_OK) return s;
    if (!ctx || !d_out) return MS_ERR_INVALID_ARGUMENT;
    if (m > 0 && n > 0 && (cdiv(n, 64) > mshost::NOALLOC_MAX_WORDS ||
                           mshost::max_probe_tiles(m, n) > mshost::NOALLOC_MAX_TILES))
        return MS_ERR_WORKSPACE_TOO_SMALL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return MS_ERR_HIP;
    const ms_config cfg = config_for(ctx, m, n);
    mshost::LaunchEnv env{ctx->num_cus, (hipStream_t)stream};
    return hip_status(mshost::launch_max_square_noalloc(env, ctx->device, cfg.probe_variant,
                                                        d_bits, m, n, ld_words, d_out));
}

ms_status ms_square_map(ms_ctx *ctx, const uint64_t *d_bits, int64_t m, int64_t n,
                        int64_t ld_words, int32_t *d_dp, int64_t ld_dp, ms_square *d_out,
                        void *stream) {
    ms_status s = validate_packed(d_bits, m, n, ld_words);
    if (s != MS_OK) return s;
    if (ld_dp < 0) return MS_ERR_INVALID_ARGUMENT;
    if (m > 0 && n > 0) {
        if (!d_dp || ld_dp < n || mul_overflows(m, ld_dp)) return MS_ERR_INVALID_ARGUMENT;
    }
    ms_ctx *c = nullptr;
    s = resolve(ctx, &c);
    if (s != MS_OK) return s;
    std::lock_guard<std::mutex> lk(c->mu);
    const ms_config cfg = config_for(c, m, n);
    hipStream_t st = (hipStream_t)stream;
    s = run_max_square(c, cfg, d_bits, m, n, ld_words, d_out, st);
    if (s != MS_OK || m == 0 || n == 0) return s;
    mshost::LaunchEnv env{c->num_cus, st};
    // the search just ran on these bits: its per-tile bounds let the map size halos by region
    const mshost::MapRegions regions{bounds_of(c), mshost::probe_tile_rows(cfg.probe_variant),
                                     cdiv(cdiv(n, 64), mshost::PROBE_TILE_WORDS),
                                     hdr_of(c)->big_box};
    hipError_t e = mshost::launch_square_map(env, cfg.map_cols, cfg.map_band_rows, d_bits, m, n,
                                             ld_words, d_dp, ld_dp, &hdr_of(c)->result,
                                             state_of(c), &regions, hdr_of(c), strips_for(c, m, n),
                                             mshost::strip_rows_setting());
    return hip_status(e);
}

ms_status ms_square_map_from_max(ms_ctx *ctx, const uint64_t *d_bits, int64_t m, int64_t n,
                                 int64_t ld_words, const ms_square *d_max, int32_t *d_dp,
                                 int64_t ld_dp, void *stream) {
    ms_status s = validate_packed(d_bits, m, n, ld_words);
    if (s != MS_OK) return s;
    if (ld_dp < 0 || !d_max) return MS_ERR_INVALID_ARGUMENT;
    if (m > 0 && n > 0) {
        if (!d_dp || ld_dp < n || mul_overflows(m, ld_dp)) return MS_ERR_INVALID_ARGUMENT;
    }
    ms_ctx *c = nullptr;
    s = resolve(ctx, &c);
    if (s != MS_OK) return s;
    if (m == 0 || n == 0) return MS_OK;
    std::lock_guard<std::mutex> lk(c->mu);
    const ms_config cfg = config_for(c, m, n);
    hipStream_t st = (hipStream_t)stream;
    if (hipSetDevice(c->device) != hipSuccess) return MS_ERR_HIP;
    s = ensure_scratch(c, m, n, st);
    if (s != MS_OK) return s;
    mshost::LaunchEnv env{c->num_cus, st};
    // d_max is the result of this context's last search, on these bits: that search's per-tile
    // bounds are still in the scratch (calls on a context are ordered on one stream), so the
    // halos follow them as in ms_square_map
    const bool same = c->last.out != nullptr && c->last.out == d_max && c->last.bits == d_bits &&
                      c->last.m == m && c->last.n == n && c->last.ldw == ld_words &&
                      c->last.variant == cfg.probe_variant;
    const mshost::MapRegions regions{bounds_of(c), mshost::probe_tile_rows(cfg.probe_variant),
                                     cdiv(cdiv(n, 64), mshost::PROBE_TILE_WORDS),
                                     hdr_of(c)->big_box};
    return hip_status(mshost::launch_square_map(env, cfg.map_cols, cfg.map_band_rows, d_bits, m,
                                                n, ld_words, d_dp, ld_dp, d_max, state_of(c),
                                                same ? &regions : nullptr, hdr_of(c),
                                                strips_for(c, m, n),
                                                mshost::strip_rows_setting()));
}

ms_status ms_batched_workspace_size(ms_ctx *ctx, const ms_matrix *h_mats, int64_t count,
                                    size_t *bytes) {
    if (count < 0 || !bytes || (count > 0 && !h_mats)) return MS_ERR_INVALID_ARGUMENT;
    for (int64_t i = 0; i < count; ++i) {
        ms_status s = validate_packed(h_mats[i].bits, h_mats[i].m, h_mats[i].n, h_mats[i].ld_words);
        if (s != MS_OK) return s;
    }
    if (count >= (int64_t(1) << 24)) return MS_ERR_INVALID_ARGUMENT;
    (void)ctx;
    // a bound for every probe variant and tile width, so a tuned choice always fits
    *bytes = mshost::batch_layout(0, -1, h_mats, count).total;
    return MS_OK;
}

ms_status ms_max_square_batched(ms_ctx *ctx, const ms_matrix *h_mats, const ms_matrix *d_mats,
                                int64_t count, ms_square *d_out, void *d_workspace,
                                size_t workspace_bytes, void *stream) {
    if (count < 0) return MS_ERR_INVALID_ARGUMENT;
    if (count == 0) return MS_OK;
    if (!h_mats || !d_mats || !d_out || !d_workspace) return MS_ERR_INVALID_ARGUMENT;
    if (count >= (int64_t(1) << 24)) return MS_ERR_INVALID_ARGUMENT;
    for (int64_t i = 0; i < count; ++i) {
        ms_status s = validate_packed(h_mats[i].bits, h_mats[i].m, h_mats[i].n, h_mats[i].ld_words);
        if (s != MS_OK) return s;
    }
    ms_ctx *c = nullptr;
    ms_status s = resolve(ctx, &c);
    if (s != MS_OK) return s;
    std::lock_guard<std::mutex> lk(c->mu);
    const int variant = c->has_forced ? c->forced.probe_variant
                        : c->batched_variant >= 0 ? c->batched_variant
                                                  : default_batched_variant(h_mats, count);
    const int narrow = !c->has_forced && c->batched_narrow >= 0 ? c->batched_narrow
                                                                : mshost::NARROW_WEIGHTS[0];
    const mshost::BatchLayout L = mshost::batch_layout(variant, narrow, h_mats, count);
    if (workspace_bytes < L.total) return MS_ERR_WORKSPACE_TOO_SMALL;
    if (hipSetDevice(c->device) != hipSuccess) return MS_ERR_HIP;
    hipStream_t st = (hipStream_t)stream;
    // a batch met for the first time runs its launches eagerly and is remembered; a repeat of
    // it (same descriptor, output and workspace buffers, count, variant and shapes) is captured
    // once into a graph and replayed from then on: one submission per call (the context's
    // graph mode, or MAXSQ_GRAPH=0 / 1, turns this off or captures on the first call).
    // A stream the caller is capturing records the eager launches into the caller's graph.
    const char *gv = std::getenv("MAXSQ_GRAPH");
    const int mode = gv && gv[0] == '0'   ? MS_GRAPHS_OFF
                     : gv && gv[0] == '1' ? MS_GRAPHS_ALWAYS
                                          : c->graph_mode;
    mshost::LaunchEnv eager{c->num_cus, st};
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cap) != hipSuccess) return MS_ERR_HIP;
    if (mode == MS_GRAPHS_OFF || cap != hipStreamCaptureStatusNone)
        return hip_status(mshost::launch_batched(eager, variant, d_mats, count, d_out, d_workspace, L));
    const uint64_t sh = shape_hash(h_mats, count);
    const auto same = [&](const GraphEntry &g) {
        return g.mats == d_mats && g.count == count && g.out == d_out && g.ws == d_workspace &&
               g.variant == variant && g.narrow == narrow && g.shape_hash == sh;
    };
    for (auto &g : c->graphs)
        if (same(g)) return hip_status(hipGraphLaunch(g.exec, st));
    if (mode == MS_GRAPHS_ON_REPEAT) {
        bool repeat = false;
        for (size_t k = 0; k < c->seen.size() && !repeat; ++k) repeat = same(c->seen[k]);
        if (!repeat) {
            if (c->seen.size() >= 16) c->seen.erase(c->seen.begin());
            c->seen.push_back(
                GraphEntry{d_mats, count, d_out, d_workspace, variant, narrow, sh, nullptr});
            return hip_status(
                mshost::launch_batched(eager, variant, d_mats, count, d_out, d_workspace, L));
        }
    }
    if (!c->capture_stream) {
        if (hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking) != hipSuccess)
            return MS_ERR_HIP;
    }
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_status(e);
    mshost::LaunchEnv env{c->num_cus, c->capture_stream};
    hipError_t le = mshost::launch_batched(env, variant, d_mats, count, d_out, d_workspace, L);
    e = hipStreamEndCapture(c->capture_stream, &graph);
    if (le != hipSuccess || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return MS_ERR_HIP;
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_status(e);
    if (c->graphs.size() >= 8) {
        if (hipDeviceSynchronize() != hipSuccess) return MS_ERR_HIP;
        (void)hipGraphExecDestroy(c->graphs.front().exec);
        c->graphs.erase(c->graphs.begin());
    }
    c->graphs.push_back(GraphEntry{d_mats, count, d_out, d_workspace, variant, narrow, sh, exec});
    return hip_status(hipGraphLaunch(exec, st));
}

ms_status ms_max_rectangle(ms_ctx *ctx, const uint64_t *d_bits, int64_t m, int64_t n,
                           int64_t ld_words, ms_rect *d_out, void *stream) {
    ms_status s = validate_packed(d_bits, m, n, ld_words);
    if (s != MS_OK) return s;
    if (!d_out) return MS_ERR_INVALID_ARGUMENT;
    if (cdiv(n, 64) > mshost::RECT_MAX_WORDS) return MS_ERR_UNSUPPORTED;
    ms_ctx *c = nullptr;
    s = resolve(ctx, &c);
    if (s != MS_OK) return s;
    std::lock_guard<std::mutex> lk(c->mu);
    if (hipSetDevice(c->device) != hipSuccess) return MS_ERR_HIP;
    hipStream_t st = (hipStream_t)stream;
    mshost::LaunchEnv env{c->num_cus, st};
    if (!c->rect_scratch) {
        const size_t bytes = sizeof(mshost::RectScratch) +
                             (size_t)mshost::rect_max_blocks(c->num_cus) * sizeof(mshost::RectRecord);
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) return hip_status(e);
        // zeroed on the call's stream, ahead of the launch there (see ensure_scratch)
        if (mshost::launch_zero_header(env, p, sizeof(mshost::RectScratch)) != hipSuccess) {
            (void)hipFree(p);
            return MS_ERR_HIP;
        }
        c->rect_scratch = p;
    } else if (c->rect_dirty) {
        if (mshost::launch_zero_header(env, c->rect_scratch, sizeof(mshost::RectScratch)) !=
            hipSuccess)
            return MS_ERR_HIP;
    }
    c->rect_dirty = false;
    hipError_t e = mshost::launch_max_rect(env, d_bits, m, n, ld_words,
                                           static_cast<mshost::RectScratch *>(c->rect_scratch),
                                           d_out);
    if (e != hipSuccess) c->rect_dirty = true;
    return hip_status(e);
}

namespace {

ms_status validate_volume(const uint64_t *bits, int64_t D, int64_t M, int64_t N, int64_t ldw) {
    if (D < 0 || M < 0 || N < 0 || ldw < 0) return MS_ERR_INVALID_ARGUMENT;
    if (D == 0 || M == 0 || N == 0) return MS_OK;
    if (!bits || ldw < cdiv(N, 64)) return MS_ERR_INVALID_ARGUMENT;
    if (mul_overflows(D, M) || mul_overflows(D * M, N) || D * M * N >= POS_LIMIT)
        return MS_ERR_INVALID_ARGUMENT;
    if (mul_overflows(D * M, ldw)) return MS_ERR_INVALID_ARGUMENT;
    if (D * M * cdiv(N, 64) >= (int64_t(1) << 32)) return MS_ERR_UNSUPPORTED;
    return MS_OK;
}

}  // namespace

ms_status ms_max_cube_workspace_size(ms_ctx *ctx, int64_t D, int64_t M, int64_t N,
                                     size_t *bytes) {
    (void)ctx;
    if (!bytes || D < 0 || M < 0 || N < 0) return MS_ERR_INVALID_ARGUMENT;
    if (mul_overflows(D, M) || mul_overflows(D * M, std::max<int64_t>(cdiv(N, 64), 1)))
        return MS_ERR_INVALID_ARGUMENT;
    *bytes = mshost::cube_workspace_bytes(D, M, N);
    return MS_OK;
}

ms_status ms_max_cube(ms_ctx *ctx, const uint64_t *d_bits, int64_t D, int64_t M, int64_t N,
                      int64_t ld_words, ms_cube *d_out, void *d_workspace,
                      size_t workspace_bytes, void *stream) {
    ms_status s = validate_volume(d_bits, D, M, N, ld_words);
    if (s != MS_OK) return s;
    if (!d_out) return MS_ERR_INVALID_ARGUMENT;
    const bool empty = D == 0 || M == 0 || N == 0;
    if (!empty && !d_workspace) return MS_ERR_INVALID_ARGUMENT;
    if (!empty && workspace_bytes < mshost::cube_workspace_bytes(D, M, N))
        return MS_ERR_WORKSPACE_TOO_SMALL;
    ms_ctx *c = nullptr;
    s = resolve(ctx, &c);
    if (s != MS_OK) return s;
    std::lock_guard<std::mutex> lk(c->mu);
    if (hipSetDevice(c->device) != hipSuccess) return MS_ERR_HIP;
    if (!c->pinned) {
        void *p = nullptr;
        if (hipHostMalloc(&p, 64, hipHostMallocDefault) != hipSuccess) return MS_ERR_OUT_OF_MEMORY;
        c->pinned = static_cast<uint64_t *>(p);
    }
    hipStream_t st = (hipStream_t)stream;
    if (!empty) {
        mshost::LaunchEnv env{c->num_cus, st};
        auto *ctl = static_cast<mshost::CubeControl *>(d_workspace);
        uint64_t *V[3];
        for (int k = 0; k < 3; ++k) V[k] = mshost::cube_volume(d_workspace, D, M, N, k);
        const int64_t smax = std::min(D, std::min(M, N));
        // E_1: the input copied into volume 0 with its padding cleared; then the search runs on
        // the device (gallop, then bisection, decided by a one-thread kernel after each probe),
        // which writes d_out when done.  The host enqueues probes in rounds of PROBES_PER_ROUND
        // and reads the phase once per round: a round that finds the search done costs only its
        // idle launches, and no probe waits for the host.
        constexpr int PROBES_PER_ROUND = 8;
        int lg = 0;
        while ((int64_t(1) << lg) < smax) ++lg;
        const int rounds = (2 * lg + 2 + PROBES_PER_ROUND - 1) / PROBES_PER_ROUND + 1;
        if (mshost::launch_cube_begin(env, ctl, smax) != hipSuccess ||
            mshost::launch_cube_copy(env, d_bits, ld_words, V[0], D, M, N, ctl) != hipSuccess ||
            mshost::launch_cube_control(env, ctl, d_out, M, N) != hipSuccess)
            return MS_ERR_HIP;
        for (int round = 0; round < rounds; ++round) {
            for (int k = 0; k < PROBES_PER_ROUND; ++k)
                if (mshost::launch_cube_probe(env, V, D, M, N, ctl) != hipSuccess ||
                    mshost::launch_cube_control(env, ctl, d_out, M, N) != hipSuccess)
                    return MS_ERR_HIP;
            if (hipMemcpyAsync(c->pinned, &ctl->phase, sizeof(int32_t), hipMemcpyDeviceToHost,
                               st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                return MS_ERR_HIP;
            int32_t phase = 0;
            std::memcpy(&phase, c->pinned, sizeof(phase));
            if (phase == mshost::CUBE_DONE) return MS_OK;
        }
        return MS_ERR_HIP;  // more probes than the bound on the search allows
    }
    // an empty volume: the result through pinned memory (d_out may be device or pinned host
    // memory)
    const ms_cube res{0, -1, -1, -1};
    std::memcpy(c->pinned, &res, sizeof(res));
    if (hipMemcpyAsync(d_out, c->pinned, sizeof(res), hipMemcpyDefault, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return MS_ERR_HIP;
    return MS_OK;
}

ms_status ms_all_max_squares_workspace_size(ms_ctx *ctx, int64_t m, int64_t n, size_t *bytes) {
    (void)ctx;
    if (!bytes || m < 0 || n < 0 || mul_overflows(m, std::max<int64_t>(n, 1)))
        return MS_ERR_INVALID_ARGUMENT;
    *bytes = mshost::all_max_layout(m, n).total;
    return MS_OK;
}

ms_status ms_all_max_squares(ms_ctx *ctx, const uint64_t *d_bits, int64_t m, int64_t n,
                             int64_t ld_words, const ms_square *d_max, int64_t *d_pos,
                             int64_t capacity, int64_t *d_count, void *d_workspace,
                             size_t workspace_bytes, void *stream) {
    ms_status s = validate_packed(d_bits, m, n, ld_words);
    if (s != MS_OK) return s;
    if (capacity < 0 || (capacity > 0 && !d_pos) || !d_count) return MS_ERR_INVALID_ARGUMENT;
    const bool empty = m == 0 || n == 0;
    if (!empty && (!d_max || !d_workspace)) return MS_ERR_INVALID_ARGUMENT;
    if (!empty && workspace_bytes < mshost::all_max_layout(m, n).total)
        return MS_ERR_WORKSPACE_TOO_SMALL;
    ms_ctx *c = nullptr;
    s = resolve(ctx, &c);
    if (s != MS_OK) return s;
    std::lock_guard<std::mutex> lk(c->mu);
    if (hipSetDevice(c->device) != hipSuccess) return MS_ERR_HIP;
    mshost::LaunchEnv env{c->num_cus, (hipStream_t)stream};
    return hip_status(mshost::launch_all_max(env, d_bits, m, n, ld_words, d_max, d_pos, capacity,
                                             d_count, d_workspace));
}

int ms_num_candidates(void) { return mshost::NUM_PROBE_VARIANTS * 2 * 3; }

ms_status ms_candidate(int index, ms_config *cfg) {
    if (!cfg || index < 0 || index >= ms_num_candidates()) return MS_ERR_INVALID_ARGUMENT;
    static const int bands[3] = {32, 64, 128};
    cfg->probe_variant = index / 6;
    cfg->map_cols = (index / 3) % 2 ? 8 : 4;
    cfg->map_band_rows = bands[index % 3];
    return MS_OK;
}

ms_status ms_set_config(ms_ctx *ctx, const ms_config *cfg) {
    if (cfg && !config_valid(*cfg)) return MS_ERR_INVALID_ARGUMENT;
    ms_ctx *c = nullptr;
    ms_status s = resolve(ctx, &c);
    if (s != MS_OK) return s;
    std::lock_guard<std::mutex> lk(c->mu);
    c->has_forced = cfg != nullptr;
    if (cfg) c->forced = *cfg;
    return MS_OK;
}

ms_status ms_set_batched_graphs(ms_ctx *ctx, int mode) {
    if (mode != MS_GRAPHS_OFF && mode != MS_GRAPHS_ON_REPEAT && mode != MS_GRAPHS_ALWAYS)
        return MS_ERR_INVALID_ARGUMENT;
    ms_ctx *c = nullptr;
    ms_status s = resolve(ctx, &c);
    if (s != MS_OK) return s;
    std::lock_guard<std::mutex> lk(c->mu);
    c->graph_mode = mode;
    return MS_OK;
}

ms_status ms_get_config(ms_ctx *ctx, int64_t m, int64_t n, ms_config *cfg) {
    if (!cfg || m < 0 || n < 0) return MS_ERR_INVALID_ARGUMENT;
    if (!ctx) {
        *cfg = default_config(m, n);
        ms_ctx *c = nullptr;
        if (resolve(nullptr, &c) != MS_OK) return MS_OK;
        ctx = c;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    *cfg = config_for(ctx, m, n);
    return MS_OK;
}

ms_status ms_autotune(ms_ctx *ctx, const uint64_t *d_bits, int64_t m, int64_t n,
                      int64_t ld_words, int32_t *d_dp_scratch, int64_t ld_dp, void *stream) {
    ms_status s = validate_packed(d_bits, m, n, ld_words);
    if (s != MS_OK) return s;
    if (m == 0 || n == 0) return MS_ERR_INVALID_ARGUMENT;
    if (d_dp_scratch && (ld_dp < n || mul_overflows(m, ld_dp))) return MS_ERR_INVALID_ARGUMENT;
    ms_ctx *c = nullptr;
    s = resolve(ctx, &c);
    if (s != MS_OK) return s;
    std::lock_guard<std::mutex> lk(c->mu);
    hipStream_t st = (hipStream_t)stream;
    if (hipSetDevice(c->device) != hipSuccess) return MS_ERR_HIP;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return MS_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return MS_ERR_HIP;
    }
    auto time_it = [&](auto &&body, float *ms_out) -> ms_status {
        const int reps = 5;
        ms_status r = body();  // warm-up
        if (r != MS_OK) return r;
        if (hipEventRecord(e0, st) != hipSuccess) return MS_ERR_HIP;
        for (int i = 0; i < reps; ++i) {
            r = body();
            if (r != MS_OK) return r;
        }
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
            return MS_ERR_HIP;
        float ms = 0;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return MS_ERR_HIP;
        *ms_out = ms / reps;
        return MS_OK;
    };
    ms_config best = DEFAULT_CONFIG;
    float best_probe = 1e30f;
    for (int v = 0; v < mshost::NUM_PROBE_VARIANTS && s == MS_OK; ++v) {
        ms_config cfg = DEFAULT_CONFIG;
        cfg.probe_variant = v;
        float t = 0;
        s = time_it([&]() { return run_max_square(c, cfg, d_bits, m, n, ld_words, nullptr, st); }, &t);
        if (s == MS_OK && t < best_probe) {
            best_probe = t;
            best.probe_variant = v;
        }
    }
    if (s == MS_OK && d_dp_scratch) {
        float best_map = 1e30f;
        for (int i = 0; i < ms_num_candidates() && s == MS_OK; ++i) {
            ms_config cfg;
            ms_candidate(i, &cfg);
            if (cfg.probe_variant != best.probe_variant) continue;
            float t = 0;
            s = time_it([&]() {
                ms_status r = run_max_square(c, cfg, d_bits, m, n, ld_words, nullptr, st);
                if (r != MS_OK) return r;
                mshost::LaunchEnv env{c->num_cus, st};
                return hip_status(mshost::launch_square_map(env, cfg.map_cols, cfg.map_band_rows,
                                                            d_bits, m, n, ld_words, d_dp_scratch,
                                                            ld_dp, &hdr_of(c)->result,
                                                            state_of(c), nullptr,
                                                            hdr_of(c),
                                                            strips_for(c, m, n),
                                                            mshost::strip_rows_setting()));
            }, &t);
            if (s == MS_OK && t < best_map) {
                best_map = t;
                best.map_cols = cfg.map_cols;
                best.map_band_rows = cfg.map_band_rows;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s == MS_OK) c->tuned[bucket_of(m, n)] = best;
    return s;
}

ms_status ms_autotune_batched(ms_ctx *ctx, const ms_matrix *h_mats, const ms_matrix *d_mats,
                              int64_t count, ms_square *d_out, void *d_workspace,
                              size_t workspace_bytes, void *stream) {
    if (count <= 0 || !h_mats || !d_mats || !d_out || !d_workspace) return MS_ERR_INVALID_ARGUMENT;
    if (count >= (int64_t(1) << 24)) return MS_ERR_INVALID_ARGUMENT;
    for (int64_t i = 0; i < count; ++i) {
        ms_status s = validate_packed(h_mats[i].bits, h_mats[i].m, h_mats[i].n, h_mats[i].ld_words);
        if (s != MS_OK) return s;
    }
    ms_ctx *c = nullptr;
    ms_status s = resolve(ctx, &c);
    if (s != MS_OK) return s;
    std::lock_guard<std::mutex> lk(c->mu);
    if (hipSetDevice(c->device) != hipSuccess) return MS_ERR_HIP;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return MS_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return MS_ERR_HIP;
    }
    mshost::LaunchEnv env{c->num_cus, st};
    int best_v = DEFAULT_CONFIG.probe_variant, best_q = mshost::NARROW_WEIGHTS[0];
    // every probe variant with every tile-width weight, in two interleaved rounds, each keeping
    // its faster round (a single round's pick moved by a few per cent from run to run)
    constexpr int NC = mshost::NUM_PROBE_VARIANTS * mshost::NUM_NARROW_WEIGHTS;
    float cand_t[NC];
    for (int i = 0; i < NC; ++i) cand_t[i] = 1e30f;
    for (int round = 0; round < 2 && s == MS_OK; ++round) {
        for (int i = 0; i < NC && s == MS_OK; ++i) {
            const int v = i / mshost::NUM_NARROW_WEIGHTS;
            const int q = mshost::NARROW_WEIGHTS[i % mshost::NUM_NARROW_WEIGHTS];
            const mshost::BatchLayout L = mshost::batch_layout(v, q, h_mats, count);
            if (workspace_bytes < L.total) {
                s = MS_ERR_WORKSPACE_TOO_SMALL;
                break;
            }
            const int reps = 3;
            hipError_t e = mshost::launch_batched(env, v, d_mats, count, d_out, d_workspace, L);
            if (e == hipSuccess) e = hipEventRecord(e0, st);
            for (int r = 0; r < reps && e == hipSuccess; ++r)
                e = mshost::launch_batched(env, v, d_mats, count, d_out, d_workspace, L);
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                s = hip_status(e);
                break;
            }
            cand_t[i] = ms < cand_t[i] ? ms : cand_t[i];
        }
    }
    float best_t = 1e30f;
    for (int i = 0; i < NC; ++i)
        if (cand_t[i] < best_t) {
            best_t = cand_t[i];
            best_v = i / mshost::NUM_NARROW_WEIGHTS;
            best_q = mshost::NARROW_WEIGHTS[i % mshost::NUM_NARROW_WEIGHTS];
        }
    // leave the results of the chosen launch shape in d_out
    if (s == MS_OK) {
        const mshost::BatchLayout L = mshost::batch_layout(best_v, best_q, h_mats, count);
        s = hip_status(mshost::launch_batched(env, best_v, d_mats, count, d_out, d_workspace, L));
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s == MS_OK) {
        c->batched_variant = best_v;
        c->batched_narrow = best_q;
    }
    return s;
}

ms_status ms_autotune_save(ms_ctx *ctx, const char *path) {
    if (!ctx || !path) return MS_ERR_INVALID_ARGUMENT;
    std::lock_guard<std::mutex> lk(ctx->mu);
    FILE *f = std::fopen(path, "w");
    if (!f) return MS_ERR_INVALID_ARGUMENT;
    std::fprintf(f, "# maxsq autotune table: bucket probe_variant map_cols map_band_rows; "
                    "batched probe_variant tile_width_weight\n");
    if (ctx->batched_variant >= 0)
        std::fprintf(f, "batched %d %d\n", ctx->batched_variant,
                     ctx->batched_narrow >= 0 ? ctx->batched_narrow : mshost::NARROW_WEIGHTS[0]);
    for (auto &kv : ctx->tuned)
        std::fprintf(f, "%d %d %d %d\n", kv.first, kv.second.probe_variant, kv.second.map_cols,
                     kv.second.map_band_rows);
    std::fclose(f);
    return MS_OK;
}

ms_status ms_autotune_load(ms_ctx *ctx, const char *path) {
    if (!ctx || !path) return MS_ERR_INVALID_ARGUMENT;
    FILE *f = std::fopen(path, "r");
    if (!f) return MS_ERR_INVALID_ARGUMENT;
    std::map<int, ms_config> table;
    int batched = -1, batched_q = -1;
    char line[256];
    ms_status s = MS_OK;
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        int bv = -1, bq = mshost::NARROW_WEIGHTS[0];
        const int nb = std::sscanf(line, "batched %d %d", &bv, &bq);
        if (nb >= 1) {  // "batched <variant> [<tile-width weight>]"
            if (bv < 0 || bv >= mshost::NUM_PROBE_VARIANTS || !mshost::narrow_weight_valid(bq)) {
                s = MS_ERR_INVALID_ARGUMENT;
                break;
            }
            batched = bv;
            batched_q = bq;
            continue;
        }
        int b = 0;
        ms_config cfg{};
        if (std::sscanf(line, "%d %d %d %d", &b, &cfg.probe_variant, &cfg.map_cols,
                        &cfg.map_band_rows) != 4 || !config_valid(cfg)) {
            s = MS_ERR_INVALID_ARGUMENT;
            break;
        }
        table[b] = cfg;
    }
    std::fclose(f);
    if (s != MS_OK) return s;
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (auto &kv : table) ctx->tuned[kv.first] = kv.second;
    if (batched >= 0) {
        ctx->batched_variant = batched;
        ctx->batched_narrow = batched_q;
    }
    return MS_OK;
}

}  // extern "C"
