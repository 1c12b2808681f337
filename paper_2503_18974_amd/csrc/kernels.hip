// kernels.hip -- libmaxsq kernels for gfx950 and their host launchers.
//
// Single matrix, largest square (two launches):
//   k_probe    : erosion search over register tiles (device.hpp tile_search).  Each tile pushes
//                its exact side (up to the side its halo certifies) with its first corner into
//                one atomic key, and writes a saturation byte: 1 when it holds a larger square.
//   k_resolve  : if any tile saturated, finishes those tiles exactly with column heights and a
//                per-row test (device.hpp resolve_tile_block, one block per tile); the last wave to
//                finish (or, with no saturated tile, the first wave) turns the key into the
//                result (running the serial pass for a square too wide for the resolve pass)
//                and clears the scratch.
// dp map (one more launch): k_dpmap reads S on the device and covers the matrix with row bands
// and column windows that start S rows / columns early (zero state there is exact); after a
// search in the same call, the halos follow each probe tile's bound.
// Batched: k_batch_count and k_batch_offsets (tile starts, clear keys, check the descriptors),
// k_probe_batched (every tile of every matrix in one grid-stride pass), k_batch_finish (the
// saturated tiles of every matrix if any, then key -> result per matrix).
#include <algorithm>
#include <cstdlib>
#include <mutex>

#include "device.hpp"
#include "launch.hpp"

namespace msk {

// ---------------------------------------------------------------------------------- pack
// Byte flags of a dword: bit 7 of each byte set iff the byte is non-zero; the multiply moves
// bits 7, 15, 23, 31 to bits 28..31 (no carries: the partial products never overlap).
__device__ __forceinline__ uint32_t nz4(uint32_t x) {
    uint32_t t = (((x & 0x7f7f7f7fu) + 0x7f7f7f7fu) | x) & 0x80808080u;
    return (t * 0x00204081u) >> 28;
}

// Load 16 bytes starting at p, using the widest loads that ALIGN (a power of two dividing the
// address) allows.
template <int ALIGN>
__device__ __forceinline__ uint4 load16(const uint8_t *__restrict__ p) {
    if constexpr (ALIGN >= 16) {
        return *reinterpret_cast<const uint4 *>(p);
    } else if constexpr (ALIGN == 8) {
        const uint2 a = reinterpret_cast<const uint2 *>(p)[0];
        const uint2 b = reinterpret_cast<const uint2 *>(p)[1];
        return make_uint4(a.x, a.y, b.x, b.y);
    } else if constexpr (ALIGN == 4) {
        const uint32_t *q = reinterpret_cast<const uint32_t *>(p);
        return make_uint4(q[0], q[1], q[2], q[3]);
    } else {
        uint32_t w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            w[k] = (uint32_t)p[4 * k] | ((uint32_t)p[4 * k + 1] << 8) |
                   ((uint32_t)p[4 * k + 2] << 16) | ((uint32_t)p[4 * k + 3] << 24);
        return make_uint4(w[0], w[1], w[2], w[3]);
    }
}

// One 16-byte chunk per lane, so a wave's loads cover 1 KB of a row contiguously; the four lanes
// of a quad hold the four chunks of one packed word and merge their 16-bit masks with two DPP
// quad permutes, and the quad's first lane stores the word.  Chunks past n (the row's padding)
// give zero bits.  Row starts are ALIGN-byte aligned (ALIGN divides the base and ld_bytes).
template <int ALIGN>
__global__ __launch_bounds__(256) void k_pack_u8(const uint8_t *__restrict__ a, int64_t m,
                                                 int64_t n, int64_t ldb,
                                                 uint64_t *__restrict__ bits, int64_t ldw) {
    const int64_t cpr = ((n + 63) >> 6) * 4;  // 16-byte chunks per packed row
    const int64_t total = m * cpr;            // a multiple of 4, as is the stride below
    const int q = __lane_id() & 3;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
        int64_t row, c;
        if (total <= 0xFFFFFFFFll) {
            row = (uint32_t)t / (uint32_t)cpr;
            c = (uint32_t)t - (uint32_t)row * (uint32_t)cpr;
        } else {
            row = t / cpr;
            c = t - row * cpr;
        }
        const int64_t off = c * 16;
        const uint8_t *__restrict__ src = a + row * ldb + off;
        uint32_t m16 = 0;
        if (off + 16 <= n) {
            const uint4 v = load16<ALIGN>(src);
            m16 = nz4(v.x) | (nz4(v.y) << 4) | (nz4(v.z) << 8) | (nz4(v.w) << 12);
        } else if (off < n) {
            for (int64_t k = 0; k < n - off; ++k)
                if (src[k] != 0) m16 |= 1u << k;
        }
        // quad_perm [1,0,3,2]: lanes 0 and 2 of the quad receive lanes 1 and 3
        const uint32_t pair = (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)m16, 0xB1, 0xf, 0xf, false);
        const uint32_t half = m16 | (pair << 16);
        // quad_perm [2,3,0,1]: lane 0 receives lane 2's upper half
        const uint32_t upper = (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)half, 0x4E, 0xf, 0xf, false);
        if (q == 0) bits[row * ldw + (c >> 2)] = ((uint64_t)upper << 32) | half;
    }
}

// ---------------------------------------------------------------------------------- probe
template <class TS>
__global__ __launch_bounds__(256) void k_probe(const uint64_t *__restrict__ bits, int64_t m,
                                               int64_t n, int64_t ldw, int64_t ntiles,
                                               int64_t ntx, mshost::ScratchHeader *hdr,
                                               uint8_t *__restrict__ sat,
                                               int32_t *__restrict__ bounds,
                                               uint32_t *__restrict__ box_rec) {
    const int64_t wave = wave_index();
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) / WAVE;
    SatBatch sb{sat};
    sb.bounds = bounds;
    sb.want_box = box_rec != nullptr;
    sb.ntx = ntx;
    sb.stride = nwave;
    for (int64_t t = wave; t < ntiles; t += nwave) {
        const int64_t ty = udiv(t, ntx), tx = t - ty * ntx;
        sb.add(t, tile_search<TS>(bits, m, n, ldw, ty, tx, TileSink{&hdr->key}));
    }
    sb.flush();
    if (__lane_id() == 0 && sb.nsat) atomicAdd(&hdr->nsat, (uint32_t)sb.nsat);
    if (box_rec) {
        // the block's box, one record per block (no atomics: many blocks can hold large
        // tiles, and same-address atomics from thousands of waves cost more than the search)
        __shared__ uint32_t s_box[4][4];
        const int wv = threadIdx.x / WAVE;
        if (__lane_id() == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) s_box[wv][k] = sb.box[k];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                v[k] = s_box[0][k];
                for (int w = 1; w < 4; ++w) v[k] = s_box[w][k] > v[k] ? s_box[w][k] : v[k];
            }
            reinterpret_cast<uint4 *>(box_rec)[blockIdx.x] = make_uint4(v[0], v[1], v[2], v[3]);
        }
    }
}

__device__ void write_result(unsigned long long key, int64_t n, ms_square *dst) {
    ms_square r;
    r.side = key_side(key);
    if (r.side == 0) {
        r.row = -1;
        r.col = -1;
    } else {
        const int64_t pos = key_pos(key);
        r.row = pos / n;
        r.col = pos - r.row * n;
    }
    *dst = r;
}

// ----------------------------------------------------------------------------------------------
// Strip sweep: the recurrence over the whole matrix, for a square too wide for the windowed
// passes, by every wave that takes part.  The columns are cut into strips of STRIP_WORDS words;
// a wave takes strips in ticket order and walks its strip top to bottom with the column heights
// and previous-row dp of its columns in registers.  Strip s needs, per row, the row run and the
// dp at the last column of strip s - 1, which that strip publishes 64 rows at a time as 64-bit
// words tagged with the launch's epoch, so the reader polls the words themselves (no flag, no
// fence).  A strip only waits on the strip before it, whose ticket was taken earlier by a wave
// that is running, so every wait ends; one that still outlasts SPIN_LIMIT polls gives up and
// sets hdr->timeout to the launch's tag, after which no wait of that launch lingers.  The row
// run is published capped at RUN_CAP: min(m, n) < 2^20, so when n > RUN_CAP every column height
// is below the cap and the cap never decides a minimum.
// ----------------------------------------------------------------------------------------------
constexpr int32_t RUN_CAP = (1 << 20) - 1;
constexpr int32_t HEIGHT_CAP = 1 << 30;
constexpr uint32_t SPIN_LIMIT = 1u << 20;

__device__ __forceinline__ void store_relaxed_u64(unsigned long long *p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t lane_u64(uint64_t v, int l) {
    return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int32_t)(v >> 32), l) << 32) |
           (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)v, l);
}

// The next strip for the calling wave: one atomic add on a counter holding epoch << 32 | count.
// The first takers of a launch find an earlier launch's epoch there; one of them installs this
// launch's epoch with ticket 0 taken (a compare-and-swap that only they race on), and the others
// add again.  The counter thus never needs a reset.
__device__ int64_t take_strip(unsigned long long *tick, uint32_t epoch) {
    uint32_t t = 0;
    if (__lane_id() == 0) {
        for (bool got = false; !got;) {
            const unsigned long long old = atomicAdd(tick, 1ull);
            if ((uint32_t)(old >> 32) == epoch) {
                t = (uint32_t)old;
                break;
            }
            const unsigned long long mine = ((unsigned long long)epoch << 32) | 1ull;
            unsigned long long cur = old + 1ull;
            for (;;) {
                const unsigned long long seen = atomicCAS(tick, cur, mine);
                if (seen == cur) {
                    t = 0;
                    got = true;
                    break;
                }
                if ((uint32_t)(seen >> 32) == epoch) break;  // installed by another wave
                cur = seen;
            }
        }
    }
    return (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane(t);
}

// Waves that take part in a sweep of nstrips strips: one per strip at most, so that the ticket
// counter sees few contenders (a wave finishing its strip takes the next one).
__device__ __forceinline__ int64_t strip_takers(int64_t nstrips, int64_t nwave) {
    return nstrips < nwave ? nstrips : nwave;
}

// Rows a strip hands on at a time (one per lane).  A sweep takes about m / R + nstrips batch
// times of R t + L (t per row, L the hand-over latency), least at R = sqrt(m L / (nstrips t));
// measured L / t is about 8 (all-ones 8192^2: R = 32 best, 4096 x 32768: 8-16, 3000 x 40000: 8),
// so R is the power of two in 8..64 nearest that.  `forced` in 1..64 overrides the choice.
__device__ __forceinline__ int strip_rows(int64_t m, int64_t nstrips, int forced) {
    if (forced >= 1 && forced <= WAVE) return forced;
    const int64_t x = 8 * m / (nstrips > 0 ? nstrips : 1);
    int r = 8;
    while (r < WAVE && 2 * (int64_t)r * r <= x) r *= 2;
    return r;
}

__device__ __forceinline__ int64_t strip_count(int64_t n) {
    return (((n + 63) >> 6) + mshost::STRIP_WORDS - 1) / mshost::STRIP_WORDS;
}

template <bool STORE>
__device__ void strip_sweep(const uint64_t *__restrict__ bits, int64_t m, int64_t n, int64_t ldw,
                            int32_t *__restrict__ dp, int64_t ld_dp, int64_t s,
                            unsigned long long *bnd, uint32_t epoch, uint32_t *timeout,
                            int R, Track &tr) {
    constexpr int SW = mshost::STRIP_WORDS;
    const int lane = __lane_id();
    const int64_t nwords = (n + 63) >> 6;
    const uint64_t lastmask = last_word_mask(n);
    const unsigned long long tag = (unsigned long long)epoch + 1ull;
    const int64_t w0 = s * SW;
    unsigned long long *mine = bnd + s * m * 2;
    const unsigned long long *left = s > 0 ? bnd + (s - 1) * m * 2 : nullptr;
    const bool publish = s + 1 < strip_count(n);
    int32_t H[SW], D[SW];
#pragma unroll
    for (int u = 0; u < SW; ++u) H[u] = D[u] = 0;
    int32_t dl = 0;  // dp of the previous row at the column just left of the strip
    // the strip's words of rows i0 .. i0 + R - 1, row i0 + l in lane l
    auto load_rows = [&](int64_t i0, uint64_t(&v)[SW]) {
        const int64_t i = i0 + lane;
#pragma unroll
        for (int u = 0; u < SW; ++u)
            v[u] = (lane < R && i < m) ? row_word(bits + i * ldw, w0 + u, nwords, lastmask)
                                       : 0ull;
    };
    uint64_t x[SW];
    load_rows(0, x);
    for (int64_t i0 = 0; i0 < m; i0 += R) {
        uint64_t nx[SW];
        load_rows(i0 + R, nx);
        int32_t win = 0, din = 0;
        if (left) {
            const int64_t i = i0 + lane;
            unsigned long long a = tag << 20, b = tag << 20;
            const bool mine_row = lane < R && i < m;
            if (mine_row) {
                a = load_relaxed(left + 2 * i);
                b = load_relaxed(left + 2 * i + 1);
            }
            for (uint32_t polls = 0;; ++polls) {
                const bool ok = (a >> 20) == tag && (b >> 20) == tag;
                if (__ballot(!ok) == 0ull) break;
                // once any wait of the launch has given up, none waits any longer
                if (polls >= SPIN_LIMIT ||
                    (polls % 1024u == 1023u && load_relaxed_u32(timeout) == epoch + 1u)) {
                    if (lane == 0) atomicExch(timeout, epoch + 1u);
                    break;
                }
                __builtin_amdgcn_s_sleep(4);
                if (!ok) {
                    a = load_relaxed(left + 2 * i);
                    b = load_relaxed(left + 2 * i + 1);
                }
            }
            win = (int32_t)(a & 0xFFFFFull);
            din = (int32_t)(b & 0xFFFFFull);
        }
        const int rows = (int)(m - i0 < R ? m - i0 : R);
        int32_t ow = 0, od = 0;
        for (int r = 0; r < rows; ++r) {
            int32_t wc = __builtin_amdgcn_readlane(win, r);  // row run entering the strip
            int32_t dleft = dl;                              // previous row, column left of word
            dl = __builtin_amdgcn_readlane(din, r);
            const int64_t i = i0 + r;
#pragma unroll
            for (int u = 0; u < SW; ++u) {
                const uint64_t xv = lane_u64(x[u], r);
                const int32_t a = (int32_t)((xv >> lane) & 1u);
                const int32_t lo = (int32_t)__clzll(~(xv << (63 - lane)));
                const int32_t wl = a ? ((lo == lane + 1) ? lane + 1 + wc : lo) : 0;
                const int32_t h = a ? (H[u] < HEIGHT_CAP ? H[u] + 1 : HEIGHT_CAP) : 0;
                const int32_t dprev = from_left_lane(D[u], dleft);
                dleft = __builtin_amdgcn_readlane(D[u], WAVE - 1);
                int32_t d = h < wl ? h : wl;
                d = d < dprev + 1 ? d : dprev + 1;
                if (!a) d = 0;
                H[u] = h;
                D[u] = d;
                const int64_t c = (w0 + u) * 64 + lane;
                if (c < n) {
                    if (STORE) dp[i * ld_dp + c] = d;
                    if (d > tr.v) {
                        tr.v = d;
                        tr.pos = i * n + c;
                    }
                }
                wc = (xv == ~0ull) ? (wc < RUN_CAP - 64 ? wc + 64 : RUN_CAP) : leading_ones(xv);
            }
            const int32_t dlast = __builtin_amdgcn_readlane(D[SW - 1], WAVE - 1);
            ow = lane == r ? wc : ow;
            od = lane == r ? dlast : od;
        }
        if (publish && lane < R && i0 + lane < m) {
            const int64_t i = i0 + lane;
            store_relaxed_u64(mine + 2 * i, (tag << 20) | (unsigned long long)(uint32_t)ow);
            store_relaxed_u64(mine + 2 * i + 1, (tag << 20) | (unsigned long long)(uint32_t)od);
        }
#pragma unroll
        for (int u = 0; u < SW; ++u) x[u] = nx[u];
    }
}

// The map's sweep: the first strip_takers waves of the launch take strips until none is left;
// the wave taking the launch's last ticket (each taker ends on one past the strips) bumps the
// epoch for the next launch (every taker read it before its first ticket).
__device__ void strip_map(const uint64_t *__restrict__ bits, int64_t m, int64_t n, int64_t ldw,
                          int32_t *__restrict__ dp, int64_t ld_dp, mshost::ScratchHeader *hdr,
                          unsigned long long *bnd, int forced_rows) {
    const int64_t nstrips = strip_count(n);
    const int64_t takers = strip_takers(nstrips, ((int64_t)gridDim.x * blockDim.x) / WAVE);
    if (wave_index() >= takers) return;
    const uint32_t epoch = (uint32_t)uniform((int32_t)(load_relaxed(&hdr->done_epoch) >> 32));
    const int R = strip_rows(m, nstrips, forced_rows);
    for (;;) {
        const int64_t s = take_strip(&hdr->tick, epoch);
        if (s >= nstrips) {
            if (s == nstrips + takers - 1 && __lane_id() == 0)
                __hip_atomic_store(&hdr->done_epoch, (unsigned long long)(epoch + 1u) << 32,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        Track tr{0, INT64_MAX};
        strip_sweep<true>(bits, m, n, ldw, dp, ld_dp, s, bnd, epoch, &hdr->timeout, R, tr);
    }
}

// One wave: key -> result (for a square too wide for the resolve pass, the strip sweep's key,
// or without boundary words the one-wave serial pass), then clear the header for the next call
// and bump its epoch.
__device__ void finalize_wave(const uint64_t *__restrict__ bits, int64_t m, int64_t n,
                              int64_t ldw, mshost::ScratchHeader *hdr, int32_t *serial_state,
                              ms_square *out, const uint32_t *__restrict__ box_rec,
                              int64_t nrec, bool strips, uint32_t epoch) {
    const int lane = __lane_id();
    if (box_rec) {
        // fold the probe blocks' box records for the map of the same call
        // 16-byte records, eight per lane in flight at a time
        static_assert(mshost::BOX_RECORD_WORDS == 4, "one uint4 per record");
        const uint4 *rec = reinterpret_cast<const uint4 *>(box_rec);
        uint32_t b[4] = {0, 0, 0, 0};
        for (int64_t i0 = 0; i0 < nrec; i0 += 8 * WAVE) {
            uint4 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t i = i0 + u * WAVE + lane;
                v[u] = i < nrec ? rec[i] : make_uint4(0, 0, 0, 0);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                b[0] = v[u].x > b[0] ? v[u].x : b[0];
                b[1] = v[u].y > b[1] ? v[u].y : b[1];
                b[2] = v[u].z > b[2] ? v[u].z : b[2];
                b[3] = v[u].w > b[3] ? v[u].w : b[3];
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) b[k] = (uint32_t)wave_max_i32((int32_t)b[k]);
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) hdr->big_box[k] = b[k];
        }
    }
    // both loads in flight together (device-scope: written by other waves' atomics)
    unsigned long long key = load_relaxed(&hdr->key);
    const uint32_t flag = load_relaxed_u32(&hdr->serial_flag);
    bool failed = false;
    if (flag && strips) {
        key = load_relaxed(&hdr->skey);
        failed = load_relaxed_u32(&hdr->timeout) == epoch + 1u;
    } else if (flag) {
        const int64_t nw64 = ((n + 63) >> 6) * 64;
        Track tr{0, INT64_MAX};
        serial_dp<false>(bits, m, n, ldw, nullptr, 0, serial_state, serial_state + nw64, tr);
        const Track w = wave_track(tr);
        key = w.v > 0 ? make_key(w.v, w.pos) : 0ull;
    }
    if (lane == 0) {
        ms_square r;
        write_result(key, n, &r);
        if (failed) r = ms_square{-1, -1, -1};
        hdr->result = r;
        if (out) *out = r;
        hdr->key = 0;
        hdr->serial_flag = 0;
        hdr->nsat = 0;
        hdr->done_epoch = (unsigned long long)(epoch + 1u) << 32;  // count 0, next epoch
        hdr->skey = 0;
        hdr->fin = 0;
        hdr->sdone = 0;
    }
}

// One of the two arrivals that end a search with a strip sweep (the last resolve wave, and the
// wave that finished the last strip): true for the second, which then writes the result.
__device__ bool fin_arrive(mshost::ScratchHeader *hdr) {
    __threadfence();
    uint32_t f = 0;
    if (__lane_id() == 0) f = atomicAdd(&hdr->fin, 1u);
    f = (uint32_t)__builtin_amdgcn_readfirstlane(f);
    if (f == 1u) __threadfence();
    return f == 1u;
}

// After the probe: if any tile saturated, finish those tiles exactly, then the last wave to
// finish (a completion count, no waiting) writes the result.  With no saturated tile, the first
// wave writes it at once and every other wave returns.  The wave that writes the result also
// folds the probe blocks' large-tile box records.
//  * Few saturated tiles (at most one per block: wide squares, whose tiles have long height
//    scans): one block of RESOLVE_WAVES waves per tile (resolve_tile_block), tiles dealt to
//    blocks by index modulo the grid so that clustered tiles land on different blocks.
//  * Many (blob images): one wave per RESOLVE_GROUP neighbouring tiles of a tile row
//    (resolve_group), sharing one window and one height scan; there the work, not the length
//    of each chain, is what costs, and one wave per group does the least of it.
// Neighbouring tile columns one wave resolves together in the second case (at most 32).  On a
// 16384^2 blob image (2804 of 3042 tiles saturated) the search takes 440 us one tile per wave
// and 339 / 343 / 355 us with groups of 2 / 3 / 4.
constexpr int RESOLVE_GROUP = 2;
// At most this many waves of a search sweep strips (each takes strip after strip).
constexpr int64_t RESOLVE_SWEEPERS = 256;

// The strip words the host recorded in the header, if they cover an m x n sweep.
__device__ __forceinline__ unsigned long long *header_strips(mshost::ScratchHeader *hdr,
                                                             int64_t m, int64_t n) {
    unsigned long long *w = reinterpret_cast<unsigned long long *>(hdr->strips_ptr);
    return (w && strip_count(n) * m * 2 <= hdr->strip_cap) ? w : nullptr;
}

// The search's strip sweep, by one of the waves that saw the serial flag (the last wave to
// arrive among them): strips until none is left, each strip's best pushed into hdr->skey.
// Returns whether the calling wave writes the result.  Kept out of line: the resolve pass's own
// code and registers stay as they are without it.
__device__ __attribute__((noinline)) bool resolve_sweep(
    const uint64_t *__restrict__ bits, int64_t m, int64_t n, int64_t ldw,
    mshost::ScratchHeader *hdr, unsigned long long *bnd, uint32_t epoch, bool last,
    int forced_rows) {
    const int lane = __lane_id();
    const int64_t nstrips = strip_count(n);
    bool finish = last && fin_arrive(hdr);
    const int R = strip_rows(m, nstrips, forced_rows);
    for (;;) {
        const int64_t st = take_strip(&hdr->tick, epoch);
        if (st >= nstrips) break;
        Track tr{0, INT64_MAX};
        strip_sweep<false>(bits, m, n, ldw, nullptr, 0, st, bnd, epoch, &hdr->timeout, R, tr);
        const Track w = wave_track(tr);
        if (lane == 0 && w.v > 0) atomicMax(&hdr->skey, make_key(w.v, w.pos));
        __threadfence();
        uint32_t k = 0;
        if (lane == 0) k = atomicAdd(&hdr->sdone, 1u);
        k = (uint32_t)__builtin_amdgcn_readfirstlane(k);
        if (k == (uint32_t)(nstrips - 1) && fin_arrive(hdr)) finish = true;
    }
    return finish;
}

template <class TS>
__global__ __launch_bounds__(64 * RESOLVE_WAVES) void k_resolve(
    const uint64_t *__restrict__ bits, int64_t m, int64_t n, int64_t ldw, int64_t ntiles,
    int64_t ntx, mshost::ScratchHeader *hdr, const uint8_t *__restrict__ sat,
    int32_t *__restrict__ bounds, const uint32_t *__restrict__ box_rec, int64_t nrec,
    int32_t *serial_state, ms_square *out) {
    __shared__ ResolveLds L;
    const int lane = __lane_id();
    const int64_t wave = wave_index();
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) / WAVE;
    const int64_t nblk = gridDim.x;
    const uint32_t nsat = (uint32_t)uniform((int32_t)load_relaxed_u32(&hdr->nsat));
    if (nsat == 0) {
        if (wave == 0)
            finalize_wave(bits, m, n, ldw, hdr, serial_state, out, box_rec, nrec, false,
                          (uint32_t)(load_relaxed(&hdr->done_epoch) >> 32));
        return;
    }
    if ((int64_t)nsat <= nblk) {
        // saturated tiles t = blockIdx.x + k * gridDim.x, found 64 at a time; every wave of the
        // block reads the same bytes, so the block agrees on its sequence of tiles
        for (int64_t base = blockIdx.x; base < ntiles; base += 64 * nblk) {
            const int64_t t = base + (int64_t)lane * nblk;
            uint64_t b = __ballot(t < ntiles && sat[t] != 0);
            while (b) {
                const int l = __ffsll((long long)b) - 1;
                b &= b - 1;
                const int64_t tt = base + (int64_t)l * nblk;
                const int64_t ty = tt / ntx, tx = tt - ty * ntx;
                resolve_tile_block<TS, RESOLVE_WAVES>(bits, m, n, ldw, ty, tx, ntx, sat,
                                                      &hdr->key, &hdr->serial_flag, bounds, L);
            }
        }
    } else {
        const int64_t ngx = (ntx + RESOLVE_GROUP - 1) / RESOLVE_GROUP;
        const int64_t ngroups = (ntiles / ntx) * ngx;
        for (int64_t base = wave; base < ngroups; base += 64 * nwave) {
            const int64_t gi = base + (int64_t)lane * nwave;
            bool any = false;
            if (gi < ngroups) {
                const int64_t gy = gi / ngx, tx0 = (gi - gy * ngx) * RESOLVE_GROUP;
                for (int k = 0; k < RESOLVE_GROUP && tx0 + k < ntx; ++k)
                    any |= sat[gy * ntx + tx0 + k] != 0;
            }
            uint64_t b = __ballot(any);
            while (b) {
                const int l = __ffsll((long long)b) - 1;
                b &= b - 1;
                const int64_t gg = base + (int64_t)l * nwave;
                const int64_t gy = gg / ngx, tx0 = (gg - gy * ngx) * RESOLVE_GROUP;
                const int64_t tx1 = tx0 + RESOLVE_GROUP - 1 < ntx ? tx0 + RESOLVE_GROUP - 1 : ntx - 1;
                uint32_t rest = resolve_group<TS>(bits, m, n, ldw, gy, tx0, tx1, ntx, sat,
                                                  &hdr->key, bounds);
                for (; rest; rest &= rest - 1)
                    resolve_tile<TS>(bits, m, n, ldw, gy, tx0 + (__ffs(rest) - 1), ntx, sat,
                                     &hdr->key, &hdr->serial_flag, bounds);
            }
        }
    }
    __threadfence();
    unsigned long long prev64 = 0;
    if (lane == 0) prev64 = atomicAdd(&hdr->done_epoch, 1ull);
    const uint32_t prev = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)prev64);
    const uint32_t epoch = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(prev64 >> 32));
    const bool last = prev == (uint32_t)(nwave - 1);
    if (last) __threadfence();
    // The possible sweepers: the last few waves to arrive (the last one among them).  Every wave
    // that raised the flag did so before its completion count, so the last wave sees it; an
    // earlier one that misses it only leaves the sweep to the others.  The other waves read
    // nothing more (an extra read per wave here measured 25 % slower searches).
    const int64_t nstrips = strip_count(n);
    const int64_t takers = strip_takers(nstrips, nwave < RESOLVE_SWEEPERS ? nwave
                                                                           : RESOLVE_SWEEPERS);
    unsigned long long *bnd = nullptr;
    if (nwave - 1 - (int64_t)prev < takers &&
        uniform((int32_t)load_relaxed_u32(&hdr->serial_flag)) != 0)
        bnd = header_strips(hdr, m, n);
    if (!bnd) {
        // with the flag raised and no strip words for this shape: the one-wave serial pass
        if (last)
            finalize_wave(bits, m, n, ldw, hdr, serial_state, out, box_rec, nrec, false, epoch);
        return;
    }
    if (resolve_sweep(bits, m, n, ldw, hdr, bnd, epoch, last, hdr->strip_rows_forced))
        finalize_wave(bits, m, n, ldw, hdr, serial_state, out, box_rec, nrec, true, epoch);
}

// The narrow pass of the map (one wave per item, windows of NGMAX groups of 64 * CPL columns):
// every cell when S <= MAP_NARROW_REACH; in region mode (S beyond the reach, per-tile bounds of
// a search in the same call) the cells of the tiles bounded by REGION_SMALL, with REGION_SMALL
// halos.  Band height: at least band_rows and 4 S (so the S-row head start costs at most a
// quarter), halved while that leaves fewer items than min_items, down to S (or 8 rows): on a
// small matrix each item's chain of rows is the latency, and shorter bands shorten it.  Items go
// to waves wave, wave + nwave, ... (the caller's numbering of the waves taking part).
template <int NGMAX, int CPL>
__device__ void narrow_pass(const uint64_t *__restrict__ bits, int64_t m, int64_t n, int64_t ldw,
                            int32_t *__restrict__ dp, int64_t ld_dp, int64_t S,
                            int64_t band_rows, int vec_ok, bool region,
                            const int32_t *__restrict__ bounds, int64_t tile_rows,
                            int64_t tile_ntx, int64_t min_items, WaveLds lds, int64_t wave,
                            int64_t nwave) {
    constexpr int64_t GW = 64 * CPL;
    constexpr int64_t TILE_COLS = 64 * mshost::PROBE_TILE_WORDS;
    const int64_t Sg = region ? REGION_SMALL : S;  // the side the halos must cover
    const int64_t hc = (Sg + 63) & ~(int64_t)63;
    int64_t ng = (hc + (4 * hc > 256 ? 4 * hc : 256) + GW - 1) / GW;
    ng = ng < 1 ? 1 : (ng > NGMAX ? NGMAX : ng);
    const int64_t rmin = Sg > 8 ? Sg : 8;
    // where even the shortest bands leave fewer items than min_items (a small matrix: each
    // wave's sequence of rows is the latency), a window one group narrower halves every row's
    // work, as long as it still leaves a 64-column output
    if (ng > 1 && (ng - 1) * GW >= hc + 64 &&
        udiv(m + rmin - 1, rmin) * udiv(n + ng * GW - hc - 1, ng * GW - hc) < min_items)
        ng -= 1;
    const int64_t ow = ng * GW - hc;
    const int64_t nwin = udiv(n + ow - 1, ow);
    // the tallest bands (the least halo work) that still leave min_items items
    int64_t R = band_rows > 4 * Sg ? band_rows : 4 * Sg;
    while (R > rmin && udiv(m + R - 1, R) * nwin < min_items) R = (R / 2 > rmin) ? R / 2 : rmin;
    // in region mode an item stays within 32 tile rows (one mask bit per tile row)
    if (region) R = R < 32 * tile_rows ? R : 32 * tile_rows;
    R = R < m ? R : m;
    const int64_t items = udiv(m + R - 1, R) * nwin;
    const int lane = __lane_id();
    Track dummy{0, 0};
    for (int64_t it = wave; it < items; it += nwave) {
        const int64_t b = udiv(it, nwin), wdx = it - b * nwin;
        const int64_t ra = b * R, rb = ra + R < m ? ra + R : m;
        const int64_t rh = ra - Sg > 0 ? ra - Sg : 0;
        const int64_t xa = wdx * ow, xb = xa + ow < n ? xa + ow : n;
        const int64_t xh = xa - hc > 0 ? xa - hc : 0;
        const int ngi = (int)((xb - xh + GW - 1) / GW);
        StoreClass<NGMAX> sc;
        if (region) {
            sc.on = true;
            sc.tile_rows = tile_rows;
            sc.ty0 = udiv(ra, tile_rows);
            const int64_t nk = udiv(rb - 1, tile_rows) - sc.ty0 + 1;  // <= 33
            bool any = false;
#pragma unroll
            for (int g = 0; g < NGMAX; ++g) {
                sc.cls[g] = 0;
                const int64_t col = xh + (int64_t)g * GW + (int64_t)lane * CPL;
                if (g < ngi && col >= xa && col < xb) {
                    const int64_t tc = col / TILE_COLS;
                    for (int64_t k = 0; k < nk; ++k) {
                        const int32_t bnd = bounds[(sc.ty0 + k) * tile_ntx + tc];
                        const bool big = bnd < 0 || bnd > REGION_SMALL;
                        if (!big) sc.cls[g] |= 1ull << k;
                    }
                }
                any |= sc.cls[g] != 0;
            }
            if (!__ballot(any)) continue;  // no small tile here
            dprun<NGMAX, CPL, true, false, true>(bits, ldw, n, rh, ra, rb, xh, xa, xb, ngi, dp,
                                                 ld_dp, vec_ok != 0, dummy, lds, sc);
        } else {
            dprun<NGMAX, CPL, true, false>(bits, ldw, n, rh, ra, rb, xh, xa, xb, ngi, dp, ld_dp,
                                           vec_ok != 0, dummy, lds);
        }
    }
}

// The wide pass of the map (MAP_NARROW_REACH < S <= 1984): windows of 2048 columns, one window
// per block (dprun_block), items distributed per block so that the block's barriers stay
// uniform.  In region mode only the cells of tiles bounded above REGION_SMALL (or saturated) are
// stored, with S halos, and the pass returns how many items it dealt (the k-th to block
// k mod gridDim.x).  Beyond 1984 one wave sweeps the whole matrix.
__device__ int64_t wide_pass(const uint64_t *__restrict__ bits, int64_t m, int64_t n, int64_t ldw,
                          int32_t *__restrict__ dp, int64_t ld_dp, int64_t S, int64_t band_rows,
                          int32_t *serial_state, int vec_ok, bool region,
                          const int32_t *__restrict__ bounds, int64_t tile_rows,
                          int64_t tile_ntx, BlockLds L, const uint32_t *box,
                          mshost::ScratchHeader *hdr, unsigned long long *bnd, int forced_rows) {
    constexpr int64_t GW = 256, NGB = 8, WIN = NGB * GW, REACH = WIN - 64;
    constexpr int64_t TILE_COLS = 64 * mshost::PROBE_TILE_WORDS;
    const int64_t hc = (S + 63) & ~(int64_t)63;
    if (hc > REACH) {
        if (bnd) {  // every wave of the launch sweeps strips; every cell is stored
            strip_map(bits, m, n, ldw, dp, ld_dp, hdr, bnd, forced_rows);
            return -1;
        }
        if (blockIdx.x == 0 && threadIdx.x < WAVE) {
            const int64_t nw64 = ((n + 63) >> 6) * 64;
            Track tr{0, INT64_MAX};
            serial_dp<true>(bits, m, n, ldw, dp, ld_dp, serial_state, serial_state + nw64, tr);
        }
        return 0;
    }
    const int64_t ow = WIN - hc;
    const int64_t nwin = (n + ow - 1) / ow;
    const int64_t nblk = gridDim.x;
    int64_t R;
    if (region) {
        R = 2 * tile_rows;  // few items touch wide tiles: short bands spread them out
    } else {
        R = band_rows > 4 * S ? band_rows : 4 * S;
        const int64_t rmin = 2 * S;
        while (R > rmin && ((m + R - 1) / R) * nwin < nblk) R = (R / 2 > rmin) ? R / 2 : rmin;
    }
    R = R < m ? R : m;
    const int64_t items = ((m + R - 1) / R) * nwin;
    const int wv = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    if (!region) {
        for (int64_t it = blockIdx.x; it < items; it += nblk) {
            const int64_t bnd_i = it / nwin, wdx = it - bnd_i * nwin;
            const int64_t ra = bnd_i * R, rb = ra + R < m ? ra + R : m;
            const int64_t rh = ra - S > 0 ? ra - S : 0;
            const int64_t xa = wdx * ow, xb = xa + ow < n ? xa + ow : n;
            const int64_t xh = xa - hc > 0 ? xa - hc : 0;
            const int ngi = (int)((xb - xh + GW - 1) / GW);
            dprun_block<false>(bits, ldw, n, rh, ra, rb, xh, xa, xb, ngi, dp, ld_dp, vec_ok != 0,
                               L, StoreClass<2>{});
        }
        return 0;
    }
    // Region mode: only items touching a tile bounded above REGION_SMALL (or saturated) have
    // cells to store, and they cluster around the large squares, so dealing items to blocks by
    // index would stack several on one block.  Every block instead ranks those items in item
    // order (256 per round: a ballot per wave and the four wave counts) and maps the ones whose
    // rank is its index modulo the grid.  Only the items meeting the search's bounding box of
    // such tiles are ranked: bands kb0..kb1 and windows kw0..kw1, in item order.
    const uint32_t e0 = box[0], e1 = box[1], e2 = box[2], e3 = box[3];
    if (e1 == 0) return 0;  // no tile beyond the narrow pass's halo
    const int64_t ty_lo = (int64_t)(BOX_LOW - e0), ty_hi = (int64_t)e1 - 1;
    const int64_t tx_lo = (int64_t)(BOX_LOW - e2), tx_hi = (int64_t)e3 - 1;
    const int64_t nbands = (m + R - 1) / R;
    const int64_t kb0 = ty_lo * tile_rows / R;
    int64_t kb1 = ((ty_hi + 1) * tile_rows - 1) / R;
    kb1 = kb1 < nbands - 1 ? kb1 : nbands - 1;
    const int64_t kw0 = tx_lo * TILE_COLS / ow;
    int64_t kw1 = ((tx_hi + 1) * TILE_COLS - 1) / ow;
    kw1 = kw1 < nwin - 1 ? kw1 : nwin - 1;
    const int64_t bw = kw1 - kw0 + 1;
    const int64_t boxed = (kb1 - kb0 + 1) * bw;
    __shared__ int32_t s_cnt[4];
    __shared__ int32_t s_nsel;
    __shared__ int64_t s_sel[256];
    int64_t before = 0;  // active items in earlier rounds (the same in every thread)
    for (int64_t c0 = 0; c0 < boxed; c0 += 256) {
        const int64_t bi = c0 + threadIdx.x;  // index among the boxed items
        const int64_t kb = bi / bw;
        const int64_t it = (kb0 + kb) * nwin + kw0 + (bi - kb * bw);
        bool act = false;
        if (bi < boxed) {
            const int64_t bnd_i = it / nwin, wdx = it - bnd_i * nwin;
            const int64_t ra = bnd_i * R, rb = ra + R < m ? ra + R : m;
            const int64_t xa = wdx * ow, xb = xa + ow < n ? xa + ow : n;
            for (int64_t ty = ra / tile_rows; ty <= (rb - 1) / tile_rows; ++ty)
                for (int64_t tc = xa / TILE_COLS; tc <= (xb - 1) / TILE_COLS; ++tc) {
                    const int32_t bv = bounds[ty * tile_ntx + tc];
                    act |= bv < 0 || bv > REGION_SMALL;
                }
        }
        const uint64_t bal = __ballot(act);
        if (lane == 0) s_cnt[wv] = __popcll(bal);
        if (threadIdx.x == 0) s_nsel = 0;
        __syncthreads();
        int32_t wbase = 0;
        for (int w = 0; w < wv; ++w) wbase += s_cnt[w];
        const int64_t ctotal = (int64_t)s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
        if (act) {
            const int64_t rank = before + wbase + __popcll(bal & ((1ull << lane) - 1));
            if (rank % nblk == blockIdx.x) s_sel[atomicAdd(&s_nsel, 1)] = it;
        }
        __syncthreads();
        const int nsel = s_nsel;
        for (int k = 0; k < nsel; ++k) {
            const int64_t it2 = s_sel[k];
            const int64_t bnd_i = it2 / nwin, wdx = it2 - bnd_i * nwin;
            const int64_t ra = bnd_i * R, rb = ra + R < m ? ra + R : m;
            const int64_t rh = ra - S > 0 ? ra - S : 0;
            const int64_t xa = wdx * ow, xb = xa + ow < n ? xa + ow : n;
            const int64_t xh = xa - hc > 0 ? xa - hc : 0;
            const int ngi = (int)((xb - xh + GW - 1) / GW);
            StoreClass<2> sc;
            sc.on = true;
            sc.tile_rows = tile_rows;
            sc.ty0 = ra / tile_rows;
            const int64_t nk = (rb - 1) / tile_rows - sc.ty0 + 1;  // 2 or 3
#pragma unroll
            for (int gl = 0; gl < 2; ++gl) {
                sc.cls[gl] = 0;
                const int64_t col = xh + (int64_t)(wv * 2 + gl) * GW + (int64_t)lane * 4;
                if (wv * 2 + gl < ngi && col >= xa && col < xb) {
                    const int64_t tc = col / TILE_COLS;
                    for (int64_t kk = 0; kk < nk; ++kk) {
                        const int32_t bv = bounds[(sc.ty0 + kk) * tile_ntx + tc];
                        if (bv < 0 || bv > REGION_SMALL) sc.cls[gl] |= 1ull << kk;
                    }
                }
            }
            dprun_block<true>(bits, ldw, n, rh, ra, rb, xh, xa, xb, ngi, dp, ld_dp, vec_ok != 0,
                              L, sc);
        }
        before += ctotal;
        __syncthreads();  // the next round rewrites s_cnt, s_nsel and s_sel
    }
    return before;  // the items dealt, the same count in every block
}

// ---------------------------------------------------------------------------------- map
// One launch per map: a narrow pass (one wave per item, 512-column windows) for S up to
// MAP_NARROW_REACH, a wide pass (one block per item, 2048-column windows) beyond it, and in region
// mode (bounds != nullptr: each probe tile of a search in the same call carries an upper bound on
// its largest side) both, split by tile: the narrow pass maps the tiles bounded by REGION_SMALL
// with REGION_SMALL halos, the wide pass the others with S halos.  A cell is exact whenever its
// halo is at least its own dp.  Both passes share the block's 24 KB of LDS (the narrow pass as
// four per-wave regions); registers are held to five waves per SIMD without spilling.
template <int NGMAX, int CPL>
__global__ __launch_bounds__(256, 5) void k_dpmap(const uint64_t *__restrict__ bits, int64_t m,
                                               int64_t n, int64_t ldw, int32_t *__restrict__ dp,
                                               int64_t ld_dp,
                                               const ms_square *__restrict__ maxsq,
                                               int64_t band_rows, int32_t *serial_state,
                                               int vec_ok, const int32_t *__restrict__ bounds,
                                               int64_t tile_rows, int64_t tile_ntx,
                                               const uint32_t *big_box, int64_t min_items,
                                               mshost::ScratchHeader *hdr,
                                               unsigned long long *bnd, int forced_rows) {
    constexpr int LDSW = BLK_WORDS / 4;  // words per wave in the narrow pass
    static_assert(NGMAX * CPL * 64 <= LDSW, "a row chunk holds at least 64 rows");
    __shared__ uint64_t lx[BLK_WORDS];
    __shared__ int32_t lc[BLK_WORDS];
    __shared__ int32_t lslot[8];
    const int64_t S = uniform(maxsq->side);
    const bool region = bounds != nullptr && S > MAP_NARROW_REACH;
    const int wv = threadIdx.x / WAVE;
    const WaveLds wave_lds{lx + wv * LDSW, lc + wv * LDSW, LDSW};
    const int64_t nblk = gridDim.x;
    if (region) {
        // The block-wide items are long chains (S + R rows each) and few: they start first, and
        // the blocks holding one take no one-wave item, which the other blocks share.
        const int64_t dealt = wide_pass(bits, m, n, ldw, dp, ld_dp, S, band_rows, serial_state,
                                        vec_ok, true, bounds, tile_rows, tile_ntx,
                                        BlockLds{lx, lc, lslot}, big_box, hdr, bnd, forced_rows);
        if (dealt < 0) return;  // the strip sweep stored every cell
        const int64_t busy = dealt < nblk ? dealt : 0;  // blocks 0 .. busy-1 held a chain
        if ((int64_t)blockIdx.x < busy) return;
        __syncthreads();  // the narrow pass takes the block's LDS as four per-wave regions
        narrow_pass<NGMAX, CPL>(bits, m, n, ldw, dp, ld_dp, S, band_rows, vec_ok, true, bounds,
                                tile_rows, tile_ntx, min_items, wave_lds,
                                ((int64_t)blockIdx.x - busy) * 4 + wv, (nblk - busy) * 4);
    } else if (S <= MAP_NARROW_REACH) {
        narrow_pass<NGMAX, CPL>(bits, m, n, ldw, dp, ld_dp, S, band_rows, vec_ok, false, bounds,
                                tile_rows, tile_ntx, min_items, wave_lds, wave_index(),
                                nblk * 4);
    } else {
        wide_pass(bits, m, n, ldw, dp, ld_dp, S, band_rows, serial_state, vec_ok, false, bounds,
                  tile_rows, tile_ntx, BlockLds{lx, lc, lslot}, nullptr, hdr, bnd,
                  forced_rows);
    }
}

__global__ void k_write_result(ms_square *out, mshost::ScratchHeader *hdr, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = ms_square{0, -1, -1};
    if (hdr && blockIdx.x == 0 && threadIdx.x == 0) hdr->result = ms_square{0, -1, -1};
}

// Zero a scratch header with plain stores (a kernel rather than a memset, so that a captured
// graph replays it correctly).
__global__ void k_clear_header(mshost::ScratchHeader *hdr) {
    constexpr int W = (int)(sizeof(mshost::ScratchHeader) / sizeof(uint32_t));
    if (threadIdx.x < W) reinterpret_cast<uint32_t *>(hdr)[threadIdx.x] = 0u;
}

// Zero `words` 32-bit words (a context header) on the caller's stream: ordered before the
// launches that follow it there, which a memset on the null stream is not.
__global__ void k_zero_u64(uint64_t *p, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

__global__ void k_set_strips(mshost::ScratchHeader *hdr, unsigned long long words, int64_t count,
                             int forced_rows) {
    if (threadIdx.x == 0) {
        hdr->strips_ptr = words;
        hdr->strip_cap = count;
        hdr->strip_rows_forced = forced_rows;
    }
}

__global__ void k_zero_words(uint32_t *p, int words) {
    for (int i = threadIdx.x; i < words; i += blockDim.x) p[i] = 0u;
}

// ---------------------------------------------------------------------------------- batched
struct BatchCounters {
    uint32_t error;    // bit 1: the device tile total disagrees with the host's
    uint32_t nsat;     // saturated tiles over the whole batch
    uint32_t nserial;  // matrices flagged for the serial pass
    uint32_t done;     // blocks of the finishing kernel done with their saturated tiles
    uint32_t pad[4];
};

// The narrow tile of the batched path: 4 word columns (3 owned) x 16 row groups of 16 rows.
// Matrices a few words wide leave most of a 16-word tile empty; per matrix, the batch takes
// whichever tile does less erosion work (tiles x rows per lane, every tile being 64 lanes).
// The same rule runs on the host (the tile total) and on the device (tile starts, probe, resolve).
using TSN = TileShape<16, 16, 4>;

template <class TS>
__host__ __device__ __forceinline__ int64_t tile_count(int64_t m, int64_t n) {
    if (m <= 0 || n <= 0) return 0;
    const int64_t nwords = (n + 63) >> 6;
    return ((m + TS::TR - 1) / TS::TR) * ((nwords + TS::OWN_WORDS - 1) / TS::OWN_WORDS);
}

// The tile width of one matrix: narrow when 4 x its narrow-tile work is below q x its wide-tile
// work.  The default, q = 2, takes the narrow tile only where its work is below half the wide
// tile's: a narrow tile spends a quarter of its words on the halo and measures slower than its
// work alone says (the 45-matrix grid in one batch: 90 us with q = 2, 152 us with q = 4; the
// 10000-matrix batch 0.447 against 0.483 ms).  The batched autotuner also tries 0 (never
// narrow), 4 (the two works as they are) and 8 (narrow up to twice the wide tile's work).
constexpr int NARROW_DEFAULT = 2;
template <class TS>
__host__ __device__ __forceinline__ bool narrow_tiles(int64_t m, int64_t n, int q) {
    return tile_count<TSN>(m, n) * TSN::RPL * 4 < tile_count<TS>(m, n) * TS::RPL * q;
}

// Tiles of one matrix of a batch whose wide tile is TS.
template <class TS>
__device__ __forceinline__ uint64_t tiles_in(const ms_matrix &d, int q) {
    return (uint64_t)(narrow_tiles<TS>(d.m, d.n, q) ? tile_count<TSN>(d.m, d.n)
                                                     : tile_count<TS>(d.m, d.n));
}

// Fingerprint of a batch's shapes: the wrapping sum over i of a mix of (i, m, n, ld_words),
// computed the same way on the host (from its copy of the descriptors) and on the device.
__host__ __device__ __forceinline__ uint64_t shape_mix(uint64_t i, uint64_t m, uint64_t n,
                                                       uint64_t ldw) {
    uint64_t x = i * 0x9E3779B97F4A7C15ull ^ m * 0xC2B2AE3D27D4EB4Full ^
                 n * 0x165667B19E3779F9ull ^ ldw * 0xD6E8FEB86659FD93ull;
    x ^= x >> 31;  // splitmix64 finalizer
    x *= 0xBF58476D1CE4E5B9ull;
    x ^= x >> 29;
    x *= 0x94D049BB133111EBull;
    return x ^ (x >> 32);
}

// Where each matrix's tiles start in the batch's tile numbering, kept in two levels: the
// matrices are cut into init blocks of INIT_BLOCK; local[i] is the start of matrix i within its
// block and off[b] the start of block b (off[nblk] the total, or ~0 when the device
// descriptors disagree with the host's fingerprint).
constexpr int INIT_BLOCK = 256;

struct BatchIndex {
    const uint64_t *local;
    const uint64_t *off;
    int64_t count, nblk;
    __device__ uint64_t start(int64_t i) const { return off[i / INIT_BLOCK] + local[i]; }
    // The matrix holding tile `item` (< the total): the last matrix whose start is <= item
    // (matrices without tiles share the next one's start and are skipped).
    __device__ int64_t find(uint64_t item) const {
        int64_t lo = 0, hi = nblk;  // off[lo] <= item < off[hi]
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if (off[mid] <= item) lo = mid;
            else hi = mid;
        }
        const uint64_t rel = item - off[lo];
        int64_t a = lo * INIT_BLOCK;
        int64_t c = a + INIT_BLOCK < count ? a + INIT_BLOCK : count;  // local[a] <= rel
        while (c - a > 1) {
            const int64_t mid = (a + c) >> 1;
            if (local[mid] <= rel) a = mid;
            else c = mid;
        }
        return a;
    }
};

struct InitPart {
    uint64_t tiles, mix;  // an init block's tile count and wrapping sum of shape_mix
};

// Batch setup, first pass: one matrix per thread, INIT_BLOCK per block.  Clears the matrix's
// key and flag, writes its tile start within the block (an exclusive scan of tiles_in) and the
// block's totals; block 0 clears the counters.
template <class TS>
__global__ __launch_bounds__(INIT_BLOCK) void k_batch_count(const ms_matrix *__restrict__ mats,
                                                            int64_t count,
                                                            unsigned long long *__restrict__ keys,
                                                            uint64_t *__restrict__ local,
                                                            uint32_t *__restrict__ flags,
                                                            InitPart *__restrict__ parts,
                                                            BatchCounters *ctr, int q) {
    constexpr int NW = INIT_BLOCK / WAVE;
    __shared__ uint64_t wt[NW], wm[NW];
    const int lane = __lane_id(), wv = threadIdx.x / WAVE;
    const int64_t i = (int64_t)blockIdx.x * INIT_BLOCK + threadIdx.x;
    uint64_t t = 0, h = 0;
    if (i < count) {
        const ms_matrix d = mats[i];
        keys[i] = 0;
        flags[i] = 0;
        t = tiles_in<TS>(d, q);
        h = shape_mix((uint64_t)i, (uint64_t)d.m, (uint64_t)d.n, (uint64_t)d.ld_words);
    }
    uint64_t incl = t, hs = h;  // inclusive scan of t and sum of h over the wave
    for (int o = 1; o < WAVE; o <<= 1) {
        const uint64_t v = __shfl_up(incl, o);
        if (lane >= o) incl += v;
        hs += __shfl_xor(hs, o);
    }
    if (lane == WAVE - 1) wt[wv] = incl;
    if (lane == 0) wm[wv] = hs;
    __syncthreads();
    uint64_t before = 0, tot = 0, mtot = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        before += w < wv ? wt[w] : 0;
        tot += wt[w];
        mtot += wm[w];
    }
    if (i < count) local[i] = before + incl - t;
    if (threadIdx.x == 0) {
        parts[blockIdx.x] = InitPart{tot, mtot};
        if (blockIdx.x == 0) {
            ctr->error = 0;
            ctr->nsat = 0;
            ctr->nserial = 0;
            ctr->done = 0;
        }
    }
}

// Batch setup, second pass (one block): off[b] = exclusive scan of the blocks' tile counts, and
// off[nblk] = the total when the fingerprint of the device descriptors equals the host's, else
// an impossible value, so the probe refuses the batch and every result reads -1.
__global__ __launch_bounds__(1024) void k_batch_offsets(const InitPart *__restrict__ parts,
                                                        int64_t nblk, uint64_t *__restrict__ off,
                                                        uint64_t host_mix) {
    constexpr int NT = 1024, NW = NT / WAVE;
    __shared__ uint64_t wt[NW], wm[NW];
    const int lane = __lane_id(), wv = threadIdx.x / WAVE;
    uint64_t carry = 0, mix = 0;
    for (int64_t c0 = 0; c0 < nblk; c0 += NT) {
        const int64_t j = c0 + threadIdx.x;
        const InitPart p = j < nblk ? parts[j] : InitPart{0, 0};
        uint64_t incl = p.tiles, hs = p.mix;
        for (int o = 1; o < WAVE; o <<= 1) {
            const uint64_t v = __shfl_up(incl, o);
            if (lane >= o) incl += v;
            hs += __shfl_xor(hs, o);
        }
        if (lane == WAVE - 1) wt[wv] = incl;
        if (lane == 0) wm[wv] = hs;
        __syncthreads();
        uint64_t before = 0, tot = 0, mtot = 0;
        for (int w = 0; w < NW; ++w) {
            before += w < wv ? wt[w] : 0;
            tot += wt[w];
            mtot += wm[w];
        }
        if (j < nblk) off[j] = carry + before + incl - p.tiles;
        carry += tot;
        mix += mtot;
        __syncthreads();  // wt and wm are rewritten by the next chunk
    }
    if (threadIdx.x == 0) off[nblk] = mix == host_mix ? carry : ~0ull;
}

// Tiles of all matrices in one grid-stride pass; the item count comes from the host (it is
// computed from the same descriptors), so the loop is bounded by construction.  A mismatch with
// the device-side total marks the whole batch as failed instead of running.  The batched path
// keeps the probe's plain saturated search (DEEP = false): its small matrices rarely saturate,
// and the deep-row search made the common unsaturated tile slower.
template <class TS>
__global__ __launch_bounds__(256) void k_probe_batched(const ms_matrix *__restrict__ mats,
                                                       unsigned long long *__restrict__ keys,
                                                       const uint64_t *__restrict__ local,
                                                       const uint64_t *__restrict__ off,
                                                       int64_t count, int64_t nblk,
                                                       BatchCounters *ctr,
                                                       uint8_t *__restrict__ sat, uint64_t total,
                                                       int q) {
    // the index arrays come in as restrict-qualified kernel arguments (nothing in the kernel
    // writes them), so their wave-uniform reads can go through the scalar cache
    const BatchIndex ix{local, off, count, nblk};
    if (__hip_atomic_load(ix.off + ix.nblk, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != total) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&ctr->error, 2u);
        return;
    }
    // each wave takes a contiguous run of items and walks it matrix by matrix: one lookup per
    // matrix rather than per tile, and a matrix's tiles in row-major order, each seeing the best
    // side its predecessors pushed
    const uint64_t wave = (uint64_t)wave_index();
    const uint64_t nwave = ((uint64_t)gridDim.x * blockDim.x) / WAVE;
    const uint64_t per = (total + nwave - 1) / nwave;
    uint64_t item = wave * per;
    const uint64_t end = item + per < total ? item + per : total;
    SatBatch sb{sat};
    sb.stride = 1;
    while (item < end) {
        const int64_t mi = ix.find(item);
        const ms_matrix d = mats[mi];
        const int64_t nwords = (d.n + 63) >> 6;
        const uint64_t st = ix.start(mi);
        const bool narrow = uniform((int32_t)narrow_tiles<TS>(d.m, d.n, q)) != 0;
        const int64_t ntx = narrow ? (nwords + TSN::OWN_WORDS - 1) / TSN::OWN_WORDS
                                   : (nwords + TS::OWN_WORDS - 1) / TS::OWN_WORDS;
        const uint64_t mend = st + (uint64_t)(narrow ? tile_count<TSN>(d.m, d.n)
                                                     : tile_count<TS>(d.m, d.n));
        const uint64_t stop = mend < end ? mend : end;  // > item: item is one of mi's tiles
        const int64_t t = (int64_t)(item - st);
        int64_t ty = t / ntx, tx = t - ty * ntx;
        for (; item < stop; ++item) {
            const int32_t r =
                narrow ? tile_search<TSN, false>(d.bits, d.m, d.n, d.ld_words, ty, tx,
                                                 TileSink{keys + mi})
                       : tile_search<TS, false>(d.bits, d.m, d.n, d.ld_words, ty, tx,
                                                TileSink{keys + mi});
            sb.add((int64_t)item, r);
            if (++tx == ntx) {
                tx = 0;
                ++ty;
            }
        }
    }
    sb.flush();
    if (__lane_id() == 0 && sb.nsat) atomicAdd(&ctr->nsat, (uint32_t)sb.nsat);
}

// Key -> result of matrix i (the serial pass for a matrix flagged by the resolve pass, by the
// calling wave, within the workspace's serial state).
__device__ void batch_result(const ms_matrix *__restrict__ mats, int64_t i,
                             const unsigned long long *__restrict__ keys,
                             int32_t *serial_state, int64_t state_words, ms_square *out) {
    const ms_matrix d = mats[i];
    const int lane = __lane_id();
    const int64_t nwords = (d.n + 63) >> 6;
    if (uniform(nwords) > state_words) {  // wider than the state the workspace holds
        if (lane == 0) out[i] = ms_square{-1, -1, -1};
        return;
    }
    Track tr{0, INT64_MAX};
    serial_dp<false>(d.bits, d.m, d.n, d.ld_words, nullptr, 0, serial_state,
                     serial_state + nwords * 64, tr);
    const Track w = wave_track(tr);
    const unsigned long long key = w.v > 0 ? make_key(w.v, w.pos) : 0ull;
    if (lane == 0) write_result(key, d.n, out + i);
    (void)keys;
}

// After the probe: the results of every matrix.
//  * An inconsistent batch (the probe refused it): every result -1.
//  * No saturated tile (the common case): the keys are final; the grid writes the results,
//    one matrix per thread, at once.
//  * Otherwise the saturated tiles of every matrix are finished, each by a block of four waves
//    sharing its height scan (resolve_tile_block) when there are at most as many as blocks,
//    else each by one wave (resolve_tile); blocks count themselves done (a completion count,
//    nothing waits), and the last block writes every result; its first wave runs the serial
//    pass for the matrices whose square was too wide for the resolve window.
template <class TS>
__global__ __launch_bounds__(256) void k_batch_finish(const ms_matrix *__restrict__ mats,
                                                      unsigned long long *__restrict__ keys,
                                                      const uint64_t *__restrict__ local,
                                                      const uint64_t *__restrict__ off,
                                                      int64_t count, int64_t nblk,
                                                      uint32_t *__restrict__ flags,
                                                      BatchCounters *ctr,
                                                      const uint8_t *__restrict__ sat,
                                                      uint64_t total, int32_t *serial_state,
                                                      int64_t state_words, ms_square *out,
                                                      int q) {
    __shared__ ResolveLds L;
    const int lane = __lane_id();
    const BatchIndex ix{local, off, count, nblk};
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nthr = (int64_t)gridDim.x * blockDim.x;
    if (uniform((int32_t)load_relaxed_u32(&ctr->error)) & 2) {
        for (int64_t i = tid; i < count; i += nthr) out[i] = ms_square{-1, -1, -1};
        return;
    }
    const uint32_t nsat = (uint32_t)uniform((int32_t)load_relaxed_u32(&ctr->nsat));
    if (nsat == 0) {
        for (int64_t i = tid; i < count; i += nthr) {
            const ms_matrix d = mats[i];
            write_result(load_relaxed(keys + i), d.n, out + i);
        }
        return;
    }
    const uint64_t wave = (uint64_t)wave_index();
    const uint64_t nwave = ((uint64_t)gridDim.x * blockDim.x) / WAVE;
    const uint64_t nb = gridDim.x;
    // Few saturated tiles (a large square or a blob in a small batch): one block per tile, its
    // four waves sharing the tile's height scan, tiles dealt to blocks by index modulo the grid;
    // every wave of a block reads the same bytes, so the block agrees on its sequence of tiles.
    for (uint64_t base = blockIdx.x; nsat <= nb && base < total; base += 64 * nb) {
        const uint64_t g = base + (uint64_t)lane * nb;
        uint64_t b = __ballot(g < total && sat[g] != 0);
        while (b) {
            const int l = __ffsll((long long)b) - 1;
            b &= b - 1;
            const uint64_t item = base + (uint64_t)l * nb;
            const int64_t mi = ix.find(item);
            const ms_matrix d = mats[mi];
            const int64_t nwords = (d.n + 63) >> 6;
            const uint64_t st = ix.start(mi);
            const int64_t t = (int64_t)(item - st);
            if (uniform((int32_t)narrow_tiles<TS>(d.m, d.n, q))) {
                const int64_t ntx = (nwords + TSN::OWN_WORDS - 1) / TSN::OWN_WORDS;
                const int64_t ty = udiv(t, ntx), tx = t - ty * ntx;
                resolve_tile_block<TSN, RESOLVE_WAVES>(d.bits, d.m, d.n, d.ld_words, ty, tx, ntx,
                                                       sat + st, keys + mi, flags + mi, nullptr,
                                                       L, &ctr->nserial);
            } else {
                const int64_t ntx = (nwords + TS::OWN_WORDS - 1) / TS::OWN_WORDS;
                const int64_t ty = udiv(t, ntx), tx = t - ty * ntx;
                resolve_tile_block<TS, RESOLVE_WAVES>(d.bits, d.m, d.n, d.ld_words, ty, tx, ntx,
                                                      sat + st, keys + mi, flags + mi, nullptr,
                                                      L, &ctr->nserial);
            }
        }
    }
    // many: one wave per tile
    for (uint64_t base = wave; nsat > nb && base < total; base += 64 * nwave) {
        const uint64_t g = base + (uint64_t)lane * nwave;
        uint64_t b = __ballot(g < total && sat[g] != 0);
        while (b) {
            const int l = __ffsll((long long)b) - 1;
            b &= b - 1;
            const uint64_t item = base + (uint64_t)l * nwave;
            const int64_t mi = ix.find(item);
            const ms_matrix d = mats[mi];
            const int64_t nwords = (d.n + 63) >> 6;
            const uint64_t st = ix.start(mi);
            const int64_t t = (int64_t)(item - st);
            if (uniform((int32_t)narrow_tiles<TS>(d.m, d.n, q))) {
                const int64_t ntx = (nwords + TSN::OWN_WORDS - 1) / TSN::OWN_WORDS;
                const int64_t ty = udiv(t, ntx), tx = t - ty * ntx;
                resolve_tile<TSN>(d.bits, d.m, d.n, d.ld_words, ty, tx, ntx, sat + st,
                                  keys + mi, flags + mi, nullptr, 0, 1, &ctr->nserial);
            } else {
                const int64_t ntx = (nwords + TS::OWN_WORDS - 1) / TS::OWN_WORDS;
                const int64_t ty = udiv(t, ntx), tx = t - ty * ntx;
                resolve_tile<TS>(d.bits, d.m, d.n, d.ld_words, ty, tx, ntx, sat + st,
                                 keys + mi, flags + mi, nullptr, 0, 1, &ctr->nserial);
            }
        }
    }
    // the last block to finish writes every result
    __threadfence();
    __syncthreads();
    __shared__ uint32_t s_last;
    if (threadIdx.x == 0) s_last = atomicAdd(&ctr->done, 1u) == gridDim.x - 1;
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    for (int64_t i = threadIdx.x; i < count; i += blockDim.x) {
        const ms_matrix d = mats[i];
        const bool serial = d.m > 0 && d.n > 0 && load_relaxed_u32(flags + i);
        if (!serial) write_result(load_relaxed(keys + i), d.n, out + i);
    }
    if (threadIdx.x >= WAVE || load_relaxed_u32(&ctr->nserial) == 0) return;
    for (int64_t b0 = 0; b0 < count; b0 += WAVE) {
        bool flagged = false;
        if (b0 + lane < count) {
            const ms_matrix d = mats[b0 + lane];
            flagged = d.m > 0 && d.n > 0 && load_relaxed_u32(flags + b0 + lane);
        }
        for (uint64_t todo = __ballot(flagged); todo; todo &= todo - 1)
            batch_result(mats, b0 + __ffsll((long long)todo) - 1, keys, serial_state,
                         state_words, out);
    }
}

// ---------------------------------------------------------------------------------- all squares
// counts[i * nux + ux]: cells of row i, unit column ux whose side equals S (the maximum).
__global__ __launch_bounds__(256) void k_allmax_count(const uint64_t *__restrict__ bits,
                                                      int64_t m, int64_t n, int64_t ldw,
                                                      const ms_square *__restrict__ maxsq,
                                                      uint32_t *__restrict__ counts, int64_t nux,
                                                      int64_t nunits) {
    const int64_t S = uniform(maxsq->side);
    if (S <= 0 || S > ALL_MAX_SIDE) return;  // nothing to list / reported by the scan
    const int lane = __lane_id();
    const int64_t wave = wave_index();
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) / WAVE;
    for (int64_t u = wave; u < nunits; u += nwave) {
        const int64_t uy = u / nux, ux = u - uy * nux;
        unit_rows_ge(bits, m, n, ldw, uy, ux, (int32_t)S,
                     [&](int64_t i, uint64_t y, int64_t) {
                         uint32_t tot;
                         (void)wave_excl_sum((uint32_t)__popcll(y), &tot);
                         if (lane == 0) counts[i * nux + ux] = tot;
                     });
    }
}

// The exclusive prefix of the counts in row-major (row, unit column) order, in three passes over
// chunks of SCAN_CHUNK consecutive entries: each block sums its chunk (k_allmax_chunks), one block
// scans the chunk sums and writes the total (k_allmax_scan: 0 when S = 0, -1 when S is wider than
// the enumeration supports), and each block scans its chunk from the chunk's prefix
// (k_allmax_offsets).  Every pass reads its chunk with consecutive threads on consecutive words.
constexpr int SCAN_PER_THREAD = 16;
constexpr int64_t SCAN_CHUNK = 256 * SCAN_PER_THREAD;

__global__ __launch_bounds__(256) void k_allmax_chunks(const ms_square *__restrict__ maxsq,
                                                       const uint32_t *__restrict__ counts,
                                                       int64_t entries,
                                                       uint64_t *__restrict__ chunk_sums) {
    const int64_t S = uniform(maxsq->side);
    if (S <= 0 || S > ALL_MAX_SIDE) return;
    __shared__ uint64_t wsum[4];
    const int64_t nchunks = (entries + SCAN_CHUNK - 1) / SCAN_CHUNK;
    for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const int64_t base = c * SCAN_CHUNK;
        uint64_t sum = 0;
#pragma unroll
        for (int k = 0; k < SCAN_PER_THREAD; ++k) {
            const int64_t e = base + (int64_t)k * 256 + threadIdx.x;
            if (e < entries) sum += counts[e];
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
        if (__lane_id() == 0) wsum[threadIdx.x / WAVE] = sum;
        __syncthreads();
        if (threadIdx.x == 0) chunk_sums[c] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        __syncthreads();
    }
}

// One block: exclusive prefix of the chunk sums (in place) and the total.
__global__ __launch_bounds__(1024) void k_allmax_scan(const ms_square *__restrict__ maxsq,
                                                      uint64_t *__restrict__ chunk_sums,
                                                      int64_t nchunks,
                                                      int64_t *__restrict__ total_out) {
    __shared__ uint64_t part[1024];
    const int64_t S = maxsq->side;
    const int tid = threadIdx.x;
    if (S <= 0 || S > ALL_MAX_SIDE) {
        if (tid == 0) *total_out = S <= 0 ? 0 : -1;
        return;
    }
    const int64_t per = (nchunks + 1023) / 1024;
    const int64_t lo = tid * per < nchunks ? tid * per : nchunks;
    const int64_t hi = lo + per < nchunks ? lo + per : nchunks;
    uint64_t sum = 0;
    for (int64_t e = lo; e < hi; ++e) sum += chunk_sums[e];
    part[tid] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint64_t v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    uint64_t run = part[tid] - sum;
    for (int64_t e = lo; e < hi; ++e) {
        const uint64_t c = chunk_sums[e];
        chunk_sums[e] = run;
        run += c;
    }
    if (tid == 1023) *total_out = (int64_t)part[1023];
}

// offsets[e] = the chunk's prefix + the counts before e within the chunk.
__global__ __launch_bounds__(256) void k_allmax_offsets(const ms_square *__restrict__ maxsq,
                                                        const uint32_t *__restrict__ counts,
                                                        int64_t entries,
                                                        const uint64_t *__restrict__ chunk_pre,
                                                        uint64_t *__restrict__ offsets) {
    const int64_t S = uniform(maxsq->side);
    if (S <= 0 || S > ALL_MAX_SIDE) return;
    __shared__ uint64_t carry[SCAN_PER_THREAD][4];
    const int lane = __lane_id(), wv = threadIdx.x / WAVE;
    const int64_t nchunks = (entries + SCAN_CHUNK - 1) / SCAN_CHUNK;
    for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const int64_t base = c * SCAN_CHUNK;
        // row k of the chunk: entries base + 256 k .. + 255, one per thread
        uint32_t v[SCAN_PER_THREAD];
        uint64_t incl[SCAN_PER_THREAD];
#pragma unroll
        for (int k = 0; k < SCAN_PER_THREAD; ++k) {
            const int64_t e = base + (int64_t)k * 256 + threadIdx.x;
            v[k] = e < entries ? counts[e] : 0u;
        }
#pragma unroll
        for (int k = 0; k < SCAN_PER_THREAD; ++k) {
            uint64_t x = v[k];
#pragma unroll
            for (int off = 1; off < WAVE; off <<= 1) {
                const uint64_t y = __shfl_up(x, off);
                if (lane >= off) x += y;
            }
            incl[k] = x;
            if (lane == WAVE - 1) carry[k][wv] = x;
        }
        __syncthreads();
        uint64_t run = chunk_pre[c];
#pragma unroll
        for (int k = 0; k < SCAN_PER_THREAD; ++k) {
            uint64_t before = run;
            for (int w = 0; w < wv; ++w) before += carry[k][w];
            const int64_t e = base + (int64_t)k * 256 + threadIdx.x;
            if (e < entries) offsets[e] = before + incl[k] - v[k];
            run += carry[k][0] + carry[k][1] + carry[k][2] + carry[k][3];
        }
        __syncthreads();
    }
}

// The positions i * n + j of those cells, in row-major order, the first `capacity` of them.
__global__ __launch_bounds__(256) void k_allmax_write(const uint64_t *__restrict__ bits,
                                                      int64_t m, int64_t n, int64_t ldw,
                                                      const ms_square *__restrict__ maxsq,
                                                      const uint64_t *__restrict__ offsets,
                                                      int64_t nux, int64_t nunits,
                                                      int64_t *__restrict__ pos, int64_t capacity) {
    const int64_t S = uniform(maxsq->side);
    if (S <= 0 || S > ALL_MAX_SIDE) return;
    const int lane = __lane_id();
    const int64_t wave = wave_index();
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) / WAVE;
    for (int64_t u = wave; u < nunits; u += nwave) {
        const int64_t uy = u / nux, ux = u - uy * nux;
        unit_rows_ge(bits, m, n, ldw, uy, ux, (int32_t)S,
                     [&](int64_t i, uint64_t y, int64_t w0) {
                         uint32_t tot;
                         const uint32_t before = wave_excl_sum((uint32_t)__popcll(y), &tot);
                         if (tot == 0) return;
                         uint64_t k = offsets[i * nux + ux] + before;
                         const int64_t rowpos = i * n + (w0 + lane) * 64;
                         while (y) {
                             const int b = __ffsll((long long)y) - 1;
                             y &= y - 1;
                             if ((int64_t)k < capacity) pos[k] = rowpos + b;
                             ++k;
                         }
                     });
    }
}

__global__ void k_write_i64(int64_t *dst, int64_t v) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *dst = v;
}

} // namespace msk

// Scratch of the allocation-free search (ms_max_square_noalloc), one copy per GPU, held until
// the process ends.  Host code reaches it only through the device address that noalloc_setup
// obtains: in host code this name is a host-side stand-in, not a device address.
static __device__ __align__(256) unsigned char scratch[mshost::NOALLOC_SCRATCH_BYTES];

// ====================================================================================== host
namespace mshost {

using TS0 = msk::TileShape<16, 16>;
using TS1 = msk::TileShape<32, 16>;
using TS2 = msk::TileShape<32, 32>;
// certifies side 64 (its halo spans two row groups; 65 owned rows): for images whose squares
// are mostly between 32 and 64 (blobs), where the 32-certified tile saturates nearly everywhere
using TS3 = msk::TileShape<32, 64>;

const ProbeVariant PROBE_VARIANTS[NUM_PROBE_VARIANTS] = {{16, 16}, {32, 16}, {32, 32}, {32, 64}};

int64_t probe_tile_rows(int variant) {
    switch (variant) {
    case 0: return TS0::TR;
    case 1: return TS1::TR;
    case 2: return TS2::TR;
    default: return TS3::TR;
    }
}

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

hipError_t launch_pack_u8(const LaunchEnv &env, const uint8_t *a, int64_t m, int64_t n,
                          int64_t ldb, uint64_t *bits, int64_t ldw) {
    const int64_t chunks = m * cdiv(n, 64) * 4;
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(cdiv(chunks, 256),
                                                                   (int64_t)env.num_cus * 32));
    const uintptr_t al = (uintptr_t)a | (uintptr_t)ldb;
    const dim3 g((unsigned)blocks), b(256);
    if (al % 16 == 0) hipLaunchKernelGGL(msk::k_pack_u8<16>, g, b, 0, env.stream, a, m, n, ldb, bits, ldw);
    else if (al % 8 == 0) hipLaunchKernelGGL(msk::k_pack_u8<8>, g, b, 0, env.stream, a, m, n, ldb, bits, ldw);
    else if (al % 4 == 0) hipLaunchKernelGGL(msk::k_pack_u8<4>, g, b, 0, env.stream, a, m, n, ldb, bits, ldw);
    else hipLaunchKernelGGL(msk::k_pack_u8<1>, g, b, 0, env.stream, a, m, n, ldb, bits, ldw);
    return hipGetLastError();
}

template <class TS>
static hipError_t launch_max_square_t(const LaunchEnv &env, const uint64_t *bits, int64_t m,
                                      int64_t n, int64_t ldw, ScratchHeader *hdr,
                                      int32_t *serial_state, uint8_t *sat, int32_t *bounds,
                                      uint32_t *box_rec, ms_square *out) {
    const int64_t ntx = cdiv(cdiv(n, 64), TS::OWN_WORDS);
    const int64_t ntiles = cdiv(m, TS::TR) * ntx;
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(cdiv(ntiles, 4),
                                                                   max_probe_blocks(env.num_cus)));
    if (!bounds) box_rec = nullptr;
    hipLaunchKernelGGL(msk::k_probe<TS>, dim3((unsigned)blocks), dim3(256), 0, env.stream, bits,
                       m, n, ldw, ntiles, ntx, hdr, sat, bounds, box_rec);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // one block per saturated tile when they are few, each block several tiles when many
    const int64_t rblocks = std::max<int64_t>(1, std::min<int64_t>(ntiles,
                                                                    (int64_t)env.num_cus * 4));
    hipLaunchKernelGGL(msk::k_resolve<TS>, dim3((unsigned)rblocks),
                       dim3(64 * msk::RESOLVE_WAVES), 0, env.stream,
                       bits, m, n, ldw, ntiles, ntx, hdr, sat, bounds, box_rec, blocks,
                       serial_state, out);
    return hipGetLastError();
}

int64_t max_probe_blocks(int num_cus) { return (int64_t)num_cus * 8; }

int64_t max_probe_tiles(int64_t m, int64_t n) {
    const int64_t nw = cdiv(std::max<int64_t>(n, 1), 64);
    const int64_t rows = std::min<int64_t>({TS0::TR, TS1::TR, TS2::TR, TS3::TR});
    return cdiv(std::max<int64_t>(m, 1), rows) * cdiv(nw, (int64_t)PROBE_TILE_WORDS);
}

hipError_t launch_max_square(const LaunchEnv &env, int variant, const uint64_t *bits, int64_t m,
                             int64_t n, int64_t ldw, ScratchHeader *hdr, int32_t *serial_state,
                             uint8_t *sat, int32_t *bounds, uint32_t *box_rec, ms_square *out) {
    switch (variant) {
    case 0:
        return launch_max_square_t<TS0>(env, bits, m, n, ldw, hdr, serial_state, sat, bounds,
                                         box_rec, out);
    case 1:
        return launch_max_square_t<TS1>(env, bits, m, n, ldw, hdr, serial_state, sat, bounds,
                                         box_rec, out);
    case 2:
        return launch_max_square_t<TS2>(env, bits, m, n, ldw, hdr, serial_state, sat, bounds,
                                        box_rec, out);
    default:
        return launch_max_square_t<TS3>(env, bits, m, n, ldw, hdr, serial_state, sat, bounds,
                                        box_rec, out);
    }
}

hipError_t launch_square_map(const LaunchEnv &env, int map_cols, int band_rows,
                             const uint64_t *bits, int64_t m, int64_t n, int64_t ldw, int32_t *dp,
                             int64_t ld_dp, const ms_square *maxsq, int32_t *serial_state,
                             const MapRegions *regions, ScratchHeader *hdr, uint64_t *bnd,
                             int strip_rows) {
    if (!hdr) bnd = nullptr;
    unsigned long long *bw = reinterpret_cast<unsigned long long *>(bnd);
    const int vec_ok = ((uintptr_t)dp % 16 == 0) && (ld_dp % 4 == 0);
    const int64_t items_bound = cdiv(m, 16) * cdiv(n, 64);
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(cdiv(items_bound, 4),
                                                                   (int64_t)env.num_cus * 8));
    const dim3 g((unsigned)blocks), b(256);
    const int32_t *bounds = regions ? regions->bounds : nullptr;
    const int64_t trows = regions ? regions->tile_rows : 1;
    const int64_t tntx = regions ? regions->tile_ntx : 1;
    const uint32_t *box = regions ? regions->big_box : nullptr;
    const int64_t min_items = (int64_t)env.num_cus * 4 * MAP_ITEMS_PER_SIMD;
    // one kernel: the narrow pass (512-column windows as 2 x 4 or 1 x 8 columns per lane) and,
    // for squares beyond its reach, the block-wide pass
    if (map_cols == 8) {
        hipLaunchKernelGGL((msk::k_dpmap<1, 8>), g, b, 0, env.stream, bits, m, n, ldw, dp, ld_dp,
                           maxsq, (int64_t)band_rows, serial_state, vec_ok, bounds, trows, tntx,
                           box, min_items, hdr, bw, strip_rows);
    } else {
        hipLaunchKernelGGL((msk::k_dpmap<2, 4>), g, b, 0, env.stream, bits, m, n, ldw, dp, ld_dp,
                           maxsq, (int64_t)band_rows, serial_state, vec_ok, bounds, trows, tntx,
                           box, min_items, hdr, bw, strip_rows);
    }
    return hipGetLastError();
}

int strip_rows_setting() {
    static const int v = [] {
        const char *e = std::getenv("MAXSQ_STRIP_ROWS");
        const int r = e ? std::atoi(e) : 0;
        return (r >= 1 && r <= 64) ? r : 0;
    }();
    return v;
}

int64_t strip_words_needed(int64_t m, int64_t n) {
    if (std::min(m, n) <= STRIP_MIN_SIDE) return 0;
    return cdiv(cdiv(n, 64), (int64_t)STRIP_WORDS) * m * 2;
}

hipError_t launch_zero_u64(const LaunchEnv &env, uint64_t *p, int64_t count) {
    if (count <= 0) return hipSuccess;
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(cdiv(count, 256 * 8),
                                                                   (int64_t)env.num_cus * 8));
    hipLaunchKernelGGL(msk::k_zero_u64, dim3((unsigned)blocks), dim3(256), 0, env.stream, p,
                       count);
    return hipGetLastError();
}

hipError_t launch_set_strips(const LaunchEnv &env, ScratchHeader *hdr, uint64_t *words,
                             int64_t count, int forced_rows) {
    hipLaunchKernelGGL(msk::k_set_strips, dim3(1), dim3(64), 0, env.stream, hdr,
                       reinterpret_cast<unsigned long long>(words), words ? count : 0,
                       forced_rows);
    return hipGetLastError();
}

hipError_t launch_zero_header(const LaunchEnv &env, void *p, size_t bytes) {
    hipLaunchKernelGGL(msk::k_zero_words, dim3(1), dim3(64), 0, env.stream,
                       static_cast<uint32_t *>(p), (int)(bytes / sizeof(uint32_t)));
    return hipGetLastError();
}

hipError_t launch_write_result(const LaunchEnv &env, ms_square *out, ScratchHeader *hdr,
                               int64_t count) {
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(cdiv(count, 256), 1024));
    hipLaunchKernelGGL(msk::k_write_result, dim3((unsigned)blocks), dim3(256), 0, env.stream, out,
                       hdr, count);
    return hipGetLastError();
}

// ------------------------------------------------------------------ allocation-free search
// Per device: the address of `scratch` on that device (found once by noalloc_setup), and
// whether its header may hold a failed call's state (true until the first call has cleared it).
static std::mutex g_noalloc_mu;
static void *g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};
static bool g_noalloc_dirty[NOALLOC_MAX_DEVICES] = {};

hipError_t noalloc_setup(int device) {
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (g_noalloc_ptr[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_noalloc_ptr[device] = p;
    g_noalloc_dirty[device] = true;
    return hipSuccess;
}

hipError_t launch_max_square_noalloc(const LaunchEnv &env, int device, int variant,
                                     const uint64_t *bits, int64_t m, int64_t n, int64_t ldw,
                                     ms_square *out) {
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    char *base = static_cast<char *>(g_noalloc_ptr[device]);  // never the array's host name
    if (!base) return hipErrorNotInitialized;
    auto *hdr = reinterpret_cast<ScratchHeader *>(base);
    auto *state = reinterpret_cast<int32_t *>(base + 256);
    auto *sat = reinterpret_cast<uint8_t *>(base + 256 + NOALLOC_STATE_BYTES);
    hipError_t e = hipSuccess;
    if (g_noalloc_dirty[device]) {
        hipLaunchKernelGGL(msk::k_clear_header, dim3(1), dim3(64), 0, env.stream, hdr);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        g_noalloc_dirty[device] = false;
    }
    if (m == 0 || n == 0) {
        e = launch_write_result(env, out, hdr, 1);
    } else {
        // no per-tile bounds or box records: no map follows in this call
        e = launch_max_square(env, variant, bits, m, n, ldw, hdr, state, sat, nullptr, nullptr,
                              out);
    }
    if (e != hipSuccess) g_noalloc_dirty[device] = true;
    return e;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Tiles of one matrix of a batch whose wide tile is TS (the device's rule, msk::tiles_in).
template <class TS>
static uint64_t tiles_of(const ms_matrix &d, int q) {
    return (uint64_t)(msk::narrow_tiles<TS>(d.m, d.n, q) ? msk::tile_count<msk::TSN>(d.m, d.n)
                                                          : msk::tile_count<TS>(d.m, d.n));
}

bool narrow_weight_valid(int q) {
    for (int k = 0; k < NUM_NARROW_WEIGHTS; ++k)
        if (NARROW_WEIGHTS[k] == q) return true;
    return false;
}
const int NARROW_WEIGHTS[NUM_NARROW_WEIGHTS] = {msk::NARROW_DEFAULT, 0, 4, 8};

BatchLayout batch_layout(int variant, int q, const ms_matrix *h_mats, int64_t count) {
    BatchLayout L{};
    L.narrow_q = q;
    uint64_t tiles = 0, mix = 0;
    int64_t maxn = 1;
    const auto pass = [&](auto ts) {  // one pass: tiles, widest row, fingerprint
        using TS = decltype(ts);
        for (int64_t i = 0; i < count; ++i) {
            const ms_matrix &d = h_mats[i];
            tiles += q >= 0 ? tiles_of<TS>(d, q)  // q < 0: a bound for every tile choice
                            : std::max<uint64_t>({(uint64_t)msk::tile_count<TS0>(d.m, d.n),
                                                  (uint64_t)msk::tile_count<TS1>(d.m, d.n),
                                                  (uint64_t)msk::tile_count<TS2>(d.m, d.n),
                                                  (uint64_t)msk::tile_count<TS3>(d.m, d.n),
                                                  (uint64_t)msk::tile_count<msk::TSN>(d.m, d.n)});
            maxn = std::max<int64_t>(maxn, d.n);
            mix += msk::shape_mix((uint64_t)i, (uint64_t)d.m, (uint64_t)d.n,
                                  (uint64_t)d.ld_words);
        }
    };
    switch (variant) {
    case 0: pass(TS0{}); break;
    case 1: pass(TS1{}); break;
    case 2: pass(TS2{}); break;
    default: pass(TS3{}); break;
    }
    L.total_tiles = tiles;
    L.max_nwords = cdiv(maxn, 64);
    L.shape_mix = mix;
    size_t off = 0;
    L.counters = off; off = align256(off + sizeof(msk::BatchCounters));
    L.nblk = std::max<int64_t>(1, cdiv(count, msk::INIT_BLOCK));
    L.keys = off; off = align256(off + sizeof(unsigned long long) * (size_t)count);
    L.local = off; off = align256(off + sizeof(uint64_t) * (size_t)count);
    L.parts = off; off = align256(off + sizeof(msk::InitPart) * (size_t)L.nblk);
    L.offsets = off; off = align256(off + sizeof(uint64_t) * (size_t)(L.nblk + 1));
    L.flags = off; off = align256(off + sizeof(uint32_t) * (size_t)count);
    L.serial_state = off; off = align256(off + sizeof(int32_t) * 2 * 64 * (size_t)L.max_nwords);
    L.sat = off; off = align256(off + (size_t)tiles);
    L.total = off;
    return L;
}

template <class TS>
static hipError_t launch_batched_t(const LaunchEnv &env, const ms_matrix *mats, int64_t count,
                                   ms_square *out, char *ws, const BatchLayout &L) {
    auto *ctr = reinterpret_cast<msk::BatchCounters *>(ws + L.counters);
    auto *keys = reinterpret_cast<unsigned long long *>(ws + L.keys);
    auto *local = reinterpret_cast<uint64_t *>(ws + L.local);
    auto *parts = reinterpret_cast<msk::InitPart *>(ws + L.parts);
    auto *offs = reinterpret_cast<uint64_t *>(ws + L.offsets);
    auto *flags = reinterpret_cast<uint32_t *>(ws + L.flags);
    auto *state = reinterpret_cast<int32_t *>(ws + L.serial_state);
    auto *sat = reinterpret_cast<uint8_t *>(ws + L.sat);
    // setup: per-matrix tile starts within init blocks and the blocks' totals, then the blocks'
    // starts and the fingerprint check
    hipLaunchKernelGGL(msk::k_batch_count<TS>, dim3((unsigned)L.nblk), dim3(msk::INIT_BLOCK), 0,
                       env.stream, mats, count, keys, local, flags, parts, ctr, L.narrow_q);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(msk::k_batch_offsets, dim3(1), dim3(1024), 0, env.stream, parts, L.nblk,
                       offs, L.shape_mix);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t pblocks = std::max<int64_t>(
        1, std::min<int64_t>(cdiv((int64_t)L.total_tiles, 4), (int64_t)env.num_cus * 8));
    hipLaunchKernelGGL(msk::k_probe_batched<TS>, dim3((unsigned)pblocks), dim3(256), 0,
                       env.stream, mats, keys, local, offs, count, L.nblk, ctr, sat,
                       (uint64_t)L.total_tiles, L.narrow_q);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // results, and the saturated tiles first if any (one launch): a block per tile up to four
    // per CU, so that a few saturated tiles get a block each
    const int64_t fblocks = std::max<int64_t>(
        1, std::min<int64_t>(std::max<int64_t>((int64_t)L.total_tiles, cdiv(count, 256)),
                             (int64_t)env.num_cus * 4));
    hipLaunchKernelGGL(msk::k_batch_finish<TS>, dim3((unsigned)fblocks), dim3(256), 0,
                       env.stream, mats, keys, local, offs, count, L.nblk, flags, ctr, sat,
                       (uint64_t)L.total_tiles, state, L.max_nwords, out, L.narrow_q);
    return hipGetLastError();
}

hipError_t launch_batched(const LaunchEnv &env, int variant, const ms_matrix *d_mats,
                          int64_t count, ms_square *out, void *ws, const BatchLayout &L) {
    char *w = static_cast<char *>(ws);
    switch (variant) {
    case 0: return launch_batched_t<TS0>(env, d_mats, count, out, w, L);
    case 1: return launch_batched_t<TS1>(env, d_mats, count, out, w, L);
    case 2: return launch_batched_t<TS2>(env, d_mats, count, out, w, L);
    default: return launch_batched_t<TS3>(env, d_mats, count, out, w, L);
    }
}

AllMaxLayout all_max_layout(int64_t m, int64_t n) {
    AllMaxLayout L{};
    L.nux = cdiv(std::max<int64_t>(cdiv(n, 64), 1), (int64_t)msk::ALL_WORDS);
    L.entries = std::max<int64_t>(m, 0) * L.nux;
    L.counts = 0;
    L.offsets = align256(sizeof(uint32_t) * (size_t)L.entries);
    L.chunks = L.offsets + align256(sizeof(uint64_t) * (size_t)(L.entries + 1));
    L.total = L.chunks +
              align256(sizeof(uint64_t) * (size_t)(cdiv(L.entries, msk::SCAN_CHUNK) + 1));
    return L;
}

hipError_t launch_all_max(const LaunchEnv &env, const uint64_t *bits, int64_t m, int64_t n,
                          int64_t ldw, const ms_square *maxsq, int64_t *pos, int64_t capacity,
                          int64_t *count, void *ws) {
    if (m == 0 || n == 0) {
        hipLaunchKernelGGL(msk::k_write_i64, dim3(1), dim3(64), 0, env.stream, count, (int64_t)0);
        return hipGetLastError();
    }
    const AllMaxLayout L = all_max_layout(m, n);
    auto *counts = reinterpret_cast<uint32_t *>(static_cast<char *>(ws) + L.counts);
    auto *offsets = reinterpret_cast<uint64_t *>(static_cast<char *>(ws) + L.offsets);
    auto *chunk_sums = reinterpret_cast<uint64_t *>(static_cast<char *>(ws) + L.chunks);
    const int64_t nchunks = cdiv(L.entries, msk::SCAN_CHUNK);
    const int64_t cblocks = std::max<int64_t>(1, std::min<int64_t>(nchunks,
                                                                    (int64_t)env.num_cus * 8));
    const int64_t nunits = cdiv(m, (int64_t)msk::ALL_ROWS) * L.nux;
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(cdiv(nunits, 4),
                                                                   (int64_t)env.num_cus * 8));
    hipLaunchKernelGGL(msk::k_allmax_count, dim3((unsigned)blocks), dim3(256), 0, env.stream,
                       bits, m, n, ldw, maxsq, counts, L.nux, nunits);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(msk::k_allmax_chunks, dim3((unsigned)cblocks), dim3(256), 0, env.stream,
                       maxsq, counts, L.entries, chunk_sums);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(msk::k_allmax_scan, dim3(1), dim3(1024), 0, env.stream, maxsq, chunk_sums,
                       nchunks, count);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(msk::k_allmax_offsets, dim3((unsigned)cblocks), dim3(256), 0, env.stream,
                       maxsq, counts, L.entries, chunk_sums, offsets);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(msk::k_allmax_write, dim3((unsigned)blocks), dim3(256), 0, env.stream,
                       bits, m, n, ldw, maxsq, offsets, L.nux, nunits, pos, capacity);
    return hipGetLastError();
}

} // namespace mshost
