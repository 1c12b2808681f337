// kernels.hip -- libmaxsq kernels for gfx950 and their host launchers.
//
// Single matrix, largest square (two launches):
//   k_probe    : erosion search over register tiles (device.hpp tile_search); each tile pushes
//                its exact side (if below the tile's certified bound) with its first corner into
//                one atomic key, or queues itself as saturated.
//   k_exact    : saturated tiles get their exact side from the windowed dp pass with a doubling
//                halo; the last wave to finish turns the key into the result and clears the
//                scratch for the next call.
// dp map (one more launch): k_dpmap reads S on the device and covers the matrix with row bands
// and column windows that start S rows / columns early (zero state there is exact).
// Batched: k_batch_init (prefix of tile counts, clear keys), k_probe_batched (one persistent
// grid pulling (matrix, tile) items from an atomic queue), k_exact_batched, k_batch_final.
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

__global__ __launch_bounds__(256) void k_pack_u8(const uint8_t *__restrict__ a, int64_t m,
                                                 int64_t n, int64_t ldb,
                                                 uint64_t *__restrict__ bits, int64_t ldw,
                                                 int aligned) {
    const int64_t groups = 4 * ((n + 63) >> 6);  // 16-column groups of the valid words
    for (int64_t i = blockIdx.y; i < m; i += gridDim.y) {
        const uint8_t *__restrict__ src = a + i * ldb;
        uint16_t *__restrict__ dst = reinterpret_cast<uint16_t *>(bits + i * ldw);
        for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < groups;
             g += (int64_t)gridDim.x * blockDim.x) {
            const int64_t c = g * 16;
            uint32_t mask = 0;
            if (aligned && c + 16 <= n) {
                const uint4 v = *reinterpret_cast<const uint4 *>(src + c);
                mask = nz4(v.x) | (nz4(v.y) << 4) | (nz4(v.z) << 8) | (nz4(v.w) << 12);
            } else {
                for (int t = 0; t < 16; ++t)
                    if (c + t < n && src[c + t] != 0) mask |= 1u << t;
            }
            dst[g] = (uint16_t)mask;
        }
    }
}

// ---------------------------------------------------------------------------------- probe
template <class TS>
__global__ __launch_bounds__(256) void k_probe(const uint64_t *__restrict__ bits, int64_t m,
                                               int64_t n, int64_t ldw, int64_t ntiles,
                                               int64_t ntx, TileSink sink) {
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) / WAVE;
    for (int64_t t = wave; t < ntiles; t += nwave) {
        const int64_t ty = t / ntx, tx = t - ty * ntx;
        tile_search<TS>(bits, m, n, ldw, ty, tx, t, sink);
    }
}

constexpr int EX_NG = 8;   // exact pass window: 8 groups x 256 columns
constexpr int EX_CPL = 4;

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

__global__ __launch_bounds__(64) void k_exact(const uint64_t *__restrict__ bits, int64_t m,
                                              int64_t n, int64_t ldw,
                                              mshost::ScratchHeader *hdr,
                                              const uint64_t *__restrict__ sat_list,
                                              int64_t sat_cap, int64_t ntx, int64_t tile_rows,
                                              int64_t kc, int32_t *serial_state,
                                              ms_square *out) {
    __shared__ uint64_t lx[LDS_WORDS];
    __shared__ int32_t lc[LDS_WORDS];
    const WaveLds lds{lx, lc};
    const int lane = __lane_id();
    const uint32_t cnt = load_relaxed_u32(&hdr->sat_count);
    if ((int64_t)cnt > sat_cap) {
        if (lane == 0 && blockIdx.x == 0) atomicOr(&hdr->serial_flag, 1u);
    } else {
        for (int64_t s = blockIdx.x; s < (int64_t)cnt; s += gridDim.x) {
            const int64_t tid = (int64_t)(sat_list[s] & 0xFFFFFFFFFFFFull);
            const int64_t ty = tid / ntx, tx = tid - ty * ntx;
            const int64_t ra = ty * tile_rows, rb = ra + tile_rows < m ? ra + tile_rows : m;
            const int64_t xa = tx * mshost::PROBE_TILE_WORDS * 64;
            const int64_t xe = xa + mshost::PROBE_TILE_WORDS * 64;
            const int64_t xb = xe < n ? xe : n;
            Track t{0, INT64_MAX};
            if (exact_region<EX_NG, EX_CPL>(bits, m, n, ldw, ra, rb, xa, xb, kc, t, lds)) {
                if (lane == 0 && t.v > 0) atomicMax(&hdr->key, make_key(t.v, t.pos));
            } else if (lane == 0) {
                atomicOr(&hdr->serial_flag, 1u);
            }
        }
    }
    __threadfence();
    uint32_t prev = 0;
    if (lane == 0) prev = atomicAdd(&hdr->done, 1u);
    prev = __shfl(prev, 0);
    if (prev != gridDim.x - 1) return;
    __threadfence();
    unsigned long long key;
    if (__hip_atomic_load(&hdr->serial_flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)) {
        const int64_t nw64 = ((n + 63) >> 6) * 64;
        Track tr{0, INT64_MAX};
        serial_dp<false>(bits, m, n, ldw, nullptr, 0, serial_state, serial_state + nw64, tr);
        const Track w = wave_track(tr);
        key = w.v > 0 ? make_key(w.v, w.pos) : 0ull;
    } else {
        key = __hip_atomic_load(&hdr->key, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (lane == 0) {
        write_result(key, n, &hdr->result);
        if (out) write_result(key, n, out);
        hdr->key = 0;
        hdr->sat_count = 0;
        hdr->done = 0;
        hdr->serial_flag = 0;
    }
}

// ---------------------------------------------------------------------------------- map
template <int NGMAX, int CPL>
__global__ __launch_bounds__(256) void k_dpmap(const uint64_t *__restrict__ bits, int64_t m,
                                               int64_t n, int64_t ldw, int32_t *__restrict__ dp,
                                               int64_t ld_dp,
                                               const ms_square *__restrict__ maxsq,
                                               int64_t band_rows, int32_t *serial_state,
                                               int vec_ok) {
    constexpr int64_t GW = 64 * CPL;
    constexpr int64_t WIN = NGMAX * GW;
    __shared__ uint64_t lx[4][LDS_WORDS];
    __shared__ int32_t lc[4][LDS_WORDS];
    const WaveLds lds{lx[threadIdx.x / WAVE], lc[threadIdx.x / WAVE]};
    const int64_t S = __hip_atomic_load(&maxsq->side, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int64_t hc = (S + 63) & ~(int64_t)63;
    if (hc + 64 > WIN) {
        // too large for a register window: one wave sweeps the whole matrix
        if (blockIdx.x == 0 && threadIdx.x < WAVE) {
            const int64_t nw64 = ((n + 63) >> 6) * 64;
            Track tr{0, INT64_MAX};
            serial_dp<true>(bits, m, n, ldw, dp, ld_dp, serial_state, serial_state + nw64, tr);
        }
        return;
    }
    int64_t ng = (hc + (4 * hc > 256 ? 4 * hc : 256) + GW - 1) / GW;
    ng = ng < 1 ? 1 : (ng > NGMAX ? NGMAX : ng);
    const int64_t ow = ng * GW - hc;
    int64_t R = band_rows > 4 * S ? band_rows : 4 * S;
    R = R < m ? R : m;
    const int64_t nwin = (n + ow - 1) / ow;
    const int64_t items = ((m + R - 1) / R) * nwin;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) / WAVE;
    Track dummy{0, 0};
    for (int64_t it = wave; it < items; it += nwave) {
        const int64_t b = it / nwin, wdx = it - b * nwin;
        const int64_t ra = b * R, rb = ra + R < m ? ra + R : m;
        const int64_t rh = ra - S > 0 ? ra - S : 0;
        const int64_t xa = wdx * ow, xb = xa + ow < n ? xa + ow : n;
        const int64_t xh = xa - hc > 0 ? xa - hc : 0;
        const int ngi = (int)((xb - xh + GW - 1) / GW);
        dprun<NGMAX, CPL, true, false>(bits, ldw, n, rh, ra, rb, xh, xa, xb, ngi, dp, ld_dp,
                                       vec_ok != 0, dummy, lds);
    }
}

__global__ void k_write_result(ms_square *out, mshost::ScratchHeader *hdr, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = ms_square{0, -1, -1};
    if (hdr && blockIdx.x == 0 && threadIdx.x == 0) hdr->result = ms_square{0, -1, -1};
}

// ---------------------------------------------------------------------------------- batched
struct BatchCounters {
    unsigned long long head;    // next work item
    unsigned long long total;   // total tiles
    uint32_t sat_count;
    uint32_t done;
    uint32_t overflow;
    uint32_t pad;
};

// One block: clear per-matrix keys and flags, tile-count prefix (exclusive), counters.
template <class TS>
__global__ __launch_bounds__(1024) void k_batch_init(const ms_matrix *__restrict__ mats,
                                                     int64_t count,
                                                     unsigned long long *__restrict__ keys,
                                                     uint64_t *__restrict__ prefix,
                                                     uint32_t *__restrict__ flags,
                                                     BatchCounters *ctr) {
    __shared__ uint64_t part[1024];
    const int tid = threadIdx.x;
    const int64_t per = (count + 1023) / 1024;
    const int64_t lo = tid * per, hi = lo + per < count ? lo + per : count;
    uint64_t s = 0;
    for (int64_t i = lo; i < hi; ++i) {
        keys[i] = 0;
        flags[i] = 0;
        const ms_matrix d = mats[i];
        const int64_t nwords = (d.n + 63) >> 6;
        const int64_t nt = (d.m > 0 && d.n > 0)
                               ? ((d.m + TS::TR - 1) / TS::TR) *
                                     ((nwords + TS::OWN_WORDS - 1) / TS::OWN_WORDS)
                               : 0;
        s += (uint64_t)nt;
    }
    part[tid] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint64_t v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    uint64_t run = part[tid] - s;  // exclusive start of this thread's range
    for (int64_t i = lo; i < hi; ++i) {
        prefix[i] = run;
        const ms_matrix d = mats[i];
        const int64_t nwords = (d.n + 63) >> 6;
        const int64_t nt = (d.m > 0 && d.n > 0)
                               ? ((d.m + TS::TR - 1) / TS::TR) *
                                     ((nwords + TS::OWN_WORDS - 1) / TS::OWN_WORDS)
                               : 0;
        run += (uint64_t)nt;
    }
    if (tid == 1023) {
        prefix[count] = part[1023];
        ctr->head = 0;
        ctr->total = part[1023];
        ctr->sat_count = 0;
        ctr->done = 0;
        ctr->overflow = 0;
    }
}

__device__ __forceinline__ int64_t find_matrix(const uint64_t *__restrict__ prefix, int64_t count,
                                               uint64_t item) {
    int64_t lo = 0, hi = count;  // prefix[lo] <= item < prefix[hi]
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (prefix[mid] <= item) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Tiles of all matrices in one grid-stride pass; the item count comes from the host (it is
// computed from the same descriptors), so the loop is bounded by construction.  A mismatch with
// the device-side prefix marks the whole batch as failed instead of running.
template <class TS>
__global__ __launch_bounds__(256) void k_probe_batched(const ms_matrix *__restrict__ mats,
                                                       int64_t count,
                                                       unsigned long long *__restrict__ keys,
                                                       const uint64_t *__restrict__ prefix,
                                                       BatchCounters *ctr,
                                                       uint64_t *__restrict__ sat_list,
                                                       uint64_t sat_cap, uint64_t total) {
    const int lane = __lane_id();
    if (__hip_atomic_load(prefix + count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != total) {
        if (lane == 0 && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&ctr->overflow, 2u);
        return;
    }
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const uint64_t nwave = ((uint64_t)gridDim.x * blockDim.x) / WAVE;
    for (uint64_t item = wave; item < total; item += nwave) {
        const int64_t mi = find_matrix(prefix, count, item);
        const ms_matrix d = mats[mi];
        const int64_t nwords = (d.n + 63) >> 6;
        const int64_t ntx = (nwords + TS::OWN_WORDS - 1) / TS::OWN_WORDS;
        const int64_t t = (int64_t)(item - prefix[mi]);
        const int64_t ty = t / ntx, tx = t - ty * ntx;
        TileSink sink{keys + mi, &ctr->sat_count, sat_list, sat_cap, (uint64_t)mi << 40};
        tile_search<TS>(d.bits, d.m, d.n, d.ld_words, ty, tx, t, sink);
    }
}

__global__ __launch_bounds__(64) void k_exact_batched(const ms_matrix *__restrict__ mats,
                                                      unsigned long long *__restrict__ keys,
                                                      uint32_t *__restrict__ flags,
                                                      BatchCounters *ctr,
                                                      const uint64_t *__restrict__ sat_list,
                                                      uint64_t sat_cap, int64_t tile_rows,
                                                      int64_t kc) {
    __shared__ uint64_t lx[LDS_WORDS];
    __shared__ int32_t lc[LDS_WORDS];
    const WaveLds lds{lx, lc};
    const int lane = __lane_id();
    const uint32_t cnt = load_relaxed_u32(&ctr->sat_count);
    if (load_relaxed_u32(&ctr->overflow) & 2u) return;
    if ((uint64_t)cnt > sat_cap) {
        if (lane == 0 && blockIdx.x == 0) atomicOr(&ctr->overflow, 1u);
        return;
    }
    for (int64_t s = blockIdx.x; s < (int64_t)cnt; s += gridDim.x) {
        const uint64_t e = sat_list[s];
        const int64_t mi = (int64_t)(e >> 40);
        const int64_t tid = (int64_t)(e & 0xFFFFFFFFFFull);
        const ms_matrix d = mats[mi];
        const int64_t nwords = (d.n + 63) >> 6;
        const int64_t ntx = (nwords + mshost::PROBE_TILE_WORDS - 1) / mshost::PROBE_TILE_WORDS;
        const int64_t ty = tid / ntx, tx = tid - ty * ntx;
        const int64_t ra = ty * tile_rows, rb = ra + tile_rows < d.m ? ra + tile_rows : d.m;
        const int64_t xa = tx * mshost::PROBE_TILE_WORDS * 64;
        const int64_t xe = xa + mshost::PROBE_TILE_WORDS * 64;
        const int64_t xb = xe < d.n ? xe : d.n;
        Track t{0, INT64_MAX};
        if (exact_region<EX_NG, EX_CPL>(d.bits, d.m, d.n, d.ld_words, ra, rb, xa, xb, kc, t, lds)) {
            if (lane == 0 && t.v > 0) atomicMax(keys + mi, make_key(t.v, t.pos));
        } else if (lane == 0) {
            atomicOr(flags + mi, 1u);
        }
    }
}

// Key -> result per matrix; matrices whose saturated tiles needed a halo wider than the exact
// pass supports are finished by block 0 with the serial pass (it owns the state buffer).
__global__ __launch_bounds__(64) void k_batch_final(const ms_matrix *__restrict__ mats,
                                                    int64_t count,
                                                    const unsigned long long *__restrict__ keys,
                                                    const uint32_t *__restrict__ flags,
                                                    const BatchCounters *ctr,
                                                    int32_t *serial_state, ms_square *out) {
    const int lane = __lane_id();
    const uint32_t ovf = load_relaxed_u32(&ctr->overflow);
    if (ovf & 2u) {  // inconsistent batch: report every result as failed
        for (int64_t i = blockIdx.x; i < count; i += gridDim.x)
            if (lane == 0) out[i] = ms_square{-1, -1, -1};
        return;
    }
    const bool overflow = ovf != 0;
    for (int64_t i = blockIdx.x; i < count; i += gridDim.x) {
        const ms_matrix d = mats[i];
        const bool serial = d.m > 0 && d.n > 0 && (load_relaxed_u32(flags + i) || overflow);
        if (!serial && lane == 0) write_result(load_relaxed(keys + i), d.n, out + i);
    }
    if (blockIdx.x != 0) return;
    for (int64_t i = 0; i < count; ++i) {
        const ms_matrix d = mats[i];
        if (!(d.m > 0 && d.n > 0 && (load_relaxed_u32(flags + i) || overflow))) continue;
        const int64_t nw64 = ((d.n + 63) >> 6) * 64;
        Track tr{0, INT64_MAX};
        serial_dp<false>(d.bits, d.m, d.n, d.ld_words, nullptr, 0, serial_state,
                         serial_state + nw64, tr);
        const Track w = wave_track(tr);
        const unsigned long long key = w.v > 0 ? make_key(w.v, w.pos) : 0ull;
        if (lane == 0) write_result(key, d.n, out + i);
    }
}

} // namespace msk

// ====================================================================================== host
namespace mshost {

using TS0 = msk::TileShape<16, 16>;
using TS1 = msk::TileShape<32, 16>;
using TS2 = msk::TileShape<32, 32>;

const ProbeVariant PROBE_VARIANTS[NUM_PROBE_VARIANTS] = {{16, 16}, {32, 16}, {32, 32}};

int64_t probe_tile_rows(int variant) {
    switch (variant) {
    case 0: return TS0::TR;
    case 1: return TS1::TR;
    default: return TS2::TR;
    }
}

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

hipError_t launch_pack_u8(const LaunchEnv &env, const uint8_t *a, int64_t m, int64_t n,
                          int64_t ldb, uint64_t *bits, int64_t ldw) {
    const int64_t groups = 4 * cdiv(n, 64);
    dim3 block(256);
    dim3 grid((unsigned)std::min<int64_t>(cdiv(groups, 256), 1 << 20),
              (unsigned)std::min<int64_t>(m, 65535));
    const int aligned = ((uintptr_t)a % 16 == 0) && (ldb % 16 == 0);
    hipLaunchKernelGGL(msk::k_pack_u8, grid, block, 0, env.stream, a, m, n, ldb, bits, ldw,
                       aligned);
    return hipGetLastError();
}

template <class TS>
static void launch_probe(const LaunchEnv &env, const uint64_t *bits, int64_t m, int64_t n,
                         int64_t ldw, ScratchHeader *hdr, uint64_t *sat_list, uint64_t sat_cap,
                         int64_t *ntx_out) {
    const int64_t nwords = cdiv(n, 64);
    const int64_t ntx = cdiv(nwords, TS::OWN_WORDS);
    const int64_t ntiles = cdiv(m, TS::TR) * ntx;
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(cdiv(ntiles, 4),
                                                                   (int64_t)env.num_cus * 8));
    msk::TileSink sink{&hdr->key, &hdr->sat_count, sat_list, sat_cap, 0};
    hipLaunchKernelGGL(msk::k_probe<TS>, dim3((unsigned)blocks), dim3(256), 0, env.stream, bits,
                       m, n, ldw, ntiles, ntx, sink);
    *ntx_out = ntx;
}

hipError_t launch_max_square(const LaunchEnv &env, int variant, const uint64_t *bits, int64_t m,
                             int64_t n, int64_t ldw, ScratchHeader *hdr, uint64_t *sat_list,
                             uint64_t sat_cap, int32_t *serial_state, ms_square *out) {
    int64_t ntx = 0;
    int kc = 16;
    switch (variant) {
    case 0: launch_probe<TS0>(env, bits, m, n, ldw, hdr, sat_list, sat_cap, &ntx); kc = TS0::KC; break;
    case 1: launch_probe<TS1>(env, bits, m, n, ldw, hdr, sat_list, sat_cap, &ntx); kc = TS1::KC; break;
    default: launch_probe<TS2>(env, bits, m, n, ldw, hdr, sat_list, sat_cap, &ntx); kc = TS2::KC; break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t blocks = (int64_t)env.num_cus * 4;
    hipLaunchKernelGGL(msk::k_exact, dim3((unsigned)blocks), dim3(64), 0, env.stream, bits, m, n,
                       ldw, hdr, sat_list, (int64_t)sat_cap, ntx, probe_tile_rows(variant),
                       (int64_t)kc, serial_state, out);
    return hipGetLastError();
}

hipError_t launch_square_map(const LaunchEnv &env, int map_cols, int band_rows,
                             const uint64_t *bits, int64_t m, int64_t n, int64_t ldw, int32_t *dp,
                             int64_t ld_dp, const ms_square *maxsq, int32_t *serial_state) {
    const int vec_ok = ((uintptr_t)dp % 16 == 0) && (ld_dp % 4 == 0);
    const int64_t items_bound = cdiv(m, band_rows) * cdiv(n, 64);
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(cdiv(items_bound, 4),
                                                                   (int64_t)env.num_cus * 8));
    if (map_cols == 8) {
        hipLaunchKernelGGL((msk::k_dpmap<4, 8>), dim3((unsigned)blocks), dim3(256), 0, env.stream,
                           bits, m, n, ldw, dp, ld_dp, maxsq, (int64_t)band_rows, serial_state,
                           vec_ok);
    } else {
        hipLaunchKernelGGL((msk::k_dpmap<8, 4>), dim3((unsigned)blocks), dim3(256), 0, env.stream,
                           bits, m, n, ldw, dp, ld_dp, maxsq, (int64_t)band_rows, serial_state,
                           vec_ok);
    }
    return hipGetLastError();
}

hipError_t launch_write_result(const LaunchEnv &env, ms_square *out, ScratchHeader *hdr,
                               int64_t count) {
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(cdiv(count, 256), 1024));
    hipLaunchKernelGGL(msk::k_write_result, dim3((unsigned)blocks), dim3(256), 0, env.stream, out,
                       hdr, count);
    return hipGetLastError();
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

template <class TS>
static uint64_t tiles_of(const ms_matrix &d) {
    if (d.m <= 0 || d.n <= 0) return 0;
    const int64_t nwords = cdiv(d.n, 64);
    return (uint64_t)(cdiv(d.m, TS::TR) * cdiv(nwords, TS::OWN_WORDS));
}

BatchLayout batch_layout(int variant, const ms_matrix *h_mats, int64_t count) {
    BatchLayout L{};
    uint64_t tiles = 0;
    int64_t maxw = 1;
    for (int64_t i = 0; i < count; ++i) {
        switch (variant) {
        case 0: tiles += tiles_of<TS0>(h_mats[i]); break;
        case 1: tiles += tiles_of<TS1>(h_mats[i]); break;
        default: tiles += tiles_of<TS2>(h_mats[i]); break;
        }
        maxw = std::max<int64_t>(maxw, cdiv(std::max<int64_t>(h_mats[i].n, 1), 64));
    }
    L.sat_cap = tiles;
    L.total_tiles = tiles;
    L.max_nwords = maxw;
    size_t off = 0;
    L.counters = off; off = align256(off + sizeof(msk::BatchCounters));
    L.keys = off; off = align256(off + sizeof(unsigned long long) * (size_t)count);
    L.prefix = off; off = align256(off + sizeof(uint64_t) * (size_t)(count + 1));
    L.flags = off; off = align256(off + sizeof(uint32_t) * (size_t)count);
    L.sat_list = off; off = align256(off + sizeof(uint64_t) * (size_t)std::max<uint64_t>(tiles, 1));
    L.serial_state = off; off = align256(off + sizeof(int32_t) * 2 * 64 * (size_t)maxw);
    L.total = off;
    return L;
}

template <class TS>
static hipError_t launch_batched_t(const LaunchEnv &env, const ms_matrix *mats, int64_t count,
                                   ms_square *out, char *ws, const BatchLayout &L) {
    auto *ctr = reinterpret_cast<msk::BatchCounters *>(ws + L.counters);
    auto *keys = reinterpret_cast<unsigned long long *>(ws + L.keys);
    auto *prefix = reinterpret_cast<uint64_t *>(ws + L.prefix);
    auto *flags = reinterpret_cast<uint32_t *>(ws + L.flags);
    auto *sat = reinterpret_cast<uint64_t *>(ws + L.sat_list);
    auto *state = reinterpret_cast<int32_t *>(ws + L.serial_state);
    hipLaunchKernelGGL(msk::k_batch_init<TS>, dim3(1), dim3(1024), 0, env.stream, mats, count,
                       keys, prefix, flags, ctr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t pblocks = std::max<int64_t>(
        1, std::min<int64_t>(cdiv((int64_t)L.total_tiles, 4), (int64_t)env.num_cus * 8));
    hipLaunchKernelGGL(msk::k_probe_batched<TS>, dim3((unsigned)pblocks), dim3(256), 0,
                       env.stream, mats, count, keys, prefix, ctr, sat, L.sat_cap,
                       (uint64_t)L.total_tiles);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(msk::k_exact_batched, dim3((unsigned)(env.num_cus * 4)), dim3(64), 0,
                       env.stream, mats, keys, flags, ctr, sat, L.sat_cap, (int64_t)TS::TR,
                       (int64_t)TS::KC);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t fb = std::max<int64_t>(1, std::min<int64_t>(count, (int64_t)env.num_cus * 4));
    hipLaunchKernelGGL(msk::k_batch_final, dim3((unsigned)fb), dim3(64), 0, env.stream, mats,
                       count, keys, flags, ctr, state, out);
    return hipGetLastError();
}

hipError_t launch_batched(const LaunchEnv &env, int variant, const ms_matrix *d_mats,
                          int64_t count, ms_square *out, void *ws, const BatchLayout &L) {
    char *w = static_cast<char *>(ws);
    switch (variant) {
    case 0: return launch_batched_t<TS0>(env, d_mats, count, out, w, L);
    case 1: return launch_batched_t<TS1>(env, d_mats, count, out, w, L);
    default: return launch_batched_t<TS2>(env, d_mats, count, out, w, L);
    }
}

} // namespace mshost
