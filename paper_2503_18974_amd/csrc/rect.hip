// rect.hip -- largest all-ones rectangle of a packed binary matrix, and its host launcher.
//
// This extends the square problem the way the paper's future work proposes (Section 6), with
// the histogram view its related work describes (Section 2.3): each row is a histogram of the
// heights H[i][j] of the runs of ones ending at row i.  For bottom row i and height h, the
// columns with H[i][j] >= h are the set bits of
//     V_h[i] = AND of the packed rows i-h+1 .. i,
// and the widest all-ones rectangle of height h whose bottom row is i spans the longest run of
// ones in V_h[i].  The largest area is the maximum of h * longest_run(V_h[i]) over all (i, h).
//
// Work split: a wave owns one bottom row at a time, holding it as WPL consecutive packed words
// per lane (so a run is a carry chain across lanes), and walks h upwards, ANDing one more row
// per step (the next QD rows above always in flight) until V_h is empty.  The longest run is measured
// only at heights that can still reach the best area known: with L the longest run at height
// h, every height below ceil(best / L) is skipped, because V_{h'} is a subset of V_h for h' > h.
// Ties are kept (>=), so the tie-break below stays exact.
//
// Result: the largest area; among the rectangles reaching it, the bottom-right corner first in
// row-major order, then the smallest height.  Each block folds its rows into one record; a
// one-block kernel that follows on the stream (k_rect_final) reduces the records, writes the
// result and clears the scratch header for the next call.
#include "device.hpp"
#include "launch.hpp"

namespace msk {

// Rows kept in flight while walking up: QD rows of WPL words per lane.
template <int WPL>
struct RectQueue {
    static constexpr int QD = WPL <= 2 ? 8 : (WPL == 4 ? 4 : 2);
};

__device__ __forceinline__ int32_t ctz64(uint64_t v) {
    return v ? (int32_t)__builtin_ctzll(v) : 64;
}
__device__ __forceinline__ int32_t clz64(uint64_t v) {
    return v ? (int32_t)__builtin_clzll(v) : 64;
}

// A run as one sortable 32-bit key: longer first, then the smaller end column (rows are at most
// 32768 columns, so both fit in 16 bits).
__device__ __forceinline__ uint32_t run_key(int32_t len, int32_t end) {
    return ((uint32_t)len << 16) | (uint32_t)(0xFFFF - end);
}

// Wave maximum, returned to every lane: DPP shifts within each row of 16 lanes (lane 15 of a row
// ends with the row's maximum; lanes shifted in from outside the row read 0), then the four row
// results through scalar registers.  No LDS round trips.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
    uint32_t t;
    t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)v, 0x111, 0xf, 0xf, true);  // row_shr:1
    v = t > v ? t : v;
    t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)v, 0x112, 0xf, 0xf, true);  // row_shr:2
    v = t > v ? t : v;
    t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)v, 0x114, 0xf, 0xf, true);  // row_shr:4
    v = t > v ? t : v;
    t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)v, 0x118, 0xf, 0xf, true);  // row_shr:8
    v = t > v ? t : v;
    const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int32_t)v, 15);
    const uint32_t r1 = (uint32_t)__builtin_amdgcn_readlane((int32_t)v, 31);
    const uint32_t r2 = (uint32_t)__builtin_amdgcn_readlane((int32_t)v, 47);
    const uint32_t r3 = (uint32_t)__builtin_amdgcn_readlane((int32_t)v, 63);
    const uint32_t a = r0 > r1 ? r0 : r1, b = r2 > r3 ? r2 : r3;
    return a > b ? a : b;
}

__device__ __forceinline__ int64_t wave_max_i64(int64_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const int64_t o = __shfl_xor(v, off);
        v = o > v ? o : v;
    }
    return v;
}

// Folds the candidate (a, p, h) into the best (ba, bp, bh): the larger area, then the smaller
// corner position, then the smaller height.
__device__ __forceinline__ void better(int64_t a, int64_t p, int64_t h, int64_t &ba, int64_t &bp,
                                       int64_t &bh) {
    if (a > ba || (a == ba && a > 0 && (p < bp || (p == bp && h < bh)))) {
        ba = a;
        bp = p;
        bh = h;
    }
}

// Longest run of ones inside one word and the bit where its first occurrence ends.  E_k marks
// the bits ending k consecutive ones (E_{2k} = E_k & E_k << k); a descent over k = 32 .. 1
// grows the run while E_{L+k} = E_L & (E_k << L) stays non-empty.  x must not be all ones.
__device__ __forceinline__ void word_longest_run(uint64_t x, int32_t &len, int32_t &end) {
    uint64_t E[6];
    E[0] = x;
#pragma unroll
    for (int b = 1; b < 6; ++b) E[b] = E[b - 1] & (E[b - 1] << (1 << (b - 1)));
    uint64_t cur = ~0ull;
    int32_t L = 0;
#pragma unroll
    for (int b = 5; b >= 0; --b) {
        const uint64_t t = cur & (E[b] << L);
        if (t) {
            cur = t;
            L += 1 << b;
        }
    }
    len = L;
    end = L ? ctz64(cur) : 0;
}

// Longest run of ones of a row held as WPL consecutive words per lane (lane l: words
// l * WPL .. l * WPL + WPL - 1), as a run_key: the leftmost among the longest; 0 when empty.
template <int WPL>
__device__ uint32_t row_longest_run(const uint64_t (&V)[WPL], int lane) {
    int32_t P[WPL], S[WPL];
    bool F[WPL];
    int32_t ls = 0;  // run reaching the lane's last column, from the lane's own words
    bool lf = true;
#pragma unroll
    for (int k = 0; k < WPL; ++k) {
        const uint64_t x = V[k];
        F[k] = x == ~0ull;
        P[k] = ctz64(~x);   // 64 when the word is full
        S[k] = clz64(~x);
        ls = F[k] ? ls + 64 : S[k];
        lf = lf && F[k];
    }
    // Carry into each lane: the run ending just left of its first column.  A lane maps the run
    // entering it, c, to a c + b (a = 1 when all its words are full, b = ls); an inclusive scan
    // composes these maps left to right and a one-lane shift makes it exclusive.  With no full
    // lane (the common case once a few rows are ANDed) the carry is the left lane's ls.
    int32_t b = ls;
    if (__ballot(lf)) {
        int32_t a = lf ? 1 : 0;
#pragma unroll
        for (int d = 1; d < WAVE; d <<= 1) {
            const int32_t ap = __shfl_up(a, d), bp = __shfl_up(b, d);
            if (lane >= d) {
                b = a ? b + bp : b;
                a = a & ap;
            }
        }
    }
    int32_t c = from_left_lane(b, 0);
    uint32_t best = 0;
    const int32_t base0 = lane * WPL * 64;
#pragma unroll
    for (int k = 0; k < WPL; ++k) {
        const int32_t base = base0 + 64 * k;
        if (F[k]) {
            c += 64;
        } else {
            // the run entering the word ends at its first zero
            const int32_t len = c + P[k];
            if (len > 0) {
                const uint32_t key = run_key(len, base + P[k] - 1);
                best = key > best ? key : best;
            }
            // runs touching neither end of the word
            const uint64_t lo = P[k] ? (~0ull >> (64 - P[k])) : 0ull;
            const uint64_t hi = S[k] ? (~0ull << (64 - S[k])) : 0ull;
            int32_t il, ie;
            word_longest_run(V[k] & ~lo & ~hi, il, ie);
            if (il > 0) {
                const uint32_t key = run_key(il, base + ie);
                best = key > best ? key : best;
            }
            c = S[k];
        }
    }
    // the run reaching the lane's last column (the next lane may extend it; a longer run it
    // belongs to is then reported there, so this shorter prefix never wins)
    if (c > 0) {
        const uint32_t key = run_key(c, base0 + 64 * WPL - 1);
        best = key > best ? key : best;
    }
    return wave_max_u32(best);
}

template <int WPL>
__global__ __launch_bounds__(256) void k_max_rect(const uint64_t *__restrict__ bits, int64_t m,
                                                  int64_t n, int64_t ldw,
                                                  mshost::RectScratch *rs,
                                                  mshost::RectRecord *rec) {
    const int lane = __lane_id();
    const int64_t wave = wave_index();
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) / WAVE;
    constexpr int QD = RectQueue<WPL>::QD;
    m = uniform(m);
    n = uniform(n);
    ldw = uniform(ldw);
    const int64_t nwords = (n + 63) >> 6;
    const uint64_t lastmask = last_word_mask(n);
    // this lane's words: an in-bounds index (clamped) and a mask clearing padding and absent words
    int64_t wc[WPL];
    uint64_t wm[WPL];
#pragma unroll
    for (int k = 0; k < WPL; ++k) {
        const int64_t w = (int64_t)lane * WPL + k;
        wm[k] = w < nwords ? (w == nwords - 1 ? lastmask : ~0ull) : 0ull;
        wc[k] = w < nwords ? w : nwords - 1;
    }
    int64_t wa = 0, wp = -1, wh = 0;  // the wave's best: area, position i * n + col, height
    for (int64_t i = wave; i < m; i += nwave) {
        uint64_t V[WPL];
#pragma unroll
        for (int k = 0; k < WPL; ++k) V[k] = bits[i * ldw + wc[k]] & wm[k];
        int64_t ra = 0, re = -1, rh = 0;  // the row's best: area, end column, height
        // the best area any finished row has published: g is what the previous evaluation
        // loaded (its device-scope load has the steps in between to arrive)
        int64_t g = uniform((int64_t)load_relaxed(&rs->best_area));
        // Q[u] holds a row above: at height h the next row to AND (row i - h) sits in slot
        // (h - 1) % QD, loaded QD heights earlier, so QD loads stay in flight.  The walk is
        // unrolled by QD so that every slot index is static (a register, never moved while its
        // load is in flight).
        uint64_t Q[QD][WPL];
#pragma unroll
        for (int u = 0; u < QD; ++u) {
            const int64_t r = i - 1 - u;
            const int64_t rc = r >= 0 ? r : 0;
#pragma unroll
            for (int k = 0; k < WPL; ++k) Q[u][k] = bits[rc * ldw + wc[k]];
        }
        int64_t h = 1, next_eval = 1;
        bool done = false;
        // every round raises h by QD unless the walk ends; h never passes i + 1
        while (!done) {
#pragma unroll
            for (int u = 0; u < QD; ++u) {
                if (done) continue;
                uint64_t any = 0;
#pragma unroll
                for (int k = 0; k < WPL; ++k) any |= V[k];
                if (!__ballot(any != 0)) {
                    done = true;
                    continue;
                }
                if (h >= next_eval) {
                    const uint32_t key = row_longest_run<WPL>(V, lane);
                    const int64_t len = uniform((int32_t)(key >> 16));
                    const int64_t end = uniform((int32_t)(0xFFFF - (key & 0xFFFF)));
                    const int64_t area = h * len;
                    if (area > ra || (area == ra && end < re)) {
                        ra = area;
                        re = end;
                        rh = h;
                    }
                    const int64_t best = g > ra ? g : ra;
                    g = uniform((int64_t)load_relaxed(&rs->best_area));
                    next_eval = (best + len - 1) / len;
                    if (next_eval <= h) next_eval = h + 1;
                }
                if (h >= i + 1 || next_eval > i + 1) {
                    done = true;
                    continue;
                }
                // height h + 1: AND row i - h (inside the matrix, since h <= i), then refill the
                // slot with the row QD heights further up (zeros above the matrix)
#pragma unroll
                for (int k = 0; k < WPL; ++k) V[k] &= Q[u][k] & wm[k];
                const int64_t r = i - h - QD;
                const int64_t rc = r >= 0 ? r : 0;
                const uint64_t keep = r >= 0 ? ~0ull : 0ull;
#pragma unroll
                for (int k = 0; k < WPL; ++k) Q[u][k] = bits[rc * ldw + wc[k]] & keep;
                h += 1;
            }
        }
        if (ra > 0) {
            const int64_t pos = i * n + re;
            if (ra > wa || (ra == wa && (pos < wp || (pos == wp && rh < wh)))) {
                wa = ra;
                wp = pos;
                wh = rh;
            }
            // publish only what beats the last value seen: one address takes every atomic
            if (ra > g && lane == 0) atomicMax(&rs->best_area, (unsigned long long)ra);
        }
    }
    // fold the four waves' bests into one record per block; k_rect_final reduces the records
    __shared__ int64_t s_a[4], s_p[4], s_h[4];
    const int wv = threadIdx.x / WAVE;
    if (lane == 0) {
        s_a[wv] = wa;
        s_p[wv] = wp;
        s_h[wv] = wh;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t ba = 0, bp = -1, bh = 0;
        for (int w = 0; w < 4; ++w) better(s_a[w], s_p[w], s_h[w], ba, bp, bh);
        rec[blockIdx.x].area = ba;
        rec[blockIdx.x].pos = bp;
        rec[blockIdx.x].height = bh;
    }
}

// One block, after k_max_rect on the same stream: reduces the per-block records (largest area,
// then smallest position, then smallest height), writes the result and clears the best area
// for the next call.
__global__ __launch_bounds__(256) void k_rect_final(const mshost::RectRecord *__restrict__ rec,
                                                    int64_t nrec, int64_t n,
                                                    mshost::RectScratch *rs, ms_rect *out) {
    __shared__ int64_t s_a[4], s_p[4], s_h[4];
    const int lane = __lane_id(), wv = threadIdx.x / WAVE;
    int64_t ba = 0, bp = -1, bh = 0;
    for (int64_t r = threadIdx.x; r < nrec; r += blockDim.x)
        better(rec[r].area, rec[r].pos, rec[r].height, ba, bp, bh);
    const int64_t A = wave_max_i64(ba);
    const int64_t P = wave_min_i64(ba == A ? bp : INT64_MAX);
    const int64_t Hh = wave_min_i64(ba == A && bp == P ? bh : INT64_MAX);
    if (lane == 0) {
        s_a[wv] = A;
        s_p[wv] = P;
        s_h[wv] = Hh;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t fa = 0, fp = -1, fh = 0;
        for (int w = 0; w < 4; ++w) better(s_a[w], s_p[w], s_h[w], fa, fp, fh);
        ms_rect res;
        if (fa > 0) {
            res.area = fa;
            res.row = fp / n;
            res.col = fp % n;
            res.height = fh;
            res.width = fa / fh;
        } else {
            res.area = 0;
            res.row = -1;
            res.col = -1;
            res.height = 0;
            res.width = 0;
        }
        *out = res;
        rs->best_area = 0;
    }
}

} // namespace msk

namespace mshost {

int64_t rect_max_blocks(int num_cus) { return (int64_t)num_cus * RECT_BLOCKS_PER_CU; }

hipError_t launch_max_rect(const LaunchEnv &env, const uint64_t *bits, int64_t m, int64_t n,
                           int64_t ldw, RectScratch *rs, ms_rect *out) {
    RectRecord *rec = reinterpret_cast<RectRecord *>(rs + 1);
    const int64_t nwords = (n + 63) / 64;
    if (m == 0 || n == 0) m = 0;  // no rows: the single block reports the empty result
    const int64_t blocks = std::max<int64_t>(
        1, std::min<int64_t>((m + 3) / 4, (int64_t)env.num_cus * RECT_BLOCKS_PER_CU));
    const dim3 g((unsigned)blocks), b(256);
    if (nwords <= 64) {
        hipLaunchKernelGGL(msk::k_max_rect<1>, g, b, 0, env.stream, bits, m, n, ldw, rs, rec);
    } else if (nwords <= 128) {
        hipLaunchKernelGGL(msk::k_max_rect<2>, g, b, 0, env.stream, bits, m, n, ldw, rs, rec);
    } else if (nwords <= 256) {
        hipLaunchKernelGGL(msk::k_max_rect<4>, g, b, 0, env.stream, bits, m, n, ldw, rs, rec);
    } else {
        hipLaunchKernelGGL(msk::k_max_rect<8>, g, b, 0, env.stream, bits, m, n, ldw, rs, rec);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(msk::k_rect_final, dim3(1), dim3(256), 0, env.stream, rec, blocks,
                       std::max<int64_t>(n, 1), rs, out);
    return hipGetLastError();
}

} // namespace mshost
