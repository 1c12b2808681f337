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
// per step (rows loaded RECT_GROUP at a time) until V_h is empty.  The longest run is measured
// only at heights that can still reach the best area known: with L the longest run at height
// h, every height below ceil(best / L) is skipped, because V_{h'} is a subset of V_h for h' > h.
// Ties are kept (>=), so the tie-break below stays exact.
//
// Result: the largest area; among the rectangles reaching it, the bottom-right corner first in
// row-major order, then the smallest height.  Each wave folds its rows into one record; the
// last wave to finish (a completion count; nothing waits) reduces the records, writes the
// result and clears the scratch header for the next call.
#include "device.hpp"
#include "launch.hpp"

namespace msk {

constexpr int RECT_GROUP = 4;  // rows loaded together while walking up

__device__ __forceinline__ int32_t ctz64(uint64_t v) {
    return v ? (int32_t)__builtin_ctzll(v) : 64;
}
__device__ __forceinline__ int32_t clz64(uint64_t v) {
    return v ? (int32_t)__builtin_clzll(v) : 64;
}

// A run as one sortable key: longer first, then the smaller end column.
__device__ __forceinline__ uint64_t run_key(int64_t len, int64_t end) {
    return ((uint64_t)len << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)end);
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = __shfl_xor(v, off);
        v = o > v ? o : v;
    }
    return v;
}

__device__ __forceinline__ int64_t wave_max_i64(int64_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const int64_t o = __shfl_xor(v, off);
        v = o > v ? o : v;
    }
    return v;
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
__device__ uint64_t row_longest_run(const uint64_t (&V)[WPL], int lane) {
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
    // composes these maps left to right and a one-lane shift makes it exclusive.
    int32_t a = lf ? 1 : 0, b = ls;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        const int32_t ap = __shfl_up(a, d), bp = __shfl_up(b, d);
        if (lane >= d) {
            b = a ? b + bp : b;
            a = a & ap;
        }
    }
    int32_t c = __shfl_up(b, 1);
    if (lane == 0) c = 0;
    uint64_t best = 0;
    const int64_t base0 = (int64_t)lane * WPL * 64;
#pragma unroll
    for (int k = 0; k < WPL; ++k) {
        const int64_t base = base0 + 64 * k;
        if (F[k]) {
            c += 64;
        } else {
            // the run entering the word ends at its first zero
            const int32_t len = c + P[k];
            if (len > 0) {
                const uint64_t key = run_key(len, base + P[k] - 1);
                best = key > best ? key : best;
            }
            // runs touching neither end of the word
            const uint64_t lo = P[k] ? (~0ull >> (64 - P[k])) : 0ull;
            const uint64_t hi = S[k] ? (~0ull << (64 - S[k])) : 0ull;
            int32_t il, ie;
            word_longest_run(V[k] & ~lo & ~hi, il, ie);
            if (il > 0) {
                const uint64_t key = run_key(il, base + ie);
                best = key > best ? key : best;
            }
            c = S[k];
        }
    }
    // the run reaching the lane's last column (the next lane may extend it; a longer run it
    // belongs to is then reported there, so this shorter prefix never wins)
    if (c > 0) {
        const uint64_t key = run_key(c, base0 + 64 * WPL - 1);
        best = key > best ? key : best;
    }
    return wave_max_u64(best);
}

template <int WPL>
__global__ __launch_bounds__(256) void k_max_rect(const uint64_t *__restrict__ bits, int64_t m,
                                                  int64_t n, int64_t ldw,
                                                  mshost::RectScratch *rs,
                                                  mshost::RectRecord *rec, ms_rect *out) {
    const int lane = __lane_id();
    const int64_t wave = wave_index();
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) / WAVE;
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
        int64_t h = 1, next_eval = 1;
        // every trip raises h by at least one and h never passes i + 1
        while (true) {
            uint64_t any = 0;
#pragma unroll
            for (int k = 0; k < WPL; ++k) any |= V[k];
            if (!__ballot(any != 0)) break;
            if (h >= next_eval) {
                const uint64_t key = row_longest_run<WPL>(V, lane);
                const int64_t len = uniform((int64_t)(key >> 32));
                const int64_t end = uniform((int64_t)(0xFFFFFFFFu - (uint32_t)key));
                const int64_t area = h * len;
                if (area > ra || (area == ra && end < re)) {
                    ra = area;
                    re = end;
                    rh = h;
                }
                const int64_t g = uniform((int64_t)load_relaxed(&rs->best_area));
                const int64_t best = g > ra ? g : ra;
                next_eval = (best + len - 1) / len;
                if (next_eval <= h) next_eval = h + 1;
            }
            if (h >= i + 1 || next_eval > i + 1) break;
            // heights h + 1 .. : the rows above, RECT_GROUP loads in flight together
            const int64_t h0 = h;
            uint64_t R[RECT_GROUP][WPL];
#pragma unroll
            for (int u = 0; u < RECT_GROUP; ++u) {
                const int64_t r = i - h0 - u;
                const int64_t rc = r >= 0 ? r : 0;
#pragma unroll
                for (int k = 0; k < WPL; ++k) R[u][k] = bits[rc * ldw + wc[k]] & wm[k];
            }
            bool stop = false;
#pragma unroll
            for (int u = 0; u < RECT_GROUP; ++u) {
                if (!stop) {
                    const bool inside = i - h0 - u >= 0;  // rows above the matrix are zeros
#pragma unroll
                    for (int k = 0; k < WPL; ++k) V[k] = inside ? (V[k] & R[u][k]) : 0ull;
                    h += 1;
                    stop = h >= next_eval || h >= i + 1;
                }
            }
        }
        if (ra > 0) {
            const int64_t pos = i * n + re;
            if (ra > wa || (ra == wa && (pos < wp || (pos == wp && rh < wh)))) {
                wa = ra;
                wp = pos;
                wh = rh;
            }
            if (lane == 0) atomicMax(&rs->best_area, (unsigned long long)ra);
        }
    }
    if (lane == 0) {
        rec[wave].area = wa;
        rec[wave].pos = wp;
        rec[wave].height = wh;
    }
    __threadfence();
    uint32_t prev = 0;
    if (lane == 0) prev = atomicAdd(&rs->done, 1u);
    prev = (uint32_t)uniform((int32_t)prev);
    if (prev != (uint32_t)(nwave - 1)) return;
    // last wave: every record is written; reduce them (area desc, position asc, height asc)
    __threadfence();
    int64_t ba = 0, bp = -1, bh = 0;
    for (int64_t r = lane; r < nwave; r += WAVE) {
        const int64_t a = __hip_atomic_load(&rec[r].area, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
        const int64_t p = __hip_atomic_load(&rec[r].pos, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
        const int64_t hh = __hip_atomic_load(&rec[r].height, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
        if (a > ba || (a == ba && a > 0 && (p < bp || (p == bp && hh < bh)))) {
            ba = a;
            bp = p;
            bh = hh;
        }
    }
    const int64_t A = wave_max_i64(ba);
    const int64_t P = wave_min_i64(ba == A ? bp : INT64_MAX);
    const int64_t Hh = wave_min_i64(ba == A && bp == P ? bh : INT64_MAX);
    if (lane == 0) {
        ms_rect res;
        if (A > 0) {
            res.area = A;
            res.row = P / n;
            res.col = P % n;
            res.height = Hh;
            res.width = A / Hh;
        } else {
            res.area = 0;
            res.row = -1;
            res.col = -1;
            res.height = 0;
            res.width = 0;
        }
        *out = res;
        rs->best_area = 0;
        rs->done = 0;
    }
}

} // namespace msk

namespace mshost {

int64_t rect_max_waves(int num_cus) { return (int64_t)num_cus * RECT_BLOCKS_PER_CU * 4; }

hipError_t launch_max_rect(const LaunchEnv &env, const uint64_t *bits, int64_t m, int64_t n,
                           int64_t ldw, RectScratch *rs, ms_rect *out) {
    RectRecord *rec = reinterpret_cast<RectRecord *>(rs + 1);
    const int64_t nwords = (n + 63) / 64;
    if (m == 0 || n == 0) m = 0;  // no rows: the single block reports the empty result
    const int64_t blocks = std::max<int64_t>(
        1, std::min<int64_t>((m + 3) / 4, (int64_t)env.num_cus * RECT_BLOCKS_PER_CU));
    const dim3 g((unsigned)blocks), b(256);
    if (nwords <= 64) {
        hipLaunchKernelGGL(msk::k_max_rect<1>, g, b, 0, env.stream, bits, m, n, ldw, rs, rec,
                           out);
    } else if (nwords <= 128) {
        hipLaunchKernelGGL(msk::k_max_rect<2>, g, b, 0, env.stream, bits, m, n, ldw, rs, rec,
                           out);
    } else if (nwords <= 256) {
        hipLaunchKernelGGL(msk::k_max_rect<4>, g, b, 0, env.stream, bits, m, n, ldw, rs, rec,
                           out);
    } else {
        hipLaunchKernelGGL(msk::k_max_rect<8>, g, b, 0, env.stream, bits, m, n, ldw, rs, rec,
                           out);
    }
    return hipGetLastError();
}

} // namespace mshost
