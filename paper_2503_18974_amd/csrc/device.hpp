// device.hpp -- device-side building blocks of libmaxsq (gfx950, wave64).
//
//  * dprun      : the per-cell side map dp[i][j] (Section 2.1 eq. (1)) evaluated row by row
//                 over a column window, in the rows-parallel form
//                     dp = A ? min(H, W, dp[i-1][j-1] + 1) : 0
//                 where H is the column run of ones ending at (i, j) -- the paper's frequency
//                 array freq[j] (Section 3, Algorithm 1) -- and W is the row run of ones
//                 ending at (i, j).  A zero state at the window's top-left edge is exact for
//                 every cell whose true value is at most the distance to that edge, so bands
//                 and windows that start at least S rows / columns early are exact.
//  * tile_search: the greedy validation of Algorithm 1 turned into a bitwise test: does the
//                 tile contain a k x k all-ones square?  E_k (k x k squares ending at each cell)
//                 is built by erosion, E_{a+d} = E_a & up_d(E_a) & left_d(E_a) & upleft_d(E_a)
//                 for d <= a, inside a register tile, with a galloping-then-bisecting search
//                 over k.  The paper's invariant that a side k + 1 is only considered once k is
//                 validated is what makes the search monotone (E_{k+1} is a subset of E_k).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace msk {

constexpr int WAVE = 64;
constexpr unsigned long long KEY_POS_MASK = (1ull << 44) - 1;

// Result key: larger side wins, then the smaller row-major position (i * n + j).
__device__ __forceinline__ unsigned long long make_key(int64_t side, int64_t pos) {
    return ((unsigned long long)side << 44) | (KEY_POS_MASK - (unsigned long long)pos);
}
__device__ __forceinline__ int64_t key_side(unsigned long long k) { return (int64_t)(k >> 44); }
__device__ __forceinline__ int64_t key_pos(unsigned long long k) {
    return (int64_t)(KEY_POS_MASK - (k & KEY_POS_MASK));
}

__device__ __forceinline__ unsigned long long load_relaxed(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t load_relaxed_u32(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int64_t wave_min_i64(int64_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        int64_t o = __shfl_xor(v, off);
        v = o < v ? o : v;
    }
    return v;
}

__device__ __forceinline__ int32_t wave_max_i32(int32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        int32_t o = __shfl_xor(v, off);
        v = o > v ? o : v;
    }
    return v;
}

// Word k of a packed row with the padding bits of the last word cleared; 0 beyond the row.
__device__ __forceinline__ uint64_t row_word(const uint64_t *__restrict__ row, int64_t k,
                                             int64_t nwords, uint64_t lastmask) {
    if (k < 0 || k >= nwords) return 0;
    uint64_t v = row[k];
    return (k == nwords - 1) ? (v & lastmask) : v;
}

__device__ __forceinline__ uint64_t last_word_mask(int64_t n) {
    return (n & 63) ? ((1ull << (n & 63)) - 1) : ~0ull;
}

// Number of consecutive ones at the top (most significant end) of v.
__device__ __forceinline__ int32_t leading_ones(uint64_t v) {
    return (v == ~0ull) ? 64 : (int32_t)__clzll(~v);
}

// A value every lane of the wave holds equally, moved to a scalar register so the compiler
// treats what depends on it (loop bounds, branches, addresses) as wave-uniform.
__device__ __forceinline__ int64_t uniform(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ int32_t uniform(int32_t v) {
    return (int32_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
}

// a / b for a >= 0, b > 0: one 32-bit division when both fit (every matrix dimension and tile
// count short of 2^32), instead of the ~100-instruction 64-bit routine.
__device__ __forceinline__ int64_t udiv(int64_t a, int64_t b) {
    if ((((uint64_t)a | (uint64_t)b) >> 32) == 0) return (int64_t)((uint32_t)a / (uint32_t)b);
    return a / b;
}

// Global index of the calling wave (uniform).
__device__ __forceinline__ int64_t wave_index() {
    return uniform((int64_t)(((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE));
}

// Lane l receives lane l-1's value, lane 0 receives `first` (DPP wave_shr:1).
__device__ __forceinline__ int32_t from_left_lane(int32_t v, int32_t first) {
    return __builtin_amdgcn_update_dpp(first, v, 0x138, 0xf, 0xf, false);
}

// Within each row of 16 lanes, lane l receives lane l-1's value; the first lane of every row
// receives 0 (DPP row_shr:1 with bound control).
__device__ __forceinline__ uint32_t from_left_in_row16(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)v, 0x111, 0xf, 0xf, true);
}

// Per-lane running maximum with the first row-major position (for the tracking mode).
struct Track {
    int32_t v;
    int64_t pos;
};

// Reduce per-lane Track to the wave's (max value, smallest position among lanes at max).
__device__ __forceinline__ Track wave_track(Track t) {
    int32_t best = wave_max_i32(t.v);
    int64_t p = (t.v == best) ? t.pos : INT64_MAX;
    p = wave_min_i64(p);
    return Track{best, p};
}

// Length of the run of ones that ends just left of bit b of the packed word x (LSB first), given
// `carry`, the run entering x, and lowmask = the bits below b: b - 1 minus the index of the
// highest zero below b, or b + carry when there is none (the count of leading zeros of an empty
// mask is 64).
__device__ __forceinline__ int32_t run_into(uint64_t x, uint64_t lowmask, int b, int32_t carry) {
    const int32_t lz = (int32_t)__clzll(~x & lowmask);
    return lz + (b - 64) + (lz == 64 ? carry : 0);
}

// One cell of the recurrence, for a cell with value `bit` (0 or 1), column height H above it, row
// run w ending just left of it and dp[i-1][j-1] = dprev: since every term of the minimum gains
// one when the cell is set,
//     dp = bit ? 1 + min(H, w, dprev) : 0,    H <- bit ? H + 1 : 0,    w <- bit ? w + 1 : 0,
// each "bit ? v + 1 : 0" being the 24-bit multiply-add v * bit + bit.  The windowed passes keep
// every operand below 2^24: heights count the rows of one item (a band plus its halo), runs the
// columns of one window.
__device__ __forceinline__ int32_t cell_step(int32_t &H, int32_t &w, int32_t dprev, uint32_t bit) {
    int32_t m3 = H < w ? H : w;
    m3 = m3 < dprev ? m3 : dprev;
    H = (int32_t)(__umul24((uint32_t)H, bit) + bit);
    w = (int32_t)(__umul24((uint32_t)w, bit) + bit);
    return (int32_t)(__umul24((uint32_t)m3, bit) + bit);
}

// ----------------------------------------------------------------------------------------------
// dprun: dp over rows [rh, rb) x columns [xh, xh + ng * 64 * CPL), zero state above row rh and
// left of column xh (xh is a multiple of 64).  Lane l of group g owns the CPL consecutive
// columns xh + g * 64 * CPL + l * CPL + t.  Cells with row >= ra and xa <= col < xb are owned:
// stored into dp (STORE) and/or folded into the per-lane Track (TRACK).
//
// Rows are staged through LDS in chunks: the wave first loads a chunk of the window's packed
// words (all loads in flight at once), then one lane per row scans that row's words once to get
// the row run W entering every word, and only then walks the rows.  Per row and group a lane
// reads its word and its entering run from LDS; dp[i-1][c-1] for its first column comes from
// the lane to its left (previous row), and for lane 0 from the previous group's last column,
// saved before that group was overwritten.
// ----------------------------------------------------------------------------------------------
constexpr int LDS_WORDS = 1024;  // staged packed words per wave

struct WaveLds {
    uint64_t *x;   // `cap` packed words
    int32_t *c;    // `cap` entering row runs
    int cap = LDS_WORDS;
};

// Which owned cells a pass stores, when the map is split by tile class: bit k of cls[g] is set
// when the lane's columns of group g in tile row ty0 + k (tile rows of `tile_rows` rows) belong
// to the pass.  With `on` false every owned cell is stored.
template <int NGMAX>
struct StoreClass {
    bool on = false;
    int64_t tile_rows = 1, ty0 = 0;
    uint64_t cls[NGMAX];
};

template <int NGMAX, int CPL, bool STORE, bool TRACK, bool CLASSED = false>
__device__ void dprun(const uint64_t *__restrict__ bits, int64_t ldw, int64_t n, int64_t rh,
                      int64_t ra, int64_t rb, int64_t xh, int64_t xa, int64_t xb, int ng,
                      int32_t *__restrict__ dp, int64_t ld_dp, bool vec_ok, Track &tr,
                      WaveLds lds, const StoreClass<NGMAX> &sc = StoreClass<NGMAX>{}) {
    static_assert(CPL == 4 || CPL == 8, "columns per lane");
    static_assert(NGMAX * CPL <= 64, "window words must fit one wave");
    rh = uniform(rh);
    ra = uniform(ra);
    rb = uniform(rb);
    xh = uniform(xh);
    xa = uniform(xa);
    xb = uniform(xb);
    ng = uniform(ng);
    ldw = uniform(ldw);
    n = uniform(n);
    ld_dp = uniform(ld_dp);
    constexpr int GW = 64 * CPL;  // columns per group
    constexpr int LPW = 64 / CPL; // lanes per word
    const int lane = __lane_id();
    const int q = lane / LPW;           // word of the group holding this lane's columns
    const int b = (lane % LPW) * CPL;   // bit offset of the lane's first column in that word
    const uint64_t lowmask = (1ull << b) - 1;  // the word's bits left of the lane's columns
    const int64_t nwords = (n + 63) >> 6;
    const uint64_t lastmask = last_word_mask(n);
    // 1 <= ng <= NGMAX whatever the caller computed, so nww is 4..64 words and both loop steps
    // below (rows per chunk, staging rows per pass) are at least one
    ng = ng < 1 ? 1 : (ng > NGMAX ? NGMAX : ng);
    const int nww = ng * CPL;                    // window words
    const int rc_max = lds.cap / nww;            // rows per chunk
    const int fl_w = lane % nww, fl_r = lane / nww, fl_rpp = 64 / nww;
    const int64_t fl_word = (xh >> 6) + fl_w;
    const bool fl_ok = fl_r < fl_rpp && fl_word < nwords;
    const uint64_t fl_mask = (fl_word == nwords - 1) ? lastmask : ~0ull;
    const int64_t fl_wc = fl_word < nwords ? fl_word : nwords - 1;  // always a valid word

    int32_t H[NGMAX][CPL], D[NGMAX][CPL];
#pragma unroll
    for (int g = 0; g < NGMAX; ++g)
#pragma unroll
        for (int t = 0; t < CPL; ++t) {
            H[g][t] = 0;
            D[g][t] = 0;
        }
    // tile row of the current row relative to ty0, and the row's offset in its tile row,
    // advanced per row (no division in the row loop)
    int64_t kq = 0, kr = 0;
    if (CLASSED) {
        kq = uniform(rh / sc.tile_rows - sc.ty0);
        kr = uniform(rh % sc.tile_rows);
    }

    for (int64_t r0 = rh; r0 < rb; r0 += rc_max) {
        const int rc = (int)(rb - r0 < rc_max ? rb - r0 : rc_max);
        // stage the chunk's words: eight rows' loads in flight per batch, from in-bounds
        // (clamped) addresses, masked afterwards
        constexpr int FB = 8;
        for (int rb0 = fl_r; rb0 < rc; rb0 += FB * fl_rpp) {
            uint64_t v[FB];
#pragma unroll
            for (int u = 0; u < FB; ++u) {
                const int r = rb0 + u * fl_rpp;
                const int r_c = r < rc ? r : rc - 1;
                v[u] = bits[(r0 + r_c) * ldw + fl_wc];
            }
#pragma unroll
            for (int u = 0; u < FB; ++u) {
                const int r = rb0 + u * fl_rpp;
                if (r < rc && fl_r < fl_rpp) lds.x[r * nww + fl_w] = fl_ok ? (v[u] & fl_mask) : 0ull;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        // row run entering each word (zero at the window's left edge)
        for (int r = lane; r < rc; r += WAVE) {
            int32_t run = 0;
            for (int w = 0; w < nww; ++w) {
                const uint64_t v = lds.x[r * nww + w];
                lds.c[r * nww + w] = run;
                run = (v == ~0ull) ? run + 64 : leading_ones(v);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        // rows are walked two at a time through two register sets, so that the next row's
        // words and entering runs are read from LDS while the current row is computed.  The
        // reads are unconditional (a group past ng rereads group 0, a row past the chunk rereads
        // its last row; neither is used), so that no branch or register reset sits between a
        // read and its use and the wait before a row covers only that row's reads.
        const auto load_row = [&](int rr, uint64_t (&x)[NGMAX], int32_t (&cr)[NGMAX]) {
#pragma unroll
            for (int g = 0; g < NGMAX; ++g) {
                const int o = rr * nww + (g < ng ? g : 0) * CPL + q;
                x[g] = lds.x[o];
                cr[g] = lds.c[o];
            }
        };
        // rows of the chunk from own_from on are owned (32-bit, uniform)
        const int own_from = (int)(ra - r0 > 0 ? (ra - r0 < rc ? ra - r0 : rc) : 0);
        // common case: 16-byte stores, and every lane owns all or none of its columns (xa is a
        // multiple of 64, so only a right edge that is not a multiple of CPL splits a lane)
        const bool whole = vec_ok && (CPL % 4 == 0) && (xb % CPL) == 0;
        const auto row = [&](int rr, const uint64_t (&cx)[NGMAX], const int32_t (&ccr)[NGMAX]) {
            const int64_t i = r0 + rr;
            const bool own_row = rr >= own_from;
            int32_t dleft_old = 0;  // previous-row dp just left of the group
            const int krow = (CLASSED && own_row) ? (int)kq : 0;
            if (CLASSED && ++kr == sc.tile_rows) {
                kr = 0;
                ++kq;
            }
#pragma unroll
            for (int g = 0; g < NGMAX; ++g) {
                if (g < ng) {
                    const uint64_t x = cx[g];
                    const int32_t carry = ccr[g];
                    const int32_t wrun = run_into(x, lowmask, b, carry);
                    const uint32_t nib = (uint32_t)(x >> b) & ((1u << CPL) - 1u);
                    int32_t dprev = from_left_lane(D[g][CPL - 1], dleft_old);
                    dleft_old = __builtin_amdgcn_readlane(D[g][CPL - 1], WAVE - 1);
                    int32_t w = wrun;
#pragma unroll
                    for (int t = 0; t < CPL; ++t) {
                        const int32_t old = D[g][t];
                        D[g][t] = cell_step(H[g][t], w, dprev, (nib >> t) & 1u);
                        dprev = old;
                    }
                    const int64_t col = xh + (int64_t)g * GW + (int64_t)lane * CPL;
                    if (STORE && !TRACK && whole) {
                        if (own_row && col >= xa && col < xb &&
                            (!CLASSED || ((sc.cls[g] >> krow) & 1))) {
                            int32_t *p = dp + i * ld_dp + col;
#pragma unroll
                            for (int t = 0; t < CPL; t += 4)
                                *reinterpret_cast<int4 *>(p + t) =
                                    make_int4(D[g][t], D[g][t + 1], D[g][t + 2], D[g][t + 3]);
                        }
                    } else if (own_row && (!CLASSED || ((sc.cls[g] >> krow) & 1))) {
                        if (STORE) {
                            int32_t *p = dp + i * ld_dp + col;
                            if (col >= xa && col + CPL <= xb) {
                                if (vec_ok) {
#pragma unroll
                                    for (int t = 0; t < CPL; t += 4)
                                        *reinterpret_cast<int4 *>(p + t) = make_int4(
                                            D[g][t], D[g][t + 1], D[g][t + 2], D[g][t + 3]);
                                } else {
#pragma unroll
                                    for (int t = 0; t < CPL; ++t) p[t] = D[g][t];
                                }
                            } else {
#pragma unroll
                                for (int t = 0; t < CPL; ++t)
                                    if (col + t >= xa && col + t < xb) p[t] = D[g][t];
                            }
                        }
                        if (TRACK) {
#pragma unroll
                            for (int t = 0; t < CPL; ++t) {
                                const bool own = col + t >= xa && col + t < xb;
                                if (own && D[g][t] > tr.v) {
                                    tr.v = D[g][t];
                                    tr.pos = i * n + col + t;
                                }
                            }
                        }
                    }
                }
            }
        };
        uint64_t rx0[NGMAX], rx1[NGMAX];
        int32_t rc0[NGMAX], rc1[NGMAX];
        load_row(0, rx0, rc0);
        for (int rr = 0; rr < rc; rr += 2) {
            load_row(rr + 1 < rc ? rr + 1 : rr, rx1, rc1);
            row(rr, rx0, rc0);
            if (rr + 1 >= rc) break;
            load_row(rr + 2 < rc ? rr + 2 : rr + 1, rx0, rc0);
            row(rr + 1, rx1, rc1);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
}

// ----------------------------------------------------------------------------------------------
// Serial evaluation by one wave over the whole matrix, per-column state in global scratch
// (2 * n int32).  Used only when the square is too large for the windowed passes.  Lane l
// handles bit l of each word; words are visited left to right, carrying the row run and the
// previous-row dp of the last column across words in uniform registers.
// ----------------------------------------------------------------------------------------------
template <bool STORE>
__device__ void serial_dp(const uint64_t *__restrict__ bits, int64_t m, int64_t n, int64_t ldw,
                          int32_t *__restrict__ dp, int64_t ld_dp, int32_t *__restrict__ stH,
                          int32_t *__restrict__ stD, Track &tr) {
    const int lane = __lane_id();
    m = uniform(m);
    n = uniform(n);
    ldw = uniform(ldw);
    const int64_t nwords = (n + 63) >> 6;
    const uint64_t lastmask = last_word_mask(n);
    for (int64_t c = lane; c < nwords * 64; c += WAVE) {
        stH[c] = 0;
        stD[c] = 0;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    constexpr int UNROLL = 8;
    for (int64_t i = 0; i < m; ++i) {
        const uint64_t *__restrict__ row = bits + i * ldw;
        int32_t wcarry = 0, dleft_old = 0;
        for (int64_t k0 = 0; k0 < nwords; k0 += UNROLL) {
            int32_t h0[UNROLL], d0[UNROLL];
            uint64_t v[UNROLL];
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                const int64_t k = k0 + u < nwords ? k0 + u : nwords - 1;  // clamped: loads batch
                const uint64_t raw = row[k];
                v[u] = (k0 + u < nwords) ? ((k == nwords - 1) ? (raw & lastmask) : raw) : 0ull;
                const int64_t c = k * 64 + lane;
                h0[u] = stH[c];
                d0[u] = stD[c];
            }
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                const int64_t k = k0 + u;
                if (k >= nwords) break;
                const int64_t c = k * 64 + lane;
                const uint64_t x = v[u];
                const int32_t a = (int32_t)((x >> lane) & 1u);
                const int32_t lo = (int32_t)__clzll(~(x << (63 - lane)));
                const int32_t w = a ? ((lo == lane + 1) ? lane + 1 + wcarry : lo) : 0;
                const int32_t h = a ? h0[u] + 1 : 0;
                int32_t dprev = __shfl_up(d0[u], 1);
                if (lane == 0) dprev = dleft_old;
                dleft_old = __shfl(d0[u], WAVE - 1);
                int32_t d = h < w ? h : w;
                d = d < dprev + 1 ? d : dprev + 1;
                if (!a) d = 0;
                stH[c] = h;
                stD[c] = d;
                if (c < n) {
                    if (STORE) dp[i * ld_dp + c] = d;
                    if (d > tr.v) {
                        tr.v = d;
                        tr.pos = i * n + c;
                    }
                }
                wcarry = (x == ~0ull) ? wcarry + 64 : leading_ones(x);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    }
}

// ----------------------------------------------------------------------------------------------
// Erosion tile: 64 lanes = NWT word columns x NRG = 64 / NWT row groups; lane (rg, wl) holds RPL
// consecutive rows of word wl.  Word column 0 is the left halo (its results are not owned); the
// first KC - 1 rows of row group 0 are the top halo.  With that halo every E_k with k <= KC is
// exact on the owned cells.  NWT = 16 is the wide tile (15 owned words, 64 / 128 rows); NWT = 4
// suits matrices a few words wide (3 owned words, 16 row groups).
// ----------------------------------------------------------------------------------------------
template <int RPL_, int KC_, int NWT_ = 16>
struct TileShape {
    static constexpr int RPL = RPL_;
    static constexpr int KC = KC_;
    static constexpr int NWT = NWT_;
    static constexpr int NRG = WAVE / NWT;
    static constexpr int ROWS = NRG * RPL;
    static constexpr int HALO = KC - 1;
    static constexpr int TR = ROWS - HALO;  // owned rows per tile
    static constexpr int OWN_WORDS = NWT - 1;
    static constexpr int HALO_RG = HALO / RPL;  // the row group where the owned rows start
    static constexpr int HALO_R = HALO % RPL;   // and their first row in it
    static_assert(NWT == 4 || NWT == 8 || NWT == 16, "word columns per row group");
    static_assert(HALO < ROWS / 2, "owned rows are most of the tile");
    static_assert(KC <= 64 && (KC & (KC - 1)) == 0, "KC power of two <= 64");
};

// Within each group of NWT lanes, lane l receives lane l-1's value; the first lane of every
// group receives 0 (DPP row_shr:1, whose bound control zeroes the first lane of each 16-lane
// row; narrower groups also clear their own first lane).
template <int NWT>
__device__ __forceinline__ uint32_t from_left_in_group(uint32_t v, int wl) {
    const uint32_t x = from_left_in_row16(v);
    if constexpr (NWT == 16) return x;
    else return wl ? x : 0u;
}

template <int RPL, int D, int NWT>
__device__ __forceinline__ void erode(const uint64_t (&E)[RPL], uint64_t (&T)[RPL], int rg,
                                      int wl) {
    static_assert(D >= 1 && D <= 16 && D <= RPL, "shift");
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        uint64_t up;
        if (r >= D) {
            up = E[r - D];
        } else {
            const uint64_t v = __shfl_up(E[RPL - D + r], NWT);
            up = rg ? v : 0ull;
        }
        T[r] = E[r] & up;
    }
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const uint64_t f = T[r];
        const uint32_t lh = from_left_in_group<NWT>((uint32_t)(f >> 32), wl);
        T[r] = f & ((f << D) | (uint64_t)(lh >> (32 - D)));
    }
}

template <int RPL, int NWT>
__device__ __forceinline__ void erode_by(const uint64_t (&E)[RPL], uint64_t (&T)[RPL], int d,
                                         int rg, int wl) {
    switch (d) {
    case 1: erode<RPL, 1, NWT>(E, T, rg, wl); break;
    case 2: erode<RPL, 2, NWT>(E, T, rg, wl); break;
    case 4: erode<RPL, 4, NWT>(E, T, rg, wl); break;
    case 8: erode<RPL, 8, NWT>(E, T, rg, wl); break;
    default:
        if constexpr (RPL >= 16) erode<RPL, 16, NWT>(E, T, rg, wl);
        break;
    }
}

// Owned rows: every row of the row groups past HALO_RG, and rows >= HALO_R of group HALO_RG.
template <class TS>
__device__ __forceinline__ bool any_owned(const uint64_t (&T)[TS::RPL], int rg, bool lane_ok) {
    uint64_t a = 0, h = 0;
#pragma unroll
    for (int r = 0; r < TS::RPL; ++r) {
        if (r < TS::HALO_R) h |= T[r];
        else a |= T[r];
    }
    const uint64_t acc = rg > TS::HALO_RG ? (a | h) : (rg == TS::HALO_RG ? a : 0ull);
    return __ballot(lane_ok && acc != 0) != 0;
}

// The deep rows of a tile: owned rows at least KC below its first owned row, i.e. register rows
// >= 2 KC - 1.  Erosion inside the register tile treats what lies above it as zero, so a row
// there is exact for every side up to 2 KC (2 KC - 1 rows above it are in the tile, and an
// owned word has a whole word to its left).
template <class TS>
struct DeepRows {
    static constexpr int FIRST = 2 * TS::KC - 1;
    static constexpr int RG = FIRST / TS::RPL;  // the row group where they start
    static constexpr int R = FIRST % TS::RPL;   // and the row there
    static_assert(FIRST < TS::ROWS, "deep rows inside the register tile");
};

// any_owned over the owned cells (deep = false) or over the deep rows only.
template <class TS>
__device__ __forceinline__ bool any_in(const uint64_t (&T)[TS::RPL], int rg, bool lane_ok,
                                       bool deep) {
    using DR = DeepRows<TS>;
    uint64_t a = 0, h = 0, t = 0;
#pragma unroll
    for (int r = 0; r < TS::RPL; ++r) {
        if (r < TS::HALO_R) h |= T[r];
        else a |= T[r];
        if constexpr (DR::R != TS::HALO_R) {
            if (r >= DR::R) t |= T[r];
        }
    }
    if constexpr (DR::R == TS::HALO_R) t = a;
    // every row of the lane past row group thr counts, and in group thr the rows from the split
    const int thr = deep ? DR::RG : TS::HALO_RG;
    const uint64_t acc = rg > thr ? (a | h) : (rg == thr ? (deep ? t : a) : 0ull);
    return __ballot(lane_ok && acc != 0) != 0;
}

// Where the outcome of one tile goes.
struct TileSink {
    unsigned long long *key;   // atomicMax target: (side, first position) of the best square
};

// Per-tile outcome of the probe for the tiles a wave visits (tile t0 + k * stride, k < 64):
// the saturation byte (read by the resolve pass) and, when `bounds` is set, an upper bound on
// the tile's largest side (read by the dp map; negative for a saturated tile until the resolve
// pass records its bound).  Written with one store per array per 64 tiles: a store per tile
// would make the next tile's loads wait for it.
//
// Saturated tiles come in two kinds.  SAT_FULL: the resolve pass finishes every owned row.
// SAT_TOP: the probe finished the deep rows exactly, and the resolve pass finishes the first KC
// owned rows only.  tile_search returns SAT_BOUND for the first kind and top_code(b) for the
// second, b being the deep rows' largest side (0 when it is below KC, where the first rows,
// which reach KC, decide).  The saturation byte is 0 (not saturated), SAT_FULL or SAT_TOP; the
// bounds array holds the code until the resolve pass replaces it with the tile's bound.
constexpr int32_t SAT_BOUND = -1;
constexpr uint8_t SAT_FULL = 1, SAT_TOP = 2;
__host__ __device__ __forceinline__ int32_t top_code(int32_t b) { return -2 - b; }
// The deep rows' side kept in a bounds entry (0 unless the entry is a top_code).
__host__ __device__ __forceinline__ int32_t deep_side(int32_t code) {
    return code < -1 ? -2 - code : 0;
}
// The saturation byte of a probe return.
__host__ __device__ __forceinline__ uint8_t sat_byte(int32_t code) {
    return code >= 0 ? 0 : (code == SAT_BOUND ? SAT_FULL : SAT_TOP);
}
// Largest side the dp map's narrow pass (512-column windows) covers.
constexpr int32_t MAP_NARROW_REACH = 448;
// When a square exceeds that reach, the map is split by tile: tiles bounded by REGION_SMALL are
// mapped by the narrow pass with a REGION_SMALL halo, the others by the block-wide pass.
constexpr int32_t REGION_SMALL = 64;

// Encoding of a tile row or column as the low corner of a bounding box kept with atomicMax.
constexpr uint32_t BOX_LOW = 1u << 30;

struct SatBatch {
    uint8_t *base;
    int32_t *bounds = nullptr;
    bool want_box = false;     // with bounds: keep the box of tiles bounded above REGION_SMALL
    int64_t ntx = 1;           // tiles per tile row (for the box)
    uint32_t box[4] = {0, 0, 0, 0};  // the wave's box so far (wave-uniform; BOX_LOW encoding)
    int64_t t0 = 0, stride = 1;
    int count = 0, nsat = 0;
    int32_t mine = 0;  // lane k: the probe's return for the k-th collected tile
    __device__ void add(int64_t t, int32_t bound) {
        const int32_t bu = uniform(bound);   // wave-uniform: keep the state in SGPRs
        if (count == 0) t0 = uniform(t);
        nsat += bu < 0 ? 1 : 0;
        if (__lane_id() == count) mine = bu;
        if (++count == 64) flush();
    }
    __device__ void flush() {
        const int lane = __lane_id();
        if (lane < count) {
            base[t0 + lane * stride] = sat_byte(mine);
            if (bounds) bounds[t0 + lane * stride] = mine;
        }
        const bool big = want_box && lane < count && (mine < 0 || mine > REGION_SMALL);
        if (want_box && __ballot(big)) {
            const int64_t t = t0 + lane * stride;
            const int64_t ty = t / ntx, tx = t - ty * ntx;
            const uint32_t e[4] = {
                (uint32_t)wave_max_i32(big ? (int32_t)(BOX_LOW - (uint32_t)ty) : 0),
                (uint32_t)wave_max_i32(big ? (int32_t)(ty + 1) : 0),
                (uint32_t)wave_max_i32(big ? (int32_t)(BOX_LOW - (uint32_t)tx) : 0),
                (uint32_t)wave_max_i32(big ? (int32_t)(tx + 1) : 0)};
#pragma unroll
            for (int k = 0; k < 4; ++k) box[k] = e[k] > box[k] ? e[k] : box[k];
        }
        count = 0;
    }
};

// Search one tile: the largest k <= KC with an owned k x k all-ones square (exact), pushed as a
// key with the first owned cell of E_k.  Returns an upper bound on the tile's largest side (exact
// unless the search stopped early because the tile could not reach the best side so far), or a
// negative code when E_KC is non-empty among the owned cells ("saturated": the resolve pass
// finishes such a tile).  A saturated tile goes on eroding inside its register tile, over its
// deep rows only (exact there up to 2 KC): when they hold no E_2KC cell, their largest side and
// its first cell are exact and pushed, and the tile is of kind SAT_TOP; otherwise it is SAT_FULL
// and pushes (2 KC, the first deep cell of E_2KC), a real square.  Either push is later beaten
// or matched by the exact pass over the remaining rows when those hold a larger side or the same
// side earlier (the key keeps the larger side, then the smaller position).
// With DEEP = false a saturated tile is always SAT_FULL and pushes a lower bound instead: the
// largest k whose erosion, continued inside the register tile past its halo, still holds an
// owned cell (a subset of the true E_k: a real square).
template <class TS, bool DEEP = (4 * TS::KC <= TS::ROWS)>
__device__ __forceinline__ int32_t tile_search(const uint64_t *__restrict__ bits, int64_t m, int64_t n, int64_t ldw,
                            int64_t ty, int64_t tx, const TileSink &sink) {
    constexpr int RPL = TS::RPL;
    m = uniform(m);
    n = uniform(n);
    ldw = uniform(ldw);
    ty = uniform(ty);
    tx = uniform(tx);
    const int lane = __lane_id();
    const int wl = lane % TS::NWT, rg = lane / TS::NWT;
    const int64_t nwords = (n + 63) >> 6;
    const int64_t tile_r0 = ty * TS::TR - TS::HALO;
    const int64_t wlane = tx * TS::OWN_WORDS - 1 + wl;
    const bool wvalid = wlane >= 0 && wlane < nwords;
    const uint64_t wmask = (wlane == nwords - 1) ? last_word_mask(n) : ~0ull;
    uint64_t E[RPL], T[RPL];
    // all loads from clamped (in-bounds) addresses first, so they are in flight together; the
    // rows and words outside the matrix are zeroed afterwards
    const int64_t wl_c = wlane < 0 ? 0 : (wlane < nwords ? wlane : nwords - 1);
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int64_t row = tile_r0 + rg * RPL + r;
        const int64_t row_c = row < 0 ? 0 : (row < m ? row : m - 1);
        E[r] = bits[row_c * ldw + wl_c];
    }
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int64_t row = tile_r0 + rg * RPL + r;
        E[r] = (wvalid && row >= 0 && row < m) ? (E[r] & wmask) : 0ull;
    }
    const bool lane_ok = wl != 0 && wvalid;
    // best side found so far by any tile (read now so the load overlaps the erosion steps)
    const int64_t best = key_side(load_relaxed(sink.key));
    if (!any_owned<TS>(E, rg, lane_ok)) return 0;

    // Two loops, two erosion call sites (each inlines the erosion bodies, and the register tile
    // leaves little room).  E holds E_cur; a step tries E_{cur + d} with d <= cur.
    //  * Growing: d = cur (doubling) up to KC; a tile reaching KC is saturated and goes on over
    //    its deep rows by DSTEP rows a step, up to 2 KC.
    //  * Halving: d = (last step) / 2 down to 1.  Unsaturated tiles stop as soon as their bracket
    //    cannot reach the best side published so far.
    constexpr int DMAX = TS::RPL < 16 ? TS::RPL : 16;
    constexpr int DSTEP = DMAX < TS::KC ? DMAX : TS::KC;  // divides KC: the steps end at 2 KC
    constexpr int DEEP_MAX = 2 * TS::KC;
    int cur = 1, dl = 1;  // dl: the last step tried
    bool saturated = false;
    for (;;) {
        // doubling, at most DMAX rows a step (a step of d reads d rows up, within one row group)
        const int d = cur < TS::KC ? (cur < DMAX ? cur : DMAX) : (DEEP ? DSTEP : DMAX);
        dl = d;
        if (DEEP ? (saturated && cur + d > DEEP_MAX) : (saturated && cur + DMAX > TS::ROWS)) break;
        erode_by<RPL, TS::NWT>(E, T, d, rg, wl);
        if (DEEP ? !any_in<TS>(T, rg, lane_ok, saturated) : !any_owned<TS>(T, rg, lane_ok)) break;
#pragma unroll
        for (int r = 0; r < RPL; ++r) E[r] = T[r];
        cur += d;
        if (!saturated && cur >= TS::KC) {
            saturated = true;
            // no deep row reaches KC: the first KC owned rows, which do, decide the tile
            if (DEEP && !any_in<TS>(E, rg, lane_ok, true)) return top_code(0);
        }
    }
    const bool full = saturated && (!DEEP || cur >= DEEP_MAX);
    // the side (over the deep rows when saturated) is in [cur, cur + dl - 1] (unsaturated), in
    // [cur, cur + DSTEP - 1] (saturated), or at least 2 KC (full)
    if (!saturated && cur + dl - 1 < best) return cur + dl - 1;
    const int d0 = DEEP ? (full ? 0 : DSTEP >> 1) : DMAX >> 1;
    for (int d = saturated ? d0 : dl >> 1; d >= 1; d >>= 1) {
        erode_by<RPL, TS::NWT>(E, T, d, rg, wl);
        if (DEEP ? any_in<TS>(T, rg, lane_ok, saturated) : any_owned<TS>(T, rg, lane_ok)) {
#pragma unroll
            for (int r = 0; r < RPL; ++r) E[r] = T[r];
            cur += d;
        }
        if (!saturated && cur + d - 1 < best) return cur + d - 1;
    }
    const int32_t ret = saturated ? (full ? SAT_BOUND : top_code(cur)) : cur;
    if (DEEP ? cur < best : !saturated && cur < best) return ret;
    // first owned (saturated: deep) cell of E_cur in row-major order
    int64_t pos = INT64_MAX;
    if (lane_ok) {
#pragma unroll
        for (int r = RPL - 1; r >= 0; --r) {
            using DR = DeepRows<TS>;
            const bool take = DEEP && saturated
                                  ? (rg > DR::RG || (r >= DR::R && rg == DR::RG))
                                  : (rg > TS::HALO_RG || (r >= TS::HALO_R && rg == TS::HALO_RG));
            const int64_t row = tile_r0 + rg * RPL + r;
            if (take && E[r]) pos = row * n + wlane * 64 + (__ffsll((long long)E[r]) - 1);
        }
    }
    pos = wave_min_i64(pos);
    if (lane == 0) atomicMax(sink.key, make_key(cur, pos));
    return ret;
}

// ----------------------------------------------------------------------------------------------
// resolve_tile: the exact largest side and first corner of a saturated tile, computed with the
// paper's frequency array instead of a dp halo.
//
// Bound.  A square of side s >= KC whose bottom-right cell (i, j) lies in the tile puts an E_KC
// cell at (i', j) for every i - s + KC <= i' <= i and at (i, j') for every j - s + KC <= j' <= j,
// so every tile holding one of them is saturated:
//     s <= U = min(Vrun * TR, Hrun * 64 * OWN_WORDS) + KC - 1,
// with Vrun / Hrun the runs of consecutive saturated tiles ending at this one in its tile column
// and tile row.
//
// Search.  H (run of ones ending at each cell down its column, the paper's freq) is built at the
// row above the tile by scanning at most U rows upwards (U is the bound above when one pass can
// hold it, else it doubles from twice the best side so far until the tile's result is below U
// or U reaches the bound), over the tile's columns
// and the U columns to their left, and kept bit-sliced: plane p holds bit p of H for the 64 columns of a
// lane's word.  A cell has dp >= k iff the k columns ending at it all have H >= k (the side map
// in its rows-independent form), i.e. iff the horizontal erosion by k of the mask (H >= k) holds
// it.  As in Algorithm 1 the best side over the rows seen so far grows by at most one per row
// (dp[i][j] <= dp[i-1][j] + 1), so the tile's first row gets a gallop-and-bisect search over k
// and each later row a single test of k = best + 1.  The first row reaching the final best, and
// its first column there, give the tile's first corner in row-major order.
//
// Rows.  A SAT_TOP tile's deep rows were finished exactly by the probe (their side and first
// cell are in the key already), so the pass covers its first KC owned rows only; the tile's
// bound is the larger of the two parts.
// ----------------------------------------------------------------------------------------------
constexpr int HB = 12;  // bit planes of H: heights up to 4095 (U + TR stays below)

__device__ __forceinline__ void planes_inc_masked(uint64_t (&P)[HB], uint64_t c) {
#pragma unroll
    for (int p = 0; p < HB; ++p) {
        const uint64_t t = P[p] & c;
        P[p] ^= c;
        c = t;
    }
}

// Mask of the columns whose H >= k (k wave-uniform).
__device__ __forceinline__ uint64_t planes_ge(const uint64_t (&P)[HB], int32_t k) {
    uint64_t gt = 0, eq = ~0ull;
#pragma unroll
    for (int p = HB - 1; p >= 0; --p) {
        if ((k >> p) & 1) {
            eq &= P[p];
        } else {
            gt |= eq & P[p];
            eq &= ~P[p];
        }
    }
    return gt | eq;
}

// Lane l receives lane l-1's 64-bit value, lane 0 receives 0 (two DPP moves).
__device__ __forceinline__ uint64_t from_left_lane64(uint64_t v) {
    const uint32_t lo = (uint32_t)from_left_lane((int32_t)(uint32_t)v, 0);
    const uint32_t hi = (uint32_t)from_left_lane((int32_t)(uint32_t)(v >> 32), 0);
    return ((uint64_t)hi << 32) | lo;
}

// A row bitmask held one word per lane (lane l: word w0 + l).  Bit j of the result is bit j - t
// of v's row; columns left of the window read 0.  Word offsets 0 and 1 (t < 128) move through
// DPP; larger ones through a lane permute.
__device__ __forceinline__ uint64_t row_from_left(uint64_t v, int32_t t, int lane) {
    const int q = t >> 6, r = t & 63;
    uint64_t a, b;
    if (q == 0) {
        a = v;
        b = from_left_lane64(v);
    } else if (q == 1) {
        a = from_left_lane64(v);
        b = from_left_lane64(a);
    } else {
        const uint64_t pa = __shfl(v, lane - q);
        const uint64_t pb = __shfl(v, lane - q - 1);
        a = lane - q >= 0 ? pa : 0ull;
        b = lane - q - 1 >= 0 ? pb : 0ull;
    }
    return r ? ((a << r) | (b >> (64 - r))) : a;
}

// Bit j set iff bits j - k + 1 .. j of v's row are all set.
//  * k <= 64: log-doubling shift-AND; every shift is below 128 columns, so through DPP.
//  * k > 64: a run of ones that long ending at bit j of a word covers all of the word's bits up
//    to j (a run inside one word is at most 64 long), so only bits below the word's first zero
//    qualify, each with the run j + 1 + e, e being the run entering the word from the left.
//    e comes from the nearest lane to the left whose word has a zero: the ones at its top plus
//    64 per full word between.  One ballot and one lane read instead of about log2(k) shifts,
//    most of them lane permutes.
__device__ __forceinline__ uint64_t row_erode(uint64_t v, int32_t k, int lane) {
    if (k > 64) {
        const bool full = v == ~0ull;
        const uint64_t nonfull = __ballot(!full);
        const int32_t top = full ? 64 : (int32_t)__clzll(~v);  // ones at the word's top
        const uint64_t left = lane ? nonfull & (~0ull >> (64 - lane)) : 0ull;
        const int p = left ? 63 - (int)__clzll(left) : -1;      // nearest such lane to the left
        const int32_t top_p = __shfl(top, p < 0 ? 0 : p);
        const int32_t enter = p < 0 ? 64 * lane : top_p + 64 * (lane - 1 - p);
        const int32_t t = full ? 64 : __ffsll((long long)~v) - 1;  // ones at the word's bottom
        const int32_t lo = k - 1 - enter;  // the first bit whose run reaches k
        if (lo >= t) return 0ull;
        const uint64_t below_t = t == 64 ? ~0ull : ((1ull << t) - 1);
        return lo <= 0 ? below_t : below_t & ~((1ull << lo) - 1);
    }
    int32_t a = 1;
    while (2 * a <= k) {
        v &= row_from_left(v, a, lane);
        a <<= 1;
    }
    if (k > a) v &= row_from_left(v, k - a, lane);
    return v;
}

// Does an owned cell of the current row have dp >= k?  If so, *col = the first such column.
__device__ __forceinline__ bool row_test(const uint64_t (&P)[HB], int32_t k, uint64_t own,
                                         int lane, int64_t w0, int64_t *col) {
    const uint64_t y = row_erode(planes_ge(P, k), k, lane) & own;
    const uint64_t b = __ballot(y != 0);
    if (!b) return false;
    const int fl = __ffsll((long long)b) - 1;
    const uint64_t yf = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int32_t)(y >> 32), fl) << 32) |
                        (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)y, fl);
    *col = (w0 + fl) * 64 + (__ffsll((long long)yf) - 1);
    return true;
}

// The first row of a stretch of rows: the largest k <= kmax such that an owned cell of the
// row has dp >= k, searched upwards from g (the best side any tile had published): sides below
// g cannot change the result.  Returns g - 1 with *pos = -1 when no cell of the row reaches g
// (g >= 2); otherwise the row's largest side, with *pos = i * n + its first column.
__device__ __forceinline__ int32_t first_row_search(const uint64_t (&P)[HB], int32_t g,
                                                    int32_t kmax, uint64_t own, int lane,
                                                    int64_t w0, int64_t i, int64_t n,
                                                    int64_t *pos) {
    // one search loop, one row_test call site: gallop from g - 1 (treated as reached) by steps
    // of 1, 2, 4, ..., then bisect between the last success lo and the first failure hi
    int32_t lo = g >= 2 ? g - 1 : 0, hi = kmax + 1, step = 1;
    bool gallop = true;
    *pos = -1;
    while (hi - lo > 1) {
        int32_t k = gallop ? lo + step : (lo + hi) >> 1;
        k = k < hi ? k : hi - 1;
        int64_t col = 0;
        if (row_test(P, k, own, lane, w0, &col)) {
            lo = k;
            *pos = i * n + col;
            step <<= 1;
        } else {
            hi = k;
            gallop = false;
        }
    }
    return lo;
}

// Consecutive set saturation bytes at idx0, idx0 - step, idx0 - 2 step, ... (idx0 - k step >= 0
// while k < limit), 64 per round.
__device__ __forceinline__ int64_t sat_run(const uint8_t *__restrict__ sat, int64_t idx0,
                                           int64_t step, int64_t limit, int lane) {
    int64_t run = 0;
    for (;;) {
        const int64_t k = run + lane;
        const bool s = k < limit && sat[idx0 - k * step] != 0;
        const uint64_t b = __ballot(s);
        const int c = (~b) ? __ffsll((long long)~b) - 1 : 64;
        run += c;
        if (c < 64) return run;
    }
}

// One pass over rows [ra, rb) of the tiles in tile columns txa..txb (one tile row) with heights
// clamped at depth U and a window of U columns to the left of them: *best / *bpos receive the
// rows' largest computed side and its first cell.  A
// true side s >= U still computes as >= U (clamping and clipping cannot push a value below U),
// so a result below U is exact.  Returns false if the window exceeds one word per lane.
template <class TS>
__device__ bool resolve_pass(const uint64_t *__restrict__ bits, int64_t m, int64_t n,
                             int64_t ldw, int64_t ra, int64_t rb, int64_t txa, int64_t txb,
                             int64_t U, int32_t g, int32_t *best_out, int64_t *bpos_out) {
    constexpr int64_t OWN_COLS = 64 * TS::OWN_WORDS;
    const int lane = __lane_id();
    const int64_t xa = txa * OWN_COLS;
    const int64_t xb = (txb + 1) * OWN_COLS < n ? (txb + 1) * OWN_COLS : n;
    const int64_t nwords = (n + 63) >> 6;
    const int64_t w0 = xa - U > 0 ? ((xa - U) >> 6) : 0;
    const int64_t w1 = (xb + 63) >> 6;
    if (w1 - w0 > WAVE || U + TS::TR + 1 >= (1 << HB)) return false;  // heights and tested k fit
    const int64_t wl = w0 + lane;
    const bool valid = wl < w1;
    const int64_t wl_c = valid ? wl : w0;
    const uint64_t wmask = !valid ? 0ull : (wl == nwords - 1 ? last_word_mask(n) : ~0ull);
    uint64_t own = 0;
    if (valid) {
        const int64_t lo = (xa > wl * 64 ? xa : wl * 64) - wl * 64;
        const int64_t hi = (xb < wl * 64 + 64 ? xb : wl * 64 + 64) - wl * 64;
        if (hi > lo) own = (hi - lo == 64 ? ~0ull : ((1ull << (hi - lo)) - 1)) << lo;
    }
    // heights at row ra - 1, at most U rows deep
    uint64_t P[HB];
#pragma unroll
    for (int p = 0; p < HB; ++p) P[p] = 0;
    uint64_t acc = valid ? ~0ull : 0ull;
    const int64_t rstop = ra - U > 0 ? ra - U : 0;
    constexpr int FB = 16;  // rows loaded per round (all in flight together)
    // the next round's rows are loaded while this round's are counted (a long scan, as above a
    // large square, is otherwise one load latency per round)
    uint64_t nv[FB];
#pragma unroll
    for (int u = 0; u < FB; ++u) {
        const int64_t r = ra - 1 - u >= rstop ? ra - 1 - u : rstop;  // clamped: the loads batch
        nv[u] = rstop <= ra - 1 ? bits[r * ldw + wl_c] : 0ull;
    }
    for (int64_t r0 = ra - 1; r0 >= rstop; r0 -= FB) {
        uint64_t v[FB];
#pragma unroll
        for (int u = 0; u < FB; ++u) v[u] = nv[u];
        if (r0 - FB >= rstop) {
#pragma unroll
            for (int u = 0; u < FB; ++u) {
                const int64_t r = r0 - FB - u >= rstop ? r0 - FB - u : rstop;
                nv[u] = bits[r * ldw + wl_c];
            }
        }
        for (int u = 0; u < FB; ++u) {  // stops at the scan's top: not unrolled
            if (r0 - u < rstop) break;
            acc &= v[u] & wmask;
            planes_inc_masked(P, acc);
        }
        if (!__ballot(acc != 0)) break;
    }
    // the tile's rows, FB at a time
    int32_t best = 0;
    int64_t bpos = -1;
    for (int64_t i0 = ra; i0 < rb; i0 += FB) {
        uint64_t v[FB];
#pragma unroll
        for (int u = 0; u < FB; ++u) {
            const int64_t r = i0 + u < rb ? i0 + u : rb - 1;
            v[u] = bits[r * ldw + wl_c];
        }
        for (int u = 0; u < FB; ++u) {
            const int64_t i = i0 + u;
            if (i >= rb) break;
            const uint64_t x = v[u] & wmask;
            planes_inc_masked(P, ~0ull);
#pragma unroll
            for (int p = 0; p < HB; ++p) P[p] &= x;
            int64_t col = 0;
            if (i == ra) {
                best = first_row_search(P, g, (int32_t)(U + TS::TR), own, lane, w0, i, n, &bpos);
            } else if (row_test(P, best + 1, own, lane, w0, &col)) {
                ++best;
                bpos = i * n + col;
            }
        }
    }
    *best_out = best;
    *bpos_out = bpos;
    return true;
}

// Records the tile's bound when the caller keeps bounds: the largest over the parts of the tile
// and, for a SAT_TOP tile, its deep rows (the probe left SAT_BOUND or a top_code there).
__device__ __forceinline__ void note_bound(int32_t *bounds, int64_t t, int64_t bound) {
    if (bounds && __lane_id() == 0) {
        const int32_t deep = deep_side(bounds[t]);
        atomicMax(&bounds[t], (int32_t)(bound > deep ? bound : deep));
    }
}

// The rows of a saturated tile left to the resolve pass: its first KC owned rows for a SAT_TOP
// tile (the probe finished the rest), all TR otherwise.
template <class TS>
__device__ __forceinline__ int64_t resolve_rows(uint8_t sb) {
    return sb == SAT_TOP ? TS::KC : TS::TR;
}

// The bound U of a saturated tile from the runs of saturated tiles (see above), at most
// min(m, n).
template <class TS>
__device__ __forceinline__ int64_t resolve_bound(const uint8_t *__restrict__ sat, int64_t ty,
                                                 int64_t tx, int64_t ntx, int64_t mn, int lane) {
    constexpr int64_t OWN_COLS = 64 * TS::OWN_WORDS;
    const int64_t t = ty * ntx + tx;
    const int64_t vrun = uniform(sat_run(sat, t, ntx, ty + 1, lane));
    const int64_t hrun = uniform(sat_run(sat, t, 1, tx + 1, lane));
    const int64_t u =
        (vrun * TS::TR < hrun * OWN_COLS ? vrun * TS::TR : hrun * OWN_COLS) + TS::KC - 1;
    return u < mn ? u : mn;
}

// Finishes rows [ra + part * ceil(TR / nparts), ...) of a saturated tile: the tile's rows split
// into nparts parts handled by different waves, each exact for its rows.
template <class TS>
__device__ void resolve_tile(const uint64_t *__restrict__ bits, int64_t m, int64_t n,
                             int64_t ldw, int64_t ty, int64_t tx, int64_t ntx,
                             const uint8_t *__restrict__ sat, unsigned long long *key,
                             uint32_t *serial_flag, int32_t *bounds = nullptr, int part = 0,
                             int nparts = 1, uint32_t *serial_count = nullptr) {
    constexpr int64_t OWN_COLS = 64 * TS::OWN_WORDS;
    const int lane = __lane_id();
    m = uniform(m);
    n = uniform(n);
    ldw = uniform(ldw);
    ty = uniform(ty);
    tx = uniform(tx);
    const int64_t rows = resolve_rows<TS>((uint8_t)uniform((int32_t)sat[ty * ntx + tx]));
    const int64_t prow = (rows + nparts - 1) / nparts;
    const int64_t ta = ty * TS::TR, tb = ta + rows < m ? ta + rows : m;
    const int64_t ra = ta + part * prow < tb ? ta + part * prow : tb;
    const int64_t rb = ra + prow < tb ? ra + prow : tb;
    if (ra >= rb) return;
    const int64_t ucap = resolve_bound<TS>(sat, ty, tx, ntx, m < n ? m : n, lane);
    const int64_t g = uniform(key_side(load_relaxed(key)));
    if (ucap < g) {  // cannot reach the best side found so far
        note_bound(bounds, ty * ntx + tx, ucap);
        return;
    }
    // one pass at the bound when its window fits (exact at once), else doubling from twice
    // the best side so far (the bound is loose where most tiles saturate)
    const int64_t w0cap = tx * OWN_COLS - ucap > 0 ? ((tx * OWN_COLS - ucap) >> 6) : 0;
    const int64_t w1cap = ((tx + 1) * OWN_COLS < n ? (tx + 1) * OWN_COLS + 63 : n + 63) >> 6;
    const bool cap_fits = w1cap - w0cap <= WAVE && ucap + TS::TR + 1 < (1 << HB);
    int64_t U = cap_fits ? ucap : 2 * (g > TS::KC ? g : TS::KC);
    for (;;) {
        U = U < ucap ? U : ucap;
        int32_t best = 0;
        int64_t bpos = -1;
        if (!resolve_pass<TS>(bits, m, n, ldw, ra, rb, tx, tx, U, (int32_t)g, &best, &bpos)) {
            // the serial pass finishes the matrix; serial_count counts the matrices so flagged
            if (lane == 0 && atomicOr(serial_flag, 1u) == 0u && serial_count)
                atomicAdd(serial_count, 1u);
            return;
        }
        best = uniform(best);
        if (best < U || U >= ucap) {
            if (lane == 0 && best > 0 && bpos >= 0) atomicMax(key, make_key(best, bpos));
            note_bound(bounds, ty * ntx + tx, best);
            return;
        }
        U = 2 * (int64_t)best;
    }
}

// Saturated tiles of one tile row handled together: the tiles in columns tx0..tx1 (some of them
// saturated) share one window and one height scan, and each row test covers all of them, so a
// blob image whose tiles nearly all saturate needs fewer waves' worth of row tests (all the
// groups then fit the device at once).  Each saturated tile's bound is computed as in resolve_tile; tiles that cannot reach the
// best side so far keep that bound and drop out.  The span's largest side is exact for every
// member (a member's true side is at most its bound, at most U once U reaches the span's bound)
// and becomes each member's recorded bound.  Returns the members (bit k: column tx0 + k) still to
// be resolved one at a time with resolve_tile: all of them where the span's window outgrows one
// word per lane, or the single one left; 0 when the group is done.
template <class TS>
__device__ uint32_t resolve_group(const uint64_t *__restrict__ bits, int64_t m, int64_t n,
                                  int64_t ldw, int64_t ty, int64_t tx0, int64_t tx1,
                                  int64_t ntx, const uint8_t *__restrict__ sat,
                                  unsigned long long *key, int32_t *bounds) {
    constexpr int64_t OWN_COLS = 64 * TS::OWN_WORDS;
    const int lane = __lane_id();
    m = uniform(m);
    n = uniform(n);
    ldw = uniform(ldw);
    ty = uniform(ty);
    tx0 = uniform(tx0);
    tx1 = uniform(tx1);
    const int64_t mn = m < n ? m : n;
    const int64_t g = uniform(key_side(load_relaxed(key)));
    // members still in the running (bit k), the largest of their bounds, and the rows the span
    // covers (every member's rows)
    uint32_t live = 0;
    int64_t lo = -1, hi = -1, ucap = 0, rows = 0;
    for (int64_t tx = tx0; tx <= tx1; ++tx) {
        const uint8_t sb = (uint8_t)uniform((int32_t)sat[ty * ntx + tx]);
        if (!sb) continue;
        const int64_t u = resolve_bound<TS>(sat, ty, tx, ntx, mn, lane);
        if (u < g) {  // cannot reach the best side found so far
            note_bound(bounds, ty * ntx + tx, u);
            continue;
        }
        live |= 1u << (tx - tx0);
        if (lo < 0) lo = tx;
        hi = tx;
        ucap = u > ucap ? u : ucap;
        rows = resolve_rows<TS>(sb) > rows ? resolve_rows<TS>(sb) : rows;
    }
    if (__popc(live) <= 1) return live;
    const int64_t ta = ty * TS::TR, tb = ta + rows < m ? ta + rows : m;
    const auto fits = [&](int64_t U) {
        const int64_t w0 = lo * OWN_COLS - U > 0 ? ((lo * OWN_COLS - U) >> 6) : 0;
        const int64_t w1 = ((hi + 1) * OWN_COLS < n ? (hi + 1) * OWN_COLS + 63 : n + 63) >> 6;
        return w1 - w0 <= WAVE && U + TS::TR + 1 < (1 << HB);
    };
    int64_t U = fits(ucap) ? ucap : 2 * (g > TS::KC ? g : TS::KC);
    for (;;) {
        U = U < ucap ? U : ucap;
        int32_t best = 0;
        int64_t bpos = -1;
        if (!fits(U) ||
            !resolve_pass<TS>(bits, m, n, ldw, ta, tb, lo, hi, U, (int32_t)g, &best, &bpos))
            return live;
        best = uniform(best);
        if (best < U || U >= ucap) {
            if (lane == 0 && best > 0 && bpos >= 0) atomicMax(key, make_key(best, bpos));
            for (uint32_t b = live; b; b &= b - 1)
                note_bound(bounds, ty * ntx + tx0 + (__ffs(b) - 1), best);
            return 0;
        }
        U = 2 * (int64_t)best;
    }
}

// ----------------------------------------------------------------------------------------------
// resolve_tile_block: a saturated tile finished by the NW waves of a block together.
//
// One wave alone spends most of a tile's time in chains of dependent steps (the upward height
// scan, then one row test after another), so here the block splits both.  The rows above the
// tile, [ta - U, ta), are cut into NW segments and the tile's own rows into NW parts, one of
// each per wave.  Each wave scans its segment and its part once, bottom to top, giving per
// column F (every row of the piece is one) and B (the run of ones ending at the piece's last
// row, bit-sliced like the heights).  Heights then flow down the pieces in order, top to
// bottom, through LDS: H after a piece is F ? H before + its length : B.  The wave owning
// part p takes the heights at the row above its part from that chain and runs the row tests
// of its rows only.  Every part is exact for its own rows (its heights are those of a scan
// starting U rows above the tile); the block's largest side decides, as in resolve_tile,
// whether U was deep enough.
//
// The first row of a part searches upward from g, the best side any tile had published when
// the block started: sides below g cannot change the result, so a part whose rows never reach
// g reports g - 1 as its bound and nothing to the key.  Later rows test best + 1 only (the
// running maximum grows by at most one per row).
// ----------------------------------------------------------------------------------------------
constexpr int RESOLVE_WAVES = 4;  // waves per block in k_resolve, one part of a tile each

struct ResolveLds {
    uint64_t H[HB][WAVE];        // heights at the bottom of the last piece folded in
    int32_t best[RESOLVE_WAVES];
    int64_t scal[2];             // the tile's bound and the best side, for the whole block
};

// Scan rows [sa, sb) of the lane's word upwards: F = columns that are one in every row,
// B = per column, the run of ones ending at row sb - 1 (clamped at the piece's length).
__device__ __forceinline__ void piece_scan(const uint64_t *__restrict__ bits, int64_t ldw,
                                           int64_t wl_c, uint64_t wmask, int64_t sa, int64_t sb,
                                           uint64_t &F, uint64_t (&B)[HB]) {
#pragma unroll
    for (int p = 0; p < HB; ++p) B[p] = 0;
    uint64_t acc = wmask;
    // row pointers are wave-uniform, the lane's word a 32-bit offset: no 64-bit address per load
    const uint32_t wo = (uint32_t)wl_c;
    constexpr int FB = 8;  // rows per round, the next round's loads issued before counting
    uint64_t nv[FB];
#pragma unroll
    for (int u = 0; u < FB; ++u) {
        const int64_t r = sb - 1 - u >= sa ? sb - 1 - u : sa;  // clamped: the loads batch
        nv[u] = sa < sb ? (bits + r * ldw)[wo] : 0ull;
    }
    for (int64_t r0 = sb - 1; r0 >= sa; r0 -= FB) {
        uint64_t v[FB];
#pragma unroll
        for (int u = 0; u < FB; ++u) v[u] = nv[u];
        if (r0 - FB >= sa) {
#pragma unroll
            for (int u = 0; u < FB; ++u) {
                const int64_t r = r0 - FB - u >= sa ? r0 - FB - u : sa;
                nv[u] = (bits + r * ldw)[wo];
            }
        }
        for (int u = 0; u < FB; ++u) {  // stops at the piece's top: not unrolled
            if (r0 - u < sa) break;
            acc &= v[u] & wmask;
            planes_inc_masked(B, acc);
        }
        if (!__ballot(acc != 0)) break;
    }
    F = acc;
}

// One step of the chain: H = the heights in LDS (zero for the first piece); LDS <- F ? H + len :
// B; on return B holds H (the heights above the piece).
__device__ __forceinline__ void chain_step(ResolveLds &L, int lane, bool has_prev, uint64_t F,
                                           uint64_t (&B)[HB], int64_t len) {
    uint64_t c = 0;
#pragma unroll
    for (int p = 0; p < HB; ++p) {
        const uint64_t a = has_prev ? L.H[p][lane] : 0ull;
        const uint64_t sum = (len >> p) & 1 ? ~(a ^ c) : (a ^ c);
        c = (len >> p) & 1 ? (a | c) : (a & c);
        L.H[p][lane] = (F & sum) | (~F & B[p]);
        B[p] = a;
    }
}

template <class TS, int NW>
__device__ void resolve_tile_block(const uint64_t *__restrict__ bits, int64_t m, int64_t n,
                                   int64_t ldw, int64_t ty, int64_t tx, int64_t ntx,
                                   const uint8_t *__restrict__ sat, unsigned long long *key,
                                   uint32_t *serial_flag, int32_t *bounds, ResolveLds &L,
                                   uint32_t *serial_count = nullptr) {
    constexpr int64_t OWN_COLS = 64 * TS::OWN_WORDS;
    const int lane = __lane_id();
    const int wv = uniform((int32_t)(threadIdx.x / WAVE));  // wave-uniform: keep it scalar
    m = uniform(m);
    n = uniform(n);
    ldw = uniform(ldw);
    ty = uniform(ty);
    tx = uniform(tx);
    const int64_t t = ty * ntx + tx;
    const int64_t rows = resolve_rows<TS>((uint8_t)uniform((int32_t)sat[t]));
    const int64_t ta = ty * TS::TR, tb = ta + rows < m ? ta + rows : m;
    const int64_t mn = m < n ? m : n;
    if (wv == 0) {
        const int64_t u = resolve_bound<TS>(sat, ty, tx, ntx, mn, lane);
        const int64_t g0 = uniform(key_side(load_relaxed(key)));
        if (lane == 0) {
            L.scal[0] = u;
            L.scal[1] = g0;
        }
    }
    __syncthreads();
    const int64_t ucap = uniform(L.scal[0]);
    const int64_t g = uniform(L.scal[1]);
    __syncthreads();  // the next tile rewrites scal
    if (ucap < g) {   // cannot reach the best side found so far
        if (wv == 0) note_bound(bounds, t, ucap);
        return;
    }
    const int64_t xa = tx * OWN_COLS, xb = (tx + 1) * OWN_COLS < n ? (tx + 1) * OWN_COLS : n;
    const auto fits = [&](int64_t U) {
        const int64_t w0 = xa - U > 0 ? ((xa - U) >> 6) : 0;
        return ((xb + 63) >> 6) - w0 <= WAVE && U + TS::TR + 1 < (1 << HB);
    };
    // one pass at the bound when its window fits (exact at once), else doubling from twice the
    // best side so far
    int64_t U = fits(ucap) ? ucap : 2 * (g > TS::KC ? g : TS::KC);
    const int64_t prow = (rows + NW - 1) / NW;
    const int64_t ra = uniform(ta + wv * prow < tb ? ta + wv * prow : tb);
    const int64_t rb = uniform(ra + prow < tb ? ra + prow : tb);
    const int64_t nwords = (n + 63) >> 6;
    for (;;) {
        U = U < ucap ? U : ucap;
        if (!fits(U)) {  // the serial pass finishes the matrix (serial_count: matrices flagged)
            if (wv == 0 && lane == 0 && atomicOr(serial_flag, 1u) == 0u && serial_count)
                atomicAdd(serial_count, 1u);
            return;
        }
        const int64_t w0 = xa - U > 0 ? ((xa - U) >> 6) : 0;
        const int64_t w1 = (xb + 63) >> 6;
        const int64_t wl = w0 + lane;
        const bool valid = wl < w1;
        const int64_t wl_c = valid ? wl : w0;
        const uint64_t wmask = !valid ? 0ull : (wl == nwords - 1 ? last_word_mask(n) : ~0ull);
        uint64_t own = 0;
        if (valid) {
            const int64_t lo = (xa > wl * 64 ? xa : wl * 64) - wl * 64;
            const int64_t hi = (xb < wl * 64 + 64 ? xb : wl * 64 + 64) - wl * 64;
            if (hi > lo) own = (hi - lo == 64 ? ~0ull : ((1ull << (hi - lo)) - 1)) << lo;
        }
        // this wave's segment above the tile and its part of the tile
        const int64_t rstop = ta - U > 0 ? ta - U : 0;
        const int64_t seg = (ta - rstop + NW - 1) / NW;
        const int64_t sa = uniform(rstop + wv * seg < ta ? rstop + wv * seg : ta);
        const int64_t sb = uniform(sa + seg < ta ? sa + seg : ta);
        // the chain: segments 0 .. NW-1, then parts 0 .. NW-1, each folded by its wave in turn
        // (a part is scanned only once the segments are folded, so the two scans' registers
        // are never live together)
        uint64_t F, P[HB];
        piece_scan(bits, ldw, wl_c, wmask, sa, sb, F, P);
        for (int s = 0; s < NW; ++s) {
            __syncthreads();
            if (s == wv) chain_step(L, lane, s > 0, F, P, sb - sa);
        }
        // then the part: P ends as the heights at row ra - 1, read from the chain before the
        // part is folded in
        piece_scan(bits, ldw, wl_c, wmask, ra, rb, F, P);
        for (int s = 0; s < NW; ++s) {
            __syncthreads();
            if (s == wv) chain_step(L, lane, true, F, P, rb - ra);
        }
        // the part's rows: the first searched upwards from g, the rest tested at best + 1
        const int32_t kmax = (int32_t)(U + TS::TR);
        int32_t best = 0;
        int64_t bpos = -1;
        constexpr int FB = 8;
        for (int64_t i0 = ra; i0 < rb; i0 += FB) {
            uint64_t v[FB];
#pragma unroll
            for (int u = 0; u < FB; ++u) {
                const int64_t r = i0 + u < rb ? i0 + u : rb - 1;
                v[u] = (bits + r * ldw)[(uint32_t)wl_c];
            }
            for (int u = 0; u < FB; ++u) {
                const int64_t i = i0 + u;
                if (i >= rb) break;
                const uint64_t x = v[u] & wmask;
                planes_inc_masked(P, ~0ull);
#pragma unroll
                for (int p = 0; p < HB; ++p) P[p] &= x;
                int64_t col = 0;
                if (i == ra) {
                    best = first_row_search(P, (int32_t)g, kmax, own, lane, w0, i, n, &bpos);
                } else if (row_test(P, best + 1, own, lane, w0, &col)) {
                    ++best;
                    bpos = i * n + col;
                }
            }
        }
        best = uniform(best);
        if (lane == 0) L.best[wv] = best;
        __syncthreads();
        int32_t bmax = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) bmax = L.best[w] > bmax ? L.best[w] : bmax;
        bmax = uniform(bmax);
        __syncthreads();  // L.best is rewritten by the next pass
        if (bmax < U || U >= ucap) {
            if (lane == 0 && best > 0 && bpos >= 0 && best >= g) atomicMax(key, make_key(best, bpos));
            if (wv == 0) note_bound(bounds, t, bmax);
            return;
        }
        U = 2 * (int64_t)bmax;
    }
}

// ----------------------------------------------------------------------------------------------
// dprun_block: the rows-parallel recurrence over a window of up to 8 groups of 256 columns shared
// by the 4 waves of a block (wave w owns groups 2w and 2w + 1), for squares too wide for a
// one-wave window.  The window's packed words and entering row runs are staged once per row
// chunk for the whole block; dp[i-1][j-1] crosses from wave w-1 to wave w through a
// double-buffered LDS slot written after each row, with one barrier per row.  Every loop trip
// count here is uniform over the block, so all waves meet every barrier.
// ----------------------------------------------------------------------------------------------
constexpr int BLK_WORDS = 2048;  // staged packed words per block (24 KB with the row runs)

struct BlockLds {
    uint64_t *x;     // BLK_WORDS packed words
    int32_t *c;      // BLK_WORDS entering row runs
    int32_t *slot;   // [2][4] last-column dp of each wave, by row parity
};

template <bool CLASSED>
__device__ void dprun_block(const uint64_t *__restrict__ bits, int64_t ldw, int64_t n,
                            int64_t rh, int64_t ra, int64_t rb, int64_t xh, int64_t xa,
                            int64_t xb, int ng, int32_t *__restrict__ dp, int64_t ld_dp,
                            bool vec_ok, BlockLds L, const StoreClass<2> &sc) {
    constexpr int CPL = 4, GW = 64 * CPL, LPW = 64 / CPL, GPW = 2, NTH = 256;
    rh = uniform(rh);
    ra = uniform(ra);
    rb = uniform(rb);
    xh = uniform(xh);
    xa = uniform(xa);
    xb = uniform(xb);
    ng = uniform(ng);
    ldw = uniform(ldw);
    n = uniform(n);
    ld_dp = uniform(ld_dp);
    const int tid = threadIdx.x;
    const int wv = tid / WAVE, lane = tid % WAVE;
    const int q = lane / LPW;
    const int b = (lane % LPW) * CPL;
    const uint64_t lowmask = (1ull << b) - 1;
    const int64_t nwords = (n + 63) >> 6;
    const uint64_t lastmask = last_word_mask(n);
    ng = ng < 1 ? 1 : (ng > 8 ? 8 : ng);  // 4..32 window words: every loop step below >= 1
    const int nww = ng * CPL;
    const int rc_max = BLK_WORDS / nww;
    const int fl_w = tid % nww, fl_r = tid / nww, fl_rpp = NTH / nww;
    const int64_t fl_word = (xh >> 6) + fl_w;
    const bool fl_ok = fl_r < fl_rpp && fl_word < nwords;
    const uint64_t fl_mask = (fl_word == nwords - 1) ? lastmask : ~0ull;
    const int64_t fl_wc = fl_word < nwords ? fl_word : nwords - 1;

    int32_t H[GPW][CPL], D[GPW][CPL];
#pragma unroll
    for (int g = 0; g < GPW; ++g)
#pragma unroll
        for (int t = 0; t < CPL; ++t) {
            H[g][t] = 0;
            D[g][t] = 0;
        }
    if (tid < 8) L.slot[tid] = 0;   // zero state left of every wave before the first row
    // tile row of the current row relative to ty0 and the row's offset in it (see dprun)
    int64_t kq = 0, kr = 0;
    if (CLASSED) {
        kq = uniform(rh / sc.tile_rows - sc.ty0);
        kr = uniform(rh % sc.tile_rows);
    }

    for (int64_t r0 = rh; r0 < rb; r0 += rc_max) {
        const int rc = (int)(rb - r0 < rc_max ? rb - r0 : rc_max);
        constexpr int FB = 8;
        for (int rb0 = fl_r; rb0 < rc; rb0 += FB * fl_rpp) {
            uint64_t v[FB];
#pragma unroll
            for (int u = 0; u < FB; ++u) {
                const int r = rb0 + u * fl_rpp;
                const int r_c = r < rc ? r : rc - 1;
                v[u] = bits[(r0 + r_c) * ldw + fl_wc];
            }
#pragma unroll
            for (int u = 0; u < FB; ++u) {
                const int r = rb0 + u * fl_rpp;
                if (r < rc && fl_r < fl_rpp) L.x[r * nww + fl_w] = fl_ok ? (v[u] & fl_mask) : 0ull;
            }
        }
        __syncthreads();
        for (int r = tid; r < rc; r += NTH) {
            int32_t run = 0;
            for (int w = 0; w < nww; ++w) {
                const uint64_t v = L.x[r * nww + w];
                L.c[r * nww + w] = run;
                run = (v == ~0ull) ? run + 64 : leading_ones(v);
            }
        }
        __syncthreads();
        for (int rr = 0; rr < rc; ++rr) {
            const int64_t i = r0 + rr;
            const bool own_row = i >= ra;
            const int par = (int)(i & 1);
            // previous-row dp just left of this wave's first group (from wave wv - 1)
            int32_t dleft_old = wv > 0 ? L.slot[par * 4 + wv - 1] : 0;
            const int krow = (CLASSED && own_row) ? (int)kq : 0;
            if (CLASSED && ++kr == sc.tile_rows) {
                kr = 0;
                ++kq;
            }
#pragma unroll
            for (int gl = 0; gl < GPW; ++gl) {
                const int g = wv * GPW + gl;
                if (g < ng) {
                    const uint64_t x = L.x[rr * nww + g * CPL + q];
                    const int32_t carry = L.c[rr * nww + g * CPL + q];
                    const int32_t wrun = run_into(x, lowmask, b, carry);
                    const uint32_t nib = (uint32_t)(x >> b) & ((1u << CPL) - 1u);
                    int32_t dprev = from_left_lane(D[gl][CPL - 1], dleft_old);
                    dleft_old = __builtin_amdgcn_readlane(D[gl][CPL - 1], WAVE - 1);
                    int32_t w = wrun;
#pragma unroll
                    for (int t = 0; t < CPL; ++t) {
                        const int32_t old = D[gl][t];
                        D[gl][t] = cell_step(H[gl][t], w, dprev, (nib >> t) & 1u);
                        dprev = old;
                    }
                    const int64_t col = xh + (int64_t)g * GW + (int64_t)lane * CPL;
                    if (own_row && (!CLASSED || ((sc.cls[gl] >> krow) & 1))) {
                        int32_t *p = dp + i * ld_dp + col;
                        if (col >= xa && col + CPL <= xb) {
                            if (vec_ok) {
                                *reinterpret_cast<int4 *>(p) =
                                    make_int4(D[gl][0], D[gl][1], D[gl][2], D[gl][3]);
                            } else {
#pragma unroll
                                for (int t = 0; t < CPL; ++t) p[t] = D[gl][t];
                            }
                        } else {
#pragma unroll
                            for (int t = 0; t < CPL; ++t)
                                if (col + t >= xa && col + t < xb) p[t] = D[gl][t];
                        }
                    }
                }
            }
            // this row's last-column dp of the wave, for wave wv + 1 at the next row
            if (lane == WAVE - 1) L.slot[(par ^ 1) * 4 + wv] = D[GPW - 1][CPL - 1];
            __syncthreads();
        }
    }
}

// ----------------------------------------------------------------------------------------------
// All maximal squares.  A cell is the bottom-right corner of a maximal square iff dp = S, and
// since S is the largest side, iff dp >= S: per row, the horizontal erosion by S of the mask of
// columns whose height is >= S (the frequency-array test of resolve_tile with k fixed at S).
// The matrix is walked in units of ALL_ROWS rows x ALL_WORDS words; a unit's heights start from
// a scan of at most S rows above it, over its columns and the S columns to their left.
// ----------------------------------------------------------------------------------------------
constexpr int ALL_ROWS = 128;
constexpr int ALL_WORDS = 16;
constexpr int64_t ALL_MAX_SIDE = 64 * (WAVE - ALL_WORDS - 1);  // window of one word per lane

// Calls row_fn(i, mask, w0) for every row i of unit (uy, ux), where lane l's `mask` holds the
// unit's cells of row i with dp >= k in word w0 + l.  k in [1, ALL_MAX_SIDE].
template <class RowFn>
__device__ void unit_rows_ge(const uint64_t *__restrict__ bits, int64_t m, int64_t n,
                             int64_t ldw, int64_t uy, int64_t ux, int32_t k, RowFn &&row_fn) {
    const int lane = __lane_id();
    const int64_t ra = uy * ALL_ROWS, rb = ra + ALL_ROWS < m ? ra + ALL_ROWS : m;
    const int64_t xa = ux * ALL_WORDS * 64, xb = xa + ALL_WORDS * 64 < n ? xa + ALL_WORDS * 64 : n;
    const int64_t nwords = (n + 63) >> 6;
    const int64_t w0 = xa - k > 0 ? ((xa - k) >> 6) : 0;
    const int64_t w1 = (xb + 63) >> 6;
    const int64_t wl = w0 + lane;
    const bool valid = wl < w1;
    const int64_t wl_c = valid ? wl : w0;
    const uint64_t wmask = !valid ? 0ull : (wl == nwords - 1 ? last_word_mask(n) : ~0ull);
    uint64_t own = 0;
    if (valid) {
        const int64_t lo = (xa > wl * 64 ? xa : wl * 64) - wl * 64;
        const int64_t hi = (xb < wl * 64 + 64 ? xb : wl * 64 + 64) - wl * 64;
        if (hi > lo) own = (hi - lo == 64 ? ~0ull : ((1ull << (hi - lo)) - 1)) << lo;
    }
    uint64_t P[HB];
#pragma unroll
    for (int p = 0; p < HB; ++p) P[p] = 0;
    // heights at row ra - 1, clamped at k (only H >= k matters)
    uint64_t acc = valid ? ~0ull : 0ull;
    const int64_t rstop = ra - k > 0 ? ra - k : 0;
    constexpr int FB = 16;
    for (int64_t r0 = ra - 1; r0 >= rstop; r0 -= FB) {
        uint64_t v[FB];
#pragma unroll
        for (int u = 0; u < FB; ++u) {
            const int64_t r = r0 - u >= rstop ? r0 - u : rstop;
            v[u] = bits[r * ldw + wl_c];
        }
        for (int u = 0; u < FB; ++u) {  // stops at the scan's top: not unrolled
            if (r0 - u < rstop) break;
            acc &= v[u] & wmask;
            planes_inc_masked(P, acc);
        }
        if (!__ballot(acc != 0)) break;
    }
    for (int64_t i0 = ra; i0 < rb; i0 += FB) {
        uint64_t v[FB];
#pragma unroll
        for (int u = 0; u < FB; ++u) {
            const int64_t r = i0 + u < rb ? i0 + u : rb - 1;
            v[u] = bits[r * ldw + wl_c];
        }
        for (int u = 0; u < FB; ++u) {
            const int64_t i = i0 + u;
            if (i >= rb) break;
            const uint64_t x = v[u] & wmask;
            planes_inc_masked(P, ~0ull);
#pragma unroll
            for (int p = 0; p < HB; ++p) P[p] &= x;
            row_fn(i, row_erode(planes_ge(P, k), k, lane) & own, w0);
        }
    }
}

// Exclusive prefix sum of a per-lane count over the wave (lane order), and the total.
__device__ __forceinline__ uint32_t wave_excl_sum(uint32_t v, uint32_t *total) {
    const int lane = __lane_id();
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    *total = __shfl(x, WAVE - 1);
    return x - v;
}

} // namespace msk
