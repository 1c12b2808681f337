// cube.hip -- largest all-ones cube of a packed binary volume (the higher-dimensional
// generalization the paper proposes as future work, Section 6), and the search over its side.
//
// E_k marks the voxels that are the far corner (largest z, y and x) of an all-ones k x k x k cube.
// Since cubes of side a tile a cube of side a + b (b <= a) when shifted by 0 or b along each axis,
//     E_{a+b}(z, y, x) = AND over (dz, dy, dx) in {0, b}^3 of E_a(z - dz, y - dy, x - dx).
// E_{k+1} is a subset of E_k, so the side S is found by galloping (E_1, E_2, E_4, ... until one is
// empty) and bisecting, as in the plane case.  A probe takes the eight shifted copies in one pass
// (k_cube_probe, after k_cube_copy has copied the input into E_1), which also reports whether the
// result is empty and its first set voxel in (z, y, x) order, which for E_S is the reported
// corner.  A one-thread kernel after each probe steers the search on the device.
#include "device.hpp"
#include "launch.hpp"

namespace msk {

// E_1: the input volume (row stride lds words, plane stride M * lds) copied into a compact volume
// (row stride W) with its padding bits cleared, lowering ctl->first to the smallest position
// z * M * n + y * n + x of a set voxel.
__global__ __launch_bounds__(256) void k_cube_copy(const uint64_t *__restrict__ src, int64_t lds,
                                                   uint64_t *__restrict__ dst, uint32_t D,
                                                   uint32_t M, int64_t n, uint32_t W,
                                                   mshost::CubeControl *ctl) {
    const uint32_t total = D * M * W;
    const uint64_t lastmask = last_word_mask(n);
    const uint32_t stride = gridDim.x * blockDim.x;
    unsigned long long best = ~0ull;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
        const uint32_t row = t / W, w = t - row * W;
        const uint32_t z = row / M, y = row - z * M;
        uint64_t v = src[((int64_t)z * M + y) * lds + w];
        if (w == W - 1) v &= lastmask;
        dst[(int64_t)row * W + w] = v;
        if (v) {
            const unsigned long long p =
                ((unsigned long long)z * M + y) * (unsigned long long)n +
                (unsigned long long)w * 64 + (unsigned long long)__builtin_ctzll(v);
            best = p < best ? p : best;
        }
    }
    // one atomic per block, and only when it can lower the current first position
    __shared__ unsigned long long s_min[4];
    unsigned long long wb = best;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o2 = __shfl_xor(wb, off);
        wb = o2 < wb ? o2 : wb;
    }
    if (__lane_id() == 0) s_min[threadIdx.x / WAVE] = wb;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long b = s_min[0];
        for (int k = 1; k < 4; ++k) b = s_min[k] < b ? s_min[k] : b;
        if (b != ~0ull && b < load_relaxed(&ctl->first)) atomicMin(&ctl->first, b);
    }
}

// One probe in one pass: E_{a+b} from E_a, the AND of the eight copies of E_a shifted by 0 or b
// along each axis, taken directly (four (z, y) corner rows, each with its x-shifted self) rather
// than as three single-axis passes; the rows the shifts reach are mostly still in the L2 from
// neighbouring threads.  Voxels shifted in from outside are zeros.  The shift and the volumes
// come from the search state; once the search is done the launch does nothing.  Also lowers
// ctl->first to the result's first set voxel, as the x pass does.
__global__ __launch_bounds__(256) void k_cube_probe(uint64_t *V0, uint64_t *V1, uint64_t *V2,
                                                    uint32_t D, uint32_t M, int64_t n, uint32_t W,
                                                    mshost::CubeControl *ctl) {
    const int32_t phase = uniform(__hip_atomic_load(&ctl->phase, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT));
    if (phase != mshost::CUBE_GALLOP && phase != mshost::CUBE_BISECT) return;
    const int32_t cur = uniform(ctl->cur), nxt = uniform(ctl->nxt);
    const uint32_t d = (uint32_t)uniform((int32_t)ctl->b);
    const uint64_t *__restrict__ src = cur == 0 ? V0 : (cur == 1 ? V1 : V2);
    uint64_t *__restrict__ dst = nxt == 0 ? V0 : (nxt == 1 ? V1 : V2);
    const uint32_t total = D * M * W;
    const uint64_t lastmask = last_word_mask(n);
    const uint32_t stride = gridDim.x * blockDim.x;
    const uint32_t q = d >> 6, r = d & 63;
    unsigned long long best = ~0ull;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
        const uint32_t row = t / W, w = t - row * W;
        const uint32_t z = row / M, y = row - z * M;
        uint64_t acc = (z >= d && y >= d) ? ~0ull : 0ull;  // a corner outside: all zero
        for (int c = 0; c < 4 && acc; ++c) {
            const uint32_t dz = (c & 2) ? d : 0, dy = (c & 1) ? d : 0;
            const uint64_t *s = src + ((int64_t)(z - dz) * M + (y - dy)) * W;
            const uint64_t hi = w >= q ? s[w - q] : 0ull;
            const uint64_t lo = w >= q + 1 ? s[w - q - 1] : 0ull;
            const uint64_t o = r ? ((hi << r) | (lo >> (64 - r))) : hi;
            acc &= s[w] & o;
        }
        if (w == W - 1) acc &= lastmask;
        dst[(int64_t)row * W + w] = acc;
        if (acc) {
            const unsigned long long p =
                ((unsigned long long)z * M + y) * (unsigned long long)n +
                (unsigned long long)w * 64 + (unsigned long long)__builtin_ctzll(acc);
            best = p < best ? p : best;
        }
    }
    __shared__ unsigned long long s_min[4];
    unsigned long long wb = best;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o2 = __shfl_xor(wb, off);
        wb = o2 < wb ? o2 : wb;
    }
    if (__lane_id() == 0) s_min[threadIdx.x / WAVE] = wb;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long b = s_min[0];
        for (int k = 1; k < 4; ++k) b = s_min[k] < b ? s_min[k] : b;
        if (b != ~0ull && b < load_relaxed(&ctl->first)) atomicMin(&ctl->first, b);
    }
}

__global__ void k_cube_begin(mshost::CubeControl *ctl, int64_t smax) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    ctl->first = ~0ull;
    ctl->fa = ~0ull;
    ctl->a = ctl->b = ctl->failed = ctl->limit = ctl->bstep = 0;
    ctl->smax = smax;
    ctl->phase = mshost::CUBE_INIT;
    ctl->cur = 0;
    ctl->nxt = 1;
}

// After a pass: take its first set voxel, choose the next shift, clear the voxel word for the
// next probe.  Gallop a = 1, 2, 4, ... (shift min(a, smax - a)) while E_{a+b} is non-empty; after
// the first empty one (shift `failed`) the side is in [a, a + failed - 1], and powers of two
// below `failed`, largest first, are added while the sum stays in range and E stays non-empty.
// Done: S = a and the corner from E_a's first voxel go to *out.
__global__ void k_cube_control(mshost::CubeControl *ctl, ms_cube *out, int64_t M, int64_t n) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    mshost::CubeControl &c = *ctl;
    if (c.phase == mshost::CUBE_DONE) return;
    const unsigned long long f = c.first;
    const bool got = f != ~0ull;
    bool done = false;
    bool bisect_next = false;
    if (c.phase == mshost::CUBE_INIT) {
        if (!got) {
            *out = ms_cube{0, -1, -1, -1};
            c.phase = mshost::CUBE_DONE;
            return;
        }
        c.fa = f;
        c.a = 1;
        c.cur = 0;
        if (c.a < c.smax) {
            c.b = c.a < c.smax - c.a ? c.a : c.smax - c.a;
            c.phase = mshost::CUBE_GALLOP;
        } else {
            done = true;
        }
    } else if (c.phase == mshost::CUBE_GALLOP) {
        if (got) {
            c.cur = c.nxt;
            c.a += c.b;
            c.fa = f;
            if (c.a < c.smax) c.b = c.a < c.smax - c.a ? c.a : c.smax - c.a;
            else done = true;
        } else {
            c.failed = c.b;
            c.limit = c.a + c.failed - 1;
            int64_t bs = 1;
            while (bs * 2 <= c.failed - 1) bs *= 2;
            c.bstep = bs;
            c.phase = mshost::CUBE_BISECT;
            bisect_next = true;
        }
    } else {  // CUBE_BISECT: the probe just run added bstep
        if (got) {
            c.cur = c.nxt;
            c.a += c.b;
            c.fa = f;
        }
        c.bstep /= 2;
        bisect_next = true;
    }
    if (bisect_next) {
        while (c.bstep >= 1 && c.a + c.bstep > c.limit) c.bstep /= 2;
        if (c.failed > 1 && c.bstep >= 1) c.b = c.bstep;
        else done = true;
    }
    if (done) {
        const unsigned long long plane = (unsigned long long)M * (unsigned long long)n;
        const unsigned long long rem = c.fa % plane;
        *out = ms_cube{c.a, (int64_t)(c.fa / plane), (int64_t)(rem / (unsigned long long)n),
                       (int64_t)(rem % (unsigned long long)n)};
        c.phase = mshost::CUBE_DONE;
        return;
    }
    c.nxt = (c.cur + 1) % 3;
    c.first = ~0ull;
}

} // namespace msk

namespace mshost {

size_t cube_workspace_bytes(int64_t D, int64_t M, int64_t n) {
    const int64_t W = std::max<int64_t>(1, (n + 63) / 64);
    const size_t vol = (size_t)D * (size_t)M * (size_t)W * sizeof(uint64_t);
    return 256 + 3 * ((vol + 255) & ~(size_t)255);
}

uint64_t *cube_volume(void *ws, int64_t D, int64_t M, int64_t n, int k) {
    const int64_t W = std::max<int64_t>(1, (n + 63) / 64);
    const size_t vol = (size_t)D * (size_t)M * (size_t)W * sizeof(uint64_t);
    return reinterpret_cast<uint64_t *>(static_cast<char *>(ws) + 256 +
                                        (size_t)k * ((vol + 255) & ~(size_t)255));
}

hipError_t launch_cube_begin(const LaunchEnv &env, CubeControl *ctl, int64_t smax) {
    hipLaunchKernelGGL(msk::k_cube_begin, dim3(1), dim3(64), 0, env.stream, ctl, smax);
    return hipGetLastError();
}

hipError_t launch_cube_control(const LaunchEnv &env, CubeControl *ctl, ms_cube *out, int64_t M,
                               int64_t n) {
    hipLaunchKernelGGL(msk::k_cube_control, dim3(1), dim3(64), 0, env.stream, ctl, out, M, n);
    return hipGetLastError();
}

hipError_t launch_cube_probe(const LaunchEnv &env, uint64_t *const V[3], int64_t D, int64_t M,
                             int64_t n, CubeControl *ctl) {
    const int64_t W = std::max<int64_t>(1, (n + 63) / 64);
    const int64_t total = D * M * W;
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256,
                                                                   (int64_t)env.num_cus * 16));
    hipLaunchKernelGGL(msk::k_cube_probe, dim3((unsigned)blocks), dim3(256), 0, env.stream, V[0],
                       V[1], V[2], (uint32_t)D, (uint32_t)M, n, (uint32_t)W, ctl);
    return hipGetLastError();
}

hipError_t launch_cube_copy(const LaunchEnv &env, const uint64_t *src, int64_t lds,
                            uint64_t *dst, int64_t D, int64_t M, int64_t n, CubeControl *ctl) {
    const int64_t W = std::max<int64_t>(1, (n + 63) / 64);
    const int64_t total = D * M * W;
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256,
                                                                   (int64_t)env.num_cus * 16));
    hipLaunchKernelGGL(msk::k_cube_copy, dim3((unsigned)blocks), dim3(256), 0, env.stream, src,
                       lds, dst, (uint32_t)D, (uint32_t)M, n, (uint32_t)W, ctl);
    return hipGetLastError();
}

} // namespace mshost
