// abm_device.h -- device helpers shared by the kernels of libabm.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "abm_internal.h"

namespace abm {

#define ABM_ABORTED(d) (__builtin_expect((d).ctl->abort != 0, 0))

constexpr double kPi = 3.14159265358979323846;

// 256 threads x 4 items: this thread's exclusive prefix of its first item and
// the block total.
__device__ inline uint32_t block_excl_scan_4(const uint32_t v[4], uint32_t *sh, uint32_t &total) {
    uint32_t s = v[0] + v[1] + v[2] + v[3];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t x = s;
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) sh[wid] = x;
    __syncthreads();
    uint32_t wpre = 0;
    total = 0;
    for (int w = 0; w < 4; ++w) {
        if (w < wid) wpre += sh[w];
        total += sh[w];
    }
    __syncthreads();
    return wpre + x - s;
}

// Morton rank of box (bx,by,bz) in a dims[0] x dims[1] x dims[2] grid: the
// number of in-grid boxes whose Morton code (x in the lowest bit, Fig 5.4) is
// smaller.  For every set bit p of the code, the boxes that agree with the
// code above p and have 0 at p are counted per axis in closed form: their free
// low bits span a range that is intersected with the grid.  Ranks of the
// in-grid boxes are dense, so they index box arrays directly.
__device__ inline uint32_t morton_rank(int bx, int by, int bz, const int32_t dims[3]) {
    const int c[3] = {bx, by, bz};
    uint64_t rank = 0;
    for (int level = 10; level >= 0; --level) {
        for (int a = 2; a >= 0; --a) {
            if (!((c[a] >> level) & 1)) continue;
            const int p = 3 * level + a;
            uint64_t prod = 1;
            for (int b = 0; b < 3; ++b) {
                int freebits;
                int64_t base;
                if (b == a) {
                    freebits = level;
                    base = (int64_t)(c[b] >> (level + 1)) << (level + 1);
                } else {
                    freebits = p < b ? 0 : (p - b + 2) / 3;
                    base = (int64_t)(c[b] >> freebits) << freebits;
                }
                int64_t span = (int64_t)1 << freebits;
                int64_t cnt = (int64_t)dims[b] - base;
                cnt = cnt < 0 ? 0 : (cnt > span ? span : cnt);
                prod *= (uint64_t)cnt;
            }
            rank += prod;
        }
    }
    return (uint32_t)rank;
}

// Box slot of box (bx,by,bz): boxes are ordered by the Morton rank of their
// aligned 4x4x4 block, then by the Morton code of the box within the block
// (two bits per axis, x lowest).  For aligned power-of-two blocks this is the
// Morton order of the boxes; edge blocks that stick out of the grid keep
// their unused slots empty.  The block ranks form a small table (one entry
// per block), so no per-box table is read.
static_assert(kBlk == 4, "box slots interleave two bits per axis within a block");
__device__ inline uint32_t local_morton(int bx, int by, int bz) {
    return (uint32_t)((bx & 1) | ((by & 1) << 1) | ((bz & 1) << 2) | ((bx & 2) << 2) | ((by & 2) << 3) |
                      ((bz & 2) << 4));
}
__device__ inline uint32_t box_rank(const Dev &d, const SimDesc &S, int bx, int by, int bz) {
    const int64_t blk =
        (int64_t)(bx >> 2) + (int64_t)S.bdims[0] * ((int64_t)(by >> 2) + (int64_t)S.bdims[1] * (int64_t)(bz >> 2));
    return d.brank[S.b_off + blk] * 64u + local_morton(bx, by, bz);
}

// Box slot of the box holding (x, y, z) in the current grid of S.
__device__ inline uint32_t box_rank_of(const Dev &d, const SimDesc &S, double x, double y, double z) {
    int bx = box_coord(x, S.lo[0], S.L, S.dims[0]);
    int by = box_coord(y, S.lo[1], S.L, S.dims[1]);
    int bz = box_coord(z, S.lo[2], S.L, S.dims[2]);
    return box_rank(d, S, bx, by, bz);
}

__device__ inline uint32_t key_rank(const Dev &d, const SimDesc &S, uint32_t key) {
    int bx, by, bz;
    unpack_key(key, bx, by, bz);
    return box_rank(d, S, bx, by, bz);
}

// Box marks of the static rule, kept per box slot and per aligned block.
__device__ inline void mark_box(uint8_t *box_marks, uint8_t *blk_marks, const SimDesc &S, uint32_t m) {
    box_marks[S.b_off + m] = 1;
    blk_marks[S.b_off + (m >> 6)] = 1;
}

// Atomic counting in which runs of equal keys in consecutive lanes of a wave
// share one atomic add of the run length at base[key]; returns this lane's
// position among the adds to its counter.  Same-address atomics of one
// instruction serialize, and agents in Morton order arrive in such runs.
// Every lane of the wave must call this; lanes with valid == false take no
// position and must be the last lanes of the wave.
__device__ inline uint32_t run_atomic_add(uint32_t *base, uint32_t key, bool valid) {
    const int lane = threadIdx.x & 63;
    const uint32_t kp = __shfl_up(key, 1);
    const bool head = valid && (lane == 0 || kp != key);
    const uint64_t hm = __ballot(head);
    const uint64_t vm = __ballot(valid);
    const uint64_t upto = (2ull << lane) - 1;  // lanes 0..lane (all lanes for lane 63)
    const uint64_t below = hm & upto;
    const int start = below ? 63 - __clzll(below) : 0;
    uint32_t r = 0;
    if (head) {
        const uint64_t after = hm & ~upto;
        const int next = after ? __ffsll((long long)after) - 1 : 64;
        const int last = 63 - __clzll(vm);
        const int end = next < last + 1 ? next : last + 1;
        r = atomicAdd(&base[key], (uint32_t)(end - lane));
    }
    return __shfl(r, start) + (uint32_t)(lane - start);
}

// Philox4x32-10 (Salmon et al., SC 2011): ten rounds on the counter c with
// key (k0, k1); c is replaced by the output block.
__device__ inline void philox(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        // each product's high and low words from one 32 x 32 -> 64-bit multiply
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0], p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Per-agent random words of the cell behaviour (Algorithm 2): Philox4x32-10
// with counter (uid low, uid high, iteration, simulation) and key (seed low
// XOR a per-purpose tag, seed high), so that every draw is a pure function
// of the agent and the iteration.  A word w gives the uniform (w + 1/2) 2^-32
// in the open interval (0, 1), exact in FP64.
constexpr uint32_t kTagBrownian = 0x42524f57u, kTagDeath = 0x44454154u, kTagDivision = 0x44495650u;
__device__ inline void agent_draw(uint64_t seed, uint32_t tag, uint32_t sim, uint64_t uid, uint64_t iter,
                                  uint32_t c[4]) {
    c[0] = (uint32_t)uid;
    c[1] = (uint32_t)(uid >> 32);
    c[2] = (uint32_t)iter;
    c[3] = sim;
    philox(c, (uint32_t)seed ^ tag, (uint32_t)(seed >> 32));
}
__device__ inline double uniform_open(uint32_t w) { return ((double)w + 0.5) * 0x1.0p-32; }

// Brownian step of Algorithm 2: three uniforms in (-1, 1), divided
// by their Euclidean norm, times the displacement rate (correctly rounded FP64
// division and square root, no contraction).
__device__ inline void brownian_step(uint64_t seed, uint32_t sim, uint64_t uid, uint64_t iter, double rate,
                                     double b[3]) {
#pragma clang fp contract(off)
    uint32_t c[4];
    agent_draw(seed, kTagBrownian, sim, uid, iter, c);
    double v[3];
    for (int a = 0; a < 3; ++a) v[a] = 2.0 * uniform_open(c[a]) - 1.0;
    const double norm = sqrt(fma(v[2], v[2], fma(v[1], v[1], v[0] * v[0])));
    for (int a = 0; a < 3; ++a) b[a] = (v[a] / norm) * rate;
}

// Squared distance below L^2 with the neighbour predicate's exact expression.
__device__ inline bool near_point(double x, double y, double z, double px, double py, double pz, double L2) {
#pragma clang fp contract(off)
    double ddx = x - px, ddy = y - py, ddz = z - pz;
    return fma(ddz, ddz, fma(ddy, ddy, ddx * ddx)) < L2;
}

}  // namespace abm
