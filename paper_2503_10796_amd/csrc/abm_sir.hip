// abm_sir.hip -- SIR epidemiology on the GPU (Sec 4.6.3, Algorithms 3-5,
// Table 4.3) with toroidal or closed space boundaries (Sec 4.4.11).
//
// Persons live in a cubic space [0, S]^3 and are updated in place.  Only
// infected persons can pass on an infection, so the neighbourhood search of
// Algorithm 3 runs over an index of the infected persons alone: their
// start-of-iteration positions, copied in the order of the boxes of a uniform
// grid whose box length Lb is at least twice the infection radius (three radii
// where the space allows).  Every infected person within the radius of a point
// then lies in the point's own box or in the one neighbour box per axis on the
// side of the box's half the point is in: eight boxes, not 27.  Late in an
// epidemic nearly all persons have recovered and the index is small.
// One iteration:
//   k_sir_behave   per person, in storage order: infection (Algorithm 3)
//                  against the index, recovery (Algorithm 4), random step and
//                  boundary (Algorithm 5), written in place; a person infected
//                  after its behaviours gets the box of its new position and
//                  its rank in that box (one atomic on the box count); counts
//                  per state
//   k_sir_tiles / k_sir_top / k_sir_apply
//                  exclusive scan of the box counts into box starts (and the
//                  counts cleared for the next binning)
//   k_sir_iscatter the new index: every infected person's position to its
//                  slot (box start + rank)
//   k_sir_end      iteration counter and the next history slot
// Every kResortEvery iterations the persons themselves are sorted by box
// (the same scan, a destination pass and a gather), so that persons next to
// each other in storage stay close in space and the searches and index
// writes of a wave touch few lines.  Each of the two iteration forms is
// captured once into a HIP graph and replayed.  The order of persons inside
// a box depends on the order of the atomics, but nothing computed depends on
// it (the infection test is an OR over neighbours, every draw is keyed by the
// person's uid), so results are deterministic.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "abm_device.h"

namespace abm {
namespace sir {

constexpr uint32_t kTagInfection = 0x494e4645u;  // 'INFE'
constexpr uint32_t kTagRecovery = 0x5245434fu;   // 'RECO'
constexpr uint32_t kTagMove = 0x4d4f5645u;       // 'MOVE'
constexpr uint8_t kSusceptible = ABM_SIR_SUSCEPTIBLE, kInfected = ABM_SIR_INFECTED, kRecovered = ABM_SIR_RECOVERED;
constexpr int kThreads = 256;
constexpr int kScanTile = 4096;     // boxes per scan tile: 4 rounds of 256 threads x 4
constexpr int kTopThreads = 1024;   // the single work group of the tile-offset scan
constexpr int64_t kMaxDims = 1600;  // boxes per axis: D^3 < 2^32
constexpr int kBehaveGrid = 4096;   // persistent work groups of the person kernel (16 per CU)
constexpr int kResortEvery = 64;    // iterations between two sorts of the persons by box

struct alignas(64) Ctl {
    int64_t iter;
};

// Device view of one population (passed by value to every kernel).
struct Dev {
    int64_t n, nbox, ntiles;
    int32_t D, boundary, hist_cap, pad;
    double S, halfS, Lb, halfLb, r2, p_inf, p_rec, speed;
    uint64_t seed;
    uint32_t sim_id;
    Ctl *ctl;
    double *pos;                 // persons in storage order: x block, y block, z block
    uint8_t *state;
    uint32_t *uid;
    double *tmp;                 // staging of the person sort (and of queries)
    uint8_t *state_t;
    uint32_t *uid_t;
    uint32_t *key, *rank;        // box of a position and rank within it (index, person sort)
    uint32_t *src;               // person sort: person (in the staging order) of every sorted slot
    uint32_t *count;             // nbox: binning counters, cleared by the scan
    uint32_t *start;             // nbox + 1: box starts of the index of infected persons
    uint32_t *pstart;            // nbox + 1: box starts of the person sort
    uint32_t *tile;              // ntiles: tile sums, then their exclusive prefix
    double *ipos;                // the index: infected persons' positions in box order (x, y, z per slot)
    unsigned long long *hist;    // hist_cap x 3
};

// Box coordinate along one axis of a coordinate in [0, S] (FP64 division).
__device__ inline int box_axis(const Dev &d, double v) {
    double q = floor(v / d.Lb);
    int b = (int)q;
    return b < 0 ? 0 : (b >= d.D ? d.D - 1 : b);
}

// Offset from a to b along one axis, minimum image on the torus.
__device__ inline double axis_offset(const Dev &d, double a, double b) {
#pragma clang fp contract(off)
    double o = b - a;
    if (d.boundary == ABM_BOUNDARY_TOROIDAL) {
        if (o > d.halfS) o -= d.S;
        else if (o < -d.halfS) o += d.S;
    }
    return o;
}

// A coordinate after the step (Sec 4.4.11).  Toroidal: the fmod wrap of
// Algorithm 5; for |v| < 2S (the step is shorter than S) it reduces exactly
// to one subtraction or addition of S (Sterbenz: S <= v < 2S makes v - S
// exact, and fmod returns v itself for -S < v < S).  Closed: clamped.
__device__ inline double bound(const Dev &d, double v) {
#pragma clang fp contract(off)
    if (d.boundary == ABM_BOUNDARY_CLOSED) return v < 0.0 ? 0.0 : (v > d.S ? d.S : v);
    if (v >= d.S) return v - d.S;
    if (v < 0.0) return d.S + v;
    return v;
}

// Algorithm 3's neighbourhood test: an infected person strictly within the
// radius of (x, y, z) in the start-of-iteration state (the index holds the
// infected persons only).  Per axis the own box and the neighbour box on the
// side of the point's half of it: Lb >= 2 r (1 + 2^-20), so the far side is
// out of reach with a margin far above the rounding of the box coordinate.
// The starts and ends of the (up to) eight boxes are loaded first, all in
// flight together; then the boxes are scanned two at a time in lock-step, so
// that two entry loads are in flight (more cost the occupancy that hides the
// latency of the searches).
__device__ bool infected_near(const Dev &d, double x, double y, double z) {
#pragma clang fp contract(off)
    const double c[3] = {x, y, z};
    uint32_t nb[3][2];
    bool two[3];
    for (int a = 0; a < 3; ++a) {
        const int b = box_axis(d, c[a]);
        const double o = c[a] - (double)b * d.Lb;
        int other = b + (o < d.halfLb ? -1 : 1);
        bool ok;
        if (d.boundary == ABM_BOUNDARY_TOROIDAL) {
            other = other < 0 ? other + d.D : (other >= d.D ? other - d.D : other);
            ok = other != b;
        } else {
            ok = other >= 0 && other < d.D;
        }
        nb[a][0] = (uint32_t)b;
        nb[a][1] = ok ? (uint32_t)other : (uint32_t)b;  // a valid box either way; unused unless ok
        two[a] = ok;
    }
    uint32_t j0[8], j1[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int ix = k & 1, iy = (k >> 1) & 1, iz = k >> 2;
        const uint32_t box = nb[0][ix] + (uint32_t)d.D * (nb[1][iy] + (uint32_t)d.D * nb[2][iz]);
        const bool use = (ix == 0 || two[0]) && (iy == 0 || two[1]) && (iz == 0 || two[2]);
        j0[k] = d.start[box];
        const uint32_t e = d.start[box + 1];
        j1[k] = use ? e : j0[k];
    }
#pragma unroll
    for (int k = 0; k < 8; k += 2) {
        uint32_t ja = j0[k], jb = j0[k + 1];
        while (ja < j1[k] || jb < j1[k + 1]) {
            const bool ia = ja < j1[k], ib = jb < j1[k + 1];
            const size_t sa = ia ? ja : 0u, sb = ib ? jb : 0u;  // slot 0 exists (n >= 1 slots); read but ignored
            const double ax = d.ipos[3 * sa], ay = d.ipos[3 * sa + 1], az = d.ipos[3 * sa + 2];
            const double bx = d.ipos[3 * sb], by = d.ipos[3 * sb + 1], bz = d.ipos[3 * sb + 2];
            const double dax = axis_offset(d, x, ax), day = axis_offset(d, y, ay), daz = axis_offset(d, z, az);
            const double dbx = axis_offset(d, x, bx), dby = axis_offset(d, y, by), dbz = axis_offset(d, z, bz);
            if ((ia && fma(daz, daz, fma(day, day, dax * dax)) < d.r2) ||
                (ib && fma(dbz, dbz, fma(dby, dby, dbx * dbx)) < d.r2))
                return true;
            ja += ia ? 1u : 0u;
            jb += ib ? 1u : 0u;
        }
    }
    return false;
}

__device__ inline uint32_t box_key(const Dev &d, double x, double y, double z) {
    return (uint32_t)box_axis(d, x) + (uint32_t)d.D * ((uint32_t)box_axis(d, y) + (uint32_t)d.D * (uint32_t)box_axis(d, z));
}

// Adds this wave's persons per state to the work group's counters.
__device__ inline void count_states(bool active, uint8_t st, uint32_t *cnt) {
    const uint64_t m0 = __ballot(active && st == kSusceptible);
    const uint64_t m1 = __ballot(active && st == kInfected);
    const uint64_t m2 = __ballot(active && st == kRecovered);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&cnt[0], (uint32_t)__popcll(m0));
        atomicAdd(&cnt[1], (uint32_t)__popcll(m1));
        atomicAdd(&cnt[2], (uint32_t)__popcll(m2));
    }
}

// Persons of one work group in the kernels that run per person in storage
// order: group b runs on XCD b mod 8, and the groups of XCD k take tiles of
// the k-th contiguous eighth of the persons in turn.  Between two person
// sorts storage order follows the boxes, so an XCD's searches and index
// writes stay in one slab of the space and share its L2.  The grid is a
// multiple of 8 work groups.
struct XcdTiles {
    int64_t lo, hi, first, stride;
    __device__ XcdTiles(int64_t n) {
        const int64_t chunk = ((n + 7) / 8 + kThreads - 1) / kThreads * kThreads;
        lo = (int64_t)(blockIdx.x & 7) * chunk;
        hi = lo + chunk < n ? lo + chunk : n;
        first = lo + (int64_t)(blockIdx.x >> 3) * kThreads;
        stride = (int64_t)(gridDim.x >> 3) * kThreads;
    }
};

// One iteration of the behaviours of every person (Algorithms 3, 4, 5), in
// place: the search reads the index, never the persons' arrays.  Eight
// waves per SIMD (the launch bound keeps the scalar registers below the
// limit of seven): the early iterations wait on the searches' loads, and
// more waves hide more of that latency.
__global__ __launch_bounds__(kThreads, 8) void k_sir_behave(Dev d) {
#pragma clang fp contract(off)
    __shared__ uint32_t cnt[3];
    if (threadIdx.x < 3) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t iter = d.ctl->iter;
    const int64_t n = d.n;
    const XcdTiles tl(n);
    for (int64_t base = tl.first; base < tl.hi; base += tl.stride) {
        const int64_t i = base + threadIdx.x;
        const bool active = i < tl.hi;
        uint8_t st = 0;
        if (active) {
            const double x = d.pos[i], y = d.pos[n + i], z = d.pos[2 * n + i];
            st = d.state[i];
            const uint32_t u = d.uid[i];
            uint32_t c[4];
            if (st == kSusceptible) {
                agent_draw(d.seed, kTagInfection, d.sim_id, u, (uint64_t)iter, c);
                if (uniform_open(c[0]) < d.p_inf && infected_near(d, x, y, z)) st = kInfected;
            }
            if (st == kInfected) {
                agent_draw(d.seed, kTagRecovery, d.sim_id, u, (uint64_t)iter, c);
                if (uniform_open(c[0]) < d.p_rec) st = kRecovered;
            }
            agent_draw(d.seed, kTagMove, d.sim_id, u, (uint64_t)iter, c);
            double v[3];
            for (int a = 0; a < 3; ++a) v[a] = 2.0 * uniform_open(c[a]) - 1.0;
            const double norm = sqrt(fma(v[2], v[2], fma(v[1], v[1], v[0] * v[0])));
            const double nx = bound(d, x + (v[0] / norm) * d.speed);
            const double ny = bound(d, y + (v[1] / norm) * d.speed);
            const double nz = bound(d, z + (v[2] / norm) * d.speed);
            if (st == kInfected) {  // into the next iteration's index
                const uint32_t k = box_key(d, nx, ny, nz);
                d.rank[i] = atomicAdd(&d.count[k], 1u);
                d.key[i] = k;
            }
            d.pos[i] = nx;
            d.pos[n + i] = ny;
            d.pos[2 * n + i] = nz;
            d.state[i] = st;
        }
        count_states(active, st, cnt);
    }
    __syncthreads();
    if (threadIdx.x < 3 && cnt[threadIdx.x])
        atomicAdd(&d.hist[(iter % d.hist_cap) * 3 + threadIdx.x], (unsigned long long)cnt[threadIdx.x]);
}

// Box and rank of every infected person (the index at creation).
__global__ __launch_bounds__(kThreads) void k_sir_ibin(Dev d) {
    const int64_t n = d.n;
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        if (d.state[i] != kInfected) continue;
        const uint32_t k = box_key(d, d.pos[i], d.pos[n + i], d.pos[2 * n + i]);
        d.rank[i] = atomicAdd(&d.count[k], 1u);
        d.key[i] = k;
    }
}

// Every infected person's position to its slot of the index.
__global__ __launch_bounds__(kThreads) void k_sir_iscatter(Dev d) {
    const int64_t n = d.n;
    const XcdTiles tl(n);
    for (int64_t i = tl.first + threadIdx.x; i < tl.hi; i += tl.stride) {
        if (d.state[i] != kInfected) continue;
        const size_t j = (size_t)d.start[d.key[i]] + d.rank[i];
        d.ipos[3 * j] = d.pos[i];
        d.ipos[3 * j + 1] = d.pos[n + i];
        d.ipos[3 * j + 2] = d.pos[2 * n + i];
    }
}

// The persons into the staging arrays (before a person sort).
__global__ __launch_bounds__(kThreads) void k_sir_stash(Dev d) {
    const int64_t n = d.n;
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        d.tmp[i] = d.pos[i];
        d.tmp[n + i] = d.pos[n + i];
        d.tmp[2 * n + i] = d.pos[2 * n + i];
        d.state_t[i] = d.state[i];
        d.uid_t[i] = d.uid[i];
    }
}

// Box and rank of every person of the staging arrays (person sort).
__global__ __launch_bounds__(kThreads) void k_sir_bin(Dev d) {
    const int64_t n = d.n;
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const uint32_t k = box_key(d, d.tmp[i], d.tmp[n + i], d.tmp[2 * n + i]);
        d.rank[i] = atomicAdd(&d.count[k], 1u);
        d.key[i] = k;
    }
}

// Sum of the box counts of one scan tile: four rounds of 1,024 boxes, each
// thread loading four consecutive counts per round (16-byte loads).
__global__ __launch_bounds__(kThreads) void k_sir_tiles(Dev d) {
    __shared__ uint32_t sh[kThreads / 64];
    const int64_t t0 = (int64_t)blockIdx.x * kScanTile;
    uint32_t s = 0;
    for (int r = 0; r < kScanTile / (4 * kThreads); ++r) {
        const int64_t b = t0 + (int64_t)r * 4 * kThreads + 4 * (int64_t)threadIdx.x;
        if (b + 4 <= d.nbox) {
            const uint4 c = *reinterpret_cast<const uint4 *>(d.count + b);
            s += c.x + c.y + c.z + c.w;
        } else {
            for (int k = 0; k < 4; ++k)
                if (b + k < d.nbox) s += d.count[b + k];
        }
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) d.tile[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// Exclusive prefix of the tile sums, in place (one work group); the end of
// the last box is the total.
__global__ __launch_bounds__(kTopThreads) void k_sir_top(Dev d, uint32_t *start) {
    __shared__ uint32_t sh[kTopThreads / 64];
    __shared__ uint32_t carry_sh;
    if (threadIdx.x == 0) carry_sh = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int64_t base = 0; base < d.ntiles; base += kTopThreads) {
        const int64_t t = base + threadIdx.x;
        const uint32_t v = t < d.ntiles ? d.tile[t] : 0u;
        uint32_t x = v;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (lane == 63) sh[wid] = x;
        __syncthreads();
        uint32_t wpre = 0, total = 0;
        for (int w = 0; w < kTopThreads / 64; ++w) {
            if (w < wid) wpre += sh[w];
            total += sh[w];
        }
        const uint32_t carry = carry_sh;
        if (t < d.ntiles) d.tile[t] = carry + wpre + x - v;
        __syncthreads();
        if (threadIdx.x == 0) carry_sh = carry + total;
        __syncthreads();
    }
    if (threadIdx.x == 0) start[d.nbox] = carry_sh;
}

// Box starts of one tile (its offset plus the exclusive prefix of its
// counts), in four rounds of 1,024 boxes with 16-byte loads and stores; the
// counts are cleared for the next binning.
__global__ __launch_bounds__(kThreads) void k_sir_apply(Dev d, uint32_t *start) {
    __shared__ uint32_t sh[kThreads / 64];
    const int64_t t0 = (int64_t)blockIdx.x * kScanTile;
    uint32_t carry = d.tile[blockIdx.x];
    for (int r = 0; r < kScanTile / (4 * kThreads); ++r) {
        const int64_t b = t0 + (int64_t)r * 4 * kThreads + 4 * (int64_t)threadIdx.x;
        if (t0 + (int64_t)r * 4 * kThreads >= d.nbox) break;  // the whole round is past the end (uniform)
        const bool full = b + 4 <= d.nbox;
        uint32_t v[4];
        if (full) {
            const uint4 c = *reinterpret_cast<const uint4 *>(d.count + b);
            v[0] = c.x; v[1] = c.y; v[2] = c.z; v[3] = c.w;
        } else {
            for (int k = 0; k < 4; ++k) v[k] = b + k < d.nbox ? d.count[b + k] : 0u;
        }
        uint32_t total;
        const uint32_t pre = carry + block_excl_scan_4(v, sh, total);
        const uint32_t s0 = pre, s1 = s0 + v[0], s2 = s1 + v[1], s3 = s2 + v[2];
        if (full) {
            *reinterpret_cast<uint4 *>(start + b) = make_uint4(s0, s1, s2, s3);
            *reinterpret_cast<uint4 *>(d.count + b) = make_uint4(0u, 0u, 0u, 0u);
        } else {
            const uint32_t sv[4] = {s0, s1, s2, s3};
            for (int k = 0; k < 4; ++k)
                if (b + k < d.nbox) {
                    start[b + k] = sv[k];
                    d.count[b + k] = 0u;
                }
        }
        carry += total;
    }
}

// Person sort: the source of every slot of the new box order.
__global__ __launch_bounds__(kThreads) void k_sir_dest(Dev d) {
    const int64_t n = d.n;
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        d.src[(int64_t)d.pstart[d.key[i]] + d.rank[i]] = (uint32_t)i;
}

// Person sort: every slot gathers its person from the staging arrays.  One
// slot per thread; work group b runs on XCD b mod 8 and the groups of XCD k
// take the k-th contiguous eighth of the slots in order, so that the lines of
// the staging arrays that neighbouring slots read (their persons came from
// nearby boxes) stay in one L2.
__global__ __launch_bounds__(kThreads) void k_sir_gather(Dev d) {
    const int64_t n = d.n;
    const int64_t per_xcd = gridDim.x / 8;
    const int64_t lb = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    const int64_t j = lb * kThreads + threadIdx.x;
    if (j < n) {
        const int64_t i = d.src[j];
        d.pos[j] = d.tmp[i];
        d.pos[n + j] = d.tmp[n + i];
        d.pos[2 * n + j] = d.tmp[2 * n + i];
        d.state[j] = d.state_t[i];
        d.uid[j] = d.uid_t[i];
    }
}

__global__ void k_sir_end(Dev d) {
    const int64_t next = d.ctl->iter + 1;
    unsigned long long *h = d.hist + (next % d.hist_cap) * 3;
    h[0] = h[1] = h[2] = 0ull;
    d.ctl->iter = next;
}

// Interleaved n x 3 positions from the coordinate blocks (src) into dst.
__global__ void k_sir_interleave(const double *src, double *dst, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        dst[3 * i] = src[i];
        dst[3 * i + 1] = src[n + i];
        dst[3 * i + 2] = src[2 * n + i];
    }
}
__global__ void k_sir_deinterleave(const double *src, double *dst, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        dst[i] = src[3 * i];
        dst[n + i] = src[3 * i + 1];
        dst[2 * n + i] = src[3 * i + 2];
    }
}
__global__ void k_sir_iota(uint32_t *u, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        u[i] = (uint32_t)i;
}
// Fill with a kernel (not a memset node: the graph replays it).
__global__ void k_sir_zero(uint32_t *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

inline int grid_for(int64_t n, int cap) {
    int64_t g = (n + kThreads - 1) / kThreads;
    return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}
// The same rounded up to a multiple of 8 work groups (XcdTiles kernels).
inline int grid_for_xcd(int64_t n, int cap) { return (grid_for(n, cap) + 7) / 8 * 8; }

// Exclusive scan of the box counts into `start` (the counts are cleared).
void launch_scan(const Dev &d, uint32_t *start, hipStream_t s) {
    hipLaunchKernelGGL(k_sir_tiles, dim3((unsigned)d.ntiles), dim3(kThreads), 0, s, d);
    hipLaunchKernelGGL(k_sir_top, dim3(1), dim3(kTopThreads), 0, s, d, start);
    hipLaunchKernelGGL(k_sir_apply, dim3((unsigned)d.ntiles), dim3(kThreads), 0, s, d, start);
}

// The index of infected persons from their binning.
void launch_index(const Dev &d, hipStream_t s) {
    launch_scan(d, d.start, s);
    if (d.n > 0) hipLaunchKernelGGL(k_sir_iscatter, dim3(grid_for_xcd(d.n, 65536)), dim3(kThreads), 0, s, d);
}

// The persons of the staging arrays into pos / state / uid in box order.
void launch_person_sort(const Dev &d, hipStream_t s) {
    if (d.n > 0) hipLaunchKernelGGL(k_sir_bin, dim3(grid_for(d.n, 65536)), dim3(kThreads), 0, s, d);
    launch_scan(d, d.pstart, s);
    if (d.n > 0) {
        hipLaunchKernelGGL(k_sir_dest, dim3(grid_for(d.n, 65536)), dim3(kThreads), 0, s, d);
        hipLaunchKernelGGL(k_sir_gather, dim3(((d.n + kThreads - 1) / kThreads + 7) / 8 * 8), dim3(kThreads), 0, s, d);
    }
}

void launch_behave(const Dev &d, hipStream_t s) {
    if (d.n > 0) hipLaunchKernelGGL(k_sir_behave, dim3(grid_for_xcd(d.n, kBehaveGrid)), dim3(kThreads), 0, s, d);
}

// Everything after the person kernel; with `resort` the persons are sorted
// by box at the end.
void launch_rest(const Dev &d, bool resort, hipStream_t s) {
    launch_index(d, s);
    if (resort && d.n > 0) {
        hipLaunchKernelGGL(k_sir_stash, dim3(grid_for(d.n, 65536)), dim3(kThreads), 0, s, d);
        launch_person_sort(d, s);
    }
    hipLaunchKernelGGL(k_sir_end, dim3(1), dim3(1), 0, s, d);
}

// ---------------------------------------------------------------- layout
struct Carver {
    size_t off = 0;
    template <class T>
    size_t take(size_t count) {
        size_t o = (off + 255) & ~size_t(255);
        off = o + count * sizeof(T);
        return o;
    }
};

struct Layout {
    size_t ctl, pos, tmp, state, state_t, uid, uid_t, key, rank, src, count, start, pstart, tile, ipos, hist, total;
};

bool geometry(const abm_sir_params &p, int64_t &D, double &Lb) {
    if (!(p.space > 0.0) || !isfinite(p.space) || !(p.radius > 0.0) || !isfinite(p.radius)) return false;
    // The eight-box search is exact for any box of at least twice the radius
    // (with a relative margin of 2^-20).  Boxes of three radii are taken: at
    // the person densities of Table 4.3 (about 2e-3 per um^3, radius 3.2 um)
    // boxes of 2r hold 0.55 persons on average and the search spends most of
    // its time on empty boxes; 3r (1.9 persons per box) measured fastest among
    // 2r, 2.5r, 3r, 3.5r and 4r.
    double q = floor(p.space / (3.0 * p.radius * (1.0 + 0x1.0p-20)));
    D = q < 1.0 ? 1 : (q > (double)kMaxDims ? kMaxDims : (int64_t)q);
    Lb = p.space / (double)D;
    return Lb >= 2.0 * p.radius;
}

bool params_ok(const abm_sir_params &p) {
    int64_t D;
    double Lb;
    if (!geometry(p, D, Lb)) return false;
    if (!(p.infection_prob >= 0.0 && p.infection_prob <= 1.0)) return false;
    if (!(p.recovery_prob >= 0.0 && p.recovery_prob <= 1.0)) return false;
    if (!(p.speed >= 0.0) || !isfinite(p.speed)) return false;
    if (p.boundary != ABM_BOUNDARY_TOROIDAL && p.boundary != ABM_BOUNDARY_CLOSED) return false;
    // the toroidal wrap reduces to one subtraction or addition of S only for steps shorter than S
    if (p.boundary == ABM_BOUNDARY_TOROIDAL && !(p.speed < p.space)) return false;
    return true;
}

bool make_layout(const abm_sir_params &p, int64_t n, int hist_cap, Layout &L, int64_t &nbox, int64_t &ntiles) {
    if (n < 0 || n >= ((int64_t)1 << 31) || hist_cap < 2 || hist_cap > (1 << 24) || !params_ok(p)) return false;
    int64_t D;
    double Lb;
    geometry(p, D, Lb);
    nbox = D * D * D;
    ntiles = (nbox + kScanTile - 1) / kScanTile;
    const size_t N = (size_t)(n > 0 ? n : 1);
    Carver c;
    L.ctl = c.take<Ctl>(1);
    L.pos = c.take<double>(3 * N);
    L.tmp = c.take<double>(3 * N);
    L.state = c.take<uint8_t>(N);
    L.state_t = c.take<uint8_t>(N);
    L.uid = c.take<uint32_t>(N);
    L.uid_t = c.take<uint32_t>(N);
    L.key = c.take<uint32_t>(N);
    L.rank = c.take<uint32_t>(N);
    L.src = c.take<uint32_t>(N);
    L.count = c.take<uint32_t>((size_t)nbox + 16);
    L.start = c.take<uint32_t>((size_t)nbox + 16);
    L.pstart = c.take<uint32_t>((size_t)nbox + 16);
    L.tile = c.take<uint32_t>((size_t)ntiles);
    L.ipos = c.take<double>(3 * N);
    L.hist = c.take<unsigned long long>((size_t)hist_cap * 3);
    L.total = c.off + 256;
    return true;
}

}  // namespace sir
}  // namespace abm

using abm::set_error;
using abm::clear_error;
namespace sirk = abm::sir;

struct abm_sir {
    sirk::Dev d;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    // 0: a whole iteration, 1: the person kernel, 2: the rest; 3 and 4: the
    // same as 0 and 2 with the person sort at the end
    hipGraphExec_t exec[5] = {};
    int64_t iter = 0;
    bool timing = false;
    std::vector<hipEvent_t> ev;
    double ms_total = 0.0;
    int64_t n_timed = 0;
};

#define SIRCHK(expr)                                                                  \
    do {                                                                              \
        hipError_t _e = (expr);                                                       \
        if (_e != hipSuccess) return set_error(ABM_ERR_HIP, hipGetErrorString(_e));   \
    } while (0)

static int capture(abm_sir *s, int part) {
    if (s->exec[part]) return ABM_OK;
    if (!s->cap_stream) SIRCHK(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
    SIRCHK(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
    if (part == 0 || part == 1 || part == 3) sirk::launch_behave(s->d, s->cap_stream);
    if (part == 0 || part == 2) sirk::launch_rest(s->d, false, s->cap_stream);
    if (part == 3 || part == 4) sirk::launch_rest(s->d, true, s->cap_stream);
    hipGraph_t g;
    hipError_t e = hipStreamEndCapture(s->cap_stream, &g);
    if (e != hipSuccess) return set_error(ABM_ERR_HIP, hipGetErrorString(e));
    e = hipGraphInstantiate(&s->exec[part], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);  // the instantiated graph no longer needs its template
    if (e != hipSuccess) return set_error(ABM_ERR_HIP, hipGetErrorString(e));
    return ABM_OK;
}

extern "C" size_t abm_sir_workspace_bytes(const abm_sir_params *p, int64_t n, int hist_cap) {
    if (!p) return 0;
    sirk::Layout L;
    int64_t nbox, ntiles;
    if (!sirk::make_layout(*p, n, hist_cap, L, nbox, ntiles)) return 0;
    return L.total;
}

extern "C" int abm_sir_create(const abm_sir_params *p, int64_t n, const double *pos, const uint8_t *state,
                              int hist_cap, void *workspace, size_t ws_bytes, void *hip_stream, abm_sir **out) {
    clear_error();
    if (!p || !out || !workspace || (n > 0 && (!pos || !state))) return set_error(ABM_ERR_ARG, "null argument");
    *out = nullptr;
    sirk::Layout L;
    int64_t nbox, ntiles;
    if (!sirk::make_layout(*p, n, hist_cap, L, nbox, ntiles))
        return set_error(ABM_ERR_ARG, "bad SIR parameters, person count or history length");
    if (ws_bytes < L.total) return set_error(ABM_ERR_ARG, "workspace too small");
    for (int64_t i = 0; i < 3 * n; ++i) {
        if (!isfinite(pos[i])) return set_error(ABM_ERR_NONFINITE, "non-finite position");
        if (pos[i] < 0.0 || pos[i] > p->space) return set_error(ABM_ERR_ARG, "position outside [0, space]");
    }
    int64_t counts[3] = {0, 0, 0};
    for (int64_t i = 0; i < n; ++i) {
        if (state[i] > ABM_SIR_RECOVERED) return set_error(ABM_ERR_ARG, "state outside 0..2");
        counts[state[i]] += 1;
    }
    abm_sir *s = new (std::nothrow) abm_sir();
    if (!s) return set_error(ABM_ERR_ARG, "out of host memory");
    int64_t D;
    double Lb;
    sirk::geometry(*p, D, Lb);
    char *base = (char *)(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
    sirk::Dev &d = s->d;
    d.n = n;
    d.nbox = nbox;
    d.ntiles = ntiles;
    d.D = (int32_t)D;
    d.boundary = p->boundary;
    d.hist_cap = hist_cap;
    d.S = p->space;
    d.halfS = 0.5 * p->space;
    d.Lb = Lb;
    d.halfLb = 0.5 * Lb;
    d.r2 = p->radius * p->radius;
    d.p_inf = p->infection_prob;
    d.p_rec = p->recovery_prob;
    d.speed = p->speed;
    d.seed = p->seed;
    d.sim_id = p->sim_id;
    d.ctl = (sirk::Ctl *)(base + L.ctl);
    d.pos = (double *)(base + L.pos);
    d.tmp = (double *)(base + L.tmp);
    d.state = (uint8_t *)(base + L.state);
    d.state_t = (uint8_t *)(base + L.state_t);
    d.uid = (uint32_t *)(base + L.uid);
    d.uid_t = (uint32_t *)(base + L.uid_t);
    d.key = (uint32_t *)(base + L.key);
    d.rank = (uint32_t *)(base + L.rank);
    d.src = (uint32_t *)(base + L.src);
    d.count = (uint32_t *)(base + L.count);
    d.start = (uint32_t *)(base + L.start);
    d.pstart = (uint32_t *)(base + L.pstart);
    d.tile = (uint32_t *)(base + L.tile);
    d.ipos = (double *)(base + L.ipos);
    d.hist = (unsigned long long *)(base + L.hist);
    s->stream = (hipStream_t)hip_stream;
    hipStream_t st = s->stream;
    auto undo = [&](int rc) {
        delete s;
        return rc;
    };
    hipError_t e = hipSuccess;
    if (n > 0) {
        // positions: interleaved upload into pos, de-interleaved into tmp
        e = hipMemcpyAsync(d.pos, pos, sizeof(double) * 3 * (size_t)n, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(d.state_t, state, (size_t)n, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return undo(set_error(ABM_ERR_HIP, hipGetErrorString(e)));
        hipLaunchKernelGGL(sirk::k_sir_deinterleave, dim3(sirk::grid_for(n, 65536)), dim3(sirk::kThreads), 0, st, d.pos, d.tmp, n);
        hipLaunchKernelGGL(sirk::k_sir_iota, dim3(sirk::grid_for(n, 65536)), dim3(sirk::kThreads), 0, st, d.uid_t, n);
    }
    hipLaunchKernelGGL(sirk::k_sir_zero, dim3(sirk::grid_for(nbox, 65536)), dim3(sirk::kThreads), 0, st, d.count, nbox);
    hipLaunchKernelGGL(sirk::k_sir_zero, dim3(sirk::grid_for(2 * (int64_t)hist_cap * 3, 65536)), dim3(sirk::kThreads), 0, st,
                       (uint32_t *)d.hist, 2 * (int64_t)hist_cap * 3);
    hipLaunchKernelGGL(sirk::k_sir_zero, dim3(1), dim3(64), 0, st, (uint32_t *)d.ctl, (int64_t)(sizeof(sirk::Ctl) / 4));
    // persons sorted by box, then the index of the infected ones
    sirk::launch_person_sort(d, st);
    if (n > 0) hipLaunchKernelGGL(sirk::k_sir_ibin, dim3(sirk::grid_for(n, 65536)), dim3(sirk::kThreads), 0, st, d);
    sirk::launch_index(d, st);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return undo(set_error(ABM_ERR_HIP, hipGetErrorString(e)));
    *out = s;
    return ABM_OK;
}

extern "C" int abm_sir_step(abm_sir *s, int n_iter, int64_t *counts) {
    clear_error();
    if (!s || n_iter < 0) return set_error(ABM_ERR_ARG, "bad handle or iteration count");
    if (n_iter == 0) return ABM_OK;
    int rc = s->timing ? capture(s, 1) : capture(s, 0);
    if (!rc) rc = s->timing ? capture(s, 2) : capture(s, 3);
    if (!rc && s->timing) rc = capture(s, 4);
    if (rc) return rc;
    // iteration t ends with the person sort when t + 1 is a multiple of kResortEvery
    auto resort = [&](int64_t t) { return (t + 1) % sirk::kResortEvery == 0; };
    const int cap = s->d.hist_cap;
    std::vector<unsigned long long> h;
    for (int done = 0; done < n_iter;) {
        // fewer iterations than history slots between reads of the counts (the
        // end of an iteration clears the slot of the next one)
        const int chunk = counts ? std::min(cap - 1, n_iter - done) : n_iter - done;
        if (s->timing) {
            while ((int)s->ev.size() < 2 * chunk) {
                hipEvent_t e;
                SIRCHK(hipEventCreate(&e));
                s->ev.push_back(e);
            }
            for (int it = 0; it < chunk; ++it) {
                SIRCHK(hipEventRecord(s->ev[2 * it], s->stream));
                SIRCHK(hipGraphLaunch(s->exec[1], s->stream));
                SIRCHK(hipEventRecord(s->ev[2 * it + 1], s->stream));
                SIRCHK(hipGraphLaunch(s->exec[resort(s->iter + it) ? 4 : 2], s->stream));
            }
            SIRCHK(hipStreamSynchronize(s->stream));
            for (int it = 0; it < chunk; ++it) {
                float ms = 0.0f;
                SIRCHK(hipEventElapsedTime(&ms, s->ev[2 * it], s->ev[2 * it + 1]));
                s->ms_total += ms;
            }
            s->n_timed += chunk;
        } else {
            for (int it = 0; it < chunk; ++it) SIRCHK(hipGraphLaunch(s->exec[resort(s->iter + it) ? 3 : 0], s->stream));
        }
        if (counts) {
            h.resize((size_t)cap * 3);
            SIRCHK(hipMemcpyAsync(h.data(), s->d.hist, sizeof(unsigned long long) * 3 * (size_t)cap,
                                  hipMemcpyDeviceToHost, s->stream));
            SIRCHK(hipStreamSynchronize(s->stream));
            for (int it = 0; it < chunk; ++it) {
                const int64_t slot = (s->iter + it) % cap;
                for (int k = 0; k < 3; ++k) counts[3 * (int64_t)(done + it) + k] = (int64_t)h[3 * slot + k];
            }
        }
        s->iter += chunk;
        done += chunk;
    }
    SIRCHK(hipGetLastError());
    return ABM_OK;
}

extern "C" int abm_sir_query(abm_sir *s, int field, void *dst, int dst_on_device, int64_t cap) {
    clear_error();
    if (!s || !dst) return set_error(ABM_ERR_ARG, "null argument");
    const int64_t n = s->d.n;
    if (cap < n) return set_error(ABM_ERR_ARG, "destination holds fewer rows than persons");
    if (n == 0) return ABM_OK;
    const hipMemcpyKind kind = dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    hipStream_t st = s->stream;
    if (field == ABM_SIR_POS) {
        // the temporary arrays are free between iterations
        double *src = s->d.tmp;
        hipLaunchKernelGGL(sirk::k_sir_interleave, dim3(sirk::grid_for(n, 65536)), dim3(sirk::kThreads), 0, st, s->d.pos, src, n);
        SIRCHK(hipMemcpyAsync(dst, src, sizeof(double) * 3 * (size_t)n, kind, st));
    } else if (field == ABM_SIR_STATE) {
        SIRCHK(hipMemcpyAsync(dst, s->d.state, (size_t)n, kind, st));
    } else if (field == ABM_SIR_UID) {
        SIRCHK(hipMemcpyAsync(dst, s->d.uid, sizeof(uint32_t) * (size_t)n, kind, st));
    } else {
        return set_error(ABM_ERR_ARG, "unknown field");
    }
    SIRCHK(hipGetLastError());
    SIRCHK(hipStreamSynchronize(st));
    return ABM_OK;
}

extern "C" int abm_sir_counts(abm_sir *s, int64_t *iteration, int64_t counts[3]) {
    clear_error();
    if (!s || !iteration || !counts) return set_error(ABM_ERR_ARG, "null argument");
    *iteration = s->iter;
    counts[0] = counts[1] = counts[2] = 0;
    const int64_t n = s->d.n;
    if (n == 0) return ABM_OK;
    std::vector<uint8_t> st((size_t)n);
    SIRCHK(hipMemcpyAsync(st.data(), s->d.state, (size_t)n, hipMemcpyDeviceToHost, s->stream));
    SIRCHK(hipStreamSynchronize(s->stream));
    for (uint8_t v : st) counts[v < 3 ? v : 2] += 1;
    return ABM_OK;
}

extern "C" int abm_sir_grid(abm_sir *s, int64_t *dims, double *box_len) {
    clear_error();
    if (!s || !dims || !box_len) return set_error(ABM_ERR_ARG, "null argument");
    *dims = s->d.D;
    *box_len = s->d.Lb;
    return ABM_OK;
}

extern "C" int abm_sir_set_timing(abm_sir *s, int on) {
    clear_error();
    if (!s) return set_error(ABM_ERR_ARG, "null handle");
    s->timing = on != 0;
    return ABM_OK;
}

extern "C" int abm_sir_kernel_time(abm_sir *s, double *ms_total, int64_t *n_launches) {
    clear_error();
    if (!s || !ms_total || !n_launches) return set_error(ABM_ERR_ARG, "null argument");
    *ms_total = s->ms_total;
    *n_launches = s->n_timed;
    s->ms_total = 0.0;
    s->n_timed = 0;
    return ABM_OK;
}

extern "C" int abm_sir_destroy(abm_sir *s) {
    clear_error();
    if (!s) return ABM_OK;
    if (s->stream) (void)hipStreamSynchronize(s->stream);  // teardown: nothing to recover
    for (hipGraphExec_t &g : s->exec)
        if (g) (void)hipGraphExecDestroy(g);
    for (hipEvent_t e : s->ev) (void)hipEventDestroy(e);
    if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
    delete s;
    return ABM_OK;
}
