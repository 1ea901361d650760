// abm_internal.h -- device data layout and helpers of libabm (gfx950).
//
// Every simulation of a batch owns a contiguous agent range [a_off, a_off+cap)
// of the flattened structure-of-arrays state and a grid-box range.  Positions
// are FP64 and double-buffered (the force sweep reads the start-of-iteration
// buffer and writes the other one: copy semantics, Sec 5.2.1).  The other
// per-agent fields are double-buffered only for the periodic Morton re-sort.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "abm.h"

namespace abm {

constexpr int kTile = 256;           // agents per work tile
constexpr int kBoxTile = 1024;       // boxes per scan tile (256 threads x 4)
constexpr int kMaxSims = 4096;
constexpr int kDimX = 2048, kDimY = 2048, kDimZ = 1024;  // packed box key 11/11/10 bits

// per-agent flag bits (flags[]): static for the coming iteration, position
// buffers differ, and what changed in the last iteration (moved, grew,
// divided, new) -- kept in the flags so they follow the Morton re-sort.
constexpr uint8_t kStatic = 1;
constexpr uint8_t kBufDiff = 2;
constexpr uint8_t kMoved = 4, kGrew = 8, kDivided = 16, kNew = 32;
constexpr uint8_t kChgMask = kMoved | kGrew | kDivided | kNew;
constexpr uint8_t kDead = 64;  // removed at the end of this iteration (Algorithm 2)

// Sweep payload of one agent: its centre relative to the origin of its grid
// box in fixed point, units of U = L 2^-kFixBits (exact integer offsets
// between boxes), and its radius in units of U (FP32).
constexpr int kFixBits = 28;
struct alignas(16) Pay {
    int32_t x, y, z;
    float r;
};

// error bits (SimDesc::err, Ctl::err)
constexpr int kErrCapacity = 1, kErrNonfinite = 2, kErrGrid = 4;

struct alignas(256) SimDesc {
    // set at creation
    int64_t a_off, cap;      // agent range
    int64_t b_off, box_cap;  // box-slot range (count, dirty, arrive) and block tables (brank, blist)
    int64_t sb_off;          // box_start range: box_cap + 1 entries
    double dt, k, gamma, adherence, mass, max_disp, box_len, div_vol, shift_frac;
    int32_t detect_static, resort_every;
    uint64_t seed;
    uint32_t sim_id, flags;
    double brownian_rate, death_prob, division_prob;  // Algorithm 2 cell behaviour
    int32_t min_age;
    // dynamic
    int64_t n, n_start, next_uid, n_div;
    int64_t n_dead;  // cells removed at the end of this iteration
    double lo[3], hi[3], L;
    double L_prev;  // box length of the previous grid (static rule radius)
    int32_t dims[3];
    int32_t err;
    int64_t nboxes;        // box slots in use: 64 per aligned 4x4x4 block (edge blocks padded)
    int32_t bdims[3];      // blocks per axis, ceil(dims / 4)
    int32_t dims_prev[3];  // dims of the block-rank tables
    int32_t remap;         // the tables must be rebuilt for new dims
    int64_t nblocks;       // aligned 4x4x4 box blocks (sweep work units)
    double rmax;           // largest agent radius at the start of the iteration
    unsigned int nonfinite;
    float kU, gU;  // k U and gamma U (U = L 2^-kFixBits in um): Eq 4.1 with lengths in units of U
};

constexpr int kBndSlots = 64;  // spread of the bounds atomics (slots per simulation)
constexpr int kBlk = 4;        // aligned blocks of kBlk^3 boxes: box order and sweep work unit

struct alignas(256) Ctl {
    int64_t iter;
    int32_t pos_par, lay_par;
    int32_t err;
    int32_t abort;
    uint32_t n_fix;
    uint32_t n_fp64_last;  // agents the FP64 path decided in the last iteration
    unsigned long long n_dense;  // (unit, core box, pass group) items queued for the box-wise sweep
    int64_t total_tiles, total_btiles, total_utiles, total_units;
    int32_t resort_now;
    int32_t any_growth;
};

// Device pointers of one batch (passed by value to every kernel).
struct Dev {
    int n_sims;
    int resort_every;
    SimDesc *sims;
    Ctl *ctl;
    int64_t *tile_begin;   // n_sims + 1: prefix of agent tiles
    int64_t *btile_begin;  // n_sims + 1: prefix of box tiles
    int64_t *utile_begin;  // n_sims + 1: prefix of uid tiles
    int64_t *a_begin;      // n_sims + 1: agent range starts (for agent -> sim)
    int64_t *wblk_begin;   // n_sims + 1: prefix of sweep work units (box blocks)
    int64_t *mv_begin;     // n_sims + 1: prefix of the removals (movers of the compaction)
    unsigned long long *bnd;  // n_sims x kBndSlots x 7 bounds accumulators
    uint32_t *blist;       // per simulation: packed block coords in Morton order
    double *pos[2];        // each 3*A: x block, y block, z block
    double *diam[2], *vol[2], *growth[2];
    uint64_t *uid[2];
    uint8_t *flags[2], *nz[2];
    int32_t *birth[2];  // iteration at whose start the agent was first present (age = iteration - birth)
    uint8_t *stage8;  // byte staging for host transfers (free between steps)
    uint32_t *key, *rank;
    Pay *payload;
    uint32_t *sorted_idx;
    int32_t *nbr, *contacts;
    double *force, *disp;  // 3*A interleaved
    int64_t *boxid;
    uint32_t *count, *box_start;  // indexed by the Morton rank of the box (box slot)
    uint32_t *brank;              // linear block id -> Morton rank of the block
    uint8_t *dirty;   // boxes holding the start position of a changed agent
    uint8_t *arrive;  // boxes of the new grid holding a changed agent
    uint8_t *dirty_blk, *arrive_blk;  // the same marks per aligned 4x4x4 block (index: box slot / 64)
    uint8_t *active_blk;  // blocks of the current grid holding an agent the next sweep must visit
    uint8_t *near_blk;    // a dirty (or arrival) mark in the block or one of its 26 neighbours
    uint32_t *tile_sum, *tile_off;
    uint32_t *rm_sum, *rm_off;  // per agent tile: removals, and their exclusive prefix per simulation
    uint32_t *fix_list;
    uint64_t *dense_list;  // box-wise sweep items: unit << 9 | core box << 3 | pass group
    int64_t dense_cap;     // entries of dense_list
    uint32_t *divflag, *divrank;
    double *stat_part;  // per agent tile: 6 doubles
    unsigned int *hist_cnt;  // n_sims x 32
    int64_t A;             // total agent capacity
};

// ---------------------------------------------------------------- helpers
__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Tile t -> simulation (tile prefix `begin` has n_sims + 1 entries, begin[0] = 0).
__device__ inline int find_sim(const int64_t *__restrict__ begin, int n_sims, int64_t t) {
    int lo = 0, hi = n_sims;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (begin[mid] <= t) lo = mid; else hi = mid;
    }
    return lo;
}

// Order-preserving map of doubles to unsigned integers (for atomic min/max).
__device__ inline unsigned long long enc_double(double v) {
    unsigned long long b = __double_as_longlong(v);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__host__ __device__ inline double dec_double(unsigned long long e) {
    unsigned long long b = (e >> 63) ? (e & 0x7fffffffffffffffull) : ~e;
    double v;
    memcpy(&v, &b, sizeof v);
    return v;
}

// Box coordinate of v (floor((v-lo)/L), clamped to [0, dim-1]), FP64 division.
__device__ inline int box_coord(double v, double lo, double L, int dim) {
    double q = floor((v - lo) / L);
    int b = (int)q;
    if (q < 0.0) b = 0;
    if (q > (double)(dim - 1)) b = dim - 1;
    return b;
}

__device__ inline uint32_t pack_key(int bx, int by, int bz) {
    return (uint32_t)bx | ((uint32_t)by << 11) | ((uint32_t)bz << 22);
}
__device__ inline void unpack_key(uint32_t k, int &bx, int &by, int &bz) {
    bx = (int)(k & 2047u);
    by = (int)((k >> 11) & 2047u);
    bz = (int)(k >> 22);
}
__device__ inline int64_t linear_box(int bx, int by, int bz, const int32_t dims[3]) {
    return (int64_t)bx + (int64_t)dims[0] * ((int64_t)by + (int64_t)dims[1] * (int64_t)bz);
}

// Payload coordinate of an agent: its offset from the origin of its box in
// units of U = L 2^-kFixBits, rounded to the nearest integer (in [0, 2^28]
// for an agent inside its box).  The FP64 offset and the division by L are
// exact to about 2^-52 relative; the rounding to an integer is the only
// error of note (at most U/2).
__device__ inline int32_t fix_coord(double v, double lo, double L, int b) {
    const double origin = lo + (double)b * L;
    return (int32_t)rint(ldexp((v - origin) / L, kFixBits));
}
// Radius of an agent of diameter dm in units of U (FP32, relative error 2^-24).
__device__ inline float fix_radius(double dm, double L) { return (float)ldexp(0.5 * dm / L, kFixBits); }

// Error message of the last failed call on this thread (abm_last_error).
void clear_error();
int set_error(int code, const char *msg);

// Launch schedule of the force sweep (picked by the autotuner): persistent
// work groups of the unit sweep, and work groups and waves per work group of
// the box-wise sweep (multiples of 8 work groups: one share per XCD).
struct Sched {
    int sweep_grid = 2048;
    int dense_grid = 1024;
    int dense_waves = 4;  // 2 or 4
};

// Host-side launch helpers implemented in the .hip files.
void launch_iteration(const Dev &d, hipStream_t s, int grid_agents, int grid_boxes, const Sched &sc, bool diag,
                      bool any_growth, bool any_static, bool resort, bool any_death, bool any_record);
void launch_grid_build(const Dev &d, hipStream_t s, int grid_agents, int grid_boxes, bool any_static);
void launch_sweep(const Dev &d, hipStream_t s, const Sched &sc, bool diag, bool any_static);
void launch_after_sweep(const Dev &d, hipStream_t s, int grid_agents, int grid_boxes, bool diag, bool any_growth,
                        bool any_static, bool resort, bool any_death, bool any_record);
void launch_resort(const Dev &d, hipStream_t s, int grid_agents, int grid_boxes, bool force, bool any_static);
void launch_end(const Dev &d, hipStream_t s, int grid_boxes, bool any_static);
void launch_near_marks(const Dev &d, hipStream_t s, int grid_boxes, bool arrivals);
void launch_stats(const Dev &d, hipStream_t s, int grid_agents, double hist_rmax, double *out_dev);
void launch_gather_pos(const Dev &d, hipStream_t s, int sim, double *dst, int64_t n, int64_t a_off);
void launch_scatter_init(const Dev &d, hipStream_t s, int grid_agents);

}  // namespace abm
