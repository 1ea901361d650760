// abm_grid.hip -- uniform grid of the agents (Sec 4.4.3, Sec 5.3.1), the
// periodic Morton-order re-sort of agent storage (Sec 5.4.2) and statistics.
//
// The grid is a counting sort of agents by the Morton rank of their box:
//   begin    per-simulation counters and agent-tile prefix
//   bounds   open boundary: min/max of positions and largest diameter (Sec 4.4.11)
//   grid     box length, dims; Morton tables are rebuilt when the dims change
//   brank    linear block id -> Morton rank of the block; Morton list of blocks
//   bin      per-box counts with arrival rank (slot order = Morton order of boxes)
//   scan_*   per-box exclusive scan -> slot start of every box
//   scatter  box-ordered FP32 payload (box-relative centre, radius) + agent index
// The force sweep (abm_mech.hip) reads the payload block by block.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "abm_device.h"

namespace abm {

// ------------------------------------------------------------------ begin
__global__ void k_begin(Dev d) {
    if (ABM_ABORTED(d)) return;
    for (int s = threadIdx.x; s < d.n_sims; s += blockDim.x) {
        SimDesc &S = d.sims[s];
        S.n_start = S.n;
        S.n_div = 0;
        S.n_dead = 0;
        S.nonfinite = 0;
        S.L_prev = S.L;
    }
    for (int q = threadIdx.x; q < d.n_sims * kBndSlots; q += blockDim.x) {
        unsigned long long *b = d.bnd + 7 * (size_t)q;
        for (int a = 0; a < 6; ++a) b[a] = ~0ull;  // min of x, y, z, -x, -y, -z (encoded)
        b[6] = 0ull;                               // max of the diameter (encoded)
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int s = 0; s < d.n_sims; ++s) {
            d.tile_begin[s] = t;
            t += ceil_div(d.sims[s].n_start, kTile);
        }
        d.tile_begin[d.n_sims] = t;
        d.ctl->total_tiles = t;
        d.ctl->n_fp64_last = d.ctl->n_fix;
        d.ctl->n_fix = 0;
        d.ctl->n_dense = 0;
    }
}

// ------------------------------------------------------------------ bounds
// Each block reduces all its tiles of one simulation before touching global
// memory, then updates one of kBndSlots accumulator copies (spreads the atomics).
__device__ inline void bounds_flush(const Dev &d, int s, double acc[7], double (*red)[4]) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int off = 32; off > 0; off >>= 1) {
        for (int a = 0; a < 6; ++a) acc[a] = fmin(acc[a], __shfl_xor(acc[a], off));
        acc[6] = fmax(acc[6], __shfl_xor(acc[6], off));
    }
    if (lane == 0)
        for (int a = 0; a < 7; ++a) red[a][wid] = acc[a];
    __syncthreads();
    if (threadIdx.x < 7) {
        int a = threadIdx.x;
        double v = red[a][0];
        for (int w = 1; w < 4; ++w) v = a < 6 ? fmin(v, red[a][w]) : fmax(v, red[a][w]);
        unsigned long long *b = d.bnd + 7 * ((size_t)s * kBndSlots + (blockIdx.x % kBndSlots));
        if (a < 6) {
            if (v < __builtin_huge_val()) atomicMin(&b[a], enc_double(v));
        } else if (v > -__builtin_huge_val()) {
            atomicMax(&b[6], enc_double(v));
        }
    }
    __syncthreads();
    for (int a = 0; a < 6; ++a) acc[a] = __builtin_huge_val();
    acc[6] = -__builtin_huge_val();
}

// (sims, tiles: read through non-aliased pointers, so that their wave-uniform
// reads are scalar loads; the only write to a descriptor, the non-finite flag,
// goes through d.sims to a field that is never read here)
__global__ void __launch_bounds__(256) k_bounds(Dev d, const SimDesc *__restrict__ sims,
                                                const int64_t *__restrict__ tiles) {
    if (ABM_ABORTED(d)) return;
    __shared__ double red[7][4];
    const int P = d.ctl->pos_par, lp = d.ctl->lay_par;
    const int64_t A = d.A;
    const int64_t total = d.ctl->total_tiles;
    double acc[7];
    for (int a = 0; a < 6; ++a) acc[a] = __builtin_huge_val();
    acc[6] = -__builtin_huge_val();
    int cur = -1;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int s = find_sim(tiles, d.n_sims, t);
        if (s != cur && cur >= 0) bounds_flush(d, cur, acc, red);
        cur = s;
        const SimDesc &S = sims[s];
        int64_t loc = (t - tiles[s]) * kTile + threadIdx.x;
        if (loc < S.n_start) {
            int64_t i = S.a_off + loc;
            double x = d.pos[P][i], y = d.pos[P][A + i], z = d.pos[P][2 * A + i];
            double dm = d.diam[lp][i];
            if (!(isfinite(x) && isfinite(y) && isfinite(z) && isfinite(dm))) atomicOr(&d.sims[s].nonfinite, 1u);
            acc[0] = fmin(acc[0], x);
            acc[1] = fmin(acc[1], y);
            acc[2] = fmin(acc[2], z);
            acc[3] = fmin(acc[3], -x);
            acc[4] = fmin(acc[4], -y);
            acc[5] = fmin(acc[5], -z);
            acc[6] = fmax(acc[6], dm);
        }
    }
    if (cur >= 0) bounds_flush(d, cur, acc, red);
}

// ------------------------------------------------------------------ grid
__global__ void k_grid(Dev d) {
    if (ABM_ABORTED(d)) return;
    for (int s = threadIdx.x; s < d.n_sims; s += blockDim.x) {
        SimDesc &S = d.sims[s];
        if (S.nonfinite) {
            S.err |= kErrNonfinite;
            atomicOr(&d.ctl->err, kErrNonfinite);
            atomicExch(&d.ctl->abort, 1);
        }
        if (S.n_start == 0) {
            S.nboxes = 0;
            S.nblocks = 0;
            S.dims[0] = S.dims[1] = S.dims[2] = 0;
            S.remap = 0;
            continue;
        }
        unsigned long long e[7];
        for (int a = 0; a < 6; ++a) e[a] = ~0ull;
        e[6] = 0ull;
        for (int q = 0; q < kBndSlots; ++q) {
            const unsigned long long *b = d.bnd + 7 * ((size_t)s * kBndSlots + q);
            for (int a = 0; a < 6; ++a) e[a] = b[a] < e[a] ? b[a] : e[a];
            e[6] = b[6] > e[6] ? b[6] : e[6];
        }
        double L = S.box_len > 0.0 ? S.box_len : dec_double(e[6]);
        S.L = L;
        int64_t nbl = 1;
        bool bad = !(L > 0.0);
        for (int a = 0; a < 3; ++a) {
            S.lo[a] = dec_double(e[a]);
            S.hi[a] = -dec_double(e[3 + a]);
            double q = floor((S.hi[a] - S.lo[a]) / L) + 1.0;
            int lim = a == 2 ? kDimZ : (a == 1 ? kDimY : kDimX);
            if (!(q <= (double)lim)) {
                bad = true;
                q = 1.0;
            }
            S.dims[a] = (int32_t)q;
            S.bdims[a] = (int32_t)ceil_div((int64_t)q, kBlk);
            nbl *= (int64_t)S.bdims[a];
        }
        int64_t nb = nbl * kBlk * kBlk * kBlk;  // box slots
        if (bad || nb > S.box_cap) {
            S.err |= kErrGrid;
            atomicOr(&d.ctl->err, kErrGrid);
            atomicExch(&d.ctl->abort, 1);
            nb = 0;
            nbl = 0;
        }
        S.nboxes = nb;
        S.nblocks = nbl;
        S.remap = (S.dims[0] != S.dims_prev[0] || S.dims[1] != S.dims_prev[1] || S.dims[2] != S.dims_prev[2]) ? 1 : 0;
        // Eq 4.1 in units of U = L 2^-kFixBits: F_N = kU delta_U - gU sqrt(rbar_U delta_U)
        S.kU = (float)(S.k * ldexp(L, -kFixBits));
        S.gU = (float)(S.gamma * ldexp(L, -kFixBits));
        S.rmax = 0.5 * dec_double(e[6]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0, u = 0;
        for (int s = 0; s < d.n_sims; ++s) {
            d.btile_begin[s] = t;
            t += ceil_div(d.sims[s].nboxes, kBoxTile);
            d.wblk_begin[s] = u;
            u += d.sims[s].nblocks;
        }
        d.btile_begin[d.n_sims] = t;
        d.wblk_begin[d.n_sims] = u;
        d.ctl->total_btiles = t;
        d.ctl->total_units = u;
    }
}

// Morton rank of every aligned 4^3 block and the Morton-ordered block list;
// only for simulations whose grid dims changed.
__global__ void __launch_bounds__(256) k_brank(Dev d) {
    if (ABM_ABORTED(d)) return;
    const int64_t total = d.ctl->total_btiles;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int s = find_sim(d.btile_begin, d.n_sims, t);
        const SimDesc &S = d.sims[s];
        if (!S.remap) continue;
        int64_t k0 = (t - d.btile_begin[s]) * kBoxTile;
        for (int q = threadIdx.x; q < kBoxTile; q += blockDim.x) {
            int64_t k = k0 + q;
            if (k >= S.nblocks) break;
            int qx = (int)(k % S.bdims[0]);
            int64_t r = k / S.bdims[0];
            int qy = (int)(r % S.bdims[1]);
            int qz = (int)(r / S.bdims[1]);
            const uint32_t m = morton_rank(qx, qy, qz, S.bdims);
            d.brank[S.b_off + k] = m;
            d.blist[S.b_off + m] = pack_key(qx, qy, qz);
        }
    }
}

__global__ void k_grid_done(Dev d) {
    for (int s = threadIdx.x; s < d.n_sims; s += blockDim.x) {
        SimDesc &S = d.sims[s];
        for (int a = 0; a < 3; ++a) S.dims_prev[a] = S.dims[a];
        S.remap = 0;
    }
}

// ------------------------------------------------------------------ bin
// (sims, tiles: the descriptors and the tile prefix, read-only and not
// aliased, so that their wave-uniform reads are scalar loads)
__global__ void __launch_bounds__(256) k_bin(Dev d, const SimDesc *__restrict__ sims,
                                             const int64_t *__restrict__ tiles) {
    if (ABM_ABORTED(d)) return;
    const int P = d.ctl->pos_par, lp = d.ctl->lay_par;
    const int64_t A = d.A;
    const int64_t total = d.ctl->total_tiles;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int s = find_sim(tiles, d.n_sims, t);
        const SimDesc &S = sims[s];
        const int64_t loc = (t - tiles[s]) * kTile + threadIdx.x;
        const bool valid = loc < S.n_start;  // the invalid lanes are the last of the tile
        const int64_t i = S.a_off + (valid ? loc : 0);
        uint32_t m = 0;
        int bx = 0, by = 0, bz = 0;
        if (valid) {
            const double L = S.L;
            bx = box_coord(d.pos[P][i], S.lo[0], L, S.dims[0]);
            by = box_coord(d.pos[P][A + i], S.lo[1], L, S.dims[1]);
            bz = box_coord(d.pos[P][2 * A + i], S.lo[2], L, S.dims[2]);
            m = box_rank(d, S, bx, by, bz);
        }
        const uint32_t r = run_atomic_add(d.count + S.b_off, m, valid);
        if (!valid) continue;
        d.key[i] = pack_key(bx, by, bz);
        d.rank[i] = r;
        if (S.detect_static) {
            const uint8_t fl = d.flags[lp][i];
            if (fl & kChgMask) mark_box(d.arrive, d.arrive_blk, S, m);
            // the next sweep visits the block unless its agents are static and settled
            if (!(fl & kStatic) || (fl & (kBufDiff | kChgMask))) d.active_blk[S.b_off + (m >> 6)] = 1;
        }
    }
}

// ------------------------------------------------------------------ segmented scan
// Exclusive scan of per-box counts (Morton-rank order) into slot starts.
// The scan kernels serve the grid build (resort = 0) and the Morton re-sort
// (resort = 1: they do nothing in iterations without a re-sort).
// Four consecutive box counts of a thread: one 16-byte load where the four
// lie in range and the address is 16-byte aligned (box ranges of a batch
// start at arbitrary offsets), else one by one.
__device__ inline void load_counts4(const uint32_t *count, int64_t at, int64_t k0, int64_t nboxes, uint32_t v[4]) {
    if (k0 + 4 <= nboxes && (at & 3) == 0) {
        const uint4 c = *reinterpret_cast<const uint4 *>(count + at);
        v[0] = c.x;
        v[1] = c.y;
        v[2] = c.z;
        v[3] = c.w;
    } else {
        for (int q = 0; q < 4; ++q) v[q] = (k0 + q < nboxes) ? count[at + q] : 0u;
    }
}

// (sims, btiles: the descriptors and the box-tile prefix, read-only and not
// aliased, so that their wave-uniform reads are scalar loads)
__global__ void __launch_bounds__(256) k_scan_tiles(Dev d, const SimDesc *__restrict__ sims,
                                                    const int64_t *__restrict__ btiles, int resort) {
    if (ABM_ABORTED(d) || (resort && !d.ctl->resort_now)) return;
    __shared__ uint32_t sh[4];
    const int64_t total = d.ctl->total_btiles;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int s = find_sim(btiles, d.n_sims, t);
        const SimDesc &S = sims[s];
        int64_t k0 = (t - btiles[s]) * kBoxTile + threadIdx.x * 4;
        uint32_t v[4];
        load_counts4(d.count, S.b_off + k0, k0, S.nboxes, v);
        uint32_t tot;
        block_excl_scan_4(v, sh, tot);
        if (threadIdx.x == 0) d.tile_sum[t] = tot;
    }
}

// One block: per simulation, exclusive scan of the tile sums (tiles in order).
__device__ inline void scan_tile_sums(const Dev &d, const int64_t *begin) {
    __shared__ uint32_t sh[16];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int s = 0; s < d.n_sims; ++s) {
        int64_t b0 = begin[s], b1 = begin[s + 1];
        uint32_t carry = 0;
        for (int64_t c = b0; c < b1; c += blockDim.x) {
            int64_t t = c + threadIdx.x;
            uint32_t v = t < b1 ? d.tile_sum[t] : 0u;
            uint32_t x = v;
            for (int off = 1; off < 64; off <<= 1) {
                uint32_t y = __shfl_up(x, off);
                if (lane >= off) x += y;
            }
            if (lane == 63) sh[wid] = x;
            __syncthreads();
            uint32_t wpre = 0, tot = 0;
            for (int w = 0; w < 16; ++w) {
                if (w < wid) wpre += sh[w];
                tot += sh[w];
            }
            if (t < b1) d.tile_off[t] = carry + wpre + x - v;
            carry += tot;
            __syncthreads();
        }
    }
}

__global__ void __launch_bounds__(1024) k_scan_top(Dev d, int resort) {
    if (ABM_ABORTED(d) || (resort && !d.ctl->resort_now)) return;
    scan_tile_sums(d, d.btile_begin);
}

// box_start[sb_off + m] = a_off + prefix; zeroes the counts.
__global__ void __launch_bounds__(256) k_scan_apply(Dev d, const SimDesc *__restrict__ sims,
                                                    const int64_t *__restrict__ btiles, int resort) {
    if (ABM_ABORTED(d) || (resort && !d.ctl->resort_now)) return;
    __shared__ uint32_t sh[4];
    const int64_t total = d.ctl->total_btiles;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int s = find_sim(btiles, d.n_sims, t);
        const SimDesc &S = sims[s];
        int64_t k0 = (t - btiles[s]) * kBoxTile + threadIdx.x * 4;
        uint32_t v[4];
        load_counts4(d.count, S.b_off + k0, k0, S.nboxes, v);
        uint32_t tot;
        uint32_t pre = block_excl_scan_4(v, sh, tot);
        const uint32_t base = (uint32_t)S.a_off + d.tile_off[t] + pre;
        const uint32_t st[4] = {base, base + v[0], base + v[0] + v[1], base + v[0] + v[1] + v[2]};
        const bool full = k0 + 4 <= S.nboxes;
        if (full && ((S.sb_off + k0) & 3) == 0) {
            *reinterpret_cast<uint4 *>(d.box_start + S.sb_off + k0) = make_uint4(st[0], st[1], st[2], st[3]);
        } else {
            for (int q = 0; q < 4; ++q)
                if (k0 + q < S.nboxes) d.box_start[S.sb_off + k0 + q] = st[q];
        }
        if (full && ((S.b_off + k0) & 3) == 0) {
            *reinterpret_cast<uint4 *>(d.count + S.b_off + k0) = make_uint4(0u, 0u, 0u, 0u);
        } else {
            for (int q = 0; q < 4; ++q)
                if (k0 + q < S.nboxes) d.count[S.b_off + k0 + q] = 0u;
        }
        if (t == btiles[s + 1] - 1 && threadIdx.x == 0)
            d.box_start[S.sb_off + S.nboxes] = (uint32_t)(S.a_off + S.n_start);
    }
}

// ------------------------------------------------------------------ scatter
__global__ void __launch_bounds__(256) k_scatter(Dev d, const SimDesc *__restrict__ sims,
                                                 const int64_t *__restrict__ tiles) {
    if (ABM_ABORTED(d)) return;
    const int P = d.ctl->pos_par, lp = d.ctl->lay_par;
    const int64_t A = d.A;
    const int64_t total = d.ctl->total_tiles;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int s = find_sim(tiles, d.n_sims, t);
        const SimDesc &S = sims[s];
        int64_t loc = (t - tiles[s]) * kTile + threadIdx.x;
        if (loc >= S.n_start) continue;
        int64_t i = S.a_off + loc;
        int bx, by, bz;
        unpack_key(d.key[i], bx, by, bz);
        uint32_t m = box_rank(d, S, bx, by, bz);
        uint32_t slot = d.box_start[S.sb_off + m] + d.rank[i];
        Pay p;
        p.x = fix_coord(d.pos[P][i], S.lo[0], S.L, bx);
        p.y = fix_coord(d.pos[P][A + i], S.lo[1], S.L, by);
        p.z = fix_coord(d.pos[P][2 * A + i], S.lo[2], S.L, bz);
        p.r = fix_radius(d.diam[lp][i], S.L);
        d.payload[slot] = p;
        d.sorted_idx[slot] = (uint32_t)i;
    }
}

// ------------------------------------------------------------------ static rule, arrivals
// After the grid of the committed positions is built: a static agent stops
// being static when a changed agent (including a new daughter) lies within
// the previous iteration's radius of it (Sec 5.5).  Boxes holding a changed
// agent were marked by k_bin.
// One wave per aligned block; only blocks next to an arrival can lose a
// static flag (or every block, when the box length shrank).
// Each wave checks 64 aligned blocks at a time, one per lane, strided by the
// number of waves of the grid (so that blocks to visit spread over all waves,
// one per wave when there are few): whether a block needs a visit; the wave
// then visits those blocks.
// (sims, btiles: read-only and not aliased, so that their wave-uniform reads
// are scalar loads.)
__global__ void __launch_bounds__(256) k_static_fix(Dev d, const SimDesc *__restrict__ sims,
                                                    const int64_t *__restrict__ btiles) {
    if (ABM_ABORTED(d)) return;
    constexpr int kTB = kBoxTile / 64;
    const int P = d.ctl->pos_par, lp = d.ctl->lay_par;
    const int64_t A = d.A;
    const int64_t nq = d.ctl->total_btiles * kTB;
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * 4;  // waves of the grid
    for (int64_t q0 = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); q0 < nq; q0 += 64 * nw) {
        const int64_t qc = q0 + lane * nw;  // the block this lane checks
        bool need = false;
        if (qc < nq) {
            const int64_t tl = qc / kTB;
            const int sl = find_sim(btiles, d.n_sims, tl);
            const SimDesc &Sl = sims[sl];
            const int64_t bl = (tl - btiles[sl]) * kTB + qc % kTB;
            // a shrunken grid cannot cover the old radius: every block is visited
            need = Sl.detect_static && bl < Sl.nblocks && (!(Sl.L >= Sl.L_prev) || d.near_blk[Sl.b_off + bl]);
        }
        for (uint64_t mv = __builtin_amdgcn_ballot_w64(need); mv; mv &= mv - 1) {
            const int64_t q = q0 + (__ffsll((long long)mv) - 1) * nw;
            const int64_t t = q / kTB;
            int s = find_sim(btiles, d.n_sims, t);
            const SimDesc &S = sims[s];
            const int64_t blk = (t - btiles[s]) * kTB + q % kTB;
            const bool shrunk = !(S.L >= S.L_prev);  // a shrunken grid cannot cover the old radius: be conservative
            const uint32_t s0 = d.box_start[S.sb_off + blk * 64], s1 = d.box_start[S.sb_off + blk * 64 + 64];
            for (uint32_t slot0 = s0; slot0 < s1; slot0 += 64) {
                const uint32_t slot = slot0 + (uint32_t)lane;
                if (slot >= s1) continue;
                const int64_t i = d.sorted_idx[slot];
                const uint8_t fl = d.flags[lp][i];
                if (!(fl & kStatic)) continue;
                bool st = !shrunk;
                int bx, by, bz;
                unpack_key(d.key[i], bx, by, bz);
                if (st) {
                    const double x = d.pos[P][i], y = d.pos[P][A + i], z = d.pos[P][2 * A + i];
                    const double L2 = S.L_prev * S.L_prev;
                    for (int oz = -1; oz <= 1 && st; ++oz)
                        for (int oy = -1; oy <= 1 && st; ++oy)
                            for (int ox = -1; ox <= 1 && st; ++ox) {
                                int cx = bx + ox, cy = by + oy, cz = bz + oz;
                                if (cx < 0 || cy < 0 || cz < 0 || cx >= S.dims[0] || cy >= S.dims[1] || cz >= S.dims[2])
                                    continue;
                                uint32_t m = box_rank(d, S, cx, cy, cz);
                                if (!d.arrive[S.b_off + m]) continue;
                                uint32_t b0 = d.box_start[S.sb_off + m], b1 = d.box_start[S.sb_off + m + 1];
                                for (uint32_t sl = b0; sl < b1 && st; ++sl) {
                                    int64_t j = d.sorted_idx[sl];
                                    if (j == i || !(d.flags[lp][j] & kChgMask)) continue;
                                    if (near_point(x, y, z, d.pos[P][j], d.pos[P][A + j], d.pos[P][2 * A + j], L2))
                                        st = false;
                                }
                            }
                }
                if (!st) {
                    d.flags[lp][i] = fl & ~kStatic;
                    d.active_blk[S.b_off + blk] = 1;
                }
            }
        }
    }
}

// near_blk[b] = any dirty (or arrival) mark in block b or its 26 neighbours:
// a static agent whose block is not near a mark has no changed agent within
// one box of it.  One thread per block (block tiles of 16 blocks).
__global__ void __launch_bounds__(256) k_near_marks(Dev d, int arrivals) {
    if (ABM_ABORTED(d)) return;
    constexpr int kTB = kBoxTile / 64;  // aligned blocks per box tile
    const int64_t total = d.ctl->total_btiles;
    const uint8_t *marks = arrivals ? d.arrive_blk : d.dirty_blk;
    // one thread per aligned block: 256 / kTB box tiles per pass of a thread block
    for (int64_t t0 = (int64_t)blockIdx.x * (256 / kTB); t0 < total; t0 += (int64_t)gridDim.x * (256 / kTB)) {
        const int64_t t = t0 + threadIdx.x / kTB;
        if (t >= total) continue;
        int s = find_sim(d.btile_begin, d.n_sims, t);
        const SimDesc &S = d.sims[s];
        if (!S.detect_static) continue;
        const int64_t blk = (t - d.btile_begin[s]) * kTB + threadIdx.x % kTB;
        if (blk >= S.nblocks) continue;
        int qx, qy, qz;
        unpack_key(d.blist[S.b_off + blk], qx, qy, qz);
        uint8_t any = 0;
        for (int oz = -1; oz <= 1; ++oz)
            for (int oy = -1; oy <= 1; ++oy)
                for (int ox = -1; ox <= 1; ++ox) {
                    const int cx = qx + ox, cy = qy + oy, cz = qz + oz;
                    if (cx < 0 || cy < 0 || cz < 0 || cx >= S.bdims[0] || cy >= S.bdims[1] || cz >= S.bdims[2]) continue;
                    const int64_t lin = (int64_t)cx + (int64_t)S.bdims[0] * ((int64_t)cy + (int64_t)S.bdims[1] * cz);
                    any |= marks[S.b_off + d.brank[S.b_off + lin]];
                }
        d.near_blk[S.b_off + blk] = any;
    }
}

// Clears the dirty and arrival marks of the current grid: the 64 box marks
// of every marked block, then the block marks (a box tile holds 16 blocks).
// (sims, btiles: read-only and not aliased, so that their wave-uniform reads
// are scalar loads)
__global__ void __launch_bounds__(256) k_clear_marks(Dev d, const SimDesc *__restrict__ sims,
                                                     const int64_t *__restrict__ btiles) {
    if (ABM_ABORTED(d)) return;
    const int64_t total = d.ctl->total_btiles;
    const int q = threadIdx.x >> 4, e = threadIdx.x & 15;  // block of the tile, 16 threads per block
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int s = find_sim(btiles, d.n_sims, t);
        const SimDesc &S = sims[s];
        if (!S.detect_static) continue;
        const int64_t blk = (t - btiles[s]) * (kBoxTile / 64) + q;
        if (blk >= S.nblocks) continue;
        const int64_t bi = S.b_off + blk;
        if (!d.dirty_blk[bi] && !d.arrive_blk[bi]) continue;
        for (int k = e; k < 64; k += 16) {
            d.dirty[S.b_off + blk * 64 + k] = 0;
            d.arrive[S.b_off + blk * 64 + k] = 0;
        }
    }
    __syncthreads();
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int s = find_sim(btiles, d.n_sims, t);
        const SimDesc &S = sims[s];
        if (!S.detect_static || e != 0) continue;
        const int64_t blk = (t - btiles[s]) * (kBoxTile / 64) + q;
        if (blk >= S.nblocks) continue;
        d.dirty_blk[S.b_off + blk] = 0;
        d.arrive_blk[S.b_off + blk] = 0;
        d.active_blk[S.b_off + blk] = 0;
    }
}

// ------------------------------------------------------------------ end of iteration
__global__ void k_end(Dev d) {
    if (ABM_ABORTED(d)) return;
    for (int s = threadIdx.x; s < d.n_sims; s += blockDim.x) {
        SimDesc &S = d.sims[s];
        S.n = S.n_start + S.n_div - S.n_dead;
        S.next_uid += S.n_div;
        S.n_start = S.n;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        d.ctl->pos_par ^= 1;
        d.ctl->iter += 1;
        int64_t t = 0;
        for (int s = 0; s < d.n_sims; ++s) {
            d.tile_begin[s] = t;
            t += ceil_div(d.sims[s].n, kTile);
        }
        d.tile_begin[d.n_sims] = t;
        d.ctl->total_tiles = t;
        d.ctl->resort_now = (d.resort_every > 0 && d.ctl->iter % d.resort_every == 0) ? 1 : 0;
    }
}

// ------------------------------------------------------------------ Morton re-sort
// Every R iterations agents are moved into the Morton order of their box in
// the grid of the iteration just finished (a counting sort by Morton rank:
// one radix digit of the size of the grid).  The next grid then finds agents
// already in slot order, so the sweep's own-agent reads and writes coalesce.
__global__ void k_force_resort(Dev d) {
    if (threadIdx.x == 0) d.ctl->resort_now = 1;
}

__global__ void __launch_bounds__(256) k_rs_count(Dev d) {
    if (ABM_ABORTED(d) || !d.ctl->resort_now) return;
    const int P = d.ctl->pos_par;
    const int64_t A = d.A;
    const int64_t total = d.ctl->total_tiles;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int s = find_sim(d.tile_begin, d.n_sims, t);
        const SimDesc &S = d.sims[s];
        if (S.nboxes == 0) continue;  // uniform over the block
        const int64_t loc = (t - d.tile_begin[s]) * kTile + threadIdx.x;
        const bool valid = loc < S.n;  // the invalid lanes are the last of the tile
        const int64_t i = S.a_off + (valid ? loc : 0);
        const uint32_t m = valid ? box_rank_of(d, S, d.pos[P][i], d.pos[P][A + i], d.pos[P][2 * A + i]) : 0u;
        const uint32_t r = run_atomic_add(d.count + S.b_off, m, valid);
        if (!valid) continue;
        d.key[i] = m;
        d.rank[i] = r;
    }
}

// The move is a gather: k_rs_dest writes the source of every destination
// slot into sorted_idx (rebuilt by the grid build that follows), and
// k_rs_move copies each destination's fields from its source, so that the
// writes are coalesced.  Out of place: the source buffers are only read.
// Positions land in the other position buffer only, so every agent is
// marked as having differing buffers.
__global__ void __launch_bounds__(256) k_rs_dest(Dev d) {
    if (ABM_ABORTED(d) || !d.ctl->resort_now) return;
    const int64_t total = d.ctl->total_tiles;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int s = find_sim(d.tile_begin, d.n_sims, t);
        const SimDesc &S = d.sims[s];
        int64_t loc = (t - d.tile_begin[s]) * kTile + threadIdx.x;
        if (loc >= S.n || S.nboxes == 0) continue;
        const int64_t i = S.a_off + loc;
        const int64_t j = (int64_t)d.box_start[S.sb_off + d.key[i]] + d.rank[i];
        d.sorted_idx[j] = (uint32_t)i;
    }
}

__global__ void __launch_bounds__(256) k_rs_move(Dev d) {
    if (ABM_ABORTED(d) || !d.ctl->resort_now) return;
    const int P = d.ctl->pos_par, lp = d.ctl->lay_par;
    const int64_t A = d.A;
    const int64_t total = d.ctl->total_tiles;
    const int nl = 1 - lp;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int s = find_sim(d.tile_begin, d.n_sims, t);
        const SimDesc &S = d.sims[s];
        int64_t loc = (t - d.tile_begin[s]) * kTile + threadIdx.x;
        if (loc >= S.n || S.nboxes == 0) continue;
        const int64_t j = S.a_off + loc;
        const int64_t i = d.sorted_idx[j];
        for (int a = 0; a < 3; ++a) d.pos[1 - P][a * A + j] = d.pos[P][a * A + i];
        d.diam[nl][j] = d.diam[lp][i];
        d.vol[nl][j] = d.vol[lp][i];
        d.growth[nl][j] = d.growth[lp][i];
        d.uid[nl][j] = d.uid[lp][i];
        d.flags[nl][j] = d.flags[lp][i] | kBufDiff;
        d.nz[nl][j] = d.nz[lp][i];
        d.birth[nl][j] = d.birth[lp][i];
    }
}

// After a re-sort of a simulation with static detection, both position
// buffers receive the new arrangement, so that static agents need no
// visit to settle differing buffers (runs before the parities flip).
__global__ void __launch_bounds__(256) k_rs_sync(Dev d) {
    if (ABM_ABORTED(d) || !d.ctl->resort_now) return;
    const int P = d.ctl->pos_par, lp = d.ctl->lay_par;  // buffers of the old arrangement
    const int64_t A = d.A;
    const int64_t total = d.ctl->total_tiles;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int s = find_sim(d.tile_begin, d.n_sims, t);
        const SimDesc &S = d.sims[s];
        if (!S.detect_static || S.nboxes == 0) continue;
        const int64_t loc = (t - d.tile_begin[s]) * kTile + threadIdx.x;
        if (loc >= S.n) continue;
        const int64_t i = S.a_off + loc;
        d.pos[P][i] = d.pos[1 - P][i];
        d.pos[P][A + i] = d.pos[1 - P][A + i];
        d.pos[P][2 * A + i] = d.pos[1 - P][2 * A + i];
        d.flags[1 - lp][i] &= (uint8_t)~kBufDiff;
    }
}

__global__ void k_rs_end(Dev d) {
    if (ABM_ABORTED(d) || !d.ctl->resort_now) return;
    if (threadIdx.x == 0) {
        d.ctl->lay_par ^= 1;
        d.ctl->pos_par ^= 1;
        d.ctl->resort_now = 0;
    }
}

// ------------------------------------------------------------------ statistics
// Deterministic two-level FP64 reductions: per-tile partials, then a fixed
// order per simulation.
__global__ void __launch_bounds__(256) k_stats_sum(Dev d, int pass, double *out) {
    __shared__ double red[3][4];
    __shared__ uint32_t hb[32];  // this tile's histogram counts
    const int P = d.ctl->pos_par;
    const int64_t A = d.A;
    const int64_t total = d.ctl->total_tiles;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int s = find_sim(d.tile_begin, d.n_sims, t);
        const SimDesc &S = d.sims[s];
        int64_t loc = (t - d.tile_begin[s]) * kTile + threadIdx.x;
        double v[3] = {0.0, 0.0, 0.0};
        if (pass == 1 && threadIdx.x < 32) hb[threadIdx.x] = 0u;
        __syncthreads();
        if (loc < S.n) {
            int64_t i = S.a_off + loc;
            double x = d.pos[P][i], y = d.pos[P][A + i], z = d.pos[P][2 * A + i];
            if (pass == 0) {
                v[0] = x;
                v[1] = y;
                v[2] = z;
            } else {
                const double *c = out + 40 * s;
                double ddx = x - c[0], ddy = y - c[1], ddz = z - c[2];
                double d2 = fma(ddz, ddz, fma(ddy, ddy, ddx * ddx));
                double r = sqrt(d2);
                v[0] = d2;
                v[1] = r;
                double w = c[3] / 32.0;
                int64_t b = (int64_t)floor(r / w);
                if (b > 31) b = 31;
                if (b < 0) b = 0;
                atomicAdd(&hb[b], 1u);
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            v[0] += __shfl_xor(v[0], off);
            v[2] += __shfl_xor(v[2], off);
            if (pass == 0) v[1] += __shfl_xor(v[1], off);
            else v[1] = fmax(v[1], __shfl_xor(v[1], off));
        }
        if (lane == 0)
            for (int a = 0; a < 3; ++a) red[a][wid] = v[a];
        __syncthreads();
        if (threadIdx.x == 0) {
            double a0 = red[0][0], a1 = red[1][0], a2 = red[2][0];
            for (int w = 1; w < 4; ++w) {
                a0 += red[0][w];
                a2 += red[2][w];
                a1 = pass == 0 ? a1 + red[1][w] : fmax(a1, red[1][w]);
            }
            d.stat_part[3 * t] = a0;
            d.stat_part[3 * t + 1] = a1;
            d.stat_part[3 * t + 2] = a2;
        }
        if (pass == 1 && threadIdx.x < 32 && hb[threadIdx.x]) atomicAdd(&d.hist_cnt[32 * s + threadIdx.x], hb[threadIdx.x]);
        __syncthreads();
    }
}

// out per simulation (40 doubles): centroid x, y, z, histogram radius, r_gyr, r_max.
// One block per simulation: each thread folds a fixed set of tiles, then a
// fixed-order tree over the threads.
__global__ void __launch_bounds__(256) k_stats_fold(Dev d, int pass, double *out, double hist_rmax) {
    __shared__ double red[3][256];
    const int s = blockIdx.x;
    const SimDesc &S = d.sims[s];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int64_t t = d.tile_begin[s] + threadIdx.x; t < d.tile_begin[s + 1]; t += blockDim.x) {
        a0 += d.stat_part[3 * t];
        a2 += d.stat_part[3 * t + 2];
        a1 = pass == 0 ? a1 + d.stat_part[3 * t + 1] : fmax(a1, d.stat_part[3 * t + 1]);
    }
    red[0][threadIdx.x] = a0;
    red[1][threadIdx.x] = a1;
    red[2][threadIdx.x] = a2;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[0][threadIdx.x] += red[0][threadIdx.x + h];
            red[2][threadIdx.x] += red[2][threadIdx.x + h];
            red[1][threadIdx.x] = pass == 0 ? red[1][threadIdx.x] + red[1][threadIdx.x + h]
                                            : fmax(red[1][threadIdx.x], red[1][threadIdx.x + h]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 32 && pass == 0) d.hist_cnt[32 * s + threadIdx.x] = 0u;
    if (threadIdx.x == 0) {
        double *o = out + 40 * s;
        const double n = (double)S.n;
        if (pass == 0) {
            o[0] = S.n > 0 ? red[0][0] / n : 0.0;
            o[1] = S.n > 0 ? red[1][0] / n : 0.0;
            o[2] = S.n > 0 ? red[2][0] / n : 0.0;
            o[3] = hist_rmax;
        } else {
            o[4] = S.n > 0 ? sqrt(red[0][0] / n) : 0.0;
            o[5] = red[1][0];
        }
    }
}

// agents per 1000 um^3 of each of the 32 shells of [0, hist_rmax)
__global__ void k_stats_hist(Dev d, double *out, float *hist) {
    for (int q = threadIdx.x; q < 32 * d.n_sims; q += blockDim.x) {
        int s = q / 32, b = q % 32;
        double w = out[40 * s + 3] / 32.0;
        double r0 = w * b, r1 = w * (b + 1);
        double shell = 4.0 / 3.0 * kPi * (r1 * r1 * r1 - r0 * r0 * r0);
        hist[q] = (float)((double)d.hist_cnt[q] / shell * 1000.0);
    }
}

__global__ void k_gather_pos(Dev d, int sim, double *dst) {
    const int P = d.ctl->pos_par;
    const SimDesc &S = d.sims[sim];
    const int64_t A = d.A;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < S.n; q += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = S.a_off + q;
        dst[3 * q] = d.pos[P][i];
        dst[3 * q + 1] = d.pos[P][A + i];
        dst[3 * q + 2] = d.pos[P][2 * A + i];
    }
}

__global__ void k_init_tiles(Dev d) {
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int s = 0; s < d.n_sims; ++s) {
            d.tile_begin[s] = t;
            t += ceil_div(d.sims[s].n, kTile);
            d.sims[s].n_start = d.sims[s].n;
        }
        d.tile_begin[d.n_sims] = t;
        d.ctl->total_tiles = t;
    }
}

// ------------------------------------------------------------------ launchers
void launch_grid_build(const Dev &d, hipStream_t st, int grid_agents, int grid_boxes, bool any_static) {
    hipLaunchKernelGGL(k_begin, dim3(1), dim3(256), 0, st, d);
    hipLaunchKernelGGL(k_bounds, dim3(grid_agents), dim3(256), 0, st, d, (const SimDesc *)d.sims,
                       (const int64_t *)d.tile_begin);
    hipLaunchKernelGGL(k_grid, dim3(1), dim3(256), 0, st, d);
    hipLaunchKernelGGL(k_brank, dim3(grid_boxes), dim3(256), 0, st, d);
    hipLaunchKernelGGL(k_grid_done, dim3(1), dim3(256), 0, st, d);
    hipLaunchKernelGGL(k_bin, dim3(grid_agents), dim3(256), 0, st, d, (const SimDesc *)d.sims,
                       (const int64_t *)d.tile_begin);
    hipLaunchKernelGGL(k_scan_tiles, dim3(grid_boxes), dim3(256), 0, st, d, (const SimDesc *)d.sims,
                       (const int64_t *)d.btile_begin, 0);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, d, 0);
    hipLaunchKernelGGL(k_scan_apply, dim3(grid_boxes), dim3(256), 0, st, d, (const SimDesc *)d.sims,
                       (const int64_t *)d.btile_begin, 0);
    hipLaunchKernelGGL(k_scatter, dim3(grid_agents), dim3(256), 0, st, d, (const SimDesc *)d.sims,
                       (const int64_t *)d.tile_begin);
    if (any_static) {
        launch_near_marks(d, st, grid_boxes, true);
        hipLaunchKernelGGL(k_static_fix, dim3(grid_agents), dim3(256), 0, st, d, (const SimDesc *)d.sims,
                           (const int64_t *)d.btile_begin);
    }
}

void launch_resort(const Dev &d, hipStream_t st, int grid_agents, int grid_boxes, bool force, bool any_static) {
    if (force) hipLaunchKernelGGL(k_force_resort, dim3(1), dim3(64), 0, st, d);
    hipLaunchKernelGGL(k_rs_count, dim3(grid_agents), dim3(256), 0, st, d);
    hipLaunchKernelGGL(k_scan_tiles, dim3(grid_boxes), dim3(256), 0, st, d, (const SimDesc *)d.sims,
                       (const int64_t *)d.btile_begin, 1);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, d, 1);
    hipLaunchKernelGGL(k_scan_apply, dim3(grid_boxes), dim3(256), 0, st, d, (const SimDesc *)d.sims,
                       (const int64_t *)d.btile_begin, 1);
    hipLaunchKernelGGL(k_rs_dest, dim3(grid_agents), dim3(256), 0, st, d);
    hipLaunchKernelGGL(k_rs_move, dim3(grid_agents), dim3(256), 0, st, d);
    if (any_static) hipLaunchKernelGGL(k_rs_sync, dim3(grid_agents), dim3(256), 0, st, d);
    hipLaunchKernelGGL(k_rs_end, dim3(1), dim3(64), 0, st, d);
}

void launch_near_marks(const Dev &d, hipStream_t st, int grid_boxes, bool arrivals) {
    hipLaunchKernelGGL(k_near_marks, dim3(grid_boxes), dim3(256), 0, st, d, arrivals ? 1 : 0);
}

void launch_end(const Dev &d, hipStream_t st, int grid_boxes, bool any_static) {
    if (any_static)
        hipLaunchKernelGGL(k_clear_marks, dim3(grid_boxes), dim3(256), 0, st, d, (const SimDesc *)d.sims,
                           (const int64_t *)d.btile_begin);
    hipLaunchKernelGGL(k_end, dim3(1), dim3(256), 0, st, d);
}

// Statistics: out_dev holds 40 doubles per simulation followed by the
// histograms (n_sims x 32 floats).
void launch_stats(const Dev &d, hipStream_t st, int grid_agents, double hist_rmax, double *out_dev) {
    float *hist = (float *)(out_dev + 40 * d.n_sims);
    hipLaunchKernelGGL(k_stats_sum, dim3(grid_agents), dim3(256), 0, st, d, 0, out_dev);
    hipLaunchKernelGGL(k_stats_fold, dim3(d.n_sims), dim3(256), 0, st, d, 0, out_dev, hist_rmax);
    hipLaunchKernelGGL(k_stats_sum, dim3(grid_agents), dim3(256), 0, st, d, 1, out_dev);
    hipLaunchKernelGGL(k_stats_fold, dim3(d.n_sims), dim3(256), 0, st, d, 1, out_dev, hist_rmax);
    hipLaunchKernelGGL(k_stats_hist, dim3(1), dim3(1024), 0, st, d, out_dev, hist);
}

void launch_gather_pos(const Dev &d, hipStream_t st, int sim, double *dst, int64_t n, int64_t a_off) {
    int grid = (int)(n / 256 + 1);
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(k_gather_pos, dim3(grid), dim3(256), 0, st, d, sim, dst);
}

void launch_scatter_init(const Dev &d, hipStream_t st, int grid_agents) {
    hipLaunchKernelGGL(k_init_tiles, dim3(1), dim3(64), 0, st, d);
}

}  // namespace abm
