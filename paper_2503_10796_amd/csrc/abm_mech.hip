// abm_mech.hip -- HIP kernels of one mechanics iteration on gfx950.
//
// Per iteration (all simulations of a batch in each launch):
//   begin     per-simulation counters, agent-tile prefix
//   bounds    open-boundary grid: min/max of positions, largest diameter (Sec 4.4.11, 4.4.3)
//   grid      box length, dims, box-tile prefix
//   bin       box key of every agent, per-box counts with arrival rank
//   scan_*    per-box exclusive scan (counting sort, Sec 5.3.1)
//   scatter   box-ordered FP32 payload (box-relative centre, radius) + index
//   sweep     27-box force sum (Eq 4.1-4.2), threshold + cap (Sec 5.5), commit
//   fixup     FP64 re-evaluation of agents whose FP32 result cannot decide an
//             integer outcome (contact, non-zero force, neighbour, move)
//   div_*     grow-or-divide with prefix-sum append (Algorithm 2, Sec 5.3.2)
//   static    static flags for the next iteration (Sec 5.5)
//   end       commit: flip position buffers, counts, iteration
//   resort    every R iterations: Morton-order counting sort of agent storage (Sec 5.4.2)
//
// Forces are summed as exact 64-bit fixed-point integers (2^-40 units), so the
// result does not depend on the order in which neighbours are visited: every
// run is bitwise reproducible regardless of atomics (Sec 7.1.4 asks for this).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "abm_internal.h"

namespace abm {

#define ABM_ABORTED(d) (__builtin_expect((d).ctl->abort != 0, 0))

constexpr double kFixMagic = 6144.0;  // 1.5 * 2^12: fma(a, b, M) rounds a*b to 2^-40
constexpr double kFixUnit = 0x1.0p-40;
constexpr double kPi = 3.14159265358979323846;

__device__ inline long long fixbits(double v) { return __double_as_longlong(v); }

// ------------------------------------------------------------------ begin
__global__ void k_begin(Dev d) {
    if (ABM_ABORTED(d)) return;
    for (int s = threadIdx.x; s < d.n_sims; s += blockDim.x) {
        SimDesc &S = d.sims[s];
        S.n_start = S.n;
        S.n_div = 0;
        S.nonfinite = 0;
        S.L_prev = S.L;
        for (int a = 0; a < 3; ++a) {
            S.enc_lo[a] = ~0ull;
            S.enc_hi[a] = 0ull;
        }
        S.enc_maxd = 0ull;
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
        d.ctl->n_fix = 0;
    }
}

// ------------------------------------------------------------------ bounds
__global__ void __launch_bounds__(256) k_bounds(Dev d) {
    if (ABM_ABORTED(d)) return;
    __shared__ double red[7][8];
    const int P = d.ctl->pos_par, lp = d.ctl->lay_par;
    const int64_t A = d.A;
    const int64_t total = d.ctl->total_tiles;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int s = find_sim(d.tile_begin, d.n_sims, t);
        const SimDesc &S = d.sims[s];
        int64_t loc = (t - d.tile_begin[s]) * kTile + threadIdx.x;
        double v[7];
        bool ok = loc < S.n_start;
        bool bad = false;
        if (ok) {
            int64_t i = S.a_off + loc;
            double x = d.pos[P][i], y = d.pos[P][A + i], z = d.pos[P][2 * A + i];
            double dm = d.diam[lp][i];
            bad = !(isfinite(x) && isfinite(y) && isfinite(z) && isfinite(dm));
            v[0] = x; v[1] = y; v[2] = z; v[3] = -x; v[4] = -y; v[5] = -z; v[6] = dm;
        } else {
            for (int a = 0; a < 6; ++a) v[a] = __builtin_huge_val();
            v[6] = -__builtin_huge_val();
        }
        // min of (x,y,z,-x,-y,-z) and max of d via wave then block reduction
        for (int off = 32; off > 0; off >>= 1) {
            for (int a = 0; a < 6; ++a) v[a] = fmin(v[a], __shfl_xor(v[a], off));
            v[6] = fmax(v[6], __shfl_xor(v[6], off));
        }
        if (lane == 0)
            for (int a = 0; a < 7; ++a) red[a][wid] = v[a];
        if (bad) atomicOr(&d.sims[s].nonfinite, 1u);
        __syncthreads();
        if (threadIdx.x == 0) {
            int nw = blockDim.x >> 6;
            for (int w = 1; w < nw; ++w) {
                for (int a = 0; a < 6; ++a) red[a][0] = fmin(red[a][0], red[a][w]);
                red[6][0] = fmax(red[6][0], red[6][w]);
            }
            SimDesc &W = d.sims[s];
            for (int a = 0; a < 3; ++a) {
                if (red[a][0] < __builtin_huge_val()) {
                    atomicMin(&W.enc_lo[a], enc_double(red[a][0]));
                    atomicMax(&W.enc_hi[a], enc_double(-red[3 + a][0]));
                }
            }
            if (red[6][0] > -__builtin_huge_val()) atomicMax(&W.enc_maxd, enc_double(red[6][0]));
        }
        __syncthreads();
    }
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
            S.dims[0] = S.dims[1] = S.dims[2] = 0;
            continue;
        }
        double L = S.box_len > 0.0 ? S.box_len : dec_double(S.enc_maxd);
        S.L = L;
        int64_t nb = 1;
        bool bad = !(L > 0.0);
        for (int a = 0; a < 3; ++a) {
            S.lo[a] = dec_double(S.enc_lo[a]);
            S.hi[a] = dec_double(S.enc_hi[a]);
            double q = floor((S.hi[a] - S.lo[a]) / L) + 1.0;
            int lim = a == 2 ? kDimZ : (a == 1 ? kDimY : kDimX);
            if (!(q <= (double)lim)) { bad = true; q = 1.0; }
            S.dims[a] = (int32_t)q;
            nb *= (int64_t)q;
        }
        if (bad || nb > S.box_cap) {
            S.err |= kErrGrid;
            atomicOr(&d.ctl->err, kErrGrid);
            atomicExch(&d.ctl->abort, 1);
            nb = 0;
        }
        S.nboxes = nb;
        S.e_delta = (float)ldexp(L, -19);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int s = 0; s < d.n_sims; ++s) {
            d.btile_begin[s] = t;
            t += ceil_div(d.sims[s].nboxes, kBoxTile);
        }
        d.btile_begin[d.n_sims] = t;
        d.ctl->total_btiles = t;
    }
}

// ------------------------------------------------------------------ bin
__global__ void __launch_bounds__(256) k_bin(Dev d) {
    if (ABM_ABORTED(d)) return;
    const int P = d.ctl->pos_par;
    const int64_t A = d.A;
    const int64_t total = d.ctl->total_tiles;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int s = find_sim(d.tile_begin, d.n_sims, t);
        const SimDesc &S = d.sims[s];
        int64_t loc = (t - d.tile_begin[s]) * kTile + threadIdx.x;
        if (loc >= S.n_start) continue;
        int64_t i = S.a_off + loc;
        double L = S.L;
        int bx = box_coord(d.pos[P][i], S.lo[0], L, S.dims[0]);
        int by = box_coord(d.pos[P][A + i], S.lo[1], L, S.dims[1]);
        int bz = box_coord(d.pos[P][2 * A + i], S.lo[2], L, S.dims[2]);
        int64_t lin = linear_box(bx, by, bz, S.dims);
        d.key[i] = pack_key(bx, by, bz);
        d.rank[i] = atomicAdd(&d.count[S.b_off + lin], 1u);
        if (S.detect_static && (d.flags[d.ctl->lay_par][i] & kChgMask)) d.arrive[S.b_off + lin] = 1;
    }
}

// ------------------------------------------------------------------ scan
// Segmented exclusive scan of per-box counts into global slot starts.
__device__ inline uint32_t block_excl_scan_4(uint32_t v[4], uint32_t *sh, uint32_t &total) {
    // 256 threads x 4 items; returns this thread's exclusive prefix of its first item
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

__global__ void __launch_bounds__(256) k_scan_tiles(Dev d) {
    if (ABM_ABORTED(d)) return;
    __shared__ uint32_t sh[4];
    const int64_t total = d.ctl->total_btiles;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int s = find_sim(d.btile_begin, d.n_sims, t);
        const SimDesc &S = d.sims[s];
        int64_t k0 = (t - d.btile_begin[s]) * kBoxTile + threadIdx.x * 4;
        uint32_t v[4];
        for (int q = 0; q < 4; ++q) v[q] = (k0 + q < S.nboxes) ? d.count[S.b_off + k0 + q] : 0u;
        uint32_t tot;
        block_excl_scan_4(v, sh, tot);
        if (threadIdx.x == 0) d.tile_sum[t] = tot;
    }
}

__global__ void __launch_bounds__(1024) k_scan_top(Dev d) {
    if (ABM_ABORTED(d)) return;
    __shared__ uint32_t sh[16];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int s = 0; s < d.n_sims; ++s) {
        int64_t b0 = d.btile_begin[s], b1 = d.btile_begin[s + 1];
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

// Writes box_start[sb_off + k] = a_off + prefix; zeroes the counts.
__global__ void __launch_bounds__(256) k_scan_apply(Dev d) {
    if (ABM_ABORTED(d)) return;
    __shared__ uint32_t sh[4];
    const int64_t total = d.ctl->total_btiles;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int s = find_sim(d.btile_begin, d.n_sims, t);
        const SimDesc &S = d.sims[s];
        int64_t k0 = (t - d.btile_begin[s]) * kBoxTile + threadIdx.x * 4;
        uint32_t v[4];
        for (int q = 0; q < 4; ++q) v[q] = (k0 + q < S.nboxes) ? d.count[S.b_off + k0 + q] : 0u;
        uint32_t tot;
        uint32_t pre = block_excl_scan_4(v, sh, tot);
        uint32_t base = (uint32_t)S.a_off + d.tile_off[t] + pre;
        for (int q = 0; q < 4; ++q) {
            if (k0 + q < S.nboxes) {
                d.box_start[S.sb_off + k0 + q] = base;
                d.count[S.b_off + k0 + q] = 0u;
            }
            base += v[q];
        }
        if (t == d.btile_begin[s + 1] - 1 && threadIdx.x == 0)
            d.box_start[S.sb_off + S.nboxes] = (uint32_t)(S.a_off + S.n_start);
    }
}

// ------------------------------------------------------------------ scatter
__global__ void __launch_bounds__(256) k_scatter(Dev d) {
    if (ABM_ABORTED(d)) return;
    const int P = d.ctl->pos_par, lp = d.ctl->lay_par;
    const int64_t A = d.A;
    const int64_t total = d.ctl->total_tiles;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int s = find_sim(d.tile_begin, d.n_sims, t);
        const SimDesc &S = d.sims[s];
        int64_t loc = (t - d.tile_begin[s]) * kTile + threadIdx.x;
        if (loc >= S.n_start) continue;
        int64_t i = S.a_off + loc;
        int bx, by, bz;
        unpack_key(d.key[i], bx, by, bz);
        int64_t lin = linear_box(bx, by, bz, S.dims);
        uint32_t slot = d.box_start[S.sb_off + lin] + d.rank[i];
        float4 p;
        p.x = rel_coord(d.pos[P][i], S.lo[0], S.L, bx);
        p.y = rel_coord(d.pos[P][A + i], S.lo[1], S.L, by);
        p.z = rel_coord(d.pos[P][2 * A + i], S.lo[2], S.L, bz);
        p.w = (float)(0.5 * d.diam[lp][i]);
        d.payload[slot] = p;
        d.sorted_idx[slot] = (uint32_t)i;
    }
}

// ------------------------------------------------------------------ commit helpers
// Displacement exactly as the thesis's rule reads: no motion unless |F| > a,
// else F*dt/m capped in Euclidean norm (FP64, IEEE ops, no contraction).
__device__ inline bool displacement64(double fx, double fy, double fz, const SimDesc &S, double &dx, double &dy,
                                      double &dz) {
#pragma clang fp contract(off)
    double fn = sqrt(fma(fz, fz, fma(fy, fy, fx * fx)));
    if (!(fn > S.adherence)) {
        dx = dy = dz = 0.0;
        return false;
    }
    double scale = S.dt / S.mass;
    dx = fx * scale;
    dy = fy * scale;
    dz = fz * scale;
    double dn = sqrt(fma(dz, dz, fma(dy, dy, dx * dx)));
    if (dn > S.max_disp) {
        double c = S.max_disp / dn;
        dx *= c;
        dy *= c;
        dz *= c;
    }
    return true;
}

// Writes the outcome of one agent's mechanics (shared by sweep and fixup).
template <bool DIAG>
__device__ inline void commit_agent(const Dev &d, const SimDesc &S, int64_t i, int P, int lp, uint8_t fl, double x,
                                    double y, double z, double fx, double fy, double fz, int nz, int nbr,
                                    int contacts) {
    const int64_t A = d.A;
    double dx, dy, dz;
    bool moved = displacement64(fx, fy, fz, S, dx, dy, dz);
    d.nz[lp][i] = (uint8_t)(nz > 255 ? 255 : nz);
    fl &= (uint8_t)~kChgMask;
    if (moved) {
        d.pos[1 - P][i] = x + dx;
        d.pos[1 - P][A + i] = y + dy;
        d.pos[1 - P][2 * A + i] = z + dz;
        d.flags[lp][i] = fl | kBufDiff | kMoved;
        if (S.detect_static) {
            int bx, by, bz;
            unpack_key(d.key[i], bx, by, bz);
            d.dirty[S.b_off + linear_box(bx, by, bz, S.dims)] = 1;
        }
    } else {
        if (fl & kBufDiff) {
            d.pos[1 - P][i] = x;
            d.pos[1 - P][A + i] = y;
            d.pos[1 - P][2 * A + i] = z;
            fl &= (uint8_t)~kBufDiff;
        }
        d.flags[lp][i] = fl;
    }
    if (DIAG) {
        d.nbr[i] = nbr;
        d.contacts[i] = contacts;
        d.force[3 * i] = fx;
        d.force[3 * i + 1] = fy;
        d.force[3 * i + 2] = fz;
        d.disp[3 * i] = dx;
        d.disp[3 * i + 1] = dy;
        d.disp[3 * i + 2] = dz;
        int bx, by, bz;
        unpack_key(d.key[i], bx, by, bz);
        d.boxid[i] = linear_box(bx, by, bz, S.dims);
    }
}

template <bool DIAG>
__device__ inline void skip_static(const Dev &d, const SimDesc &S, int64_t i, int P, int lp, uint8_t fl) {
    const int64_t A = d.A;
    if (fl & kBufDiff) {
        d.pos[1 - P][i] = d.pos[P][i];
        d.pos[1 - P][A + i] = d.pos[P][A + i];
        d.pos[1 - P][2 * A + i] = d.pos[P][2 * A + i];
    }
    if (fl & (kBufDiff | kChgMask)) d.flags[lp][i] = fl & (uint8_t) ~(kBufDiff | kChgMask);
    if (DIAG) {
        d.nbr[i] = -1;
        d.contacts[i] = -1;
        for (int a = 0; a < 3; ++a) {
            d.force[3 * i + a] = 0.0;
            d.disp[3 * i + a] = 0.0;
        }
        int bx, by, bz;
        unpack_key(d.key[i], bx, by, bz);
        d.boxid[i] = linear_box(bx, by, bz, S.dims);
    }
}

// ------------------------------------------------------------------ sweep
// One thread per target agent, agents in storage (Morton) order.  The 27
// neighbour boxes are visited as 9 rows of 3 consecutive boxes, each row a
// contiguous range of the box-ordered payload.  All FP32 work is on
// box-relative coordinates; every integer decision that FP32 cannot certify
// sends the agent to the FP64 fix-up kernel instead.
template <bool DIAG>
__global__ void __launch_bounds__(256) k_sweep(Dev d) {
    if (ABM_ABORTED(d)) return;
    const int P = d.ctl->pos_par, lp = d.ctl->lay_par;
    const int64_t A = d.A;
    const int64_t total = d.ctl->total_tiles;
    const int tpb = blockDim.x;
    const int64_t per_tile = kTile;
    // a tile of kTile agents is covered by kTile / blockDim.x passes
    const int passes = (int)(per_tile / tpb) > 0 ? (int)(per_tile / tpb) : 1;
    for (int64_t w = blockIdx.x; w < total * passes; w += gridDim.x) {
        int64_t t = w / passes;
        int part = (int)(w - t * passes);
        int s = find_sim(d.tile_begin, d.n_sims, t);
        const SimDesc &S = d.sims[s];
        int64_t loc = (t - d.tile_begin[s]) * kTile + part * tpb + threadIdx.x;
        if (loc >= S.n_start) continue;
        int64_t i = S.a_off + loc;
        uint8_t fl = d.flags[lp][i];
        if (S.detect_static && (fl & kStatic)) {
            skip_static<DIAG>(d, S, i, P, lp, fl);
            continue;
        }
        const double x = d.pos[P][i], y = d.pos[P][A + i], z = d.pos[P][2 * A + i];
        int bx, by, bz;
        unpack_key(d.key[i], bx, by, bz);
        const int nx = S.dims[0], ny = S.dims[1], nzd = S.dims[2];
        const float Lf = (float)S.L;
        const float rxi = rel_coord(x, S.lo[0], S.L, bx);
        const float ryi = rel_coord(y, S.lo[1], S.L, by);
        const float rzi = rel_coord(z, S.lo[2], S.L, bz);
        const float ri = (float)(0.5 * d.diam[lp][i]);
        const uint32_t self = d.box_start[S.sb_off + linear_box(bx, by, bz, S.dims)] + d.rank[i];
        const float e = S.e_delta;
        const float g = 2.0f * e;
        const float kf = (float)S.k, gf = (float)S.gamma;
        const float L2 = (float)(S.L * S.L);
        const float G = (float)ldexp(S.L * S.L, -18);
        const float L2m = L2 - G, L2p = L2 + G;
        long long ax = 0, ay = 0, az = 0;
        uint32_t eacc = 0;
        int contacts = 0, nzc = 0, nbr = 0, nfix = 0;
        bool unc = false;
        for (int oz = -1; oz <= 1; ++oz) {
            int cz = bz + oz;
            if (cz < 0 || cz >= nzd) continue;
            for (int oy = -1; oy <= 1; ++oy) {
                int cy = by + oy;
                if (cy < 0 || cy >= ny) continue;
                const int bx0 = bx > 0 ? bx - 1 : 0;
                const int bx1 = bx < nx - 1 ? bx + 1 : nx - 1;
                const int64_t rowlin = (int64_t)nx * ((int64_t)cy + (int64_t)ny * cz);
                const uint32_t *bs = d.box_start + S.sb_off + rowlin;
                const float qy = ryi - (float)oy * Lf;
                const float qz = rzi - (float)oz * Lf;
                uint32_t sb = bs[bx0];
                for (int cx = bx0; cx <= bx1; ++cx) {
                    const uint32_t se = bs[cx + 1];
                    const float qx = rxi - (float)(cx - bx) * Lf;
                    for (uint32_t slot = sb; slot < se; ++slot) {
                        if (slot == self) continue;
                        const float4 c = d.payload[slot];
                        const float ddx = qx - c.x, ddy = qy - c.y, ddz = qz - c.z;
                        const float d2 = fmaf(ddz, ddz, fmaf(ddy, ddy, ddx * ddx));
                        if (DIAG) {
                            if (d2 < L2m) ++nbr;
                            else if (d2 < L2p) unc = true;
                        }
                        const float sr = ri + c.w;
                        const float sg = sr + g;
                        if (d2 < sg * sg) {
                            if (d2 >= L2m) {  // only possible when box_len < largest diameter
                                if (d2 < L2p) unc = true;
                                continue;
                            }
                            const float dist = sqrtf(d2);
                            const float delta = sr - dist;
                            if (delta <= e) {
                                if (delta >= -e) unc = true;
                                continue;
                            }
                            ++contacts;
                            const float rbar = ri * c.w / sr;
                            const float sq = sqrtf(rbar * delta);
                            const float fn = kf * delta - gf * sq;
                            const float ep = (kf + gf * sq / (2.0f * delta)) * e + fabsf(fn) * 0x1.0p-19f;
                            if (ep >= 0x1.0p-6f || fabsf(fn) <= ep) {
                                unc = true;
                                continue;
                            }
                            ++nzc;
                            const double f = (double)(fn / dist);
                            ax += fixbits(fma(f, (double)ddx, kFixMagic));
                            ay += fixbits(fma(f, (double)ddy, kFixMagic));
                            az += fixbits(fma(f, (double)ddz, kFixMagic));
                            ++nfix;
                            eacc += (uint32_t)ceilf(ep * 0x1.0p26f);
                        }
                    }
                    sb = se;
                }
            }
        }
        if (!unc) {
            const long long mb = fixbits(kFixMagic);
            const double fx = (double)(ax - (long long)nfix * mb) * kFixUnit;
            const double fy = (double)(ay - (long long)nfix * mb) * kFixUnit;
            const double fz = (double)(az - (long long)nfix * mb) * kFixUnit;
            const double fnorm = sqrt(fx * fx + fy * fy + fz * fz);
            const double ebound = (double)eacc * 0x1.0p-26 + 1e-9;
            if (fabs(fnorm - S.adherence) <= ebound) unc = true;
            else commit_agent<DIAG>(d, S, i, P, lp, fl, x, y, z, fx, fy, fz, nzc, nbr, contacts);
        }
        if (unc) {
            uint32_t q = atomicAdd(&d.ctl->n_fix, 1u);
            d.fix_list[q] = (uint32_t)i;
        }
    }
}

// ------------------------------------------------------------------ fixup
// FP64 re-evaluation with the exact expressions of the method for agents the
// FP32 sweep could not decide.  Neighbours are read from the start-of-iteration
// FP64 state through the grid (copy semantics).
template <bool DIAG>
__global__ void __launch_bounds__(256) k_fixup(Dev d) {
#pragma clang fp contract(off)
    if (ABM_ABORTED(d)) return;
    const int P = d.ctl->pos_par, lp = d.ctl->lay_par;
    const int64_t A = d.A;
    const uint32_t nf = d.ctl->n_fix;
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < nf; q += gridDim.x * blockDim.x) {
        const int64_t i = d.fix_list[q];
        const int s = find_sim(d.a_begin, d.n_sims, i);
        const SimDesc &S = d.sims[s];
        const uint8_t fl = d.flags[lp][i];
        const double x = d.pos[P][i], y = d.pos[P][A + i], z = d.pos[P][2 * A + i];
        const double ri = 0.5 * d.diam[lp][i];
        const double L2 = S.L * S.L;
        int bx, by, bz;
        unpack_key(d.key[i], bx, by, bz);
        double fx = 0.0, fy = 0.0, fz = 0.0;
        int nbr = 0, contacts = 0, nzc = 0;
        for (int oz = -1; oz <= 1; ++oz)
            for (int oy = -1; oy <= 1; ++oy)
                for (int ox = -1; ox <= 1; ++ox) {
                    int cx = bx + ox, cy = by + oy, cz = bz + oz;
                    if (cx < 0 || cy < 0 || cz < 0 || cx >= S.dims[0] || cy >= S.dims[1] || cz >= S.dims[2]) continue;
                    int64_t lin = linear_box(cx, cy, cz, S.dims);
                    uint32_t s0 = d.box_start[S.sb_off + lin], s1 = d.box_start[S.sb_off + lin + 1];
                    for (uint32_t slot = s0; slot < s1; ++slot) {
                        int64_t j = d.sorted_idx[slot];
                        if (j == i) continue;
                        double ddx = x - d.pos[P][j], ddy = y - d.pos[P][A + j], ddz = z - d.pos[P][2 * A + j];
                        double d2 = fma(ddz, ddz, fma(ddy, ddy, ddx * ddx));
                        if (!(d2 < L2)) continue;
                        ++nbr;
                        double rj = 0.5 * d.diam[lp][j];
                        double dist = sqrt(d2);
                        double delta = ri + rj - dist;
                        if (!(delta > 0.0)) continue;
                        ++contacts;
                        double rbar = ri * rj / (ri + rj);
                        double fn = S.k * delta - S.gamma * sqrt(rbar * delta);
                        if (fn != 0.0) ++nzc;
                        if (dist > 0.0) {
                            fx += fn * ddx / dist;
                            fy += fn * ddy / dist;
                            fz += fn * ddz / dist;
                        }
                    }
                }
        commit_agent<DIAG>(d, S, i, P, lp, fl, x, y, z, fx, fy, fz, nzc, nbr, contacts);
    }
}

// ------------------------------------------------------------------ growth and division
// Correctly rounded cube root: ocml's cbrt is within one ulp; the candidate
// is corrected by the sign of (y +- ulp/2)^3 - t, evaluated with error-free
// products (Dekker/Ogita-Rump-Oishi TwoProd via fma).
__device__ inline double cube_minus(double y, double h, double t) {
#pragma clang fp contract(off)
    double p = y * y, e1 = fma(y, y, -p);
    double q = p * y, e2 = fma(p, y, -q);
    double r = e1 * y, e3 = fma(e1, y, -r);
    double hp = h * p;  // exact: h is a power of two
    double s1 = 3.0 * hp, s2 = fma(3.0, hp, -s1);
    double s3 = 3.0 * h * e1;
    double s4 = 3.0 * y * h * h;
    double big = (q - t) + s1;
    return big + ((e2 + r) + ((s2 + e3) + (s3 + s4)));
}

__device__ inline double cbrt_cr(double t) {
    double y = cbrt(t);
    double up = nextafter(y, __builtin_huge_val());
    if (cube_minus(y, 0.5 * (up - y), t) < 0.0) return up;
    double dn = nextafter(y, 0.0);
    if (cube_minus(y, -0.5 * (y - dn), t) > 0.0) return dn;
    return y;
}

__device__ inline double diameter_from_volume(double v) { return cbrt_cr((6.0 * v) / kPi); }

// Philox4x32-10 (Salmon et al., SC'11).
__device__ inline void philox(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        uint32_t hi0 = __umulhi(0xD2511F53u, c[0]), lo0 = 0xD2511F53u * c[0];
        uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]), lo1 = 0xCD9E8D57u * c[2];
        uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Uniform unit vector for a division, keyed by (seed; uid, iteration, sim).
__device__ inline void division_direction(uint64_t seed, uint32_t sim, uint64_t uid, uint64_t iter, double u[3]) {
#pragma clang fp contract(off)
    uint32_t c[4] = {(uint32_t)uid, (uint32_t)(uid >> 32), (uint32_t)iter, sim};
    philox(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    double u1 = (double)(((((uint64_t)c[0]) << 32) | c[1]) >> 11) * 0x1.0p-53;
    double u2 = (double)(((((uint64_t)c[2]) << 32) | c[3]) >> 11) * 0x1.0p-53;
    double zc = 2.0 * u1 - 1.0;
    double phi = 2.0 * kPi * u2;
    double rho = sqrt((1.0 - zc) * (1.0 + zc));
    double sn, cs;
    sincos(phi, &sn, &cs);
    u[0] = rho * cs;
    u[1] = rho * sn;
    u[2] = zc;
}

__global__ void __launch_bounds__(256) k_div_mark(Dev d) {
    if (ABM_ABORTED(d)) return;
    const int lp = d.ctl->lay_par;
    const int64_t total = d.ctl->total_tiles;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int s = find_sim(d.tile_begin, d.n_sims, t);
        SimDesc &S = d.sims[s];
        if (!(S.div_vol > 0.0)) continue;
        int64_t loc = (t - d.tile_begin[s]) * kTile + threadIdx.x;
        bool div = false;
        if (loc < S.n_start) {
            int64_t i = S.a_off + loc;
            if (d.vol[lp][i] >= S.div_vol) {
                div = true;
                d.divflag[S.a_off + d.uid[lp][i]] = 1u;
            }
        }
        unsigned long long b = __ballot(div);
        if ((threadIdx.x & 63) == 0 && b) atomicAdd((unsigned long long *)&S.n_div, (unsigned long long)__popcll(b));
    }
}

__global__ void k_div_check(Dev d) {
    if (ABM_ABORTED(d)) return;
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int s = threadIdx.x; s < d.n_sims; s += blockDim.x) {
        SimDesc &S = d.sims[s];
        if (S.n_start + S.n_div > S.cap || S.next_uid + S.n_div > S.cap) {
            S.err |= kErrCapacity;
            atomicOr(&d.ctl->err, kErrCapacity);
            bad = 1;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int s = 0; s < d.n_sims; ++s) {
            d.utile_begin[s] = t;
            t += d.sims[s].div_vol > 0.0 ? ceil_div(d.sims[s].next_uid, kBoxTile) : 0;
        }
        d.utile_begin[d.n_sims] = t;
        d.ctl->total_utiles = t;
        if (bad) d.ctl->abort = 1;
    }
}

// Segmented exclusive scan of the divider flags (indexed by uid) -> rank.
__global__ void __launch_bounds__(256) k_uscan_tiles(Dev d) {
    if (ABM_ABORTED(d)) return;
    __shared__ uint32_t sh[4];
    const int64_t total = d.ctl->total_utiles;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int s = find_sim(d.utile_begin, d.n_sims, t);
        const SimDesc &S = d.sims[s];
        int64_t k0 = (t - d.utile_begin[s]) * kBoxTile + threadIdx.x * 4;
        uint32_t v[4];
        for (int q = 0; q < 4; ++q) v[q] = (k0 + q < S.next_uid) ? d.divflag[S.a_off + k0 + q] : 0u;
        uint32_t tot;
        block_excl_scan_4(v, sh, tot);
        if (threadIdx.x == 0) d.tile_sum[t] = tot;
    }
}

__global__ void __launch_bounds__(1024) k_uscan_top(Dev d) {
    if (ABM_ABORTED(d)) return;
    __shared__ uint32_t sh[16];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int s = 0; s < d.n_sims; ++s) {
        int64_t b0 = d.utile_begin[s], b1 = d.utile_begin[s + 1];
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

__global__ void __launch_bounds__(256) k_uscan_apply(Dev d) {
    if (ABM_ABORTED(d)) return;
    __shared__ uint32_t sh[4];
    const int64_t total = d.ctl->total_utiles;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int s = find_sim(d.utile_begin, d.n_sims, t);
        const SimDesc &S = d.sims[s];
        int64_t k0 = (t - d.utile_begin[s]) * kBoxTile + threadIdx.x * 4;
        uint32_t v[4];
        for (int q = 0; q < 4; ++q) v[q] = (k0 + q < S.next_uid) ? d.divflag[S.a_off + k0 + q] : 0u;
        uint32_t tot;
        uint32_t pre = block_excl_scan_4(v, sh, tot);
        uint32_t base = d.tile_off[t] + pre;
        for (int q = 0; q < 4; ++q) {
            if (k0 + q < S.next_uid && v[q]) d.divrank[S.a_off + k0 + q] = base;
            base += v[q];
        }
    }
}

// Grow (V += g) or divide (two cells of V/2 shifted +-s along a random unit
// vector, daughter appended at n_start + rank) from the start-of-iteration
// volume, applied to the committed position.
__global__ void __launch_bounds__(256) k_div_apply(Dev d) {
#pragma clang fp contract(off)
    if (ABM_ABORTED(d)) return;
    const int P = d.ctl->pos_par, lp = d.ctl->lay_par;
    const int64_t A = d.A;
    const int64_t total = d.ctl->total_tiles;
    const uint64_t iter = (uint64_t)d.ctl->iter;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int s = find_sim(d.tile_begin, d.n_sims, t);
        const SimDesc &S = d.sims[s];
        if (!(S.div_vol > 0.0)) continue;
        int64_t loc = (t - d.tile_begin[s]) * kTile + threadIdx.x;
        if (loc >= S.n_start) continue;
        int64_t i = S.a_off + loc;
        double v = d.vol[lp][i];
        const int Q = 1 - P;  // buffer of committed positions
        if (v >= S.div_vol) {
            uint64_t u_id = d.uid[lp][i];
            uint32_t rank = d.divrank[S.a_off + u_id];
            d.divflag[S.a_off + u_id] = 0u;
            int64_t j = S.a_off + S.n_start + rank;
            double u[3];
            division_direction(S.seed, S.sim_id, u_id, iter, u);
            double shift = S.shift_frac * (0.5 * d.diam[lp][i]);
            double half = 0.5 * v;
            double dnew = diameter_from_volume(half);
            double cx = d.pos[Q][i], cy = d.pos[Q][A + i], cz = d.pos[Q][2 * A + i];
            double jx = cx + shift * u[0], jy = cy + shift * u[1], jz = cz + shift * u[2];
            double mx = cx - shift * u[0], my = cy - shift * u[1], mz = cz - shift * u[2];
            d.pos[Q][j] = jx; d.pos[Q][A + j] = jy; d.pos[Q][2 * A + j] = jz;
            d.pos[Q][i] = mx; d.pos[Q][A + i] = my; d.pos[Q][2 * A + i] = mz;
            d.vol[lp][i] = half; d.vol[lp][j] = half;
            d.diam[lp][i] = dnew; d.diam[lp][j] = dnew;
            d.growth[lp][j] = d.growth[lp][i];
            d.uid[lp][j] = (uint64_t)S.next_uid + rank;
            d.nz[lp][j] = 0;
            d.flags[lp][j] = kBufDiff | kNew;
            d.flags[lp][i] = (d.flags[lp][i] & ~kStatic) | kBufDiff | kMoved | kDivided;
        } else {
            double nv = v + d.growth[lp][i];
            d.vol[lp][i] = nv;
            d.diam[lp][i] = diameter_from_volume(nv);
            d.flags[lp][i] |= kGrew;
        }
        if (S.detect_static) {
            // the start box of a changed agent (the new grid catches arrivals)
            int bx, by, bz;
            unpack_key(d.key[i], bx, by, bz);
            d.dirty[S.b_off + linear_box(bx, by, bz, S.dims)] = 1;
        }
    }
}

// ------------------------------------------------------------------ static flags
// Sec 5.5: an agent is static in the coming iteration when it did not change
// itself, had at most one non-zero neighbour force, and no changed agent lies
// within the interaction radius L of it, at the changed agent's start or
// committed position.  The test is radius-exact (FP64, same expression as the
// neighbour predicate).  Here, changed agents whose start position is in the
// 27-box neighbourhood are checked (boxes marked dirty prune the search);
// changed agents that arrive from farther away are caught by k_static_fix on
// the next grid.
__device__ inline bool near_point(double x, double y, double z, double px, double py, double pz, double L2) {
#pragma clang fp contract(off)
    double ddx = x - px, ddy = y - py, ddz = z - pz;
    return fma(ddz, ddz, fma(ddy, ddy, ddx * ddx)) < L2;
}

__global__ void __launch_bounds__(256) k_static(Dev d) {
    if (ABM_ABORTED(d)) return;
    const int P = d.ctl->pos_par, lp = d.ctl->lay_par;
    const int64_t A = d.A;
    const int64_t total = d.ctl->total_tiles;  // tiles over n_start (daughters are new: never static)
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int s = find_sim(d.tile_begin, d.n_sims, t);
        const SimDesc &S = d.sims[s];
        if (!S.detect_static) continue;
        int64_t loc = (t - d.tile_begin[s]) * kTile + threadIdx.x;
        if (loc >= S.n_start) continue;
        int64_t i = S.a_off + loc;
        uint8_t fl = d.flags[lp][i];
        bool st = !(fl & kChgMask) && d.nz[lp][i] <= 1;
        if (st) {
            const double x = d.pos[P][i], y = d.pos[P][A + i], z = d.pos[P][2 * A + i];
            const double L2 = S.L * S.L;
            int bx, by, bz;
            unpack_key(d.key[i], bx, by, bz);
            for (int oz = -1; oz <= 1 && st; ++oz)
                for (int oy = -1; oy <= 1 && st; ++oy)
                    for (int ox = -1; ox <= 1 && st; ++ox) {
                        int cx = bx + ox, cy = by + oy, cz = bz + oz;
                        if (cx < 0 || cy < 0 || cz < 0 || cx >= S.dims[0] || cy >= S.dims[1] || cz >= S.dims[2]) continue;
                        int64_t lin = linear_box(cx, cy, cz, S.dims);
                        if (!d.dirty[S.b_off + lin]) continue;
                        uint32_t s0 = d.box_start[S.sb_off + lin], s1 = d.box_start[S.sb_off + lin + 1];
                        for (uint32_t slot = s0; slot < s1 && st; ++slot) {
                            int64_t j = d.sorted_idx[slot];
                            if (j == i || !(d.flags[lp][j] & kChgMask)) continue;
                            // start position (buffer P) and committed position (buffer 1-P)
                            if (near_point(x, y, z, d.pos[P][j], d.pos[P][A + j], d.pos[P][2 * A + j], L2) ||
                                near_point(x, y, z, d.pos[1 - P][j], d.pos[1 - P][A + j], d.pos[1 - P][2 * A + j], L2))
                                st = false;
                        }
                    }
        }
        d.flags[lp][i] = st ? (fl | kStatic) : (fl & ~kStatic);
    }
}

// After the next grid is built (positions = committed positions): a static
// agent stops being static when a changed agent (including a new daughter)
// now lies within the previous iteration's radius.  Boxes holding a changed
// agent were marked by k_bin.
__global__ void __launch_bounds__(256) k_static_fix(Dev d) {
    if (ABM_ABORTED(d)) return;
    const int P = d.ctl->pos_par, lp = d.ctl->lay_par;
    const int64_t A = d.A;
    const int64_t total = d.ctl->total_tiles;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int s = find_sim(d.tile_begin, d.n_sims, t);
        const SimDesc &S = d.sims[s];
        if (!S.detect_static) continue;
        int64_t loc = (t - d.tile_begin[s]) * kTile + threadIdx.x;
        if (loc >= S.n_start) continue;
        int64_t i = S.a_off + loc;
        uint8_t fl = d.flags[lp][i];
        if (!(fl & kStatic)) continue;
        bool st = S.L >= S.L_prev;  // a shrunken grid cannot cover the old radius: be conservative
        if (st) {
            const double x = d.pos[P][i], y = d.pos[P][A + i], z = d.pos[P][2 * A + i];
            const double L2 = S.L_prev * S.L_prev;
            int bx, by, bz;
            unpack_key(d.key[i], bx, by, bz);
            for (int oz = -1; oz <= 1 && st; ++oz)
                for (int oy = -1; oy <= 1 && st; ++oy)
                    for (int ox = -1; ox <= 1 && st; ++ox) {
                        int cx = bx + ox, cy = by + oy, cz = bz + oz;
                        if (cx < 0 || cy < 0 || cz < 0 || cx >= S.dims[0] || cy >= S.dims[1] || cz >= S.dims[2]) continue;
                        int64_t lin = linear_box(cx, cy, cz, S.dims);
                        if (!d.arrive[S.b_off + lin]) continue;
                        uint32_t s0 = d.box_start[S.sb_off + lin], s1 = d.box_start[S.sb_off + lin + 1];
                        for (uint32_t slot = s0; slot < s1 && st; ++slot) {
                            int64_t j = d.sorted_idx[slot];
                            if (j == i || !(d.flags[lp][j] & kChgMask)) continue;
                            if (near_point(x, y, z, d.pos[P][j], d.pos[P][A + j], d.pos[P][2 * A + j], L2)) st = false;
                        }
                    }
        }
        if (!st) d.flags[lp][i] = fl & ~kStatic;
    }
}

// Clears the dirty and arrival marks of the current grid.
__global__ void __launch_bounds__(256) k_clear_marks(Dev d) {
    if (ABM_ABORTED(d)) return;
    const int64_t total = d.ctl->total_btiles;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int s = find_sim(d.btile_begin, d.n_sims, t);
        const SimDesc &S = d.sims[s];
        if (!S.detect_static) continue;
        int64_t k0 = (t - d.btile_begin[s]) * kBoxTile;
        for (int q = threadIdx.x; q < kBoxTile; q += blockDim.x) {
            if (k0 + q < S.nboxes) {
                d.dirty[S.b_off + k0 + q] = 0;
                d.arrive[S.b_off + k0 + q] = 0;
            }
        }
    }
}

// ------------------------------------------------------------------ end of iteration
__global__ void k_end(Dev d) {
    if (ABM_ABORTED(d)) return;
    for (int s = threadIdx.x; s < d.n_sims; s += blockDim.x) {
        SimDesc &S = d.sims[s];
        S.n = S.n_start + S.n_div;
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
// Rank of box (bx,by,bz) among the boxes of an nx x ny x nz grid in Morton
// order (x in the lowest bit, Fig 5.4): the number of in-grid boxes whose code
// is smaller, counted bit by bit.  For every set bit p of the code, the boxes
// sharing the bits above p and having 0 at p are counted per axis in closed
// form (their free low bits form a range intersected with the grid).
__device__ inline uint64_t morton_rank(int bx, int by, int bz, const int32_t dims[3]) {
    const int c[3] = {bx, by, bz};
    uint64_t rank = 0;
    for (int level = 10; level >= 0; --level) {
        for (int a = 2; a >= 0; --a) {
            int p = 3 * level + a;
            if (!((c[a] >> level) & 1)) continue;
            uint64_t prod = 1;
            for (int b = 0; b < 3; ++b) {
                int freebits;
                int64_t base;
                if (b == a) {
                    freebits = level;
                    base = ((int64_t)(c[b] >> (level + 1)) << (level + 1));
                } else {
                    freebits = (p - b + 2) / 3;
                    if (p < b) freebits = 0;
                    base = ((int64_t)(c[b] >> freebits) << freebits);
                }
                int64_t span = (int64_t)1 << freebits;
                int64_t cnt = (int64_t)dims[b] - base;
                if (cnt < 0) cnt = 0;
                if (cnt > span) cnt = span;
                prod *= (uint64_t)cnt;
            }
            rank += prod;
        }
    }
    return rank;
}

__global__ void __launch_bounds__(256) k_rs_rank(Dev d) {
    if (ABM_ABORTED(d) || !d.ctl->resort_now) return;
    const int64_t total = d.ctl->total_btiles;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int s = find_sim(d.btile_begin, d.n_sims, t);
        const SimDesc &S = d.sims[s];
        int64_t k0 = (t - d.btile_begin[s]) * kBoxTile;
        for (int q = threadIdx.x; q < kBoxTile; q += blockDim.x) {
            int64_t k = k0 + q;
            if (k >= S.nboxes) break;
            int bx = (int)(k % S.dims[0]);
            int64_t r = k / S.dims[0];
            int by = (int)(r % S.dims[1]);
            int bz = (int)(r / S.dims[1]);
            d.mrank[S.b_off + k] = (uint32_t)morton_rank(bx, by, bz, S.dims);
        }
    }
}

// Count agents per Morton rank of their current box (grid of this iteration).
__global__ void __launch_bounds__(256) k_rs_count(Dev d) {
    if (ABM_ABORTED(d) || !d.ctl->resort_now) return;
    const int P = d.ctl->pos_par;  // already flipped: the committed positions
    const int64_t A = d.A;
    const int64_t total = d.ctl->total_tiles;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int s = find_sim(d.tile_begin, d.n_sims, t);
        const SimDesc &S = d.sims[s];
        int64_t loc = (t - d.tile_begin[s]) * kTile + threadIdx.x;
        if (loc >= S.n || S.nboxes == 0) continue;
        int64_t i = S.a_off + loc;
        int bx = box_coord(d.pos[P][i], S.lo[0], S.L, S.dims[0]);
        int by = box_coord(d.pos[P][A + i], S.lo[1], S.L, S.dims[1]);
        int bz = box_coord(d.pos[P][2 * A + i], S.lo[2], S.L, S.dims[2]);
        uint32_t mr = d.mrank[S.b_off + linear_box(bx, by, bz, S.dims)];
        d.key[i] = mr;
        d.rank[i] = atomicAdd(&d.count[S.b_off + mr], 1u);
    }
}

// Move every agent to its Morton slot in the other buffers (out of place: the
// source buffers are only read).  Positions land in the other position
// buffer only, so every agent is marked as having differing buffers.
__global__ void __launch_bounds__(256) k_rs_move(Dev d) {
    if (ABM_ABORTED(d) || !d.ctl->resort_now) return;
    const int P = d.ctl->pos_par, lp = d.ctl->lay_par;
    const int64_t A = d.A;
    const int64_t total = d.ctl->total_tiles;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int s = find_sim(d.tile_begin, d.n_sims, t);
        const SimDesc &S = d.sims[s];
        int64_t loc = (t - d.tile_begin[s]) * kTile + threadIdx.x;
        if (loc >= S.n || S.nboxes == 0) continue;
        int64_t i = S.a_off + loc;
        int64_t j = (int64_t)d.box_start[S.sb_off + d.key[i]] + d.rank[i];
        const int nl = 1 - lp;
        for (int a = 0; a < 3; ++a) d.pos[1 - P][a * A + j] = d.pos[P][a * A + i];
        d.diam[nl][j] = d.diam[lp][i];
        d.vol[nl][j] = d.vol[lp][i];
        d.growth[nl][j] = d.growth[lp][i];
        d.uid[nl][j] = d.uid[lp][i];
        d.flags[nl][j] = d.flags[lp][i] | kBufDiff;
        d.nz[nl][j] = d.nz[lp][i];
    }
}

__global__ void k_rs_end(Dev d) {
    if (ABM_ABORTED(d) || !d.ctl->resort_now) return;
    if (threadIdx.x == 0) {
        d.ctl->lay_par ^= 1;
        d.ctl->pos_par ^= 1;
    }
}

// ------------------------------------------------------------------ statistics
// Deterministic two-level FP64 reductions: per-tile partials, then a fixed
// order per simulation.
__global__ void __launch_bounds__(256) k_stats_sum(Dev d, int pass, double *out) {
    __shared__ double red[4][4];
    const int P = d.ctl->pos_par;
    const int64_t A = d.A;
    const int64_t total = d.ctl->total_tiles;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int s = find_sim(d.tile_begin, d.n_sims, t);
        const SimDesc &S = d.sims[s];
        int64_t loc = (t - d.tile_begin[s]) * kTile + threadIdx.x;
        double v[3] = {0.0, 0.0, 0.0};
        if (loc < S.n) {
            int64_t i = S.a_off + loc;
            double x = d.pos[P][i], y = d.pos[P][A + i], z = d.pos[P][2 * A + i];
            if (pass == 0) {
                v[0] = x; v[1] = y; v[2] = z;
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
                atomicAdd(&d.hist_cnt[32 * s + b], 1u);
            }
        }
        // fixed-shape tree reduction: deterministic
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
        __syncthreads();
    }
}

// out layout per simulation (40 doubles): cx, cy, cz, hist_rmax, r_gyr, r_max, ...
__global__ void k_stats_fold(Dev d, int pass, double *out, double hist_rmax) {
    for (int s = threadIdx.x; s < d.n_sims; s += blockDim.x) {
        const SimDesc &S = d.sims[s];
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        for (int64_t t = d.tile_begin[s]; t < d.tile_begin[s + 1]; ++t) {
            a0 += d.stat_part[3 * t];
            a2 += d.stat_part[3 * t + 2];
            a1 = pass == 0 ? a1 + d.stat_part[3 * t + 1] : fmax(a1, d.stat_part[3 * t + 1]);
        }
        double *o = out + 40 * s;
        double n = (double)S.n;
        if (pass == 0) {
            o[0] = S.n > 0 ? a0 / n : 0.0;
            o[1] = S.n > 0 ? a1 / n : 0.0;
            o[2] = S.n > 0 ? a2 / n : 0.0;
            o[3] = hist_rmax;
            for (int b = 0; b < 32; ++b) d.hist_cnt[32 * s + b] = 0u;
        } else {
            o[4] = S.n > 0 ? sqrt(a0 / n) : 0.0;
            o[5] = a1;
        }
    }
}

__global__ void k_stats_hist(Dev d, double *out, float *hist) {
    for (int q = threadIdx.x; q < 32 * d.n_sims; q += blockDim.x) {
        int s = q / 32, b = q % 32;
        double w = out[40 * s + 3] / 32.0;
        double r0 = w * b, r1 = w * (b + 1);
        double shell = 4.0 / 3.0 * kPi * (r1 * r1 * r1 - r0 * r0 * r0);
        hist[q] = (float)((double)d.hist_cnt[q] / shell * 1000.0);
    }
}

// ------------------------------------------------------------------ launchers
static int grid_of(int want, int64_t cap_tiles) {
    int64_t g = cap_tiles < want ? cap_tiles : want;
    return g < 1 ? 1 : (int)g;
}

// Grid of the current positions (counting sort by box), then the arrival
// part of the static rule on that grid.
void launch_grid_build(const Dev &d, hipStream_t st, int grid_agents, int grid_boxes, bool any_static) {
    hipLaunchKernelGGL(k_begin, dim3(1), dim3(256), 0, st, d);
    hipLaunchKernelGGL(k_bounds, dim3(grid_agents), dim3(256), 0, st, d);
    hipLaunchKernelGGL(k_grid, dim3(1), dim3(256), 0, st, d);
    hipLaunchKernelGGL(k_bin, dim3(grid_agents), dim3(256), 0, st, d);
    hipLaunchKernelGGL(k_scan_tiles, dim3(grid_boxes), dim3(256), 0, st, d);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, d);
    hipLaunchKernelGGL(k_scan_apply, dim3(grid_boxes), dim3(256), 0, st, d);
    hipLaunchKernelGGL(k_scatter, dim3(grid_agents), dim3(256), 0, st, d);
    if (any_static) hipLaunchKernelGGL(k_static_fix, dim3(grid_agents), dim3(256), 0, st, d);
}

// The force sweep of one iteration (the dominant kernel).
void launch_sweep(const Dev &d, hipStream_t st, int grid_agents, int sweep_block, bool diag) {
    int sb = sweep_block;
    int sweep_grid = grid_agents * (kTile / sb > 0 ? kTile / sb : 1);
    if (diag) hipLaunchKernelGGL(k_sweep<true>, dim3(sweep_grid), dim3(sb), 0, st, d);
    else hipLaunchKernelGGL(k_sweep<false>, dim3(sweep_grid), dim3(sb), 0, st, d);
}

// Everything of one iteration after the sweep; ends by building the grid of
// the committed state.
void launch_after_sweep(const Dev &d, hipStream_t st, int grid_agents, int grid_boxes, bool diag, bool any_growth,
                        bool any_static, bool resort) {
    if (diag) hipLaunchKernelGGL(k_fixup<true>, dim3(256), dim3(256), 0, st, d);
    else hipLaunchKernelGGL(k_fixup<false>, dim3(256), dim3(256), 0, st, d);
    if (any_growth) {
        hipLaunchKernelGGL(k_div_mark, dim3(grid_agents), dim3(256), 0, st, d);
        hipLaunchKernelGGL(k_div_check, dim3(1), dim3(256), 0, st, d);
        hipLaunchKernelGGL(k_uscan_tiles, dim3(grid_boxes), dim3(256), 0, st, d);
        hipLaunchKernelGGL(k_uscan_top, dim3(1), dim3(1024), 0, st, d);
        hipLaunchKernelGGL(k_uscan_apply, dim3(grid_boxes), dim3(256), 0, st, d);
        hipLaunchKernelGGL(k_div_apply, dim3(grid_agents), dim3(256), 0, st, d);
    }
    if (any_static) {
        hipLaunchKernelGGL(k_static, dim3(grid_agents), dim3(256), 0, st, d);
        hipLaunchKernelGGL(k_clear_marks, dim3(grid_boxes), dim3(256), 0, st, d);
    }
    hipLaunchKernelGGL(k_end, dim3(1), dim3(256), 0, st, d);
    if (resort) {
        hipLaunchKernelGGL(k_rs_rank, dim3(grid_boxes), dim3(256), 0, st, d);
        hipLaunchKernelGGL(k_rs_count, dim3(grid_agents), dim3(256), 0, st, d);
        hipLaunchKernelGGL(k_scan_tiles, dim3(grid_boxes), dim3(256), 0, st, d);
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, d);
        hipLaunchKernelGGL(k_scan_apply, dim3(grid_boxes), dim3(256), 0, st, d);
        hipLaunchKernelGGL(k_rs_move, dim3(grid_agents), dim3(256), 0, st, d);
        hipLaunchKernelGGL(k_rs_end, dim3(1), dim3(64), 0, st, d);
    }
    launch_grid_build(d, st, grid_agents, grid_boxes, any_static);
}

// One iteration on the grid built at the end of the previous one.
void launch_iteration(const Dev &d, hipStream_t st, int grid_agents, int grid_boxes, int sweep_block, bool diag,
                      bool any_growth, bool any_static, bool resort) {
    launch_sweep(d, st, grid_agents, sweep_block, diag);
    launch_after_sweep(d, st, grid_agents, grid_boxes, diag, any_growth, any_static, resort);
}

// Statistics: out_dev holds 40 doubles per simulation followed by the
// histograms (n_sims x 32 floats).
void launch_stats(const Dev &d, hipStream_t st, int grid_agents, double hist_rmax, double *out_dev) {
    float *hist = (float *)(out_dev + 40 * d.n_sims);
    hipLaunchKernelGGL(k_stats_sum, dim3(grid_agents), dim3(256), 0, st, d, 0, out_dev);
    hipLaunchKernelGGL(k_stats_fold, dim3(1), dim3(256), 0, st, d, 0, out_dev, hist_rmax);
    hipLaunchKernelGGL(k_stats_sum, dim3(grid_agents), dim3(256), 0, st, d, 1, out_dev);
    hipLaunchKernelGGL(k_stats_fold, dim3(1), dim3(256), 0, st, d, 1, out_dev, hist_rmax);
    hipLaunchKernelGGL(k_stats_hist, dim3(1), dim3(1024), 0, st, d, out_dev, hist);
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

void launch_gather_pos(const Dev &d, hipStream_t st, int sim, double *dst, int64_t n, int64_t a_off) {
    int grid = (int)(n / 256 + 1);
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(k_gather_pos, dim3(grid), dim3(256), 0, st, d, sim, dst);
}

// Initial tile prefix (after create) so that statistics and queries work
// before the first step.
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

void launch_scatter_init(const Dev &d, hipStream_t st, int grid_agents) {
    hipLaunchKernelGGL(k_init_tiles, dim3(1), dim3(64), 0, st, d);
}

}  // namespace abm
