// abm_mech.hip -- force sweep, displacement, static rule, growth and division.
//
// Per iteration, on the grid built at the end of the previous one:
//   sweep     27-box force sum (Eq 4.1-4.2), threshold + cap (Sec 5.5), commit
//   fixup     FP64 re-evaluation of agents whose FP32 result cannot decide an
//             integer outcome (contact, non-zero force, neighbour, move)
//   div_*     grow-or-divide with prefix-sum append (Algorithm 2, Sec 5.3.2)
//   static    static flags for the next iteration (Sec 5.5)
//
// The sweep works on aligned 4x4x4 blocks of boxes, visited in Morton order
// with each XCD taking a contiguous range (its L2 then holds the shared halo).
// A workgroup stages the FP32 payload of the block and its one-box halo
// (6x6x6 boxes, about 730 agents at 3.4 agents per box) into LDS with
// coalesced reads, then each thread sweeps one target's 27 boxes from LDS.
//
// Forces are summed as exact 64-bit fixed-point integers (2^-40 units), so the
// result does not depend on the order in which neighbours are visited: every
// run is bitwise reproducible regardless of atomics (Sec 7.1.4 asks for this).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "abm_device.h"

namespace abm {

constexpr double kFixMagic = 6144.0;  // 1.5 * 2^12: fma(a, b, M) rounds a*b to 2^-40
constexpr double kFixUnit = 0x1.0p-40;
constexpr int kHalo = kBlk + 2;              // 6
constexpr int kNb = kHalo * kHalo * kHalo;   // 216 staged boxes
constexpr int kCore = kBlk * kBlk * kBlk;    // 64 target boxes
constexpr int kStage = 2048;                 // staged agents (32 KB of float4)

__device__ inline unsigned long long fixbits(double v) { return (unsigned long long)__double_as_longlong(v); }

// ------------------------------------------------------------------ commit helpers
// Displacement as the thesis's rule reads: no motion unless |F| > a, else
// F*dt/m capped in Euclidean norm (FP64, IEEE ops, no contraction).
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
// m: Morton rank of the agent's box; lin: its linear id (diagnostics).
template <bool DIAG>
__device__ inline void commit_agent(const Dev &d, const SimDesc &S, int64_t i, int P, int lp, uint8_t fl, double x,
                                    double y, double z, double fx, double fy, double fz, int nz, int nbr,
                                    int contacts, uint32_t m, int64_t lin) {
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
        if (S.detect_static) d.dirty[S.b_off + m] = 1;  // start box of a changed agent
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
        d.boxid[i] = lin;
    }
}

// A static agent: no force, no motion, non-zero-force count kept (Sec 5.5).
template <bool DIAG>
__device__ inline void skip_static(const Dev &d, int64_t i, int P, int lp, uint8_t fl, int64_t lin) {
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
        d.boxid[i] = lin;
    }
}

// Per-target accumulator of the FP32 sweep.
struct Acc {
    unsigned long long ax, ay, az;  // force components in 2^-40 units, plus nfix * magic bits (mod 2^64)
    uint32_t eacc;         // error bound in 2^-26 units (rounded up per pair)
    int contacts, nz, nbr, nfix;
    bool unc;              // an integer outcome is not decidable in FP32
};

// Contact part of one pair: (ddx,ddy,ddz) = target minus candidate, d2 its
// squared length, ri/rj the radii.  Decides contact (delta > 0) and non-zero
// force, accumulates the force in fixed point and its error bound; marks the
// target undecidable when FP32 cannot certify an integer outcome.
__device__ inline void pair_contact(Acc &a, float ddx, float ddy, float ddz, float d2, float ri, float rj, float e,
                                    float g, float kf, float gf, float L2m, float L2p) {
    const float sr = ri + rj;
    const float sg = sr + g;
    if (!(d2 < sg * sg)) return;
    if (d2 >= L2m) {  // only possible when the box length is below the largest diameter
        if (d2 < L2p) a.unc = true;
        return;
    }
    const float dist = sqrtf(d2);
    const float delta = sr - dist;
    if (delta <= e) {
        if (delta >= -e) a.unc = true;
        return;
    }
    ++a.contacts;
    const float rbar = ri * rj * __builtin_amdgcn_rcpf(sr);
    const float sq = sqrtf(rbar * delta);
    const float kd = kf * delta, gs = gf * sq;
    const float fn = kd - gs;
    // bound on |fn error|: conditioning of Eq 4.1 times the overlap error,
    // plus FP32 rounding relative to the magnitudes of both terms
    const float ep = (kf + 0.5f * gs * __builtin_amdgcn_rcpf(delta)) * e + (kd + gs) * 0x1.0p-19f;
    if (ep >= 0x1.0p-6f || fabsf(fn) <= ep) {
        a.unc = true;
        return;
    }
    ++a.nz;
    const double f = (double)(fn * __builtin_amdgcn_rcpf(dist));
    a.ax += fixbits(fma(f, (double)ddx, kFixMagic));
    a.ay += fixbits(fma(f, (double)ddy, kFixMagic));
    a.az += fixbits(fma(f, (double)ddz, kFixMagic));
    ++a.nfix;
    a.eacc += (uint32_t)ceilf(ep * 0x1.0p26f);
}

// One candidate pair in FP32 box-relative coordinates (global-memory path).
// (qx,qy,qz) = target coordinate minus the box offset of the candidate's box.
template <bool DIAG>
__device__ inline void pair_fp32(Acc &a, float qx, float qy, float qz, float ri, float4 c, float e, float g, float kf,
                                 float gf, float L2m, float L2p) {
    const float ddx = qx - c.x, ddy = qy - c.y, ddz = qz - c.z;
    const float d2 = fmaf(ddz, ddz, fmaf(ddy, ddy, ddx * ddx));
    if (DIAG) {
        if (d2 < L2m) ++a.nbr;
        else if (d2 < L2p) a.unc = true;
    }
    pair_contact(a, ddx, ddy, ddz, d2, ri, c.w, e, g, kf, gf, L2m, L2p);
}

// ------------------------------------------------------------------ sweep
constexpr int kList = 32;  // per-thread list of candidates within reach (u16 LDS indices)
constexpr int kChunk = 16;  // candidates tested between two list-room checks

__device__ inline uint32_t wave_max_u32(uint32_t v) {
    for (int off = 32; off > 0; off >>= 1) {
        uint32_t o = __shfl_xor(v, off);
        v = o > v ? o : v;
    }
    return __builtin_amdgcn_readfirstlane(v);
}

// Contact math of the listed candidates (phase 2), block-relative FP32
// coordinates.  Wave-uniform loop with predication: no branches per entry.
// Coincident or near-coincident centres, overlaps and forces within their
// FP32 error bound of a decision threshold mark the target for FP64.
__device__ inline void drain_list(Acc &a, const float4 *sp, const uint16_t *lst, uint32_t n, uint32_t self, float4 own,
                                  float e, float g, float kf, float gf, float L2m, float L2p) {
    const uint32_t nmax = wave_max_u32(n);
    for (uint32_t k = 0; k < nmax; ++k) {
        uint32_t q = lst[k * 256 + threadIdx.x];
        q = q < (uint32_t)kStage ? q : 0u;
        const bool valid = k < n && q != self;
        const float4 c = sp[q];
        const float ddx = valid ? own.x - c.x : 0.0f;
        const float ddy = valid ? own.y - c.y : 0.0f;
        const float ddz = valid ? own.z - c.z : 0.0f;
        const float rj = valid ? c.w : 0.0f;
        const float d2 = fmaf(ddz, ddz, fmaf(ddy, ddy, ddx * ddx));
        const float sr = own.w + rj;
        const float sg = sr + g;
        bool cand = valid && d2 < sg * sg;
        const bool beyond = d2 >= L2m;  // only when the box length is below the largest diameter
        bool unc = cand && beyond && d2 < L2p;
        unc |= cand && d2 < g * g;  // (near-)coincident centres: direction left to FP64
        cand = cand && !beyond && d2 >= g * g;
        const float dist = __builtin_amdgcn_sqrtf(d2);
        const float delta = sr - dist;
        unc |= cand && delta <= e && delta >= -e;
        bool contact = cand && delta > e;
        const float rbar = own.w * rj * __builtin_amdgcn_rcpf(sr);
        const float sq = __builtin_amdgcn_sqrtf(fmaxf(rbar * delta, 0.0f));
        const float kd = kf * delta, gs = gf * sq;
        const float fn = kd - gs;
        const float ep = (kf + 0.5f * gs * __builtin_amdgcn_rcpf(delta)) * e + (kd + gs) * 0x1.0p-19f;
        const bool bad = contact && (ep >= 0x1.0p-6f || fabsf(fn) <= ep);
        unc |= bad;
        contact = contact && !bad;
        a.unc |= unc;
        a.contacts += contact ? 1 : 0;
        a.nz += contact ? 1 : 0;
        const double f = contact ? (double)(fn * __builtin_amdgcn_rcpf(dist)) : 0.0;
        a.ax += fixbits(fma(f, (double)ddx, kFixMagic));
        a.ay += fixbits(fma(f, (double)ddy, kFixMagic));
        a.az += fixbits(fma(f, (double)ddz, kFixMagic));
        ++a.nfix;
        a.eacc += contact ? (uint32_t)ceilf(ep * 0x1.0p26f) : 0u;
    }
}

template <bool DIAG>
__global__ void __launch_bounds__(256) k_sweep(Dev d) {
    __shared__ float4 sp[kStage];            // staged payload, block-relative coordinates
    __shared__ uint16_t lst[kList * 256];    // per-thread candidate lists, thread-interleaved
    __shared__ uint32_t sbeg[kNb + 1];       // exclusive prefix of the staged box counts
    __shared__ uint32_t gsrc[kNb];           // global slot start of every staged box
    __shared__ uint32_t coff[kCore + 1];
    __shared__ uint32_t scnt[kNb];
    __shared__ uint32_t sh[4];
    if (ABM_ABORTED(d)) return;
    const int P = d.ctl->pos_par, lp = d.ctl->lay_par;
    const int64_t A = d.A;
    const int64_t U = d.ctl->total_units;
    const int tid = threadIdx.x;
    // blocks are dealt to the 8 XCDs round-robin: give each XCD a contiguous
    // Morton range of work units so that neighbouring blocks share its L2
    const int xcd = blockIdx.x & 7;
    const int64_t per_xcd = (int64_t)(gridDim.x >> 3);
    const int64_t chunk = ceil_div(U, 8);
    const int64_t u_end = (xcd + 1) * chunk < U ? (xcd + 1) * chunk : U;
    for (int64_t u = xcd * chunk + (blockIdx.x >> 3); u < u_end; u += per_xcd) {
        const int s = find_sim(d.wblk_begin, d.n_sims, u);
        const SimDesc &S = d.sims[s];
        int qx, qy, qz;
        unpack_key(d.blist[S.b_off + (u - d.wblk_begin[s])], qx, qy, qz);
        // table of the 6x6x6 staged boxes (x fastest)
        uint32_t cnt = 0;
        if (tid < kNb) {
            const int lx = tid % kHalo, ly = (tid / kHalo) % kHalo, lz = tid / (kHalo * kHalo);
            const int gx = qx * kBlk + lx - 1, gy = qy * kBlk + ly - 1, gz = qz * kBlk + lz - 1;
            uint32_t src = 0;
            if (gx >= 0 && gy >= 0 && gz >= 0 && gx < S.dims[0] && gy < S.dims[1] && gz < S.dims[2]) {
                const uint32_t m = d.mrank[S.b_off + linear_box(gx, gy, gz, S.dims)];
                src = d.box_start[S.sb_off + m];
                cnt = d.box_start[S.sb_off + m + 1] - src;
            }
            gsrc[tid] = src;
            scnt[tid] = cnt;
        }
        uint32_t v[4] = {cnt, 0u, 0u, 0u};
        uint32_t total;
        const uint32_t pre = block_excl_scan_4(v, sh, total);
        if (tid < kNb) sbeg[tid] = pre;
        if (tid == 0) sbeg[kNb] = total;
        __syncthreads();
        if (tid < 64) {  // prefix of the target counts over the 64 core boxes (one wave)
            const int lb = (tid % 4 + 1) + kHalo * ((tid / 4 % 4 + 1) + kHalo * (tid / 16 + 1));
            const uint32_t cc = scnt[lb];
            uint32_t x = cc;
            for (int off = 1; off < 64; off <<= 1) {
                uint32_t y = __shfl_up(x, off);
                if (tid >= off) x += y;
            }
            coff[tid] = x - cc;
            if (tid == 63) coff[64] = x;
        }
        const float Lf = (float)S.L;
        const bool staged = total <= (uint32_t)kStage;
        if (staged) {
            // box-relative -> relative to the centre of the 6x6x6 region (|x| < 3L)
            for (uint32_t e = tid; e < total; e += blockDim.x) {
                int lo = 0, hi = kNb;  // largest lb with sbeg[lb] <= e
                while (hi - lo > 1) {
                    int mid = (lo + hi) >> 1;
                    if (sbeg[mid] <= e) lo = mid; else hi = mid;
                }
                float4 c = d.payload[gsrc[lo] + (e - sbeg[lo])];
                const int lx = lo % kHalo, ly = (lo / kHalo) % kHalo, lz = lo / (kHalo * kHalo);
                c.x += (float)(lx - 3) * Lf;
                c.y += (float)(ly - 3) * Lf;
                c.z += (float)(lz - 3) * Lf;
                sp[e] = c;
            }
        }
        __syncthreads();
        const uint32_t nt = coff[64];
        const float e = S.e_delta, g = 2.0f * e;
        const float kf = (float)S.k, gf = (float)S.gamma;
        const float L2 = (float)(S.L * S.L);
        const float G = (float)ldexp(S.L * S.L, -18);
        const float L2m = L2 - G, L2p = L2 + G;
        const float rmaxg = (float)S.rmax + g;
        for (uint32_t t0 = 0; t0 < nt; t0 += blockDim.x) {
            // all lanes run the loop body (wave-uniform inner loops); lanes
            // without a target, and static targets, are predicated off
            const uint32_t t = t0 + tid < nt ? t0 + tid : nt - 1;
            bool act = t0 + tid < nt;
            int c = 0, hi = kCore;  // core box of target t
            while (hi - c > 1) {
                int mid = (c + hi) >> 1;
                if (coff[mid] <= t) c = mid; else hi = mid;
            }
            const int cx = c % 4, cy = c / 4 % 4, cz = c / 16;
            const int lb = (cx + 1) + kHalo * ((cy + 1) + kHalo * (cz + 1));
            const uint32_t k = t - coff[c];
            const uint32_t slot = gsrc[lb] + k;
            const uint32_t self = staged ? sbeg[lb] + k : slot;
            const int64_t i = d.sorted_idx[slot];
            const int bx = qx * kBlk + cx, by = qy * kBlk + cy, bz = qz * kBlk + cz;
            const int64_t lin = linear_box(bx, by, bz, S.dims);
            const uint8_t fl = d.flags[lp][i];
            if (act && S.detect_static && (fl & kStatic)) {
                skip_static<DIAG>(d, i, P, lp, fl, lin);
                act = false;
            }
            Acc a = {0, 0, 0, 0u, 0, 0, 0, 0, false};
            if (staged) {
                // phase 1: distance pre-test against the reach of the largest
                // agent; survivors go to the thread's list; phase 2: contacts
                const float4 own = sp[self];
                const float R = own.w + rmaxg;
                const float R2 = fminf(R * R, L2p);
                uint32_t n = 0;
                for (int r = 0; r < 9; ++r) {
                    const int row = cx + kHalo * ((cy + r % 3) + kHalo * (cz + r / 3));  // boxes cx..cx+2
                    const uint32_t b0 = sbeg[row];
                    const uint32_t len = act ? sbeg[row + 3] - b0 : 0u;
                    const uint32_t kmax = wave_max_u32(len);
                    for (uint32_t k0 = 0; k0 < kmax; k0 += kChunk) {
                        if (__ballot(n + kChunk > (uint32_t)kList)) {
                            drain_list(a, sp, lst, n, self, own, e, g, kf, gf, L2m, L2p);
                            n = 0;
                        }
                        const uint32_t k1 = k0 + kChunk < kmax ? k0 + kChunk : kmax;
                        for (uint32_t kk = k0; kk < k1; ++kk) {
                            const bool in = kk < len;
                            const uint32_t q = in ? b0 + kk : 0u;
                            const float4 cc = sp[q];
                            const float ddx = own.x - cc.x, ddy = own.y - cc.y, ddz = own.z - cc.z;
                            const float d2 = fmaf(ddz, ddz, fmaf(ddy, ddy, ddx * ddx));
                            if (DIAG) {
                                const bool other = in && q != self;
                                a.nbr += (other && d2 < L2m) ? 1 : 0;
                                a.unc |= other && d2 >= L2m && d2 < L2p;
                            }
                            lst[n * 256 + tid] = (uint16_t)q;
                            n += (in && d2 < R2) ? 1u : 0u;
                        }
                    }
                }
                drain_list(a, sp, lst, n, self, own, e, g, kf, gf, L2m, L2p);
            } else if (act) {
                const float4 own = d.payload[slot];
                for (int oz = -1; oz <= 1; ++oz) {
                    for (int oy = -1; oy <= 1; ++oy) {
                        const int row = cx + kHalo * ((cy + 1 + oy) + kHalo * (cz + 1 + oz));
                        const float qy2 = own.y - (float)oy * Lf;
                        const float qz2 = own.z - (float)oz * Lf;
                        for (int ox = -1; ox <= 1; ++ox) {
                            const int lbb = row + ox + 1;
                            const float qx2 = own.x - (float)ox * Lf;
                            const uint32_t b0 = gsrc[lbb], nn = sbeg[lbb + 1] - sbeg[lbb];
                            for (uint32_t q = b0; q < b0 + nn; ++q)
                                if (q != self)
                                    pair_fp32<DIAG>(a, qx2, qy2, qz2, own.w, d.payload[q], e, g, kf, gf, L2m, L2p);
                        }
                    }
                }
            }
            if (!act) continue;
            bool unc = a.unc;
            if (!unc) {
                const unsigned long long mb = (unsigned long long)a.nfix * fixbits(kFixMagic);
                const double fx = (double)(long long)(a.ax - mb) * kFixUnit;
                const double fy = (double)(long long)(a.ay - mb) * kFixUnit;
                const double fz = (double)(long long)(a.az - mb) * kFixUnit;
                const double fnorm = sqrt(fx * fx + fy * fy + fz * fz);
                const double ebound = (double)a.eacc * 0x1.0p-26 + 1e-9;
                if (fabs(fnorm - S.adherence) <= ebound) {
                    unc = true;
                } else {
                    const uint32_t m = d.mrank[S.b_off + lin];
                    commit_agent<DIAG>(d, S, i, P, lp, fl, d.pos[P][i], d.pos[P][A + i], d.pos[P][2 * A + i], fx, fy,
                                       fz, a.nz, a.nbr, a.contacts, m, lin);
                }
            }
            if (unc) {
                uint32_t q = atomicAdd(&d.ctl->n_fix, 1u);
                d.fix_list[q] = (uint32_t)i;
            }
        }
        __syncthreads();  // the next unit reuses the LDS tables
    }
}

// ------------------------------------------------------------------ fixup
// Order-independent sum of FP64 terms: every term is rounded to a multiple
// of 2^-80 (round half up in magnitude) and added into a 128-bit two's
// complement integer, so the result does not depend on the order in which
// the neighbours are met.  Terms of magnitude 2^36 and above set `wide`
// (the caller then falls back to a plain FP64 sum); with fewer than 2^11
// terms the integer cannot overflow.
struct Fix128 {
    uint64_t lo = 0, hi = 0;
    bool wide = false;
    __device__ void add(double t) {
        const uint64_t bits = (uint64_t)__double_as_longlong(t);
        const int E = (int)((bits >> 52) & 0x7ff);
        if (E == 0) return;  // zero or subnormal: below 2^-80
        if (E >= 1023 + 36) {
            wide = true;
            return;
        }
        const uint64_t m = (bits & 0xfffffffffffffull) | (1ull << 52);
        const int sh = E - 1075 + 80;  // value = m * 2^sh units of 2^-80, sh < 49
        uint64_t vlo, vhi;
        if (sh >= 0) {
            vlo = m << sh;
            vhi = sh == 0 ? 0ull : m >> (64 - sh);
        } else if (sh > -54) {
            const uint64_t half = 1ull << (-sh - 1);
            vlo = (m + half) >> (-sh);
            vhi = 0;
        } else {
            return;
        }
        if (bits >> 63) {  // subtract
            const uint64_t nlo = lo - vlo;
            hi = hi - vhi - (nlo > lo ? 1ull : 0ull);
            lo = nlo;
        } else {
            const uint64_t nlo = lo + vlo;
            hi = hi + vhi + (nlo < lo ? 1ull : 0ull);
            lo = nlo;
        }
    }
    __device__ double value() const {
        uint64_t l = lo, h = hi;
        const bool neg = (int64_t)h < 0;
        if (neg) {  // magnitude
            l = ~l + 1ull;
            h = ~h + (l == 0 ? 1ull : 0ull);
        }
        // two roundings: deterministic, within one ulp of the exact sum
        const double r = ((double)h * 0x1.0p64 + (double)l) * 0x1.0p-80;
        return neg ? -r : r;
    }
};

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
        double fx = 0.0, fy = 0.0, fz = 0.0;  // plain sums, used only when a term is huge
        Fix128 sx, sy, sz;
        int nbr = 0, contacts = 0, nzc = 0;
        for (int oz = -1; oz <= 1; ++oz)
            for (int oy = -1; oy <= 1; ++oy)
                for (int ox = -1; ox <= 1; ++ox) {
                    int cx = bx + ox, cy = by + oy, cz = bz + oz;
                    if (cx < 0 || cy < 0 || cz < 0 || cx >= S.dims[0] || cy >= S.dims[1] || cz >= S.dims[2]) continue;
                    uint32_t m = d.mrank[S.b_off + linear_box(cx, cy, cz, S.dims)];
                    uint32_t s0 = d.box_start[S.sb_off + m], s1 = d.box_start[S.sb_off + m + 1];
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
                            const double tx = fn * ddx / dist, ty = fn * ddy / dist, tz = fn * ddz / dist;
                            fx += tx;
                            fy += ty;
                            fz += tz;
                            sx.add(tx);
                            sy.add(ty);
                            sz.add(tz);
                        }
                    }
                }
        if (!(sx.wide || sy.wide || sz.wide)) {
            fx = sx.value();
            fy = sy.value();
            fz = sz.value();
        }
        const int64_t lin = linear_box(bx, by, bz, S.dims);
        commit_agent<DIAG>(d, S, i, P, lp, fl, x, y, z, fx, fy, fz, nzc, nbr, contacts, d.mrank[S.b_off + lin], lin);
    }
}

// ------------------------------------------------------------------ growth and division
// Correctly rounded cube root: ocml's cbrt is within one ulp; the candidate
// is corrected by the sign of (y +- ulp/2)^3 - t, evaluated with error-free
// products (TwoProd via fma, Ogita-Rump-Oishi).
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
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Uniform unit vector for a division, keyed by (seed; uid, iteration, sim):
// Archimedes' construction, z uniform in [-1, 1) and a uniform azimuth.
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
            d.pos[Q][j] = jx;
            d.pos[Q][A + j] = jy;
            d.pos[Q][2 * A + j] = jz;
            d.pos[Q][i] = mx;
            d.pos[Q][A + i] = my;
            d.pos[Q][2 * A + i] = mz;
            d.vol[lp][i] = half;
            d.vol[lp][j] = half;
            d.diam[lp][i] = dnew;
            d.diam[lp][j] = dnew;
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
        if (S.detect_static) d.dirty[S.b_off + key_rank(d, S, d.key[i])] = 1;  // start box of a changed agent
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
                        uint32_t m = d.mrank[S.b_off + linear_box(cx, cy, cz, S.dims)];
                        if (!d.dirty[S.b_off + m]) continue;
                        uint32_t s0 = d.box_start[S.sb_off + m], s1 = d.box_start[S.sb_off + m + 1];
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

// ------------------------------------------------------------------ launchers
void launch_sweep(const Dev &d, hipStream_t st, int sweep_grid, bool diag) {
    if (diag) hipLaunchKernelGGL(k_sweep<true>, dim3(sweep_grid), dim3(256), 0, st, d);
    else hipLaunchKernelGGL(k_sweep<false>, dim3(sweep_grid), dim3(256), 0, st, d);
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
    if (any_static) hipLaunchKernelGGL(k_static, dim3(grid_agents), dim3(256), 0, st, d);
    launch_end(d, st, grid_boxes, any_static);
    if (resort) launch_resort(d, st, grid_agents, grid_boxes, false);
    launch_grid_build(d, st, grid_agents, grid_boxes, any_static);
}

// One iteration on the grid built at the end of the previous one.
void launch_iteration(const Dev &d, hipStream_t st, int grid_agents, int grid_boxes, int sweep_grid, bool diag,
                      bool any_growth, bool any_static, bool resort) {
    launch_sweep(d, st, sweep_grid, diag);
    launch_after_sweep(d, st, grid_agents, grid_boxes, diag, any_growth, any_static, resort);
}

}  // namespace abm
