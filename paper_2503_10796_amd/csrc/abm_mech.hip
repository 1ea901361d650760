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
// coalesced reads, then sweeps the targets' candidate rows from LDS as
// length-sorted tasks, one per lane.
//
// Forces are summed as exact 64-bit fixed-point integers (2^-40 units), so the
// result does not depend on the order in which neighbours are visited: every
// run is bitwise reproducible regardless of atomics (Sec 7.1.4 asks for this).
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "abm_device.h"

namespace abm {

// Force sums are exact fixed-point integers in units of 2^-34: fma(a, b, M)
// with M = 1.5 * 2^18 rounds a*b (|a*b| < 2^17) to a multiple of 2^-34, and
// the bits of the result minus those of M are that multiple.
constexpr double kFixMagic = 393216.0;
constexpr double kFixUnit = 0x1.0p-34;
// Lengths in the sweep are in units of U = L 2^-kFixBits (payload coordinates,
// radii).  In these units the box length and its square are powers of two.
constexpr int32_t kUnitL = 1 << kFixBits;               // L
constexpr float kUnitLf = (float)(1 << kFixBits);
constexpr double kL2U = 0x1.0p56;                        // L^2
// Band around L^2 where the neighbour test is left to FP64: the quantised
// centres are within sqrt(3) U of the true ones, so d^2 moves by at most
// 2 L sqrt(3) U + 3 U^2 < 2^30 U^2 near d = L (plus both sides' FP64 rounding).
constexpr double kNbrBand = 0x1.0p30 + 64.0;
// The FP32 reach test keeps every pair with d < r_i + r_j + kReach (U units,
// 2^-18 L): it covers the FP32 rounding of the squared distance (about 2^-22
// relative), the quantisation of the centres and the radii.
constexpr float kReach = 1024.0f;
constexpr int kHalo = kBlk + 2;              // 6
constexpr int kNb = kHalo * kHalo * kHalo;   // 216 staged boxes
constexpr int kCore = kBlk * kBlk * kBlk;    // 64 target boxes
constexpr int kStage = 928;                  // staged agents (14.5 KB of payload)
static_assert(kStage >= 4 * 64, "the dense path uses 64 staged entries per wave of a 256-thread block");

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
// m: Morton rank of the agent's box; lin: its linear id (recorded fields).
// With DIAG or the ABM_RECORD flag of the simulation, the force, displacement,
// contact count and box are recorded (the neighbour count only with DIAG).
template <bool DIAG>
__device__ inline void commit_agent(const Dev &d, const SimDesc &S, int64_t i, int P, int lp, uint8_t fl, double x,
                                    double y, double z, double fx, double fy, double fz, int nz, int nbr,
                                    int contacts, uint32_t m, int64_t lin) {
#pragma clang fp contract(off)
    const int64_t A = d.A;
    double dx, dy, dz;
    displacement64(fx, fy, fz, S, dx, dy, dz);
    // Algorithm 2: the Brownian step comes first, then the mechanical
    // displacement: x' = (x + b) + d
    double b[3] = {0.0, 0.0, 0.0};
    if (S.brownian_rate > 0.0) brownian_step(S.seed, S.sim_id, d.uid[lp][i], (uint64_t)d.ctl->iter, S.brownian_rate, b);
    const double nx = (x + b[0]) + dx, ny = (y + b[1]) + dy, nzz = (z + b[2]) + dz;
    const bool moved = nx != x || ny != y || nzz != z;
    d.nz[lp][i] = (uint8_t)(nz > 255 ? 255 : nz);
    fl &= (uint8_t)~kChgMask;
    if (moved) {
        d.pos[1 - P][i] = nx;
        d.pos[1 - P][A + i] = ny;
        d.pos[1 - P][2 * A + i] = nzz;
        d.flags[lp][i] = fl | kBufDiff | kMoved;
        if (S.detect_static) mark_box(d.dirty, d.dirty_blk, S, m);  // start box of a changed agent
    } else {
        if (fl & kBufDiff) {
            d.pos[1 - P][i] = x;
            d.pos[1 - P][A + i] = y;
            d.pos[1 - P][2 * A + i] = z;
            fl &= (uint8_t)~kBufDiff;
        }
        d.flags[lp][i] = fl;
    }
    if (DIAG || (S.flags & ABM_RECORD)) {
        d.nbr[i] = DIAG ? nbr : -1;
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
__device__ inline void skip_static(const Dev &d, const SimDesc &S, int64_t i, int P, int lp, uint8_t fl, int64_t lin) {
    const int64_t A = d.A;
    if (fl & kBufDiff) {
        d.pos[1 - P][i] = d.pos[P][i];
        d.pos[1 - P][A + i] = d.pos[P][A + i];
        d.pos[1 - P][2 * A + i] = d.pos[P][2 * A + i];
    }
    if (fl & (kBufDiff | kChgMask)) d.flags[lp][i] = fl & (uint8_t) ~(kBufDiff | kChgMask);
    if (DIAG || (S.flags & ABM_RECORD)) {
        d.nbr[i] = -1;
        d.contacts[i] = -1;
        for (int a = 0; a < 3; ++a) {
            d.force[3 * i + a] = 0.0;
            d.disp[3 * i + a] = 0.0;
        }
        d.boxid[i] = lin;
    }
}

// ------------------------------------------------------------------ sweep
// Per work unit (an aligned 4x4x4 block of boxes):
//   table    start and count of the 6x6x6 staged boxes (block scan)
//   stage    FP32 payload of the region into LDS, relative to its centre
//   setup    per target: static skip (Sec 5.5) or up to ten tasks, one per row
//            of three boxes (x-1..x+1) of its 27-box neighbourhood trimmed to
//            the reach (plus the own row's halo box under the half shell); the
//            tasks are counting-sorted by row length, so the 64 lanes of a
//            wave hold rows of about equal length and run equal trip counts
//   sweep    each lane tests its row against the pair's contact reach plus
//            the guard band; survivors go to a per-wave LDS queue, which is
//            drained 64 pairs at a time through the contact math (Eq 4.1-4.2)
//            with exact fixed-point LDS atomics into per-target accumulators
//   commit   per target: threshold, displacement, write-back (or FP64 path)
// Units whose region does not fit in LDS (dense packings) take a box-wise
// path that reads the payload from global memory.
constexpr int kMaxT = 280;      // targets per unit on the LDS path (mean 216 at 1 agent per 1000 um^3)
constexpr int kRows = 10;       // tasks per target: nine rows, the own row's left halo box apart
constexpr int kTaskCap = 2048;  // tasks per unit on the LDS path (about 7.5 per target)
constexpr int kBuckets = 64;    // task lengths 1..63, longer rows share the last bucket
constexpr int kQueue = 128;     // per-wave survivor queue (entries: target << 20 | target's staged
                                // index << 10 | candidate's staged index)
constexpr uint16_t kNoTarget = 0xffff;
// Accumulator words of a target on the LDS path.  acc[0..2]: the force
// components as 52-bit two's complement fixed point (2^-34 units, |F| < 2^17)
// with a count in the top 12 bits: contacts (x word) and pairs FP32 could not
// decide (y word).  Both fields are linear, so any order of additions gives
// the same words.  At most kStage - 1 pairs per target keep every field in
// range (forces of at most 64 per pair, counts below 4096).
constexpr int kCntShift = 52;
constexpr unsigned long long kCnt1 = 1ull << kCntShift;
__device__ inline long long fix_field(unsigned long long w) { return (long long)(w << 12) >> 12; }
__device__ inline uint32_t cnt_field(unsigned long long w, long long f) {
    return (uint32_t)((w - (unsigned long long)f) >> kCntShift);
}
// acm: the pairs' force error bounds (2^-28 units, rounded up) << 32 | lower
// bounds of their |F_N| (2^-17 units, each at most 32): below 2^32 each for
// kStage - 1 pairs.

template <bool DIAG>
struct SweepLds {
    Pay sp[kStage + 1];                     // staged payload, relative to the region centre (one
                                            // entry past the largest stage: read ahead, unused)
    unsigned long long acc[3][kMaxT];       // force x | contacts, force y | undecided pairs, force z
    unsigned long long acm[kMaxT];          // error bound << 32 | lower bound of sum |F_N|
    uint32_t anbr[DIAG ? kMaxT : 1];        // neighbours within the box length
    uint32_t sbeg[kNb + 1];                 // exclusive prefix of the staged box counts
    uint32_t gsrc[kNb];                     // global slot start of every staged box
    uint32_t coff[kCore + 1];               // prefix of the target counts of the core boxes
    uint32_t bcnt[kBuckets], boff[kBuckets];
    uint32_t queue[4][kQueue + 1];          // (+1: a spare slot that lanes without a survivor write)
    uint32_t sh[4];                         // per-wave flags: an active target, a static target
    unsigned long long sh64[4];             // per-wave totals of the table scan
    uint32_t ntask;
    unsigned long long ahead[2][4];         // look-ahead over units: active-unit ballots of the 4 waves
    uint32_t task[kTaskCap];                // target | first candidate << 9 | candidates << 19,
                                            // sorted by length (longest first); before the
                                            // setup, the staged box of every staged agent (bytes)
    uint16_t tself[kMaxT];                  // staged index of each target (kNoTarget: static)
    uint32_t tidx[kMaxT];                   // agent index of each target
    uint16_t tmap[kStage];                  // target of each staged agent (kNoTarget: halo or static)
    uint8_t tbox[kMaxT];                    // core box of each target
};
static_assert(sizeof(SweepLds<false>) <= 40960, "four blocks of 256 threads per CU");
static_assert(kStage < 1024 && kMaxT < 512, "queue and task entries: 9-bit target, 10-bit staged indices");
static_assert(kNb <= 256 && kStage <= 4 * kTaskCap, "the stage map: one byte per staged agent in the task list");
static_assert(kStage < 4096, "count fields of the accumulator words");

// Per-target accumulator of the global-memory path (diagnostic box-wise sweep).
struct Acc {
    unsigned long long ax, ay, az;  // force components in 2^-34 units, plus nfix * magic bits (mod 2^64)
    unsigned long long eacc, sacc;  // error bound (2^-28 units), lower bound of sum |F_N| (2^-17 units)
    int contacts, nbr, nfix;
    int unc;                        // pairs whose integer outcome FP32 cannot decide
};

// Contact math of one pair (Eq 4.1-4.2).  (dx, dy, dz): target minus candidate
// centre, exact integers in units of U = L 2^-kFixBits held in doubles; d2:
// their squared length (FP64); ri, rj: radii in units of U (FP32).
//   overlap   delta = r_i + r_j - d = ((r_i + r_j)^2 - d^2) / (r_i + r_j + d):
//             the numerator in FP64 (no cancellation error), the rest in FP32
//             (at most 3.75 * 2^-23 relative with one-ulp sqrt and rcp), plus
//             the quantisation of the inputs (centres within U/2 per axis,
//             radii within 2^-24 relative):
//             e = 1.74 U + 1.01 * 2^-24 (r_i + r_j) + 2^-21 |delta| bounds it
//   force     F_N = k delta - gamma sqrt(rbar delta) in FP32 (kU = k U,
//             gU = gamma U: lengths in units of U), factor F_N / d
// Certain outcomes: contact iff delta > 4e (below, the pair is undecided);
// a neighbour within the box length iff d^2 < L^2 - band.  The pair is
// undecided (the target goes to the FP64 path) when the overlap is within
// 4e of zero, d^2 is within the band of L^2, the centres (nearly) coincide,
// its force cannot be told from zero (so the non-zero-force count is exact),
// or its error bound or force is too large for the accumulator words.
//   ep        bound on the error of the pair's force vector: the overlap
//             error times a bound of |dF_N/d delta| = |k - h(delta)| over
//             [delta - e, delta + e], h = gamma sqrt(rbar) / (2 sqrt(delta)):
//             |k - h| + 0.16 h with delta > 4e (h grows by at most
//             sqrt(4/3) there); the FP32 rounding of Eq 4.1 (k delta to 2
//             ulp, the square-root term to 8.5 ulp with the radii's
//             quantisation in rbar, the difference to one); the error of the
//             unit vector times |F_N| (2 sqrt(3) U / d from the quantised
//             centres, 5.5 ulp from the distance, rcp and product); and the
//             fixed-point rounding of the sum.
struct PairOut {
    bool contact;  // a certain contact with a certain non-zero force
    bool unc;      // an integer outcome is not decidable here
    float f;       // F_N / d (force per unit U)
    uint32_t eu;   // ep in 2^-28 units, rounded up (contacts only)
    uint32_t su;   // lower bound of |F_N|, at most 32, in 2^-17 units (contacts only)
};
__device__ inline PairOut pair_math(double dx, double dy, double dz, double d2, float ri, float rj, float kU, float gU,
                                    bool valid) {
    PairOut o;
    const double sr = (double)ri + (double)rj;  // exact
    const double num = fma(sr, sr, -d2);        // (r_i + r_j)^2 - d^2, one rounding
    const float dist = __builtin_amdgcn_sqrtf((float)d2);
    const float srf = (float)sr;
    const float delta = (float)num * __builtin_amdgcn_rcpf(srf + dist);
    const float e = 1.74f + srf * 0x1.02p-24f + fabsf(delta) * 0x1.0p-21f;
    const bool near = valid && delta > -e;  // possibly a contact
    const bool beyond = d2 >= kL2U - kNbrBand;  // (only when the box is shorter than r_i + r_j)
    bool unc = near && beyond && d2 < kL2U + kNbrBand;
    const bool coinc = d2 < 64.0;  // centres within 8 U: the direction is left to FP64
    const bool cand = near && !beyond && !coinc;
    unc |= near && !beyond && coinc;
    unc |= cand && delta <= 4.0f * e;
    const bool contact = cand && delta > 4.0f * e;
    const float rbar = ri * rj * __builtin_amdgcn_rcpf(srf);
    const float sq = __builtin_amdgcn_sqrtf(fmaxf(rbar * delta, 0.0f));
    const float kd = kU * delta, gs = gU * sq;
    const float fn = kd - gs;
    const float rd = __builtin_amdgcn_rcpf(dist);
    const float afn = fabsf(fn);
    const float hg = 0.5f * gs * __builtin_amdgcn_rcpf(delta);  // gamma sqrt(rbar) / (2 sqrt(delta))
    const float ep = (fabsf(kU - hg) + 0.16f * hg) * e + (3.0f * kd + 9.0f * gs) * 0x1.0p-24f +
                     afn * (3.5f * rd + 0x1.8p-22f) + 0x1.0p-33f;
    const bool bad = contact && !(ep < 0x1.0p-6f && afn <= 64.0f && afn > ep);
    o.unc = unc || bad;
    o.contact = contact && !bad;
    o.f = fn * rd;
    o.eu = o.contact ? (uint32_t)ceilf(ep * 0x1.0p28f) : 0u;
    o.su = o.contact ? (uint32_t)(fminf(afn - ep, 32.0f) * 0x1.0p17f) : 0u;
    return o;
}

// Force contribution of a pair in the fixed-point units of the sums.
__device__ inline unsigned long long fix_term(float f, double dd) {
    return fixbits(fma((double)f, dd, kFixMagic)) - fixbits(kFixMagic);
}

// One candidate pair of the diagnostic box-wise path: the target's payload
// (qx, qy, qz: already shifted into the frame of the candidate's box), the
// candidate's payload c.
template <bool DIAG>
__device__ inline void pair_acc(Acc &a, int32_t qx, int32_t qy, int32_t qz, float ri, Pay c, float kU, float gU) {
    const double dx = (double)(qx - c.x), dy = (double)(qy - c.y), dz = (double)(qz - c.z);
    const double d2 = fma(dz, dz, fma(dy, dy, dx * dx));
    if (DIAG) {
        if (d2 < kL2U - kNbrBand) ++a.nbr;
        else if (d2 < kL2U + kNbrBand) ++a.unc;
    }
    const PairOut o = pair_math(dx, dy, dz, d2, ri, c.r, kU, gU, true);
    a.unc += o.unc ? 1 : 0;
    if (o.contact) {
        ++a.contacts;
        const double f = (double)o.f;
        a.ax += fixbits(fma(f, dx, kFixMagic));
        a.ay += fixbits(fma(f, dy, kFixMagic));
        a.az += fixbits(fma(f, dz, kFixMagic));
        ++a.nfix;
        a.eacc += o.eu;
        a.sacc += o.su;
    }
}

// Whether a target's FP32 result is certified: its force within 1e-5 of the
// sum of |F_N| of its contacts (the error bound e_sum against the lower bound
// s_sum of that sum; the oracle's own FP64 rounding is far below the margin)
// and its move decision (|F| > a) outside the error bound.
__device__ inline bool fp32_certified(const SimDesc &S, double fx, double fy, double fz, double e_sum, double s_sum) {
    if (!(e_sum <= 0.99999e-5 * s_sum)) return false;
    const double fnorm = sqrt(fma(fz, fz, fma(fy, fy, fx * fx)));
    return fabs(fnorm - S.adherence) > e_sum + 0x1.0p-40 * (1.0 + S.adherence);
}

// Drains `cnt` (<= 64) queued pairs of this wave (lane l takes entry l).
// With the half shell (n3), a pair of two targets is drained once and adds
// the opposite force (exact in fixed point) and the same counts and bounds to
// the candidate's accumulators.
template <bool DIAG>
__device__ inline void drain_queue(SweepLds<DIAG> &L, const uint32_t *qw, uint32_t cnt, float kU, float gU, bool n3) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t ent = lane < cnt ? qw[lane] : 0u;
    const uint32_t t = ent >> 20, self = (ent >> 10) & 1023u, q = ent & 1023u;
    const bool valid = lane < cnt && q != self;
    const Pay own = L.sp[self];
    const Pay c = L.sp[q];
    const double dx = (double)(own.x - c.x), dy = (double)(own.y - c.y), dz = (double)(own.z - c.z);
    const double d2 = fma(dz, dz, fma(dy, dy, dx * dx));
    const PairOut o = pair_math(dx, dy, dz, d2, own.r, c.r, kU, gU, valid);
    const uint32_t tq = n3 ? L.tmap[q] : kNoTarget;
    if (o.contact || o.unc) {
        const unsigned long long fx = o.contact ? fix_term(o.f, dx) : 0ull;
        const unsigned long long fy = o.contact ? fix_term(o.f, dy) : 0ull;
        const unsigned long long fz = o.contact ? fix_term(o.f, dz) : 0ull;
        const unsigned long long cx = o.contact ? kCnt1 : 0ull, cy = o.unc ? kCnt1 : 0ull;
        const unsigned long long cm = ((unsigned long long)o.eu << 32) | o.su;
        atomicAdd(&L.acc[0][t], fx + cx);
        atomicAdd(&L.acc[1][t], fy + cy);
        atomicAdd(&L.acc[2][t], fz);
        atomicAdd(&L.acm[t], cm);
        if (tq != kNoTarget) {
            atomicAdd(&L.acc[0][tq], (0ull - fx) + cx);
            atomicAdd(&L.acc[1][tq], (0ull - fy) + cy);
            atomicAdd(&L.acc[2][tq], 0ull - fz);
            atomicAdd(&L.acm[tq], cm);
        }
    }
}

// Reach test of candidate kk of a lane's task (staged payload c, staged index
// b0 + kk) against the lane's target: FP32 squared distance from the exact
// integer offset, against (r_i + kReach + r_j)^2.  Survivors go to the wave's
// queue, which is drained whenever it holds 64 pairs (qn: wave-uniform
// fill).  CHECK: some lane's task may have fewer than kk + 1 candidates.
// DIAG also counts the neighbours within the box length (FP32 test with a
// band of 2^-18 L^2 around L^2; inside it the target goes to the FP64 path).
constexpr float kL2f = 0x1.0p56f, kL2Bandf = 0x1.0p38f;
template <bool DIAG, bool CHECK>
__device__ inline void reach_test(SweepLds<DIAG> &L, uint32_t *qw, uint32_t &qn, Pay own, float owg, Pay c,
                                  uint32_t kk, uint32_t len, uint32_t tq, uint32_t self, uint32_t b0, uint32_t &nb,
                                  bool &un, float kU, float gU, bool n3) {
    const uint32_t lane = threadIdx.x & 63;
    const bool in = !CHECK || kk < len;
    const float ddx = (float)(own.x - c.x), ddy = (float)(own.y - c.y), ddz = (float)(own.z - c.z);
    const float d2 = fmaf(ddz, ddz, fmaf(ddy, ddy, ddx * ddx));
    const float sg = owg + c.r;
    const bool hit = in && d2 < sg * sg;
    if (DIAG) {
        const bool other = in && b0 + kk != self;
        nb += (other && d2 < kL2f - kL2Bandf) ? 1u : 0u;
        un |= other && d2 >= kL2f - kL2Bandf && d2 < kL2f + kL2Bandf;
    }
    // every lane stores (a survivor at its queue position, the others in the
    // spare slot): no branch on the ballot and no exec mask per candidate
    const uint64_t m = __builtin_amdgcn_ballot_w64(hit);
    const uint32_t pos = qn + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    qw[hit ? pos : (uint32_t)kQueue] = tq + kk;
    qn += (uint32_t)__popcll(m);
    if (qn >= 64) {
        __builtin_amdgcn_wave_barrier();
        drain_queue<DIAG>(L, qw, 64u, kU, gU, n3);
        __builtin_amdgcn_wave_barrier();
        qn -= 64;
        if (lane < qn) qw[lane] = qw[64 + lane];
        __builtin_amdgcn_wave_barrier();
    }
}

__device__ inline void core_box_coords(int c, int &cx, int &cy, int &cz) {
    cx = c & 3;
    cy = (c >> 2) & 3;
    cz = c >> 4;
}
// Staged row (boxes x-1..x+1 around core box (cx,cy,cz)) of task row r.
__device__ inline int task_row(int cx, int cy, int cz, int r) {
    return cx + kHalo * ((cy + r % 3) + kHalo * (cz + r / 3));
}

// Rows of a target's 27-box neighbourhood that can hold a pair within reach
// (bits 3r..3r+2 per row r: row used, its left box, its right box).  `reach`
// bounds the pair's contact distance plus the reach guard, with a margin for
// the FP32 face distances (U units): a box whose distance from the target
// exceeds it cannot hold a pair that the sweep keeps.  With DIAG every box is
// visited (all neighbours within the box length are counted).
template <bool DIAG>
__device__ inline uint32_t row_mask(Pay own, int cx, int cy, int cz, float reach_add) {
    if (DIAG) return 0x7ffffffu;
    const float reach = own.r + reach_add;
    const float r2 = reach * reach;
    // distances to the faces of the target box (local box c+1 spans [(c-2)L, (c-1)L)),
    // exact integers up to the FP32 rounding
    const float fx0 = (float)(own.x - (cx - 2) * kUnitL), fx1 = kUnitLf - fx0;
    const float fy0 = (float)(own.y - (cy - 2) * kUnitL), fy1 = kUnitLf - fy0;
    const float fz0 = (float)(own.z - (cz - 2) * kUnitL), fz1 = kUnitLf - fz0;
    uint32_t m = 0;
    for (int r = 0; r < 9; ++r) {
        const int dy = r % 3 - 1, dz = r / 3 - 1;
        const float gy = dy < 0 ? fy0 : (dy > 0 ? fy1 : 0.0f);
        const float gz = dz < 0 ? fz0 : (dz > 0 ? fz1 : 0.0f);
        const float rem = r2 - gy * gy - gz * gz;
        if (rem > 0.0f) {
            const uint32_t b = 1u | (fx0 * fx0 < rem ? 2u : 0u) | (fx1 * fx1 < rem ? 4u : 0u);
            m |= b << (3 * r);
        }
    }
    return m;
}

// Candidate range of task r of a target in core box (cx,cy,cz) with staged
// index self and kept boxes `rows` (row_mask): r < 9 is row r, r == 9 the
// own row's left halo box under the half shell.  Without the half shell a
// row is its kept boxes.  With it (n3: every target of the unit active), a
// pair of two targets is taken once, by the one with the smaller staged
// index (staging runs in box order, x fastest): rows before the own row keep
// only their halo box (core lines have at most one, at x = -1 or x = 4),
// the own row keeps the candidates after the target (task r) and its halo
// left box (task 9), rows after it are kept whole.  Lines outside the core
// hold no targets and are kept whole.
template <bool DIAG>
__device__ inline void task_range(const SweepLds<DIAG> &L, uint32_t rows, int cx, int cy, int cz, int r, bool n3,
                                  uint32_t self, uint32_t &b0, uint32_t &len) {
    const int rr = r < 9 ? r : 4;  // task 9 belongs to the own row
    const int dy = rr % 3 - 1, dz = rr / 3 - 1;
    const uint32_t rb = (rows >> (3 * rr)) & 7u;
    const int row = task_row(cx, cy, cz, rr);  // staged box of the row's left box
    const bool lk = (rb & 2u) != 0, rk = (rb & 4u) != 0;  // left / right box kept
    int lo_i = lk ? row : row + 1, hi_i = rk ? row + 3 : row + 2;
    bool keep = rb != 0 && r < 9;
    bool after_self = false;
    // (r is a constant once the task loop is unrolled: the cases below
    // reduce to a few selects)
    const bool inner = (unsigned)(cy + dy) < (unsigned)kBlk && (unsigned)(cz + dz) < (unsigned)kBlk;
    const bool lh = cx == 0 && lk, rh = cx == kBlk - 1 && rk;  // kept halo boxes
    if (r == 9) {  // own row, halo left box
        keep = n3 && lh;
        hi_i = row + 1;
    } else if (dz < 0 || (dz == 0 && dy < 0)) {  // before the own row: its halo box only
        if (n3 && inner) {
            keep = keep && (lh || rh);
            hi_i = lh ? row + 1 : hi_i;
            lo_i = lh ? lo_i : row + 2;
        }
    } else if (dz == 0 && dy == 0) {  // own row: the candidates after the target
        after_self = n3;
    }
    const uint32_t lo = after_self ? self + 1u : L.sbeg[lo_i], hi = L.sbeg[hi_i];
    b0 = lo;
    len = keep && hi > lo ? hi - lo : 0u;
}

// Exact sum of the accumulators of the lanes lane ^ off for off = g, 2g, ..., 32
// (the streams of one target, see sweep_unit_dense).
__device__ inline void acc_reduce_streams(Acc &a, int g) {
    for (int off = g; off < 64; off <<= 1) {
        a.ax += __shfl_xor(a.ax, off);
        a.ay += __shfl_xor(a.ay, off);
        a.az += __shfl_xor(a.az, off);
        a.eacc += __shfl_xor(a.eacc, off);
        a.sacc += __shfl_xor(a.sacc, off);
        a.contacts += __shfl_xor(a.contacts, off);
        a.nbr += __shfl_xor(a.nbr, off);
        a.nfix += __shfl_xor(a.nfix, off);
        a.unc += __shfl_xor(a.unc, off);
    }
}

// Box-wise path of the production sweep: candidates per wave and chunk.
constexpr int kDenseChunk = 192;
// Targets per sub-pass: the up to 64 targets of a pass are grouped by the
// octant of their box, and each group of kSubTargets tests only the
// candidates within reach of its own bounding box.
constexpr int kSubTargets = 16;
// Margin of that cull in U units, above the FP32 rounding of the distance
// from a candidate to the box (about 2^-22 relative of at most 2^30 U).
constexpr float kCullMargin = 1024.0f;
// Target slot word: bits 0-30 the slot, bit 31 a target without pairs
// (static, or past the pass's targets).
constexpr uint32_t kTsSlot = 0x7fffffffu, kTsIdle = 0x80000000u;
// Candidates per box (its 27-box neighbourhood) beyond which the box-wise
// path leaves the box's targets to the FP64 path: below it the packed error
// and force-sum words of a target cannot overflow.
constexpr uint32_t kDenseMaxCand = 16000;
// Accumulator words per target on the box-wise path: force x, y, z (2^-34
// units, full 64-bit words), contacts | undecided pairs << 32, error bound
// (2^-24 units, rounded up) << 32 | lower bound of sum |F_N| (2^-12 units).
constexpr int kDenseWords = 5;

// Drain of the box-wise path: lane l takes queue entry l (target index |
// candidate index in the staged chunk << 6) and adds the pair's contact
// force, counts and bounds to the target's LDS accumulators.  Candidates are
// staged in the frame of the targets' box; cs holds their slots and ts the
// targets' (low 31 bits: a target is not its own candidate).
__device__ inline void drain_dense(const uint32_t *qw, uint32_t cnt, const Pay *ob, const Pay *buf, const uint32_t *cs,
                                   const uint32_t *ts, unsigned long long *acc, float kU, float gU) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t ent = lane < cnt ? qw[lane] : 0u;
    const uint32_t tl = ent & 63u, j = ent >> 6;
    const bool valid = lane < cnt && cs[j] != (ts[tl] & kTsSlot);
    const Pay own = ob[tl];
    const Pay c = buf[j];
    const double dx = (double)(own.x - c.x), dy = (double)(own.y - c.y), dz = (double)(own.z - c.z);
    const double d2 = fma(dz, dz, fma(dy, dy, dx * dx));
    const PairOut o = pair_math(dx, dy, dz, d2, own.r, c.r, kU, gU, valid);
    unsigned long long *a = acc + kDenseWords * tl;
    if (o.contact) {
        atomicAdd(&a[0], fix_term(o.f, dx));
        atomicAdd(&a[1], fix_term(o.f, dy));
        atomicAdd(&a[2], fix_term(o.f, dz));
        atomicAdd(&a[3], 1ull);
        atomicAdd(&a[4], ((unsigned long long)((o.eu + 15u) >> 4) << 32) | (o.su >> 5));
    }
    if (o.unc) atomicAdd(&a[3], 1ull << 32);
}

// Box-wise path of the production sweep, for units whose region does not fit
// the LDS stage (or whose task list overflows).  The sweep queues such units
// as (unit, core box, pass group) items, one per core box with targets and
// pass group, for k_sweep_dense, so that the boxes of the densest units spread
// over the whole chip instead of over the four waves of one block.
// Within an item, the up to 64 targets of a pass are grouped by the octant of
// their box and split into sub-passes of kSubTargets.  The candidates of all
// 27 boxes are staged in chunks of up to kDenseChunk per wave, all of a
// chunk's loads in flight together, and shifted into the frame of the
// targets' box; each sub-pass first keeps the chunk's candidates within reach
// of its targets' bounding box, then its lanes hold (target, stream) pairs
// over them.  Each lane only tests the pair against its contact reach;
// survivors go to a per-wave queue and the contact math runs on full 64-pair
// drains (and on the rest at the end of each chunk), with exact fixed-point
// LDS accumulators per target.
constexpr int kDensePassGroups = 8;  // pass p (64 targets) of a box is in group p % 8

struct DenseWave {
    Pay buf[kDenseChunk];                      // staged candidates, in the frame of the targets' box
    Pay ob[64];                                // the targets of the pass, grouped by octant
    uint32_t cs[kDenseChunk];                  // slots of the staged candidates
    uint32_t ts[64];                           // slot word of each target (kTsSlot, kTsIdle)
    unsigned long long acc[kDenseWords * 64];  // per target, see kDenseWords
    uint32_t pre[28];                          // prefix of the candidate counts of the 27 boxes (entry 27: total)
    uint32_t src[27];                          // first slot of each of the 27 boxes
    uint32_t queue[2 * 64];                    // survivors: target index | staged candidate << 6
    int32_t sbox[64 / kSubTargets][8];         // per sub-pass: min x, y, z, max x, y, z, largest radius (bits)
    uint8_t cl[kDenseChunk];                   // the chunk's candidates within a sub-pass's reach
};

// The passes of group pg of box (gx, gy, gz): targets pg * 64 .. pg * 64 + 63,
// then every kDensePassGroups-th block of 64 after them.
__device__ void sweep_box_dense(const Dev &d, const SimDesc &S, DenseWave &W, int P, int lp, int gx, int gy, int gz,
                                int pg) {
    const int64_t A = d.A;
    const int lane = threadIdx.x & 63;
    if (gx >= S.dims[0] || gy >= S.dims[1] || gz >= S.dims[2]) return;  // padding of an edge block
    const uint32_t m = box_rank(d, S, gx, gy, gz);
    const uint32_t tbeg = d.box_start[S.sb_off + m];
    const uint32_t cnt = d.box_start[S.sb_off + m + 1] - tbeg;
    if (cnt <= (uint32_t)pg * 64u) return;  // no pass in this group
    const float kU = S.kU, gU = S.gU;
    const int64_t lin = linear_box(gx, gy, gz, S.dims);
    Pay *buf = W.buf, *ob = W.ob;
    uint32_t *cs = W.cs, *pre = W.pre, *src = W.src, *qw = W.queue, *ts = W.ts;
    uint8_t *cl = W.cl;
    int32_t(*sbox)[8] = W.sbox;
    unsigned long long *acc = W.acc;
    // prefix of the candidate counts of the 27 boxes (lane b: box b, x fastest)
    uint32_t nnb = 0, srcb = 0;
    if (lane < 27) {
        const int bx = gx + lane % 3 - 1, by = gy + lane / 3 % 3 - 1, bz = gz + lane / 9 - 1;
        if (bx >= 0 && by >= 0 && bz >= 0 && bx < S.dims[0] && by < S.dims[1] && bz < S.dims[2]) {
            const uint32_t mb = box_rank(d, S, bx, by, bz);
            srcb = d.box_start[S.sb_off + mb];
            nnb = d.box_start[S.sb_off + mb + 1] - srcb;
        }
    }
    uint32_t inc = nnb;
    for (int off = 1; off < 32; off <<= 1) {
        const uint32_t o = __shfl_up(inc, off);
        if (lane >= off) inc += o;
    }
    const uint32_t T = __shfl(inc, 26);  // candidates of the 27 boxes
    const bool huge = T > kDenseMaxCand;  // (wave-uniform) every target goes to the FP64 path
    __builtin_amdgcn_wave_barrier();
    if (lane < 28) pre[lane] = inc - nnb;  // lane 27: T
    if (lane < 27) src[lane] = srcb;
    __builtin_amdgcn_wave_barrier();
    for (uint32_t p0 = (uint32_t)pg * 64u; p0 < cnt; p0 += 64u * (uint32_t)kDensePassGroups) {
        const int gsz = cnt - p0 < 64u ? (int)(cnt - p0) : 64;  // targets in this pass
        const bool tv = lane < gsz;
        const uint32_t tslot0 = tbeg + p0;
        const uint32_t slot = tslot0 + (tv ? (uint32_t)lane : 0u);
        const int64_t i = d.sorted_idx[slot];
        const uint8_t fl = d.flags[lp][i];
        const bool stat = tv && S.detect_static && (fl & kStatic);
        const bool act = tv && !stat;
        if (stat) skip_static<false>(d, S, i, P, lp, fl, lin);
        if (huge) {
            if (act) d.fix_list[atomicAdd(&d.ctl->n_fix, 1u)] = (uint32_t)i;
            continue;
        }
        const Pay own = d.payload[slot];
        // targets grouped by the octant of their box (the top bit of each
        // box-relative coordinate; only the grouping depends on it)
        const int oct = tv ? (int)((((uint32_t)own.x >> 27) & 1u) | (((uint32_t)own.y >> 26) & 2u) |
                                   (((uint32_t)own.z >> 25) & 4u))
                           : 8;
        uint32_t gpos = 0;
        for (int k = 0; k < 8; ++k) {
            const uint64_t m = __builtin_amdgcn_ballot_w64(oct == k);
            if (oct > k) gpos += (uint32_t)__popcll(m);
            if (oct == k) gpos += __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        }
        __builtin_amdgcn_wave_barrier();
        if (tv) {
            ob[gpos] = own;
            ts[gpos] = slot | (act ? 0u : kTsIdle);
            for (int w = 0; w < kDenseWords; ++w) acc[kDenseWords * gpos + w] = 0;
        }
        __builtin_amdgcn_wave_barrier();
        // bounding box and largest radius of every sub-pass's targets (lane l:
        // grouped target l; lanes past the targets repeat the last one)
        const int nsub = (gsz + kSubTargets - 1) / kSubTargets;
        {
            const Pay t = ob[tv ? lane : (uint32_t)(gsz - 1)];
            int32_t lo[3] = {t.x, t.y, t.z}, hi[3] = {t.x, t.y, t.z};
            float rr = t.r;
            for (int off = 1; off < kSubTargets; off <<= 1) {
                for (int a = 0; a < 3; ++a) {
                    lo[a] = min(lo[a], __shfl_xor(lo[a], off));
                    hi[a] = max(hi[a], __shfl_xor(hi[a], off));
                }
                rr = fmaxf(rr, __shfl_xor(rr, off));
            }
            const int sp = lane / kSubTargets;
            if (lane % kSubTargets == 0 && sp < nsub) {
                for (int a = 0; a < 3; ++a) {
                    sbox[sp][a] = lo[a];
                    sbox[sp][3 + a] = hi[a];
                }
                sbox[sp][6] = __float_as_int(rr);
            }
        }
        __builtin_amdgcn_wave_barrier();
        uint32_t qn = 0;  // wave-uniform queue fill
        for (uint32_t cb0 = 0; cb0 < T; cb0 += kDenseChunk) {
            const uint32_t mc = T - cb0 < (uint32_t)kDenseChunk ? T - cb0 : (uint32_t)kDenseChunk;
            // stage the chunk (up to three candidates per lane, all loads in
            // flight together): box and slot first (the slot goes to LDS at
            // once, the boxes stay packed in one register), then the shift
            // into the targets' frame (box b is at offset (b % 3 - 1,
            // b / 3 % 3 - 1, b / 9 - 1) boxes: exact integer multiples of L)
            static_assert(kDenseChunk <= 3 * 64, "three candidates per lane");
            uint32_t vb = 0;
            for (int h = 0; h < 3; ++h) {
                const uint32_t q = (uint32_t)lane + 64u * (uint32_t)h;
                if (q < mc) {
                    const uint32_t kk = cb0 + q;
                    int lo = 0, hi = 27;  // the box of candidate kk: largest b with pre[b] <= kk
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (pre[mid] <= kk) lo = mid; else hi = mid;
                    }
                    vb |= (uint32_t)lo << (8 * h);
                    cs[q] = src[lo] + (kk - pre[lo]);
                }
            }
            Pay v[3];
#pragma unroll
            for (int h = 0; h < 3; ++h) {
                const uint32_t q = (uint32_t)lane + 64u * (uint32_t)h;
                if (q < mc) v[h] = d.payload[cs[q]];
            }
#pragma unroll
            for (int h = 0; h < 3; ++h) {
                const uint32_t q = (uint32_t)lane + 64u * (uint32_t)h;
                if (q < mc) {
                    const int b = (int)((vb >> (8 * h)) & 0xffu);
                    Pay cc = v[h];
                    cc.x += (b % 3 - 1) * kUnitL;
                    cc.y += (b / 3 % 3 - 1) * kUnitL;
                    cc.z += (b / 9 - 1) * kUnitL;
                    buf[q] = cc;
                }
            }
            __builtin_amdgcn_wave_barrier();
            for (int sp = 0; sp < nsub; ++sp) {
                const int sb = sp * kSubTargets;
                const int sgsz = gsz - sb < kSubTargets ? gsz - sb : kSubTargets;
                const int nstream = 64 / sgsz;
                const int tl = sb + lane % sgsz, sid = lane / sgsz;
                // the chunk's candidates within reach of the sub-pass's box: a
                // pair test below can succeed only if the candidate is closer
                // to some target than that target's radius + its own + kReach
                const int32_t b0x = sbox[sp][0], b0y = sbox[sp][1], b0z = sbox[sp][2];
                const int32_t b1x = sbox[sp][3], b1y = sbox[sp][4], b1z = sbox[sp][5];
                const float rreach = __int_as_float(sbox[sp][6]) + (kReach + kCullMargin);
                uint32_t nc = 0;  // wave-uniform
#pragma unroll
                for (int h = 0; h < 3; ++h) {
                    const uint32_t q = (uint32_t)lane + 64u * (uint32_t)h;
                    bool keep = false;
                    if (q < mc) {
                        const Pay c = buf[q];
                        const float ex = (float)max(max(b0x - c.x, c.x - b1x), 0);
                        const float ey = (float)max(max(b0y - c.y, c.y - b1y), 0);
                        const float ez = (float)max(max(b0z - c.z, c.z - b1z), 0);
                        const float rc = rreach + c.r;
                        keep = fmaf(ez, ez, fmaf(ey, ey, ex * ex)) < rc * rc;
                    }
                    const uint64_t km = __builtin_amdgcn_ballot_w64(keep);
                    if (keep)
                        cl[nc + __builtin_amdgcn_mbcnt_hi((uint32_t)(km >> 32),
                                                          __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u))] = (uint8_t)q;
                    nc += (uint32_t)__popcll(km);
                }
                __builtin_amdgcn_wave_barrier();
                const Pay ot = ob[tl];
                const bool at = sid < nstream && !(ts[tl] & kTsIdle);
                const float owg = ot.r + kReach;
                for (uint32_t j0 = 0; j0 < nc; j0 += (uint32_t)nstream) {  // same trip count on all lanes
                    const uint32_t jj = j0 + (uint32_t)sid;
                    const bool in = jj < nc && at;
                    const uint32_t j = cl[jj < nc ? jj : 0u];
                    const Pay cc = buf[j];
                    const float ddx = (float)(ot.x - cc.x), ddy = (float)(ot.y - cc.y), ddz = (float)(ot.z - cc.z);
                    const float d2 = fmaf(ddz, ddz, fmaf(ddy, ddy, ddx * ddx));
                    const float sg = owg + cc.r;
                    const bool hit = in && d2 < sg * sg;
                    // (many trips have no survivor at all: the append is skipped on those)
                    const uint64_t mh = __builtin_amdgcn_ballot_w64(hit);
                    if (mh) {
                        if (hit)
                            qw[qn + __builtin_amdgcn_mbcnt_hi((uint32_t)(mh >> 32),
                                                              __builtin_amdgcn_mbcnt_lo((uint32_t)mh, 0u))] =
                                (uint32_t)tl | (j << 6);
                        qn += (uint32_t)__popcll(mh);
                        if (qn >= 64) {
                            __builtin_amdgcn_wave_barrier();
                            drain_dense(qw, 64u, ob, buf, cs, ts, acc, kU, gU);
                            __builtin_amdgcn_wave_barrier();
                            qn -= 64;
                            if ((uint32_t)lane < qn) qw[lane] = qw[64 + lane];
                            __builtin_amdgcn_wave_barrier();
                        }
                    }
                }
                __builtin_amdgcn_wave_barrier();  // the next sub-pass rewrites cl
            }
            if (qn) {  // the chunk is restaged next: drain the rest now
                __builtin_amdgcn_wave_barrier();
                drain_dense(qw, qn, ob, buf, cs, ts, acc, kU, gU);
                qn = 0;
            }
            __builtin_amdgcn_wave_barrier();
        }
        // commit: lane l takes grouped target l
        if (!tv) continue;
        const uint32_t tw = ts[lane];
        if (tw & kTsIdle) continue;
        const int64_t ic = d.sorted_idx[tw & kTsSlot];
        const uint8_t flc = d.flags[lp][ic];
        const unsigned long long *a = acc + kDenseWords * lane;
        const unsigned long long ac = a[3], am = a[4];
        bool unc = (ac >> 32) != 0;
        if (!unc) {
            const double fx = (double)(long long)a[0] * kFixUnit;
            const double fy = (double)(long long)a[1] * kFixUnit;
            const double fz = (double)(long long)a[2] * kFixUnit;
            const int nc = (int)(uint32_t)ac;
            if (fp32_certified(S, fx, fy, fz, (double)(am >> 32) * 0x1.0p-24, (double)(uint32_t)am * 0x1.0p-12))
                commit_agent<false>(d, S, ic, P, lp, flc, d.pos[P][ic], d.pos[P][A + ic], d.pos[P][2 * A + ic], fx, fy,
                                    fz, nc, 0, nc, m, lin);
            else
                unc = true;
        }
        if (unc) d.fix_list[atomicAdd(&d.ctl->n_fix, 1u)] = (uint32_t)ic;
    }
}

// Queues the box-wise work of a unit for k_sweep_dense: one item per core box
// with targets and pass group, ceil(targets / 64) groups at most
// kDensePassGroups; one atomic per wave.  sbeg: the unit's staged-box prefix
// (core boxes are the staged boxes 1..4 on every axis).  Every thread of the
// block calls it.
__device__ inline void queue_dense_unit(const Dev &d, const uint32_t *sbeg, int64_t u) {
    const int tid = threadIdx.x;
    const uint32_t lane = tid & 63;
    uint32_t ng = 0;
    int cb = 0;
    if (tid < kNb) {
        const int lx = tid % kHalo, ly = (tid / kHalo) % kHalo, lz = tid / (kHalo * kHalo);
        if (lx >= 1 && lx <= kBlk && ly >= 1 && ly <= kBlk && lz >= 1 && lz <= kBlk) {
            cb = (lx - 1) + kBlk * ((ly - 1) + kBlk * (lz - 1));
            const uint32_t np = (sbeg[tid + 1] - sbeg[tid] + 63u) / 64u;
            ng = np < (uint32_t)kDensePassGroups ? np : (uint32_t)kDensePassGroups;
        }
    }
    uint32_t x = ng;  // inclusive scan over the wave
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= (uint32_t)off) x += y;
    }
    const uint32_t tot = __shfl(x, 63);
    if (tot == 0) return;
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(&d.ctl->n_dense, (unsigned long long)tot);
    base = __shfl(base, 0);
    for (uint32_t k = 0; k < ng; ++k) {
        const unsigned long long q = base + (x - ng) + k;
        if (q < (unsigned long long)d.dense_cap) {
            d.dense_list[q] = ((uint64_t)u << 9) | ((uint64_t)cb << 3) | (uint64_t)k;
        } else {  // cannot happen with the list sized as above; fail the step rather than skip agents
            atomicOr(&d.ctl->err, kErrGrid);
            atomicExch(&d.ctl->abort, 1);
        }
    }
}

// Dense units (region larger than the LDS stage, or more targets than
// kMaxT), diagnostic form: each wave takes one core box at a time.  All
// targets of a box share its 27-box candidate set, so the lanes hold (target,
// stream) pairs, g targets by 64 / g streams, and walk the candidates in
// wave-uniform loops with the streams interleaved, the contact math inline for
// every candidate (every neighbour within the box length is counted); the
// exact fixed-point sums of a target's streams are then added across lanes.
// Payload is read from global memory in coalesced chunks of 64 candidates
// staged in the wave's slice of the LDS stage.
template <bool DIAG>
__device__ void sweep_unit_dense(const Dev &d, const SimDesc &S, SweepLds<DIAG> &L, int P, int lp, int qx, int qy,
                                 int qz) {
    const int64_t A = d.A;
    const float kU = S.kU, gU = S.gU;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    Pay *buf = L.sp + 64 * w;  // the LDS stage is free on this path: 64 candidates per wave
    for (int c = w; c < kCore; c += blockDim.x >> 6) {
        int cx, cy, cz;
        core_box_coords(c, cx, cy, cz);
        const int lb = (cx + 1) + kHalo * ((cy + 1) + kHalo * (cz + 1));
        const uint32_t cnt = L.sbeg[lb + 1] - L.sbeg[lb];
        if (cnt == 0) continue;
        const int64_t lin = linear_box(qx * kBlk + cx, qy * kBlk + cy, qz * kBlk + cz, S.dims);
        for (uint32_t p0 = 0; p0 < cnt;) {
            // gsz targets in this pass (a power of two >= the remaining ones, at
            // most 64), 64 / gsz streams each
            int gsz = 1;
            while (gsz < 64 && (uint32_t)gsz < cnt - p0) gsz <<= 1;
            const int nstream = 64 / gsz;
            const int tl = lane & (gsz - 1), sid = lane / gsz;
            const uint32_t k = p0 + (uint32_t)tl;
            const bool tv = k < cnt;
            const uint32_t slot = L.gsrc[lb] + (tv ? k : 0u);
            const int64_t i = d.sorted_idx[slot];
            const uint8_t fl = d.flags[lp][i];
            const bool stat = tv && S.detect_static && (fl & kStatic);
            const bool act = tv && !stat;
            if (stat && sid == 0) skip_static<DIAG>(d, S, i, P, lp, fl, lin);
            Acc a = {0ull, 0ull, 0ull, 0ull, 0ull, 0, 0, 0, 0};
            const Pay own = d.payload[slot];
            for (int oz = -1; oz <= 1; ++oz)
                for (int oy = -1; oy <= 1; ++oy) {
                    const int row = cx + kHalo * ((cy + 1 + oy) + kHalo * (cz + 1 + oz));
                    // the target in the frame of the candidate's box (exact integers)
                    const int32_t qy2 = own.y - oy * kUnitL;
                    const int32_t qz2 = own.z - oz * kUnitL;
                    for (int ox = -1; ox <= 1; ++ox) {
                        const int lbb = row + ox + 1;
                        const int32_t qx2 = own.x - ox * kUnitL;
                        const uint32_t b0 = L.gsrc[lbb], nn = L.sbeg[lbb + 1] - L.sbeg[lbb];
                        // the box's candidates 64 at a time: one coalesced load
                        // per chunk into this wave's LDS slice, then broadcast reads
                        for (uint32_t c0 = 0; c0 < nn; c0 += 64) {
                            const uint32_t mc = nn - c0 < 64u ? nn - c0 : 64u;
                            __builtin_amdgcn_wave_barrier();
                            if ((uint32_t)lane < mc) buf[lane] = d.payload[b0 + c0 + (uint32_t)lane];
                            __builtin_amdgcn_wave_barrier();
                            for (uint32_t j0 = 0; j0 < mc; j0 += (uint32_t)nstream) {  // same trip count on all lanes
                                const uint32_t j = j0 + (uint32_t)sid;
                                const bool in = j < mc && act;
                                const Pay cc = buf[j < mc ? j : 0u];
                                if (in && b0 + c0 + j != slot) pair_acc<DIAG>(a, qx2, qy2, qz2, own.r, cc, kU, gU);
                            }
                        }
                    }
                }
            acc_reduce_streams(a, gsz);
            p0 += (uint32_t)gsz;
            if (!act || sid != 0) continue;
            bool unc = a.unc != 0;
            if (!unc) {
                const unsigned long long mb = (unsigned long long)a.nfix * fixbits(kFixMagic);
                const double fx = (double)(long long)(a.ax - mb) * kFixUnit;
                const double fy = (double)(long long)(a.ay - mb) * kFixUnit;
                const double fz = (double)(long long)(a.az - mb) * kFixUnit;
                if (fp32_certified(S, fx, fy, fz, (double)a.eacc * 0x1.0p-28, (double)a.sacc * 0x1.0p-17)) {
                    const uint32_t m = box_rank(d, S, qx * kBlk + cx, qy * kBlk + cy, qz * kBlk + cz);
                    commit_agent<DIAG>(d, S, i, P, lp, fl, d.pos[P][i], d.pos[P][A + i], d.pos[P][2 * A + i], fx, fy,
                                       fz, a.contacts, a.nbr, a.contacts, m, lin);
                } else {
                    unc = true;
                }
            }
            if (unc) d.fix_list[atomicAdd(&d.ctl->n_fix, 1u)] = (uint32_t)i;
        }
    }
}

// The simulation descriptors and unit tables come in as read-only,
// non-aliased arguments as well, so that their wave-uniform reads are scalar
// loads.
template <bool DIAG>
__global__ void __launch_bounds__(256, 4)  // 4 blocks per CU: at most 128 VGPRs
    k_sweep(Dev d, const SimDesc *__restrict__ sims, const int64_t *__restrict__ wblk,
            const uint32_t *__restrict__ blist, const uint8_t *__restrict__ active_blk, int lookahead) {
    __shared__ SweepLds<DIAG> L;
    if (ABM_ABORTED(d)) return;
    const int P = d.ctl->pos_par, lp = d.ctl->lay_par;
    const int64_t A = d.A;
    const int64_t U = d.ctl->total_units;
    const int tid = threadIdx.x;
    const uint32_t lane = tid & 63, w = tid >> 6;
    // blocks are dealt to the 8 XCDs round-robin: give each XCD a contiguous
    // Morton range of work units so that neighbouring blocks share its L2
    const int xcd = blockIdx.x & 7;
    const int64_t per_xcd = (int64_t)(gridDim.x >> 3);
    const int64_t chunk = ceil_div(U, 8);
    const int64_t u_end = (xcd + 1) * chunk < U ? (xcd + 1) * chunk : U;
    int par = 0;
    for (int64_t u = xcd * chunk + (blockIdx.x >> 3); u < u_end; u += per_xcd) {
        if (!DIAG && lookahead) {
            // with static detection most units may have no active agent: the
            // 256 threads test the next 256 units of this block at once and
            // jump to the first active one
            for (;;) {
                const int64_t uu = u + (int64_t)tid * per_xcd;
                bool act = false;
                if (uu < u_end) {
                    const int s2 = find_sim(wblk, d.n_sims, uu);
                    const SimDesc &S2 = sims[s2];
                    act = !S2.detect_static || active_blk[S2.b_off + (uu - wblk[s2])] != 0;
                }
                const uint64_t am = __builtin_amdgcn_ballot_w64(act);
                if (lane == 0) L.ahead[par][w] = am;
                __syncthreads();  // (two buffers: the next pass writes the other one)
                int first = -1;
                for (int v = 0; v < 4 && first < 0; ++v) {
                    const uint64_t mv = L.ahead[par][v];
                    if (mv) first = v * 64 + __ffsll((long long)mv) - 1;
                }
                par ^= 1;
                if (first >= 0) {
                    u += (int64_t)first * per_xcd;
                    break;
                }
                u += 256 * per_xcd;
                if (u >= u_end) break;
            }
            if (u >= u_end) break;
        }
        const int s = find_sim(wblk, d.n_sims, u);
        const SimDesc &S = sims[s];
        // with static detection, a block whose agents are all static and
        // settled needs no visit (marked while binning the grid); the
        // diagnostic mode visits every block to write its per-agent fields
        if (!DIAG && S.detect_static && !active_blk[S.b_off + (u - wblk[s])]) continue;
        int qx, qy, qz;
        unpack_key(blist[S.b_off + (u - wblk[s])], qx, qy, qz);
        // Wave priority rises as a unit advances through its phases (table 0,
        // stage 1, setup 2, pair tests and commit 3): waves further along issue
        // first, so the waves of a block reach its barriers together while
        // other blocks' loads fill the gaps.
        __builtin_amdgcn_s_setprio(0);
        // ---- table of the 6x6x6 staged boxes (x fastest).  One scan of packed
        // counts gives the staged index of every box (low word) and the target
        // index of every core box (high word).
        uint32_t cnt = 0;
        int cb = -1;  // core box index (targets), or -1
        if (tid < kNb) {
            const int lx = tid % kHalo, ly = (tid / kHalo) % kHalo, lz = tid / (kHalo * kHalo);
            const int gx = qx * kBlk + lx - 1, gy = qy * kBlk + ly - 1, gz = qz * kBlk + lz - 1;
            uint32_t src = 0;
            if (gx >= 0 && gy >= 0 && gz >= 0 && gx < S.dims[0] && gy < S.dims[1] && gz < S.dims[2]) {
                const uint32_t m = box_rank(d, S, gx, gy, gz);
                src = d.box_start[S.sb_off + m];
                cnt = d.box_start[S.sb_off + m + 1] - src;
            }
            L.gsrc[tid] = src;
            if (lx >= 1 && lx <= kBlk && ly >= 1 && ly <= kBlk && lz >= 1 && lz <= kBlk)
                cb = (lx - 1) + kBlk * ((ly - 1) + kBlk * (lz - 1));
        }
        uint32_t total, nt;
        {
            const unsigned long long pv = (unsigned long long)cnt | ((unsigned long long)(cb >= 0 ? cnt : 0u) << 32);
            unsigned long long x = pv;
            for (int off = 1; off < 64; off <<= 1) {
                const unsigned long long y = __shfl_up(x, off);
                if ((int)lane >= off) x += y;
            }
            if (lane == 63) L.sh64[w] = x;  // read after the barrier; rewritten only in the next unit
            __syncthreads();
            unsigned long long pre = x - pv, tot = 0;
            for (int v = 0; v < 4; ++v) {
                const unsigned long long sv = L.sh64[v];
                if (v < (int)w) pre += sv;
                tot += sv;
            }
            if (tid < kNb) L.sbeg[tid] = (uint32_t)pre;
            if (cb >= 0) L.coff[cb] = (uint32_t)(pre >> 32);
            if ((uint32_t)tot <= (uint32_t)kStage) {
                // staged box of every staged agent, for the stage loop (the
                // task list is free until the setup)
                uint8_t *smap = reinterpret_cast<uint8_t *>(L.task);
                for (uint32_t j = 0; j < cnt; ++j) smap[(uint32_t)pre + j] = (uint8_t)tid;
            }
            if (tid == 0) {
                L.sbeg[kNb] = (uint32_t)tot;
                L.coff[kCore] = (uint32_t)(tot >> 32);
            }
            if (tid < kBuckets) L.bcnt[tid] = 0;
            total = (uint32_t)tot;
            nt = (uint32_t)(tot >> 32);
        }
        __syncthreads();
        const float kU = S.kU, gU = S.gU;
        // largest reach beyond the target radius (U units): largest radius,
        // reach guard and a margin of 2^-10 L for the FP32 face distances
        const float reach_add = (float)ldexp(S.rmax / S.L, kFixBits) + kReach + (float)(1 << (kFixBits - 10));
        const bool lds_path = total <= (uint32_t)kStage && nt <= (uint32_t)kMaxT;
        if (!lds_path) {  // box-wise: in the diagnostic mode here, else queued for k_sweep_dense
            if constexpr (DIAG) sweep_unit_dense<DIAG>(d, S, L, P, lp, qx, qy, qz);
            else queue_dense_unit(d, L.sbeg, u);
            __syncthreads();  // the next unit reuses the LDS tables
            continue;
        }
        __builtin_amdgcn_s_setprio(1);
        // ---- stage: box-relative -> relative to the centre of the 6x6x6 region
        // (|x| < 3L).  A staged agent of a core box is a target: static skip
        // (Sec 5.5), staged index, core box, agent index, zero accumulators.
        int active = 0, anystat = 0;
        const uint8_t *smap = reinterpret_cast<const uint8_t *>(L.task);
        for (uint32_t k = tid; k < total; k += blockDim.x) {
            const int lo = smap[k];
            const uint32_t kb = k - L.sbeg[lo];
            Pay c = d.payload[L.gsrc[lo] + kb];
            const int lx = lo % kHalo, ly = (lo / kHalo) % kHalo, lz = lo / (kHalo * kHalo);
            uint16_t tm = kNoTarget;
            if (lx >= 1 && lx <= kBlk && ly >= 1 && ly <= kBlk && lz >= 1 && lz <= kBlk) {
                const int cb = (lx - 1) + kBlk * ((ly - 1) + kBlk * (lz - 1));
                const uint32_t t = L.coff[cb] + kb;
                const uint32_t ia = d.sorted_idx[L.gsrc[lo] + kb];
                bool stat = false;
                if (S.detect_static) {
                    const int64_t i = ia;
                    const uint8_t fl = d.flags[lp][i];
                    if (fl & kStatic) {
                        skip_static<DIAG>(d, S, i, P, lp, fl,
                                          linear_box(qx * kBlk + lx - 1, qy * kBlk + ly - 1, qz * kBlk + lz - 1,
                                                     S.dims));
                        stat = true;
                    }
                }
                active |= stat ? 0 : 1;
                anystat |= stat ? 1 : 0;
                L.tself[t] = stat ? kNoTarget : (uint16_t)k;
                L.tbox[t] = (uint8_t)cb;
                L.tidx[t] = ia;
                L.acc[0][t] = 0;
                L.acc[1][t] = 0;
                L.acc[2][t] = 0;
                L.acm[t] = 0;
                if (DIAG) L.anbr[t] = 0;
                if (!stat) tm = (uint16_t)t;
            }
            // relative to the region centre: exact integer shifts, |x| <= 3L
            c.x += (lx - 3) * kUnitL;
            c.y += (ly - 3) * kUnitL;
            c.z += (lz - 3) * kUnitL;
            L.sp[k] = c;
            L.tmap[k] = tm;
        }
        // whether any target is active, and whether any is static: the waves'
        // ballots meet in LDS (one barrier)
        {
            const uint64_t ba = __builtin_amdgcn_ballot_w64(active != 0);
            const uint64_t bs = __builtin_amdgcn_ballot_w64(anystat != 0);
            if (lane == 0) L.sh[w] = (ba ? 1u : 0u) | (bs ? 2u : 0u);  // read below; rewritten a unit later
        }
        __syncthreads();
        const uint32_t any = L.sh[0] | L.sh[1] | L.sh[2] | L.sh[3];
        if (!(any & 1u)) continue;  // every target static: nothing to sweep
        // the half shell needs every core agent of the unit to be a target
        const bool n3 = !DIAG && !(S.detect_static && (any & 2u));
        __builtin_amdgcn_s_setprio(2);
        // ---- setup: candidate ranges of every active target (at most two per
        // thread), task counts per length; the ranges stay in registers for
        // the task scatter
        static_assert(kMaxT <= 512, "two targets per thread");
        uint32_t rw[2][kRows];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t t = (uint32_t)tid + 256u * (uint32_t)h;
#pragma unroll
            for (int r = 0; r < kRows; ++r) rw[h][r] = 0u;
            if (t >= nt) continue;
            const uint32_t self = L.tself[t];
            if (self == kNoTarget) continue;
            int cx, cy, cz;
            core_box_coords(L.tbox[t], cx, cy, cz);
            const uint32_t rows = row_mask<DIAG>(L.sp[self], cx, cy, cz, reach_add);
#pragma unroll
            for (int r = 0; r < kRows; ++r) {
                uint32_t b0, len;
                task_range<DIAG>(L, rows, cx, cy, cz, r, n3, self, b0, len);
                if (len) {
                    atomicAdd(&L.bcnt[len < kBuckets ? len : kBuckets - 1], 1u);
                    rw[h][r] = (b0 << 9) | (len << 19);
                }
            }
        }
        __syncthreads();
        if (tid < 64) {  // bucket offsets, longest tasks first (one wave)
            const uint32_t b = kBuckets - 1 - tid;
            const uint32_t cc = L.bcnt[b];
            uint32_t x = cc;
            for (int off = 1; off < 64; off <<= 1) {
                uint32_t y = __shfl_up(x, off);
                if (tid >= off) x += y;
            }
            L.boff[b] = x - cc;
            if (tid == 63) L.ntask = x;
        }
        __syncthreads();
        if (L.ntask > (uint32_t)kTaskCap) {  // rare: more tasks than the list holds; box-wise as above
            if constexpr (DIAG) sweep_unit_dense<DIAG>(d, S, L, P, lp, qx, qy, qz);
            else queue_dense_unit(d, L.sbeg, u);
            __syncthreads();  // the next unit reuses the LDS tables
            continue;
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t t = (uint32_t)tid + 256u * (uint32_t)h;
#pragma unroll
            for (int r = 0; r < kRows; ++r) {
                const uint32_t len = rw[h][r] >> 19;
                if (len) {
                    const uint32_t p = atomicAdd(&L.boff[len < kBuckets ? len : kBuckets - 1], 1u);
                    L.task[p] = rw[h][r] | t;
                }
            }
        }
        __syncthreads();
        __builtin_amdgcn_s_setprio(3);
        // ---- sweep: chunks of 64 tasks per wave, survivors through the queue
        {
            uint32_t *qw = L.queue[w];
            uint32_t qn = 0;  // wave-uniform queue fill
            const uint32_t ntask = L.ntask;
            for (uint32_t c0 = w * 64; c0 < ntask; c0 += 256) {
                const uint32_t j = c0 + lane;
                const bool tv = j < ntask;
                const uint32_t tk = L.task[tv ? j : c0];
                const uint32_t t = tk & 511u;
                const uint32_t b0 = (tk >> 9) & 1023u;
                const uint32_t len = tv ? tk >> 19 : 0u;
                const uint32_t self = L.tself[t];
                const Pay own = L.sp[self];
                const float owg = own.r + kReach;
                const uint32_t tq = (t << 20) | (self << 10) | b0;  // + kk: b0 + kk < kStage
                uint32_t nb = 0;
                bool un = false;
                // wave-uniform trip counts: the tasks are sorted by length, longest
                // first, and buckets below the last (kBuckets - 1 and up) hold one
                // length each, so the chunk's first task is its longest unless it
                // lies in the last bucket, and every task has at least as many
                // candidates as the last lane's (an invalid lane has none) or
                // kBuckets - 1, whichever is smaller
                uint32_t maxlen = __builtin_amdgcn_readlane(len, 0);
                if (maxlen >= (uint32_t)kBuckets - 1u) {
                    uint32_t mx = len;
                    for (int off = 1; off < 64; off <<= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, off));
                    maxlen = __builtin_amdgcn_readlane(mx, 0);
                }
                const uint32_t minlen = min((uint32_t)__builtin_amdgcn_readlane(len, 63), (uint32_t)kBuckets - 1u);
                // candidates b0, b0+1, ... two per trip, each loaded one test ahead.
                // Below minlen every lane is inside its row (the read-ahead stays
                // within the stage's guard entry); past it, lanes beyond their row
                // end read clamped indices and are masked
                uint32_t kk = 0;
                if (minlen >= 2) {
                    const Pay *row = L.sp + b0;
                    Pay ca = row[0];
                    for (; kk + 1u < minlen; kk += 2) {
                        const Pay cb = row[kk + 1u];
                        reach_test<DIAG, false>(L, qw, qn, own, owg, ca, kk, len, tq, self, b0, nb, un, kU, gU, n3);
                        ca = row[kk + 2u];
                        reach_test<DIAG, false>(L, qw, qn, own, owg, cb, kk + 1u, len, tq, self, b0, nb, un, kU, gU,
                                                n3);
                    }
                }
                if (kk < maxlen) {
                    const uint32_t last = (uint32_t)kStage - 1u;
                    Pay ca = L.sp[min(b0 + kk, last)];
                    for (; kk < maxlen; kk += 2) {
                        const Pay cb = L.sp[min(b0 + kk + 1u, last)];
                        reach_test<DIAG, true>(L, qw, qn, own, owg, ca, kk, len, tq, self, b0, nb, un, kU, gU, n3);
                        ca = L.sp[min(b0 + kk + 2u, last)];
                        if (kk + 1u < maxlen)
                            reach_test<DIAG, true>(L, qw, qn, own, owg, cb, kk + 1u, len, tq, self, b0, nb, un, kU,
                                                   gU, n3);
                    }
                }
                if (DIAG && tv) {
                    atomicAdd(&L.anbr[t], nb);
                    if (un) atomicAdd(&L.acc[1][t], kCnt1);
                }
            }
            if (qn) {
                __builtin_amdgcn_wave_barrier();
                drain_queue<DIAG>(L, qw, qn, kU, gU, n3);
            }
        }
        __syncthreads();
        // ---- commit
        for (uint32_t t = tid; t < nt; t += blockDim.x) {
            if (L.tself[t] == kNoTarget) continue;
            const int c = L.tbox[t];
            int cx, cy, cz;
            core_box_coords(c, cx, cy, cz);
            const int64_t i = L.tidx[t];
            const int64_t lin = linear_box(qx * kBlk + cx, qy * kBlk + cy, qz * kBlk + cz, S.dims);
            const unsigned long long w0 = L.acc[0][t], w1 = L.acc[1][t], w2 = L.acc[2][t], wm = L.acm[t];
            const long long fxi = fix_field(w0), fyi = fix_field(w1), fzi = fix_field(w2);
            bool unc = cnt_field(w1, fyi) != 0;
            if (!unc) {
                const double fx = (double)fxi * kFixUnit, fy = (double)fyi * kFixUnit, fz = (double)fzi * kFixUnit;
                if (fp32_certified(S, fx, fy, fz, (double)(uint32_t)(wm >> 32) * 0x1.0p-28,
                                   (double)(uint32_t)wm * 0x1.0p-17)) {
                    const int nc = (int)cnt_field(w0, fxi);
                    // box slot: the unit's block has Morton rank u - wblk_begin (its blist entry)
                    const uint32_t m = (uint32_t)(u - wblk[s]) * 64u + local_morton(cx, cy, cz);
                    const uint8_t fl = d.flags[lp][i];
                    commit_agent<DIAG>(d, S, i, P, lp, fl, d.pos[P][i], d.pos[P][A + i], d.pos[P][2 * A + i], fx, fy,
                                       fz, nc, DIAG ? (int)L.anbr[t] : 0, nc, m, lin);
                } else {
                    unc = true;
                }
            }
            if (unc) d.fix_list[atomicAdd(&d.ctl->n_fix, 1u)] = (uint32_t)i;
        }
        __syncthreads();  // the next unit reuses the LDS
    }
}

// ------------------------------------------------------------------ box-wise sweep
// The items the sweep queued, dealt to the waves in order (item q to wave
// q mod the number of waves, waves numbered XCD by XCD so that the boxes of a
// unit share an L2).  A box's pass groups are separate items, so the targets
// of the densest boxes spread over several waves.
// (sims, wblk, blist: read-only and not aliased, so that their wave-uniform
// reads are scalar loads)
// NW waves per work group (a schedule parameter: the waves are independent).
template <int NW>
__global__ void __launch_bounds__(64 * NW)
    k_sweep_dense(Dev d, const SimDesc *__restrict__ sims, const int64_t *__restrict__ wblk,
                  const uint32_t *__restrict__ blist) {
    if (ABM_ABORTED(d)) return;
    const unsigned long long nq = d.ctl->n_dense;
    if (nq == 0) return;
    __shared__ DenseWave W[NW];
    const int P = d.ctl->pos_par, lp = d.ctl->lay_par;
    const uint32_t w = threadIdx.x >> 6;
    const unsigned long long n = nq < (unsigned long long)d.dense_cap ? nq : (unsigned long long)d.dense_cap;
    const unsigned long long nw = (unsigned long long)NW * gridDim.x;  // (gridDim.x: a multiple of 8)
    const unsigned long long gw = (unsigned long long)NW * ((blockIdx.x & 7u) * (gridDim.x >> 3) + (blockIdx.x >> 3)) + w;
    for (unsigned long long q = gw; q < n; q += nw) {
        const uint64_t e = d.dense_list[q];
        const int64_t u = (int64_t)(e >> 9);
        const int s = find_sim(wblk, d.n_sims, u);
        const SimDesc &S = sims[s];
        int qx, qy, qz, cx, cy, cz;
        unpack_key(blist[S.b_off + (u - wblk[s])], qx, qy, qz);
        core_box_coords((int)((e >> 3) & 63u), cx, cy, cz);
        sweep_box_dense(d, S, W[w], P, lp, qx * kBlk + cx, qy * kBlk + cy, qz * kBlk + cz, (int)(e & 7u));
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
// 128-bit sum over the lanes of a half wave (two's complement, exact).
__device__ inline void half_sum128(uint64_t &lo, uint64_t &hi) {
    for (int off = 16; off > 0; off >>= 1) {
        const uint64_t olo = __shfl_xor(lo, off), ohi = __shfl_xor(hi, off);
        const uint64_t nlo = lo + olo;
        hi = hi + ohi + (nlo < lo ? 1ull : 0ull);
        lo = nlo;
    }
}
__device__ inline int half_sum_i32(int v) {
    for (int off = 16; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}
__device__ inline double half_sum_f64(double v) {
    for (int off = 16; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Two agents per wave on the FP64 path, one per half wave: lane b < 27 of a
// half reads the slot range of neighbour box b, the candidates of all 27
// boxes are dealt to the half's lanes, and the exact per-lane sums are added
// over the half.  (All shuffles stay within a half, so a half that has no
// agent left may drop out while the other goes on.)
template <bool DIAG>
__global__ void __launch_bounds__(256)
    k_fixup(Dev d, const SimDesc *__restrict__ sims, const int64_t *__restrict__ a_begin) {  // (read-only, not aliased)
#pragma clang fp contract(off)
    __shared__ uint32_t bst[8][27], bpre[8][28];
    if (ABM_ABORTED(d)) return;
    const int P = d.ctl->pos_par, lp = d.ctl->lay_par;
    const int64_t A = d.A;
    const uint32_t nf = d.ctl->n_fix;
    const uint32_t w = threadIdx.x >> 5, lane = threadIdx.x & 31;  // half wave, lane in it
    for (uint32_t q = blockIdx.x * 8 + w; q < nf; q += gridDim.x * 8) {
        const int64_t i = d.fix_list[q];
        const int s = find_sim(a_begin, d.n_sims, i);
        const SimDesc &S = sims[s];
        const double x = d.pos[P][i], y = d.pos[P][A + i], z = d.pos[P][2 * A + i];
        const double ri = 0.5 * d.diam[lp][i];
        const double L2 = S.L * S.L;
        int bx, by, bz;
        unpack_key(d.key[i], bx, by, bz);
        uint32_t cnt = 0, st = 0;
        if (lane < 27) {
            const int cx = bx + (int)(lane % 3) - 1, cy = by + (int)(lane / 3 % 3) - 1, cz = bz + (int)(lane / 9) - 1;
            if (cx >= 0 && cy >= 0 && cz >= 0 && cx < S.dims[0] && cy < S.dims[1] && cz < S.dims[2]) {
                const uint32_t m = box_rank(d, S, cx, cy, cz);
                st = d.box_start[S.sb_off + m];
                cnt = d.box_start[S.sb_off + m + 1] - st;
            }
        }
        uint32_t pre = cnt;  // inclusive scan over the half's lanes
        for (int off = 1; off < 32; off <<= 1) {
            const uint32_t o = __shfl_up(pre, off, 32);
            if (lane >= (uint32_t)off) pre += o;
        }
        const uint32_t total = __shfl(pre, 31, 32);
        if (lane < 27) {
            bst[w][lane] = st;
            bpre[w][lane] = pre - cnt;
        }
        if (lane == 27) bpre[w][27] = total;
        __builtin_amdgcn_wave_barrier();
        double fx = 0.0, fy = 0.0, fz = 0.0;  // plain sums, used only when a term is huge
        Fix128 sx, sy, sz;
        int nbr = 0, contacts = 0, nzc = 0;
        for (uint32_t c = lane; c < total; c += 32) {
            int lo = 0, hi = 27;  // box of candidate c: the largest b with bpre[b] <= c
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (bpre[w][mid] <= c) lo = mid; else hi = mid;
            }
            const int64_t j = d.sorted_idx[bst[w][lo] + (c - bpre[w][lo])];
            if (j == i) continue;
            const double ddx = x - d.pos[P][j], ddy = y - d.pos[P][A + j], ddz = z - d.pos[P][2 * A + j];
            const double d2 = fma(ddz, ddz, fma(ddy, ddy, ddx * ddx));
            if (!(d2 < L2)) continue;
            ++nbr;
            const double rj = 0.5 * d.diam[lp][j];
            const double dist = sqrt(d2);
            const double delta = ri + rj - dist;
            if (!(delta > 0.0)) continue;
            ++contacts;
            const double rbar = ri * rj / (ri + rj);
            const double fn = S.k * delta - S.gamma * sqrt(rbar * delta);
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
        __builtin_amdgcn_wave_barrier();  // the box tables are rewritten for the next agent
        nbr = half_sum_i32(nbr);
        contacts = half_sum_i32(contacts);
        nzc = half_sum_i32(nzc);
        const uint64_t bw = __builtin_amdgcn_ballot_w64(sx.wide || sy.wide || sz.wide);
        const bool wide = ((w & 1u) ? (bw >> 32) : (bw & 0xffffffffull)) != 0;
        if (wide) {
            fx = half_sum_f64(fx);
            fy = half_sum_f64(fy);
            fz = half_sum_f64(fz);
        } else {
            half_sum128(sx.lo, sx.hi);
            half_sum128(sy.lo, sy.hi);
            half_sum128(sz.lo, sz.hi);
            fx = sx.value();
            fy = sy.value();
            fz = sz.value();
        }
        if (lane == 0) {
            const uint8_t fl = d.flags[lp][i];
            const int64_t lin = linear_box(bx, by, bz, S.dims);
            commit_agent<DIAG>(d, S, i, P, lp, fl, x, y, z, fx, fy, fz, nzc, nbr, contacts, box_rank(d, S, bx, by, bz),
                               lin);
        }
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

// Fate of every cell from the start-of-iteration state (Algorithm 2): removal
// (at least min_age iterations old and the death draw below the death
// probability), then, for the cells that stay, division (at or above the
// division volume and the division draw below the division probability).  A removed cell is no change for the static rule (Sec 5.5,
// condition iv): its change bits are cleared.  Each agent tile also writes
// its number of removals (rm_sum) for the compaction's scan; the totals come
// from the scans, not from atomics.
__global__ void __launch_bounds__(256) k_fate(Dev d) {
    if (ABM_ABORTED(d)) return;
    __shared__ uint32_t wsum[4];
    const int lp = d.ctl->lay_par;
    const int64_t total = d.ctl->total_tiles;
    const int64_t iter = d.ctl->iter;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int s = find_sim(d.tile_begin, d.n_sims, t);
        const SimDesc &S = d.sims[s];
        const bool growth = S.div_vol > 0.0, death = S.death_prob > 0.0;
        int64_t loc = (t - d.tile_begin[s]) * kTile + threadIdx.x;
        bool dead = false;
        if ((growth || death) && loc < S.n_start) {
            const int64_t i = S.a_off + loc;
            const uint64_t u_id = d.uid[lp][i];
            uint32_t c[4];
            if (death && iter - (int64_t)d.birth[lp][i] >= (int64_t)S.min_age) {
                agent_draw(S.seed, kTagDeath, S.sim_id, u_id, (uint64_t)iter, c);
                dead = uniform_open(c[0]) < S.death_prob;
            }
            if (dead) {
                d.flags[lp][i] = (uint8_t)((d.flags[lp][i] & ~kChgMask) | kDead);
            } else if (growth && d.vol[lp][i] >= S.div_vol) {
                bool div = S.division_prob >= 1.0;
                if (!div) {
                    agent_draw(S.seed, kTagDivision, S.sim_id, u_id, (uint64_t)iter, c);
                    div = uniform_open(c[0]) < S.division_prob;
                }
                if (div) d.divflag[S.a_off + u_id] = 1u;
            }
        }
        const uint64_t bd = __ballot(dead);
        if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = (uint32_t)__popcll(bd);
        __syncthreads();
        if (threadIdx.x == 0) d.rm_sum[t] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        __syncthreads();
    }
}

// Layout of the divider scan: tiles of kBoxTile uids per simulation with growth.
__global__ void k_div_plan(Dev d) {
    if (ABM_ABORTED(d)) return;
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int s = 0; s < d.n_sims; ++s) {
            d.utile_begin[s] = t;
            t += d.sims[s].div_vol > 0.0 ? ceil_div(d.sims[s].next_uid, kBoxTile) : 0;
        }
        d.utile_begin[d.n_sims] = t;
        d.ctl->total_utiles = t;
    }
}

// Capacity check once the divider scan has counted the divisions (n_div).
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
    if (threadIdx.x == 0 && bad) d.ctl->abort = 1;
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

// Exclusive scan of per-tile counts within each simulation's tile range
// (begin: n_sims + 1 tile prefix): offsets into off; each simulation's total
// goes to its n_div (what = 0) or n_dead (what = 1).
__global__ void __launch_bounds__(1024) k_tile_scan(Dev d, const int64_t *begin, const uint32_t *sum, uint32_t *off,
                                                    int what) {
    if (ABM_ABORTED(d)) return;
    __shared__ uint32_t sh[16];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int s = blockIdx.x; s < d.n_sims; s += gridDim.x) {  // one work group per simulation
        int64_t b0 = begin[s], b1 = begin[s + 1];
        uint32_t carry = 0;
        for (int64_t c = b0; c < b1; c += blockDim.x) {
            int64_t t = c + threadIdx.x;
            uint32_t v = t < b1 ? sum[t] : 0u;
            uint32_t x = v;
            for (int o = 1; o < 64; o <<= 1) {
                uint32_t y = __shfl_up(x, o);
                if (lane >= o) x += y;
            }
            if (lane == 63) sh[wid] = x;
            __syncthreads();
            uint32_t wpre = 0, tot = 0;
            for (int w = 0; w < 16; ++w) {
                if (w < wid) wpre += sh[w];
                tot += sh[w];
            }
            if (t < b1) off[t] = carry + wpre + x - v;
            carry += tot;
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (what == 0) d.sims[s].n_div = carry;
            else d.sims[s].n_dead = carry;
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
        if (d.flags[lp][i] & kDead) continue;  // removed: neither grows nor divides
        const uint64_t u_id = d.uid[lp][i];
        if (v >= S.div_vol && d.divflag[S.a_off + u_id]) {
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
            d.birth[lp][j] = (int32_t)(iter + 1);  // present from the next iteration, at age 0
            d.flags[lp][j] = kBufDiff | kNew;
            d.flags[lp][i] = (d.flags[lp][i] & ~kStatic) | kBufDiff | kMoved | kDivided;
        } else if (v < S.div_vol) {
            double nv = v + d.growth[lp][i];
            d.vol[lp][i] = nv;
            d.diam[lp][i] = diameter_from_volume(nv);
            d.flags[lp][i] |= kGrew;
        } else {
            continue;  // at the division volume with a failed division draw: no change
        }
        if (S.detect_static) mark_box(d.dirty, d.dirty_blk, S, key_rank(d, S, d.key[i]));  // start box of a changed agent
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
// One wave per aligned block.  A block with no active agent and no changed
// agent within one box keeps the flags of its agents: they stay static.
// Each wave checks 64 aligned blocks at a time, one per lane, strided by the
// number of waves of the grid (so that blocks to visit spread over all waves,
// one per wave when there are few): whether a block needs a visit (near a
// change, or holding active agents); the wave then visits those blocks.  (sims, btiles: read-only and not
// aliased, so that their wave-uniform reads are scalar loads.)
__global__ void __launch_bounds__(256) k_static(Dev d, const SimDesc *__restrict__ sims,
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
        uint32_t need = 0;  // bit 0: visit, bit 1: near a change
        if (qc < nq) {
            const int64_t tl = qc / kTB;
            const int sl = find_sim(btiles, d.n_sims, tl);
            const SimDesc &Sl = sims[sl];
            const int64_t bl = (tl - btiles[sl]) * kTB + qc % kTB;
            if (Sl.detect_static && bl < Sl.nblocks) {
                const bool nr = d.near_blk[Sl.b_off + bl] != 0;
                need = (nr || d.active_blk[Sl.b_off + bl]) ? (nr ? 3u : 1u) : 0u;
            }
        }
        for (uint64_t mv = __builtin_amdgcn_ballot_w64(need != 0); mv; mv &= mv - 1) {
            const int l = __ffsll((long long)mv) - 1;
            const int64_t q = q0 + l * nw;
            const bool near = (__shfl(need, l) & 2u) != 0;
            const int64_t t = q / kTB;
            int s = find_sim(btiles, d.n_sims, t);
            const SimDesc &S = sims[s];
            const int64_t blk = (t - btiles[s]) * kTB + q % kTB;
            // the agents binned at the start of the iteration (daughters are new: never static)
            const uint32_t s0 = d.box_start[S.sb_off + blk * 64], s1 = d.box_start[S.sb_off + blk * 64 + 64];
            for (uint32_t slot0 = s0; slot0 < s1; slot0 += 64) {
                const uint32_t slot = slot0 + (uint32_t)lane;
                if (slot >= s1) continue;
                const int64_t i = d.sorted_idx[slot];
                const uint8_t fl = d.flags[lp][i];
                bool st = !(fl & kChgMask) && d.nz[lp][i] <= 1;
                if (st && near) {
                    int bx, by, bz;
                    unpack_key(d.key[i], bx, by, bz);
                    const double x = d.pos[P][i], y = d.pos[P][A + i], z = d.pos[P][2 * A + i];
                    const double L2 = S.L * S.L;
                    for (int oz = -1; oz <= 1 && st; ++oz)
                        for (int oy = -1; oy <= 1 && st; ++oy)
                            for (int ox = -1; ox <= 1 && st; ++ox) {
                                int cx = bx + ox, cy = by + oy, cz = bz + oz;
                                if (cx < 0 || cy < 0 || cz < 0 || cx >= S.dims[0] || cy >= S.dims[1] || cz >= S.dims[2])
                                    continue;
                                uint32_t m = box_rank(d, S, cx, cy, cz);
                                if (!d.dirty[S.b_off + m]) continue;
                                uint32_t b0 = d.box_start[S.sb_off + m], b1 = d.box_start[S.sb_off + m + 1];
                                for (uint32_t sl = b0; sl < b1 && st; ++sl) {
                                    int64_t j = d.sorted_idx[sl];
                                    if (j == i || !(d.flags[lp][j] & kChgMask)) continue;
                                    // start position (buffer P) and committed position (buffer 1-P)
                                    if (near_point(x, y, z, d.pos[P][j], d.pos[P][A + j], d.pos[P][2 * A + j], L2) ||
                                        near_point(x, y, z, d.pos[1 - P][j], d.pos[1 - P][A + j], d.pos[1 - P][2 * A + j],
                                                   L2))
                                        st = false;
                                }
                            }
                }
                const uint8_t nf = st ? (fl | kStatic) : (fl & ~kStatic);
                if (nf != fl) d.flags[lp][i] = nf;
            }
        }
    }
}

// ------------------------------------------------------------------ removals
// Removed cells leave the state at the end of the iteration without gaps
// (Sec 5.3.2, Fig 5.1): with R removals out of m agents (daughters included,
// never removed in the iteration that creates them) the state shrinks to
// m - R.  Removed cells left of m - R are holes; living cells right of it
// are movers; there are as many of each, and the k-th mover (ascending index)
// fills the k-th hole.  Both ranks come from one index-ordered exclusive scan
// of the removal flags (dp = removals before an index): a hole's rank is dp,
// a mover's is its offset past m - R minus the removals in between.  Only
// the R movers are copied, and the result does not depend on any timing.

// Prefix of the mover counts (the removals R) over the simulations, once
// the scan of k_fate's per-tile counts has given each simulation's R.
__global__ void k_rm_plan(Dev d) {
    if (ABM_ABORTED(d)) return;
    if (threadIdx.x == 0) {
        int64_t mv = 0;
        for (int s = 0; s < d.n_sims; ++s) {
            d.mv_begin[s] = mv;
            mv += d.sims[s].n_dead;
        }
        d.mv_begin[d.n_sims] = mv;
    }
}

// Per agent tile (kTile agents of [0, n_start)): the removals before each
// agent (dp, from the tile's offset and a block scan); each hole writes its
// index at its rank (into fix_list, free after the FP64 path), and agents of
// the tail [keep, n_start) keep dp for the movers (into divrank, free after
// the divisions).
__global__ void __launch_bounds__(256) k_rm_apply(Dev d) {
    if (ABM_ABORTED(d)) return;
    __shared__ uint32_t wsum[4];
    const int lp = d.ctl->lay_par;
    const int64_t total = d.ctl->total_tiles;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        const int s = find_sim(d.tile_begin, d.n_sims, t);
        const SimDesc &S = d.sims[s];
        if (S.n_dead == 0) continue;  // (block-uniform)
        const int64_t k = (t - d.tile_begin[s]) * kTile + threadIdx.x;
        const bool dead = k < S.n_start && (d.flags[lp][S.a_off + k] & kDead);
        const uint64_t bd = __ballot(dead);
        if (lane == 0) wsum[w] = (uint32_t)__popcll(bd);
        __syncthreads();
        uint32_t dp = d.rm_off[t] + (uint32_t)__popcll(bd & ((1ull << lane) - 1ull));
        for (int v = 0; v < w; ++v) dp += wsum[v];
        const int64_t keep = S.n_start + S.n_div - S.n_dead;
        if (dead && k < keep) d.fix_list[S.a_off + dp] = (uint32_t)k;
        if (k >= keep && k < S.n_start) d.divrank[S.a_off + k] = dp;
        __syncthreads();
    }
}

__device__ inline bool dead_flag(const Dev &d, const SimDesc &S, int lp, int64_t k) {
    return k < S.n_start && (d.flags[lp][S.a_off + k] & kDead);
}

// The movers fill the holes: every per-agent field of the state (both
// position buffers) and, when recorded, the iteration's recorded fields.
__global__ void __launch_bounds__(256) k_rm_move(Dev d, int record) {
    if (ABM_ABORTED(d)) return;
    const int lp = d.ctl->lay_par;
    const int64_t A = d.A;
    const int64_t total = d.mv_begin[d.n_sims];
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int s = find_sim(d.mv_begin, d.n_sims, g);
        const SimDesc &S = d.sims[s];
        const int64_t R = S.n_dead, keep = S.n_start + S.n_div - R;
        const int64_t k = keep + (g - d.mv_begin[s]);  // in [keep, m)
        if (dead_flag(d, S, lp, k)) continue;           // a removed cell past the new end
        const int64_t dpk = k < S.n_start ? (int64_t)d.divrank[S.a_off + k] : R;
        const int64_t dpe = keep < S.n_start ? (int64_t)d.divrank[S.a_off + keep] : R;  // (k >= keep: written)
        const int64_t rank = (k - keep) - (dpk - dpe);
        const int64_t i = S.a_off + k, j = S.a_off + (int64_t)d.fix_list[S.a_off + rank];
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 3; ++a) d.pos[b][a * A + j] = d.pos[b][a * A + i];
        d.diam[lp][j] = d.diam[lp][i];
        d.vol[lp][j] = d.vol[lp][i];
        d.growth[lp][j] = d.growth[lp][i];
        d.uid[lp][j] = d.uid[lp][i];
        d.flags[lp][j] = d.flags[lp][i];
        d.nz[lp][j] = d.nz[lp][i];
        d.birth[lp][j] = d.birth[lp][i];
        if (record) {
            for (int a = 0; a < 3; ++a) {
                d.force[3 * j + a] = d.force[3 * i + a];
                d.disp[3 * j + a] = d.disp[3 * i + a];
            }
            d.nbr[j] = d.nbr[i];
            d.contacts[j] = d.contacts[i];
            d.boxid[j] = d.boxid[i];
        }
    }
}

// ------------------------------------------------------------------ launchers
void launch_sweep(const Dev &d, hipStream_t st, const Sched &sc, bool diag, bool any_static) {
    const SimDesc *sims = d.sims;
    if (diag) {
        hipLaunchKernelGGL(k_sweep<true>, dim3(sc.sweep_grid), dim3(256), 0, st, d, sims, d.wblk_begin, d.blist,
                           d.active_blk, 0);
    } else {
        hipLaunchKernelGGL(k_sweep<false>, dim3(sc.sweep_grid), dim3(256), 0, st, d, sims, d.wblk_begin, d.blist,
                           d.active_blk, any_static ? 1 : 0);
        // the units queued for the box-wise path (the kernel returns at once
        // when there are none)
        if (sc.dense_waves == 2)
            hipLaunchKernelGGL(k_sweep_dense<2>, dim3(sc.dense_grid), dim3(128), 0, st, d, sims,
                               (const int64_t *)d.wblk_begin, (const uint32_t *)d.blist);
        else
            hipLaunchKernelGGL(k_sweep_dense<4>, dim3(sc.dense_grid), dim3(256), 0, st, d, sims,
                               (const int64_t *)d.wblk_begin, (const uint32_t *)d.blist);
    }
}

// Everything of one iteration after the sweep; ends by building the grid of
// the committed state.
void launch_after_sweep(const Dev &d, hipStream_t st, int grid_agents, int grid_boxes, bool diag, bool any_growth,
                        bool any_static, bool resort, bool any_death, bool any_record) {
    // two agents per wave on the FP64 path (32768 at a time, grid-stride beyond)
    const SimDesc *sims = d.sims;
    const int64_t *a_begin = d.a_begin;
    if (diag) hipLaunchKernelGGL(k_fixup<true>, dim3(4096), dim3(256), 0, st, d, sims, a_begin);
    else hipLaunchKernelGGL(k_fixup<false>, dim3(4096), dim3(256), 0, st, d, sims, a_begin);
    if (any_growth || any_death) hipLaunchKernelGGL(k_fate, dim3(grid_agents), dim3(256), 0, st, d);
    if (any_growth) {
        hipLaunchKernelGGL(k_div_plan, dim3(1), dim3(64), 0, st, d);
        hipLaunchKernelGGL(k_uscan_tiles, dim3(grid_boxes), dim3(256), 0, st, d);
        hipLaunchKernelGGL(k_tile_scan, dim3(d.n_sims), dim3(1024), 0, st, d, (const int64_t *)d.utile_begin,
                           (const uint32_t *)d.tile_sum, d.tile_off, 0);
        hipLaunchKernelGGL(k_div_check, dim3(1), dim3(256), 0, st, d);
        hipLaunchKernelGGL(k_uscan_apply, dim3(grid_boxes), dim3(256), 0, st, d);
        hipLaunchKernelGGL(k_div_apply, dim3(grid_agents), dim3(256), 0, st, d);
    }
    if (any_static) {
        launch_near_marks(d, st, grid_boxes, false);
        hipLaunchKernelGGL(k_static, dim3(grid_boxes), dim3(256), 0, st, d, (const SimDesc *)d.sims,
                           (const int64_t *)d.btile_begin);
    }
    if (any_death) {
        hipLaunchKernelGGL(k_tile_scan, dim3(d.n_sims), dim3(1024), 0, st, d, (const int64_t *)d.tile_begin,
                           (const uint32_t *)d.rm_sum, d.rm_off, 1);
        hipLaunchKernelGGL(k_rm_plan, dim3(1), dim3(64), 0, st, d);
        hipLaunchKernelGGL(k_rm_apply, dim3(grid_agents), dim3(256), 0, st, d);
        hipLaunchKernelGGL(k_rm_move, dim3(grid_agents), dim3(256), 0, st, d, (diag || any_record) ? 1 : 0);
    }
    launch_end(d, st, grid_boxes, any_static);
    if (resort) launch_resort(d, st, grid_agents, grid_boxes, false, any_static);
    launch_grid_build(d, st, grid_agents, grid_boxes, any_static);
}

// One iteration on the grid built at the end of the previous one.
void launch_iteration(const Dev &d, hipStream_t st, int grid_agents, int grid_boxes, const Sched &sc, bool diag,
                      bool any_growth, bool any_static, bool resort, bool any_death, bool any_record) {
    launch_sweep(d, st, sc, diag, any_static);
    launch_after_sweep(d, st, grid_agents, grid_boxes, diag, any_growth, any_static, resort, any_death, any_record);
}

}  // namespace abm
