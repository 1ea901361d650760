// abm_api.hip -- host runtime and C ABI of libabm (see include/abm.h).
//
// Device state of a batch is carved from the caller's workspace; one
// iteration (all kernels of every simulation) is captured once into a HIP
// graph and replayed per iteration.  No CPU fallback exists: every step of the
// method runs in the kernels of abm_mech.hip.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "abm_internal.h"

using namespace abm;

static thread_local std::string g_err;

namespace abm {
void clear_error() { g_err.clear(); }
int set_error(int code, const char *msg) {
    g_err = msg;
    return code;
}
}  // namespace abm

static int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                        \
    do {                                                                                    \
        hipError_t _e = (expr);                                                             \
        if (_e != hipSuccess) return fail(ABM_ERR_HIP, "%s: %s", #expr, hipGetErrorString(_e)); \
    } while (0)

extern "C" const char *abm_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------- layout
namespace {

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
    size_t sims, ctl, tile_begin, btile_begin, utile_begin, a_begin, wblk_begin, mv_begin, bnd, blist;
    size_t pos[2], diam[2], vol[2], growth[2], uid[2], flags[2], nz[2], birth[2];
    size_t stage8, key, rank, payload, sorted_idx, nbr, contacts, force, disp, boxid;
    size_t count, box_start, brank, dirty, arrive, dirty_blk, arrive_blk, active_blk, near_blk, tile_sum, tile_off, rm_sum, rm_off, fix_list, dense_list, divflag, divrank;
    size_t stat_part, hist_cnt, stat_out;
    size_t total;
};

// Items of the box-wise sweep: per core box with targets, at most
// ceil(targets / 64) pass groups, so over all units at most A / 64 plus the
// number of non-empty boxes, min(A, B).
int64_t dense_capacity(int64_t A, int64_t B) { return A / 64 + std::min(A, B) + 64; }

bool make_layout(int n_sims, const int64_t *cap, const int64_t *bcap, Layout &L, int64_t &A, int64_t &B,
                 int64_t &SB, int64_t &T, int64_t &BT) {
    if (n_sims < 1 || n_sims > kMaxSims) return false;
    A = B = SB = T = BT = 0;
    int64_t UT = 0;
    for (int s = 0; s < n_sims; ++s) {
        if (cap[s] < 1 || bcap[s] < 1) return false;
        A += cap[s];
        B += bcap[s];
        SB += bcap[s] + 1;
        T += ceil_div(cap[s], kTile);
        BT += ceil_div(bcap[s], kBoxTile);
        UT += ceil_div(cap[s], kBoxTile);
    }
    if (A >= (int64_t)0xFFFFFFF0ll || SB >= (int64_t)0xFFFFFFF0ll) return false;
    int64_t ST = std::max(BT, UT);
    Carver c;
    L.sims = c.take<SimDesc>(n_sims);
    L.ctl = c.take<Ctl>(1);
    L.tile_begin = c.take<int64_t>(n_sims + 1);
    L.btile_begin = c.take<int64_t>(n_sims + 1);
    L.utile_begin = c.take<int64_t>(n_sims + 1);
    L.a_begin = c.take<int64_t>(n_sims + 1);
    L.wblk_begin = c.take<int64_t>(n_sims + 1);
    L.mv_begin = c.take<int64_t>(n_sims + 1);
    L.bnd = c.take<unsigned long long>((size_t)n_sims * kBndSlots * 7);
    for (int b = 0; b < 2; ++b) {
        L.pos[b] = c.take<double>(3 * A);
        L.diam[b] = c.take<double>(A);
        L.vol[b] = c.take<double>(A);
        L.growth[b] = c.take<double>(A);
        L.uid[b] = c.take<uint64_t>(A);
        L.flags[b] = c.take<uint8_t>(A);
        L.nz[b] = c.take<uint8_t>(A);
        L.birth[b] = c.take<int32_t>(A);
    }
    L.stage8 = c.take<uint8_t>(A);
    L.key = c.take<uint32_t>(A);
    L.rank = c.take<uint32_t>(A);
    L.payload = c.take<Pay>(A);
    L.sorted_idx = c.take<uint32_t>(A);
    L.nbr = c.take<int32_t>(A);
    L.contacts = c.take<int32_t>(A);
    L.force = c.take<double>(3 * A);
    L.disp = c.take<double>(3 * A);
    L.boxid = c.take<int64_t>(A);
    L.count = c.take<uint32_t>(B);
    L.box_start = c.take<uint32_t>(SB);
    L.brank = c.take<uint32_t>(B);
    L.blist = c.take<uint32_t>(B);
    L.dirty = c.take<uint8_t>(B);
    L.arrive = c.take<uint8_t>(B);
    L.dirty_blk = c.take<uint8_t>(B);
    L.arrive_blk = c.take<uint8_t>(B);
    L.active_blk = c.take<uint8_t>(B);
    L.near_blk = c.take<uint8_t>(B);
    L.tile_sum = c.take<uint32_t>(ST);
    L.tile_off = c.take<uint32_t>(ST);
    L.rm_sum = c.take<uint32_t>(T);
    L.rm_off = c.take<uint32_t>(T);
    L.fix_list = c.take<uint32_t>(A);
    L.dense_list = c.take<uint64_t>(dense_capacity(A, B));
    L.divflag = c.take<uint32_t>(A);
    L.divrank = c.take<uint32_t>(A);
    L.stat_part = c.take<double>(3 * T);
    L.hist_cnt = c.take<unsigned int>(32 * (size_t)n_sims);
    L.stat_out = c.take<double>(40 * (size_t)n_sims + 16 * (size_t)n_sims);
    L.total = c.off + 256;
    return true;
}

__global__ void k_load_pos(double *p0, double *p1, int64_t A, int64_t a_off, int64_t n, const double *xyz) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        for (int a = 0; a < 3; ++a) {
            double v = xyz[3 * q + a];
            p0[a * A + a_off + q] = v;
            p1[a * A + a_off + q] = v;
        }
    }
}

// volume of a sphere of diameter d: pi d^3 / 6
__global__ void k_vol_from_diam(double *vol, const double *diam, int64_t a_off, int64_t n) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        double d = diam[a_off + q];
        vol[a_off + q] = 3.14159265358979323846 * d * d * d / 6.0;
    }
}

__global__ void k_iota_uid(uint64_t *uid, int64_t a_off, int64_t n) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        uid[a_off + q] = (uint64_t)q;
}

__global__ void k_max_uid(const uint64_t *uid, int64_t a_off, int64_t n, unsigned long long *out) {
    unsigned long long m = 0;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
    {
        unsigned long long v = (unsigned long long)uid[a_off + q] + 1ull;
        m = v > m ? v : m;
    }
    atomicMax(out, m);
}

__global__ void k_u8_from_host_layout(uint8_t *dst, const uint8_t *src, int64_t a_off, int64_t n) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        dst[a_off + q] = src[q] ? kStatic : 0;
}

__global__ void k_nz_from_i32(uint8_t *dst, const int32_t *src, int64_t a_off, int64_t n) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        int32_t v = src[q];
        dst[a_off + q] = (uint8_t)(v < 0 ? 0 : (v > 255 ? 255 : v));
    }
}

// birth = iteration - age (age = 0 where src is null)
__global__ void k_birth_from_age(int32_t *dst, const int32_t *src, int64_t a_off, int64_t n, int64_t iteration) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        dst[a_off + q] = (int32_t)(iteration - (src ? (int64_t)src[q] : 0));
}

// age = iteration - birth
__global__ void k_age(int32_t *dst, const int32_t *birth, int64_t n, int64_t iteration) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        dst[q] = (int32_t)(iteration - (int64_t)birth[q]);
}

__global__ void k_widen_u8(int32_t *dst, const uint8_t *src, int64_t n, int mask) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        dst[q] = mask ? ((src[q] & mask) ? 1 : 0) : (int32_t)src[q];
}

__global__ void k_static_u8(uint8_t *dst, const uint8_t *flags, int64_t n) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        dst[q] = (flags[q] & kStatic) ? 1 : 0;
}

int grid_for(int64_t n) {
    int64_t g = n / 256 + 1;
    return (int)std::min<int64_t>(g, 4096);
}

}  // namespace

// ---------------------------------------------------------------- handle
struct abm_batch {
    int n_sims = 0;
    Dev d{};
    Layout L{};
    char *ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;      // the caller's stream: all work is ordered on it
    hipStream_t cap_stream = nullptr;  // private stream used only to capture the graph
    std::vector<SimDesc> host_sims;
    int64_t A = 0, T = 0, BT = 0;
    Sched sched;            // launch schedule of the force sweep (autotuned)
    int grid_agents = 2048, grid_boxes = 2048;
    bool any_growth = false, any_static = false;
    bool any_death = false, any_record = false;  // Algorithm 2 removals; recorded fields
    int resort_every = 0;
    hipGraphExec_t exec[3][2] = {};  // [part][diag], see capture()
    bool grid_valid = false;         // grid of the current state is built
    bool fresh = true;               // nothing has run since create (restore is allowed)
    bool timing = false;             // bracket every sweep with events
    std::vector<hipEvent_t> ev;      // event pairs of the last step
    double sweep_ms = 0.0;
    int64_t n_sweeps = 0;
};

static void destroy_graphs(abm_batch *b) {
    for (int part = 0; part < 3; ++part)
        for (int k = 0; k < 2; ++k) {
            if (b->exec[part][k]) (void)hipGraphExecDestroy(b->exec[part][k]);  // teardown: nothing to recover
            b->exec[part][k] = nullptr;
        }
}

// part 0: one whole iteration; 1: its force sweep; 2: everything after the sweep.
static int capture(abm_batch *b, int part, int diag) {
    if (b->exec[part][diag]) return ABM_OK;
    hipGraph_t g;
    // the caller's stream may be the legacy default stream, which cannot be
    // captured: capture on a private stream, replay on the caller's
    if (!b->cap_stream) HIPCHK(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    b->d.resort_every = b->resort_every;
    bool resort = b->resort_every > 0;
    if (part == 0)
        launch_iteration(b->d, b->cap_stream, b->grid_agents, b->grid_boxes, b->sched, diag != 0, b->any_growth,
                         b->any_static, resort, b->any_death, b->any_record);
    else if (part == 1)
        launch_sweep(b->d, b->cap_stream, b->sched, diag != 0, b->any_static);
    else
        launch_after_sweep(b->d, b->cap_stream, b->grid_agents, b->grid_boxes, diag != 0, b->any_growth, b->any_static,
                           resort, b->any_death, b->any_record);
    hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (e != hipSuccess) return fail(ABM_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&b->exec[part][diag], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);  // the instantiated graph no longer needs its template
    if (e != hipSuccess) return fail(ABM_ERR_HIP, "graph instantiate failed: %s", hipGetErrorString(e));
    return ABM_OK;
}

static bool params_ok(const abm_params &p) {
    if (!(p.dt > 0.0) || !(p.mass > 0.0) || !(p.max_disp > 0.0) || !(p.adherence >= 0.0)) return false;
    if (!isfinite(p.k) || !isfinite(p.gamma) || !(p.box_len >= 0.0) || !(p.div_vol >= 0.0)) return false;
    if (!(p.shift_frac >= 0.0) || !isfinite(p.shift_frac)) return false;
    // Algorithm 2 cell behaviour
    if (!(p.brownian_rate >= 0.0) || !isfinite(p.brownian_rate)) return false;
    if (!(p.death_prob >= 0.0 && p.death_prob <= 1.0) || p.min_age < 0) return false;
    if (p.div_vol > 0.0 && !(p.division_prob > 0.0 && p.division_prob <= 1.0)) return false;
    if (p.detect_static && p.brownian_rate > 0.0) return false;  // every agent moves: none can be static
    return true;
}

extern "C" size_t abm_batch_workspace_bytes(int n_sims, const int64_t *capacity, const int64_t *box_capacity) {
    if (!capacity || !box_capacity) return 0;
    Layout L;
    int64_t A, B, SB, T, BT;
    if (!make_layout(n_sims, capacity, box_capacity, L, A, B, SB, T, BT)) return 0;
    return L.total;
}

extern "C" int abm_batch_create(int n_sims, const abm_params *per_sim, const int64_t *n0, const double *xyz,
                                const double *diam, const double *vol, const double *growth, const uint64_t *uid,
                                int inputs_on_device, const int64_t *capacity, const int64_t *box_capacity,
                                void *workspace, size_t ws_bytes, void *hip_stream, abm_batch **out) {
    g_err.clear();
    if (!out || !per_sim || !n0 || !capacity || !box_capacity || !workspace) return fail(ABM_ERR_ARG, "null argument");
    *out = nullptr;
    Layout L;
    int64_t A, B, SB, T, BT;
    if (!make_layout(n_sims, capacity, box_capacity, L, A, B, SB, T, BT))
        return fail(ABM_ERR_ARG, "invalid simulation count or capacities");
    if (ws_bytes < L.total) return fail(ABM_ERR_ARG, "workspace too small: %zu < %zu", ws_bytes, L.total);
    int64_t ntot = 0;
    for (int s = 0; s < n_sims; ++s) {
        if (n0[s] < 0 || n0[s] > capacity[s]) return fail(ABM_ERR_ARG, "sim %d: n0 %lld outside [0, capacity]", s, (long long)n0[s]);
        if (!params_ok(per_sim[s])) return fail(ABM_ERR_ARG, "sim %d: invalid parameters", s);
        ntot += n0[s];
    }
    if (ntot > 0 && (!xyz || !diam)) return fail(ABM_ERR_ARG, "positions and diameters are required");
    if (!inputs_on_device) {
        for (int64_t q = 0; q < 3 * ntot; ++q)
            if (!isfinite(xyz[q])) return fail(ABM_ERR_NONFINITE, "non-finite position at %lld", (long long)(q / 3));
        for (int64_t q = 0; q < ntot; ++q)
            if (!(diam[q] > 0.0) || !isfinite(diam[q])) return fail(ABM_ERR_ARG, "invalid diameter at %lld", (long long)q);
    }

    abm_batch *b = new abm_batch();
    b->n_sims = n_sims;
    b->L = L;
    b->ws = (char *)(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
    b->ws_bytes = ws_bytes;
    b->stream = (hipStream_t)hip_stream;
    b->A = A;
    b->T = T;
    b->BT = BT;
    char *w = b->ws;
    Dev &d = b->d;
    d.n_sims = n_sims;
    d.sims = (SimDesc *)(w + L.sims);
    d.ctl = (Ctl *)(w + L.ctl);
    d.tile_begin = (int64_t *)(w + L.tile_begin);
    d.btile_begin = (int64_t *)(w + L.btile_begin);
    d.utile_begin = (int64_t *)(w + L.utile_begin);
    d.a_begin = (int64_t *)(w + L.a_begin);
    d.wblk_begin = (int64_t *)(w + L.wblk_begin);
    d.mv_begin = (int64_t *)(w + L.mv_begin);
    d.bnd = (unsigned long long *)(w + L.bnd);
    for (int k = 0; k < 2; ++k) {
        d.pos[k] = (double *)(w + L.pos[k]);
        d.diam[k] = (double *)(w + L.diam[k]);
        d.vol[k] = (double *)(w + L.vol[k]);
        d.growth[k] = (double *)(w + L.growth[k]);
        d.uid[k] = (uint64_t *)(w + L.uid[k]);
        d.flags[k] = (uint8_t *)(w + L.flags[k]);
        d.nz[k] = (uint8_t *)(w + L.nz[k]);
        d.birth[k] = (int32_t *)(w + L.birth[k]);
    }
    d.stage8 = (uint8_t *)(w + L.stage8);
    d.key = (uint32_t *)(w + L.key);
    d.rank = (uint32_t *)(w + L.rank);
    d.payload = (Pay *)(w + L.payload);
    d.sorted_idx = (uint32_t *)(w + L.sorted_idx);
    d.nbr = (int32_t *)(w + L.nbr);
    d.contacts = (int32_t *)(w + L.contacts);
    d.force = (double *)(w + L.force);
    d.disp = (double *)(w + L.disp);
    d.boxid = (int64_t *)(w + L.boxid);
    d.count = (uint32_t *)(w + L.count);
    d.box_start = (uint32_t *)(w + L.box_start);
    d.brank = (uint32_t *)(w + L.brank);
    d.blist = (uint32_t *)(w + L.blist);
    d.dirty = (uint8_t *)(w + L.dirty);
    d.arrive = (uint8_t *)(w + L.arrive);
    d.dirty_blk = (uint8_t *)(w + L.dirty_blk);
    d.arrive_blk = (uint8_t *)(w + L.arrive_blk);
    d.active_blk = (uint8_t *)(w + L.active_blk);
    d.near_blk = (uint8_t *)(w + L.near_blk);
    d.tile_sum = (uint32_t *)(w + L.tile_sum);
    d.tile_off = (uint32_t *)(w + L.tile_off);
    d.rm_sum = (uint32_t *)(w + L.rm_sum);
    d.rm_off = (uint32_t *)(w + L.rm_off);
    d.fix_list = (uint32_t *)(w + L.fix_list);
    d.dense_list = (uint64_t *)(w + L.dense_list);
    d.dense_cap = dense_capacity(A, B);
    d.divflag = (uint32_t *)(w + L.divflag);
    d.divrank = (uint32_t *)(w + L.divrank);
    d.stat_part = (double *)(w + L.stat_part);
    d.hist_cnt = (unsigned int *)(w + L.hist_cnt);
    d.A = A;

    hipStream_t st = b->stream;
    auto cleanup = [&](int rc) { delete b; return rc; };
#define HIPCHK_C(expr)                                                                          \
    do {                                                                                        \
        hipError_t _e = (expr);                                                                 \
        if (_e != hipSuccess) return cleanup(fail(ABM_ERR_HIP, "%s: %s", #expr, hipGetErrorString(_e))); \
    } while (0)

    // zero what must start at zero (outside any graph)
    HIPCHK_C(hipMemsetAsync(d.count, 0, sizeof(uint32_t) * B, st));
    HIPCHK_C(hipMemsetAsync(d.dirty, 0, B, st));
    HIPCHK_C(hipMemsetAsync(d.divflag, 0, sizeof(uint32_t) * A, st));
    HIPCHK_C(hipMemsetAsync(d.flags[0], 0, A, st));
    HIPCHK_C(hipMemsetAsync(d.flags[1], 0, A, st));
    HIPCHK_C(hipMemsetAsync(d.birth[0], 0, sizeof(int32_t) * A, st));  // age 0 at iteration 0
    HIPCHK_C(hipMemsetAsync(d.birth[1], 0, sizeof(int32_t) * A, st));
    HIPCHK_C(hipMemsetAsync(d.nz[0], 0, A, st));
    HIPCHK_C(hipMemsetAsync(d.arrive, 0, B, st));
    HIPCHK_C(hipMemsetAsync(d.dirty_blk, 0, B, st));
    HIPCHK_C(hipMemsetAsync(d.arrive_blk, 0, B, st));
    HIPCHK_C(hipMemsetAsync(d.active_blk, 0, B, st));
    HIPCHK_C(hipMemsetAsync(d.growth[0], 0, sizeof(double) * A, st));
    HIPCHK_C(hipMemsetAsync(d.hist_cnt, 0, sizeof(unsigned) * 32 * n_sims, st));

    // simulation descriptors
    b->host_sims.assign(n_sims, SimDesc{});
    std::vector<int64_t> a_begin(n_sims + 1);
    int64_t aoff = 0, boff = 0, sboff = 0, in_off = 0;
    b->any_growth = false;
    b->any_static = false;
    b->any_death = false;
    b->any_record = false;
    for (int s = 0; s < n_sims; ++s) {
        SimDesc &S = b->host_sims[s];
        memset(&S, 0, sizeof S);
        const abm_params &p = per_sim[s];
        S.a_off = aoff;
        S.cap = capacity[s];
        S.b_off = boff;
        S.box_cap = box_capacity[s];
        S.sb_off = sboff;
        S.dt = p.dt; S.k = p.k; S.gamma = p.gamma; S.adherence = p.adherence; S.mass = p.mass;
        S.max_disp = p.max_disp; S.box_len = p.box_len; S.div_vol = p.div_vol; S.shift_frac = p.shift_frac;
        S.detect_static = p.detect_static ? 1 : 0;
        S.resort_every = p.resort_every;
        S.seed = p.seed;
        S.sim_id = p.sim_id;
        S.flags = p.flags;
        S.brownian_rate = p.brownian_rate;
        S.death_prob = p.death_prob;
        S.division_prob = p.division_prob;
        S.min_age = p.min_age;
        S.n = n0[s];
        S.n_start = n0[s];
        S.next_uid = n0[s];
        a_begin[s] = aoff;
        b->any_growth |= p.div_vol > 0.0;
        b->any_death |= p.death_prob > 0.0;
        b->any_record |= (p.flags & ABM_RECORD) != 0;
        b->any_static |= p.detect_static != 0;
        // inputs
        if (n0[s] > 0) {
            const double *src = xyz + 3 * in_off;
            if (!inputs_on_device) {
                // stage on the device in the force buffer (scratch until a diagnostic step)
                HIPCHK_C(hipMemcpyAsync(d.force, src, sizeof(double) * 3 * n0[s], hipMemcpyHostToDevice, st));
                src = d.force;
            }
            hipLaunchKernelGGL(k_load_pos, dim3(grid_for(n0[s])), dim3(256), 0, st, d.pos[0], d.pos[1], A, aoff, n0[s], src);
            hipMemcpyKind kind = inputs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
            HIPCHK_C(hipMemcpyAsync(d.diam[0] + aoff, diam + in_off, sizeof(double) * n0[s], kind, st));
            if (vol) HIPCHK_C(hipMemcpyAsync(d.vol[0] + aoff, vol + in_off, sizeof(double) * n0[s], kind, st));
            else hipLaunchKernelGGL(k_vol_from_diam, dim3(grid_for(n0[s])), dim3(256), 0, st, d.vol[0], d.diam[0], aoff, n0[s]);
            if (growth) HIPCHK_C(hipMemcpyAsync(d.growth[0] + aoff, growth + in_off, sizeof(double) * n0[s], kind, st));
            if (uid) HIPCHK_C(hipMemcpyAsync(d.uid[0] + aoff, uid + in_off, sizeof(uint64_t) * n0[s], kind, st));
            else hipLaunchKernelGGL(k_iota_uid, dim3(grid_for(n0[s])), dim3(256), 0, st, d.uid[0], aoff, n0[s]);
            HIPCHK_C(hipStreamSynchronize(st));  // the staging buffer is reused by the next simulation
        }
        aoff += capacity[s];
        boff += box_capacity[s];
        sboff += box_capacity[s] + 1;
        in_off += n0[s];
    }
    a_begin[n_sims] = aoff;
    b->resort_every = per_sim[0].resort_every > 0 ? per_sim[0].resort_every : 0;

    // next uid = max uid + 1 (uids must stay below the capacity: they index per-simulation tables)
    if (uid) {
        unsigned long long *tmp = (unsigned long long *)d.tile_sum;
        for (int s = 0; s < n_sims; ++s) {
            if (n0[s] == 0) continue;
            HIPCHK_C(hipMemsetAsync(tmp, 0, sizeof(unsigned long long), st));
            hipLaunchKernelGGL(k_max_uid, dim3(grid_for(n0[s])), dim3(256), 0, st, d.uid[0], b->host_sims[s].a_off, n0[s], tmp);
            unsigned long long mu = 0;
            HIPCHK_C(hipMemcpyAsync(&mu, tmp, sizeof mu, hipMemcpyDeviceToHost, st));
            HIPCHK_C(hipStreamSynchronize(st));
            if ((int64_t)mu > capacity[s]) return cleanup(fail(ABM_ERR_ARG, "sim %d: uids must be below the capacity", s));
            b->host_sims[s].next_uid = (int64_t)mu;
        }
    }
    HIPCHK_C(hipMemcpyAsync(d.sims, b->host_sims.data(), sizeof(SimDesc) * n_sims, hipMemcpyHostToDevice, st));
    HIPCHK_C(hipMemcpyAsync(d.a_begin, a_begin.data(), sizeof(int64_t) * (n_sims + 1), hipMemcpyHostToDevice, st));
    Ctl c;
    memset(&c, 0, sizeof c);
    c.any_growth = b->any_growth;
    HIPCHK_C(hipMemcpyAsync(d.ctl, &c, sizeof c, hipMemcpyHostToDevice, st));
    launch_scatter_init(d, st, 1);
    HIPCHK_C(hipStreamSynchronize(st));
    HIPCHK_C(hipGetLastError());
    int64_t tiles_cap = T;
    b->grid_agents = (int)std::min<int64_t>(std::max<int64_t>(tiles_cap, 1), 8192);
    b->grid_boxes = (int)std::min<int64_t>(std::max<int64_t>(BT, 1), 4096);
    *out = b;
#undef HIPCHK_C
    return ABM_OK;
}

static int read_ctl(abm_batch *b, Ctl &c) {
    HIPCHK(hipMemcpyAsync(&c, b->d.ctl, sizeof c, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    return ABM_OK;
}

static int read_sims(abm_batch *b, std::vector<SimDesc> &v) {
    v.resize(b->n_sims);
    HIPCHK(hipMemcpyAsync(v.data(), b->d.sims, sizeof(SimDesc) * b->n_sims, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    return ABM_OK;
}

extern "C" int abm_batch_restore(abm_batch *b, const uint8_t *is_static, const int32_t *nz, const int32_t *age,
                                 const uint64_t *next_uid, int64_t iteration, int on_device) {
    g_err.clear();
    if (!b) return fail(ABM_ERR_ARG, "null handle");
    // the arrays are in creation order: only the untouched state of a new
    // handle is in that order (a step, the tuner or a restore re-sorts or
    // changes it)
    if (!b->fresh) return fail(ABM_ERR_ARG, "restore must directly follow abm_batch_create");
    if (iteration < 0 || iteration > INT32_MAX) return fail(ABM_ERR_ARG, "iteration outside 0..2^31-1");
    std::vector<SimDesc> sims;
    int rc = read_sims(b, sims);
    if (rc) return rc;
    hipStream_t st = b->stream;
    if (age && !on_device) {
        int64_t tot = 0;
        for (int s = 0; s < b->n_sims; ++s) tot += sims[s].n;
        for (int64_t q = 0; q < tot; ++q)
            if (age[q] < 0 || age[q] > iteration + (int64_t)INT32_MAX) return fail(ABM_ERR_ARG, "negative age");
    }
    int64_t in_off = 0;
    for (int s = 0; s < b->n_sims; ++s) {
        int64_t n = sims[s].n;
        if (n > 0) {
            if (is_static) {
                const uint8_t *src = is_static + in_off;
                if (!on_device) {
                    HIPCHK(hipMemcpyAsync(b->d.stage8, src, n, hipMemcpyHostToDevice, st));
                    src = b->d.stage8;
                }
                hipLaunchKernelGGL(k_u8_from_host_layout, dim3(grid_for(n)), dim3(256), 0, st, b->d.flags[0], src, sims[s].a_off, n);
            }
            if (nz) {
                const int32_t *src = nz + in_off;
                if (!on_device) {
                    HIPCHK(hipMemcpyAsync(b->d.nbr, src, sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
                    src = b->d.nbr;
                }
                hipLaunchKernelGGL(k_nz_from_i32, dim3(grid_for(n)), dim3(256), 0, st, b->d.nz[0], src, sims[s].a_off, n);
            }
            {  // birth iteration = iteration - age (age 0 without ages)
                const int32_t *src = age ? age + in_off : nullptr;
                if (src && !on_device) {
                    HIPCHK(hipMemcpyAsync(b->d.contacts, src, sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
                    src = b->d.contacts;
                }
                hipLaunchKernelGGL(k_birth_from_age, dim3(grid_for(n)), dim3(256), 0, st, b->d.birth[0], src,
                                   sims[s].a_off, n, iteration);
            }
            HIPCHK(hipStreamSynchronize(st));
        }
        if (next_uid) {
            uint64_t nu;
            if (on_device) {
                HIPCHK(hipMemcpyAsync(&nu, next_uid + s, sizeof nu, hipMemcpyDeviceToHost, st));
                HIPCHK(hipStreamSynchronize(st));
            } else {
                nu = next_uid[s];
            }
            if ((int64_t)nu > sims[s].cap) return fail(ABM_ERR_ARG, "next_uid above capacity");
            sims[s].next_uid = (int64_t)nu;
        }
        in_off += n;
    }
    HIPCHK(hipMemsetAsync(b->d.stage8, 0, b->A, st));
    HIPCHK(hipMemcpyAsync(b->d.sims, sims.data(), sizeof(SimDesc) * b->n_sims, hipMemcpyHostToDevice, st));
    Ctl c;
    rc = read_ctl(b, c);
    if (rc) return rc;
    c.iter = iteration;
    HIPCHK(hipMemcpyAsync(b->d.ctl, &c, sizeof c, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    b->fresh = false;
    return ABM_OK;
}

static int status_from_ctl(abm_batch *b, const Ctl &c) {
    if (c.err & kErrNonfinite) return fail(ABM_ERR_NONFINITE, "non-finite position or diameter");
    if (c.err & kErrCapacity) return fail(ABM_ERR_CAPACITY, "divisions would exceed the agent capacity");
    if (c.err & kErrGrid) return fail(ABM_ERR_CAPACITY, "grid exceeds the box capacity or 2048x2048x1024 boxes");
    return ABM_OK;
}

static int clear_abort(abm_batch *b) {
    // the state is that of the last completed iteration; clear the flags so the
    // handle stays usable (queries, restore, smaller steps)
    Ctl c;
    int rc = read_ctl(b, c);
    if (rc) return rc;
    c.abort = 0;
    c.err = 0;
    std::vector<SimDesc> sims;
    rc = read_sims(b, sims);
    if (rc) return rc;
    for (auto &S : sims) {
        S.err = 0;
        S.n_div = 0;
        S.n_start = S.n;
    }
    HIPCHK(hipMemcpyAsync(b->d.sims, sims.data(), sizeof(SimDesc) * b->n_sims, hipMemcpyHostToDevice, b->stream));
    HIPCHK(hipMemcpyAsync(b->d.ctl, &c, sizeof c, hipMemcpyHostToDevice, b->stream));
    // stale divider flags and dirty marks of the aborted iteration
    HIPCHK(hipMemsetAsync(b->d.divflag, 0, sizeof(uint32_t) * b->A, b->stream));
    int64_t B = 0;
    for (auto &S : sims) B += S.box_cap;
    HIPCHK(hipMemsetAsync(b->d.dirty, 0, B, b->stream));
    HIPCHK(hipMemsetAsync(b->d.arrive, 0, B, b->stream));
    HIPCHK(hipMemsetAsync(b->d.dirty_blk, 0, B, b->stream));
    HIPCHK(hipMemsetAsync(b->d.arrive_blk, 0, B, b->stream));
    HIPCHK(hipMemsetAsync(b->d.active_blk, 0, B, b->stream));
    HIPCHK(hipMemsetAsync(b->d.count, 0, sizeof(uint32_t) * B, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    return ABM_OK;
}

static bool any_diag(const abm_batch *b) {
    for (auto &S : b->host_sims)
        if (S.flags & ABM_DIAG) return true;
    return false;
}

// Every iteration ends by building the grid of its result, and the iteration
// graph relies on it.  The first step (and a step after an error) builds it
// first, and puts agents into Morton order when re-sorting is on; so does the
// tuner before it replays iterations.
static int ensure_grid(abm_batch *b) {
    b->fresh = false;
    if (b->grid_valid) return ABM_OK;
    b->d.resort_every = b->resort_every;
    launch_grid_build(b->d, b->stream, b->grid_agents, b->grid_boxes, b->any_static);
    if (b->resort_every > 0) {
        launch_resort(b->d, b->stream, b->grid_agents, b->grid_boxes, true, b->any_static);
        launch_grid_build(b->d, b->stream, b->grid_agents, b->grid_boxes, b->any_static);
    }
    HIPCHK(hipGetLastError());
    b->grid_valid = true;
    return ABM_OK;
}

extern "C" int abm_batch_step(abm_batch *b, int n_iter) {
    g_err.clear();
    if (!b || n_iter < 0) return fail(ABM_ERR_ARG, "bad handle or iteration count");
    if (n_iter == 0) return ABM_OK;
    int diag = any_diag(b) ? 1 : 0;
    int rc = b->timing ? capture(b, 1, diag) : capture(b, 0, diag);
    if (!rc && b->timing) rc = capture(b, 2, diag);
    if (rc) return rc;
    rc = ensure_grid(b);
    if (rc) return rc;
    if (b->timing) {
        while ((int)b->ev.size() < 2 * n_iter) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            b->ev.push_back(e);
        }
        for (int it = 0; it < n_iter; ++it) {
            HIPCHK(hipEventRecord(b->ev[2 * it], b->stream));
            HIPCHK(hipGraphLaunch(b->exec[1][diag], b->stream));
            HIPCHK(hipEventRecord(b->ev[2 * it + 1], b->stream));
            HIPCHK(hipGraphLaunch(b->exec[2][diag], b->stream));
        }
    } else {
        for (int it = 0; it < n_iter; ++it) HIPCHK(hipGraphLaunch(b->exec[0][diag], b->stream));
    }
    Ctl c;
    rc = read_ctl(b, c);
    if (rc) return rc;
    if (b->timing) {
        for (int it = 0; it < n_iter; ++it) {
            float ms = 0.0f;
            HIPCHK(hipEventElapsedTime(&ms, b->ev[2 * it], b->ev[2 * it + 1]));
            b->sweep_ms += ms;
        }
        b->n_sweeps += n_iter;
    }
    HIPCHK(hipGetLastError());
    if (c.abort || c.err) {
        b->grid_valid = false;
        int st = status_from_ctl(b, c);
        std::string msg = g_err;
        int rc2 = clear_abort(b);
        if (rc2) return rc2;
        g_err = msg;
        return st ? st : fail(ABM_ERR_HIP, "iteration aborted");
    }
    return ABM_OK;
}

extern "C" int abm_batch_num_agents(abm_batch *b, int64_t *n_out) {
    g_err.clear();
    if (!b || !n_out) return fail(ABM_ERR_ARG, "null argument");
    std::vector<SimDesc> sims;
    int rc = read_sims(b, sims);
    if (rc) return rc;
    for (int s = 0; s < b->n_sims; ++s) n_out[s] = sims[s].n;
    return ABM_OK;
}

extern "C" int abm_batch_fp64_agents(abm_batch *b, int64_t *n_out) {
    g_err.clear();
    if (!b || !n_out) return fail(ABM_ERR_ARG, "null argument");
    Ctl c;
    int rc = read_ctl(b, c);
    if (rc) return rc;
    *n_out = c.n_fp64_last;
    return ABM_OK;
}

extern "C" int abm_batch_grid(abm_batch *b, int sim, double lo[3], double *L, int64_t dims[3]) {
    g_err.clear();
    if (!b || sim < 0 || sim >= b->n_sims) return fail(ABM_ERR_ARG, "bad handle or simulation");
    std::vector<SimDesc> sims;
    int rc = read_sims(b, sims);
    if (rc) return rc;
    for (int a = 0; a < 3; ++a) {
        if (lo) lo[a] = sims[sim].lo[a];
        if (dims) dims[a] = sims[sim].dims[a];
    }
    if (L) *L = sims[sim].L;
    return ABM_OK;
}

extern "C" int abm_batch_query(abm_batch *b, int sim, int field, void *dst, int dst_on_device, int64_t cap,
                               int64_t *n_out) {
    g_err.clear();
    if (!b || sim < 0 || sim >= b->n_sims || !dst) return fail(ABM_ERR_ARG, "bad handle, simulation or destination");
    std::vector<SimDesc> sims;
    int rc = read_sims(b, sims);
    if (rc) return rc;
    Ctl c;
    rc = read_ctl(b, c);
    if (rc) return rc;
    const SimDesc &S = sims[sim];
    int64_t n = S.n;
    if (n_out) *n_out = n;
    if (n > cap) return fail(ABM_ERR_ARG, "destination holds %lld agents, need %lld", (long long)cap, (long long)n);
    if (n == 0) return ABM_OK;
    hipStream_t st = b->stream;
    const int lp = c.lay_par, P = c.pos_par;
    const int64_t a = S.a_off, A = b->A;
    hipMemcpyKind kind = dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    auto copy = [&](const void *src, size_t bytes) -> int {
        HIPCHK(hipMemcpyAsync(dst, src, bytes, kind, st));
        HIPCHK(hipStreamSynchronize(st));
        return ABM_OK;
    };
    switch (field) {
    case ABM_POS: {
        if (dst_on_device) {
            launch_gather_pos(b->d, st, sim, (double *)dst, n, a);
            HIPCHK(hipStreamSynchronize(st));
            return ABM_OK;
        }
        std::vector<double> tmp(3 * n);
        for (int k = 0; k < 3; ++k)
            HIPCHK(hipMemcpyAsync(tmp.data() + k * n, b->d.pos[P] + k * A + a, sizeof(double) * n, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        double *o = (double *)dst;
        for (int64_t q = 0; q < n; ++q)
            for (int k = 0; k < 3; ++k) o[3 * q + k] = tmp[k * n + q];
        return ABM_OK;
    }
    case ABM_DIAM: return copy(b->d.diam[lp] + a, sizeof(double) * n);
    case ABM_VOL: return copy(b->d.vol[lp] + a, sizeof(double) * n);
    case ABM_GROWTH: return copy(b->d.growth[lp] + a, sizeof(double) * n);
    case ABM_UID: return copy(b->d.uid[lp] + a, sizeof(uint64_t) * n);
    case ABM_STATIC: {
        // the per-iteration change bytes are free between steps: use them as staging
        hipLaunchKernelGGL(k_static_u8, dim3(grid_for(n)), dim3(256), 0, st, b->d.stage8, b->d.flags[lp] + a, n);
        return copy(b->d.stage8, n);
    }
    case ABM_NZ: {
        int32_t *tmp = (int32_t *)b->d.fix_list;  // free between steps
        hipLaunchKernelGGL(k_widen_u8, dim3(grid_for(n)), dim3(256), 0, st, tmp, b->d.nz[lp] + a, n, 0);
        return copy(tmp, sizeof(int32_t) * n);
    }
    case ABM_AGE: {
        int32_t *tmp = (int32_t *)b->d.fix_list;  // free between steps
        hipLaunchKernelGGL(k_age, dim3(grid_for(n)), dim3(256), 0, st, tmp, b->d.birth[lp] + a, n, c.iter);
        return copy(tmp, sizeof(int32_t) * n);
    }
    case ABM_NBR_COUNT: return copy(b->d.nbr + a, sizeof(int32_t) * n);
    case ABM_CONTACT_COUNT: return copy(b->d.contacts + a, sizeof(int32_t) * n);
    case ABM_FORCE: return copy(b->d.force + 3 * a, sizeof(double) * 3 * n);
    case ABM_DISP: return copy(b->d.disp + 3 * a, sizeof(double) * 3 * n);
    case ABM_BOX: return copy(b->d.boxid + a, sizeof(int64_t) * n);
    default: return fail(ABM_ERR_ARG, "unknown field %d", field);
    }
}

extern "C" int abm_batch_stats(abm_batch *b, double hist_rmax, double *centroid, double *r_gyr, double *r_max,
                               float *hist) {
    g_err.clear();
    if (!b || !(hist_rmax > 0.0)) return fail(ABM_ERR_ARG, "bad handle or histogram radius");
    double *out = (double *)(b->ws + b->L.stat_out);
    launch_stats(b->d, b->stream, b->grid_agents, hist_rmax, out);
    HIPCHK(hipGetLastError());
    std::vector<double> h(40 * b->n_sims);
    std::vector<float> hh(32 * b->n_sims);
    HIPCHK(hipMemcpyAsync(h.data(), out, sizeof(double) * 40 * b->n_sims, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipMemcpyAsync(hh.data(), out + 40 * b->n_sims, sizeof(float) * 32 * b->n_sims, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    for (int s = 0; s < b->n_sims; ++s) {
        if (centroid)
            for (int a = 0; a < 3; ++a) centroid[3 * s + a] = h[40 * s + a];
        if (r_gyr) r_gyr[s] = h[40 * s + 4];
        if (r_max) r_max[s] = h[40 * s + 5];
        if (hist)
            for (int q = 0; q < 32; ++q) hist[32 * s + q] = hh[32 * s + q];
    }
    return ABM_OK;
}

extern "C" int abm_batch_hist(abm_batch *b, double hist_rmax, float *out, int out_on_device) {
    g_err.clear();
    if (!b || !out || !(hist_rmax > 0.0)) return fail(ABM_ERR_ARG, "bad arguments");
    double *so = (double *)(b->ws + b->L.stat_out);
    launch_stats(b->d, b->stream, b->grid_agents, hist_rmax, so);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(out, so + 40 * b->n_sims, sizeof(float) * 32 * b->n_sims,
                          out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    return ABM_OK;
}

extern "C" int abm_batch_set_sweep_grid(abm_batch *b, int workgroups) {
    g_err.clear();
    if (!b || workgroups < 8 || workgroups > 65536 || workgroups % 8)
        return fail(ABM_ERR_ARG, "workgroups must be a multiple of 8 in [8, 65536]");
    if (workgroups != b->sched.sweep_grid) {
        b->sched.sweep_grid = workgroups;
        destroy_graphs(b);
    }
    return ABM_OK;
}

// One trial of the tuner: from the snapshot, the current schedule replays
// one warm-up iteration and then `iters` timed iterations.  Returns the
// milliseconds, or a negative value when the trial aborted (a capacity error:
// the schedule is then not taken).
static int tune_trial(abm_batch *b, void *snap, size_t bytes, int iters, hipEvent_t e0, hipEvent_t e1, float *ms) {
    hipStream_t st = b->stream;
    destroy_graphs(b);
    int rc = capture(b, 0, 0);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(b->ws, snap, bytes, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipGraphLaunch(b->exec[0][0], st));  // warm-up
    HIPCHK(hipEventRecord(e0, st));
    for (int it = 0; it < iters; ++it) HIPCHK(hipGraphLaunch(b->exec[0][0], st));
    HIPCHK(hipEventRecord(e1, st));
    HIPCHK(hipEventSynchronize(e1));
    HIPCHK(hipEventElapsedTime(ms, e0, e1));
    Ctl c;
    rc = read_ctl(b, c);
    if (rc) return rc;
    if (c.abort) *ms = -1.0f;
    return ABM_OK;
}

extern "C" int abm_batch_tune(abm_batch *b, int n_trial_iters, int *grid_out) {
    g_err.clear();
    if (!b || n_trial_iters < 1) return fail(ABM_ERR_ARG, "bad arguments");
    int rc = ensure_grid(b);  // the trials replay iterations, which need the grid
    if (rc) return rc;
    // snapshot of the whole workspace so that trials leave the batch unchanged
    void *snap = nullptr;
    size_t bytes = b->L.total - 256;
    HIPCHK(hipMalloc(&snap, bytes));
    hipStream_t st = b->stream;
    hipError_t e = hipMemcpyAsync(snap, b->ws, bytes, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) {
        (void)hipFree(snap);
        return fail(ABM_ERR_HIP, "snapshot copy failed: %s", hipGetErrorString(e));
    }
    bool tune_resort = false;
    for (auto &S : b->host_sims) tune_resort |= S.resort_every < 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess)
        rc = fail(ABM_ERR_HIP, "event creation failed: %s", hipGetErrorString(e));
    Sched best = b->sched;
    int best_resort = b->resort_every;
    // stage 1: persistent work groups of the unit sweep
    float best_ms = 1e30f;
    const int grids[4] = {512, 1024, 2048, 4096};
    for (int k = 0; k < 4 && rc == ABM_OK; ++k) {
        b->sched = best;
        b->sched.sweep_grid = grids[k];
        float ms;
        if ((rc = tune_trial(b, snap, bytes, n_trial_iters, e0, e1, &ms))) break;
        if (ms >= 0.0f && ms < best_ms) best_ms = ms, best.sweep_grid = grids[k];
    }
    // stage 2: work groups and waves per work group of the box-wise sweep
    const int dense[6][2] = {{512, 4}, {1024, 4}, {2048, 4}, {1024, 2}, {2048, 2}, {4096, 2}};
    best_ms = 1e30f;
    Sched base = best;
    for (int k = 0; k < 6 && rc == ABM_OK; ++k) {
        b->sched = base;
        b->sched.dense_grid = dense[k][0];
        b->sched.dense_waves = dense[k][1];
        float ms;
        if ((rc = tune_trial(b, snap, bytes, n_trial_iters, e0, e1, &ms))) break;
        if (ms >= 0.0f && ms < best_ms) best_ms = ms, best.dense_grid = dense[k][0], best.dense_waves = dense[k][1];
    }
    // stage 3 (on request): the Morton re-sort period, each candidate timed
    // over 20 iterations so that its re-sorts are part of the time
    if (tune_resort) {
        const int resorts[3] = {5, 10, 20};
        best_ms = 1e30f;
        b->sched = best;
        for (int k = 0; k < 3 && rc == ABM_OK; ++k) {
            b->resort_every = resorts[k];
            float ms;
            if ((rc = tune_trial(b, snap, bytes, n_trial_iters > 20 ? n_trial_iters : 20, e0, e1, &ms))) break;
            if (ms >= 0.0f && ms < best_ms) best_ms = ms, best_resort = resorts[k];
        }
    }
    // restore the batch as it was before the trials
    if ((e = hipMemcpyAsync(b->ws, snap, bytes, hipMemcpyDeviceToDevice, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess) {
        if (rc == ABM_OK) rc = fail(ABM_ERR_HIP, "autotuner: restoring the batch failed: %s", hipGetErrorString(e));
    }
    (void)hipFree(snap);  // teardown: nothing to recover
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    b->sched = best;
    b->resort_every = best_resort;
    destroy_graphs(b);
    if (rc) return rc;
    if (grid_out) *grid_out = best.sweep_grid;
    return ABM_OK;
}

extern "C" int abm_batch_schedule(abm_batch *b, int *sweep_grid, int *dense_grid, int *dense_waves, int *resort_every) {
    g_err.clear();
    if (!b) return fail(ABM_ERR_ARG, "null handle");
    if (sweep_grid) *sweep_grid = b->sched.sweep_grid;
    if (dense_grid) *dense_grid = b->sched.dense_grid;
    if (dense_waves) *dense_waves = b->sched.dense_waves;
    if (resort_every) *resort_every = b->resort_every;
    return ABM_OK;
}

extern "C" int abm_batch_set_timing(abm_batch *b, int on) {
    g_err.clear();
    if (!b) return fail(ABM_ERR_ARG, "null handle");
    b->timing = on != 0;
    return ABM_OK;
}

extern "C" int abm_batch_sweep_time(abm_batch *b, double *ms_total, int64_t *n_sweeps) {
    g_err.clear();
    if (!b) return fail(ABM_ERR_ARG, "null handle");
    if (ms_total) *ms_total = b->sweep_ms;
    if (n_sweeps) *n_sweeps = b->n_sweeps;
    b->sweep_ms = 0.0;
    b->n_sweeps = 0;
    return ABM_OK;
}

extern "C" int abm_batch_destroy(abm_batch *b) {
    g_err.clear();
    if (!b) return ABM_OK;
    destroy_graphs(b);
    for (hipEvent_t e : b->ev) (void)hipEventDestroy(e);  // teardown: nothing to recover
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    delete b;
    return ABM_OK;
}

// ---------------------------------------------------------------- single population
extern "C" size_t abm_pop_workspace_bytes(const abm_params *p, int64_t capacity, int64_t box_capacity) {
    (void)p;
    return abm_batch_workspace_bytes(1, &capacity, &box_capacity);
}

extern "C" int abm_pop_create(const abm_params *p, int64_t n, const double *xyz, const double *diam, const double *vol,
                              const double *growth, const uint64_t *uid, int inputs_on_device, void *workspace,
                              size_t ws_bytes, int64_t capacity, int64_t box_capacity, void *hip_stream, abm_pop **out) {
    return abm_batch_create(1, p, &n, xyz, diam, vol, growth, uid, inputs_on_device, &capacity, &box_capacity,
                            workspace, ws_bytes, hip_stream, out);
}

extern "C" int abm_pop_step(abm_pop *p, int n_iter) { return abm_batch_step(p, n_iter); }

extern "C" int abm_pop_num_agents(abm_pop *p, int64_t *n) { return abm_batch_num_agents(p, n); }

extern "C" int abm_pop_query(abm_pop *p, int field, void *dst, int dst_on_device, int64_t cap, int64_t *n_out) {
    return abm_batch_query(p, 0, field, dst, dst_on_device, cap, n_out);
}

extern "C" int abm_pop_stats(abm_pop *p, double hist_rmax, double centroid[3], double *r_gyr, double *r_max,
                             float hist[32]) {
    return abm_batch_stats(p, hist_rmax, centroid, r_gyr, r_max, hist);
}

extern "C" int abm_pop_destroy(abm_pop *p) { return abm_batch_destroy(p); }
