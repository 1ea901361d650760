// abm_soma.hip -- extracellular diffusion (Sec 4.5.2, Eq 4.3) with the
// secreting, chemotactic cells of the soma clustering model (Sec 4.7.1,
// Algorithms 6-7).
//
// One iteration (captured once into a HIP graph and replayed):
//   k_soma_cells    per cell: chemotaxis on the start-of-iteration
//                   concentrations (Algorithm 7), and the cell's voxel with
//                   its rank among the voxel's cells (one integer atomic)
//   k_soma_secrete  per cell of rank 0: its voxel gains the count of cells
//                   times the quantity in one addition (Algorithm 6); the
//                   count is cleared for the next iteration
//   k_diffuse       Eq 4.3 over every substance, from one buffer to the other
//   k_soma_end      buffer parity and iteration counter
// The stencil is bound by HBM: every point is read once from memory and
// written once (16 bytes).  A work group owns a 64 x 16 tile of (x, y) and
// marches along z over a chunk of planes, holding the planes z - 1, z and
// z + 1 of its points in registers (the z neighbours cost no memory
// traffic) and staging plane z with its one-point x and y halo in LDS.  The
// next plane's points and halo are loaded one plane ahead.  Tiles are dealt
// to the XCDs in contiguous ranges so the halos of neighbouring tiles meet
// in the same L2.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <vector>

#include "abm_device.h"

namespace abm {
namespace soma {

constexpr int kThreads = 256;
constexpr int kTX = 64, kTY = 16, kRows = kTY / 4;  // tile: 64 x 16 points, 4 rows per thread
constexpr int kZChunk = 16;                           // planes per work group
constexpr int kXcds = 8;
constexpr int64_t kMaxRes = 2048;
constexpr int kMaxSubstances = 16;

struct alignas(64) Ctl {
    int64_t iter;
    int32_t par;  // buffer holding the current concentrations
};

struct Dev {
    int64_t n, V;  // cells, points per substance
    int32_t R, nsub;
    double lo, S, hi, dx, keep, c, q, w;
    Ctl *ctl;
    double *u[2];      // nsub x V each
    uint32_t *cnt;     // nsub x V cell counts (zero between iterations)
    double *pos;       // cells: x block, y block, z block
    int32_t *type;
    int64_t *vox;      // substance * V + voxel of each cell
    uint32_t *rank;    // rank of the cell among the cells of its voxel
    int64_t *orig;     // creation index of the cell in each storage slot
    double *stage;     // 3 x n: queries in creation order
    int64_t tiles_x, tiles_y, tiles_z, tiles;  // stencil work groups per substance
};

__device__ inline int64_t voxel_axis(const Dev &d, double v) {
    double q = floor((v - d.lo) / d.dx);
    if (q < 0.0) return 0;
    if (q > (double)(d.R - 1)) return d.R - 1;
    return (int64_t)q;
}

// Concentration at (x, y, z), zero beyond the grid.
__device__ inline double at(const Dev &d, const double *u, int64_t x, int64_t y, int64_t z) {
    if (x < 0 || y < 0 || z < 0 || x >= d.R || y >= d.R || z >= d.R) return 0.0;
    return u[x + (int64_t)d.R * (y + (int64_t)d.R * z)];
}

__device__ inline double clamp_space(const Dev &d, double v) { return v < d.lo ? d.lo : (v > d.hi ? d.hi : v); }

// Algorithm 7 (chemotaxis) and the voxel and rank for Algorithm 6.
__global__ __launch_bounds__(kThreads) void k_soma_cells(Dev d) {
#pragma clang fp contract(off)
    const double *u = d.u[d.ctl->par];
    const int64_t n = d.n;
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const double x = d.pos[i], y = d.pos[n + i], z = d.pos[2 * n + i];
        const int64_t t = d.type[i];
        const int64_t a = voxel_axis(d, x), b = voxel_axis(d, y), c = voxel_axis(d, z);
        const double *us = u + t * d.V;
        const double g0 = (at(d, us, a + 1, b, c) - at(d, us, a - 1, b, c)) / (2.0 * d.dx);
        const double g1 = (at(d, us, a, b + 1, c) - at(d, us, a, b - 1, c)) / (2.0 * d.dx);
        const double g2 = (at(d, us, a, b, c + 1) - at(d, us, a, b, c - 1)) / (2.0 * d.dx);
        const double norm = sqrt(fma(g2, g2, fma(g1, g1, g0 * g0)));
        if (norm > 0.0) {
            d.pos[i] = clamp_space(d, x + (g0 / norm) * d.w);
            d.pos[n + i] = clamp_space(d, y + (g1 / norm) * d.w);
            d.pos[2 * n + i] = clamp_space(d, z + (g2 / norm) * d.w);
        }
        const int64_t v = t * d.V + a + (int64_t)d.R * (b + (int64_t)d.R * c);
        d.vox[i] = v;
        d.rank[i] = atomicAdd(&d.cnt[v], 1u);
    }
}

// Algorithm 6: one addition per occupied voxel, by the cell of rank 0.
__global__ __launch_bounds__(kThreads) void k_soma_secrete(Dev d) {
#pragma clang fp contract(off)
    double *u = d.u[d.ctl->par];
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < d.n; i += (int64_t)gridDim.x * kThreads) {
        if (d.rank[i] != 0) continue;
        const int64_t v = d.vox[i];
        const uint32_t k = d.cnt[v];
        u[v] = u[v] + (double)k * d.q;
        d.cnt[v] = 0u;
    }
}

// Cells back in creation order: interleaved positions or types.
__global__ void k_soma_unsort_pos(Dev d, double *dst) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < d.n; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = d.orig[j];
        dst[3 * i] = d.pos[j];
        dst[3 * i + 1] = d.pos[d.n + j];
        dst[3 * i + 2] = d.pos[2 * d.n + j];
    }
}
__global__ void k_soma_unsort_type(Dev d, int32_t *dst) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < d.n; j += (int64_t)gridDim.x * blockDim.x)
        dst[d.orig[j]] = d.type[j];
}

// Eq 4.3 on every substance (see the file comment for the tiling).
__global__ __launch_bounds__(kThreads, 6) void k_diffuse(Dev d) {
#pragma clang fp contract(off)
    __shared__ double pl[kTY + 2][kTX + 2];
    // tiles dealt to XCDs in contiguous ranges (work group b runs on XCD b mod 8)
    const int nt = (int)(d.tiles * d.nsub);
    const int per = (nt + kXcds - 1) / kXcds;
    const int t = (int)(blockIdx.x % kXcds) * per + (int)(blockIdx.x / kXcds);
    if (t >= nt) return;
    const int tiles = (int)d.tiles, txs = (int)d.tiles_x, tys = (int)d.tiles_y;
    const int sub = t / tiles;
    int r = t - sub * tiles;
    const int tx = r % txs;
    r /= txs;
    const int ty = r % tys;
    const int tz = r / tys;
    const int R = d.R;
    const int64_t plane = (int64_t)R * R;
    const int par = d.ctl->par;
    const double *__restrict__ src = d.u[par] + sub * d.V;
    double *__restrict__ dst = d.u[par ^ 1] + sub * d.V;
    const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;  // wave ly holds rows ly, ly + 4, ly + 8, ly + 12
    const int x = tx * kTX + lx;
    const int y0 = ty * kTY;
    const int z0 = tz * kZChunk;
    const int z1 = z0 + kZChunk < R ? z0 + kZChunk : R;
    // in-plane offsets of this thread's points, of its x halo (lanes 0 and 1)
    // and of its y halo (waves 0 and 3); -1: beyond the grid (zero)
    const int hxx = tx * kTX + (lx == 0 ? -1 : kTX);
    const int hyy = ly == 0 ? y0 - 1 : y0 + kTY;
    int off[kRows], hoff[kRows];
    for (int k = 0; k < kRows; ++k) {
        const int y = y0 + ly + 4 * k;
        off[k] = (x < R && y < R) ? y * R + x : -1;
        hoff[k] = (lx < 2 && hxx >= 0 && hxx < R && y < R) ? y * R + hxx : -1;
    }
    const int yoff = ((ly == 0 || ly == 3) && hyy >= 0 && hyy < R && x < R) ? hyy * R + x : -1;
    auto ld = [&](int o, int z) -> double {
        return (o >= 0 && z >= 0 && z < R) ? src[(int64_t)z * plane + o] : 0.0;
    };
    double zm[kRows], zc[kRows], zp[kRows], hx[kRows];
    for (int k = 0; k < kRows; ++k) {
        zm[k] = ld(off[k], z0 - 1);
        zc[k] = ld(off[k], z0);
        zp[k] = ld(off[k], z0 + 1);
        hx[k] = ld(hoff[k], z0);
    }
    double hy = ld(yoff, z0);
    for (int z = z0; z < z1; ++z) {
        for (int k = 0; k < kRows; ++k) {
            pl[1 + ly + 4 * k][1 + lx] = zc[k];
            if (lx < 2) pl[1 + ly + 4 * k][lx == 0 ? 0 : kTX + 1] = hx[k];
        }
        if (ly == 0) pl[0][1 + lx] = hy;
        if (ly == 3) pl[kTY + 1][1 + lx] = hy;
        __syncthreads();
        // loads of the next plane's halo and of the plane after next, in flight during the update
        double nzp[kRows];
        for (int k = 0; k < kRows; ++k) {
            nzp[k] = ld(off[k], z + 2);
            hx[k] = ld(hoff[k], z + 1);
        }
        hy = ld(yoff, z + 1);
        double *dz = dst + (int64_t)z * plane;
        for (int k = 0; k < kRows; ++k) {
            const int row = 1 + ly + 4 * k;
            const double c = zc[k];
            double v = c * d.keep;
            v = v + d.c * ((pl[row][lx + 2] - 2.0 * c) + pl[row][lx]);
            v = v + d.c * ((pl[row + 1][lx + 1] - 2.0 * c) + pl[row - 1][lx + 1]);
            v = v + d.c * ((zp[k] - 2.0 * c) + zm[k]);
            if (off[k] >= 0) dz[off[k]] = v;
        }
        __syncthreads();
        for (int k = 0; k < kRows; ++k) {
            zm[k] = zc[k];
            zc[k] = zp[k];
            zp[k] = nzp[k];
        }
    }
}

__global__ void k_soma_end(Dev d) {
    d.ctl->par ^= 1;
    d.ctl->iter += 1;
}

__global__ void k_soma_zero(uint32_t *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

inline int grid_for(int64_t n, int cap) {
    int64_t g = (n + kThreads - 1) / kThreads;
    return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

void launch_cells(const Dev &d, hipStream_t s) {
    if (d.n == 0) return;
    hipLaunchKernelGGL(k_soma_cells, dim3(grid_for(d.n, 8192)), dim3(kThreads), 0, s, d);
    hipLaunchKernelGGL(k_soma_secrete, dim3(grid_for(d.n, 8192)), dim3(kThreads), 0, s, d);
}
void launch_diffuse(const Dev &d, hipStream_t s) {
    const int64_t nt = d.tiles * d.nsub;
    const int64_t grid = ((nt + kXcds - 1) / kXcds) * kXcds;
    hipLaunchKernelGGL(k_diffuse, dim3((unsigned)grid), dim3(kThreads), 0, s, d);
}
void launch_end(const Dev &d, hipStream_t s) { hipLaunchKernelGGL(k_soma_end, dim3(1), dim3(1), 0, s, d); }

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
    size_t ctl, u0, u1, cnt, pos, type, vox, rank, orig, stage, total;
};

bool params_ok(const abm_soma_params &p) {
    if (!isfinite(p.lo) || !(p.space > 0.0) || !isfinite(p.space)) return false;
    if (p.resolution < 1 || p.resolution > kMaxRes || p.n_substances < 1 || p.n_substances > kMaxSubstances)
        return false;
    if (!(p.diffusion >= 0.0) || !isfinite(p.diffusion) || !(p.decay >= 0.0) || !isfinite(p.decay)) return false;
    if (!(p.dt > 0.0) || !isfinite(p.dt) || !isfinite(p.secretion) || !isfinite(p.gradient_weight)) return false;
    return true;
}

bool make_layout(const abm_soma_params &p, int64_t n, Layout &L) {
    if (n < 0 || n >= ((int64_t)1 << 40) || !params_ok(p)) return false;
    const int64_t R = p.resolution;
    const size_t pts = (size_t)(R * R * R) * (size_t)p.n_substances;
    const size_t N = (size_t)(n > 0 ? n : 1);
    Carver c;
    L.ctl = c.take<Ctl>(1);
    L.u0 = c.take<double>(pts);
    L.u1 = c.take<double>(pts);
    L.cnt = c.take<uint32_t>(pts);
    L.pos = c.take<double>(3 * N);
    L.type = c.take<int32_t>(N);
    L.vox = c.take<int64_t>(N);
    L.rank = c.take<uint32_t>(N);
    L.orig = c.take<int64_t>(N);
    L.stage = c.take<double>(3 * N);
    L.total = c.off + 256;
    return true;
}

}  // namespace soma
}  // namespace abm

using abm::clear_error;
using abm::set_error;
namespace sk = abm::soma;

struct abm_soma {
    sk::Dev d;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t exec[4] = {};  // 0: a whole iteration; 1: the cells; 2: the diffusion; 3: the end
    bool timing = false;
    std::vector<hipEvent_t> ev;
    double ms_total = 0.0;
    int64_t n_timed = 0;
};

#define SOMACHK(expr)                                                                 \
    do {                                                                              \
        hipError_t _e = (expr);                                                       \
        if (_e != hipSuccess) return set_error(ABM_ERR_HIP, hipGetErrorString(_e));   \
    } while (0)

static int capture(abm_soma *s, int part) {
    if (s->exec[part]) return ABM_OK;
    if (part == 1 && s->d.n == 0) return ABM_OK;  // no cells: nothing to capture
    if (!s->cap_stream) SOMACHK(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
    SOMACHK(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
    if (part == 0 || part == 1) sk::launch_cells(s->d, s->cap_stream);
    if (part == 0 || part == 2) sk::launch_diffuse(s->d, s->cap_stream);
    if (part == 0 || part == 3) sk::launch_end(s->d, s->cap_stream);
    hipGraph_t g;
    hipError_t e = hipStreamEndCapture(s->cap_stream, &g);
    if (e != hipSuccess) return set_error(ABM_ERR_HIP, hipGetErrorString(e));
    e = hipGraphInstantiate(&s->exec[part], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);  // the instantiated graph no longer needs its template
    if (e != hipSuccess) return set_error(ABM_ERR_HIP, hipGetErrorString(e));
    return ABM_OK;
}

// Coefficients of Eq 4.3 in the order the scheme states them (no contraction).
static void coefficients(const abm_soma_params &p, double &dx, double &keep, double &c) {
#pragma clang fp contract(off)
    dx = p.space / (double)p.resolution;
    keep = 1.0 - p.decay * p.dt;
    c = p.diffusion * p.dt / (dx * dx);
}

extern "C" size_t abm_soma_workspace_bytes(const abm_soma_params *p, int64_t n_cells) {
    if (!p) return 0;
    sk::Layout L;
    if (!sk::make_layout(*p, n_cells, L)) return 0;
    return L.total;
}

extern "C" int abm_soma_create(const abm_soma_params *p, int64_t n, const double *pos, const int32_t *type,
                               const double *conc, void *workspace, size_t ws_bytes, void *hip_stream,
                               abm_soma **out) {
    clear_error();
    if (!p || !out || !workspace || (n > 0 && (!pos || !type))) return set_error(ABM_ERR_ARG, "null argument");
    *out = nullptr;
    sk::Layout L;
    if (!sk::make_layout(*p, n, L)) return set_error(ABM_ERR_ARG, "bad diffusion parameters or cell count");
    if (ws_bytes < L.total) return set_error(ABM_ERR_ARG, "workspace too small");
    const double hi = p->lo + p->space;
    for (int64_t i = 0; i < 3 * n; ++i) {
        if (!isfinite(pos[i])) return set_error(ABM_ERR_NONFINITE, "non-finite position");
        if (pos[i] < p->lo || pos[i] > hi) return set_error(ABM_ERR_ARG, "position outside the space");
    }
    for (int64_t i = 0; i < n; ++i)
        if (type[i] < 0 || type[i] >= p->n_substances) return set_error(ABM_ERR_ARG, "cell type outside 0..n_substances-1");
    const int64_t R = p->resolution, V = R * R * R, pts = V * p->n_substances;
    if (conc)
        for (int64_t i = 0; i < pts; ++i)
            if (!isfinite(conc[i])) return set_error(ABM_ERR_NONFINITE, "non-finite concentration");
    abm_soma *s = new (std::nothrow) abm_soma();
    if (!s) return set_error(ABM_ERR_ARG, "out of host memory");
    char *base = (char *)(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
    sk::Dev &d = s->d;
    d.n = n;
    d.V = V;
    d.R = (int32_t)R;
    d.nsub = p->n_substances;
    d.lo = p->lo;
    d.S = p->space;
    d.hi = hi;
    coefficients(*p, d.dx, d.keep, d.c);
    d.q = p->secretion;
    d.w = p->gradient_weight;
    d.ctl = (sk::Ctl *)(base + L.ctl);
    d.u[0] = (double *)(base + L.u0);
    d.u[1] = (double *)(base + L.u1);
    d.cnt = (uint32_t *)(base + L.cnt);
    d.pos = (double *)(base + L.pos);
    d.type = (int32_t *)(base + L.type);
    d.vox = (int64_t *)(base + L.vox);
    d.rank = (uint32_t *)(base + L.rank);
    d.orig = (int64_t *)(base + L.orig);
    d.stage = (double *)(base + L.stage);
    d.tiles_x = (R + sk::kTX - 1) / sk::kTX;
    d.tiles_y = (R + sk::kTY - 1) / sk::kTY;
    d.tiles_z = (R + sk::kZChunk - 1) / sk::kZChunk;
    d.tiles = d.tiles_x * d.tiles_y * d.tiles_z;
    s->stream = (hipStream_t)hip_stream;
    hipStream_t st = s->stream;
    hipError_t e = hipSuccess;
    if (conc) e = hipMemcpyAsync(d.u[0], conc, sizeof(double) * (size_t)pts, hipMemcpyHostToDevice, st);
    else hipLaunchKernelGGL(sk::k_soma_zero, dim3(sk::grid_for(2 * pts, 65536)), dim3(sk::kThreads), 0, st,
                            (uint32_t *)d.u[0], 2 * pts);
    if (e == hipSuccess && n > 0) {
        // cells stored in the order of their substance and voxel (x fastest):
        // cells that are near each other read the same lines of the grid
        std::vector<int64_t> key((size_t)n), perm((size_t)n);
        auto vaxis = [&](double v) {
            double q = floor((v - d.lo) / d.dx);
            return q < 0.0 ? (int64_t)0 : (q > (double)(R - 1) ? R - 1 : (int64_t)q);
        };
        for (int64_t i = 0; i < n; ++i)
            key[i] = (int64_t)type[i] * V + vaxis(pos[3 * i]) + R * (vaxis(pos[3 * i + 1]) + R * vaxis(pos[3 * i + 2]));
        std::iota(perm.begin(), perm.end(), (int64_t)0);
        std::stable_sort(perm.begin(), perm.end(), [&](int64_t a, int64_t b) { return key[a] < key[b]; });
        std::vector<double> blocks((size_t)n * 3);
        std::vector<int32_t> ts((size_t)n);
        for (int64_t j = 0; j < n; ++j) {
            const int64_t i = perm[j];
            for (int a = 0; a < 3; ++a) blocks[(size_t)a * n + j] = pos[3 * i + a];
            ts[j] = type[i];
        }
        e = hipMemcpyAsync(d.pos, blocks.data(), sizeof(double) * 3 * (size_t)n, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(d.type, ts.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(d.orig, perm.data(), sizeof(int64_t) * (size_t)n, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);  // the host arrays end with this scope
    }
    if (e != hipSuccess) {
        delete s;
        return set_error(ABM_ERR_HIP, hipGetErrorString(e));
    }
    hipLaunchKernelGGL(sk::k_soma_zero, dim3(sk::grid_for(pts, 65536)), dim3(sk::kThreads), 0, st, d.cnt, pts);
    hipLaunchKernelGGL(sk::k_soma_zero, dim3(1), dim3(64), 0, st, (uint32_t *)d.ctl, (int64_t)(sizeof(sk::Ctl) / 4));
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        delete s;
        return set_error(ABM_ERR_HIP, hipGetErrorString(e));
    }
    *out = s;
    return ABM_OK;
}

extern "C" int abm_soma_step(abm_soma *s, int n_iter) {
    clear_error();
    if (!s || n_iter < 0) return set_error(ABM_ERR_ARG, "bad handle or iteration count");
    if (n_iter == 0) return ABM_OK;
    if (s->timing) {
        for (int part = 1; part <= 3; ++part) {
            int rc = capture(s, part);
            if (rc) return rc;
        }
        while ((int)s->ev.size() < 2 * n_iter) {
            hipEvent_t e;
            SOMACHK(hipEventCreate(&e));
            s->ev.push_back(e);
        }
        for (int it = 0; it < n_iter; ++it) {
            if (s->exec[1]) SOMACHK(hipGraphLaunch(s->exec[1], s->stream));
            SOMACHK(hipEventRecord(s->ev[2 * it], s->stream));
            SOMACHK(hipGraphLaunch(s->exec[2], s->stream));
            SOMACHK(hipEventRecord(s->ev[2 * it + 1], s->stream));
            SOMACHK(hipGraphLaunch(s->exec[3], s->stream));
        }
        SOMACHK(hipStreamSynchronize(s->stream));
        for (int it = 0; it < n_iter; ++it) {
            float ms = 0.0f;
            SOMACHK(hipEventElapsedTime(&ms, s->ev[2 * it], s->ev[2 * it + 1]));
            s->ms_total += ms;
        }
        s->n_timed += n_iter;
    } else {
        int rc = capture(s, 0);
        if (rc) return rc;
        for (int it = 0; it < n_iter; ++it) SOMACHK(hipGraphLaunch(s->exec[0], s->stream));
    }
    SOMACHK(hipGetLastError());
    return ABM_OK;
}

extern "C" int abm_soma_query(abm_soma *s, int field, void *dst, int dst_on_device, int64_t cap) {
    clear_error();
    if (!s || !dst) return set_error(ABM_ERR_ARG, "null argument");
    const sk::Dev &d = s->d;
    const hipMemcpyKind kind = dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    hipStream_t st = s->stream;
    sk::Ctl c;
    SOMACHK(hipMemcpyAsync(&c, d.ctl, sizeof c, hipMemcpyDeviceToHost, st));
    SOMACHK(hipStreamSynchronize(st));
    if (field == ABM_SOMA_POS || field == ABM_SOMA_TYPE) {
        if (cap < d.n) return set_error(ABM_ERR_ARG, "destination too small");
        if (d.n == 0) return ABM_OK;
        const size_t bytes = field == ABM_SOMA_POS ? sizeof(double) * 3 * (size_t)d.n : sizeof(int32_t) * (size_t)d.n;
        void *tmp = d.stage;
        if (field == ABM_SOMA_POS)
            hipLaunchKernelGGL(sk::k_soma_unsort_pos, dim3(sk::grid_for(d.n, 65536)), dim3(sk::kThreads), 0, st, d,
                               (double *)tmp);
        else
            hipLaunchKernelGGL(sk::k_soma_unsort_type, dim3(sk::grid_for(d.n, 65536)), dim3(sk::kThreads), 0, st, d,
                               (int32_t *)tmp);
        hipError_t e = hipMemcpyAsync(dst, tmp, bytes, kind, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return set_error(ABM_ERR_HIP, hipGetErrorString(e));
    } else if (field == ABM_SOMA_CONC) {
        const int64_t pts = d.V * d.nsub;
        if (cap < pts) return set_error(ABM_ERR_ARG, "destination too small");
        SOMACHK(hipMemcpyAsync(dst, d.u[c.par], sizeof(double) * (size_t)pts, kind, st));
    } else {
        return set_error(ABM_ERR_ARG, "unknown field");
    }
    SOMACHK(hipGetLastError());
    SOMACHK(hipStreamSynchronize(st));
    return ABM_OK;
}

extern "C" int abm_soma_set_timing(abm_soma *s, int on) {
    clear_error();
    if (!s) return set_error(ABM_ERR_ARG, "null handle");
    s->timing = on != 0;
    return ABM_OK;
}

extern "C" int abm_soma_kernel_time(abm_soma *s, double *ms_total, int64_t *n_launches) {
    clear_error();
    if (!s || !ms_total || !n_launches) return set_error(ABM_ERR_ARG, "null argument");
    *ms_total = s->ms_total;
    *n_launches = s->n_timed;
    s->ms_total = 0.0;
    s->n_timed = 0;
    return ABM_OK;
}

extern "C" int abm_soma_destroy(abm_soma *s) {
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
