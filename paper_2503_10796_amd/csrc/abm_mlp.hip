// abm_mlp.hip -- the surrogate MLP on the matrix cores of gfx950.
//
// Layers Linear -> GELU (exact erf form) on every hidden layer, Linear at the
// output; loss = mean squared error over batch x outputs; Adam with bias
// correction.  FP32 master weights and Adam moments; the GEMMs read BF16
// copies of weights and activations and accumulate in FP32 with
// v_mfma_f32_16x16x32_bf16.  One tiled GEMM kernel serves the forward pass
// (bias + GELU epilogue), the input gradient (GELU' epilogue) and the weight
// gradient (transposed A operand); bias gradients are column sums.  Every
// reduction runs in a fixed order, so a step is bitwise reproducible.
//
// Parameter layout (get/set, gradients): per layer W [out][in] row-major,
// then b [out].
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>

#include "abm_device.h"

using namespace abm;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kMaxLayers = 8;
constexpr int kBM = 64, kBN = 64, kBK = 32;  // GEMM block tile; 4 waves of 32 x 32
constexpr int kLdsK = kBK + 8;               // padded LDS row (bf16 elements, 80 bytes)

enum GemmMode { kFwdHidden = 0, kFwdOut = 1, kBwdInput = 2, kBwdWeight = 3, kFwdHiddenAct = 4 };

struct GemmArgs {
    int M, N, K;
    const __bf16 *A;  // A[m][k] = transA ? A[k * lda + m] : A[m * lda + k]
    int lda, transA;
    const __bf16 *B;  // B[k][n] = transB ? B[n * ldb + k] : B[k * ldb + n]
    int ldb, transB;
    int mode;
    const float *bias;   // [N] (forward)
    float *outf;         // FP32 result, leading dimension ldo
    int ldo;
    __bf16 *outb;        // BF16 result (forward hidden, backward input), leading dimension ldob
    int ldob;
    const float *zprev;  // pre-activation of the layer below (backward input), leading dimension ldz
    int ldz;
};

__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// C[M x N] = A[M x K] * B[K x N] with the mode's epilogue.  Block (64 x 64)
// tiles, K in steps of 32 staged through LDS; operands out of range read 0.
__global__ void __launch_bounds__(256) k_gemm(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) __bf16 As[kBM][kLdsK];
    __shared__ __attribute__((aligned(16))) __bf16 Bt[kBN][kLdsK];  // B tile transposed: Bt[n][k]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int m0 = blockIdx.y * kBM, n0 = blockIdx.x * kBN;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    f32x4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const __bf16 zero = (__bf16)0.0f;
    for (int k0 = 0; k0 < g.K; k0 += kBK) {
        // 2048 elements per tile, 8 per thread
        for (int e = 0; e < 8; ++e) {
            const int idx = tid * 8 + e;
            // A tile element (r, c): row r of 64, column c of 32
            {
                const int r = g.transA ? idx % kBM : idx / kBK;
                const int c = g.transA ? idx / kBM : idx % kBK;
                const int m = m0 + r, k = k0 + c;
                __bf16 v = zero;
                if (m < g.M && k < g.K) v = g.transA ? g.A[(size_t)k * g.lda + m] : g.A[(size_t)m * g.lda + k];
                As[r][c] = v;
            }
            // B tile element (k, n) stored at Bt[n][k]
            {
                const int n = g.transB ? idx / kBK : idx % kBN;
                const int c = g.transB ? idx % kBK : idx / kBN;
                const int nn = n0 + n, k = k0 + c;
                __bf16 v = zero;
                if (nn < g.N && k < g.K) v = g.transB ? g.B[(size_t)nn * g.ldb + k] : g.B[(size_t)k * g.ldb + nn];
                Bt[n][c] = v;
            }
        }
        __syncthreads();
        bf16x8 a[2], b[2];
        for (int i = 0; i < 2; ++i) a[i] = *(const bf16x8 *)&As[wm + 16 * i + (lane & 15)][8 * (lane >> 4)];
        for (int j = 0; j < 2; ++j) b[j] = *(const bf16x8 *)&Bt[wn + 16 * j + (lane & 15)][8 * (lane >> 4)];
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    // lane holds column (lane & 15) and rows 4 * (lane >> 4) + e of each 16 x 16 block
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + wn + 16 * j + (lane & 15);
            if (n >= g.N) continue;
            for (int e = 0; e < 4; ++e) {
                const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + e;
                if (m >= g.M) continue;
                const float v = acc[i][j][e];
                switch (g.mode) {
                    case kFwdHidden: {
                        const float z = v + g.bias[n];
                        g.outf[(size_t)m * g.ldo + n] = z;
                        g.outb[(size_t)m * g.ldob + n] = (__bf16)gelu(z);
                        break;
                    }
                    case kFwdHiddenAct:  // inference: the BF16 activation only
                        g.outb[(size_t)m * g.ldob + n] = (__bf16)gelu(v + g.bias[n]);
                        break;
                    case kFwdOut:
                        g.outf[(size_t)m * g.ldo + n] = v + g.bias[n];
                        break;
                    case kBwdInput: {
                        const float dz = v * gelu_grad(g.zprev[(size_t)m * g.ldz + n]);
                        g.outf[(size_t)m * g.ldo + n] = dz;
                        g.outb[(size_t)m * g.ldob + n] = (__bf16)dz;
                        break;
                    }
                    default:
                        g.outf[(size_t)m * g.ldo + n] = v;
                        break;
                }
            }
        }
}

// x [B x in] FP32 -> [B x ldk] BF16, zero padded.
__global__ void k_to_bf16(const float *x, __bf16 *out, int B, int in, int ldk) {
    const int64_t n = (int64_t)B * ldk;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(t / ldk), c = (int)(t % ldk);
        out[t] = (__bf16)(c < in ? x[(size_t)r * in + c] : 0.0f);
    }
}

struct Layers {
    int nl;
    int in[kMaxLayers], out[kMaxLayers], ldk[kMaxLayers];
    int64_t woff[kMaxLayers], boff[kMaxLayers], wbf_off[kMaxLayers];
};

// BF16 copies of all weights, each [out x ldk] zero padded.
__global__ void k_weights_bf16(const float *theta, __bf16 *wbf, Layers Ls) {
    for (int l = 0; l < Ls.nl; ++l) {
        const int64_t n = (int64_t)Ls.out[l] * Ls.ldk[l];
        for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
            const int o = (int)(t / Ls.ldk[l]), c = (int)(t % Ls.ldk[l]);
            wbf[Ls.wbf_off[l] + t] = (__bf16)(c < Ls.in[l] ? theta[Ls.woff[l] + (int64_t)o * Ls.in[l] + c] : 0.0f);
        }
    }
}

// Inference of the whole network in one kernel, for networks whose padded
// widths are at most kFuseMax: a work group (4 waves) carries 16 rows of the
// batch through every layer, with the activations in LDS (BF16, zero padded
// to the next layer's K) and the weights read from L2.  Each wave takes the
// 16-column output tiles w, w + 4, ... of a layer, four at a time, with the
// B fragments of all K steps of the four tiles loaded before the first MFMA
// (so the L2 latency is paid once per layer, not once per K step).  The MFMA
// operands and their K order are those of k_gemm, and the epilogues are the
// same expressions, so the outputs equal the layer-by-layer path bit for bit.
constexpr int kFuseRows = 16, kFuseMax = 256, kFuseLd = kFuseMax + 8;

__global__ void __launch_bounds__(256) k_mlp_fused(const float *__restrict__ x, float *__restrict__ y, int batch,
                                                    const __bf16 *__restrict__ wbf, const float *__restrict__ theta,
                                                    Layers Lsa) {
    __shared__ __attribute__((aligned(16))) __bf16 act[2][kFuseRows][kFuseLd];
    __shared__ Layers Ls;  // indexed by the layer below: kept in LDS, not in private memory
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) Ls = Lsa;
    __syncthreads();
    const int row0 = blockIdx.x * kFuseRows;
    const __bf16 zero = (__bf16)0.0f;
    {  // the input rows, converted and zero padded to ldk[0] (rows past the batch: zero)
        const int in = Ls.in[0], ld = Ls.ldk[0];
        for (int t = tid; t < kFuseRows * ld; t += 256) {
            const int r = t / ld, c = t % ld;
            act[0][r][c] = (row0 + r < batch && c < in) ? (__bf16)x[(size_t)(row0 + r) * in + c] : zero;
        }
    }
    __syncthreads();
    for (int l = 0; l < Ls.nl; ++l) {
        const int cur = l & 1, nxt = cur ^ 1;
        const int K = Ls.ldk[l], N = Ls.out[l], nsteps = K / kBK;
        const bool last = l == Ls.nl - 1;
        const __bf16 *W = wbf + Ls.wbf_off[l];  // [N][K], zero padded
        const float *bias = theta + Ls.boff[l];
        const int ntiles = (N + 15) / 16;
        for (int j0 = w; j0 < ntiles; j0 += 16) {
            const int jt[4] = {j0, j0 + 4, j0 + 8, j0 + 12};
            bf16x8 bw[4][kFuseMax / kBK];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int n = jt[q] * 16 + (lane & 15);
                const bool ok = jt[q] < ntiles && n < N;
#pragma unroll
                for (int st = 0; st < kFuseMax / kBK; ++st) {
                    if (st < nsteps && ok) bw[q][st] = *(const bf16x8 *)&W[(size_t)n * K + st * kBK + 8 * (lane >> 4)];
                    else bw[q][st] = bf16x8{zero, zero, zero, zero, zero, zero, zero, zero};
                }
            }
            f32x4 acc[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int st = 0; st < kFuseMax / kBK; ++st) {
                if (st >= nsteps) break;
                const bf16x8 a = *(const bf16x8 *)&act[cur][lane & 15][st * kBK + 8 * (lane >> 4)];
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[q][st], acc[q], 0, 0, 0);
            }
            // lane holds column (lane & 15) and rows 4 * (lane >> 4) + e of each tile
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int n = jt[q] * 16 + (lane & 15);
                if (jt[q] >= ntiles || n >= N) continue;
                const float b = bias[n];
                for (int e = 0; e < 4; ++e) {
                    const int m = 4 * (lane >> 4) + e;
                    if (last) {
                        if (row0 + m < batch) y[(size_t)(row0 + m) * N + n] = acc[q][e] + b;
                    } else {
                        act[nxt][m][n] = (__bf16)gelu(acc[q][e] + b);
                    }
                }
            }
        }
        if (!last) {
            // zero the padding of the next layer's K (columns N .. ldk[l + 1])
            const int ld = Ls.ldk[l + 1];
            for (int t = tid; t < kFuseRows * (ld - N); t += 256) act[nxt][t / (ld - N)][N + t % (ld - N)] = zero;
        }
        __syncthreads();
    }
}

// He-normal weights (std sqrt(2 / fan_in)), zero biases.  Normal deviates by
// Box-Muller from Philox4x32-10, counter (parameter index, 0, 0, 0), key = seed.
__global__ void k_init(float *theta, Layers Ls, uint64_t seed) {
    for (int l = 0; l < Ls.nl; ++l) {
        const int64_t nw = (int64_t)Ls.out[l] * Ls.in[l];
        const float sd = sqrtf(2.0f / (float)Ls.in[l]);
        for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nw + Ls.out[l];
             t += (int64_t)gridDim.x * blockDim.x) {
            if (t >= nw) {
                theta[Ls.boff[l] + (t - nw)] = 0.0f;
                continue;
            }
            const uint64_t idx = (uint64_t)(Ls.woff[l] + t);
            uint32_t c[4] = {(uint32_t)idx, (uint32_t)(idx >> 32), 0u, 0u};
            philox(c, (uint32_t)seed, (uint32_t)(seed >> 32));
            const float u1 = ((float)(c[0] >> 8) + 1.0f) * 0x1.0p-24f;  // (0, 1]
            const float u2 = (float)(c[1] >> 8) * 0x1.0p-24f;           // [0, 1)
            theta[Ls.woff[l] + t] = sd * sqrtf(-2.0f * logf(u1)) * cospif(2.0f * u2);
        }
    }
}

// Output error: d = yhat - y; per-block partial sums of d^2 (fixed order);
// dz = 2 d / (B * out) in FP32 and BF16.
__global__ void __launch_bounds__(256) k_loss(const float *yhat, const float *y, int64_t n, float scale, float *dzf,
                                              __bf16 *dzb, float *part) {
    __shared__ float sh[256];
    float s = 0.0f;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const float d = yhat[t] - y[t];
        s += d * d;
        const float g = 2.0f * d * scale;
        dzf[t] = g;
        dzb[t] = (__bf16)g;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_loss_final(const float *part, int np, float scale, float *loss) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < np; ++i) s += part[i];
        *loss = (float)(s * scale);
    }
}

// db[n] = sum over rows of dz[m][n] (32 columns per block, 8 row lanes, fixed order).
__global__ void __launch_bounds__(256) k_colsum(const float *dz, int M, int N, float *db) {
    __shared__ float sh[8][33];
    const int c = threadIdx.x & 31, r = threadIdx.x >> 5;
    const int n = blockIdx.x * 32 + c;
    float s = 0.0f;
    if (n < N)
        for (int m = r; m < M; m += 8) s += dz[(size_t)m * N + n];
    sh[r][c] = s;
    __syncthreads();
    if (r == 0 && n < N) {
        float t = 0.0f;
        for (int q = 0; q < 8; ++q) t += sh[q][c];
        db[n] = t;
    }
}

__global__ void k_adam(float *theta, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
                       float c1, float c2, float eps) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const float gt = g[t];
        const float mt = b1 * m[t] + (1.0f - b1) * gt;
        const float vt = b2 * v[t] + (1.0f - b2) * gt * gt;
        m[t] = mt;
        v[t] = vt;
        theta[t] -= lr * (mt / c1) / (sqrtf(vt / c2) + eps);
    }
}

inline int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

}  // namespace

struct abm_mlp {
    Layers Ls;
    int max_batch;
    int64_t nparams;
    hipStream_t stream;
    int64_t t;  // Adam steps taken
    float *theta, *grad, *am, *av;
    __bf16 *wbf;
    __bf16 *hbf[kMaxLayers + 1];  // hbf[0]: input [B x ldk0]; hbf[l]: GELU(z[l-1]) [B x out(l-1)]
    float *z[kMaxLayers];         // pre-activations [B x out(l)]
    float *dzf[2];
    __bf16 *dzb[2];
    float *yout;
    float *part, *loss;
    int nparts;
};

namespace {

struct Carve {
    char *base;
    int64_t off = 0;
    template <typename T>
    T *take(int64_t n) {
        off = align_up(off, 256);
        T *p = base ? (T *)(base + off) : nullptr;
        off += n * (int64_t)sizeof(T);
        return p;
    }
};

bool valid_dims(const int *dims, int n_dims) {
    if (!dims || n_dims < 2 || n_dims > kMaxLayers + 1) return false;
    for (int i = 0; i < n_dims; ++i)
        if (dims[i] <= 0 || dims[i] > 65536) return false;
    for (int i = 1; i < n_dims - 1; ++i)
        if (dims[i] % 16) return false;
    return true;
}

// Lays the handle's buffers out in the workspace (base == nullptr: sizing only).
int64_t layout(abm_mlp &h, const int *dims, int n_dims, int max_batch, char *base) {
    Carve c{base};
    Layers &Ls = h.Ls;
    Ls.nl = n_dims - 1;
    int64_t p = 0, wb = 0;
    for (int l = 0; l < Ls.nl; ++l) {
        Ls.in[l] = dims[l];
        Ls.out[l] = dims[l + 1];
        Ls.ldk[l] = (int)align_up(dims[l], kBK);
        Ls.woff[l] = p;
        p += (int64_t)dims[l + 1] * dims[l];
        Ls.boff[l] = p;
        p += dims[l + 1];
        Ls.wbf_off[l] = wb;
        wb += (int64_t)dims[l + 1] * Ls.ldk[l];
    }
    h.nparams = p;
    h.max_batch = max_batch;
    h.theta = c.take<float>(p);
    h.grad = c.take<float>(p);
    h.am = c.take<float>(p);
    h.av = c.take<float>(p);
    h.wbf = c.take<__bf16>(wb);
    h.hbf[0] = c.take<__bf16>((int64_t)max_batch * Ls.ldk[0]);
    int widest = 0;
    for (int l = 0; l < Ls.nl; ++l) {
        h.z[l] = c.take<float>((int64_t)max_batch * Ls.out[l]);
        h.hbf[l + 1] = c.take<__bf16>((int64_t)max_batch * Ls.out[l]);
        widest = std::max(widest, Ls.out[l]);
    }
    for (int q = 0; q < 2; ++q) {
        h.dzf[q] = c.take<float>((int64_t)max_batch * widest);
        h.dzb[q] = c.take<__bf16>((int64_t)max_batch * widest);
    }
    h.yout = c.take<float>((int64_t)max_batch * Ls.out[Ls.nl - 1]);
    h.nparts = 256;
    h.part = c.take<float>(h.nparts);
    h.loss = c.take<float>(1);
    return c.off;
}

#define MLPCHK(expr)                                                               \
    do {                                                                           \
        hipError_t _e = (expr);                                                    \
        if (_e != hipSuccess) return set_error(ABM_ERR_HIP, hipGetErrorString(_e)); \
    } while (0)

void gemm(hipStream_t s, const GemmArgs &g) {
    dim3 grid((g.N + kBN - 1) / kBN, (g.M + kBM - 1) / kBM);
    hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, s, g);
}

// Forward pass of a batch already converted into hbf[0]; the output lands in yout.
void forward(abm_mlp *h, int B) {
    const Layers &Ls = h->Ls;
    for (int l = 0; l < Ls.nl; ++l) {
        const bool last = l == Ls.nl - 1;
        GemmArgs g{};
        g.M = B;
        g.N = Ls.out[l];
        // the input is zero padded to ldk[0]; hidden activations are rows of
        // out[l - 1] (the tile reads zeros past K)
        g.K = l == 0 ? Ls.ldk[0] : Ls.in[l];
        g.A = h->hbf[l];
        g.lda = l == 0 ? Ls.ldk[0] : Ls.out[l - 1];
        g.transA = 0;
        g.B = h->wbf + Ls.wbf_off[l];  // B[k][n] = W[n][k]
        g.ldb = Ls.ldk[l];
        g.transB = 1;
        g.mode = last ? kFwdOut : kFwdHidden;
        g.bias = h->theta + Ls.boff[l];
        g.outf = last ? h->yout : h->z[l];
        g.ldo = Ls.out[l];
        g.outb = last ? nullptr : h->hbf[l + 1];
        g.ldob = Ls.out[l];
        gemm(h->stream, g);
    }
}

// Loss and gradient of a batch (x, y device FP32) into h->grad and h->loss.
void loss_and_grad(abm_mlp *h, const float *x, const float *y, int B) {
    const Layers &Ls = h->Ls;
    hipStream_t s = h->stream;
    hipLaunchKernelGGL(k_to_bf16, dim3(std::min(4096, (B * Ls.ldk[0] + 255) / 256)), dim3(256), 0, s, x, h->hbf[0], B,
                       Ls.in[0], Ls.ldk[0]);
    forward(h, B);
    const int L = Ls.nl;
    const int64_t nout = (int64_t)B * Ls.out[L - 1];
    const float scale = 1.0f / (float)nout;
    hipLaunchKernelGGL(k_loss, dim3(h->nparts), dim3(256), 0, s, h->yout, y, nout, scale, h->dzf[0], h->dzb[0], h->part);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, s, h->part, h->nparts, scale, h->loss);
    int cur = 0;
    for (int l = L - 1; l >= 0; --l) {
        // dW[o][i] = sum_b dz[b][o] h[b][i]
        GemmArgs gw{};
        gw.M = Ls.out[l];
        gw.N = Ls.in[l];
        gw.K = B;
        gw.A = h->dzb[cur];
        gw.lda = Ls.out[l];
        gw.transA = 1;
        gw.B = h->hbf[l];
        gw.ldb = l == 0 ? Ls.ldk[0] : Ls.out[l - 1];
        gw.transB = 0;
        gw.mode = kBwdWeight;
        gw.outf = h->grad + Ls.woff[l];
        gw.ldo = Ls.in[l];
        gemm(s, gw);
        hipLaunchKernelGGL(k_colsum, dim3((Ls.out[l] + 31) / 32), dim3(256), 0, s, h->dzf[cur], B, Ls.out[l],
                           h->grad + Ls.boff[l]);
        if (l == 0) break;
        // dz below = (dz W) * GELU'(z below)
        GemmArgs gi{};
        gi.M = B;
        gi.N = Ls.in[l];
        gi.K = Ls.out[l];
        gi.A = h->dzb[cur];
        gi.lda = Ls.out[l];
        gi.transA = 0;
        gi.B = h->wbf + Ls.wbf_off[l];  // B[k][n] = W[k][n]
        gi.ldb = Ls.ldk[l];
        gi.transB = 0;
        gi.mode = kBwdInput;
        gi.zprev = h->z[l - 1];
        gi.ldz = Ls.out[l - 1];
        gi.outf = h->dzf[1 - cur];
        gi.ldo = Ls.in[l];
        gi.outb = h->dzb[1 - cur];
        gi.ldob = Ls.in[l];
        gemm(s, gi);
        cur = 1 - cur;
    }
}

int check_batch(abm_mlp *m, int batch) {
    if (!m) return set_error(ABM_ERR_ARG, "null handle");
    if (batch <= 0 || batch > m->max_batch) return set_error(ABM_ERR_ARG, "batch outside 1..max_batch");
    return ABM_OK;
}

}  // namespace

extern "C" size_t abm_mlp_workspace_bytes(const int *dims, int n_dims, int max_batch) {
    if (!valid_dims(dims, n_dims) || max_batch <= 0) return 0;
    abm_mlp h{};
    return (size_t)layout(h, dims, n_dims, max_batch, nullptr);
}

extern "C" int abm_mlp_create(const int *dims, int n_dims, int max_batch, uint64_t seed, void *workspace,
                              size_t ws_bytes, void *hip_stream, abm_mlp **out) {
    clear_error();
    if (!out || !workspace) return set_error(ABM_ERR_ARG, "null argument");
    if (!valid_dims(dims, n_dims) || max_batch <= 0)
        return set_error(ABM_ERR_ARG, "dims must be 2..9 positive widths, hidden widths multiples of 16");
    abm_mlp *h = new (std::nothrow) abm_mlp{};
    if (!h) return set_error(ABM_ERR_ARG, "out of host memory");
    const int64_t need = layout(*h, dims, n_dims, max_batch, (char *)workspace);
    if ((size_t)need > ws_bytes) {
        delete h;
        return set_error(ABM_ERR_ARG, "workspace too small");
    }
    h->stream = (hipStream_t)hip_stream;
    h->t = 0;
    hipStream_t s = h->stream;
    hipError_t e = hipMemsetAsync(h->am, 0, sizeof(float) * h->nparams, s);
    if (e == hipSuccess) e = hipMemsetAsync(h->av, 0, sizeof(float) * h->nparams, s);
    if (e != hipSuccess) {
        delete h;
        return set_error(ABM_ERR_HIP, hipGetErrorString(e));
    }
    hipLaunchKernelGGL(k_init, dim3(256), dim3(256), 0, s, h->theta, h->Ls, seed);
    hipLaunchKernelGGL(k_weights_bf16, dim3(256), dim3(256), 0, s, h->theta, h->wbf, h->Ls);
    e = hipGetLastError();
    if (e != hipSuccess) {
        delete h;
        return set_error(ABM_ERR_HIP, hipGetErrorString(e));
    }
    *out = h;
    return ABM_OK;
}

extern "C" int abm_mlp_train_step(abm_mlp *m, const float *x, const float *y, int batch, float lr, float *loss_out) {
    clear_error();
    int rc = check_batch(m, batch);
    if (rc) return rc;
    if (!x || !y || !(lr > 0.0f)) return set_error(ABM_ERR_ARG, "null input or non-positive learning rate");
    loss_and_grad(m, x, y, batch);
    m->t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = (float)(1.0 - std::pow(0.9, (double)m->t)), c2 = (float)(1.0 - std::pow(0.999, (double)m->t));
    hipLaunchKernelGGL(k_adam, dim3(256), dim3(256), 0, m->stream, m->theta, m->grad, m->am, m->av, m->nparams, lr,
                       b1, b2, c1, c2, 1e-8f);
    hipLaunchKernelGGL(k_weights_bf16, dim3(256), dim3(256), 0, m->stream, m->theta, m->wbf, m->Ls);
    MLPCHK(hipGetLastError());
    if (loss_out) {
        MLPCHK(hipMemcpyAsync(loss_out, m->loss, sizeof(float), hipMemcpyDeviceToHost, m->stream));
        MLPCHK(hipStreamSynchronize(m->stream));
    }
    return ABM_OK;
}

extern "C" int abm_mlp_grads(abm_mlp *m, const float *x, const float *y, int batch, float *grads_out,
                             float *loss_out) {
    clear_error();
    int rc = check_batch(m, batch);
    if (rc) return rc;
    if (!x || !y || !grads_out) return set_error(ABM_ERR_ARG, "null argument");
    loss_and_grad(m, x, y, batch);
    MLPCHK(hipMemcpyAsync(grads_out, m->grad, sizeof(float) * m->nparams, hipMemcpyDeviceToDevice, m->stream));
    if (loss_out) {
        MLPCHK(hipMemcpyAsync(loss_out, m->loss, sizeof(float), hipMemcpyDeviceToHost, m->stream));
        MLPCHK(hipStreamSynchronize(m->stream));
    }
    MLPCHK(hipGetLastError());
    return ABM_OK;
}

extern "C" int abm_mlp_infer(abm_mlp *m, const float *x, float *y, int batch) {
    clear_error();
    int rc = check_batch(m, batch);
    if (rc) return rc;
    if (!x || !y) return set_error(ABM_ERR_ARG, "null argument");
    const Layers &Ls = m->Ls;
    bool fits = true;
    for (int l = 0; l < Ls.nl; ++l) fits = fits && Ls.ldk[l] <= kFuseMax && Ls.out[l] <= kFuseMax;
    if (fits) {
        hipLaunchKernelGGL(k_mlp_fused, dim3((batch + kFuseRows - 1) / kFuseRows), dim3(256), 0, m->stream, x, y, batch,
                           m->wbf, m->theta, Ls);
        MLPCHK(hipGetLastError());
        return ABM_OK;
    }
    hipLaunchKernelGGL(k_to_bf16, dim3(std::min(4096, (batch * Ls.ldk[0] + 255) / 256)), dim3(256), 0, m->stream, x,
                       m->hbf[0], batch, Ls.in[0], Ls.ldk[0]);
    forward(m, batch);
    MLPCHK(hipMemcpyAsync(y, m->yout, sizeof(float) * (size_t)batch * Ls.out[Ls.nl - 1], hipMemcpyDeviceToDevice,
                          m->stream));
    MLPCHK(hipGetLastError());
    return ABM_OK;
}

extern "C" int abm_mlp_get_params(abm_mlp *m, float *dst, size_t n) {
    clear_error();
    if (!m || !dst || n != (size_t)m->nparams) return set_error(ABM_ERR_ARG, "bad handle, buffer or size");
    MLPCHK(hipMemcpyAsync(dst, m->theta, sizeof(float) * n, hipMemcpyDeviceToDevice, m->stream));
    return ABM_OK;
}

extern "C" int abm_mlp_set_params(abm_mlp *m, const float *src, size_t n) {
    clear_error();
    if (!m || !src || n != (size_t)m->nparams) return set_error(ABM_ERR_ARG, "bad handle, buffer or size");
    MLPCHK(hipMemcpyAsync(m->theta, src, sizeof(float) * n, hipMemcpyDeviceToDevice, m->stream));
    MLPCHK(hipMemsetAsync(m->am, 0, sizeof(float) * n, m->stream));
    MLPCHK(hipMemsetAsync(m->av, 0, sizeof(float) * n, m->stream));
    m->t = 0;
    hipLaunchKernelGGL(k_weights_bf16, dim3(256), dim3(256), 0, m->stream, m->theta, m->wbf, m->Ls);
    MLPCHK(hipGetLastError());
    return ABM_OK;
}

extern "C" size_t abm_mlp_num_params(abm_mlp *m) { return m ? (size_t)m->nparams : 0; }

extern "C" int abm_mlp_destroy(abm_mlp *m) {
    clear_error();
    if (!m) return set_error(ABM_ERR_ARG, "null handle");
    delete m;
    return ABM_OK;
}

// ------------------------------------------------------------------ inference without allocation
// abm_mlp_infer_noalloc: the forward pass of abm_mlp_infer with its
// activations in a file-scope device array instead of the handle's
// workspace.  Layout of the array: the BF16 input [B x ldk0], then two BF16
// activation buffers [B x width] used in turn by the hidden layers; the output
// layer writes the caller's y.  Each GPU holds its own copy of the array
// until the process ends, and every call on that GPU shares it.
namespace {
constexpr int kNoAllocMaxBatch = 4096;
constexpr int kNoAllocMaxWidth = 512;  // input width (padded) and hidden widths
constexpr size_t kNoAllocActBytes = (size_t)kNoAllocMaxBatch * kNoAllocMaxWidth * sizeof(__bf16);
constexpr size_t kNoAllocBytes = 3 * kNoAllocActBytes;  // 12 MiB
constexpr int kNoAllocMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
std::mutex g_scratch_mu;
char *g_scratch_ptr[kNoAllocMaxDevices];  // device address of `scratch` on each device (null: not looked up)

// Device address of the array on the current device, looked up once per
// device with that device current.
int noalloc_scratch(char **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(ABM_ERR_HIP, hipGetErrorString(e));
    if (dev < 0 || dev >= kNoAllocMaxDevices) return set_error(ABM_ERR_ARG, "device ordinal beyond 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return set_error(ABM_ERR_HIP, "hipGetSymbolAddress of the inference scratch failed");
        g_scratch_ptr[dev] = (char *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return ABM_OK;
}
}  // namespace

extern "C" int abm_mlp_infer_noalloc(abm_mlp *m, const float *x, float *y, int batch) {
    clear_error();
    if (!m || !x || !y) return set_error(ABM_ERR_ARG, "null argument");
    if (batch <= 0 || batch > kNoAllocMaxBatch) return set_error(ABM_ERR_ARG, "batch outside 1..4096");
    const Layers &Ls = m->Ls;
    if (Ls.ldk[0] > kNoAllocMaxWidth) return set_error(ABM_ERR_ARG, "input width beyond 512");
    for (int l = 0; l + 1 < Ls.nl; ++l)
        if (Ls.out[l] > kNoAllocMaxWidth) return set_error(ABM_ERR_ARG, "hidden width beyond 512");
    char *base = nullptr;
    int rc = noalloc_scratch(&base);
    if (rc) return rc;
    __bf16 *in = (__bf16 *)base;
    __bf16 *act[2] = {(__bf16 *)(base + kNoAllocActBytes), (__bf16 *)(base + 2 * kNoAllocActBytes)};
    hipStream_t s = m->stream;
    hipLaunchKernelGGL(k_to_bf16, dim3(std::min(4096, (batch * Ls.ldk[0] + 255) / 256)), dim3(256), 0, s, x, in, batch,
                       Ls.in[0], Ls.ldk[0]);
    for (int l = 0; l < Ls.nl; ++l) {
        const bool last = l == Ls.nl - 1;
        GemmArgs g{};
        g.M = batch;
        g.N = Ls.out[l];
        g.K = l == 0 ? Ls.ldk[0] : Ls.in[l];
        g.A = l == 0 ? in : act[(l - 1) & 1];
        g.lda = l == 0 ? Ls.ldk[0] : Ls.out[l - 1];
        g.transA = 0;
        g.B = m->wbf + Ls.wbf_off[l];
        g.ldb = Ls.ldk[l];
        g.transB = 1;
        g.mode = last ? kFwdOut : kFwdHiddenAct;
        g.bias = m->theta + Ls.boff[l];
        g.outf = last ? y : nullptr;
        g.ldo = Ls.out[l];
        g.outb = last ? nullptr : act[l & 1];
        g.ldob = Ls.out[l];
        gemm(s, g);
    }
    MLPCHK(hipGetLastError());
    return ABM_OK;
}
