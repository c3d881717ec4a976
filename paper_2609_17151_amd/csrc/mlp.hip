// Warm-start network on the matrix cores: every layer, forward and backward,
// is one BF16 product with FP32 accumulation (v_mfma_f32_16x16x32_bf16) whose
// epilogue applies the elementwise work of the layer, so no activation makes
// an extra round trip to memory.
//
// A layer's parameters are the matrix [n_out][n_in + 1] with the bias as the
// last column; the products see the layer input extended by a column of ones,
// so the bias rides in the product both forward (z = [a 1] Wa^T) and backward
// (dWa = dz^T [a 1], whose last column is the bias gradient).
//
// Product C[M][N] = sum_k A(m, k) B(k, n), operands read through strides from
// FP32 or BF16 memory and rounded to BF16 into LDS.  Tile 64 x 64 x 32, four
// waves in a 2 x 2 arrangement, each wave a 32 x 32 block of four 16 x 16
// matrix-core tiles.  Epilogues:
//   STORE  C = acc
//   GELU   C = acc (pre-activation), C2 = acc Phi(acc)
//   LOSS   d = acc - T, C = scale d (the output gradient), sum of d^2 per workgroup
//   DGELU  C = acc * g'(Z) with g' the derivative of z Phi(z)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "pic_mlp.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kBM = 64, kBN = 64, kBK = 32;
constexpr int kPad = 8;                    // LDS row = 40 BF16 = 80 B: rows land on different banks
constexpr int kThreads = 256;

enum { EPI_STORE = 0, EPI_GELU = 1, EPI_LOSS = 2, EPI_DGELU = 3 };

struct Operand {
    const void* p;
    int64_t s0, s1;        // A: element (m, k) at m*s0 + k*s1;  B: element (k, n) at k*s0 + n*s1
    int32_t bf16;          // storage type: 1 = BF16, 0 = FP32
    int32_t one;           // A: k index that reads as 1; B: n index that reads as 1; -1: none
};

struct GemmArgs {
    int32_t M, N, K, epi;
    Operand a, b;
    float* c;
    float* c2;
    int64_t ldc;
    const float* aux;      // LOSS: targets, DGELU: pre-activation of the layer below
    int64_t ldaux;
    float scale;
    float* loss_part;      // LOSS: one partial sum per workgroup
};

__device__ __forceinline__ float gelu(float z)
{
    return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}

__device__ __forceinline__ float gelu_grad(float z)
{
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

__device__ __forceinline__ float ld(const Operand& o, int64_t idx)
{
    return o.bf16 ? (float)reinterpret_cast<const __bf16*>(o.p)[idx] : reinterpret_cast<const float*>(o.p)[idx];
}

__global__ __launch_bounds__(kThreads) void gemm_kernel(GemmArgs g)
{
    __shared__ __align__(16) __bf16 As[kBM][kBK + kPad];
    __shared__ __align__(16) __bf16 Bs[kBN][kBK + kPad];   // [n][k]
    __shared__ float s_red[kThreads / 64];

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int m0 = blockIdx.y * kBM, n0 = blockIdx.x * kBN;
    const int wm = wid >> 1, wn = wid & 1;
    // loader: thread t fills row t/4 of a tile, k = 8 (t%4) .. 8 (t%4) + 7
    const int lr = tid >> 2, lk = (tid & 3) * 8;

    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    for (int k0 = 0; k0 < g.K; k0 += kBK) {
        bf16x8 va, vb;
        const int m = m0 + lr, n = n0 + lr;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = k0 + lk + e;
            float x = 0.0f, y = 0.0f;
            if (m < g.M && k < g.K) x = (k == g.a.one) ? 1.0f : ld(g.a, (int64_t)m * g.a.s0 + (int64_t)k * g.a.s1);
            if (n < g.N && k < g.K) y = (n == g.b.one) ? 1.0f : ld(g.b, (int64_t)k * g.b.s0 + (int64_t)n * g.b.s1);
            va[e] = (__bf16)x;
            vb[e] = (__bf16)y;
        }
        __syncthreads();                                   // the previous tile is consumed
        *reinterpret_cast<bf16x8*>(&As[lr][lk]) = va;
        *reinterpret_cast<bf16x8*>(&Bs[lr][lk]) = vb;
        __syncthreads();
        // lane l holds row (l % 16) of A and column (l % 16) of B, k = 8 (l / 16) .. + 7
        const int fr = lane & 15, fk = (lane >> 4) * 8;
        bf16x8 fa[2], fb[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) fa[i] = *reinterpret_cast<const bf16x8*>(&As[wm * 32 + i * 16 + fr][fk]);
#pragma unroll
        for (int j = 0; j < 2; ++j) fb[j] = *reinterpret_cast<const bf16x8*>(&Bs[wn * 32 + j * 16 + fr][fk]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
    }

    // lane l holds rows 4 (l / 16) + r, r = 0..3, of column l % 16 of each 16 x 16 tile
    float sq = 0.0f;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm * 32 + i * 16 + (lane >> 4) * 4 + r;
                const int n = n0 + wn * 32 + j * 16 + (lane & 15);
                if (m >= g.M || n >= g.N) continue;
                const float v = acc[i][j][r];
                const int64_t ci = (int64_t)m * g.ldc + n;
                if (g.epi == EPI_STORE) {
                    g.c[ci] = v;
                } else if (g.epi == EPI_GELU) {
                    g.c[ci] = v;
                    g.c2[ci] = gelu(v);
                } else if (g.epi == EPI_LOSS) {
                    const float d = v - g.aux[(int64_t)m * g.ldaux + n];
                    g.c[ci] = g.scale * d;
                    sq += d * d;
                } else {
                    g.c[ci] = v * gelu_grad(g.aux[(int64_t)m * g.ldaux + n]);
                }
            }
    if (g.epi == EPI_LOSS) {
        // fixed-order reduction: lanes by butterfly, waves in order
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) sq += __shfl_xor(sq, o, 64);
        if (lane == 0) s_red[wid] = sq;
        __syncthreads();
        if (tid == 0) {
            float t = 0.0f;
            for (int w = 0; w < kThreads / 64; ++w) t += s_red[w];
            g.loss_part[blockIdx.y * gridDim.x + blockIdx.x] = t;
        }
    }
}

// sum of the loss partials in a fixed order, divided by the element count
__global__ __launch_bounds__(256) void loss_kernel(const float* part, int n, float inv_count, float* out,
                                                   float* out2)
{
    __shared__ double s[256];
    double t = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) t += (double)part[i];
    s[threadIdx.x] = t;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const float v = (float)(s[0] * (double)inv_count);
        out[0] = v;
        if (out2) out2[0] = v;
    }
}

__global__ __launch_bounds__(256) void adam_kernel(float* w, float* m, float* v, const float* grad, __bf16* wb,
                                                   int64_t n, float lr, float b1, float b2, float eps, float c1,
                                                   float c2)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = grad[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    w[i] = wi;
    wb[i] = (__bf16)wi;
}

__global__ __launch_bounds__(256) void to_bf16_kernel(const float* w, __bf16* wb, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) wb[i] = (__bf16)w[i];
}

}  // namespace

struct pic_mlp {
    std::vector<int32_t> widths;
    std::vector<int64_t> off;      // parameter offset of every layer
    int64_t P = 0;
    int32_t max_batch = 0;
    int has_alloc = 0;
    pic_allocator alloc{};
    hipStream_t stream = nullptr;
    std::vector<void*> blocks;
    float *w = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    __bf16* wb = nullptr;
    std::vector<float*> z, h;      // per hidden layer: pre-activation and activation [max_batch][width]
    float* dz[2] = {nullptr, nullptr};
    float* loss_part = nullptr;
    float* loss = nullptr;         // [1]
    int64_t max_parts = 0;
    int64_t updates = 0;
};

namespace {

void* net_alloc(pic_mlp* n, size_t bytes)
{
    bytes = (std::max<size_t>(bytes, 256) + 255) & ~(size_t)255;
    void* p = nullptr;
    if (n->has_alloc) p = n->alloc.alloc(bytes, n->alloc.user);
    else if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
    if (p) n->blocks.push_back(p);
    return p;
}

hipError_t gemm(const GemmArgs& g, hipStream_t st)
{
    const dim3 grid((unsigned)((g.N + kBN - 1) / kBN), (unsigned)((g.M + kBM - 1) / kBM));
    hipLaunchKernelGGL(gemm_kernel, grid, dim3(kThreads), 0, st, g);
    return hipGetLastError();
}

int64_t parts_for(int M, int N) { return (int64_t)((M + kBM - 1) / kBM) * ((N + kBN - 1) / kBN); }

// forward pass; `t` non-null: the last layer writes the loss gradient into dz[0]
// and the loss partials instead of the outputs
hipError_t run_forward(pic_mlp* n, int batch, const float* x, float* y, const float* t)
{
    const int L = (int)n->widths.size() - 1;
    const float* a = x;
    for (int l = 0; l < L; ++l) {
        const int ni = n->widths[l], no = n->widths[l + 1];
        GemmArgs g{};
        g.M = batch;
        g.N = no;
        g.K = ni + 1;
        g.a = Operand{a, ni, 1, 0, ni};
        g.b = Operand{n->wb + n->off[l], 1, ni + 1, 1, -1};
        g.ldc = no;
        if (l < L - 1) {
            g.epi = EPI_GELU;
            g.c = n->z[l];
            g.c2 = n->h[l];
        } else if (t) {
            g.epi = EPI_LOSS;
            g.c = n->dz[0];
            g.aux = t;
            g.ldaux = no;
            g.scale = 2.0f / ((float)batch * (float)no);
            g.loss_part = n->loss_part;
        } else {
            g.epi = EPI_STORE;
            g.c = y;
        }
        const hipError_t e = gemm(g, n->stream);
        if (e != hipSuccess) return e;
        a = (l < L - 1) ? n->h[l] : nullptr;
    }
    return hipSuccess;
}

// loss and gradient of the batch into n->loss and n->grad
hipError_t run_grad(pic_mlp* n, int batch, const float* x, const float* t, float* loss_out)
{
    const int L = (int)n->widths.size() - 1;
    hipError_t e = run_forward(n, batch, x, nullptr, t);
    if (e != hipSuccess) return e;
    const int no_last = n->widths[L];
    hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(256), 0, n->stream, n->loss_part, (int)parts_for(batch, no_last),
                       1.0f / ((float)batch * (float)no_last), n->loss, loss_out);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int cur = 0;
    for (int l = L - 1; l >= 0; --l) {
        const int ni = n->widths[l], no = n->widths[l + 1];
        const float* a = l == 0 ? x : n->h[l - 1];
        // dWa = dz^T [a 1]
        GemmArgs g{};
        g.M = no;
        g.N = ni + 1;
        g.K = batch;
        g.epi = EPI_STORE;
        g.a = Operand{n->dz[cur], 1, no, 0, -1};
        g.b = Operand{a, ni, 1, 0, ni};
        g.c = n->grad + n->off[l];
        g.ldc = ni + 1;
        if ((e = gemm(g, n->stream)) != hipSuccess) return e;
        if (l > 0) {
            // dz of the layer below = (dz W) * g'(z below)
            GemmArgs h{};
            h.M = batch;
            h.N = ni;
            h.K = no;
            h.epi = EPI_DGELU;
            h.a = Operand{n->dz[cur], no, 1, 0, -1};
            h.b = Operand{n->wb + n->off[l], ni + 1, 1, 1, -1};
            h.c = n->dz[cur ^ 1];
            h.ldc = ni;
            h.aux = n->z[l - 1];
            h.ldaux = ni;
            if ((e = gemm(h, n->stream)) != hipSuccess) return e;
            cur ^= 1;
        }
    }
    return hipSuccess;
}

bool batch_ok(const pic_mlp* n, int32_t batch) { return batch >= 1 && batch <= n->max_batch; }

}  // namespace

extern "C" {

pic_status pic_mlp_create(const int32_t* widths, int32_t n_widths, int32_t max_batch, const pic_allocator* alloc,
                          void* hip_stream, pic_mlp** out)
{
    if (!widths || !out || n_widths < 2 || n_widths > PIC_MLP_MAX_LAYERS + 1 || max_batch < 1 ||
        max_batch > (1 << 20))
        return PIC_EINVAL;
    for (int i = 0; i < n_widths; ++i)
        if (widths[i] < 1 || widths[i] > PIC_MLP_MAX_WIDTH) return PIC_EINVAL;
    if (alloc && (!alloc->alloc || !alloc->free)) return PIC_EINVAL;
    pic_mlp* n = new pic_mlp();
    n->widths.assign(widths, widths + n_widths);
    n->max_batch = max_batch;
    n->stream = (hipStream_t)hip_stream;
    if (alloc) {
        n->has_alloc = 1;
        n->alloc = *alloc;
    }
    int wmax = 0;
    for (int l = 0; l + 1 < n_widths; ++l) {
        n->off.push_back(n->P);
        n->P += (int64_t)widths[l + 1] * (widths[l] + 1);
        wmax = std::max(wmax, widths[l + 1]);
        n->max_parts = std::max(n->max_parts, parts_for(max_batch, widths[l + 1]));
    }
    bool ok = true;
    auto A = [&](size_t bytes) {
        void* p = net_alloc(n, bytes);
        ok = ok && p;
        return p;
    };
    n->w = (float*)A(4 * n->P);
    n->m = (float*)A(4 * n->P);
    n->v = (float*)A(4 * n->P);
    n->grad = (float*)A(4 * n->P);
    n->wb = (__bf16*)A(2 * n->P);
    for (int l = 0; l + 2 < n_widths; ++l) {
        n->z.push_back((float*)A(4ull * max_batch * widths[l + 1]));
        n->h.push_back((float*)A(4ull * max_batch * widths[l + 1]));
    }
    n->dz[0] = (float*)A(4ull * max_batch * wmax);
    n->dz[1] = (float*)A(4ull * max_batch * wmax);
    n->loss_part = (float*)A(4ull * n->max_parts);
    n->loss = (float*)A(4);
    if (ok) {
        ok = hipMemsetAsync(n->w, 0, 4 * n->P, n->stream) == hipSuccess &&
             hipMemsetAsync(n->m, 0, 4 * n->P, n->stream) == hipSuccess &&
             hipMemsetAsync(n->v, 0, 4 * n->P, n->stream) == hipSuccess &&
             hipMemsetAsync(n->wb, 0, 2 * n->P, n->stream) == hipSuccess &&
             hipStreamSynchronize(n->stream) == hipSuccess;
        if (!ok) {
            pic_mlp_free(n);
            return PIC_EHIP;
        }
    } else {
        pic_mlp_free(n);
        return PIC_ENOMEM;
    }
    *out = n;
    return PIC_OK;
}

int64_t pic_mlp_n_params(const pic_mlp* net) { return net ? net->P : 0; }

pic_status pic_mlp_set_params(pic_mlp* n, const float* params, int64_t count)
{
    if (!n || !params || count != n->P) return PIC_EINVAL;
    if (hipMemcpyAsync(n->w, params, 4 * n->P, hipMemcpyHostToDevice, n->stream) != hipSuccess) return PIC_EHIP;
    hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)((n->P + 255) / 256)), dim3(256), 0, n->stream, n->w, n->wb,
                       n->P);
    if (hipGetLastError() != hipSuccess) return PIC_EHIP;
    if (hipMemsetAsync(n->m, 0, 4 * n->P, n->stream) != hipSuccess ||
        hipMemsetAsync(n->v, 0, 4 * n->P, n->stream) != hipSuccess)
        return PIC_EHIP;
    n->updates = 0;
    return hipStreamSynchronize(n->stream) == hipSuccess ? PIC_OK : PIC_EHIP;
}

pic_status pic_mlp_get_params(pic_mlp* n, float* params, int64_t count)
{
    if (!n || !params || count != n->P) return PIC_EINVAL;
    if (hipMemcpyAsync(params, n->w, 4 * n->P, hipMemcpyDeviceToHost, n->stream) != hipSuccess) return PIC_EHIP;
    return hipStreamSynchronize(n->stream) == hipSuccess ? PIC_OK : PIC_EHIP;
}

pic_status pic_mlp_forward(pic_mlp* n, int32_t batch, const float* x_dev, float* y_dev)
{
    if (!n || !x_dev || !y_dev || !batch_ok(n, batch)) return PIC_EINVAL;
    return run_forward(n, batch, x_dev, y_dev, nullptr) == hipSuccess ? PIC_OK : PIC_EHIP;
}

pic_status pic_mlp_train_step(pic_mlp* n, int32_t batch, const float* x_dev, const float* t_dev, float lr,
                              float beta1, float beta2, float eps, float* loss_dev)
{
    if (!n || !x_dev || !t_dev || !batch_ok(n, batch)) return PIC_EINVAL;
    if (!(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return PIC_EINVAL;
    if (run_grad(n, batch, x_dev, t_dev, loss_dev) != hipSuccess) return PIC_EHIP;
    n->updates += 1;
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)n->updates)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)n->updates)));
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n->P + 255) / 256)), dim3(256), 0, n->stream, n->w, n->m, n->v,
                       n->grad, n->wb, n->P, lr, beta1, beta2, eps, c1, c2);
    return hipGetLastError() == hipSuccess ? PIC_OK : PIC_EHIP;
}

pic_status pic_mlp_grad(pic_mlp* n, int32_t batch, const float* x_dev, const float* t_dev, float* grad, float* loss)
{
    if (!n || !x_dev || !t_dev || !grad || !loss || !batch_ok(n, batch)) return PIC_EINVAL;
    if (run_grad(n, batch, x_dev, t_dev, nullptr) != hipSuccess) return PIC_EHIP;
    if (hipMemcpyAsync(grad, n->grad, 4 * n->P, hipMemcpyDeviceToHost, n->stream) != hipSuccess ||
        hipMemcpyAsync(loss, n->loss, 4, hipMemcpyDeviceToHost, n->stream) != hipSuccess)
        return PIC_EHIP;
    return hipStreamSynchronize(n->stream) == hipSuccess ? PIC_OK : PIC_EHIP;
}

pic_status pic_mlp_sync(pic_mlp* n)
{
    if (!n) return PIC_EINVAL;
    return hipStreamSynchronize(n->stream) == hipSuccess ? PIC_OK : PIC_EHIP;
}

void pic_mlp_free(pic_mlp* n)
{
    if (!n) return;
    (void)hipStreamSynchronize(n->stream);
    for (void* p : n->blocks) {
        if (n->has_alloc) n->alloc.free(p, n->alloc.user);
        else (void)hipFree(p);
    }
    delete n;
}

}  // extern "C"
