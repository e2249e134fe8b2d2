// Surrogate network kernels and their C ABI (include/dybond_mlp.h).
//
// A 4 -> 128 -> 128 -> 2 perceptron trained with mean-squared error and
// Adam.  The 128 x 128 layer is a dense contraction over the minibatch, so
// it and both GEMMs of its backward pass run on the matrix cores
// (v_mfma_f32_16x16x16_bf16: bf16 operands, FP32 accumulation), one wave per
// 16 x 16 output tile; the 4-wide input layer, the 2-wide output layer, the
// bias and weight reductions over the minibatch and Adam are plain FP32
// lanes.  Reductions run over the minibatch in a fixed order, so a training
// run is reproducible bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <random>
#include <string>
#include <vector>

#include "../../include/dybond_mlp.h"

namespace {

constexpr int kIn = 4, kHid = 128, kOut = 2;
// offsets in the flat parameter vector
constexpr uint32_t kW1 = 0, kB1 = kW1 + kHid * kIn, kW2 = kB1 + kHid, kB2 = kW2 + kHid * kHid,
                   kW3 = kB2 + kHid, kB3 = kW3 + kOut * kHid, kNP = kB3 + kOut;
static_assert(kNP == DB_MLP_PARAMS, "parameter count");

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> bf16, round to nearest even (NaN kept quiet).
__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float sigmoidf_(float z) { return 1.0f / (1.0f + expf(-z)); }
__device__ __forceinline__ float siluf_(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float dsiluf_(float z) {
    const float s = sigmoidf_(z);
    return s * (1.0f + z * (1.0f - s));
}

struct Net {
    float* p;          // FP32 master parameters
    float* m;          // Adam first moments
    float* v;          // Adam second moments
    float* g;          // gradient
    uint16_t* wb;      // bf16 copy of the parameter vector (weights used; biases unused)
    // minibatch (bp rows, bp a multiple of 16) and intermediates
    float* x;          // bp x 4
    float* t;          // bp x 2
    float* z1;         // bp x 128
    uint16_t* a1b;     // bp x 128, bf16 SiLU(z1)
    float* z2;         // bp x 128
    float* a2;         // bp x 128
    float* y;          // bp x 2
    float* dz3;        // bp x 2
    float* dz2;        // bp x 128
    uint16_t* dz2b;    // bp x 128
    float* dz1;        // bp x 128
    float* loss;       // [0] loss of the last full evaluation
};

// One 16 x 16 tile of C = A B with bf16 operands and FP32 accumulation on
// the matrix cores.  A(m, k) = a[m * sam + k * sak], B(k, n) = b[k * sbk + n * sbn]
// for m, n < 16 (tile origin folded into the pointers) and k < K (a
// multiple of 16).  Lane l supplies A(l % 16, 4 (l / 16) + j) and
// B(4 (l / 16) + j, l % 16), j = 0..3, and receives C(4 (l / 16) + j, l % 16).
__device__ __forceinline__ f32x4 mfma_tile(const uint16_t* a, int sam, int sak, const uint16_t* b, int sbk,
                                           int sbn, int K) {
    const int l = (int)(threadIdx.x & 63u);
    const int r = l & 15, kq = (l >> 4) * 4;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 16) {
        bf16x4 av, bv;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            av[j] = (short)a[r * sam + (k0 + kq + j) * sak];
            bv[j] = (short)b[(k0 + kq + j) * sbk + r * sbn];
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
    }
    return acc;
}

// bf16 copies of the three weight matrices (biases are read in FP32).
__global__ void k_mlp_round(Net N) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < kNP) N.wb[k] = to_bf16(N.p[k]);
}

// rows [0, bp) of the minibatch gathered from the full data set by index
// (rows at or past nb are zero inputs whose outputs are ignored)
__global__ void k_mlp_gather(Net N, const float* __restrict__ X, const float* __restrict__ Tt,
                             const uint32_t* __restrict__ idx, uint32_t nb, uint32_t bp) {
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= bp) return;
    const uint32_t r = b < nb ? idx[b] : 0u;
#pragma unroll
    for (int k = 0; k < kIn; ++k) N.x[b * kIn + k] = b < nb ? X[(size_t)r * kIn + k] : 0.0f;
    if (Tt)
#pragma unroll
        for (int k = 0; k < kOut; ++k) N.t[b * kOut + k] = b < nb ? Tt[(size_t)r * kOut + k] : 0.0f;
}

// layer 1: z1 = W1 x + b1, a1 = SiLU(z1) rounded to bf16
__global__ void k_mlp_fwd1(Net N, uint32_t bp) {
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= bp * kHid) return;
    const uint32_t b = e / kHid, h = e % kHid;
    float z = N.p[kB1 + h];
#pragma unroll
    for (int k = 0; k < kIn; ++k) z = fmaf(from_bf16(N.wb[kW1 + h * kIn + k]), N.x[b * kIn + k], z);
    N.z1[e] = z;
    N.a1b[e] = to_bf16(siluf_(z));
}

// layer 2 on the matrix cores: z2(b, h) = sum_k a1(b, k) W2(h, k) + b2(h);
// one wave per 16 x 16 tile of (b, h)
__global__ void k_mlp_fwd2(Net N, uint32_t bp) {
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t ntn = kHid / 16;
    if (wave >= (bp / 16) * ntn) return;
    const uint32_t bm = (wave / ntn) * 16, hn = (wave % ntn) * 16;
    const f32x4 acc = mfma_tile(N.a1b + bm * kHid, kHid, 1, N.wb + kW2 + hn * kHid, 1, kHid, kHid);
    const int l = (int)(threadIdx.x & 63u);
    const uint32_t h = hn + (l & 15);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t b = bm + (l >> 4) * 4 + j;
        const float z = acc[j] + N.p[kB2 + h];
        N.z2[b * kHid + h] = z;
        N.a2[b * kHid + h] = siluf_(z);
    }
}

// layer 3: y = sigmoid(W3 a2 + b3); with targets, dz3 = dL/dz3 for the
// mean-squared error over the nb valid rows
__global__ void k_mlp_fwd3(Net N, uint32_t bp, uint32_t nb, int with_grad) {
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= bp * kOut) return;
    const uint32_t b = e / kOut, o = e % kOut;
    float z = N.p[kB3 + o];
    for (int h = 0; h < kHid; ++h) z = fmaf(from_bf16(N.wb[kW3 + o * kHid + h]), N.a2[b * kHid + h], z);
    const float y = sigmoidf_(z);
    N.y[e] = y;
    if (with_grad) {
        const float dy = b < nb ? 2.0f * (y - N.t[e]) / (float)(nb * kOut) : 0.0f;
        N.dz3[e] = dy * y * (1.0f - y);
    }
}

// mean-squared error of the nb valid rows (one workgroup, fixed order)
__global__ __launch_bounds__(256) void k_mlp_loss(Net N, uint32_t nb) {
    __shared__ float part[256];
    float s = 0.0f;
    for (uint32_t e = threadIdx.x; e < nb * kOut; e += 256) {
        const float d = N.y[e] - N.t[e];
        s = fmaf(d, d, s);
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) N.loss[0] = part[0] / (float)(nb * kOut);
}

// back through layer 3: dz2 = (dz3 W3) * SiLU'(z2), kept in FP32 and bf16
__global__ void k_mlp_bwd3(Net N, uint32_t bp) {
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= bp * kHid) return;
    const uint32_t b = e / kHid, h = e % kHid;
    float da = 0.0f;
#pragma unroll
    for (int o = 0; o < kOut; ++o) da = fmaf(N.dz3[b * kOut + o], from_bf16(N.wb[kW3 + o * kHid + h]), da);
    const float dz = da * dsiluf_(N.z2[e]);
    N.dz2[e] = dz;
    N.dz2b[e] = to_bf16(dz);
}

// parameter gradients that reduce over the minibatch in FP32, one thread
// per parameter: W3, b3, b2 (and, after the layer-2 GEMMs, W1, b1)
__global__ void k_mlp_grad3(Net N, uint32_t bp) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < kOut * kHid) {                                // dW3(o, h) = sum_b dz3(b, o) a2(b, h)
        const uint32_t o = k / kHid, h = k % kHid;
        float s = 0.0f;
        for (uint32_t b = 0; b < bp; ++b) s = fmaf(N.dz3[b * kOut + o], N.a2[b * kHid + h], s);
        N.g[kW3 + k] = s;
    } else if (k < kOut * kHid + kOut) {                  // db3
        const uint32_t o = k - kOut * kHid;
        float s = 0.0f;
        for (uint32_t b = 0; b < bp; ++b) s += N.dz3[b * kOut + o];
        N.g[kB3 + o] = s;
    } else if (k < kOut * kHid + kOut + kHid) {           // db2
        const uint32_t h = k - kOut * kHid - kOut;
        float s = 0.0f;
        for (uint32_t b = 0; b < bp; ++b) s += N.dz2[b * kHid + h];
        N.g[kB2 + h] = s;
    }
}

// both GEMMs of layer 2's backward pass on the matrix cores, one wave per
// 16 x 16 tile: waves [0, 64) make dW2(h, k) = sum_b dz2(b, h) a1(b, k);
// the rest make da1(b, k) = sum_h dz2(b, h) W2(h, k), then
// dz1 = da1 * SiLU'(z1)
__global__ void k_mlp_bwd2(Net N, uint32_t bp) {
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t ntn = kHid / 16;
    const int l = (int)(threadIdx.x & 63u);
    if (wave < ntn * ntn) {
        const uint32_t hm = (wave / ntn) * 16, kn = (wave % ntn) * 16;
        const f32x4 acc = mfma_tile(N.dz2b + hm, 1, kHid, N.a1b + kn, kHid, 1, (int)bp);
        const uint32_t k = kn + (l & 15);
#pragma unroll
        for (int j = 0; j < 4; ++j) N.g[kW2 + (hm + (l >> 4) * 4 + j) * kHid + k] = acc[j];
        return;
    }
    const uint32_t w2 = wave - ntn * ntn;
    if (w2 >= (bp / 16) * ntn) return;
    const uint32_t bm = (w2 / ntn) * 16, kn = (w2 % ntn) * 16;
    const f32x4 acc = mfma_tile(N.dz2b + bm * kHid, kHid, 1, N.wb + kW2 + kn, kHid, 1, kHid);
    const uint32_t k = kn + (l & 15);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t b = bm + (l >> 4) * 4 + j;
        N.dz1[b * kHid + k] = acc[j] * dsiluf_(N.z1[b * kHid + k]);
    }
}

// dW1(h, k) = sum_b dz1(b, h) x(b, k), db1(h) = sum_b dz1(b, h)
__global__ void k_mlp_grad1(Net N, uint32_t bp) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < kHid * kIn) {
        const uint32_t h = k / kIn, c = k % kIn;
        float s = 0.0f;
        for (uint32_t b = 0; b < bp; ++b) s = fmaf(N.dz1[b * kHid + h], N.x[b * kIn + c], s);
        N.g[kW1 + k] = s;
    } else if (k < kHid * kIn + kHid) {
        const uint32_t h = k - kHid * kIn;
        float s = 0.0f;
        for (uint32_t b = 0; b < bp; ++b) s += N.dz1[b * kHid + h];
        N.g[kB1 + h] = s;
    }
}

// Adam on the FP32 master parameters (Kingma & Ba, bias-corrected), then
// the bf16 copy; c1 = 1 - beta1^t, c2 = 1 - beta2^t
__global__ void k_mlp_adam(Net N, float lr, float c1, float c2) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kNP) return;
    const float g = N.g[k];
    const float m = 0.9f * N.m[k] + 0.1f * g;
    const float v = 0.999f * N.v[k] + 0.001f * g * g;
    N.m[k] = m;
    N.v[k] = v;
    const float p = N.p[k] - lr * (m / c1) / (sqrtf(v / c2) + 1e-8f);
    N.p[k] = p;
    N.wb[k] = to_bf16(p);
}

}  // namespace

struct db_mlp {
    int device = 0;
    hipStream_t stream = nullptr;
    uint32_t bmax = 0;           // rows per minibatch, multiple of 16
    uint64_t adam_t = 0;
    Net N{};
    std::vector<void*> allocs;
    std::string err;
    float* dX = nullptr;         // training set on the device
    float* dT = nullptr;
    uint32_t* dIdx = nullptr;
    uint64_t cap_rows = 0;
};

namespace {

db_status mfail(db_mlp* s, db_status st, const char* fmt, ...) {
    if (s) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        s->err = buf;
    }
    return st;
}

#define MCHK(s, call)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess) return mfail((s), DB_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

template <class T>
db_status malloc_n(db_mlp* s, T*& p, size_t n) {
    void* q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess)
        return mfail(s, DB_ENOMEM, "device allocation of %zu bytes failed", n * sizeof(T));
    s->allocs.push_back(q);
    p = static_cast<T*>(q);
    return DB_OK;
}

#define MALLOC(s, p, n)                               \
    do {                                              \
        db_status st_ = malloc_n((s), (p), (n));      \
        if (st_ != DB_OK) return st_;                 \
    } while (0)

inline unsigned blocks(uint64_t n, unsigned bs) { return (unsigned)((n + bs - 1) / bs); }

// forward (and, with targets, backward) over the bp-row minibatch already in N.x / N.t
void run_pass(db_mlp* s, uint32_t nb, bool grad) {
    const uint32_t bp = (nb + 15u) & ~15u;
    Net& N = s->N;
    hipLaunchKernelGGL(k_mlp_fwd1, dim3(blocks((uint64_t)bp * kHid, 256)), dim3(256), 0, s->stream, N, bp);
    hipLaunchKernelGGL(k_mlp_fwd2, dim3(blocks((uint64_t)(bp / 16) * (kHid / 16) * 64, 256)), dim3(256), 0,
                       s->stream, N, bp);
    hipLaunchKernelGGL(k_mlp_fwd3, dim3(blocks((uint64_t)bp * kOut, 256)), dim3(256), 0, s->stream, N, bp, nb,
                       grad ? 1 : 0);
    if (!grad) return;
    hipLaunchKernelGGL(k_mlp_bwd3, dim3(blocks((uint64_t)bp * kHid, 256)), dim3(256), 0, s->stream, N, bp);
    hipLaunchKernelGGL(k_mlp_grad3, dim3(blocks(kOut * kHid + kOut + kHid, 256)), dim3(256), 0, s->stream, N, bp);
    const uint64_t waves = (uint64_t)(kHid / 16) * (kHid / 16) + (uint64_t)(bp / 16) * (kHid / 16);
    hipLaunchKernelGGL(k_mlp_bwd2, dim3(blocks(waves * 64, 256)), dim3(256), 0, s->stream, N, bp);
    hipLaunchKernelGGL(k_mlp_grad1, dim3(blocks(kHid * kIn + kHid, 256)), dim3(256), 0, s->stream, N, bp);
}

db_status upload_rows(db_mlp* s, const float* x, const float* t, uint64_t n) {
    if (n > s->cap_rows) {
        for (void* q : {(void*)s->dX, (void*)s->dT, (void*)s->dIdx}) {
            auto it = std::find(s->allocs.begin(), s->allocs.end(), q);
            if (it != s->allocs.end()) {
                (void)hipFree(q);
                s->allocs.erase(it);
            }
        }
        s->dX = nullptr;
        s->dT = nullptr;
        s->dIdx = nullptr;
        s->cap_rows = 0;
        MALLOC(s, s->dX, n * kIn);
        MALLOC(s, s->dT, n * kOut);
        MALLOC(s, s->dIdx, n);
        s->cap_rows = n;
    }
    MCHK(s, hipMemcpyAsync(s->dX, x, n * kIn * sizeof(float), hipMemcpyHostToDevice, s->stream));
    if (t) MCHK(s, hipMemcpyAsync(s->dT, t, n * kOut * sizeof(float), hipMemcpyHostToDevice, s->stream));
    return DB_OK;
}

bool finite_rows(const float* a, uint64_t count) {
    for (uint64_t k = 0; k < count; ++k)
        if (!std::isfinite(a[k])) return false;
    return true;
}

}  // namespace

extern "C" {

db_status db_mlp_create(uint32_t batch_max, int device, db_mlp** out) {
    if (!out) return DB_EINVAL;
    *out = nullptr;
    if (batch_max < 1 || batch_max > 4096) return DB_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        return DB_EDEVICE;
    }
    db_mlp* s = new db_mlp();
    s->device = device;
    s->bmax = (batch_max + 15u) & ~15u;
    auto bad = [&](db_status st) {
        db_mlp_destroy(s);
        return st;
    };
    if (hipSetDevice(device) != hipSuccess || hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess)
        return bad(DB_EDEVICE);
    Net& N = s->N;
    const size_t b = s->bmax;
    db_status st = DB_OK;
    auto A = [&](auto*& p, size_t n) { if (st == DB_OK) st = malloc_n(s, p, n); };
    A(N.p, kNP); A(N.m, kNP); A(N.v, kNP); A(N.g, kNP); A(N.wb, kNP);
    A(N.x, b * kIn); A(N.t, b * kOut); A(N.z1, b * kHid); A(N.a1b, b * kHid); A(N.z2, b * kHid);
    A(N.a2, b * kHid); A(N.y, b * kOut); A(N.dz3, b * kOut); A(N.dz2, b * kHid); A(N.dz2b, b * kHid);
    A(N.dz1, b * kHid); A(N.loss, 1);
    if (st != DB_OK) return bad(st);
    for (void* q : {(void*)N.p, (void*)N.m, (void*)N.v, (void*)N.g})
        if (hipMemsetAsync(q, 0, kNP * sizeof(float), s->stream) != hipSuccess) return bad(DB_EDEVICE);
    if (hipMemsetAsync(N.wb, 0, kNP * sizeof(uint16_t), s->stream) != hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess)
        return bad(DB_EDEVICE);
    *out = s;
    return DB_OK;
}

void db_mlp_destroy(db_mlp* s) {
    if (!s) return;
    (void)hipSetDevice(s->device);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (void* q : s->allocs) (void)hipFree(q);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

db_status db_mlp_set_params(db_mlp* s, const float* params, uint64_t count) {
    if (!s || !params) return DB_EINVAL;
    if (count != kNP) return mfail(s, DB_EINVAL, "expected %u parameters, got %llu", kNP, (unsigned long long)count);
    MCHK(s, hipSetDevice(s->device));
    MCHK(s, hipMemcpyAsync(s->N.p, params, kNP * sizeof(float), hipMemcpyHostToDevice, s->stream));
    MCHK(s, hipMemsetAsync(s->N.m, 0, kNP * sizeof(float), s->stream));
    MCHK(s, hipMemsetAsync(s->N.v, 0, kNP * sizeof(float), s->stream));
    hipLaunchKernelGGL(k_mlp_round, dim3(blocks(kNP, 256)), dim3(256), 0, s->stream, s->N);
    MCHK(s, hipGetLastError());
    MCHK(s, hipStreamSynchronize(s->stream));
    s->adam_t = 0;
    return DB_OK;
}

db_status db_mlp_get_params(db_mlp* s, float* params, uint64_t count) {
    if (!s || !params) return DB_EINVAL;
    if (count != kNP) return mfail(s, DB_EINVAL, "expected %u parameters, got %llu", kNP, (unsigned long long)count);
    MCHK(s, hipSetDevice(s->device));
    MCHK(s, hipMemcpyAsync(params, s->N.p, kNP * sizeof(float), hipMemcpyDeviceToHost, s->stream));
    MCHK(s, hipStreamSynchronize(s->stream));
    return DB_OK;
}

db_status db_mlp_predict(db_mlp* s, const float* x, uint64_t n, float* y) {
    if (!s || (!x && n) || (!y && n)) return DB_EINVAL;
    if (n == 0) return DB_OK;
    if (!finite_rows(x, n * kIn)) return mfail(s, DB_EINVAL, "non-finite input");
    MCHK(s, hipSetDevice(s->device));
    db_status st = upload_rows(s, x, nullptr, n);
    if (st != DB_OK) return st;
    std::vector<uint32_t> idx(s->bmax);
    for (uint64_t r0 = 0; r0 < n; r0 += s->bmax) {
        const uint32_t nb = (uint32_t)std::min<uint64_t>(s->bmax, n - r0);
        for (uint32_t k = 0; k < nb; ++k) idx[k] = (uint32_t)(r0 + k);
        MCHK(s, hipMemcpyAsync(s->dIdx, idx.data(), nb * sizeof(uint32_t), hipMemcpyHostToDevice, s->stream));
        const uint32_t bp = (nb + 15u) & ~15u;
        hipLaunchKernelGGL(k_mlp_gather, dim3(blocks(bp, 256)), dim3(256), 0, s->stream, s->N, s->dX,
                           (const float*)nullptr, s->dIdx, nb, bp);
        run_pass(s, nb, false);
        MCHK(s, hipGetLastError());
        MCHK(s, hipMemcpyAsync(y + r0 * kOut, s->N.y, nb * kOut * sizeof(float), hipMemcpyDeviceToHost, s->stream));
        MCHK(s, hipStreamSynchronize(s->stream));
    }
    return DB_OK;
}

db_status db_mlp_loss_grad(db_mlp* s, const float* x, const float* t, uint32_t n, float* loss, float* grad) {
    if (!s || !x || !t || !loss || !grad) return DB_EINVAL;
    if (n < 1 || n > s->bmax) return mfail(s, DB_EINVAL, "n must be in [1, %u]", s->bmax);
    if (!finite_rows(x, (uint64_t)n * kIn) || !finite_rows(t, (uint64_t)n * kOut))
        return mfail(s, DB_EINVAL, "non-finite input or target");
    MCHK(s, hipSetDevice(s->device));
    db_status st = upload_rows(s, x, t, n);
    if (st != DB_OK) return st;
    std::vector<uint32_t> idx(n);
    std::iota(idx.begin(), idx.end(), 0u);
    MCHK(s, hipMemcpyAsync(s->dIdx, idx.data(), n * sizeof(uint32_t), hipMemcpyHostToDevice, s->stream));
    const uint32_t bp = (n + 15u) & ~15u;
    hipLaunchKernelGGL(k_mlp_gather, dim3(blocks(bp, 256)), dim3(256), 0, s->stream, s->N, s->dX, s->dT, s->dIdx,
                       n, bp);
    run_pass(s, n, true);
    hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(256), 0, s->stream, s->N, n);
    MCHK(s, hipGetLastError());
    MCHK(s, hipMemcpyAsync(grad, s->N.g, kNP * sizeof(float), hipMemcpyDeviceToHost, s->stream));
    MCHK(s, hipMemcpyAsync(loss, s->N.loss, sizeof(float), hipMemcpyDeviceToHost, s->stream));
    MCHK(s, hipStreamSynchronize(s->stream));
    return DB_OK;
}

db_status db_mlp_train(db_mlp* s, const float* x, const float* t, uint64_t n, uint32_t batch, uint32_t epochs,
                       float lr, uint64_t seed, float* final_loss) {
    if (!s || !x || !t) return DB_EINVAL;
    if (n < 1 || n > 0xFFFFFFFFull) return mfail(s, DB_EINVAL, "n out of range");
    if (batch < 1 || batch > s->bmax) return mfail(s, DB_EINVAL, "batch must be in [1, %u]", s->bmax);
    if (!(lr > 0.0f) || !std::isfinite(lr)) return mfail(s, DB_EINVAL, "learning rate must be positive");
    if (!finite_rows(x, n * kIn) || !finite_rows(t, n * kOut)) return mfail(s, DB_EINVAL, "non-finite input or target");
    MCHK(s, hipSetDevice(s->device));
    db_status st = upload_rows(s, x, t, n);
    if (st != DB_OK) return st;
    std::mt19937_64 gen(seed);
    std::vector<uint32_t> perm(n);
    std::iota(perm.begin(), perm.end(), 0u);
    for (uint32_t ep = 0; ep < epochs; ++ep) {
        for (uint64_t k = n - 1; k > 0; --k) std::swap(perm[k], perm[gen() % (k + 1)]);
        MCHK(s, hipMemcpyAsync(s->dIdx, perm.data(), n * sizeof(uint32_t), hipMemcpyHostToDevice, s->stream));
        for (uint64_t r0 = 0; r0 < n; r0 += batch) {
            const uint32_t nb = (uint32_t)std::min<uint64_t>(batch, n - r0);
            const uint32_t bp = (nb + 15u) & ~15u;
            hipLaunchKernelGGL(k_mlp_gather, dim3(blocks(bp, 256)), dim3(256), 0, s->stream, s->N, s->dX, s->dT,
                               s->dIdx + r0, nb, bp);
            run_pass(s, nb, true);
            ++s->adam_t;
            const float c1 = (float)(1.0 - std::pow(0.9, (double)s->adam_t));
            const float c2 = (float)(1.0 - std::pow(0.999, (double)s->adam_t));
            hipLaunchKernelGGL(k_mlp_adam, dim3(blocks(kNP, 256)), dim3(256), 0, s->stream, s->N, lr, c1, c2);
        }
        MCHK(s, hipGetLastError());
        // the host copies the next epoch's order into the index buffer: wait for this one
        MCHK(s, hipStreamSynchronize(s->stream));
    }
    if (final_loss) {
        // mean-squared error over all rows, batch_max rows at a time
        double acc = 0.0;
        std::vector<uint32_t> idx(s->bmax);
        for (uint64_t r0 = 0; r0 < n; r0 += s->bmax) {
            const uint32_t nb = (uint32_t)std::min<uint64_t>(s->bmax, n - r0);
            for (uint32_t k = 0; k < nb; ++k) idx[k] = (uint32_t)(r0 + k);
            MCHK(s, hipMemcpyAsync(s->dIdx, idx.data(), nb * sizeof(uint32_t), hipMemcpyHostToDevice, s->stream));
            const uint32_t bp = (nb + 15u) & ~15u;
            hipLaunchKernelGGL(k_mlp_gather, dim3(blocks(bp, 256)), dim3(256), 0, s->stream, s->N, s->dX, s->dT,
                               s->dIdx, nb, bp);
            run_pass(s, nb, false);
            hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(256), 0, s->stream, s->N, nb);
            float l = 0.0f;
            MCHK(s, hipMemcpyAsync(&l, s->N.loss, sizeof(float), hipMemcpyDeviceToHost, s->stream));
            MCHK(s, hipStreamSynchronize(s->stream));
            acc += (double)l * nb;
        }
        *final_loss = (float)(acc / (double)n);
    }
    return DB_OK;
}

const char* db_mlp_last_error(const db_mlp* s) { return s ? s->err.c_str() : "null handle"; }

}  // extern "C"
