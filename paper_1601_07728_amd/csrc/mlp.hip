// Learned continued-fraction terminator: a 64 -> 256 -> 256 -> 256 -> 448 ReLU MLP that
// predicts Haydock coefficients 32..255 from the first 32 pairs (extends the recursion of
// section 3.2 so the continued fraction of eq. loss.fcn reaches depth 256 from 32 H*v).
// Forward, backward and Adam run in these kernels; the GEMMs use the gfx950 matrix
// cores (bf16 16x16x32 with FP32 accumulation, or f32 16x16x4 in the FP32 mode).
// Parameters are FP32 masters packed [W1, b1, W2, b2, W3, b3, W4, b4], W stored [in][out].
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include <cstdio>
#include "internal.h"

namespace ocean {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kLayers = 4;
constexpr int kSizes[kLayers + 1] = {64, 256, 256, 256, 448};
constexpr int kMIn = 32, kNOut = 224, kDepth = kMIn + kNOut;

__host__ __device__ constexpr int layer_offset(int l) {
    int off = 0;
    for (int i = 0; i < l; ++i) off += kSizes[i] * kSizes[i + 1] + kSizes[i + 1];
    return off;
}
constexpr int kParams = layer_offset(kLayers);

// C[M][N] = op(A)[M][K] op(B)[K][N] (+ bias[N]) (ReLU) (* (mask > 0)), FP32 in memory.
// op(A)(m, k) = ta ? A[k * lda + m] : A[m * lda + k];  op(B)(k, n) = tb ? B[n * ldb + k] : B[k * ldb + n].
// Block = 4 waves = a 32 x 32 tile; lane l = i + 16 kq.  Result register r holds row 4 kq + r.
template <bool BF16>
__global__ __launch_bounds__(256) void mlp_gemm_kernel(const float* __restrict__ A, int lda, int ta,
                                                      const float* __restrict__ B, int ldb, int tb,
                                                      float* __restrict__ C, int M, int N, int K,
                                                      const float* __restrict__ bias, int relu,
                                                      const float* __restrict__ mask) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, kq = lane >> 4;
    const int m0 = blockIdx.y * 32 + (wave >> 1) * 16;
    const int n0 = blockIdx.x * 32 + (wave & 1) * 16;
    const int row = m0 + i, col = n0 + i;
    auto ga = [&](int m, int k) -> float {
        if (m >= M || k >= K) return 0.f;
        return ta ? A[(size_t)k * lda + m] : A[(size_t)m * lda + k];
    };
    auto gb = [&](int k, int n) -> float {
        if (k >= K || n >= N) return 0.f;
        return tb ? B[(size_t)n * ldb + k] : B[(size_t)k * ldb + n];
    };
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    if constexpr (BF16) {
        for (int k0 = 0; k0 < K; k0 += 32) {
            bf16x8 av, bv;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = k0 + kq * 8 + j;
                av[j] = (__bf16)ga(row, k);
                bv[j] = (__bf16)gb(k, col);
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
        }
    } else {
        for (int k0 = 0; k0 < K; k0 += 4) {
            const int k = k0 + kq;
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ga(row, k), gb(k, col), acc, 0, 0, 0);
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int orow = m0 + 4 * kq + r, ocol = n0 + i;
        if (orow >= M || ocol >= N) continue;
        float c = acc[r];
        if (bias) c += bias[ocol];
        if (relu) c = fmaxf(c, 0.f);
        if (mask && !(mask[(size_t)orow * N + ocol] > 0.f)) c = 0.f;
        C[(size_t)orow * N + ocol] = c;
    }
}

// dY = 2 w (Y - T) / n and per-block partial sums of w (Y - T)^2 / n, with w the weight of the
// output position (e % 448), or 1 without weights
__global__ __launch_bounds__(256) void mse_grad_kernel(const float* __restrict__ Y, const float* __restrict__ T,
                                                      const float* __restrict__ W, float* __restrict__ dY,
                                                      double* __restrict__ part, long long n) {
    __shared__ double sh[256];
    double s = 0.0;
    const double inv = 1.0 / (double)n;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const float r = Y[e] - T[e];
        const double w = W ? (double)W[e % kSizes[kLayers]] : 1.0;
        dY[e] = (float)(2.0 * w * r * inv);
        s += w * (double)r * r * inv;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void sum_parts_kernel(const double* __restrict__ part, int n, double* __restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += part[i];
        *out = s;
    }
}

// db[n] = sum over rows of G[row][n] (fixed order)
__global__ __launch_bounds__(256) void colsum_kernel(const float* __restrict__ G, int rows, int N,
                                                    float* __restrict__ db) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int r = 0; r < rows; ++r) s += G[(size_t)r * N + n];
    db[n] = s;
}

__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                                                  float* __restrict__ m, float* __restrict__ v, int n,
                                                  float lr, float b1, float b2, float c1, float c2,
                                                  float eps) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float gg = g[e];
    const float mm = b1 * m[e] + (1.f - b1) * gg;
    const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    const float mh = mm / c1, vh = vv / c2;
    p[e] -= lr * mh / (sqrtf(vh) + eps);
}

// Features (and targets when the sequences are long enough) of each coefficient sequence.
__global__ __launch_bounds__(64) void encode_kernel(const double* __restrict__ a, const double* __restrict__ b,
                                                   int n_seq, int stride, float* __restrict__ x,
                                                   float* __restrict__ t, double* __restrict__ cs) {
    const int sq = blockIdx.x;
    if (sq >= n_seq) return;
    const double* as = a + (size_t)sq * stride;
    const double* bs = b + (size_t)sq * stride;
    double c = 0.0, s = 0.0;
    for (int j = 16; j < kMIn; ++j) {
        c += as[j];
        s += bs[j];
    }
    c /= 16.0;
    s /= 16.0;
    for (int j = threadIdx.x; j < kMIn; j += blockDim.x) {
        x[(size_t)sq * 64 + j] = (float)((as[j] - c) / s);
        x[(size_t)sq * 64 + kMIn + j] = (float)(bs[j] / s);
    }
    if (t && stride >= kDepth)
        for (int j = threadIdx.x; j < kNOut; j += blockDim.x) {
            t[(size_t)sq * 448 + j] = (float)((as[kMIn + j] - c) / s);
            t[(size_t)sq * 448 + kNOut + j] = (float)log(bs[kMIn + j] / s);
        }
    if (cs && threadIdx.x == 0) {
        cs[2 * sq] = c;
        cs[2 * sq + 1] = s;
    }
}

// Extended coefficients: the known 32 pairs, then the decoded prediction; valid[sq] = 0 if any
// predicted value is not finite or a predicted b is not positive.
__global__ __launch_bounds__(256) void decode_kernel(const double* __restrict__ a, const double* __restrict__ b,
                                                    int stride, const float* __restrict__ y,
                                                    const double* __restrict__ cs, int n_seq,
                                                    double* __restrict__ ae, double* __restrict__ be,
                                                    int* __restrict__ valid) {
    const int sq = blockIdx.x;
    if (sq >= n_seq) return;
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    const double c = cs[2 * sq], s = cs[2 * sq + 1];
    for (int j = threadIdx.x; j < kDepth; j += blockDim.x) {
        double av, bv;
        if (j < kMIn) {
            av = a[(size_t)sq * stride + j];
            bv = b[(size_t)sq * stride + j];
        } else {
            av = (double)y[(size_t)sq * 448 + (j - kMIn)] * s + c;
            bv = exp((double)y[(size_t)sq * 448 + kNOut + (j - kMIn)]) * s;
            if (!isfinite(av) || !isfinite(bv) || !(bv > 0.0)) atomicOr(&bad, 1);
        }
        ae[(size_t)sq * kDepth + j] = av;
        be[(size_t)sq * kDepth + j] = bv;
    }
    __syncthreads();
    if (threadIdx.x == 0) valid[sq] = bad ? 0 : 1;
}

}  // namespace
}  // namespace ocean

struct ocean_mlp_s {
    int precision;  // OCEAN_MLP_BF16 or OCEAN_MLP_FP32
    int device;
    hipStream_t stream;
    float* p = nullptr;
    float* g = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    int t = 0;
    int cap = 0;
    float* act[ocean::kLayers + 1] = {};
    float* dact[ocean::kLayers + 1] = {};
    double* part = nullptr;
    double* loss = nullptr;
    float* lw = nullptr;   // per-output loss weights [448], or NULL for 1
};

namespace ocean {
namespace {

int mlp_fail(const std::string& msg, int code) {
    set_error(msg);
    return code;
}

int mlp_hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return OCEAN_OK;
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return OCEAN_ERR_DEVICE;
}

void mlp_free_acts(ocean_mlp_s* h) {
    for (int l = 0; l <= kLayers; ++l) {
        if (h->act[l]) (void)hipFree(h->act[l]);
        if (h->dact[l]) (void)hipFree(h->dact[l]);
        h->act[l] = h->dact[l] = nullptr;
    }
    h->cap = 0;
}

int mlp_ensure(ocean_mlp_s* h, int batch) {
    if (batch <= h->cap) return OCEAN_OK;
    mlp_free_acts(h);
    for (int l = 0; l <= kLayers; ++l) {
        const size_t bytes = (size_t)batch * kSizes[l] * sizeof(float);
        if (hipMalloc((void**)&h->act[l], bytes) != hipSuccess || hipMalloc((void**)&h->dact[l], bytes) != hipSuccess) {
            (void)hipGetLastError();
            mlp_free_acts(h);
            return mlp_fail("ocean_mlp: hipMalloc failed for activations", OCEAN_ERR_OUT_OF_MEMORY);
        }
    }
    h->cap = batch;
    return OCEAN_OK;
}

hipError_t gemm_on(ocean_mlp_s* h, hipStream_t st, const float* A, int lda, int ta, const float* B, int ldb,
                   int tb, float* C, int M, int N, int K, const float* bias, int relu, const float* mask) {
    dim3 grid((N + 31) / 32, (M + 31) / 32);
    if (h->precision == OCEAN_MLP_BF16)
        mlp_gemm_kernel<true><<<grid, 256, 0, st>>>(A, lda, ta, B, ldb, tb, C, M, N, K, bias, relu, mask);
    else
        mlp_gemm_kernel<false><<<grid, 256, 0, st>>>(A, lda, ta, B, ldb, tb, C, M, N, K, bias, relu, mask);
    return hipGetLastError();
}

hipError_t gemm(ocean_mlp_s* h, const float* A, int lda, int ta, const float* B, int ldb, int tb, float* C,
                int M, int N, int K, const float* bias, int relu, const float* mask) {
    return gemm_on(h, h->stream, A, lda, ta, B, ldb, tb, C, M, N, K, bias, relu, mask);
}

// act[0] must hold the input; fills act[1..4] on stream st
int mlp_forward_on(ocean_mlp_s* h, float* const* act, int batch, hipStream_t st) {
    for (int l = 0; l < kLayers; ++l) {
        const float* W = h->p + layer_offset(l);
        const float* bias = W + kSizes[l] * kSizes[l + 1];
        const hipError_t e = gemm_on(h, st, act[l], kSizes[l], 0, W, kSizes[l + 1], 0, act[l + 1], batch,
                                     kSizes[l + 1], kSizes[l], bias, l < kLayers - 1 ? 1 : 0, nullptr);
        if (e != hipSuccess) return mlp_hip(e, "mlp forward");
    }
    return OCEAN_OK;
}

int mlp_forward(ocean_mlp_s* h, int batch) { return mlp_forward_on(h, h->act, batch, h->stream); }

// ---- fixed scratch for ocean_mlp_predict_noalloc ----------------------------------------------
// Per sequence: the encoding constants (c, s) and the activations of the five layers.  The
// array lives in every device's memory for the life of the process; host code reaches it only
// through the address hipGetSymbolAddress returns for the current device.
constexpr int kNoAllocMaxSeq = OCEAN_MLP_NOALLOC_MAX_SEQ;
constexpr size_t kActFloatsPerSeq = 64 + 3 * 256 + 448;
constexpr size_t kScratchBytes = (size_t)kNoAllocMaxSeq * (2 * sizeof(double) + kActFloatsPerSeq * sizeof(float));
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Resolve (once per device, with that device current) the device address of `scratch`.
int scratch_address(int device, void** out) {
    if (device < 0 || device >= kMaxDevices) return mlp_fail("ocean_mlp: device index out of range", OCEAN_ERR_DEVICE);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess) return mlp_fail("ocean_mlp: hipGetDevice failed", OCEAN_ERR_DEVICE);
        if (cur != device && hipSetDevice(device) != hipSuccess)
            return mlp_fail("ocean_mlp: hipSetDevice failed", OCEAN_ERR_DEVICE);
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess || p == nullptr) {
            (void)hipGetLastError();
            return mlp_fail(std::string("ocean_mlp: hipGetSymbolAddress of the fixed scratch array failed: ") +
                                hipGetErrorString(e),
                            OCEAN_ERR_DEVICE);
        }
        g_scratch_dev[device] = p;
    }
    *out = g_scratch_dev[device];
    return OCEAN_OK;
}

// Gradients of the MSE w.r.t. all parameters into h->g; loss into h->loss (device)
int mlp_backward(ocean_mlp_s* h, const float* t_dev, int batch) {
    const long long n = (long long)batch * kSizes[kLayers];
    const int nblk = 120;
    mse_grad_kernel<<<nblk, 256, 0, h->stream>>>(h->act[kLayers], t_dev, h->lw, h->dact[kLayers], h->part, n);
    sum_parts_kernel<<<1, 64, 0, h->stream>>>(h->part, nblk, h->loss);
    for (int l = kLayers - 1; l >= 0; --l) {
        const int in = kSizes[l], out = kSizes[l + 1];
        float* gW = h->g + layer_offset(l);
        float* gb = gW + in * out;
        const float* W = h->p + layer_offset(l);
        hipError_t e = gemm(h, h->act[l], in, 1, h->dact[l + 1], out, 0, gW, in, out, batch, nullptr, 0, nullptr);
        if (e != hipSuccess) return mlp_hip(e, "mlp backward");
        colsum_kernel<<<(out + 255) / 256, 256, 0, h->stream>>>(h->dact[l + 1], batch, out, gb);
        if (l > 0) {
            e = gemm(h, h->dact[l + 1], out, 0, W, out, 1, h->dact[l], batch, in, out, nullptr, 0, h->act[l]);
            if (e != hipSuccess) return mlp_hip(e, "mlp backward");
        }
    }
    return mlp_hip(hipGetLastError(), "mlp backward");
}

}  // namespace
}  // namespace ocean

using namespace ocean;

extern "C" {

int ocean_mlp_param_count(void) { return kParams; }

int ocean_mlp_create(int precision, ocean_mlp_t* out) {
    if (!out || (precision != OCEAN_MLP_BF16 && precision != OCEAN_MLP_FP32))
        return mlp_fail("ocean_mlp_create: invalid argument", OCEAN_ERR_INVALID_ARG);
    *out = nullptr;
    ocean_mlp_s* h = new (std::nothrow) ocean_mlp_s();
    if (!h) return mlp_fail("ocean_mlp_create: host allocation failed", OCEAN_ERR_OUT_OF_MEMORY);
    h->precision = precision;
    (void)hipGetDevice(&h->device);
    if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) {
        delete h;
        return mlp_fail("ocean_mlp_create: hipStreamCreate failed", OCEAN_ERR_DEVICE);
    }
    const size_t pb = (size_t)kParams * sizeof(float);
    if (hipMalloc((void**)&h->p, pb) != hipSuccess || hipMalloc((void**)&h->g, pb) != hipSuccess ||
        hipMalloc((void**)&h->m, pb) != hipSuccess || hipMalloc((void**)&h->v, pb) != hipSuccess ||
        hipMalloc((void**)&h->part, 1024 * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&h->loss, sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        ocean_mlp_destroy(h);
        return mlp_fail("ocean_mlp_create: hipMalloc failed", OCEAN_ERR_OUT_OF_MEMORY);
    }
    (void)hipMemsetAsync(h->p, 0, pb, h->stream);
    (void)hipMemsetAsync(h->m, 0, pb, h->stream);
    (void)hipMemsetAsync(h->v, 0, pb, h->stream);
    (void)hipStreamSynchronize(h->stream);
    // set-up of the allocation-free prediction path: the fixed scratch array's address on
    // this device
    void* scr = nullptr;
    if (const int rc = scratch_address(h->device, &scr); rc != OCEAN_OK) {
        ocean_mlp_destroy(h);
        return rc;
    }
    *out = h;
    return OCEAN_OK;
}

void ocean_mlp_destroy(ocean_mlp_t h) {
    if (!h) return;
    (void)hipSetDevice(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    mlp_free_acts(h);
    for (void* q : {(void*)h->p, (void*)h->g, (void*)h->m, (void*)h->v, (void*)h->part, (void*)h->loss, (void*)h->lw})
        if (q) (void)hipFree(q);
    if (h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

int ocean_mlp_set_params(ocean_mlp_t h, const float* params) {
    if (!h || !params) return mlp_fail("ocean_mlp_set_params: invalid argument", OCEAN_ERR_INVALID_ARG);
    const size_t pb = (size_t)kParams * sizeof(float);
    int rc = mlp_hip(hipMemcpyAsync(h->p, params, pb, hipMemcpyHostToDevice, h->stream), "upload");
    if (rc == OCEAN_OK) rc = mlp_hip(hipMemsetAsync(h->m, 0, pb, h->stream), "reset");
    if (rc == OCEAN_OK) rc = mlp_hip(hipMemsetAsync(h->v, 0, pb, h->stream), "reset");
    if (rc == OCEAN_OK) rc = mlp_hip(hipStreamSynchronize(h->stream), "set_params");
    h->t = 0;
    return rc;
}

int ocean_mlp_set_loss_weights(ocean_mlp_t h, const float* w) {
    if (!h) return mlp_fail("ocean_mlp_set_loss_weights: NULL handle", OCEAN_ERR_INVALID_ARG);
    if (!w) {
        if (h->lw) {
            (void)hipStreamSynchronize(h->stream);
            (void)hipFree(h->lw);
            h->lw = nullptr;
        }
        return OCEAN_OK;
    }
    for (int j = 0; j < kSizes[kLayers]; ++j)
        if (!std::isfinite(w[j]) || w[j] < 0.f)
            return mlp_fail("ocean_mlp_set_loss_weights: weights must be finite and >= 0", OCEAN_ERR_INVALID_ARG);
    (void)hipSetDevice(h->device);
    if (!h->lw && hipMalloc((void**)&h->lw, kSizes[kLayers] * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        h->lw = nullptr;
        return mlp_fail("ocean_mlp_set_loss_weights: hipMalloc failed", OCEAN_ERR_OUT_OF_MEMORY);
    }
    int rc = mlp_hip(hipMemcpyAsync(h->lw, w, kSizes[kLayers] * sizeof(float), hipMemcpyHostToDevice, h->stream),
                     "upload");
    if (rc == OCEAN_OK) rc = mlp_hip(hipStreamSynchronize(h->stream), "set_loss_weights");
    return rc;
}

int ocean_mlp_get_params(ocean_mlp_t h, float* params) {
    if (!h || !params) return mlp_fail("ocean_mlp_get_params: invalid argument", OCEAN_ERR_INVALID_ARG);
    int rc = mlp_hip(hipMemcpyAsync(params, h->p, (size_t)kParams * sizeof(float), hipMemcpyDeviceToHost, h->stream), "download");
    if (rc == OCEAN_OK) rc = mlp_hip(hipStreamSynchronize(h->stream), "get_params");
    return rc;
}

int ocean_mlp_save(ocean_mlp_t h, const char* path) {
    if (!h || !path) return mlp_fail("ocean_mlp_save: invalid argument", OCEAN_ERR_INVALID_ARG);
    std::vector<float> buf((size_t)3 * kParams);
    const size_t pb = (size_t)kParams * sizeof(float);
    int rc = mlp_hip(hipMemcpyAsync(buf.data(), h->p, pb, hipMemcpyDeviceToHost, h->stream), "download");
    if (rc == OCEAN_OK) rc = mlp_hip(hipMemcpyAsync(buf.data() + kParams, h->m, pb, hipMemcpyDeviceToHost, h->stream), "download");
    if (rc == OCEAN_OK) rc = mlp_hip(hipMemcpyAsync(buf.data() + 2 * (size_t)kParams, h->v, pb, hipMemcpyDeviceToHost, h->stream), "download");
    if (rc == OCEAN_OK) rc = mlp_hip(hipStreamSynchronize(h->stream), "save");
    if (rc != OCEAN_OK) return rc;
    FILE* f = std::fopen(path, "wb");
    if (!f) return mlp_fail(std::string("ocean_mlp_save: cannot open ") + path, OCEAN_ERR_INVALID_ARG);
    const int32_t head[4] = {1, h->precision, h->t, kParams};
    bool ok = std::fwrite("OCEANMLP", 1, 8, f) == 8 && std::fwrite(head, sizeof(int32_t), 4, f) == 4 &&
              std::fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return mlp_fail(std::string("ocean_mlp_save: write failed for ") + path, OCEAN_ERR_INVALID_ARG);
    return OCEAN_OK;
}

int ocean_mlp_load(ocean_mlp_t h, const char* path) {
    if (!h || !path) return mlp_fail("ocean_mlp_load: invalid argument", OCEAN_ERR_INVALID_ARG);
    FILE* f = std::fopen(path, "rb");
    if (!f) return mlp_fail(std::string("ocean_mlp_load: cannot open ") + path, OCEAN_ERR_INVALID_ARG);
    char magic[8];
    int32_t head[4];
    std::vector<float> buf((size_t)3 * kParams);
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "OCEANMLP", 8) == 0 &&
              std::fread(head, sizeof(int32_t), 4, f) == 4 && head[0] == 1 && head[3] == kParams &&
              head[1] == h->precision && head[2] >= 0 &&
              std::fread(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    std::fclose(f);
    if (!ok)
        return mlp_fail(std::string("ocean_mlp_load: not a checkpoint of this network and precision: ") + path,
                        OCEAN_ERR_INVALID_ARG);
    const size_t pb = (size_t)kParams * sizeof(float);
    int rc = mlp_hip(hipMemcpyAsync(h->p, buf.data(), pb, hipMemcpyHostToDevice, h->stream), "upload");
    if (rc == OCEAN_OK) rc = mlp_hip(hipMemcpyAsync(h->m, buf.data() + kParams, pb, hipMemcpyHostToDevice, h->stream), "upload");
    if (rc == OCEAN_OK) rc = mlp_hip(hipMemcpyAsync(h->v, buf.data() + 2 * (size_t)kParams, pb, hipMemcpyHostToDevice, h->stream), "upload");
    if (rc == OCEAN_OK) rc = mlp_hip(hipStreamSynchronize(h->stream), "load");
    if (rc == OCEAN_OK) h->t = head[2];
    return rc;
}

int ocean_mlp_encode(const double* a_dev, const double* b_dev, int n_seq, int stride, float* x_dev,
                     float* t_dev) {
    if (!a_dev || !b_dev || !x_dev || n_seq < 1 || stride < kMIn || (t_dev && stride < kDepth))
        return mlp_fail("ocean_mlp_encode: invalid argument", OCEAN_ERR_INVALID_ARG);
    encode_kernel<<<n_seq, 64, 0, 0>>>(a_dev, b_dev, n_seq, stride, x_dev, t_dev, nullptr);
    int rc = mlp_hip(hipGetLastError(), "encode launch");
    if (rc == OCEAN_OK) rc = mlp_hip(hipDeviceSynchronize(), "encode");
    return rc;
}

int ocean_mlp_forward(ocean_mlp_t h, const float* x_dev, int batch, float* y_dev) {
    if (!h || !x_dev || !y_dev || batch < 1) return mlp_fail("ocean_mlp_forward: invalid argument", OCEAN_ERR_INVALID_ARG);
    (void)hipSetDevice(h->device);
    int rc = mlp_ensure(h, batch);
    if (rc != OCEAN_OK) return rc;
    rc = mlp_hip(hipMemcpyAsync(h->act[0], x_dev, (size_t)batch * 64 * sizeof(float), hipMemcpyDeviceToDevice, h->stream), "copy");
    if (rc == OCEAN_OK) rc = mlp_forward(h, batch);
    if (rc == OCEAN_OK)
        rc = mlp_hip(hipMemcpyAsync(y_dev, h->act[kLayers], (size_t)batch * 448 * sizeof(float), hipMemcpyDeviceToDevice, h->stream), "copy");
    if (rc == OCEAN_OK) rc = mlp_hip(hipStreamSynchronize(h->stream), "forward");
    return rc;
}

int ocean_mlp_loss_grad(ocean_mlp_t h, const float* x_dev, const float* t_dev, int batch, double* loss,
                        float* grad) {
    if (!h || !x_dev || !t_dev || batch < 1) return mlp_fail("ocean_mlp_loss_grad: invalid argument", OCEAN_ERR_INVALID_ARG);
    (void)hipSetDevice(h->device);
    int rc = mlp_ensure(h, batch);
    if (rc != OCEAN_OK) return rc;
    rc = mlp_hip(hipMemcpyAsync(h->act[0], x_dev, (size_t)batch * 64 * sizeof(float), hipMemcpyDeviceToDevice, h->stream), "copy");
    if (rc == OCEAN_OK) rc = mlp_forward(h, batch);
    if (rc == OCEAN_OK) rc = mlp_backward(h, t_dev, batch);
    if (rc == OCEAN_OK && loss) rc = mlp_hip(hipMemcpyAsync(loss, h->loss, sizeof(double), hipMemcpyDeviceToHost, h->stream), "copy");
    if (rc == OCEAN_OK && grad)
        rc = mlp_hip(hipMemcpyAsync(grad, h->g, (size_t)kParams * sizeof(float), hipMemcpyDeviceToHost, h->stream), "copy");
    if (rc == OCEAN_OK) rc = mlp_hip(hipStreamSynchronize(h->stream), "loss_grad");
    return rc;
}

int ocean_mlp_train_step(ocean_mlp_t h, const float* x_dev, const float* t_dev, int batch, float lr,
                         double* loss) {
    if (!h || !x_dev || !t_dev || batch < 1 || !(lr > 0.f))
        return mlp_fail("ocean_mlp_train_step: invalid argument", OCEAN_ERR_INVALID_ARG);
    (void)hipSetDevice(h->device);
    int rc = mlp_ensure(h, batch);
    if (rc != OCEAN_OK) return rc;
    rc = mlp_hip(hipMemcpyAsync(h->act[0], x_dev, (size_t)batch * 64 * sizeof(float), hipMemcpyDeviceToDevice, h->stream), "copy");
    if (rc == OCEAN_OK) rc = mlp_forward(h, batch);
    if (rc == OCEAN_OK) rc = mlp_backward(h, t_dev, batch);
    if (rc != OCEAN_OK) return rc;
    h->t += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 - std::pow(b1, h->t)), c2 = (float)(1.0 - std::pow(b2, h->t));
    adam_kernel<<<(kParams + 255) / 256, 256, 0, h->stream>>>(h->p, h->g, h->m, h->v, kParams, lr, (float)b1,
                                                              (float)b2, c1, c2, 1e-8f);
    rc = mlp_hip(hipGetLastError(), "adam launch");
    if (rc == OCEAN_OK && loss) {
        rc = mlp_hip(hipMemcpyAsync(loss, h->loss, sizeof(double), hipMemcpyDeviceToHost, h->stream), "copy");
        if (rc == OCEAN_OK) rc = mlp_hip(hipStreamSynchronize(h->stream), "train_step");
    }
    return rc;
}

int ocean_mlp_predict(ocean_mlp_t h, const double* a, const double* b, int n_seq, int stride, double* a_ext,
                      double* b_ext, int* valid) {
    if (!h || !a || !b || !a_ext || !b_ext || !valid || n_seq < 1 || stride < kMIn)
        return mlp_fail("ocean_mlp_predict: invalid argument", OCEAN_ERR_INVALID_ARG);
    (void)hipSetDevice(h->device);
    int rc = mlp_ensure(h, n_seq);
    if (rc != OCEAN_OK) return rc;
    const size_t nab = (size_t)n_seq * stride, next = (size_t)n_seq * kDepth;
    char* buf = nullptr;
    const size_t bytes = nab * 16 + next * 16 + (size_t)n_seq * 16 + (size_t)n_seq * 4 + 64;
    if (hipMalloc((void**)&buf, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return mlp_fail("ocean_mlp_predict: hipMalloc failed", OCEAN_ERR_OUT_OF_MEMORY);
    }
    double* da = reinterpret_cast<double*>(buf);
    double* db = da + nab;
    double* dae = db + nab;
    double* dbe = dae + next;
    double* cs = dbe + next;
    int* dv = reinterpret_cast<int*>(cs + 2 * n_seq);
    rc = mlp_hip(hipMemcpyAsync(da, a, nab * 8, hipMemcpyHostToDevice, h->stream), "upload");
    if (rc == OCEAN_OK) rc = mlp_hip(hipMemcpyAsync(db, b, nab * 8, hipMemcpyHostToDevice, h->stream), "upload");
    if (rc == OCEAN_OK) {
        encode_kernel<<<n_seq, 64, 0, h->stream>>>(da, db, n_seq, stride, h->act[0], nullptr, cs);
        rc = mlp_hip(hipGetLastError(), "encode launch");
    }
    if (rc == OCEAN_OK) rc = mlp_forward(h, n_seq);
    if (rc == OCEAN_OK) {
        decode_kernel<<<n_seq, 256, 0, h->stream>>>(da, db, stride, h->act[kLayers], cs, n_seq, dae, dbe, dv);
        rc = mlp_hip(hipGetLastError(), "decode launch");
    }
    if (rc == OCEAN_OK) rc = mlp_hip(hipMemcpyAsync(a_ext, dae, next * 8, hipMemcpyDeviceToHost, h->stream), "download");
    if (rc == OCEAN_OK) rc = mlp_hip(hipMemcpyAsync(b_ext, dbe, next * 8, hipMemcpyDeviceToHost, h->stream), "download");
    if (rc == OCEAN_OK) rc = mlp_hip(hipMemcpyAsync(valid, dv, (size_t)n_seq * 4, hipMemcpyDeviceToHost, h->stream), "download");
    if (rc == OCEAN_OK) rc = mlp_hip(hipStreamSynchronize(h->stream), "predict");
    (void)hipFree(buf);
    return rc;
}

int ocean_mlp_predict_noalloc(ocean_mlp_t h, const double* a_dev, const double* b_dev, int n_seq, int stride,
                              double* a_ext_dev, double* b_ext_dev, int* valid_dev, void* stream) {
    if (!h || !a_dev || !b_dev || !a_ext_dev || !b_ext_dev || !valid_dev || n_seq < 1 || stride < kMIn)
        return mlp_fail("ocean_mlp_predict_noalloc: NULL argument, n_seq < 1 or stride < 32", OCEAN_ERR_INVALID_ARG);
    if (n_seq > kNoAllocMaxSeq)
        return mlp_fail("ocean_mlp_predict_noalloc: n_seq " + std::to_string(n_seq) + " exceeds the fixed scratch (" +
                            std::to_string(kNoAllocMaxSeq) + " sequences)",
                        OCEAN_ERR_INVALID_ARG);
    void* base = nullptr;
    if (const int rc = scratch_address(h->device, &base); rc != OCEAN_OK) return rc;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || (cur != h->device && hipSetDevice(h->device) != hipSuccess))
        return mlp_fail("ocean_mlp_predict_noalloc: cannot select the handle's device", OCEAN_ERR_DEVICE);
    // fixed layout: [kNoAllocMaxSeq][2] doubles, then act[0..4] each sized for kNoAllocMaxSeq
    double* cs = static_cast<double*>(base);
    float* act[kLayers + 1];
    float* f = reinterpret_cast<float*>(cs + 2 * (size_t)kNoAllocMaxSeq);
    for (int l = 0; l <= kLayers; ++l) {
        act[l] = f;
        f += (size_t)kNoAllocMaxSeq * kSizes[l];
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    encode_kernel<<<n_seq, 64, 0, st>>>(a_dev, b_dev, n_seq, stride, act[0], nullptr, cs);
    int rc = mlp_hip(hipGetLastError(), "ocean_mlp_predict_noalloc: encode launch");
    if (rc == OCEAN_OK) rc = mlp_forward_on(h, act, n_seq, st);
    if (rc == OCEAN_OK) {
        decode_kernel<<<n_seq, 256, 0, st>>>(a_dev, b_dev, stride, act[kLayers], cs, n_seq, a_ext_dev, b_ext_dev,
                                              valid_dev);
        rc = mlp_hip(hipGetLastError(), "ocean_mlp_predict_noalloc: decode launch");
    }
    if (cur != h->device) (void)hipSetDevice(cur);
    return rc;
}

}  // extern "C"
