// Measured ceilings of the device, for the roofline of the projections: what one FP64
// matrix-core instruction stream, one FP64 multiply-add stream, one plain copy and one plain
// read reach on this part, next to the published peaks.  The projections of Algorithm 1 issue both
// instruction kinds (matrix cores for whole 16-column tiles, multiply-adds for the last
// columns), and stream u and phi through HBM.
#include "internal.h"

namespace ocean {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

// Four independent 16x16x4 FP64 accumulations per wave (operands nonzero so that the
// units see data-dependent switching, as on real inputs).
__global__ __launch_bounds__(256) void rate_mfma_f64_kernel(double* __restrict__ out, int iters) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const double a = 1.0 + 1e-9 * threadIdx.x, b = 1.0 - 1e-9 * threadIdx.x;
    v4d acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = v4d{0.25 * c, 0.5, 0.75, 1.0};
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    out[gid] = s;
}

// Eight independent FP64 multiply-add chains per lane, 32 per loop turn.
__global__ __launch_bounds__(256) void rate_fma_f64_kernel(double* __restrict__ out, int iters) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const double a = 1.0 - 1e-12 * threadIdx.x, b = 1e-3;
    double f[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) f[j] = 1e-3 * (j + threadIdx.x);
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int j = 0; j < 8; ++j) f[j] = __builtin_fma(f[j], a, b);
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += f[j];
    out[gid] = s;
}

// One 16-byte element per thread over a grid covering the array: on this part short blocks
// stream faster than grid-stride loops (measured), so this shape gives the copy ceiling.
__global__ __launch_bounds__(256) void copy16_kernel(const float4* __restrict__ src, float4* __restrict__ dst,
                                                     size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// Read-only stream: block b reads the 1024 consecutive elements [1024 b, 1024 b + 1024), four
// per thread at a stride of 256, and writes one partial sum per wave (4 per block).
__global__ __launch_bounds__(256) void read16_kernel(const float4* __restrict__ src, float* __restrict__ part,
                                                     size_t n) {
    const size_t b = (size_t)blockIdx.x * 1024 + threadIdx.x;
    float acc = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (b + 256 * j < n) {
            const float4 v = src[b + 256 * j];
            acc += (v.x + v.y) + (v.z + v.w);
        }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0) part[(size_t)blockIdx.x * 4 + (threadIdx.x >> 6)] = acc;
}

}  // namespace
}  // namespace ocean

using namespace ocean;

extern "C" int ocean_device_ceilings(long long copy_bytes, double* mfma_f64_tflops, double* fma_f64_tflops,
                                     double* copy_gbs, double* read_gbs) {
    set_error("");
    if (copy_bytes < (1ll << 20) || !mfma_f64_tflops || !fma_f64_tflops || !copy_gbs || !read_gbs) {
        set_error("ocean_device_ceilings: copy_bytes >= 1 MiB and four output pointers required");
        return OCEAN_ERR_INVALID_ARG;
    }
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) {
        (void)hipGetLastError();
        set_error("ocean_device_ceilings: no device");
        return OCEAN_ERR_DEVICE;
    }
    const int blocks = 4 * cus;   // four 4-wave blocks per CU: four waves per SIMD
    const size_t n16 = (size_t)copy_bytes / 16;
    const size_t rblocks = (n16 + 1023) / 1024;
    double* out = nullptr;
    float* part = nullptr;
    float4* src = nullptr;
    float4* dst = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = OCEAN_OK;
    auto fail = [&](int code, const char* what) {
        (void)hipGetLastError();
        set_error(std::string("ocean_device_ceilings: ") + what);
        rc = code;
    };
    if (hipMalloc((void**)&out, sizeof(double) * blocks * 256) != hipSuccess ||
        hipMalloc((void**)&src, n16 * 16) != hipSuccess || hipMalloc((void**)&dst, n16 * 16) != hipSuccess ||
        hipMalloc((void**)&part, sizeof(float) * 4 * rblocks) != hipSuccess)
        fail(OCEAN_ERR_OUT_OF_MEMORY, "hipMalloc failed");
    if (rc == OCEAN_OK && (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
                           hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        fail(OCEAN_ERR_DEVICE, "stream or event creation failed");
    // fastest of three timed launches after one untimed run; milliseconds
    auto timed = [&](auto launch, float* ms) {
        launch();
        *ms = 1e30f;
        for (int r = 0; r < 3 && rc == OCEAN_OK; ++r) {
            float t = 0.f;
            (void)hipEventRecord(e0, st);
            launch();
            (void)hipEventRecord(e1, st);
            if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess ||
                hipGetLastError() != hipSuccess)
                fail(OCEAN_ERR_DEVICE, "timed launch failed");
            else if (t < *ms)
                *ms = t;
        }
    };
    if (rc == OCEAN_OK) {
        const int it = 4000;
        float ms = 0.f;
        timed([&] { rate_mfma_f64_kernel<<<blocks, 256, 0, st>>>(out, it); }, &ms);
        // 16*16*4 multiply-adds per wave-level instruction, 4 per turn, 4 waves per block
        *mfma_f64_tflops = rc == OCEAN_OK ? (double)blocks * 4 * it * 4 * (16.0 * 16 * 4 * 2) / (ms * 1e9) : 0.0;
    }
    if (rc == OCEAN_OK) {
        const int it = 8000;
        float ms = 0.f;
        timed([&] { rate_fma_f64_kernel<<<blocks, 256, 0, st>>>(out, it); }, &ms);
        *fma_f64_tflops = rc == OCEAN_OK ? (double)blocks * 256 * it * 32 * 2.0 / (ms * 1e9) : 0.0;
    }
    if (rc == OCEAN_OK) {
        if (hipMemsetAsync(src, 0, n16 * 16, st) != hipSuccess) fail(OCEAN_ERR_DEVICE, "memset failed");
        float ms = 0.f;
        if (rc == OCEAN_OK)
            timed([&] { copy16_kernel<<<(unsigned)((n16 + 255) / 256), 256, 0, st>>>(src, dst, n16); }, &ms);
        *copy_gbs = rc == OCEAN_OK ? 2.0 * n16 * 16 / (ms * 1e6) : 0.0;   // bytes read + written
    }
    if (rc == OCEAN_OK) {
        float ms = 0.f;
        timed([&] { read16_kernel<<<(unsigned)rblocks, 256, 0, st>>>(src, part, n16); }, &ms);
        *read_gbs = rc == OCEAN_OK ? (double)n16 * 16 / (ms * 1e6) : 0.0;
    }
    if (st) (void)hipStreamSynchronize(st);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    if (out) (void)hipFree(out);
    if (src) (void)hipFree(src);
    if (dst) (void)hipFree(dst);
    if (part) (void)hipFree(part);
    return rc;
}
