// ccd_ceil.hip -- measured ceilings of the GPU: HBM copy bandwidth and the
// matrix-core rates the kernels of this library use (FP64 16x16x4 and 4x4x4,
// FP32 16x16x4, BF16 16x16x32), each from a resident loop with several
// independent accumulators per wave and three workgroups per compute unit.
// The roofline of a kernel is stated against the published peak; these
// figures say what this part reaches in practice.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>

#include "ccd_internal.h"

namespace {

typedef double d4c __attribute__((ext_vector_type(4)));
typedef float f4c __attribute__((ext_vector_type(4)));
typedef __bf16 bf8c __attribute__((ext_vector_type(8)));

constexpr int kIters = 2000;

// one copy pass: 16-byte vectors, grid-stride
__global__ void __launch_bounds__(256) k_copy(const double2* __restrict__ src, double2* __restrict__ dst, size_t n) {
    for (size_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) dst[i] = src[i];
}

template <int KIND>
__global__ void __launch_bounds__(256) k_mfma(double* out, int iters) {
    const double x = 1e-3 * (threadIdx.x + 1), y = 2e-3;
    double acc = 0.0;
    if constexpr (KIND == 0) {  // FP64 16x16x4
        d4c a0 = {0, 0, 0, 0}, a1 = a0, a2 = a0, a3 = a0;
        for (int i = 0; i < iters; i++) {
            a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, a0, 0, 0, 0);
            a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, a1, 0, 0, 0);
            a2 = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, a2, 0, 0, 0);
            a3 = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, a3, 0, 0, 0);
        }
        const d4c s = a0 + a1 + a2 + a3;
        acc = s[0] + s[1] + s[2] + s[3];
    } else if constexpr (KIND == 1) {  // FP64 4x4x4, four blocks
        double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
        for (int i = 0; i < iters; i++) {
            a0 = __builtin_amdgcn_mfma_f64_4x4x4f64(x, y, a0, 0, 0, 0);
            a1 = __builtin_amdgcn_mfma_f64_4x4x4f64(x, y, a1, 0, 0, 0);
            a2 = __builtin_amdgcn_mfma_f64_4x4x4f64(x, y, a2, 0, 0, 0);
            a3 = __builtin_amdgcn_mfma_f64_4x4x4f64(x, y, a3, 0, 0, 0);
        }
        acc = a0 + a1 + a2 + a3;
    } else if constexpr (KIND == 2) {  // FP32 16x16x4
        f4c a0 = {0, 0, 0, 0}, a1 = a0, a2 = a0, a3 = a0;
        const float xf = (float)x, yf = (float)y;
        for (int i = 0; i < iters; i++) {
            a0 = __builtin_amdgcn_mfma_f32_16x16x4f32(xf, yf, a0, 0, 0, 0);
            a1 = __builtin_amdgcn_mfma_f32_16x16x4f32(xf, yf, a1, 0, 0, 0);
            a2 = __builtin_amdgcn_mfma_f32_16x16x4f32(xf, yf, a2, 0, 0, 0);
            a3 = __builtin_amdgcn_mfma_f32_16x16x4f32(xf, yf, a3, 0, 0, 0);
        }
        const f4c s = a0 + a1 + a2 + a3;
        acc = (double)(s[0] + s[1] + s[2] + s[3]);
    } else {  // BF16 16x16x32
        bf8c xb, yb;
        for (int j = 0; j < 8; j++) { xb[j] = (__bf16)(float)x; yb[j] = (__bf16)(float)y; }
        f4c a0 = {0, 0, 0, 0}, a1 = a0, a2 = a0, a3 = a0;
        for (int i = 0; i < iters; i++) {
            a0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xb, yb, a0, 0, 0, 0);
            a1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xb, yb, a1, 0, 0, 0);
            a2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xb, yb, a2, 0, 0, 0);
            a3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xb, yb, a3, 0, 0, 0);
        }
        const f4c s = a0 + a1 + a2 + a3;
        acc = (double)(s[0] + s[1] + s[2] + s[3]);
    }
    out[blockIdx.x * 256 + threadIdx.x] = acc;
}

// flops of one instruction of each kind
constexpr double kFlops[4] = {2.0 * 16 * 16 * 4, 4 * 2.0 * 4 * 4 * 4, 2.0 * 16 * 16 * 4, 2.0 * 16 * 16 * 32};

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    ~Timer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

#define CEIL_TRY(x)                                                                      \
    do {                                                                                 \
        hipError_t e_ = (x);                                                             \
        if (e_ != hipSuccess) {                                                          \
            ccd::set_error(std::string("ccd_measure_ceilings: ") + hipGetErrorString(e_)); \
            return CCD_EHIP;                                                             \
        }                                                                                \
    } while (0)

}  // namespace

extern "C" ccd_status ccd_measure_ceilings(void* dev_buf, size_t bytes, void* hip_stream, double* out) {
    if (!dev_buf || !out || (((uintptr_t)dev_buf) & 255)) {
        ccd::set_error("ccd_measure_ceilings: need a 256-byte aligned device buffer and out[5]");
        return CCD_EINVAL;
    }
    int dev = 0, ncu = 0;
    CEIL_TRY(hipGetDevice(&dev));
    CEIL_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    const size_t need_mfma = (size_t)3 * ncu * 256 * sizeof(double);
    if (bytes < need_mfma || bytes < ((size_t)64 << 20)) {
        ccd::set_error("ccd_measure_ceilings: the buffer must hold at least 64 MiB");
        return CCD_EINVAL;
    }
    hipStream_t s = (hipStream_t)hip_stream;
    Timer t;
    CEIL_TRY(hipEventCreate(&t.a));
    CEIL_TRY(hipEventCreate(&t.b));
    float ms = 0.0f;
    // HBM: copy one half of the buffer onto the other, read + write bytes counted
    const size_t n2 = (bytes / 2) / sizeof(double2);
    const double2* src = (const double2*)dev_buf;
    double2* dst = (double2*)dev_buf + n2;
    const int cgrid = ncu * 8;
    k_copy<<<cgrid, 256, 0, s>>>(src, dst, n2);
    CEIL_TRY(hipGetLastError());
    CEIL_TRY(hipEventRecord(t.a, s));
    for (int r = 0; r < 5; r++) k_copy<<<cgrid, 256, 0, s>>>(src, dst, n2);
    CEIL_TRY(hipGetLastError());
    CEIL_TRY(hipEventRecord(t.b, s));
    CEIL_TRY(hipEventSynchronize(t.b));
    CEIL_TRY(hipEventElapsedTime(&ms, t.a, t.b));
    out[0] = 5.0 * 2.0 * (double)n2 * sizeof(double2) / (ms * 1e-3) / 1e9;
    // matrix cores: three workgroups of four waves per compute unit
    double* o = (double*)dev_buf;
    const int grid = 3 * ncu;
    for (int kind = 0; kind < 4; kind++) {
        auto launch = [&](int iters) {
            switch (kind) {
                case 0: k_mfma<0><<<grid, 256, 0, s>>>(o, iters); break;
                case 1: k_mfma<1><<<grid, 256, 0, s>>>(o, iters); break;
                case 2: k_mfma<2><<<grid, 256, 0, s>>>(o, iters); break;
                default: k_mfma<3><<<grid, 256, 0, s>>>(o, iters); break;
            }
        };
        launch(kIters / 10);
        CEIL_TRY(hipGetLastError());
        CEIL_TRY(hipEventRecord(t.a, s));
        launch(kIters);
        CEIL_TRY(hipGetLastError());
        CEIL_TRY(hipEventRecord(t.b, s));
        CEIL_TRY(hipEventSynchronize(t.b));
        CEIL_TRY(hipEventElapsedTime(&ms, t.a, t.b));
        const double instr = (double)grid * 4 /* waves */ * kIters * 4 /* chains */;
        out[1 + kind] = instr * kFlops[kind] / (ms * 1e-3) / 1e12;
    }
    return CCD_OK;
}
