// ccd_mlp.hip -- training and inference kernels of the warm-start network
// (include/ccd_mlp.h): forward on a feature buffer (FP32 or BF16 MFMA), loss
// and gradient (FP32 MFMA), and the Adam update of Kingma and Ba (2015),
// Algorithm 1.  Gradients are summed in a fixed order (per-block partials,
// then one reduction), so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "../../include/ccd_mlp.h"
#include "ccd_internal.h"
#include "mlp_net.h"

using namespace mlp;

namespace {

#define MLP_TRY(x)                                                                      \
    do {                                                                                \
        hipError_t e_ = (x);                                                            \
        if (e_ != hipSuccess) {                                                         \
            ccd::set_error(std::string(#x) + ": " + hipGetErrorString(e_));             \
            return CCD_EHIP;                                                            \
        }                                                                               \
    } while (0)

// ---- forward on a buffer of packed features -----------------------------------
// wave tiles of four amplitudes (16 rows); grid-stride over tiles
template <bool BF16>
__global__ void __launch_bounds__(256) k_mlp_fwd(const float* __restrict__ P, const float* __restrict__ feat,
                                                 int64_t n, float* __restrict__ y) {
    extern __shared__ __attribute__((aligned(16))) char lds[];
    const Lds s = lds_carve<BF16>(lds);
    lds_load<BF16>(P, s, threadIdx.x, 256);
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t ntile = (n + 3) / 4;
    for (int64_t t = (int64_t)blockIdx.x * 4 + w; t < ntile; t += (int64_t)gridDim.x * 4) {
        const int64_t e = 4 * t + ((lane & 15) >> 2);
        float f[kPack];
#pragma unroll
        for (int q = 0; q < kPack; q++) f[q] = e < n ? feat[e * kPack + q] : 0.0f;
        const float yp = tile_predict<BF16>(f, s, lane);
        const int64_t eo = 4 * t + (lane >> 4);
        if ((lane & 15) == 0 && eo < n) y[eo] = yp;
    }
}

// ---- loss and gradient ----------------------------------------------------------
// One block takes kEPB amplitudes of the batch in chunks of 8 (32 rows = 8
// amplitudes x 4 swap variants).  Wave w = (rt, ch): row tile rt = w / 2
// (amplitudes 4 rt .. 4 rt + 3 of the chunk) and column half ch = w % 2 of the
// 128 x 128 layer.  Per chunk:
//   h1 = relu(W1 x + b1)                      (VALU, into LDS)
//   z2 = h1 W2^T + b2, g = W3 relu(z2)        (MFMA, W2 in LDS)
//   y = sum_k sign_k g_k / 4, dL/dg_k = sign_k (y - y*) / (4 M)
//   dz2 = dg W3 relu'(z2)                     (into LDS)
//   dW2 += dz2^T h1                            (MFMA, 16 tiles per wave held in registers)
//   dh1 = dz2 W2, dz1 = dh1 relu'(z1)         (MFMA; z1 recomputed)
//   dW1 += dz1^T x, db1 += sum dz1, db2 += sum dz2, dW3 += dg^T relu(z2)
// The block's sums go to its row of the partial-gradient buffer.
constexpr int kEPB = 64;   // amplitudes per block
constexpr int kLdH = kW + 4;

__host__ __device__ constexpr size_t grad_lds_bytes() {
    return lds_bytes<false>() + (size_t)2 * 32 * kLdH * 4 + (size_t)(8 * kPack + 8 + 8 + 2 * 32) * 4;
}

// Indices of `order` outside [0, n_rows) are skipped (the amplitude counts as
// absent) and counted in *bad.
__global__ void __launch_bounds__(256) k_mlp_grad(const float* __restrict__ P, const float* __restrict__ feat,
                                                  const float* __restrict__ target, const int32_t* __restrict__ order,
                                                  int64_t base, int64_t n, int64_t n_rows, float inv_m,
                                                  float* __restrict__ work, float* __restrict__ work_loss,
                                                  int32_t* __restrict__ bad) {
    extern __shared__ __attribute__((aligned(16))) char lds[];
    const Lds s = lds_carve<false>(lds);
    float* H1 = (float*)(lds + lds_bytes<false>());  // [32][kLdH]
    float* DZ2 = H1 + 32 * kLdH;                     // [32][kLdH]
    float* Fs = DZ2 + 32 * kLdH;                     // [8][8]
    float* Ys = Fs + 8 * kPack;                      // [8]
    float* Vs = Ys + 8;                              // [8] 1 = amplitude present
    float* Gs = Vs + 8;                              // [2][32]
    const float* W2 = (const float*)s.W2;
    lds_load<false>(P, s, threadIdx.x, 256);

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, rt = w >> 1, ch = w & 1;
    const int r16 = lane & 15, kq = lane >> 4;
    const int64_t e0 = (int64_t)blockIdx.x * kEPB;
    const int ne = (int)std::min<int64_t>(kEPB, n - e0);

    f4v aW2[16];
#pragma unroll
    for (int t = 0; t < 16; t++) aW2[t] = f4v{0.f, 0.f, 0.f, 0.f};
    float aW3[4] = {0.f, 0.f, 0.f, 0.f}, aB2[4] = {0.f, 0.f, 0.f, 0.f}, aB1[4] = {0.f, 0.f, 0.f, 0.f};
    float aW1[4][7];
#pragma unroll
    for (int j = 0; j < 4; j++)
#pragma unroll
        for (int q = 0; q < 7; q++) aW1[j][q] = 0.f;
    float loss = 0.f;

    for (int cb = 0; cb * 8 < ne; cb++) {
        __syncthreads();  // previous chunk done with Fs, H1, DZ2, Gs (and W2 staged)
        if (tid < 8 * kPack) {
            const int el = tid >> 3, q = tid & 7;
            const int64_t li = e0 + cb * 8 + el;
            int64_t gi = li < n ? (order ? (int64_t)order[base + li] : base + li) : -1;
            if (li < n && (gi < 0 || gi >= n_rows)) {
                if (q == 0) atomicAdd(bad, 1);
                gi = -1;
            }
            const bool ok = gi >= 0;
            Fs[el * kPack + q] = ok ? feat[gi * kPack + q] : 0.f;
            if (q == 0) {
                Ys[el] = ok ? target[gi] : 0.f;
                Vs[el] = ok ? 1.f : 0.f;
            }
        }
        __syncthreads();
        // layer 1 into LDS: unit c, rows r = (tid >> 7) + 2 m
        {
            const int c = tid & 127;
            for (int r = tid >> 7; r < 32; r += 2) {
                float x[7];
                variant_inputs(&Fs[(r >> 2) * kPack], r & 3, x);
                H1[r * kLdH + c] = act(layer1(s.W1, s.b1, c, x));
            }
        }
        __syncthreads();
        // layer 2 and the wave's share of g
        f4v z2[4];
#pragma unroll
        for (int j = 0; j < 4; j++) z2[j] = f4v{0.f, 0.f, 0.f, 0.f};
        for (int st = 0; st < 32; st++) {
            const float a = H1[(rt * 16 + r16) * kLdH + 4 * st + kq];
#pragma unroll
            for (int j = 0; j < 4; j++)
                z2[j] = mfma_f32(a, W2[((ch * 4 + j) * 16 + r16) * kLd32 + 4 * st + kq], z2[j]);
        }
        float gp[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int col = (ch * 4 + j) * 16 + r16;
            const float b2 = s.b2[col], w3 = s.W3[col];
#pragma unroll
            for (int i = 0; i < 4; i++) {
                z2[j][i] += b2;
                gp[i] += act(z2[j][i]) * w3;
            }
        }
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) gp[i] += __shfl_xor(gp[i], o);
        if (r16 == 0)
#pragma unroll
            for (int i = 0; i < 4; i++) Gs[ch * 32 + rt * 16 + 4 * kq + i] = gp[i];
        __syncthreads();
        // residual of amplitude el = 4 rt + kq; dL/dg of its four rows
        const int el = rt * 4 + kq;
        float g[4];
#pragma unroll
        for (int i = 0; i < 4; i++) g[i] = Gs[4 * el + i] + Gs[32 + 4 * el + i];
        const float yp = 0.25f * ((g[0] - g[1]) - (g[2] - g[3]));
        const float res = Vs[el] != 0.f ? yp - Ys[el] : 0.f;
        if (ch == 0 && r16 == 0) loss += 0.5f * res * res * inv_m;
        float dg[4];
#pragma unroll
        for (int i = 0; i < 4; i++) dg[i] = variant_sign(i) * 0.25f * res * inv_m;
        // dz2, dW3, db2
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int col = (ch * 4 + j) * 16 + r16;
            const float w3 = s.W3[col];
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const float dz = dg[i] * w3 * dact(z2[j][i]);
                aW3[j] += dg[i] * act(z2[j][i]);
                aB2[j] += dz;
                DZ2[(rt * 16 + 4 * kq + i) * kLdH + col] = dz;
            }
        }
        __syncthreads();
        // dW2 += dz2^T h1: wave w owns output rows (units) n-tiles 2w, 2w+1, all k-tiles
        for (int st = 0; st < 8; st++) {
            const int r = 4 * st + kq;
            float av[2], bv[8];
#pragma unroll
            for (int u = 0; u < 2; u++) av[u] = DZ2[r * kLdH + (2 * w + u) * 16 + r16];
#pragma unroll
            for (int kt = 0; kt < 8; kt++) bv[kt] = H1[r * kLdH + kt * 16 + r16];
#pragma unroll
            for (int u = 0; u < 2; u++)
#pragma unroll
                for (int kt = 0; kt < 8; kt++) aW2[u * 8 + kt] = mfma_f32(av[u], bv[kt], aW2[u * 8 + kt]);
        }
        // dh1 = dz2 W2 for rows of tile rt, k-tiles ch*4 .. ch*4+3
        f4v dh[4];
#pragma unroll
        for (int j = 0; j < 4; j++) dh[j] = f4v{0.f, 0.f, 0.f, 0.f};
        for (int st = 0; st < 32; st++) {
            const float a = DZ2[(rt * 16 + r16) * kLdH + 4 * st + kq];
#pragma unroll
            for (int j = 0; j < 4; j++)
                dh[j] = mfma_f32(a, W2[(4 * st + kq) * kLd32 + (ch * 4 + j) * 16 + r16], dh[j]);
        }
        // dz1 = dh1 relu'(z1), rows 4 el + i (variant i of amplitude el)
        float xv[4][7];
#pragma unroll
        for (int i = 0; i < 4; i++) variant_inputs(&Fs[el * kPack], i, xv[i]);
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int c = (ch * 4 + j) * 16 + r16;
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const float dz1 = dh[j][i] * dact(layer1(s.W1, s.b1, c, xv[i]));
                aB1[j] += dz1;
#pragma unroll
                for (int q = 0; q < 7; q++) aW1[j][q] += dz1 * xv[i][q];
            }
        }
    }
    // ---- block sums -> partial-gradient row of this block
    float* out = work + (size_t)blockIdx.x * kParams;
    // lane groups kq hold partial sums over their rows: reduce over kq
#pragma unroll
    for (int j = 0; j < 4; j++) {
#pragma unroll
        for (int o = 16; o < 64; o <<= 1) {
            aW3[j] += __shfl_xor(aW3[j], o);
            aB2[j] += __shfl_xor(aB2[j], o);
            aB1[j] += __shfl_xor(aB1[j], o);
#pragma unroll
            for (int q = 0; q < 7; q++) aW1[j][q] += __shfl_xor(aW1[j][q], o);
        }
    }
    // waves rt = 1 hand their column sums to the waves rt = 0 of the same half
    __syncthreads();
    float* X = H1;  // [2 halves][4][16][10] scratch
    if (rt == 1 && kq == 0) {
#pragma unroll
        for (int j = 0; j < 4; j++) {
            float* q = X + ((ch * 4 + j) * 16 + r16) * 10;
            q[0] = aW3[j]; q[1] = aB2[j]; q[2] = aB1[j];
#pragma unroll
            for (int f = 0; f < 7; f++) q[3 + f] = aW1[j][f];
        }
    }
    __syncthreads();
    if (rt == 0 && kq == 0) {
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int col = (ch * 4 + j) * 16 + r16;
            const float* q = X + col * 10;
            out[OFF_W3 + col] = aW3[j] + q[0];
            out[OFF_B2 + col] = aB2[j] + q[1];
            out[OFF_B1 + col] = aB1[j] + q[2];
#pragma unroll
            for (int f = 0; f < 7; f++) out[OFF_W1 + col * kPack + f] = aW1[j][f] + q[3 + f];
            out[OFF_W1 + col * kPack + 7] = 0.f;
        }
    }
    // dW2 tiles of this wave: rows n = (2w+u)*16 + 4 kq + i, columns k = kt*16 + r16
#pragma unroll
    for (int u = 0; u < 2; u++)
#pragma unroll
        for (int kt = 0; kt < 8; kt++)
#pragma unroll
            for (int i = 0; i < 4; i++)
                out[OFF_W2 + ((2 * w + u) * 16 + 4 * kq + i) * kW + kt * 16 + r16] = aW2[u * 8 + kt][i];
    // b3 cancels in the antisymmetrised output; padding stays zero
    if (tid < kParams - OFF_B3) out[OFF_B3 + tid] = 0.f;
    // loss: lanes r16 == 0 of waves ch == 0 hold it
    loss += __shfl_xor(loss, 16);
    loss += __shfl_xor(loss, 32);
    __syncthreads();
    if (ch == 0 && lane == 0) Gs[rt] = loss;
    __syncthreads();
    if (tid == 0) work_loss[blockIdx.x] = Gs[0] + Gs[1];
}

// sum of the block partials (fixed order); mode 0 writes the gradient, mode 1
// applies one Adam step.  Block 0 adds the batch loss to acc[0].
__global__ void __launch_bounds__(256) k_mlp_reduce(const float* __restrict__ work, const float* __restrict__ work_loss,
                                                    int nblk, int mode, float* __restrict__ grad, float* __restrict__ P,
                                                    float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                                                    float b2, float eps, float bc1, float bc2, double* acc) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p < kParams) {
        float g = 0.f;
        for (int b = 0; b < nblk; b++) g += work[(size_t)b * kParams + p];
        if (mode == 0) {
            grad[p] = g;
        } else {
            const float mn = b1 * m[p] + (1.f - b1) * g;
            const float vn = b2 * v[p] + (1.f - b2) * g * g;
            m[p] = mn;
            v[p] = vn;
            P[p] -= lr * (mn / bc1) / (sqrtf(vn / bc2) + eps);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double l = 0.0;
        for (int b = 0; b < nblk; b++) l += (double)work_loss[b];
        acc[0] += l;
    }
}

__global__ void k_mlp_zero(double* acc, int32_t* bad) {
    acc[0] = 0.0;
    bad[0] = 0;
}

struct Work {
    float* part;
    float* loss;
    double* acc;
    int32_t* bad;   // count of out-of-range indices
};

size_t work_bytes_for(int64_t n) {
    const int64_t nblk = std::max<int64_t>(1, (n + kEPB - 1) / kEPB);
    return (size_t)nblk * kParams * 4 + (size_t)((nblk + 63) / 64) * 256 + 256;
}

Work carve(void* w, int64_t n) {
    const int64_t nblk = std::max<int64_t>(1, (n + kEPB - 1) / kEPB);
    Work k;
    k.part = (float*)w;
    k.loss = k.part + (size_t)nblk * kParams;
    k.acc = (double*)((char*)w + work_bytes_for(n) - 256);
    k.bad = (int32_t*)(k.acc + 1);
    return k;
}

ccd_status grad_attrs() {
    static bool done = false;
    if (done) return CCD_OK;
    MLP_TRY(hipFuncSetAttribute((const void*)k_mlp_grad, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)grad_lds_bytes()));
    MLP_TRY(hipFuncSetAttribute((const void*)k_mlp_fwd<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds_bytes<false>()));
    done = true;
    return CCD_OK;
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

}  // namespace

extern "C" {

ccd_status ccd_mlp_forward(const float* params, const float* feat, int64_t n, int32_t precision, float* y,
                           void* stream) {
    if (!params || (n > 0 && (!feat || !y)) || n < 0 ||
        (precision != CCD_PREC_FP32 && precision != CCD_PREC_BF16)) {
        ccd::set_error("ccd_mlp_forward: need params, feat, y, n >= 0 and precision FP32 or BF16");
        return CCD_EINVAL;
    }
    if (!aligned(params, 16) || !aligned(feat, 16)) {
        ccd::set_error("ccd_mlp_forward: params and feat must be 16-byte aligned");
        return CCD_EINVAL;
    }
    if (n == 0) return CCD_OK;
    ccd_status s = grad_attrs();
    if (s != CCD_OK) return s;
    const int64_t ntile = (n + 3) / 4;
    const int grid = (int)std::min<int64_t>((ntile + 3) / 4, 2048);
    if (precision == CCD_PREC_BF16)
        hipLaunchKernelGGL(k_mlp_fwd<true>, dim3(grid), dim3(256), lds_bytes<true>(), (hipStream_t)stream, params,
                           feat, n, y);
    else
        hipLaunchKernelGGL(k_mlp_fwd<false>, dim3(grid), dim3(256), lds_bytes<false>(), (hipStream_t)stream, params,
                           feat, n, y);
    MLP_TRY(hipGetLastError());
    return CCD_OK;
}

ccd_status ccd_mlp_work_size(int64_t n, size_t* bytes) {
    if (!bytes || n < 1) {
        ccd::set_error("ccd_mlp_work_size: need n >= 1 and bytes");
        return CCD_EINVAL;
    }
    *bytes = work_bytes_for(n);
    return CCD_OK;
}

ccd_status ccd_mlp_loss_grad(const float* params, const float* feat, const float* target, int64_t n, float* grad,
                             double* loss, void* work, size_t work_bytes, void* stream) {
    if (!params || !feat || !target || !grad || !work || n < 1) {
        ccd::set_error("ccd_mlp_loss_grad: NULL argument or n < 1");
        return CCD_EINVAL;
    }
    if (work_bytes < work_bytes_for(n) || !aligned(work, 256)) {
        ccd::set_error("ccd_mlp_loss_grad: work buffer too small or not 256-byte aligned");
        return CCD_EINVAL;
    }
    ccd_status s = grad_attrs();
    if (s != CCD_OK) return s;
    const Work k = carve(work, n);
    const int nblk = (int)((n + kEPB - 1) / kEPB);
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_mlp_zero, dim3(1), dim3(1), 0, st, k.acc, k.bad);
    hipLaunchKernelGGL(k_mlp_grad, dim3(nblk), dim3(256), grad_lds_bytes(), st, params, feat, target,
                       (const int32_t*)nullptr, (int64_t)0, n, n, 1.0f / (float)n, k.part, k.loss, k.bad);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kParams + 255) / 256), dim3(256), 0, st, k.part, k.loss, nblk, 0, grad,
                       (float*)nullptr, (float*)nullptr, (float*)nullptr, 0.f, 0.f, 0.f, 0.f, 1.f, 1.f, k.acc);
    MLP_TRY(hipGetLastError());
    if (loss) {
        MLP_TRY(hipMemcpyAsync(loss, k.acc, 8, hipMemcpyDeviceToHost, st));
        MLP_TRY(hipStreamSynchronize(st));
    }
    return CCD_OK;
}

ccd_status ccd_mlp_train(float* params, float* adam_m, float* adam_v, int64_t* step, const float* feat,
                         const float* target, int64_t n_rows, const int32_t* order, int64_t n_order,
                         const ccd_adam_opts* o, void* work, size_t work_bytes, double* mean_loss, void* stream) {
    if (!params || !adam_m || !adam_v || !step || !feat || !target || !order || !o || !work || n_rows < 1) {
        ccd::set_error("ccd_mlp_train: NULL argument or n_rows < 1");
        return CCD_EINVAL;
    }
    if (o->batch < 1 || n_order < o->batch || !(o->lr > 0.f) || !(o->beta1 >= 0.f && o->beta1 < 1.f) ||
        !(o->beta2 >= 0.f && o->beta2 < 1.f) || !(o->eps > 0.f) || *step < 0) {
        ccd::set_error("ccd_mlp_train: need 1 <= batch <= n_order, lr > 0, 0 <= beta < 1, eps > 0, step >= 0");
        return CCD_EINVAL;
    }
    if (work_bytes < work_bytes_for(o->batch) || !aligned(work, 256)) {
        ccd::set_error("ccd_mlp_train: work buffer smaller than ccd_mlp_work_size(batch) or misaligned");
        return CCD_EINVAL;
    }
    ccd_status s = grad_attrs();
    if (s != CCD_OK) return s;
    const Work k = carve(work, o->batch);
    const int nblk = (int)((o->batch + kEPB - 1) / kEPB);
    const int64_t nsteps = n_order / o->batch;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_mlp_zero, dim3(1), dim3(1), 0, st, k.acc, k.bad);
    for (int64_t q = 0; q < nsteps; q++) {
        const int64_t t = *step + 1;
        const float bc1 = (float)(1.0 - std::pow((double)o->beta1, (double)t));
        const float bc2 = (float)(1.0 - std::pow((double)o->beta2, (double)t));
        hipLaunchKernelGGL(k_mlp_grad, dim3(nblk), dim3(256), grad_lds_bytes(), st, params, feat, target, order,
                           q * o->batch, (int64_t)o->batch, n_rows, 1.0f / (float)o->batch, k.part, k.loss, k.bad);
        hipLaunchKernelGGL(k_mlp_reduce, dim3((kParams + 255) / 256), dim3(256), 0, st, k.part, k.loss, nblk, 1,
                           (float*)nullptr, params, adam_m, adam_v, o->lr, o->beta1, o->beta2, o->eps, bc1, bc2,
                           k.acc);
        MLP_TRY(hipGetLastError());
        *step = t;
    }
    double acc = 0.0;
    int32_t bad = 0;
    MLP_TRY(hipMemcpyAsync(&acc, k.acc, 8, hipMemcpyDeviceToHost, st));
    MLP_TRY(hipMemcpyAsync(&bad, k.bad, 4, hipMemcpyDeviceToHost, st));
    MLP_TRY(hipStreamSynchronize(st));
    if (mean_loss) *mean_loss = acc / (double)nsteps;
    if (bad) {
        ccd::set_error("ccd_mlp_train: " + std::to_string(bad) + " indices of order outside [0, n_rows) were skipped");
        return CCD_EINVAL;
    }
    return CCD_OK;
}

}  // extern "C"
