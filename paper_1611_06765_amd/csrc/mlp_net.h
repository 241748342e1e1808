// Device code of the warm-start network (declared in include/ccd_mlp.h):
// g(x) = W3 relu(W2 relu(W1 x + b1) + b2) + b3 on 7 inputs, width 128, and
// its antisymmetrised prediction y = (g(x) - g(x_ab) - g(x_ij) + g(x_abij))/4
// over the swaps a <-> b and i <-> j of t_ij^ab.
//
// A wave evaluates 16 input rows at once: four amplitudes times their four
// swap variants, row 4e + k.  The 128 x 128 layer runs on MFMA with W2 in LDS
// (FP32 16x16x4, or BF16 16x16x32 with FP32 accumulation).  In the FP32 form
// the 7-input layer is computed per lane straight into the A-operand layout.
// In the BF16 form it runs on MFMA too, one FP16 16x16x32 step per unit tile
// with the 7 inputs padded to K = 32 (W1 and the inputs in FP16, FP32
// accumulation; the output transposed: units by rows), and W2 is stored with
// its K dimension permuted so that each lane's accumulators are its A operand
// of the next layer without any data movement.  The last layer is a 16-lane reduction of the
// accumulator tiles, whose lane layout puts the four variants of one
// amplitude in one lane group.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mlp {

constexpr int kW = 128;      // width
constexpr int kPack = 8;     // packed features per amplitude (7 inputs + 1 spare)
constexpr int OFF_W1 = 0;                      // [128][8]
constexpr int OFF_B1 = OFF_W1 + kW * kPack;    // [128]
constexpr int OFF_W2 = OFF_B1 + kW;            // [128][128], row = output unit
constexpr int OFF_B2 = OFF_W2 + kW * kW;       // [128]
constexpr int OFF_W3 = OFF_B2 + kW;            // [128]
constexpr int OFF_B3 = OFF_W3 + kW;            // [1]
constexpr int kParams = 17800;                 // OFF_B3 + 1 rounded up to 8
constexpr int kLd32 = kW + 4;                  // LDS row stride of W2 (FP32)
constexpr int kLd16 = kW + 8;                  // LDS row stride of W2 (BF16), 16-byte rows

// feature scales
constexpr double kRho0 = 0.16;     // fm^-3
constexpr double kE0 = 100.0;      // MeV
constexpr double kVScale = 1000.0; // MeV fm^3: v and y are carried as v L^3 / kVScale

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef _Float16 h8v __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f4v mfma_f32(float a, float b, f4v c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4v mfma_bf16(bf8v a, bf8v b, f4v c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4v mfma_f16(h8v a, h8v b, f4v c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// the activation, relu(z) = max(z, 0), and its derivative (0 at z <= 0): one
// full-rate VALU operation each
__device__ __forceinline__ float act(float z) { return fmaxf(z, 0.0f); }
__device__ __forceinline__ float dact(float z) { return z > 0.0f ? 1.0f : 0.0f; }

// network inputs of swap variant k (0 identity, 1 a<->b, 2 i<->j, 3 both) from
// the packed features (rho, |q|, |q'|, eps_i, eps_j, eps_a, eps_b, v)
__device__ __forceinline__ void variant_inputs(const float* f, int k, float* x) {
    const bool sab = k == 1 || k == 3, sij = k == 2 || k == 3;
    x[0] = f[0];
    x[1] = (k == 1 || k == 2) ? f[2] : f[1];
    x[2] = sij ? f[4] : f[3];
    x[3] = sij ? f[3] : f[4];
    x[4] = sab ? f[6] : f[5];
    x[5] = sab ? f[5] : f[6];
    x[6] = (k == 1 || k == 2) ? -f[7] : f[7];
}
__device__ __forceinline__ float variant_sign(int k) { return (k == 1 || k == 2) ? -1.0f : 1.0f; }

// first-layer pre-activation of unit c for inputs x (W1 rows of 8 floats and
// b1 in LDS; two 16-byte reads per row)
__device__ __forceinline__ float layer1(const float* W1s, const float* b1s, int c, const float* x) {
    const float4 w0 = *(const float4*)&W1s[c * kPack], w1 = *(const float4*)&W1s[c * kPack + 4];
    float z = b1s[c];
    z += w0.x * x[0];
    z += w0.y * x[1];
    z += w0.z * x[2];
    z += w0.w * x[3];
    z += w1.x * x[4];
    z += w1.y * x[5];
    z += w1.z * x[6];
    return z;
}

// parameters staged in LDS; W2 as FP32 (ld kLd32) or BF16 (ld kLd16)
struct Lds {
    float* W1;   // [128][8] (BF16 form: FP16 [128][8] in the same space)
    float* b1;   // [128]
    float* b2;   // [128]
    float* W3;   // [128]
    void* W2;
};

template <bool BF16>
__host__ __device__ constexpr size_t lds_bytes() {
    return (size_t)(kW * kPack + 3 * kW) * 4 + (BF16 ? (size_t)kW * kLd16 * 2 : (size_t)kW * kLd32 * 4);
}

template <bool BF16>
__device__ __forceinline__ Lds lds_carve(char* base) {
    Lds s;
    s.W1 = (float*)base;
    s.b1 = s.W1 + kW * kPack;
    s.b2 = s.b1 + kW;
    s.W3 = s.b2 + kW;
    s.W2 = (void*)(s.W3 + kW);
    return s;
}

template <bool BF16>
__device__ __forceinline__ void lds_load(const float* __restrict__ P, const Lds& s, int tid, int nthreads) {
    for (int e = tid; e < kW * kPack; e += nthreads) {
        if constexpr (BF16) ((_Float16*)s.W1)[e] = (_Float16)P[OFF_W1 + e];
        else s.W1[e] = P[OFF_W1 + e];
    }
    for (int e = tid; e < kW; e += nthreads) {
        s.b1[e] = P[OFF_B1 + e];
        s.b2[e] = P[OFF_B2 + e];
        s.W3[e] = P[OFF_W3 + e];
    }
    for (int e = tid; e < kW * kW; e += nthreads) {
        const int n = e / kW, k = e - n * kW;
        if constexpr (BF16) {
            // stored column k = 32 st + 8 q + j holds unit 32 st + 16 (j / 4) + 4 q + j % 4
            const int st = k >> 5, q = (k >> 3) & 3, j = k & 7;
            const int u = 32 * st + 16 * (j >> 2) + 4 * q + (j & 3);
            ((__bf16*)s.W2)[n * kLd16 + k] = (__bf16)P[OFF_W2 + n * kW + u];
        } else {
            ((float*)s.W2)[n * kLd32 + k] = P[OFF_W2 + e];
        }
    }
}

// Prediction y of amplitude (lane >> 4) of a 16-row tile.  f: packed features
// of the amplitude of this lane's A-operand row, i.e. amplitude (lane & 15) >> 2.
// The result is valid in every lane of the 16-lane group.
template <bool BF16>
__device__ __forceinline__ float tile_predict(const float* f, const Lds& s, int lane) {
    const int row = lane & 15, kq = lane >> 4;
    float x[7];
    variant_inputs(f, row & 3, x);
    f4v acc[8];
#pragma unroll
    for (int ct = 0; ct < 8; ct++) acc[ct] = f4v{0.f, 0.f, 0.f, 0.f};
    if constexpr (BF16) {
        // layer 1, transposed: D[unit][row] = sum_k W1[unit][k] x_row[k].  Every
        // lane supplies W1's row 16 ct + row as A[row][8 kq .. 8 kq + 7]; the B
        // operand B[8 kq + j][row] is input j of this lane's own row in the
        // lanes of group 0 and zero in the others, so only K = 0..7 counts.
        // The lane receives units 16 ct + 4 (lane / 16) + i.
        h8v xb;
#pragma unroll
        for (int j = 0; j < 7; j++) xb[j] = kq == 0 ? (_Float16)x[j] : (_Float16)0.f;
        xb[7] = (_Float16)0.f;
        const _Float16* W1h = (const _Float16*)s.W1;
        bf8v a[4];
#pragma unroll
        for (int ct = 0; ct < 8; ct++) {
            const h8v wa = *(const h8v*)&W1h[(16 * ct + row) * kPack];
            const f4v z = mfma_f16(wa, xb, f4v{0.f, 0.f, 0.f, 0.f});
            const float4 bb = *(const float4*)&s.b1[16 * ct + 4 * kq];
            // unit 16 ct + 4 kq + i is logical K index 8 kq + 4 (ct % 2) + i of step ct / 2
            a[ct >> 1][4 * (ct & 1) + 0] = (__bf16)act(z[0] + bb.x);
            a[ct >> 1][4 * (ct & 1) + 1] = (__bf16)act(z[1] + bb.y);
            a[ct >> 1][4 * (ct & 1) + 2] = (__bf16)act(z[2] + bb.z);
            a[ct >> 1][4 * (ct & 1) + 3] = (__bf16)act(z[3] + bb.w);
        }
        const __bf16* W2 = (const __bf16*)s.W2;
#pragma unroll
        for (int st = 0; st < 4; st++) {
#pragma unroll
            for (int ct = 0; ct < 8; ct++) {
                const bf8v b = *(const bf8v*)&W2[(ct * 16 + row) * kLd16 + 32 * st + 8 * kq];
                acc[ct] = mfma_bf16(a[st], b, acc[ct]);
            }
            // keep the next step's W2 loads below this point (register pressure)
            __builtin_amdgcn_sched_barrier(0);
        }
    } else {
        const float* W2 = (const float*)s.W2;
        for (int st = 0; st < 32; st++) {
            const int c = 4 * st + kq;
            const float a = act(layer1(s.W1, s.b1, c, x));
#pragma unroll
            for (int ct = 0; ct < 8; ct++) acc[ct] = mfma_f32(a, W2[(ct * 16 + row) * kLd32 + c], acc[ct]);
        }
    }
    // accumulator lane layout: rows 4 kq + i (amplitude kq, variant i), column ct*16 + row
    float gp[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ct = 0; ct < 8; ct++) {
        const int col = ct * 16 + row;
        const float b2 = s.b2[col], w3 = s.W3[col];
#pragma unroll
        for (int i = 0; i < 4; i++) gp[i] += act(acc[ct][i] + b2) * w3;
    }
#pragma unroll
    for (int i = 0; i < 4; i++) {
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) gp[i] += __shfl_xor(gp[i], o);
    }
    return 0.25f * ((gp[0] - gp[1]) - (gp[2] - gp[3]));
}

}  // namespace mlp
