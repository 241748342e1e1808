// ccd_device.hip -- gfx950 kernels of the CCD sweep and the C ABI around them.
//
// One Jacobi sweep of eq. ccd3 in the intermediates form (sec. "Developing a
// CCD code for infinite matter"), every term from the current amplitudes t:
//   k_direct  per S_z = 0 block: the parts of 1/2 sum_cd <kl||cd> t_ij^cd
//   k_dsum    (MFMA), and the row / column sums of t <ab||ij>; k_dsum adds the
//             parts and <kl||ij> into chi_klij
//   k_dchi    one-body intermediates, diagonal by momentum conservation:
//             chi_bb - f_bb = -1/2 sum_kld t_kl^bd <kl||bd>,
//             chi_jj - f_jj = +1/2 sum_cdl <jl||cd> t_jl^cd
//   k_ringp   per pair {Q, -Q} of cross channels: gather T~_Q, generate the
//             interaction blocks, the two ring terms of every amplitude in three
//             MFMA products in LDS, stored to the amplitude's ring slots
//   k_ladder  per S_z = 0 block, 128-pair and 16-column tile: pp ladder
//             1/2 sum_cd <ab||cd> t_ij^cd as a product over the block's momentum
//             pairs {p, K - p} on MFMA, the interaction generated in registers
//             from W(m), plus the hh ladder 1/2 sum_kl t_kl^ab chi_klij
//             (k_ladder64 in FP64)
//   k_update  every amplitude: <ab||ij> + ladder sums + ring slots + one-body
//             terms, t_new = R / eps_ij^ab, linear mixing, energy partial sums
//   k_energy  deterministic per-problem energy and convergence flag (inside a
//             run of sweeps: the last blocks of the next sweep's k_direct)
// Problems with the same (N, nmax2, twist) form a group that shares the integer
// tables (states, pair lists, position maps, work lists); the sweep kernels'
// work items are (item, problem) pairs over them, and the work lists are cut
// per XCD by problem so each XCD's L2 sees about one problem's amplitudes.
// Reductions are fixed-order trees (no floating-point atomics): energies are
// bit-identical from run to run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <thread>
#include <tuple>
#include <type_traits>
#include <vector>

#include "ccd_internal.h"
#include "mlp_net.h"
#include "../../include/ccd_mlp.h"

using namespace ccd;

namespace ccd {
static thread_local std::string g_err;
void set_error(const std::string& m) { g_err = m; }
}  // namespace ccd

#define HIP_TRY(x)                                                                      \
    do {                                                                                \
        hipError_t e_ = (x);                                                            \
        if (e_ != hipSuccess) {                                                         \
            set_error(std::string(#x) + ": " + hipGetErrorString(e_));                  \
            return CCD_EHIP;                                                            \
        }                                                                               \
    } while (0)

typedef double d4 __attribute__((ext_vector_type(4)));

// D = A B + C for 16x16x4 FP64 tiles.  Lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; it receives D[l/16 + 4r][l%16], r = 0..3.
__device__ __forceinline__ d4 mfma64(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// Four independent 4x4x4 FP64 products (blocks q = 0..3).  Lane l supplies
// A_q[i][k] and B_q[k][j] at l = 16k + 4q + i (resp. + j) and receives
// D_q[i][j] at l = 16i + 4q + j.  With the rows of a 16-row tile as 4q + i, the
// A operand is laid out as for mfma64 (row l%16, k = l/16); every block takes
// the same 4-column group of B (column l%4), and lane l receives row
// 4 ((l%16)/4) + l/16, column l%4.  Narrow column groups waste 4x less than
// 16-column tiles, and the instruction itself runs faster per flop.
__device__ __forceinline__ double mfma4(double a, double b, double c) {
    return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}


// Mixed precision: FP32 operands on the 16x16x4 FP32 MFMA, or BF16 operands on
// the 16x16x32 BF16 MFMA, both accumulating in FP32.  For both, lane l
// receives D[4 (l/16) + r][l%16].  BF16: lane l supplies A[l%16][8 (l/16) + j]
// and B[8 (l/16) + j][l%16], j = 0..7.
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ f4 mfma32(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfmabf(bf8 a, bf8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
enum Prec { P_F64 = 0, P_F32 = 1, P_BF16 = 2 };
template <int P> struct AccT { using T = f4; using E = float; };
template <> struct AccT<P_F64> { using T = d4; using E = double; };
// row of accumulator element r held by lane l (16x16 output tile)
template <int P> __device__ __forceinline__ int orow(int lane, int r) {
    return P == P_F64 ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r;
}

// --------------------------------------------------------------------------
// device pointers, passed by value to every kernel
// --------------------------------------------------------------------------
struct DevPtrs {
    const int32_t* st;       // packed states (per group structure)
    const double* eps;       // Fock energies (per problem)
    const double* lut;       // W(m)/2 (per problem)
    const DevGroup* groups;
    const DevChan* chans;
    const DevPh* ph;
    const int32_t* hh;       // packed pairs (per structure)
    const int32_t* pp;
    const int32_t* phst;     // per member (p, h) of a cross channel: the packed states of p and h
    const int32_t* phmap;
    const int32_t* csr_ptr;
    const int32_t* csr_idx;
    const int32_t* zs;       // per pair-block position: ring slot << 1 | sign, or -1 (shared by a group)
    const double* rowE;      // per particle-pair row: eps_a + eps_b (per problem)
    const double* colE;      // per hole-pair column: eps_i + eps_j (per problem)
    const int32_t* pgrp;     // per problem: group
    const int32_t* pgi;      // per problem: index inside the group
    const double* pscale;    // per problem: rho, 2 pi / L, L^3 / 1000 (network features)
    const Item* it_elem;     // elementwise items, all channels
    const Item* it_ladder;   // ladder items over momentum pairs (S_z = 0)
    const int32_t* it_sz0;   // S_z = 0 channel ids
    const Item* it_dchi;     // (group, first state)
    const Item* it_dsub;     // (S_z = 0 channel, first row) of the chi_klij product items
    const Item* it_direct;   // (product item, problem in group)
    const Item* it_dsum;     // (S_z = 0 channel, problem in group)
    const Item* it_ring_s;   // (primary cross channel with n <= 16, problem in group)
    const Item* it_ring_b;   // (primary cross channel with n > 16, problem in group)
    const Item* it_lg;       // (ladder item, problem in group)
    const int4* lpinfo;      // per momentum pair {p, q} of an S_z = 0 block: (p as int8 x, y, z, 0;
                             // |p|^2 | |q|^2 << 10; row of (p up, q down); row of (p down, q up)), -1 = none
    const Item* it_ue;       // (elementwise item, problem in group): the update
    double* t[2];
    double* vt;              // <ab||ij>
    double* chh;
    double* dpart;           // partial chi_klij per product item
    double* dcolp;           // partial column sums per product item
    double* rowsum;
    double* colsum;
    double* dchi;
    double* zc;              // ring result: two slots per amplitude, canonical order
    double* rowX;            // per row: one-body intermediates of a and b
    double* colX;            // per column: one-body intermediates of i and j
    double* rmm;             // ladder sums of the S_z = 0 amplitudes (t layout)
    double* epart_elem;
    double* ecorr;
    double* eprev;
    int32_t* active;
    int32_t* sweeps;
    double* ehist;           // per problem: energies of the last kHistCap sweeps (ring)
    double* dprev;           // per problem: |dE| of the previous sweep (0 = none yet)
    int32_t* streak;         // per problem: consecutive sweeps that passed the tail test
};

constexpr int kHistCap = 64;  // sweeps between two host reads of the energy history

// --------------------------------------------------------------------------
// small device helpers
// --------------------------------------------------------------------------
__device__ __forceinline__ int s_x(int32_t s) { return (int)(int8_t)(s & 0xff); }
__device__ __forceinline__ int s_y(int32_t s) { return (int)(int8_t)((s >> 8) & 0xff); }
__device__ __forceinline__ int s_z(int32_t s) { return (int)(int8_t)((s >> 16) & 0xff); }
__device__ __forceinline__ int s_s(int32_t s) { return s >> 24; }
__device__ __forceinline__ int pa(int32_t p) { return p & 0xffff; }
__device__ __forceinline__ int pb(int32_t p) { return (int)((uint32_t)p >> 16); }

__device__ __forceinline__ int dist2(int32_t a, int32_t b) {
    int x = s_x(a) - s_x(b), y = s_y(a) - s_y(b), z = s_z(a) - s_z(b);
    return x * x + y * y + z * z;
}

// <pq||rs> for a momentum-conserving quadruple of packed states; lut holds W/2.
__device__ __forceinline__ double vas(const double* __restrict__ lut, int32_t p, int32_t q,
                                      int32_t r, int32_t s) {
    int sp = s_s(p), sq = s_s(q), sr = s_s(r), ss = s_s(s);
    int f = (int)(sp == sr && sq == ss) - (int)(sp == ss && sq == sr);
    if (f == 0) return 0.0;
    double w = lut[dist2(p, r)] + lut[dist2(p, s)];
    return f > 0 ? w : -w;
}

// The same element when |n_p - n_r|^2 is known to be a constant of the block
// (every ring element: p, r are the hole and particle of one member of a cross
// channel Q, so |n_p - n_r|^2 = |Q|^2), with wr = W(|Q|^2)/2 read once.
__device__ __forceinline__ double vas_q(const double* __restrict__ lut, double wr, int32_t p, int32_t q,
                                        int32_t r, int32_t s) {
    int sp = s_s(p), sq = s_s(q), sr = s_s(r), ss = s_s(s);
    int f = (int)(sp == sr && sq == ss) - (int)(sp == ss && sq == sr);
    if (f == 0) return 0.0;
    double w = wr + lut[dist2(p, s)];
    return f > 0 ? w : -w;
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// deterministic sum over a 256-thread block; result valid in thread 0
__device__ __forceinline__ double block_sum256(double v, double* sh) {
    v = wave_sum(v);
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    return r;
}

// --------------------------------------------------------------------------
// set-up kernels
// --------------------------------------------------------------------------

// <ab||ij>, t0 = <ab||ij> / eps_ij^ab (eq. ccdGuess), energy partials
__global__ void __launch_bounds__(256) k_init(DevPtrs d, int cur, int only) {
    __shared__ double sh[4];
    const int item = blockIdx.x;
    const Item it = d.it_elem[item];
    const DevChan c = d.chans[it.chan];
    const DevGroup G = d.groups[c.group];
    const int nel = c.nhh * c.npp;
    const int32_t* st = d.st + G.st_off;
    for (int g = 0; g < G.G; g++) {
        if (only >= 0 && G.p0 + g != only) continue;
        const double* eps = d.eps + G.eps_base + g * G.ns;
        const double* lut = d.lut + G.lut_base + g * G.nlut;
        const int64_t E0 = G.t_base + g * G.n_amp + c.t_off;
        double es = 0.0;
        for (int k = 0; k < kElemChunk / 256; k++) {
            int e = it.start + threadIdx.x + 256 * k;
            if (e < nel && e < it.start + kElemChunk) {
                int r = e / c.nhh, col = e - r * c.nhh;
                int32_t ab = d.pp[c.pp_off + r], ij = d.hh[c.hh_off + col];
                int a = pa(ab), b = pb(ab), i = pa(ij), j = pb(ij);
                double v = vas(lut, st[a], st[b], st[i], st[j]);
                double t0 = v / (eps[i] + eps[j] - eps[a] - eps[b]);
                d.vt[E0 + e] = v;
                d.t[cur][E0 + e] = t0;
                es += v * t0;
            }
        }
        double s = block_sum256(es, sh);
        if (threadIdx.x == 0) d.epart_elem[G.eelem_base + g * (G.elem_hi - G.elem_lo) + (item - G.elem_lo)] = s;
    }
}

// energy partials sum v t of the current amplitudes per elementwise item
__global__ void __launch_bounds__(256) k_dot(DevPtrs d, int cur) {
    __shared__ double sh[4];
    const int item = blockIdx.x;
    const Item it = d.it_elem[item];
    const DevChan c = d.chans[it.chan];
    const DevGroup G = d.groups[c.group];
    const int nel = c.nhh * c.npp;
    for (int g = 0; g < G.G; g++) {
        const int64_t E0 = G.t_base + g * G.n_amp + c.t_off;
        double es = 0.0;
        for (int k = 0; k < kElemChunk / 256; k++) {
            int e = it.start + threadIdx.x + 256 * k;
            if (e < nel && e < it.start + kElemChunk) es += d.vt[E0 + e] * d.t[cur][E0 + e];
        }
        double s = block_sum256(es, sh);
        if (threadIdx.x == 0) d.epart_elem[G.eelem_base + g * (G.elem_hi - G.elem_lo) + (item - G.elem_lo)] = s;
    }
}

// per-problem energy from the elementwise partials; sets ecorr = eprev
__global__ void __launch_bounds__(256) k_energy_elem(DevPtrs d) {
    __shared__ double sh[4];
    const int p = blockIdx.x;
    const DevGroup G = d.groups[d.pgrp[p]];
    const int g = d.pgi[p], n = G.elem_hi - G.elem_lo;
    const double* part = d.epart_elem + G.eelem_base + g * n;
    double s = 0.0;
    for (int x = threadIdx.x; x < n; x += 256) s += part[x];
    double e = block_sum256(s, sh);
    if (threadIdx.x == 0) { d.ecorr[p] = e; d.eprev[p] = e; }
}

// --------------------------------------------------------------------------
// learned warm start: features and prediction of the amplitude network
// --------------------------------------------------------------------------

// packed features of canonical amplitude e of channel c, problem g of group G
// (rho, |q|, |q'|, eps_i, eps_j, eps_a, eps_b scaled, v L^3 / 1000), and the
// FP64 quantities of the decoding t = (v + y / s) / D
__device__ __forceinline__ void amp_features(const DevPtrs& d, const DevChan& c, const DevGroup& G, int g, int e,
                                             float* f, double& D, double& v, double& sc) {
    const int r = e / c.nhh, col = e - r * c.nhh;
    const int32_t ab = d.pp[c.pp_off + r], ij = d.hh[c.hh_off + col];
    const int a = pa(ab), b = pb(ab), i = pa(ij), j = pb(ij);
    const int32_t* st = d.st + G.st_off;
    const int32_t sa = st[a], sb = st[b], si = st[i], sj = st[j];
    const double* eps = d.eps + G.eps_base + g * G.ns;
    const int slot = G.p0 + g;
    const double rho = d.pscale[3 * slot], ku = d.pscale[3 * slot + 1];
    sc = d.pscale[3 * slot + 2];
    // twice the transfers, in units of 2 pi / L
    const int qx = s_x(sa) - s_x(sb) - s_x(si) + s_x(sj), qy = s_y(sa) - s_y(sb) - s_y(si) + s_y(sj),
              qz = s_z(sa) - s_z(sb) - s_z(si) + s_z(sj);
    const int px = s_x(sb) - s_x(sa) - s_x(si) + s_x(sj), py = s_y(sb) - s_y(sa) - s_y(si) + s_y(sj),
              pz = s_z(sb) - s_z(sa) - s_z(si) + s_z(sj);
    v = d.vt[G.t_base + g * G.n_amp + c.t_off + e];
    D = eps[i] + eps[j] - eps[a] - eps[b];
    f[0] = (float)(rho / mlp::kRho0);
    f[1] = (float)(0.5 * ku * sqrt((double)(qx * qx + qy * qy + qz * qz)));
    f[2] = (float)(0.5 * ku * sqrt((double)(px * px + py * py + pz * pz)));
    f[3] = (float)(eps[i] / mlp::kE0);
    f[4] = (float)(eps[j] / mlp::kE0);
    f[5] = (float)(eps[a] / mlp::kE0);
    f[6] = (float)(eps[b] / mlp::kE0);
    f[7] = (float)(v * sc);
}

// features (and targets y* = (t D - v) s of the current amplitudes) of one
// problem, canonical order; one block per elementwise item of its group
__global__ void __launch_bounds__(256) k_features(DevPtrs d, int cur, int gi, int g, float* feat, float* target) {
    const DevGroup G = d.groups[gi];
    const Item it = d.it_elem[G.elem_lo + blockIdx.x];
    const DevChan c = d.chans[it.chan];
    const int nel = c.nhh * c.npp;
    for (int k = 0; k < kElemChunk / 256; k++) {
        const int e = it.start + threadIdx.x + 256 * k;
        if (e < nel && e < it.start + kElemChunk) {
            float f[mlp::kPack];
            double D, v, sc;
            amp_features(d, c, G, g, e, f, D, v, sc);
            const int64_t loc = c.t_off + e;
            float4* o = (float4*)(feat + loc * mlp::kPack);
            o[0] = make_float4(f[0], f[1], f[2], f[3]);
            o[1] = make_float4(f[4], f[5], f[6], f[7]);
            if (target) {
                const double t = d.t[cur][G.t_base + g * G.n_amp + loc];
                target[loc] = (float)((t * D - v) * sc);
            }
        }
    }
}

// warm start of every problem: per (elementwise item, problem), chunks of 256
// amplitudes: every thread gathers the features of one amplitude into LDS
// (the table loads of a whole chunk in flight at once), then the wave tiles of
// four amplitudes go through the network (W2 staged once per block) and the
// decoded amplitudes replace the current ones
constexpr int kWarmChunk = 256;  // amplitudes per feature chunk (one per thread)
template <bool BF16> __host__ __device__ constexpr size_t warm_lds() {
    return mlp::lds_bytes<BF16>() + (size_t)kWarmChunk * (mlp::kPack * 4 + 16);
}
template <bool BF16>
__global__ void __launch_bounds__(256, 3) k_warm(DevPtrs d, int cur, const float* __restrict__ P, int n_items,
                                                int max_g) {
    extern __shared__ __attribute__((aligned(16))) char lds[];
    const mlp::Lds s = mlp::lds_carve<BF16>(lds);
    float* Fs = (float*)(lds + mlp::lds_bytes<BF16>());    // [kWarmChunk][kPack] features
    double* Ds = (double*)(Fs + kWarmChunk * mlp::kPack);  // [kWarmChunk] eps_ij^ab
    double* Vs = Ds + kWarmChunk;                          // [kWarmChunk] <ab||ij>
    mlp::lds_load<BF16>(P, s, threadIdx.x, 256);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, kq = lane >> 4;
    // work units (elementwise item, problem of its group), max_g problem slots per item
    for (int wi = blockIdx.x; wi < n_items * max_g; wi += gridDim.x) {
        const int bi = wi / max_g, g = wi - bi * max_g;
        const Item it = d.it_elem[bi];
        const DevChan c = d.chans[it.chan];
        const DevGroup G = d.groups[c.group];
        if (g >= G.G) continue;
        const int nel = c.nhh * c.npp;
        const int lim = min(nel, it.start + kElemChunk);
        const double sc = d.pscale[3 * (G.p0 + g) + 2];
        double* tout = d.t[cur] + G.t_base + g * G.n_amp + c.t_off;
        for (int c0 = it.start; c0 < lim; c0 += kWarmChunk) {
            const int n = min(kWarmChunk, lim - c0);
            __syncthreads();  // the previous chunk's reads of LDS are done
            {
                float f[mlp::kPack];
                double D = 1.0, v = 0.0, scx;
#pragma unroll
                for (int q = 0; q < mlp::kPack; q++) f[q] = 0.f;
                if ((int)threadIdx.x < n) amp_features(d, c, G, g, c0 + threadIdx.x, f, D, v, scx);
                float4* fw = (float4*)&Fs[threadIdx.x * mlp::kPack];
                fw[0] = make_float4(f[0], f[1], f[2], f[3]);
                fw[1] = make_float4(f[4], f[5], f[6], f[7]);
                Ds[threadIdx.x] = D;
                Vs[threadIdx.x] = v;
            }
            __syncthreads();
            // wave w: amplitudes 64 w .. 64 w + 63 of the chunk, four per tile
            for (int a0 = 64 * w; a0 < min(n, 64 * w + 64); a0 += 4) {
                const float4* fr = (const float4*)&Fs[(a0 + ((lane & 15) >> 2)) * mlp::kPack];
                const float4 f0 = fr[0], f1 = fr[1];
                const float f[mlp::kPack] = {f0.x, f0.y, f0.z, f0.w, f1.x, f1.y, f1.z, f1.w};
                const float y = mlp::tile_predict<BF16>(f, s, lane);
                // lane 20 kq: A-operand row 4 kq, i.e. amplitude kq of the tile, variant 0
                const int o = a0 + kq;
                if ((lane & 15) == 4 * kq && o < n) tout[c0 + o] = (Vs[o] + (double)y / sc) / Ds[o];
            }
        }
    }
}

// --------------------------------------------------------------------------
// sweep kernels
// --------------------------------------------------------------------------
// per-problem energy after a sweep, convergence test, divergence flag (block p
// of k_energy, or the last blocks of the next sweep's k_direct launch)
// rule 0: stop when |dE_n| < tol + tol_rel |E_n| (the paper's test); rule 1:
// the geometric-tail estimate |dE_n| r / (1 - r), r = |dE_n / dE_(n-1)|, of the
// remaining change must also be below the same threshold (r < 1), in two
// consecutive sweeps (a turning point of E_n makes one |dE| small)
__device__ __forceinline__ void energy_of(const DevPtrs& d, int p, double tol, double tol_rel, int rule, double* sh) {
    const DevGroup G = d.groups[d.pgrp[p]];
    const int g = d.pgi[p], n = G.elem_hi - G.elem_lo;
    const double* part = d.epart_elem + G.eelem_base + g * n;
    double s = 0.0;
    for (int x = threadIdx.x; x < n; x += 256) s += part[x];
    double e = block_sum256(s, sh);
    if (threadIdx.x == 0 && d.active[p]) {
        double old = d.ecorr[p];
        d.eprev[p] = old;
        d.ecorr[p] = e;
        d.ehist[(size_t)p * kHistCap + d.sweeps[p] % kHistCap] = e;
        d.sweeps[p] += 1;
        if (!isfinite(e)) d.active[p] = 0;
        else if (tol > 0.0 || tol_rel > 0.0) {
            const double de = fabs(e - old), thr = tol + tol_rel * fabs(e), dp = d.dprev[p];
            bool stop = de < thr;
            if (rule == 1) {
                const double r = dp > 0.0 ? de / dp : 1.0;
                const bool pass = stop && r < 1.0 && de * r < thr * (1.0 - r);
                d.streak[p] = pass ? d.streak[p] + 1 : 0;
                stop = d.streak[p] >= 2;
            }
            if (stop) d.active[p] = 0;
        }
        d.dprev[p] = fabs(e - old);
    }
}


// per (item of kDirSplit particle-pair rows of an S_z = 0 channel, problem):
// row sums of t v, the item's part of 1/2 sum_cd <kl||cd> t_ij^cd on MFMA over
// LDS-staged chunks of rows (FP64 in LDS, converted at the MFMA in the mixed
// modes), and its part of the column sums (the diagonal of that product in
// FP64; summed from the staged chunk in the mixed modes).  Both operands are
// amplitude-shaped blocks ([n_pp][n_hh] rows of <ab||ij> and t).  The staging
// row stride follows the channel's tiles, so narrow channels stage more rows
// per barrier.  With at most four 16x16 output tiles (n_hh <= 32) every wave
// computes all tiles over every fourth 4-row K step of a chunk and the four
// partial tiles are added in LDS in wave order; with more tiles wave w owns
// tiles w, w+4, ...  k_dsum adds the items' parts in item order.
constexpr int kDirBuf = 2048;  // doubles per staged operand
template <int P>
__global__ void __launch_bounds__(256) k_direct(DevPtrs d, int cur, uint32_t mask, int n_items, int nd, int energy,
                                                double tol, double tol_rel, int rule) {
    using E = double;
    using AT = typename std::conditional<P == P_F64, d4, f4>::type;
    constexpr int PM = P == P_F64 ? P_F64 : P_F32;   // contraction precision used here
    __shared__ __attribute__((aligned(16))) E vs[kDirBuf];
    __shared__ __attribute__((aligned(16))) E ts[kDirBuf];
    __shared__ AT red[3][64];  // partial tiles of waves 1..3
    __shared__ int live_s;
    // blocks nd .. nd + P - 1 (energy set): the previous sweep's energy step,
    // one problem each; it only reads the previous update's partial sums
    if (energy && (int)blockIdx.x >= nd) {
        energy_of(d, blockIdx.x - nd, tol, tol_rel, rule, vs);
        return;
    }
    for (int bi = blockIdx.x; bi < n_items; bi += nd) {
    const Item it = d.it_direct[bi];
    if (it.chan < 0) continue;
    const Item sub = d.it_dsub[it.chan];
    const DevChan c = d.chans[sub.chan];
    const DevGroup G = d.groups[c.group];
    const int g = it.start;
    // the problem's flag, read once for the block: an energy block of this
    // launch may clear it meanwhile, and waves that read it at different
    // times would otherwise take different paths through the barriers below
    __syncthreads();  // the previous item's readers of live_s are done
    if (threadIdx.x == 0) live_s = d.active[G.p0 + g];
    __syncthreads();
    if (!live_s) continue;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nhh = c.nhh, npp = c.npp, nt = (nhh + 15) >> 4, ntt = nt * nt;
    const int ld = nt * 16 + 1;                    // staging row stride
    const int crows = (kDirBuf / ld) & ~3;         // rows per staged chunk
    const int k0 = sub.start, k1 = min(npp, k0 + kDirSplit), si = it.chan - c.dsub_lo;
    const int64_t E0 = G.t_base + g * G.n_amp + c.t_off;
    const double* t = d.t[cur] + E0;
    const double* vt = d.vt + E0;
    const bool quad = (mask & (CCD_T_QHH | CCD_T_QHOLE)) != 0;
    const bool split = ntt <= 4;  // waves split K, each holding all tiles
    double* rows = d.rowsum + G.rows_base + g * G.n_rows + c.row_off;
    AT acc[4];
#pragma unroll
    for (int k = 0; k < 4; k++) acc[k] = AT{0, 0, 0, 0};
    double cpart = 0.0;  // mixed modes: this thread's share of a column sum
    // a chunk in the padded layout [crows][16 nt]: element e of it is loaded by
    // thread e % 256 into register e / 256 (zero past the chunk and the block),
    // one chunk ahead of the work on the previous one
    constexpr int kPerD = kDirBuf / 256;
    const int cw = 16 * nt;
    double vr[kPerD], tr[kPerD];
    auto load_chunk = [&](int r0) {
        const int rc = min(crows, k1 - r0);
#pragma unroll
        for (int i = 0; i < kPerD; i++) {
            const int e = threadIdx.x + 256 * i, r = e / cw, j = e - r * cw;
            const bool ok = r < rc && j < nhh;
            vr[i] = ok ? vt[(int64_t)(r0 + r) * nhh + j] : 0.0;
            tr[i] = ok ? t[(int64_t)(r0 + r) * nhh + j] : 0.0;
        }
    };
    load_chunk(k0);
    for (int r0 = k0; r0 < k1; r0 += crows) {
        const int rc = min(crows, k1 - r0);
        const int rpad = (rc + 3) & ~3;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kPerD; i++) {
            const int e = threadIdx.x + 256 * i, r = e / cw, j = e - r * cw;
            if (r < crows) { vs[r * ld + j] = vr[i]; ts[r * ld + j] = tr[i]; }
        }
        __syncthreads();
        if (r0 + crows < k1) load_chunk(r0 + crows);
        // row sums of t v (one-body particle terms), FP64 in every mode
        if (mask & CCD_T_QPART) {
            for (int r = threadIdx.x; r < rc; r += 256) {
                double sum = 0.0;
                for (int j = 0; j < nhh; j++) sum += ts[r * ld + j] * vs[r * ld + j];
                rows[r0 + r] = sum;
            }
        }
        // mixed modes: this thread's share of a column sum, rows phase, phase + 4, ...
        if constexpr (P != P_F64) {
            const int j = threadIdx.x & 63;
            if ((mask & CCD_T_QHOLE) && j < nhh)
                for (int r = threadIdx.x >> 6; r < rc; r += 4) cpart += ts[r * ld + j] * vs[r * ld + j];
        }
        if (quad) {
            const int col = lane & 15;
            if (split) {
                for (int kk = 4 * w; kk < rpad; kk += 16) {
                    const int r = kk + (lane >> 4);
                    // second column tile (nt = 2); with nt = 1 the same in-range
                    // column is read and not used
                    const int c1 = nt > 1 ? 16 + col : col;
                    const E a0 = vs[r * ld + col], b0 = ts[r * ld + col];
                    const E a1 = vs[r * ld + c1], b1 = ts[r * ld + c1];
                    if constexpr (P == P_F64) {
                        acc[0] = mfma64(a0, b0, acc[0]);
                        if (nt > 1) {
                            acc[1] = mfma64(a0, b1, acc[1]);
                            acc[2] = mfma64(a1, b0, acc[2]);
                            acc[3] = mfma64(a1, b1, acc[3]);
                        }
                    } else {
                        acc[0] = mfma32((float)a0, (float)b0, acc[0]);
                        if (nt > 1) {
                            acc[1] = mfma32((float)a0, (float)b1, acc[1]);
                            acc[2] = mfma32((float)a1, (float)b0, acc[2]);
                            acc[3] = mfma32((float)a1, (float)b1, acc[3]);
                        }
                    }
                }
            } else {
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    const int tile = w + 4 * k;
                    if (tile < ntt) {
                        const int ti = tile / nt, tj = tile - ti * nt;
                        for (int kk = 0; kk < rpad; kk += 4) {
                            const int r = kk + (lane >> 4);
                            const E av = vs[r * ld + ti * 16 + col];
                            const E bv = ts[r * ld + tj * 16 + col];
                            if constexpr (P == P_F64) acc[k] = mfma64(av, bv, acc[k]);
                            else acc[k] = mfma32((float)av, (float)bv, acc[k]);
                        }
                    }
                }
            }
        }
    }
    double* part = d.dpart + G.dpart_base + (int64_t)g * G.n_dpart + c.dpart_off + (int64_t)si * nhh * nhh;
    double* colp = d.dcolp + G.dcolp_base + (int64_t)g * G.n_dcolp + c.dcolp_off + (int64_t)si * nhh;
    if (quad) {
        if (split) {
            // add the partial tiles of waves 1..3 to wave 0's, tile by tile, in wave order
            for (int k = 0; k < ntt; k++) {
                __syncthreads();
                if (w > 0) red[w - 1][lane] = acc[k];
                __syncthreads();
                if (w == 0) acc[k] = ((acc[k] + red[0][lane]) + red[1][lane]) + red[2][lane];
            }
        }
#pragma unroll
        for (int k = 0; k < 4; k++) {
            int ti, tj;
            if (split) {
                // acc[k] holds tile (k / 2, k % 2) of the 2 x 2 layout
                ti = k >> 1; tj = k & 1;
                if (w != 0 || ti >= nt || tj >= nt) continue;
            } else {
                const int tile = w + 4 * k;
                if (tile >= ntt) continue;
                ti = tile / nt; tj = tile - ti * nt;
            }
#pragma unroll
            for (int q = 0; q < 4; q++) {
                int kl = ti * 16 + orow<PM>(lane, q), ij = tj * 16 + (lane & 15);
                if (kl < nhh && ij < nhh) {
                    const double qv = (double)acc[k][q];
                    part[kl * nhh + ij] = qv;
                    if (P == P_F64 && kl == ij) colp[kl] = qv;
                }
            }
        }
    }
    if constexpr (P != P_F64) {
        if (mask & CCD_T_QHOLE) {
            double* cred = vs;  // 4 x 64 doubles
            __syncthreads();
            cred[threadIdx.x] = cpart;
            __syncthreads();
            if (threadIdx.x < nhh)
                colp[threadIdx.x] = (cred[threadIdx.x] + cred[64 + threadIdx.x]) + (cred[128 + threadIdx.x] + cred[192 + threadIdx.x]);
        }
    }
    }
}

// per (S_z = 0 channel, problem): chi_klij = <kl||ij> + sum of the product
// items' parts, and the column sums, in item order
__global__ void __launch_bounds__(256) k_dsum(DevPtrs d, uint32_t mask, int n_items) {
    for (int bi = blockIdx.x; bi < n_items; bi += gridDim.x) {
        const Item it = d.it_dsum[bi];
        if (it.chan < 0) continue;
        const DevChan c = d.chans[it.chan];
        const DevGroup G = d.groups[c.group];
        const int g = it.start;
        if (!d.active[G.p0 + g]) continue;
        const int nhh = c.nhh, nsub = c.dsub_n;
        const double* part = d.dpart + G.dpart_base + (int64_t)g * G.n_dpart + c.dpart_off;
        const double* colp = d.dcolp + G.dcolp_base + (int64_t)g * G.n_dcolp + c.dcolp_off;
        double* chh = d.chh + G.chh_base + g * G.n_chh + c.chh_off;
        double* cols = d.colsum + G.cols_base + g * G.n_cols + c.col_off;
        const double* lut = d.lut + G.lut_base + g * G.nlut;
        const int32_t* st = d.st + G.st_off;
        for (int e = threadIdx.x; e < nhh * nhh; e += 256) {
            const int kl = e / nhh, ij = e - kl * nhh;
            double v = 0.0;
            if (mask & CCD_T_HH) {
                const int32_t p1 = d.hh[c.hh_off + kl], p2 = d.hh[c.hh_off + ij];
                v = vas(lut, st[pa(p1)], st[pb(p1)], st[pa(p2)], st[pb(p2)]);
            }
            if (mask & CCD_T_QHH) {
                double q = 0.0;
                for (int s = 0; s < nsub; s++) q += part[(int64_t)s * nhh * nhh + e];
                v += q;
            }
            chh[e] = v;
        }
        if ((mask & CCD_T_QHOLE) && threadIdx.x < nhh) {
            double q = 0.0;
            for (int s = 0; s < nsub; s++) q += colp[s * nhh + threadIdx.x];
            cols[threadIdx.x] = q;
        }
    }
}

// one-body intermediates: one wave per (state, problem); CSR entries x >= 0
// name a column sum (holes, +), x < 0 the row sum -x-1 (particles, -)
__global__ void __launch_bounds__(256) k_dchi(DevPtrs d, uint32_t mask, int n_items) {
    for (int bi = blockIdx.x; bi < n_items; bi += gridDim.x) {
    const Item it = d.it_dchi[bi];
    const DevGroup G = d.groups[it.chan];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int s = (it.start & 0xffff) + w, g = it.start >> 16;  // state of this wave, problem
    if (s >= G.ns) continue;
    const int x0 = d.csr_ptr[G.csr_off + s], x1 = d.csr_ptr[G.csr_off + s + 1];
    {
        if (!d.active[G.p0 + g]) continue;
        const double* rows = d.rowsum + G.rows_base + g * G.n_rows;
        const double* cols = d.colsum + G.cols_base + g * G.n_cols;
        double acc = 0.0;
        for (int x = x0 + lane; x < x1; x += 64) {
            int idx = d.csr_idx[x];
            if (idx >= 0) {
                if (mask & CCD_T_QHOLE) acc += cols[idx];
            } else {
                if (mask & CCD_T_QPART) acc -= rows[-idx - 1];
            }
        }
        acc = wave_sum(acc);
        if (lane == 0) d.dchi[G.eps_base + g * G.ns + s] = acc;
    }
    }
}

// ring per pair {Q, P = -Q} of cross channels and problem.  With
//   A[u][x] = T~_Q  = t_ik^ac,  (a,i) = member u of Q, (c,k) = member x of P
//   B[x][m] = <kl||cd>,         (c,k) = member x of P, (d,l) = member m of Q
// (A is n_Q x n_P and B n_P x n_Q; the two sizes differ under a twist)
// the partner's blocks are the transposes (T~_P = A^T, its Vbar = B^T), so
//   chi_P = <kb||cj>_P + 1/2 B A      (chi_kbcj for the ring of Q)
//   M_Q   = <kb||cj>_Q + 1/2 A B      (the transpose of chi_kbcj for the ring of P)
//   Out   = A chi_P + M_Q A  =  Z_Q[u][y] + Z_P[y][u]
// i.e. the sum of the two P(ij)P(ab) ring terms (with their common sign) that
// land on one canonical amplitude.  The two halves of A B A combine, so
//   Out = X A + A V_P,  X = A B + V_Q,  V = <kb||cj>
// takes three products instead of four.  Each entry of Out is stored once,
// to the ring slot (2e + k) of the amplitude e it feeds (k = which of its two
// ring terms), so the amplitude update reads its two slots with one 16-byte
// load.  The products run on MFMA from LDS (matrices padded to n16 >= both
// sizes, row stride n16 + 1), their K loops cut at the contracted size rounded
// up to the MFMA K step.
struct PairCtx {
    const int32_t* map;    // position map of Q, [nq][np]
    const double* t;       // amplitudes of the problem
    double* zc;            // ring slots of the problem
    const int32_t* zs;     // position -> slot table of the pair block, [nq][np]
    int nq, np;            // members of Q and of P = -Q
    bool self;             // Q is its own partner
};

__device__ __forceinline__ bool pair_ctx(const DevPtrs& d, const Item it, int cur, PairCtx& r,
                                         int32_t& memQ, int32_t& memP, int32_t& lut_off, int32_t& nlut) {
    const DevPh q = d.ph[it.chan];
    const DevGroup G = d.groups[q.group];
    const int g = it.start;
    r.map = d.phmap + q.map_off;
    r.t = d.t[cur] + G.t_base + g * G.n_amp;
    r.zc = d.zc + 2 * (G.t_base + g * G.n_amp);
    r.zs = d.zs + G.zidx_off + q.zp_off;
    r.nq = q.n;
    r.np = q.m;
    r.self = q.partner == it.chan;
    memQ = q.mem_off;
    memP = q.pmem_off;
    lut_off = G.lut_base + g * G.nlut;
    nlut = G.nlut;
    return d.active[G.p0 + g] != 0;
}

// stage the (p, h) states of both member lists and the problem's W/2 table
__device__ __forceinline__ void pair_stage(const DevPtrs& d, int memQ, int memP, int lut_off, int nlut,
                                           int nq, int np, int32_t* qs, int32_t* ps, double* lutS, int t0,
                                           int stride) {
    const int2* ms = (const int2*)d.phst;
    for (int e = t0; e < nq; e += stride) {
        const int2 m = ms[memQ + e];
        qs[2 * e] = m.x; qs[2 * e + 1] = m.y;
    }
    for (int e = t0; e < np; e += stride) {
        const int2 o = ms[memP + e];
        ps[2 * e] = o.x; ps[2 * e + 1] = o.y;
    }
    for (int e = t0; e < nlut; e += stride) lutS[e] = d.lut[lut_off + e];
}

// This thread's position-map entries of A, entries t0, t0 + stride, ...
// (issued before the staging barrier, so that the amplitude gathers can start
// right after it)
template <int n16, int stride, int J>
__device__ __forceinline__ void pair_maps(const PairCtx& r, int t0, int32_t* m) {
    constexpr int tot = n16 * n16;
#pragma unroll
    for (int j = 0; j < J; j++) {
        const int e = t0 + j * stride, u = e / n16, x = e - u * n16;
        m[j] = (e < tot && u < r.nq && x < r.np) ? r.map[u * r.np + x] : -1;
    }
}

// A = gathered T~_Q (signed), B = Vbar, zero padded.  The gathers are issued
// first and B is generated while they are in flight.  With TR set (BF16), A,
// At = A^T and Bt = B^T are written instead of A and B.
template <typename E, int n16, int lda, int stride, int J, bool TR>
__device__ __forceinline__ void pair_fill(const PairCtx& r, const int32_t* m, const int32_t* qs, const int32_t* ps,
                                          const double* lutS, double wq, E* A, E* B, E* At, E* Bt, int t0,
                                          bool qring) {
    const int nq = r.nq, np = r.np;
    constexpr int tot = n16 * n16;
    double tv[J];
#pragma unroll
    for (int j = 0; j < J; j++) tv[j] = m[j] >= 0 ? r.t[m[j] >> 3] : 0.0;
#pragma unroll
    for (int j = 0; j < J; j++) {
        const int e = t0 + j * stride;
        if (e < tot) {
            const int u = e / n16, x = e - u * n16;
            double b = 0.0;
            if (qring && u < np && x < nq)  // <kl||cd>: (c,k) = P member u, (d,l) = Q member x
                b = vas_q(lutS, wq, ps[2 * u + 1], qs[2 * x + 1], ps[2 * u], qs[2 * x]);
            if constexpr (TR) Bt[x * lda + u] = (E)b;
            else B[u * lda + x] = (E)b;
        }
    }
#pragma unroll
    for (int j = 0; j < J; j++) {
        const int e = t0 + j * stride;
        if (e < tot) {
            const int u = e / n16, x = e - u * n16;
            const E av = (E)((m[j] & 1) ? -tv[j] : tv[j]);
            A[u * lda + x] = av;
            if constexpr (TR) At[x * lda + u] = av;
        }
    }
}

// <kb||cj> between members x, y of one list (states interleaved (p, h))
__device__ __forceinline__ double pair_vph(const int32_t* s2, const double* lutS, double wq, int x, int y) {
    return vas_q(lutS, wq, s2[2 * x + 1], s2[2 * y], s2[2 * x], s2[2 * y + 1]);
}

// the ring slots of this lane's four output positions of tile (tu, ty), -1 for
// none (a self pair holds both orders of one amplitude; only the p < p' one
// has a slot); loaded before the products so that the stores do not wait
template <int P>
__device__ __forceinline__ void pair_slots(const PairCtx& r, int tu, int ty, int lane, int32_t* z) {
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int u = tu * 16 + orow<P>(lane, q), y = ty * 16 + (lane & 15);
        z[q] = (u < r.nq && y < r.np) ? r.zs[u * r.np + y] : -1;
    }
}

template <typename AT>
__device__ __forceinline__ void pair_store(const PairCtx& r, AT acc, const int32_t* z) {
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const double v = (double)acc[q];
        if (z[q] >= 0) r.zc[z[q] >> 1] = (z[q] & 1) ? -v : v;
    }
}

// products of one 16x16 output tile, k from 0 to kmax (a multiple of 4; FP64 /
// FP32: 16x16x4); operands of four steps are loaded before their MFMAs
template <int P, typename E, typename AT>
__device__ __forceinline__ AT mm4(const E* X, const E* Y, int lda, int tx, int ty, int kmax, int lane, AT acc) {
    const E* xr = X + (tx * 16 + (lane & 15)) * lda + (lane >> 4);
    const E* yc = Y + (lane >> 4) * lda + ty * 16 + (lane & 15);
    int k0 = 0;
    for (; k0 + 16 <= kmax; k0 += 16) {
        E a[4], b[4];
#pragma unroll
        for (int s = 0; s < 4; s++) {
            a[s] = xr[k0 + 4 * s];
            b[s] = yc[(k0 + 4 * s) * lda];
        }
#pragma unroll
        for (int s = 0; s < 4; s++) {
            if constexpr (P == P_F64) acc = mfma64(a[s], b[s], acc);
            else acc = mfma32(a[s], b[s], acc);
        }
    }
    for (; k0 < kmax; k0 += 4) {
        if constexpr (P == P_F64) acc = mfma64(xr[k0], yc[k0 * lda], acc);
        else acc = mfma32(xr[k0], yc[k0 * lda], acc);
    }
    return acc;
}
// BF16: X row-major, Yt = Y^T row-major, k from 0 to kmax (a multiple of 32)
__device__ __forceinline__ f4 mmbf(const __bf16* X, const __bf16* Yt, int lda, int tx, int ty, int kmax,
                                   int lane, f4 acc) {
    const __bf16* xr = X + (tx * 16 + (lane & 15)) * lda + 8 * (lane >> 4);
    const __bf16* yr = Yt + (ty * 16 + (lane & 15)) * lda + 8 * (lane >> 4);
    int k0 = 0;
    for (; k0 + 64 <= kmax; k0 += 64) {
        const bf8 a0 = *(const bf8*)&xr[k0], b0 = *(const bf8*)&yr[k0];
        const bf8 a1 = *(const bf8*)&xr[k0 + 32], b1 = *(const bf8*)&yr[k0 + 32];
        acc = mfmabf(a0, b0, acc);
        acc = mfmabf(a1, b1, acc);
    }
    if (k0 < kmax) acc = mfmabf(*(const bf8*)&xr[k0], *(const bf8*)&yr[k0], acc);
    return acc;
}

// byte offset of the matrices in a pair item's LDS (after W/2 and member states)
__host__ __device__ constexpr size_t pair_mat_off() {
    return ((size_t)kMaxLut * 8 + 4 * (size_t)kMaxPH * 4 + 15) & ~(size_t)15;
}

// One pair item with NW waves, wave w owning output tiles w, w + NW, ...
// Matrices padded to n16 (K padded to kpad = n16 for 16x16x4, 32-multiple for
// BF16) with row stride lda.
template <int P, int N16, int NW>
__device__ __forceinline__ void pair_body(const DevPtrs& d, const Item it, int cur, uint32_t mask, char* lds,
                                          int tid) {
    using E = typename std::conditional<P == P_F64, double, typename std::conditional<P == P_F32, float, __bf16>::type>::type;
    using AT = typename AccT<P>::T;
    constexpr int n16 = N16, nt = N16 / 16, ntt = nt * nt, TPW = (ntt + NW - 1) / NW;
    constexpr int kpad = P == P_BF16 ? ((N16 + 31) & ~31) : N16;
    constexpr int lda = P == P_BF16 ? kpad + 8 : N16 + 1;
    constexpr int rows = P == P_BF16 ? kpad : N16;  // rows allocated per matrix
    PairCtx r;
    r.nq = 0; r.np = 0; r.self = false; r.map = nullptr; r.t = nullptr; r.zc = nullptr; r.zs = nullptr;
    int32_t memQ = 0, memP = 0, lo = 0, nlut = 0;
    // every wave reaches every barrier below; only the work is guarded by live
    const bool live = it.chan >= 0 && pair_ctx(d, it, cur, r, memQ, memP, lo, nlut);
    const int lane = tid & 63, w = tid >> 6;
    double* lutS = (double*)lds;
    int32_t* qs = (int32_t*)(lutS + kMaxLut);
    int32_t* ps = qs + 2 * kMaxPH;
    // FP64 / FP32: A and B (B later holds X, then V_P);
    // BF16: A, At = A^T and Bt = B^T (Bt later holds X, then V_P^T)
    E* A = (E*)(lds + pair_mat_off());
    E* B = A + rows * lda;
    E* At = B;                // BF16 only (same storage as B)
    E* Bt = At + rows * lda;  // BF16 only
    const bool qring = (mask & CCD_T_QRING) != 0, ring = (mask & CCD_T_RING) != 0;
    constexpr int J = (n16 * n16 + 64 * NW - 1) / (64 * NW);  // entries of A per thread
    int32_t mp[J];
#pragma unroll
    for (int j = 0; j < J; j++) mp[j] = -1;
    if (live) pair_maps<n16, 64 * NW, J>(r, tid, mp);
    if (live) {
        pair_stage(d, memQ, memP, lo, nlut, r.nq, r.np, qs, ps, lutS, tid, 64 * NW);
        if constexpr (P == P_BF16) {
            // zero the K padding (rows and columns n16 .. kpad) of all three matrices
            for (int e = tid; e < 3 * rows * lda; e += 64 * NW) A[e] = (E)0.0f;
        }
    }
    __syncthreads();
    // W(|Q|^2)/2, the first table entry of every element of the pair (member 0
    // of Q: hole qs[1], particle qs[0])
    const double wq = live ? lutS[dist2(qs[1], qs[0])] : 0.0;
    if (live) pair_fill<E, n16, lda, 64 * NW, J, P == P_BF16>(r, mp, qs, ps, lutS, wq, A, B, At, Bt, tid, qring);
    int32_t zsl[TPW][4];
#pragma unroll
    for (int k = 0; k < TPW; k++) {
        const int tile = w + NW * k;
        if (live && tile < ntt) pair_slots<P>(r, tile / nt, tile - (tile / nt) * nt, lane, zsl[k]);
    }
    __syncthreads();
    // K extents: the contracted size rounded up to the MFMA K step (n_P for
    // A B and A V_P, n_Q for X A)
    const int kp = P == P_BF16 ? ((r.np + 31) & ~31) : ((r.np + 3) & ~3);
    const int kq = P == P_BF16 ? ((r.nq + 31) & ~31) : ((r.nq + 3) & ~3);
    // X = A B for this wave's tiles (quadratic ring)
    AT xq[TPW];
#pragma unroll
    for (int k = 0; k < TPW; k++) {
        xq[k] = AT{0, 0, 0, 0};
        const int tile = w + NW * k;
        if (live && qring && tile < ntt) {
            const int tx = tile / nt, ty = tile - tx * nt;
            if constexpr (P == P_BF16) xq[k] = mmbf(A, Bt, lda, tx, ty, kp, lane, xq[k]);
            else xq[k] = mm4<P>(A, B, lda, tx, ty, kp, lane, xq[k]);
        }
    }
    __syncthreads();  // every wave has finished reading B (Bt)
    // X = A B + V_Q replaces B (FP64 / FP32) or Bt (BF16), row-major; zero outside the block
    E* XB = P == P_BF16 ? Bt : B;
#pragma unroll
    for (int k = 0; k < TPW; k++) {
        const int tile = w + NW * k;
        if (live && tile < ntt) {
            const int tx = tile / nt, ty = tile - tx * nt;
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int x = tx * 16 + orow<P>(lane, q), y = ty * 16 + (lane & 15);
                double xv = (double)xq[k][q];
                if (ring && x < r.nq && y < r.nq) xv += pair_vph(qs, lutS, wq, x, y);
                XB[x * lda + y] = (E)xv;
            }
        }
    }
    __syncthreads();
    // Out = X A, accumulators kept across the next barrier
    AT acc[TPW];
#pragma unroll
    for (int k = 0; k < TPW; k++) {
        acc[k] = AT{0, 0, 0, 0};
        const int tile = w + NW * k;
        if (live && tile < ntt) {
            const int tu = tile / nt, ty = tile - tu * nt;
            if constexpr (P == P_BF16) acc[k] = mmbf(XB, At, lda, tu, ty, kq, lane, acc[k]);
            else acc[k] = mm4<P>(XB, A, lda, tu, ty, kq, lane, acc[k]);
        }
    }
    __syncthreads();  // every wave has finished reading X
    // V_P replaces X: row-major for FP64 / FP32, transposed for BF16
#pragma unroll
    for (int k = 0; k < TPW; k++) {
        const int tile = w + NW * k;
        if (live && tile < ntt) {
            const int tx = tile / nt, ty = tile - tx * nt;
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int x = tx * 16 + orow<P>(lane, q), y = ty * 16 + (lane & 15);
                const double vp = (ring && x < r.np && y < r.np) ? pair_vph(ps, lutS, wq, x, y) : 0.0;
                if constexpr (P == P_BF16) XB[y * lda + x] = (E)(float)vp;
                else XB[x * lda + y] = (E)vp;
            }
        }
    }
    __syncthreads();
    // Out += A V_P
#pragma unroll
    for (int k = 0; k < TPW; k++) {
        const int tile = w + NW * k;
        if (live && tile < ntt) {
            const int tu = tile / nt, ty = tile - tu * nt;
            if constexpr (P == P_BF16) acc[k] = mmbf(A, XB, lda, tu, ty, kp, lane, acc[k]);
            else acc[k] = mm4<P>(A, XB, lda, tu, ty, kp, lane, acc[k]);
            pair_store(r, acc[k], zsl[k]);
        }
    }
}

template <int P> __host__ __device__ constexpr size_t pair_lds(int n16) {
    const size_t es = P == P_F64 ? 8 : (P == P_F32 ? 4 : 2);
    const size_t kpad = P == P_BF16 ? ((n16 + 31) & ~31) : n16;
    const size_t lda = P == P_BF16 ? kpad + 8 : n16 + 1;
    const size_t rows = P == P_BF16 ? kpad : n16;
    const size_t mats = P == P_BF16 ? 3 : 2;
    return pair_mat_off() + mats * rows * lda * es;
}

// pairs with n <= 16: one wave per item, four items per block
template <int P>
__global__ void __launch_bounds__(256) k_ringp_small(DevPtrs d, int cur, uint32_t mask, int n_items) {
    constexpr size_t per = (pair_lds<P>(16) + 15) & ~(size_t)15;
    __shared__ __attribute__((aligned(16))) char lds[4 * per];
    const int w = threadIdx.x >> 6;
    const int nb = (n_items + 3) / 4;
    for (int bi = blockIdx.x; bi < nb; bi += gridDim.x) {
        const int idx = bi * 4 + w;
        Item it = d.it_ring_s[min(idx, n_items - 1)];
        if (idx >= n_items) it.chan = -1;
        __syncthreads();  // the previous item's reads of LDS are done
        pair_body<P, 16, 1>(d, it, cur, mask, lds + w * per, threadIdx.x & 63);
    }
}

// pairs with n > 16: one block per item, one wave per output tile
template <int P, int N16, int NW>
__global__ void __launch_bounds__(64 * NW) k_ringp(DevPtrs d, int cur, uint32_t mask, int base, int n_items) {
    extern __shared__ __attribute__((aligned(16))) char dyn_lds[];
    for (int bi = blockIdx.x; bi < n_items; bi += gridDim.x) {
        __syncthreads();  // the previous item's reads of LDS are done
        pair_body<P, N16, NW>(d, d.it_ring_b[base + bi], cur, mask, dyn_lds, threadIdx.x);
    }
}

// the ring contribution to amplitude e of problem g: its two ring slots
__device__ __forceinline__ double ring_term(const DevPtrs& d, const DevGroup& G, int g, int64_t e) {
    const double2 z = *(const double2*)(d.zc + 2 * (G.t_base + g * G.n_amp + e));
    return z.x + z.y;
}

// one-body sums per row (delta chi_a + delta chi_b) and column (delta chi_i +
// delta chi_j); grid (blocks over rows + columns, problem slot)
__global__ void __launch_bounds__(256) k_onebody(DevPtrs d) {
    const int p = blockIdx.y;
    const DevGroup G = d.groups[d.pgrp[p]];
    const int g = d.pgi[p];
    if (!d.active[G.p0 + g]) return;
    const int e = blockIdx.x * 256 + threadIdx.x;
    const double* dc = d.dchi + G.eps_base + g * G.ns;
    if (e < G.n_rows_all) {
        int32_t ab = d.pp[G.pp0 + e];
        d.rowX[G.rowa_base + g * G.n_rows_all + e] = dc[pa(ab)] + dc[pb(ab)];
    } else if (e < G.n_rows_all + G.n_cols_all) {
        int q = e - G.n_rows_all;
        int32_t ij = d.hh[G.hh0 + q];
        d.colX[G.cola_base + g * G.n_cols_all + q] = dc[pa(ij)] + dc[pb(ij)];
    }
}

// ladder sums per (128-pair tile, 16-column tile of an S_z = 0 channel,
// problem): 1/2 sum_cd <ab||cd> t_ij^cd + 1/2 sum_kl t_kl^ab chi_klij into rmm.
// They need t and chi_klij only, so they run beside the ring.  Both kernels
// run the pp sum as a product over the momentum pairs P = {p, K - p} of the
// block (see k_ladder64 below for the identity): wave w owns pairs 32w ..
// 32w+31 of the tile as two 16-row MFMA tiles that share each staged operand
// and column descriptor, and each finished sum goes to the two spin rows of
// its pair with signs + and -.
//
// Generator.  With p' the row pair's first momentum and (p, q = K - p) the
// column pair's, M[P'][P] = (W(|p' - p|^2) + W(|p' - q|^2)) / 2.  With S the
// byte size of a table entry both table byte offsets follow from one dot
// product: |p' - p|^2 = A2 + C2 - 2 p'.p and |p' - q|^2 = A2 - 2 p'.K + D2 +
// 2 p'.p (A2 = |p'|^2, C2 = |p|^2, D2 = |q|^2), so o1 = S A2 + S C2 - 2S p'.p
// (sdot4 of -(S/2) p' and 4 p, both packed int8, accumulated onto the row and
// column constants) and o2 = S (2 A2 - 2 p'.K) + S (C2 + D2) - o1.  Padding
// columns carry p = K and D2 = 0, so both offsets stay inside the table
// (|q'|^2 and A2); their delta is zero.  Padding rows carry p' = 0.
constexpr int kKP = 128;  // momentum pairs staged per barrier

// the mixed modes: FP32 operands on the 16x16x4 FP32 MFMA or BF16 operands on
// the 16x16x32 BF16 MFMA, FP32 accumulation; staging as in k_ladder64
template <int P>
__global__ void __launch_bounds__(256, 3) k_ladder(DevPtrs d, int cur, uint32_t mask, int n_items) {
    static_assert(P != P_F64, "the FP64 ladder is k_ladder64");
    constexpr int S = 4;
    __shared__ float lutS[kMaxLut];
    // delta chunk: [k][16] FP32, transposed [16][k] BF16
    __shared__ __attribute__((aligned(16))) char tks[P == P_F32 ? kKP * 16 * 4 : 16 * (kKP + 8) * 2];
    // per staged pair: (4 p as int8, S |p|^2, S (|p|^2 + |q|^2), rows + 1 as two 16-bit fields)
    __shared__ int4 cvi[2][kKP];
    __shared__ int2 prs[kLadderRows];  // the two spin rows of the tile's pairs
    const char* lutB = (const char*)lutS;
    for (int bi = blockIdx.x; bi < n_items; bi += gridDim.x) {
    const Item lg = d.it_lg[bi];
    if (lg.chan < 0) continue;
    const int g = lg.start;
    const Item it = d.it_ladder[lg.chan];
    const int r0 = it.start & 0xfffff, ct = it.start >> 20;  // pair tile and column tile of the item
    const DevChan c = d.chans[it.chan];
    const DevGroup G = d.groups[c.group];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nhh = c.nhh, nlp = c.n_lp;
    const bool act = d.active[G.p0 + g] != 0;
    const bool pp_on = act && (mask & CCD_T_PP) != 0;
    const bool hh_on = act && (mask & (CCD_T_HH | CCD_T_QHH)) != 0;
    const int64_t T0 = G.t_base + g * G.n_amp + c.t_off;
    const double* tcur = d.t[cur] + T0;
    const int4* lp = d.lpinfo + c.lp_off;
    const int rbase = r0 + 32 * w;
    const int32_t kpack = (int32_t)((uint32_t)(uint8_t)(int8_t)c.kx | ((uint32_t)(uint8_t)(int8_t)c.ky << 8) |
                                    ((uint32_t)(uint8_t)(int8_t)c.kz << 16));
    const int K2 = c.kx * c.kx + c.ky * c.ky + c.kz * c.kz;
    // 4 n as packed int8 (|4 n_i| <= 64): shift each byte left by two, dropping
    // the bits carried into the next byte
    auto times4 = [](int32_t x) { return (int32_t)(((uint32_t)x << 2) & 0xfcfcfcfcu); };
    int32_t apack[2] = {0, 0};  // -(S/2) p' as packed int8
    int rowA[2] = {0, 0}, rowS[2] = {0, 0};
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const int pr = rbase + 16 * h + (lane & 15);
        const int4 li = pr < nlp ? lp[pr] : make_int4(0, 0, -1, -1);
        const int ax = (int8_t)(li.x & 0xff), ay = (int8_t)((li.x >> 8) & 0xff), az = (int8_t)((li.x >> 16) & 0xff);
        apack[h] = (int32_t)((uint32_t)(uint8_t)(int8_t)(-2 * ax) | ((uint32_t)(uint8_t)(int8_t)(-2 * ay) << 8) |
                             ((uint32_t)(uint8_t)(int8_t)(-2 * az) << 16));
        const int A2 = li.y & 1023;
        const int aK = ax * c.kx + ay * c.ky + az * c.kz;
        rowA[h] = S * A2;
        rowS[h] = S * (2 * A2 - 2 * aK);
    }
    const int4 cpad = make_int4(times4(kpack), S * K2, S * K2, 0);
    auto cdesc = [&](const int4& li) {
        const int C2 = li.y & 1023, D2 = (li.y >> 10) & 1023;
        return make_int4(times4(li.x), S * C2, S * (C2 + D2),
                         (int)((uint32_t)(li.z + 1) | ((uint32_t)(li.w + 1) << 16)));
    };
    constexpr int kPer = kKP * 16 / 256;
    double tv[kPer];
    auto load_delta = [&](int kp, int b) {
        const int kn = min(kKP, nlp - kp);
#pragma unroll
        for (int i = 0; i < kPer; i++) {
            const int e = threadIdx.x + 256 * i, kk = e >> 4, cc = ct * 16 + (e & 15);
            double v = 0.0;
            if (kk < kn && cc < nhh) {
                const uint32_t rr = (uint32_t)cvi[b][kk].w;
                const int rp = (int)(rr & 0xffff) - 1, rm = (int)(rr >> 16) - 1;
                const double tp = rp >= 0 ? tcur[(int64_t)rp * nhh + cc] : 0.0;
                const double tm = rm >= 0 ? tcur[(int64_t)rm * nhh + cc] : 0.0;
                v = tp - tm;
            }
            tv[i] = v;
        }
    };
    auto store_delta = [&]() {
#pragma unroll
        for (int i = 0; i < kPer; i++) {
            const int e = threadIdx.x + 256 * i, kk = e >> 4, jj = e & 15;
            if constexpr (P == P_F32) ((float*)tks)[kk * 16 + jj] = (float)tv[i];
            else ((__bf16*)tks)[jj * (kKP + 8) + kk] = (__bf16)tv[i];
        }
    };
    // M[P'][P] of tile h's row for column descriptor ci
    auto gen = [&](const int4 ci, int h) -> float {
        const int o1 = __builtin_amdgcn_sdot4(apack[h], ci.x, rowA[h] + ci.y, false);
        const int o2 = rowS[h] + ci.z - o1;
        return *(const float*)(lutB + o1) + *(const float*)(lutB + o2);
    };
    const int col = ct * 16 + (lane & 15);
    f4 acc[2], acc2[2];
#pragma unroll
    for (int h = 0; h < 2; h++) { acc[h] = f4{0, 0, 0, 0}; acc2[h] = f4{0, 0, 0, 0}; }

    const double* lutg = d.lut + G.lut_base + g * G.nlut;
    const float lv0 = threadIdx.x < G.nlut ? (float)lutg[threadIdx.x] : 0.0f;
    const float lv1 = threadIdx.x + 256 < G.nlut ? (float)lutg[threadIdx.x + 256] : 0.0f;
    int4 lpc = cpad;
    if (pp_on && threadIdx.x < kKP && threadIdx.x < nlp) lpc = lp[threadIdx.x];
    const int2* lpr = (const int2*)lp;
    const int2 myr = (threadIdx.x < kLadderRows && r0 + threadIdx.x < nlp) ? lpr[2 * (r0 + threadIdx.x) + 1]
                                                                           : make_int2(-1, -1);
    __syncthreads();  // the previous item's reads of LDS are done
    lutS[threadIdx.x] = lv0;
    if (threadIdx.x + 256 < kMaxLut) lutS[threadIdx.x + 256] = lv1;
    if (threadIdx.x < kLadderRows) prs[threadIdx.x] = myr;
    if (pp_on) {
        if (threadIdx.x < kKP) cvi[0][threadIdx.x] = threadIdx.x < nlp ? cdesc(lpc) : cpad;
        lpc = cpad;
        if (threadIdx.x < kKP && kKP + threadIdx.x < nlp) lpc = lp[kKP + threadIdx.x];
    }
    __syncthreads();
    if (pp_on) {
        load_delta(0, 0);
        store_delta();
        for (int kp = 0; kp < nlp; kp += kKP) {
            const int b = (kp / kKP) & 1;
            const bool more = kp + kKP < nlp;
            if (more && threadIdx.x < kKP) {
                cvi[b ^ 1][threadIdx.x] = kp + kKP + threadIdx.x < nlp ? cdesc(lpc) : cpad;
                lpc = cpad;
                if (kp + 2 * kKP + threadIdx.x < nlp) lpc = lp[kp + 2 * kKP + threadIdx.x];
            }
            __syncthreads();  // this chunk's delta and the next chunk's descriptors are in LDS
            if (more) load_delta(kp + kKP, b ^ 1);
            const int kn = min(kKP, nlp - kp);
            if constexpr (P == P_BF16) {
                const int ksteps = (kn + 31) & ~31;
                for (int kk = 0; kk < ksteps; kk += 32) {
                    const int k0 = kk + 8 * (lane >> 4);
                    bf8 av[2];
#pragma unroll
                    for (int j = 0; j < 8; j++) {
                        const int4 ci = cvi[b][k0 + j];
                        av[0][j] = (__bf16)gen(ci, 0);
                        av[1][j] = (__bf16)gen(ci, 1);
                    }
                    const bf8 bv = *(const bf8*)&((const __bf16*)tks)[(lane & 15) * (kKP + 8) + k0];
                    acc[0] = mfmabf(av[0], bv, acc[0]);
                    acc[1] = mfmabf(av[1], bv, acc[1]);
                }
            } else {
                // four MFMA steps per batch for both tiles: all operands are
                // produced first, each phase's LDS reads issued together
                const int ksteps = (kn + 15) & ~15;
                for (int kk = 0; kk < ksteps; kk += 16) {
                    float vb[4], x1[2][4], x2[2][4];
                    int o1[2][4], o2[2][4];
#pragma unroll
                    for (int s2 = 0; s2 < 4; s2++) {
                        const int4 ci = cvi[b][kk + 4 * s2 + (lane >> 4)];
#pragma unroll
                        for (int h = 0; h < 2; h++) {
                            o1[h][s2] = __builtin_amdgcn_sdot4(apack[h], ci.x, rowA[h] + ci.y, false);
                            o2[h][s2] = rowS[h] + ci.z - o1[h][s2];
                        }
                    }
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int s2 = 0; s2 < 4; s2++) {
#pragma unroll
                        for (int h = 0; h < 2; h++) {
                            x1[h][s2] = *(const float*)(lutB + o1[h][s2]);
                            x2[h][s2] = *(const float*)(lutB + o2[h][s2]);
                        }
                        vb[s2] = ((const float*)tks)[(kk + 4 * s2 + (lane >> 4)) * 16 + (lane & 15)];
                    }
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int s2 = 0; s2 < 4; s2 += 2) {
#pragma unroll
                        for (int h = 0; h < 2; h++) {
                            const float va0 = x1[h][s2] + x2[h][s2], va1 = x1[h][s2 + 1] + x2[h][s2 + 1];
                            acc[h] = mfma32(va0, vb[s2], acc[h]);
                            acc2[h] = mfma32(va1, vb[s2 + 1], acc2[h]);
                        }
                    }
                }
            }
            __syncthreads();  // every wave is done with this chunk
            if (more) store_delta();
        }
        // u of the lane's output pairs: + to the (p up, q down) row, - to the other
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const f4 u = acc[h] + acc2[h];
            acc[h] = u;
            acc2[h] = -u;
        }
    }
    if (hh_on) {
        // 1/2 sum_kl t_kl^ab chi_klij per spin row: A = t rows, B = chi_klij columns
        const double* xg = d.chh + G.chh_base + g * G.n_chh + c.chh_off;
        int2 arow[2];
#pragma unroll
        for (int h = 0; h < 2; h++) arow[h] = prs[32 * w + 16 * h + (lane & 15)];
        for (int k0 = 0; k0 < nhh; k0 += 16) {
            double bq[4];
#pragma unroll
            for (int s2 = 0; s2 < 4; s2++) {
                const int kq = k0 + 4 * s2 + (lane >> 4);
                bq[s2] = (kq < nhh && col < nhh) ? xg[kq * nhh + col] : 0.0;
            }
#pragma unroll
            for (int h = 0; h < 2; h++) {
                double ap[4], am[4];
#pragma unroll
                for (int s2 = 0; s2 < 4; s2++) {
                    const int kq = k0 + 4 * s2 + (lane >> 4);
                    ap[s2] = (arow[h].x >= 0 && kq < nhh) ? tcur[(int64_t)arow[h].x * nhh + kq] : 0.0;
                    am[s2] = (arow[h].y >= 0 && kq < nhh) ? tcur[(int64_t)arow[h].y * nhh + kq] : 0.0;
                }
#pragma unroll
                for (int s2 = 0; s2 < 4; s2++) {
                    acc[h] = mfma32((float)ap[s2], (float)bq[s2], acc[h]);
                    acc2[h] = mfma32((float)am[s2], (float)bq[s2], acc2[h]);
                }
            }
        }
    }
    // this lane owns pairs orow(lane, r) of each tile, column col
    if (act) {
#pragma unroll
        for (int h = 0; h < 2; h++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int po = rbase + 16 * h + orow<P>(lane, r);
                if (po < nlp && col < nhh) {
                    const int2 rr = prs[32 * w + 16 * h + orow<P>(lane, r)];
                    if (rr.x >= 0) d.rmm[T0 + (int64_t)rr.x * nhh + col] = (double)acc[h][r];
                    if (rr.y >= 0) d.rmm[T0 + (int64_t)rr.y * nhh + col] = (double)acc2[h][r];
                }
            }
    }
    }
}

// FP64 ladder sums over momentum pairs, on the 4x4x4 MFMA.
//
// In an S_z = 0 block the generated <ab||cd> = s_a s_c (W(|n_a - n_c|^2) +
// W(|n_a - n_d|^2)) / 2 depends on the row only through s_a and n_a and on the
// column only through s_c and the momenta (n_c, n_d).  The rows of a block come
// in momentum pairs P = {p, q = K - p}: (p up, q down) and (p down, q up), or
// the one row (p down, p up) when p = q; both rows of a pair have n_a = p.  So
//   sum_cd <ab||cd> t_ij^cd = s_a u_ij(P_a),   u(P') = sum_P M[P'][P] delta(P),
//   M[P'][P] = (W(|p' - p|^2) + W(|p' - q|^2)) / 2,
//   delta(P) = t(p up, q down) - t(p down, q up)   (-t(p down, p up) if p = q),
// a square product over the momentum pairs: a quarter of the multiply-adds and
// of the table reads of the product over spin pairs.  M is generated per lane
// in the A-operand layout with the generator of k_ladder (row p', column
// (p, q), no column sign: it is in delta), delta is formed while a chunk of
// kKP pairs is staged in LDS, and the finished u goes to the two rows of P' with
// signs + and -.  The hh ladder 1/2 sum_kl t_kl^ab chi_klij then runs per row on
// the same accumulators (one set per spin row).
//
// The 16-row tiles of pairs map onto the four blocks of the instruction and the
// 16-column tile is cut into NG groups of four columns (NG = 1 .. 4, the groups
// that hold columns of the channel).  Staging is pipelined one chunk ahead: the
// column descriptors (with the two rows of each pair) of chunk c + 1 are in LDS
// while chunk c is multiplied, so the t loads of chunk c + 1 are in flight then.
template <int NG>
__device__ __forceinline__ void ladder64_item(const DevPtrs& d, const DevChan& c, const DevGroup& G, int g, int cur,
                                              int r0, int ct, uint32_t mask, bool act, double* lutS,
                                              double* tks, int4 (*cvi)[kKP], int2* prs) {
    constexpr int S = 8;
    const char* lutB = (const char*)lutS;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nhh = c.nhh, nlp = c.n_lp;
    const bool pp_on = act && (mask & CCD_T_PP) != 0;
    const bool hh_on = act && (mask & (CCD_T_HH | CCD_T_QHH)) != 0;
    const int64_t T0 = G.t_base + g * G.n_amp + c.t_off;
    const double* tcur = d.t[cur] + T0;
    const int4* lp = d.lpinfo + c.lp_off;
    const int rbase = r0 + 32 * w;
    // this lane's B column inside a group and its output row inside a tile
    const int bj = lane & 3;
    const int orow4 = 4 * ((lane & 15) >> 2) + (lane >> 4);
    const int32_t kpack = (int32_t)((uint32_t)(uint8_t)(int8_t)c.kx | ((uint32_t)(uint8_t)(int8_t)c.ky << 8) |
                                    ((uint32_t)(uint8_t)(int8_t)c.kz << 16));
    const int K2 = c.kx * c.kx + c.ky * c.ky + c.kz * c.kz;
    auto times4 = [](int32_t x) { return (int32_t)(((uint32_t)x << 2) & 0xfcfcfcfcu); };

    // generator rows (A layout)
    int32_t apack[2] = {0, 0};
    int rowA[2] = {0, 0}, rowS[2] = {0, 0};
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const int pr = rbase + 16 * h + (lane & 15);
        const int4 li = pr < nlp ? lp[pr] : make_int4(0, 0, -1, -1);
        const int ax = (int8_t)(li.x & 0xff), ay = (int8_t)((li.x >> 8) & 0xff), az = (int8_t)((li.x >> 16) & 0xff);
        apack[h] = (int32_t)((uint32_t)(uint8_t)(int8_t)(-4 * ax) | ((uint32_t)(uint8_t)(int8_t)(-4 * ay) << 8) |
                             ((uint32_t)(uint8_t)(int8_t)(-4 * az) << 16));
        const int A2 = li.y & 1023;
        const int aK = ax * c.kx + ay * c.ky + az * c.kz;
        rowA[h] = S * A2;
        rowS[h] = S * (2 * A2 - 2 * aK);
    }
    // column descriptor: (4 p as int8, S |p|^2, S (|p|^2 + |q|^2), rows + 1 as
    // two 16-bit fields); padding columns carry p = K, q = 0 and no rows, so
    // both table offsets stay in range and delta is zero
    const int4 cpad = make_int4(times4(kpack), S * K2, S * K2, 0);
    auto cdesc = [&](const int4& li) {
        const int C2 = li.y & 1023, D2 = (li.y >> 10) & 1023;
        return make_int4(times4(li.x), S * C2, S * (C2 + D2),
                         (int)((uint32_t)(li.z + 1) | ((uint32_t)(li.w + 1) << 16)));
    };
    constexpr int kPer = kKP * 16 / 256;
    double tv[kPer];
    // delta of chunk kp from the rows in cvi[b]
    auto load_delta = [&](int kp, int b) {
        const int kn = min(kKP, nlp - kp);
#pragma unroll
        for (int i = 0; i < kPer; i++) {
            const int e = threadIdx.x + 256 * i, kk = e >> 4, cc = ct * 16 + (e & 15);
            double v = 0.0;
            if (kk < kn && cc < nhh) {
                const uint32_t rr = (uint32_t)cvi[b][kk].w;
                const int rp = (int)(rr & 0xffff) - 1, rm = (int)(rr >> 16) - 1;
                const double tp = rp >= 0 ? tcur[(int64_t)rp * nhh + cc] : 0.0;
                const double tm = rm >= 0 ? tcur[(int64_t)rm * nhh + cc] : 0.0;
                v = tp - tm;
            }
            tv[i] = v;
        }
    };
    auto store_delta = [&]() {
#pragma unroll
        for (int i = 0; i < kPer; i++) {
            const int e = threadIdx.x + 256 * i;
            tks[(e >> 4) * 16 + (e & 15)] = tv[i];
        }
    };

    double acc[2][NG][2];
#pragma unroll
    for (int h = 0; h < 2; h++)
#pragma unroll
        for (int q = 0; q < NG; q++) { acc[h][q][0] = 0.0; acc[h][q][1] = 0.0; }

    const double* lutg = d.lut + G.lut_base + g * G.nlut;
    const double lv0 = threadIdx.x < G.nlut ? lutg[threadIdx.x] : 0.0;
    const double lv1 = threadIdx.x + 256 < G.nlut ? lutg[threadIdx.x + 256] : 0.0;
    int4 lpc = cpad;
    if (pp_on && threadIdx.x < kKP && threadIdx.x < nlp) lpc = lp[threadIdx.x];
    // the two spin rows of the tile's pairs, for the hh operands and the stores
    const int2* lpr = (const int2*)lp;
    const int2 myr = (threadIdx.x < kLadderRows && r0 + threadIdx.x < nlp) ? lpr[2 * (r0 + threadIdx.x) + 1]
                                                                           : make_int2(-1, -1);
    __syncthreads();  // the previous item's reads of LDS are done
    lutS[threadIdx.x] = lv0;
    if (threadIdx.x + 256 < kMaxLut) lutS[threadIdx.x + 256] = lv1;
    if (threadIdx.x < kLadderRows) prs[threadIdx.x] = myr;
    if (pp_on) {
        if (threadIdx.x < kKP) cvi[0][threadIdx.x] = threadIdx.x < nlp ? cdesc(lpc) : cpad;
        lpc = cpad;
        if (threadIdx.x < kKP && kKP + threadIdx.x < nlp) lpc = lp[kKP + threadIdx.x];
    }
    __syncthreads();
    if (pp_on) {
        load_delta(0, 0);
        store_delta();
        for (int kp = 0; kp < nlp; kp += kKP) {
            const int b = (kp / kKP) & 1;
            const bool more = kp + kKP < nlp;
            if (more && threadIdx.x < kKP) {
                cvi[b ^ 1][threadIdx.x] = kp + kKP + threadIdx.x < nlp ? cdesc(lpc) : cpad;
                lpc = cpad;
                if (kp + 2 * kKP + threadIdx.x < nlp) lpc = lp[kp + 2 * kKP + threadIdx.x];
            }
            __syncthreads();  // this chunk's delta and the next chunk's descriptors are in LDS
            if (more) load_delta(kp + kKP, b ^ 1);
            const int kn = min(kKP, nlp - kp);
            const int ksteps = (kn + 15) & ~15;
            for (int kk = 0; kk < ksteps; kk += 16) {
                int o1[2][4], o2[2][4];
#pragma unroll
                for (int s2 = 0; s2 < 4; s2++) {
                    const int4 ci = cvi[b][kk + 4 * s2 + (lane >> 4)];
#pragma unroll
                    for (int h = 0; h < 2; h++) {
                        o1[h][s2] = __builtin_amdgcn_sdot4(apack[h], ci.x, rowA[h] + ci.y, false);
                        o2[h][s2] = rowS[h] + ci.z - o1[h][s2];
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
                double x1[2][4], x2[2][4], vb[4][NG];
#pragma unroll
                for (int s2 = 0; s2 < 4; s2++) {
#pragma unroll
                    for (int h = 0; h < 2; h++) {
                        x1[h][s2] = *(const double*)(lutB + o1[h][s2]);
                        x2[h][s2] = *(const double*)(lutB + o2[h][s2]);
                    }
#pragma unroll
                    for (int q = 0; q < NG; q++) vb[s2][q] = tks[(kk + 4 * s2 + (lane >> 4)) * 16 + 4 * q + bj];
                }
#pragma unroll
                for (int s2 = 0; s2 < 4; s2++) {
#pragma unroll
                    for (int h = 0; h < 2; h++) {
                        const double va = x1[h][s2] + x2[h][s2];
#pragma unroll
                        for (int q = 0; q < NG; q++) acc[h][q][s2 & 1] = mfma4(va, vb[s2][q], acc[h][q][s2 & 1]);
                    }
                }
            }
            __syncthreads();  // every wave is done with this chunk
            if (more) store_delta();
        }
        // u of the lane's output pair: + to the (p up, q down) row, - to the other
#pragma unroll
        for (int h = 0; h < 2; h++)
#pragma unroll
            for (int q = 0; q < NG; q++) {
                const double u = acc[h][q][0] + acc[h][q][1];
                acc[h][q][0] = u;
                acc[h][q][1] = -u;
            }
    }
    // the two spin rows of the lane's A-operand pairs and of its output pairs
    int arow[2][2], orow[2][2];
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const int2 ra = prs[32 * w + 16 * h + (lane & 15)], ro = prs[32 * w + 16 * h + orow4];
        arow[h][0] = ra.x; arow[h][1] = ra.y;
        orow[h][0] = ro.x; orow[h][1] = ro.y;
    }
    if (hh_on) {
        // 1/2 sum_kl t_kl^ab chi_klij per spin row: A = t rows, B = chi_klij columns
        const double* xg = d.chh + G.chh_base + g * G.n_chh + c.chh_off;
        for (int k0 = 0; k0 < nhh; k0 += 4) {
            const int kq = k0 + (lane >> 4);
            double bb[NG];
#pragma unroll
            for (int q = 0; q < NG; q++) {
                const int cc = ct * 16 + 4 * q + bj;
                bb[q] = (kq < nhh && cc < nhh) ? xg[kq * nhh + cc] : 0.0;
            }
#pragma unroll
            for (int h = 0; h < 2; h++)
#pragma unroll
                for (int s = 0; s < 2; s++) {
                    const int r = arow[h][s];
                    const double a = (r >= 0 && kq < nhh) ? tcur[(int64_t)r * nhh + kq] : 0.0;
#pragma unroll
                    for (int q = 0; q < NG; q++) acc[h][q][s] = mfma4(a, bb[q], acc[h][q][s]);
                }
        }
    }
    if (act) {
#pragma unroll
        for (int h = 0; h < 2; h++)
#pragma unroll
            for (int s = 0; s < 2; s++) {
                const int r = orow[h][s];
#pragma unroll
                for (int q = 0; q < NG; q++) {
                    const int cc = ct * 16 + 4 * q + bj;
                    if (r >= 0 && cc < nhh) d.rmm[T0 + (int64_t)r * nhh + cc] = acc[h][q][s];
                }
            }
    }
}

__global__ void __launch_bounds__(256, 3) k_ladder64(DevPtrs d, int cur, uint32_t mask, int n_items) {
    __shared__ double lutS[kMaxLut];
    __shared__ __attribute__((aligned(16))) double tks[kKP * 16];
    __shared__ int4 cvi[2][kKP];
    __shared__ int2 prs[kLadderRows];
    for (int bi = blockIdx.x; bi < n_items; bi += gridDim.x) {
        const Item lg = d.it_lg[bi];
        if (lg.chan < 0) continue;
        const int g = lg.start;
        const Item it = d.it_ladder[lg.chan];
        const int r0 = it.start & 0xfffff, ct = it.start >> 20;
        const DevChan c = d.chans[it.chan];
        const DevGroup G = d.groups[c.group];
        const bool act = d.active[G.p0 + g] != 0;
        // groups of four columns of this column tile that hold columns
        const int ng = min(4, (min(16, c.nhh - 16 * ct) + 3) >> 2);
        switch (ng) {
            case 1: ladder64_item<1>(d, c, G, g, cur, r0, ct, mask, act, lutS, tks, cvi, prs); break;
            case 2: ladder64_item<2>(d, c, G, g, cur, r0, ct, mask, act, lutS, tks, cvi, prs); break;
            case 3: ladder64_item<3>(d, c, G, g, cur, r0, ct, mask, act, lutS, tks, cvi, prs); break;
            default: ladder64_item<4>(d, c, G, g, cur, r0, ct, mask, act, lutS, tks, cvi, prs); break;
        }
    }
}

// the update of every amplitude per (elementwise item, problem):
// R = <ab||ij> (S_z = 0) + ladder sums (S_z = 0) + ring slots + one-body terms,
// t_new = R / eps_ij^ab, mixing, and the energy partial of the item
__global__ void __launch_bounds__(256) k_update(DevPtrs d, int cur, double alpha, uint32_t mask, int n_items) {
    __shared__ double sh[4];
    const bool ring_on = (mask & (CCD_T_RING | CCD_T_QRING)) != 0;
    const bool lad_on = (mask & (CCD_T_PP | CCD_T_HH | CCD_T_QHH)) != 0;
    for (int bi = blockIdx.x; bi < n_items; bi += gridDim.x) {
        const Item ig = d.it_ue[bi];
        if (ig.chan < 0) continue;
        const int item = ig.chan, g = ig.start;
        const Item it = d.it_elem[item];
        const DevChan c = d.chans[it.chan];
        const DevGroup G = d.groups[c.group];
        const int nel = c.nhh * c.npp;
        const bool act = d.active[G.p0 + g] != 0;
        const bool lad = lad_on && c.sz == 0;
        const int64_t T0 = G.t_base + g * G.n_amp + c.t_off;
        const double* rowE = d.rowE + G.rowa_base + g * G.n_rows_all + c.rowa_off;
        const double* rowX = d.rowX + G.rowa_base + g * G.n_rows_all + c.rowa_off;
        const double* colE = d.colE + G.cola_base + g * G.n_cols_all + c.cola_off;
        const double* colX = d.colX + G.cola_base + g * G.n_cols_all + c.cola_off;
        double es = 0.0;
        for (int k = 0; k < kElemChunk / 256; k++) {
            const int e = it.start + threadIdx.x + 256 * k;
            if (e < nel && e < it.start + kElemChunk) {
                const int64_t E = T0 + e;
                // <ab||ij> = 0 in S_z = +-1 blocks (two neutrons interact only
                // in the spin singlet), so only S_z = 0 blocks read it
                const double tc = d.t[cur][E], v = c.sz == 0 ? d.vt[E] : 0.0;
                double tm = tc;
                if (act) {
                    const int r = e / c.nhh, col = e - r * c.nhh;
                    double R = v;
                    if (lad) R += d.rmm[E];
                    if (ring_on) R += ring_term(d, G, g, c.t_off + e);
                    R += (rowX[r] - colX[col]) * tc;
                    tm = alpha * (R / (colE[col] - rowE[r])) + (1.0 - alpha) * tc;
                }
                d.t[cur ^ 1][E] = tm;
                es += v * tm;
            }
        }
        const double s = block_sum256(es, sh);
        if (threadIdx.x == 0) d.epart_elem[G.eelem_base + g * (G.elem_hi - G.elem_lo) + (item - G.elem_lo)] = s;
    }
}

__global__ void __launch_bounds__(256) k_energy(DevPtrs d, double tol, double tol_rel, int rule) {
    __shared__ double sh[4];
    energy_of(d, blockIdx.x, tol, tol_rel, rule, sh);
}

// --------------------------------------------------------------------------
// context
// --------------------------------------------------------------------------
enum Family {
    F_INIT = 0, F_DIRECT, F_DSUM, F_DCHI, F_RING_S, F_RING32, F_RING48, F_RING64, F_RING80, F_LADDER, F_UPDATE,
    F_ENERGY, F_NUM
};
// one name per family, in the order above (direct is the chi_klij product
// items, dsum their sums; ring32 .. ring80 are the pair blocks of padded order
// 32 .. 80; the ladder family is the pp + hh ladder sums; update covers every
// amplitude)
static const char* kFamilyNames[F_NUM] = {"init", "direct", "dsum", "dchi", "ring_small", "ring32", "ring48",
                                          "ring64", "ring80", "ladder", "update", "energy"};

struct Region {
    size_t off = 0, bytes = 0;
};

// a captured run of n sweeps and the arguments it was captured with
struct GraphEntry {
    int prec, cur, n, rule;
    uint32_t mask;
    double alpha, tol, tol_rel;
    int32_t tune[CCD_TUNE_LEN];
    hipGraphExec_t exec;
    bool same(int p, int c0, int n0, uint32_t m, double a, double t, double tr, int ru, const int32_t* tu) const {
        return prec == p && cur == c0 && n == n0 && mask == m && alpha == a && tol == t && tol_rel == tr && rule == ru &&
               std::memcmp(tune, tu, sizeof(tune)) == 0;
    }
};

struct ccd_ctx {
    std::vector<HostProblem> probs;
    hipStream_t stream = nullptr;
    // concatenated host tables
    std::vector<DevGroup> dgroups;
    std::vector<DevChan> dchans;
    std::vector<DevPh> dph;
    std::vector<int32_t> lpinfo;
    std::vector<int32_t> st, hh, pp, phst, phmap, zs, csr_ptr, csr_idx, pgrp, pgi, it_sz0;
    std::vector<double> eps, lut, rowE, colE, pscale;
    std::vector<Item> it_elem, it_ladder, it_dchi, it_direct, it_ring_s, it_ring_b, it_lg, it_ue, it_dsub,
        it_dsum;
    int64_t n_dpart = 0, n_dcolp = 0;
    int ring_lo[4] = {0}, ring_n[4] = {0};  // big pair items by padded size n16 = 32, 48, 64, 80
    std::vector<int64_t> prob_t0;  // amplitude index of each problem (caller order)
    std::vector<int> slot_of;      // caller problem -> slot (group order) of the device flags
    int64_t NT = 0;
    int n_rows = 0, n_cols = 0, n_chh = 0, n_eps = 0, n_eparte = 0, max_ph = 0;
    // workspace
    Region r_static, r_t0, r_t1, r_vt, r_chh, r_rows, r_cols, r_dchi, r_zc, r_rowx, r_colx, r_rmm, r_eparte,
        r_ecorr, r_eprev, r_active, r_sweeps, r_ehist, r_dpart, r_dcolp, r_dprev, r_streak;
    size_t ws_bytes = 0;
    char* ws = nullptr;
    bool bound = false;
    int cur = 0;
    std::vector<double> emp2;
    // timing
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, int>> pending;  // (family, first event index)
    size_t ev_used = 0;
    double ms[F_NUM] = {0};
    int64_t launches[F_NUM] = {0};
    // launch shapes (CCD_TUNE_* slots), chosen by ccd_autotune or set by the caller
    int32_t tune[CCD_TUNE_LEN] = {0};
    // replayable sweep graphs
    hipStream_t cap_stream = nullptr;
    // three more streams (ring size buckets, ladder sums), forked from and
    // joined back into the caller's stream with events (default priority)
    hipStream_t aux[3] = {nullptr, nullptr, nullptr};
    hipEvent_t ev_fork = nullptr, ev_mid = nullptr, ev_join[3] = {nullptr, nullptr, nullptr};
    bool aux_ok = false;
    // inside run_sweeps (kernel timing off) a sweep's energy step is left to
    // the next sweep's k_direct launch, or to the end of the run
    bool defer_energy = false, energy_pending = false;
    double pend_tol = 0.0, pend_tol_rel = 0.0;
    int pend_rule = 0;
    std::vector<GraphEntry> graphs;
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

#define STATIC_TABLES(X)                                                  \
    X(st, int32_t) X(eps, double) X(lut, double) X(dgroups, DevGroup)     \
    X(dchans, DevChan) X(dph, DevPh) X(hh, int32_t) X(pp, int32_t)        \
    X(phst, int32_t) X(phmap, int32_t) X(zs, int32_t) X(rowE, double) X(colE, double) \
    X(csr_ptr, int32_t)                                                   \
    X(csr_idx, int32_t) X(pgrp, int32_t) X(pgi, int32_t) X(pscale, double) \
    X(it_elem, Item) X(it_ladder, Item) X(it_sz0, int32_t) X(it_dchi, Item) \
    X(it_direct, Item) X(it_ring_s, Item) X(it_ring_b, Item) X(it_lg, Item) X(it_ue, Item) \
    X(it_dsub, Item) X(it_dsum, Item) X(lpinfo, int32_t)

static DevPtrs make_ptrs(ccd_ctx* c) {
    DevPtrs d;
    char* base = c->ws;
    size_t o = c->r_static.off;
    const void* p_st; const void* p_eps; const void* p_lut; const void* p_dgroups; const void* p_dchans;
    const void* p_dph; const void* p_hh; const void* p_pp; const void* p_phst; const void* p_phmap;
    const void* p_csr_ptr; const void* p_csr_idx; const void* p_pgrp; const void* p_pgi;
    const void* p_it_elem; const void* p_it_ladder; const void* p_it_sz0;
    const void* p_it_dchi; const void* p_it_direct; const void* p_it_ring_s; const void* p_it_ring_b;
    const void* p_it_lg; const void* p_it_ue; const void* p_zs; const void* p_rowE; const void* p_colE;
    const void* p_pscale; const void* p_it_dsub; const void* p_it_dsum;
    const void* p_lpinfo;
#define TAKE(name, T)             \
    p_##name = base + o;          \
    o += align256(c->name.size() * sizeof(T));
    STATIC_TABLES(TAKE)
#undef TAKE
    d.st = (const int32_t*)p_st; d.eps = (const double*)p_eps; d.lut = (const double*)p_lut;
    d.groups = (const DevGroup*)p_dgroups; d.chans = (const DevChan*)p_dchans; d.ph = (const DevPh*)p_dph;
    d.hh = (const int32_t*)p_hh; d.pp = (const int32_t*)p_pp; d.phst = (const int32_t*)p_phst;
    d.phmap = (const int32_t*)p_phmap; d.csr_ptr = (const int32_t*)p_csr_ptr;
    d.csr_idx = (const int32_t*)p_csr_idx; d.pgrp = (const int32_t*)p_pgrp; d.pgi = (const int32_t*)p_pgi;
    d.it_elem = (const Item*)p_it_elem;
    d.it_ladder = (const Item*)p_it_ladder; d.it_sz0 = (const int32_t*)p_it_sz0;
    d.it_dchi = (const Item*)p_it_dchi;
    d.it_direct = (const Item*)p_it_direct; d.it_ring_s = (const Item*)p_it_ring_s;
    d.it_ring_b = (const Item*)p_it_ring_b; d.it_lg = (const Item*)p_it_lg;
    d.it_ue = (const Item*)p_it_ue; d.zs = (const int32_t*)p_zs;
    d.rowE = (const double*)p_rowE; d.colE = (const double*)p_colE;
    d.pscale = (const double*)p_pscale;
    d.it_dsub = (const Item*)p_it_dsub; d.it_dsum = (const Item*)p_it_dsum;
    d.lpinfo = (const int4*)p_lpinfo;
    d.dpart = (double*)(base + c->r_dpart.off);
    d.dcolp = (double*)(base + c->r_dcolp.off);
    d.t[0] = (double*)(base + c->r_t0.off);
    d.t[1] = (double*)(base + c->r_t1.off);
    d.vt = (double*)(base + c->r_vt.off);
    d.chh = (double*)(base + c->r_chh.off);
    d.rowsum = (double*)(base + c->r_rows.off);
    d.colsum = (double*)(base + c->r_cols.off);
    d.dchi = (double*)(base + c->r_dchi.off);
    d.zc = (double*)(base + c->r_zc.off);
    d.rowX = (double*)(base + c->r_rowx.off);
    d.colX = (double*)(base + c->r_colx.off);
    d.rmm = (double*)(base + c->r_rmm.off);
    d.epart_elem = (double*)(base + c->r_eparte.off);
    d.ecorr = (double*)(base + c->r_ecorr.off);
    d.eprev = (double*)(base + c->r_eprev.off);
    d.active = (int32_t*)(base + c->r_active.off);
    d.sweeps = (int32_t*)(base + c->r_sweeps.off);
    d.ehist = (double*)(base + c->r_ehist.off);
    d.dprev = (double*)(base + c->r_dprev.off);
    d.streak = (int32_t*)(base + c->r_streak.off);
    return d;
}

// host image of the static tables, in the order make_ptrs takes them
static std::vector<char> static_image(const ccd_ctx* c) {
    std::vector<char> img(c->r_static.bytes, 0);
    size_t o = 0;
#define PUT(name, T)                                                              \
    if (!c->name.empty()) std::memcpy(img.data() + o, c->name.data(), c->name.size() * sizeof(T)); \
    o += align256(c->name.size() * sizeof(T));
    STATIC_TABLES(PUT)
#undef PUT
    return img;
}

static void layout(ccd_ctx* c) {
    size_t s = 0;
#define ADD(name, T) s += align256(c->name.size() * sizeof(T));
    STATIC_TABLES(ADD)
#undef ADD
    size_t o = 0;
    auto region = [&](Region& r, size_t bytes) {
        r.off = o;
        r.bytes = bytes;
        o += align256(std::max<size_t>(bytes, 8));
    };
    size_t P = c->probs.size();
    region(c->r_static, s);
    region(c->r_t0, c->NT * 8);
    region(c->r_t1, c->NT * 8);
    region(c->r_vt, c->NT * 8);
    region(c->r_chh, (size_t)c->n_chh * 8);
    region(c->r_dpart, (size_t)c->n_dpart * 8);
    region(c->r_dcolp, (size_t)c->n_dcolp * 8);
    region(c->r_rows, (size_t)c->n_rows * 8);
    region(c->r_cols, (size_t)c->n_cols * 8);
    region(c->r_dchi, (size_t)c->n_eps * 8);
    region(c->r_zc, (size_t)c->NT * 16);
    region(c->r_rowx, c->rowE.size() * 8);
    region(c->r_colx, c->colE.size() * 8);
    region(c->r_rmm, (size_t)c->NT * 8);
    region(c->r_eparte, (size_t)c->n_eparte * 8);
    region(c->r_ecorr, P * 8);
    region(c->r_eprev, P * 8);
    region(c->r_active, P * 4);
    region(c->r_sweeps, P * 4);
    region(c->r_ehist, P * kHistCap * 8);
    region(c->r_dprev, P * 8);
    region(c->r_streak, P * 4);
    c->ws_bytes = o;
}

// Blocks are dispatched to the eight XCDs round-robin by block index.  Work
// lists sorted by problem are cut into eight contiguous pieces, piece x going
// to XCD x, so each XCD's L2 sees the data of about one problem.  Units of u
// consecutive items stay together; padding items have chan = -1.
static std::vector<Item> xcd_order(std::vector<std::pair<int, Item>> v, int u = 1) {
    std::stable_sort(v.begin(), v.end(), [](const std::pair<int, Item>& a, const std::pair<int, Item>& b) {
        return a.first < b.first;
    });
    const size_t nunits = (v.size() + u - 1) / u;
    if (nunits == 0) return {};
    const size_t per = (nunits + 7) / 8;
    std::vector<Item> out(per * 8 * u, Item{-1, 0});
    for (size_t k = 0; k < v.size(); k++) {
        const size_t unit = k / u, x = unit / per, j = unit % per;
        out[(j * 8 + x) * u + k % u] = v[k].second;
    }
    return out;
}

// The same for items of uneven cost: the eight pieces are cut at equal shares
// of the total cost (still contiguous in problem order), and inside a piece the
// costliest items come first, so long items do not start last (with
// per_problem, costliest first within each problem's run of the piece, so
// the piece still works through one problem's data at a time).
static std::vector<Item> xcd_order_cost(const std::vector<std::pair<int, Item>>& v, const std::vector<double>& cost,
                                        bool per_problem = false) {
    std::vector<size_t> idx(v.size());
    for (size_t k = 0; k < idx.size(); k++) idx[k] = k;
    std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return v[a].first < v[b].first; });
    double total = 0.0;
    for (double x : cost) total += x;
    std::vector<std::vector<size_t>> piece(8);
    double run = 0.0;
    for (size_t k : idx) {
        const int x = total > 0.0 ? std::min(7, (int)(8.0 * run / total)) : 0;
        piece[x].push_back(k);
        run += cost[k];
    }
    size_t per = 0;
    for (auto& pc : piece) {
        std::stable_sort(pc.begin(), pc.end(), [&](size_t a, size_t b) {
            if (per_problem && v[a].first != v[b].first) return v[a].first < v[b].first;
            return cost[a] > cost[b];
        });
        per = std::max(per, pc.size());
    }
    std::vector<Item> out(per * 8, Item{-1, 0});
    for (int x = 0; x < 8; x++)
        for (size_t j = 0; j < piece[x].size(); j++) out[j * 8 + x] = v[piece[x][j]].second;
    return out;
}

// group the problems by structure (N, nmax2 and the twist, which decides the
// hole set) and lay out the device tables
static ccd_status assemble(ccd_ctx* c) {
    using SKey = std::tuple<int, int, double, double, double>;
    std::map<SKey, std::vector<int>> by_structure;
    for (size_t p = 0; p < c->probs.size(); p++) {
        const ccd_problem& q = c->probs[p].par;
        // +0.0 folds -0.0 into 0.0, so a zero twist of either sign is one structure
        by_structure[SKey{q.n_particles, q.nmax2, q.twist[0] + 0.0, q.twist[1] + 0.0, q.twist[2] + 0.0}]
            .push_back((int)p);
    }
    const size_t P = c->probs.size();
    c->pgrp.assign(P, 0);
    c->pgi.assign(P, 0);
    c->prob_t0.assign(P, 0);
    c->slot_of.assign(P, 0);
    std::vector<std::pair<int, Item>> lg, ue, dir, dsum, rs, rb[4];
    std::vector<double> lg_cost, dir_cost, rb_cost[4];
    int64_t t_base = 0;
    int gi = 0, slot0 = 0;
    for (auto& kv : by_structure) {
        const std::vector<int>& members = kv.second;
        const HostProblem& H = c->probs[members[0]];
        DevGroup D;
        std::memset(&D, 0, sizeof(D));
        D.G = (int)members.size();
        D.p0 = slot0;
        D.ns = H.ns; D.nh = H.nh; D.np = H.np; D.nlut = (int)H.W.size();
        D.n_amp = H.n_amp;
        D.t_base = t_base;
        D.st_off = (int)c->st.size();
        D.eps_base = c->n_eps;
        D.lut_base = (int)c->lut.size();
        for (int s = 0; s < H.ns; s++) c->st.push_back(pack_state(H.nx[s], H.ny[s], H.nz[s], H.sz[s]));
        for (int g = 0; g < D.G; g++) {
            const HostProblem& Hg = c->probs[members[g]];
            c->eps.insert(c->eps.end(), Hg.eps.begin(), Hg.eps.end());
            for (double wv : Hg.W) c->lut.push_back(0.5 * wv);
            c->pgrp[members[g]] = gi;
            c->pgi[members[g]] = g;
            c->slot_of[members[g]] = slot0 + g;
            c->prob_t0[members[g]] = t_base + (int64_t)g * H.n_amp;
        }
        c->n_eps += D.G * H.ns;
        // direct channels
        const int hh0 = (int)c->hh.size(), pp0 = (int)c->pp.size();
        for (size_t k = 0; k < H.hh.size() / 2; k++) c->hh.push_back(pack_pair(H.hh[2 * k], H.hh[2 * k + 1]));
        for (size_t k = 0; k < H.pp.size() / 2; k++) c->pp.push_back(pack_pair(H.pp[2 * k], H.pp[2 * k + 1]));
        int rows = 0, cols = 0, chh = 0, dpart = 0, dcolp = 0;
        std::vector<std::vector<int32_t>> lists(H.ns);
        D.ladder_lo = (int)c->it_ladder.size();
        D.elem_lo = (int)c->it_elem.size();
        for (const Chan& h : H.chans) {
            DevChan dc;
            std::memset(&dc, 0, sizeof(dc));
            dc.t_off = h.t_off;
            dc.group = gi;
            dc.nhh = h.nhh; dc.npp = h.npp; dc.sz = h.Sz;
            dc.hh_off = hh0 + h.hh_off;
            dc.pp_off = pp0 + h.pp_off;
            dc.chh_off = -1; dc.row_off = -1; dc.col_off = -1;
            dc.kx = h.Kx; dc.ky = h.Ky; dc.kz = h.Kz;
            dc.rowa_off = h.pp_off;
            dc.cola_off = h.hh_off;
            const int id = (int)c->dchans.size();
            if (h.Sz == 0) {
                dc.chh_off = chh; chh += h.nhh * h.nhh;
                dc.row_off = rows;
                dc.col_off = cols;
                for (int r = 0; r < h.npp; r++) {
                    lists[H.pp[2 * (h.pp_off + r)]].push_back(-(rows + r) - 1);
                    lists[H.pp[2 * (h.pp_off + r) + 1]].push_back(-(rows + r) - 1);
                }
                for (int q = 0; q < h.nhh; q++) {
                    lists[H.hh[2 * (h.hh_off + q)]].push_back(cols + q);
                    lists[H.hh[2 * (h.hh_off + q) + 1]].push_back(cols + q);
                }
                rows += h.npp; cols += h.nhh;
                c->it_sz0.push_back(id);
                dc.dsub_lo = (int)c->it_dsub.size();
                dc.dpart_off = dpart;
                dc.dcolp_off = dcolp;
                for (int k0 = 0; k0 < h.npp; k0 += kDirSplit) {
                    const int si = (int)c->it_dsub.size();
                    c->it_dsub.push_back({id, k0});
                    // staged rows times output tiles: the long items go first,
                    // so that they do not run alone at the end of the launch
                    const int nt = (h.nhh + 15) / 16;
                    for (int g = 0; g < D.G; g++) {
                        dir.push_back({slot0 + g, Item{si, g}});
                        dir_cost.push_back((double)std::min(kDirSplit, h.npp - k0) * nt * nt + 64.0);
                    }
                    dpart += h.nhh * h.nhh;
                    dcolp += h.nhh;
                }
                dc.dsub_n = (int)c->it_dsub.size() - dc.dsub_lo;
                for (int g = 0; g < D.G; g++) dsum.push_back({slot0 + g, Item{id, g}});
                // momentum pairs {n_a, n_b} of the rows, in order of first row;
                // a row's pair is keyed by n_a (b follows from K and the spins)
                if (h.npp >= 0xffff) {  // rows travel as 16-bit fields in the kernel
                    set_error("an S_z = 0 block has more than 65534 particle pairs");
                    return CCD_EINVAL;
                }
                dc.lp_off = (int)(c->lpinfo.size() / 4);
                std::map<std::tuple<int, int, int>, int> lp_of;
                std::vector<std::array<int32_t, 4>> lps;
                for (int r = 0; r < h.npp; r++) {
                    const int a = H.pp[2 * (h.pp_off + r)], b = H.pp[2 * (h.pp_off + r) + 1];
                    auto ins = lp_of.insert({{H.nx[a], H.ny[a], H.nz[a]}, (int)lps.size()});
                    if (ins.second) {
                        const int A2 = H.nx[a] * H.nx[a] + H.ny[a] * H.ny[a] + H.nz[a] * H.nz[a];
                        const int B2 = H.nx[b] * H.nx[b] + H.ny[b] * H.ny[b] + H.nz[b] * H.nz[b];
                        lps.push_back({pack_state(H.nx[a], H.ny[a], H.nz[a], 0), A2 | (B2 << 10), -1, -1});
                    }
                    int32_t& slot = lps[ins.first->second][H.sz[a] > 0 ? 2 : 3];
                    if (slot >= 0) {
                        set_error("internal: two rows of one S_z = 0 block share a and its spin");
                        return CCD_EINVAL;
                    }
                    slot = r;
                }
                if ((int)lps.size() != h.nlp) {
                    set_error("internal: momentum-pair count of an S_z = 0 block");
                    return CCD_EINVAL;
                }
                for (auto& e : lps) c->lpinfo.insert(c->lpinfo.end(), e.begin(), e.end());
                dc.n_lp = h.nlp;
                // ladder items: kLadderRows pairs by 16 columns
                for (int r0 = 0; r0 < h.nlp; r0 += kLadderRows)
                    for (int ct = 0; ct < (h.nhh + 15) / 16; ct++) {
                        const int li = (int)c->it_ladder.size();
                        c->it_ladder.push_back({id, r0 | (ct << 20)});
                        for (int g = 0; g < D.G; g++) {
                            lg.push_back({slot0 + g, Item{li, g}});
                            lg_cost.push_back((double)h.nlp);  // MFMA steps of the item
                        }
                    }
            }
            const int nel = h.nhh * h.npp;
            for (int e0 = 0; e0 < nel; e0 += kElemChunk) {
                const int ei = (int)c->it_elem.size();
                c->it_elem.push_back({id, e0});
                for (int g = 0; g < D.G; g++) ue.push_back({slot0 + g, Item{ei, g}});
            }
            c->dchans.push_back(dc);
        }
        D.ladder_hi = (int)c->it_ladder.size();
        D.elem_hi = (int)c->it_elem.size();
        D.n_rows = rows; D.n_cols = cols; D.n_chh = chh;
        D.n_dpart = dpart; D.n_dcolp = dcolp;
        D.dpart_base = c->n_dpart; D.dcolp_base = c->n_dcolp;
        c->n_dpart += (int64_t)D.G * dpart; c->n_dcolp += (int64_t)D.G * dcolp;
        D.rows_base = c->n_rows; D.cols_base = c->n_cols; D.chh_base = c->n_chh;
        c->n_rows += D.G * rows; c->n_cols += D.G * cols; c->n_chh += D.G * chh;
        D.eelem_base = c->n_eparte;
        c->n_eparte += D.G * (D.elem_hi - D.elem_lo);
        // one-body CSR
        D.csr_off = (int)c->csr_ptr.size();
        c->csr_ptr.push_back((int32_t)c->csr_idx.size());
        for (auto& l : lists) {
            c->csr_idx.insert(c->csr_idx.end(), l.begin(), l.end());
            c->csr_ptr.push_back((int32_t)c->csr_idx.size());
        }
        for (int g = 0; g < D.G; g++)
            for (int s0 = 0; s0 < H.ns; s0 += 4) c->it_dchi.push_back({gi, s0 | (g << 16)});
        // per-row / per-column Fock sums of every problem, ring indices
        D.pp0 = pp0; D.hh0 = hh0;
        D.n_rows_all = (int)H.pp.size() / 2;
        D.n_cols_all = (int)H.hh.size() / 2;
        D.rowa_base = (int)c->rowE.size();
        D.cola_base = (int)c->colE.size();
        for (int g = 0; g < D.G; g++) {
            const HostProblem& Hg = c->probs[members[g]];
            for (size_t k = 0; k < H.pp.size() / 2; k++) c->rowE.push_back(Hg.eps[H.pp[2 * k]] + Hg.eps[H.pp[2 * k + 1]]);
            for (size_t k = 0; k < H.hh.size() / 2; k++) c->colE.push_back(Hg.eps[H.hh[2 * k]] + Hg.eps[H.hh[2 * k + 1]]);
        }
        D.zidx_off = (int64_t)c->zs.size();
        c->zs.insert(c->zs.end(), H.zs.begin(), H.zs.end());
        // cross channels and their pairs {Q, -Q}; the lower index is the primary
        const int ph0 = (int)c->dph.size(), mem0 = (int)c->phst.size() / 2;
        const int64_t map0 = (int64_t)c->phmap.size();
        const int64_t nzp = H.n_zp;
        for (size_t qi = 0; qi < H.ph.size(); qi++) {
            const PhChan& h = H.ph[qi];
            DevPh dp;
            std::memset(&dp, 0, sizeof(dp));
            dp.map_off = map0 + h.z_off;
            dp.group = gi;
            dp.n = h.n;
            dp.m = H.ph[h.partner].n;
            dp.partner = ph0 + h.partner;
            dp.mem_off = mem0 + h.mem_off;
            dp.pmem_off = mem0 + H.ph[h.partner].mem_off;
            dp.zp_off = h.zp_off;
            const int pid = (int)c->dph.size();
            if (h.zp_off >= 0) {
                const int nb = std::max(h.n, dp.m);  // the pair's padded order
                for (int g = 0; g < D.G; g++) {
                    if (nb <= 16) rs.push_back({slot0 + g, Item{pid, g}});
                    else {
                        // an item's gather grows with n m, its products with n m (n + m)
                        const int k = ((nb + 15) >> 4) - 2;
                        rb[k].push_back({slot0 + g, Item{pid, g}});
                        rb_cost[k].push_back((double)h.n * dp.m * (h.n + dp.m + 16));
                    }
                }
            }
            c->dph.push_back(dp);
            c->max_ph = std::max(c->max_ph, h.n);
        }
        for (size_t k = 0; k < H.phmem.size(); k++) {
            const int x = H.phmem[k];
            c->phst.push_back(pack_state(H.nx[x], H.ny[x], H.nz[x], H.sz[x]));
        }
        c->phmap.insert(c->phmap.end(), H.phmap.begin(), H.phmap.end());
        D.phq_off = 0;
        D.ph_base = (int)map0;
        D.n_zp = nzp;
        c->dgroups.push_back(D);
        t_base += (int64_t)D.G * H.n_amp;
        slot0 += D.G;
        gi++;
    }
    c->NT = t_base;

    if (c->csr_idx.empty()) c->csr_idx.push_back(0);
    c->it_lg = xcd_order_cost(lg, lg_cost);
    c->it_ue = xcd_order(ue);
    c->it_direct = xcd_order_cost(dir, dir_cost);
    c->it_dsum = xcd_order(dsum);
    c->it_ring_s = xcd_order(rs, 4);
    c->it_ring_b.clear();
    for (int k = 0; k < 4; k++) {
        // a bucket that fits one round of two blocks per compute unit ends with
        // its longest item: its pieces are cut at equal cost, costliest first;
        // over several rounds the problem and pair order keeps the L2 working set
        // of a piece smaller (10 problems at N=66, n^2<=20: ring32 46 -> 50 us
        // in cost order)
        std::vector<Item> o = rb[k].size() <= 512 ? xcd_order_cost(rb[k], rb_cost[k], true) : xcd_order(rb[k]);
        c->ring_lo[k] = (int)c->it_ring_b.size();
        c->ring_n[k] = (int)o.size();
        c->it_ring_b.insert(c->it_ring_b.end(), o.begin(), o.end());
    }
    // per-slot copies of (group, index in group) for the per-problem kernels
    std::vector<int32_t> sg(P), sgi(P);
    for (size_t p = 0; p < P; p++) {
        sg[c->slot_of[p]] = c->pgrp[p];
        sgi[c->slot_of[p]] = c->pgi[p];
    }
    c->pgrp = sg;
    c->pgi = sgi;
    c->pscale.assign(3 * P, 0.0);
    for (size_t p = 0; p < P; p++) {
        const HostProblem& H = c->probs[p];
        const int sl = c->slot_of[p];
        c->pscale[3 * sl] = H.par.density;
        c->pscale[3 * sl + 1] = 2.0 * M_PI / H.L;
        c->pscale[3 * sl + 2] = H.L * H.L * H.L / mlp::kVScale;
    }
    layout(c);
    return CCD_OK;
}

// ---- timing ----------------------------------------------------------------
static hipError_t ev_begin(ccd_ctx* c, int fam) {
    if (!c->timing) return hipSuccess;
    while (c->ev_used + 2 > c->ev_pool.size()) {
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        c->ev_pool.push_back(e);
    }
    c->pending.push_back({fam, (int)c->ev_used});
    hipError_t r = hipEventRecord(c->ev_pool[c->ev_used], c->stream);
    c->ev_used += 2;
    return r;
}
static hipError_t ev_end(ccd_ctx* c) {
    if (!c->timing) return hipSuccess;
    return hipEventRecord(c->ev_pool[c->pending.back().second + 1], c->stream);
}
static ccd_status harvest(ccd_ctx* c) {
    if (c->pending.empty()) return CCD_OK;
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (auto& p : c->pending) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, c->ev_pool[p.second], c->ev_pool[p.second + 1]));
        c->ms[p.first] += ms;
        c->launches[p.first] += 1;
    }
    c->pending.clear();
    c->ev_used = 0;
    return CCD_OK;
}

#define LAUNCH(fam, kernel, grid, block, shmem, ...)                                    \
    do {                                                                                \
        if ((grid) > 0) {                                                               \
            HIP_TRY(ev_begin(c, fam));                                                  \
            hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), shmem, c->stream, __VA_ARGS__); \
            HIP_TRY(hipGetLastError());                                                 \
            HIP_TRY(ev_end(c));                                                         \
        }                                                                               \
    } while (0)


static ccd_status refresh_energy(ccd_ctx* c) {
    DevPtrs d = make_ptrs(c);
    LAUNCH(F_INIT, k_dot, (int)c->it_elem.size(), 256, 0, d, c->cur);
    LAUNCH(F_ENERGY, k_energy_elem, (int)c->probs.size(), 256, 0, d);
    return CCD_OK;
}

// grid of a family: one block per item, or (slot value m > 0) a persistent
// grid of m blocks per compute unit looping over the items; a multiple of 8
// keeps every item on the XCD that xcd_order chose for it
static int grid_for(const ccd_ctx* c, int slot, int nb) {
    const int m = c->tune[slot];
    if (m <= 0 || nb <= 0) return nb;
    return std::min(nb, m * 256);
}

// the energy step left over from the previous sweep, as its own launch
static ccd_status flush_energy(ccd_ctx* c, const DevPtrs& d) {
    if (!c->energy_pending) return CCD_OK;
    c->energy_pending = false;
    LAUNCH(F_ENERGY, k_energy, (int)c->probs.size(), 256, 0, d, c->pend_tol, c->pend_tol_rel, c->pend_rule);
    return CCD_OK;
}

template <int P>
static ccd_status L_direct(ccd_ctx* c, const DevPtrs& d, int cur, uint32_t mask) {
    const int n = (int)c->it_direct.size(), ns = (int)c->it_dsum.size();
    if (mask & (CCD_T_QHH | CCD_T_QHOLE | CCD_T_QPART)) {
        const int nd = grid_for(c, CCD_TUNE_DIRECT, n);
        if (c->energy_pending && nd > 0) {
            // the previous sweep's energy step rides on this launch (its last blocks)
            c->energy_pending = false;
            LAUNCH(F_DIRECT, k_direct<P>, nd + (int)c->probs.size(), 256, 0, d, cur, mask, n, nd, 1, c->pend_tol,
                   c->pend_tol_rel, c->pend_rule);
        } else {
            LAUNCH(F_DIRECT, k_direct<P>, nd, 256, 0, d, cur, mask, n, nd, 0, 0.0, 0.0, 0);
        }
    }
    if (mask & (CCD_T_HH | CCD_T_QHH | CCD_T_QHOLE))
        LAUNCH(F_DSUM, k_dsum, ns, 256, 0, d, mask, ns);
    return CCD_OK;
}

static ccd_status L_dchi(ccd_ctx* c, const DevPtrs& d, uint32_t mask) {
    const int n = (int)c->it_dchi.size();
    LAUNCH(F_DCHI, k_dchi, grid_for(c, CCD_TUNE_DCHI, n), 256, 0, d, mask, n);
    int maxe = 0;
    for (const DevGroup& D : c->dgroups) maxe = std::max(maxe, D.n_rows_all + D.n_cols_all);
    HIP_TRY(ev_begin(c, F_DCHI));
    hipLaunchKernelGGL(k_onebody, dim3((maxe + 255) / 256, (int)c->probs.size()), dim3(256), 0, c->stream, d);
    HIP_TRY(hipGetLastError());
    HIP_TRY(ev_end(c));
    return CCD_OK;
}

template <int P>
static ccd_status L_ring_small(ccd_ctx* c, const DevPtrs& d, int cur, uint32_t mask) {
    const int n = (int)c->it_ring_s.size();
    if (mask & (CCD_T_RING | CCD_T_QRING))
        LAUNCH(F_RING_S, k_ringp_small<P>, grid_for(c, CCD_TUNE_RING_SMALL, (n + 3) / 4), 256, 0, d, cur, mask, n);
    return CCD_OK;
}

// waves per block of each ring size class: slot value 0 -> NWA, 1 -> NWB
template <int P, int N16, int NWA, int NWB>
static ccd_status L_ring_class(ccd_ctx* c, const DevPtrs& d, int cur, uint32_t mask, int k) {
    const int n = c->ring_n[k], lo = c->ring_lo[k];
    const int grid = grid_for(c, CCD_TUNE_RING, n);
    if (c->tune[CCD_TUNE_RING_NW32 + k] == 0)
        LAUNCH(F_RING32 + k, (k_ringp<P, N16, NWA>), grid, 64 * NWA, pair_lds<P>(N16), d, cur, mask, lo, n);
    else
        LAUNCH(F_RING32 + k, (k_ringp<P, N16, NWB>), grid, 64 * NWB, pair_lds<P>(N16), d, cur, mask, lo, n);
    return CCD_OK;
}

template <int P>
static ccd_status L_ring(ccd_ctx* c, const DevPtrs& d, int cur, uint32_t mask, int only = -1) {
    if (!(mask & (CCD_T_RING | CCD_T_QRING))) return CCD_OK;
    ccd_status s = CCD_OK;
    if (s == CCD_OK && (only < 0 || only == 0)) s = L_ring_class<P, 32, 4, 2>(c, d, cur, mask, 0);
    if (s == CCD_OK && (only < 0 || only == 1)) s = L_ring_class<P, 48, 9, 3>(c, d, cur, mask, 1);
    if (s == CCD_OK && (only < 0 || only == 2)) s = L_ring_class<P, 64, 16, 8>(c, d, cur, mask, 2);
    if (s == CCD_OK && (only < 0 || only == 3)) s = L_ring_class<P, 80, 16, 9>(c, d, cur, mask, 3);
    return s;
}

template <int P>
static ccd_status L_ladder(ccd_ctx* c, const DevPtrs& d, int cur, uint32_t mask) {
    const int n = (int)c->it_lg.size();
    if (mask & (CCD_T_PP | CCD_T_HH | CCD_T_QHH)) {
        if constexpr (P == P_F64) {
            LAUNCH(F_LADDER, k_ladder64, grid_for(c, CCD_TUNE_LADDER, n), 256, 0, d, cur, mask, n);
        } else {
            LAUNCH(F_LADDER, k_ladder<P>, grid_for(c, CCD_TUNE_LADDER, n), 256, 0, d, cur, mask, n);
        }
    }
    return CCD_OK;
}

static ccd_status L_update(ccd_ctx* c, const DevPtrs& d, int cur, double alpha, uint32_t mask) {
    const int n = (int)c->it_ue.size();
    LAUNCH(F_UPDATE, k_update, grid_for(c, CCD_TUNE_UPDATE, n), 256, 0, d, cur, alpha, mask, n);
    return CCD_OK;
}

// launches made while it lives go to stream `to` instead of the context's stream
struct StreamSwap {
    ccd_ctx* c;
    hipStream_t saved;
    StreamSwap(ccd_ctx* cc, hipStream_t to) : c(cc), saved(cc->stream) { c->stream = to; }
    ~StreamSwap() { c->stream = saved; }
};

// The ring reads only t[cur] and static tables and writes only the ring
// slots; the ladder sums read t[cur] and chi_klij and write only rmm; the
// one-body sums read the row and column sums and write only their own arrays.
// So the ring size buckets run on two auxiliary streams from the start of the
// sweep, and once chi_klij is complete the one-body sums fork to a third while
// the ladder, the longest chain, stays on the context's stream (a cross-stream
// wait costs ~10 us on this ROCm, and the chain direct -> dsum -> ladder ->
// update is the critical one); the update waits for all of them.  With kernel
// timing on, everything stays on the context's stream so that the per-family
// event times are not overlapped.
template <int P>
static ccd_status launch_contractions(ccd_ctx* c, const DevPtrs& d, int cur, uint32_t mask) {
    const bool fork = c->aux_ok && !c->timing;
    ccd_status s = CCD_OK;
    // a pending energy step that no k_direct launch of this sweep can carry
    // runs first, on its own
    if (c->energy_pending && !((mask & (CCD_T_QHH | CCD_T_QHOLE | CCD_T_QPART)) && !c->it_direct.empty())) {
        s = flush_energy(c, d);
        if (s != CCD_OK) return s;
    }
    if (fork) {
        HIP_TRY(hipEventRecord(c->ev_fork, c->stream));
        for (int k = 0; k < 2; k++) HIP_TRY(hipStreamWaitEvent(c->aux[k], c->ev_fork, 0));
        // the critical chain's first kernel is submitted before the rings: the
        // dependencies are the same, but when the host runs close behind the
        // GPU (a profiler, a busy host) it reaches the GPU first
        s = L_direct<P>(c, d, cur, mask);
        if (s == CCD_OK) {
            StreamSwap sw(c, c->aux[0]);
            s = L_ring<P>(c, d, cur, mask, 2);
            if (s == CCD_OK) s = L_ring<P>(c, d, cur, mask, 3);
            if (s == CCD_OK) s = L_ring_small<P>(c, d, cur, mask);
        }
        if (s == CCD_OK) {
            StreamSwap sw(c, c->aux[1]);
            s = L_ring<P>(c, d, cur, mask, 1);
            if (s == CCD_OK) s = L_ring<P>(c, d, cur, mask, 0);
        }
        if (s == CCD_OK) {
            HIP_TRY(hipEventRecord(c->ev_mid, c->stream));
            s = L_ladder<P>(c, d, cur, mask);  // submitted first, as k_direct above
        }
        if (s == CCD_OK) {
            HIP_TRY(hipStreamWaitEvent(c->aux[2], c->ev_mid, 0));
            StreamSwap sw(c, c->aux[2]);
            s = L_dchi(c, d, mask);
        }
        // one join on the context's stream: the third stream, whose one-body
        // sums end well before the ladder, takes the waits for the two ring
        // streams (every wait is a barrier packet that costs a few us even when
        // its event has completed)
        for (int k = 0; k < 2; k++) {
            HIP_TRY(hipEventRecord(c->ev_join[k], c->aux[k]));
            HIP_TRY(hipStreamWaitEvent(c->aux[2], c->ev_join[k], 0));
        }
        HIP_TRY(hipEventRecord(c->ev_join[2], c->aux[2]));
        HIP_TRY(hipStreamWaitEvent(c->stream, c->ev_join[2], 0));
    } else {
        s = L_direct<P>(c, d, cur, mask);
        if (s == CCD_OK) s = L_dchi(c, d, mask);
        if (s == CCD_OK) s = L_ring_small<P>(c, d, cur, mask);
        if (s == CCD_OK) s = L_ring<P>(c, d, cur, mask);
        if (s == CCD_OK) s = L_ladder<P>(c, d, cur, mask);
    }
    return s;
}

template <int P, int N16, int NWA, int NWB>
static hipError_t set_ring_attr_pair() {
    hipError_t e = hipFuncSetAttribute((const void*)k_ringp<P, N16, NWA>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)pair_lds<P>(N16));
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_ringp<P, N16, NWB>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)pair_lds<P>(N16));
}

template <int P>
static hipError_t set_ring_attrs() {
    hipError_t e;
    if ((e = set_ring_attr_pair<P, 32, 4, 2>()) != hipSuccess) return e;
    if ((e = set_ring_attr_pair<P, 48, 9, 3>()) != hipSuccess) return e;
    if ((e = set_ring_attr_pair<P, 64, 16, 8>()) != hipSuccess) return e;
    return set_ring_attr_pair<P, 80, 16, 9>();
}

static ccd_status sweep(ccd_ctx* c, double alpha, double tol, double tol_rel, int rule, uint32_t mask, int prec) {
    DevPtrs d = make_ptrs(c);
    const int cur = c->cur;
    ccd_status s = prec == CCD_PREC_BF16 ? launch_contractions<P_BF16>(c, d, cur, mask)
                 : prec == CCD_PREC_FP32 ? launch_contractions<P_F32>(c, d, cur, mask)
                                         : launch_contractions<P_F64>(c, d, cur, mask);
    if (s != CCD_OK) return s;
    s = L_update(c, d, cur, alpha, mask);
    if (s != CCD_OK) return s;
    s = flush_energy(c, d);  // not left by a k_direct launch of this sweep (none)
    if (s != CCD_OK) return s;
    if (c->defer_energy && !c->timing) {
        // the energy step of this sweep rides on the next sweep's k_direct launch
        // (or runs at the end of the run), so that nothing sits between this
        // update and the next sweep's fork
        c->energy_pending = true;
        c->pend_tol = tol;
        c->pend_tol_rel = tol_rel;
        c->pend_rule = rule;
    } else {
        LAUNCH(F_ENERGY, k_energy, (int)c->probs.size(), 256, 0, d, tol, tol_rel, rule);
    }
    c->cur ^= 1;
    return CCD_OK;
}

// n sweeps: launched one by one, or (graph) as one replay of a captured graph
// of the same n sweeps; kernel timing disables the graph
static constexpr size_t kMaxGraphs = 4;
// the energy steps of a run's sweeps are deferred (see sweep) and the last one
// is launched before the run returns
struct DeferEnergy {
    ccd_ctx* c;
    explicit DeferEnergy(ccd_ctx* cc) : c(cc) { c->defer_energy = true; c->energy_pending = false; }
    ~DeferEnergy() { c->defer_energy = false; c->energy_pending = false; }
};
static ccd_status run_sweeps(ccd_ctx* c, int n, double alpha, double tol, double tol_rel, int rule, uint32_t mask,
                             int prec, bool graph) {
    DeferEnergy de(c);
    if (!graph || c->timing) {
        for (int k = 0; k < n; k++) {
            ccd_status s = sweep(c, alpha, tol, tol_rel, rule, mask, prec);
            if (s != CCD_OK) return s;
        }
        return flush_energy(c, make_ptrs(c));
    }
    GraphEntry* ge = nullptr;
    for (GraphEntry& g : c->graphs)
        if (g.same(prec, c->cur, n, mask, alpha, tol, tol_rel, rule, c->tune)) ge = &g;
    if (!ge) {
        // captured on a private stream (the caller's may be the null stream),
        // replayed on the caller's stream in order with its other work
        if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        const hipStream_t user = c->stream;
        const int cur0 = c->cur;
        HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        c->stream = c->cap_stream;
        ccd_status s = CCD_OK;
        for (int k = 0; k < n && s == CCD_OK; k++) s = sweep(c, alpha, tol, tol_rel, rule, mask, prec);
        if (s == CCD_OK) s = flush_energy(c, make_ptrs(c));  // inside the captured graph
        c->energy_pending = false;
        hipGraph_t gr = nullptr;
        const hipError_t ec = hipStreamEndCapture(c->cap_stream, &gr);
        c->stream = user;
        c->cur = cur0;
        if (s != CCD_OK) {
            if (gr) (void)hipGraphDestroy(gr);
            return s;
        }
        if (ec != hipSuccess) {
            set_error(std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
            return CCD_EHIP;
        }
        hipGraphExec_t ex = nullptr;
        const hipError_t ei = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        if (ei != hipSuccess) {
            set_error(std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
            return CCD_EHIP;
        }
        if (c->graphs.size() >= kMaxGraphs) {
            (void)hipGraphExecDestroy(c->graphs.front().exec);
            c->graphs.erase(c->graphs.begin());
        }
        GraphEntry e;
        e.prec = prec; e.cur = cur0; e.n = n; e.mask = mask; e.alpha = alpha; e.tol = tol; e.tol_rel = tol_rel;
        e.rule = rule;
        std::memcpy(e.tune, c->tune, sizeof(e.tune));
        e.exec = ex;
        c->graphs.push_back(e);
        ge = &c->graphs.back();
    }
    HIP_TRY(hipGraphLaunch(ge->exec, c->stream));
    c->cur ^= (n & 1);
    return CCD_OK;
}

// ---- autotuner ---------------------------------------------------------------
// Every family launch is idempotent for a fixed cur (it rewrites its outputs
// from t[cur] and the other families' outputs), so the sweep's contractions
// and update can be launched repeatedly without advancing the iteration.
// Slots are tuned one at a time in pipeline order, each candidate timed over
// reps such passes after one warm pass; a candidate replaces the incumbent
// only when it is 2% faster.
template <typename F>
static ccd_status time_family(ccd_ctx* c, F&& launch, int reps, hipEvent_t e0, hipEvent_t e1, double& ms) {
    ccd_status s = launch();
    if (s != CCD_OK) return s;
    HIP_TRY(hipEventRecord(e0, c->stream));
    for (int r = 0; r < reps && s == CCD_OK; r++) s = launch();
    if (s != CCD_OK) return s;
    HIP_TRY(hipEventRecord(e1, c->stream));
    HIP_TRY(hipEventSynchronize(e1));
    float f = 0.f;
    HIP_TRY(hipEventElapsedTime(&f, e0, e1));
    ms = (double)f / reps;
    return CCD_OK;
}

template <int P>
static ccd_status autotune_impl(ccd_ctx* c, int reps, double* best_ms, hipEvent_t e0, hipEvent_t e1) {
    const DevPtrs d = make_ptrs(c);
    const int cur = c->cur;
    const uint32_t mask = CCD_T_ALL;
    const double alpha = 0.5;
    ccd_status s = launch_contractions<P>(c, d, cur, mask);
    if (s == CCD_OK) s = L_update(c, d, cur, alpha, mask);
    if (s != CCD_OK) return s;
    struct Spec {
        int slot, ncand;
        int cand[4];
    };
    const Spec specs[] = {
        {CCD_TUNE_DIRECT, 4, {0, 1, 2, 4}},  {CCD_TUNE_DCHI, 4, {0, 1, 2, 4}},
        {CCD_TUNE_RING_SMALL, 4, {0, 1, 2, 4}}, {CCD_TUNE_RING_NW32, 2, {0, 1}},
        {CCD_TUNE_RING_NW48, 2, {0, 1}},     {CCD_TUNE_RING_NW64, 2, {0, 1}},
        {CCD_TUNE_RING_NW80, 2, {0, 1}},     {CCD_TUNE_RING, 4, {0, 1, 2, 4}},
        {CCD_TUNE_LADDER, 4, {0, 1, 2, 4}},  {CCD_TUNE_UPDATE, 4, {0, 1, 2, 4}},
    };
    // every candidate is timed on the sweep's contractions and update as they
    // run (forked streams included): a shape that is faster alone can be slower
    // beside the kernels it shares the compute units with
    auto sweep_body = [&] {
        ccd_status r = launch_contractions<P>(c, d, cur, mask);
        return r == CCD_OK ? L_update(c, d, cur, alpha, mask) : r;
    };
    for (const Spec& sp : specs) {
        double best = 0.0;
        int bestv = sp.cand[0];
        for (int k = 0; k < sp.ncand; k++) {
            c->tune[sp.slot] = sp.cand[k];
            double ms = 0.0;
            s = time_family(c, sweep_body, reps, e0, e1, ms);
            if (s != CCD_OK) return s;
            if (k == 0 || ms < 0.98 * best) { best = ms; bestv = sp.cand[k]; }
        }
        c->tune[sp.slot] = bestv;
        if (best_ms) best_ms[sp.slot] = best;
    }
    return CCD_OK;
}

// --------------------------------------------------------------------------
// C ABI
// --------------------------------------------------------------------------
extern "C" {

const char* ccd_last_error(void) { return g_err.c_str(); }
const char* ccd_version(void) { return "ccd-mi355x 0.3 (gfx950; FP64, FP32 and BF16 MFMA contractions)"; }

ccd_status ccd_build_channels(const ccd_problem* probs, int32_t n, void* stream, ccd_ctx** out) {
    if (!probs || !out || n < 1 || n > 4096) {
        set_error("ccd_build_channels: need probs, out and 1 <= n_problems <= 4096");
        return CCD_EINVAL;
    }
    *out = nullptr;
    ccd_ctx* c = new (std::nothrow) ccd_ctx();
    if (!c) { set_error("out of host memory"); return CCD_ENOMEM; }
    c->stream = (hipStream_t)stream;
    c->probs.resize(n);
    // the plans are independent: host threads take problems i = w, w + T, ...
    std::vector<ccd_status> st(n, CCD_OK);
    std::vector<std::string> errs(n);
    {
        const int T = std::max(1, std::min({n, 16, (int)std::thread::hardware_concurrency()}));
        auto work = [&](int w) {
            for (int i = w; i < n; i += T) st[i] = build_problem(probs[i], c->probs[i], errs[i]);
        };
        std::vector<std::thread> pool;
        for (int w = 1; w < T; w++) pool.emplace_back(work, w);
        work(0);
        for (auto& th : pool) th.join();
    }
    for (int i = 0; i < n; i++)
        if (st[i] != CCD_OK) {
            set_error("problem " + std::to_string(i) + ": " + errs[i]);
            const ccd_status s = st[i];
            delete c;
            return s;
        }
    ccd_status s = assemble(c);
    if (s != CCD_OK) { delete c; return s; }
    c->emp2.assign(n, 0.0);
    *out = c;
    return CCD_OK;
}

ccd_status ccd_workspace_size(const ccd_ctx* c, size_t* bytes) {
    if (!c || !bytes) { set_error("ccd_workspace_size: NULL argument"); return CCD_EINVAL; }
    *bytes = c->ws_bytes;
    return CCD_OK;
}

ccd_status ccd_reset_amplitudes(ccd_ctx* c) {
    if (!c) { set_error("NULL context"); return CCD_EINVAL; }
    if (!c->bound) { set_error("no workspace bound"); return CCD_ESTATE; }
    c->cur = 0;
    DevPtrs d = make_ptrs(c);
    LAUNCH(F_INIT, k_init, (int)c->it_elem.size(), 256, 0, d, 0, -1);
    LAUNCH(F_ENERGY, k_energy_elem, (int)c->probs.size(), 256, 0, d);
    return CCD_OK;
}

ccd_status ccd_bind_workspace(ccd_ctx* c, void* ptr, size_t bytes) {
    if (!c || !ptr) { set_error("ccd_bind_workspace: NULL argument"); return CCD_EINVAL; }
    if (c->bound) { set_error("a workspace is already bound"); return CCD_ESTATE; }
    if (bytes < c->ws_bytes) { set_error("workspace too small"); return CCD_EINVAL; }
    if (((uintptr_t)ptr) & 255) { set_error("workspace must be 256-byte aligned"); return CCD_EINVAL; }
    c->ws = (char*)ptr;
    if (!c->aux_ok) {
        bool ok = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) == hipSuccess &&
                  hipEventCreateWithFlags(&c->ev_mid, hipEventDisableTiming) == hipSuccess;
        for (int k = 0; k < 3 && ok; k++)
            ok = hipStreamCreateWithFlags(&c->aux[k], hipStreamNonBlocking) == hipSuccess &&
                 hipEventCreateWithFlags(&c->ev_join[k], hipEventDisableTiming) == hipSuccess;
        c->aux_ok = ok;  // without them the ring stays on the caller's stream
    }
    HIP_TRY(set_ring_attrs<P_F64>());
    HIP_TRY(set_ring_attrs<P_F32>());
    HIP_TRY(set_ring_attrs<P_BF16>());
    std::vector<char> img = static_image(c);
    HIP_TRY(hipMemcpyAsync(c->ws + c->r_static.off, img.data(), img.size(), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemsetAsync(c->ws + c->r_t0.off, 0, c->ws_bytes - c->r_t0.off, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->bound = true;
    ccd_status s = ccd_reset_amplitudes(c);
    if (s != CCD_OK) return s;
    const int P = (int)c->probs.size();
    std::vector<double> e(P);
    HIP_TRY(hipMemcpyAsync(e.data(), c->ws + c->r_ecorr.off, P * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (int p = 0; p < P; p++) c->emp2[p] = e[c->slot_of[p]];
    return CCD_OK;
}

// one phase of sweeps in precision prec.  Sweeps run in chunks of up to
// check_every (graph replays when asked); after each chunk the host reads the
// per-problem sweep counters, active flags and the device energy history.
// min_sweeps: sweeps run before the convergence test may stop a problem.
static ccd_status run_phase(ccd_ctx* c, const ccd_solver_opts* o, int prec, double tol_phase, double rel_phase,
                            int rule, int budget, int min_sweeps, double* e_hist, int& used) {
    const int P = (int)c->probs.size();
    std::vector<int32_t> ones(P, 1);
    HIP_TRY(hipMemcpyAsync(c->ws + c->r_active.off, ones.data(), P * 4, hipMemcpyHostToDevice, c->stream));
    const bool stops = tol_phase > 0.0 || rel_phase > 0.0;
    const bool check = stops || e_hist;
    const int every = check ? std::max(1, std::min(o->check_every > 0 ? o->check_every : 1, kHistCap)) : kHistCap;
    const bool graph = o->use_graph != 0;
    std::vector<int32_t> sw(P, 0), sw0(P, 0), act(P, 1);
    std::vector<double> hb((size_t)P * kHistCap);
    if (e_hist) {
        HIP_TRY(hipMemcpyAsync(sw.data(), c->ws + c->r_sweeps.off, P * 4, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
    }
    bool all_done = false;
    used = 0;
    // Chunk length: `every` sweeps, or fewer once the sweeps that the slowest
    // problem still needs can be estimated from its geometric rate of
    // convergence: sweeps launched after every problem has stopped still cost
    // most of a live sweep (launches, barriers, the update's copy of t), while
    // a short chunk costs one more host read.  Only the host's reads move; the
    // device decides when each problem stops, so results do not change.
    std::vector<double> ec(P), dq(P), d_then(P, 0.0);
    std::vector<int32_t> sw_then(P, 0);
    int next = every;
    while (used < budget && !all_done) {
        int n;
        double tol, rel;
        if (used + 1 < min_sweeps) {
            n = std::min(std::min(min_sweeps - 1 - used, budget - used), every);
            tol = rel = 0.0;
        } else {
            n = std::min(next, budget - used);
            tol = tol_phase;
            rel = rel_phase;
        }
        ccd_status st = run_sweeps(c, n, o->mixing, tol, rel, rule, o->terms, prec, graph);
        if (st != CCD_OK) return st;
        used += n;
        if (check) {
            sw0 = sw;
            HIP_TRY(hipMemcpyAsync(sw.data(), c->ws + c->r_sweeps.off, P * 4, hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(hipMemcpyAsync(act.data(), c->ws + c->r_active.off, P * 4, hipMemcpyDeviceToHost, c->stream));
            if (e_hist || stops)
                HIP_TRY(hipMemcpyAsync(hb.data(), c->ws + c->r_ehist.off, hb.size() * 8, hipMemcpyDeviceToHost,
                                       c->stream));
            if (stops) {
                HIP_TRY(hipMemcpyAsync(ec.data(), c->ws + c->r_ecorr.off, P * 8, hipMemcpyDeviceToHost, c->stream));
                HIP_TRY(hipMemcpyAsync(dq.data(), c->ws + c->r_dprev.off, P * 8, hipMemcpyDeviceToHost, c->stream));
            }
            HIP_TRY(hipStreamSynchronize(c->stream));
            all_done = stops;
            for (int p = 0; p < P; p++) {
                const int sl = c->slot_of[p];
                if (e_hist)
                    for (int k = sw0[sl]; k < sw[sl] && k < o->max_iter; k++)
                        e_hist[(size_t)p * o->max_iter + k] = hb[(size_t)sl * kHistCap + k % kHistCap];
                if (act[sl]) all_done = false;
            }
            // (with graph replay every chunk length is a graph of its own to
            // capture, so the chunks keep the one length there)
            if (stops && !graph && used + 1 >= min_sweeps) {
                next = 0;
                for (int sl = 0; sl < P; sl++) {
                    if (!act[sl]) continue;
                    const double de = dq[sl], thr = tol_phase + rel_phase * std::fabs(ec[sl]);
                    int need = every;
                    // the rate over the last chunk, else over the last sweep (the
                    // energy history holds E after sweep s at (s - 1) mod kHistCap)
                    double rate = -1.0;
                    if (sw[sl] > sw_then[sl] && d_then[sl] > 0.0 && de > 0.0) {
                        rate = std::pow(de / d_then[sl], 1.0 / (sw[sl] - sw_then[sl]));
                    } else if (sw[sl] >= 3 && de > 0.0) {
                        const double* h = hb.data() + (size_t)sl * kHistCap;
                        const double d1 = std::fabs(h[(sw[sl] - 2) % kHistCap] - h[(sw[sl] - 3) % kHistCap]);
                        if (d1 > 0.0) rate = de / d1;
                    }
                    if (std::isfinite(rate) && rate > 0.0 && rate < 1.0) {
                        // rule 1 stops after two sweeps with |dE| r / (1 - r) < thr
                        const double target = rule == 1 ? thr * (1.0 - rate) / rate : thr;
                        const int extra = rule == 1 ? 2 : 1;
                        // (clamped before the cast: a rate near 1 gives a huge count)
                        const double k = de < target ? 0.0 : std::floor(std::log(target / de) / std::log(rate));
                        need = k >= (double)every ? every : (int)k + extra;
                    }
                    next = std::max(next, std::min(std::max(need, 1), every));
                    d_then[sl] = de;
                    sw_then[sl] = sw[sl];
                }
                if (next < 1) next = every;
            }
        }
    }
    return CCD_OK;
}

ccd_status ccd_iterate(ccd_ctx* c, const ccd_solver_opts* o, int32_t* sweeps_done, double* e_hist) {
    if (!c || !o) { set_error("ccd_iterate: NULL argument"); return CCD_EINVAL; }
    if (!c->bound) { set_error("ccd_iterate: no workspace bound"); return CCD_ESTATE; }
    if (!(o->mixing > 0.0 && o->mixing <= 1.0) || o->max_iter < 1) {
        set_error("ccd_iterate: need 0 < mixing <= 1 and max_iter >= 1");
        return CCD_EINVAL;
    }
    if (o->precision != CCD_PREC_FP64 && o->precision != CCD_PREC_FP32 && o->precision != CCD_PREC_BF16) {
        set_error("ccd_iterate: unknown precision");
        return CCD_EINVAL;
    }
    if (o->refine_sweeps < 0 || o->check_every < 0 || o->stop_rule < 0 || o->stop_rule > 1) {
        set_error("ccd_iterate: refine_sweeps and check_every must be >= 0, stop_rule 0 or 1");
        return CCD_EINVAL;
    }
    const int P = (int)c->probs.size();
    std::vector<int32_t> zeros(P, 0);
    std::vector<double> dzero(P, 0.0);
    HIP_TRY(hipMemcpyAsync(c->ws + c->r_sweeps.off, zeros.data(), P * 4, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->ws + c->r_dprev.off, dzero.data(), P * 8, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->ws + c->r_streak.off, zeros.data(), P * 4, hipMemcpyHostToDevice, c->stream));
    if (e_hist)
        for (size_t k = 0; k < (size_t)P * o->max_iter; k++) e_hist[k] = NAN;
    int used = 0;
    const bool mixed = o->precision != CCD_PREC_FP64;
    const bool own = mixed && o->mixed_tol > 0.0;  // the mixed phase has its own (absolute) criterion
    // a mixed phase with its own criterion uses the plain |dE| test: near its
    // rounding floor the ratio of successive changes hovers around 1
    ccd_status st = run_phase(c, o, o->precision, own ? o->mixed_tol : o->tol, own ? 0.0 : o->tol_rel,
                              own ? 0 : o->stop_rule, o->max_iter, 1, e_hist, used);
    if (st != CCD_OK) return st;
    if (mixed && used < o->max_iter) {
        // FP64 refinement: continue the FP64 iteration from the mixed-precision iterate
        int used2 = 0;
        st = run_phase(c, o, CCD_PREC_FP64, o->tol, o->tol_rel, o->stop_rule, o->max_iter - used,
                       std::max(1, o->refine_sweeps), e_hist, used2);
        if (st != CCD_OK) return st;
    }
    std::vector<int32_t> sw(P), act(P);
    std::vector<double> e(P);
    HIP_TRY(hipMemcpyAsync(sw.data(), c->ws + c->r_sweeps.off, P * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(e.data(), c->ws + c->r_ecorr.off, P * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(act.data(), c->ws + c->r_active.off, P * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (sweeps_done)
        for (int p = 0; p < P; p++) sweeps_done[p] = sw[c->slot_of[p]];
    for (int p = 0; p < P; p++)
        if (!std::isfinite(e[c->slot_of[p]])) {
            set_error("problem " + std::to_string(p) + ": correlation energy is not finite");
            return CCD_DIVERGED;
        }
    if (o->tol > 0.0 || o->tol_rel > 0.0)
        for (int p = 0; p < P; p++)
            if (act[c->slot_of[p]]) return CCD_NOT_CONVERGED;
    return CCD_OK;
}

ccd_status ccd_mbpt3(ccd_ctx* c, double* out) {
    if (!c || !out) { set_error("ccd_mbpt3: NULL argument"); return CCD_EINVAL; }
    if (!c->bound) { set_error("ccd_mbpt3: no workspace bound"); return CCD_ESTATE; }
    const int P = (int)c->probs.size();
    const uint32_t masks[4] = {CCD_T_PP, CCD_T_HH, CCD_T_RING, CCD_T_PP | CCD_T_HH | CCD_T_RING};
    ccd_solver_opts o;
    std::memset(&o, 0, sizeof(o));
    o.mixing = 1.0;
    o.max_iter = 1;
    o.precision = CCD_PREC_FP64;
    o.check_every = 1;
    std::vector<double> e(P);
    for (int k = 0; k < 4; k++) {
        ccd_status s = ccd_reset_amplitudes(c);
        if (s != CCD_OK) return s;
        o.terms = masks[k];
        s = ccd_iterate(c, &o, nullptr, nullptr);
        if (s != CCD_OK && s != CCD_NOT_CONVERGED) {
            (void)ccd_reset_amplitudes(c);
            return s;
        }
        HIP_TRY(hipMemcpyAsync(e.data(), c->ws + c->r_ecorr.off, 8 * P, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        for (int p = 0; p < P; p++) out[4 * p + k] = e[c->slot_of[p]] - c->emp2[p];
    }
    return ccd_reset_amplitudes(c);
}

ccd_status ccd_energy(const ccd_ctx* cc, int32_t p, double* eref, double* emp2, double* ecorr) {
    ccd_ctx* c = (ccd_ctx*)cc;
    if (!c || p < 0 || p >= (int)c->probs.size()) { set_error("ccd_energy: bad problem"); return CCD_EINVAL; }
    if (eref) *eref = c->probs[p].eref;
    if (emp2 || ecorr) {
        if (!c->bound) { set_error("ccd_energy: no workspace bound"); return CCD_ESTATE; }
        double e = 0;
        HIP_TRY(hipMemcpyAsync(&e, c->ws + c->r_ecorr.off + 8 * c->slot_of[p], 8, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        if (emp2) *emp2 = c->emp2[p];
        if (ecorr) *ecorr = e;
    }
    return CCD_OK;
}

ccd_status ccd_reference_parts(const ccd_ctx* c, int32_t p, double* kinetic, double* hf_potential) {
    if (!c || p < 0 || p >= (int)c->probs.size()) { set_error("ccd_reference_parts: bad problem"); return CCD_EINVAL; }
    if (kinetic) *kinetic = c->probs[p].ekin;
    if (hf_potential) *hf_potential = c->probs[p].eref - c->probs[p].ekin;
    return CCD_OK;
}

ccd_status ccd_twist_average(const ccd_ctx* cc, const double* weight, double* out) {
    ccd_ctx* c = (ccd_ctx*)cc;
    if (!c || !weight || !out) { set_error("ccd_twist_average: NULL argument"); return CCD_EINVAL; }
    if (!c->bound) { set_error("ccd_twist_average: no workspace bound"); return CCD_ESTATE; }
    const size_t P = c->probs.size();
    std::vector<double> ec(P);
    HIP_TRY(hipMemcpyAsync(ec.data(), c->ws + c->r_ecorr.off, 8 * P, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    double acc[5] = {0, 0, 0, 0, 0};
    for (size_t p = 0; p < P; p++) {
        const HostProblem& H = c->probs[p];
        const double w = weight[p];
        if (!std::isfinite(w)) { set_error("ccd_twist_average: weight not finite"); return CCD_EINVAL; }
        acc[0] += w * H.ekin;
        acc[1] += w * (H.eref - H.ekin);
        acc[2] += w * H.eref;
        acc[3] += w * c->emp2[p];
        acc[4] += w * ec[c->slot_of[p]];
    }
    for (int k = 0; k < 5; k++) out[k] = acc[k];
    return CCD_OK;
}

ccd_status ccd_problem_info(const ccd_ctx* c, int32_t p, ccd_info* info) {
    if (!c || !info || p < 0 || p >= (int)c->probs.size()) { set_error("ccd_problem_info: bad argument"); return CCD_EINVAL; }
    const HostProblem& H = c->probs[p];
    info->n_states = H.ns; info->n_holes = H.nh; info->n_particles_states = H.np;
    info->n_channels = (int)H.chans.size(); info->n_channels_sz0 = H.n_sz0;
    info->n_ph_channels = (int)H.ph.size();
    info->max_hh = H.max_hh; info->max_pp = H.max_pp; info->max_ph = H.max_ph;
    info->n_amplitudes = H.n_amp;
    info->lut_size = (int)H.W.size();
    info->box_L = H.L;
    info->flops_pp = H.flops_pp; info->flops_hh = H.flops_hh; info->flops_ring = H.flops_ring;
    info->flops_ordered = H.flops_ordered;
    return CCD_OK;
}

ccd_status ccd_get_amplitudes(const ccd_ctx* c, int32_t p, double* dst, size_t n) {
    if (!c || !dst || p < 0 || p >= (int)c->probs.size()) { set_error("ccd_get_amplitudes: bad argument"); return CCD_EINVAL; }
    if (!c->bound) { set_error("no workspace bound"); return CCD_ESTATE; }
    if (n != (size_t)c->probs[p].n_amp) { set_error("ccd_get_amplitudes: n != n_amplitudes"); return CCD_EINVAL; }
    const Region& r = c->cur ? c->r_t1 : c->r_t0;
    HIP_TRY(hipMemcpyAsync(dst, c->ws + r.off + 8 * c->prob_t0[p], n * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return CCD_OK;
}

ccd_status ccd_set_amplitudes(ccd_ctx* c, int32_t p, const double* src, size_t n) {
    if (!c || !src || p < 0 || p >= (int)c->probs.size()) { set_error("ccd_set_amplitudes: bad argument"); return CCD_EINVAL; }
    if (!c->bound) { set_error("no workspace bound"); return CCD_ESTATE; }
    if (n != (size_t)c->probs[p].n_amp) { set_error("ccd_set_amplitudes: n != n_amplitudes"); return CCD_EINVAL; }
    for (size_t k = 0; k < n; k++)
        if (!std::isfinite(src[k])) { set_error("ccd_set_amplitudes: non-finite amplitude"); return CCD_EINVAL; }
    const Region& r = c->cur ? c->r_t1 : c->r_t0;
    HIP_TRY(hipMemcpyAsync(c->ws + r.off + 8 * c->prob_t0[p], src, n * 8, hipMemcpyHostToDevice, c->stream));
    ccd_status s = refresh_energy(c);
    if (s != CCD_OK) return s;
    HIP_TRY(hipStreamSynchronize(c->stream));
    return CCD_OK;
}

ccd_status ccd_export_maps(const ccd_ctx* c, int32_t p, int32_t which, int32_t* dst, size_t n, size_t* need) {
    if (!c || p < 0 || p >= (int)c->probs.size()) { set_error("ccd_export_maps: bad problem"); return CCD_EINVAL; }
    const HostProblem& H = c->probs[p];
    std::vector<int32_t> v;
    switch (which) {
        case CCD_MAP_STATES:
            for (int s = 0; s < H.ns; s++) { v.push_back(H.nx[s]); v.push_back(H.ny[s]); v.push_back(H.nz[s]); v.push_back(H.sz[s]); }
            break;
        case CCD_MAP_CHANNELS:
            for (auto& ch : H.chans) { v.push_back(ch.Kx); v.push_back(ch.Ky); v.push_back(ch.Kz); v.push_back(ch.Sz); v.push_back(ch.nhh); v.push_back(ch.npp); }
            break;
        case CCD_MAP_HH: v = H.hh; break;
        case CCD_MAP_PP: v = H.pp; break;
        case CCD_MAP_PH_CHANNELS:
            for (auto& ch : H.ph) { v.push_back(ch.Qx); v.push_back(ch.Qy); v.push_back(ch.Qz); v.push_back(ch.sig); v.push_back(ch.n); v.push_back(ch.partner); }
            break;
        case CCD_MAP_PH: v = H.phmem; break;
        default: set_error("ccd_export_maps: unknown map"); return CCD_EINVAL;
    }
    if (need) *need = v.size();
    if (!dst) return CCD_OK;
    if (n < v.size()) { set_error("ccd_export_maps: destination too small"); return CCD_EINVAL; }
    std::copy(v.begin(), v.end(), dst);
    return CCD_OK;
}

ccd_status ccd_export_tables(const ccd_ctx* c, int32_t p, double* tkin, double* eps, double* w) {
    if (!c || p < 0 || p >= (int)c->probs.size()) { set_error("ccd_export_tables: bad problem"); return CCD_EINVAL; }
    const HostProblem& H = c->probs[p];
    if (tkin) std::copy(H.tkin.begin(), H.tkin.end(), tkin);
    if (eps) std::copy(H.eps.begin(), H.eps.end(), eps);
    if (w) std::copy(H.W.begin(), H.W.end(), w);
    return CCD_OK;
}

ccd_status ccd_set_timing(ccd_ctx* c, int32_t on) {
    if (!c) { set_error("NULL context"); return CCD_EINVAL; }
    ccd_status s = harvest(c);
    if (s != CCD_OK) return s;
    c->timing = on != 0;
    return CCD_OK;
}

ccd_status ccd_autotune(ccd_ctx* c, int32_t precision, int32_t reps, double* best_ms) {
    if (!c) { set_error("ccd_autotune: NULL context"); return CCD_EINVAL; }
    if (!c->bound) { set_error("ccd_autotune: no workspace bound"); return CCD_ESTATE; }
    if (precision < CCD_PREC_FP64 || precision > CCD_PREC_BF16 || reps < 1 || reps > 1000) {
        set_error("ccd_autotune: need a CCD_PREC_* precision and 1 <= reps <= 1000");
        return CCD_EINVAL;
    }
    ccd_status s = harvest(c);
    if (s != CCD_OK) return s;
    const bool timing = c->timing;
    c->timing = false;
    const int P = (int)c->probs.size();
    std::vector<int32_t> ones(P, 1);
    HIP_TRY(hipMemcpyAsync(c->ws + c->r_active.off, ones.data(), P * 4, hipMemcpyHostToDevice, c->stream));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        set_error(std::string("hipEventCreate: ") + hipGetErrorString(he));
        return CCD_EHIP;
    }
    s = precision == CCD_PREC_BF16 ? autotune_impl<P_BF16>(c, reps, best_ms, e0, e1)
      : precision == CCD_PREC_FP32 ? autotune_impl<P_F32>(c, reps, best_ms, e0, e1)
                                   : autotune_impl<P_F64>(c, reps, best_ms, e0, e1);
    (void)hipStreamSynchronize(c->stream);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->timing = timing;
    return s;
}

ccd_status ccd_mlp_features(const ccd_ctx* cc, int32_t p, float* feat, float* target) {
    ccd_ctx* c = const_cast<ccd_ctx*>(cc);
    if (!c || !feat || p < 0 || p >= (int)c->probs.size()) {
        set_error("ccd_mlp_features: bad argument");
        return CCD_EINVAL;
    }
    if (!c->bound) { set_error("ccd_mlp_features: no workspace bound"); return CCD_ESTATE; }
    if (((uintptr_t)feat) & 15) { set_error("ccd_mlp_features: feat must be 16-byte aligned"); return CCD_EINVAL; }
    const int sl = c->slot_of[p];
    const int gi = c->pgrp[sl], g = c->pgi[sl];
    const DevGroup& G = c->dgroups[gi];
    DevPtrs d = make_ptrs(c);
    LAUNCH(F_INIT, k_features, G.elem_hi - G.elem_lo, 256, 0, d, c->cur, gi, g, feat, target);
    return CCD_OK;
}

ccd_status ccd_warm_start(ccd_ctx* c, const float* params, int32_t precision, int32_t* used_net) {
    if (!c) { set_error("ccd_warm_start: NULL context"); return CCD_EINVAL; }
    if (!c->bound) { set_error("ccd_warm_start: no workspace bound"); return CCD_ESTATE; }
    const int P = (int)c->probs.size();
    if (!params) {
        ccd_status s = ccd_reset_amplitudes(c);
        if (s != CCD_OK) return s;
        HIP_TRY(hipStreamSynchronize(c->stream));
        if (used_net) std::fill(used_net, used_net + P, 0);
        return CCD_OK;
    }
    if (precision != CCD_PREC_FP32 && precision != CCD_PREC_BF16) {
        set_error("ccd_warm_start: precision must be CCD_PREC_FP32 or CCD_PREC_BF16");
        return CCD_EINVAL;
    }
    if (((uintptr_t)params) & 15) { set_error("ccd_warm_start: params must be 16-byte aligned"); return CCD_EINVAL; }
    static bool attr = false;
    if (!attr) {
        HIP_TRY(hipFuncSetAttribute((const void*)k_warm<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)warm_lds<false>()));
        HIP_TRY(hipFuncSetAttribute((const void*)k_warm<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)warm_lds<true>()));
        attr = true;
    }
    DevPtrs d = make_ptrs(c);
    const int n = (int)c->it_elem.size();
    int max_g = 1;
    for (const DevGroup& D : c->dgroups) max_g = std::max(max_g, D.G);
    // persistent: three blocks per compute unit (the LDS of one block allows
    // three), each staging the weights once for all its work units
    int dev = 0, ncu = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    const int grid = (int)std::min<int64_t>((int64_t)n * max_g, (int64_t)std::max(ncu, 1) * 3);
    if (precision == CCD_PREC_BF16)
        LAUNCH(F_INIT, k_warm<true>, grid, 256, warm_lds<true>(), d, c->cur, params, n, max_g);
    else
        LAUNCH(F_INIT, k_warm<false>, grid, 256, warm_lds<false>(), d, c->cur, params, n, max_g);
    ccd_status s = refresh_energy(c);
    if (s != CCD_OK) return s;
    std::vector<double> e(P);
    HIP_TRY(hipMemcpyAsync(e.data(), c->ws + c->r_ecorr.off, P * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    bool any = false;
    for (int p = 0; p < P; p++) {
        const double ew = e[c->slot_of[p]], r = ew / c->emp2[p];
        const bool keep = std::isfinite(ew) && r >= 0.5 && r <= 2.0;
        if (used_net) used_net[p] = keep ? 1 : 0;
        if (!keep) {
            LAUNCH(F_INIT, k_init, n, 256, 0, d, c->cur, c->slot_of[p]);
            any = true;
        }
    }
    if (any) {
        s = refresh_energy(c);
        if (s != CCD_OK) return s;
        HIP_TRY(hipStreamSynchronize(c->stream));
    }
    return CCD_OK;
}

ccd_status ccd_get_tuning(const ccd_ctx* c, int32_t* dst, int32_t n) {
    if (!c || !dst || n < CCD_TUNE_LEN) { set_error("ccd_get_tuning: need dst of CCD_TUNE_LEN entries"); return CCD_EINVAL; }
    std::copy(c->tune, c->tune + CCD_TUNE_LEN, dst);
    return CCD_OK;
}

ccd_status ccd_set_tuning(ccd_ctx* c, const int32_t* src, int32_t n) {
    if (!c || !src || n < CCD_TUNE_LEN) { set_error("ccd_set_tuning: need src of CCD_TUNE_LEN entries"); return CCD_EINVAL; }
    for (int k = 0; k < CCD_TUNE_LEN; k++) {
        const bool ok = k < CCD_TUNE_RING_NW32 ? (src[k] == 0 || src[k] == 1 || src[k] == 2 || src[k] == 4)
                                              : (src[k] == 0 || src[k] == 1);
        if (!ok) { set_error("ccd_set_tuning: value out of range in slot " + std::to_string(k)); return CCD_EINVAL; }
    }
    std::copy(src, src + CCD_TUNE_LEN, c->tune);
    return CCD_OK;
}

int32_t ccd_kernel_families(void) { return F_NUM; }
const char* ccd_kernel_name(int32_t f) { return (f >= 0 && f < F_NUM) ? kFamilyNames[f] : ""; }

ccd_status ccd_kernel_times(ccd_ctx* c, double* ms, int64_t* launches, int32_t reset) {
    if (!c) { set_error("NULL context"); return CCD_EINVAL; }
    ccd_status s = harvest(c);
    if (s != CCD_OK) return s;
    for (int f = 0; f < F_NUM; f++) {
        if (ms) ms[f] = c->ms[f];
        if (launches) launches[f] = c->launches[f];
        if (reset) { c->ms[f] = 0; c->launches[f] = 0; }
    }
    return CCD_OK;
}

void ccd_destroy(ccd_ctx* c) {
    if (!c) return;
    if (!c->graphs.empty() || c->cap_stream || c->aux_ok) (void)hipStreamSynchronize(c->stream);
    for (GraphEntry& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (int k = 0; k < 3; k++) {
        if (c->aux[k]) {
            (void)hipStreamSynchronize(c->aux[k]);
            (void)hipStreamDestroy(c->aux[k]);
        }
        if (c->ev_join[k]) (void)hipEventDestroy(c->ev_join[k]);
    }
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_mid) (void)hipEventDestroy(c->ev_mid);
    if (!c->ev_pool.empty()) {
        if (!c->pending.empty()) (void)hipStreamSynchronize(c->stream);
        for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    }
    delete c;
}

}  // extern "C"
