// ccd_device.hip -- gfx950 kernels of the CCD sweep and the C ABI around them.
//
// One Jacobi sweep (eq. ccd3 in the intermediates form of sec. "Developing a
// CCD code for infinite matter"), all terms from the current amplitudes t:
//   k_rowcol   row and column sums of t <ab||ij> over S_z = 0 blocks
//   k_dchi     one-body intermediates, diagonal by momentum conservation:
//              chi_bb - f_bb = -1/2 sum_kld t_kl^bd <kl||bd>,
//              chi_jj - f_jj = +1/2 sum_cdl <jl||cd> t_jl^cd
//   k_chh      chi_klij = <kl||ij> + 1/2 sum_cd <kl||cd> t_ij^cd per S_z = 0 block
//   k_scatter  t -> particle-hole layout T~_Q[(a,i),(c,k)] = t_ik^ac
//   k_ring     per cross channel Q: chi~ = V_ph + 1/2 Vbar T~_Q (chi_kbcj),
//              Z_Q = T~_Q chi~ (sum_kc t_ik^ac chi_kbcj)
//   k_ladder   per S_z = 0 block and 64-row tile: pp ladder sum_{c<d} <ab||cd> t_ij^cd
//              with <ab||cd> generated on the fly from W(m), hh ladder
//              sum_{k<l} t_kl^ab chi_klij, the ring P(ij)P(ab) gather from Z,
//              the one-body terms, t_new = R / eps_ij^ab, linear mixing and the
//              energy partial sums
//   k_update   the same update for the S_z = +-1 blocks (no ladders: <ab||cd> = 0)
//   k_energy   deterministic per-problem energy, convergence flag
// Reductions use fixed-order trees (no floating-point atomics), so energies are
// bit-identical from run to run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ccd_internal.h"

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

// --------------------------------------------------------------------------
// device pointers, passed by value to every kernel
// --------------------------------------------------------------------------
struct DevPtrs {
    const int32_t* st;     // packed states
    const double* eps;     // Fock energies
    const double* lut;     // W(m) / 2
    const DevProb* probs;
    const DevChan* chans;
    const DevPh* ph;
    const int32_t* hh;     // packed pairs
    const int32_t* pp;
    const int32_t* phmem;
    const int32_t* phq;
    const int32_t* phpos;
    const int32_t* dchi_ptr;
    const int32_t* dchi_idx;
    const Item* it_elem;   // elementwise items, all channels
    const Item* it_nsz0;   // elementwise items, S_z != 0 channels
    const Item* it_ladder; // ladder items (S_z = 0)
    const int32_t* it_sz0; // S_z = 0 channel ids
    double* t[2];
    double* vt;            // <ab||ij>
    double* chh;
    double* rowsum;
    double* colsum;
    double* dchi;
    double* tt;            // particle-hole layout of t
    double* z;             // ring result
    double* epart;         // energy partials (ladder items)
    double* epart_elem;    // energy partials (elementwise items)
    double* ecorr;
    double* eprev;
    int32_t* active;
    int32_t* sweeps;
};

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

// deterministic sum over a 256-thread block; result valid in thread 0
__device__ __forceinline__ double block_sum256(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    return r;
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// index of Z[(p,h),(p2,h2)] in the particle-hole layout
__device__ __forceinline__ int64_t zidx(const DevPtrs& d, const DevProb& P, int p, int h, int p2, int h2) {
    int u = P.ph_off + (p - P.nh) * P.nh + h;
    int v = P.ph_off + (p2 - P.nh) * P.nh + h2;
    const DevPh q = d.ph[d.phq[u]];
    return q.z_off + (int64_t)d.phpos[u] * q.n + d.phpos[v];
}

// P(ij)P(ab) sum_kc t_ik^ac chi_kbcj from the ring result Z
__device__ __forceinline__ double ring_gather(const DevPtrs& d, const DevProb& P, int a, int b, int i, int j) {
    return d.z[zidx(d, P, a, i, b, j)] - d.z[zidx(d, P, a, j, b, i)] - d.z[zidx(d, P, b, i, a, j)] +
           d.z[zidx(d, P, b, j, a, i)];
}

// --------------------------------------------------------------------------
// kernels
// --------------------------------------------------------------------------

// <ab||ij>, t0 = <ab||ij> / eps_ij^ab (eq. ccdGuess); energy partial per item
__global__ void __launch_bounds__(256) k_init(DevPtrs d, int cur) {
    __shared__ double sh[4];
    const Item it = d.it_elem[blockIdx.x];
    const DevChan c = d.chans[it.chan];
    const DevProb P = d.probs[c.prob];
    const int nel = c.nhh * c.npp;
    double es = 0.0;
    for (int k = 0; k < kElemChunk / 256; k++) {
        int e = it.start + threadIdx.x + 256 * k;
        if (e < nel && e < it.start + kElemChunk) {
            int r = e / c.nhh, col = e - r * c.nhh;
            int32_t ab = d.pp[c.pp_off + r], ij = d.hh[c.hh_off + col];
            int a = pa(ab), b = pb(ab), i = pa(ij), j = pb(ij);
            const int32_t* st = d.st + P.st_off;
            const double* eps = d.eps + P.st_off;
            double v = vas(d.lut + P.lut_off, st[a], st[b], st[i], st[j]);
            double den = eps[i] + eps[j] - eps[a] - eps[b];
            double t0 = v / den;
            d.vt[c.t_off + e] = v;
            d.t[cur][c.t_off + e] = t0;
            es += v * t0;
        }
    }
    double s = block_sum256(es, sh);
    if (threadIdx.x == 0) d.epart_elem[blockIdx.x] = s;
}

// energy partial sums sum v t of the current amplitudes per elementwise item
__global__ void __launch_bounds__(256) k_dot(DevPtrs d, int cur) {
    __shared__ double sh[4];
    const Item it = d.it_elem[blockIdx.x];
    const DevChan c = d.chans[it.chan];
    const int nel = c.nhh * c.npp;
    double es = 0.0;
    for (int k = 0; k < kElemChunk / 256; k++) {
        int e = it.start + threadIdx.x + 256 * k;
        if (e < nel && e < it.start + kElemChunk) es += d.vt[c.t_off + e] * d.t[cur][c.t_off + e];
    }
    double s = block_sum256(es, sh);
    if (threadIdx.x == 0) d.epart_elem[blockIdx.x] = s;
}

// per-problem energy from the elementwise partials; sets ecorr = eprev
__global__ void __launch_bounds__(256) k_energy_elem(DevPtrs d) {
    __shared__ double sh[4];
    const DevProb P = d.probs[blockIdx.x];
    double s = 0.0;
    for (int x = P.elem_lo + threadIdx.x; x < P.elem_hi; x += 256) s += d.epart_elem[x];
    double e = block_sum256(s, sh);
    if (threadIdx.x == 0) { d.ecorr[blockIdx.x] = e; d.eprev[blockIdx.x] = e; }
}

// row and column sums of t <ab||ij> for the S_z = 0 blocks (one block per channel)
__global__ void __launch_bounds__(256) k_rowcol(DevPtrs d, int cur) {
    __shared__ double sh[4][64];
    const DevChan c = d.chans[d.it_sz0[blockIdx.x]];
    if (!d.active[c.prob]) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const double* t = d.t[cur] + c.t_off;
    const double* vt = d.vt + c.t_off;
    for (int r = w; r < c.npp; r += 4) {
        double v = lane < c.nhh ? t[(int64_t)r * c.nhh + lane] * vt[(int64_t)r * c.nhh + lane] : 0.0;
        v = wave_sum(v);
        if (lane == 0) d.rowsum[c.row_off + r] = v;
    }
    double s = 0.0;
    if (lane < c.nhh)
        for (int r = w; r < c.npp; r += 4) s += t[(int64_t)r * c.nhh + lane] * vt[(int64_t)r * c.nhh + lane];
    sh[w][lane] = s;
    __syncthreads();
    if (w == 0 && lane < c.nhh) d.colsum[c.col_off + lane] = (sh[0][lane] + sh[1][lane]) + (sh[2][lane] + sh[3][lane]);
}

// one-body intermediates per state from the row/column sums (fixed CSR order):
// entry x >= 0: + colsum[x] (holes); x < 0: - rowsum[-x-1] (particles)
__global__ void __launch_bounds__(256) k_dchi(DevPtrs d, int n_states, uint32_t mask) {
    int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n_states) return;
    double acc = 0.0;
    for (int x = d.dchi_ptr[s]; x < d.dchi_ptr[s + 1]; x++) {
        int idx = d.dchi_idx[x];
        if (idx >= 0) {
            if (mask & CCD_T_QHOLE) acc += d.colsum[idx];
        } else {
            if (mask & CCD_T_QPART) acc -= d.rowsum[-idx - 1];
        }
    }
    d.dchi[s] = acc;
}

// chi_klij = [HH] <kl||ij> + [QHH] sum_{c<d} <kl||cd> t_ij^cd (one block per S_z = 0 channel)
__global__ void __launch_bounds__(256) k_chh(DevPtrs d, int cur, uint32_t mask) {
    __shared__ double sv[32][kMaxHH];
    __shared__ double stt[32][kMaxHH];
    const DevChan c = d.chans[d.it_sz0[blockIdx.x]];
    if (!d.active[c.prob]) return;
    const DevProb P = d.probs[c.prob];
    const int nhh = c.nhh, npp = c.npp, n2 = nhh * nhh;
    double acc[kMaxHH * kMaxHH / 256];
#pragma unroll
    for (int k = 0; k < kMaxHH * kMaxHH / 256; k++) acc[k] = 0.0;
    if (mask & CCD_T_QHH) {
        const double* t = d.t[cur] + c.t_off;
        const double* vt = d.vt + c.t_off;
        for (int r0 = 0; r0 < npp; r0 += 32) {
            int rc = min(32, npp - r0);
            for (int e = threadIdx.x; e < 32 * nhh; e += 256) {
                int r = e / nhh, col = e - r * nhh;
                bool ok = r < rc;
                sv[r][col] = ok ? vt[(int64_t)(r0 + r) * nhh + col] : 0.0;
                stt[r][col] = ok ? t[(int64_t)(r0 + r) * nhh + col] : 0.0;
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kMaxHH * kMaxHH / 256; k++) {
                int o = threadIdx.x + 256 * k;
                if (o < n2) {
                    int kl = o / nhh, ij = o - kl * nhh;
                    double s = 0.0;
                    for (int r = 0; r < rc; r++) s += sv[r][kl] * stt[r][ij];
                    acc[k] += s;
                }
            }
            __syncthreads();
        }
    }
    const int32_t* st = d.st + P.st_off;
#pragma unroll
    for (int k = 0; k < kMaxHH * kMaxHH / 256; k++) {
        int o = threadIdx.x + 256 * k;
        if (o < n2) {
            int kl = o / nhh, ij = o - kl * nhh;
            double v = 0.0;
            if (mask & CCD_T_HH) {
                int32_t p1 = d.hh[c.hh_off + kl], p2 = d.hh[c.hh_off + ij];
                v = vas(d.lut + P.lut_off, st[pa(p1)], st[pb(p1)], st[pa(p2)], st[pb(p2)]);
            }
            d.chh[c.chh_off + o] = v + acc[k];
        }
    }
}

// t -> particle-hole layout: each canonical amplitude lands at four places
__global__ void __launch_bounds__(256) k_scatter(DevPtrs d, int cur) {
    const Item it = d.it_elem[blockIdx.x];
    const DevChan c = d.chans[it.chan];
    if (!d.active[c.prob]) return;
    const DevProb P = d.probs[c.prob];
    const int nel = c.nhh * c.npp;
    for (int k = 0; k < kElemChunk / 256; k++) {
        int e = it.start + threadIdx.x + 256 * k;
        if (e < nel && e < it.start + kElemChunk) {
            int r = e / c.nhh, col = e - r * c.nhh;
            int32_t ab = d.pp[c.pp_off + r], ij = d.hh[c.hh_off + col];
            int a = pa(ab), b = pb(ab), i = pa(ij), j = pb(ij);
            double tv = d.t[cur][c.t_off + e];
            d.tt[zidx(d, P, a, i, b, j)] = tv;
            d.tt[zidx(d, P, a, j, b, i)] = -tv;
            d.tt[zidx(d, P, b, i, a, j)] = -tv;
            d.tt[zidx(d, P, b, j, a, i)] = tv;
        }
    }
}

// ring per cross channel Q (one block; 2 n^2 doubles of dynamic LDS):
//   B[x][m] = <kl||cd>, (c,k) in -Q, (d,l) in Q;   A = T~_Q
//   chi[x][y] = [RING] <kb||cj> + [QRING] 1/2 sum_m B[x][m] A[m][y]
//   Z_Q[u][y] = sum_x A[u][x] chi[x][y]
constexpr int kRingPer = (kMaxPH * kMaxPH + 255) / 256;
__global__ void __launch_bounds__(256) k_ring(DevPtrs d, uint32_t mask) {
    extern __shared__ double lds[];
    const DevPh q = d.ph[blockIdx.x];
    if (!d.active[q.prob]) return;
    const DevPh pq = d.ph[q.partner];
    const DevProb P = d.probs[q.prob];
    const int n = q.n, n2 = n * n;
    double* A = lds;
    double* B = lds + n2;
    const int32_t* st = d.st + P.st_off;
    const double* lut = d.lut + P.lut_off;
    for (int e = threadIdx.x; e < n2; e += 256) {
        A[e] = d.tt[q.z_off + e];
        double v = 0.0;
        if (mask & CCD_T_QRING) {
            int x = e / n, m = e - x * n;
            int32_t ck = d.phmem[pq.mem_off + x], dl = d.phmem[q.mem_off + m];
            v = vas(lut, st[pb(ck)], st[pb(dl)], st[pa(ck)], st[pa(dl)]);
        }
        B[e] = v;
    }
    __syncthreads();
    double acc[kRingPer];
#pragma unroll
    for (int k = 0; k < kRingPer; k++) {
        int e = threadIdx.x + 256 * k;
        double s = 0.0;
        if (e < n2) {
            int x = e / n, y = e - x * n;
            if (mask & CCD_T_QRING) {
                for (int m = 0; m < n; m++) s += B[x * n + m] * A[m * n + y];
                s *= 0.5;
            }
            if (mask & CCD_T_RING) {
                int32_t ck = d.phmem[pq.mem_off + x], bj = d.phmem[pq.mem_off + y];
                s += vas(lut, st[pb(ck)], st[pa(bj)], st[pa(ck)], st[pb(bj)]);
            }
        }
        acc[k] = s;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kRingPer; k++) {
        int e = threadIdx.x + 256 * k;
        if (e < n2) B[e] = acc[k];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n2; e += 256) {
        int u = e / n, y = e - u * n;
        double s = 0.0;
        for (int x = 0; x < n; x++) s += A[u * n + x] * B[x * n + y];
        d.z[q.z_off + e] = s;
    }
}

// fused S_z = 0 update: ladders, ring gather, one-body terms, division, mixing, energy
constexpr int kKC = 32;
__global__ void __launch_bounds__(256) k_ladder(DevPtrs d, int cur, double alpha, uint32_t mask) {
    // the K-loop tiles and the chi_klij block share the same LDS
    static_assert(kKC * kMaxHH + kKC * kLadderRows >= kMaxHH * kMaxHH, "LDS union too small");
    __shared__ double smem[kKC * kMaxHH + kKC * kLadderRows];
    __shared__ int32_t pcs[kKC][2];
    __shared__ double sh[4];
    double (*Ts)[kMaxHH] = reinterpret_cast<double (*)[kMaxHH]>(smem);
    double (*Vs)[kLadderRows] = reinterpret_cast<double (*)[kLadderRows]>(smem + kKC * kMaxHH);
    double* chi = smem;
    const Item it = d.it_ladder[blockIdx.x];
    const DevChan c = d.chans[it.chan];
    const DevProb P = d.probs[c.prob];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nhh = c.nhh, npp = c.npp;
    const int row = it.start + lane;
    const bool rv = row < npp;
    const int32_t* st = d.st + P.st_off;
    const double* eps = d.eps + P.st_off;
    const double* lut = d.lut + P.lut_off;
    const double* t = d.t[cur] + c.t_off;
    double* tn = d.t[cur ^ 1] + c.t_off;
    const double* vt = d.vt + c.t_off;
    const bool act = d.active[c.prob] != 0;
    const double al = act ? alpha : 0.0;

    int a = 0, b = 0;
    int32_t sa = 0, sb = 0;
    if (rv) {
        int32_t ab = d.pp[c.pp_off + row];
        a = pa(ab); b = pb(ab);
        sa = st[a]; sb = st[b];
    }
    constexpr int NC = kMaxHH / 4;
    double acc[NC];
#pragma unroll
    for (int k = 0; k < NC; k++) acc[k] = 0.0;

    if (act && (mask & CCD_T_PP)) {
        for (int c0 = 0; c0 < npp; c0 += kKC) {
            const int kc = min(kKC, npp - c0);
            for (int e = threadIdx.x; e < kKC * nhh; e += 256) {
                int rr = e / nhh, cc = e - rr * nhh;
                Ts[rr][cc] = rr < kc ? t[(int64_t)(c0 + rr) * nhh + cc] : 0.0;
            }
            if (threadIdx.x < kKC) {
                int32_t cd = threadIdx.x < kc ? d.pp[c.pp_off + c0 + threadIdx.x] : 0;
                pcs[threadIdx.x][0] = threadIdx.x < kc ? st[pa(cd)] : 0;
                pcs[threadIdx.x][1] = threadIdx.x < kc ? st[pb(cd)] : 0;
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kKC / 4; k++) {
                int cl = w + 4 * k;
                double v = 0.0;
                if (rv && cl < kc) v = vas(lut, sa, sb, pcs[cl][0], pcs[cl][1]);
                Vs[cl][lane] = v;
            }
            __syncthreads();
            for (int cl = 0; cl < kc; cl++) {
                double v = Vs[cl][lane];
#pragma unroll
                for (int k = 0; k < NC; k++) {
                    int col = w + 4 * k;
                    if (col < nhh) acc[k] += v * Ts[cl][col];
                }
            }
            __syncthreads();
        }
    }
    const bool hh_on = act && (mask & (CCD_T_HH | CCD_T_QHH));
    if (hh_on) {
        for (int e = threadIdx.x; e < nhh * nhh; e += 256) chi[e] = d.chh[c.chh_off + e];
        __syncthreads();
    }
    const bool ring_on = act && (mask & (CCD_T_RING | CCD_T_QRING));
    double es = 0.0;
    if (rv) {
#pragma unroll
        for (int k = 0; k < NC; k++) {
            int col = w + 4 * k;
            if (col < nhh) {
                int64_t e = (int64_t)row * nhh + col;
                double tc = t[e], v = vt[e];
                double tm = tc;
                if (act) {
                    int32_t ij = d.hh[c.hh_off + col];
                    int i = pa(ij), j = pb(ij);
                    double R = v + acc[k];
                    if (hh_on) {
                        double s = 0.0;
                        for (int kl = 0; kl < nhh; kl++) s += t[(int64_t)row * nhh + kl] * chi[kl * nhh + col];
                        R += s;
                    }
                    if (ring_on) R += ring_gather(d, P, a, b, i, j);
                    const double* dc = d.dchi + P.st_off;
                    R += (dc[a] + dc[b] - dc[i] - dc[j]) * tc;
                    double den = eps[i] + eps[j] - eps[a] - eps[b];
                    tm = al * (R / den) + (1.0 - al) * tc;
                }
                tn[e] = tm;
                es += v * tm;
            }
        }
    }
    double s = block_sum256(es, sh);
    if (threadIdx.x == 0) d.epart[blockIdx.x] = s;
}

// update of the S_z = +-1 blocks: only the ring and one-body terms survive
__global__ void __launch_bounds__(256) k_update(DevPtrs d, int cur, double alpha, uint32_t mask) {
    const Item it = d.it_nsz0[blockIdx.x];
    const DevChan c = d.chans[it.chan];
    const DevProb P = d.probs[c.prob];
    const bool act = d.active[c.prob] != 0;
    const bool ring_on = act && (mask & (CCD_T_RING | CCD_T_QRING));
    const int nel = c.nhh * c.npp;
    const double* eps = d.eps + P.st_off;
    const double* dc = d.dchi + P.st_off;
    for (int k = 0; k < kElemChunk / 256; k++) {
        int e = it.start + threadIdx.x + 256 * k;
        if (e < nel && e < it.start + kElemChunk) {
            double tc = d.t[cur][c.t_off + e];
            double tm = tc;
            if (act) {
                int r = e / c.nhh, col = e - r * c.nhh;
                int32_t ab = d.pp[c.pp_off + r], ij = d.hh[c.hh_off + col];
                int a = pa(ab), b = pb(ab), i = pa(ij), j = pb(ij);
                double R = d.vt[c.t_off + e];
                if (ring_on) R += ring_gather(d, P, a, b, i, j);
                R += (dc[a] + dc[b] - dc[i] - dc[j]) * tc;
                double den = eps[i] + eps[j] - eps[a] - eps[b];
                tm = alpha * (R / den) + (1.0 - alpha) * tc;
            }
            d.t[cur ^ 1][c.t_off + e] = tm;
        }
    }
}

// per-problem energy after a sweep, convergence test, divergence flag
__global__ void __launch_bounds__(256) k_energy(DevPtrs d, double tol) {
    __shared__ double sh[4];
    const int p = blockIdx.x;
    const DevProb P = d.probs[p];
    double s = 0.0;
    for (int x = P.ladder_lo + threadIdx.x; x < P.ladder_hi; x += 256) s += d.epart[x];
    double e = block_sum256(s, sh);
    if (threadIdx.x == 0 && d.active[p]) {
        double old = d.ecorr[p];
        d.eprev[p] = old;
        d.ecorr[p] = e;
        d.sweeps[p] += 1;
        if (!isfinite(e)) d.active[p] = 0;
        else if (tol > 0.0 && fabs(e - old) < tol) d.active[p] = 0;
    }
}

// --------------------------------------------------------------------------
// context
// --------------------------------------------------------------------------
enum Family { F_INIT = 0, F_ROWCOL, F_DCHI, F_CHH, F_SCATTER, F_RING, F_LADDER, F_UPDATE, F_ENERGY, F_NUM };
static const char* kFamilyNames[F_NUM] = {"init", "rowcol", "dchi", "chi_hhhh", "ph_scatter",
                                          "ring", "ladder_update", "update_sz1", "energy"};

struct Region {
    size_t off = 0, bytes = 0;
};

struct ccd_ctx {
    std::vector<HostProblem> probs;
    hipStream_t stream = nullptr;
    // concatenated host tables
    std::vector<DevProb> dprobs;
    std::vector<DevChan> dchans;
    std::vector<DevPh> dph;
    std::vector<int32_t> st, hh, pp, phmem, phq, phpos, dchi_ptr, dchi_idx, it_sz0;
    std::vector<double> eps, lut;
    std::vector<Item> it_elem, it_nsz0, it_ladder;
    int64_t NT = 0, NZ = 0;
    int n_rows = 0, n_cols = 0, n_chh = 0, ns_tot = 0, max_ph = 0;
    // workspace
    Region r_static, r_t0, r_t1, r_vt, r_chh, r_rows, r_cols, r_dchi, r_tt, r_z, r_epart, r_eparte,
        r_ecorr, r_eprev, r_emp2, r_active, r_sweeps;
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
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static DevPtrs make_ptrs(ccd_ctx* c) {
    DevPtrs d;
    char* base = c->ws;
    size_t o = c->r_static.off;
    auto take = [&](size_t bytes) {
        char* p = base + o;
        o += align256(bytes);
        return p;
    };
    d.st = (const int32_t*)take(c->st.size() * 4);
    d.eps = (const double*)take(c->eps.size() * 8);
    d.lut = (const double*)take(c->lut.size() * 8);
    d.probs = (const DevProb*)take(c->dprobs.size() * sizeof(DevProb));
    d.chans = (const DevChan*)take(c->dchans.size() * sizeof(DevChan));
    d.ph = (const DevPh*)take(c->dph.size() * sizeof(DevPh));
    d.hh = (const int32_t*)take(c->hh.size() * 4);
    d.pp = (const int32_t*)take(c->pp.size() * 4);
    d.phmem = (const int32_t*)take(c->phmem.size() * 4);
    d.phq = (const int32_t*)take(c->phq.size() * 4);
    d.phpos = (const int32_t*)take(c->phpos.size() * 4);
    d.dchi_ptr = (const int32_t*)take(c->dchi_ptr.size() * 4);
    d.dchi_idx = (const int32_t*)take(c->dchi_idx.size() * 4);
    d.it_elem = (const Item*)take(c->it_elem.size() * sizeof(Item));
    d.it_nsz0 = (const Item*)take(c->it_nsz0.size() * sizeof(Item));
    d.it_ladder = (const Item*)take(c->it_ladder.size() * sizeof(Item));
    d.it_sz0 = (const int32_t*)take(c->it_sz0.size() * 4);
    d.t[0] = (double*)(base + c->r_t0.off);
    d.t[1] = (double*)(base + c->r_t1.off);
    d.vt = (double*)(base + c->r_vt.off);
    d.chh = (double*)(base + c->r_chh.off);
    d.rowsum = (double*)(base + c->r_rows.off);
    d.colsum = (double*)(base + c->r_cols.off);
    d.dchi = (double*)(base + c->r_dchi.off);
    d.tt = (double*)(base + c->r_tt.off);
    d.z = (double*)(base + c->r_z.off);
    d.epart = (double*)(base + c->r_epart.off);
    d.epart_elem = (double*)(base + c->r_eparte.off);
    d.ecorr = (double*)(base + c->r_ecorr.off);
    d.eprev = (double*)(base + c->r_eprev.off);
    d.active = (int32_t*)(base + c->r_active.off);
    d.sweeps = (int32_t*)(base + c->r_sweeps.off);
    return d;
}

// host image of the static tables, in the order make_ptrs takes them
static std::vector<char> static_image(const ccd_ctx* c) {
    std::vector<char> img(c->r_static.bytes, 0);
    size_t o = 0;
    auto put = [&](const void* src, size_t bytes) {
        if (bytes) std::memcpy(img.data() + o, src, bytes);
        o += align256(bytes);
    };
    put(c->st.data(), c->st.size() * 4);
    put(c->eps.data(), c->eps.size() * 8);
    put(c->lut.data(), c->lut.size() * 8);
    put(c->dprobs.data(), c->dprobs.size() * sizeof(DevProb));
    put(c->dchans.data(), c->dchans.size() * sizeof(DevChan));
    put(c->dph.data(), c->dph.size() * sizeof(DevPh));
    put(c->hh.data(), c->hh.size() * 4);
    put(c->pp.data(), c->pp.size() * 4);
    put(c->phmem.data(), c->phmem.size() * 4);
    put(c->phq.data(), c->phq.size() * 4);
    put(c->phpos.data(), c->phpos.size() * 4);
    put(c->dchi_ptr.data(), c->dchi_ptr.size() * 4);
    put(c->dchi_idx.data(), c->dchi_idx.size() * 4);
    put(c->it_elem.data(), c->it_elem.size() * sizeof(Item));
    put(c->it_nsz0.data(), c->it_nsz0.size() * sizeof(Item));
    put(c->it_ladder.data(), c->it_ladder.size() * sizeof(Item));
    put(c->it_sz0.data(), c->it_sz0.size() * 4);
    return img;
}

static void layout(ccd_ctx* c) {
    size_t s = 0;
    auto add = [&](size_t bytes) { s += align256(bytes); };
    add(c->st.size() * 4); add(c->eps.size() * 8); add(c->lut.size() * 8);
    add(c->dprobs.size() * sizeof(DevProb)); add(c->dchans.size() * sizeof(DevChan));
    add(c->dph.size() * sizeof(DevPh)); add(c->hh.size() * 4); add(c->pp.size() * 4);
    add(c->phmem.size() * 4); add(c->phq.size() * 4); add(c->phpos.size() * 4);
    add(c->dchi_ptr.size() * 4); add(c->dchi_idx.size() * 4);
    add(c->it_elem.size() * sizeof(Item)); add(c->it_nsz0.size() * sizeof(Item));
    add(c->it_ladder.size() * sizeof(Item)); add(c->it_sz0.size() * 4);
    size_t o = 0;
    auto region = [&](Region& r, size_t bytes) {
        r.off = o;
        r.bytes = bytes;
        o += align256(bytes);
    };
    size_t P = c->probs.size();
    region(c->r_static, s);
    region(c->r_t0, c->NT * 8);
    region(c->r_t1, c->NT * 8);
    region(c->r_vt, c->NT * 8);
    region(c->r_chh, (size_t)std::max(1, c->n_chh) * 8);
    region(c->r_rows, (size_t)std::max(1, c->n_rows) * 8);
    region(c->r_cols, (size_t)std::max(1, c->n_cols) * 8);
    region(c->r_dchi, (size_t)c->ns_tot * 8);
    region(c->r_tt, c->NZ * 8);
    region(c->r_z, c->NZ * 8);
    region(c->r_epart, std::max<size_t>(1, c->it_ladder.size()) * 8);
    region(c->r_eparte, std::max<size_t>(1, c->it_elem.size()) * 8);
    region(c->r_ecorr, P * 8);
    region(c->r_eprev, P * 8);
    region(c->r_emp2, P * 8);
    region(c->r_active, P * 4);
    region(c->r_sweeps, P * 4);
    c->ws_bytes = o;
}

static ccd_status assemble(ccd_ctx* c) {
    int st_off = 0, lut_off = 0, ph_off = 0, hh_off = 0, pp_off = 0, phm_off = 0, phc_off = 0;
    int64_t t_off = 0, z_off = 0;
    int row_off = 0, col_off = 0, chh_off = 0;
    // per-state CSR lists for the one-body intermediates
    std::vector<std::vector<int32_t>> lists;
    for (size_t pi = 0; pi < c->probs.size(); pi++) {
        HostProblem& H = c->probs[pi];
        DevProb P;
        P.ns = H.ns; P.nh = H.nh; P.np = H.np;
        P.st_off = st_off; P.lut_off = lut_off; P.ph_off = ph_off;
        for (int s = 0; s < H.ns; s++) c->st.push_back(pack_state(H.nx[s], H.ny[s], H.nz[s], H.sz[s]));
        c->eps.insert(c->eps.end(), H.eps.begin(), H.eps.end());
        for (double w : H.W) c->lut.push_back(0.5 * w);
        lists.resize(st_off + H.ns);
        // direct channels
        P.elem_lo = (int)c->it_elem.size();
        P.ladder_lo = (int)c->it_ladder.size();
        for (size_t ci = 0; ci < H.chans.size(); ci++) {
            const Chan& h = H.chans[ci];
            DevChan d;
            d.t_off = t_off + h.t_off;
            d.prob = (int)pi;
            d.nhh = h.nhh; d.npp = h.npp; d.sz = h.Sz;
            d.hh_off = hh_off + h.hh_off;
            d.pp_off = pp_off + h.pp_off;
            d.chh_off = -1; d.row_off = -1; d.col_off = -1; d.pad = 0;
            int gid = (int)c->dchans.size();
            if (h.Sz == 0) {
                d.chh_off = chh_off; chh_off += h.nhh * h.nhh;
                d.row_off = row_off;
                d.col_off = col_off;
                for (int r = 0; r < h.npp; r++) {
                    int a = H.pp[2 * (h.pp_off + r)], b = H.pp[2 * (h.pp_off + r) + 1];
                    lists[st_off + a].push_back(-(row_off + r) - 1);
                    lists[st_off + b].push_back(-(row_off + r) - 1);
                }
                for (int q = 0; q < h.nhh; q++) {
                    int i = H.hh[2 * (h.hh_off + q)], j = H.hh[2 * (h.hh_off + q) + 1];
                    lists[st_off + i].push_back(col_off + q);
                    lists[st_off + j].push_back(col_off + q);
                }
                row_off += h.npp; col_off += h.nhh;
                c->it_sz0.push_back(gid);
                for (int r0 = 0; r0 < h.npp; r0 += kLadderRows) c->it_ladder.push_back({gid, r0});
            }
            int nel = h.nhh * h.npp;
            for (int e0 = 0; e0 < nel; e0 += kElemChunk) {
                c->it_elem.push_back({gid, e0});
                if (h.Sz != 0) c->it_nsz0.push_back({gid, e0});
            }
            c->dchans.push_back(d);
        }
        P.elem_hi = (int)c->it_elem.size();
        P.ladder_hi = (int)c->it_ladder.size();
        for (size_t k = 0; k < H.hh.size() / 2; k++) c->hh.push_back(pack_pair(H.hh[2 * k], H.hh[2 * k + 1]));
        for (size_t k = 0; k < H.pp.size() / 2; k++) c->pp.push_back(pack_pair(H.pp[2 * k], H.pp[2 * k + 1]));
        // cross channels
        for (const PhChan& h : H.ph) {
            DevPh d;
            d.z_off = z_off + h.z_off;
            d.prob = (int)pi;
            d.n = h.n;
            d.partner = phc_off + h.partner;
            d.mem_off = phm_off + h.mem_off;
            c->dph.push_back(d);
            c->max_ph = std::max(c->max_ph, h.n);
        }
        for (size_t k = 0; k < H.phmem.size() / 2; k++)
            c->phmem.push_back(pack_pair(H.phmem[2 * k], H.phmem[2 * k + 1]));
        for (size_t k = 0; k < H.phq.size(); k++) {
            c->phq.push_back(phc_off + H.phq[k]);
            c->phpos.push_back(H.phpos[k]);
        }
        c->dprobs.push_back(P);
        st_off += H.ns;
        lut_off += (int)H.W.size();
        ph_off += (int)H.phq.size();
        hh_off += (int)H.hh.size() / 2;
        pp_off += (int)H.pp.size() / 2;
        phm_off += (int)H.phmem.size() / 2;
        phc_off += (int)H.ph.size();
        t_off += H.n_amp;
        z_off += H.nz_ph;
    }
    c->NT = t_off;
    c->NZ = z_off;
    c->n_rows = row_off;
    c->n_cols = col_off;
    c->n_chh = chh_off;
    c->ns_tot = st_off;
    c->dchi_ptr.push_back(0);
    for (auto& l : lists) {
        c->dchi_idx.insert(c->dchi_idx.end(), l.begin(), l.end());
        c->dchi_ptr.push_back((int32_t)c->dchi_idx.size());
    }
    if (c->dchi_idx.empty()) c->dchi_idx.push_back(0);
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

static ccd_status sweep(ccd_ctx* c, double alpha, double tol, uint32_t mask) {
    DevPtrs d = make_ptrs(c);
    const int cur = c->cur;
    const int nsz0 = (int)c->it_sz0.size();
    if (mask & (CCD_T_QHOLE | CCD_T_QPART)) {
        LAUNCH(F_ROWCOL, k_rowcol, nsz0, 256, 0, d, cur);
    }
    LAUNCH(F_DCHI, k_dchi, (c->ns_tot + 255) / 256, 256, 0, d, c->ns_tot, mask);
    if (mask & (CCD_T_HH | CCD_T_QHH)) {
        LAUNCH(F_CHH, k_chh, nsz0, 256, 0, d, cur, mask);
    }
    if (mask & (CCD_T_RING | CCD_T_QRING)) {
        LAUNCH(F_SCATTER, k_scatter, (int)c->it_elem.size(), 256, 0, d, cur);
        size_t lds = (size_t)2 * c->max_ph * c->max_ph * sizeof(double);
        LAUNCH(F_RING, k_ring, (int)c->dph.size(), 256, lds, d, mask);
    }
    LAUNCH(F_LADDER, k_ladder, (int)c->it_ladder.size(), 256, 0, d, cur, alpha, mask);
    LAUNCH(F_UPDATE, k_update, (int)c->it_nsz0.size(), 256, 0, d, cur, alpha, mask);
    LAUNCH(F_ENERGY, k_energy, (int)c->probs.size(), 256, 0, d, tol);
    c->cur ^= 1;
    return CCD_OK;
}

// --------------------------------------------------------------------------
// C ABI
// --------------------------------------------------------------------------
extern "C" {

const char* ccd_last_error(void) { return g_err.c_str(); }
const char* ccd_version(void) { return "ccd-mi355x 0.1 (gfx950)"; }

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
    for (int i = 0; i < n; i++) {
        std::string err;
        ccd_status s = build_problem(probs[i], c->probs[i], err);
        if (s != CCD_OK) {
            set_error("problem " + std::to_string(i) + ": " + err);
            delete c;
            return s;
        }
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
    LAUNCH(F_INIT, k_init, (int)c->it_elem.size(), 256, 0, d, 0);
    LAUNCH(F_ENERGY, k_energy_elem, (int)c->probs.size(), 256, 0, d);
    return CCD_OK;
}

ccd_status ccd_bind_workspace(ccd_ctx* c, void* ptr, size_t bytes) {
    if (!c || !ptr) { set_error("ccd_bind_workspace: NULL argument"); return CCD_EINVAL; }
    if (c->bound) { set_error("a workspace is already bound"); return CCD_ESTATE; }
    if (bytes < c->ws_bytes) { set_error("workspace too small"); return CCD_EINVAL; }
    if (((uintptr_t)ptr) & 255) { set_error("workspace must be 256-byte aligned"); return CCD_EINVAL; }
    c->ws = (char*)ptr;
    size_t lds = (size_t)2 * c->max_ph * c->max_ph * sizeof(double);
    HIP_TRY(hipFuncSetAttribute((const void*)k_ring, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    std::vector<char> img = static_image(c);
    HIP_TRY(hipMemcpyAsync(c->ws + c->r_static.off, img.data(), img.size(), hipMemcpyHostToDevice, c->stream));
    // dynamic regions start at zero (particle-hole positions with i = k or a = c stay zero)
    HIP_TRY(hipMemsetAsync(c->ws + c->r_t0.off, 0, c->ws_bytes - c->r_t0.off, c->stream));
    c->bound = true;
    ccd_status s = ccd_reset_amplitudes(c);
    if (s != CCD_OK) return s;
    std::vector<double> e(c->probs.size());
    HIP_TRY(hipMemcpyAsync(e.data(), c->ws + c->r_ecorr.off, e.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->emp2 = e;
    HIP_TRY(hipMemcpyAsync(c->ws + c->r_emp2.off, e.data(), e.size() * 8, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return CCD_OK;
}

ccd_status ccd_iterate(ccd_ctx* c, const ccd_solver_opts* o, int32_t* sweeps_done, double* e_hist) {
    if (!c || !o) { set_error("ccd_iterate: NULL argument"); return CCD_EINVAL; }
    if (!c->bound) { set_error("ccd_iterate: no workspace bound"); return CCD_ESTATE; }
    if (!(o->mixing > 0.0 && o->mixing <= 1.0) || o->max_iter < 1) {
        set_error("ccd_iterate: need 0 < mixing <= 1 and max_iter >= 1");
        return CCD_EINVAL;
    }
    if (o->precision != CCD_PREC_FP64) {
        set_error("ccd_iterate: this build runs the FP64 contraction path only");
        return CCD_EINVAL;
    }
    const int P = (int)c->probs.size();
    std::vector<int32_t> ones(P, 1), zeros(P, 0);
    HIP_TRY(hipMemcpyAsync(c->ws + c->r_active.off, ones.data(), P * 4, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->ws + c->r_sweeps.off, zeros.data(), P * 4, hipMemcpyHostToDevice, c->stream));
    const bool check = o->tol > 0.0 || e_hist;
    std::vector<double> e(P);
    std::vector<int32_t> act(P, 1);
    if (e_hist)
        for (size_t k = 0; k < (size_t)P * o->max_iter; k++) e_hist[k] = NAN;
    bool all_done = false;
    for (int s = 0; s < o->max_iter && !all_done; s++) {
        ccd_status st = sweep(c, o->mixing, o->tol, o->terms);
        if (st != CCD_OK) return st;
        if (check) {
            std::vector<int32_t> was = act;
            HIP_TRY(hipMemcpyAsync(e.data(), c->ws + c->r_ecorr.off, P * 8, hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(hipMemcpyAsync(act.data(), c->ws + c->r_active.off, P * 4, hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(hipStreamSynchronize(c->stream));
            all_done = true;
            for (int p = 0; p < P; p++) {
                if (e_hist && was[p]) e_hist[(size_t)p * o->max_iter + s] = e[p];
                if (act[p]) all_done = false;
            }
            if (o->tol <= 0.0) all_done = false;
        }
    }
    std::vector<int32_t> sw(P);
    HIP_TRY(hipMemcpyAsync(sw.data(), c->ws + c->r_sweeps.off, P * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(e.data(), c->ws + c->r_ecorr.off, P * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(act.data(), c->ws + c->r_active.off, P * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (sweeps_done)
        for (int p = 0; p < P; p++) sweeps_done[p] = sw[p];
    for (int p = 0; p < P; p++)
        if (!std::isfinite(e[p])) {
            set_error("problem " + std::to_string(p) + ": correlation energy is not finite");
            return CCD_DIVERGED;
        }
    if (o->tol > 0.0)
        for (int p = 0; p < P; p++)
            if (act[p]) return CCD_NOT_CONVERGED;
    return CCD_OK;
}

ccd_status ccd_energy(const ccd_ctx* cc, int32_t p, double* eref, double* emp2, double* ecorr) {
    ccd_ctx* c = (ccd_ctx*)cc;
    if (!c || p < 0 || p >= (int)c->probs.size()) { set_error("ccd_energy: bad problem"); return CCD_EINVAL; }
    if (eref) *eref = c->probs[p].eref;
    if (emp2 || ecorr) {
        if (!c->bound) { set_error("ccd_energy: no workspace bound"); return CCD_ESTATE; }
        double e = 0;
        HIP_TRY(hipMemcpyAsync(&e, c->ws + c->r_ecorr.off + 8 * p, 8, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        if (emp2) *emp2 = c->emp2[p];
        if (ecorr) *ecorr = e;
    }
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

static int64_t prob_t_off(const ccd_ctx* c, int p) {
    int64_t o = 0;
    for (int q = 0; q < p; q++) o += c->probs[q].n_amp;
    return o;
}

ccd_status ccd_get_amplitudes(const ccd_ctx* c, int32_t p, double* dst, size_t n) {
    if (!c || !dst || p < 0 || p >= (int)c->probs.size()) { set_error("ccd_get_amplitudes: bad argument"); return CCD_EINVAL; }
    if (!c->bound) { set_error("no workspace bound"); return CCD_ESTATE; }
    if (n != (size_t)c->probs[p].n_amp) { set_error("ccd_get_amplitudes: n != n_amplitudes"); return CCD_EINVAL; }
    const Region& r = c->cur ? c->r_t1 : c->r_t0;
    HIP_TRY(hipMemcpyAsync(dst, c->ws + r.off + 8 * prob_t_off(c, p), n * 8, hipMemcpyDeviceToHost, c->stream));
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
    HIP_TRY(hipMemcpyAsync(c->ws + r.off + 8 * prob_t_off(c, p), src, n * 8, hipMemcpyHostToDevice, c->stream));
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
    if (!c->ev_pool.empty()) {
        if (!c->pending.empty()) (void)hipStreamSynchronize(c->stream);
        for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    }
    delete c;
}

}  // extern "C"
