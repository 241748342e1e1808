// ccd_nm.hip -- CCD for infinite nuclear matter with isospin (protons and
// neutrons) on gfx950: host plan, kernels and the C ABI of include/ccd_nm.h.
//
// One Jacobi sweep of eq. ccd3 in the intermediates form (sec. "Developing a
// CCD code for infinite matter"), every term from the current amplitudes t:
//   k_nm_gather   T~_Q[(a,i)][(c,k)] = t_ik^ac for every cross channel Q
//   k_nm_rowcol   row and column sums of t <ab||ij> per direct channel, from
//   k_nm_colsum   chunks of whole rows (column parts added in chunk order)
//   k_nm_gemm     (launch 1) chi_klij = <kl||ij> + sum_{c<d} <kl||cd> t_ij^cd per
//                 direct channel; C_P = <kb||cj>_P + 1/2 Vbar T~_Q per cross
//                 channel (chi_kbcj of the ring of Q, P = -Q)
//                 (launch 2) ladders sum_{c<d} <ab||cd> t_ij^cd +
//                 sum_{k<l} t_kl^ab chi_klij per direct channel; the ring
//                 Z_Q = T~_Q C_P per cross channel, scattered to the four ring
//                 slots of the amplitudes it feeds
//   k_nm_update   R / eps_ij^ab with the one-body terms, mixing, energy parts
//   k_nm_energy   fixed-order energy sum
// The products run on the FP64 16x16x4 MFMA over LDS-staged chunks; the
// interaction is generated where a product reads it, from four tables of the
// spin-isospin classes of the Minnesota operator.  No floating-point atomics:
// every sum has a fixed order, so results are bit-identical run to run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "ccd_internal.h"
#include "../../include/ccd_nm.h"

namespace {

#define NM_TRY(x)                                                                   \
    do {                                                                            \
        hipError_t e_ = (x);                                                        \
        if (e_ != hipSuccess) {                                                     \
            ccd::set_error(std::string("ccd_nm: ") + #x + ": " + hipGetErrorString(e_)); \
            return CCD_EHIP;                                                        \
        }                                                                           \
    } while (0)

constexpr int kNmMaxNmax2 = 64;
constexpr int kNmChunk = 1024;   // amplitudes per elementwise work item
constexpr int kNmHist = 64;

// A state: bytes 0..2 n_x, n_y, n_z (int8); byte 3 bit 0 = spin up, bit 1 = neutron.
__host__ __device__ inline int32_t nm_pack(int x, int y, int z, int s, int t) {
    return (int32_t)((uint32_t)(uint8_t)(int8_t)x | ((uint32_t)(uint8_t)(int8_t)y << 8) |
                     ((uint32_t)(uint8_t)(int8_t)z << 16) | ((uint32_t)((s > 0) | ((t > 0) << 1)) << 24));
}
__host__ __device__ inline int nm_x(int32_t s) { return (int)(int8_t)(s & 0xff); }
__host__ __device__ inline int nm_y(int32_t s) { return (int)(int8_t)((s >> 8) & 0xff); }
__host__ __device__ inline int nm_z(int32_t s) { return (int)(int8_t)((s >> 16) & 0xff); }
__host__ __device__ inline int nm_st(int32_t s) { return (s >> 24) & 3; }
__host__ __device__ inline int nm_d2(int32_t a, int32_t b) {
    const int x = nm_x(a) - nm_x(b), y = nm_y(a) - nm_y(b), z = nm_z(a) - nm_z(b);
    return x * x + y * y + z * z;
}

// The antisymmetrised Minnesota element for a momentum-conserving quadruple.
// With the spin (isospin) factors of the direct term d_s = [s_p = s_r][s_q = s_s]
// and of the exchange term x_s = [s_p = s_s][s_q = s_r] (d_t, x_t alike), the
// operator of each Gaussian channel a is a combination of 1, P_s, P_t, P_s P_t
// whose matrix element is c_a = (R: (d_s d_t - x_s x_t)/2,
// T: (d_s d_t + x_s d_t - d_s x_t - x_s x_t)/4, S: (d_s d_t - x_s d_t + d_s x_t - x_s x_t)/4),
// and the exchange term carries -c_a, so
//   <pq||rs> = sum_a c_a (W_a(|n_p - n_r|^2) + W_a(|n_p - n_s|^2)).
// The nonzero (c_R, c_T, c_S) are +-(1/2, 0, 1/2), +-(1/2, 1/2, 0),
// +-(1/2, 1/4, 1/4) and +-(0, 1/4, -1/4); u holds the four combined tables
// U_k(m) = c . W(m) for k = 0..3 (nlut entries each), and the 4-bit code
// (d_s, x_s, d_t, x_t) picks the table and the sign.
// The table k and sign of the element from the spin-isospin labels (bit 0 spin
// up, bit 1 neutron) of p, q, r, s; false when the element is zero.
__host__ __device__ inline bool nm_class(int a, int b, int c, int d, int& k, bool& neg) {
    const int ds = ((a & 1) == (c & 1)) & ((b & 1) == (d & 1));
    const int xs = ((a & 1) == (d & 1)) & ((b & 1) == (c & 1));
    const int dt = ((a >> 1) == (c >> 1)) & ((b >> 1) == (d >> 1));
    const int xt = ((a >> 1) == (d >> 1)) & ((b >> 1) == (c >> 1));
    const int code = (ds << 3) | (xs << 2) | (dt << 1) | xt;
    neg = false;
    switch (code) {
        case 11: k = 0; break;               // (1,0,1,1)
        case 7: k = 0; neg = true; break;    // (0,1,1,1)
        case 14: k = 1; break;               // (1,1,1,0)
        case 13: k = 1; neg = true; break;   // (1,1,0,1)
        case 10: k = 2; break;               // (1,0,1,0)
        case 5: k = 2; neg = true; break;    // (0,1,0,1)
        case 6: k = 3; break;                // (0,1,1,0)
        case 9: k = 3; neg = true; break;    // (1,0,0,1)
        default: return false;
    }
    return true;
}

__host__ __device__ inline double nm_vas(const double* u, int nlut, int32_t p, int32_t q, int32_t r, int32_t s) {
    int k = 0;
    bool neg = false;
    if (!nm_class(nm_st(p), nm_st(q), nm_st(r), nm_st(s), k, neg)) return 0.0;
    const double w = u[k * nlut + nm_d2(p, r)] + u[k * nlut + nm_d2(p, s)];
    return neg ? -w : w;
}

__host__ __device__ inline int pr_a(int32_t v) { return v & 0xffff; }
__host__ __device__ inline int pr_b(int32_t v) { return (int)((uint32_t)v >> 16); }

// ---------------------------------------------------------------------------
// device data
// ---------------------------------------------------------------------------
struct NmItem {
    int32_t chan, start;  // direct channel, first amplitude (local to the channel)
};

struct NmChanD {
    int64_t t_off;
    int32_t nhh, npp, hh_off, pp_off, chh_off;
    int32_t rc_lo, rc_n;   // its row-chunk items of the row and column sums
};

// a chunk of whole rows of a block for the row and column sums; its column
// parts (n_hh of them) start at poff
struct NmRcItem {
    int32_t chan, r0, nr, poff;
};

// arrays a product reads or writes
enum { ARR_T = 0, ARR_VT = 1, ARR_CHH = 2, ARR_TQ = 3, ARR_CP = 4, ARR_LAD = 5 };
// operand / output modes of the channel products
enum { AM_ROW = 0, AM_COL = 1, AM_GPAIR = 2, AM_GVBAR = 3 };
enum { CM_NONE = 0, CM_GPAIR = 1, CM_GVPH = 2 };
enum { OM_ROW = 0, OM_SCATTER = 1, OM_ROW_ADD = 2 };  // OM_ROW_ADD: added to the output array's value

struct NmSeg {
    int32_t K, amode, lda, term;   // term: mask bits that enable the segment
    int64_t a_off;                 // AM_ROW / AM_COL: element offset into the A array
    int32_t a_rows, a_cols;        // generated: offsets of the row / column lists
    int32_t a_arr;                 // the A array (ARR_*) of AM_ROW / AM_COL
    int32_t b_arr;                 // the B array (ARR_*)
    int64_t b_off;
    int32_t ldb;
    double alpha;
};

struct NmJob {
    int32_t M, N, nseg, cmode, cterm, omode, ldo, c_rows, c_cols, tiles_n;
    int64_t o_off;                 // OM_ROW: offset into the output array; OM_SCATTER: into the map
    int32_t o_arr;                 // OM_ROW: the output array (ARR_CHH, ARR_CP or ARR_LAD)
    NmSeg seg[2];
};

struct NmTile {
    int32_t job, tm, tn;
};

// The pp ladder of a direct channel as products over its momentum pairs (see
// k_nm_ladpp).  Row slots 0..3 of a momentum pair are the rows X_0, Y_0, X_1,
// Y_1 of the differences delta_j = t(X_j) - t(Y_j); rec[slot] gives, for j = 0
// and 1, the coefficient of u_(class, j) in that row's sum (bits 0-1 and 3-4:
// 0 none, 1 plus, 2 minus) and its class (bits 2 and 5).
struct NmLadD {
    int32_t chan, lp_off, n_lp;    // direct channel; its momentum pairs (offset in pairs, count)
    int32_t nd, nk;                // differences (0..2) and element classes (0..2)
    int32_t tab[2];                // the table of each class
    int32_t kx, ky, kz;            // total momentum
    int32_t rec[4];
};

struct NmLadItem {
    int32_t lad, start;            // channel entry; first momentum pair | 16-column tile << 20
};

struct NmDev {
    const int32_t* st;      // packed states
    const double* u;        // the four element tables
    const double* eps;
    const int32_t* hh;      // hole pairs (i | j << 16), channel after channel
    const int32_t* pp;      // particle pairs
    const int32_t* mem;     // cross-channel members (p | h << 16)
    const int32_t* pmap;    // ring position maps
    const NmChanD* ch;
    const NmItem* items;
    const NmRcItem* rcit;   // row chunks of the row and column sums
    double* cpart;          // their column parts
    const NmJob* jobs;
    const NmTile* tiles;
    const NmLadD* ladd;     // pp ladder over momentum pairs: channels,
    const int4* ladlp;      // two int4 per momentum pair: (p packed, |p|^2 | |q|^2 << 10, X_0, Y_0), (X_1, Y_1, 0, 0)
    const NmLadItem* ladit; // and work items
    const int32_t* csr_ptr; // per state: rows (particles) or columns (holes) holding it
    const int32_t* csr_idx;
    const int32_t* row_chan;  // global row -> channel ; global column -> channel
    double* t[2];
    double* vt;
    double* chh;
    double* tq;             // gathered T~_Q blocks
    double* cp;             // C_P blocks
    double* lad;            // ladder sums (t layout)
    double* ring;           // four ring slots per amplitude
    double* rowsum;         // per global row: sum_cols t vt
    double* colsum;         // per global column: sum_rows t vt
    double* dchi;           // per state
    double* epart;
    double* ehist;          // [kNmHist]
    int32_t ns, nlut, n_items, n_tq;
    int64_t n_amp;
};

__device__ __forceinline__ double nm_wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// fixed-order sum over a 256-thread block: wave sums, then the four in order
__device__ __forceinline__ double nm_block_sum(double v, double* sh) {
    v = nm_wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = ((sh[0] + sh[1]) + sh[2]) + sh[3];
    __syncthreads();
    return r;
}

// <ab||ij>, t0 = <ab||ij> / eps_ij^ab, energy parts (eq. ccdGuess)
__global__ void __launch_bounds__(256) k_nm_init(NmDev d) {
    __shared__ double sh[4];
    for (int w = blockIdx.x; w < d.n_items; w += gridDim.x) {
        const NmItem it = d.items[w];
        const NmChanD C = d.ch[it.chan];
        const int64_t n = (int64_t)C.nhh * C.npp;
        double acc = 0.0;
        for (int k = threadIdx.x; k < kNmChunk; k += 256) {
            const int64_t e = (int64_t)it.start + k;
            if (e < n) {
                const int r = (int)(e / C.nhh), c = (int)(e - (int64_t)r * C.nhh);
                const int32_t P = d.pp[C.pp_off + r], H = d.hh[C.hh_off + c];
                const int a = pr_a(P), b = pr_b(P), i = pr_a(H), j = pr_b(H);
                const double v = nm_vas(d.u, d.nlut, d.st[a], d.st[b], d.st[i], d.st[j]);
                const double den = d.eps[i] + d.eps[j] - d.eps[a] - d.eps[b];
                const double t0 = v / den;
                d.vt[C.t_off + e] = v;
                d.t[0][C.t_off + e] = t0;
                acc += v * t0;
            }
        }
        acc = nm_block_sum(acc, sh);
        if (threadIdx.x == 0) d.epart[w] = acc;
    }
}

// energy parts sum vt t of amplitudes `cur`
__global__ void __launch_bounds__(256) k_nm_dot(NmDev d, int cur) {
    __shared__ double sh[4];
    for (int w = blockIdx.x; w < d.n_items; w += gridDim.x) {
        const NmItem it = d.items[w];
        const NmChanD C = d.ch[it.chan];
        const int64_t n = (int64_t)C.nhh * C.npp;
        double acc = 0.0;
        for (int k = threadIdx.x; k < kNmChunk; k += 256) {
            const int64_t e = (int64_t)it.start + k;
            if (e < n) acc += d.vt[C.t_off + e] * d.t[cur][C.t_off + e];
        }
        acc = nm_block_sum(acc, sh);
        if (threadIdx.x == 0) d.epart[w] = acc;
    }
}

// energy (eq. ccdcorr with unordered pairs): the item parts in item order;
// written to ehist[slot]
__global__ void __launch_bounds__(256) k_nm_energy(NmDev d, int slot) {
    __shared__ double sh[256];
    // each thread sums a contiguous run of items in order, then a fixed tree
    const int per = (d.n_items + 255) / 256;
    double s = 0.0;
    for (int k = 0; k < per; k++) {
        const int w = threadIdx.x * per + k;
        if (w < d.n_items) s += d.epart[w];
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) d.ehist[slot] = sh[0];
}

// T~_Q[u][x] = t_ik^ac, (a,i) member u of Q, (c,k) member x of its partner;
// the position map gives the canonical amplitude e and the sign
__global__ void __launch_bounds__(256) k_nm_gather(NmDev d, int cur) {
    const double* t = d.t[cur];
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < d.n_tq; k += (int64_t)gridDim.x * 256) {
        const int32_t m = d.pmap[k];
        double v = 0.0;
        if (m >= 0) {
            v = t[m >> 3];
            if (m & 1) v = -v;
        }
        d.tq[k] = v;
    }
}

// row and column sums of t <ab||ij> per block, from chunks of whole rows (at
// most kNmChunk amplitudes) loaded with coalesced reads: the products in LDS,
// then each row's sum in column order and each column's part over the chunk's
// rows in row order; k_nm_colsum adds a column's parts in chunk order.
__global__ void __launch_bounds__(256) k_nm_rowcol(NmDev d, int cur, int n_items) {
    __shared__ double ps[kNmChunk];
    const double* t = d.t[cur];
    for (int bi = blockIdx.x; bi < n_items; bi += gridDim.x) {
        const NmRcItem it = d.rcit[bi];
        const NmChanD C = d.ch[it.chan];
        const int nhh = C.nhh, ne = it.nr * nhh;
        const int64_t o = C.t_off + (int64_t)it.r0 * nhh;
        if (ne > kNmChunk) {  // one row longer than the buffer (nr = 1): straight from memory
            for (int q = threadIdx.x; q < nhh; q += 256) d.cpart[it.poff + q] = t[o + q] * d.vt[o + q];
            if (threadIdx.x == 0) {
                double s = 0.0;
                for (int x = 0; x < nhh; x++) s += t[o + x] * d.vt[o + x];
                d.rowsum[C.pp_off + it.r0] = s;
            }
            continue;
        }
        __syncthreads();  // the previous item's reads of ps are done
        for (int x = threadIdx.x; x < ne; x += 256) ps[x] = t[o + x] * d.vt[o + x];
        __syncthreads();
        for (int r = threadIdx.x; r < it.nr; r += 256) {
            double s = 0.0;
            for (int x = 0; x < nhh; x++) s += ps[r * nhh + x];
            d.rowsum[C.pp_off + it.r0 + r] = s;
        }
        for (int q = threadIdx.x; q < nhh; q += 256) {
            double s = 0.0;
            for (int r = 0; r < it.nr; r++) s += ps[r * nhh + q];
            d.cpart[it.poff + q] = s;
        }
    }
}

// a block's chunks are consecutive and each holds n_hh parts, so the parts of
// column lc are n_hh apart from the first chunk's; eight loads are issued
// before they are added in chunk order
__global__ void __launch_bounds__(256) k_nm_colsum(NmDev d, int n_rows, int n_cols) {
    for (int q = blockIdx.x * 256 + threadIdx.x; q < n_cols; q += gridDim.x * 256) {
        const NmChanD C = d.ch[d.row_chan[n_rows + q]];
        const double* pc = d.cpart + d.rcit[C.rc_lo].poff + (q - C.hh_off);
        const int n = C.rc_n, step = C.nhh;
        double s = 0.0;
        int i = 0;
        for (; i + 8 <= n; i += 8) {
            double v[8];
#pragma unroll
            for (int k = 0; k < 8; k++) v[k] = pc[(int64_t)(i + k) * step];
#pragma unroll
            for (int k = 0; k < 8; k++) s += v[k];
        }
        for (; i < n; i++) s += pc[(int64_t)i * step];
        d.colsum[q] = s;
    }
}

// one-body intermediates, diagonal by momentum, spin and isospin conservation:
//   chi_bb - f_bb = -1/2 sum_kld t_kl^bd <kl||bd> = -(sum of the row sums of
//   the rows holding b), chi_jj - f_jj = +1/2 sum_cdl <jl||cd> t_jl^cd = +(sum of
//   the column sums of the columns holding j); one wave per state: lane l sums
//   entries l, l + 64, ... of its CSR list, then a fixed butterfly over the lanes
__global__ void __launch_bounds__(256) k_nm_dchi(NmDev d, uint32_t mask, int nh) {
    const int lane = threadIdx.x & 63;
    const int wid = (blockIdx.x * 256 + threadIdx.x) >> 6, nw = (gridDim.x * 256) >> 6;
    for (int s = wid; s < d.ns; s += nw) {
        double acc = 0.0;
        const bool hole = s < nh;
        if (hole ? (mask & CCD_T_QHOLE) : (mask & CCD_T_QPART)) {
            for (int k = d.csr_ptr[s] + lane; k < d.csr_ptr[s + 1]; k += 64)
                acc += hole ? d.colsum[d.csr_idx[k]] : d.rowsum[d.csr_idx[k]];
        }
        acc = nm_wave_sum(acc);
        if (lane == 0) d.dchi[s] = hole ? acc : -acc;
    }
}

// ---- the channel products ---------------------------------------------------
typedef double nm_d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double* nm_arr(const NmDev& d, int which, int cur) {
    switch (which) {
        case ARR_T: return d.t[cur];
        case ARR_VT: return d.vt;
        case ARR_CHH: return d.chh;
        case ARR_TQ: return d.tq;
        case ARR_CP: return d.cp;
        default: return d.lad;
    }
}

// the packed states (first, second) of entry x of a pair list (pp pairs for
// AM_GPAIR, cross-channel members (particle, hole) for AM_GVBAR)
__device__ __forceinline__ int2 nm_pair_states(const NmDev& d, int amode, int list, int x) {
    const int32_t P = amode == AM_GPAIR ? d.pp[list + x] : d.mem[list + x];
    return make_int2(d.st[pr_a(P)], d.st[pr_b(P)]);
}

// element (m, k) of a generated A operand from the staged pair states:
// AM_GPAIR <ab||cd> with row (a, b), column (c, d); AM_GVBAR <kl||cd> with row
// x = (c, k) of P and column m = (d, l) of Q
__device__ __forceinline__ double nm_genA(int amode, const double* u, int nlut, int2 R, int2 C) {
    return amode == AM_GPAIR ? nm_vas(u, nlut, R.x, R.y, C.x, C.y) : nm_vas(u, nlut, R.y, C.y, R.x, C.x);
}

// K extent of a staged chunk, and each thread's share of its A (32 x kNmKC)
// and B (kNmKC x 32) entries
constexpr int kNmKC = 32;
constexpr int kNmPer = 32 * kNmKC / 256;

// this thread's A and B entries of the chunk at k0 (array operands; zero
// outside the block); generated A entries are made when staged
__device__ __forceinline__ void nm_fetch(const NmSeg& S, const NmJob& J, const double* A, const double* B, int m0,
                                         int n0, int k0, double* ra, double* rb) {
#pragma unroll
    for (int h = 0; h < kNmPer; h++) {
        const int q = threadIdx.x + 256 * h;
        const int am = q / kNmKC, ak = q % kNmKC, m = m0 + am, kk = k0 + ak;
        ra[h] = 0.0;
        if (m < J.M && kk < S.K) {
            if (S.amode == AM_ROW) ra[h] = A[S.a_off + (int64_t)m * S.lda + kk];
            else if (S.amode == AM_COL) ra[h] = A[S.a_off + (int64_t)kk * S.lda + m];
        }
        const int bk = q >> 5, bn = q & 31, kb = k0 + bk, n = n0 + bn;
        rb[h] = (kb < S.K && n < J.N) ? B[S.b_off + (int64_t)kb * S.ldb + n] : 0.0;
    }
}

// One 32 x 32 output tile of one job per workgroup, four waves of 16 x 16;
// K in chunks of kNmKC staged in LDS, kNmKC / 4 FP64 16x16x4 MFMA steps per chunk;
// the array operands of chunk c + 1 are loaded into registers before chunk c
// is multiplied.
// Lane l of a wave supplies A[l%16][l/16], B[l/16][l%16] and receives
// D[l/16 + 4r][l%16].
__global__ void __launch_bounds__(256) k_nm_gemm(NmDev d, int cur, uint32_t mask, int tile0, int n_tiles) {
    __shared__ double u[4 * (4 * kNmMaxNmax2 + 1)];
    __shared__ double sA[32][kNmKC + 1];
    __shared__ double sB[kNmKC][33];
    __shared__ int2 rst[32], cst[kNmKC];  // pair states of a generated A operand: tile rows, chunk columns
    for (int k = threadIdx.x; k < 4 * d.nlut; k += 256) u[k] = d.u[k];
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wm = w >> 1, wn = w & 1;
    for (int ti = blockIdx.x; ti < n_tiles; ti += gridDim.x) {
        const NmTile T = d.tiles[tile0 + ti];
        // the job is read through a reference to the list: a local copy of it,
        // whose segment array is indexed at run time, would live in scratch
        const NmJob& J = d.jobs[T.job];
        const int m0 = T.tm * 32, n0 = T.tn * 32;
        nm_d4 acc = {0.0, 0.0, 0.0, 0.0};
        for (int sg = 0; sg < J.nseg; sg++) {
            const NmSeg S = J.seg[sg];
            if (!(mask & (uint32_t)S.term)) continue;
            const double* A = nm_arr(d, S.a_arr, cur);
            const double* B = nm_arr(d, S.b_arr, cur);
            const bool gen = S.amode == AM_GPAIR || S.amode == AM_GVBAR;
            double ra[kNmPer], rb[kNmPer];
            nm_fetch(S, J, A, B, m0, n0, 0, ra, rb);
            for (int k0 = 0; k0 < S.K; k0 += kNmKC) {
                __syncthreads();  // the previous chunk's reads are done
                if (gen) {
                    if (k0 == 0 && threadIdx.x < 32 && m0 + (int)threadIdx.x < J.M)
                        rst[threadIdx.x] = nm_pair_states(d, S.amode, S.a_rows, m0 + threadIdx.x);
                    if (threadIdx.x >= 64 && threadIdx.x < 64 + kNmKC && k0 + (int)threadIdx.x - 64 < S.K)
                        cst[threadIdx.x - 64] = nm_pair_states(d, S.amode, S.a_cols, k0 + threadIdx.x - 64);
                    __syncthreads();
                }
#pragma unroll
                for (int h = 0; h < kNmPer; h++) {
                    const int q = threadIdx.x + 256 * h;
                    const int am = q / kNmKC, ak = q % kNmKC;
                    double av = ra[h];
                    if (gen) av = (m0 + am < J.M && k0 + ak < S.K) ? nm_genA(S.amode, u, d.nlut, rst[am], cst[ak]) : 0.0;
                    sA[am][ak] = S.alpha * av;
                    sB[q >> 5][q & 31] = rb[h];
                }
                __syncthreads();
                if (k0 + kNmKC < S.K) nm_fetch(S, J, A, B, m0, n0, k0 + kNmKC, ra, rb);
#pragma unroll
                for (int s = 0; s < kNmKC / 4; s++) {
                    const double a = sA[wm * 16 + (lane & 15)][4 * s + (lane >> 4)];
                    const double b = sB[4 * s + (lane >> 4)][wn * 16 + (lane & 15)];
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
                }
            }
        }
        const bool cinit = J.cmode != CM_NONE && (mask & (uint32_t)J.cterm);
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int m = m0 + wm * 16 + (lane >> 4) + 4 * r, n = n0 + wn * 16 + (lane & 15);
            if (m >= J.M || n >= J.N) continue;
            double v = acc[r];
            if (cinit) {
                if (J.cmode == CM_GPAIR) {
                    const int32_t R = d.hh[J.c_rows + m], C = d.hh[J.c_cols + n];
                    v += nm_vas(u, d.nlut, d.st[pr_a(R)], d.st[pr_b(R)], d.st[pr_a(C)], d.st[pr_b(C)]);
                } else {  // <kb||cj>, x = (c, k) row member, y = (b, j) column member
                    const int32_t X = d.mem[J.c_rows + m], Y = d.mem[J.c_cols + n];
                    v += nm_vas(u, d.nlut, d.st[pr_b(X)], d.st[pr_a(Y)], d.st[pr_a(X)], d.st[pr_b(Y)]);
                }
            }
            if (J.omode == OM_ROW) {
                nm_arr(d, J.o_arr, cur)[J.o_off + (int64_t)m * J.ldo + n] = v;
            } else if (J.omode == OM_ROW_ADD) {
                double* o = nm_arr(d, J.o_arr, cur) + J.o_off + (int64_t)m * J.ldo + n;
                *o = *o + v;
            } else {
                const int32_t z = d.pmap[J.o_off + (int64_t)m * J.ldo + n];
                if (z >= 0) d.ring[4 * (int64_t)(z >> 3) + ((z >> 1) & 3)] = (z & 1) ? -v : v;
            }
        }
    }
}


// pp ladder over momentum pairs.  In a direct channel (K, S_z, T_z) the element
// <ab||cd> = +-(U_k(|n_a - n_c|^2) + U_k(|n_a - n_d|^2)) depends on the row only
// through n_a and the labels of a and b, on the column through its momenta
// {n_c, n_d} and labels, and its table k and sign only on the four labels.
// The rows of a momentum pair P = {p, K - p} (the first state at p) are its
// label pairs; with the channel's labels sorted into pairs (X_j, Y_j) whose
// columns enter every row with the same table and opposite signs,
//   sum_{c<d} <ab||cd> t_ij^cd = sum_j c_(ab, j) u_(k(ab, j), j)(n_a),
//   u_(k, j)(p') = sum_P M_k[p'][P] delta_j(P),  M_k[p'][P] = U_k(|p' - p|^2) + U_k(|p' - q|^2),
//   delta_j(P) = t(P, X_j) - t(P, Y_j),
// a square product over the momentum pairs per (class, difference): one for
// the S_z = 0 blocks of like particles and the |S_z| = 1 blocks of unlike ones
// (n_lp^2 n_hh multiply-adds against the 4 n_lp^2 n_hh of the product over
// label pairs), four for the S_z = T_z = 0 blocks (against 16 n_lp^2 n_hh),
// none for |S_z| = |T_z| = 1, where the element vanishes.  M_k is generated per lane with the
// offsets of the neutron ladder (one sdot4 and three integer ops), the
// differences are formed when a chunk of kNmKP pairs is staged, and each row
// takes its combination of the products.  A wave holds one 16-row tile; the
// 16-column tile is cut into NG groups of four for the 4x4x4 FP64 MFMA.
constexpr int kNmKP = 128;       // column momentum pairs staged per chunk
constexpr int kNmLadRows = 64;   // row momentum pairs per work item
__device__ __forceinline__ double nm_mfma4(double a, double b, double c) {
    return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}
template <int NG, int ND, int NK>
__device__ __forceinline__ void nm_ladpp_item(const NmDev& d, const NmLadD& L, const NmChanD& C, int cur, int r0,
                                              int ct, bool pp_on, const double* lutS, double* tks,
                                              int4 (*cvi)[kNmKP], int (*cvj)[kNmKP], int4* prs) {
    constexpr int S = 8;  // bytes per table entry
    constexpr int NA = ND * NK == 1 ? 2 : 1;  // independent accumulators per product
    const char* lutB = (const char*)lutS;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nhh = C.nhh, nlp = L.n_lp;
    const double* tcur = d.t[cur] + C.t_off;
    const int4* lp = d.ladlp + 2 * (int64_t)L.lp_off;
    const int rbase = r0 + 16 * w;
    const int bj = lane & 3;
    const int orow4 = 4 * ((lane & 15) >> 2) + (lane >> 4);
    int tb[2] = {0, 0};  // byte offsets of the classes' tables
#pragma unroll
    for (int c = 0; c < NK; c++) tb[c] = L.tab[c] * d.nlut * S;
    const int32_t kpack = (int32_t)((uint32_t)(uint8_t)(int8_t)L.kx | ((uint32_t)(uint8_t)(int8_t)L.ky << 8) |
                                    ((uint32_t)(uint8_t)(int8_t)L.kz << 16));
    const int K2 = L.kx * L.kx + L.ky * L.ky + L.kz * L.kz;
    auto times4 = [](int32_t x) { return (int32_t)(((uint32_t)x << 2) & 0xfcfcfcfcu); };
    // generator row (A layout): -(S/2) p' packed, S |p'|^2, S (2 |p'|^2 - 2 p'.K)
    int32_t apack = 0;
    int rowA = 0, rowS = 0;
    {
        const int pr = rbase + (lane & 15);
        const int4 li = pr < nlp ? lp[2 * pr] : make_int4(0, 0, -1, -1);
        const int ax = (int8_t)(li.x & 0xff), ay = (int8_t)((li.x >> 8) & 0xff), az = (int8_t)((li.x >> 16) & 0xff);
        apack = (int32_t)((uint32_t)(uint8_t)(int8_t)(-4 * ax) | ((uint32_t)(uint8_t)(int8_t)(-4 * ay) << 8) |
                          ((uint32_t)(uint8_t)(int8_t)(-4 * az) << 16));
        const int A2 = li.y & 1023;
        rowA = S * A2;
        rowS = S * (2 * A2 - 2 * (ax * L.kx + ay * L.ky + az * L.kz));
    }
    // column descriptor: (4 p packed, S |p|^2, S (|p|^2 + |q|^2), X_0 + 1 | (Y_0 + 1) << 16)
    // and (X_1 + 1 | (Y_1 + 1) << 16); padding columns carry p = K, q = 0, no rows
    const int4 cpad = make_int4(times4(kpack), S * K2, S * K2, 0);
    auto cdesc = [&](const int4& li) {
        const int C2 = li.y & 1023, D2 = (li.y >> 10) & 1023;
        return make_int4(times4(li.x), S * C2, S * (C2 + D2),
                         (int)((uint32_t)(li.z + 1) | ((uint32_t)(li.w + 1) << 16)));
    };
    auto cdesc2 = [&](const int4& lj) { return (int)((uint32_t)(lj.x + 1) | ((uint32_t)(lj.y + 1) << 16)); };
    constexpr int kPer = kNmKP * 16 / 256;
    double tv[ND][kPer];
    auto load_delta = [&](int kp, int b) {
        const int kn = min(kNmKP, nlp - kp);
#pragma unroll
        for (int i = 0; i < kPer; i++) {
            const int e = threadIdx.x + 256 * i, kk = e >> 4, cc = ct * 16 + (e & 15);
            const bool in = kk < kn && cc < nhh;
#pragma unroll
            for (int j = 0; j < ND; j++) {
                const uint32_t rr = in ? (uint32_t)(j == 0 ? cvi[b][kk].w : cvj[b][kk]) : 0u;
                const int rp = (int)(rr & 0xffff) - 1, rm = (int)(rr >> 16) - 1;
                const double tp = rp >= 0 ? tcur[(int64_t)rp * nhh + cc] : 0.0;
                const double tm = rm >= 0 ? tcur[(int64_t)rm * nhh + cc] : 0.0;
                tv[j][i] = tp - tm;
            }
        }
    };
    auto store_delta = [&]() {
#pragma unroll
        for (int j = 0; j < ND; j++)
#pragma unroll
            for (int i = 0; i < kPer; i++) {
                const int e = threadIdx.x + 256 * i;
                tks[j * kNmKP * 16 + (e >> 4) * 16 + (e & 15)] = tv[j][i];
            }
    };
    double acc[NK][ND][NG][NA];
#pragma unroll
    for (int c = 0; c < NK; c++)
#pragma unroll
        for (int j = 0; j < ND; j++)
#pragma unroll
            for (int q = 0; q < NG; q++)
#pragma unroll
                for (int a = 0; a < NA; a++) acc[c][j][q][a] = 0.0;
    int4 lpc = cpad, lpd = make_int4(-1, -1, 0, 0);
    if (pp_on && threadIdx.x < kNmKP && threadIdx.x < nlp) { lpc = lp[2 * threadIdx.x]; lpd = lp[2 * threadIdx.x + 1]; }
    const int4 myr = (threadIdx.x < kNmLadRows && r0 + threadIdx.x < nlp)
                         ? make_int4(lp[2 * (r0 + threadIdx.x)].z, lp[2 * (r0 + threadIdx.x)].w,
                                     lp[2 * (r0 + threadIdx.x) + 1].x, lp[2 * (r0 + threadIdx.x) + 1].y)
                         : make_int4(-1, -1, -1, -1);
    __syncthreads();  // the previous item's reads of LDS are done
    if (threadIdx.x < kNmLadRows) prs[threadIdx.x] = myr;
    if (pp_on) {
        if (threadIdx.x < kNmKP) {
            cvi[0][threadIdx.x] = threadIdx.x < nlp ? cdesc(lpc) : cpad;
            cvj[0][threadIdx.x] = threadIdx.x < nlp ? cdesc2(lpd) : 0;
        }
        lpc = cpad; lpd = make_int4(-1, -1, 0, 0);
        if (threadIdx.x < kNmKP && kNmKP + threadIdx.x < nlp) {
            lpc = lp[2 * (kNmKP + threadIdx.x)];
            lpd = lp[2 * (kNmKP + threadIdx.x) + 1];
        }
    }
    __syncthreads();
    if (pp_on) {
        load_delta(0, 0);
        store_delta();
        for (int kp = 0; kp < nlp; kp += kNmKP) {
            const int b = (kp / kNmKP) & 1;
            const bool more = kp + kNmKP < nlp;
            if (more && threadIdx.x < kNmKP) {
                const bool in = kp + kNmKP + threadIdx.x < nlp;
                cvi[b ^ 1][threadIdx.x] = in ? cdesc(lpc) : cpad;
                cvj[b ^ 1][threadIdx.x] = in ? cdesc2(lpd) : 0;
                lpc = cpad; lpd = make_int4(-1, -1, 0, 0);
                if (kp + 2 * kNmKP + threadIdx.x < nlp) {
                    lpc = lp[2 * (kp + 2 * kNmKP + threadIdx.x)];
                    lpd = lp[2 * (kp + 2 * kNmKP + threadIdx.x) + 1];
                }
            }
            __syncthreads();  // this chunk's differences and the next chunk's descriptors are in LDS
            if (more) load_delta(kp + kNmKP, b ^ 1);
            const int kn = min(kNmKP, nlp - kp);
            const int ksteps = (kn + 15) & ~15;
            for (int kk = 0; kk < ksteps; kk += 16) {
#pragma unroll
                for (int s2 = 0; s2 < 4; s2++) {
                    const int kc = kk + 4 * s2 + (lane >> 4);
                    const int4 ci = cvi[b][kc];
                    const int o1 = __builtin_amdgcn_sdot4(apack, ci.x, rowA + ci.y, false);
                    const int o2 = rowS + ci.z - o1;
                    double va[NK];
#pragma unroll
                    for (int c = 0; c < NK; c++)
                        va[c] = *(const double*)(lutB + tb[c] + o1) + *(const double*)(lutB + tb[c] + o2);
#pragma unroll
                    for (int j = 0; j < ND; j++)
#pragma unroll
                        for (int q = 0; q < NG; q++) {
                            const double vb = tks[j * kNmKP * 16 + kc * 16 + 4 * q + bj];
#pragma unroll
                            for (int c = 0; c < NK; c++)
                                acc[c][j][q][s2 % NA] = nm_mfma4(va[c], vb, acc[c][j][q][s2 % NA]);
                        }
                }
            }
            __syncthreads();  // every wave is done with this chunk
            if (more) store_delta();
        }
    }
    // the four rows of the lane's output pair, each with its combination
    const int4 ro = prs[16 * w + orow4];
    const int rows[4] = {ro.x, ro.y, ro.z, ro.w};
    double* lad = d.lad + C.t_off;
#pragma unroll
    for (int r = 0; r < 4; r++) {
        if (rows[r] < 0) continue;
        const int rc = L.rec[r];
#pragma unroll
        for (int q = 0; q < NG; q++) {
            const int cc = ct * 16 + 4 * q + bj;
            if (cc >= nhh) continue;
            double v = 0.0;
#pragma unroll
            for (int j = 0; j < ND; j++) {
                const int cf = (rc >> (3 * j)) & 3, cl = (rc >> (3 * j + 2)) & 1;
                double u = 0.0;
#pragma unroll
                for (int c = 0; c < NK; c++)
                    if (c == cl) {
#pragma unroll
                        for (int a = 0; a < NA; a++) u += acc[c][j][q][a];
                    }
                if (cf == 1) v += u;
                else if (cf == 2) v -= u;
            }
            lad[(int64_t)rows[r] * nhh + cc] = pp_on ? v : 0.0;
        }
    }
}

template <int ND, int NK>
__device__ __forceinline__ void nm_ladpp_ng(const NmDev& d, const NmLadD& L, const NmChanD& C, int cur, int r0,
                                            int ct, bool pp_on, double* lutS, double* tks, int4 (*cvi)[kNmKP],
                                            int (*cvj)[kNmKP], int4* prs) {
    const int ng = min(4, (min(16, C.nhh - 16 * ct) + 3) >> 2);
    switch (ng) {
        case 1: nm_ladpp_item<1, ND, NK>(d, L, C, cur, r0, ct, pp_on, lutS, tks, cvi, cvj, prs); break;
        case 2: nm_ladpp_item<2, ND, NK>(d, L, C, cur, r0, ct, pp_on, lutS, tks, cvi, cvj, prs); break;
        case 3: nm_ladpp_item<3, ND, NK>(d, L, C, cur, r0, ct, pp_on, lutS, tks, cvi, cvj, prs); break;
        default: nm_ladpp_item<4, ND, NK>(d, L, C, cur, r0, ct, pp_on, lutS, tks, cvi, cvj, prs); break;
    }
}

// one work item (channel, 64 row momentum pairs, 16 columns) per workgroup
// iteration; the four class tables are staged once per workgroup
__global__ void __launch_bounds__(256, 2) k_nm_ladpp(NmDev d, int cur, uint32_t mask, int n_items) {
    __shared__ double lutS[4 * (4 * kNmMaxNmax2 + 1)];
    __shared__ __attribute__((aligned(16))) double tks[2 * kNmKP * 16];
    __shared__ int4 cvi[2][kNmKP];
    __shared__ int cvj[2][kNmKP];
    __shared__ int4 prs[kNmLadRows];
    for (int k = threadIdx.x; k < 4 * d.nlut; k += 256) lutS[k] = d.u[k];
    const bool pp = (mask & CCD_T_PP) != 0;
    for (int bi = blockIdx.x; bi < n_items; bi += gridDim.x) {
        const NmLadItem it = d.ladit[bi];
        const NmLadD& L = d.ladd[it.lad];
        const NmChanD C = d.ch[L.chan];
        const int r0 = it.start & 0xfffff, ct = it.start >> 20;
        if (L.nd == 2 && L.nk == 2) nm_ladpp_ng<2, 2>(d, L, C, cur, r0, ct, pp, lutS, tks, cvi, cvj, prs);
        else if (L.nd == 2 && L.nk == 1) nm_ladpp_ng<2, 1>(d, L, C, cur, r0, ct, pp, lutS, tks, cvi, cvj, prs);
        else if (L.nd == 1 && L.nk == 2) nm_ladpp_ng<1, 2>(d, L, C, cur, r0, ct, pp, lutS, tks, cvi, cvj, prs);
        else if (L.nd == 1) nm_ladpp_ng<1, 1>(d, L, C, cur, r0, ct, pp, lutS, tks, cvi, cvj, prs);
        else nm_ladpp_ng<1, 1>(d, L, C, cur, r0, ct, false, lutS, tks, cvi, cvj, prs);  // no element: zeros
    }
}

// R = <ab||ij> + ladder sums + ring slots + (dchi_a + dchi_b - dchi_i - dchi_j) t,
// t_new = R / eps_ij^ab, t <- alpha t_new + (1 - alpha) t, energy parts
__global__ void __launch_bounds__(256) k_nm_update(NmDev d, int cur, double alpha, uint32_t mask) {
    __shared__ double sh[4];
    const double* t = d.t[cur];
    double* tn = d.t[cur ^ 1];
    const bool lad = (mask & (CCD_T_PP | CCD_T_HH | CCD_T_QHH)) != 0;
    const bool rng = (mask & (CCD_T_RING | CCD_T_QRING)) != 0;
    for (int w = blockIdx.x; w < d.n_items; w += gridDim.x) {
        const NmItem it = d.items[w];
        const NmChanD C = d.ch[it.chan];
        const int64_t n = (int64_t)C.nhh * C.npp;
        double acc = 0.0;
        for (int k = threadIdx.x; k < kNmChunk; k += 256) {
            const int64_t e = (int64_t)it.start + k;
            if (e >= n) continue;
            const int r = (int)(e / C.nhh), c = (int)(e - (int64_t)r * C.nhh);
            const int32_t P = d.pp[C.pp_off + r], H = d.hh[C.hh_off + c];
            const int a = pr_a(P), b = pr_b(P), i = pr_a(H), j = pr_b(H);
            const int64_t g = C.t_off + e;
            const double told = t[g], v = d.vt[g];
            double R = v;
            if (lad) R += d.lad[g];
            if (rng) {
                const double* z = d.ring + 4 * g;
                R += (z[0] + z[1]) + (z[2] + z[3]);
            }
            R += ((d.dchi[a] + d.dchi[b]) - (d.dchi[i] + d.dchi[j])) * told;
            const double den = d.eps[i] + d.eps[j] - d.eps[a] - d.eps[b];
            const double x = alpha * (R / den) + (1.0 - alpha) * told;
            tn[g] = x;
            acc += v * x;
        }
        acc = nm_block_sum(acc, sh);
        if (threadIdx.x == 0) d.epart[w] = acc;
    }
}

// ---------------------------------------------------------------------------
// host plan
// ---------------------------------------------------------------------------
struct HChan {
    int Kx, Ky, Kz, Sz, Tz;
    std::vector<int32_t> hh, pp;
    int64_t t_off = 0;
    int hh_off = 0, pp_off = 0;
    int64_t chh_off = 0;
};

struct HPh {
    int Qx, Qy, Qz, sig, tau;
    std::vector<int32_t> mem;  // (p | h << 16)
    int partner = -1, mem_off = 0;
    int64_t tq_off = -1, cp_off = -1;  // T~_Q block [n][n_P], C_P block [n_P][n_P]
};

inline size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

// kernel families of a sweep, for per-launch timing
enum { NF_GATHER = 0, NF_ROWCOL, NF_DCHI, NF_GEMM1, NF_GEMM2, NF_UPDATE, NF_ENERGY, NF_LADPP, NF_NUM };
const char* const kNmFamily[NF_NUM] = {"gather", "rowcol", "dchi", "gemm_chi", "gemm_ladder_ring", "update", "energy",
                                       "ladder_pp"};

struct ccd_nm_ctx {
    ccd_nm_problem par;
    bool timing = false;
    double fam_ms[NF_NUM] = {0};
    int64_t fam_n[NF_NUM] = {0};
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;  // (family, events)
    hipStream_t stream = nullptr;
    int ns = 0, nh = 0, nlut = 0;
    double L = 0.0, eref = 0.0, emp2 = 0.0, ecorr = 0.0, last_ms = 0.0;
    std::vector<int> nx, ny, nz, sz, tz;
    std::vector<int32_t> st;
    std::vector<double> tkin, eps, u;
    std::vector<HChan> ch;
    std::vector<HPh> ph;
    std::vector<int32_t> hh_all, pp_all, mem_all, pmap, csr_ptr, csr_idx, row_chan;
    std::vector<NmChanD> chd;
    std::vector<NmItem> items;
    std::vector<NmRcItem> rcit;
    int64_t n_cpart = 0;
    std::vector<NmJob> jobs;
    std::vector<NmTile> tiles;
    int tiles_a = 0, tiles_b = 0;  // tiles of the first launch, then of the second
    int64_t n_amp = 0, n_chh = 0, n_tq = 0, n_cp = 0;
    int n_rows = 0, n_cols = 0, max_hh = 0, max_pp = 0, max_ph = 0;
    double flops = 0.0, flops_a = 0.0;  // all products; those of the first launch
    double flops_lad = 0.0;             // the pp ladder over momentum pairs
    std::vector<NmLadD> ladd;           // its channels, momentum pairs and work items
    std::vector<int32_t> ladlp;
    std::vector<NmLadItem> ladit;
    // workspace
    char* ws = nullptr;
    size_t ws_bytes = 0;
    std::vector<std::pair<size_t, size_t>> region;  // offset, bytes
    NmDev dev{};
    int cur = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

namespace {

double nm_vas_host(const ccd_nm_ctx* c, int p, int q, int r, int s) {
    if (c->nx[p] + c->nx[q] != c->nx[r] + c->nx[s] || c->ny[p] + c->ny[q] != c->ny[r] + c->ny[s] ||
        c->nz[p] + c->nz[q] != c->nz[r] + c->nz[s])
        return 0.0;
    return nm_vas(c->u.data(), c->nlut, c->st[p], c->st[q], c->st[r], c->st[s]);
}

// The pp ladder of channel k over its momentum pairs (k_nm_ladpp): the pairs
// of its rows (keyed by the momentum of the first state), the pairing of its
// label pairs into differences and each label's combination of the products.
// False when the channel's elements do not take that form; its ladder then
// stays a product over label pairs.  Every row's elements against a sample of
// columns are checked against the element itself.
bool nm_ladpp_channel(const ccd_nm_ctx* c, int k, NmLadD& L, std::vector<int32_t>& lp) {
    const HChan& h = c->ch[k];
    const int npp = (int)h.pp.size();
    if (npp >= 0xffff) return false;
    std::vector<int> labs;
    std::map<std::tuple<int, int, int>, int> pidx;
    std::vector<std::vector<std::pair<int, int>>> prl;  // per momentum pair: (label pair, row)
    std::vector<std::array<int, 2>> pst;                // per momentum pair: its first row's states
    for (int r = 0; r < npp; r++) {
        const int a = pr_a(h.pp[r]), b = pr_b(h.pp[r]);
        const int lab = nm_st(c->st[a]) | (nm_st(c->st[b]) << 2);
        if (std::find(labs.begin(), labs.end(), lab) == labs.end()) labs.push_back(lab);
        auto ins = pidx.insert({{c->nx[a], c->ny[a], c->nz[a]}, (int)prl.size()});
        if (ins.second) {
            prl.emplace_back();
            pst.push_back({a, b});
        }
        prl[ins.first->second].push_back({lab, r});
    }
    const int nl = (int)labs.size();
    if (nl > 4) return false;
    std::sort(labs.begin(), labs.end());
    int tk[4][4] = {}, sg[4][4] = {};
    bool any = false;
    for (int x = 0; x < nl; x++)
        for (int y = 0; y < nl; y++) {
            int kk = 0;
            bool neg = false;
            if (nm_class(labs[x] & 3, labs[x] >> 2, labs[y] & 3, labs[y] >> 2, kk, neg)) {
                tk[x][y] = kk;
                sg[x][y] = neg ? -1 : 1;
                any = true;
            }
        }
    int slot_of[4] = {0, 1, 2, 3};
    std::memset(&L, 0, sizeof(L));
    L.chan = k;
    L.kx = h.Kx; L.ky = h.Ky; L.kz = h.Kz;
    std::vector<int> cls;
    if (any) {
        std::vector<int> X, Y;
        bool used[4] = {false, false, false, false};
        for (int x = 0; x < nl; x++) {
            if (used[x]) continue;
            int y = -1;
            for (int z = x + 1; z < nl && y < 0; z++) {
                if (used[z]) continue;
                bool ok = true;
                for (int r = 0; r < nl && ok; r++) {
                    if (sg[r][x] == 0 && sg[r][z] == 0) continue;
                    ok = sg[r][x] != 0 && sg[r][z] == -sg[r][x] && tk[r][x] == tk[r][z];
                }
                if (ok) y = z;
            }
            if (y < 0) return false;
            used[x] = used[y] = true;
            X.push_back(x);
            Y.push_back(y);
        }
        if (X.size() > 2) return false;
        for (int r = 0; r < nl; r++)
            for (size_t j = 0; j < X.size(); j++)
                if (sg[r][X[j]] != 0 && std::find(cls.begin(), cls.end(), tk[r][X[j]]) == cls.end())
                    cls.push_back(tk[r][X[j]]);
        if (cls.empty() || cls.size() > 2) return false;
        L.nd = (int)X.size();
        L.nk = (int)cls.size();
        for (int q = 0; q < L.nk; q++) L.tab[q] = cls[q];
        for (size_t j = 0; j < X.size(); j++) {
            slot_of[X[j]] = 2 * (int)j;
            slot_of[Y[j]] = 2 * (int)j + 1;
        }
        for (int r = 0; r < nl; r++) {
            int rc = 0;
            for (size_t j = 0; j < X.size(); j++) {
                const int sgn = sg[r][X[j]];
                if (sgn == 0) continue;
                const int ci = (int)(std::find(cls.begin(), cls.end(), tk[r][X[j]]) - cls.begin());
                rc |= ((sgn > 0 ? 1 : 2) | (ci << 2)) << (3 * j);
            }
            L.rec[slot_of[r]] = rc;
        }
    }
    // the rows' elements against a sample of columns, from the recipe
    const int step = std::max(1, npp / 16);
    for (int r = 0; r < npp; r++) {
        const int a = pr_a(h.pp[r]), b = pr_b(h.pp[r]);
        const int lr = (int)(std::find(labs.begin(), labs.end(), nm_st(c->st[a]) | (nm_st(c->st[b]) << 2)) -
                             labs.begin());
        for (int q = 0; q < npp; q += step) {
            const int cc = pr_a(h.pp[q]), dd = pr_b(h.pp[q]);
            const int lq = (int)(std::find(labs.begin(), labs.end(), nm_st(c->st[cc]) | (nm_st(c->st[dd]) << 2)) -
                                 labs.begin());
            double want = 0.0;
            if (L.nd > 0) {
                const int sl = slot_of[lq], j = sl >> 1, rc = (L.rec[slot_of[lr]] >> (3 * j)) & 7;
                const int cf = rc & 3;
                if (cf != 0) {
                    const int kk = L.tab[(rc >> 2) & 1];
                    const auto d2 = [&](int x, int y) {
                        const int dx = c->nx[x] - c->nx[y], dy = c->ny[x] - c->ny[y], dz = c->nz[x] - c->nz[y];
                        return dx * dx + dy * dy + dz * dz;
                    };
                    const double m = c->u[kk * c->nlut + d2(a, cc)] + c->u[kk * c->nlut + d2(a, dd)];
                    want = ((cf == 1) == ((sl & 1) == 0)) ? m : -m;
                }
            }
            const double got = nm_vas_host(c, a, b, cc, dd);
            if (std::fabs(got - want) > 1e-12 * (std::fabs(got) + 1e-300) && got != want) return false;
        }
    }
    // momentum pairs: (p packed, |p|^2 | |q|^2 << 10, slot rows 0 and 1), (slot rows 2 and 3, 0, 0)
    L.lp_off = (int)(lp.size() / 8);
    L.n_lp = (int)prl.size();
    for (size_t P = 0; P < prl.size(); P++) {
        const int a = pst[P][0], b = pst[P][1];
        int rows[4] = {-1, -1, -1, -1};
        for (auto& e : prl[P]) {
            const int li = (int)(std::find(labs.begin(), labs.end(), e.first) - labs.begin());
            rows[slot_of[li]] = e.second;
        }
        const int p2 = c->nx[a] * c->nx[a] + c->ny[a] * c->ny[a] + c->nz[a] * c->nz[a];
        const int q2 = c->nx[b] * c->nx[b] + c->ny[b] * c->ny[b] + c->nz[b] * c->nz[b];
        const int32_t pk = (int32_t)((uint32_t)(uint8_t)(int8_t)c->nx[a] | ((uint32_t)(uint8_t)(int8_t)c->ny[a] << 8) |
                                     ((uint32_t)(uint8_t)(int8_t)c->nz[a] << 16));
        const int32_t e[8] = {pk, p2 | (q2 << 10), rows[0], rows[1], rows[2], rows[3], 0, 0};
        lp.insert(lp.end(), e, e + 8);
    }
    return true;
}

ccd_status nm_plan(ccd_nm_ctx* c) {
    const ccd_nm_problem& P = c->par;
    if (P.species != 1 && P.species != 2) {
        ccd::set_error("ccd_nm_build: species must be 1 (neutrons) or 2 (protons and neutrons)");
        return CCD_EINVAL;
    }
    if (P.nmax2 < 0 || P.nmax2 > kNmMaxNmax2 || !(P.density > 0.0) || !(P.hbar2_over_m > 0.0) ||
        !(P.kappa_R > 0.0) || !(P.kappa_T > 0.0) || !(P.kappa_S > 0.0) || P.n_nucleons <= 0) {
        ccd::set_error("ccd_nm_build: need 0 <= nmax2 <= 64, positive density, hbar^2/m, kappas and A");
        return CCD_EINVAL;
    }
    // model space: shell, n_x, n_y, n_z, s_z, t_z (innermost)
    int R = 0;
    while ((R + 1) * (R + 1) <= P.nmax2) R++;
    for (int shell = 0; shell <= P.nmax2; shell++)
        for (int x = -R; x <= R; x++)
            for (int y = -R; y <= R; y++)
                for (int z = -R; z <= R; z++)
                    for (int s = -1; s <= 1; s += 2)
                        for (int t = (P.species == 2 ? -1 : 1); t <= 1; t += 2)
                            if (x * x + y * y + z * z == shell) {
                                c->nx.push_back(x); c->ny.push_back(y); c->nz.push_back(z);
                                c->sz.push_back(s); c->tz.push_back(t);
                                c->st.push_back(nm_pack(x, y, z, s, t));
                            }
    c->ns = (int)c->st.size();
    c->nh = P.n_nucleons;
    const int A = c->nh;
    auto shell_of = [&](int p) { return c->nx[p] * c->nx[p] + c->ny[p] * c->ny[p] + c->nz[p] * c->nz[p]; };
    if (A >= c->ns || shell_of(A - 1) == shell_of(A)) {
        ccd::set_error("ccd_nm_build: A = " + std::to_string(A) + " does not close a shell of the basis "
                       "or leaves no particle states");
        return CCD_ENOTMAGIC;
    }
    if (c->ns >= 65536) {
        ccd::set_error("ccd_nm_build: more than 65535 states");
        return CCD_EINVAL;
    }
    c->L = std::cbrt((double)A / P.density);
    const double k0 = 2.0 * M_PI / c->L;
    c->tkin.resize(c->ns);
    for (int p = 0; p < c->ns; p++) c->tkin[p] = 0.5 * P.hbar2_over_m * k0 * k0 * (double)shell_of(p);
    // element tables: W_a(m) = V_a / L^3 (pi / kappa_a)^{3/2} exp(-(2 pi / L)^2 m / (4 kappa_a))
    c->nlut = 4 * P.nmax2 + 1;
    const double L3 = c->L * c->L * c->L;
    std::vector<double> W[3];
    const double V[3] = {P.V_R, P.V_T, P.V_S}, K[3] = {P.kappa_R, P.kappa_T, P.kappa_S};
    for (int a = 0; a < 3; a++) {
        W[a].resize(c->nlut);
        for (int m = 0; m < c->nlut; m++)
            W[a][m] = V[a] / L3 * std::pow(M_PI / K[a], 1.5) * std::exp(-k0 * k0 * (double)m / (4.0 * K[a]));
    }
    c->u.resize(4 * (size_t)c->nlut);
    for (int m = 0; m < c->nlut; m++) {
        c->u[0 * c->nlut + m] = 0.5 * W[0][m] + 0.5 * W[2][m];
        c->u[1 * c->nlut + m] = 0.5 * W[0][m] + 0.5 * W[1][m];
        c->u[2 * c->nlut + m] = 0.5 * W[0][m] + 0.25 * W[1][m] + 0.25 * W[2][m];
        c->u[3 * c->nlut + m] = 0.25 * W[1][m] - 0.25 * W[2][m];
    }
    // Fock energies and E_ref
    c->eps.resize(c->ns);
    for (int p = 0; p < c->ns; p++) {
        double s = c->tkin[p];
        for (int i = 0; i < A; i++) s += nm_vas_host(c, p, i, p, i);
        c->eps[p] = s;
    }
    for (int i = 0; i < A; i++)
        for (int a = A; a < c->ns; a++)
            if (!(c->eps[i] < c->eps[a])) {
                ccd::set_error("ccd_nm_build: a hole lies at or above a particle in Fock energy");
                return CCD_EINVAL;
            }
    {
        double e = 0.0, v = 0.0;
        for (int i = 0; i < A; i++) e += c->tkin[i];
        for (int i = 0; i < A; i++)
            for (int j = 0; j < A; j++) v += nm_vas_host(c, i, j, i, j);
        c->eref = e + 0.5 * v;
    }
    // direct channels (K, S_z, T_z)
    typedef std::tuple<int, int, int, int, int> Key;  // T_z, S_z, K_x, K_y, K_z
    std::map<Key, int> idx;
    std::vector<HChan> all;
    auto key_of = [&](int p, int q) {
        return Key(c->tz[p] + c->tz[q], c->sz[p] + c->sz[q], c->nx[p] + c->nx[q], c->ny[p] + c->ny[q],
                   c->nz[p] + c->nz[q]);
    };
    auto chan_of = [&](const Key& k) {
        auto f = idx.find(k);
        if (f != idx.end()) return f->second;
        HChan h;
        h.Tz = std::get<0>(k); h.Sz = std::get<1>(k);
        h.Kx = std::get<2>(k); h.Ky = std::get<3>(k); h.Kz = std::get<4>(k);
        all.push_back(h);
        idx[k] = (int)all.size() - 1;
        return (int)all.size() - 1;
    };
    for (int i = 0; i < A; i++)
        for (int j = i + 1; j < A; j++) all[chan_of(key_of(i, j))].hh.push_back((int32_t)(i | (j << 16)));
    for (int a = A; a < c->ns; a++)
        for (int b = a + 1; b < c->ns; b++) {
            auto f = idx.find(key_of(a, b));
            if (f != idx.end()) all[f->second].pp.push_back((int32_t)(a | (b << 16)));
        }
    // keep channels with both kinds of pairs, in key order
    std::map<Key, int> kept_idx;
    for (auto& kv : idx) {
        HChan& h = all[kv.second];
        if (h.hh.empty() || h.pp.empty()) continue;
        kept_idx[kv.first] = (int)c->ch.size();
        c->ch.push_back(h);
    }
    // pair -> (channel, position)
    std::map<int32_t, std::pair<int, int>> hpos, ppos;
    int64_t toff = 0, choff = 0;
    for (size_t k = 0; k < c->ch.size(); k++) {
        HChan& h = c->ch[k];
        h.t_off = toff;
        h.chh_off = choff;
        h.hh_off = (int)c->hh_all.size();
        h.pp_off = (int)c->pp_all.size();
        for (size_t x = 0; x < h.hh.size(); x++) {
            hpos[h.hh[x]] = {(int)k, (int)x};
            c->hh_all.push_back(h.hh[x]);
        }
        for (size_t x = 0; x < h.pp.size(); x++) {
            ppos[h.pp[x]] = {(int)k, (int)x};
            c->pp_all.push_back(h.pp[x]);
        }
        toff += (int64_t)h.hh.size() * h.pp.size();
        choff += (int64_t)h.hh.size() * h.hh.size();
        c->max_hh = std::max(c->max_hh, (int)h.hh.size());
        c->max_pp = std::max(c->max_pp, (int)h.pp.size());
        NmChanD d;
        d.t_off = h.t_off;
        d.nhh = (int)h.hh.size();
        d.npp = (int)h.pp.size();
        d.hh_off = h.hh_off;
        d.pp_off = h.pp_off;
        d.chh_off = (int32_t)h.chh_off;
        d.rc_lo = (int32_t)c->rcit.size();
        {
            const int R = std::max(1, kNmChunk / d.nhh);
            for (int r0 = 0; r0 < d.npp; r0 += R) {
                const int nr = std::min(R, d.npp - r0);
                c->rcit.push_back({(int32_t)k, r0, nr, (int32_t)c->n_cpart});
                c->n_cpart += d.nhh;
            }
        }
        d.rc_n = (int32_t)c->rcit.size() - d.rc_lo;
        c->chd.push_back(d);
        for (int64_t s0 = 0; s0 < (int64_t)d.nhh * d.npp; s0 += kNmChunk) c->items.push_back({(int32_t)k, (int32_t)s0});
    }
    c->n_amp = toff;
    c->n_chh = choff;
    c->n_rows = (int)c->pp_all.size();
    c->n_cols = (int)c->hh_all.size();
    if (c->n_amp == 0 || c->n_amp >= ((int64_t)1 << 28)) {
        ccd::set_error("ccd_nm_build: no amplitudes, or more than 2^28");
        return CCD_EINVAL;
    }
    c->row_chan.resize(c->n_rows + c->n_cols);
    for (size_t k = 0; k < c->ch.size(); k++) {
        for (int x = 0; x < c->chd[k].npp; x++) c->row_chan[c->chd[k].pp_off + x] = (int32_t)k;
        for (int x = 0; x < c->chd[k].nhh; x++) c->row_chan[c->n_rows + c->chd[k].hh_off + x] = (int32_t)k;
    }
    // one-body CSR: rows holding each particle, columns holding each hole
    {
        std::vector<std::vector<int32_t>> lists(c->ns);
        for (int r = 0; r < c->n_rows; r++) {
            lists[pr_a(c->pp_all[r])].push_back(r);
            lists[pr_b(c->pp_all[r])].push_back(r);
        }
        for (int q = 0; q < c->n_cols; q++) {
            lists[pr_a(c->hh_all[q])].push_back(q);
            lists[pr_b(c->hh_all[q])].push_back(q);
        }
        c->csr_ptr.assign(1, 0);
        for (int s = 0; s < c->ns; s++) {
            for (int32_t x : lists[s]) c->csr_idx.push_back(x);
            c->csr_ptr.push_back((int32_t)c->csr_idx.size());
        }
    }
    // cross channels (Q, sigma, tau): members (particle p, hole h)
    std::map<Key, int> pidx;
    for (int p = A; p < c->ns; p++)
        for (int h = 0; h < A; h++) {
            Key k(c->tz[p] - c->tz[h], c->sz[p] - c->sz[h], c->nx[p] - c->nx[h], c->ny[p] - c->ny[h],
                  c->nz[p] - c->nz[h]);
            auto f = pidx.find(k);
            int id;
            if (f == pidx.end()) {
                HPh q;
                q.tau = std::get<0>(k); q.sig = std::get<1>(k);
                q.Qx = std::get<2>(k); q.Qy = std::get<3>(k); q.Qz = std::get<4>(k);
                c->ph.push_back(q);
                id = (int)c->ph.size() - 1;
                pidx[k] = id;
            } else {
                id = f->second;
            }
            c->ph[id].mem.push_back((int32_t)(p | (h << 16)));
        }
    for (auto& q : c->ph) {
        q.mem_off = (int)c->mem_all.size();
        for (int32_t m : q.mem) c->mem_all.push_back(m);
        auto f = pidx.find(Key(-q.tau, -q.sig, -q.Qx, -q.Qy, -q.Qz));
        q.partner = f == pidx.end() ? -1 : f->second;
        c->max_ph = std::max(c->max_ph, (int)q.mem.size());
    }
    // ring blocks and position maps: entry (u, y) of Q's block, (a,i) = member u
    // of Q and (b,j) = member y of its partner, names the canonical amplitude of
    // {i, j}, {a, b}: (e << 3) | (slot << 1) | negative, slot = 2 [a > b] + [i > j],
    // negative when exactly one of the two pairs is out of order; -1 when
    // i = j or a = b
    for (auto& q : c->ph) {
        if (q.partner < 0) continue;
        const HPh& P = c->ph[q.partner];
        q.tq_off = c->n_tq;
        q.cp_off = c->n_cp;
        const int nQ = (int)q.mem.size(), nP = (int)P.mem.size();
        c->n_tq += (int64_t)nQ * nP;
        c->n_cp += (int64_t)nP * nP;
        for (int u = 0; u < nQ; u++)
            for (int y = 0; y < nP; y++) {
                const int a = pr_a(q.mem[u]), i = pr_b(q.mem[u]), b = pr_a(P.mem[y]), j = pr_b(P.mem[y]);
                if (a == b || i == j) {
                    c->pmap.push_back(-1);
                    continue;
                }
                const int32_t hp = (int32_t)(std::min(i, j) | (std::max(i, j) << 16));
                const int32_t pq = (int32_t)(std::min(a, b) | (std::max(a, b) << 16));
                const auto hx = hpos.find(hp), px = ppos.find(pq);
                if (hx == hpos.end() || px == ppos.end() || hx->second.first != px->second.first) {
                    ccd::set_error("ccd_nm_build: internal error, a ring position has no amplitude");
                    return CCD_EINVAL;
                }
                const NmChanD& C = c->chd[hx->second.first];
                const int64_t e = C.t_off + (int64_t)px->second.second * C.nhh + hx->second.second;
                const int slot = 2 * (a > b) + (i > j);
                const int neg = (a > b) != (i > j);
                c->pmap.push_back((int32_t)((e << 3) | (slot << 1) | neg));
            }
    }
    // products: launch 1 (chi_klij, C_P), launch 2 (ladders, ring Z)
    auto add_tiles = [&](const NmJob& J) {
        const int jid = (int)c->jobs.size();
        c->jobs.push_back(J);
        for (int tm = 0; tm < (J.M + 31) / 32; tm++)
            for (int tn = 0; tn < (J.N + 31) / 32; tn++) c->tiles.push_back({jid, tm, tn});
    };
    auto blank = []() {
        NmJob J;
        std::memset(&J, 0, sizeof(J));
        for (auto& s : J.seg) s.alpha = 1.0;
        return J;
    };
    for (size_t k = 0; k < c->ch.size(); k++) {  // chi_klij
        const NmChanD& C = c->chd[k];
        NmJob J = blank();
        J.M = C.nhh; J.N = C.nhh; J.nseg = 1;
        J.seg[0].K = C.npp; J.seg[0].amode = AM_COL; J.seg[0].a_arr = ARR_VT; J.seg[0].a_off = C.t_off;
        J.seg[0].lda = C.nhh; J.seg[0].b_arr = ARR_T; J.seg[0].b_off = C.t_off; J.seg[0].ldb = C.nhh;
        J.seg[0].term = CCD_T_QHH;
        J.cmode = CM_GPAIR; J.cterm = CCD_T_HH; J.c_rows = C.hh_off; J.c_cols = C.hh_off;
        J.omode = OM_ROW; J.o_arr = ARR_CHH; J.o_off = C.chh_off; J.ldo = C.nhh;
        add_tiles(J);
        c->flops += 2.0 * C.nhh * C.nhh * C.npp;
    }
    for (auto& q : c->ph) {  // C_P = <kb||cj>_P + 1/2 Vbar T~_Q
        if (q.partner < 0) continue;
        const HPh& P = c->ph[q.partner];
        const int nQ = (int)q.mem.size(), nP = (int)P.mem.size();
        NmJob J = blank();
        J.M = nP; J.N = nP; J.nseg = 1;
        J.seg[0].K = nQ; J.seg[0].amode = AM_GVBAR; J.seg[0].a_rows = P.mem_off; J.seg[0].a_cols = q.mem_off;
        J.seg[0].alpha = 0.5; J.seg[0].b_arr = ARR_TQ; J.seg[0].b_off = q.tq_off; J.seg[0].ldb = nP;
        J.seg[0].term = CCD_T_QRING;
        J.cmode = CM_GVPH; J.cterm = CCD_T_RING; J.c_rows = P.mem_off; J.c_cols = P.mem_off;
        J.omode = OM_ROW; J.o_arr = ARR_CP; J.o_off = q.cp_off; J.ldo = nP;
        add_tiles(J);
        c->flops += 2.0 * nP * nP * nQ;
    }
    c->tiles_a = (int)c->tiles.size();
    c->flops_a = c->flops;
    // the pp ladder over momentum pairs where the channel's elements allow it
    std::vector<std::pair<int, NmLadItem>> lit;
    std::vector<bool> by_pairs(c->ch.size(), false);
    std::vector<int32_t> lpall;
    for (size_t k = 0; k < c->ch.size(); k++) {
        NmLadD L;
        const size_t lp0 = lpall.size();
        if (!nm_ladpp_channel(c, (int)k, L, lpall)) {
            lpall.resize(lp0);
            continue;
        }
        by_pairs[k] = true;
        const int li = (int)c->ladd.size();
        c->ladd.push_back(L);
        const NmChanD& C = c->chd[k];
        for (int r0 = 0; r0 < L.n_lp; r0 += kNmLadRows)
            for (int ct = 0; ct < (C.nhh + 15) / 16; ct++) lit.push_back({L.n_lp, NmLadItem{li, r0 | (ct << 20)}});
        c->flops_lad += 2.0 * L.nd * L.nk * (double)L.n_lp * L.n_lp * C.nhh;
    }
    // the longest items (K extent n_lp) first, so that they do not start last
    std::stable_sort(lit.begin(), lit.end(), [](const std::pair<int, NmLadItem>& x,
                                               const std::pair<int, NmLadItem>& y) { return x.first > y.first; });
    for (auto& e : lit) c->ladit.push_back(e.second);
    c->ladlp = std::move(lpall);
    for (size_t k = 0; k < c->ch.size(); k++) {  // ladders (the pp part here only without the pairs form)
        const NmChanD& C = c->chd[k];
        NmJob J = blank();
        J.M = C.npp; J.N = C.nhh; J.nseg = 2;
        J.seg[0].K = C.npp; J.seg[0].amode = AM_GPAIR; J.seg[0].a_rows = C.pp_off; J.seg[0].a_cols = C.pp_off;
        J.seg[0].b_arr = ARR_T; J.seg[0].b_off = C.t_off; J.seg[0].ldb = C.nhh;
        J.seg[0].term = by_pairs[k] ? 0 : CCD_T_PP;
        J.seg[1].K = C.nhh; J.seg[1].amode = AM_ROW; J.seg[1].a_arr = ARR_T; J.seg[1].a_off = C.t_off;
        J.seg[1].lda = C.nhh; J.seg[1].b_arr = ARR_CHH; J.seg[1].b_off = C.chh_off; J.seg[1].ldb = C.nhh;
        J.seg[1].term = CCD_T_HH | CCD_T_QHH;
        // with the pairs form the pp sums are already in the output (k_nm_ladpp runs first)
        J.omode = by_pairs[k] ? OM_ROW_ADD : OM_ROW; J.o_arr = ARR_LAD; J.o_off = C.t_off; J.ldo = C.nhh;
        add_tiles(J);
        c->flops += (by_pairs[k] ? 0.0 : 2.0 * C.npp * C.npp * C.nhh) + 2.0 * C.npp * C.nhh * C.nhh;
    }
    {
        int64_t moff = 0;
        for (auto& q : c->ph) {  // Z_Q = T~_Q C_P, scattered
            if (q.partner < 0) continue;
            const HPh& P = c->ph[q.partner];
            const int nQ = (int)q.mem.size(), nP = (int)P.mem.size();
            NmJob J = blank();
            J.M = nQ; J.N = nP; J.nseg = 1;
            J.seg[0].K = nP; J.seg[0].amode = AM_ROW; J.seg[0].a_arr = ARR_TQ; J.seg[0].a_off = q.tq_off;
            J.seg[0].lda = nP; J.seg[0].b_arr = ARR_CP; J.seg[0].b_off = q.cp_off; J.seg[0].ldb = nP;
            J.seg[0].term = CCD_T_RING | CCD_T_QRING;
            J.omode = OM_SCATTER; J.o_off = moff; J.ldo = nP;
            moff += (int64_t)nQ * nP;
            add_tiles(J);
            c->flops += 2.0 * nQ * nP * nP;
        }
    }
    c->tiles_b = (int)c->tiles.size() - c->tiles_a;
    if (c->n_tq >= ((int64_t)1 << 31) || c->n_cp >= ((int64_t)1 << 40)) {
        ccd::set_error("ccd_nm_build: ring blocks beyond 2^31 entries");
        return CCD_EINVAL;
    }
    return CCD_OK;
}

// workspace regions, in order
enum {
    R_ST, R_U, R_EPS, R_HH, R_PP, R_MEM, R_PMAP, R_CH, R_ITEMS, R_JOBS, R_TILES, R_CSRP, R_CSRI, R_RCH,
    R_LADD, R_LADLP, R_LADIT, R_RCIT, R_T0, R_T1, R_VT, R_CHH, R_TQ, R_CP, R_LAD, R_RING, R_ROWS, R_COLS, R_CPART,
    R_DCHI, R_EPART, R_EHIST, R_COUNT
};

void nm_layout(ccd_nm_ctx* c) {
    const size_t sz[R_COUNT] = {
        4 * (size_t)c->ns, 8 * c->u.size(), 8 * (size_t)c->ns, 4 * c->hh_all.size(), 4 * c->pp_all.size(),
        4 * c->mem_all.size(), 4 * std::max<size_t>(1, c->pmap.size()), sizeof(NmChanD) * c->chd.size(),
        sizeof(NmItem) * c->items.size(), sizeof(NmJob) * c->jobs.size(), sizeof(NmTile) * c->tiles.size(),
        4 * c->csr_ptr.size(), 4 * std::max<size_t>(1, c->csr_idx.size()), 4 * c->row_chan.size(),
        sizeof(NmLadD) * c->ladd.size(), 4 * c->ladlp.size(), sizeof(NmLadItem) * c->ladit.size(),
        sizeof(NmRcItem) * c->rcit.size(),
        8 * (size_t)c->n_amp, 8 * (size_t)c->n_amp, 8 * (size_t)c->n_amp, 8 * (size_t)std::max<int64_t>(1, c->n_chh),
        8 * (size_t)std::max<int64_t>(1, c->n_tq), 8 * (size_t)std::max<int64_t>(1, c->n_cp), 8 * (size_t)c->n_amp,
        32 * (size_t)c->n_amp, 8 * (size_t)c->n_rows, 8 * (size_t)c->n_cols, 8 * (size_t)std::max<int64_t>(1, c->n_cpart),
        8 * (size_t)c->ns,
        8 * c->items.size(), 8 * (size_t)kNmHist};
    c->region.clear();
    size_t off = 0;
    for (int k = 0; k < R_COUNT; k++) {
        c->region.push_back({off, sz[k]});
        off = up256(off + sz[k]);
    }
    c->ws_bytes = off;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" ccd_status ccd_nm_build(const ccd_nm_problem* prob, void* hip_stream, ccd_nm_ctx** out) {
    if (!prob || !out) {
        ccd::set_error("ccd_nm_build: NULL argument");
        return CCD_EINVAL;
    }
    *out = nullptr;
    ccd_nm_ctx* c = new (std::nothrow) ccd_nm_ctx();
    if (!c) {
        ccd::set_error("ccd_nm_build: out of host memory");
        return CCD_ENOMEM;
    }
    c->par = *prob;
    c->stream = (hipStream_t)hip_stream;
    ccd_status st;
    try {
        st = nm_plan(c);
    } catch (const std::bad_alloc&) {
        ccd::set_error("ccd_nm_build: out of host memory");
        st = CCD_ENOMEM;
    }
    if (st != CCD_OK) {
        delete c;
        return st;
    }
    nm_layout(c);
    *out = c;
    return CCD_OK;
}

extern "C" ccd_status ccd_nm_info_get(const ccd_nm_ctx* c, ccd_nm_info* info) {
    if (!c || !info) {
        ccd::set_error("ccd_nm_info_get: NULL argument");
        return CCD_EINVAL;
    }
    info->n_states = c->ns;
    info->n_holes = c->nh;
    info->n_channels = (int32_t)c->ch.size();
    info->n_ph_channels = (int32_t)c->ph.size();
    info->max_hh = c->max_hh;
    info->max_pp = c->max_pp;
    info->max_ph = c->max_ph;
    info->n_amplitudes = c->n_amp;
    info->box_L = c->L;
    info->flops_per_sweep = c->flops + c->flops_lad;
    return CCD_OK;
}

extern "C" ccd_status ccd_nm_workspace_size(const ccd_nm_ctx* c, size_t* bytes) {
    if (!c || !bytes) {
        ccd::set_error("ccd_nm_workspace_size: NULL argument");
        return CCD_EINVAL;
    }
    *bytes = c->ws_bytes;
    return CCD_OK;
}

namespace {

int nm_grid(int64_t work, int per) {
    return (int)std::max<int64_t>(1, std::min<int64_t>((work + per - 1) / per, 8192));
}

ccd_status nm_energy_now(ccd_nm_ctx* c, int slot, double* e) {
    k_nm_energy<<<1, 256, 0, c->stream>>>(c->dev, slot);
    NM_TRY(hipGetLastError());
    NM_TRY(hipMemcpyAsync(e, c->dev.ehist + slot, 8, hipMemcpyDeviceToHost, c->stream));
    NM_TRY(hipStreamSynchronize(c->stream));
    return CCD_OK;
}

// with timing on, every launch is bracketed by two events (collected when
// the stream is next synchronised)
struct NmTimed {
    ccd_nm_ctx* c;
    int fam;
    hipEvent_t a = nullptr, b = nullptr;
    NmTimed(ccd_nm_ctx* cc, int f) : c(cc), fam(f) {
        if (c->timing && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess)
            (void)hipEventRecord(a, c->stream);
    }
    ~NmTimed() {
        if (a && b) {
            (void)hipEventRecord(b, c->stream);
            c->pending.push_back({fam, {a, b}});
        } else {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    }
};

ccd_status nm_harvest(ccd_nm_ctx* c) {
    if (c->pending.empty()) return CCD_OK;
    NM_TRY(hipStreamSynchronize(c->stream));
    for (auto& p : c->pending) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, p.second.first, p.second.second) == hipSuccess) {
            c->fam_ms[p.first] += ms;
            c->fam_n[p.first] += 1;
        }
        (void)hipEventDestroy(p.second.first);
        (void)hipEventDestroy(p.second.second);
    }
    c->pending.clear();
    return CCD_OK;
}

// one sweep from t[cur] into t[cur ^ 1]; the energy lands in ehist[slot]
ccd_status nm_sweep(ccd_nm_ctx* c, double alpha, uint32_t mask, int slot) {
    NmDev& d = c->dev;
    hipStream_t s = c->stream;
    const int cur = c->cur;
    if (d.n_tq > 0) {
        NmTimed tm(c, NF_GATHER);
        k_nm_gather<<<nm_grid(d.n_tq, 256), 256, 0, s>>>(d, cur);
    }
    {
        NmTimed tm(c, NF_ROWCOL);
        k_nm_rowcol<<<std::min<int>((int)c->rcit.size(), 8192), 256, 0, s>>>(d, cur, (int)c->rcit.size());
        k_nm_colsum<<<nm_grid(c->n_cols, 256), 256, 0, s>>>(d, c->n_rows, c->n_cols);
    }
    {
        NmTimed tm(c, NF_DCHI);
        k_nm_dchi<<<nm_grid((int64_t)c->ns * 64, 256), 256, 0, s>>>(d, mask, c->nh);
    }
    if (c->tiles_a > 0) {
        NmTimed tm(c, NF_GEMM1);
        k_nm_gemm<<<std::min(c->tiles_a, 8192), 256, 0, s>>>(d, cur, mask, 0, c->tiles_a);
    }
    if (!c->ladit.empty() && (mask & (CCD_T_PP | CCD_T_HH | CCD_T_QHH))) {
        // the pp sums of the channels with the pairs form, before the ladder jobs add the rest
        NmTimed tm(c, NF_LADPP);
        k_nm_ladpp<<<std::min<int>((int)c->ladit.size(), 4096), 256, 0, s>>>(d, cur, mask, (int)c->ladit.size());
    }
    if (c->tiles_b > 0) {
        NmTimed tm(c, NF_GEMM2);
        k_nm_gemm<<<std::min(c->tiles_b, 8192), 256, 0, s>>>(d, cur, mask, c->tiles_a, c->tiles_b);
    }
    {
        NmTimed tm(c, NF_UPDATE);
        k_nm_update<<<std::min<int>((int)c->items.size(), 8192), 256, 0, s>>>(d, cur, alpha, mask);
    }
    {
        NmTimed tm(c, NF_ENERGY);
        k_nm_energy<<<1, 256, 0, s>>>(d, slot);
    }
    NM_TRY(hipGetLastError());
    c->cur ^= 1;
    return CCD_OK;
}

}  // namespace

extern "C" ccd_status ccd_nm_bind_workspace(ccd_nm_ctx* c, void* ptr, size_t bytes) {
    if (!c || !ptr || (((uintptr_t)ptr) & 255) || bytes < c->ws_bytes) {
        ccd::set_error("ccd_nm_bind_workspace: need a 256-byte aligned buffer of ccd_nm_workspace_size bytes");
        return CCD_EINVAL;
    }
    if (c->ws) {
        ccd::set_error("ccd_nm_bind_workspace: already bound");
        return CCD_ESTATE;
    }
    c->ws = (char*)ptr;
    char* b = c->ws;
    auto at = [&](int r) { return (void*)(b + c->region[r].first); };
    auto up = [&](int r, const void* src) -> hipError_t {
        if (c->region[r].second == 0) return hipSuccess;
        return hipMemcpyAsync(at(r), src, c->region[r].second, hipMemcpyHostToDevice, c->stream);
    };
    const int32_t zero = -1;
    NM_TRY(up(R_ST, c->st.data()));
    NM_TRY(up(R_U, c->u.data()));
    NM_TRY(up(R_EPS, c->eps.data()));
    NM_TRY(up(R_HH, c->hh_all.data()));
    NM_TRY(up(R_PP, c->pp_all.data()));
    if (!c->mem_all.empty()) NM_TRY(up(R_MEM, c->mem_all.data()));
    if (!c->pmap.empty()) NM_TRY(up(R_PMAP, c->pmap.data()));
    else NM_TRY(hipMemcpyAsync(at(R_PMAP), &zero, 4, hipMemcpyHostToDevice, c->stream));
    NM_TRY(up(R_CH, c->chd.data()));
    NM_TRY(up(R_ITEMS, c->items.data()));
    NM_TRY(up(R_JOBS, c->jobs.data()));
    NM_TRY(up(R_TILES, c->tiles.data()));
    NM_TRY(up(R_CSRP, c->csr_ptr.data()));
    if (!c->csr_idx.empty()) NM_TRY(up(R_CSRI, c->csr_idx.data()));
    NM_TRY(up(R_RCH, c->row_chan.data()));
    if (!c->ladd.empty()) NM_TRY(up(R_LADD, c->ladd.data()));
    if (!c->ladlp.empty()) NM_TRY(up(R_LADLP, c->ladlp.data()));
    if (!c->ladit.empty()) NM_TRY(up(R_LADIT, c->ladit.data()));
    NM_TRY(up(R_RCIT, c->rcit.data()));
    NmDev& d = c->dev;
    d.st = (const int32_t*)at(R_ST);
    d.u = (const double*)at(R_U);
    d.eps = (const double*)at(R_EPS);
    d.hh = (const int32_t*)at(R_HH);
    d.pp = (const int32_t*)at(R_PP);
    d.mem = (const int32_t*)at(R_MEM);
    d.pmap = (const int32_t*)at(R_PMAP);
    d.ch = (const NmChanD*)at(R_CH);
    d.items = (const NmItem*)at(R_ITEMS);
    d.jobs = (const NmJob*)at(R_JOBS);
    d.tiles = (const NmTile*)at(R_TILES);
    d.csr_ptr = (const int32_t*)at(R_CSRP);
    d.csr_idx = (const int32_t*)at(R_CSRI);
    d.row_chan = (const int32_t*)at(R_RCH);
    d.ladd = (const NmLadD*)at(R_LADD);
    d.ladlp = (const int4*)at(R_LADLP);
    d.ladit = (const NmLadItem*)at(R_LADIT);
    d.rcit = (const NmRcItem*)at(R_RCIT);
    d.cpart = (double*)at(R_CPART);
    d.t[0] = (double*)at(R_T0);
    d.t[1] = (double*)at(R_T1);
    d.vt = (double*)at(R_VT);
    d.chh = (double*)at(R_CHH);
    d.tq = (double*)at(R_TQ);
    d.cp = (double*)at(R_CP);
    d.lad = (double*)at(R_LAD);
    d.ring = (double*)at(R_RING);
    d.rowsum = (double*)at(R_ROWS);
    d.colsum = (double*)at(R_COLS);
    d.dchi = (double*)at(R_DCHI);
    d.epart = (double*)at(R_EPART);
    d.ehist = (double*)at(R_EHIST);
    d.ns = c->ns;
    d.nlut = c->nlut;
    d.n_items = (int32_t)c->items.size();
    d.n_tq = (int32_t)c->n_tq;
    d.n_amp = c->n_amp;
    c->cur = 0;
    k_nm_init<<<std::min<int>((int)c->items.size(), 8192), 256, 0, c->stream>>>(d);
    NM_TRY(hipGetLastError());
    ccd_status st = nm_energy_now(c, 0, &c->emp2);
    if (st != CCD_OK) return st;
    c->ecorr = c->emp2;
    if (!c->ev0) NM_TRY(hipEventCreate(&c->ev0));
    if (!c->ev1) NM_TRY(hipEventCreate(&c->ev1));
    return CCD_OK;
}

extern "C" ccd_status ccd_nm_iterate(ccd_nm_ctx* c, const ccd_solver_opts* o, int32_t* sweeps_done,
                                     double* e_hist) {
    if (!c || !o) {
        ccd::set_error("ccd_nm_iterate: NULL argument");
        return CCD_EINVAL;
    }
    if (!c->ws) {
        ccd::set_error("ccd_nm_iterate: bind a workspace first");
        return CCD_ESTATE;
    }
    if (!(o->mixing > 0.0 && o->mixing <= 1.0) || o->max_iter < 1 || o->precision != CCD_PREC_FP64) {
        ccd::set_error("ccd_nm_iterate: need 0 < mixing <= 1, max_iter >= 1 and FP64 precision");
        return CCD_EINVAL;
    }
    if (e_hist)
        for (int k = 0; k < o->max_iter; k++) e_hist[k] = NAN;
    const bool test = o->tol > 0.0 || o->tol_rel > 0.0;
    double e = c->ecorr;
    int done = 0;
    bool conv = false, bad = false;
    std::vector<double> h(kNmHist);
    float ms_total = 0.0f;
    while (done < o->max_iter && !conv && !bad) {
        const int chunk = test ? 1 : std::min(kNmHist, o->max_iter - done);
        NM_TRY(hipEventRecord(c->ev0, c->stream));
        for (int k = 0; k < chunk; k++) {
            ccd_status st = nm_sweep(c, o->mixing, o->terms, k);
            if (st != CCD_OK) return st;
        }
        NM_TRY(hipEventRecord(c->ev1, c->stream));
        NM_TRY(hipMemcpyAsync(h.data(), c->dev.ehist, 8 * (size_t)chunk, hipMemcpyDeviceToHost, c->stream));
        NM_TRY(hipStreamSynchronize(c->stream));
        float ms = 0.0f;
        NM_TRY(hipEventElapsedTime(&ms, c->ev0, c->ev1));
        ms_total += ms;
        for (int k = 0; k < chunk; k++) {
            const double en = h[k];
            if (e_hist) e_hist[done] = en;
            done++;
            if (!std::isfinite(en)) {
                bad = true;
                e = en;
                break;
            }
            const double de = std::fabs(en - e);
            e = en;
            if (test && de < o->tol + o->tol_rel * std::fabs(en)) {
                conv = true;
                break;
            }
        }
    }
    c->ecorr = e;
    c->last_ms = ms_total;
    if (sweeps_done) *sweeps_done = done;
    if (bad) {
        ccd::set_error("ccd_nm_iterate: correlation energy is not finite");
        return CCD_DIVERGED;
    }
    return test && !conv ? CCD_NOT_CONVERGED : CCD_OK;
}

extern "C" ccd_status ccd_nm_energy(const ccd_nm_ctx* c, double* e_ref, double* e_mbpt2, double* e_corr) {
    if (!c) {
        ccd::set_error("ccd_nm_energy: NULL context");
        return CCD_EINVAL;
    }
    if (e_ref) *e_ref = c->eref;
    if (e_mbpt2) *e_mbpt2 = c->emp2;
    if (e_corr) *e_corr = c->ecorr;
    return CCD_OK;
}

extern "C" ccd_status ccd_nm_get_amplitudes(const ccd_nm_ctx* c, double* dst, size_t n) {
    if (!c || !dst || n != (size_t)c->n_amp) {
        ccd::set_error("ccd_nm_get_amplitudes: need n = n_amplitudes and a host buffer");
        return CCD_EINVAL;
    }
    if (!c->ws) {
        ccd::set_error("ccd_nm_get_amplitudes: no workspace");
        return CCD_ESTATE;
    }
    NM_TRY(hipMemcpyAsync(dst, c->dev.t[c->cur], 8 * n, hipMemcpyDeviceToHost, c->stream));
    NM_TRY(hipStreamSynchronize(c->stream));
    return CCD_OK;
}

extern "C" ccd_status ccd_nm_set_amplitudes(ccd_nm_ctx* c, const double* src, size_t n) {
    if (!c || !src || n != (size_t)c->n_amp) {
        ccd::set_error("ccd_nm_set_amplitudes: need n = n_amplitudes and a host buffer");
        return CCD_EINVAL;
    }
    if (!c->ws) {
        ccd::set_error("ccd_nm_set_amplitudes: no workspace");
        return CCD_ESTATE;
    }
    NM_TRY(hipMemcpyAsync(c->dev.t[c->cur], src, 8 * n, hipMemcpyHostToDevice, c->stream));
    k_nm_dot<<<std::min<int>((int)c->items.size(), 8192), 256, 0, c->stream>>>(c->dev, c->cur);
    NM_TRY(hipGetLastError());
    return nm_energy_now(c, 0, &c->ecorr);
}

extern "C" ccd_status ccd_nm_export_maps(const ccd_nm_ctx* c, int32_t which, int32_t* dst, size_t n,
                                         size_t* n_needed) {
    if (!c) {
        ccd::set_error("ccd_nm_export_maps: NULL context");
        return CCD_EINVAL;
    }
    std::vector<int32_t> v;
    switch (which) {
        case CCD_NM_MAP_STATES:
            for (int p = 0; p < c->ns; p++)
                v.insert(v.end(), {c->nx[p], c->ny[p], c->nz[p], c->sz[p], c->tz[p]});
            break;
        case CCD_NM_MAP_CHANNELS:
            for (const auto& h : c->ch)
                v.insert(v.end(), {h.Kx, h.Ky, h.Kz, h.Sz, h.Tz, (int)h.hh.size(), (int)h.pp.size()});
            break;
        case CCD_NM_MAP_HH:
            for (int32_t x : c->hh_all) v.insert(v.end(), {pr_a(x), pr_b(x)});
            break;
        case CCD_NM_MAP_PP:
            for (int32_t x : c->pp_all) v.insert(v.end(), {pr_a(x), pr_b(x)});
            break;
        default:
            ccd::set_error("ccd_nm_export_maps: unknown map");
            return CCD_EINVAL;
    }
    if (n_needed) *n_needed = v.size();
    if (!dst) return CCD_OK;
    if (n < v.size()) {
        ccd::set_error("ccd_nm_export_maps: buffer too small");
        return CCD_EINVAL;
    }
    std::memcpy(dst, v.data(), 4 * v.size());
    return CCD_OK;
}

extern "C" ccd_status ccd_nm_export_tables(const ccd_nm_ctx* c, double* tkin, double* eps, double* e_ref) {
    if (!c) {
        ccd::set_error("ccd_nm_export_tables: NULL context");
        return CCD_EINVAL;
    }
    if (tkin) std::memcpy(tkin, c->tkin.data(), 8 * (size_t)c->ns);
    if (eps) std::memcpy(eps, c->eps.data(), 8 * (size_t)c->ns);
    if (e_ref) *e_ref = c->eref;
    return CCD_OK;
}

extern "C" ccd_status ccd_nm_element(const ccd_nm_ctx* c, int32_t p, int32_t q, int32_t r, int32_t s, double* v) {
    if (!c || !v || p < 0 || q < 0 || r < 0 || s < 0 || p >= c->ns || q >= c->ns || r >= c->ns || s >= c->ns) {
        ccd::set_error("ccd_nm_element: bad state index");
        return CCD_EINVAL;
    }
    if (c->sz[p] + c->sz[q] != c->sz[r] + c->sz[s] || c->tz[p] + c->tz[q] != c->tz[r] + c->tz[s]) {
        *v = 0.0;
        return CCD_OK;
    }
    *v = nm_vas_host(c, p, q, r, s);
    return CCD_OK;
}

extern "C" ccd_status ccd_nm_set_timing(ccd_nm_ctx* c, int32_t enabled) {
    if (!c) {
        ccd::set_error("ccd_nm_set_timing: NULL context");
        return CCD_EINVAL;
    }
    ccd_status st = nm_harvest(c);
    c->timing = enabled != 0;
    return st;
}

extern "C" ccd_status ccd_nm_kernel_times(ccd_nm_ctx* c, double* ms, int64_t* launches, double* flops,
                                          int32_t reset) {
    if (!c) {
        ccd::set_error("ccd_nm_kernel_times: NULL context");
        return CCD_EINVAL;
    }
    ccd_status st = nm_harvest(c);
    if (st != CCD_OK) return st;
    for (int f = 0; f < NF_NUM; f++) {
        if (ms) ms[f] = c->fam_ms[f];
        if (launches) launches[f] = c->fam_n[f];
        if (flops)
            flops[f] = f == NF_GEMM1 ? c->flops_a
                     : f == NF_GEMM2 ? c->flops - c->flops_a
                     : f == NF_LADPP ? c->flops_lad : 0.0;
        if (reset) { c->fam_ms[f] = 0.0; c->fam_n[f] = 0; }
    }
    return CCD_OK;
}

extern "C" const char* ccd_nm_kernel_name(int32_t family) {
    return family >= 0 && family < NF_NUM ? kNmFamily[family] : "";
}

extern "C" ccd_status ccd_nm_last_ms(const ccd_nm_ctx* c, double* ms) {
    if (!c || !ms) {
        ccd::set_error("ccd_nm_last_ms: NULL argument");
        return CCD_EINVAL;
    }
    *ms = c->last_ms;
    return CCD_OK;
}

extern "C" void ccd_nm_destroy(ccd_nm_ctx* c) {
    if (!c) return;
    (void)nm_harvest(c);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    delete c;
}
