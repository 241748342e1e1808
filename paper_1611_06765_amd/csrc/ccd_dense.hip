// ccd_dense.hip -- CCD for small model spaces given by dense matrix elements
// (the pairing model of sec. "Developing a CCD code for infinite matter",
// eqs. sppairing / intpairing, or any Hamiltonian in a canonical Hartree-Fock
// basis): the Fock energies of eq. pairingsp, the MBPT2 start of eq. ccdGuess
// and Jacobi sweeps of eq. ccd3 with all eight terms, one GPU thread per
// ordered amplitude (i, j, a, b), every sum in a fixed order.  It is a
// validation path (cost O(n_h^4 n_p^4)), not a fast one: the plane-wave
// problems run on the channel-blocked kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ccd_internal.h"

namespace {

constexpr int kDenseMaxN = 48;

struct Dense {
    const double* v;    // <pq||rs> at ((p n + q) n + r) n + s
    const double* eps;  // Fock energies
    int n, nh, np;
};

__device__ __forceinline__ double dv(const Dense& q, int p, int r, int s, int u) {
    return q.v[(((size_t)p * q.n + r) * q.n + s) * q.n + u];
}
// t_ij^ab at ((i nh + j) np + a - nh) np + b - nh
__device__ __forceinline__ size_t tix(const Dense& q, int i, int j, int a, int b) {
    return ((size_t)(i * q.nh + j) * q.np + (a - q.nh)) * q.np + (b - q.nh);
}

__global__ void __launch_bounds__(256) k_dense_mbpt2(Dense q, double* t) {
    const size_t m = (size_t)q.nh * q.nh * q.np * q.np;
    for (size_t e = blockIdx.x * 256 + threadIdx.x; e < m; e += (size_t)gridDim.x * 256) {
        const int b = q.nh + (int)(e % q.np), a = q.nh + (int)((e / q.np) % q.np);
        const int j = (int)((e / ((size_t)q.np * q.np)) % q.nh), i = (int)(e / ((size_t)q.np * q.np * q.nh));
        t[e] = dv(q, a, b, i, j) / (q.eps[i] + q.eps[j] - q.eps[a] - q.eps[b]);
    }
}

// the right-hand side of eq. ccd3 for (i, j, a, b) from amplitudes t
__device__ double ccd3_rhs(const Dense& q, const double* t, int i, int j, int a, int b, uint32_t m) {
    const int nh = q.nh, n = q.n;
    double r = dv(q, a, b, i, j);
    if (m & CCD_T_PP) {
        double s = 0.0;
        for (int c = nh; c < n; c++)
            for (int d = nh; d < n; d++) s += dv(q, a, b, c, d) * t[tix(q, i, j, c, d)];
        r += 0.5 * s;
    }
    if (m & CCD_T_HH) {
        double s = 0.0;
        for (int k = 0; k < nh; k++)
            for (int l = 0; l < nh; l++) s += dv(q, k, l, i, j) * t[tix(q, k, l, a, b)];
        r += 0.5 * s;
    }
    if (m & CCD_T_RING) {
        // P(ij|ab) f(i,j,a,b) = f(ijab) - f(jiab) - f(ijba) + f(jiba),
        // f = sum_kc <kb||cj> t_ik^ac
        auto f = [&](int i_, int j_, int a_, int b_) {
            double s = 0.0;
            for (int k = 0; k < nh; k++)
                for (int c = nh; c < n; c++) s += dv(q, k, b_, c, j_) * t[tix(q, i_, k, a_, c)];
            return s;
        };
        r += f(i, j, a, b) - f(j, i, a, b) - f(i, j, b, a) + f(j, i, b, a);
    }
    if (m & (CCD_T_QHH | CCD_T_QRING | CCD_T_QHOLE | CCD_T_QPART)) {
        double s_hh = 0.0, s_ring = 0.0, s_hole = 0.0, s_part = 0.0;
        for (int k = 0; k < nh; k++)
            for (int l = 0; l < nh; l++)
                for (int c = nh; c < n; c++)
                    for (int d = nh; d < n; d++) {
                        const double w = dv(q, k, l, c, d);
                        if (w == 0.0) continue;
                        if (m & CCD_T_QHH) s_hh += w * t[tix(q, i, j, c, d)] * t[tix(q, k, l, a, b)];
                        if (m & CCD_T_QRING)
                            s_ring += w * (t[tix(q, i, k, a, c)] * t[tix(q, j, l, b, d)] -
                                           t[tix(q, j, k, a, c)] * t[tix(q, i, l, b, d)]);
                        if (m & CCD_T_QHOLE)
                            s_hole += w * (t[tix(q, i, k, d, c)] * t[tix(q, l, j, a, b)] -
                                           t[tix(q, j, k, d, c)] * t[tix(q, l, i, a, b)]);
                        if (m & CCD_T_QPART)
                            s_part += w * (t[tix(q, l, k, a, c)] * t[tix(q, i, j, d, b)] -
                                           t[tix(q, l, k, b, c)] * t[tix(q, i, j, d, a)]);
                    }
        r += 0.25 * s_hh + s_ring - 0.5 * s_hole - 0.5 * s_part;
    }
    return r;
}

__global__ void __launch_bounds__(256) k_dense_sweep(Dense q, const double* t, double* tn, double alpha, uint32_t m) {
    const size_t mm = (size_t)q.nh * q.nh * q.np * q.np;
    for (size_t e = blockIdx.x * 256 + threadIdx.x; e < mm; e += (size_t)gridDim.x * 256) {
        const int b = q.nh + (int)(e % q.np), a = q.nh + (int)((e / q.np) % q.np);
        const int j = (int)((e / ((size_t)q.np * q.np)) % q.nh), i = (int)(e / ((size_t)q.np * q.np * q.nh));
        double tnew = 0.0;
        if (i != j && a != b) {
            const double r = ccd3_rhs(q, t, i, j, a, b, m);
            tnew = r / (q.eps[i] + q.eps[j] - q.eps[a] - q.eps[b]);
        }
        tn[e] = alpha * tnew + (1.0 - alpha) * t[e];
    }
}

// 1/4 sum <ij||ab> t_ij^ab: one partial per block (fixed order in the block)
__global__ void __launch_bounds__(256) k_dense_energy(Dense q, const double* t, double* part) {
    __shared__ double sh[256];
    const size_t mm = (size_t)q.nh * q.nh * q.np * q.np;
    const size_t e = blockIdx.x * 256 + threadIdx.x;
    double x = 0.0;
    if (e < mm) {
        const int b = q.nh + (int)(e % q.np), a = q.nh + (int)((e / q.np) % q.np);
        const int j = (int)((e / ((size_t)q.np * q.np)) % q.nh), i = (int)(e / ((size_t)q.np * q.np * q.nh));
        x = dv(q, i, j, a, b) * t[e];
    }
    sh[threadIdx.x] = x;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = 0.25 * sh[0];
}

struct DenseLayout {
    size_t v, eps, t0, t1, part, total;
    int nblk;
};

DenseLayout dense_layout(int n, int nh) {
    const size_t np = (size_t)(n - nh), m = (size_t)nh * nh * np * np;
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    DenseLayout L;
    L.nblk = (int)((m + 255) / 256);
    L.v = 0;
    L.eps = up(L.v + 8 * (size_t)n * n * n * n);
    L.t0 = up(L.eps + 8 * (size_t)n);
    L.t1 = up(L.t0 + 8 * m);
    L.part = up(L.t1 + 8 * m);
    L.total = up(L.part + 8 * (size_t)L.nblk);
    return L;
}

#define DENSE_TRY(x)                                                                 \
    do {                                                                             \
        hipError_t e_ = (x);                                                         \
        if (e_ != hipSuccess) {                                                      \
            ccd::set_error(std::string("ccd_dense_solve: ") + hipGetErrorString(e_)); \
            return CCD_EHIP;                                                         \
        }                                                                            \
    } while (0)

}  // namespace

extern "C" ccd_status ccd_dense_workspace_size(int32_t n, int32_t n_holes, size_t* bytes) {
    if (!bytes || n < 2 || n > kDenseMaxN || n_holes < 1 || n_holes >= n) {
        ccd::set_error("ccd_dense_workspace_size: need 2 <= n <= 48 and 1 <= n_holes < n");
        return CCD_EINVAL;
    }
    *bytes = dense_layout(n, n_holes).total;
    return CCD_OK;
}

// The work area of ccd_dense_solve_static (8 MiB per GPU; see
// scratch_address below for how host code reaches it).
constexpr size_t kDenseScratchBytes = CCD_DENSE_STATIC_BYTES;
static __device__ __align__(256) unsigned char scratch[kDenseScratchBytes];

namespace {

// The solve itself, on a work area `dev_work` of at least dense_layout(n,
// n_holes).total bytes (sizes and options already checked).  Every byte of the
// area that a kernel reads is written first in this call: v and eps by the
// uploads, t0 by the MBPT2 kernel, t1 by the first sweep, the energy partials
// by the energy kernel, so a reused area needs no clearing.
ccd_status dense_solve_on(const double* h, const double* v, int32_t n, int32_t n_holes,
                          const ccd_solver_opts* o, void* dev_work, hipStream_t s, double* e_ref,
                          double* e_mbpt2, double* e_ccd, int32_t* sweeps, double* e_hist) {
    ccd_status st = CCD_OK;
    const int nh = n_holes, np = n - n_holes;
    auto V = [&](int p, int q, int r, int s) { return v[(((size_t)p * n + q) * n + r) * n + s]; };
    // Fock energies (eq. pairingsp) and the reference energy
    std::vector<double> eps(n);
    for (int p = 0; p < n; p++) {
        double s = h[p];
        for (int i = 0; i < nh; i++) s += V(p, i, p, i);
        eps[p] = s;
    }
    double eref = 0.0, pot = 0.0;
    for (int i = 0; i < nh; i++) eref += h[i];
    for (int i = 0; i < nh; i++)
        for (int j = 0; j < nh; j++) pot += V(i, j, i, j);
    eref += 0.5 * pot;
    for (int i = 0; i < nh; i++)
        for (int a = nh; a < n; a++)
            if (!(eps[i] < eps[a])) {
                ccd::set_error("ccd_dense_solve: a hole lies at or above a particle in Fock energy");
                return CCD_EINVAL;
            }
    const DenseLayout L = dense_layout(n, nh);
    char* base = (char*)dev_work;
    DENSE_TRY(hipMemcpyAsync(base + L.v, v, 8 * (size_t)n * n * n * n, hipMemcpyHostToDevice, s));
    DENSE_TRY(hipMemcpyAsync(base + L.eps, eps.data(), 8 * (size_t)n, hipMemcpyHostToDevice, s));
    Dense q;
    q.v = (const double*)(base + L.v);
    q.eps = (const double*)(base + L.eps);
    q.n = n; q.nh = nh; q.np = np;
    double* t[2] = {(double*)(base + L.t0), (double*)(base + L.t1)};
    double* part = (double*)(base + L.part);
    std::vector<double> ph(L.nblk);
    auto energy = [&](const double* tt, double& e) -> ccd_status {
        k_dense_energy<<<L.nblk, 256, 0, s>>>(q, tt, part);
        DENSE_TRY(hipGetLastError());
        DENSE_TRY(hipMemcpyAsync(ph.data(), part, 8 * (size_t)L.nblk, hipMemcpyDeviceToHost, s));
        DENSE_TRY(hipStreamSynchronize(s));
        e = 0.0;
        for (int b = 0; b < L.nblk; b++) e += ph[b];
        return CCD_OK;
    };
    const int grid = std::min(L.nblk, 4096);
    k_dense_mbpt2<<<grid, 256, 0, s>>>(q, t[0]);
    DENSE_TRY(hipGetLastError());
    double e2 = 0.0;
    if ((st = energy(t[0], e2)) != CCD_OK) return st;
    if (e_ref) *e_ref = eref;
    if (e_mbpt2) *e_mbpt2 = e2;
    if (e_hist)
        for (int k = 0; k < o->max_iter; k++) e_hist[k] = NAN;
    double e = e2;
    int cur = 0, done = 0;
    bool conv = false;
    for (int it = 0; it < o->max_iter; it++) {
        k_dense_sweep<<<grid, 256, 0, s>>>(q, t[cur], t[cur ^ 1], o->mixing, o->terms);
        DENSE_TRY(hipGetLastError());
        cur ^= 1;
        double en = 0.0;
        if ((st = energy(t[cur], en)) != CCD_OK) return st;
        done = it + 1;
        if (e_hist) e_hist[it] = en;
        if (!std::isfinite(en)) {
            if (e_ccd) *e_ccd = en;
            if (sweeps) *sweeps = done;
            ccd::set_error("ccd_dense_solve: correlation energy is not finite");
            return CCD_DIVERGED;
        }
        const double de = std::fabs(en - e);
        e = en;
        if ((o->tol > 0.0 || o->tol_rel > 0.0) && de < o->tol + o->tol_rel * std::fabs(en)) {
            conv = true;
            break;
        }
    }
    if (e_ccd) *e_ccd = e;
    if (sweeps) *sweeps = done;
    return (o->tol > 0.0 || o->tol_rel > 0.0) && !conv ? CCD_NOT_CONVERGED : CCD_OK;
}

ccd_status dense_check_opts(const char* who, const double* h, const double* v, const ccd_solver_opts* o) {
    if (!h || !v || !o) {
        ccd::set_error(std::string(who) + ": need h, v and opts");
        return CCD_EINVAL;
    }
    if (!(o->mixing > 0.0 && o->mixing <= 1.0) || o->max_iter < 1) {
        ccd::set_error(std::string(who) + ": need 0 < mixing <= 1 and max_iter >= 1");
        return CCD_EINVAL;
    }
    return CCD_OK;
}

// Work area of ccd_dense_solve_static: one per GPU, alive until the process
// ends.  Host code never passes `scratch` itself to a kernel or a copy (on the
// host the name is only a stand-in); it uses the device address that
// hipGetSymbolAddress returns for the current device, kept per device.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

ccd_status scratch_address(void** out) {
    int dev = -1;
    DENSE_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        ccd::set_error("ccd_dense_solve_static: device index out of range");
        return CCD_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* p = nullptr;
        DENSE_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || (((uintptr_t)p) & 255)) {
            ccd::set_error("ccd_dense_solve_static: scratch array has no aligned device address");
            return CCD_EHIP;
        }
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return CCD_OK;
}

}  // namespace

extern "C" ccd_status ccd_dense_solve(const double* h, const double* v, int32_t n, int32_t n_holes,
                                      const ccd_solver_opts* o, void* dev_work, size_t work_bytes, void* hip_stream,
                                      double* e_ref, double* e_mbpt2, double* e_ccd, int32_t* sweeps,
                                      double* e_hist) {
    size_t need = 0;
    ccd_status st = ccd_dense_workspace_size(n, n_holes, &need);
    if (st != CCD_OK) return st;
    if ((st = dense_check_opts("ccd_dense_solve", h, v, o)) != CCD_OK) return st;
    if (!dev_work || (((uintptr_t)dev_work) & 255) || work_bytes < need) {
        ccd::set_error("ccd_dense_solve: need a 256-byte aligned work buffer of ccd_dense_workspace_size bytes");
        return CCD_EINVAL;
    }
    return dense_solve_on(h, v, n, n_holes, o, dev_work, (hipStream_t)hip_stream, e_ref, e_mbpt2, e_ccd,
                          sweeps, e_hist);
}

extern "C" ccd_status ccd_dense_solve_static(const double* h, const double* v, int32_t n, int32_t n_holes,
                                             const ccd_solver_opts* o, void* hip_stream, double* e_ref,
                                             double* e_mbpt2, double* e_ccd, int32_t* sweeps, double* e_hist) {
    size_t need = 0;
    ccd_status st = ccd_dense_workspace_size(n, n_holes, &need);
    if (st != CCD_OK) return st;
    if ((st = dense_check_opts("ccd_dense_solve_static", h, v, o)) != CCD_OK) return st;
    if (need > kDenseScratchBytes) {
        ccd::set_error("ccd_dense_solve_static: this model space needs " + std::to_string(need) +
                       " bytes of work area, more than the " + std::to_string(kDenseScratchBytes) +
                       " of the static one; use ccd_dense_solve with a caller buffer");
        return CCD_EINVAL;
    }
    void* work = nullptr;
    if ((st = scratch_address(&work)) != CCD_OK) return st;
    return dense_solve_on(h, v, n, n_holes, o, work, (hipStream_t)hip_stream, e_ref, e_mbpt2, e_ccd, sweeps,
                          e_hist);
}
