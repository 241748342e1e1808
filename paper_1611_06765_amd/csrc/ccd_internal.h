// ccd_internal.h -- host plan and device-side descriptors of the CCD library.
// Private to the library: the public interface is include/ccd.h.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ccd.h"

namespace ccd {

// Limits of the kernels (checked when the plan is built).
constexpr int kMaxHH = 64;        // hole pairs of one direct channel (ladder tile width)
constexpr int kMaxPH = 90;        // pairs of one particle-hole channel (2 N^2 doubles in LDS)
constexpr int kLadderRows = 64;   // particle-pair rows per ladder work item
constexpr int kElemChunk = 1024;  // amplitudes per elementwise work item

// A state is packed into 32 bits: bytes 0..2 = n_x, n_y, n_z (int8), byte 3 = 2 s_z (int8).
inline int32_t pack_state(int x, int y, int z, int s) {
    return (int32_t)((uint32_t)(uint8_t)(int8_t)x | ((uint32_t)(uint8_t)(int8_t)y << 8) |
                     ((uint32_t)(uint8_t)(int8_t)z << 16) | ((uint32_t)(uint8_t)(int8_t)s << 24));
}
// A pair of state indices (local to the problem) is packed as p | q << 16.
inline int32_t pack_pair(int p, int q) { return (int32_t)((uint32_t)p | ((uint32_t)q << 16)); }

// ---- descriptors shared with the kernels (plain data, 8-byte aligned) ------
struct DevProb {
    int32_t ns, nh, np;
    int32_t st_off;       // offset into states / eps / dchi
    int32_t lut_off;      // offset into the W/2 table
    int32_t ph_off;       // offset into phq / phpos ([(p-nh)*nh + h])
    int32_t ladder_lo, ladder_hi;  // ladder work items of this problem (energy partial slots)
    int32_t elem_lo, elem_hi;      // elementwise work items of this problem
};

struct DevChan {
    int64_t t_off;        // element offset of the [npp][nhh] block
    int32_t prob;         // problem index
    int32_t nhh, npp;
    int32_t sz;           // 2 S_z: -2, 0, +2
    int32_t hh_off, pp_off;   // offsets into hh_pairs / pp_pairs
    int32_t chh_off;      // offset of the chi_klij block (S_z = 0), else -1
    int32_t row_off;      // global row id of row 0 (S_z = 0), for row sums
    int32_t col_off;      // global column id of column 0 (S_z = 0), for column sums
    int32_t pad;
};

struct DevPh {
    int64_t z_off;        // offset of the [n][n] block in the ph-layout buffers
    int32_t prob, n, partner, mem_off;
};

struct Item {             // work item: a channel and a start (row or element)
    int32_t chan, start;
};

// ---- host-side plan of one problem ----------------------------------------
struct Chan {
    int Kx, Ky, Kz, Sz;   // Sz = 2 S_z
    int nhh, npp;
    int64_t t_off;        // local to the problem
    int hh_off, pp_off;   // local to the problem (in pairs)
};

struct PhChan {
    int Qx, Qy, Qz, sig;  // sig = 2 (s_p - s_h)/... in units of 1/2: -2, 0, +2
    int n, partner;       // local partner index
    int mem_off;          // local offset in phmem (pairs)
    int64_t z_off;        // local
};

struct HostProblem {
    ccd_problem par;
    int ns = 0, nh = 0, np = 0, R = 0;
    double L = 0;
    std::vector<int> nx, ny, nz, sz;     // sz = 2 s_z = -1 or +1
    std::vector<double> tkin, eps;       // kinetic and Fock energies
    std::vector<double> W;               // W(m), m = 0 .. 4 nmax2
    double eref = 0;
    std::vector<Chan> chans;
    std::vector<int32_t> hh, pp;         // pairs, 2 ints each, channel after channel
    int64_t n_amp = 0;
    int n_sz0 = 0;
    std::vector<PhChan> ph;
    std::vector<int32_t> phmem;          // (p, h), 2 ints each
    std::vector<int32_t> phq, phpos;     // [(p-nh)*nh + h] -> local ph channel, position
    int64_t nz_ph = 0;                   // sum n^2 over ph channels
    int max_hh = 0, max_pp = 0, max_ph = 0;
    double flops_pp = 0, flops_hh = 0, flops_ring = 0, flops_ordered = 0;
};

// build one problem's plan; returns CCD_OK or an error with message
ccd_status build_problem(const ccd_problem& p, HostProblem& out, std::string& err);

void set_error(const std::string& msg);

}  // namespace ccd
