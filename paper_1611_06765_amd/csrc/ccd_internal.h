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
constexpr int kMaxPH = 80;        // pairs of one particle-hole channel (2 N^2 doubles in LDS)
constexpr int kLadderRows = 128;  // momentum pairs (rows of the pair product) per ladder work item
constexpr int kElemChunk = 1024;  // amplitudes per elementwise work item
constexpr int kDirSplit = 256;    // particle-pair rows per work item of the chi_klij product
constexpr int kMaxNmax2 = 64;     // cutoff limit: W(m) tables of 4 nmax2 + 1 entries live in LDS
constexpr int kMaxLut = 4 * kMaxNmax2 + 1;

// A state is packed into 32 bits: bytes 0..2 = n_x, n_y, n_z (int8), byte 3 = 2 s_z (int8).
inline int32_t pack_state(int x, int y, int z, int s) {
    return (int32_t)((uint32_t)(uint8_t)(int8_t)x | ((uint32_t)(uint8_t)(int8_t)y << 8) |
                     ((uint32_t)(uint8_t)(int8_t)z << 16) | ((uint32_t)(uint8_t)(int8_t)s << 24));
}
// A pair of state indices (local to the problem) is packed as p | q << 16.
inline int32_t pack_pair(int p, int q) { return (int32_t)((uint32_t)p | ((uint32_t)q << 16)); }

// ---- descriptors shared with the kernels (plain data) -----------------------
// Problems with the same (N, nmax2) have identical channel structure; they form
// a group whose integer tables are stored once.  Per-problem data (W table,
// Fock energies, amplitudes, intermediates) is stored problem after problem, so
// problem g of a group is found at base + g * stride.
struct DevGroup {
    int64_t n_amp;        // canonical amplitudes per problem
    int64_t t_base;       // amplitude index of the group's first problem
    int64_t n_zp;         // pair-block positions per problem
    int64_t zidx_off;     // pair-block position -> ring slot table (shared)
    int32_t phq_off;      // (p, h) -> cross channel / position tables (shared)
    int32_t n_rows_all, n_cols_all; // particle-pair rows / hole-pair columns of all channels
    int32_t rowa_base, cola_base;   // per-row / per-column arrays: + g * n_rows_all / n_cols_all
    int32_t pp0, hh0;               // first particle / hole pair of the structure in the pair tables
    int32_t G, p0;        // problems in the group, index of the first one
    int32_t ns, nh, np, nlut;
    int32_t st_off;       // packed states (shared)
    int32_t eps_base;     // Fock energies / one-body intermediates: eps_base + g * ns
    int32_t lut_base;     // W/2 tables: lut_base + g * nlut
    int32_t ph_base;      // ph-map offset of the group (shared)
    int32_t n_rows, n_cols, n_chh;  // S_z = 0 rows, columns, chi_klij entries per problem
    int32_t rows_base, cols_base, chh_base;  // + g * n_rows / n_cols / n_chh
    int32_t ladder_lo, ladder_hi;   // ladder items of the group
    int32_t elem_lo, elem_hi;       // elementwise items of the group
    int32_t eelem_base;   // elementwise energy partial of (item, g)
    int32_t csr_off;      // one-body CSR row pointers of the group: csr_off + s
    int32_t n_dpart, n_dcolp;       // partial chi_klij / column sums per problem
    int64_t dpart_base, dcolp_base; // + g * n_dpart / n_dcolp
};

struct DevChan {
    int64_t t_off;        // element offset of the [npp][nhh] block inside a problem
    int32_t group;
    int32_t nhh, npp;
    int32_t sz;           // 2 S_z: -2, 0, +2
    int32_t hh_off, pp_off;   // global offsets into hh / pp pair tables (shared)
    int32_t chh_off;      // local offset of the chi_klij block (S_z = 0), else -1
    int32_t row_off;      // local row id of row 0 (S_z = 0)
    int32_t col_off;      // local column id of column 0 (S_z = 0)
    int32_t kx, ky, kz;   // total momentum
    int32_t rowa_off, cola_off;     // first row / column of the block among all rows / columns
    int32_t dsub_lo, dsub_n;        // S_z = 0: items of kDirSplit rows of the chi_klij product
    int32_t dpart_off, dcolp_off;   // S_z = 0: local offsets of their partial sums
    int32_t lp_off, n_lp;           // S_z = 0: momentum pairs of the rows (global offset, count)
};

struct DevPh {
    int64_t map_off;      // global offset of the [n][m] position map (shared)
    int64_t zp_off;       // offset of the [n][m] pair block if this channel is the
                          // primary of its pair {Q, -Q} (the lower index), else -1
    int32_t group, n, partner, mem_off;  // partner / mem_off global (members in the packed-state table)
    int32_t m;            // the partner's size (differs from n under a twist)
    int32_t pmem_off;     // the partner's mem_off
};

struct Item {             // work item: a channel and a start (row or element)
    int32_t chan, start;
};

// ---- host-side plan of one problem ----------------------------------------
struct Chan {
    int Kx, Ky, Kz, Sz;   // Sz = 2 S_z
    int nhh, npp;
    int nlp;              // S_z = 0: momentum pairs {n_a, n_b} of the rows
    int64_t t_off;        // local to the problem
    int hh_off, pp_off;   // local to the problem (in pairs)
};

struct PhChan {
    int Qx, Qy, Qz, sig;  // sig = 2 (s_p - s_h): -2, 0, +2
    int n, partner;       // local partner index
    int mem_off;          // local offset in phmem (pairs)
    int64_t z_off;        // local offset of the position map [n][partner's n]
    int64_t zp_off;       // pair-block offset if primary of {Q, -Q} (lower index), else -1
};

struct HostProblem {
    ccd_problem par;
    int ns = 0, nh = 0, np = 0, R = 0;
    double L = 0;
    std::vector<int> nx, ny, nz, sz;     // sz = 2 s_z = -1 or +1
    std::vector<double> tkin, eps;       // kinetic and Fock energies
    std::vector<double> W;               // W(m), m = 0 .. 4 nmax2
    double ekin = 0, eref = 0;           // kinetic and reference energy of the Fermi sea
    std::vector<Chan> chans;
    std::vector<int32_t> hh, pp;         // pairs, 2 ints each, channel after channel
    int64_t n_amp = 0;
    int n_sz0 = 0;
    std::vector<PhChan> ph;
    std::vector<int32_t> phmem;          // (p, h), 2 ints each
    std::vector<int32_t> phq, phpos;     // [(p-nh)*nh + h] -> local ph channel, position
    int64_t nz_ph = 0;                   // sum n^2 over ph channels
    // position map of the particle-hole blocks: entry (Q, u, y) for the pairs
    // (p,h) = member u of Q and (p',h') = member y of the partner of Q names the
    // canonical amplitude of {h,h'},{p,p'}: (e << 3) | (slot << 1) | negative,
    // slot = 2 [p > p'] + [h > h'], or -1 when h = h' or p = p'.
    std::vector<int32_t> phmap;
    int64_t n_zp = 0;                    // entries of the pair blocks
    // per canonical amplitude: the two pair-block entries that hold its ring
    // term, positions (a,i)(b,j) and (a,j)(b,i)
    std::vector<int32_t> zidx;           // 2 per amplitude: the pair-block positions of its ring terms
    std::vector<int32_t> zs;             // per pair-block position: (ring slot 2e + k) << 1 | sign, or -1
    int max_hh = 0, max_pp = 0, max_ph = 0;
    double flops_pp = 0, flops_hh = 0, flops_ring = 0, flops_ordered = 0;
};

// build one problem's plan; returns CCD_OK or an error with message
ccd_status build_problem(const ccd_problem& p, HostProblem& out, std::string& err);

void set_error(const std::string& msg);

}  // namespace ccd
