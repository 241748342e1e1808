/*
 * ccd_nm.h -- C ABI of the CCD solver for infinite nuclear matter with
 * isospin (symmetric nuclear matter, SNM: protons and neutrons), in the same
 * library as ccd.h.  After Lietz, Novario, Jansen, Hagen and Hjorth-Jensen,
 * "Computational Nuclear Physics and Post Hartree-Fock Methods"
 * (arXiv:1611.06765).
 *
 * The problem (sec. "Developing a CCD code for infinite matter"): A nucleons,
 * A/2 protons and A/2 neutrons, at density rho = A / L^3 in a periodic box,
 * plane waves k = 2 pi n / L with n^2 <= nmax2, both spins and both isospins;
 * the model-space loop with its extra isospin loop (innermost, t_z = -1/2
 * proton first) orders the states and the first A are holes, so A must be one
 * of Table 1's fillings doubled (4, 28, 76, 108, 132, 228, ...).  The
 * interaction is the full Minnesota operator
 *   V = 1/2 (V_R + 1/2 (1 + P_s) V_T + 1/2 (1 - P_s) V_S) (1 - P_s P_t)
 * with Gaussian form factors (sec. "Two-body interaction"), whose V_T channel
 * acts between a proton and a neutron.  Direct channels carry (K, S_z, T_z),
 * cross channels (Q, sigma, tau) (the channel discussion after the
 * intermediates, with T_z in the index function).  Species = 1 is pure
 * neutron matter through the same code (a cross-check of the specialised
 * path of ccd.h).
 *
 * Conventions as in ccd.h: plain C types, status codes, ccd_last_error(),
 * energies as box totals in MeV, all device memory from the caller, work on
 * the stream given at creation.  One problem per context, FP64 throughout.
 *
 * Amplitude layout: the direct channels in the order of CCD_NM_MAP_CHANNELS,
 * each a row-major [n_pp][n_hh] block of t_ij^ab with (a < b) particle pairs
 * as rows and (i < j) hole pairs as columns, pairs in the order of
 * CCD_NM_MAP_PP / CCD_NM_MAP_HH.
 */
#ifndef CCD_NM_H
#define CCD_NM_H

#include <stddef.h>
#include <stdint.h>

#include "ccd.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t n_nucleons;   /* A: closed shell of the basis (species 2: 4, 28, 76, 108, 132, ...;
                             species 1: 2, 14, 38, 54, 66, ...) */
    int32_t species;      /* 2: protons and neutrons, A/2 each; 1: neutrons only */
    int32_t nmax2;        /* keep states with n_x^2+n_y^2+n_z^2 <= nmax2 (<= 64) */
    double density;       /* rho = A / L^3 in fm^-3 */
    double hbar2_over_m;  /* MeV fm^2 (one mass for both species), e.g. 41.47 */
    double V_R, kappa_R;  /* e.g. 200 MeV, 1.487 fm^-2 */
    double V_T, kappa_T;  /* e.g. -178 MeV, 0.639 fm^-2 (acts between a proton and a neutron) */
    double V_S, kappa_S;  /* e.g. -91.85 MeV, 0.465 fm^-2 */
} ccd_nm_problem;

typedef struct {
    int32_t n_states, n_holes;
    int32_t n_channels;       /* direct channels (K, S_z, T_z) holding amplitudes */
    int32_t n_ph_channels;    /* cross channels (Q, sigma, tau) */
    int32_t max_hh, max_pp, max_ph;
    int64_t n_amplitudes;
    double box_L;
    double flops_per_sweep;   /* FP64 flops of the channel products as executed */
} ccd_nm_info;

typedef struct ccd_nm_ctx ccd_nm_ctx;

/* Host plan: states, Minnesota tables, Fock energies (f_pp = t_p + sum_i
 * <pi||pi>), E_ref, direct and cross channels, the ring's position maps and the
 * work lists of the sweep.  No GPU work.  Errors: CCD_EINVAL, CCD_ENOTMAGIC
 * (A does not close a shell or leaves no particle states), CCD_ENOMEM. */
ccd_status ccd_nm_build(const ccd_nm_problem* prob, void* hip_stream, ccd_nm_ctx** out);
ccd_status ccd_nm_info_get(const ccd_nm_ctx* ctx, ccd_nm_info* info);
ccd_status ccd_nm_workspace_size(const ccd_nm_ctx* ctx, size_t* bytes);
/* Caller-owned device memory of ccd_nm_workspace_size bytes, 256-byte aligned,
 * kept alive until ccd_nm_destroy.  Uploads the tables and builds <ab||ij>, the
 * MBPT2 amplitudes and energy (eq. ccdGuess) on the device. */
ccd_status ccd_nm_bind_workspace(ccd_nm_ctx* ctx, void* device_ptr, size_t bytes);
/* Jacobi sweeps of eq. ccd3 in the intermediates form (FP64; opts: mixing,
 * tol, tol_rel, max_iter and terms are used, the rest ignored).  sweeps_done
 * (nullable) receives the sweeps run; e_hist (nullable, max_iter doubles)
 * the energy after each sweep, NaN past the last.  Synchronises the stream once
 * per sweep when a tolerance is set, else once at the end.  Returns CCD_OK,
 * CCD_NOT_CONVERGED, CCD_DIVERGED, CCD_EINVAL, CCD_ESTATE, CCD_EHIP. */
ccd_status ccd_nm_iterate(ccd_nm_ctx* ctx, const ccd_solver_opts* opts, int32_t* sweeps_done, double* e_hist);
/* E_ref, the MBPT2 and the current correlation energy (box totals, MeV). */
ccd_status ccd_nm_energy(const ccd_nm_ctx* ctx, double* e_ref, double* e_mbpt2, double* e_corr);
/* Canonical amplitudes to / from host memory (n = n_amplitudes doubles); set
 * recomputes the energy and makes them the current iterate. */
ccd_status ccd_nm_get_amplitudes(const ccd_nm_ctx* ctx, double* host_dst, size_t n);
ccd_status ccd_nm_set_amplitudes(ccd_nm_ctx* ctx, const double* host_src, size_t n);
/* Host copies of the plan (no GPU needed).  dst NULL or n too small: only
 * *n_needed is written (CCD_OK for NULL, CCD_EINVAL otherwise). */
#define CCD_NM_MAP_STATES   0 /* 5 per state: n_x, n_y, n_z, 2 s_z, 2 t_z                   */
#define CCD_NM_MAP_CHANNELS 1 /* 7 per direct channel: K_x, K_y, K_z, 2 S_z, 2 T_z, n_hh, n_pp */
#define CCD_NM_MAP_HH       2 /* 2 per hole pair (i, j), channel after channel               */
#define CCD_NM_MAP_PP       3 /* 2 per particle pair (a, b), channel after channel           */
ccd_status ccd_nm_export_maps(const ccd_nm_ctx* ctx, int32_t which, int32_t* dst, size_t n, size_t* n_needed);
/* Host tables: kinetic and Fock energies (n_states each, nullable) and E_ref. */
ccd_status ccd_nm_export_tables(const ccd_nm_ctx* ctx, double* tkin, double* eps, double* e_ref);
/* The plan's antisymmetrised element <pq||rs> (host arithmetic, the same
 * formula the kernels use), zero unless momentum, S_z and T_z are conserved. */
ccd_status ccd_nm_element(const ccd_nm_ctx* ctx, int32_t p, int32_t q, int32_t r, int32_t s, double* v);
/* Milliseconds of GPU time (HIP events on the context's stream) of the last
 * ccd_nm_iterate call's sweeps, excluding host reads. */
ccd_status ccd_nm_last_ms(const ccd_nm_ctx* ctx, double* ms);
/* Per-launch timing: while enabled every launch of a sweep is bracketed by two
 * HIP events on the context's stream.  ccd_nm_kernel_times returns, per kernel
 * family (CCD_NM_FAMILIES of them, named by ccd_nm_kernel_name: gather,
 * rowcol, dchi, gemm_chi (chi_klij and the ring's C_P), gemm_ladder_ring (the
 * hh ladder, the pp ladder of blocks without the momentum-pair form, and the
 * ring's Z_Q), update, energy, ladder_pp (the pp ladder as products over the
 * blocks' momentum pairs)), the summed milliseconds, the
 * launch count and the FP64 flops of one launch of that family (0 for the
 * non-product families), and optionally resets the sums.  Both synchronise the
 * stream. */
#define CCD_NM_FAMILIES 8
ccd_status ccd_nm_set_timing(ccd_nm_ctx* ctx, int32_t enabled);
ccd_status ccd_nm_kernel_times(ccd_nm_ctx* ctx, double* ms, int64_t* launches, double* flops, int32_t reset);
const char* ccd_nm_kernel_name(int32_t family);
void ccd_nm_destroy(ccd_nm_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* CCD_NM_H */
