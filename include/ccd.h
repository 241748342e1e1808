/*
 * ccd.h -- C ABI of the MI355X (gfx950) coupled-cluster doubles (CCD) library
 * for pure neutron matter (PNM) in a periodic box with the Minnesota
 * interaction, after Lietz, Novario, Jansen, Hagen and Hjorth-Jensen,
 * "Computational Nuclear Physics and Post Hartree-Fock Methods"
 * (arXiv:1611.06765).
 *
 * The problem stated by the paper (sec. "Developing a CCD code for infinite
 * matter"): for N neutrons (a closed shell of the plane-wave basis) at density
 * rho, in a basis of plane waves k = 2 pi n / L with n_x^2+n_y^2+n_z^2 <= nmax2
 * and both spin projections, find the reference energy E_ref, the MBPT2
 * correlation energy and the CCD correlation energy of eq. ccdcorr, by the
 * iteration of eq. ccd3 (in its intermediates form) started from the MBPT2
 * amplitudes of eq. ccdGuess, with linear mixing, until the correlation energy
 * changes by less than a tolerance.
 *
 * Conventions
 *  - Energies are box totals in MeV (divide by N for E/N).
 *  - Plain C types only.  "Host" pointers are ordinary CPU memory owned by the
 *    caller; "device" pointers are GPU memory owned by the caller.
 *  - Every call returns a ccd_status; nothing aborts.  On failure the message
 *    of ccd_last_error() (thread-local) says why.
 *  - A context is used by one host thread at a time.  All device work of a
 *    context is ordered on the HIP stream given at creation (NULL = the default
 *    stream); calls that return numbers to the host synchronise that stream.
 *  - Amplitude layout ("canonical"): the direct channels of a problem in the
 *    order of ccd_export_maps(CCD_MAP_CHANNELS); each channel holds a row-major
 *    block [n_pp][n_hh] of t_ij^ab with (a<b) particle pairs as rows and (i<j)
 *    hole pairs as columns, pairs in the order of CCD_MAP_PP / CCD_MAP_HH.
 *    Only channels that hold at least one hole pair and one particle pair are
 *    present.  The other orderings follow from t_ij^ab = -t_ji^ab = -t_ij^ba.
 */
#ifndef CCD_H
#define CCD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CCD_OK = 0,
    CCD_NOT_CONVERGED = 1, /* max_iter sweeps done, some problem not converged */
    CCD_DIVERGED = 2,      /* a correlation energy became non-finite */
    CCD_EINVAL = -1,       /* bad argument (message in ccd_last_error) */
    CCD_ENOTMAGIC = -2,    /* N does not close a shell, or no particle states */
    CCD_ENOMEM = -3,       /* host allocation failed or workspace too small */
    CCD_EHIP = -4,         /* a HIP runtime call failed */
    CCD_ESTATE = -5        /* call out of order (e.g. iterate before a workspace is bound) */
} ccd_status;

/* One PNM problem (sec. "Single-particle basis for infinite matter" and
 * sec. "Two-body interaction").  The Minnesota triplet channel does not act
 * between two neutrons, so only its R and S channels are parameters.
 *
 * twist (the twist-averaging passage of sec. "Developing a CCD code for
 * infinite matter"): phi(x + L) = e^{i theta} phi(x) in each direction, so
 * k = (2 pi n + theta) / L; all zero is the periodic box, pi antiperiodic.
 * With a twist the states of the same basis are ordered by energy (key
 * |n|^2 + 2 n.theta/2pi in FP64, ties kept in the periodic order) and the
 * lowest N are holes; N must then be even, but need not close a shell. */
typedef struct {
    int32_t n_particles;  /* N: closed shell of the basis (2, 14, 38, 54, 66, 114, ...) */
    int32_t nmax2;        /* keep states with n_x^2+n_y^2+n_z^2 <= nmax2 */
    double density;       /* rho in fm^-3; box side L = (N/rho)^(1/3) */
    double hbar2_over_m;  /* MeV fm^2, e.g. 41.47 */
    double V_R, kappa_R;  /* repulsive Gaussian, e.g. 200 MeV, 1.487 fm^-2 */
    double V_S, kappa_S;  /* singlet Gaussian, e.g. -91.85 MeV, 0.465 fm^-2 */
    double twist[3];      /* theta_x, theta_y, theta_z in radians (finite) */
} ccd_problem;

/* Term bits of eq. ccd3 (all set = full CCD) */
#define CCD_T_PP     1u  /* 1/2 sum_cd <ab|v|cd> t_ij^cd                       */
#define CCD_T_HH     2u  /* 1/2 sum_kl <kl|v|ij> t_kl^ab                       */
#define CCD_T_RING   4u  /* P(ij|ab) sum_kc <kb|v|cj> t_ik^ac                  */
#define CCD_T_QHH    8u  /* 1/4 sum_klcd <kl|v|cd> t_ij^cd t_kl^ab             */
#define CCD_T_QRING 16u  /* P(ij) sum_klcd <kl|v|cd> t_ik^ac t_jl^bd           */
#define CCD_T_QHOLE 32u  /* -1/2 P(ij) sum_klcd <kl|v|cd> t_ik^dc t_lj^ab      */
#define CCD_T_QPART 64u  /* -1/2 P(ab) sum_klcd <kl|v|cd> t_lk^ac t_ij^db      */
#define CCD_T_ALL  127u

/* Precision of the channel contractions (ladders and ring).  Denominators,
 * the amplitude update, mixing and the energy are FP64 in every mode. */
#define CCD_PREC_FP64 0
#define CCD_PREC_FP32 1 /* FP32 operands, FP32 accumulation on MFMA */
#define CCD_PREC_BF16 2 /* BF16 operands, FP32 accumulation on MFMA */

typedef struct {
    double mixing;         /* alpha in (0, 1]: t <- alpha t_new + (1-alpha) t_old */
    double tol;            /* stop when |dE_n - dE_(n-1)| < tol (MeV, box total),
                              see also tol_rel */
    int32_t max_iter;      /* sweeps in this call (>= 1) */
    int32_t precision;     /* CCD_PREC_* for the sweeps of this call */
    int32_t refine_sweeps; /* mixed precision: after the mixed phase stops, at
                              least this many FP64 sweeps, then FP64 iteration
                              until |dE| < tol, within max_iter sweeps in total */
    uint32_t terms;        /* CCD_T_* mask; CCD_T_ALL for CCD */
    double mixed_tol;      /* mixed precision: the mixed phase stops when
                              |dE_n - dE_(n-1)| < mixed_tol (MeV); <= 0 means tol.
                              Rounding in BF16 keeps |dE| from falling far below
                              ~1e-4 |E|, so give BF16 a loose value. */
    int32_t check_every;   /* sweeps between host reads of the convergence flags
                              and energies (1..64; 0 = 1).  Problems that converge
                              inside a chunk stop there; the rest of the chunk
                              passes them over, so results do not depend on it. */
    int32_t use_graph;     /* nonzero: each chunk of sweeps is captured once as a
                              HIP graph and replayed (up to 4 captured shapes are
                              kept per context); ignored while kernel timing is on */
    double tol_rel;        /* relative part of the stop test: a problem stops when
                              |dE_n - dE_(n-1)| < tol + tol_rel |dE_n|; both <= 0
                              run exactly max_iter sweeps */
    int32_t stop_rule;     /* 0: the test above (the paper's).  1: additionally the
                              estimate of the remaining change of a linearly
                              converging iteration, |dE_n| r / (1 - r) with
                              r = |dE_n| / |dE_(n-1)|, must pass the same threshold
                              (and r < 1), in two consecutive sweeps; this bounds
                              the distance to the limit when a slow mode dominates
                              or E_n passes a turning point. */
} ccd_solver_opts;

typedef struct ccd_ctx ccd_ctx; /* opaque */

typedef struct {
    int32_t n_states, n_holes, n_particles_states;
    int32_t n_channels;      /* direct channels (K, S_z) in the amplitude layout */
    int32_t n_channels_sz0;  /* of which S_z = 0 (the only ones with nonzero <ab|v|ij>) */
    int32_t n_ph_channels;   /* particle-hole cross channels (Q, sigma) */
    int32_t max_hh, max_pp, max_ph;  /* largest block dimensions */
    int64_t n_amplitudes;    /* elements of the canonical amplitude vector */
    int32_t lut_size;        /* entries of the interaction table W(m), m = |dn|^2 */
    double box_L;            /* fm */
    double flops_pp;         /* flops of one sweep's pp ladder as executed:
                                the product over the momentum pairs {n_a, n_b}
                                of each S_z = 0 block (a quarter of the product
                                over spin pairs) */
    double flops_hh;         /* hh ladder + chi_klij contraction */
    double flops_ring;       /* both ring contractions */
    double flops_ordered;    /* the same three with ordered pairs, the paper's
                                unrestricted-index form */
} ccd_info;

/* Build the host plan of n_problems independent problems: model space and
 * hole filling (model-space loop of sec. "Developing a CCD code for infinite
 * matter"), Minnesota table W(m) and Fock energies (sec. "Two-body
 * interaction", normal-ordering section), direct channels T (quantum numbers
 * added) and particle-hole cross channels X (subtracted) with their pair lists
 * (channel discussion after the intermediates).  No GPU work and no device
 * memory: the GPU is first touched by ccd_bind_workspace.
 *   probs       host array of n_problems problems (n_problems >= 1)
 *   hip_stream  hipStream_t for all later device work (NULL = default stream)
 *   out         receives the new context; free with ccd_destroy.
 * Errors: CCD_EINVAL (bad sizes / parameters, blocks beyond the kernels'
 * limits), CCD_ENOTMAGIC, CCD_ENOMEM. */
ccd_status ccd_build_channels(const ccd_problem* probs, int32_t n_problems, void* hip_stream,
                              ccd_ctx** out);

/* Device bytes the context needs (all amplitudes, intermediates, tables). */
ccd_status ccd_workspace_size(const ccd_ctx* ctx, size_t* bytes);

/* Hand the context device memory of at least ccd_workspace_size bytes, owned
 * by the caller (e.g. a torch uint8 tensor) and kept alive until ccd_destroy.
 * Uploads the tables, then on the device builds <ab||ij>, the MBPT2 amplitudes
 * t0 = <ab||ij>/eps_ij^ab and the MBPT2 energy (eq. ccdGuess).  The library
 * itself allocates no device memory.  Errors: CCD_EINVAL (NULL / too small /
 * misaligned: 256-byte alignment required), CCD_EHIP, CCD_ESTATE (bound twice). */
ccd_status ccd_bind_workspace(ccd_ctx* ctx, void* device_ptr, size_t bytes);

/* Jacobi sweeps of eq. ccd3 in the intermediates form on the GPU (every term
 * from t^(n), linear mixing, energy of the mixed amplitudes), for all
 * problems of the context.  A problem whose |dE_n - dE_(n-1)| < tol + tol_rel |dE_n| stops
 * changing; the call returns when all problems have converged or after
 * max_iter sweeps.
 *   sweeps_done  host, n_problems entries (nullable): sweeps each problem ran in this call
 *   e_hist       host, n_problems * max_iter entries (nullable): correlation energy
 *                of problem p after its sweep s at e_hist[p*max_iter + s] (NaN
 *                after the problem stopped).  The device keeps the energies of the
 *                last 64 sweeps; the host collects them after every chunk.
 * Returns CCD_OK, CCD_NOT_CONVERGED (tol > 0 and a problem is still moving;
 * with tol <= 0 always CCD_OK), CCD_DIVERGED, CCD_EINVAL, CCD_ESTATE, CCD_EHIP. */
ccd_status ccd_iterate(ccd_ctx* ctx, const ccd_solver_opts* opts, int32_t* sweeps_done,
                       double* e_hist);

/* Launch shapes.  A context holds CCD_TUNE_LEN integer slots:
 *  - slots CCD_TUNE_DIRECT .. CCD_TUNE_UPDATE, one per kernel family: 0 = one
 *    workgroup per work item; m in {1, 2, 4} = a persistent grid of m
 *    workgroups per compute unit, each looping over the work items.
 *  - slots CCD_TUNE_RING_NW32 .. NW80, one per size bucket of the ring pair
 *    blocks (padded order 32, 48, 64, 80): 0 or 1 picks one of two waves-per-
 *    workgroup shapes (32: 4|2, 48: 9|3, 64: 16|8, 80: 16|9).
 * Shapes change speed only: every choice gives bit-identical results.
 * ccd_autotune times the candidates of each slot, one slot after another, on
 * the context's own problems: reps passes of the sweep's contractions and
 * update (forked streams included, since a shape that is faster alone can be
 * slower beside the kernels it shares the GPU with), after a warm pass, and
 * keeps a candidate only if it beats the current one by 2%; best_ms
 * (nullable, CCD_TUNE_LEN entries) receives each slot's best time per pass.
 * It recomputes the sweep's intermediates from the current amplitudes but does
 * not advance the iteration.  A fresh context has all slots 0. */
#define CCD_TUNE_DIRECT      0
#define CCD_TUNE_DCHI        1
#define CCD_TUNE_RING_SMALL  2
#define CCD_TUNE_RING        3
#define CCD_TUNE_LADDER      4
#define CCD_TUNE_UPDATE      5
#define CCD_TUNE_RING_NW32   6
#define CCD_TUNE_RING_NW48   7
#define CCD_TUNE_RING_NW64   8
#define CCD_TUNE_RING_NW80   9
#define CCD_TUNE_LEN        10
ccd_status ccd_autotune(ccd_ctx* ctx, int32_t precision, int32_t reps, double* best_ms);
ccd_status ccd_get_tuning(const ccd_ctx* ctx, int32_t* dst, int32_t n);
ccd_status ccd_set_tuning(ccd_ctx* ctx, const int32_t* src, int32_t n);

/* Energies of problem `problem` (MeV, box totals): E_ref, the MBPT2
 * correlation energy and the current correlation energy 1/4 sum <ij||ab> t
 * (eq. ccdcorr).  Synchronises the stream.  Any pointer may be NULL. */
ccd_status ccd_energy(const ccd_ctx* ctx, int32_t problem, double* e_ref, double* e_mbpt2,
                      double* e_corr);

/* Kinetic energy T = sum_i t_i of the Fermi sea of problem `problem` and the
 * first-order (Hartree-Fock) potential energy E_ref - T, box totals in MeV:
 * the two quantities the twist-averaging passage compares with infinite
 * matter.  Host data only (no GPU work).  Either pointer may be NULL. */
ccd_status ccd_reference_parts(const ccd_ctx* ctx, int32_t problem, double* kinetic, double* hf_potential);

/* Gauss-Legendre twist mesh of the twist-averaging algorithm: n points on
 * [0, pi] in each direction, n^3 twists theta[3k .. 3k+2] (x slowest, nodes
 * ascending) with weights weight[k] = w_x w_y w_z / pi^3, which sum to 1, so
 * that sum_k weight[k] E(theta_k) is the twist average.  Nodes by Newton's
 * method on the Legendre polynomial P_n.  n in [1, 64]; host buffers of 3 n^3
 * and n^3 doubles.  No GPU work.  Errors: CCD_EINVAL. */
ccd_status ccd_twist_mesh(int32_t n, double* theta, double* weight);

/* Weighted sums over all problems p of a context (e.g. one problem per twist,
 * weights from ccd_twist_mesh): out[0..4] = sum_p weight[p] (T, E_ref - T,
 * E_ref, MBPT2 correlation energy, current correlation energy).  weight: host,
 * n_problems finite doubles; out: host, 5 doubles.  Synchronises the stream.
 * Errors: CCD_EINVAL, CCD_ESTATE (no workspace), CCD_EHIP. */
ccd_status ccd_twist_average(const ccd_ctx* ctx, const double* weight, double* out);

/* Third-order MBPT energies (sec. "Developing a CCD code for infinite
 * matter", eqs. diag3-diag5): one Jacobi sweep of eq. ccd3 from the MBPT2
 * amplitudes with only linear terms and no mixing changes the correlation
 * energy by exactly the corresponding third-order diagrams, so for each of
 * the pp ladder (4), the hh ladder (5), the ring (3) and all three,
 * E3 = E(t1) - E_MBPT2.  out: host, 4 doubles per problem,
 * [n_problems][4] = (pp, hh, ring, total), box totals in MeV.  FP64.  Leaves
 * every problem at its MBPT2 amplitudes (as ccd_reset_amplitudes).
 * Synchronises the stream.  Errors: CCD_EINVAL, CCD_ESTATE, CCD_EHIP,
 * CCD_DIVERGED. */
ccd_status ccd_mbpt3(ccd_ctx* ctx, double* out);

/* Measured ceilings of the current GPU, for stating kernel rates against what
 * the part reaches rather than only its published peaks:
 *   out[0] HBM copy bandwidth, GB/s (read + write bytes; one half of dev_buf
 *          copied onto the other, five passes);
 *   out[1] FP64 MFMA 16x16x4, out[2] FP64 MFMA 4x4x4 (four blocks),
 *   out[3] FP32 MFMA 16x16x4, out[4] BF16 MFMA 16x16x32 (FP32 accumulation),
 *          TFLOP/s of resident loops (three workgroups of four waves per
 *          compute unit, four independent accumulators per wave).
 * dev_buf: caller-owned device memory, 256-byte aligned, at least 64 MiB (its
 * contents are overwritten); work on hip_stream (NULL = default), which is
 * synchronised.  No context needed.  Errors: CCD_EINVAL, CCD_EHIP. */
ccd_status ccd_measure_ceilings(void* dev_buf, size_t bytes, void* hip_stream, double* out);

/* Dense CCD for small model spaces given by their matrix elements, e.g. the
 * pairing model of eqs. sppairing / intpairing (sec. "Developing a CCD code
 * for infinite matter"): h[n] the one-body diagonal (canonical Hartree-Fock
 * basis), v[n^4] the antisymmetrised <pq||rs> at ((p n + q) n + r) n + s (host,
 * caller-owned), the lowest n_holes states are holes.  Fock energies
 * eps_p = h_p + sum_i <pi||pi> (eq. pairingsp), E_ref = sum_i h_i +
 * 1/2 sum_ij <ij||ij>, the MBPT2 start (eq. ccdGuess), then Jacobi sweeps of
 * eq. ccd3 with the terms opts->terms (all eight = CCD_T_ALL), linear mixing
 * opts->mixing, stop when |dE_n - dE_(n-1)| < tol + tol_rel |dE_n| (FP64; the
 * other options are ignored).  One GPU thread per ordered amplitude: cost
 * O(n_h^4 n_p^4) per sweep, a validation path, not the fast one.  2 <= n <= 48.
 * dev_work: ccd_dense_workspace_size bytes of caller-owned device memory,
 * 256-byte aligned.  Outputs are host pointers (nullable; e_hist: max_iter
 * doubles, NAN past the last sweep).  Synchronises hip_stream once per sweep.
 * Returns CCD_OK, CCD_NOT_CONVERGED, CCD_DIVERGED, CCD_EINVAL (also when a hole
 * is not below every particle in Fock energy), CCD_EHIP. */
ccd_status ccd_dense_workspace_size(int32_t n, int32_t n_holes, size_t* bytes);
ccd_status ccd_dense_solve(const double* h, const double* v, int32_t n, int32_t n_holes,
                           const ccd_solver_opts* opts, void* dev_work, size_t work_bytes, void* hip_stream,
                           double* e_ref, double* e_mbpt2, double* e_ccd, int32_t* sweeps, double* e_hist);

/* The same dense CCD for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid hipMalloc):
 * arguments and results as ccd_dense_solve, but the work area is a static
 * device array of CCD_DENSE_STATIC_BYTES that the library holds on every GPU
 * it runs on until the process ends.  No hipMalloc, hipFree or other
 * allocating call is made.  The work area is that of the current device
 * (hipGetDevice), which must be the device of hip_stream.  Every call on one
 * GPU uses the same array and leaves its contents there; each call writes
 * every byte it reads before reading it, so no clearing is needed, but calls
 * that overlap on one GPU (other host threads, other streams) race and must
 * be serialised by the caller.  Errors: as ccd_dense_solve, and CCD_EINVAL
 * when ccd_dense_workspace_size(n, n_holes) exceeds CCD_DENSE_STATIC_BYTES
 * (for example n = 28 with 4 holes fits; n = 40 does not). */
#define CCD_DENSE_STATIC_BYTES (8u << 20)
ccd_status ccd_dense_solve_static(const double* h, const double* v, int32_t n, int32_t n_holes,
                                  const ccd_solver_opts* opts, void* hip_stream, double* e_ref,
                                  double* e_mbpt2, double* e_ccd, int32_t* sweeps, double* e_hist);

/* Sizes and operation counts of problem `problem`. */
ccd_status ccd_problem_info(const ccd_ctx* ctx, int32_t problem, ccd_info* info);

/* Copy the canonical amplitude vector of a problem to / from host memory
 * (n = ccd_info.n_amplitudes doubles).  set also recomputes the energy and
 * makes the set amplitudes the current iterate (warm start, checkpoint
 * restore).  reset returns every problem to its MBPT2 amplitudes. */
ccd_status ccd_get_amplitudes(const ccd_ctx* ctx, int32_t problem, double* host_dst, size_t n);
ccd_status ccd_set_amplitudes(ccd_ctx* ctx, int32_t problem, const double* host_src, size_t n);
ccd_status ccd_reset_amplitudes(ccd_ctx* ctx);

/* Host copies of the plan's integer maps of a problem, for bit-exact tests.
 * Works without a GPU.  If dst is NULL or n is too small, only *n_needed is
 * written (and CCD_OK returned when dst is NULL, CCD_EINVAL otherwise). */
#define CCD_MAP_STATES   0 /* 4 per state: n_x, n_y, n_z, 2 s_z                         */
#define CCD_MAP_CHANNELS 1 /* 6 per direct channel: K_x, K_y, K_z, 2 S_z, n_hh, n_pp      */
#define CCD_MAP_HH       2 /* 2 per hole pair (i, j), channel after channel                */
#define CCD_MAP_PP       3 /* 2 per particle pair (a, b), channel after channel            */
#define CCD_MAP_PH_CHANNELS 4 /* 6 per cross channel: Q_x, Q_y, Q_z, 2 sigma, n, partner     */
#define CCD_MAP_PH       5 /* 2 per particle-hole pair (p, h), channel after channel       */
ccd_status ccd_export_maps(const ccd_ctx* ctx, int32_t problem, int32_t which, int32_t* dst,
                           size_t n, size_t* n_needed);

/* Host copies of a problem's single-particle tables: kinetic energies,
 * Fock energies (n_states each) and the interaction table W(m) (lut_size). */
ccd_status ccd_export_tables(const ccd_ctx* ctx, int32_t problem, double* tkin, double* eps,
                             double* w_table);

/* Per-kernel GPU timing with HIP events recorded on the context's stream.
 * While enabled every launch is bracketed by two events and the sweep runs on
 * the context's stream alone (no forked streams), so the times do not overlap;
 * ccd_kernel_times returns, per kernel family, the summed milliseconds and
 * launch counts since the last reset.  Families (ccd_kernel_name, in order):
 * init, direct (the chi_klij product items), dsum (their column sums), dchi
 * (one-body sums), ring_small, ring32, ring48, ring64, ring80 (the ring pair
 * blocks by padded order), ladder, update, energy.  ms and launches hold
 * ccd_kernel_families() entries.  Synchronises the stream. */
ccd_status ccd_set_timing(ccd_ctx* ctx, int32_t enabled);
int32_t ccd_kernel_families(void);
const char* ccd_kernel_name(int32_t family);
ccd_status ccd_kernel_times(ccd_ctx* ctx, double* ms, int64_t* launches, int32_t reset);

const char* ccd_last_error(void);
const char* ccd_version(void);
void ccd_destroy(ccd_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* CCD_H */
