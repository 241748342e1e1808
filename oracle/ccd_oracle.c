/*
 * ccd_oracle.c -- plain, slow, FP64 CPU oracle for the coupled-cluster doubles
 * (CCD) method of Lietz, Novario, Jansen, Hagen and Hjorth-Jensen,
 * "Computational Nuclear Physics and Post Hartree-Fock Methods"
 * (arXiv:1611.06765).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file: only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no code, header, table or constant generator with
 * the GPU path.
 *
 * Contents (each function cites the passage it follows):
 *   - nuclear matter model space: plane waves in a periodic box, spherical
 *     cutoff, spin, and for symmetric nuclear matter (SNM) isospin; holes =
 *     lowest A states; pure neutron matter (PNM) has neutrons only
 *                                                          (sec. "Single-particle
 *     basis for infinite matter"; the model-space loop of sec. "Developing a CCD
 *     code for infinite matter" with its extra isospin loop; Table 1's magic
 *     numbers doubled for SNM)
 *   - twisted boundary conditions: momenta k = (2 pi n + theta) / L, states
 *     ordered by energy and the lowest N filled for each twist  (the
 *     twist-averaging passage and its algorithm, sec. "Developing a CCD code
 *     for infinite matter")
 *   - Minnesota interaction from its operator form, with the spin- and
 *     isospin-exchange algebra evaluated as explicit 16x16 matrices in
 *     two-nucleon spin-isospin space and the Gaussian Fourier transform                         (sec. "Two-body
 *     interaction", Table "Parameters used to define the Minnesota interaction")
 *   - antisymmetrised elements <pq||rs> = <pq|v|rs> - <pq|v|sr>
 *   - Fock energies and reference energy                 (normal-ordering section)
 *   - O1: the iterative CCD equation (eq. ccd3) with all eight terms, written
 *     over dense four-index arrays indexed p*n^3+q*n^2+r*n+s, usable for any
 *     Hamiltonian given as dense arrays (pairing model, tiny PNM bases)
 *   - O3: the same iteration in the intermediates form (chi(b,c), chi(k,j),
 *     chi(kl,ij), chi(kb,cj)) for nuclear matter, where the fourth index of
 *     every amplitude and matrix element is deduced from momentum, spin and
 *     isospin conservation (elements that violate it are zero).
 *
 * Precision: IEEE binary64, fixed loop order, no fast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* term selection bits, shared meaning with the test-suite (eq. ccd3):
 *   PP      1/2 sum_cd <ab|v|cd> t_ij^cd
 *   HH      1/2 sum_kl <kl|v|ij> t_kl^ab
 *   RING    P(ij|ab) sum_kc <kb|v|cj> t_ik^ac
 *   Q_HH    1/4 sum_klcd <kl|v|cd> t_ij^cd t_kl^ab
 *   Q_RING  P(ij) sum_klcd <kl|v|cd> t_ik^ac t_jl^bd
 *   Q_HOLE  -1/2 P(ij) sum_klcd <kl|v|cd> t_ik^dc t_lj^ab
 *   Q_PART  -1/2 P(ab) sum_klcd <kl|v|cd> t_lk^ac t_ij^db                     */
#define T_PP 1u
#define T_HH 2u
#define T_RING 4u
#define T_QHH 8u
#define T_QRING 16u
#define T_QHOLE 32u
#define T_QPART 64u

/* ------------------------------------------------------------------------- */
/* PNM model space and interaction                                            */
/* ------------------------------------------------------------------------- */

typedef struct {
    int nmax2;     /* keep n_x^2+n_y^2+n_z^2 <= nmax2 */
    int nh;        /* number of neutrons = number of hole states */
    int ns;        /* number of single-particle states */
    int R;         /* floor(sqrt(nmax2)) */
    double rho, L, hb2m; /* density (fm^-3), box side (fm), hbar^2/m (MeV fm^2) */
    double theta[3];     /* twist angles (radians); 0 = periodic, pi = antiperiodic */
    int species;         /* 1: neutrons only (PNM); 2: protons and neutrons */
    double Va[3], ka[3]; /* Minnesota strengths / ranges, channels R, T, S */
    double Oa[3][16][16];/* spin-isospin operators of the three channels, two-nucleon basis */
    int *nx, *ny, *nz, *sz; /* sz = -1 or +1 (twice s_z) */
    int *tz;             /* twice t_z: -1 proton, +1 neutron */
    double *tkin;        /* kinetic energies */
    double *eps;         /* Fock energies */
    int *grid;           /* (n, s) -> state index or -1 */
    double *gcache[3];   /* exp cache per channel, indexed by |n_p-n_q-n_r+n_s|^2 */
    int mcache;
} orc_pnm;

static int isqrt_floor(int x) {
    int r = 0;
    while ((r + 1) * (r + 1) <= x) r++;
    return r;
}

/* internal state of one nucleon, c = 2 [s_z > 0] + [t_z > 0], and of two
 * nucleons, 4 c1 + c2 (16 states: spin and isospin of both) */
static int cint(int s, int t) { return 2 * (s > 0) + (t > 0); }
static int cidx(const void* hv, int p, int q);

static void mat16_mul(double a[16][16], double b[16][16], double c[16][16]) {
    double t[16][16];
    for (int i = 0; i < 16; i++)
        for (int j = 0; j < 16; j++) {
            double s = 0.0;
            for (int k = 0; k < 16; k++) s += a[i][k] * b[k][j];
            t[i][j] = s;
        }
    memcpy(c, t, sizeof(t));
}

/* Spin/isospin operator of the Minnesota potential (sec. "Two-body
 * interaction"):
 *   V = 1/2 ( V_R + 1/2(1+P_s) V_T + 1/2(1-P_s) V_S ) (1 - P_s P_t).
 * P_s swaps the spins of the two nucleons, P_t their isospins.  Both are built
 * as explicit 16x16 permutation matrices on |s1 t1, s2 t2>, and each channel's
 * operator as a product of such matrices.  Between two neutrons P_t acts as
 * +1, which leaves only the spin singlet in the R and S channels and nothing
 * in the T channel. */
static void build_spin_operators(orc_pnm* h) {
    double one[16][16] = {{0}}, Ps[16][16] = {{0}}, Pt[16][16] = {{0}};
    for (int i = 0; i < 16; i++) one[i][i] = 1.0;
    for (int s1 = -1; s1 <= 1; s1 += 2)
        for (int t1 = -1; t1 <= 1; t1 += 2)
            for (int s2 = -1; s2 <= 1; s2 += 2)
                for (int t2 = -1; t2 <= 1; t2 += 2) {
                    int ket = 4 * cint(s1, t1) + cint(s2, t2);
                    Ps[4 * cint(s2, t1) + cint(s1, t2)][ket] = 1.0;
                    Pt[4 * cint(s1, t2) + cint(s2, t1)][ket] = 1.0;
                }
    double PsPt[16][16], ex[16][16], plus[16][16], minus[16][16], tmp[16][16];
    mat16_mul(Ps, Pt, PsPt);
    for (int i = 0; i < 16; i++)
        for (int j = 0; j < 16; j++) {
            ex[i][j] = one[i][j] - PsPt[i][j];
            plus[i][j] = 0.5 * (one[i][j] + Ps[i][j]);
            minus[i][j] = 0.5 * (one[i][j] - Ps[i][j]);
        }
    /* R: 1/2 * (1 - P_s P_t) */
    for (int i = 0; i < 16; i++)
        for (int j = 0; j < 16; j++) h->Oa[0][i][j] = 0.5 * ex[i][j];
    /* T: 1/2 * 1/2(1+P_s) * (1 - P_s P_t) */
    mat16_mul(plus, ex, tmp);
    for (int i = 0; i < 16; i++)
        for (int j = 0; j < 16; j++) h->Oa[1][i][j] = 0.5 * tmp[i][j];
    /* S: 1/2 * 1/2(1-P_s) * (1 - P_s P_t) */
    mat16_mul(minus, ex, tmp);
    for (int i = 0; i < 16; i++)
        for (int j = 0; j < 16; j++) h->Oa[2][i][j] = 0.5 * tmp[i][j];
}

static int grid_slot(const orc_pnm* h, int x, int y, int z, int s, int t) {
    int R = h->R, W = 2 * R + 1;
    return (((((x + R) * W) + (y + R)) * W + (z + R)) * 2 + (s > 0)) * 2 + (t > 0);
}

static int grid_index(const orc_pnm* h, int x, int y, int z, int s, int t) {
    int R = h->R;
    if (x < -R || x > R || y < -R || y > R || z < -R || z > R) return -1;
    if ((s != -1 && s != 1) || (t != -1 && t != 1)) return -1;
    return h->grid[grid_slot(h, x, y, z, s, t)];
}

static int cidx(const void* hv, int p, int q) {
    const orc_pnm* h = (const orc_pnm*)hv;
    return 4 * cint(h->sz[p], h->tz[p]) + cint(h->sz[q], h->tz[q]);
}

void orc_pnm_free(orc_pnm* h) {
    if (!h) return;
    free(h->nx); free(h->ny); free(h->nz); free(h->sz); free(h->tz);
    free(h->tkin); free(h->eps); free(h->grid);
    for (int a = 0; a < 3; a++) free(h->gcache[a]);
    free(h);
}

double orc_pnm_vas_direct(const orc_pnm* h, int p, int q, int r, int s);

/* Model space: the loop over shells, then n_x, n_y, n_z, then s_z = -1/2, +1/2,
 * of sec. "Developing a CCD code for infinite matter", with the extra innermost
 * loop over isospin (t_z = -1/2 proton, +1/2 neutron) that the passage asks for
 * symmetric nuclear matter; pure neutron matter has neutrons only.  Box side
 * from rho = A / L^3 (A = all nucleons), momenta k = (2 pi n + theta) / L,
 * kinetic energy hbar^2 k^2 / 2m with one mass for both species (sec.
 * "Single-particle basis for infinite matter" and the twist-averaging
 * passage).  The states are then ordered by single-particle energy and the
 * first A are holes ("Order States by Energy and Fill Holes").  The order is
 * decided on the exact-shaped key |n|^2 + 2 n.phi, phi = theta/2pi (the
 * kinetic energy is (hbar^2/2m)(2pi/L)^2 (key + |phi|^2)), evaluated in FP64
 * left to right; equal keys keep the loop order.  Without a twist the key is
 * the integer shell, so the loop order is kept as it is, and with both species
 * the first A states fill whole momenta with all four spin-isospin states.
 * Returns NULL if A leaves no particle states, if A is not a multiple of the
 * 2 species spins, or, without a twist and unless open_ok, if A does not close
 * a shell. */
static orc_pnm* nm_build(int nmax2, int nparticles, int species, double rho, double hb2m,
                         double VR, double kR, double VT, double kT, double VS, double kS,
                         double thx, double thy, double thz, int open_ok) {
    if (nmax2 < 0 || nparticles <= 0 || rho <= 0.0 || (species != 1 && species != 2)) return NULL;
    if (species == 1 && (nparticles & 1)) return NULL;
    orc_pnm* h = (orc_pnm*)calloc(1, sizeof(orc_pnm));
    h->nmax2 = nmax2;
    h->nh = nparticles;
    h->species = species;
    h->rho = rho;
    h->hb2m = hb2m;
    h->theta[0] = thx; h->theta[1] = thy; h->theta[2] = thz;
    const int twisted = thx != 0.0 || thy != 0.0 || thz != 0.0;
    h->Va[0] = VR; h->ka[0] = kR;
    h->Va[1] = VT; h->ka[1] = kT;
    h->Va[2] = VS; h->ka[2] = kS;
    h->L = cbrt((double)nparticles / rho);
    int R = isqrt_floor(nmax2);
    h->R = R;
    int cap = (2 * R + 1) * (2 * R + 1) * (2 * R + 1) * 4;
    h->nx = (int*)malloc(sizeof(int) * cap);
    h->ny = (int*)malloc(sizeof(int) * cap);
    h->nz = (int*)malloc(sizeof(int) * cap);
    h->sz = (int*)malloc(sizeof(int) * cap);
    h->tz = (int*)malloc(sizeof(int) * cap);
    h->grid = (int*)malloc(sizeof(int) * cap);
    for (int i = 0; i < cap; i++) h->grid[i] = -1;
    int n = 0;
    for (int shell = 0; shell <= nmax2; shell++)
        for (int x = -R; x <= R; x++)
            for (int y = -R; y <= R; y++)
                for (int z = -R; z <= R; z++)
                    for (int s = -1; s <= 1; s += 2)
                        for (int t = (species == 2 ? -1 : 1); t <= 1; t += 2)
                            if (x * x + y * y + z * z == shell) {
                                h->nx[n] = x; h->ny[n] = y; h->nz[n] = z; h->sz[n] = s; h->tz[n] = t;
                                n++;
                            }
    h->ns = n;
    if (nparticles >= n) { orc_pnm_free(h); return NULL; }
    /* order by energy: insertion sort on the key, stable */
    {
        const double phx = thx / (2.0 * M_PI), phy = thy / (2.0 * M_PI), phz = thz / (2.0 * M_PI);
        double* key = (double*)malloc(sizeof(double) * n);
        for (int p = 0; p < n; p++) {
            int n2 = h->nx[p] * h->nx[p] + h->ny[p] * h->ny[p] + h->nz[p] * h->nz[p];
            key[p] = (double)n2 + 2.0 * ((double)h->nx[p] * phx + (double)h->ny[p] * phy + (double)h->nz[p] * phz);
        }
        for (int p = 1; p < n; p++) {
            double k = key[p];
            int x = h->nx[p], y = h->ny[p], z = h->nz[p], s = h->sz[p], t = h->tz[p];
            int q = p - 1;
            while (q >= 0 && key[q] > k) {
                key[q + 1] = key[q];
                h->nx[q + 1] = h->nx[q]; h->ny[q + 1] = h->ny[q]; h->nz[q + 1] = h->nz[q];
                h->sz[q + 1] = h->sz[q]; h->tz[q + 1] = h->tz[q];
                q--;
            }
            key[q + 1] = k;
            h->nx[q + 1] = x; h->ny[q + 1] = y; h->nz[q + 1] = z; h->sz[q + 1] = s; h->tz[q + 1] = t;
        }
        free(key);
    }
    for (int p = 0; p < n; p++) h->grid[grid_slot(h, h->nx[p], h->ny[p], h->nz[p], h->sz[p], h->tz[p])] = p;
    /* periodic box: closed shell, i.e. last hole and first particle lie in
     * different shells */
    if (!twisted && !open_ok) {
        int a = nparticles - 1, b = nparticles;
        int sa = h->nx[a] * h->nx[a] + h->ny[a] * h->ny[a] + h->nz[a] * h->nz[a];
        int sb = h->nx[b] * h->nx[b] + h->ny[b] * h->ny[b] + h->nz[b] * h->nz[b];
        if (sa == sb) { orc_pnm_free(h); return NULL; }
    }
    build_spin_operators(h);
    h->tkin = (double*)malloc(sizeof(double) * n);
    for (int p = 0; p < n; p++) {
        double kx = (2.0 * M_PI * h->nx[p] + thx) / h->L;
        double ky = (2.0 * M_PI * h->ny[p] + thy) / h->L;
        double kz = (2.0 * M_PI * h->nz[p] + thz) / h->L;
        h->tkin[p] = 0.5 * hb2m * (kx * kx + ky * ky + kz * kz);
    }
    /* exp cache for the fast element used by O3: index m = |n_p-n_q-n_r+n_s|^2
     * (the twist cancels in that combination of momenta) */
    h->mcache = 16 * 3 * R * R + 1;
    for (int a = 0; a < 3; a++) {
        h->gcache[a] = (double*)malloc(sizeof(double) * h->mcache);
        for (int m = 0; m < h->mcache; m++) {
            double q2 = (M_PI / h->L) * (M_PI / h->L) * (double)m; /* q = (pi/L) * vec */
            h->gcache[a][m] = h->Va[a] / (h->L * h->L * h->L) *
                              pow(M_PI / h->ka[a], 1.5) * exp(-q2 / (4.0 * h->ka[a]));
        }
    }
    /* Fock energies: f_pp = t_p + sum_i <pi||pi> (normal-ordering section) */
    h->eps = (double*)malloc(sizeof(double) * n);
    for (int p = 0; p < n; p++) {
        double s = h->tkin[p];
        for (int i = 0; i < h->nh; i++) s += orc_pnm_vas_direct(h, p, i, p, i);
        h->eps[p] = s;
    }
    return h;
}

/* pure neutron matter, periodic or twisted */
orc_pnm* orc_pnm_new_twist(int nmax2, int nparticles, double rho, double hb2m,
                           double VR, double kR, double VT, double kT, double VS, double kS,
                           double thx, double thy, double thz) {
    return nm_build(nmax2, nparticles, 1, rho, hb2m, VR, kR, VT, kT, VS, kS, thx, thy, thz, 0);
}

/* nuclear matter: species = 1 (neutrons) or 2 (protons and neutrons, A/2
 * of each when A fills whole momenta), periodic box; open_ok accepts an A
 * that does not close a shell (small exact test systems) */
orc_pnm* orc_nm_new(int nmax2, int nparticles, int species, double rho, double hb2m,
                    double VR, double kR, double VT, double kT, double VS, double kS, int open_ok) {
    return nm_build(nmax2, nparticles, species, rho, hb2m, VR, kR, VT, kT, VS, kS, 0.0, 0.0, 0.0, open_ok);
}

/* periodic boundary conditions: no twist */
orc_pnm* orc_pnm_new(int nmax2, int nparticles, double rho, double hb2m,
                     double VR, double kR, double VT, double kT, double VS, double kS) {
    return orc_pnm_new_twist(nmax2, nparticles, rho, hb2m, VR, kR, VT, kT, VS, kS, 0.0, 0.0, 0.0);
}

/* Non-antisymmetrised element <pq|v|rs> of the Minnesota interaction:
 * V_a/L^3 (pi/kappa_a)^{3/2} exp(-q^2 / 4 kappa_a) delta_{k_p+k_q, k_r+k_s}
 * with q = (k_p - k_q - k_r + k_s)/2, times the spin-isospin matrix element of
 * each channel's operator (sec. "Two-body interaction"). */
static double kmom(const orc_pnm* h, int n, int d) { return (2.0 * M_PI * n + h->theta[d]) / h->L; }

static double v_direct(const orc_pnm* h, int p, int q, int r, int s) {
    /* k_p + k_q = k_r + k_s: the twists of both sides are equal */
    if (h->nx[p] + h->nx[q] != h->nx[r] + h->nx[s]) return 0.0;
    if (h->ny[p] + h->ny[q] != h->ny[r] + h->ny[s]) return 0.0;
    if (h->nz[p] + h->nz[q] != h->nz[r] + h->nz[s]) return 0.0;
    double qx = 0.5 * (kmom(h, h->nx[p], 0) - kmom(h, h->nx[q], 0) - kmom(h, h->nx[r], 0) + kmom(h, h->nx[s], 0));
    double qy = 0.5 * (kmom(h, h->ny[p], 1) - kmom(h, h->ny[q], 1) - kmom(h, h->ny[r], 1) + kmom(h, h->ny[s], 1));
    double qz = 0.5 * (kmom(h, h->nz[p], 2) - kmom(h, h->nz[q], 2) - kmom(h, h->nz[r], 2) + kmom(h, h->nz[s], 2));
    double q2 = qx * qx + qy * qy + qz * qz;
    double L3 = h->L * h->L * h->L;
    int bra = cidx(h, p, q), ket = cidx(h, r, s);
    double v = 0.0;
    for (int a = 0; a < 3; a++) {
        double spin = h->Oa[a][bra][ket];
        if (spin == 0.0) continue;
        v += h->Va[a] / L3 * pow(M_PI / h->ka[a], 1.5) * exp(-q2 / (4.0 * h->ka[a])) * spin;
    }
    return v;
}

/* Antisymmetrised element <pq||rs> = <pq|v|rs> - <pq|v|sr>. */
double orc_pnm_vas_direct(const orc_pnm* h, int p, int q, int r, int s) {
    return v_direct(h, p, q, r, s) - v_direct(h, p, q, s, r);
}

/* Same value, for callers that guarantee momentum conservation, with the
 * Gaussian factors read from the per-|2q|^2 cache built in orc_pnm_new. */
static inline double vas_fast(const orc_pnm* h, int p, int q, int r, int s) {
    int bra = cidx(h, p, q);
    int k1 = cidx(h, r, s), k2 = cidx(h, s, r);
    int dx = h->nx[p] - h->nx[q] - h->nx[r] + h->nx[s];
    int dy = h->ny[p] - h->ny[q] - h->ny[r] + h->ny[s];
    int dz = h->nz[p] - h->nz[q] - h->nz[r] + h->nz[s];
    int m1 = dx * dx + dy * dy + dz * dz;
    dx = h->nx[p] - h->nx[q] - h->nx[s] + h->nx[r];
    dy = h->ny[p] - h->ny[q] - h->ny[s] + h->ny[r];
    dz = h->nz[p] - h->nz[q] - h->nz[s] + h->nz[r];
    int m2 = dx * dx + dy * dy + dz * dz;
    double v = 0.0;
    for (int a = 0; a < 3; a++) {
        double s1 = h->Oa[a][bra][k1], s2 = h->Oa[a][bra][k2];
        if (s1 != 0.0) v += h->gcache[a][m1] * s1;
        if (s2 != 0.0) v -= h->gcache[a][m2] * s2;
    }
    return v;
}

double orc_pnm_vas_fast(const orc_pnm* h, int p, int q, int r, int s) {
    if (h->nx[p] + h->nx[q] != h->nx[r] + h->nx[s]) return 0.0;
    if (h->ny[p] + h->ny[q] != h->ny[r] + h->ny[s]) return 0.0;
    if (h->nz[p] + h->nz[q] != h->nz[r] + h->nz[s]) return 0.0;
    return vas_fast(h, p, q, r, s);
}

int orc_pnm_nstates(const orc_pnm* h) { return h->ns; }
double orc_pnm_L(const orc_pnm* h) { return h->L; }

void orc_pnm_states(const orc_pnm* h, int* nx, int* ny, int* nz, int* sz) {
    for (int p = 0; p < h->ns; p++) {
        nx[p] = h->nx[p]; ny[p] = h->ny[p]; nz[p] = h->nz[p]; sz[p] = h->sz[p];
    }
}

void orc_pnm_isospins(const orc_pnm* h, int* tz) {
    for (int p = 0; p < h->ns; p++) tz[p] = h->tz[p];
}
int orc_pnm_species(const orc_pnm* h) { return h->species; }

void orc_pnm_kinetic(const orc_pnm* h, double* out) { memcpy(out, h->tkin, sizeof(double) * h->ns); }
void orc_pnm_fock(const orc_pnm* h, double* out) { memcpy(out, h->eps, sizeof(double) * h->ns); }

/* E_Ref = sum_i <i|t|i> + 1/2 sum_ij <ij||ij> (normal-ordering section). */
double orc_pnm_eref(const orc_pnm* h) {
    double e = 0.0;
    for (int i = 0; i < h->nh; i++) e += h->tkin[i];
    double v = 0.0;
    for (int i = 0; i < h->nh; i++)
        for (int j = 0; j < h->nh; j++) v += orc_pnm_vas_direct(h, i, j, i, j);
    return e + 0.5 * v;
}

/* Dense n^4 array of <pq||rs>, index p n^3 + q n^2 + r n + s (tiny bases). */
void orc_pnm_dense_v(const orc_pnm* h, double* out) {
    int n = h->ns;
    for (int p = 0; p < n; p++)
        for (int q = 0; q < n; q++)
            for (int r = 0; r < n; r++)
                for (int s = 0; s < n; s++)
                    out[(((size_t)p * n + q) * n + r) * n + s] = orc_pnm_vas_direct(h, p, q, r, s);
}

/* ------------------------------------------------------------------------- */
/* O1: eq. ccd3 verbatim over dense four-index arrays                          */
/* ------------------------------------------------------------------------- */

typedef struct {
    int n, nh;
    double *v;    /* <pq||rs>, dense */
    double *eps;  /* Fock energies f_pp = h_pp + sum_i <pi||pi> */
    double *t, *tnew;
    double eref, emp2, ecorr;
} orc_o1;

#define IDX4(n, p, q, r, s) ((((size_t)(p) * (n) + (q)) * (n) + (r)) * (n) + (s))

/* Correlation energy 1/4 sum_ijab <ij||ab> t_ij^ab (eq. ccdcorr). */
static double o1_energy(const orc_o1* o, const double* t) {
    int n = o->n, nh = o->nh;
    double e = 0.0;
    for (int i = 0; i < nh; i++)
        for (int j = 0; j < nh; j++)
            for (int a = nh; a < n; a++)
                for (int b = nh; b < n; b++)
                    e += o->v[IDX4(n, i, j, a, b)] * t[IDX4(n, a, b, i, j)];
    return 0.25 * e;
}

void orc_o1_free(orc_o1* o) {
    if (!o) return;
    free(o->v); free(o->eps); free(o->t); free(o->tnew); free(o);
}

/* Set-up: Fock energies (eq. pairingsp / normal-ordering section), reference
 * energy, and the MBPT2 start t^(0) = <ab||ij> / eps_ij^ab (eq. ccdGuess). */
orc_o1* orc_o1_new(int n, int nh, const double* hdiag, const double* v) {
    orc_o1* o = (orc_o1*)calloc(1, sizeof(orc_o1));
    o->n = n; o->nh = nh;
    size_t n4 = (size_t)n * n * n * n;
    o->v = (double*)malloc(sizeof(double) * n4);
    memcpy(o->v, v, sizeof(double) * n4);
    o->eps = (double*)malloc(sizeof(double) * n);
    for (int p = 0; p < n; p++) {
        double s = hdiag[p];
        for (int i = 0; i < nh; i++) s += v[IDX4(n, p, i, p, i)];
        o->eps[p] = s;
    }
    double e = 0.0;
    for (int i = 0; i < nh; i++) e += hdiag[i];
    double w = 0.0;
    for (int i = 0; i < nh; i++)
        for (int j = 0; j < nh; j++) w += v[IDX4(n, i, j, i, j)];
    o->eref = e + 0.5 * w;
    o->t = (double*)calloc(n4, sizeof(double));
    o->tnew = (double*)calloc(n4, sizeof(double));
    for (int i = 0; i < nh; i++)
        for (int j = 0; j < nh; j++)
            for (int a = nh; a < n; a++)
                for (int b = nh; b < n; b++) {
                    double d = o->eps[i] + o->eps[j] - o->eps[a] - o->eps[b];
                    o->t[IDX4(n, a, b, i, j)] = v[IDX4(n, a, b, i, j)] / d;
                }
    o->emp2 = o1_energy(o, o->t);
    o->ecorr = o->emp2;
    return o;
}

double orc_o1_eref(const orc_o1* o) { return o->eref; }
double orc_o1_emp2(const orc_o1* o) { return o->emp2; }
double orc_o1_ecorr(const orc_o1* o) { return o->ecorr; }
void orc_o1_eps(const orc_o1* o, double* out) { memcpy(out, o->eps, sizeof(double) * o->n); }
double orc_o1_t(const orc_o1* o, int a, int b, int i, int j) { return o->t[IDX4(o->n, a, b, i, j)]; }

/* One Jacobi sweep of eq. ccd3: every term from t^(n); t_new = RHS/eps_ij^ab,
 * then linear mixing t^(n+1) = alpha t_new + (1-alpha) t^(n) (sec. "Approximations
 * to the full CCD equations"), and the energy of the mixed amplitudes.  All
 * i, j, a, b are visited (unrestricted indices).  Inner loops skip a term as
 * soon as a factor is exactly zero.  Returns the new correlation energy. */
double orc_o1_sweep(orc_o1* o, double alpha, unsigned mask) {
    int n = o->n, nh = o->nh;
    const double* v = o->v;
    const double* t = o->t;
#define V(p, q, r, s) v[IDX4(n, p, q, r, s)]
#define T(a, b, i, j) t[IDX4(n, a, b, i, j)]
#pragma omp parallel for collapse(2) schedule(dynamic)
    for (int i = 0; i < nh; i++)
        for (int j = 0; j < nh; j++)
            for (int a = nh; a < n; a++)
                for (int b = nh; b < n; b++) {
                    double sum = V(a, b, i, j);
                    if (mask & T_PP) {
                        double s = 0.0;
                        for (int c = nh; c < n; c++)
                            for (int d = nh; d < n; d++) {
                                double x = T(c, d, i, j);
                                if (x != 0.0) s += V(a, b, c, d) * x;
                            }
                        sum += 0.5 * s;
                    }
                    if (mask & T_HH) {
                        double s = 0.0;
                        for (int k = 0; k < nh; k++)
                            for (int l = 0; l < nh; l++) {
                                double x = T(a, b, k, l);
                                if (x != 0.0) s += V(k, l, i, j) * x;
                            }
                        sum += 0.5 * s;
                    }
                    if (mask & T_RING) {
                        /* P(ij|ab) f(i,j,a,b), f = sum_kc <kb||cj> t_ik^ac */
                        double s = 0.0;
                        for (int k = 0; k < nh; k++)
                            for (int c = nh; c < n; c++) {
                                double f1 = T(a, c, i, k), f2 = T(a, c, j, k);
                                double f3 = T(b, c, i, k), f4 = T(b, c, j, k);
                                if (f1 != 0.0) s += V(k, b, c, j) * f1;
                                if (f2 != 0.0) s -= V(k, b, c, i) * f2;
                                if (f3 != 0.0) s -= V(k, a, c, j) * f3;
                                if (f4 != 0.0) s += V(k, a, c, i) * f4;
                            }
                        sum += s;
                    }
                    if (mask & T_QHH) {
                        double s = 0.0;
                        for (int c = nh; c < n; c++)
                            for (int d = nh; d < n; d++) {
                                double x = T(c, d, i, j);
                                if (x == 0.0) continue;
                                for (int k = 0; k < nh; k++)
                                    for (int l = 0; l < nh; l++) {
                                        double y = T(a, b, k, l);
                                        if (y != 0.0) s += V(k, l, c, d) * x * y;
                                    }
                            }
                        sum += 0.25 * s;
                    }
                    if (mask & T_QRING) {
                        /* P(ij) g(i,j), g = sum_klcd <kl||cd> t_ik^ac t_jl^bd */
                        double s = 0.0;
                        for (int k = 0; k < nh; k++)
                            for (int c = nh; c < n; c++) {
                                double x1 = T(a, c, i, k), x2 = T(a, c, j, k);
                                if (x1 == 0.0 && x2 == 0.0) continue;
                                for (int l = 0; l < nh; l++)
                                    for (int d = nh; d < n; d++) {
                                        double vv = V(k, l, c, d);
                                        if (vv == 0.0) continue;
                                        s += vv * (x1 * T(b, d, j, l) - x2 * T(b, d, i, l));
                                    }
                            }
                        sum += s;
                    }
                    if (mask & T_QHOLE) {
                        /* -1/2 P(ij) h(i,j), h = sum_klcd <kl||cd> t_ik^dc t_lj^ab */
                        double s = 0.0;
                        for (int l = 0; l < nh; l++) {
                            double y1 = T(a, b, l, j), y2 = T(a, b, l, i);
                            if (y1 == 0.0 && y2 == 0.0) continue;
                            double u1 = 0.0, u2 = 0.0;
                            for (int k = 0; k < nh; k++)
                                for (int c = nh; c < n; c++)
                                    for (int d = nh; d < n; d++) {
                                        double vv = V(k, l, c, d);
                                        if (vv == 0.0) continue;
                                        u1 += vv * T(d, c, i, k);
                                        u2 += vv * T(d, c, j, k);
                                    }
                            s += u1 * y1 - u2 * y2;
                        }
                        sum += -0.5 * s;
                    }
                    if (mask & T_QPART) {
                        /* -1/2 P(ab) p(a,b), p = sum_klcd <kl||cd> t_lk^ac t_ij^db */
                        double s = 0.0;
                        for (int d = nh; d < n; d++) {
                            double y1 = T(d, b, i, j), y2 = T(d, a, i, j);
                            if (y1 == 0.0 && y2 == 0.0) continue;
                            double u1 = 0.0, u2 = 0.0;
                            for (int k = 0; k < nh; k++)
                                for (int l = 0; l < nh; l++)
                                    for (int c = nh; c < n; c++) {
                                        double vv = V(k, l, c, d);
                                        if (vv == 0.0) continue;
                                        u1 += vv * T(a, c, l, k);
                                        u2 += vv * T(b, c, l, k);
                                    }
                            s += u1 * y1 - u2 * y2;
                        }
                        sum += -0.5 * s;
                    }
                    double den = o->eps[i] + o->eps[j] - o->eps[a] - o->eps[b];
                    double tn = sum / den;
                    o->tnew[IDX4(n, a, b, i, j)] = alpha * tn + (1.0 - alpha) * T(a, b, i, j);
                }
#undef V
#undef T
    double* sw = o->t; o->t = o->tnew; o->tnew = sw;
    o->ecorr = o1_energy(o, o->t);
    return o->ecorr;
}

/* ------------------------------------------------------------------------- */
/* O3: PNM CCD in the intermediates form, fourth index deduced                */
/* ------------------------------------------------------------------------- */

typedef struct {
    const orc_pnm* h;
    int nh, np, ns;
    /* amplitudes t_ij^ab stored at [i][j][a-nh]; b is deduced from momentum and
     * spin conservation (bidx), -1 if b is not a particle state of the basis. */
    int* bidx;      /* nh*nh*np */
    double *t, *tnew, *vt;  /* vt = <ab||ij> */
    double *dchi;   /* one-body intermediates per state (diagonal) */
    double *chh;    /* chi_klij at [k][l][i] (j deduced) */
    int* jidx;      /* j for [k][l][i], -1 if not a hole */
    double* cph;    /* chi_kbcj at [k][b-nh][j] (c deduced) */
    int* cidx;      /* c for [k][b][j], -1 if not a particle */
    double eref, emp2, ecorr;
} orc_o3;

static int partner(const orc_pnm* h, int p, int q, int r) {
    /* state s with n_s = n_p + n_q - n_r, s_s = s_p + s_q - s_r, t_s = t_p + t_q - t_r */
    int x = h->nx[p] + h->nx[q] - h->nx[r];
    int y = h->ny[p] + h->ny[q] - h->ny[r];
    int z = h->nz[p] + h->nz[q] - h->nz[r];
    int s = h->sz[p] + h->sz[q] - h->sz[r];
    int t = h->tz[p] + h->tz[q] - h->tz[r];
    return grid_index(h, x, y, z, s, t);
}

#define O3I(o, i, j, a) (((size_t)(i) * (o)->nh + (j)) * (o)->np + ((a) - (o)->nh))

static double o3_energy(const orc_o3* o, const double* t) {
    double e = 0.0;
    for (size_t x = 0; x < (size_t)o->nh * o->nh * o->np; x++)
        if (o->bidx[x] >= 0) e += o->vt[x] * t[x];
    return 0.25 * e;
}

void orc_o3_free(orc_o3* o) {
    if (!o) return;
    free(o->bidx); free(o->t); free(o->tnew); free(o->vt); free(o->dchi);
    free(o->chh); free(o->jidx); free(o->cph); free(o->cidx); free(o);
}

/* Set-up and MBPT2 start (eq. ccdGuess); E_MBPT2 = 1/4 sum v t^(0). */
orc_o3* orc_o3_new(const orc_pnm* h) {
    orc_o3* o = (orc_o3*)calloc(1, sizeof(orc_o3));
    o->h = h;
    o->nh = h->nh; o->ns = h->ns; o->np = h->ns - h->nh;
    int nh = o->nh, np = o->np;
    size_t nt = (size_t)nh * nh * np;
    o->bidx = (int*)malloc(sizeof(int) * nt);
    o->t = (double*)calloc(nt, sizeof(double));
    o->tnew = (double*)calloc(nt, sizeof(double));
    o->vt = (double*)calloc(nt, sizeof(double));
    o->dchi = (double*)calloc(h->ns, sizeof(double));
    o->chh = (double*)calloc((size_t)nh * nh * nh, sizeof(double));
    o->jidx = (int*)malloc(sizeof(int) * (size_t)nh * nh * nh);
    o->cph = (double*)calloc((size_t)nh * np * nh, sizeof(double));
    o->cidx = (int*)malloc(sizeof(int) * (size_t)nh * np * nh);
    for (int i = 0; i < nh; i++)
        for (int j = 0; j < nh; j++)
            for (int a = nh; a < h->ns; a++) {
                size_t x = O3I(o, i, j, a);
                int b = partner(h, i, j, a);
                if (b < nh || i == j || a == b) b = -1;
                o->bidx[x] = b;
                if (b >= 0) {
                    o->vt[x] = orc_pnm_vas_direct(h, a, b, i, j);
                    double d = h->eps[i] + h->eps[j] - h->eps[a] - h->eps[b];
                    o->t[x] = o->vt[x] / d;
                }
            }
    for (int k = 0; k < nh; k++)
        for (int l = 0; l < nh; l++)
            for (int i = 0; i < nh; i++) {
                int j = partner(h, k, l, i);
                if (j < 0 || j >= nh) j = -1;
                o->jidx[((size_t)k * nh + l) * nh + i] = j;
            }
    for (int k = 0; k < nh; k++)
        for (int b = nh; b < h->ns; b++)
            for (int j = 0; j < nh; j++) {
                int c = partner(h, k, b, j);
                if (c < nh) c = -1;
                o->cidx[((size_t)k * np + (b - nh)) * nh + j] = c;
            }
    o->eref = orc_pnm_eref(h);
    o->emp2 = o3_energy(o, o->t);
    o->ecorr = o->emp2;
    return o;
}

double orc_o3_eref(const orc_o3* o) { return o->eref; }
double orc_o3_emp2(const orc_o3* o) { return o->emp2; }
double orc_o3_ecorr(const orc_o3* o) { return o->ecorr; }

/* t_ij^ab for arbitrary states; 0 when the element violates conservation */
double orc_o3_t(const orc_o3* o, int a, int b, int i, int j) {
    if (i < 0 || j < 0 || i >= o->nh || j >= o->nh || a < o->nh || b < o->nh) return 0.0;
    size_t x = O3I(o, i, j, a);
    return o->bidx[x] == b ? o->t[x] : 0.0;
}

/* number of stored (i, j, a) with a valid b, and export (i, j, a, b, t) */
long orc_o3_count(const orc_o3* o) {
    long c = 0;
    for (size_t x = 0; x < (size_t)o->nh * o->nh * o->np; x++) c += o->bidx[x] >= 0;
    return c;
}
void orc_o3_export(const orc_o3* o, int* ijab, double* tv) {
    long c = 0;
    for (int i = 0; i < o->nh; i++)
        for (int j = 0; j < o->nh; j++)
            for (int a = o->nh; a < o->ns; a++) {
                size_t x = O3I(o, i, j, a);
                if (o->bidx[x] < 0) continue;
                ijab[4 * c + 0] = i; ijab[4 * c + 1] = j;
                ijab[4 * c + 2] = a; ijab[4 * c + 3] = o->bidx[x];
                tv[c] = o->t[x];
                c++;
            }
}

/* overwrite the amplitudes (used to start both forms from identical t) */
void orc_o3_set_t(orc_o3* o, const double* tv_in_export_order) {
    long c = 0;
    for (size_t x = 0; x < (size_t)o->nh * o->nh * o->np; x++)
        if (o->bidx[x] >= 0) o->t[x] = tv_in_export_order[c++];
    o->ecorr = o3_energy(o, o->t);
}

/* One Jacobi sweep in the intermediates form (sec. "Developing a CCD code for
 * infinite matter", the rewrite with chi(b,c), chi(k,j), chi(kl,ij),
 * chi(kb,cj) and chi(ab,cd) = <ab||cd>):
 *   eps_ij^ab t = <ab||ij> + P(ab) sum_c dchi_bc t_ij^ac - P(ij) sum_k dchi_kj t_ik^ab
 *               + 1/2 sum_cd <ab||cd> t_ij^cd + 1/2 sum_kl t_kl^ab chi_klij
 *               + P(ij)P(ab) sum_kc t_ik^ac chi_kbcj,
 * where dchi is chi minus the Fock matrix (whose diagonal is moved to the left
 * as eps_ij^ab).  Momentum and spin conservation make chi_bc and chi_kj
 * diagonal, and fix the fourth index of every sum.  The term mask selects the
 * same pieces of eq. ccd3 as in O1.  Returns the new correlation energy. */
double orc_o3_sweep(orc_o3* o, double alpha, unsigned mask) {
    const orc_pnm* h = o->h;
    int nh = o->nh, np = o->np, ns = o->ns;
    const double* t = o->t;
    const double* vt = o->vt;

    /* one-body pieces: chi_bb - f_bb = -1/2 sum_kld t_kl^bd <kl||bd>,
     *                  chi_jj - f_jj = +1/2 sum_cdl <jl||cd> t_jl^cd          */
    for (int p = 0; p < ns; p++) o->dchi[p] = 0.0;
    if (mask & T_QPART) {
#pragma omp parallel for schedule(static)
        for (int b = nh; b < ns; b++) {
            double s = 0.0;
            for (int k = 0; k < nh; k++)
                for (int l = 0; l < nh; l++) {
                    size_t x = O3I(o, k, l, b);
                    if (o->bidx[x] >= 0) s += t[x] * vt[x];
                }
            o->dchi[b] = -0.5 * s;
        }
    }
    if (mask & T_QHOLE) {
#pragma omp parallel for schedule(static)
        for (int j = 0; j < nh; j++) {
            double s = 0.0;
            for (int l = 0; l < nh; l++)
                for (int c = nh; c < ns; c++) {
                    size_t x = O3I(o, j, l, c);
                    if (o->bidx[x] >= 0) s += vt[x] * t[x];
                }
            o->dchi[j] = 0.5 * s;
        }
    }
    /* chi_klij = <kl||ij> [HH] + 1/2 sum_cd <kl||cd> t_ij^cd [Q_HH] */
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nh; k++)
        for (int l = 0; l < nh; l++)
            for (int i = 0; i < nh; i++) {
                size_t y = ((size_t)k * nh + l) * nh + i;
                int j = o->jidx[y];
                double s = 0.0;
                if (j >= 0) {
                    if (mask & T_HH) s += vas_fast(h, k, l, i, j);
                    if (mask & T_QHH) {
                        double q = 0.0;
                        for (int c = nh; c < ns; c++) {
                            size_t x1 = O3I(o, k, l, c), x2 = O3I(o, i, j, c);
                            if (o->bidx[x1] >= 0) q += vt[x1] * t[x2];
                        }
                        s += 0.5 * q;
                    }
                }
                o->chh[y] = s;
            }
    /* chi_kbcj = <kb||cj> [RING] + 1/2 sum_dl <kl||cd> t_lj^db [Q_RING] */
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nh; k++)
        for (int b = nh; b < ns; b++)
            for (int j = 0; j < nh; j++) {
                size_t y = ((size_t)k * np + (b - nh)) * nh + j;
                int c = o->cidx[y];
                double s = 0.0;
                if (c >= 0) {
                    if (mask & T_RING) s += vas_fast(h, k, b, c, j);
                    if (mask & T_QRING) {
                        double q = 0.0;
                        for (int l = 0; l < nh; l++) {
                            size_t x1 = O3I(o, k, l, c); /* <kl||cd>, d deduced */
                            int d = o->bidx[x1];
                            if (d < 0) continue;
                            size_t x2 = O3I(o, l, j, d); /* t_lj^db */
                            if (o->bidx[x2] != b) continue;
                            q += vt[x1] * t[x2];
                        }
                        s += 0.5 * q;
                    }
                }
                o->cph[y] = s;
            }
    /* amplitude update */
#pragma omp parallel for collapse(2) schedule(dynamic)
    for (int i = 0; i < nh; i++)
        for (int j = 0; j < nh; j++)
            for (int a = nh; a < ns; a++) {
                size_t x = O3I(o, i, j, a);
                int b = o->bidx[x];
                if (b < 0) { o->tnew[x] = 0.0; continue; }
                double sum = vt[x];
                if (mask & T_PP) {
                    double s = 0.0;
                    for (int c = nh; c < ns; c++) {
                        size_t z = O3I(o, i, j, c);
                        int d = o->bidx[z];
                        if (d < 0) continue;
                        s += vas_fast(h, a, b, c, d) * t[z];
                    }
                    sum += 0.5 * s;
                }
                if (mask & (T_HH | T_QHH)) {
                    double s = 0.0;
                    for (int k = 0; k < nh; k++) {
                        int l = partner(h, i, j, k); /* n_l = n_i + n_j - n_k */
                        if (l < 0 || l >= nh) continue;
                        size_t zt = O3I(o, k, l, a);
                        if (o->bidx[zt] != b) continue;
                        s += t[zt] * o->chh[((size_t)k * nh + l) * nh + i];
                    }
                    sum += 0.5 * s;
                }
                if (mask & (T_RING | T_QRING)) {
                    /* P(ij)P(ab) f(ijab), f = sum_kc t_ik^ac chi_kbcj */
                    int pi[4] = {i, j, i, j}, pj[4] = {j, i, j, i};
                    int pa[4] = {a, a, b, b}, pb[4] = {b, b, a, a};
                    double sg[4] = {1.0, -1.0, -1.0, 1.0};
                    double s = 0.0;
                    for (int u = 0; u < 4; u++) {
                        double f = 0.0;
                        for (int k = 0; k < nh; k++) {
                            size_t z = O3I(o, pi[u], k, pa[u]); /* t_ik^ac, c deduced */
                            int c = o->bidx[z];
                            if (c < 0) continue;
                            size_t y = ((size_t)k * np + (pb[u] - nh)) * nh + pj[u];
                            if (o->cidx[y] != c) continue;
                            f += t[z] * o->cph[y];
                        }
                        s += sg[u] * f;
                    }
                    sum += s;
                }
                sum += (o->dchi[a] + o->dchi[b] - o->dchi[i] - o->dchi[j]) * t[x];
                double den = h->eps[i] + h->eps[j] - h->eps[a] - h->eps[b];
                double tn = sum / den;
                o->tnew[x] = alpha * tn + (1.0 - alpha) * t[x];
            }
    double* sw = o->t; o->t = o->tnew; o->tnew = sw;
    o->ecorr = o3_energy(o, o->t);
    return o->ecorr;
}
