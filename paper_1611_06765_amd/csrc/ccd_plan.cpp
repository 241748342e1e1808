// ccd_plan.cpp -- host side of the CCD library: model space, Minnesota table,
// Fock energies, direct and particle-hole channels, and operation counts.
//
// Model space: plane waves k = 2 pi n / L in a periodic box of side
// L = (N/rho)^(1/3), n_x^2+n_y^2+n_z^2 <= nmax2, two spin projections, ordered
// by shell, then n_x, n_y, n_z, then s_z = -1/2 before +1/2; the first N
// states are holes (sec. "Single-particle basis for infinite matter" and the
// model-space loop of sec. "Developing a CCD code for infinite matter").
//
// Twisted boundary conditions (the twist-averaging passage and its algorithm):
// phi(x + L) = e^{i theta} phi(x) gives k = (2 pi n + theta) / L.  The same
// states are then ordered by energy, i.e. by |n|^2 + 2 n.phi with
// phi = theta / 2 pi (FP64, left to right, stable in the order above), and the
// first N are holes.  Momentum transfers and momentum conservation do not see
// the twist, so the interaction table and the channel rules are unchanged; the
// hole set is no longer symmetric under n -> -n, so a cross channel Q and its
// partner -Q can differ in size.
//
// Interaction: between two neutrons the isospin exchange is +1, so the
// Minnesota operator 1/2 (V_R + 1/2(1+P_s)V_T + 1/2(1-P_s)V_S)(1 - P_s P_t)
// (sec. "Two-body interaction") reduces to 1/2 (V_R(r) + V_S(r)) (1 - P_s):
// only spin singlets interact.  With the Gaussian Fourier transform
// V_a/L^3 (pi/kappa_a)^{3/2} exp(-q^2/4 kappa_a) and q = k_p - k_r under
// momentum conservation, the antisymmetrised element is
//   <pq||rs> = 1/2 [d(s_p,s_r) d(s_q,s_s) - d(s_p,s_s) d(s_q,s_r)]
//              * (W(|n_p-n_r|^2) + W(|n_p-n_s|^2)),
//   W(m) = sum_{a=R,S} V_a/L^3 (pi/kappa_a)^{3/2} exp(-(2 pi/L)^2 m / 4 kappa_a),
// for n_p+n_q = n_r+n_s and zero otherwise.  The table W(m), m = 0 .. 4 nmax2,
// is all the device needs to generate any element.
//
// Channels (channel discussion after the intermediates): direct channels
// T = (K = n_p + n_q, S_z) hold the hole pairs (i<j) and particle pairs (a<b);
// particle-hole cross channels X = (Q = n_p - n_h, sigma = s_p - s_h) hold
// (particle, hole) pairs; the ring contraction of cross channel (Q, sigma)
// pairs it with (-Q, -sigma).
#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <set>
#include <tuple>

#include "ccd_internal.h"

// the state order is an integer decision taken on FP64 keys: no contraction
#pragma STDC FP_CONTRACT OFF

namespace ccd {

static double minnesota_W(const ccd_problem& p, double L, int m) {
    const double pi = 3.14159265358979323846;
    double dk = 2.0 * pi / L;
    double L3 = L * L * L;
    double w = 0.0;
    w += p.V_R / L3 * std::pow(pi / p.kappa_R, 1.5) * std::exp(-dk * dk * (double)m / (4.0 * p.kappa_R));
    w += p.V_S / L3 * std::pow(pi / p.kappa_S, 1.5) * std::exp(-dk * dk * (double)m / (4.0 * p.kappa_S));
    return w;
}

ccd_status build_problem(const ccd_problem& par, HostProblem& P, std::string& err) {
    P = HostProblem();
    P.par = par;
    if (par.nmax2 < 1 || par.nmax2 > kMaxNmax2) { err = "nmax2 must be in [1, 64]"; return CCD_EINVAL; }
    if (par.n_particles < 2) { err = "n_particles must be >= 2"; return CCD_EINVAL; }
    if (!(par.density > 0.0) || !std::isfinite(par.density)) { err = "density must be > 0"; return CCD_EINVAL; }
    if (!(par.hbar2_over_m > 0.0)) { err = "hbar2_over_m must be > 0"; return CCD_EINVAL; }
    if (!(par.kappa_R > 0.0) || !(par.kappa_S > 0.0)) { err = "Gaussian ranges must be > 0"; return CCD_EINVAL; }
    for (int d = 0; d < 3; d++)
        if (!std::isfinite(par.twist[d])) { err = "twist angles must be finite"; return CCD_EINVAL; }
    const bool twisted = par.twist[0] != 0.0 || par.twist[1] != 0.0 || par.twist[2] != 0.0;
    if (par.n_particles & 1) { err = "n_particles must be even"; return CCD_ENOTMAGIC; }

    // ---- model space ------------------------------------------------------
    int R = 0;
    while ((R + 1) * (R + 1) <= par.nmax2) R++;
    P.R = R;
    std::vector<std::array<int, 4>> mom;  // (n^2, nx, ny, nz)
    for (int x = -R; x <= R; x++)
        for (int y = -R; y <= R; y++)
            for (int z = -R; z <= R; z++) {
                int n2 = x * x + y * y + z * z;
                if (n2 <= par.nmax2) mom.push_back({n2, x, y, z});
            }
    std::sort(mom.begin(), mom.end());
    {
        // energy order under the twist; both spins of a momentum stay together
        const double phx = par.twist[0] / (2.0 * M_PI), phy = par.twist[1] / (2.0 * M_PI),
                     phz = par.twist[2] / (2.0 * M_PI);
        std::vector<std::pair<double, size_t>> key(mom.size());
        for (size_t k = 0; k < mom.size(); k++)
            key[k] = {(double)mom[k][0] + 2.0 * ((double)mom[k][1] * phx + (double)mom[k][2] * phy +
                                                 (double)mom[k][3] * phz),
                      k};
        std::stable_sort(key.begin(), key.end(),
                         [](const std::pair<double, size_t>& a, const std::pair<double, size_t>& b) {
                             return a.first < b.first;
                         });
        for (auto& kv : key)
            for (int s : {-1, 1}) {
                const auto& m = mom[kv.second];
                P.nx.push_back(m[1]); P.ny.push_back(m[2]); P.nz.push_back(m[3]); P.sz.push_back(s);
            }
    }
    P.ns = (int)P.nx.size();
    P.nh = par.n_particles;
    if (P.nh >= P.ns) { err = "no particle states: raise nmax2"; return CCD_ENOTMAGIC; }
    auto shell = [&](int p) { return P.nx[p] * P.nx[p] + P.ny[p] * P.ny[p] + P.nz[p] * P.nz[p]; };
    if (!twisted && shell(P.nh - 1) == shell(P.nh)) {
        err = "n_particles does not close a shell of the plane-wave basis";
        return CCD_ENOTMAGIC;
    }
    if (P.ns > 65535) { err = "basis too large"; return CCD_EINVAL; }
    P.np = P.ns - P.nh;
    P.L = std::cbrt((double)par.n_particles / par.density);

    // ---- energies and interaction table -------------------------------------
    const double pi = 3.14159265358979323846;
    P.tkin.resize(P.ns);
    for (int p = 0; p < P.ns; p++) {
        const double kx = (2.0 * pi * P.nx[p] + par.twist[0]) / P.L, ky = (2.0 * pi * P.ny[p] + par.twist[1]) / P.L,
                     kz = (2.0 * pi * P.nz[p] + par.twist[2]) / P.L;
        P.tkin[p] = 0.5 * par.hbar2_over_m * (kx * kx + ky * ky + kz * kz);
    }
    int nlut = 4 * par.nmax2 + 1;
    P.W.resize(nlut);
    for (int m = 0; m < nlut; m++) P.W[m] = minnesota_W(par, P.L, m);
    auto d2 = [&](int p, int q) {
        int x = P.nx[p] - P.nx[q], y = P.ny[p] - P.ny[q], z = P.nz[p] - P.nz[q];
        return x * x + y * y + z * z;
    };
    // <pi||pi> = 1/2 (1 - d(s_p, s_i)) (W(0) + W(|n_p - n_i|^2))
    P.eps.resize(P.ns);
    for (int p = 0; p < P.ns; p++) {
        double f = 0.0;
        for (int i = 0; i < P.nh; i++)
            if (P.sz[i] != P.sz[p]) f += 0.5 * (P.W[0] + P.W[d2(p, i)]);
        P.eps[p] = P.tkin[p] + f;
    }
    {
        double t = 0.0, v = 0.0;
        for (int i = 0; i < P.nh; i++) t += P.tkin[i];
        for (int i = 0; i < P.nh; i++)
            for (int j = 0; j < P.nh; j++)
                if (P.sz[i] != P.sz[j]) v += 0.5 * (P.W[0] + P.W[d2(i, j)]);
        P.ekin = t;
        P.eref = t + 0.5 * v;
    }

    // ---- direct channels ----------------------------------------------------
    // key = (S_z, K_x, K_y, K_z): canonical channel order is by S_z, then K.
    using Key = std::tuple<int, int, int, int>;
    std::map<Key, std::pair<std::vector<int32_t>, std::vector<int32_t>>> chmap;
    for (int i = 0; i < P.nh; i++)
        for (int j = i + 1; j < P.nh; j++) {
            Key k{P.sz[i] + P.sz[j], P.nx[i] + P.nx[j], P.ny[i] + P.ny[j], P.nz[i] + P.nz[j]};
            auto& e = chmap[k].first;
            e.push_back(i); e.push_back(j);
        }
    for (int a = P.nh; a < P.ns; a++)
        for (int b = a + 1; b < P.ns; b++) {
            Key k{P.sz[a] + P.sz[b], P.nx[a] + P.nx[b], P.ny[a] + P.ny[b], P.nz[a] + P.nz[b]};
            auto it = chmap.find(k);
            if (it == chmap.end()) continue;  // no hole pair: carries no amplitude
            it->second.second.push_back(a); it->second.second.push_back(b);
        }
    int64_t toff = 0;
    for (auto& kv : chmap) {
        int nhh = (int)kv.second.first.size() / 2, npp = (int)kv.second.second.size() / 2;
        if (nhh == 0 || npp == 0) continue;
        Chan c;
        c.Sz = std::get<0>(kv.first); c.Kx = std::get<1>(kv.first);
        c.Ky = std::get<2>(kv.first); c.Kz = std::get<3>(kv.first);
        c.nhh = nhh; c.npp = npp; c.nlp = 0;
        c.t_off = toff;
        c.hh_off = (int)P.hh.size() / 2;
        c.pp_off = (int)P.pp.size() / 2;
        P.hh.insert(P.hh.end(), kv.second.first.begin(), kv.second.first.end());
        P.pp.insert(P.pp.end(), kv.second.second.begin(), kv.second.second.end());
        toff += (int64_t)nhh * npp;
        P.chans.push_back(c);
        P.max_hh = std::max(P.max_hh, nhh);
        P.max_pp = std::max(P.max_pp, npp);
        if (c.Sz == 0) {
            P.n_sz0++;
            // rows with a spin-down a, plus spin-up rows whose spin-down
            // partner (the same momenta) is missing: one per momentum pair
            std::set<std::tuple<int, int, int>> moms;
            for (size_t k = 0; k < kv.second.second.size(); k += 2) {
                const int a = kv.second.second[k];
                moms.insert({P.nx[a], P.ny[a], P.nz[a]});
            }
            P.chans.back().nlp = (int)moms.size();
            double M = npp, Nn = nhh, Mr = (double)moms.size();
            // executed by the FP64 path: the product over momentum pairs
            P.flops_pp += 2.0 * Mr * Mr * Nn;
            P.flops_hh += 2.0 * M * Nn * Nn + 2.0 * Nn * Nn * M;  // hh ladder + chi_klij
            P.flops_ordered += 8.0 * (2.0 * M * M * Nn + 4.0 * M * Nn * Nn);
        }
    }
    P.n_amp = toff;
    if (P.max_hh > kMaxHH) {
        err = "a direct channel has more than 64 hole pairs (N too large for this library)";
        return CCD_EINVAL;
    }

    // ---- particle-hole cross channels -------------------------------------
    std::map<Key, std::vector<int32_t>> phmap;  // key (sigma, Qx, Qy, Qz)
    for (int p = P.nh; p < P.ns; p++)
        for (int h = 0; h < P.nh; h++) {
            Key k{P.sz[p] - P.sz[h], P.nx[p] - P.nx[h], P.ny[p] - P.ny[h], P.nz[p] - P.nz[h]};
            auto& e = phmap[k];
            e.push_back(p); e.push_back(h);
        }
    // a channel whose partner -Q holds no pair carries no ring term (the two
    // positions of every ring term lie in Q and -Q): it is left out
    std::map<Key, int> phid;
    for (auto& kv : phmap) {
        const Key partner{-std::get<0>(kv.first), -std::get<1>(kv.first), -std::get<2>(kv.first),
                          -std::get<3>(kv.first)};
        if (phmap.find(partner) == phmap.end()) continue;
        PhChan c;
        c.sig = std::get<0>(kv.first); c.Qx = std::get<1>(kv.first);
        c.Qy = std::get<2>(kv.first); c.Qz = std::get<3>(kv.first);
        c.n = (int)kv.second.size() / 2;
        c.mem_off = (int)P.phmem.size() / 2;
        c.partner = -1;
        phid[kv.first] = (int)P.ph.size();
        P.phmem.insert(P.phmem.end(), kv.second.begin(), kv.second.end());
        P.ph.push_back(c);
        P.max_ph = std::max(P.max_ph, c.n);
    }
    P.phq.assign((size_t)P.np * P.nh, -1);
    P.phpos.assign((size_t)P.np * P.nh, -1);
    for (size_t q = 0; q < P.ph.size(); q++) {
        PhChan& c = P.ph[q];
        Key partner{-c.sig, -c.Qx, -c.Qy, -c.Qz};
        auto it = phid.find(partner);
        if (it == phid.end()) {
            err = "internal: particle-hole channel without a partner";
            return CCD_EINVAL;
        }
        c.partner = it->second;
        for (int u = 0; u < c.n; u++) {
            int p = P.phmem[2 * (c.mem_off + u)], h = P.phmem[2 * (c.mem_off + u) + 1];
            P.phq[(size_t)(p - P.nh) * P.nh + h] = (int)q;
            P.phpos[(size_t)(p - P.nh) * P.nh + h] = u;
        }
    }
    // position maps [n_Q][n_-Q]; ring flops 2 n_-Q^2 n_Q for chi_kbcj and as
    // many for Z_Q (both square when the hole set is symmetric)
    for (PhChan& c : P.ph) {
        const int m = P.ph[c.partner].n;
        c.z_off = P.nz_ph;
        P.nz_ph += (int64_t)c.n * m;
        P.flops_ring += 4.0 * (double)c.n * m * m;
    }
    P.flops_ordered += P.flops_ring;
    if (P.max_ph > kMaxPH) {
        err = "a particle-hole channel has more than 80 pairs (N too large for this library)";
        return CCD_EINVAL;
    }
    if (P.n_amp >= (int64_t)1 << 28) { err = "too many amplitudes"; return CCD_EINVAL; }

    // ---- position map of the particle-hole blocks -------------------------
    // canonical index of the element (i<j, a<b): channel block offset +
    // row (position of (a,b)) * n_hh + column (position of (i,j))
    std::vector<int32_t> hpos((size_t)P.nh * P.nh, -1), hchan((size_t)P.nh * P.nh, -1);
    std::vector<int32_t> ppos((size_t)P.np * P.np, -1);
    for (size_t ci = 0; ci < P.chans.size(); ci++) {
        const Chan& c = P.chans[ci];
        for (int q = 0; q < c.nhh; q++) {
            int i = P.hh[2 * (c.hh_off + q)], j = P.hh[2 * (c.hh_off + q) + 1];
            hpos[(size_t)i * P.nh + j] = q;
            hchan[(size_t)i * P.nh + j] = (int)ci;
        }
        for (int r = 0; r < c.npp; r++) {
            int a = P.pp[2 * (c.pp_off + r)], b = P.pp[2 * (c.pp_off + r) + 1];
            ppos[(size_t)(a - P.nh) * P.np + (b - P.nh)] = r;
        }
    }
    P.phmap.assign((size_t)P.nz_ph, -1);
    for (const PhChan& c : P.ph) {
        const PhChan& pc = P.ph[c.partner];
        for (int u = 0; u < c.n; u++) {
            int p = P.phmem[2 * (c.mem_off + u)], h = P.phmem[2 * (c.mem_off + u) + 1];
            for (int y = 0; y < pc.n; y++) {
                int p2 = P.phmem[2 * (pc.mem_off + y)], h2 = P.phmem[2 * (pc.mem_off + y) + 1];
                if (p == p2 || h == h2) continue;
                int i = std::min(h, h2), j = std::max(h, h2);
                int a = std::min(p, p2), b = std::max(p, p2);
                int ci = hchan[(size_t)i * P.nh + j];
                int r = ppos[(size_t)(a - P.nh) * P.np + (b - P.nh)];
                if (ci < 0 || r < 0) { err = "internal: particle-hole position without amplitude"; return CCD_EINVAL; }
                const Chan& dc = P.chans[ci];
                int64_t e = dc.t_off + (int64_t)r * dc.nhh + hpos[(size_t)i * P.nh + j];
                int slot = 2 * (p > p2) + (h > h2);
                int neg = (p > p2) ^ (h > h2);
                P.phmap[(size_t)c.z_off + (size_t)u * pc.n + y] = (int32_t)((e << 3) | (slot << 1) | neg);
            }
        }
    }
    // ---- pair blocks {Q, -Q} and the ring indices of each amplitude ----------
    // the primary (lower index) Q of a pair owns the block [n_Q][n_-Q]
    for (size_t q = 0; q < P.ph.size(); q++) {
        PhChan& c = P.ph[q];
        c.zp_off = -1;
        if (c.partner >= (int)q) {
            c.zp_off = P.n_zp;
            P.n_zp += (int64_t)c.n * P.ph[c.partner].n;
        }
    }
    if (P.n_zp >= ((int64_t)1 << 31) || P.n_amp >= ((int64_t)1 << 29)) { err = "too many ring entries"; return CCD_EINVAL; }
    auto zpos = [&](int p, int h, int p2, int h2) -> int64_t {
        size_t x1 = (size_t)(p - P.nh) * P.nh + h, x2 = (size_t)(p2 - P.nh) * P.nh + h2;
        if (P.phq[x1] < 0 || P.phq[x2] < 0) return (int64_t)-1;
        const PhChan& c = P.ph[P.phq[x1]];
        const PhChan& pc = P.ph[c.partner];
        if (c.zp_off >= 0) return c.zp_off + (int64_t)P.phpos[x1] * pc.n + P.phpos[x2];
        return pc.zp_off + (int64_t)P.phpos[x2] * c.n + P.phpos[x1];
    };
    P.zidx.resize(2 * (size_t)P.n_amp);
    for (const Chan& c : P.chans)
        for (int r = 0; r < c.npp; r++) {
            int a = P.pp[2 * (c.pp_off + r)], b = P.pp[2 * (c.pp_off + r) + 1];
            for (int q = 0; q < c.nhh; q++) {
                int i = P.hh[2 * (c.hh_off + q)], j = P.hh[2 * (c.hh_off + q) + 1];
                int64_t e = c.t_off + (int64_t)r * c.nhh + q;
                const int64_t z0 = zpos(a, i, b, j), z1 = zpos(a, j, b, i);
                if (z0 < 0 || z1 < 0) { err = "internal: ring position in a channel without a partner"; return CCD_EINVAL; }
                P.zidx[2 * e] = (int32_t)z0;
                P.zidx[2 * e + 1] = (int32_t)z1;
            }
        }
    // inverse: each written pair-block position feeds one ring slot 2e + k of one
    // amplitude (zidx[2e + k] is that position); zs = (2e + k) << 1 | sign
    P.zs.assign((size_t)P.n_zp, -1);
    int64_t assigned = 0;
    for (const PhChan& c : P.ph) {
        if (c.zp_off < 0) continue;
        const bool self = c.partner == (int)(&c - P.ph.data());
        const int ncol = P.ph[c.partner].n;
        for (int u = 0; u < c.n; u++)
            for (int y = 0; y < ncol; y++) {
                const int32_t m = P.phmap[(size_t)c.z_off + (size_t)u * ncol + y];
                if (m < 0 || (self && ((m >> 2) & 1))) continue;
                const int64_t e = m >> 3, pos = c.zp_off + (int64_t)u * ncol + y;
                int k = -1;
                if (P.zidx[2 * e] == pos) k = 0;
                else if (P.zidx[2 * e + 1] == pos) k = 1;
                if (k < 0 || P.zs[pos] != -1) { err = "internal: ring position without a unique slot"; return CCD_EINVAL; }
                P.zs[pos] = (int32_t)(((2 * e + k) << 1) | (m & 1));
                assigned++;
            }
    }
    if (assigned != 2 * P.n_amp) { err = "internal: ring slots not covered"; return CCD_EINVAL; }
    return CCD_OK;
}

}  // namespace ccd

// Gauss-Legendre rule by Newton's method on P_n, evaluated with the
// three-term recurrence (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}; nodes
// ascending on [-1, 1], weights 2 / ((1 - x^2) P_n'(x)^2).
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < (n + 1) / 2; i++) {
        double z = std::cos(pi * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = z;
            for (int k = 1; k < n; k++) {
                const double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        // recompute the derivative at the converged node for the weight
        double p0 = 1.0, p1 = z;
        for (int k = 1; k < n; k++) {
            const double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        const double wt = 2.0 / ((1.0 - z * z) * dp * dp);
        x[n - 1 - i] = z;  w[n - 1 - i] = wt;
        x[i] = -z;         w[i] = wt;
    }
    if (n & 1) x[n / 2] = 0.0;
}

extern "C" ccd_status ccd_twist_mesh(int32_t n, double* theta, double* weight) {
    if (n < 1 || n > 64 || !theta || !weight) {
        ccd::set_error("ccd_twist_mesh: n must be in [1, 64] and the buffers non-NULL");
        return CCD_EINVAL;
    }
    std::vector<double> x, w;
    gauss_legendre(n, x, w);
    const double pi = 3.14159265358979323846, h = 0.5 * pi;
    size_t k = 0;
    for (int a = 0; a < n; a++)
        for (int b = 0; b < n; b++)
            for (int c = 0; c < n; c++, k++) {
                theta[3 * k] = h * (x[a] + 1.0);
                theta[3 * k + 1] = h * (x[b] + 1.0);
                theta[3 * k + 2] = h * (x[c] + 1.0);
                weight[k] = (h * w[a]) * (h * w[b]) * (h * w[c]) / (pi * pi * pi);
            }
    return CCD_OK;
}
