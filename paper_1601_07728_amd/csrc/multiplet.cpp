// Host helpers for L2,3 edges: the core spin-orbit matrix, the short-range
// direct/exchange matrix on (core spin-orbital, d channel) pairs, and dipole
// amplitudes.  Angular factors use closed forms: Wigner 3j symbols from the
// Racah formula and the standard Gaunt-coefficient identity
//   c^k(lm; l'm') = (-1)^m sqrt((2l+1)(2l'+1)) (l k l'; 0 0 0) (l k l'; -m m-m' m').
// Physics: section 2 (H_h = eps_c + chi - i Gamma; V_D screened, V_X bare) and
// section 3.2.2 (multipole expansion of the short-range terms with selection rules).
#include <cmath>
#include <complex>
#include <vector>

#include "internal.h"

namespace {

double fact(int n) {
    double r = 1.0;
    for (int i = 2; i <= n; ++i) r *= i;
    return r;
}

// Wigner 3j symbol for integer arguments (Racah formula).
double wigner3j(int j1, int j2, int j3, int m1, int m2, int m3) {
    if (m1 + m2 + m3 != 0) return 0.0;
    if (j3 < std::abs(j1 - j2) || j3 > j1 + j2) return 0.0;
    if (std::abs(m1) > j1 || std::abs(m2) > j2 || std::abs(m3) > j3) return 0.0;
    const double tri = fact(j1 + j2 - j3) * fact(j1 - j2 + j3) * fact(-j1 + j2 + j3) / fact(j1 + j2 + j3 + 1);
    const double pre = std::sqrt(tri * fact(j1 + m1) * fact(j1 - m1) * fact(j2 + m2) * fact(j2 - m2) *
                                 fact(j3 + m3) * fact(j3 - m3));
    const int tmin = std::max(0, std::max(j2 - j3 - m1, j1 - j3 + m2));
    const int tmax = std::min(j1 + j2 - j3, std::min(j1 - m1, j2 + m2));
    double s = 0.0;
    for (int t = tmin; t <= tmax; ++t) {
        const double den = fact(t) * fact(j3 - j2 + t + m1) * fact(j3 - j1 + t - m2) * fact(j1 + j2 - j3 - t) *
                           fact(j1 - t - m1) * fact(j2 - t + m2);
        s += ((t & 1) ? -1.0 : 1.0) / den;
    }
    const int ph = j1 - j2 - m3;
    return ((ph & 1) ? -1.0 : 1.0) * pre * s;
}

double gaunt_ck(int k, int l, int m, int lp, int mp) {
    const int q = m - mp;
    if (std::abs(q) > k) return 0.0;
    if ((l + k + lp) & 1) return 0.0;   // (l k l'; 0 0 0) vanishes for odd l + k + l'
    const double sgn = (m & 1) ? -1.0 : 1.0;
    return sgn * std::sqrt((2.0 * l + 1) * (2.0 * lp + 1)) * wigner3j(l, k, lp, 0, 0, 0) *
           wigner3j(l, k, lp, -m, q, mp);
}

}  // namespace

// Matrix elements on (core m_c, d channel m) of the screened direct (F2, m' - m = m_c' - m_c)
// and bare exchange (G1, G3, m' - m_c' = m - m_c) interactions.
double direct_element(double F2, int mcp, int mp, int mc, int m) {
    if (mp - m != mcp - mc) return 0.0;
    return F2 * gaunt_ck(2, 2, mp, 2, m) * gaunt_ck(2, 1, mcp, 1, mc);
}
double exchange_element(double G1, double G3, int mcp, int mp, int mc, int m) {
    if (mp - mcp != m - mc) return 0.0;
    return G1 * gaunt_ck(1, 2, mp, 1, mcp) * gaunt_ck(1, 2, m, 1, mc) +
           G3 * gaunt_ck(3, 2, mp, 1, mcp) * gaunt_ck(3, 2, m, 1, mc);
}


// <Y_lm| v.r^ |Y_l'm'> for a real vector v: v.r^ in spherical components (Y_1q, q = m - m')
// times the Gaunt coefficient c^1(lm; l'm').
static std::complex<double> vdotr_element(const double* v, int l, int m, int lp, int mp) {
    const int q = m - mp;
    if (std::abs(q) > 1) return 0.0;
    const double c1 = gaunt_ck(1, l, m, lp, mp);
    if (c1 == 0.0) return 0.0;
    const double r2 = 1.0 / std::sqrt(2.0);
    if (q == 0) return v[2] * c1;
    if (q == -1) return std::complex<double>(v[0] * r2, v[1] * r2) * c1;
    return std::complex<double>(-v[0] * r2, v[1] * r2) * c1;
}

// Y_LM at the unit vector u (Condon-Shortley phase), from the associated Legendre recurrence
// in L at fixed |M| and Y_{L,-M} = (-1)^M conj(Y_LM).
static std::complex<double> ylm_at(int L, int M, const double* u) {
    const int am = std::abs(M);
    if (am > L) return 0.0;
    const double x = std::max(-1.0, std::min(1.0, u[2]));
    const double s = std::sqrt(std::max(0.0, 1.0 - x * x));
    double pmm = 1.0;   // P_|M|^|M| = (-1)^|M| (2|M| - 1)!! s^|M|
    for (int i = 1; i <= am; ++i) pmm *= -(2.0 * i - 1.0) * s;
    double p = pmm;
    if (L > am) {
        double pm1 = pmm, pl = x * (2.0 * am + 1.0) * pmm;
        for (int ll = am + 2; ll <= L; ++ll) {
            const double pn = ((2.0 * ll - 1.0) * x * pl - (ll + am - 1.0) * pm1) / (ll - am);
            pm1 = pl;
            pl = pn;
        }
        p = pl;
    }
    const double norm = std::sqrt((2.0 * L + 1.0) / (4.0 * M_PI) * fact(L - am) / fact(L + am));
    const double phi = (u[0] == 0.0 && u[1] == 0.0) ? 0.0 : std::atan2(u[1], u[0]);
    std::complex<double> y = norm * p * std::exp(std::complex<double>(0.0, am * phi));
    if (M < 0) y = ((am & 1) ? -1.0 : 1.0) * std::conj(y);
    return y;
}

extern "C" {

int ocean_multiplet_matrices(double zeta, double F2, double G1, double G3, double* core_mat,
                             double* local_mat) {
    if (!std::isfinite(zeta) || !std::isfinite(F2) || !std::isfinite(G1) || !std::isfinite(G3)) {
        ocean::set_error("ocean_multiplet_matrices: parameters must be finite");
        return OCEAN_ERR_INVALID_ARG;
    }
    const int lc = 1, lv = 2;
    if (core_mat) {
        // -chi, chi = zeta l.s on |m_c, sigma>, index (m_c + 1) * 2 + sigma (sigma 0 = up)
        // <m s|l.s|m s> = m s_z;  <m+1, dn|l.s|m, up> = <m, up|l.s|m+1, dn> = sqrt(l(l+1)-m(m+1))/2
        for (int i = 0; i < 72; ++i) core_mat[i] = 0.0;
        auto idx = [](int mc, int s) { return (mc + 1) * 2 + s; };
        for (int mc = -lc; mc <= lc; ++mc) {
            core_mat[2 * (idx(mc, 0) * 6 + idx(mc, 0))] = -zeta * 0.5 * mc;
            core_mat[2 * (idx(mc, 1) * 6 + idx(mc, 1))] = zeta * 0.5 * mc;
            if (mc < lc) {
                const double off = -zeta * 0.5 * std::sqrt((double)(lc * (lc + 1) - mc * (mc + 1)));
                core_mat[2 * (idx(mc + 1, 1) * 6 + idx(mc, 0))] = off;
                core_mat[2 * (idx(mc, 0) * 6 + idx(mc + 1, 1))] = off;
            }
        }
    }
    if (local_mat) {
        // pairs ((m_c, sigma), m) -> ((m_c + 1) * 2 + sigma) * 5 + (m + 2)
        for (int i = 0; i < 30 * 30 * 2; ++i) local_mat[i] = 0.0;
        for (int mcp = -lc; mcp <= lc; ++mcp)
            for (int sp = 0; sp < 2; ++sp)
                for (int mp = -lv; mp <= lv; ++mp) {
                    const int row = ((mcp + 1) * 2 + sp) * 5 + (mp + 2);
                    for (int mc = -lc; mc <= lc; ++mc)
                        for (int s = 0; s < 2; ++s)
                            for (int m = -lv; m <= lv; ++m) {
                                const int col = ((mc + 1) * 2 + s) * 5 + (m + 2);
                                double v = 0.0;
                                // screened direct, diagonal in spin; bare exchange, all spin pairs
                                if (sp == s) v -= direct_element(F2, mcp, mp, mc, m);
                                v += exchange_element(G1, G3, mcp, mp, mc, m);
                                local_mat[2 * (row * 30 + col)] = v;
                            }
                }
    }
    return OCEAN_OK;
}

int ocean_multiplet_matrices_spin(double zeta, double F2, double G1, double G3, double* core_mat,
                                  double* local_mat) {
    // the restricted core matrix on (m_c, sigma_h), then the identity on sigma_e
    double core6[72];
    const int rc = ocean_multiplet_matrices(zeta, F2, G1, G3, core6, nullptr);
    if (rc != OCEAN_OK) return rc;
    if (core_mat) {
        for (int i = 0; i < 12 * 12 * 2; ++i) core_mat[i] = 0.0;
        for (int r = 0; r < 6; ++r)
            for (int c = 0; c < 6; ++c)
                for (int e = 0; e < 2; ++e) {
                    core_mat[2 * ((2 * r + e) * 12 + 2 * c + e)] = core6[2 * (r * 6 + c)];
                    core_mat[2 * ((2 * r + e) * 12 + 2 * c + e) + 1] = core6[2 * (r * 6 + c) + 1];
                }
    }
    if (local_mat) {
        // pairs ((m_c, sigma_h, sigma_e), m) -> (((m_c + 1) * 2 + sigma_h) * 2 + sigma_e) * 5 + (m + 2)
        for (int i = 0; i < 60 * 60 * 2; ++i) local_mat[i] = 0.0;
        for (int mcp = -1; mcp <= 1; ++mcp)
            for (int hp = 0; hp < 2; ++hp)
                for (int ep = 0; ep < 2; ++ep)
                    for (int mp = -2; mp <= 2; ++mp) {
                        const int row = (((mcp + 1) * 2 + hp) * 2 + ep) * 5 + (mp + 2);
                        for (int mc = -1; mc <= 1; ++mc)
                            for (int h = 0; h < 2; ++h)
                                for (int e = 0; e < 2; ++e)
                                    for (int m = -2; m <= 2; ++m) {
                                        const int col = (((mc + 1) * 2 + h) * 2 + e) * 5 + (m + 2);
                                        double v = 0.0;
                                        // direct: both spins kept
                                        if (hp == h && ep == e) v -= direct_element(F2, mcp, mp, mc, m);
                                        // exchange: a pair of equal spins annihilated, another created
                                        if (hp == ep && h == e) v += exchange_element(G1, G3, mcp, mp, mc, m);
                                        local_mat[2 * (row * 60 + col)] = v;
                                    }
                    }
    }
    return OCEAN_OK;
}

int ocean_local_matrix_channels(int n_ch, const int* l, const double* f2, const double* gk, int full_spin,
                                double* local_mat) {
    if (n_ch < 1 || !l || !f2 || !gk || !local_mat) {
        ocean::set_error("ocean_local_matrix_channels: invalid argument");
        return OCEAN_ERR_INVALID_ARG;
    }
    std::vector<int> off(n_ch + 1, 0);
    for (int i = 0; i < n_ch; ++i) {
        if (l[i] < 0 || l[i] > 3) {
            ocean::set_error("ocean_local_matrix_channels: channel l must be 0..3");
            return OCEAN_ERR_INVALID_ARG;
        }
        off[i + 1] = off[i] + 2 * l[i] + 1;
    }
    for (int e = 0; e < n_ch * n_ch * 6; ++e)
        if (!std::isfinite(e < n_ch * n_ch ? f2[e] : gk[e - n_ch * n_ch])) {
            ocean::set_error("ocean_local_matrix_channels: radial integrals must be finite");
            return OCEAN_ERR_INVALID_ARG;
        }
    const int nmu = off[n_ch];
    if (nmu > ocean::kMaxLocal) {
        ocean::set_error("ocean_local_matrix_channels: at most 64 local functions");
        return OCEAN_ERR_UNSUPPORTED;
    }
    // direct D and exchange X on (m_c, mu) pairs, mu = (channel i, m)
    std::vector<double> dm((size_t)9 * nmu * nmu, 0.0), xm((size_t)9 * nmu * nmu, 0.0);
    auto at = [nmu](int mcp, int mup, int mc, int mu) { return ((size_t)(mcp + 1) * nmu + mup) * 3 * nmu + (mc + 1) * nmu + mu; };
    for (int ip = 0; ip < n_ch; ++ip)
        for (int i = 0; i < n_ch; ++i)
            for (int mcp = -1; mcp <= 1; ++mcp)
                for (int mc = -1; mc <= 1; ++mc)
                    for (int mp = -l[ip]; mp <= l[ip]; ++mp)
                        for (int m = -l[i]; m <= l[i]; ++m) {
                            const int mup = off[ip] + mp + l[ip], mu = off[i] + m + l[i];
                            // screened direct, k = 2 (k = 0 is the long-range W0), m' - m = m_c' - m_c
                            if (mp - m == mcp - mc)
                                dm[at(mcp, mup, mc, mu)] = f2[ip * n_ch + i] * gaunt_ck(2, l[ip], mp, l[i], m) *
                                                           gaunt_ck(2, 1, mcp, 1, mc);
                            // bare exchange, every k, m' - m_c' = m - m_c
                            if (mp - mcp == m - mc) {
                                double v = 0.0;
                                for (int k = 0; k <= 4; ++k)
                                    v += gk[(k * n_ch + ip) * n_ch + i] * gaunt_ck(k, l[ip], mp, 1, mcp) *
                                         gaunt_ck(k, l[i], m, 1, mc);
                                xm[at(mcp, mup, mc, mu)] = v;
                            }
                        }
    // spin structure: restricted (core (m_c, sigma), electron spin = sigma) or full
    // ((m_c, sigma_h, sigma_e)); direct keeps the spins, exchange links equal-spin pairs
    const int ns = full_spin ? 4 : 2;
    const int np = 3 * ns * nmu;
    for (size_t e = 0; e < (size_t)np * np * 2; ++e) local_mat[e] = 0.0;
    for (int mcp = -1; mcp <= 1; ++mcp)
        for (int a = 0; a < ns; ++a)
            for (int mc = -1; mc <= 1; ++mc)
                for (int b = 0; b < ns; ++b) {
                    const int hp = full_spin ? a >> 1 : a, ep = full_spin ? a & 1 : a;
                    const int h = full_spin ? b >> 1 : b, e = full_spin ? b & 1 : b;
                    const bool direct = hp == h && ep == e, exch = hp == ep && h == e;
                    if (!direct && !exch) continue;
                    for (int mup = 0; mup < nmu; ++mup)
                        for (int mu = 0; mu < nmu; ++mu) {
                            double v = 0.0;
                            if (direct) v -= dm[at(mcp, mup, mc, mu)];
                            if (exch) v += xm[at(mcp, mup, mc, mu)];
                            const size_t row = (size_t)((mcp + 1) * ns + a) * nmu + mup;
                            const size_t col = (size_t)((mc + 1) * ns + b) * nmu + mu;
                            local_mat[2 * (row * np + col)] = v;
                        }
                }
    return OCEAN_OK;
}

int ocean_dipole_amplitudes_channels(int n_ch, const int* l, const double* radial, const double* e, double* d) {
    if (n_ch < 1 || !l || !radial || !e || !d || !std::isfinite(e[0]) || !std::isfinite(e[1]) ||
        !std::isfinite(e[2])) {
        ocean::set_error("ocean_dipole_amplitudes_channels: invalid argument");
        return OCEAN_ERR_INVALID_ARG;
    }
    const double r2 = 1.0 / std::sqrt(2.0);
    int mu0 = 0;
    for (int i = 0; i < n_ch; ++i) {
        if (l[i] < 0 || l[i] > 3 || !std::isfinite(radial[i])) {
            ocean::set_error("ocean_dipole_amplitudes_channels: channel l must be 0..3, radial finite");
            return OCEAN_ERR_INVALID_ARG;
        }
        // <Y_lm| e.r^ |Y_1mc>: the expansion of e.r^ in Y_1q as in ocean_dipole_amplitudes
        for (int m = -l[i]; m <= l[i]; ++m)
            for (int mc = -1; mc <= 1; ++mc) {
                const double c1 = gaunt_ck(1, l[i], m, 1, mc);
                const int q = m - mc;
                std::complex<double> v(0.0, 0.0);
                if (q == 0) v += e[2] * c1;
                if (q == -1) v += std::complex<double>(e[0] * r2, e[1] * r2) * c1;
                if (q == 1) v += std::complex<double>(-e[0] * r2, e[1] * r2) * c1;
                v *= radial[i];
                const int mu = mu0 + m + l[i];
                d[2 * (mu * 3 + (mc + 1))] = v.real();
                d[2 * (mu * 3 + (mc + 1)) + 1] = v.imag();
            }
        mu0 += 2 * l[i] + 1;
    }
    return OCEAN_OK;
}

int ocean_dipole_amplitudes(const double* e, double* d) {
    if (!e || !d || !std::isfinite(e[0]) || !std::isfinite(e[1]) || !std::isfinite(e[2])) {
        ocean::set_error("ocean_dipole_amplitudes: invalid argument");
        return OCEAN_ERR_INVALID_ARG;
    }
    // e.r^ = e_z z^ + e_x x^ + e_y y^ with x^ = sqrt(2pi/3)(Y_{1,-1} - Y_{11}),
    // y^ = i sqrt(2pi/3)(Y_{1,-1} + Y_{11}), z^ = sqrt(4pi/3) Y_10 and
    // <Y_2m|Y_1q|Y_1mc> = sqrt(3/(4pi)) c^1(2m; 1mc) delta_{q, m - mc}.
    const double r2 = 1.0 / std::sqrt(2.0);
    for (int m = -2; m <= 2; ++m)
        for (int mc = -1; mc <= 1; ++mc) {
            const double c1 = gaunt_ck(1, 2, m, 1, mc);
            const int q = m - mc;
            std::complex<double> v(0.0, 0.0);
            if (q == 0) v += e[2] * c1;
            if (q == -1) v += std::complex<double>(e[0] * r2, e[1] * r2) * c1;
            if (q == 1) v += std::complex<double>(-e[0] * r2, e[1] * r2) * c1;
            d[2 * ((m + 2) * 3 + (mc + 1))] = v.real();
            d[2 * ((m + 2) * 3 + (mc + 1)) + 1] = v.imag();
        }
    return OCEAN_OK;
}

int ocean_nrixs_amplitudes_channels(int n_ch, const int* l, int n_L, const double* radial, const double* q,
                                    double* d) {
    if (n_ch < 1 || n_L < 1 || n_L > 16 || !l || !radial || !q || !d || !std::isfinite(q[0]) ||
        !std::isfinite(q[1]) || !std::isfinite(q[2])) {
        ocean::set_error("ocean_nrixs_amplitudes_channels: invalid argument");
        return OCEAN_ERR_INVALID_ARG;
    }
    const double qn = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
    if (!(qn > 0.0)) {
        ocean::set_error("ocean_nrixs_amplitudes_channels: the momentum transfer must be nonzero");
        return OCEAN_ERR_INVALID_ARG;
    }
    const double u[3] = {q[0] / qn, q[1] / qn, q[2] / qn};
    for (int i = 0; i < n_ch; ++i) {
        bool ok = l[i] >= 0 && l[i] <= 3;
        for (int L = 0; L < n_L; ++L) ok = ok && std::isfinite(radial[i * n_L + L]);
        if (!ok) {
            ocean::set_error("ocean_nrixs_amplitudes_channels: channel l must be 0..3, radial finite");
            return OCEAN_ERR_INVALID_ARG;
        }
    }
    // e^{iq.r} = 4 pi sum_LM i^L j_L(q r) conj(Y_LM(q^)) Y_LM(r^) and
    // <Y_lm|Y_LM|Y_1mc> = sqrt((2L + 1) / 4 pi) c^L(lm; 1 mc) with M = m - mc
    const std::complex<double> iu(0.0, 1.0);
    int mu0 = 0;
    for (int i = 0; i < n_ch; ++i) {
        for (int m = -l[i]; m <= l[i]; ++m)
            for (int mc = -1; mc <= 1; ++mc) {
                std::complex<double> v(0.0, 0.0), ipow(1.0, 0.0);
                for (int L = 0; L < n_L; ++L, ipow *= iu) {
                    const double c = gaunt_ck(L, l[i], m, 1, mc);
                    if (c == 0.0) continue;
                    v += radial[i * n_L + L] * ipow * std::sqrt(4.0 * M_PI * (2.0 * L + 1.0)) *
                         std::conj(ylm_at(L, m - mc, u)) * c;
                }
                const int mu = mu0 + m + l[i];
                d[2 * (mu * 3 + (mc + 1))] = v.real();
                d[2 * (mu * 3 + (mc + 1)) + 1] = v.imag();
            }
        mu0 += 2 * l[i] + 1;
    }
    return OCEAN_OK;
}

int ocean_quadrupole_amplitudes_channels(int n_ch, const int* l, const double* radial1, const double* radial2,
                                         const double* e, const double* q, double* d) {
    bool ok = n_ch >= 1 && l && radial1 && radial2 && e && q && d;
    for (int a = 0; ok && a < 3; ++a) ok = std::isfinite(e[a]) && std::isfinite(q[a]);
    for (int i = 0; ok && i < n_ch; ++i)
        ok = l[i] >= 0 && l[i] <= 3 && std::isfinite(radial1[i]) && std::isfinite(radial2[i]);
    if (!ok) {
        ocean::set_error("ocean_quadrupole_amplitudes_channels: invalid argument (channel l 0..3, all finite)");
        return OCEAN_ERR_INVALID_ARG;
    }
    // (e.r^)(q.r^) Y_1mc lies in the l = 0 and l = 2 shells, so the product's matrix element is
    // the sum over those intermediate states of the two single-vector elements
    int mu0 = 0;
    for (int i = 0; i < n_ch; ++i) {
        for (int m = -l[i]; m <= l[i]; ++m)
            for (int mc = -1; mc <= 1; ++mc) {
                std::complex<double> quad(0.0, 0.0);
                for (int lm = 0; lm <= 2; lm += 2)
                    for (int mm = -lm; mm <= lm; ++mm)
                        quad += vdotr_element(e, l[i], m, lm, mm) * vdotr_element(q, lm, mm, 1, mc);
                const std::complex<double> v =
                    radial1[i] * vdotr_element(e, l[i], m, 1, mc) + std::complex<double>(0.0, 0.5) * radial2[i] * quad;
                const int mu = mu0 + m + l[i];
                d[2 * (mu * 3 + (mc + 1))] = v.real();
                d[2 * (mu * 3 + (mc + 1)) + 1] = v.imag();
            }
        mu0 += 2 * l[i] + 1;
    }
    return OCEAN_OK;
}

}  // extern "C"
