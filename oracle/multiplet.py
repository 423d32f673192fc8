"""Core-hole and local-basis matrices for an L2,3 edge, by plain quadrature.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Builds, from the multiplet parameters alone:

* the core matrix Hc = -(eps_c + chi) on the six 2p spin-orbitals, with
  chi = zeta l.s (the spin-orbit term of H_h, section 2) and eps_c = 0;
* the short-range interaction matrix on (core spin-orbital, d channel) pairs
  (section 3.2.2: the local direct term is screened -- F2 -- and the exchange term is
  bare -- G1, G3; F0 is the long-range W0 and is left out here);
* dipole amplitudes <Y_2m | e.r^ | Y_1mc> for the initial vector (eq. loss.fcn,
  dipole operator e.r), and on the general basis those of e^{iq.r} (non-resonant
  scattering, by the Legendre series of the plane wave) and of the quadrupole term
  (i/2)(e.r)(q.r), each angular factor a sphere integral of the operator itself.

Index conventions: core index c = (m_c + 1) * 2 + sigma (sigma = 0 spin up),
local channel mu = m + 2 for m = -2..2, pair index (c, mu) -> c * 5 + mu.  The general
local basis below (channels of l = 0..3, several radial functions) orders mu by channel,
then m.

Gaunt coefficients c^k(lm; l'm') = sqrt(4 pi / (2k+1)) Int Y*_{lm} Y_{k,m-m'} Y_{l'm'} dOmega are
computed here by Gauss-Legendre x uniform-phi quadrature over the sphere (exact
for these polynomial degrees), not by any closed form.
"""
from __future__ import annotations

import functools
import math

import numpy as np
from scipy.special import sph_harm_y

N_THETA = 24
N_PHI = 48


def _sphere_rule():
    xs, ws = np.polynomial.legendre.leggauss(N_THETA)
    theta = np.arccos(xs)
    phi = 2.0 * math.pi * np.arange(N_PHI) / N_PHI
    th, ph = np.meshgrid(theta, phi, indexing="ij")
    wt = np.outer(ws, np.full(N_PHI, 2.0 * math.pi / N_PHI))
    return th.ravel(), ph.ravel(), wt.ravel()


_TH, _PH, _WT = _sphere_rule()


def ylm(l, m):
    """Complex spherical harmonic (Condon-Shortley phase) on the quadrature nodes."""
    if abs(m) > l:
        return np.zeros_like(_TH, dtype=np.complex128)
    return sph_harm_y(l, m, _TH, _PH)


def sphere_integral(f):
    return np.sum(_WT * f)


@functools.lru_cache(maxsize=None)
def gaunt(k, l, m, lp, mp):
    """c^k(lm; l'm') by quadrature."""
    q = m - mp
    if abs(q) > k:
        return 0.0
    val = sphere_integral(np.conj(ylm(l, m)) * ylm(k, q) * ylm(lp, mp))
    return float(math.sqrt(4.0 * math.pi / (2 * k + 1)) * val.real)


def angular_momentum(l):
    """(Lx, Ly, Lz) for angular momentum l in the basis m = -l..l, from the ladder
    operators L+|m> = sqrt(l(l+1) - m(m+1)) |m+1>."""
    ms = np.arange(-l, l + 1)
    dim = 2 * l + 1
    lz = np.diag(ms.astype(np.float64)).astype(np.complex128)
    lp = np.zeros((dim, dim), dtype=np.complex128)
    for i, m in enumerate(ms[:-1]):
        lp[i + 1, i] = math.sqrt(l * (l + 1) - m * (m + 1))
    lm = lp.conj().T
    return 0.5 * (lp + lm), -0.5j * (lp - lm), lz


def spin_orbit(l, zeta):
    """chi = zeta l.s on |m, sigma> with index m_index * 2 + sigma."""
    lx, ly, lz = angular_momentum(l)
    sx = 0.5 * np.array([[0, 1], [1, 0]], dtype=np.complex128)
    sy = 0.5 * np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
    sz = 0.5 * np.array([[1, 0], [0, -1]], dtype=np.complex128)
    return zeta * (np.kron(lx, sx) + np.kron(ly, sy) + np.kron(lz, sz))


def core_matrix(mult):
    """Hc = -(eps_c + chi) with eps_c = 0 (the core-hole Hamiltonian enters H_BSE as -H_h)."""
    return -spin_orbit(1, mult["zeta"])


def direct_matrix(f2, l_core=1, l_val=2):
    """D[(m_c', m'), (m_c, m)] = F2 c^2(l_val m'; l_val m) c^2(l_core m_c'; l_core m_c),
    nonzero only when m' - m = m_c' - m_c.  Index (m_c + l_core)*(2 l_val + 1) + (m + l_val)."""
    nv = 2 * l_val + 1
    ncr = 2 * l_core + 1
    d = np.zeros((ncr * nv, ncr * nv))
    for mcp in range(-l_core, l_core + 1):
        for mp in range(-l_val, l_val + 1):
            for mc in range(-l_core, l_core + 1):
                for m in range(-l_val, l_val + 1):
                    if mp - m != mcp - mc:
                        continue
                    d[(mcp + l_core) * nv + mp + l_val, (mc + l_core) * nv + m + l_val] = (
                        f2 * gaunt(2, l_val, mp, l_val, m) * gaunt(2, l_core, mcp, l_core, mc))
    return d


def exchange_matrix(gks, l_core=1, l_val=2):
    """X[(m_c', m'), (m_c, m)] = sum_k G^k c^k(l_val m'; l_core m_c') c^k(l_val m; l_core m_c),
    nonzero only when m' - m_c' = m - m_c.  gks maps k -> G^k."""
    nv = 2 * l_val + 1
    ncr = 2 * l_core + 1
    x = np.zeros((ncr * nv, ncr * nv))
    for mcp in range(-l_core, l_core + 1):
        for mp in range(-l_val, l_val + 1):
            for mc in range(-l_core, l_core + 1):
                for m in range(-l_val, l_val + 1):
                    if mp - mcp != m - mc:
                        continue
                    s = 0.0
                    for k, gk in gks.items():
                        s += gk * gaunt(k, l_val, mp, l_core, mcp) * gaunt(k, l_val, m, l_core, mc)
                    x[(mcp + l_core) * nv + mp + l_val, (mc + l_core) * nv + m + l_val] = s
    return x


def local_matrix(mult):
    """K_loc on pairs ((m_c, sigma), m): -(D x I_spin) + (X x J_spin), J = all-ones 2x2.

    The direct part is diagonal in spin; the exchange part couples every
    (sigma, sigma') pair of the electron-hole spin (restricted spin model)."""
    d = direct_matrix(mult["F2"])
    x = exchange_matrix({1: mult["G1"], 3: mult["G3"]})
    ncr, nv = 3, 5
    kmat = np.zeros((6 * nv, 6 * nv), dtype=np.complex128)
    for mcp in range(ncr):
        for sp in range(2):
            for mp in range(nv):
                row = (mcp * 2 + sp) * nv + mp
                for mc in range(ncr):
                    for s in range(2):
                        for m in range(nv):
                            col = (mc * 2 + s) * nv + m
                            val = x[mcp * nv + mp, mc * nv + m]
                            if sp == s:
                                val -= d[mcp * nv + mp, mc * nv + m]
                            kmat[row, col] = val
    return kmat


# --- a general local basis: channels of any l (s, p, d, f), several radial functions each ------
# Channel i has angular momentum l_i; local index mu runs over (channel i, m = -l_i..l_i) in
# that order.  The radial integrals are inputs: F2[i, j] for the screened direct term (F0 is
# the long-range W0 and is left out; a 2p core allows k = 0, 2 only) and G[k][i, j] for the
# bare exchange term (k = 0..4, as the Gaunt selection rules allow).  With the single d
# channel this is the matrix above.

def channel_offsets(ls):
    """Start of each channel in the local index, and the total N_mu."""
    off = np.concatenate([[0], np.cumsum([2 * l + 1 for l in ls])]).astype(int)
    return off[:-1], int(off[-1])


def direct_matrix_channels(ls, f2):
    """D[(m_c', i', m'), (m_c, i, m)] = F2[i', i] c^2(l_i' m'; l_i m) c^2(1 m_c'; 1 m_c)."""
    off, nmu = channel_offsets(ls)
    d = np.zeros((3 * nmu, 3 * nmu))
    for ip, lp in enumerate(ls):
        for i, l in enumerate(ls):
            if f2[ip, i] == 0.0:
                continue
            for mcp in range(-1, 2):
                for mc in range(-1, 2):
                    for mp in range(-lp, lp + 1):
                        for m in range(-l, l + 1):
                            if mp - m != mcp - mc:
                                continue
                            d[(mcp + 1) * nmu + off[ip] + mp + lp, (mc + 1) * nmu + off[i] + m + l] = (
                                f2[ip, i] * gaunt(2, lp, mp, l, m) * gaunt(2, 1, mcp, 1, mc))
    return d


def exchange_matrix_channels(ls, gk):
    """X[(m_c', i', m'), (m_c, i, m)] = sum_k G^k[i', i] c^k(l_i' m'; 1 m_c') c^k(l_i m; 1 m_c)."""
    off, nmu = channel_offsets(ls)
    x = np.zeros((3 * nmu, 3 * nmu))
    for k, g in gk.items():
        for ip, lp in enumerate(ls):
            for i, l in enumerate(ls):
                if g[ip, i] == 0.0:
                    continue
                for mcp in range(-1, 2):
                    for mc in range(-1, 2):
                        for mp in range(-lp, lp + 1):
                            for m in range(-l, l + 1):
                                if mp - mcp != m - mc:
                                    continue
                                x[(mcp + 1) * nmu + off[ip] + mp + lp, (mc + 1) * nmu + off[i] + m + l] += (
                                    g[ip, i] * gaunt(k, lp, mp, 1, mcp) * gaunt(k, l, m, 1, mc))
    return x


def local_matrix_channels(ls, f2, gk, full_spin=False):
    """K_loc on pairs (core index, mu) -> core index * N_mu + mu, in the restricted spin
    model (core index (m_c, sigma)) or with the electron spin carried separately (core
    index (m_c, sigma_h, sigma_e)); the spin structure is the one of local_matrix and
    local_matrix_spin."""
    d = direct_matrix_channels(ls, f2)
    x = exchange_matrix_channels(ls, gk)
    _, nmu = channel_offsets(ls)
    spins = [(h, e) for h in range(2) for e in range(2)] if full_spin else [(s, s) for s in range(2)]
    ns = len(spins)
    kmat = np.zeros((3 * ns * nmu, 3 * ns * nmu), dtype=np.complex128)
    for mcp in range(3):
        for a, (hp, ep) in enumerate(spins):
            rows = slice((mcp * ns + a) * nmu, (mcp * ns + a + 1) * nmu)
            for mc in range(3):
                for b, (h, e) in enumerate(spins):
                    cols = slice((mc * ns + b) * nmu, (mc * ns + b + 1) * nmu)
                    blk = np.zeros((nmu, nmu))
                    if hp == h and ep == e:
                        blk -= d[mcp * nmu:(mcp + 1) * nmu, mc * nmu:(mc + 1) * nmu]
                    if hp == ep and h == e:
                        blk += x[mcp * nmu:(mcp + 1) * nmu, mc * nmu:(mc + 1) * nmu]
                    kmat[rows, cols] = blk
    return kmat


def dipole_psi0_channels(local_proj, ls, radial, pol, full_spin=False):
    """psi0[k, n, core index] = sum_{i, m} conj(A[k, n, (i, m)]) R_i <Y_{l_i m} | e.r^ | Y_1mc>
    with R_i the radial dipole integral of channel i (only s and d channels couple to 2p)."""
    off, nmu = channel_offsets(ls)
    e = np.asarray(pol, dtype=np.float64)
    rhat = np.stack([np.sin(_TH) * np.cos(_PH), np.sin(_TH) * np.sin(_PH), np.cos(_TH)])
    edotr = np.tensordot(e, rhat, axes=1)
    dm = np.zeros((nmu, 3), dtype=np.complex128)
    for i, l in enumerate(ls):
        for m in range(-l, l + 1):
            for mc in range(-1, 2):
                dm[off[i] + m + l, mc + 1] = radial[i] * sphere_integral(np.conj(ylm(l, m)) * edotr * ylm(1, mc))
    per_mc = np.einsum("knm,mc->knc", local_proj.conj(), dm)
    if not full_spin:
        return np.repeat(per_mc, 2, axis=2)
    out = np.zeros(per_mc.shape[:2] + (12,), dtype=np.complex128)
    for mc in range(3):
        for s in range(2):
            out[:, :, (mc * 2 + s) * 2 + s] = per_mc[:, :, mc]
    return out


# --- non-resonant inelastic scattering: O = e^{iq.r} (section 2, eq. loss.fcn) -------------
# e^{iq.r} = sum_L i^L (2L + 1) j_L(q r) P_L(q^.r^).  With radial integrals
# R[i, L] = int R_i(r) j_L(q r) R_2p(r) r^2 dr given per channel i, the amplitude of channel
# function (i, m) from core m_c is sum_L R[i, L] i^L (2L + 1) <Y_{l_i m} | P_L(q^.r^) | Y_1mc>,
# the angular integral taken here by sphere quadrature of the Legendre polynomial itself.

def nrixs_amplitudes_channels(ls, radial, qhat):
    """d[mu, m_c] for mu = (channel i, m); radial[i, L] for L = 0..L_max."""
    from scipy.special import eval_legendre
    off, nmu = channel_offsets(ls)
    qv = np.asarray(qhat, dtype=np.float64)
    qv = qv / np.linalg.norm(qv)
    rhat = np.stack([np.sin(_TH) * np.cos(_PH), np.sin(_TH) * np.sin(_PH), np.cos(_TH)])
    cosg = np.tensordot(qv, rhat, axes=1)
    radial = np.asarray(radial, dtype=np.float64)
    d = np.zeros((nmu, 3), dtype=np.complex128)
    for i, l in enumerate(ls):
        f = sum(radial[i, L] * (1j ** L) * (2 * L + 1) * eval_legendre(L, cosg) for L in range(radial.shape[1]))
        for m in range(-l, l + 1):
            for mc in range(-1, 2):
                d[off[i] + m + l, mc + 1] = sphere_integral(np.conj(ylm(l, m)) * f * ylm(1, mc))
    return d


def quadrupole_amplitudes_channels(ls, radial1, radial2, pol, q):
    """XAS beyond the dipole term: O = e.r + (i/2)(e.r)(q.r) (section 2, eq. loss.fcn).
    radial1[i] and radial2[i] are the channel's integrals of r and r^2 against the 2p
    function; the angular factors are taken by sphere quadrature."""
    off, nmu = channel_offsets(ls)
    rhat = np.stack([np.sin(_TH) * np.cos(_PH), np.sin(_TH) * np.sin(_PH), np.cos(_TH)])
    edotr = np.tensordot(np.asarray(pol, dtype=np.float64), rhat, axes=1)
    qdotr = np.tensordot(np.asarray(q, dtype=np.float64), rhat, axes=1)
    d = np.zeros((nmu, 3), dtype=np.complex128)
    for i, l in enumerate(ls):
        f = radial1[i] * edotr + 0.5j * radial2[i] * edotr * qdotr
        for m in range(-l, l + 1):
            for mc in range(-1, 2):
                d[off[i] + m + l, mc + 1] = sphere_integral(np.conj(ylm(l, m)) * f * ylm(1, mc))
    return d


def psi0_from_amplitudes(local_proj, d, full_spin=False):
    """psi0[k, n, core index] = sum_mu conj(A[k, n, mu]) d[mu, m_c], spin as in dipole_psi0."""
    per_mc = np.einsum("knm,mc->knc", local_proj.conj(), d)
    if not full_spin:
        return np.repeat(per_mc, 2, axis=2)
    out = np.zeros(per_mc.shape[:2] + (12,), dtype=np.complex128)
    for mc in range(3):
        for s in range(2):
            out[:, :, (mc * 2 + s) * 2 + s] = per_mc[:, :, mc]
    return out


# --- the full electron x hole spin space ---------------------------------------------------
# The restricted space ties the photoelectron spin to the spin of the core hole.  Carrying the
# electron spin sigma_e separately, the core index becomes (m_c, sigma_h, sigma_e), index
# ((m_c + 1) * 2 + sigma_h) * 2 + sigma_e.  The spin-orbit term acts on (m_c, sigma_h); the
# direct interaction conserves both spins; the exchange interaction annihilates a pair and
# creates another, so it only connects pairs whose two spins agree (section 2: V_D, V_X;
# the electron and hole spins carried separately, section 3.2.2).

def core_matrix_spin(mult):
    """Hc on the full spin space: -chi on (m_c, sigma_h), the identity on sigma_e."""
    return np.kron(core_matrix(mult), np.eye(2))


def local_matrix_spin(mult):
    """K_loc on pairs ((m_c, sigma_h, sigma_e), m):
    -D delta(sigma_h', sigma_h) delta(sigma_e', sigma_e) + X delta(sigma_h', sigma_e') delta(sigma_h, sigma_e)."""
    d = direct_matrix(mult["F2"])
    x = exchange_matrix({1: mult["G1"], 3: mult["G3"]})
    nv = 5
    kmat = np.zeros((12 * nv, 12 * nv), dtype=np.complex128)
    for mcp in range(3):
        for hp in range(2):
            for ep in range(2):
                for mp in range(nv):
                    row = ((mcp * 2 + hp) * 2 + ep) * nv + mp
                    for mc in range(3):
                        for h in range(2):
                            for e in range(2):
                                for m in range(nv):
                                    col = ((mc * 2 + h) * 2 + e) * nv + m
                                    val = 0.0
                                    if hp == h and ep == e:
                                        val -= d[mcp * nv + mp, mc * nv + m]
                                    if hp == ep and h == e:
                                        val += x[mcp * nv + mp, mc * nv + m]
                                    kmat[row, col] = val
    return kmat


def dipole_psi0_spin(local_proj, pol):
    """psi0[k, n, (m_c, sigma_h, sigma_e)]: the dipole operator conserves spin, so only the
    pairs with sigma_e = sigma_h are excited, with the restricted amplitudes."""
    per_c = dipole_psi0(local_proj, pol)                         # [k, n, (m_c, sigma)]
    out = np.zeros(per_c.shape[:2] + (12,), dtype=np.complex128)
    for c in range(6):
        out[:, :, 2 * c + (c % 2)] = per_c[:, :, c]
    return out


def dipole_amplitudes(pol):
    """d[m, m_c] = <Y_2m | e.r^ | Y_1mc> (radial integral 1), m = -2..2, m_c = -1..1."""
    e = np.asarray(pol, dtype=np.float64)
    rhat = np.stack([np.sin(_TH) * np.cos(_PH), np.sin(_TH) * np.sin(_PH), np.cos(_TH)])
    edotr = np.tensordot(e, rhat, axes=1)
    d = np.zeros((5, 3), dtype=np.complex128)
    for m in range(-2, 3):
        for mc in range(-1, 2):
            d[m + 2, mc + 1] = sphere_integral(np.conj(ylm(2, m)) * edotr * ylm(1, mc))
    return d


def dipole_psi0(local_proj, pol):
    """psi0[k, n, c = (m_c, sigma)] = sum_m conj(A[k, n, m]) d[m, m_c], the same for both spins."""
    d = dipole_amplitudes(pol)
    per_mc = np.einsum("knm,mc->knc", local_proj.conj(), d)     # [k, n, m_c]
    return np.repeat(per_mc, 2, axis=2)
