"""Pins of the oracle's transition operators beyond the dipole (section 2, eq. loss.fcn):
non-resonant scattering e^{iq.r} and the XAS quadrupole term (i/2)(e.r)(q.r), on the general
local basis (channels l = s..f) around a 2p core.

* e^{iq.r}: brute force -- the full three-dimensional integral of conj(R_i Y_lm) e^{iq.r}
  R_2p Y_1mc over space, for explicit radial functions, by a product rule of its own --
  equals the channel amplitudes built from the j_L radial integrals of the same functions
  (this fixes the i^L and 2L + 1 factors of the plane-wave expansion for every L);
* its L = 1 term alone is 3i times the pinned dipole amplitudes with e = q^, and its L = 0
  term is the overlap: delta(m, m_c) on p channels, zero on the others;
* the quadrupole product on a p channel equals the Cartesian closed form
  Int r_a r_b r_c r_d dOmega / 4 pi = (d_ab d_cd + d_ac d_bd + d_ad d_bc) / 15, mapped to
  Y_1m by the standard unitary, and vanishes on s and d channels (parity);
* q = 0 leaves the dipole amplitudes."""
import math

import numpy as np
from scipy.special import spherical_jn, sph_harm_y

from oracle import multiplet as mp

LS = [0, 1, 2, 3, 2]
ALPHA = [1.3, 0.9, 1.1, 0.8, 1.6]     # R_i(r) = r^l exp(-alpha_i r); R_2p(r) = r exp(-r)


def _radial_rule(n=240, rmax=40.0):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * rmax * (x + 1.0), 0.5 * rmax * w


def _angular_rule(nt=40, nph=80):
    x, w = np.polynomial.legendre.leggauss(nt)
    th = np.arccos(x)
    ph = 2.0 * math.pi * np.arange(nph) / nph
    T, P = np.meshgrid(th, ph, indexing="ij")
    W = np.outer(w, np.full(nph, 2.0 * math.pi / nph))
    return T.ravel(), P.ravel(), W.ravel()


def _brute_force_eiqr(q):
    r, wr = _radial_rule()
    th, ph, wa = _angular_rule()
    rhat = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
    phase = np.exp(1j * np.outer(r, q @ rhat))              # [r, Omega]
    r2p = r * np.exp(-r)
    off, nmu = mp.channel_offsets(LS)
    d = np.zeros((nmu, 3), dtype=np.complex128)
    for i, l in enumerate(LS):
        radial_w = wr * r ** 2 * r ** l * np.exp(-ALPHA[i] * r) * r2p
        g = radial_w @ phase                                  # [Omega]
        for m in range(-l, l + 1):
            for mc in range(-1, 2):
                y = np.conj(sph_harm_y(l, m, th, ph)) * sph_harm_y(1, mc, th, ph)
                d[off[i] + m + l, mc + 1] = np.sum(wa * y * g)
    return d


def _jl_radial(q, n_l):
    r, wr = _radial_rule()
    qn = float(np.linalg.norm(q))
    out = np.zeros((len(LS), n_l))
    for i, l in enumerate(LS):
        f = wr * r ** 2 * r ** l * np.exp(-ALPHA[i] * r) * r * np.exp(-r)
        for L in range(n_l):
            out[i, L] = np.sum(f * spherical_jn(L, qn * r))
    return out


def test_eiqr_matches_brute_force_space_integral():
    for q in (np.array([0.4, -0.7, 1.1]), np.array([0.0, 0.0, 2.5])):
        ref = _brute_force_eiqr(q)
        got = mp.nrixs_amplitudes_channels(LS, _jl_radial(q, 6), q)
        assert np.abs(ref).max() > 0.1
        assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max(), np.abs(got - ref).max()


def test_eiqr_dipole_and_monopole_terms():
    rng = np.random.default_rng(4)
    q = np.array([0.3, -0.5, 0.8])
    qh = q / np.linalg.norm(q)
    r1 = rng.normal(size=len(LS))
    rad = np.zeros((len(LS), 4))
    rad[:, 1] = r1
    eye = np.eye(sum(2 * l + 1 for l in LS))[None]
    dip = mp.dipole_psi0_channels(eye, LS, r1, qh)[0, :, ::2]
    assert np.abs(mp.nrixs_amplitudes_channels(LS, rad, q) - 3j * dip).max() <= 1e-14
    rad0 = np.zeros((len(LS), 1))
    rad0[:, 0] = 1.0
    d0 = mp.nrixs_amplitudes_channels(LS, rad0, q)
    off, _ = mp.channel_offsets(LS)
    ref = np.zeros_like(d0)
    ref[off[1]:off[1] + 3] = np.eye(3)
    assert np.abs(d0 - ref).max() <= 1e-14


def test_quadrupole_p_channel_closed_form_and_parity():
    e = np.array([0.6, 0.0, 0.8])
    q = np.array([0.7, -1.1, 0.4])
    r2 = np.arange(1.0, len(LS) + 1.0)
    d = mp.quadrupole_amplitudes_channels(LS, np.zeros(len(LS)), r2, e, q)
    # Cartesian p functions p_c = sqrt(3 / 4 pi) r^_c: <p_c|(e.r^)(q.r^)|p_d> =
    # (e_c q_d + q_c e_d + (e.q) delta_cd) / 5
    cart = (np.outer(e, q) + np.outer(q, e) + np.dot(e, q) * np.eye(3)) / 5.0
    s2 = 1.0 / math.sqrt(2.0)
    u = np.array([[s2, -1j * s2, 0.0],       # Y_1,-1 = (p_x - i p_y) / sqrt 2
                  [0.0, 0.0, 1.0],           # Y_10 = p_z
                  [-s2, -1j * s2, 0.0]])     # Y_11 = -(p_x + i p_y) / sqrt 2
    ref_p = 0.5j * r2[1] * (u.conj() @ cart @ u.T)
    off, _ = mp.channel_offsets(LS)
    assert np.abs(d[off[1]:off[1] + 3] - ref_p).max() <= 1e-14
    for i in (0, 2, 4):                       # even l: odd integrand
        assert np.abs(d[off[i]:off[i] + 2 * LS[i] + 1]).max() <= 1e-14
    assert np.abs(d[off[3]:off[3] + 7]).max() > 0.01     # f channel is reached


def test_quadrupole_at_zero_q_is_the_dipole():
    rng = np.random.default_rng(5)
    r1, r2 = rng.normal(size=len(LS)), rng.normal(size=len(LS))
    e = np.array([0.2, 0.7, -0.4])
    eye = np.eye(sum(2 * l + 1 for l in LS))[None]
    dip = mp.dipole_psi0_channels(eye, LS, r1, e)[0, :, ::2]
    assert np.abs(mp.quadrupole_amplitudes_channels(LS, r1, r2, e, np.zeros(3)) - dip).max() <= 1e-15


def test_psi0_from_amplitudes_reproduces_dipole_vectors():
    rng = np.random.default_rng(6)
    nmu = sum(2 * l + 1 for l in LS)
    a = rng.normal(size=(3, 4, nmu)) + 1j * rng.normal(size=(3, 4, nmu))
    r1 = rng.normal(size=len(LS))
    e = np.array([0.2, 0.7, -0.4])
    d = mp.dipole_psi0_channels(np.eye(nmu)[None], LS, r1, e)[0, :, ::2]
    for full in (False, True):
        ref = mp.dipole_psi0_channels(a, LS, r1, e, full_spin=full)
        assert np.abs(mp.psi0_from_amplitudes(a, d, full_spin=full) - ref).max() <= 1e-14
