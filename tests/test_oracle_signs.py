"""Pins of the signs and the lattice algebra of the oracle's Hamiltonian.

H_BSE = H_e - H_h - V_D + V_X (section 2, eq. H_BSE): the screened direct interaction
between the excited electron and the core hole enters with a minus sign (it binds the pair)
and the bare exchange with a plus sign.  The long-range part of V_D is W0, applied by
Algorithm 1 (section 3.2.1); its short-range direct part (F^2) and the exchange (G^k) act
through the local basis (section 3.2.2, multipole expansion of the Coulomb kernel).

Each pin is checked twice: on the oracle as it stands, where it must hold, and on copies of
the oracle with one plausible mistake planted in the source text (a flipped sign, a
transposed matrix), where it must fail.  The planted copies live only inside this test."""
import math
import os
import types

import numpy as np
import pytest
from scipy.special import eval_legendre, sph_harm_y

import synth
from oracle import bse
from oracle import multiplet as mp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SKEWED = np.array([[7.0, 0.0, 0.0], [2.1, 6.4, 0.0], [-1.3, 1.7, 6.9]])
HEXAGONAL = np.array([[6.0, 0.0, 0.0], [3.0, 3.0 * math.sqrt(3.0), 0.0], [0.0, 0.0, 7.5]])


def _mutant(name, old, new, occurrence=None):
    """A fresh copy of oracle/<name>.py with `old` replaced by `new` in its source text
    (every occurrence, or only the occurrence-th, counting from 1)."""
    path = os.path.join(ROOT, "oracle", name + ".py")
    with open(path) as f:
        src = f.read()
    assert old in src, f"planted mistake not applicable: {old!r} not in {name}.py"
    if occurrence is None:
        src = src.replace(old, new)
    else:
        at = -1
        for _ in range(occurrence):
            at = src.index(old, at + 1)
        src = src[:at] + new + src[at + len(old):]
    mod = types.ModuleType(f"oracle_planted_{name}")
    mod.__file__ = path
    exec(compile(src, f"{path} (planted copy)", "exec"), mod.__dict__)
    return mod


# --- the crystals the pins run on ---------------------------------------------------------------

def _cubic_l():
    return synth.small_l_edge(seed=3, nk=(2, 1, 2), nx=(4, 5, 3), n_bands=7)


def _skewed_l():
    cr = synth.small_l_edge(seed=21, nk=(2, 2, 2), nx=(3, 4, 3), n_bands=4)
    cr.lattice = SKEWED
    cr.kshift = (0.5, 0.0, 0.5)
    return cr


def _hexagonal_l():
    cr = synth.small_l_edge(seed=24, nk=(3, 2, 2), nx=(3, 3, 4), n_bands=3)
    cr.lattice = HEXAGONAL
    cr.kshift = (0.0, 0.5, 0.0)
    return cr


def _crystals():
    return [synth.config1(), _cubic_l(), _skewed_l(), _hexagonal_l()]


def _constant_w(cr, c):
    """A copy of the crystal whose radial table is the constant c out to 10^6 bohr, so that
    W(x, R) = c for every pair (x, R) of the Born-von-Karman supercell."""
    import dataclasses
    return dataclasses.replace(cr, w_r=np.array([0.0, 1.0e6]), w_val=np.array([c, c]))


def _matrices(mpm, cr):
    if cr.multiplet is None:
        return None, None
    return mpm.core_matrix(cr.multiplet), mpm.local_matrix(cr.multiplet)


# --- (i) the sign of W0: a constant screened potential shifts H by exactly -c ----------------------

def w0_shift_error(bm, mpm, cr, c=0.37):
    """max |H(W = c) - H(W = 0) + c I| / c for the explicit matrix and the matrix-free form.

    With u orthonormal per k and a unitary k <-> R pair, a potential that is the same
    constant at every (x, R) acts as c times the identity on each core index, and -V_D turns
    that into -c (section 2, eq. H_BSE; section 3.2.1)."""
    hc, kl = _matrices(mpm, cr)
    crc = _constant_w(cr, c)
    dim = cr.dim
    err_dense = np.abs(bm.h_dense(crc, hc, kl) - bm.h_dense(cr, hc, kl, w_scale=0.0) + c * np.eye(dim)).max()
    psi = synth.complex_gaussian(np.random.default_rng(5), (cr.n_k, cr.n_bands, cr.n_core))
    diff = bm.apply_h(crc, psi, hc, kl) - bm.apply_h(cr, psi, hc, kl, w_scale=0.0)
    err_free = np.abs(diff + c * psi).max() / np.abs(psi).max()
    return max(err_dense, err_free) / c


@pytest.mark.parametrize("idx", range(4), ids=["c1-cubic-K", "cubic-L", "skewed-shifted-L", "hexagonal-shifted-L"])
def test_constant_w_shifts_h_down_by_c(idx):
    cr = _crystals()[idx]
    assert w0_shift_error(bse, mp, cr) <= 1e-13


def core_hole_binding(bm, mpm, cr):
    """(largest rise, lowest-level drop) of the sorted eigenvalues of H when W0 is switched
    on.  W(r) >= 0 makes the W0 matrix positive semidefinite (it is sum_x U_x^H F^H diag(W_x)
    F U_x), so with -V_D every level can only move down (Weyl's monotonicity theorem), and
    the lowest one moves down strictly: the attractive core hole pulls a bound exciton below
    the band bottom."""
    hc, kl = _matrices(mpm, cr)
    lam_on = np.linalg.eigvalsh(bm.h_dense(cr, hc, kl))
    lam_off = np.linalg.eigvalsh(bm.h_dense(cr, hc, kl, w_scale=0.0))
    return float(np.max(lam_on - lam_off)), float(lam_off[0] - lam_on[0])


def test_attractive_core_hole_lowers_every_level():
    for cr in (synth.config1(), _cubic_l()):
        assert np.all(cr.w_val > 0)
        rise, drop = core_hole_binding(bse, mp, cr)
        assert rise <= 1e-12 and drop > 1e-3 * np.abs(cr.w_val).max()


# --- (iv) the reciprocal lattice of a cell of any shape ---------------------------------------------

def dft_unitarity_error(bm, cr):
    """The k -> R transform F[R, k] = Nk^{-1/2} e^{ik.R} and its inverse are unitary exactly
    when a_i . b_j = 2 pi delta_ij (section 3.2.1: Fourier transform over the k grid to the
    cells R of the Born-von-Karman supercell), whatever the shape of the cell and the offset
    of the k grid.  Also returns the largest |a_i . b_j - 2 pi delta_ij|."""
    f = bm.dft_matrix(cr)
    eye = np.eye(cr.n_k)
    err_u = max(np.abs(f.conj().T @ f - eye).max(), np.abs(f @ f.conj().T - eye).max())
    dual = cr.cell_vectors() @ bm.reciprocal_vectors(cr).T
    return err_u, float(np.abs(dual - 2.0 * math.pi * np.eye(3)).max())


@pytest.mark.parametrize("idx", range(4), ids=["c1-cubic-K", "cubic-L", "skewed-shifted-L", "hexagonal-shifted-L"])
def test_dft_pair_is_unitary_on_any_cell(idx):
    cr = _crystals()[idx]
    err_u, err_dual = dft_unitarity_error(bse, cr)
    assert err_u <= 1e-13 and err_dual <= 1e-13


def test_bloch_phase_is_periodic_over_the_supercell():
    """e^{ik.L} = e^{2 pi i s_d} for every k of a grid offset by s_d steps and every supercell
    vector L = n_d a_d: the k grid is the set of Bloch vectors of the Born-von-Karman
    supercell (closed form, independent of the cell's shape)."""
    for cr in (_skewed_l(), _hexagonal_l()):
        k = bse.kpoints(cr)
        sup = np.asarray(cr.nk, dtype=float)[:, None] * cr.cell_vectors()
        ph = np.exp(1j * k @ sup.T)                                       # [k, d]
        want = np.exp(2j * math.pi * np.asarray(cr.kshift))[None, :]
        assert np.abs(ph - want).max() <= 1e-12


# --- (ii), (iii) short-range direct and exchange: the Coulomb multipole integrals by brute force ----
# The direct element between pair states |(m_c, i, m)> (electron in channel function (i, m),
# hole left in core orbital m_c) is the Coulomb energy of the electron density
# conj(phi_{i'm'}) phi_{im} with the hole density, in which the hole carries the conjugate
# representation: phi_{1 m_c'} conj(phi_{1 m_c}).  The exchange element is the Coulomb energy of
# the two transition densities conj(phi_{i'm'}) phi_{1 m_c'} and conj(phi_{1 m_c}) phi_{im}.
# The angular part of the k-th multipole of 1/|r - r'| is P_k(r^.r^'); here it is integrated
# directly over two spheres, with no Gaunt coefficients and no addition theorem.

def _sphere_rule(n_theta=16, n_phi=20):
    x, w = np.polynomial.legendre.leggauss(n_theta)
    th, ph = np.meshgrid(np.arccos(x), 2.0 * math.pi * np.arange(n_phi) / n_phi, indexing="ij")
    wt = np.outer(w, np.full(n_phi, 2.0 * math.pi / n_phi))
    return th.ravel(), ph.ravel(), wt.ravel()


def coulomb_multipole_blocks(ls, f2, gk):
    """D[(m_c', mu'), (m_c, mu)] and X[(m_c', mu'), (m_c, mu)] (index (m_c + 1) N_mu + mu, mu
    over (channel, m)) by double quadrature of the angular parts of the multipole terms
    (r_<^k / r_>^(k+1)) P_k(r^.r^') of 1/|r - r'|, with unit radial integrals scaled by the
    tables:
      D = F2[i', i] Int Int conj(Y_{l'm'}(r)) Y_{lm}(r) P_2(r.r') Y_{1m_c'}(r') conj(Y_{1m_c}(r')),
      X = sum_k G^k[i', i] Int Int conj(Y_{l'm'}(r)) Y_{1m_c'}(r) P_k(r.r') conj(Y_{1m_c}(r')) Y_{lm}(r')."""
    th, ph, wt = _sphere_rule()
    rhat = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
    cosg = np.clip(rhat.T @ rhat, -1.0, 1.0)
    elec = np.concatenate([[sph_harm_y(l, m, th, ph) for m in range(-l, l + 1)] for l in ls])   # [mu, P]
    core = np.array([sph_harm_y(1, m, th, ph) for m in range(-1, 2)])                           # [m_c, P]
    chan = np.concatenate([[i] * (2 * l + 1) for i, l in enumerate(ls)])
    nmu = len(chan)
    ee = np.conj(elec)[:, None, :] * elec[None, :, :] * wt          # [mu', mu, P]
    hh = core[:, None, :] * np.conj(core)[None, :, :] * wt          # [m_c', m_c, Q]
    ang_d = np.einsum("abp,pq,cdq->cadb", ee, eval_legendre(2, cosg), hh)  # [m_c', mu', m_c, mu]
    d = ang_d * np.asarray(f2)[chan][:, chan][None, :, None, :]
    x = np.zeros_like(d)
    t1 = np.conj(elec)[:, None, :] * core[None, :, :] * wt          # [mu', m_c', P]
    t2 = np.conj(core)[:, None, :] * elec[None, :, :] * wt          # [m_c, mu, Q]
    for k, g in gk.items():
        ang_x = np.einsum("abp,pq,cdq->bacd", t1, eval_legendre(k, cosg), t2)   # [m_c', mu', m_c, mu]
        x = x + ang_x * np.asarray(g)[chan][:, chan][None, :, None, :]
    return d.reshape(3 * nmu, 3 * nmu), x.reshape(3 * nmu, 3 * nmu)


def _assemble(d, x, nmu, full_spin):
    """-V_D + V_X on (core index, mu): the direct term keeps the spins, the exchange term
    annihilates a pair of equal spins and creates another.  Restricted model: core index
    (m_c, sigma) with the electron spin tied to sigma, so the exchange couples every spin pair;
    full space: core index (m_c, sigma_h, sigma_e)."""
    spins = [(h, e) for h in range(2) for e in range(2)] if full_spin else [(s, s) for s in range(2)]
    ns = len(spins)
    out = np.zeros((3 * ns * nmu, 3 * ns * nmu), dtype=np.complex128)
    d4 = d.reshape(3, nmu, 3, nmu)
    x4 = x.reshape(3, nmu, 3, nmu)
    for mcp in range(3):
        for a, (hp, ep) in enumerate(spins):
            r0 = (mcp * ns + a) * nmu
            for mc in range(3):
                for b, (h, e) in enumerate(spins):
                    c0 = (mc * ns + b) * nmu
                    blk = np.zeros((nmu, nmu), dtype=np.complex128)
                    if hp == h and ep == e:
                        blk -= d4[mcp, :, mc, :]
                    if hp == ep and h == e:
                        blk += x4[mcp, :, mc, :]
                    out[r0:r0 + nmu, c0:c0 + nmu] = blk
    return out


MULT = {"zeta": 0.14, "F2": 0.29, "G1": 0.22, "G3": 0.13}


def local_d_channel_error(mpm):
    """max |K_loc - K_brute| over the restricted and the full-spin d-channel matrices."""
    d, x = coulomb_multipole_blocks([2], np.array([[MULT["F2"]]]),
                                    {1: np.array([[MULT["G1"]]]), 3: np.array([[MULT["G3"]]])})
    e1 = np.abs(mpm.local_matrix(MULT) - _assemble(d, x, 5, False)).max()
    e2 = np.abs(mpm.local_matrix_spin(MULT) - _assemble(d, x, 5, True)).max()
    return max(e1, e2) / MULT["F2"]


def _channel_tables(seed=8):
    rng = np.random.default_rng(seed)
    ls = [0, 1, 2, 2, 3]
    n = len(ls)

    def gram(scale):
        b = rng.normal(size=(n, n))
        return scale * (b @ b.T) / n

    return ls, gram(0.3), {k: gram(0.2) for k in range(5)}


def local_channels_error(mpm):
    """max |K_loc - K_brute| for a general basis (s, p, two d, f channels), both spin models."""
    ls, f2, gk = _channel_tables()
    d, x = coulomb_multipole_blocks(ls, f2, gk)
    nmu = sum(2 * l + 1 for l in ls)
    err = 0.0
    for full in (False, True):
        got = mpm.local_matrix_channels(ls, f2, gk, full_spin=full)
        err = max(err, np.abs(got - _assemble(d, x, nmu, full)).max())
    return err / np.abs(f2).max()


def test_local_direct_and_exchange_equal_the_coulomb_multipole_integrals():
    assert local_d_channel_error(mp) <= 1e-13
    assert local_channels_error(mp) <= 1e-13


def test_brute_force_blocks_have_the_physical_signs():
    """Closed-form checks of the brute force itself: for an electron in d(m = 0) and a hole
    in p(m_c = 0), both elongated along z, the k = 2 direct integral is F2 c^2(20;20) c^2(10;10)
    = F2 (2/7)(2/5) > 0, so -V_D makes this aligned pair's diagonal element negative
    (attraction); the exchange block is positive semidefinite (the Coulomb energy of a charge
    density with itself is never negative), and with G1 alone it has rank 3, one for each
    component of the p-d dipole transition density."""
    d, x = coulomb_multipole_blocks([2], np.array([[1.0]]), {1: np.array([[1.0]])})
    i00 = 1 * 5 + 2                       # (m_c = 0, m = 0)
    assert abs(d[i00, i00] - (2 / 7) * (2 / 5)) <= 1e-14
    assert np.linalg.eigvalsh(x).min() >= -1e-14
    assert np.linalg.matrix_rank(x, tol=1e-10) == 3
    assert abs(np.trace(d)) <= 1e-14      # a full shell averages every k > 0 multipole to zero


def exchange_expectation(mpm, cr):
    """(smallest eigenvalue of K_loc with F2 = 0, <psi0|H|psi0> / |psi0|^2) with H the local term
    alone (E = 0, W = 0, no core matrix) and psi0 the z-polarised dipole vector: bare exchange
    is repulsive (+V_X), so the first is >= 0 and the second > 0."""
    mult = dict(MULT, F2=0.0, zeta=0.0)
    kl = mpm.local_matrix(mult)
    psi0 = mpm.dipole_psi0(cr.local_proj, [0.0, 0.0, 1.0])
    y = bse.apply_local(psi0, cr.local_proj, kl)
    return float(np.linalg.eigvalsh(kl).min()), float(np.vdot(psi0, y).real / np.vdot(psi0, psi0).real)


def test_bare_exchange_is_repulsive():
    lam_min, expect = exchange_expectation(mp, _cubic_l())
    assert lam_min >= -1e-14 and expect > 1e-3 * MULT["G1"]


# --- the planted mistakes: every pin above must reject them ---------------------------------------

def test_planted_w0_sign_is_caught():
    """+W0 in place of -W0, planted in the matrix-free H and, separately, in the explicit H."""
    cr = _cubic_l()
    for old, new in [("out = out - w_scale * apply_w0(", "out = out + w_scale * apply_w0("),
                     ("h[:, :, c, :, :, c] -= w_scale * m", "h[:, :, c, :, :, c] += w_scale * m")]:
        bad = _mutant("bse", old, new)
        assert w0_shift_error(bad, mp, cr) > 1.0
    bad = _mutant("bse", "h[:, :, c, :, :, c] -= w_scale * m", "h[:, :, c, :, :, c] += w_scale * m")
    rise, drop = core_hole_binding(bad, mp, cr)
    assert rise > 1e-3 and drop < 0.0


def test_planted_transposed_reciprocal_lattice_is_caught():
    """inv(A) in place of inv(A)^T: the same on a cubic cell, wrong on a skewed one."""
    bad = _mutant("bse", "np.linalg.inv(cell_vectors(cr)).T", "np.linalg.inv(cell_vectors(cr))")
    for cr in (_skewed_l(), _hexagonal_l()):
        err_u, err_dual = dft_unitarity_error(bad, cr)
        assert err_u > 1e-2 and err_dual > 1e-2
        assert w0_shift_error(bad, mp, cr) > 1e-2
    assert max(dft_unitarity_error(bad, synth.config1())) <= 1e-13     # cubic: blind, as expected


@pytest.mark.parametrize("old,new,occurrence,which", [
    ("val -= d[", "val += d[", 1, "d"),                       # +D in the restricted d-channel matrix
    ("val -= d[", "val += d[", 2, "d"),                       # +D in the full-spin d-channel matrix
    ("blk -= d[", "blk += d[", 1, "channels"),                # +D in the general-basis matrix
    ("val = x[mcp * nv + mp, mc * nv + m]", "val = -x[mcp * nv + mp, mc * nv + m]", 1, "d"),   # -X restricted
    ("val += x[", "val -= x[", 1, "d"),                       # -X in the full-spin matrix
    ("blk += x[", "blk -= x[", 1, "channels"),                # -X in the general-basis matrix
    ("gaunt(2, 1, mcp, 1, mc)", "gaunt(2, 1, mc, 1, mcp)", 1, "channels"),   # hole not conjugated
], ids=["plusD-restricted", "plusD-spin", "plusD-channels", "minusX-restricted", "minusX-spin",
        "minusX-channels", "hole-unconjugated"])
def test_planted_local_sign_is_caught(old, new, occurrence, which):
    bad = _mutant("multiplet", old, new, occurrence)
    err = local_d_channel_error(bad) if which == "d" else local_channels_error(bad)
    assert err > 1e-2


def test_planted_exchange_sign_fails_the_repulsion_pin():
    bad = _mutant("multiplet", "val = x[mcp * nv + mp, mc * nv + m]", "val = -x[mcp * nv + mp, mc * nv + m]")
    lam_min, expect = exchange_expectation(bad, _cubic_l())
    assert lam_min < -1e-3 and expect < 0.0
