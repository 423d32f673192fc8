"""Pins of the CPU oracle to facts outside itself (closed forms, textbook values,
library routines, brute force on tiny inputs, exact identities).

Each test names the passage of the paper whose statement it pins."""
import math

import numpy as np
import pytest

import synth
from oracle import bse
from oracle import multiplet as mp


@pytest.fixture(scope="module")
def c1():
    return synth.config1()


@pytest.fixture(scope="module")
def small_l():
    return synth.small_l_edge(seed=3, nk=(2, 1, 2), nx=(4, 5, 3), n_bands=7)


def _rand(shape, seed=11):
    return synth.complex_gaussian(np.random.default_rng(seed), shape)


# --- H assembly (section 2, eq. H_BSE; section 3.2) ------------------------------------------

def test_dense_h_is_hermitian(c1, small_l):
    """H_BSE is Hermitian once the lifetime -i Gamma is moved into z = w + i Gamma."""
    for cr in (c1, small_l):
        hc = mp.core_matrix(cr.multiplet) if cr.multiplet else None
        kl = mp.local_matrix(cr.multiplet) if cr.multiplet else None
        h = bse.h_dense(cr, hc, kl)
        assert np.abs(h - h.conj().T).max() <= 1e-14 * np.abs(h).max()


def test_matrix_free_equals_dense(c1, small_l):
    for cr in (c1, small_l):
        hc = mp.core_matrix(cr.multiplet) if cr.multiplet else None
        kl = mp.local_matrix(cr.multiplet) if cr.multiplet else None
        h = bse.h_dense(cr, hc, kl)
        psi = _rand((cr.n_k, cr.n_bands, cr.n_core))
        y = bse.apply_h(cr, psi, hc, kl)
        y2 = (h @ psi.ravel()).reshape(psi.shape)
        assert np.abs(y - y2).max() <= 1e-13 * np.abs(y2).max()


def test_w0_matches_supercell_brute_force(small_l):
    """Algorithm 1 equals the plain supercell definition: the matrix element of the
    local potential W(x + R) between normalised Bloch functions
    e^{ik.(R+x)} u_nk(x) / sqrt(Nk) on the Born-von-Karman supercell (section 3.2,
    expansion of Phi_alpha(x, R)).  No DFT matrix is used on this side."""
    _w0_brute_force_check(small_l)


def _w0_brute_force_check(cr, reach=1):
    """W0 of Algorithm 1 against the matrix element of W(x + R - tau) between Bloch
    functions e^{ik.(R+x)} u_nk(x) / sqrt(Nk), built point by point, with the minimum image
    found by trying every supercell translation with coefficients in [-reach, reach]
    (no wrapping)."""
    kv = bse.kpoints(cr)
    rv = bse.lattice_vectors(cr)
    xv = bse.xpoints(cr)
    sup = np.asarray(cr.nk, dtype=float)[:, None] * cr.cell_vectors()
    shifts = [np.array(m) - reach for m in np.ndindex(*(2 * reach + 1,) * 3)]
    bloch = np.zeros((cr.n_k, cr.n_bands, cr.n_x, cr.n_k), dtype=np.complex128)
    wsc = np.zeros((cr.n_x, cr.n_k))
    for ix, x in enumerate(xv):
        for ir, r in enumerate(rv):
            pos = x + r
            best = min(np.linalg.norm(pos - cr.tau + m @ sup) for m in shifts)
            wsc[ix, ir] = bse.w_radial(cr.w_r, cr.w_val, np.array([best]))[0]
            for ik, k in enumerate(kv):
                bloch[ik, :, ix, ir] = np.exp(1j * k @ pos) * cr.u[ik, ix, :] / math.sqrt(cr.n_k)
    b = bloch.reshape(cr.n_k * cr.n_bands, cr.n_x * cr.n_k)
    m_ref = b.conj() @ (wsc.ravel()[:, None] * b.T)
    m = bse.w0_matrix(cr)
    assert np.abs(m - m_ref).max() <= 1e-13 * np.abs(m_ref).max()
    assert np.abs(bse.w_supercell(cr) - wsc).max() <= 1e-15 * wsc.max()


SKEWED = np.array([[7.0, 0.0, 0.0], [2.1, 6.4, 0.0], [-1.3, 1.7, 6.9]])   # a reduced triclinic cell
HEXAGONAL = np.array([[6.0, 0.0, 0.0], [3.0, 3.0 * math.sqrt(3.0), 0.0], [0.0, 0.0, 7.5]])


def test_w0_brute_force_skewed_cell_shifted_grid():
    """The same definition on a triclinic cell with a k grid offset by half a step, with
    images up to two supercell vectors away."""
    cr = synth.small_l_edge(seed=21, nk=(2, 1, 2), nx=(3, 4, 3), n_bands=5)
    cr.lattice = SKEWED
    cr.kshift = (0.5, 0.0, 0.5)
    _w0_brute_force_check(cr, reach=2)


def test_min_image_on_a_60_degree_lattice():
    """Closed forms on the plane hexagonal lattice of spacing L: the midpoint of a1 and
    a2 lies L/2 from the lattice points a1 and a2 (wrapping the fractional coordinates
    alone gives |a1 + a2| / 2 = L sqrt(3)/2, so the image search is needed); the centre of a
    triangle lies L/sqrt(3) from its corners; a lattice point lies at distance 0."""
    L = 6.0
    sup = HEXAGONAL
    a1, a2 = sup[0], sup[1]
    d = np.array([0.5 * (a1 + a2), (a1 + a2) / 3.0, 2.0 * (a1 + a2) / 3.0, a1 - a2, 3 * a1 + 2 * sup[2]])
    got = bse.min_image_distance(d, sup)
    want = np.array([0.5 * L, L / math.sqrt(3.0), L / math.sqrt(3.0), 0.0, 0.0])
    assert np.abs(got - want).max() <= 1e-12 * L


def test_sheared_basis_gives_the_same_supercell_potential():
    """a2' = a1 + a2 spans the same cubic lattice.  With equal counts along a1 and a2
    the x grid, the supercell and hence the set of distances |x + R - tau| are the same, so
    W(x, R) takes the same multiset of values."""
    cr = synth.small_l_edge(seed=22, nk=(2, 2, 1), nx=(4, 4, 3), n_bands=3)
    cr.tau = np.array([1.1, 0.4, 2.3])
    w_cubic = np.sort(bse.w_supercell(cr).ravel())
    cr.lattice = cr.a * np.array([[1.0, 0.0, 0.0], [1.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    w_sheared = np.sort(bse.w_supercell(cr).ravel())
    assert np.abs(w_cubic - w_sheared).max() <= 1e-14 * w_cubic.max()


def test_grid_offset_cancels_in_w0():
    """An offset of the k grid by a fraction of a step cancels in W0: the transforms meet as
    e^{-i(k - k').R} and the Bloch phases as e^{-i(k - k').x}, and k - k' is a whole number
    of steps.  Given u_nk at the offset points, W0 is the same operator as on the unshifted
    grid (the plain definition with the offset is checked point by point in
    test_w0_brute_force_skewed_cell_shifted_grid)."""
    cr = synth.small_l_edge(seed=23, nk=(2, 2, 2), nx=(4, 3, 5), n_bands=6)
    cr.lattice = SKEWED
    psi = _rand((cr.n_k, cr.n_bands, cr.n_core))
    plain = bse.apply_w0(cr, psi)
    cr.kshift = (0.5, 0.25, 0.5)
    shifted = bse.apply_w0(cr, psi)
    assert np.abs(shifted - plain).max() <= 1e-13 * np.abs(plain).max()
    # the offset does change each factor: the folded u and the transform
    assert np.abs(bse.folded_u(cr) - bse.folded_u(synth.small_l_edge(seed=23, nk=(2, 2, 2), nx=(4, 3, 5),
                                                                       n_bands=6))).max() > 0.1 * np.abs(cr.u).max()



def test_constant_w_is_rigid_shift(c1):
    """W = const in the supercell: with orthonormal u and a unitary k<->R pair the
    W0 term is exactly const * identity."""
    psi = _rand((c1.n_k, c1.n_bands, c1.n_core))
    wconst = np.full((c1.n_x, c1.n_k), 0.37)
    y = bse.apply_w0(c1, psi, w=wconst)
    assert np.abs(y - 0.37 * psi).max() <= 1e-13


def test_dft_matrix_is_numpy_fft(small_l):
    """Explicit e^{+ik.R} / sqrt(Nk) equals numpy's inverse FFT times sqrt(Nk)."""
    cr = small_l
    f = bse.dft_matrix(cr)
    g = _rand(cr.n_k, seed=2)
    ref = np.fft.ifftn(g.reshape(cr.nk)).ravel() * math.sqrt(cr.n_k)
    assert np.abs(f @ g - ref).max() <= 1e-14
    assert np.abs(f.conj().T @ f - np.eye(cr.n_k)).max() <= 1e-14


def test_w_radial_interpolation_and_tail(c1):
    r, w = c1.w_r, c1.w_val
    assert np.allclose(bse.w_radial(r, w, r[:-1]), w[:-1], rtol=0, atol=1e-16)
    mid = 0.5 * (r[3] + r[4])
    assert abs(bse.w_radial(r, w, np.array([mid]))[0] - 0.5 * (w[3] + w[4])) < 1e-15
    far = np.array([6.0, 9.0, 12.0])
    assert np.allclose(bse.w_radial(r, w, far), w[-1] * 6.0 / far, rtol=1e-15)
    # erf(r/0.5)/(eps r) is 1/(eps r) at 6 bohr to machine precision
    assert abs(w[-1] - 1.0 / (c1.eps * 6.0)) < 1e-16


# --- independent-particle limit (W = 0: Lorentzians at the band energies) ------------------

def test_ip_limit_closed_form(c1):
    """W = 0, no core matrix, no local term: sigma(w) = (1/pi) sum |psi0|^2 Gamma /
    ((w - E)^2 + Gamma^2).  Haydock at full Krylov depth reproduces it."""
    cr = c1
    psi0 = cr.psi0[0]
    a, b, n2, s, _ = bse.haydock(lambda v: bse.apply_h(cr, v, w_scale=0.0), psi0, 200, reorth=True)
    sig = bse.spectrum(a, b, n2, cr.omega, cr.gamma)
    e = cr.energies[:, :, None] + 0 * psi0.real
    wt = np.abs(psi0) ** 2
    om = cr.omega[:, None]
    ref = np.sum(wt.ravel()[None, :] * cr.gamma / ((om - e.ravel()[None, :]) ** 2 + cr.gamma ** 2),
                 axis=1) / math.pi
    assert s <= 128          # 128 distinct energies: the Krylov space closes
    assert bse.l1_relative(sig, ref) <= 1e-12


# --- Haydock and the continued fraction (section 3.2, eq. haydock1; eq. loss.fcn) -----------

def test_cf_at_full_depth_equals_dense_diagonalisation(c1):
    cr = c1
    h = bse.h_dense(cr)
    psi0 = cr.psi0[0]
    a, b, n2, s, _ = bse.haydock(lambda v: (h @ v.ravel()).reshape(v.shape), psi0, 128, reorth=True)
    sig = bse.spectrum(a, b, n2, cr.omega, cr.gamma)
    ref = bse.spectrum_dense(h, psi0, cr.omega, cr.gamma)
    assert bse.l1_relative(sig, ref) <= 1e-12
    # at 100 steps the recursion is not yet exact (truncation), as expected
    sig100 = bse.spectrum(a[:100], b[:100], n2, cr.omega, cr.gamma)
    assert bse.l1_relative(sig100, ref) > 1e-7


def test_cf_equals_tridiagonal_resolvent(c1):
    """Exact at any depth: g_N(z) = [(z - T_N)^-1]_00 with T_N the Lanczos matrix."""
    rng = np.random.default_rng(4)
    a = rng.uniform(-1, 1, 37)
    b = rng.uniform(0.1, 1, 37)
    t = np.diag(a) + np.diag(b[:-1], 1) + np.diag(b[:-1], -1)
    lam, q = np.linalg.eigh(t)
    z = np.linspace(-3, 3, 101) + 0.05j
    ref = np.sum(q[0, :][None, :] ** 2 / (z[:, None] - lam[None, :]), axis=1)
    g = bse.continued_fraction(a, b, z)
    assert np.abs(g - ref).max() <= 1e-12 * np.abs(ref).max()


def test_haydock_moments(small_l):
    """a_0 = <v0|H|v0>, b_1^2 = <v0|H^2|v0> - a_0^2, and the Ritz values stay in the spectrum."""
    cr = small_l
    hc = mp.core_matrix(cr.multiplet)
    kl = mp.local_matrix(cr.multiplet)
    h = bse.h_dense(cr, hc, kl)
    psi0 = _rand(cr.n_k * cr.n_bands * cr.n_core, seed=9)
    v0 = psi0 / np.linalg.norm(psi0)
    a, b, n2, s, _ = bse.haydock(lambda v: h @ v, psi0, 12)
    m1 = np.vdot(v0, h @ v0).real
    m2 = np.vdot(h @ v0, h @ v0).real
    assert abs(a[0] - m1) <= 1e-14 * abs(m1) + 1e-16
    assert abs(b[0] ** 2 - (m2 - m1 ** 2)) <= 1e-12 * m2
    lam = np.linalg.eigvalsh(h)
    t = np.diag(a) + np.diag(b[:-1], 1) + np.diag(b[:-1], -1)
    ritz = np.linalg.eigvalsh(t)
    assert ritz.min() >= lam.min() - 1e-12 and ritz.max() <= lam.max() + 1e-12
    assert abs(n2 - np.vdot(psi0, psi0).real) <= 1e-14 * n2


def test_breakdown_on_eigenvector(c1):
    """psi0 = one basis vector with W = 0 is an eigenvector: b_1 = 0 and the recursion stops."""
    psi0 = np.zeros((c1.n_k, c1.n_bands, c1.n_core), dtype=np.complex128)
    psi0[1, 3, 0] = 1.0
    a, b, n2, s, _ = bse.haydock(lambda v: bse.apply_h(c1, v, w_scale=0.0), psi0, 10)
    assert s == 1 and abs(a[0] - c1.energies[1, 3]) < 1e-15 and b[0] == 0.0


def test_spin_doubling(c1):
    """K edge without spin-orbit: the two spin blocks are identical, so the
    two-spin recursion equals the one-spin recursion with twice the weight."""
    psi0 = c1.psi0[0]
    a2, b2, n22, _, _ = bse.haydock(lambda v: bse.apply_h(c1, v), psi0, 40, reorth=True)
    one = psi0[:, :, :1].copy()
    a1, b1, n21, _, _ = bse.haydock(lambda v: bse.apply_h(c1, v), one, 40, reorth=True)
    assert np.abs(a2 - a1).max() <= 1e-13 and np.abs(b2 - b1).max() <= 1e-13
    assert abs(n22 - 2 * n21) <= 1e-12 * n22


def test_sqrt_terminator_fixed_point_and_semicircle():
    """The square-root terminator is the exact Green's function of a constant chain:
    t = 1/(z - a - b^2 t), and -Im t / pi tends to the semicircle sqrt(4b^2-(w-a)^2)/(2 pi b^2)."""
    a_inf, b_inf = 0.3, 0.7
    z = np.linspace(-2, 2, 201) + 1e-3j
    t = bse.sqrt_terminator(z, a_inf, b_inf)
    assert np.all(t.imag <= 0)
    assert np.abs(t - 1.0 / (z - a_inf - b_inf ** 2 * t)).max() <= 1e-12
    g = bse.continued_fraction(np.full(9, a_inf), np.full(9, b_inf), z, "sqrt", a_inf, b_inf)
    assert np.abs(g - t).max() <= 1e-10
    w = np.array([0.0, 0.5, 1.0])
    dos = -bse.sqrt_terminator(w + 1e-12j, a_inf, b_inf).imag / math.pi
    ref = np.sqrt(4 * b_inf ** 2 - (w - a_inf) ** 2) / (2 * math.pi * b_inf ** 2)
    assert np.allclose(dos, ref, rtol=1e-9)


# --- core matrix and the local short-range term (section 2 H_h; section 3.2.2) ----------------

def test_spin_orbit_spectrum():
    chi = mp.spin_orbit(1, 1.7)
    lam = np.sort(np.linalg.eigvalsh(chi))
    assert np.allclose(lam, [-1.7, -1.7, 0.85, 0.85, 0.85, 0.85], atol=1e-14)


def test_l3_l2_branching_ratio():
    """Independent-particle L2,3 edge with flat bands: summing the dipole spectra of
    three orthogonal polarisations gives the statistical 2:1 L3:L2 weight ratio
    (L3 at -zeta/2, L2 at +zeta relative to the band energy)."""
    cr = synth.small_l_edge(seed=5, nk=(1, 1, 1), nx=(3, 3, 3), n_bands=20)
    cr.energies[:] = 0.1
    hc = mp.core_matrix(cr.multiplet)
    zeta = cr.multiplet["zeta"]
    h = bse.h_dense(cr, hc, None, w_scale=0.0)
    lam, q = np.linalg.eigh(h)
    w_l3 = w_l2 = 0.0
    for pol in np.eye(3):
        p0 = mp.dipole_psi0(cr.local_proj, pol).ravel()
        wt = np.abs(q.conj().T @ p0) ** 2
        w_l3 += wt[np.abs(lam - (0.1 - zeta / 2)) < 1e-9].sum()
        w_l2 += wt[np.abs(lam - (0.1 + zeta)) < 1e-9].sum()
    assert w_l2 > 0 and abs(w_l3 / w_l2 - 2.0) < 1e-12


def test_gaunt_against_sympy_and_textbook():
    """Quadrature Gaunt coefficients equal sympy's exact Gaunt integrals, and the
    classic values c^2(20;20) = 2/7, c^2(10;10) = 2/5, c^2(11;11) = -1/5."""
    from sympy.physics.wigner import gaunt as gaunt_exact
    for (k, l, lp) in [(2, 2, 2), (2, 1, 1), (1, 2, 1), (3, 2, 1), (0, 2, 2)]:
        for m in range(-l, l + 1):
            for mp_ in range(-lp, lp + 1):
                q = m - mp_
                if abs(q) > k:
                    continue
                exact = float(gaunt_exact(l, k, lp, -m, q, mp_)) * (-1) ** m * math.sqrt(
                    4 * math.pi / (2 * k + 1))
                assert abs(mp.gaunt(k, l, m, lp, mp_) - exact) <= 1e-14
    assert abs(mp.gaunt(2, 2, 0, 2, 0) - 2 / 7) < 1e-14
    assert abs(mp.gaunt(2, 1, 0, 1, 0) - 2 / 5) < 1e-14
    assert abs(mp.gaunt(2, 1, 1, 1, 1) + 1 / 5) < 1e-14


def test_local_matrix_structure():
    mult = {"F2": 0.3, "G1": 0.2, "G3": 0.1}
    k = mp.local_matrix(mult)
    assert np.abs(k - k.conj().T).max() <= 1e-15
    x = mp.exchange_matrix({1: 0.2, 3: 0.1})
    assert np.linalg.eigvalsh(x).min() >= -1e-14
    x1 = mp.exchange_matrix({1: 1.0})
    assert np.linalg.matrix_rank(x1, tol=1e-10) == 3
    # K commutes with M = m - m_c (the e-h pair's total m) and with the spin flip
    mvals = np.array([(m - 2) - (c // 2 - 1) for c in range(6) for m in range(5)])
    kk = np.abs(k) > 1e-14
    rows, cols = np.nonzero(kk)
    assert np.all(mvals[rows] == mvals[cols])
    flip = np.zeros((30, 30))
    for c in range(6):
        for m in range(5):
            flip[(c ^ 1) * 5 + m, c * 5 + m] = 1.0
    assert np.abs(flip @ k - k @ flip).max() <= 1e-15


def test_local_term_acts_as_k_on_local_states(small_l):
    """With A orthonormal over (k, n) and E = 0, W = 0, no core matrix, the
    short-range term has the spectrum of K_loc (plus zeros): projecting onto the
    local basis and back is exact on those states."""
    cr = small_l
    kl = mp.local_matrix(cr.multiplet)
    saved = cr.energies.copy()
    cr.energies[:] = 0.0
    try:
        h = bse.h_dense(cr, None, kl, w_scale=0.0)
    finally:
        cr.energies[:] = saved
    lam = np.sort(np.linalg.eigvalsh(h))
    kl_lam = np.sort(np.linalg.eigvalsh(kl))
    nz = lam[np.abs(lam) > 1e-12]
    knz = kl_lam[np.abs(kl_lam) > 1e-12]
    assert len(nz) == len(knz) and np.allclose(nz, knz, atol=1e-13)


def test_dipole_amplitudes():
    """<Y_20 | z | Y_10> = sqrt(4/15); dipole selection rule |m - m_c| <= 1;
    summed over x, y, z the strength out of each m_c is the same (isotropy)."""
    dz = mp.dipole_amplitudes([0, 0, 1])
    assert abs(dz[2, 1] - math.sqrt(4 / 15)) < 1e-14
    for pol in np.eye(3):
        d = mp.dipole_amplitudes(pol)
        for m in range(5):
            for mc in range(3):
                if abs((m - 2) - (mc - 1)) > 1:
                    assert abs(d[m, mc]) < 1e-14
    tot = sum(np.abs(mp.dipole_amplitudes(p)) ** 2 for p in np.eye(3)).sum(axis=0)
    assert np.allclose(tot, tot[0], rtol=1e-13)
