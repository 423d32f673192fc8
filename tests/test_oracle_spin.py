"""Pins of the full electron x hole spin space of the oracle (12 core states
(m_c, sigma_h, sigma_e)), against the restricted model, which the other pins fix.

* zeta = 0: nothing flips the hole spin, the direct term keeps both spins and the
  exchange term maps aligned pairs to aligned pairs, so the aligned pairs span an invariant
  subspace isometric to the restricted space: the recursion from the dipole vector is the
  restricted one.
* no exchange: the full H is the restricted H (with its exchange removed) times the
  identity on the electron spin, so every eigenvalue appears twice.
* the exchange part annihilates every pair whose electron and hole spins differ (a pair is
  annihilated and another created, with spin conserved)."""
import numpy as np
import pytest

import synth
from oracle import bse
from oracle import multiplet as mp

HA = synth.HARTREE_EV


def _crystal(zeta_ev=3.8, g_ev=(6.0, 3.5), seed=5):
    cr = synth.small_l_edge(seed=seed, nk=(2, 1, 2), nx=(4, 4, 3), n_bands=6)
    cr.multiplet = {"zeta": zeta_ev / HA, "F2": 8.0 / HA, "G1": g_ev[0] / HA, "G3": g_ev[1] / HA}
    return cr


def _haydock(cr, hc, kl, psi0, n):
    return bse.haydock(lambda v: bse.apply_h(cr, v, hc, kl), psi0, n, reorth=True)


def test_zero_spin_orbit_full_space_recursion_is_the_restricted_one():
    cr = _crystal(zeta_ev=0.0)
    full = synth.full_spin(cr)
    m = cr.multiplet
    p_r = mp.dipole_psi0(cr.local_proj, [0.3, -0.5, 0.8])
    p_f = mp.dipole_psi0_spin(cr.local_proj, [0.3, -0.5, 0.8])
    a_r, b_r, n_r, _, _ = _haydock(cr, mp.core_matrix(m), mp.local_matrix(m), p_r, 40)
    a_f, b_f, n_f, _, _ = _haydock(full, mp.core_matrix_spin(m), mp.local_matrix_spin(m), p_f, 40)
    scale = np.abs(a_r).max() + 2 * np.abs(b_r).max()
    assert abs(n_f - n_r) <= 1e-14 * n_r
    assert np.abs(a_f - a_r).max() <= 1e-12 * scale
    assert np.abs(b_f - b_r).max() <= 1e-12 * scale


def test_without_exchange_every_level_appears_twice():
    cr = _crystal(g_ev=(0.0, 0.0))
    full = synth.full_spin(cr)
    m = cr.multiplet
    h_r = bse.h_dense(cr, mp.core_matrix(m), mp.local_matrix(m))
    h_f = bse.h_dense(full, mp.core_matrix_spin(m), mp.local_matrix_spin(m))
    assert np.abs(h_f - h_f.conj().T).max() <= 1e-14 * np.abs(h_f).max()
    ev_r = np.linalg.eigvalsh(h_r)
    ev_f = np.linalg.eigvalsh(h_f)
    assert np.abs(ev_f - np.sort(np.repeat(ev_r, 2))).max() <= 1e-12 * np.abs(ev_r).max()
    # and with exchange the doubling is lifted (the check is not vacuous)
    m2 = _crystal().multiplet
    ev_x = np.linalg.eigvalsh(bse.h_dense(full, mp.core_matrix_spin(m2), mp.local_matrix_spin(m2)))
    ev_rx = np.linalg.eigvalsh(bse.h_dense(cr, mp.core_matrix(m2), mp.local_matrix(m2)))
    assert np.abs(ev_x - np.sort(np.repeat(ev_rx, 2))).max() > 1e-4 * np.abs(ev_rx).max()


def test_exchange_only_touches_aligned_pairs():
    m = _crystal().multiplet
    m0 = dict(m, G1=0.0, G3=0.0)
    x = mp.local_matrix_spin(m) - mp.local_matrix_spin(m0)
    assert np.abs(mp.local_matrix_spin(m) - mp.local_matrix_spin(m).conj().T).max() <= 1e-15
    idx = np.arange(60)
    c = idx // 5
    aligned = ((c // 2) % 2) == (c % 2)
    assert np.abs(x[:, ~aligned]).max() == 0.0 and np.abs(x[~aligned, :]).max() == 0.0
    assert np.abs(x[np.ix_(aligned, aligned)]).max() > 0.1 * (m["G1"])
    # on the aligned pairs it is the restricted exchange block
    xr = mp.local_matrix(m) - mp.local_matrix(m0)
    assert np.abs(x[np.ix_(aligned, aligned)] - xr).max() <= 1e-15


def test_full_spin_dipole_excites_aligned_pairs_only():
    cr = _crystal()
    p = mp.dipole_psi0_spin(cr.local_proj, [0.0, 0.0, 1.0])
    c = np.arange(12)
    assert np.abs(p[:, :, ((c // 2) % 2) != (c % 2)]).max() == 0.0
    assert abs(np.sum(np.abs(p) ** 2) - np.sum(np.abs(mp.dipole_psi0(cr.local_proj, [0.0, 0.0, 1.0])) ** 2)) <= 1e-12
