"""Pins of the general local basis of the oracle (channels of l = s, p, d, f with several
radial functions, section 3.2.2):

* with one d channel it is the pinned d-channel matrix, in both spin models;
* rotational invariance: the direct and exchange interactions are scalars under a joint
  rotation of the electron and the hole, so K commutes with the pair's total angular
  momentum J = -L*_core + L_val (the hole carries the conjugate representation); this
  fixes the relative phases of the Gaunt factors, including the odd Delta m elements, and
  the same check with the hole's generator taken as +L_core fails;
* the exchange part is a sum of Gram matrices, so it is positive semidefinite when every
  G^k table is;
* dipole amplitudes: one d channel gives the pinned d-channel vector, and an s channel
  gives <Y_00 | cos theta | Y_10> = 1/sqrt(3) for light along z."""
import math

import numpy as np

from oracle import multiplet as mp

LS = [0, 1, 2, 3, 2]     # s, p, d, f and a second d radial function


def _psd(rng, n):
    a = rng.normal(size=(n, n))
    return a @ a.T / n


def _tables(seed=0):
    rng = np.random.default_rng(seed)
    n = len(LS)
    return _psd(rng, n), {k: _psd(rng, n) for k in range(5)}


def _generators(ls, hole_sign):
    off, nmu = mp.channel_offsets(ls)
    lc = mp.angular_momentum(1)
    gens = []
    for a in range(3):
        lv = np.zeros((nmu, nmu), dtype=np.complex128)
        for i, l in enumerate(ls):
            lv[off[i]:off[i] + 2 * l + 1, off[i]:off[i] + 2 * l + 1] = mp.angular_momentum(l)[a]
        core = -np.conj(lc[a]) if hole_sign < 0 else lc[a]
        gens.append(np.kron(np.kron(core, np.eye(2)), np.eye(nmu)) + np.kron(np.eye(6), lv))
    return gens


def test_single_d_channel_is_the_pinned_matrix():
    m = {"zeta": 0.14, "F2": 0.29, "G1": 0.22, "G3": 0.13}
    f2 = np.array([[m["F2"]]])
    gk = {1: np.array([[m["G1"]]]), 3: np.array([[m["G3"]]])}
    assert np.abs(mp.local_matrix_channels([2], f2, gk) - mp.local_matrix(m)).max() == 0.0
    assert np.abs(mp.local_matrix_channels([2], f2, gk, full_spin=True) - mp.local_matrix_spin(m)).max() == 0.0


def test_local_matrix_is_rotationally_invariant():
    f2, gk = _tables()
    k = mp.local_matrix_channels(LS, f2, gk)
    scale = np.abs(k).max()
    for j in _generators(LS, -1):
        assert np.abs(k @ j - j @ k).max() <= 1e-13 * scale
    wrong = _generators(LS, +1)
    assert max(np.abs(k @ j - j @ k).max() for j in wrong) > 1e-2 * scale


def test_exchange_is_positive_semidefinite_and_hermitian():
    f2, gk = _tables(seed=1)
    x = mp.exchange_matrix_channels(LS, gk)
    assert np.abs(x - x.T).max() <= 1e-15 * np.abs(x).max()
    assert np.linalg.eigvalsh(x).min() >= -1e-13 * np.abs(x).max()
    k = mp.local_matrix_channels(LS, f2, gk, full_spin=True)
    assert np.abs(k - k.conj().T).max() <= 1e-15 * np.abs(k).max()


def test_dipole_amplitudes_of_channels():
    rng = np.random.default_rng(2)
    a5 = rng.normal(size=(3, 4, 5)) + 1j * rng.normal(size=(3, 4, 5))
    pol = [0.3, -0.5, 0.8]
    assert np.abs(mp.dipole_psi0_channels(a5, [2], [1.0], pol) - mp.dipole_psi0(a5, pol)).max() <= 1e-15
    assert np.abs(mp.dipole_psi0_channels(a5, [2], [1.0], pol, full_spin=True)
                  - mp.dipole_psi0_spin(a5, pol)).max() <= 1e-15
    one = np.ones((1, 1, 1), dtype=np.complex128)       # A = 1 on a single s function
    p = mp.dipole_psi0_channels(one, [0], [1.0], [0.0, 0.0, 1.0])
    # core index (m_c, sigma): m_c = 0 sits at 2 and 3
    assert abs(p[0, 0, 2] - 1.0 / math.sqrt(3.0)) <= 1e-14 and abs(p[0, 0, 3] - 1.0 / math.sqrt(3.0)) <= 1e-14
    assert np.abs(p[0, 0, [0, 1, 4, 5]]).max() <= 1e-15
