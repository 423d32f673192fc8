"""Pins of the screening oracle (section 3.3): the imaginary-axis quadrature of
eq. chi_rpa against the static Adler-Wiser closed form (the same integral done by partial
fractions), the symmetry and sign of the static response, and the Green's function of
eq. greens.fcn against its defining sum, element by element."""
import numpy as np

import synth
from oracle import screening as sc


def test_imaginary_axis_quadrature_reaches_the_adler_wiser_sum():
    psi, eps, mu, t, w = synth.screening_inputs(seed=1, n_points=60, n_states=120, n_occ=40, n_t=64)
    quad = sc.chi0_imaginary_axis(psi, eps, mu, t, w)
    closed = sc.chi0_adler_wiser(psi, eps, mu)
    assert np.abs(quad - closed).max() <= 1e-12 * np.abs(closed).max()
    # with few nodes the quadrature is visibly off, so the check is not vacuous
    psi, eps, mu, t, w = synth.screening_inputs(seed=1, n_points=60, n_states=120, n_occ=40, n_t=8)
    assert np.abs(sc.chi0_imaginary_axis(psi, eps, mu, t, w) - closed).max() > 1e-6 * np.abs(closed).max()


def test_static_response_is_symmetric_and_negative():
    """chi0 = -sum_{o,u} (2 / (eps_u - eps_o)) Re[v v^H], v = psi_o psi_u*: real, symmetric
    and negative semidefinite."""
    psi, eps, mu, t, w = synth.screening_inputs(seed=2, n_points=50, n_states=90, n_occ=30, n_t=48)
    chi = sc.chi0_imaginary_axis(psi, eps, mu, t, w)
    assert np.abs(chi - chi.T).max() <= 1e-15 * np.abs(chi).max()
    assert np.linalg.eigvalsh(chi).max() <= 1e-13 * np.abs(chi).max()


def test_green_function_elements_by_the_defining_sum():
    psi, eps, mu, t, w = synth.screening_inputs(seed=3, n_points=20, n_states=40, n_occ=12, n_t=4)
    g = sc.greens_function(psi, eps, mu, t[1])
    for r, rp in [(0, 0), (3, 17), (19, 2)]:
        ref = sum(psi[r, s] * np.conj(psi[rp, s]) / (mu + 1j * t[1] - eps[s]) for s in range(40))
        assert abs(g[r, rp] - ref) <= 1e-14 * abs(ref)   # 40 terms in another order


def test_no_occupied_states_means_no_response():
    """Every term needs one occupied and one empty state."""
    psi, eps, mu, t, w = synth.screening_inputs(seed=4, n_points=15, n_states=30, n_occ=0, n_t=48)
    chi = sc.chi0_imaginary_axis(psi, eps, mu, t, w)
    scale = np.abs(sc.chi0_imaginary_axis(*synth.screening_inputs(seed=4, n_points=15, n_states=30,
                                                                    n_occ=10, n_t=48))).max()
    assert np.abs(chi).max() <= 1e-12 * scale
    assert np.abs(sc.chi0_adler_wiser(psi, eps, mu)).max() == 0.0
