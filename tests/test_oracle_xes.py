"""Pins of the emission (XES) reading of the oracle (oracle/xes.py) to things other than
itself:

* without the core-hole interaction the BSE path over the occupied window (Haydock at full
  depth, continued fraction; oracle/bse.py) gives the closed-form amplitude-weighted
  occupied density of states, and so does the eigen-decomposition of the dense H;
* one band and one core state: the spectrum is the textbook Lorentzian, with its peak
  height |psi0|^2 / (pi Gamma) at the line;
* the sum rule: the spectrum integrates to |psi0|^2 (less the Lorentzian tails outside the
  grid, 2 Gamma / (pi L) for a grid reaching L past the band);
* with the core-hole interaction the recursion matches the dense resolvent of the same H
  over the occupied window;
* a planted mistake (the lines put at -E, the absorption-side mirror) fails the first pin."""
import math

import numpy as np

import synth
from oracle import bse as orc
from oracle import xes


def _site(seed=3, n_occ=12, grid=6):
    return synth.xes_site(seed, n_occ=n_occ, grid=grid, box=12.0)


def test_xes_site_is_an_occupied_window():
    cr = _site()
    assert xes.is_occupied_window(cr.energies)
    assert cr.n_core == 2 and cr.n_k == 1 and cr.psi0.shape == (3, 1, 12, 2)


def test_one_particle_limit_is_the_occupied_dos():
    cr = _site()
    dim = cr.dim
    h0 = orc.h_dense(cr, w_scale=0.0)
    for v in range(3):
        p0 = cr.psi0[v]
        a, b, n2, s, _ = orc.haydock(lambda x: orc.apply_h(cr, x, w_scale=0.0), p0, dim, reorth=True)
        sig = orc.spectrum(a, b, n2, cr.omega, cr.gamma)
        ref = xes.occupied_dos_spectrum(cr.energies, p0, cr.omega, cr.gamma)
        assert np.abs(sig - ref).max() <= 1e-10 * ref.max(), (v, s)
        dense = orc.spectrum_dense(h0, p0, cr.omega, cr.gamma)
        assert np.abs(dense - ref).max() <= 1e-10 * ref.max()
        # the planted mistake: emission lines mirrored to -E
        wrong = xes.occupied_dos_spectrum(-cr.energies, p0, cr.omega, cr.gamma)
        assert np.abs(wrong - sig).max() > 0.1 * ref.max()


def test_single_line_is_the_textbook_lorentzian():
    e = np.array([[-0.3]])
    amp = np.array([[[0.6 - 0.8j]]])          # |psi0|^2 = 1
    g = 0.02
    om = np.array([-0.3, -0.3 + g, -0.3 - 2 * g])
    sig = xes.occupied_dos_spectrum(e, amp, om, g)
    assert abs(sig[0] - 1.0 / (math.pi * g)) <= 1e-12 / g
    assert abs(sig[1] - 0.5 / (math.pi * g)) <= 1e-12 / g     # half maximum at one half width
    assert abs(sig[2] - 0.2 / (math.pi * g)) <= 1e-12 / g


def test_sum_rule():
    cr = _site(seed=5, n_occ=10)
    p0 = cr.psi0[0]
    lo, hi = cr.energies.min(), cr.energies.max()
    reach = 400 * cr.gamma
    om = np.linspace(lo - reach, hi + reach, 400001)
    sig = xes.occupied_dos_spectrum(cr.energies, p0, om, cr.gamma)
    total = float(np.sum(np.abs(p0) ** 2))
    integral = float(np.trapezoid(sig, om)) if hasattr(np, "trapezoid") else float(np.trapz(sig, om))
    tails = 2 * cr.gamma / (math.pi * reach) * total
    assert abs(integral - total) <= 1.5 * tails + 1e-6 * total
    assert integral < total


def test_with_core_hole_matches_the_dense_resolvent():
    cr = _site(seed=7, n_occ=10)
    dim = cr.dim
    h = orc.h_dense(cr)
    p0 = cr.psi0[1]
    a, b, n2, s, _ = orc.haydock(lambda x: orc.apply_h(cr, x), p0, dim, reorth=True)
    sig = orc.spectrum(a, b, n2, cr.omega, cr.gamma)
    dense = orc.spectrum_dense(h, p0, cr.omega, cr.gamma)
    assert np.abs(sig - dense).max() <= 1e-10 * dense.max()
    # the interaction moves weight: the spectrum differs from the one-particle form
    free = xes.occupied_dos_spectrum(cr.energies, p0, cr.omega, cr.gamma)
    assert np.abs(sig - free).max() > 1e-3 * free.max()
