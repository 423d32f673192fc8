"""Plain FP64 reference of the RPA screening response of section 3.3 (Screening).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code with the
GPU library and never calls it.

* Green's function on the real-space grid at imaginary frequency (eq. greens.fcn):
  G(r, r', mu + i t) = sum_s psi_s(r) psi_s*(r') / (mu + i t - eps_s).
* Static response (eq. chi_rpa at omega = 0), the frequency integral taken along the
  imaginary axis through mu:  chi0(r, r') = (1/2 pi) int_{-inf}^{inf} dt G(r, r', mu + it) G(r', r, mu + it).
  The integrand at -t is the complex conjugate of the one at t, so
  chi0(r, r') = (1/pi) int_0^inf dt Re[G(r, r', mu + it) G(r', r, mu + it)], summed with
  caller-given nodes and weights.
* The same integral done exactly (partial fractions, int dt/2pi 1/(x + it) = sign(x)/2)
  gives the static Adler-Wiser sum over occupied o and empty u states:
  chi0(r, r') = sum_{o,u} 2 Re[psi_o(r) psi_o*(r') psi_u(r') psi_u*(r)] / (eps_o - eps_u).

Reading: one spin channel (no factor 2); psi are the Bloch functions already on the grid
(the paper projects them from its optimal basis functions, which is outside this path).
"""
from __future__ import annotations

import math

import numpy as np


def greens_function(psi, eps, mu, t):
    """G[r, r'] at z = mu + i t: explicit sum over states, psi[r, s]."""
    g = 1.0 / (mu + 1j * t - eps)
    return (psi * g[None, :]) @ psi.conj().T


def chi0_imaginary_axis(psi, eps, mu, t_nodes, weights):
    """chi0 by the quadrature sum over imaginary frequencies (see module docstring)."""
    out = np.zeros((psi.shape[0], psi.shape[0]))
    for t, w in zip(t_nodes, weights):
        g = greens_function(psi, eps, mu, t)
        out += (w / math.pi) * np.real(g * g.T)
    return out


def chi0_adler_wiser(psi, eps, mu):
    """The closed form: sum over occupied/empty pairs of 2 Re[...] / (eps_o - eps_u)."""
    occ = eps < mu
    po, pu = psi[:, occ], psi[:, ~occ]
    eo, eu = eps[occ], eps[~occ]
    out = np.zeros((psi.shape[0], psi.shape[0]))
    for j in range(pu.shape[1]):
        # pair functions v_o(r) = psi_o(r) psi_u*(r) for this empty state u
        v = po * pu[:, j].conj()[:, None]                      # [r, o]
        c = 1.0 / (eo - eu[j])                                  # [o]
        out += 2.0 * np.real((v * c[None, :]) @ v.conj().T)
    return out


def chi0_element(psi, eps, mu, t_nodes, weights, r, rp):
    """One element chi0[r, r'] of the quadrature sum, from the two grid rows alone."""
    out = 0.0
    for t, w in zip(t_nodes, weights):
        g = 1.0 / (mu + 1j * t - eps)
        grr = np.sum(psi[r] * g * np.conj(psi[rp]))
        gpr = np.sum(psi[rp] * g * np.conj(psi[r]))
        out += (w / math.pi) * float(np.real(grr * gpr))
    return out
