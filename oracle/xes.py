"""Plain FP64 reference of the x-ray emission (XES) spectrum on the BSE path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the GPU library and never calls it.

The paper (Gilmore et al., section 1 and section 4.5) lists XES among the spectra the
method produces and states that absorption probes the unoccupied and emission the occupied
density of states; it gives no separate formula for emission.  Reading taken here:

* Emission is the same loss function (section 2, eq. loss.fcn) with the same Hamiltonian
  (eq. H_BSE) over the occupied band window: the pair is the core hole and the valence
  electron that fills it.  Band energies below the Fermi level enter the diagonal as they
  are, so the emission lines sit at E_v - E_c (eps_c = 0), and the transition amplitudes
  connect the core level with the occupied bands.  Nothing in the operator changes sign.
* Without the core-hole interaction (W = 0, no local term, no core matrix) the spectrum is
  the amplitude-weighted occupied density of states, the statement the paper makes:
    sigma(w) = (1/pi) sum_{k, v, c} |psi0[k, v, c]|^2 Gamma / ((w - E[k, v])^2 + Gamma^2).
  ``occupied_dos_spectrum`` writes that sum out; it is the closed form the XES path must
  reach in that limit.
* Resonant scattering (RIXS) needs the absorption intermediate state carried into a
  valence-conduction final state, a second Hamiltonian the paper does not describe; it is
  not covered.
"""
from __future__ import annotations

import math

import numpy as np


def occupied_dos_spectrum(energies, psi0, omega, gamma):
    """Amplitude-weighted occupied density of states, Lorentzian half width gamma.

    energies [Nk, Nb] (Ha, the occupied window), psi0 [Nk, Nb, Nc] complex amplitudes,
    omega [n] (Ha).  Returns sigma [n]."""
    wts = np.sum(np.abs(np.asarray(psi0)) ** 2, axis=-1).ravel()      # sum over core states
    lines = np.asarray(energies, dtype=np.float64).ravel()
    om = np.asarray(omega, dtype=np.float64)[:, None]
    return np.sum(wts[None, :] * gamma / ((om - lines[None, :]) ** 2 + gamma ** 2), axis=1) / math.pi


def is_occupied_window(energies, fermi=0.0):
    """True when every band of the window lies at or below the Fermi level."""
    return bool(np.all(np.asarray(energies) <= fermi))
