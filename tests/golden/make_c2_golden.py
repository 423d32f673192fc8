"""Writes the golden Haydock coefficients and spectra of the SrTiO3-shaped Ti L2,3 edge from the
CPU oracle alone.

Workload: 5-atom cubic cell a = 7.38 bohr with the core site at the Ti position, 8^3 k grid,
96 bands with energies U[0, 40] eV, 20^3 real-space grid, 2p core (6 spin-orbitals,
zeta = 3.8 eV), d-channel local term (F2 = 8, G1 = 6, G3 = 3.5 eV), W(r) = erf(r/0.5)/(6r);
H dimension 294,912.  Inputs come from `synth.config2_shape(seed=0)`: u_nk drawn on the host and
orthonormalised per k by numpy's QR.  Start vectors: the dipole operator for x, y and z
polarisations (section 2, eq. loss.fcn).  Recursion: the Haydock (three-term Lanczos) recursion
of section 3.2, eq. haydock1, with full re-orthogonalisation, so that every coefficient is
unique; 300 steps.  Spectrum: eq. loss.fcn as a continued fraction with no terminator,
Lorentzian half width 0.5 eV, 2000 points on [-25, 55] eV.

Only `oracle/` and the input generator `synth` are called.  Outputs (text, beside this file):
  c2_l23_coefficients.txt   polarisation, step i, a_i, b_{i+1}
  c2_l23_norm2.txt          polarisation, |psi0|^2
  c2_l23_spectra.txt        omega (Ha), sigma_x, sigma_y, sigma_z

Usage: python tests/golden/make_c2_golden.py [n_steps]   (about an hour on 8 cores, 16 GB)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth                                   # noqa: E402
from oracle import bse                         # noqa: E402
from oracle import multiplet as mp             # noqa: E402


def main(n_steps=300, seed=0):
    t0 = time.time()
    cr = synth.config2_shape(seed=seed, psi0="none")
    print(f"inputs drawn in {time.time() - t0:.0f} s", flush=True)
    hc = mp.core_matrix(cr.multiplet)
    kl = mp.local_matrix(cr.multiplet)
    ut = bse.folded_u(cr)
    w = bse.w_supercell(cr)
    f = bse.dft_matrix(cr)
    cr.u = None                                # the folded copy is all that H*v reads
    calls = [0, time.time()]

    def apply(v):
        calls[0] += 1
        if calls[0] % 25 == 0:
            dt = time.time() - calls[1]
            print(f"  {calls[0]} H*v, {dt / 25:.2f} s each", flush=True)
            calls[1] = time.time()
        return bse.apply_h(cr, v, hc, kl, ut=ut, w=w, f=f)

    header = (f"SrTiO3-shaped Ti L2,3 edge, seed {seed}, H dimension {cr.dim}; Haydock recursion with full "
              f"re-orthogonalisation, {n_steps} steps; written by tests/golden/make_c2_golden.py from the CPU oracle")
    coef, norms, sig = [], [], []
    for p, pol in enumerate(np.eye(3)):
        psi0 = mp.dipole_psi0(cr.local_proj, pol)
        a, b, n2, s, _ = bse.haydock(apply, psi0, n_steps, reorth=True)
        assert s == n_steps, f"the recursion stopped after {s} steps"
        coef += [(p, i, a[i], b[i]) for i in range(n_steps)]
        norms.append((p, n2))
        sig.append(bse.spectrum(a, b, n2, cr.omega, cr.gamma))
        short = bse.spectrum(a[:n_steps - 50], b[:n_steps - 50], n2, cr.omega, cr.gamma)
        print(f"polarisation {p}: spectrum L1 between {n_steps - 50} and {n_steps} steps "
              f"{bse.l1_relative(short, sig[-1]):.2e} ({time.time() - t0:.0f} s)", flush=True)
    np.savetxt(os.path.join(HERE, "c2_l23_coefficients.txt"), np.array(coef), fmt=["%d", "%d", "%.17e", "%.17e"],
               header=header + "\ncolumns: polarisation (0 x, 1 y, 2 z), step i, a_i (Ha), b_{i+1} (Ha)")
    np.savetxt(os.path.join(HERE, "c2_l23_norm2.txt"), np.array(norms), fmt=["%d", "%.17e"],
               header=header + "\ncolumns: polarisation, |psi0|^2")
    np.savetxt(os.path.join(HERE, "c2_l23_spectra.txt"), np.column_stack([cr.omega] + sig), fmt="%.17e",
               header=header + "\nno terminator, half width 0.5 eV\ncolumns: omega (Ha), sigma_x, sigma_y, sigma_z")
    print(f"done in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 300)
