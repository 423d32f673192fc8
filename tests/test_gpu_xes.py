"""GPU parity of the emission (XES) path: the same H*v, recursion and spectrum kernels over
the occupied band window (the reading in oracle/xes.py), through the C ABI, against the
oracle.

* A small window (Gamma point, 10^3 box grid, 20 occupied bands, K edge, three amplitude
  vectors): FP64 H*v to 1e-13 of max|y|; the re-orthogonalised recursion at full depth
  (dim = 40 steps) to 1e-10 of S = max|a| + 2 max b; spectra to 1e-10 of max sigma.
* The same window without the core-hole interaction (W = 0): the GPU spectrum at full depth
  against the closed-form amplitude-weighted occupied density of states, 1e-9 of max sigma.
* The Alq3-sized site (30 bohr box, 48^3 grid, 81 occupied bands): FP64 coefficients of the
  first 40 re-orthogonalised steps against the oracle (1e-10 of S), and the BF16 path's
  200-step spectrum within L1 1e-3 of the FP64 one."""
import sys

import numpy as np
import pytest

import synth
from oracle import bse as orc
from oracle import xes

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _small(w_off=False):
    cr = synth.xes_site(seed=11, n_occ=20, grid=10, box=14.0)
    if w_off:
        cr.w_val = np.zeros_like(cr.w_val)
    return cr


def test_xes_hv_and_recursion_match_the_oracle():
    import paper_1601_07728_amd as ob
    cr = _small()
    assert xes.is_occupied_window(cr.energies)
    _say(f"[xes small] dim {cr.dim}")
    h = ob.Bse.from_crystal(cr, precision="fp64")
    y = h.apply(_dev(cr.psi0)).cpu().numpy()
    for v in range(3):
        ref = orc.apply_h(cr, cr.psi0[v])
        assert np.abs(y[v] - ref).max() <= 1e-13 * np.abs(ref).max()
    n = cr.dim
    a, b, n2, sd, rc = h.haydock(_dev(cr.psi0), n, reorth=True)
    sig = ob.spectrum(a, b, n2, cr.omega, cr.gamma, n_used=sd)
    h.close()
    for v in range(3):
        ra, rb, rn2, rs, _ = orc.haydock(lambda x: orc.apply_h(cr, x), cr.psi0[v], n, reorth=True)
        S = np.abs(ra).max() + 2 * rb.max()
        m = min(rs, int(sd[v]))
        assert np.abs(a[v, :m] - ra[:m]).max() <= 1e-10 * S
        assert np.abs(b[v, :m - 1] - rb[:m - 1]).max() <= 1e-10 * S
        assert abs(n2[v] - rn2) <= 1e-13 * rn2
        ref = orc.spectrum(ra, rb, rn2, cr.omega, cr.gamma)
        assert np.abs(sig[v] - ref).max() <= 1e-10 * ref.max()


def test_xes_without_core_hole_is_the_occupied_dos():
    import paper_1601_07728_amd as ob
    cr = _small(w_off=True)
    h = ob.Bse.from_crystal(cr, precision="fp64")
    a, b, n2, sd, rc = h.haydock(_dev(cr.psi0), cr.dim, reorth=True)
    sig = ob.spectrum(a, b, n2, cr.omega, cr.gamma, n_used=sd)
    h.close()
    for v in range(3):
        ref = xes.occupied_dos_spectrum(cr.energies, cr.psi0[v], cr.omega, cr.gamma)
        err = np.abs(sig[v] - ref).max() / ref.max()
        _say(f"[xes W = 0] vector {v}: steps {sd[v]}, max deviation {err:.2e} of max sigma")
        assert err <= 1e-9


def test_xes_alq3_sized_site():
    import paper_1601_07728_amd as ob
    cr = synth.xes_site(seed=2)
    _say(f"[xes site] {cr.n_x} points, {cr.n_bands} occupied bands, dim {cr.dim}")
    n = 40
    h = ob.Bse.from_crystal(cr, precision="fp64")
    a, b, n2, sd, rc = h.haydock(_dev(cr.psi0), n, reorth=True)
    ra, rb, rn2, rs, _ = orc.haydock(lambda x: orc.apply_h(cr, x), cr.psi0[0], n, reorth=True)
    S = np.abs(ra).max() + 2 * rb.max()
    dev = max(np.abs(a[0] - ra).max(), np.abs(b[0] - rb).max()) / S
    _say(f"[xes site] FP64 vs oracle over {n} steps: {dev:.2e} of S")
    assert rs == n and sd[0] == n and dev <= 1e-10
    steps = 200
    a64, b64, n64, s64, _ = h.haydock(_dev(cr.psi0), steps)
    h.close()
    ref = ob.spectrum(a64, b64, n64, cr.omega, cr.gamma, n_used=s64)
    hb = ob.Bse.from_crystal(cr, precision="bf16")
    ab, bb, nb, sb, _ = hb.haydock(_dev(cr.psi0), steps)
    hb.close()
    sig = ob.spectrum(ab, bb, nb, cr.omega, cr.gamma, n_used=sb)
    l1 = [float(np.sum(np.abs(sig[v] - ref[v])) / np.sum(np.abs(ref[v]))) for v in range(3)]
    _say(f"[xes site] BF16 200-step spectra vs FP64: L1 {', '.join(f'{x:.2e}' for x in l1)}")
    assert max(l1) <= 1e-3
