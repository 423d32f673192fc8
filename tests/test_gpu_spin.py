"""GPU parity on the full electron x hole spin space (12 core states), through the C ABI,
against the oracle.  Tolerances as for the restricted space: H*v 1e-13 of max|y| in FP64,
2e-5 in FP32, 1e-4 in split-BF16; recursion coefficients 1e-10 of max|a| + 2 max b."""
import sys

import numpy as np
import pytest

import synth
from oracle import bse as orc
from oracle import multiplet as omp

pytestmark = pytest.mark.gpu
HA = synth.HARTREE_EV


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _crystal(seed=41, zeta_ev=None):
    cr = synth.small_l_edge(seed=seed, nk=(2, 2, 1), nx=(5, 4, 6), n_bands=14)
    if zeta_ev is not None:
        cr.multiplet = dict(cr.multiplet, zeta=zeta_ev / HA)
    return cr


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-13), ("fp32", 2e-5), ("split_bf16", 1e-4)])
@pytest.mark.parametrize("n_vec", [1, 3])
def test_full_spin_apply_matches_oracle(precision, tol, n_vec):
    import paper_1601_07728_amd as ob
    cr = synth.full_spin(_crystal())
    _say(f"[spin apply] {precision} n_vec={n_vec} cols={12 * n_vec}")
    h = ob.Bse.from_crystal(cr, precision=precision, check_inputs=True)
    m = cr.multiplet
    hc, kl = omp.core_matrix_spin(m), omp.local_matrix_spin(m)
    x = synth.complex_gaussian(np.random.default_rng(300 + n_vec), (n_vec, cr.n_k, cr.n_bands, 12))
    y = h.apply(_dev(x)).cpu().numpy()
    for v in range(n_vec):
        ref = orc.apply_h(cr, x[v], hc, kl)
        err = float(np.abs(y[v] - ref).max() / np.abs(ref).max())
        assert err <= tol, (precision, v, err)
    h.close()


def test_full_spin_dipole_and_recursion_match_oracle():
    import paper_1601_07728_amd as ob
    cr = synth.full_spin(_crystal(seed=42))
    _say("[spin dipole + haydock]")
    h = ob.Bse.from_crystal(cr, precision="fp64")
    pol = np.array([[0.3, -0.5, 0.8]])
    p0 = h.dipole_psi0(pol)
    ref0 = omp.dipole_psi0_spin(cr.local_proj, pol[0])
    assert np.abs(p0[0].cpu().numpy() - ref0).max() <= 1e-14 * np.abs(ref0).max()
    m = cr.multiplet
    hc, kl = omp.core_matrix_spin(m), omp.local_matrix_spin(m)
    n = 60
    a, b, n2, steps, rc = h.haydock(p0, n, reorth=True)
    ar, br, n2r, _, _ = orc.haydock(lambda v: orc.apply_h(cr, v, hc, kl), ref0, n, reorth=True)
    scale = np.abs(ar).max() + 2 * np.abs(br).max()
    assert np.abs(a[0, :n] - ar).max() <= 1e-10 * scale
    assert np.abs(b[0, :n] - br).max() <= 1e-10 * scale
    assert abs(n2[0] - n2r) <= 1e-12 * n2r
    h.close()


def test_zero_spin_orbit_full_space_recursion_is_the_restricted_one_on_device():
    import paper_1601_07728_amd as ob
    cr = _crystal(seed=43, zeta_ev=0.0)
    _say("[spin zeta=0 vs restricted]")
    hr = ob.Bse.from_crystal(cr, precision="fp64")
    hf = ob.Bse.from_crystal(synth.full_spin(cr), precision="fp64")
    pol = np.eye(3)
    ar, br, n2r, _, _ = hr.haydock(hr.dipole_psi0(pol), 50, reorth=True)
    af, bf, n2f, _, _ = hf.haydock(hf.dipole_psi0(pol), 50, reorth=True)
    scale = np.abs(ar).max() + 2 * np.abs(br).max()
    assert np.abs(af - ar).max() <= 1e-11 * scale
    assert np.abs(bf - br).max() <= 1e-11 * scale
    assert np.abs(n2f - n2r).max() <= 1e-13 * np.abs(n2r).max()
    hr.close()
    hf.close()
