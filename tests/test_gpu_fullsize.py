"""Parity at the full benchmark size (SrTiO3-shaped L2,3 edge: 8^3 k, 96 bands, 20^3 x,
6 core states, H dimension 294912), in the launch configuration bench.py times (three
polarisation vectors per call, default tiles).  The oracle computes one complete H*v of
the first vector (every output element) and the first Haydock coefficients."""
import sys

import numpy as np
import pytest

import synth
from oracle import bse as orc
from oracle import multiplet as omp

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def full():
    import torch

    import paper_1601_07728_amd as ob
    cr = synth.config2_shape(seed=0, u_override="skip", psi0="none")
    u = synth.gpu_orthonormal_u(cr.n_k, cr.n_x, cr.n_bands, seed=1000)
    torch.cuda.synchronize()
    h64 = ob.Bse.from_crystal(cr, precision="fp64", u=u)
    _say(f"[fullsize] fp64 tuned {h64.autotune(n_vec=3)}")   # the tiles the benchmark times
    psi0 = h64.dipole_psi0(np.eye(3))
    y64 = h64.apply(psi0).cpu().numpy()
    a, b, n2, sd, _ = h64.haydock(psi0, 2)
    h32 = ob.Bse.from_crystal(cr, precision="fp32", u=u)
    _say(f"[fullsize] fp32 tuned {h32.autotune(n_vec=3)}")
    y32 = h32.apply(psi0).cpu().numpy()
    h32.close()
    h64.close()
    _say("[fullsize] GPU done; oracle H*v of vector 0")
    cr.u = u.cpu().numpy()
    del u
    hc, kl = omp.core_matrix(cr.multiplet), omp.local_matrix(cr.multiplet)
    ut, w, f = orc.folded_u(cr), orc.w_supercell(cr), orc.dft_matrix(cr)
    p0 = psi0.cpu().numpy()
    apply = lambda v: orc.apply_h(cr, v, hc, kl, ut=ut, w=w, f=f)  # noqa: E731
    ref = apply(p0[0])
    return dict(cr=cr, p0=p0, y64=y64, y32=y32, ref=ref, a=a, b=b, n2=n2, apply=apply)


def test_fullsize_apply_fp64(full):
    err = np.abs(full["y64"][0] - full["ref"]).max() / np.abs(full["ref"]).max()
    _say(f"[fullsize] fp64 H*v rel err {err:.2e}")
    assert err <= 1e-13


def test_fullsize_apply_fp32_projections(full):
    err = np.abs(full["y32"][0] - full["ref"]).max() / np.abs(full["ref"]).max()
    _say(f"[fullsize] fp32-projection H*v rel err {err:.2e}")
    assert err <= 1e-5


def test_fullsize_first_haydock_steps(full):
    """a_0 = <v0|H v0>, b_1 = |H v0 - a_0 v0|, a_1 from the oracle's second H*v."""
    p0 = full["p0"][0]
    n2 = float(np.vdot(p0, p0).real)
    v0 = p0 / np.sqrt(n2)
    w = full["ref"] / np.sqrt(n2)
    a0 = float(np.vdot(v0, w).real)
    r = w - a0 * v0
    b1 = float(np.linalg.norm(r))
    v1 = r / b1
    a1 = float(np.vdot(v1, full["apply"](v1)).real)
    scale = abs(a0) + 2 * b1
    assert abs(full["n2"][0] - n2) <= 1e-13 * n2
    assert abs(full["a"][0, 0] - a0) <= 1e-12 * scale
    assert abs(full["b"][0, 0] - b1) <= 1e-12 * scale
    assert abs(full["a"][0, 1] - a1) <= 1e-12 * scale
