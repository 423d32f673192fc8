"""Parity at the size of the paper's timed supercell calculation: one Ti L2,3 site of the
4x4x4 SrTiO3-shaped supercell with 3072 bands, 2^3 k and 32^3 x (u 12.9 GB in FP64, drawn on
the device).  The oracle computes the complete H*v of the z-polarised dipole vector (every
output element) from a host copy of the same u."""
import sys
import time

import numpy as np
import pytest

import synth
from oracle import bse as orc
from oracle import multiplet as omp

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_paper_shape_fullsize_apply_fp64():
    import torch

    import paper_1601_07728_amd as ob
    t0 = time.time()
    cr = synth.config3_shape(seed=0, nx=(32, 32, 32), n_bands=3072)
    u = synth.gpu_orthonormal_u(cr.n_k, cr.n_x, cr.n_bands, seed=4000)
    torch.cuda.synchronize()
    _say(f"[paper shape] u on the device ({u.numel() * 16 / 1e9:.1f} GB) in {time.time() - t0:.1f} s")
    h = ob.Bse.from_crystal(cr, precision="fp64", u=u)
    psi0 = h.dipole_psi0(np.eye(3))
    y = h.apply(psi0)[2].cpu().numpy()
    p0 = psi0[2].cpu().numpy()
    h.close()
    cr.u = u.cpu().numpy()
    del u, psi0
    torch.cuda.empty_cache()
    _say(f"[paper shape] oracle H*v from {time.time() - t0:.1f} s")
    ref = orc.apply_h(cr, p0, omp.core_matrix(cr.multiplet), omp.local_matrix(cr.multiplet))
    cr.u = None
    err = float(np.abs(y - ref).max() / np.abs(ref).max())
    _say(f"[paper shape] fp64 H*v rel err {err:.2e} at {time.time() - t0:.1f} s")
    assert err <= 1e-13
