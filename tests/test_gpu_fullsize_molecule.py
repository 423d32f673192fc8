"""Parity at the full size of the batched molecule-in-box workload: 40 sites of a 52-atom
layout in a 30 bohr box (Gamma point, 48^3 grid, 200..800 bands per site, K and L2,3
edges, 3 polarisations each), as bench.py runs it.  Every site's H*v of its three
vectors is checked against the oracle element by element for the smallest and the
largest site; the batched recursion of all 120 solves equals the stand-alone recursion
of every site bit for bit over the first steps."""
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


@pytest.fixture(scope="module")
def molecule():
    import torch

    import paper_1601_07728_amd as ob
    t0 = time.time()
    sites = synth.molecule_sites(seed=0)
    torch.cuda.synchronize()
    _say(f"[molecule] {len(sites)} sites on the device in {time.time() - t0:.1f} s")
    hs = [ob.Bse.from_crystal(cr, precision="fp64", u=u) for cr, u in sites]
    p0 = [torch.from_numpy(cr.psi0).to("cuda") if cr.psi0 is not None else h.dipole_psi0(np.eye(3))
          for h, (cr, _) in zip(hs, sites)]
    yield sites, hs, p0
    for h in hs:
        h.close()


def test_molecule_sites_apply_matches_oracle(molecule):
    sites, hs, p0 = molecule
    nbs = [cr.n_bands for cr, _ in sites]
    for s in (int(np.argmin(nbs)), int(np.argmax(nbs))):
        cr, u = sites[s]
        y = hs[s].apply(p0[s]).cpu().numpy()
        cr.u = u.cpu().numpy()
        hc = omp.core_matrix(cr.multiplet) if cr.multiplet else None
        kl = omp.local_matrix(cr.multiplet) if cr.multiplet else None
        ut, w, f = orc.folded_u(cr), orc.w_supercell(cr), orc.dft_matrix(cr)
        x = p0[s].cpu().numpy()
        for v in range(x.shape[0]):
            ref = orc.apply_h(cr, x[v], hc, kl, ut=ut, w=w, f=f)
            err = float(np.abs(y[v] - ref).max() / np.abs(ref).max())
            _say(f"[molecule] site {s} ({cr.name}, {cr.n_bands} bands) vector {v}: rel err {err:.2e}")
            assert err <= 1e-13
        cr.u = None


def test_molecule_batch_equals_standalone(molecule):
    import paper_1601_07728_amd as ob
    sites, hs, p0 = molecule
    n_steps = 12
    out, _ = ob.haydock_batch(hs, p0, n_steps)
    for s, h in enumerate(hs):
        a1, b1, n21, sd1, _ = h.haydock(p0[s], n_steps)
        a, b, n2, sd = out[s]
        assert np.array_equal(a, a1) and np.array_equal(b, b1) and np.array_equal(n2, n21), s
        assert np.array_equal(sd, sd1), s
