"""Checkpoint and resume of the Haydock recursion (ocean_haydock_export / _continue): a run
split into two calls, with the state moved to another handle of the same system in between,
gives the coefficients of the uninterrupted run bit for bit; a stopped vector stays stopped;
re-orthogonalisation is refused."""
import ctypes
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("precision", ["fp64", "bf16"])
def test_split_run_equals_uninterrupted_run(precision):
    import paper_1601_07728_amd as ob
    cr = synth.small_l_edge(seed=71, nk=(2, 2, 2), nx=(6, 5, 4), n_bands=17)
    _say(f"[resume] {precision}")
    h = ob.Bse.from_crystal(cr, precision=precision)
    p0 = h.dipole_psi0(np.eye(3))
    a, b, n2, sd, rc = h.haydock(p0, 60)
    assert rc == ob.OK and np.all(sd == 60)
    a1, b1, n21, _, _ = h.haydock(p0, 25)
    v, vp, st = h.haydock_export(3)
    assert np.array_equal(st[:, 2], n2) and np.all(st[:, 4] == 0) and np.all(st[:, 5] == 25)
    assert np.array_equal(st[:, 0], b1[:, 24])
    h.close()
    h2 = ob.Bse.from_crystal(cr, precision=precision)
    a2, b2, sd2, rc2 = h2.haydock_continue(v, vp, st, 35)
    assert rc2 == ob.OK and np.all(sd2 == 35)
    assert np.array_equal(np.concatenate([a1, a2], axis=1), a)
    assert np.array_equal(np.concatenate([b1, b2], axis=1), b)
    # the state after the continuation continues again, on the same handle
    v3, vp3, st3 = h2.haydock_export(3)
    a3, b3, _, _ = h2.haydock_continue(v3, vp3, st3, 5)
    a4, b4, _, _, _ = h2.haydock(p0, 65)
    assert np.array_equal(a3, a4[:, 60:]) and np.array_equal(b3, b4[:, 60:])
    h2.close()


def test_stopped_vector_stays_stopped_and_reorth_is_refused():
    import paper_1601_07728_amd as ob
    cr = synth.config1()
    cr.w_val = cr.w_val * 0.0
    h = ob.Bse.from_crystal(cr)
    psi0 = np.zeros((1, cr.n_k, cr.n_bands, cr.n_core), dtype=np.complex128)
    psi0[0, 1, 3, 0] = 1.0
    import torch
    a, b, n2, sd, rc = h.haydock(torch.from_numpy(psi0).to("cuda"), 10)
    assert rc == ob.INFO_INVARIANT_SUBSPACE and sd[0] == 1
    v, vp, st = h.haydock_export(1)
    assert st[0, 4] == 1.0
    a2, b2, sd2, rc2 = h.haydock_continue(v, vp, st, 4)
    assert rc2 == ob.INFO_INVARIANT_SUBSPACE and sd2[0] == 0 and np.all(a2 == 0) and np.all(b2 == 0)
    lib = ob.lib()
    aa, bb, ss = np.zeros(4), np.zeros(4), np.zeros(1, dtype=np.int32)
    p = lambda x: x.ctypes.data_as(ctypes.c_void_p)
    rc3 = lib.ocean_haydock_continue(h._h, v.data_ptr(), vp.data_ptr(), p(st), 1, 4, ob.HAYDOCK_REORTH,
                                     p(aa), p(bb), p(ss))
    assert rc3 == ob.ERR_UNSUPPORTED
    bad = st.copy()
    bad[0, 2] = -1.0
    rc4 = lib.ocean_haydock_continue(h._h, v.data_ptr(), vp.data_ptr(), p(bad), 1, 4, 0, p(aa), p(bb), p(ss))
    assert rc4 == ob.ERR_INVALID_ARG
    with pytest.raises(Exception):
        h.haydock_export(2)        # the last run had one vector
    h.close()
