"""Boundary tests that need no GPU: the library loads, exports every symbol the
header declares, its host helpers agree with the oracle, and argument
validation rejects bad input before any device work."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import paper_1601_07728_amd as ob
from oracle import multiplet as mp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "ocean_bse.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ocean_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(ob.LIB_PATH):
        pytest.fail("libocean_bse.so is not built (run __graft_entry__.build())")
    return ob.lib()


def test_exports_every_declared_symbol(lib):
    syms = _declared_symbols()
    assert len(syms) >= 13
    for s in syms:
        assert hasattr(lib, s), s
    assert sorted(ob.EXPORTED) == syms


def test_multiplet_matrices_match_oracle_quadrature(lib):
    """Closed-form (Racah 3j) helper vs the oracle's sphere quadrature."""
    zeta, f2, g1, g3 = 0.14, 0.29, 0.22, 0.13
    core, loc = ob.multiplet_matrices(zeta, f2, g1, g3)
    mult = {"zeta": zeta, "F2": f2, "G1": g1, "G3": g3}
    assert np.abs(core - mp.core_matrix(mult)).max() <= 1e-15
    assert np.abs(loc - mp.local_matrix(mult)).max() <= 1e-14


def test_full_spin_multiplet_matrices_match_oracle(lib):
    """The same on the full electron x hole spin space (12 core states)."""
    zeta, f2, g1, g3 = 0.14, 0.29, 0.22, 0.13
    core, loc = ob.multiplet_matrices(zeta, f2, g1, g3, full_spin=True)
    mult = {"zeta": zeta, "F2": f2, "G1": g1, "G3": g3}
    assert np.abs(core - mp.core_matrix_spin(mult)).max() <= 1e-15
    assert np.abs(loc - mp.local_matrix_spin(mult)).max() <= 1e-14


def test_dipole_amplitudes_match_oracle(lib):
    for pol in [(1, 0, 0), (0, 1, 0), (0, 0, 1), (0.3, -0.5, 0.81)]:
        d = ob.dipole_amplitudes(pol)
        assert np.abs(d - mp.dipole_amplitudes(pol)).max() <= 1e-14


def test_spectrum_rejects_bad_arguments(lib):
    a = np.zeros((1, 4))
    om = np.linspace(0, 1, 5)
    with pytest.raises(ob.OceanError) as e:
        ob.spectrum(a, a, [1.0], om, gamma=0.0)
    assert e.value.code == ob.ERR_INVALID_ARG
    with pytest.raises(ob.OceanError):
        ob.spectrum(a, a, [1.0], om, gamma=0.1, n_used=[9])
    # the constant chain's coefficients: both or neither, finite, b_inf > 0
    for ai, bi in ((np.zeros(1), None), (None, np.ones(1)), (np.zeros(1), np.zeros(1)),
                   (np.array([np.nan]), np.ones(1)), (np.zeros(1), np.array([np.inf]))):
        p = ob._ptr
        aa, bb = (None if ai is None else np.ascontiguousarray(ai)), (None if bi is None else np.ascontiguousarray(bi))
        n2 = np.ones(1)
        sig = np.zeros(5)
        rc = lib.ocean_spectrum(p(a), p(a), None, p(n2), 1, 4, ob.TERM_SQRT, p(aa), p(bb), p(om), 5, 0.1, p(sig))
        assert rc == ob.ERR_INVALID_ARG and len(lib.ocean_last_error()) > 0


def _set_cell(d, rows):
    for a in range(3):
        d.cell[a][:] = [float(x) for x in np.asarray(rows, dtype=float)[a]]


def _desc(**over):
    d = ob.Desc()
    d.nk[:] = (2, 2, 2)
    d.nx[:] = (4, 4, 4)
    d.n_bands, d.n_core, d.n_local = 4, 2, 0
    _set_cell(d, 7.0 * np.eye(3))
    keep = []
    e = np.zeros((8, 4))
    u = np.zeros((8, 64, 4), dtype=np.complex128)
    wr = np.linspace(0, 6, 64)
    wv = np.ones(64)
    keep += [e, u, wr, wv]
    d.energies, d.u = ob._ptr(e), ob._ptr(u)
    d.n_wr, d.w_r, d.w_val = 64, ob._ptr(wr), ob._ptr(wv)
    d.precision = ob.PREC_FP64
    for k, v in over.items():
        if k == "w_r":
            keep.append(v)
            d.w_r = ob._ptr(v)
        elif k == "energies":
            keep.append(v)
            d.energies = ob._ptr(v)
        elif k == "cell":
            _set_cell(d, v)
        elif k in ("nk", "nx"):
            getattr(d, k)[:] = v
        else:
            setattr(d, k, v)
    return d, keep


@pytest.mark.parametrize("over,code", [
    (dict(n_bands=0), ob.ERR_INVALID_ARG),
    (dict(nk=(0, 2, 2)), ob.ERR_INVALID_ARG),
    (dict(nk=(17, 1, 1)), ob.ERR_UNSUPPORTED),
    (dict(cell=[[7.0, 0.0, 0.0], [7.0, 0.0, 0.0], [0.0, 0.0, 7.0]]), ob.ERR_INVALID_ARG),   # no volume
    (dict(cell=[[7.0, 0.0, 0.0], [0.0, np.nan, 0.0], [0.0, 0.0, 7.0]]), ob.ERR_INVALID_ARG),
    (dict(n_core=13), ob.ERR_UNSUPPORTED),
    (dict(n_local=5), ob.ERR_INVALID_ARG),          # no projectors given
    (dict(precision=7), ob.ERR_UNSUPPORTED),
    (dict(w_r=np.linspace(1, 6, 64)), ob.ERR_INVALID_ARG),
    (dict(w_r=np.linspace(0, 6, 64) ** 1.5), ob.ERR_INVALID_ARG),
    (dict(energies=np.full((8, 4), np.nan), flags=ob.FLAG_CHECK_INPUTS), ob.ERR_INVALID_ARG),
])
def test_create_validates_before_device_work(lib, over, code):
    d, keep = _desc(**over)
    h = ctypes.c_void_p()
    rc = lib.ocean_bse_create(ctypes.byref(d), None, ctypes.byref(h))
    assert rc == code, lib.ocean_last_error()
    assert not h.value
    assert len(lib.ocean_last_error()) > 0


def test_null_handle_calls(lib):
    assert lib.ocean_bse_dim(None) == ob.ERR_INVALID_ARG
    assert lib.ocean_bse_apply(None, None, None, 1) == ob.ERR_INVALID_ARG
    assert lib.ocean_haydock(None, None, 1, 1, 0, None, None, None, None) == ob.ERR_INVALID_ARG
    assert lib.ocean_haydock_export(None, 1, None, None, None) == ob.ERR_INVALID_ARG
    assert lib.ocean_haydock_continue(None, None, None, None, 1, 1, 0, None, None, None) == ob.ERR_INVALID_ARG
    lib.ocean_bse_destroy(None)


def test_binding_has_no_fallback(monkeypatch, tmp_path):
    """With the library missing, the binding raises instead of computing anything."""
    monkeypatch.setattr(ob, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(ob, "_lib", None)
    with pytest.raises(RuntimeError):
        ob.lib()


def test_screening_validates_before_device_work(lib):
    """Invalid arguments are rejected before any device pointer is touched."""
    eps = np.array([0.0, 1.0])
    tn = np.array([0.5])
    wn = np.array([1.0])
    fake = ctypes.c_void_p(8)
    bad = [(None, eps, 1, 2, 0.1, tn, wn, 1),
           (fake, eps, 0, 2, 0.1, tn, wn, 1),
           (fake, np.array([0.0, np.nan]), 1, 2, 0.1, tn, wn, 1),
           (fake, eps, 1, 2, 0.1, np.array([-0.5]), wn, 1),
           (fake, eps, 1, 2, float("inf"), tn, wn, 1)]
    for psi, e, npt, ns, mu, t, w, nt in bad:
        rc = lib.ocean_screening_chi0(psi, ob._ptr(e), npt, ns, mu, ob._ptr(t), ob._ptr(w), nt, fake, None)
        assert rc == ob.ERR_INVALID_ARG
        assert len(lib.ocean_last_error()) > 0


def test_local_matrix_channels_match_oracle(lib):
    """General local basis: closed-form (Racah 3j) helper vs the oracle's quadrature, both spin
    models, and the dipole amplitudes of the channels."""
    rng = np.random.default_rng(3)
    ls = [0, 1, 2, 3, 2, 1]
    n = len(ls)
    f2 = rng.normal(size=(n, n))
    f2 = f2 @ f2.T / n
    gk = rng.normal(size=(5, n, n))
    gk = np.einsum("kij,klj->kil", gk, gk) / n
    for full in (False, True):
        got = ob.local_matrix_channels(ls, f2, gk, full_spin=full)
        ref = mp.local_matrix_channels(ls, f2, {k: gk[k] for k in range(5)}, full_spin=full)
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    radial = rng.normal(size=n)
    for pol in [(0, 0, 1), (0.3, -0.5, 0.81)]:
        d = ob.dipole_amplitudes_channels(ls, radial, pol)
        one = np.eye(d.shape[0])[None]      # A = identity: psi0 rows are the amplitudes d
        ref = mp.dipole_psi0_channels(one, ls, radial, pol)[0, :, ::2]
        assert np.abs(d - ref).max() <= 1e-14


def test_transition_amplitudes_match_oracle(lib):
    """e^{iq.r} (addition theorem with closed-form Y_LM and Gaunt factors) and the quadrupole
    term (products through the l = 0, 2 shells) against the oracle's sphere quadrature."""
    rng = np.random.default_rng(8)
    ls = [0, 1, 2, 3, 2, 1]
    n = len(ls)
    rad = rng.normal(size=(n, 6))
    for q in ([0.3, -0.5, 0.8], [0, 0, 1.0], [0, 0, -2.0], [1.0, 0, 0], [0, -1e-3, 0]):
        q = np.asarray(q)
        got = ob.nrixs_amplitudes_channels(ls, rad, q)
        ref = mp.nrixs_amplitudes_channels(ls, rad, q)
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    r1, r2 = rng.normal(size=n), rng.normal(size=n)
    for e, q in (([0.6, 0, 0.8], [0.7, -1.1, 0.4]), ([0, 0, 1.0], [1.0, 0, 0]), ([0.3, -0.5, 0.81], [0, 0, 0])):
        got = ob.quadrupole_amplitudes_channels(ls, r1, r2, e, q)
        ref = mp.quadrupole_amplitudes_channels(ls, r1, r2, e, q)
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    la = np.array(ls, dtype=np.int32)
    d = np.zeros((sum(2 * l + 1 for l in ls), 3), dtype=np.complex128)
    p = lambda a: np.ascontiguousarray(a).ctypes.data_as(ctypes.c_void_p)
    r = np.ascontiguousarray(rad)
    assert lib.ocean_nrixs_amplitudes_channels(n, p(la), 6, p(r), p(np.zeros(3)), p(d)) == ob.ERR_INVALID_ARG
    assert lib.ocean_nrixs_amplitudes_channels(n, p(la), 0, p(r), p(np.ones(3)), p(d)) == ob.ERR_INVALID_ARG
    assert lib.ocean_nrixs_amplitudes_channels(n, p(np.array([4] * n, dtype=np.int32)), 6, p(r), p(np.ones(3)),
                                               p(d)) == ob.ERR_INVALID_ARG
    assert lib.ocean_quadrupole_amplitudes_channels(n, p(la), p(r1), p(r2), p(np.array([np.nan, 0, 1.0])),
                                                    p(np.ones(3)), p(d)) == ob.ERR_INVALID_ARG
    assert lib.ocean_psi0_amplitudes(None, p(d), 1, None) == ob.ERR_INVALID_ARG
    assert len(lib.ocean_last_error()) > 0
