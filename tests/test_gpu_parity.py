"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.

Tolerances (FP64 path): H*v to 1e-13 of max|y| (the two sides differ only in
summation order, ~1e-16 per operation over <= 1e4-term sums); Haydock
coefficients with re-orthogonalisation to 1e-10 of the spectral scale
S = max|a| + 2 max b; spectra to 1e-10 of max sigma.  FP32 path: spectrum L1
<= 1e-3 relative against the converged FP64 oracle spectrum."""
import sys

import numpy as np
import pytest

import synth
from oracle import bse as orc
from oracle import multiplet as omp

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _ob():
    import paper_1601_07728_amd as ob
    return ob


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _oracle_mats(cr, with_local=True):
    if cr.multiplet is None:
        return None, None
    return omp.core_matrix(cr.multiplet), (omp.local_matrix(cr.multiplet) if with_local else None)


def _to_dev(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


HV_CASES = {
    "c1": lambda: synth.config1(),
    "l_ragged": lambda: synth.small_l_edge(seed=3, nk=(2, 1, 2), nx=(4, 5, 3), n_bands=7),
    "l_tiles": lambda: synth.small_l_edge(seed=4, nk=(4, 2, 2), nx=(10, 9, 11), n_bands=37),
    "gamma": lambda: synth.small_l_edge(seed=5, nk=(1, 1, 1), nx=(12, 12, 12), n_bands=53),
    "k8_axis": lambda: synth.small_l_edge(seed=6, nk=(8, 1, 3), nx=(3, 4, 5), n_bands=19),
    "cube4": lambda: synth.small_l_edge(seed=8, nk=(4, 4, 4), nx=(5, 4, 3), n_bands=9),
    "cube8": lambda: synth.small_l_edge(seed=9, nk=(8, 8, 8), nx=(3, 2, 2), n_bands=5),
}


@pytest.mark.parametrize("case", list(HV_CASES))
@pytest.mark.parametrize("n_vec", [1, 3, 5])
def test_apply_fp64_matches_oracle(case, n_vec):
    ob = _ob()
    cr = HV_CASES[case]()
    _say(f"[apply fp64] case={case} n_vec={n_vec} nk={cr.nk} nx={cr.nx} nb={cr.n_bands}")
    h = ob.Bse.from_crystal(cr, precision="fp64", check_inputs=True)
    hc, kl = _oracle_mats(cr)
    x = synth.complex_gaussian(np.random.default_rng(100 + n_vec),
                               (n_vec, cr.n_k, cr.n_bands, cr.n_core))
    y = h.apply(_to_dev(x)).cpu().numpy()
    f = orc.dft_matrix(cr)
    ut = orc.folded_u(cr)
    w = orc.w_supercell(cr)
    for v in range(n_vec):
        ref = orc.apply_h(cr, x[v], hc, kl, ut=ut, w=w, f=f)
        assert _rel(y[v], ref) <= 1e-13, (case, v, _rel(y[v], ref))
    h.close()


# (n_core, n_vec): the projections take the exciton columns n_vec * n_core in passes of up to
# 24 (FP64: a single pass when there are at most 40) and split each pass into 16-wide matrix-core tiles plus, in FP64, a multiply-add tail of
# 1 or 2 columns.  Odd core counts reach the one-column tail.
COLUMN_SPLITS = [(1, 2), (1, 9), (3, 3), (1, 17), (3, 5), (1, 18), (3, 8), (1, 41),
                 # one wide FP64 pass of 25..40 columns: 3 tiles + tail 1..4, 4 tiles + tail 0..4, 5 tiles
                 (5, 5), (2, 13), (3, 9), (7, 4), (6, 5), (3, 11), (2, 17), (5, 7), (12, 3), (4, 10)]


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-13), ("fp32", 2e-5)])
@pytest.mark.parametrize("n_core,n_vec", COLUMN_SPLITS)
def test_apply_column_splits_match_oracle(n_core, n_vec, precision, tol):
    ob = _ob()
    cr = synth.make_crystal(f"split-c{n_core}", a=7.0, tau=(0.5, 1.0, 1.5), nk=(2, 1, 2),
                            nx=(7, 5, 6), n_bands=23, n_core=n_core, e_range_ev=25.0, eps=4.0,
                            seed=40 + n_core, psi0="none")
    _say(f"[apply column split] n_core={n_core} n_vec={n_vec} cols={n_core * n_vec} {precision}")
    h = ob.Bse.from_crystal(cr, precision=precision, check_inputs=True)
    x = synth.complex_gaussian(np.random.default_rng(500 + n_vec), (n_vec, cr.n_k, cr.n_bands, n_core))
    y = h.apply(_to_dev(x)).cpu().numpy()
    f, ut, w = orc.dft_matrix(cr), orc.folded_u(cr), orc.w_supercell(cr)
    for v in range(n_vec):
        ref = orc.apply_h(cr, x[v], ut=ut, w=w, f=f)
        assert _rel(y[v], ref) <= tol, (n_core, n_vec, precision, v, _rel(y[v], ref))
    h.close()


def _lattice_case(name):
    """Cells of other shapes, and a k grid offset by half a step (the oracle applies the
    offset in its phases and transform; the library needs no input for it, since the
    offset cancels in W0)."""
    skewed = np.array([[7.0, 0.0, 0.0], [2.1, 6.4, 0.0], [-1.3, 1.7, 6.9]])
    hexagonal = np.array([[6.0, 0.0, 0.0], [3.0, 3.0 * np.sqrt(3.0), 0.0], [0.0, 0.0, 7.5]])
    if name == "skewed":
        cr = synth.small_l_edge(seed=31, nk=(2, 2, 2), nx=(5, 4, 6), n_bands=13)
        cr.lattice = skewed
    elif name == "hexagonal":
        cr = synth.small_l_edge(seed=32, nk=(3, 3, 2), nx=(6, 6, 5), n_bands=11)
        cr.lattice = hexagonal
    elif name == "orthorhombic":
        cr = synth.small_l_edge(seed=33, nk=(2, 4, 1), nx=(5, 6, 7), n_bands=9)
        cr.lattice = np.diag([6.5, 7.2, 8.1])
    else:   # skewed cell, grid offset by half a step along b1 and b3
        cr = synth.small_l_edge(seed=34, nk=(2, 2, 2), nx=(4, 5, 4), n_bands=10)
        cr.lattice = skewed
        cr.kshift = (0.5, 0.0, 0.5)
    cr.tau = np.array([1.3, 2.2, 0.7])
    return cr


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-13), ("fp32", 2e-5)])
@pytest.mark.parametrize("case", ["skewed", "hexagonal", "orthorhombic", "skewed_offset_grid"])
def test_apply_lattices_match_oracle(case, precision, tol):
    ob = _ob()
    cr = _lattice_case(case)
    _say(f"[apply lattice] case={case} {precision} nk={cr.nk} nx={cr.nx} nb={cr.n_bands}")
    h = ob.Bse.from_crystal(cr, precision=precision, check_inputs=True)
    hc, kl = _oracle_mats(cr)
    x = synth.complex_gaussian(np.random.default_rng(91), (3, cr.n_k, cr.n_bands, cr.n_core))
    y = h.apply(_to_dev(x)).cpu().numpy()
    f, ut, w = orc.dft_matrix(cr), orc.folded_u(cr), orc.w_supercell(cr)
    for v in range(3):
        ref = orc.apply_h(cr, x[v], hc, kl, ut=ut, w=w, f=f)
        assert _rel(y[v], ref) <= tol, (case, precision, v, _rel(y[v], ref))
    h.close()


@pytest.mark.parametrize("case", ["skewed", "skewed_offset_grid"])
def test_apply_lattice_borrowed_fp64(case):
    """The same with u borrowed from the device (the transform applies the phase)."""
    ob = _ob()
    cr = _lattice_case(case)
    _say(f"[apply lattice borrowed] case={case}")
    h = ob.Bse.from_crystal(cr, precision="fp64", u=_to_dev(cr.u))
    hc, kl = _oracle_mats(cr)
    x = synth.complex_gaussian(np.random.default_rng(92), (2, cr.n_k, cr.n_bands, cr.n_core))
    y = h.apply(_to_dev(x)).cpu().numpy()
    for v in range(2):
        ref = orc.apply_h(cr, x[v], hc, kl)
        assert _rel(y[v], ref) <= 1e-13, (case, v, _rel(y[v], ref))
    h.close()


@pytest.mark.parametrize("case", ["c1", "l_tiles", "k8_axis", "cube4", "cube8"])
def test_apply_borrowed_fp64_matches_oracle(case):
    """A borrowed FP64 u is used as given, so the k-grid transform applies the Bloch phase
    itself (owned copies carry it): both routes against the oracle."""
    ob = _ob()
    cr = HV_CASES[case]()
    _say(f"[apply fp64 borrowed] case={case} nk={cr.nk} nx={cr.nx} nb={cr.n_bands}")
    u_dev = _to_dev(cr.u)
    h = ob.Bse.from_crystal(cr, precision="fp64", u=u_dev)
    hc, kl = _oracle_mats(cr)
    x = synth.complex_gaussian(np.random.default_rng(77), (3, cr.n_k, cr.n_bands, cr.n_core))
    y = h.apply(_to_dev(x)).cpu().numpy()
    f, ut, w = orc.dft_matrix(cr), orc.folded_u(cr), orc.w_supercell(cr)
    for v in range(3):
        ref = orc.apply_h(cr, x[v], hc, kl, ut=ut, w=w, f=f)
        assert _rel(y[v], ref) <= 1e-13, (case, v, _rel(y[v], ref))
    h.close()


def test_apply_w_scaled_exercises_w0():
    """W multiplied by 50 so the long-range term is O(1) of H: a sign or index
    error in W0 cannot hide below the diagonal."""
    ob = _ob()
    cr = synth.small_l_edge(seed=8, nk=(2, 2, 2), nx=(6, 6, 6), n_bands=11)
    cr.w_val = cr.w_val * 50.0
    _say("[apply w x50]")
    h = ob.Bse.from_crystal(cr, precision="fp64")
    hc, kl = _oracle_mats(cr)
    x = synth.complex_gaussian(np.random.default_rng(7), (cr.n_k, cr.n_bands, cr.n_core))
    y = h.apply(_to_dev(x)).cpu().numpy()
    ref = orc.apply_h(cr, x, hc, kl)
    w0 = orc.apply_w0(cr, x)
    assert np.abs(w0).max() > 0.3 * np.abs(ref).max()
    assert _rel(y, ref) <= 1e-13


@pytest.fixture(scope="module")
def c1_oracle():
    cr = synth.config1()
    psi0 = cr.psi0[0]
    a, b, n2, s, _ = orc.haydock(lambda v: orc.apply_h(cr, v), psi0, cr.n_steps, reorth=True)
    sig = orc.spectrum(a, b, n2, cr.omega, cr.gamma)
    ap, bp, _, _, basis = orc.haydock(lambda v: orc.apply_h(cr, v), psi0, cr.n_steps, reorth=False)
    vs = np.stack([q.ravel() for q in basis])
    ov = np.abs(vs.conj() @ vs.T - np.eye(len(vs)))
    loss = [ov[:i + 1, :i + 1].max() for i in range(len(vs))]
    return dict(cr=cr, a=a, b=b, n2=n2, sig=sig, ap=ap, bp=bp, loss=np.array(loss))


def test_haydock_reorth_c1_matches_oracle(c1_oracle):
    ob = _ob()
    o = c1_oracle
    cr = o["cr"]
    _say("[haydock c1 reorth]")
    h = ob.Bse.from_crystal(cr)
    a, b, n2, sd, rc = h.haydock(_to_dev(cr.psi0), cr.n_steps, reorth=True)
    S = np.abs(o["a"]).max() + 2 * o["b"].max()
    assert sd[0] == cr.n_steps and rc == 0
    assert abs(n2[0] - o["n2"]) <= 1e-13 * o["n2"]
    assert np.abs(a[0] - o["a"]).max() <= 1e-10 * S
    assert np.abs(b[0] - o["b"]).max() <= 1e-10 * S
    sig = ob.spectrum(a, b, n2, cr.omega, cr.gamma)[0]
    assert np.abs(sig - o["sig"]).max() <= 1e-10 * o["sig"].max()
    # bitwise reproducible run to run (fixed reduction order)
    a2, b2, _, _, _ = h.haydock(_to_dev(cr.psi0), cr.n_steps, reorth=True)
    assert np.array_equal(a, a2) and np.array_equal(b, b2)
    h.close()


def test_haydock_plain_c1_prefix(c1_oracle):
    """Without re-orthogonalisation, coefficients are compared while the oracle's
    Lanczos basis is still orthogonal to 1e-8."""
    ob = _ob()
    o = c1_oracle
    cr = o["cr"]
    h = ob.Bse.from_crystal(cr)
    a, b, n2, sd, rc = h.haydock(_to_dev(cr.psi0), cr.n_steps, reorth=False)
    S = np.abs(o["ap"]).max() + 2 * o["bp"].max()
    good = int(np.sum(o["loss"] < 1e-8)) - 1
    assert good >= 30
    assert np.abs(a[0, :good] - o["ap"][:good]).max() <= 1e-10 * S
    assert np.abs(b[0, :good] - o["bp"][:good]).max() <= 1e-10 * S
    h.close()


def test_haydock_l_edge_multi_vector_reorth():
    """L edge with spin-orbit and local term, three polarisation vectors at once."""
    ob = _ob()
    cr = synth.small_l_edge(seed=9, nk=(2, 2, 1), nx=(5, 6, 4), n_bands=9)
    hc, kl = _oracle_mats(cr)
    _say("[haydock L edge 3 vectors]")
    h = ob.Bse.from_crystal(cr)
    psi0 = h.dipole_psi0(np.eye(3))
    p0 = psi0.cpu().numpy()
    n_steps = 60
    a, b, n2, sd, rc = h.haydock(psi0, n_steps, reorth=True)
    for v in range(3):
        ref0 = omp.dipole_psi0(cr.local_proj, np.eye(3)[v])
        assert np.abs(p0[v] - ref0).max() <= 1e-14
        ra, rb, rn2, rs, _ = orc.haydock(lambda q: orc.apply_h(cr, q, hc, kl), ref0, n_steps, reorth=True)
        S = np.abs(ra).max() + 2 * rb.max()
        assert sd[v] == rs
        assert abs(n2[v] - rn2) <= 1e-13 * rn2
        assert np.abs(a[v, :rs] - ra).max() <= 1e-10 * S
        assert np.abs(b[v, :rs] - rb).max() <= 1e-10 * S
    h.close()


def test_breakdown_on_eigenvector():
    ob = _ob()
    cr = synth.config1()
    cr.w_val = cr.w_val * 0.0
    h = ob.Bse.from_crystal(cr)
    psi0 = np.zeros((1, cr.n_k, cr.n_bands, cr.n_core), dtype=np.complex128)
    psi0[0, 1, 3, 0] = 1.0
    a, b, n2, sd, rc = h.haydock(_to_dev(psi0), 10)
    assert rc == ob.INFO_INVARIANT_SUBSPACE and sd[0] == 1
    assert abs(a[0, 0] - cr.energies[1, 3]) <= 1e-15 and b[0, 0] == 0.0
    assert np.all(a[0, 1:] == 0)
    h.close()


def test_spectrum_kernel_matches_oracle():
    ob = _ob()
    rng = np.random.default_rng(12)
    a = rng.uniform(-0.5, 0.5, (3, 40))
    b = rng.uniform(0.05, 0.4, (3, 40))
    n2 = np.array([1.0, 2.5, 0.3])
    om = np.linspace(-1.5, 1.5, 777)
    gam = 0.02
    used = [40, 25, 17]
    for term in ("none", "sqrt"):
        sig = ob.spectrum(a, b, n2, om, gam, terminator=term, n_used=used)
        for s in range(3):
            ref = orc.spectrum(a[s, :used[s]], b[s, :used[s]], n2[s], om, gam, terminator=term)
            assert np.abs(sig[s] - ref).max() <= 1e-12 * np.abs(ref).max(), (term, s)


def test_fp32_spectrum_l1_within_1e_3():
    """Mixed precision (FP32 projections, FP64 recursion) against the FP64 oracle
    at a step count where the oracle spectrum is converged (full Krylov depth)."""
    ob = _ob()
    cr = synth.small_l_edge(seed=10, nk=(2, 2, 2), nx=(6, 6, 6), n_bands=10)
    hc, kl = _oracle_mats(cr)
    _say("[fp32 L1]")
    h = ob.Bse.from_crystal(cr, precision="fp32")
    psi0 = h.dipole_psi0([0, 0, 1])
    p0 = psi0.cpu().numpy()[0]
    hd = orc.h_dense(cr, hc, kl)
    ref = orc.spectrum_dense(hd, p0, cr.omega, cr.gamma)
    a, b, n2, sd, rc = h.haydock(psi0, cr.dim + 8, reorth=True)
    sig = ob.spectrum(a, b, n2, cr.omega, cr.gamma, n_used=sd)[0]
    l1 = orc.l1_relative(sig, ref)
    _say(f"fp32 L1 = {l1:.3e}")
    assert l1 <= 1e-3
    x = synth.complex_gaussian(np.random.default_rng(3), (cr.n_k, cr.n_bands, cr.n_core))
    y = h.apply(_to_dev(x)).cpu().numpy()
    yr = orc.apply_h(cr, x, hc, kl)
    assert _rel(y, yr) <= 1e-5
    h.close()


def test_long_range_term_does_not_mix_core_states():
    """Algorithm 1 treats each core index on its own (section 3.2.1): with no core matrix and no
    local term, H*v of a vector living on one core state stays on that state, and equals the
    same vector's H*v computed alone with one core state."""
    ob = _ob()
    cr = synth.make_crystal("nomix", a=6.8, tau=(0.3, 1.1, 2.0), nk=(2, 2, 2), nx=(6, 5, 6), n_bands=13,
                            n_core=6, e_range_ev=20.0, eps=4.0, seed=91, psi0="none")
    h = ob.Bse.from_crystal(cr, precision="fp64")
    rng = np.random.default_rng(92)
    x = np.zeros((1, cr.n_k, cr.n_bands, 6), dtype=np.complex128)
    x[0, :, :, 4] = synth.complex_gaussian(rng, (cr.n_k, cr.n_bands))
    y = h.apply(_to_dev(x)).cpu().numpy()[0]
    h.close()
    assert np.abs(y[:, :, [0, 1, 2, 3, 5]]).max() == 0.0
    c1 = synth.make_crystal("nomix1", a=6.8, tau=(0.3, 1.1, 2.0), nk=(2, 2, 2), nx=(6, 5, 6), n_bands=13,
                            n_core=1, e_range_ev=20.0, eps=4.0, seed=91, psi0="none")
    h1 = ob.Bse.from_crystal(c1, precision="fp64")
    y1 = h1.apply(_to_dev(np.ascontiguousarray(x[:, :, :, 4:5]))).cpu().numpy()[0]
    h1.close()
    assert np.abs(y[:, :, 4] - y1[:, :, 0]).max() <= 1e-14 * np.abs(y1).max()


def test_one_vector_stops_while_the_other_continues():
    """Two starting vectors in one recursion, one an eigenvector (it stops after one step) and
    one generic: the stopped vector reports 1 step and zeros after it, the generic one runs on
    with exactly the coefficients it has when run alone."""
    ob = _ob()
    cr = synth.config1()
    cr.w_val = cr.w_val * 0.0
    h = ob.Bse.from_crystal(cr)
    psi = np.zeros((2, cr.n_k, cr.n_bands, cr.n_core), dtype=np.complex128)
    psi[0, 1, 3, 0] = 1.0
    psi[1] = synth.complex_gaussian(np.random.default_rng(93), (cr.n_k, cr.n_bands, cr.n_core))
    a, b, n2, sd, rc = h.haydock(_to_dev(psi), 30)
    assert rc == ob.INFO_INVARIANT_SUBSPACE and sd[0] == 1 and sd[1] == 30
    assert np.all(a[0, 1:] == 0) and np.all(b[0] == 0)
    a1, b1, n21, sd1, _ = h.haydock(_to_dev(np.ascontiguousarray(psi[1:])), 30)
    assert np.array_equal(a[1], a1[0]) and np.array_equal(b[1], b1[0]) and n2[1] == n21[0]
    h.close()


RES_CASES = {
    "l_tiles": lambda: synth.small_l_edge(seed=4, nk=(4, 2, 2), nx=(10, 9, 11), n_bands=37),
    "l_odd_bands": lambda: synth.small_l_edge(seed=12, nk=(2, 2, 2), nx=(6, 7, 5), n_bands=13),
    "k_edge": lambda: synth.config1(),
    "l_c2_bands": lambda: synth.small_l_edge(seed=13, nk=(2, 2, 1), nx=(12, 11, 10), n_bands=96),
}


@pytest.mark.parametrize("case", list(RES_CASES))
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-13), ("fp32", 1e-5), ("split_bf16", 1e-4), ("bf16", 1e-2)])
def test_resident_operand_forward_matches_chunked_and_oracle(case, precision, tol, monkeypatch):
    """The forward projection with psi[k] (in the bf16 modes its staged B chunks) resident in
    LDS (OCEAN_FWD_TILES row tiles per block: one tile, several, and more than the x grid
    holds) gives the band-chunked kernel's H*v bit for bit (the same MFMA sequence per output
    element; FP32 with the 4x4x1 remainder tiles off on both sides, and again with them on), and
    the oracle's to the precision's tolerance with them on, for 1..5 vectors (6 to 30 columns: one to three column
    tiles, with and without the FP64 multiply-add tail or the FP32 4-column remainder, one or
    two passes)."""
    torch = _torch()
    ob = _ob()
    cr = RES_CASES[case]()
    hc, kl = _oracle_mats(cr)
    nvs = (1, 2, 3) if cr.n_core == 6 else (1, 3, 5)
    for nv in nvs:
        x = synth.complex_gaussian(np.random.default_rng(40 + nv), (nv, cr.n_k, cr.n_bands, cr.n_core))
        xd = _to_dev(x)
        refs = [orc.apply_h(cr, x[v], hc, kl) for v in range(nv)]
        monkeypatch.setenv("OCEAN_QUAD_TAIL", "0")
        monkeypatch.setenv("OCEAN_FWD_TILES", "0")
        h = ob.Bse.from_crystal(cr, precision=precision)
        y0 = h.apply(xd).cpu().numpy()
        h.close()
        for ft in ("1", "4", "64"):
            _say(f"resident forward: {case} {precision} n_vec {nv} tiles {ft}")
            monkeypatch.setenv("OCEAN_FWD_TILES", ft)
            h = ob.Bse.from_crystal(cr, precision=precision)
            y = h.apply(xd).cpu().numpy()
            h.close()
            torch.cuda.synchronize()
            assert np.array_equal(y, y0), (case, precision, nv, ft, float(np.abs(y - y0).max()))
        monkeypatch.setenv("OCEAN_QUAD_TAIL", "1")
        yq = {}
        for ft in ("0", "4"):
            monkeypatch.setenv("OCEAN_FWD_TILES", ft)
            h = ob.Bse.from_crystal(cr, precision=precision)
            y = h.apply(xd).cpu().numpy()
            h.close()
            yq[ft] = y
            for v in range(nv):
                assert _rel(y[v], refs[v]) <= tol, (case, precision, nv, ft, v)
        # with the FP32 4x4x1 remainder on, both forward forms run it in the same order
        assert np.array_equal(yq["0"], yq["4"]), (case, precision, nv, float(np.abs(yq["0"] - yq["4"]).max()))
        for v in range(nv):
            assert _rel(y0[v], refs[v]) <= tol, (case, precision, nv, v)


@pytest.mark.parametrize("precision,tol", [("fp32", 2e-5), ("split_bf16", 1e-4), ("bf16", 1e-2)])
@pytest.mark.parametrize("nx,n_core,n_vec,lines", [((3, 2, 2), 6, 3, "8"), ((5, 5, 3), 3, 1, "8"),
                                                    ((5, 5, 3), 3, 1, "16"), ((3, 3, 3), 6, 5, "16")])
def test_transform_line_pairs_match_single_lines(nx, n_core, n_vec, lines, precision, tol, monkeypatch):
    """The FP32-arithmetic cube transform with two lines per thread gives the one-line-per-
    thread kernel's H*v bit for bit, on an 8^3 k grid with an even and an odd number of lines
    (x points times columns: 12 x 18; 75 x 3, whose last block holds padding lines; 27 x 30)
    and 8 or 16 lines per block, and the oracle's to the precision's tolerance."""
    ob = _ob()
    local = n_core == 6
    cr = synth.make_crystal("pairs", a=6.5, tau=(0.7, 1.9, 3.1), nk=(8, 8, 8), nx=nx, n_bands=6, n_core=n_core,
                            e_range_ev=30.0, eps=5.0, seed=21, n_local=5 if local else 0,
                            multiplet_ev=dict(synth.L_EDGE_MULTIPLET_EV) if local else None, psi0="none")
    hc, kl = _oracle_mats(cr)
    x = synth.complex_gaussian(np.random.default_rng(5), (n_vec, cr.n_k, cr.n_bands, cr.n_core))
    xd = _to_dev(x)
    monkeypatch.setenv("OCEAN_FFT_LINES", lines)
    ys = []
    for pairs in ("0", "1"):
        monkeypatch.setenv("OCEAN_FFT_PAIRS", pairs)
        _say(f"[transform line pairs] nx={nx} n_core={n_core} n_vec={n_vec} lines={lines} {precision} pairs={pairs}")
        h = ob.Bse.from_crystal(cr, precision=precision)
        ys.append(h.apply(xd).cpu().numpy())
        h.close()
    assert np.array_equal(ys[0], ys[1])
    for v in range(n_vec):
        ref = orc.apply_h(cr, x[v], hc, kl)
        assert _rel(ys[1][v], ref) <= tol, (v, _rel(ys[1][v], ref))
