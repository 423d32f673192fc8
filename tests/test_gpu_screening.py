"""GPU parity of the screening response (ocean_screening_chi0) against the oracle, through the
C ABI.  Tolerance 1e-12 of max|chi0| with the same nodes (FP64 on both sides, sums of a few
thousand terms in another order); 1e-10 against the Adler-Wiser closed form with 48 nodes
(the quadrature itself is within 1e-12 there)."""
import sys

import numpy as np
import pytest

import synth
from oracle import screening as sc

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(psi, eps, mu, t, w):
    import torch
    import paper_1601_07728_amd as ob
    p = torch.from_numpy(np.ascontiguousarray(psi)).to("cuda")
    return ob.screening_chi0(p, eps, mu, t, w).cpu().numpy()


@pytest.mark.parametrize("n_points,n_states,n_occ,n_t", [(150, 300, 100, 32), (33, 17, 5, 8), (400, 1500, 500, 16),
                                                          (1, 40, 10, 4)])
def test_chi0_matches_oracle(n_points, n_states, n_occ, n_t):
    _say(f"[screening] n_points={n_points} n_states={n_states} n_t={n_t}")
    psi, eps, mu, t, w = synth.screening_inputs(seed=n_points + n_states, n_points=n_points, n_states=n_states,
                                                n_occ=n_occ, n_t=n_t)
    got = _run(psi, eps, mu, t, w)
    ref = sc.chi0_imaginary_axis(psi, eps, mu, t, w)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_chi0_reaches_adler_wiser():
    psi, eps, mu, t, w = synth.screening_inputs(seed=7, n_points=96, n_states=260, n_occ=80, n_t=48)
    _say("[screening vs closed form]")
    got = _run(psi, eps, mu, t, w)
    ref = sc.chi0_adler_wiser(psi, eps, mu)
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()


def test_chi0_full_grid_samples_and_properties():
    """The 900-point grid with 16384 states and 16 nodes (the benchmark shape): sampled
    elements against the oracle's element formula; symmetric and negative semidefinite."""
    import torch
    import paper_1601_07728_amd as ob
    psi, eps, mu, t, w = synth.screening_inputs(seed=11, n_points=900, n_states=16384, n_occ=8192, n_t=16)
    _say("[screening full grid]")
    p = torch.from_numpy(psi).to("cuda")
    chi = ob.screening_chi0(p, eps, mu, t, w)
    c = chi.cpu().numpy()
    scale = np.abs(c).max()
    rng = np.random.default_rng(5)
    for r, rp in [(0, 0), (899, 899), (0, 899)] + [tuple(rng.integers(0, 900, 2)) for _ in range(6)]:
        ref = sc.chi0_element(psi, eps, mu, t, w, int(r), int(rp))
        assert abs(c[r, rp] - ref) <= 1e-12 * scale, (r, rp)
    assert np.abs(c - c.T).max() <= 1e-13 * scale
    ev = torch.linalg.eigvalsh(chi).cpu().numpy()
    assert ev.max() <= 1e-12 * scale


def test_kept_scratch_serves_builds_of_any_size_and_release():
    """The device scratch kept between builds: a large build, a smaller one (the kept buffer
    is larger than needed), a larger one again (it grows), then a release and a build that
    allocates afresh; each against the oracle."""
    import paper_1601_07728_amd as ob
    cases = [(150, 300, 100, 32), (33, 17, 5, 8), (200, 420, 150, 40), (33, 17, 5, 8)]
    for k, (n_points, n_states, n_occ, n_t) in enumerate(cases):
        if k == 3:
            ob.screening_release()
        _say(f"[screening scratch] build {k}: n_points={n_points} n_states={n_states} n_t={n_t}")
        psi, eps, mu, t, w = synth.screening_inputs(seed=31 + k, n_points=n_points, n_states=n_states,
                                                    n_occ=n_occ, n_t=n_t)
        got = _run(psi, eps, mu, t, w)
        ref = sc.chi0_imaginary_axis(psi, eps, mu, t, w)
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    ob.screening_release()
    ob.screening_release()   # nothing held: a no-op
