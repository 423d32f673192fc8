"""GPU parity over a seeded spread of 64 small shapes that the hand-picked cases do not list:
k grids of any size per axis (the general, power-of-two and cube transform kernels), odd
real-space grids, band counts from 1 up, 1, 2, 3, 6 or 12 core states, with and without the
local term (6 core states), 1 to 4 vectors, skewed cells, and every projection precision.  Each case compares one
H*v per vector with the oracle, element by element: once with the default kernel choices and
once with the tuner's other forms forced on (the resident-operand forward with 1 to 16 row
tiles per block, 2 to 8 waves per back-projection block, another back-projection grid
target and transform line count)."""
import sys

import numpy as np
import pytest

import synth
from oracle import bse as orc
from oracle import multiplet as omp

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-13, "fp32": 2e-5, "split_bf16": 1e-4, "bf16": 1e-2}


def _cases(n=64, seed=2024):
    rng = np.random.default_rng(seed)
    out = []
    for c in range(n):
        nk = tuple(int(rng.choice([1, 2, 3, 4, 5, 6, 8, 16])) for _ in range(3))
        while int(np.prod(nk)) > 96:
            nk = tuple(int(rng.choice([1, 2, 3, 4])) for _ in range(3))
        nx = tuple(int(rng.integers(3, 10)) for _ in range(3))
        n_bands = int(rng.integers(1, min(40, int(np.prod(nx))) + 1))
        n_core = int(rng.choice([1, 2, 3, 6, 12]))
        local = n_core == 6 and rng.random() < 0.6
        n_vec = int(rng.integers(1, 5))
        prec = str(rng.choice(list(TOL)))
        skew = rng.random() < 0.3
        knobs = dict(OCEAN_FWD_TILES=str(int(rng.choice([1, 2, 3, 16]))),
                     OCEAN_BWD_WAVES=str(int(rng.choice([2, 4, 8]))),
                     OCEAN_BWD_BLOCKS=str(int(rng.choice([64, 1024, 8192]))),
                     OCEAN_FFT_LINES=str(int(rng.choice([4, 8, 16]))))
        out.append(dict(case=c, nk=nk, nx=nx, n_bands=n_bands, n_core=n_core, local=local, n_vec=n_vec,
                        prec=prec, skew=skew, seed=int(rng.integers(1, 1 << 30)), knobs=knobs))
    return out


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _crystal(cfg):
    cr = synth.make_crystal(f"rand{cfg['case']}", a=6.5, tau=(0.7, 1.9, 3.1), nk=cfg["nk"], nx=cfg["nx"],
                            n_bands=cfg["n_bands"], n_core=cfg["n_core"], e_range_ev=30.0, eps=5.0,
                            seed=cfg["seed"], n_local=5 if cfg["local"] else 0,
                            multiplet_ev=dict(synth.L_EDGE_MULTIPLET_EV) if cfg["local"] else None, psi0="none")
    if cfg["skew"]:
        cr.lattice = np.array([[6.5, 0.0, 0.0], [1.7, 6.1, 0.0], [-0.9, 1.3, 6.8]])
    return cr


def _check(cfg, cr, y, x):
    hc = omp.core_matrix(cr.multiplet) if cfg["local"] else None
    kl = omp.local_matrix(cr.multiplet) if cfg["local"] else None
    for v in range(cfg["n_vec"]):
        ref = orc.apply_h(cr, x[v], hc, kl)
        err = float(np.abs(y[v] - ref).max() / np.abs(ref).max())
        assert np.isfinite(y[v]).all()
        assert err <= TOL[cfg["prec"]], (cfg, v, err)


def _apply(cfg, cr):
    import torch

    import paper_1601_07728_amd as ob
    h = ob.Bse.from_crystal(cr, precision=cfg["prec"], check_inputs=True)
    x = synth.complex_gaussian(np.random.default_rng(cfg["seed"] + 1), (cfg["n_vec"], cr.n_k, cr.n_bands, cr.n_core))
    y = h.apply(torch.from_numpy(x).to("cuda")).cpu().numpy()
    h.close()
    return x, y


@pytest.mark.parametrize("cfg", _cases(), ids=lambda c: f"case{c['case']}")
def test_random_shape_apply_matches_oracle(cfg, monkeypatch):
    for k in cfg["knobs"]:
        monkeypatch.delenv(k, raising=False)
    _say(f"[random shape] {cfg}")
    cr = _crystal(cfg)
    x, y = _apply(cfg, cr)
    _check(cfg, cr, y, x)


@pytest.mark.parametrize("cfg", _cases(), ids=lambda c: f"case{c['case']}")
def test_random_shape_other_kernel_forms_match_oracle(cfg, monkeypatch):
    for k, v in cfg["knobs"].items():
        monkeypatch.setenv(k, v)
    _say(f"[random shape, forced kernel forms] {cfg}")
    cr = _crystal(cfg)
    x, y = _apply(cfg, cr)
    _check(cfg, cr, y, x)
