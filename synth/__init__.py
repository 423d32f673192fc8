"""Seeded synthetic inputs for the core-level BSE solver.

This module is shared by the CPU oracle (``oracle/``) and by the GPU library
tests and benchmark.  It draws random numbers and builds the *inputs* of the
BSE stage -- the quantities that the paper's earlier stages (DFT, translator,
screening) would otherwise supply:

* quasiparticle energies E[k, n]             (stand-in for the DFT/GW stage)
* periodic Bloch parts u_nk(x) on the x grid (stand-in for the DFT/OBF stage)
* the radial screened core-hole potential W(r) (stand-in for the screening stage)
* local-basis projector coefficients A[k, n, mu] ("precomputed and stored",
  section 3.2.2 of the paper)
* the initial exciton vector(s) psi0 (transition-operator output, eq. loss.fcn)
* the energy grid and broadening of the spectrum.

It deliberately holds none of the BSE method's arithmetic: no Hamiltonian
pieces, no Fourier transforms, no Lanczos, no continued fraction, no angular
algebra.  Multiplet parameters (zeta, F2, G1, G3) are passed on as plain numbers;
each side builds its own matrices from them.

Conventions shared by both sides (fixed by the paper's notation in section 3.2
and by the published workload description):

* energies in Hartree; 1 Ha = 27.211386245988 eV (CODATA 2018)
* lengths in bohr; cubic cell of side ``a``; Gamma-centred, unshifted k grid
  k = (2 pi / a) * (i / n_k) per axis, i = 0 .. n_k - 1
* real-space points x = a * j / n_x per axis, j = 0 .. n_x - 1
* flat grid indices are row-major with the last axis fastest
* u[k, x, n] columns are orthonormal per k: sum_x |u|^2 = 1
* exciton vectors are stored [k][n][c] (core index fastest)
* complex Gaussian = (N(0,1) + i N(0,1)) / sqrt(2)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

HARTREE_EV = 27.211386245988
RADIAL_POINTS = 64
RADIAL_RMAX = 6.0


@dataclass
class Crystal:
    """One BSE problem: the inputs of ``ocean_bse_create`` plus a spectrum request."""
    name: str
    a: float                      # cubic lattice constant, bohr
    tau: np.ndarray               # core-site position, bohr, shape (3,)
    nk: tuple                     # k grid (n1, n2, n3)
    nx: tuple                     # real-space grid per cell (g1, g2, g3)
    n_bands: int
    n_core: int                   # 2 (1s, K edge) or 6 (2p, L2,3 edge)
    energies: np.ndarray          # (Nk, Nb) Ha
    u: np.ndarray                 # (Nk, Nx, Nb) complex128
    w_r: np.ndarray               # (64,) bohr, ascending, w_r[0] = 0
    w_val: np.ndarray             # (64,) Ha
    local_proj: Optional[np.ndarray] = None   # (Nk, Nb, Nmu) complex128 or None
    multiplet: Optional[dict] = None          # zeta, F2, G1, G3 in Ha (l_core=1, l_val=2)
    psi0: Optional[np.ndarray] = None         # (n_vec, Nk, Nb, Nc) complex128, or None
    polarisations: Optional[np.ndarray] = None  # (n_pol, 3) unit vectors for dipole psi0
    n_steps: int = 100
    gamma: float = 0.5 / HARTREE_EV           # Lorentzian HWHM, Ha
    omega: np.ndarray = field(default_factory=lambda: np.zeros(0))  # Ha
    eps: float = 5.0
    lattice: Optional[np.ndarray] = None      # (3, 3) rows a1, a2, a3, bohr; None: cubic cell of edge a
    kshift: tuple = (0.0, 0.0, 0.0)           # k-grid offset along b_d, in grid steps (0: Gamma-centred)
    channels: Optional[dict] = None           # general local basis: l, f2, gk, radial (see full_local_basis)

    def cell_vectors(self) -> np.ndarray:
        """Rows a1, a2, a3 of the cell (bohr)."""
        return np.asarray(self.lattice, dtype=np.float64) if self.lattice is not None else self.a * np.eye(3)

    @property
    def n_k(self) -> int:
        return int(np.prod(self.nk))

    @property
    def n_x(self) -> int:
        return int(np.prod(self.nx))

    @property
    def n_local(self) -> int:
        return 0 if self.local_proj is None else int(self.local_proj.shape[2])

    @property
    def dim(self) -> int:
        return self.n_core * self.n_k * self.n_bands


def complex_gaussian(rng: np.random.Generator, shape) -> np.ndarray:
    """(N(0,1) + i N(0,1)) / sqrt(2), real part drawn first."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) / math.sqrt(2.0)


def orthonormal_columns(z: np.ndarray) -> np.ndarray:
    """Q of a reduced QR of z (columns orthonormal), with the phase of diag(R)
    moved into Q so the result is unique."""
    q, r = np.linalg.qr(z)
    d = np.diagonal(r)
    ph = np.where(np.abs(d) > 0, d / np.abs(d), 1.0)
    return q * ph[None, :]


def radial_table(eps: float) -> tuple[np.ndarray, np.ndarray]:
    """W(r) = erf(r / 0.5) / (eps r) Ha on r_j = 6 j / 63 bohr; W(0) is the r -> 0 limit.

    This stands in for the output of the screening stage (section 3.3)."""
    r = RADIAL_RMAX * np.arange(RADIAL_POINTS) / (RADIAL_POINTS - 1)
    w = np.empty_like(r)
    w[0] = 2.0 / (math.sqrt(math.pi) * 0.5 * eps)
    for j in range(1, RADIAL_POINTS):
        w[j] = math.erf(r[j] / 0.5) / (eps * r[j])
    return r, w


def omega_grid(lo_ev: float, hi_ev: float, n: int = 2000) -> np.ndarray:
    return np.linspace(lo_ev, hi_ev, n) / HARTREE_EV


def make_crystal(name: str, *, a: float, tau, nk, nx, n_bands: int, n_core: int,
                 e_range_ev: float, eps: float, seed: int, n_local: int = 0,
                 multiplet_ev: Optional[dict] = None, psi0: str = "random",
                 n_vec: int = 1, polarisations=None, n_steps: int = 100,
                 gamma_ev: float = 0.5, omega_ev=(-20.0, 40.0), n_omega: int = 2000,
                 u_override: Optional[np.ndarray] = None, e_min_ev: float = 0.0) -> Crystal:
    """Draw one synthetic crystal.  Draw order: E (uniform on [e_min, e_min + e_range] eV),
    then U per k (real then imaginary parts), then psi0 amplitudes, then the local
    projectors A."""
    rng = np.random.default_rng(seed)
    n_k = int(np.prod(nk))
    n_x = int(np.prod(nx))
    energies = np.sort(rng.uniform(e_min_ev, e_min_ev + e_range_ev, size=(n_k, n_bands)), axis=1) / HARTREE_EV
    if isinstance(u_override, str) and u_override == "skip":
        u = None          # generated elsewhere (e.g. on the device); no host draw
    elif u_override is not None:
        u = u_override
    else:
        # the draws stay in order (k by k, real then imaginary parts); the QRs, independent per
        # k, run on a thread pool (LAPACK releases the interpreter lock)
        u = np.empty((n_k, n_x, n_bands), dtype=np.complex128)
        for k in range(n_k):
            u[k] = complex_gaussian(rng, (n_x, n_bands))

        def _qr(k):
            u[k] = orthonormal_columns(u[k])

        if n_k > 1 and n_x * n_bands >= 4096:
            from concurrent.futures import ThreadPoolExecutor
            import os
            with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
                list(ex.map(_qr, range(n_k)))
        else:
            for k in range(n_k):
                _qr(k)
    p0 = None
    if psi0 == "random":
        # dipole-like amplitudes M[k, n], identical for every core state (spin-
        # independent transition operator), one independent draw per vector
        p0 = np.empty((n_vec, n_k, n_bands, n_core), dtype=np.complex128)
        for v in range(n_vec):
            m = complex_gaussian(rng, (n_k, n_bands))
            p0[v] = m[:, :, None]
    elif psi0 == "random_full":
        p0 = complex_gaussian(rng, (n_vec, n_k, n_bands, n_core))
    local = None
    if n_local > 0:
        z = complex_gaussian(rng, (n_k * n_bands, n_local))
        local = orthonormal_columns(z).reshape(n_k, n_bands, n_local)
    mult = None
    if multiplet_ev is not None:
        mult = {key: val / HARTREE_EV for key, val in multiplet_ev.items()}
    w_r, w_val = radial_table(eps)
    pol = None if polarisations is None else np.asarray(polarisations, dtype=np.float64)
    return Crystal(name=name, a=float(a), tau=np.asarray(tau, dtype=np.float64),
                   nk=tuple(nk), nx=tuple(nx), n_bands=n_bands, n_core=n_core,
                   energies=energies, u=u, w_r=w_r, w_val=w_val, local_proj=local,
                   multiplet=mult, psi0=p0, polarisations=pol, n_steps=n_steps,
                   gamma=gamma_ev / HARTREE_EV,
                   omega=omega_grid(omega_ev[0], omega_ev[1], n_omega), eps=eps)


L_EDGE_MULTIPLET_EV = {"zeta": 3.8, "F2": 8.0, "G1": 6.0, "G3": 3.5}
XYZ_POLARISATIONS = np.eye(3)
SRTIO3_A = 7.38


def config1(seed: int = 0) -> Crystal:
    """K edge, 1 site at the origin, a = 7.38 bohr, 2^3 k, 16 bands in [0, 30] eV,
    8^3 x grid, eps = 5, complex-normal dipole amplitudes, 100 steps."""
    return make_crystal("c1", a=SRTIO3_A, tau=(0.0, 0.0, 0.0), nk=(2, 2, 2), nx=(8, 8, 8),
                        n_bands=16, n_core=2, e_range_ev=30.0, eps=5.0, seed=seed,
                        psi0="random", n_steps=100, omega_ev=(-20.0, 40.0))


def config2_shape(nk=(8, 8, 8), nx=(20, 20, 20), n_bands=96, seed: int = 0,
                  eps: float = 6.0, n_steps: int = 300, psi0: str = "random", n_vec: int = 1,
                  u_override=None, e_range_ev: float = 40.0) -> Crystal:
    """Ti L2,3 edge in a 5-atom SrTiO3-shaped cubic cell (core site at the Ti
    position (1/2,1/2,1/2) a): 2p core (6 spin-orbitals), d-channel local term,
    zeta = 3.8, F2 = 8, G1 = 6, G3 = 3.5 eV.  Defaults give the full-size
    workload (8^3 k, 96 bands, 20^3 x, H dimension 294912)."""
    return make_crystal("c2", a=SRTIO3_A, tau=(0.5 * SRTIO3_A,) * 3, nk=nk, nx=nx,
                        n_bands=n_bands, n_core=6, e_range_ev=e_range_ev, eps=eps, seed=seed,
                        n_local=5, multiplet_ev=dict(L_EDGE_MULTIPLET_EV), psi0=psi0,
                        n_vec=n_vec, polarisations=XYZ_POLARISATIONS, n_steps=n_steps,
                        omega_ev=(-25.0, 55.0), u_override=u_override)


def config3_shape(seed: int = 0, n_steps: int = 300, psi0: str = "none", u_override="skip",
                  nk=(2, 2, 2), nx=(64, 64, 64), n_bands: int = 1200) -> Crystal:
    """Ti L2,3 edge at one site of a 4x4x4 supercell of the SrTiO3-shaped cell (320 atoms,
    a_s = 4 a, the site at the first Ti, (1/2,1/2,1/2) a): 2^3 k, 1200 bands in [0, 40] eV,
    64^3 x, the c2 screening and multiplet parameters.  u (40 GB in FP64) is meant to be
    drawn on the device (gpu_orthonormal_u)."""
    return make_crystal("c3", a=4.0 * SRTIO3_A, tau=(0.5 * SRTIO3_A,) * 3, nk=nk, nx=nx,
                        n_bands=n_bands, n_core=6, e_range_ev=40.0, eps=6.0, seed=seed,
                        n_local=5, multiplet_ev=dict(L_EDGE_MULTIPLET_EV), psi0=psi0,
                        polarisations=XYZ_POLARISATIONS, n_steps=n_steps,
                        omega_ev=(-25.0, 55.0), u_override=u_override)


def small_l_edge(seed: int = 1, nk=(2, 2, 2), nx=(6, 6, 6), n_bands=12, **kw) -> Crystal:
    """A tiny L-edge crystal (dense H feasible) for parity and pin tests."""
    return config2_shape(nk=nk, nx=nx, n_bands=n_bands, seed=seed, **kw)


def full_spin(cr: Crystal) -> Crystal:
    """The same crystal with the electron spin carried separately: 12 core states
    (m_c, sigma_h, sigma_e).  Inputs are unchanged; only the space doubles."""
    import dataclasses
    out = dataclasses.replace(cr, n_core=12, psi0=None)
    if cr.psi0 is not None:
        p = np.zeros(cr.psi0.shape[:3] + (12,), dtype=np.complex128)
        for c in range(cr.n_core):
            p[..., 2 * c + (c % 2)] = cr.psi0[..., c]
        out.psi0 = p
    return out


# --- device-side generation for the full-size workloads ---------------------------------

def gpu_orthonormal_u(n_k: int, n_x: int, n_bands: int, seed: int, device="cuda"):
    """U[k] = orthonormal columns of a complex Gaussian (n_x x n_bands) per k, drawn
    with torch's device RNG and orthonormalised by two passes of Cholesky QR.
    Used where a host QR of gigabytes would dominate the run; the oracle then
    receives a host copy of exactly these values."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    u = torch.empty((n_k, n_x, n_bands), dtype=torch.complex128, device=device)
    for k in range(n_k):
        z = torch.randn((n_x, n_bands), dtype=torch.complex128, device=device, generator=g)
        for _ in range(2):
            gram = (z.conj().transpose(0, 1).contiguous() @ z)
            gram = 0.5 * (gram + gram.conj().transpose(0, 1))
            r = torch.linalg.cholesky(gram).conj().transpose(0, 1).contiguous()   # G = R^H R
            eye = torch.eye(n_bands, dtype=z.dtype, device=device)
            rinv = torch.linalg.solve_triangular(r, eye, upper=True)            # small solve
            z = z @ rinv                                                        # Q = Z R^-1
        u[k] = z
    return u


def gpu_orthonormal_u_batched(n_k: int, n_x: int, n_bands: int, seed: int, device="cuda"):
    """As gpu_orthonormal_u, with every k drawn in one call and the two Cholesky-QR passes
    batched over k (a different stream of random numbers from gpu_orthonormal_u)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    z = torch.randn((n_k, n_x, n_bands), dtype=torch.complex128, device=device, generator=g)
    eye = torch.eye(n_bands, dtype=z.dtype, device=device).expand(n_k, n_bands, n_bands)
    for _ in range(2):
        gram = torch.matmul(z.conj().transpose(1, 2).contiguous(), z)
        gram = 0.5 * (gram + gram.conj().transpose(1, 2))
        r = torch.linalg.cholesky(gram).conj().transpose(1, 2).contiguous()       # G = R^H R
        rinv = torch.linalg.solve_triangular(r, eye, upper=True)
        z = torch.matmul(z, rinv.contiguous())                                  # Q = Z R^-1
        del gram, r, rinv
    return z.contiguous()


# --- molecule in a box: many absorbing sites, Gamma point only ---------------------------

def molecule_sites(seed: int = 0, n_atoms: int = 52, n_sites: int = 40, box: float = 30.0,
                   grid: int = 48, nb_range=(200, 800), p_k_edge: float = 0.5,
                   min_spacing: float = 2.5, device_u: bool = True):
    """An Alq3-sized molecule in a periodic cubic box (Gamma point only): atoms placed by
    seeded rejection sampling at >= min_spacing bohr (minimum image), the first n_sites
    of them absorbing sites.  Each site is a K edge (2 core states, no local term) with
    probability p_k_edge, else an L2,3 edge (6 core states, d-channel local term, the
    SrTiO3 multiplet parameters).  Per site: band count uniform in nb_range, energies
    U[0, 40] eV, eps U[2, 10], its own u on the grid^3 box grid.  K edges get three
    complex-normal amplitude vectors (one per polarisation); L edges carry x, y, z
    polarisations for the dipole rule.

    Returns a list of (Crystal, u) with u a device tensor (device_u) or the host array in
    Crystal.u."""
    rng = np.random.default_rng(seed)
    pos = []
    while len(pos) < n_atoms:
        p = rng.uniform(0.0, box, size=3)
        ok = True
        for q in pos:
            d = p - q
            d = d - box * np.round(d / box)
            if np.sqrt(np.sum(d * d)) < min_spacing:
                ok = False
                break
        if ok:
            pos.append(p)
    sites = []
    for s in range(n_sites):
        k_edge = rng.uniform() < p_k_edge
        nb = int(rng.integers(nb_range[0], nb_range[1] + 1))
        eps = float(rng.uniform(2.0, 10.0))
        site_seed = int(rng.integers(0, 2 ** 31 - 1))
        common = dict(a=box, tau=pos[s], nk=(1, 1, 1), nx=(grid,) * 3, n_bands=nb,
                      e_range_ev=40.0, eps=eps, seed=site_seed, n_steps=200,
                      omega_ev=(-20.0, 45.0), u_override="skip" if device_u else None)
        if k_edge:
            cr = make_crystal(f"site{s}-K", n_core=2, psi0="random", n_vec=3, **common)
        else:
            cr = make_crystal(f"site{s}-L23", n_core=6, n_local=5,
                              multiplet_ev=dict(L_EDGE_MULTIPLET_EV), psi0="none",
                              polarisations=XYZ_POLARISATIONS, **common)
        u = None
        if device_u:
            u = gpu_orthonormal_u(1, grid ** 3, nb, seed=site_seed)
        sites.append((cr, u))
    return sites


def xes_site(seed: int = 0, n_occ: int = 81, box: float = 30.0, grid: int = 48, width_ev: float = 25.0,
             eps: float = 4.0, n_steps: int = 200, u_override=None) -> Crystal:
    """One K-edge emission (XES) site of an Alq3-sized molecule in a periodic box (Gamma point
    only): the band window is the occupied valence manifold, n_occ bands (81 = half of Alq3's
    162 valence electrons) with energies uniform on [-width, 0] eV below the Fermi level, 2
    core states (1s), no local term, three complex-normal amplitude vectors (one per
    polarisation), the site at the box centre.  The emission lines sit at E_v - E_c <= 0."""
    return make_crystal(f"xes{seed}-K", a=box, tau=(box / 2, box / 2, box / 2), nk=(1, 1, 1), nx=(grid,) * 3,
                        n_bands=n_occ, n_core=2, e_range_ev=width_ev, e_min_ev=-width_ev, eps=eps, seed=seed,
                        psi0="random", n_vec=3, n_steps=n_steps, omega_ev=(-width_ev - 12.0, 12.0),
                        u_override=u_override)


def terminator_params(seed: int) -> tuple[float, float]:
    """(eps, band width in eV) of terminator-dataset system `seed`: eps ~ U[2, 10], width ~ U[20, 60]."""
    rng = np.random.default_rng([seed, 7])
    eps = float(rng.uniform(2.0, 10.0))
    width = float(rng.uniform(20.0, 60.0))
    return eps, width


def terminator_omega(seed: int, n: int = 2000) -> np.ndarray:
    """Energy grid of system `seed`'s spectrum: n points on [-15, width + 15] eV (in Ha)."""
    return omega_grid(-15.0, terminator_params(seed)[1] + 15.0, n)


def terminator_system(seed: int, nk=(2, 2, 2), nx=(5, 5, 5), n_bands: int = 24,
                      n_steps: int = 512, u_override=None) -> Crystal:
    """One system of the learned-terminator dataset: the SrTiO3-shaped L2,3 edge (any grid
    and band count), with eps ~ U[2, 10] and band width ~ U[20, 60] eV drawn from the seed."""
    eps, width = terminator_params(seed)
    return config2_shape(nk=nk, nx=nx, n_bands=n_bands, seed=seed, eps=eps, n_steps=n_steps,
                         psi0="none", e_range_ev=width, u_override=u_override)


TERMINATOR_U_SEED_OFFSET = 1 << 20


def terminator_system_device(seed: int, nk=(8, 8, 8), nx=(20, 20, 20), n_bands: int = 96,
                             n_steps: int = 512, device="cuda"):
    """A terminator-dataset system at the full SrTiO3-shaped size (default 8^3 k, 20^3 x,
    96 bands), with u drawn on the device in one batch (gpu_orthonormal_u_batched, seed +
    TERMINATOR_U_SEED_OFFSET).  Returns (Crystal, u)."""
    cr = terminator_system(seed, nk=nk, nx=nx, n_bands=n_bands, n_steps=n_steps, u_override="skip")
    u = gpu_orthonormal_u_batched(cr.n_k, cr.n_x, cr.n_bands, seed=seed + TERMINATOR_U_SEED_OFFSET,
                                  device=device)
    return cr, u


# --- screening inputs (the RPA response on the real-space sphere around the core site) --------

def screening_inputs(seed: int = 0, n_points: int = 900, n_states: int = 2048, n_occ: int = 512,
                     n_t: int = 16, gap_ev: float = 2.0, occ_width_ev: float = 20.0,
                     unocc_width_ev: float = 60.0, t_scale_ev: float = 10.0):
    """Bloch functions on the screening grid (the paper's 36 angles x 25 radii = 900 points),
    their energies, the chemical potential in the gap, and the imaginary-frequency
    quadrature.  Draw order: psi (complex Gaussian, scaled by 1/sqrt(n_points)), then the
    occupied and empty energies.  The nodes t_j and weights w_j integrate over t in
    [0, inf): Gauss-Legendre on x in (-1, 1) (numpy.polynomial.legendre.leggauss) mapped by
    t = T (1 + x) / (1 - x), dt = 2 T / (1 - x)^2 dx, with T = t_scale.  Energies in Ha."""
    rng = np.random.default_rng(seed)
    psi = complex_gaussian(rng, (n_points, n_states)) / math.sqrt(n_points)
    e_occ = np.sort(rng.uniform(-occ_width_ev, 0.0, size=n_occ))
    e_unocc = np.sort(rng.uniform(gap_ev, gap_ev + unocc_width_ev, size=n_states - n_occ))
    eps = np.concatenate([e_occ, e_unocc]) / HARTREE_EV
    mu = 0.5 * gap_ev / HARTREE_EV
    x, wx = np.polynomial.legendre.leggauss(n_t)
    tsc = t_scale_ev / HARTREE_EV
    t = tsc * (1.0 + x) / (1.0 - x)
    w = wx * 2.0 * tsc / (1.0 - x) ** 2
    return psi, eps, mu, t, w


def full_local_basis(cr: Crystal, seed: int = 0, n_radial: int = 4, f2_ev: float = 8.0, g_ev: float = 6.0) -> Crystal:
    """The same crystal with the local basis of section 3.2.2 in full: n_radial radial functions
    for each of l = s, p, d, f (64 local functions for 4), channel order (l, radial).
    Draw order: A (QR of a complex Gaussian over (k, n)), then the radial tables: the direct
    F^2 and each exchange G^k (k = 0..4) as Gram matrices B B^T / n of Gaussian B (positive
    semidefinite, scaled to f2_ev / g_ev), then the dipole radial integrals (Gaussian, s and d
    channels only; others are ignored by the selection rules).  Energies in Ha."""
    import dataclasses
    rng = np.random.default_rng(seed)
    ls = [l for l in range(4) for _ in range(n_radial)]
    n = len(ls)
    nmu = sum(2 * l + 1 for l in ls)
    z = complex_gaussian(rng, (cr.n_k * cr.n_bands, nmu))
    a = orthonormal_columns(z).reshape(cr.n_k, cr.n_bands, nmu)

    def gram(scale):
        b = rng.normal(size=(n, n))
        return scale / HARTREE_EV * (b @ b.T) / n

    f2 = gram(f2_ev)
    gk = np.stack([gram(g_ev) for _ in range(5)])
    radial = rng.normal(size=n)
    out = dataclasses.replace(cr, local_proj=a, psi0=None)
    out.channels = {"l": ls, "f2": f2, "gk": gk, "radial": radial}
    return out
