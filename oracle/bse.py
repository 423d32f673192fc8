"""Plain FP64 reference of the BSE H*v, Haydock recursion and spectrum.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the GPU library and never calls it.

Everything here is written for checking by eye against the paper
(Gilmore et al., "Efficient implementation of core-excitation Bethe-Salpeter
equation calculations", section 2 and section 3.2):

* the loss function sigma ~ -(1/pi) Im <0|O+ G(w) O|0>, G = [w - H_BSE]^-1 (eq. loss.fcn)
* H_BSE = H_e - H_h - V_D + V_X (eq. H_BSE), with H_h = eps_c + chi - i Gamma
* the long-range direct term W0 applied by Algorithm 1 (section 3.2.1)
* the short-range terms through the local basis (eq. local_basis, section 3.2.2)
* the Haydock recursion (eq. haydock1 and the cited Haydock method)

Readings where the paper is silent:

* Fourier pair of Algorithm 1 (k -> R and back): unitary, e^{+ik.R} forward and
  e^{-ik.R} back, with Nk^{-1/2} each way.
* W(x, R) = W_rad(|x + R - tau|) with the minimum image in the Born-von-Karman
  supercell (the k grid fixes the range of W, section 3.2.1); W_rad is the
  linear interpolation of the radial table, and W(r_max) r_max / r beyond it.
* The cell is given by three lattice vectors (any shape); x and R are fractional
  multiples of them.  The k grid may be offset by a fraction of a grid step along
  each reciprocal vector (the paper's runs use shifted 2x2x2 grids, section 4).
* -V_D enters with a minus sign; eps_c = 0; Gamma is a constant Lorentzian
  broadening z = w + i Gamma.
* Haydock is the three-term Lanczos recursion; b_0 = 0; optional full
  re-orthogonalisation (two passes of classical Gram-Schmidt).
* Vectors are psi[k, n, c] (core index fastest).

Explicit sums and dense matrices only: the k <-> R transform is an explicit
DFT matrix, never an FFT.
"""
from __future__ import annotations

import math

import numpy as np


# --- grids (section 3.2.1: k-points, lattice vectors R, points x in the cell) ---

def _grid_indices(n):
    """All integer triples (i1, i2, i3), i_d in [0, n_d), last axis fastest."""
    n1, n2, n3 = n
    i1, i2, i3 = np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij")
    return np.stack([i1.ravel(), i2.ravel(), i3.ravel()], axis=1).astype(np.float64)


def cell_vectors(cr):
    """Rows a1, a2, a3 of the cell, bohr (cr.lattice, or a cubic cell of edge cr.a)."""
    lat = getattr(cr, "lattice", None)
    return np.asarray(lat, dtype=np.float64) if lat is not None else cr.a * np.eye(3)


def reciprocal_vectors(cr):
    """Rows b1, b2, b3 with a_i . b_j = 2 pi delta_ij."""
    return 2.0 * math.pi * np.linalg.inv(cell_vectors(cr)).T


def kpoints(cr):
    """k = sum_d ((i_d + s_d) / n_d) b_d: the k grid, offset by s_d grid steps along b_d
    (s = 0 is the Gamma-centred unshifted grid; the paper's runs use s = 1/2)."""
    shift = np.asarray(getattr(cr, "kshift", (0.0, 0.0, 0.0)), dtype=np.float64)
    frac = (_grid_indices(cr.nk) + shift) / np.asarray(cr.nk, dtype=np.float64)
    return frac @ reciprocal_vectors(cr)


def lattice_vectors(cr):
    """R = sum_d r_d a_d, r_d in [0, n_d): the cells of the Born-von-Karman supercell."""
    return _grid_indices(cr.nk) @ cell_vectors(cr)


def xpoints(cr):
    """x = sum_d (j_d / g_d) a_d, j_d in [0, g_d): the real-space grid of one cell."""
    return (_grid_indices(cr.nx) / np.asarray(cr.nx, dtype=np.float64)) @ cell_vectors(cr)


# --- the screened core-hole potential W(x, R) ---------------------------------------------

def w_radial(w_r, w_val, r):
    """Radial W at distances r: linear interpolation of the table; beyond the
    last node W(r_max) r_max / r (W0 goes as 1/r far from the core hole)."""
    r = np.asarray(r, dtype=np.float64)
    out = np.empty_like(r)
    rmax = w_r[-1]
    h = w_r[1] - w_r[0]
    far = r >= rmax
    out[far] = w_val[-1] * rmax / r[far]
    near = ~far
    s = r[near] / h
    j = np.floor(s).astype(np.int64)
    j = np.minimum(j, len(w_r) - 2)
    t = s - j
    out[near] = (1.0 - t) * w_val[j] + t * w_val[j + 1]
    return out


def min_image_distance(d, sup):
    """|d| for the image of d nearest the origin in the lattice whose rows are sup.  The
    fractional coordinates are wrapped into [-1/2, 1/2) and the 27 images around the
    wrapped point are compared; for an orthogonal lattice the wrapped point itself is the
    nearest.  (For a reduced, not too skewed basis the nearest image is among the 27; the
    pins compare against a wider search.)"""
    f = d @ np.linalg.inv(sup)
    f = f - np.round(f)
    if np.allclose(sup, np.diag(np.diag(sup))):
        return np.sqrt(np.sum((f @ sup) ** 2, axis=-1))
    best = None
    for m in np.ndindex(3, 3, 3):
        dist = np.sqrt(np.sum(((f + (np.array(m) - 1)) @ sup) ** 2, axis=-1))
        best = dist if best is None else np.minimum(best, dist)
    return best


def w_supercell(cr):
    """W[x, R] = W_rad(|x + R - tau|) with the minimum image in the Born-von-Karman
    supercell (rows n_d a_d)."""
    x = xpoints(cr)
    rv = lattice_vectors(cr)
    sup = np.asarray(cr.nk, dtype=np.float64)[:, None] * cell_vectors(cr)
    out = np.empty((len(x), len(rv)))
    step = max(1, (1 << 22) // max(1, len(rv)))   # x points per chunk: about 4M (x, R) pairs
    for x0 in range(0, len(x), step):
        d = x[x0:x0 + step, None, :] + rv[None, :, :] - np.asarray(cr.tau)[None, None, :]
        out[x0:x0 + step] = w_radial(cr.w_r, cr.w_val, min_image_distance(d, sup).ravel()).reshape(d.shape[:2])
    return out


def folded_u(cr):
    """e^{ik.x} u_nk(x): the phase factor of Algorithm 1's band-to-real-space step folded into u."""
    k = kpoints(cr)
    x = xpoints(cr)
    phase = np.exp(1j * (k @ x.T))            # [k, x]
    return cr.u * phase[:, :, None]


def dft_matrix(cr):
    """F[R, k] = Nk^{-1/2} e^{+ik.R} (Algorithm 1, k -> R); its conjugate transpose is R -> k."""
    return np.exp(1j * (lattice_vectors(cr) @ kpoints(cr).T)) / math.sqrt(cr.n_k)


# --- Hamiltonian pieces ----------------------------------------------------------------------

def apply_w0(cr, psi, ut=None, w=None, f=None):
    """W0 psi by Algorithm 1, every core index alpha at once (the long-range direct term
    does not mix spin or angular momentum, so alpha is a spectator column).  psi is
    [k, n, c].  The band sums are matrix products per k."""
    ut = folded_u(cr) if ut is None else ut
    w = w_supercell(cr) if w is None else w
    f = dft_matrix(cr) if f is None else f
    nk = psi.shape[0]
    # band -> real space: phi(k, x, alpha) = sum_n psi_{n,k,alpha} e^{ik.x} u_nk(x)
    phi_k = np.stack([ut[k] @ psi[k] for k in range(nk)])            # [k, x, c]
    nx, nc = phi_k.shape[1], phi_k.shape[2]
    # k -> R: phi(R) = F_{k->R}[phi(k)], one matrix product over k for every (x, alpha)
    phi_r = (f @ phi_k.reshape(nk, nx * nc)).reshape(-1, nx, nc)
    # screened potential: phi(R) = W(x, R) phi(R)
    phi_r = w.T[:, :, None] * phi_r
    # R -> k: phi(k) = F_{R->k}[phi(R)]
    phi_k = (f.conj().T @ phi_r.reshape(-1, nx * nc)).reshape(nk, nx, nc)
    # real space -> band: psi'_{n,k,alpha} = sum_x conj(e^{ik.x} u_nk(x)) phi(k, x, alpha)
    return np.stack([(ut[k].T @ phi_k[k].conj()).conj() for k in range(nk)])


def apply_local(psi, local_proj, local_mat):
    """Short-range term through the local basis (section 3.2.2): project onto the
    local channels, apply the (core x channel) interaction matrix, project back.
    b[c, mu] = sum_{k,n} A[k,n,mu] psi[k,n,c]; b' = K b; out = sum_mu conj(A) b'."""
    nmu = local_proj.shape[2]
    nc = psi.shape[2]
    b = np.einsum("knm,knc->cm", local_proj, psi).reshape(nc * nmu)
    bp = (local_mat @ b).reshape(nc, nmu)
    return np.einsum("knm,cm->knc", local_proj.conj(), bp)


def apply_h(cr, psi, core_mat=None, local_mat=None, w_scale=1.0, ut=None, w=None, f=None):
    """H psi = E psi + Hc psi - W0 psi + (local term), psi[k, n, c].

    E: diagonal quasiparticle energies (H_e); Hc = -(eps_c + chi) acts on the core
    index (-H_h, eps_c = 0); W0 enters with a minus sign (-V_D, attractive)."""
    out = cr.energies[:, :, None] * psi
    if core_mat is not None:
        out = out + np.einsum("cd,knd->knc", core_mat, psi)
    if w_scale != 0.0:
        out = out - w_scale * apply_w0(cr, psi, ut=ut, w=w, f=f)
    if local_mat is not None and cr.local_proj is not None:
        out = out + apply_local(psi, cr.local_proj, local_mat)
    return out


def w0_matrix(cr):
    """Explicit W0 on (k, n) for one core index:
    M[(k,n),(k',n')] = sum_x conj(ut[k,x,n]) ut[k',x,n'] sum_R conj(F[R,k]) W[x,R] F[R,k']."""
    ut = folded_u(cr)
    w = w_supercell(cr)
    f = dft_matrix(cr)
    kern = np.einsum("rk,xr,rq->xkq", f.conj(), w, f)      # [x, k, k']
    m = np.einsum("kxn,xkq,qxm->knqm", ut.conj(), kern, ut)
    nb = cr.n_bands
    return m.reshape(cr.n_k * nb, cr.n_k * nb)


def h_dense(cr, core_mat=None, local_mat=None, w_scale=1.0):
    """The BSE Hamiltonian as an explicit matrix over flat index ((k*Nb)+n)*Nc+c."""
    nk, nb, nc = cr.n_k, cr.n_bands, cr.n_core
    dim = nk * nb * nc
    h = np.zeros((nk, nb, nc, nk, nb, nc), dtype=np.complex128)
    e = cr.energies
    for c in range(nc):
        h[:, :, c, :, :, c] += np.diag(e.ravel()).reshape(nk, nb, nk, nb)
    if core_mat is not None:
        for k in range(nk):
            for n in range(nb):
                h[k, n, :, k, n, :] += core_mat
    if w_scale != 0.0:
        m = w0_matrix(cr).reshape(nk, nb, nk, nb)
        for c in range(nc):
            h[:, :, c, :, :, c] -= w_scale * m
    if local_mat is not None and cr.local_proj is not None:
        a = cr.local_proj
        nmu = a.shape[2]
        kl = local_mat.reshape(nc, nmu, nc, nmu)
        h += np.einsum("knm,cmdl,qpl->kncqpd", a.conj(), kl, a)
    return h.reshape(dim, dim)


# --- Haydock recursion and the continued fraction ----------------------------------------------

def haydock(apply, psi0, n_steps, reorth=False, tol=1e-14):
    """Three-term Lanczos recursion started from psi0 / |psi0|.

    Returns (a[0..s-1], b[1..s], |psi0|^2, s, basis) where s <= n_steps is the
    number of completed steps; the recursion stops early when
    b_{i+1} <= tol * max(|a_0..a_i|, b_1..b_i) (an invariant Krylov subspace)."""
    norm2 = float(np.vdot(psi0, psi0).real)
    v = psi0 / math.sqrt(norm2)
    v_prev = np.zeros_like(v)
    b_i = 0.0
    a_list, b_list = [], []
    basis = [v]
    scale = 0.0
    for i in range(n_steps):
        w = apply(v)
        a_i = float(np.vdot(v, w).real)
        w = w - a_i * v - b_i * v_prev
        if reorth:
            vs = np.stack([q.ravel() for q in basis], axis=0)
            for _ in range(2):
                h = vs.conj() @ w.ravel()
                w = w - (h @ vs).reshape(w.shape)
        b_next = float(np.sqrt(np.vdot(w, w).real))
        a_list.append(a_i)
        b_list.append(b_next)
        scale = max(scale, abs(a_i), b_i)
        if b_next <= tol * scale:
            return np.array(a_list), np.array(b_list), norm2, i + 1, basis
        v_prev, v = v, w / b_next
        b_i = b_next
        basis.append(v)
    return np.array(a_list), np.array(b_list), norm2, n_steps, basis


def sqrt_terminator(z, a_inf, b_inf):
    """Green's function of a semi-infinite chain with constant (a_inf, b_inf):
    t = [(z - a) - sqrt((z - a)^2 - 4 b^2)] / (2 b^2), the root with Im t <= 0."""
    zz = z - a_inf
    s = np.sqrt(zz * zz - 4.0 * b_inf * b_inf + 0j)
    t1 = (zz - s) / (2.0 * b_inf * b_inf)
    t2 = (zz + s) / (2.0 * b_inf * b_inf)
    return np.where(t1.imag <= 0.0, t1, t2)


def continued_fraction(a, b, z, terminator="none", a_inf=None, b_inf=None):
    """g(z) = 1/(z - a_0 - b_1^2/(z - a_1 - ... - b_{N-1}^2/(z - a_{N-1} - b_N^2 t(z)))),
    evaluated from the bottom up.  b holds b_1..b_N."""
    n = len(a)
    z = np.asarray(z, dtype=np.complex128)
    if terminator == "none":
        g = np.zeros_like(z)
    elif terminator == "sqrt":
        g = sqrt_terminator(z, a_inf, b_inf)
    else:
        raise ValueError(terminator)
    for i in range(n - 1, -1, -1):
        g = 1.0 / (z - a[i] - b[i] * b[i] * g)
    return g


def terminator_params(a, b, tail=16):
    """Asymptotic chain parameters: means of the last `tail` coefficients."""
    return float(np.mean(a[-tail:])), float(np.mean(b[-tail:]))


def spectrum(a, b, norm2, omega, gamma, terminator="none", a_inf=None, b_inf=None):
    """sigma(w) = -(1/pi) |psi0|^2 Im g(w + i Gamma) (eq. loss.fcn with G = [w - H]^-1)."""
    if terminator == "sqrt" and a_inf is None:
        a_inf, b_inf = terminator_params(a, b)
    g = continued_fraction(a, b, np.asarray(omega) + 1j * gamma, terminator, a_inf, b_inf)
    return -norm2 * g.imag / math.pi


def spectrum_dense(h, psi0, omega, gamma):
    """The same spectrum from the eigen-decomposition of an explicit Hermitian H:
    sigma(w) = (1/pi) sum_j |<q_j|psi0>|^2 Gamma / ((w - lambda_j)^2 + Gamma^2)."""
    lam, q = np.linalg.eigh(h)
    wts = np.abs(q.conj().T @ psi0.ravel()) ** 2
    om = np.asarray(omega)[:, None]
    return np.sum(wts[None, :] * gamma / ((om - lam[None, :]) ** 2 + gamma ** 2), axis=1) / math.pi


def l1_relative(sig, ref):
    return float(np.sum(np.abs(sig - ref)) / np.sum(np.abs(ref)))
