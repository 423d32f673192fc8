"""MI355X (gfx950) core-level BSE solver: Python binding of libocean_bse.so.

Thin ctypes marshalling over the C ABI declared in include/ocean_bse.h: every
computation runs in the library's HIP kernels.  PyTorch is used only to hold
device memory (exciton vectors are torch.complex128 CUDA tensors whose
data_ptr() is handed to the library).  If the shared library has not been
built, importing works but every call raises RuntimeError -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# OCEAN_BSE_LIB names another build of the same library (the AddressSanitizer build of the
# host-side checks); by default the in-tree library is loaded
LIB_PATH = os.environ.get("OCEAN_BSE_LIB") or os.path.join(_HERE, "libocean_bse.so")

OK = 0
INFO_INVARIANT_SUBSPACE = 1
ERR_INVALID_ARG = -1
ERR_OUT_OF_MEMORY = -2
ERR_DEVICE = -3
ERR_UNSUPPORTED = -4

PREC_FP64 = 0
PREC_FP32 = 1
PREC_SPLIT_BF16 = 2
PREC_BF16 = 3
PRECISIONS = {"fp64": PREC_FP64, "fp32": PREC_FP32, "split_bf16": PREC_SPLIT_BF16, "bf16": PREC_BF16}

FLAG_BORROW_DEVICE_U = 0x1
FLAG_CHECK_INPUTS = 0x2
HAYDOCK_REORTH = 0x1
HAYDOCK_STATE_LEN = 6
TERM_NONE = 0
TERM_SQRT = 1

EXPORTED = [
    "ocean_bse_create", "ocean_bse_destroy", "ocean_bse_dim", "ocean_bse_apply", "ocean_haydock",
    "ocean_spectrum", "ocean_multiplet_matrices", "ocean_multiplet_matrices_spin",
    "ocean_dipole_amplitudes", "ocean_dipole_psi0",
    "ocean_bse_set_profiling", "ocean_bse_kernel_times", "ocean_bse_device_bytes",
    "ocean_last_error", "ocean_haydock_batch", "ocean_bse_autotune", "ocean_bse_get_tuning",
    "ocean_mlp_param_count", "ocean_mlp_create", "ocean_mlp_destroy", "ocean_mlp_set_params",
    "ocean_mlp_get_params", "ocean_mlp_encode", "ocean_mlp_forward", "ocean_mlp_loss_grad",
    "ocean_mlp_train_step", "ocean_mlp_predict", "ocean_mlp_save", "ocean_mlp_load",
    "ocean_device_ceilings", "ocean_screening_chi0", "ocean_screening_release", "ocean_local_matrix_channels",
    "ocean_dipole_amplitudes_channels", "ocean_dipole_psi0_channels", "ocean_nrixs_amplitudes_channels",
    "ocean_quadrupole_amplitudes_channels", "ocean_psi0_amplitudes", "ocean_haydock_export",
    "ocean_haydock_continue", "ocean_mlp_predict_noalloc", "ocean_mlp_set_loss_weights",
]
MLP_BF16 = 0
MLP_FP32 = 1
MLP_NOALLOC_MAX_SEQ = 4096      # OCEAN_MLP_NOALLOC_MAX_SEQ


def cell_matrix(cell) -> np.ndarray:
    """Lattice vectors as the rows of a 3x3 array (bohr) from an edge length (cubic cell),
    three edge lengths (orthorhombic) or the 3x3 rows themselves."""
    c = np.asarray(cell, dtype=np.float64)
    if c.ndim == 0:
        return float(c) * np.eye(3)
    if c.shape == (3,):
        return np.diag(c)
    if c.shape == (3, 3):
        return c.copy()
    raise ValueError("cell: an edge length, three edge lengths or a 3x3 array of lattice vectors")


class OceanError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class Desc(ctypes.Structure):
    _fields_ = [
        ("nk", ctypes.c_int * 3), ("nx", ctypes.c_int * 3), ("n_bands", ctypes.c_int),
        ("n_core", ctypes.c_int), ("n_local", ctypes.c_int), ("cell", (ctypes.c_double * 3) * 3),
        ("tau", ctypes.c_double * 3), ("energies", ctypes.c_void_p), ("u", ctypes.c_void_p),
        ("n_wr", ctypes.c_int), ("w_r", ctypes.c_void_p), ("w_val", ctypes.c_void_p),
        ("local_proj", ctypes.c_void_p), ("local_mat", ctypes.c_void_p),
        ("core_mat", ctypes.c_void_p), ("precision", ctypes.c_int), ("flags", ctypes.c_uint),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(hipcc --offload-arch=gfx950); there is no CPU fallback")
    # torch holds the device memory the kernels read, through the HIP runtime it ships with; that
    # runtime has to see the GPU before the library's own runtime opens it, so it is started here
    # first (a process whose first GPU call came from the library found no GPU in torch)
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp, ci, cd, cu = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_uint
    ll = ctypes.c_longlong
    L.ocean_bse_create.argtypes = [ctypes.POINTER(Desc), vp, ctypes.POINTER(vp)]
    L.ocean_bse_create.restype = ci
    L.ocean_bse_destroy.argtypes = [vp]
    L.ocean_bse_destroy.restype = None
    L.ocean_bse_dim.argtypes = [vp]
    L.ocean_bse_dim.restype = ll
    L.ocean_bse_device_bytes.argtypes = [vp]
    L.ocean_bse_device_bytes.restype = ll
    L.ocean_device_ceilings.argtypes = [ll] + [ctypes.POINTER(ctypes.c_double)] * 4
    L.ocean_device_ceilings.restype = ci
    L.ocean_screening_chi0.argtypes = [vp, vp, ci, ci, cd, vp, vp, ci, vp, vp]
    L.ocean_screening_chi0.restype = ci
    L.ocean_screening_release.argtypes = []
    L.ocean_screening_release.restype = ci
    L.ocean_bse_apply.argtypes = [vp, vp, vp, ci]
    L.ocean_bse_apply.restype = ci
    L.ocean_haydock.argtypes = [vp, vp, ci, ci, cu, vp, vp, vp, vp]
    L.ocean_haydock.restype = ci
    L.ocean_spectrum.argtypes = [vp, vp, vp, vp, ci, ci, ci, vp, vp, vp, ci, cd, vp]
    L.ocean_spectrum.restype = ci
    L.ocean_multiplet_matrices.argtypes = [cd, cd, cd, cd, vp, vp]
    L.ocean_multiplet_matrices.restype = ci
    L.ocean_multiplet_matrices_spin.argtypes = [cd, cd, cd, cd, vp, vp]
    L.ocean_multiplet_matrices_spin.restype = ci
    L.ocean_local_matrix_channels.argtypes = [ci, vp, vp, vp, ci, vp]
    L.ocean_local_matrix_channels.restype = ci
    L.ocean_dipole_amplitudes_channels.argtypes = [ci, vp, vp, vp, vp]
    L.ocean_dipole_amplitudes_channels.restype = ci
    L.ocean_dipole_psi0_channels.argtypes = [vp, ci, vp, vp, vp, ci, vp]
    L.ocean_dipole_psi0_channels.restype = ci
    L.ocean_nrixs_amplitudes_channels.argtypes = [ci, vp, ci, vp, vp, vp]
    L.ocean_nrixs_amplitudes_channels.restype = ci
    L.ocean_quadrupole_amplitudes_channels.argtypes = [ci, vp, vp, vp, vp, vp, vp]
    L.ocean_quadrupole_amplitudes_channels.restype = ci
    L.ocean_psi0_amplitudes.argtypes = [vp, vp, ci, vp]
    L.ocean_psi0_amplitudes.restype = ci
    L.ocean_haydock_export.argtypes = [vp, ci, vp, vp, vp]
    L.ocean_haydock_export.restype = ci
    L.ocean_haydock_continue.argtypes = [vp, vp, vp, vp, ci, ci, ctypes.c_uint, vp, vp, vp]
    L.ocean_haydock_continue.restype = ci
    L.ocean_dipole_amplitudes.argtypes = [vp, vp]
    L.ocean_dipole_amplitudes.restype = ci
    L.ocean_dipole_psi0.argtypes = [vp, vp, ci, vp]
    L.ocean_dipole_psi0.restype = ci
    L.ocean_bse_set_profiling.argtypes = [vp, ci]
    L.ocean_bse_set_profiling.restype = ci
    L.ocean_bse_kernel_times.argtypes = [vp, vp, vp, vp, ci]
    L.ocean_bse_kernel_times.restype = ci
    L.ocean_haydock_batch.argtypes = [vp, ci, vp, vp, ci, cu, vp, vp, vp, vp]
    L.ocean_haydock_batch.restype = ci
    L.ocean_bse_autotune.argtypes = [vp, ci, ci]
    L.ocean_bse_autotune.restype = ci
    L.ocean_bse_get_tuning.argtypes = [vp, vp, vp, vp, vp, vp]
    L.ocean_bse_get_tuning.restype = ci
    L.ocean_mlp_param_count.argtypes = []
    L.ocean_mlp_param_count.restype = ci
    L.ocean_mlp_create.argtypes = [ci, ctypes.POINTER(vp)]
    L.ocean_mlp_create.restype = ci
    L.ocean_mlp_destroy.argtypes = [vp]
    L.ocean_mlp_destroy.restype = None
    L.ocean_mlp_set_params.argtypes = [vp, vp]
    L.ocean_mlp_set_params.restype = ci
    L.ocean_mlp_get_params.argtypes = [vp, vp]
    L.ocean_mlp_get_params.restype = ci
    L.ocean_mlp_encode.argtypes = [vp, vp, ci, ci, vp, vp]
    L.ocean_mlp_encode.restype = ci
    L.ocean_mlp_forward.argtypes = [vp, vp, ci, vp]
    L.ocean_mlp_forward.restype = ci
    L.ocean_mlp_loss_grad.argtypes = [vp, vp, vp, ci, vp, vp]
    L.ocean_mlp_loss_grad.restype = ci
    L.ocean_mlp_train_step.argtypes = [vp, vp, vp, ci, ctypes.c_float, vp]
    L.ocean_mlp_train_step.restype = ci
    L.ocean_mlp_predict.argtypes = [vp, vp, vp, ci, ci, vp, vp, vp]
    L.ocean_mlp_predict.restype = ci
    L.ocean_mlp_predict_noalloc.argtypes = [vp, vp, vp, ci, ci, vp, vp, vp, vp]
    L.ocean_mlp_predict_noalloc.restype = ci
    L.ocean_mlp_set_loss_weights.argtypes = [vp, vp]
    L.ocean_mlp_set_loss_weights.restype = ci
    L.ocean_mlp_save.argtypes = [vp, ctypes.c_char_p]
    L.ocean_mlp_save.restype = ci
    L.ocean_mlp_load.argtypes = [vp, ctypes.c_char_p]
    L.ocean_mlp_load.restype = ci
    L.ocean_last_error.argtypes = []
    L.ocean_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(rc: int, allow_info: bool = False) -> int:
    if rc < 0 or (rc > 0 and not allow_info):
        raise OceanError(rc, lib().ocean_last_error().decode())
    return rc


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _host_c128(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


def _host_f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _device_sync():
    """The library enqueues on its own stream: order it against torch's work."""
    import torch
    torch.cuda.synchronize()


def _dev_ptr(t) -> int:
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous CUDA tensor")
    if t.dtype != torch.complex128:
        raise ValueError("exciton vectors are torch.complex128")
    return t.data_ptr()


def multiplet_matrices(zeta: float, f2: float, g1: float, g3: float, full_spin: bool = False):
    """L2,3-edge core matrix and local interaction matrix, Ha: 6x6 and 30x30 with the
    electron spin tied to the hole's, or 12x12 and 60x60 with it carried separately."""
    nc = 12 if full_spin else 6
    core = np.zeros((nc, nc), dtype=np.complex128)
    loc = np.zeros((5 * nc, 5 * nc), dtype=np.complex128)
    fn = lib().ocean_multiplet_matrices_spin if full_spin else lib().ocean_multiplet_matrices
    _check(fn(zeta, f2, g1, g3, _ptr(core), _ptr(loc)))
    return core, loc


def _gk_array(gk, n):
    """G^k tables as a [5, n, n] array (from a dict k -> [n, n] or an array)."""
    if isinstance(gk, dict):
        out = np.zeros((5, n, n))
        for k, g in gk.items():
            out[int(k)] = np.asarray(g, dtype=np.float64)
        return out
    return np.ascontiguousarray(np.asarray(gk, dtype=np.float64).reshape(5, n, n))


def local_matrix_channels(ls, f2, gk, full_spin: bool = False) -> np.ndarray:
    """Short-range matrix of a general local basis (ocean_local_matrix_channels): channels of
    angular momentum ls, direct F^2 table f2 [n, n], exchange G^k tables gk ({k: [n, n]} or
    [5, n, n]); restricted (6 core states) or full spin (12)."""
    la = np.ascontiguousarray(np.asarray(ls, dtype=np.int32))
    n = len(la)
    f = _host_f64(np.asarray(f2, dtype=np.float64).reshape(n, n))
    g = _gk_array(gk, n)
    nmu = int(np.sum(2 * la + 1))
    npair = (12 if full_spin else 6) * nmu
    out = np.zeros((npair, npair), dtype=np.complex128)
    _check(lib().ocean_local_matrix_channels(n, la.ctypes.data_as(ctypes.c_void_p), _ptr(f), _ptr(g),
                                             int(bool(full_spin)), _ptr(out)))
    return out


def dipole_amplitudes_channels(ls, radial, pol) -> np.ndarray:
    la = np.ascontiguousarray(np.asarray(ls, dtype=np.int32))
    r = _host_f64(radial)
    e = _host_f64(pol)
    d = np.zeros((int(np.sum(2 * la + 1)), 3), dtype=np.complex128)
    _check(lib().ocean_dipole_amplitudes_channels(len(la), la.ctypes.data_as(ctypes.c_void_p), _ptr(r), _ptr(e),
                                                  _ptr(d)))
    return d


def nrixs_amplitudes_channels(ls, radial, q) -> np.ndarray:
    """e^{iq.r} amplitudes [N_mu][3]; radial[i][L] = channel i's j_L radial integral."""
    la = np.ascontiguousarray(np.asarray(ls, dtype=np.int32))
    r = _host_f64(np.atleast_2d(radial))
    qv = _host_f64(q)
    d = np.zeros((int(np.sum(2 * la + 1)), 3), dtype=np.complex128)
    _check(lib().ocean_nrixs_amplitudes_channels(len(la), la.ctypes.data_as(ctypes.c_void_p), r.shape[1], _ptr(r),
                                                 _ptr(qv), _ptr(d)))
    return d


def quadrupole_amplitudes_channels(ls, radial1, radial2, pol, q) -> np.ndarray:
    """e.r + (i/2)(e.r)(q.r) amplitudes [N_mu][3]."""
    la = np.ascontiguousarray(np.asarray(ls, dtype=np.int32))
    r1, r2, e, qv = _host_f64(radial1), _host_f64(radial2), _host_f64(pol), _host_f64(q)
    d = np.zeros((int(np.sum(2 * la + 1)), 3), dtype=np.complex128)
    _check(lib().ocean_quadrupole_amplitudes_channels(len(la), la.ctypes.data_as(ctypes.c_void_p), _ptr(r1),
                                                      _ptr(r2), _ptr(e), _ptr(qv), _ptr(d)))
    return d


def dipole_amplitudes(pol) -> np.ndarray:
    e = _host_f64(pol)
    d = np.zeros((5, 3), dtype=np.complex128)
    _check(lib().ocean_dipole_amplitudes(_ptr(e), _ptr(d)))
    return d


def device_ceilings(copy_bytes: int = 1 << 30) -> dict:
    """Measured FP64 matrix-core and multiply-add rates (TFLOP/s) and the streaming rates of a
    plain copy (GB/s, read + written) and a plain read on the current device
    (ocean_device_ceilings)."""
    m, f, c, r = (ctypes.c_double() for _ in range(4))
    _check(lib().ocean_device_ceilings(int(copy_bytes), ctypes.byref(m), ctypes.byref(f), ctypes.byref(c),
                                       ctypes.byref(r)))
    return {"mfma_f64_tflops": m.value, "fma_f64_tflops": f.value, "copy_GBs": c.value, "read_GBs": r.value}


def screening_chi0(psi, eps, mu: float, t, w, out=None):
    """Static RPA response chi0 [n_points, n_points] (real, device) from Bloch functions on
    the screening grid psi [n_points, n_states] (complex128, device), energies eps
    [n_states], chemical potential mu and imaginary-frequency nodes t / weights w
    (ocean_screening_chi0)."""
    import torch
    if psi.dtype != torch.complex128 or not psi.is_cuda or psi.dim() != 2 or not psi.is_contiguous():
        raise ValueError("psi must be a contiguous [n_points, n_states] complex128 CUDA tensor")
    npt, ns = psi.shape
    e = _host_f64(eps)
    tt, ww = _host_f64(t), _host_f64(w)
    if e.shape != (ns,) or tt.shape != ww.shape:
        raise ValueError("eps must have n_states entries and t, w the same length")
    if out is None:
        out = torch.empty((npt, npt), dtype=torch.float64, device=psi.device)
    if out.dtype != torch.float64 or not out.is_cuda or tuple(out.shape) != (npt, npt) or not out.is_contiguous():
        raise ValueError("out must be a contiguous [n_points, n_points] float64 CUDA tensor")
    _device_sync()
    _check(lib().ocean_screening_chi0(_dev_ptr(psi), _ptr(e), npt, ns, float(mu), _ptr(tt), _ptr(ww), len(tt),
                                      ctypes.c_void_p(out.data_ptr()), None))
    return out


def screening_release():
    """Free the device scratch the response build keeps between calls
    (ocean_screening_release)."""
    _check(lib().ocean_screening_release())


def spectrum(a, b, norm2, omega, gamma: float, terminator: str = "none", n_used=None, a_inf=None,
             b_inf=None) -> np.ndarray:
    """Continued-fraction spectra on the GPU.  a, b: [n_spec, n_steps]; norm2: [n_spec].
    With terminator "sqrt", a_inf and b_inf ([n_spec] each, or None for the means of the
    last 16 used coefficients) are the constant chain's coefficients."""
    a = _host_f64(np.atleast_2d(a))
    b = _host_f64(np.atleast_2d(b))
    n2 = _host_f64(np.atleast_1d(norm2))
    om = _host_f64(omega)
    n_spec, n_steps = a.shape
    used = None if n_used is None else np.ascontiguousarray(np.atleast_1d(n_used), dtype=np.int32)
    ai = None if a_inf is None else _host_f64(np.broadcast_to(np.asarray(a_inf, dtype=np.float64), (n_spec,)))
    bi = None if b_inf is None else _host_f64(np.broadcast_to(np.asarray(b_inf, dtype=np.float64), (n_spec,)))
    sig = np.zeros((n_spec, len(om)))
    term = {"none": TERM_NONE, "sqrt": TERM_SQRT}[terminator]
    _check(lib().ocean_spectrum(_ptr(a), _ptr(b), _ptr(used), _ptr(n2), n_spec, n_steps, term, _ptr(ai), _ptr(bi),
                                _ptr(om), len(om), float(gamma), _ptr(sig)))
    return sig


def haydock_batch(systems, psi0s, n_steps: int, reorth: bool = False):
    """Batched recursion over independent handles (one HIP graph per step).
    systems: list of Bse; psi0s: matching list of device tensors [n_vec, Nk, Nb, Nc].
    Returns a list of (a, b, norm2, steps_done) per system and the return code."""
    n = len(systems)
    if n < 1 or len(psi0s) != n:
        raise ValueError("need one psi0 per system")
    nvs = []
    for h, p in zip(systems, psi0s):
        nv = p.numel() // h.dim
        if nv * h.dim != p.numel() or nv < 1:
            raise ValueError("psi0 size is not a multiple of the vector dimension")
        nvs.append(nv)
    tot = sum(nvs)
    hs = (ctypes.c_void_p * n)(*[h._h.value for h in systems])
    ps = (ctypes.c_void_p * n)(*[_dev_ptr(p) for p in psi0s])
    nv_arr = (ctypes.c_int * n)(*nvs)
    a = np.zeros((tot, n_steps))
    b = np.zeros((tot, n_steps))
    n2 = np.zeros(tot)
    sd = np.zeros(tot, dtype=np.int32)
    _device_sync()
    rc = lib().ocean_haydock_batch(hs, n, ps, nv_arr, int(n_steps), HAYDOCK_REORTH if reorth else 0,
                                   _ptr(a), _ptr(b), _ptr(n2), _ptr(sd))
    _check(rc, allow_info=True)
    out, off = [], 0
    for nv in nvs:
        out.append((a[off:off + nv], b[off:off + nv], n2[off:off + nv], sd[off:off + nv]))
        off += nv
    return out, rc


class Bse:
    """One solver handle (ocean_bse_create ... ocean_bse_destroy)."""

    def __init__(self, *, nk, nx, cell, tau, energies, u, w_r, w_val, n_core: int,
                 local_proj=None, local_mat=None, core_mat=None, precision: str = "fp64",
                 check_inputs: bool = False, stream=None):
        import torch
        nk = tuple(int(v) for v in nk)
        nx = tuple(int(v) for v in nx)
        cell = cell_matrix(cell)
        self._keep = []
        e = _host_f64(energies)
        n_bands = e.shape[-1]
        flags = FLAG_CHECK_INPUTS if check_inputs else 0
        if isinstance(u, torch.Tensor):
            if not u.is_cuda:
                u = u.numpy()
            else:
                flags |= FLAG_BORROW_DEVICE_U
        if isinstance(u, np.ndarray) or not isinstance(u, torch.Tensor):
            uh = _host_c128(u)
            uptr = _ptr(uh)
            self._keep.append(uh)
        else:
            if u.dtype != torch.complex128 or not u.is_contiguous():
                raise ValueError("device u must be a contiguous complex128 tensor")
            uptr = ctypes.c_void_p(u.data_ptr())
            self._u_dev = u
        wr, wv = _host_f64(w_r), _host_f64(w_val)
        lp = None if local_proj is None else _host_c128(local_proj)
        lm = None if local_mat is None else _host_c128(local_mat)
        cm = None if core_mat is None else _host_c128(core_mat)
        d = Desc()
        d.nk[:] = nk
        d.nx[:] = nx
        d.n_bands = n_bands
        d.n_core = int(n_core)
        d.n_local = 0 if lp is None else lp.shape[-1]
        for a in range(3):
            d.cell[a][:] = [float(v) for v in cell[a]]
        d.tau[:] = [float(v) for v in np.asarray(tau, dtype=np.float64)]
        d.energies = _ptr(e)
        d.u = uptr
        d.n_wr = len(wr)
        d.w_r, d.w_val = _ptr(wr), _ptr(wv)
        d.local_proj, d.local_mat, d.core_mat = _ptr(lp), _ptr(lm), _ptr(cm)
        d.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        d.flags = flags
        h = ctypes.c_void_p()
        st = None if stream is None else ctypes.c_void_p(stream)
        if flags & FLAG_BORROW_DEVICE_U:
            _device_sync()
        _check(lib().ocean_bse_create(ctypes.byref(d), st, ctypes.byref(h)))
        self._h = h
        self.nk, self.nx, self.n_bands, self.n_core = nk, nx, n_bands, int(n_core)
        self.n_k = int(np.prod(nk))
        self.dim = int(lib().ocean_bse_dim(h))
        self.precision = precision

    @classmethod
    def from_crystal(cls, cr, precision: str = "fp64", with_local: bool = True, u=None, **kw):
        """Convenience constructor from a synth.Crystal (inputs only; the multiplet
        matrices are built by this library's own helper)."""
        core_mat = local_mat = None
        lp = None
        if cr.multiplet is not None:
            m = cr.multiplet
            core_mat, local_mat = multiplet_matrices(m["zeta"], m["F2"], m["G1"], m["G3"],
                                                     full_spin=cr.n_core == 12)
            if getattr(cr, "channels", None) is not None:
                ch = cr.channels
                local_mat = local_matrix_channels(ch["l"], ch["f2"], ch["gk"], full_spin=cr.n_core == 12)
            if with_local and cr.local_proj is not None:
                lp = cr.local_proj
            else:
                local_mat = None
        return cls(nk=cr.nk, nx=cr.nx, cell=cr.cell_vectors(), tau=cr.tau, energies=cr.energies,
                   u=cr.u if u is None else u, w_r=cr.w_r, w_val=cr.w_val, n_core=cr.n_core,
                   local_proj=lp, local_mat=local_mat, core_mat=core_mat, precision=precision, **kw)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ocean_bse_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def apply(self, x, y=None, sync: bool = True):
        """y = H x for x of shape [n_vec, Nk, Nb, Nc] (or [Nk, Nb, Nc]) complex128 on the GPU.
        With sync=False the caller orders the library's stream (e.g. torch.cuda.synchronize())."""
        import torch
        nv = x.numel() // self.dim
        if nv * self.dim != x.numel() or nv < 1:
            raise ValueError("x size is not a multiple of the vector dimension")
        if y is None:
            y = torch.empty_like(x)
        if sync:
            _device_sync()
        _check(lib().ocean_bse_apply(self._h, _dev_ptr(x), _dev_ptr(y), nv))
        if sync:
            _device_sync()
        return y

    def haydock(self, psi0, n_steps: int, reorth: bool = False):
        """Run the recursion; returns (a [nv, N], b [nv, N], norm2 [nv], steps_done [nv], rc)."""
        nv = psi0.numel() // self.dim
        if nv * self.dim != psi0.numel() or nv < 1:
            raise ValueError("psi0 size is not a multiple of the vector dimension")
        a = np.zeros((nv, n_steps))
        b = np.zeros((nv, n_steps))
        n2 = np.zeros(nv)
        sd = np.zeros(nv, dtype=np.int32)
        _device_sync()
        rc = lib().ocean_haydock(self._h, _dev_ptr(psi0), nv, int(n_steps),
                                 HAYDOCK_REORTH if reorth else 0, _ptr(a), _ptr(b), _ptr(n2), _ptr(sd))
        _check(rc, allow_info=True)
        return a, b, n2, sd, rc

    def dipole_psi0_channels(self, ls, radial, pols):
        """Dipole start vectors for a general local basis (ocean_dipole_psi0_channels)."""
        import torch
        la = np.ascontiguousarray(np.asarray(ls, dtype=np.int32))
        r = _host_f64(radial)
        p = _host_f64(np.atleast_2d(pols))
        out = torch.empty((p.shape[0], self.n_k, self.n_bands, self.n_core), dtype=torch.complex128,
                          device="cuda")
        _device_sync()
        _check(lib().ocean_dipole_psi0_channels(self._h, len(la), la.ctypes.data_as(ctypes.c_void_p), _ptr(r),
                                                _ptr(p), p.shape[0], _dev_ptr(out)))
        return out

    def haydock_export(self, n_vec: int):
        """State of the last recursion on this handle: (v, vprev) device tensors
        [n_vec, Nk, Nb, Nc] and the host state [n_vec, 6] (ocean_haydock_export)."""
        import torch
        shape = (n_vec, self.n_k, self.n_bands, self.n_core)
        v = torch.empty(shape, dtype=torch.complex128, device="cuda")
        vp = torch.empty(shape, dtype=torch.complex128, device="cuda")
        st = np.zeros((n_vec, HAYDOCK_STATE_LEN))
        _device_sync()
        _check(lib().ocean_haydock_export(self._h, n_vec, _dev_ptr(v), _dev_ptr(vp), _ptr(st)))
        return v, vp, st

    def haydock_continue(self, v, vprev, state, n_steps: int):
        """n_steps more steps from an exported state; returns (a, b, steps_done, rc)."""
        st = np.ascontiguousarray(np.asarray(state, dtype=np.float64))
        nv = st.shape[0]
        if v.numel() != nv * self.dim or vprev.numel() != nv * self.dim:
            raise ValueError("vectors do not match the state's vector count")
        a = np.zeros((nv, n_steps))
        b = np.zeros((nv, n_steps))
        sd = np.zeros(nv, dtype=np.int32)
        _device_sync()
        rc = lib().ocean_haydock_continue(self._h, _dev_ptr(v), _dev_ptr(vprev), _ptr(st), nv, int(n_steps), 0,
                                          _ptr(a), _ptr(b), _ptr(sd))
        _check(rc, allow_info=True)
        return a, b, sd, rc

    def psi0_amplitudes(self, d):
        """Start vectors from local amplitudes d[n_pol][N_mu][3] (ocean_psi0_amplitudes)."""
        import torch
        dd = np.ascontiguousarray(np.asarray(d, dtype=np.complex128))
        if dd.ndim == 2:
            dd = dd[None]
        out = torch.empty((dd.shape[0], self.n_k, self.n_bands, self.n_core), dtype=torch.complex128,
                          device="cuda")
        _device_sync()
        _check(lib().ocean_psi0_amplitudes(self._h, _ptr(dd), dd.shape[0], _dev_ptr(out)))
        return out

    def dipole_psi0(self, pols):
        import torch
        p = _host_f64(np.atleast_2d(pols))
        out = torch.empty((p.shape[0], self.n_k, self.n_bands, self.n_core), dtype=torch.complex128,
                          device="cuda")
        _device_sync()
        _check(lib().ocean_dipole_psi0(self._h, _ptr(p), p.shape[0], _dev_ptr(out)))
        return out

    def autotune(self, n_vec: int, reps: int = 5):
        _device_sync()
        _check(lib().ocean_bse_autotune(self._h, int(n_vec), int(reps)))
        return self.tuning

    @property
    def tuning(self):
        m, b, f, t, w = (ctypes.c_int() for _ in range(5))
        _check(lib().ocean_bse_get_tuning(self._h, ctypes.byref(m), ctypes.byref(b), ctypes.byref(f),
                                          ctypes.byref(t), ctypes.byref(w)))
        return {"fwd_ms": m.value, "bwd_blocks": b.value, "fft_lines": f.value, "fwd_tiles": t.value,
                "bwd_waves": w.value}

    def set_profiling(self, on: bool):
        _check(lib().ocean_bse_set_profiling(self._h, 1 if on else 0))

    def kernel_times(self) -> dict:
        n = lib().ocean_bse_kernel_times(self._h, None, None, None, 0)
        _check(min(n, 0))
        names = (ctypes.c_char_p * max(n, 1))()
        ms = np.zeros(max(n, 1))
        cnt = np.zeros(max(n, 1), dtype=np.int64)
        lib().ocean_bse_kernel_times(self._h, names, _ptr(ms), _ptr(cnt), n)
        return {names[i].decode(): (float(ms[i]), int(cnt[i])) for i in range(n)}

    @property
    def device_bytes(self) -> int:
        return int(lib().ocean_bse_device_bytes(self._h))


class Mlp:
    """Learned terminator network (ocean_mlp_*).  Device arrays are torch.float32 tensors."""

    def __init__(self, precision: str = "bf16"):
        h = ctypes.c_void_p()
        _check(lib().ocean_mlp_create(MLP_BF16 if precision == "bf16" else MLP_FP32, ctypes.byref(h)))
        self._h = h
        self.n_params = int(lib().ocean_mlp_param_count())

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ocean_mlp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _f32(t):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
            raise ValueError("expected a contiguous float32 CUDA tensor")
        return t.data_ptr()

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        if p.size != self.n_params:
            raise ValueError("wrong parameter count")
        _check(lib().ocean_mlp_set_params(self._h, _ptr(p)))

    def set_loss_weights(self, w):
        """Per-output weights [448] of the training loss, or None for unit weights."""
        if w is None:
            _check(lib().ocean_mlp_set_loss_weights(self._h, None))
            return
        w = np.ascontiguousarray(w, dtype=np.float32)
        if w.size != 448:
            raise ValueError("448 loss weights expected")
        _check(lib().ocean_mlp_set_loss_weights(self._h, _ptr(w)))

    def get_params(self):
        p = np.zeros(self.n_params, dtype=np.float32)
        _check(lib().ocean_mlp_get_params(self._h, _ptr(p)))
        return p

    def save(self, path):
        """Checkpoint parameters, Adam moments and step count (ocean_mlp_save)."""
        _check(lib().ocean_mlp_save(self._h, os.fsencode(path)))

    def load(self, path):
        """Restore a checkpoint written by save (ocean_mlp_load)."""
        _check(lib().ocean_mlp_load(self._h, os.fsencode(path)))

    @staticmethod
    def encode(a_dev, b_dev, with_targets: bool = True):
        """Features (and targets) from device FP64 coefficient arrays [n_seq, stride]."""
        import torch
        n, stride = a_dev.shape
        for t in (a_dev, b_dev):
            if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
                raise ValueError("expected contiguous float64 CUDA tensors")
        x = torch.empty((n, 64), dtype=torch.float32, device="cuda")
        t = torch.empty((n, 448), dtype=torch.float32, device="cuda") if with_targets else None
        _device_sync()
        _check(lib().ocean_mlp_encode(a_dev.data_ptr(), b_dev.data_ptr(), n, stride, x.data_ptr(),
                                      None if t is None else t.data_ptr()))
        return x, t

    def forward(self, x):
        import torch
        y = torch.empty((x.shape[0], 448), dtype=torch.float32, device="cuda")
        _device_sync()
        _check(lib().ocean_mlp_forward(self._h, self._f32(x), x.shape[0], self._f32(y)))
        return y

    def loss_grad(self, x, t):
        loss = ctypes.c_double()
        g = np.zeros(self.n_params, dtype=np.float32)
        _device_sync()
        _check(lib().ocean_mlp_loss_grad(self._h, self._f32(x), self._f32(t), x.shape[0], ctypes.byref(loss), _ptr(g)))
        return loss.value, g

    def train_step(self, x, t, lr: float, want_loss: bool = False):
        """One Adam step on device batch (x, t).  Without want_loss the call returns with the
        step still queued on the network's stream, which reads x and t: keep them alive until
        the device has been synchronised."""
        loss = ctypes.c_double()
        _check(lib().ocean_mlp_train_step(self._h, self._f32(x), self._f32(t), x.shape[0], float(lr),
                                          ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def predict(self, a, b):
        """Extended (a, b) [n, 256] from host arrays a, b [n, >=32]; valid flags [n]."""
        a = _host_f64(np.atleast_2d(a))
        b = _host_f64(np.atleast_2d(b))
        n, stride = a.shape
        ae = np.zeros((n, 256))
        be = np.zeros((n, 256))
        valid = np.zeros(n, dtype=np.int32)
        _check(lib().ocean_mlp_predict(self._h, _ptr(a), _ptr(b), n, stride, _ptr(ae), _ptr(be), _ptr(valid)))
        return ae, be, valid.astype(bool)

    def predict_noalloc(self, a_dev, b_dev, a_ext_dev, b_ext_dev, valid_dev, stream=None):
        """ocean_mlp_predict_noalloc on caller-owned device tensors: a_dev, b_dev float64
        [n, stride >= 32]; outputs a_ext_dev, b_ext_dev float64 [n, 256] and valid_dev int32 [n].
        Enqueued on `stream` (a torch.cuda.Stream, or None for the default stream)."""
        import torch
        n, stride = a_dev.shape
        for t, shape, dt in ((a_dev, (n, stride), torch.float64), (b_dev, (n, stride), torch.float64),
                             (a_ext_dev, (n, 256), torch.float64), (b_ext_dev, (n, 256), torch.float64),
                             (valid_dev, (n,), torch.int32)):
            if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dt or not t.is_contiguous() \
                    or tuple(t.shape) != shape:
                raise ValueError(f"expected a contiguous {dt} CUDA tensor of shape {shape}")
        st = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
        _check(lib().ocean_mlp_predict_noalloc(self._h, a_dev.data_ptr(), b_dev.data_ptr(), n, stride,
                                               a_ext_dev.data_ptr(), b_ext_dev.data_ptr(), valid_dev.data_ptr(), st))
