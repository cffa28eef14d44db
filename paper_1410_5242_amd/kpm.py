"""Thin ctypes binding of libkpm.so (include/kpm.h).

Argument marshalling only: every step of the KPM path runs in the library's
HIP kernels.  PyTorch supplies device memory (tensors) and the HIP stream.
The binding refuses to run when the compiled library is missing; there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkpm.so")

KPM_OK, KPM_EINVAL, KPM_ENOMEM, KPM_EDEVICE, KPM_ENOTSUP, KPM_ESPECTRUM, KPM_EINTERNAL = 0, -1, -2, -3, -4, -5, -6
C128, C64 = 0, 1
JACKSON, DIRICHLET, LORENTZ = 0, 1, 2
FULL, NODOT, PLAIN = 0, 1, 2
SUPPORTED_R = (1, 2, 4, 8, 16, 32, 64)

_KERNELS = {"jackson": JACKSON, "dirichlet": DIRICHLET, "lorentz": LORENTZ}
_VARIANTS = {"full": FULL, "nodot": NODOT, "plain": PLAIN}
_DTYPES = {"c128": C128, "c64": C64}
_TORCH_DTYPE = {C128: torch.complex128, C64: torch.complex64}


class KPMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"kpm status {status}: {msg}")
        self.status = status


class SweepTuning(ctypes.Structure):
    _fields_ = [("wg_per_cu", ctypes.c_int32), ("xcd_ways", ctypes.c_int32), ("chunk_tiles", ctypes.c_int32),
                ("pencil", ctypes.c_int32), ("dynamic", ctypes.c_int32), ("prefetch", ctypes.c_int32),
                ("stream", ctypes.c_int32), ("lattice", ctypes.c_int32), ("gather", ctypes.c_int32),
                ("tile_order", ctypes.c_int32), ("slab", ctypes.c_int32), ("gather_tile", ctypes.c_int32)]


class BatchTuning(ctypes.Structure):
    _fields_ = [("waves", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32), ("dynamic", ctypes.c_int32),
                ("slab", ctypes.c_int32)]


BATCH_CHECK, BATCH_GRAPH = 1, 2


class LatticeDesc(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32 * 3),
        ("periodic", ctypes.c_int32 * 3),
        ("t", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("potential", ctypes.c_void_p),
        ("dtype", ctypes.c_int32),
        ("margin", ctypes.c_double),
        ("fixed_scale", ctypes.c_int32),
        ("a", ctypes.c_double),
        ("b", ctypes.c_double),
        ("sell_C", ctypes.c_int32),
        ("sell_sigma", ctypes.c_int32),
    ]


class CsrDesc(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int64),
        ("rowptr", ctypes.c_void_p),
        ("col", ctypes.c_void_p),
        ("val", ctypes.c_void_p),
        ("dtype", ctypes.c_int32),
        ("sell_C", ctypes.c_int32),
        ("sell_sigma", ctypes.c_int32),
        ("margin", ctypes.c_double),
        ("fixed_scale", ctypes.c_int32),
        ("a", ctypes.c_double),
        ("b", ctypes.c_double),
    ]


class RunOpts(ctypes.Structure):
    _fields_ = [("check", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("mu_on_host", ctypes.c_int32), ("tuning", ctypes.POINTER(SweepTuning)),
                ("eta_out", ctypes.c_void_p), ("group", ctypes.c_int32)]


class SweepPlan(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("grid", ctypes.c_int32), ("tile_order", ctypes.c_int32),
                ("pieces", ctypes.c_int32), ("halves", ctypes.c_int32), ("group", ctypes.c_int32)]


_LIB = None
EXPORTS = ("kpm_build_hamiltonian", "kpm_hamiltonian_info", "kpm_export_csr",
           "kpm_destroy_hamiltonian", "kpm_aug_spmmv", "kpm_moments", "kpm_dos",
           "kpm_set_sweep_tuning", "kpm_get_sweep_tuning", "kpm_sweep_kernel", "kpm_sweep_plan", "kpm_sweep_profile_enable", "kpm_sweep_profile_read", "kpm_moments_batched",
           "kpm_set_batch_tuning", "kpm_get_batch_tuning", "kpm_mlp_create", "kpm_mlp_destroy",
           "kpm_mlp_param_count", "kpm_mlp_set_params", "kpm_mlp_get_params", "kpm_mlp_get_grads",
           "kpm_mlp_forward", "kpm_mlp_backward", "kpm_mlp_adam_step", "kpm_mlp_train_step",
           "kpm_mlp_gemm_bf16", "kpm_dos_batched", "kpm_moment_features", "kpm_random_phase_block",
           "kpm_moments_naive", "kpm_axpy", "kpm_scal", "kpm_dot", "kpm_dot_noalloc", "kpm_site_block", "kpm_plane_wave_block",
           "kpm_lanczos_bounds", "kpm_set_scaling", "kpm_stream", "kpm_sell_layout", "kpm_import_csr", "kpm_sell_info",
           "kpm_last_error", "kpm_version")


def lib():
    """Load libkpm.so (built by __graft_entry__.build() / paper_1410_5242_amd.build)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1410_5242_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.kpm_build_hamiltonian.restype = ctypes.c_int
    L.kpm_build_hamiltonian.argtypes = [ctypes.POINTER(LatticeDesc), vp, ctypes.POINTER(vp)]
    L.kpm_hamiltonian_info.restype = ctypes.c_int
    L.kpm_hamiltonian_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i32),
                                       ctypes.POINTER(i32), ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                       ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
    L.kpm_export_csr.restype = ctypes.c_int
    L.kpm_export_csr.argtypes = [vp, vp, vp, vp]
    L.kpm_sell_layout.restype = ctypes.c_int
    L.kpm_sell_layout.argtypes = [i64, vp, i32, i32, vp, vp, vp]
    L.kpm_import_csr.restype = ctypes.c_int
    L.kpm_import_csr.argtypes = [ctypes.POINTER(CsrDesc), vp, ctypes.POINTER(vp)]
    L.kpm_sell_info.restype = ctypes.c_int
    L.kpm_sell_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i64),
                                ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.kpm_destroy_hamiltonian.restype = None
    L.kpm_destroy_hamiltonian.argtypes = [vp]
    L.kpm_aug_spmmv.restype = ctypes.c_int
    L.kpm_aug_spmmv.argtypes = [vp, vp, vp, i32, dbl, dbl, dbl, i32, vp, vp]
    L.kpm_moments.restype = ctypes.c_int
    L.kpm_moments.argtypes = [vp, vp, i32, i32, vp, ctypes.POINTER(RunOpts), vp]
    L.kpm_moments_naive.restype = ctypes.c_int
    L.kpm_moments_naive.argtypes = [vp, vp, i32, i32, vp, i32, vp]
    L.kpm_axpy.restype = ctypes.c_int
    L.kpm_axpy.argtypes = [i32, i64, dbl, vp, vp, vp]
    L.kpm_scal.restype = ctypes.c_int
    L.kpm_scal.argtypes = [i32, i64, dbl, vp, vp]
    L.kpm_dot.restype = ctypes.c_int
    L.kpm_dot.argtypes = [i32, i64, vp, vp, vp, vp]
    L.kpm_dot_noalloc.restype = ctypes.c_int
    L.kpm_dot_noalloc.argtypes = [i32, i64, vp, vp, vp, vp]
    L.kpm_dos.restype = ctypes.c_int
    L.kpm_dos.argtypes = [vp, i32, i32, i32, dbl, dbl, dbl, vp, i32, vp, vp]
    L.kpm_set_sweep_tuning.restype = ctypes.c_int
    L.kpm_set_sweep_tuning.argtypes = [ctypes.POINTER(SweepTuning)]
    L.kpm_get_sweep_tuning.restype = ctypes.c_int
    L.kpm_get_sweep_tuning.argtypes = [ctypes.POINTER(SweepTuning)]
    L.kpm_sweep_kernel.restype = ctypes.c_int
    L.kpm_sweep_kernel.argtypes = [vp, i32, ctypes.POINTER(i32)]
    L.kpm_sweep_plan.restype = ctypes.c_int
    L.kpm_sweep_plan.argtypes = [vp, i32, ctypes.POINTER(SweepTuning), ctypes.POINTER(SweepPlan)]
    L.kpm_sweep_profile_enable.restype = ctypes.c_int
    L.kpm_sweep_profile_enable.argtypes = [i32]
    L.kpm_sweep_profile_read.restype = ctypes.c_int
    L.kpm_sweep_profile_read.argtypes = [ctypes.POINTER(i64), ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                         ctypes.POINTER(dbl)]
    L.kpm_moments_batched.restype = ctypes.c_int
    L.kpm_moments_batched.argtypes = [vp, vp, i32, i32, i32, vp, i32, vp]
    L.kpm_set_batch_tuning.restype = ctypes.c_int
    L.kpm_set_batch_tuning.argtypes = [ctypes.POINTER(BatchTuning)]
    L.kpm_get_batch_tuning.restype = ctypes.c_int
    L.kpm_get_batch_tuning.argtypes = [ctypes.POINTER(BatchTuning)]
    flt = ctypes.c_float
    L.kpm_mlp_create.restype = ctypes.c_int
    L.kpm_mlp_create.argtypes = [i32, i32, i32, i32, ctypes.POINTER(vp)]
    L.kpm_mlp_destroy.restype = None
    L.kpm_mlp_destroy.argtypes = [vp]
    L.kpm_mlp_param_count.restype = ctypes.c_int
    L.kpm_mlp_param_count.argtypes = [vp, ctypes.POINTER(i64)]
    for name in ("kpm_mlp_set_params", "kpm_mlp_get_params", "kpm_mlp_get_grads"):
        getattr(L, name).restype = ctypes.c_int
        getattr(L, name).argtypes = [vp, vp]
    L.kpm_mlp_forward.restype = ctypes.c_int
    L.kpm_mlp_forward.argtypes = [vp, vp, i32, vp, vp, vp]
    L.kpm_mlp_backward.restype = ctypes.c_int
    L.kpm_mlp_backward.argtypes = [vp, vp, vp, vp, i32, flt, vp, vp]
    L.kpm_mlp_adam_step.restype = ctypes.c_int
    L.kpm_mlp_adam_step.argtypes = [vp, flt, flt, flt, flt, vp]
    L.kpm_mlp_train_step.restype = ctypes.c_int
    L.kpm_mlp_train_step.argtypes = [vp, vp, vp, vp, i32, flt, flt, vp, vp]
    L.kpm_mlp_gemm_bf16.restype = ctypes.c_int
    L.kpm_mlp_gemm_bf16.argtypes = [vp, vp, i32, i32, i32, i32, i32, vp, vp]
    L.kpm_dos_batched.restype = ctypes.c_int
    L.kpm_dos_batched.argtypes = [vp, i32, i32, i32, i32, i32, dbl, vp, vp, vp, i32, i32, vp, vp]
    L.kpm_moment_features.restype = ctypes.c_int
    L.kpm_moment_features.argtypes = [vp, i32, i32, i32, i32, vp, vp, vp]
    L.kpm_lanczos_bounds.restype = ctypes.c_int
    L.kpm_lanczos_bounds.argtypes = [vp, i32, ctypes.c_uint64, ctypes.POINTER(dbl), ctypes.POINTER(dbl), vp]
    L.kpm_set_scaling.restype = ctypes.c_int
    L.kpm_set_scaling.argtypes = [vp, dbl, dbl]
    L.kpm_site_block.restype = ctypes.c_int
    L.kpm_site_block.argtypes = [vp, i64, i32, vp, i32, vp]
    L.kpm_plane_wave_block.restype = ctypes.c_int
    L.kpm_plane_wave_block.argtypes = [vp, vp, i32, vp, vp, i32, vp]
    L.kpm_random_phase_block.restype = ctypes.c_int
    L.kpm_random_phase_block.argtypes = [vp, i64, i32, i32, ctypes.c_uint64, vp]
    L.kpm_stream.restype = ctypes.c_int
    L.kpm_stream.argtypes = [i32, vp, vp, vp, dbl, i64, i32, i32, vp]
    L.kpm_last_error.restype = ctypes.c_char_p
    L.kpm_last_error.argtypes = []
    L.kpm_version.restype = ctypes.c_char_p
    L.kpm_version.argtypes = []
    _LIB = L
    return L


def _check(status: int):
    if status != KPM_OK:
        raise KPMError(status, lib().kpm_last_error().decode())


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t: torch.Tensor) -> ctypes.c_void_p:
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


class Hamiltonian:
    """Owning wrapper of a kpm_hamiltonian handle."""

    def __init__(self, handle: ctypes.c_void_p):
        self.handle = handle
        N, nnz = ctypes.c_int64(), ctypes.c_int64()
        width, dtype = ctypes.c_int32(), ctypes.c_int32()
        a, b, lo, hi = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(lib().kpm_hamiltonian_info(handle, N, nnz, width, dtype, a, b, lo, hi))
        self.N, self.nnz_stored, self.width = N.value, nnz.value, width.value
        self.dtype = dtype.value
        self.a, self.b, self.emin, self.emax = a.value, b.value, lo.value, hi.value

    @property
    def torch_dtype(self):
        return _TORCH_DTYPE[self.dtype]

    def close(self):
        if self.handle:
            lib().kpm_destroy_hamiltonian(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_hamiltonian(L, potential=None, t: float = 1.0, periodic=(1, 1, 1), dtype: str = "c128",
                      margin: float = 1.01, fixed_scale=None, gamma: float = 0.0, seed: int = 0,
                      sell_C: int = 0, sell_sigma: int = 0, stream=None) -> Hamiltonian:
    """kpm_build_hamiltonian: H of eq. "Ham" on the device plus its Gershgorin scaling.

    `potential` is the host array of V_n; None draws V_n ~ U[-gamma/2, gamma/2) on the device
    from the library's counter generator keyed by `seed`.  sell_C > 0 stores the built matrix in
    SELL-C-sigma (chunk height sell_C, sorting window sell_sigma) instead of the lattice layout."""
    d = LatticeDesc()
    for j in range(3):
        d.L[j] = int(L[j])
        d.periodic[j] = 1 if periodic[j] else 0
    d.t = float(t)
    d.gamma = float(gamma)
    d.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    pot = None
    if potential is not None:
        pot = np.ascontiguousarray(potential, dtype=np.float64).reshape(-1)
        d.potential = pot.ctypes.data
    d.dtype = _DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
    d.margin = float(margin)
    if fixed_scale is not None:
        d.fixed_scale = 1
        d.a, d.b = float(fixed_scale[0]), float(fixed_scale[1])
    d.sell_C, d.sell_sigma = int(sell_C), int(sell_sigma)
    h = ctypes.c_void_p()
    _check(lib().kpm_build_hamiltonian(ctypes.byref(d), _stream(stream), ctypes.byref(h)))
    return Hamiltonian(h)


def export_csr(H: Hamiltonian):
    """kpm_export_csr: (rowptr int64, col int32, val complex128) on the host."""
    rowptr = np.zeros(H.N + 1, dtype=np.int64)
    _check(lib().kpm_export_csr(H.handle, rowptr.ctypes.data, None, None))
    nnz = int(rowptr[-1])
    col = np.zeros(nnz, dtype=np.int32)
    val = np.zeros(2 * nnz, dtype=np.float64)
    _check(lib().kpm_export_csr(H.handle, rowptr.ctypes.data, col.ctypes.data, val.ctypes.data))
    return rowptr, col, val.view(np.complex128)


def _csr_arrays(rowptr, col, val):
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.complex128)
    return rowptr, col, val


def sell_layout(rowptr, C: int, sigma: int):
    """kpm_sell_layout (host only): (perm [N], width [nchunks], start [nchunks + 1]) of the
    SELL-C-sigma layout of a CRS pattern."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    N = rowptr.size - 1
    nch = (N + int(C) - 1) // int(C) if C > 0 else 0
    perm = np.zeros(max(N, 1), dtype=np.int32)
    width = np.zeros(max(nch, 1), dtype=np.int32)
    start = np.zeros(nch + 1, dtype=np.int64)
    _check(lib().kpm_sell_layout(N, rowptr.ctypes.data, int(C), int(sigma), perm.ctypes.data, width.ctypes.data,
                                 start.ctypes.data))
    return perm[:N], width[:nch], start


def import_csr(rowptr, col, val, dtype: str = "c128", C: int = 0, sigma: int = 0, margin: float = 1.01,
               fixed_scale=None, stream=None) -> Hamiltonian:
    """kpm_import_csr: a general sparse Hermitian matrix (host CRS; val complex) stored on the
    device in SELL-C-sigma, with its Gershgorin scaling.  C = 0 and sigma = 0 take the library's
    defaults."""
    rowptr, col, val = _csr_arrays(rowptr, col, val)
    d = CsrDesc()
    d.N = rowptr.size - 1
    d.rowptr = rowptr.ctypes.data
    d.col = col.ctypes.data if col.size else None
    d.val = val.ctypes.data if val.size else None
    d.dtype = _DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
    d.sell_C, d.sell_sigma = int(C), int(sigma)
    d.margin = float(margin)
    if fixed_scale is not None:
        d.fixed_scale = 1
        d.a, d.b = float(fixed_scale[0]), float(fixed_scale[1])
    h = ctypes.c_void_p()
    _check(lib().kpm_import_csr(ctypes.byref(d), _stream(stream), ctypes.byref(h)))
    return Hamiltonian(h)


def sell_info(H: Hamiltonian) -> dict:
    """kpm_sell_info: C, sigma, chunks, stored entries (padding included) and imported nonzeros."""
    C, sigma = ctypes.c_int32(), ctypes.c_int32()
    nch, stored, nnz = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib().kpm_sell_info(H.handle, C, sigma, nch, stored, nnz))
    return {"C": C.value, "sigma": sigma.value, "nchunks": nch.value, "stored": stored.value, "nnz": nnz.value}


def aug_spmmv(H: Hamiltonian, V: torch.Tensor, W: torch.Tensor, alpha: float, beta: float, gamma: float,
              variant: str = "full", eta: torch.Tensor | None = None, stream=None):
    """kpm_aug_spmmv: one fused sweep W <- alpha H V + beta V + gamma W (+ eta for "full")."""
    R = V.shape[1]
    _check(lib().kpm_aug_spmmv(H.handle, _dptr(V), _dptr(W), R, float(alpha), float(beta), float(gamma),
                               _VARIANTS[variant], _dptr(eta) if eta is not None else None, _stream(stream)))


def _tuning_struct(tuning):
    """A SweepTuning from a dict of fields (missing ones at the library defaults), or None."""
    if tuning is None:
        return None
    fields = dict(DEFAULT_SWEEP_TUNING)
    fields.update(tuning)
    return SweepTuning(*[int(fields[k]) for k, _ in SweepTuning._fields_])


def moments(H: Hamiltonian, V0: torch.Tensor, M: int, mu: torch.Tensor | None = None,
            eta: torch.Tensor | None = None, check: bool = True, graph: bool = False, variant: str = "full",
            tuning: dict | None = None, group: int = 0, stream=None):
    """kpm_moments: mu[R][M] (float64) for the [N][R] start block V0.

    mu may be a device tensor (default) or a host numpy array (filled in place, the call
    synchronises); graph=True captures the launch sequence once and replays it; variant
    "nodot" runs the recurrence without the scalar products (mu is not written); tuning is a
    per-call launch shape (dict of kpm_sweep_tuning fields); group > 0 runs the columns as
    independent groups of that width (0: only where the whole block exceeds what the sweeps
    address)."""
    if V0.dim() != 2 or V0.shape[0] != H.N:
        raise ValueError("V0 must be [N][R]")
    if V0.dtype != H.torch_dtype:
        raise ValueError(f"V0 must be {H.torch_dtype}")
    R = V0.shape[1]
    if mu is None:
        mu = torch.empty((R, M), dtype=torch.float64, device=V0.device)
    opts = RunOpts()
    opts.check = 1 if check else 0
    opts.use_graph = 1 if graph else 0
    opts.variant = _VARIANTS[variant]
    t = _tuning_struct(tuning)
    if t is not None:
        opts.tuning = ctypes.pointer(t)
    opts.eta_out = _dptr(eta).value if eta is not None else None
    opts.group = int(group)
    if isinstance(mu, np.ndarray):
        if mu.dtype != np.float64 or mu.shape != (R, M) or not mu.flags.c_contiguous:
            raise ValueError("host mu must be a contiguous float64 [R][M] array")
        opts.mu_on_host = 1
        mu_ptr = ctypes.c_void_p(mu.ctypes.data)
    else:
        mu_ptr = _dptr(mu)
    _check(lib().kpm_moments(H.handle, _dptr(V0), R, int(M), mu_ptr, ctypes.byref(opts), _stream(stream)))
    return mu


def moments_naive(H: Hamiltonian, V0: torch.Tensor, M: int, mu: torch.Tensor | None = None,
                  check: bool = True, stream=None) -> torch.Tensor:
    """kpm_moments_naive: mu[R][M] by the naive algorithm (one SpMV and five BLAS-1 calls per step)."""
    if V0.dim() != 2 or V0.shape[0] != H.N:
        raise ValueError("V0 must be [N][R]")
    if V0.dtype != H.torch_dtype:
        raise ValueError(f"V0 must be {H.torch_dtype}")
    R = V0.shape[1]
    if mu is None:
        mu = torch.empty((R, M), dtype=torch.float64, device=V0.device)
    _check(lib().kpm_moments_naive(H.handle, _dptr(V0), R, int(M), _dptr(mu), 1 if check else 0, _stream(stream)))
    return mu


_BLAS1_DTYPES = {torch.complex128: 0, torch.complex64: 1}


def _blas1_vec(x: torch.Tensor) -> int:
    if x.dtype not in _BLAS1_DTYPES or not x.is_contiguous() or not x.is_cuda:
        raise ValueError("BLAS-1 vectors must be contiguous complex128 or complex64 device tensors")
    return _BLAS1_DTYPES[x.dtype]


def axpy(alpha: float, x: torch.Tensor, y: torch.Tensor, stream=None) -> torch.Tensor:
    """kpm_axpy: y <- y + alpha x (in place)."""
    dt = _blas1_vec(x)
    if _blas1_vec(y) != dt or x.numel() != y.numel():
        raise ValueError("x and y must have the same dtype and length")
    _check(lib().kpm_axpy(dt, x.numel(), float(alpha), _dptr(x), _dptr(y), _stream(stream)))
    return y


def scal(alpha: float, x: torch.Tensor, stream=None) -> torch.Tensor:
    """kpm_scal: x <- alpha x (in place)."""
    _check(lib().kpm_scal(_blas1_vec(x), x.numel(), float(alpha), _dptr(x), _stream(stream)))
    return x


def dot(x: torch.Tensor, y: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """kpm_dot: sum_i conj(x_i) y_i in FP64 as a device tensor [re, im]."""
    dt = _blas1_vec(x)
    if _blas1_vec(y) != dt or x.numel() != y.numel():
        raise ValueError("x and y must have the same dtype and length")
    if out is None:
        out = torch.empty(2, dtype=torch.float64, device=x.device)
    _check(lib().kpm_dot(dt, x.numel(), _dptr(x), _dptr(y), _dptr(out), _stream(stream)))
    return out


def dot_noalloc(x: torch.Tensor, y: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
    """kpm_dot_noalloc: kpm_dot through the library's static per-GPU partials array (allocates
    nothing; `out` is a caller-provided float64 device tensor of 2 elements)."""
    dt = _blas1_vec(x)
    if _blas1_vec(y) != dt or x.numel() != y.numel():
        raise ValueError("x and y must have the same dtype and length")
    if out.dtype != torch.float64 or out.numel() < 2 or not out.is_cuda:
        raise ValueError("out must be a float64 device tensor with 2 elements")
    _check(lib().kpm_dot_noalloc(dt, x.numel(), _dptr(x), _dptr(y), _dptr(out), _stream(stream)))
    return out


def moments_batched(Hs, V0s, M: int, mu: torch.Tensor | None = None, check: bool = True,
                    graph: bool = False, stream=None) -> torch.Tensor:
    """kpm_moments_batched: mu[n_inst][R][M] (float64, device) for instances (Hs[i], V0s[i])."""
    n = len(Hs)
    if n == 0 or len(V0s) != n:
        raise ValueError("need one start block per Hamiltonian")
    R = V0s[0].shape[1]
    for H, V0 in zip(Hs, V0s):
        if V0.dim() != 2 or V0.shape[0] != H.N or V0.shape[1] != R:
            raise ValueError("V0s[i] must be [N_i][R] with one R for all instances")
        if V0.dtype != H.torch_dtype:
            raise ValueError(f"V0s[i] must be {H.torch_dtype}")
    if mu is None:
        mu = torch.empty((n, R, M), dtype=torch.float64, device=V0s[0].device)
    hs = (ctypes.c_void_p * n)(*[H.handle for H in Hs])
    vs = (ctypes.c_void_p * n)(*[_dptr(V0).value for V0 in V0s])
    flags = (BATCH_CHECK if check else 0) | (BATCH_GRAPH if graph else 0)
    _check(lib().kpm_moments_batched(hs, vs, n, R, int(M), _dptr(mu), flags, _stream(stream)))
    return mu


def set_batch_tuning(waves: int = 0, wg_per_cu: int = 0, dynamic: int = 1, slab: int = 0):
    """kpm_set_batch_tuning: launch shape of the batched solver (process-wide)."""
    _check(lib().kpm_set_batch_tuning(ctypes.byref(BatchTuning(waves, wg_per_cu, dynamic, slab))))


def reset_batch_tuning():
    _check(lib().kpm_set_batch_tuning(None))


def get_batch_tuning():
    t = BatchTuning()
    _check(lib().kpm_get_batch_tuning(ctypes.byref(t)))
    return {"waves": t.waves, "wg_per_cu": t.wg_per_cu, "dynamic": t.dynamic, "slab": t.slab}


def dos(mu: torch.Tensor, a: float, b: float, E: torch.Tensor, kernel: str = "jackson", kparam: float = 0.0,
        rho: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """kpm_dos: density of states per unit energy on the device energy grid E."""
    R, M = mu.shape
    K = E.numel()
    if rho is None:
        rho = torch.empty(K, dtype=torch.float64, device=E.device)
    _check(lib().kpm_dos(_dptr(mu), R, M, _KERNELS[kernel], float(kparam), float(a), float(b),
                         _dptr(E), K, _dptr(rho), _stream(stream)))
    return rho


def random_phase_block(N: int, R: int, seed: int, dtype: str = "c128", out: torch.Tensor | None = None,
                       stream=None) -> torch.Tensor:
    """kpm_random_phase_block: [N][R] random-phase start block drawn on the device."""
    dt = _DTYPES[dtype]
    if out is None:
        out = torch.empty((N, R), dtype=_TORCH_DTYPE[dt], device="cuda")
    _check(lib().kpm_random_phase_block(_dptr(out), int(N), int(R), dt, int(seed) & 0xFFFFFFFFFFFFFFFF,
                                        _stream(stream)))
    return out


def lanczos_bounds(H: Hamiltonian, steps: int = 50, seed: int = 0, stream=None):
    """kpm_lanczos_bounds: (emin, emax), the extreme Ritz values after `steps` Lanczos steps."""
    lo, hi = ctypes.c_double(), ctypes.c_double()
    _check(lib().kpm_lanczos_bounds(H.handle, int(steps), int(seed) & 0xFFFFFFFFFFFFFFFF, ctypes.byref(lo),
                                    ctypes.byref(hi), _stream(stream)))
    return lo.value, hi.value


def set_scaling(H: Hamiltonian, a: float, b: float):
    """kpm_set_scaling: the sweeps apply (H - b) / a from now on."""
    _check(lib().kpm_set_scaling(H.handle, float(a), float(b)))
    H.a, H.b = float(a), float(b)


def site_block(N: int, rows, dtype: str = "c128", out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """kpm_site_block: [N][R] block whose column r is the unit vector of row rows[r]."""
    import numpy as np
    r = np.ascontiguousarray(rows, dtype=np.int64)
    dt = _DTYPES[dtype]
    if out is None:
        out = torch.empty((N, r.size), dtype=_TORCH_DTYPE[dt], device="cuda")
    _check(lib().kpm_site_block(_dptr(out), int(N), int(r.size), r.ctypes.data_as(ctypes.c_void_p), dt,
                                _stream(stream)))
    return out


def plane_wave_block(L, k, orbitals, dtype: str = "c128", out: torch.Tensor | None = None,
                     stream=None) -> torch.Tensor:
    """kpm_plane_wave_block: [N][R] block of plane waves (momenta k [R][3], orbitals [R])."""
    import numpy as np
    Ls = np.ascontiguousarray(L, dtype=np.int32)
    kk = np.ascontiguousarray(k, dtype=np.float64).reshape(-1, 3)
    oo = np.ascontiguousarray(orbitals, dtype=np.int32)
    if kk.shape[0] != oo.size:
        raise ValueError("one orbital per momentum")
    dt = _DTYPES[dtype]
    N = 4 * int(Ls[0]) * int(Ls[1]) * int(Ls[2])
    if out is None:
        out = torch.empty((N, oo.size), dtype=_TORCH_DTYPE[dt], device="cuda")
    _check(lib().kpm_plane_wave_block(_dptr(out), Ls.ctypes.data_as(ctypes.c_void_p), int(oo.size),
                                      kk.ctypes.data_as(ctypes.c_void_p), oo.ctypes.data_as(ctypes.c_void_p), dt,
                                      _stream(stream)))
    return out


def dos_batched(mu: torch.Tensor, a: torch.Tensor, b: torch.Tensor, E: torch.Tensor, M: int | None = None,
                kernel: str = "jackson", kparam: float = 0.0, masses: bool = False,
                rho: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """kpm_dos_batched: rho [n][K] from mu [n][R][ld] (first M moments), per-instance a, b [n]."""
    n, R, ld = mu.shape
    M = ld if M is None else int(M)
    K = E.numel()
    if rho is None:
        rho = torch.empty((n, K), dtype=torch.float64, device=E.device)
    _check(lib().kpm_dos_batched(_dptr(mu), n, R, ld, M, _KERNELS[kernel], float(kparam), _dptr(a), _dptr(b),
                                 _dptr(E), K, 1 if masses else 0, _dptr(rho), _stream(stream)))
    return rho


def moment_features(mu: torch.Tensor, n_mom: int, extra: torch.Tensor | None = None,
                    stream=None) -> torch.Tensor:
    """kpm_moment_features: [n][n_mom (+1)] float32 features from mu [n][R][ld]."""
    n, R, ld = mu.shape
    x = torch.empty((n, n_mom + (1 if extra is not None else 0)), dtype=torch.float32, device=mu.device)
    _check(lib().kpm_moment_features(_dptr(mu), n, R, ld, int(n_mom), _dptr(extra) if extra is not None else None,
                                     _dptr(x), _stream(stream)))
    return x


DEFAULT_SWEEP_TUNING = {"wg_per_cu": 0, "xcd_ways": 8, "chunk_tiles": 8, "pencil": 16, "dynamic": 0,
                        "prefetch": 2, "stream": 3, "lattice": 1, "gather": 1, "tile_order": 3, "slab": 4,
                        "gather_tile": 0}


def set_sweep_tuning(wg_per_cu: int = 0, xcd_ways: int = 8, chunk_tiles: int = 8, pencil: int = 16,
                     dynamic: int = 0, prefetch: int = 2, stream: int = 3, lattice: int = 1, gather: int = 1,
                     tile_order: int = 3, slab: int = 4, gather_tile: int = 0):
    """kpm_set_sweep_tuning: launch shape and site order of the sweep kernel (process-wide)."""
    _check(lib().kpm_set_sweep_tuning(ctypes.byref(SweepTuning(wg_per_cu, xcd_ways, chunk_tiles, pencil,
                                                               dynamic, prefetch, stream, lattice, gather,
                                                               tile_order, slab, gather_tile))))


def reset_sweep_tuning():
    _check(lib().kpm_set_sweep_tuning(None))


def get_sweep_tuning():
    t = SweepTuning()
    _check(lib().kpm_get_sweep_tuning(ctypes.byref(t)))
    return {"wg_per_cu": t.wg_per_cu, "xcd_ways": t.xcd_ways, "chunk_tiles": t.chunk_tiles, "pencil": t.pencil,
            "dynamic": t.dynamic, "prefetch": t.prefetch, "stream": t.stream,
            "lattice": t.lattice, "gather": t.gather, "tile_order": t.tile_order, "slab": t.slab,
            "gather_tile": t.gather_tile}


SWEEP_KERNELS = {0: "aug_spmmv_kernel", 1: "lattice_kernel", 2: "gather_sweep_kernel", 3: "window_sweep_kernel",
                 4: "sell_sweep_kernel"}


def sweep_kernel(H: Hamiltonian, R: int) -> str:
    """kpm_sweep_kernel: name of the sweep kernel used for H at block width R."""
    k = ctypes.c_int32()
    _check(lib().kpm_sweep_kernel(H.handle, int(R), ctypes.byref(k)))
    return SWEEP_KERNELS[k.value]


def sweep_plan(H: Hamiltonian, R: int, tuning: dict | None = None) -> dict:
    """kpm_sweep_plan: kernel, grid, resolved tile order, z-pieces and 32-column halves of a sweep, and the
    column-group width kpm_moments takes for the block by default."""
    p = SweepPlan()
    t = _tuning_struct(tuning)
    _check(lib().kpm_sweep_plan(H.handle, int(R), ctypes.byref(t) if t is not None else None, ctypes.byref(p)))
    return {"kernel": SWEEP_KERNELS[p.kernel], "grid": p.grid, "tile_order": p.tile_order, "pieces": p.pieces,
            "halves": p.halves, "group": p.group}


def sweep_profile_enable(on=True):
    """kpm_sweep_profile_enable: bracket every n-th sweep kernel with HIP events (True = every one,
    an integer n > 0 = every n-th, False / 0 = off)."""
    n = int(on) if not isinstance(on, bool) else (1 if on else 0)
    _check(lib().kpm_sweep_profile_enable(n))


def sweep_profile_read():
    """kpm_sweep_profile_read: (count, total_ms, min_ms, max_ms) of the recorded sweeps; clears them."""
    n, tot, lo, hi = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib().kpm_sweep_profile_read(n, tot, lo, hi))
    return n.value, tot.value, lo.value, hi.value


MLP_PARAM_ORDER = ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4", "w5", "b5")


def flatten_params(P: dict) -> np.ndarray:
    """Parameter dict (W1 [n_in][H], b1, ..., w5 [H] or [H][1], b5) -> flat float32 vector."""
    return np.concatenate([np.asarray(P[k], dtype=np.float64).reshape(-1) for k in MLP_PARAM_ORDER]).astype(np.float32)


def unflatten_params(flat: np.ndarray, n_in: int, hidden: int, n_out: int) -> dict:
    shapes = {"W1": (n_in, hidden), "b1": (hidden,), "W2": (hidden, hidden), "b2": (hidden,),
              "W3": (hidden, hidden), "b3": (hidden,), "W4": (hidden, n_out), "b4": (n_out,),
              "w5": (hidden, 1), "b5": (1,)}
    out, o = {}, 0
    for k in MLP_PARAM_ORDER:
        n = int(np.prod(shapes[k]))
        out[k] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(shapes[k])
        o += n
    return out


class MLP:
    """Owning wrapper of a kpm_mlp network (learned DOS reconstruction)."""

    def __init__(self, n_in: int = 129, hidden: int = 512, n_out: int = 512, max_batch: int = 1024):
        h = ctypes.c_void_p()
        _check(lib().kpm_mlp_create(int(n_in), int(hidden), int(n_out), int(max_batch), ctypes.byref(h)))
        self.handle = h
        self.n_in, self.hidden, self.n_out, self.max_batch = n_in, hidden, n_out, max_batch
        c = ctypes.c_int64()
        _check(lib().kpm_mlp_param_count(self.handle, ctypes.byref(c)))
        self.param_count = c.value
        self._loss = torch.zeros(1, dtype=torch.float32, device="cuda")

    def close(self):
        if self.handle:
            lib().kpm_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, flat) -> None:
        if isinstance(flat, dict):
            flat = flatten_params(flat)
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        if flat.size != self.param_count:
            raise ValueError(f"expected {self.param_count} parameters")
        _check(lib().kpm_mlp_set_params(self.handle, flat.ctypes.data))

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.param_count, dtype=np.float32)
        _check(lib().kpm_mlp_get_params(self.handle, out.ctypes.data))
        return out

    def get_grads(self) -> np.ndarray:
        out = np.zeros(self.param_count, dtype=np.float32)
        _check(lib().kpm_mlp_get_grads(self.handle, out.ctypes.data))
        return out

    def _x(self, x):
        if x.dtype != torch.float32 or x.dim() != 2 or x.shape[1] != self.n_in:
            raise ValueError(f"x must be float32 [B][{self.n_in}]")
        return x

    def forward(self, x: torch.Tensor, stream=None):
        """(q [B][n_out], e [B]) on the device."""
        x = self._x(x)
        B = x.shape[0]
        q = torch.empty((B, self.n_out), dtype=torch.float32, device=x.device)
        e = torch.empty(B, dtype=torch.float32, device=x.device)
        _check(lib().kpm_mlp_forward(self.handle, _dptr(x), B, _dptr(q), _dptr(e), _stream(stream)))
        return q, e

    def backward(self, x: torch.Tensor, p: torch.Tensor, t: torch.Tensor | None = None, lam: float = 1.0,
                 stream=None) -> torch.Tensor:
        x = self._x(x)
        B = x.shape[0]
        if p.dtype != torch.float32 or tuple(p.shape) != (B, self.n_out):
            raise ValueError("p must be float32 [B][n_out]")
        _check(lib().kpm_mlp_backward(self.handle, _dptr(x), _dptr(p), _dptr(t) if t is not None else None, B,
                                      float(lam), _dptr(self._loss), _stream(stream)))
        return self._loss

    def adam_step(self, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
                  stream=None):
        _check(lib().kpm_mlp_adam_step(self.handle, float(lr), float(beta1), float(beta2), float(eps),
                                       _stream(stream)))

    def train_step(self, x, p, t=None, lam: float = 1.0, lr: float = 1e-3, stream=None) -> torch.Tensor:
        x = self._x(x)
        B = x.shape[0]
        _check(lib().kpm_mlp_train_step(self.handle, _dptr(x), _dptr(p), _dptr(t) if t is not None else None, B,
                                        float(lam), float(lr), _dptr(self._loss), _stream(stream)))
        return self._loss


def gemm_bf16(A: torch.Tensor, B: torch.Tensor, trans_a: bool = False, trans_b: bool = False,
              stream=None) -> torch.Tensor:
    """kpm_mlp_gemm_bf16 on BF16 bit patterns (torch.int16 / uint16 / bfloat16 tensors)."""
    if A.dtype == torch.bfloat16:
        A = A.view(torch.int16)
    if B.dtype == torch.bfloat16:
        B = B.view(torch.int16)
    M, K = (A.shape[1], A.shape[0]) if trans_a else (A.shape[0], A.shape[1])
    N = B.shape[0] if trans_b else B.shape[1]
    C = torch.empty((M, N), dtype=torch.float32, device=A.device)
    _check(lib().kpm_mlp_gemm_bf16(_dptr(A), _dptr(B), M, N, K, int(trans_a), int(trans_b), _dptr(C),
                                   _stream(stream)))
    return C


STREAM_COPY, STREAM_TRIAD, STREAM_READ = 0, 1, 2


def stream_kernel(kind: str, c: torch.Tensor, a: torch.Tensor, b: torch.Tensor | None = None, scalar: float = 3.0,
                  wg_per_cu: int = 1, nontemporal: bool = True, stream=None):
    """kpm_stream: STREAM copy (c = a) or triad (c = a + scalar b, FP64) over the bytes of c, or
    read: per-workgroup sums of a's FP64 values into c (c needs compute units x wg_per_cu doubles)."""
    k = {"copy": STREAM_COPY, "triad": STREAM_TRIAD, "read": STREAM_READ}[kind]
    nbytes = a.numel() * a.element_size()
    if k == STREAM_READ:
        cus = torch.cuda.get_device_properties(c.device).multi_processor_count
        if c.dtype != torch.float64 or c.numel() < cus * wg_per_cu:
            raise ValueError(f"read needs a float64 c of at least {cus * wg_per_cu} elements")
    elif c.numel() * c.element_size() != nbytes or (b is not None and b.numel() * b.element_size() != nbytes):
        raise ValueError("arrays must have the same size in bytes")
    _check(lib().kpm_stream(k, _dptr(c), _dptr(a), _dptr(b) if b is not None else None, float(scalar), nbytes,
                            int(wg_per_cu), 1 if nontemporal else 0, _stream(stream)))
    return c


def version() -> str:
    return lib().kpm_version().decode()
