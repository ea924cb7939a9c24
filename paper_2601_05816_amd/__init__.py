"""Multi-rhs Wilson-Dirac operator and batched GMRES on AMD MI355X.

Thin Python binding over the C-ABI of liblqcd.so (declared in include/lqcd.h).
Torch tensors provide device memory and the current HIP stream; every
computation happens in the library's HIP kernels.  The binding only checks
shapes, marshals pointers and forwards status codes as exceptions.

Tensor shapes (lattice dims (N0, N1, N2, N3), N0 = time):
  U                      complex[4, N0, N1, N2, N3, 3, 3]
  block, RHS_OUTER       complex[nrhs, N0, N1, N2, N3, 4, 3]
  block, LAYOUT1         complex[N0, N1, N2, N3, nrhs, 4, 3]
  block, LAYOUT2         complex[N0, N1, N2, N3, 4, 3, nrhs]
  half-lattice blocks    the four lattice axes replaced by one axis of V/2 sites
complex128 selects FP64, complex64 FP32; FP16 storage uses float16 tensors
with a trailing axis of 2 (re, im).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

F64, F32, F16 = 0, 1, 2
RHS_OUTER, LAYOUT1, LAYOUT2 = 0, 1, 2
DAGGER = 1
OK, NOT_CONVERGED = 0, 1

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblqcd.so")
_lib = None


class LqcdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lqcd error {code}: {msg}")
        self.code = code


class Lattice(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 4)]


class SolverParams(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int32), ("max_restarts", ctypes.c_int32), ("eo", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("x_is_guess", ctypes.c_int32), ("fixed_iters", ctypes.c_int32),
                ("tol", ctypes.c_double), ("inner_tol", ctypes.c_double), ("max_outer", ctypes.c_int32),
                ("dagger", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("rhs_block", ctypes.c_int32),
                ("gs", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Problem(ctypes.Structure):
    _fields_ = [("lat", Lattice), ("U", ctypes.c_void_p), ("psi", ctypes.c_void_p), ("eta", ctypes.c_void_p),
                ("nrhs", ctypes.c_int32), ("reserved", ctypes.c_int32), ("m0", ctypes.c_double)]


MAX_BATCH = 16
NOALLOC_SCRATCH_BYTES = 256 << 20  # LQCD_NOALLOC_SCRATCH_BYTES


class KernelConfig(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("tile_y", ctypes.c_int32), ("tile_z", ctypes.c_int32),
                ("segments", ctypes.c_int32), ("nontemporal", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32),
                ("ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class RhsStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("restarts", ctypes.c_int32), ("outer_iters", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("true_relres", ctypes.c_double), ("est_relres", ctypes.c_double)]


def load():
    """Load liblqcd.so.  Raises if it has not been built: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing; build it with `python -m paper_2601_05816_amd.build`")
    # torch first: the library then binds to the HIP runtime torch loaded, so
    # device pointers, streams and events are shared by one runtime whatever
    # order the caller imports them in
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lp = ctypes.POINTER(Lattice)
    lib.lqcd_last_error.restype = ctypes.c_char_p
    lib.lqcd_lattice_tables.argtypes = [lp, vp, vp]
    lib.dirac_apply.argtypes = [lp, vp, vp, vp, i32, dbl, i32, i32, i32, vp]
    lib.dirac_apply_eo.argtypes = [lp, vp, vp, vp, i32, dbl, i32, i32, i32, vp]
    lib.dirac_apply_eo_ws.argtypes = [lp, vp, vp, vp, i32, dbl, i32, i32, i32, vp, ctypes.c_size_t, vp]
    lib.dirac_apply_eo_ws.restype = i32
    lib.dirac_apply_eo_workspace_bytes.argtypes = [lp, i32, i32]
    lib.dirac_apply_eo_workspace_bytes.restype = ctypes.c_size_t
    lib.dirac_apply_eo_noalloc.argtypes = [lp, vp, vp, vp, i32, dbl, i32, i32, i32, vp]
    lib.dirac_apply_eo_noalloc.restype = i32
    lib.dirac_apply_clover.argtypes = [lp, vp, vp, vp, vp, i32, dbl, i32, i32, i32, vp]
    lib.dirac_apply_clover.restype = i32
    lib.clover_inverse.argtypes = [lp, vp, vp, dbl, i32, vp]
    lib.clover_inverse.restype = i32
    lib.dirac_apply_eo_clover.argtypes = [lp, vp, vp, vp, vp, vp, i32, dbl, i32, i32, i32, vp]
    lib.dirac_apply_eo_clover.restype = i32
    lib.lqcd_set_kernel_variant.argtypes = [i32, vp]
    lib.dirac_apply_batch.argtypes = [i32, ctypes.POINTER(Problem), i32, i32, vp]
    lib.dirac_apply_batch.restype = i32
    lib.lqcd_set_batch_grid.argtypes = [i32]
    lib.lqcd_set_batch_grid.restype = i32
    lib.lqcd_set_kernel_config.argtypes = [ctypes.POINTER(KernelConfig)]
    lib.lqcd_set_kernel_config.restype = i32
    lib.lqcd_autotune.argtypes = [lp, vp, vp, vp, i32, i32, i32, i32, i32, ctypes.POINTER(KernelConfig), vp]
    lib.lqcd_autotune.restype = i32
    lib.lqcd_tune_save.argtypes = [ctypes.c_char_p]
    lib.lqcd_tune_save.restype = i32
    lib.lqcd_tune_load.argtypes = [ctypes.c_char_p]
    lib.lqcd_tune_load.restype = i32
    lib.lqcd_tune_clear.argtypes = []
    lib.lqcd_tune_clear.restype = None
    lib.lqcd_autotune_batch.argtypes = [i32, ctypes.POINTER(Problem), i32, i32, ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_int), vp]
    lib.lqcd_set_batch_kernel.argtypes = [i32]
    lib.lqcd_set_batch_kernel.restype = i32
    lib.lqcd_autotune_batch.restype = i32
    lib.lqcd_hbm_probe.argtypes = [i32, vp, vp, vp, ctypes.c_size_t, i32, ctypes.POINTER(ctypes.c_double), vp]
    lib.lqcd_hbm_probe.restype = i32
    for name in ("lqcd_lattice_tables", "dirac_apply", "dirac_apply_eo", "lqcd_set_kernel_variant"):
        getattr(lib, name).restype = i32
    if hasattr(lib, "gmres_solve"):
        lib.lqcd_solver_defaults.argtypes = [ctypes.POINTER(SolverParams)]
        lib.lqcd_solver_defaults.restype = None
        lib.gmres_workspace_bytes.argtypes = [lp, i32, ctypes.POINTER(SolverParams)]
        lib.gmres_workspace_bytes.restype = ctypes.c_size_t
        lib.gmres_rhs_block.argtypes = [lp, i32, ctypes.POINTER(SolverParams), ctypes.c_size_t]
        lib.gmres_rhs_block.restype = i32
        lib.gmres_solve.argtypes = [lp, vp, vp, vp, i32, dbl, i32, ctypes.POINTER(SolverParams), vp,
                                    ctypes.c_size_t, ctypes.POINTER(RhsStats), vp]
        lib.gmres_solve.restype = i32
        lib.gmres_workspace_bytes_clover.argtypes = [lp, i32, ctypes.POINTER(SolverParams)]
        lib.gmres_workspace_bytes_clover.restype = ctypes.c_size_t
        lib.gmres_solve_clover.argtypes = [lp, vp, vp, vp, vp, i32, dbl, i32, ctypes.POINTER(SolverParams), vp,
                                           ctypes.c_size_t, ctypes.POINTER(RhsStats), vp]
        lib.gmres_solve_clover.restype = i32
        lib.gmres_workspace_bytes_batch.argtypes = [i32, ctypes.POINTER(Problem), ctypes.POINTER(SolverParams)]
        lib.gmres_workspace_bytes_batch.restype = ctypes.c_size_t
        lib.gmres_solve_batch.argtypes = [i32, ctypes.POINTER(Problem), ctypes.POINTER(SolverParams), vp,
                                          ctypes.c_size_t, ctypes.POINTER(RhsStats), vp]
        lib.gmres_solve_batch.restype = i32
        lib.block_gmres_workspace_bytes.argtypes = [lp, i32, ctypes.POINTER(SolverParams)]
        lib.block_gmres_workspace_bytes.restype = ctypes.c_size_t
        lib.block_gmres_solve.argtypes = [lp, vp, vp, vp, i32, dbl, i32, ctypes.POINTER(SolverParams), vp,
                                          ctypes.c_size_t, ctypes.POINTER(RhsStats), vp]
        lib.block_gmres_solve.restype = i32
        lib.link_force.argtypes = [lp, vp, vp, vp, vp, i32, i32, dbl, i32, vp]
        lib.link_force.restype = i32
        lib.block_dot.argtypes = [lp, vp, vp, i32, i32, vp, vp]
        lib.block_dot.restype = i32
    _lib = lib
    return lib


def _check(rc):
    if rc < 0:
        raise LqcdError(rc, load().lqcd_last_error().decode())
    return rc


def _lattice(dims):
    lat = Lattice()
    for i in range(4):
        lat.dims[i] = int(dims[i])
    return lat


def lattice_tables(dims):
    """(nbr[V, 8], eo_site[2, V/2]) as int32 numpy arrays, computed by the library."""
    v = int(np.prod(dims))
    nbr = np.empty((v, 8), dtype=np.int32)
    eo = np.empty((2, v // 2), dtype=np.int32)
    _check(load().lqcd_lattice_tables(ctypes.byref(_lattice(dims)), nbr.ctypes.data, eo.ctypes.data))
    return nbr, eo


def set_kernel_variant(variant=0, pencil=None):
    """Wilson kernel choice: 0 automatic, 1 one site per work item, 2 pencils;
    pencil = (tile Y, tile Z, t segments) with 0 = automatic."""
    arr = None
    if pencil is not None:
        arr = (ctypes.c_int32 * 3)(*[int(v) for v in pencil])
    _check(load().lqcd_set_kernel_variant(int(variant), arr))


def set_kernel_config(variant=0, tile_y=0, tile_z=0, segments=0, nontemporal=0, wg_per_cu=0):
    """Force a Wilson kernel configuration (variant 0 = automatic selection)."""
    if variant == 0 and not (tile_y or tile_z or segments or nontemporal or wg_per_cu):
        _check(load().lqcd_set_kernel_config(None))
        return
    c = KernelConfig(int(variant), int(tile_y), int(tile_z), int(segments), int(nontemporal), int(wg_per_cu), 0.0)
    _check(load().lqcd_set_kernel_config(ctypes.byref(c)))


def tune_save(path):
    _check(load().lqcd_tune_save(str(path).encode()))


def tune_load(path):
    return _check(load().lqcd_tune_load(str(path).encode()))


def tune_clear():
    load().lqcd_tune_clear()


# ------------------------------------------------------------- tensors
def _prec_of(t):
    import torch

    if t.dtype == torch.complex128:
        return F64
    if t.dtype == torch.complex64:
        return F32
    if t.dtype == torch.float16 and t.shape[-1] == 2:
        return F16
    raise TypeError(f"unsupported dtype {t.dtype} (complex128, complex64, or float16[..., 2])")


def _core_shape(t, prec):
    return tuple(t.shape[:-1]) if prec == F16 else tuple(t.shape)


def _dims_of_links(U, prec):
    s = _core_shape(U, prec)
    if len(s) != 7 or s[0] != 4 or s[5:] != (3, 3):
        raise ValueError(f"gauge field must be [4, N0, N1, N2, N3, 3, 3], got {s}")
    return s[1:5]


def _nrhs_of(t, prec, layout, nsite_axes):
    s = _core_shape(t, prec)
    if layout == RHS_OUTER:
        return s[0], s[1:1 + nsite_axes]
    if layout == LAYOUT1:
        return s[nsite_axes], s[:nsite_axes]
    if layout == LAYOUT2:
        return s[-1], s[:nsite_axes]
    raise ValueError(f"unknown layout {layout}")


def _check_device(*ts):
    for t in ts:
        if not t.is_cuda:
            raise ValueError("all tensors must live on the GPU")
        if not t.is_contiguous():
            raise ValueError("tensors must be contiguous")


def _stream():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def dirac_apply(U, psi, m0, layout=LAYOUT2, dagger=False, out=None):
    """eta = D psi (or D^dagger psi) for every rhs of a full-lattice block."""
    import torch

    prec = _prec_of(psi)
    if _prec_of(U) != prec:
        raise TypeError("U and psi must have the same precision")
    dims = _dims_of_links(U, prec)
    nrhs, sdims = _nrhs_of(psi, prec, layout, 4)
    if tuple(sdims) != tuple(dims):
        raise ValueError(f"spinor lattice {sdims} does not match gauge lattice {dims}")
    out = torch.empty_like(psi) if out is None else out
    _check_device(U, psi, out)
    _check(load().dirac_apply(ctypes.byref(_lattice(dims)), U.data_ptr(), psi.data_ptr(), out.data_ptr(), nrhs,
                              float(m0), layout, prec, DAGGER if dagger else 0, _stream()))
    return out


def dirac_apply_eo(U, psi_e, m0, layout=LAYOUT2, dagger=False, out=None):
    """eta_e = S psi_e, S = D_ee - D_eo D_oo^-1 D_oe, for an even half-lattice block."""
    import torch

    prec = _prec_of(psi_e)
    if _prec_of(U) != prec:
        raise TypeError("U and psi_e must have the same precision")
    dims = _dims_of_links(U, prec)
    nrhs, sdims = _nrhs_of(psi_e, prec, layout, 1)
    if int(sdims[0]) * 2 != int(np.prod(dims)):
        raise ValueError(f"half-lattice block has {sdims[0]} sites, lattice {dims} needs {int(np.prod(dims)) // 2}")
    out = torch.empty_like(psi_e) if out is None else out
    _check_device(U, psi_e, out)
    _check(load().dirac_apply_eo(ctypes.byref(_lattice(dims)), U.data_ptr(), psi_e.data_ptr(), out.data_ptr(),
                                 nrhs, float(m0), layout, prec, DAGGER if dagger else 0, _stream()))
    return out


def dirac_apply_eo_ws(U, psi_e, m0, work, layout=LAYOUT2, dagger=False, out=None):
    """dirac_apply_eo with the odd temporary in `work` (a device uint8 tensor
    of at least dirac_apply_eo_workspace_bytes bytes; nothing is allocated
    when `out` is given)."""
    import torch

    prec = _prec_of(psi_e)
    if _prec_of(U) != prec:
        raise TypeError("U and psi_e must have the same precision")
    dims = _dims_of_links(U, prec)
    nrhs, sdims = _nrhs_of(psi_e, prec, layout, 1)
    if int(sdims[0]) * 2 != int(np.prod(dims)):
        raise ValueError(f"half-lattice block has {sdims[0]} sites, lattice {dims} needs {int(np.prod(dims)) // 2}")
    out = torch.empty_like(psi_e) if out is None else out
    _check_device(U, psi_e, out, work)
    _check(load().dirac_apply_eo_ws(ctypes.byref(_lattice(dims)), U.data_ptr(), psi_e.data_ptr(), out.data_ptr(),
                                    nrhs, float(m0), layout, prec, DAGGER if dagger else 0, work.data_ptr(),
                                    work.numel(), _stream()))
    return out


def dirac_apply_eo_workspace_bytes(dims, nrhs, prec):
    return int(load().dirac_apply_eo_workspace_bytes(ctypes.byref(_lattice(dims)), int(nrhs), int(prec)))


def dirac_apply_eo_noalloc(U, psi_e, m0, out, layout=LAYOUT2, dagger=False):
    """dirac_apply_eo with the odd temporary in the library's fixed device
    array (no device allocation; `out` must be given).  Raises LqcdError
    (LQCD_ERR_WORKSPACE) if the odd block exceeds NOALLOC_SCRATCH_BYTES."""
    prec = _prec_of(psi_e)
    if _prec_of(U) != prec:
        raise TypeError("U and psi_e must have the same precision")
    dims = _dims_of_links(U, prec)
    nrhs, sdims = _nrhs_of(psi_e, prec, layout, 1)
    if int(sdims[0]) * 2 != int(np.prod(dims)):
        raise ValueError(f"half-lattice block has {sdims[0]} sites, lattice {dims} needs {int(np.prod(dims)) // 2}")
    if out.shape != psi_e.shape or out.dtype != psi_e.dtype:
        raise ValueError("out must have the shape and dtype of psi_e")
    _check_device(U, psi_e, out)
    _check(load().dirac_apply_eo_noalloc(ctypes.byref(_lattice(dims)), U.data_ptr(), psi_e.data_ptr(),
                                         out.data_ptr(), nrhs, float(m0), layout, prec, DAGGER if dagger else 0,
                                         _stream()))
    return out


# ---------------------------------------------------------------- clover
def _check_clover(C, dims, prec):
    if _prec_of(C) != prec:
        raise TypeError("the clover field must have the precision of U")
    want = tuple(dims) + (42,) + ((2,) if prec == F16 else ())
    if tuple(C.shape) != want:
        raise ValueError(f"clover field shape {tuple(C.shape)}, expected {want}")


def dirac_apply_clover(U, C, psi, m0, layout=LAYOUT2, dagger=False, out=None):
    """eta = (D_W - C) psi (or its adjoint) with a packed clover field C
    [N0, N1, N2, N3, 42] (two Hermitian 6x6 blocks per site)."""
    import torch

    prec = _prec_of(psi)
    if _prec_of(U) != prec:
        raise TypeError("U and psi must have the same precision")
    dims = _dims_of_links(U, prec)
    _check_clover(C, dims, prec)
    nrhs, _ = _nrhs_of(psi, prec, layout, 4)
    out = torch.empty_like(psi) if out is None else out
    _check_device(U, C, psi, out)
    _check(load().dirac_apply_clover(ctypes.byref(_lattice(dims)), U.data_ptr(), C.data_ptr(), psi.data_ptr(),
                                     out.data_ptr(), nrhs, float(m0), layout, prec, DAGGER if dagger else 0, _stream()))
    return out


def clover_inverse(C, m0, dims):
    """Packed ((4 + m0) - C(x))^{-1} for every site (same shape and precision as C)."""
    import torch

    prec = _prec_of(C)
    _check_clover(C, dims, prec)
    out = torch.empty_like(C)
    _check_device(C, out)
    _check(load().clover_inverse(ctypes.byref(_lattice(dims)), C.data_ptr(), out.data_ptr(), float(m0), prec,
                                 _stream()))
    return out


def dirac_apply_eo_clover(U, C, Cinv, psi_e, m0, layout=LAYOUT2, dagger=False, out=None):
    """eta_e = S psi_e with the clover term: S = D_ee - D_eo D_oo^-1 D_oe, Cinv
    from clover_inverse(C, m0)."""
    import torch

    prec = _prec_of(psi_e)
    if _prec_of(U) != prec:
        raise TypeError("U and psi_e must have the same precision")
    dims = _dims_of_links(U, prec)
    _check_clover(C, dims, prec)
    _check_clover(Cinv, dims, prec)
    nrhs, sdims = _nrhs_of(psi_e, prec, layout, 1)
    if int(sdims[0]) * 2 != int(np.prod(dims)):
        raise ValueError(f"half-lattice block has {sdims[0]} sites, lattice {dims} needs {int(np.prod(dims)) // 2}")
    out = torch.empty_like(psi_e) if out is None else out
    _check_device(U, C, Cinv, psi_e, out)
    _check(load().dirac_apply_eo_clover(ctypes.byref(_lattice(dims)), U.data_ptr(), C.data_ptr(), Cinv.data_ptr(),
                                        psi_e.data_ptr(), out.data_ptr(), nrhs, float(m0), layout, prec,
                                        DAGGER if dagger else 0, _stream()))
    return out


# ---------------------------------------------------------------- solver
MODES = {"f64": 0, "ir-f32": 1, "ir-f16": 2}


GS = {"cgs": 0, "cgs2": 1, "mgs": 2}


def solver_params(restart=30, max_restarts=200, eo=True, mode=0, tol=1e-10, inner_tol=0.0, max_outer=50,
                  x_is_guess=False, fixed_iters=False, dagger=False, use_graph=False, rhs_block=0, gs="cgs"):
    p = SolverParams()
    load().lqcd_solver_defaults(ctypes.byref(p))
    p.restart, p.max_restarts, p.eo = int(restart), int(max_restarts), int(bool(eo))
    p.mode = MODES[mode] if isinstance(mode, str) else int(mode)
    p.tol, p.inner_tol, p.max_outer = float(tol), float(inner_tol), int(max_outer)
    p.x_is_guess, p.fixed_iters = int(bool(x_is_guess)), int(bool(fixed_iters))
    p.dagger = int(bool(dagger))
    p.use_graph = int(bool(use_graph))
    p.rhs_block = int(rhs_block)
    p.gs = GS[gs] if isinstance(gs, str) else int(gs)
    return p


def gmres_workspace_bytes(dims, nrhs, params):
    return int(load().gmres_workspace_bytes(ctypes.byref(_lattice(dims)), int(nrhs), ctypes.byref(params)))


def gmres_rhs_block(dims, nrhs, params, work_bytes):
    """The rhs chunk width gmres_solve uses with a workspace of work_bytes."""
    return _check(load().gmres_rhs_block(ctypes.byref(_lattice(dims)), int(nrhs), ctypes.byref(params),
                                         ctypes.c_size_t(int(work_bytes))))


def gmres_solve(U, b, m0, layout=LAYOUT2, x0=None, work=None, out=None, **kw):
    """x = D^-1 b per rhs with batched GMRES (FP64 U and b, full lattice).

    Keyword arguments are those of solver_params; x0 (same shape as b) is the
    initial guess; out (same shape and type as b) receives x (else a new
    tensor).  Returns (x, stats, status) with stats a dict of per-rhs numpy
    arrays and status OK or NOT_CONVERGED."""
    import torch

    if U.dtype != torch.complex128 or b.dtype != torch.complex128:
        raise TypeError("gmres_solve takes complex128 U and b")
    dims = _dims_of_links(U, F64)
    nrhs, sdims = _nrhs_of(b, F64, layout, 4)
    if tuple(sdims) != tuple(dims):
        raise ValueError(f"source lattice {sdims} does not match gauge lattice {dims}")
    p = solver_params(x_is_guess=x0 is not None, **kw)
    if out is not None:
        if out.shape != b.shape or out.dtype != b.dtype or not out.is_contiguous():
            raise ValueError("out must be a contiguous tensor of b's shape and type")
        x = out.copy_(x0) if x0 is not None else out
    else:
        x = x0.clone() if x0 is not None else torch.empty_like(b)
    if work is None:
        work = torch.empty(gmres_workspace_bytes(dims, nrhs, p), dtype=torch.uint8, device=b.device)
    _check_device(U, b, x, work)
    st = (RhsStats * nrhs)()
    rc = _check(load().gmres_solve(ctypes.byref(_lattice(dims)), U.data_ptr(), b.data_ptr(), x.data_ptr(), nrhs,
                                   float(m0), layout, ctypes.byref(p), work.data_ptr(), work.numel(), st, _stream()))
    stats = {k: np.array([getattr(s, k) for s in st]) for k, _ in RhsStats._fields_}
    return x, stats, rc


BLOCK_MAX_RHS = 16


def block_gmres_workspace_bytes(dims, nrhs, params):
    return int(load().block_gmres_workspace_bytes(ctypes.byref(_lattice(dims)), int(nrhs), ctypes.byref(params)))


def block_gmres_solve(U, b, m0, layout=LAYOUT2, x0=None, work=None, **kw):
    """x = D^-1 b with block GMRES: all rhs of b (at most BLOCK_MAX_RHS) share
    one block Krylov space.  Same keywords (mode must be "f64", no graphs) and
    return value as gmres_solve; stats["iters"] counts block steps."""
    import torch

    if U.dtype != torch.complex128 or b.dtype != torch.complex128:
        raise TypeError("block_gmres_solve takes complex128 U and b")
    dims = _dims_of_links(U, F64)
    nrhs, sdims = _nrhs_of(b, F64, layout, 4)
    if tuple(sdims) != tuple(dims):
        raise ValueError(f"source lattice {sdims} does not match gauge lattice {dims}")
    p = solver_params(x_is_guess=x0 is not None, **kw)
    x = x0.clone() if x0 is not None else torch.empty_like(b)
    need = block_gmres_workspace_bytes(dims, nrhs, p)
    if work is None or work.numel() < need:
        work = torch.empty(max(need, 1), dtype=torch.uint8, device=b.device)
    _check_device(U, b, x, work)
    st = (RhsStats * nrhs)()
    rc = _check(load().block_gmres_solve(ctypes.byref(_lattice(dims)), U.data_ptr(), b.data_ptr(), x.data_ptr(),
                                         nrhs, float(m0), layout, ctypes.byref(p), work.data_ptr(), work.numel(), st,
                                         _stream()))
    stats = {k: np.array([getattr(s, k) for s in st]) for k, _ in RhsStats._fields_}
    return x, stats, rc


def gmres_solve_clover(U, C, b, m0, layout=LAYOUT2, x0=None, work=None, **kw):
    """x = (D_W - C)^-1 b per rhs (FP64 U, clover field C [N0..N3, 42] and b);
    same keywords and return value as gmres_solve."""
    import torch

    if U.dtype != torch.complex128 or b.dtype != torch.complex128:
        raise TypeError("gmres_solve_clover takes complex128 U, C and b")
    dims = _dims_of_links(U, F64)
    _check_clover(C, dims, F64)
    nrhs, sdims = _nrhs_of(b, F64, layout, 4)
    if tuple(sdims) != tuple(dims):
        raise ValueError(f"source lattice {sdims} does not match gauge lattice {dims}")
    p = solver_params(x_is_guess=x0 is not None, **kw)
    x = x0.clone() if x0 is not None else torch.empty_like(b)
    need = int(load().gmres_workspace_bytes_clover(ctypes.byref(_lattice(dims)), nrhs, ctypes.byref(p)))
    if need == 0:
        raise ValueError("invalid solver arguments")
    if work is None or work.numel() < need:
        work = torch.empty(need, dtype=torch.uint8, device=b.device)
    _check_device(U, C, b, x, work)
    st = (RhsStats * nrhs)()
    rc = _check(load().gmres_solve_clover(ctypes.byref(_lattice(dims)), U.data_ptr(), C.data_ptr(), b.data_ptr(),
                                          x.data_ptr(), nrhs, float(m0), layout, ctypes.byref(p), work.data_ptr(),
                                          work.numel(), st, _stream()))
    stats = {k: np.array([getattr(s, k) for s in st]) for k, _ in RhsStats._fields_}
    return x, stats, rc


def link_force(U, g, psi, coeff, layout=LAYOUT2, project=False, out=None):
    """G_mu(x) = coeff sum_rhs sum_spin {[(1-g_mu) g(x)] (x) psi(x+mu)^* + psi(x) (x) [(1+g_mu) g(x+mu)]^*},
    or the su(3) force TA(G U^dag) with project=True.  FP64 blocks."""
    import torch

    dims = _dims_of_links(U, F64)
    nrhs, _ = _nrhs_of(g, F64, layout, 4)
    out = torch.empty_like(U) if out is None else out
    _check_device(U, g, psi, out)
    _check(load().link_force(ctypes.byref(_lattice(dims)), U.data_ptr(), g.data_ptr(), psi.data_ptr(),
                             out.data_ptr(), nrhs, layout, float(coeff), int(bool(project)), _stream()))
    return out


def block_dot(a, b, dims, layout=LAYOUT2):
    """Per-rhs <a_i, b_i> (conjugate-linear in a) of two FP64 full-lattice blocks, as a complex128 tensor."""
    import torch

    nrhs, _ = _nrhs_of(a, F64, layout, 4)
    out = torch.empty(nrhs, dtype=torch.complex128, device=a.device)
    _check_device(a, b, out)
    _check(load().block_dot(ctypes.byref(_lattice(dims)), a.data_ptr(), b.data_ptr(), nrhs, layout,
                            out.data_ptr(), _stream()))
    return out


def dirac_apply_batch(problems, dagger=False, outs=None):
    """eta_k = D_k psi_k for a list of (U_k, psi_k, m0_k) on independent lattices
    (rhs-innermost blocks, one precision), in one persistent launch."""
    import torch

    if not 1 <= len(problems) <= MAX_BATCH:
        raise ValueError(f"need 1..{MAX_BATCH} problems")
    prec = _prec_of(problems[0][1])
    arr = (Problem * len(problems))()
    outs = [torch.empty_like(p[1]) for p in problems] if outs is None else outs
    for k, ((U, psi, m0), eta) in enumerate(zip(problems, outs)):
        if _prec_of(psi) != prec or _prec_of(U) != prec:
            raise TypeError("all problems of a batch share one precision")
        dims = _dims_of_links(U, prec)
        nrhs, sdims = _nrhs_of(psi, prec, LAYOUT2, 4)
        if tuple(sdims) != tuple(dims):
            raise ValueError(f"problem {k}: spinor lattice {sdims} does not match {dims}")
        _check_device(U, psi, eta)
        arr[k].lat = _lattice(dims)
        arr[k].U, arr[k].psi, arr[k].eta = U.data_ptr(), psi.data_ptr(), eta.data_ptr()
        arr[k].nrhs, arr[k].m0 = nrhs, float(m0)
    _check(load().dirac_apply_batch(len(problems), arr, prec, DAGGER if dagger else 0, _stream()))
    return outs


def set_batch_grid(blocks=0):
    _check(load().lqcd_set_batch_grid(int(blocks)))


def autotune(U, psi, eta, m0=0.0, layout=LAYOUT2, eo=False, reps=3):
    """Time the candidate Wilson kernels on these buffers (eta overwritten) and
    record the fastest for automatic selection.  Returns the winner as a dict."""
    prec = _prec_of(psi)
    dims = _dims_of_links(U, prec)
    nrhs, _ = _nrhs_of(psi, prec, layout, 1 if eo else 4)
    _check_device(U, psi, eta)
    best = KernelConfig()
    _check(load().lqcd_autotune(ctypes.byref(_lattice(dims)), U.data_ptr(), psi.data_ptr(), eta.data_ptr(), nrhs,
                                prec, layout, int(bool(eo)), int(reps), ctypes.byref(best), _stream()))
    return best.as_dict()


def set_batch_kernel(kind=0):
    """Kernel of the persistent batch launch: 0 automatic, 1 one (site, rhs) per
    work item, 2 time-streaming pencils."""
    _check(load().lqcd_set_batch_kernel(int(kind)))


def autotune_batch(problems, outs, reps=3):
    """Pick the kernel and persistent grid size for dirac_apply_batch on these
    problems; returns {"kernel": k, "grid": g}."""
    prec = _prec_of(problems[0][1])
    arr = (Problem * len(problems))()
    for k, ((U, psi, m0), eta) in enumerate(zip(problems, outs)):
        dims = _dims_of_links(U, prec)
        nrhs, _ = _nrhs_of(psi, prec, LAYOUT2, 4)
        arr[k].lat = _lattice(dims)
        arr[k].U, arr[k].psi, arr[k].eta = U.data_ptr(), psi.data_ptr(), eta.data_ptr()
        arr[k].nrhs, arr[k].m0 = nrhs, float(m0)
    kind, g = ctypes.c_int(0), ctypes.c_int(0)
    _check(load().lqcd_autotune_batch(len(problems), arr, prec, int(reps), ctypes.byref(kind), ctypes.byref(g),
                                      _stream()))
    return {"kernel": kind.value, "grid": g.value}


def hbm_probe(a, b, c=None, kind="triad", reps=5):
    """Mean time (ms) of a copy (b = a) or triad (a = b + s c) over float64 device tensors."""
    n = a.numel()
    ms = ctypes.c_double(0.0)
    k = 0 if kind == "copy" else 1
    _check(load().lqcd_hbm_probe(k, a.data_ptr(), b.data_ptr(), None if c is None else c.data_ptr(), n, int(reps),
                                 ctypes.byref(ms), _stream()))
    return ms.value


def gmres_solve_batch(problems, work=None, **kw):
    """Solve D_k x_k = b_k for a list of (U_k, b_k, m0_k) on independent
    lattices (FP64, rhs-innermost full-lattice blocks) with one lock-step
    batched GMRES.  Returns (list of x_k, list of per-problem stats dicts, status)."""
    import torch

    if not 1 <= len(problems) <= MAX_BATCH:
        raise ValueError(f"need 1..{MAX_BATCH} problems")
    p = solver_params(**kw)
    arr = (Problem * len(problems))()
    xs = []
    nrhs_list = []
    for k, (U, b, m0) in enumerate(problems):
        if U.dtype != torch.complex128 or b.dtype != torch.complex128:
            raise TypeError("gmres_solve_batch takes complex128 U and b")
        dims = _dims_of_links(U, F64)
        nrhs, sdims = _nrhs_of(b, F64, LAYOUT2, 4)
        if tuple(sdims) != tuple(dims):
            raise ValueError(f"problem {k}: source lattice {sdims} does not match {dims}")
        x = torch.empty_like(b)
        _check_device(U, b, x)
        arr[k].lat = _lattice(dims)
        arr[k].U, arr[k].psi, arr[k].eta = U.data_ptr(), b.data_ptr(), x.data_ptr()
        arr[k].nrhs, arr[k].m0 = nrhs, float(m0)
        xs.append(x)
        nrhs_list.append(nrhs)
    need = int(load().gmres_workspace_bytes_batch(len(problems), arr, ctypes.byref(p)))
    if need == 0:
        raise ValueError("invalid batch")
    if work is None or work.numel() < need:
        work = torch.empty(need, dtype=torch.uint8, device=problems[0][1].device)
    st = (RhsStats * sum(nrhs_list))()
    rc = _check(load().gmres_solve_batch(len(problems), arr, ctypes.byref(p), work.data_ptr(), work.numel(), st,
                                         _stream()))
    stats, off = [], 0
    for n in nrhs_list:
        stats.append({k: np.array([getattr(s, k) for s in st[off:off + n]]) for k, _ in RhsStats._fields_})
        off += n
    return xs, stats, rc
