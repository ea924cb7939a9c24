"""Test-side conversions between the oracle's array shapes and the tensors
the binding takes (layout permutations and precision casts only)."""
import numpy as np

import paper_2601_05816_amd as lq


def to_layout_np(block, layout):
    """oracle block (nrhs, *sites, 4, 3) -> numpy array in `layout`."""
    ns = block.ndim - 3  # number of site axes
    if layout == lq.RHS_OUTER:
        return np.ascontiguousarray(block)
    if layout == lq.LAYOUT1:
        return np.ascontiguousarray(np.moveaxis(block, 0, ns))
    return np.ascontiguousarray(np.moveaxis(block, 0, -1))


def from_layout_np(arr, layout, ns):
    if layout == lq.RHS_OUTER:
        return arr
    if layout == lq.LAYOUT1:
        return np.moveaxis(arr, ns, 0)
    return np.moveaxis(arr, -1, 0)


def to_dev(arr, prec, device="cuda"):
    import torch

    if prec == lq.F64:
        return torch.from_numpy(np.ascontiguousarray(arr.astype(np.complex128))).to(device)
    if prec == lq.F32:
        return torch.from_numpy(np.ascontiguousarray(arr.astype(np.complex64))).to(device)
    h = np.stack([arr.real, arr.imag], axis=-1).astype(np.float16)
    return torch.from_numpy(np.ascontiguousarray(h)).to(device)


def from_dev(t, prec):
    a = t.cpu().numpy()
    if prec == lq.F16:
        a = a.astype(np.float64)
        return a[..., 0] + 1j * a[..., 1]
    return a.astype(np.complex128)


def rounded(arr, prec):
    """The values a precision actually stores (what the GPU reads)."""
    if prec == lq.F64:
        return arr.astype(np.complex128)
    if prec == lq.F32:
        return arr.astype(np.complex64).astype(np.complex128)
    re = arr.real.astype(np.float16).astype(np.float64)
    im = arr.imag.astype(np.float16).astype(np.float64)
    return re + 1j * im


def rel_err_per_rhs(got, want):
    n = got.shape[0]
    g = got.reshape(n, -1)
    w = want.reshape(n, -1)
    return np.linalg.norm(g - w, axis=1) / np.linalg.norm(w, axis=1)


def neighbourhood(coord, dims, lo=-1, hi=1):
    """Site numbers of the block of offsets lo..hi (per direction) around
    coord on the periodic lattice dims, in the block's own row-major order."""
    r = np.arange(lo, hi + 1)
    offs = np.stack(np.meshgrid(r, r, r, r, indexing="ij"), axis=-1).reshape(-1, 4)
    pts = (np.asarray(coord)[None, :] + offs) % np.asarray(dims)[None, :]
    return np.ravel_multi_index(pts.T, dims)


def apply_gpu(U, psi, m0, layout, prec, dagger=False):
    """dirac_apply on oracle-shaped host arrays (nrhs first), result back in that shape."""
    Ud = to_dev(U, prec)
    pd = to_dev(to_layout_np(psi, layout), prec)
    out = lq.dirac_apply(Ud, pd, m0, layout=layout, dagger=dagger)
    return from_layout_np(from_dev(out, prec), layout, 4)


def apply_eo_gpu(U, psi_e, m0, layout, prec, dagger=False):
    """dirac_apply_eo on an oracle-shaped even half-lattice block."""
    Ud = to_dev(U, prec)
    pd = to_dev(to_layout_np(psi_e, layout), prec)
    out = lq.dirac_apply_eo(Ud, pd, m0, layout=layout, dagger=dagger)
    return from_layout_np(from_dev(out, prec), layout, 1)
