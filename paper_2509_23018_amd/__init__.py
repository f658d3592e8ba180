"""Python binding of libgw, the MI355X (gfx950) chi0 library.

Argument marshalling only: every step of MTXEL, the energy factor, the CHI0
contraction and the adjoint runs in the HIP kernels of ``libgw.so``; PyTorch
provides device memory and the stream.  There is no CPU path: if the library
is missing, or a tensor is not on a ROCm device, the call raises.

Entry points mirror the C ABI (``include/gw.h``):

* :func:`gw_mtxel`  -- plane-wave matrix elements of pair densities;
* :func:`gw_chi0`   -- polarizability chi0(z) for one or many problems;
* :func:`gw_chi0_backward` -- adjoint of ``gw_chi0``;
* :class:`Chi0` / :func:`chi0` -- ``torch.autograd.Function`` wrapper.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime that libgw binds to)

__all__ = [
    "GWError", "lib", "library_path", "GW_FP64", "GW_FP32", "GW_SPLIT_BF16", "GW_SPLIT_FP16",
    "GW_SPLIT_FP16X9",
    "GW_FLAG_NO_HERMITIAN", "GW_FLAG_ACCUMULATE", "GW_FLAG_GRAPH", "GW_FLAG_AUTOTUNE",
    "GW_FLAG_FP64_TILE128", "GW_FLAG_ACC_HERMITIAN",
    "Chi0Problem", "gw_mtxel", "gw_chi0", "gw_chi0_fixed", "workspace_bytes", "new_workspace",
    "pseudobands_workspace_bytes",
    "gw_chi0_backward", "gw_pseudobands", "gw_subspace_basis", "gw_chi0_subspace",
    "subspace_basis_workspace_bytes", "chi0_subspace_workspace_bytes", "gw_zgemm", "gw_heev",
    "gw_epsinv", "gw_gpp_sigma", "gw_chi0_keep_m", "gw_chi0_from_m", "Chi0", "chi0", "release",
    "profile_enable",
    "profile_reset",
    "profile_read",
]

GW_FP64, GW_FP32, GW_SPLIT_BF16, GW_SPLIT_FP16, GW_SPLIT_FP16X9 = 0, 1, 2, 3, 4
GW_FLAG_NO_HERMITIAN = 1 << 0
GW_FLAG_ACCUMULATE = 1 << 1
GW_FLAG_GRAPH = 1 << 2
GW_FLAG_AUTOTUNE = 1 << 3
GW_FLAG_FP64_TILE128 = 1 << 4
GW_FLAG_ACC_HERMITIAN = 1 << 5
PRECISIONS = {"fp64": GW_FP64, "fp32": GW_FP32, "split_bf16": GW_SPLIT_BF16,
              "split_fp16": GW_SPLIT_FP16, "split_fp16x9": GW_SPLIT_FP16X9}

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libgw.so")


class GWError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libgw status {status}: {msg}")
        self.status = status


class _Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("volume", ctypes.c_double)]


class _Problem(ctypes.Structure):
    _fields_ = [
        ("grid", _Grid),
        ("psi_v", ctypes.c_void_p), ("nv", ctypes.c_int32),
        ("psi_c", ctypes.c_void_p), ("nc", ctypes.c_int32),
        ("e_v", ctypes.c_void_p), ("e_c", ctypes.c_void_p),
        ("gvec", ctypes.c_void_p), ("ng", ctypes.c_int32),
        ("z", ctypes.c_void_p), ("nz", ctypes.c_int32),
        ("chi", ctypes.c_void_p),
    ]


class _Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("n_slices", ctypes.c_int32),
                ("pair_chunk", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("spin", ctypes.c_double), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t)]


class _C128(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class _DiagOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("guard", ctypes.c_int32), ("max_degree", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("weight", ctypes.c_void_p),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t)]


class _DiagInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("degree", ctypes.c_int32),
                ("residual", ctypes.c_double), ("bound", ctypes.c_double),
                ("sweeps", ctypes.c_int32)]


_LIB = None


def lib() -> ctypes.CDLL:
    """Load libgw.so (built in-tree by ``paper_2509_23018_amd.build``)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(library_path):
            raise RuntimeError(f"{library_path} is not built; run "
                               "`python -m paper_2509_23018_amd.build` first")
        L = ctypes.CDLL(library_path)
        L.gw_mtxel.restype = ctypes.c_int32
        L.gw_mtxel.argtypes = [ctypes.POINTER(_Grid), ctypes.c_void_p, ctypes.c_int32,
                               ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                               ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
        L.gw_chi0.restype = ctypes.c_int32
        L.gw_chi0.argtypes = [ctypes.POINTER(_Problem), ctypes.c_int32, ctypes.POINTER(_Opts),
                              ctypes.c_void_p]
        L.gw_chi0_backward.restype = ctypes.c_int32
        L.gw_chi0_backward.argtypes = [ctypes.POINTER(_Problem), ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.POINTER(_Opts), ctypes.c_void_p]
        L.gw_pseudobands.restype = ctypes.c_int32
        L.gw_pseudobands.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                     ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                     ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                     ctypes.c_void_p]
        L.gw_pseudobands_workspace_bytes.restype = ctypes.c_size_t
        L.gw_pseudobands_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int64,
                                                     ctypes.c_int32, ctypes.c_int32]
        L.gw_workspace_bytes.restype = ctypes.c_size_t
        L.gw_workspace_bytes.argtypes = [ctypes.POINTER(_Problem), ctypes.c_int32,
                                         ctypes.POINTER(_Opts), ctypes.c_int32]
        L.gw_subspace_basis.restype = ctypes.c_int32
        L.gw_subspace_basis.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.POINTER(_DiagOpts), ctypes.POINTER(_DiagInfo),
                                        ctypes.c_void_p]
        L.gw_subspace_basis_workspace_bytes.restype = ctypes.c_size_t
        L.gw_subspace_basis_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32,
                                                        ctypes.POINTER(_DiagOpts)]
        L.gw_chi0_subspace.restype = ctypes.c_int32
        L.gw_chi0_subspace.argtypes = [ctypes.POINTER(_Problem), ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_int32, ctypes.POINTER(_Opts), ctypes.c_void_p]
        L.gw_chi0_subspace_workspace_bytes.restype = ctypes.c_size_t
        L.gw_chi0_subspace_workspace_bytes.argtypes = [ctypes.POINTER(_Problem), ctypes.c_int32,
                                                       ctypes.POINTER(_Opts)]
        L.gw_chi0_keep_m.restype = ctypes.c_int32
        L.gw_chi0_keep_m.argtypes = [ctypes.POINTER(_Problem), ctypes.c_void_p,
                                     ctypes.POINTER(_Opts), ctypes.c_void_p]
        L.gw_chi0_from_m.restype = ctypes.c_int32
        L.gw_chi0_from_m.argtypes = [ctypes.POINTER(_Problem), ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(_Opts),
                                     ctypes.c_void_p]
        L.gw_chi0_backward_from_m.restype = ctypes.c_int32
        L.gw_chi0_backward_from_m.argtypes = [ctypes.POINTER(_Problem), ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.POINTER(_Opts), ctypes.c_void_p]
        L.gw_chi0_backward_from_m_workspace_bytes.restype = ctypes.c_size_t
        L.gw_chi0_backward_from_m_workspace_bytes.argtypes = [ctypes.POINTER(_Problem),
                                                              ctypes.POINTER(_Opts)]
        L.gw_chi0_from_m_workspace_bytes.restype = ctypes.c_size_t
        L.gw_chi0_from_m_workspace_bytes.argtypes = [ctypes.POINTER(_Problem), ctypes.c_int32,
                                                     ctypes.POINTER(_Opts)]
        L.gw_zgemm.restype = ctypes.c_int32
        L.gw_zgemm.argtypes = [ctypes.c_char, ctypes.c_char, ctypes.c_int32, ctypes.c_int32,
                               ctypes.c_int32, _C128, ctypes.c_void_p, ctypes.c_int64,
                               ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                               _C128, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                               ctypes.c_int32, ctypes.c_void_p]
        L.gw_heev.restype = ctypes.c_int32
        L.gw_heev.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                              ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p,
                              ctypes.c_size_t, ctypes.c_void_p]
        L.gw_heev_workspace_bytes.restype = ctypes.c_size_t
        L.gw_heev_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32]
        L.gw_chi0_fixed.restype = ctypes.c_int32
        L.gw_chi0_fixed.argtypes = [ctypes.POINTER(_Problem), ctypes.POINTER(_Opts),
                                    ctypes.c_void_p]
        L.gw_chi0_fixed_scratch_bytes.restype = ctypes.c_size_t
        L.gw_chi0_fixed_scratch_bytes.argtypes = []
        L.gw_epsinv.restype = ctypes.c_int32
        L.gw_epsinv.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                ctypes.c_void_p]
        L.gw_epsinv_workspace_bytes.restype = ctypes.c_size_t
        L.gw_epsinv_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32]
        L.gw_gpp_sigma.restype = ctypes.c_int32
        L.gw_gpp_sigma.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        L.gw_gpp_sigma_workspace_bytes.restype = ctypes.c_size_t
        L.gw_gpp_sigma_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32,
                                                   ctypes.c_int32]
        L.gw_last_error.restype = ctypes.c_char_p
        L.gw_last_error.argtypes = []
        L.gw_release.restype = ctypes.c_int32
        L.gw_abi_version.restype = ctypes.c_int32
        L.gw_profile_enable.restype = ctypes.c_int32
        L.gw_profile_enable.argtypes = [ctypes.c_int32]
        L.gw_profile_read.restype = ctypes.c_int32
        L.gw_profile_read.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_double)]
        L.gw_profile_reset.restype = ctypes.c_int32
        _LIB = L
    return _LIB


def _check(status: int):
    if status != 0:
        raise GWError(status, lib().gw_last_error().decode())


def _stream(device: torch.device, stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return int(s.cuda_stream)


def _dev(t: torch.Tensor, name: str, dtype) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a ROCm device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _host_i32(g) -> np.ndarray:
    if isinstance(g, torch.Tensor):
        g = g.detach().cpu().numpy()
    return np.ascontiguousarray(np.asarray(g, dtype=np.int32).reshape(-1, 3))


def _host_c128(z) -> np.ndarray:
    if isinstance(z, torch.Tensor):
        z = z.detach().cpu().numpy()
    return np.ascontiguousarray(np.asarray(z, dtype=np.complex128).reshape(-1))


def _grid(n, volume) -> _Grid:
    g = _Grid()
    for i in range(3):
        g.n[i] = int(n[i])
    g.volume = float(volume)
    return g


def _workspace(ws):
    """(pointer, bytes) of a caller workspace: a device tensor or None."""
    if ws is None:
        return None, 0
    if not isinstance(ws, torch.Tensor) or ws.device.type != "cuda" or not ws.is_contiguous():
        raise TypeError("workspace must be a contiguous ROCm device tensor")
    return ws.data_ptr(), ws.numel() * ws.element_size()


def _opts(precision="fp64", n_slices=0, pair_chunk=4096, flags=0, spin=2.0,
          workspace=None) -> _Opts:
    o = _Opts()
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.n_slices = int(n_slices)
    o.pair_chunk = int(pair_chunk)
    o.flags = int(flags)
    o.spin = float(spin)
    o.workspace, o.workspace_bytes = _workspace(workspace)
    return o


def new_workspace(nbytes: int, device=None) -> torch.Tensor:
    """A device buffer usable as a caller workspace (torch allocations are
    at least 256-byte aligned)."""
    device = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    return torch.empty(max(1, int(nbytes)), dtype=torch.uint8, device=device)


def gw_mtxel(psi_v: torch.Tensor, psi_c: torch.Tensor, gvec, n, volume: float,
             pair_begin: int = 0, pair_count: Optional[int] = None,
             out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """M[k][i] = dV sum_r conj(psi_v[v]) psi_c[c] e^{+i G_i.r}, p = pair_begin + k = v*nc + c."""
    _dev(psi_v, "psi_v", torch.complex128)
    _dev(psi_c, "psi_c", torch.complex128)
    nv, nc = psi_v.shape[0], psi_c.shape[0]
    g = _host_i32(gvec)
    if pair_count is None:
        pair_count = nv * nc - pair_begin
    if out is None:
        out = torch.empty((pair_count, g.shape[0]), dtype=torch.complex128, device=psi_v.device)
    _dev(out, "out", torch.complex128)
    if out.numel() < pair_count * g.shape[0]:
        raise ValueError("out is too small")
    grid = _grid(n, volume)
    with torch.cuda.device(psi_v.device):
        _check(lib().gw_mtxel(ctypes.byref(grid), psi_v.data_ptr(), nv, psi_c.data_ptr(), nc,
                              g.ctypes.data, g.shape[0], int(pair_begin), int(pair_count),
                              out.data_ptr(), _stream(psi_v.device, stream)))
    return out


def pseudobands_workspace_bytes(nkeep: int, nidx: int, nslices: int, n_xi: int) -> int:
    return int(lib().gw_pseudobands_workspace_bytes(int(nkeep), int(nidx), int(nslices),
                                                    int(n_xi)))


def gw_pseudobands(psi: torch.Tensor, e: torch.Tensor, keep, slices, n_xi: int, theta,
                   stream=None, workspace=None):
    """Stochastic pseudobands: returns (psi_out, e_out) with the bands `keep`
    first, then n_xi random-phase combinations of each slice (a sequence of
    band-index arrays), with phases theta[s] of shape [n_xi][len(slices[s])]
    in turns."""
    _dev(psi, "psi", torch.complex128)
    _dev(e, "e", torch.float64)
    nb, nr = psi.shape[0], psi.shape[1]
    i32 = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.int64).reshape(-1), np.int32)
    k = i32(keep)
    sl = [np.asarray(x, dtype=np.int64).reshape(-1) for x in slices]
    idx = i32(np.concatenate(sl) if sl else np.zeros(0, np.int64))
    off = i32(np.concatenate([[0], np.cumsum([len(x) for x in sl])]))
    th = np.ascontiguousarray(np.concatenate(
        [np.asarray(t, dtype=np.float64).reshape(-1) for t in theta]) if sl else np.zeros(0))
    nout = len(k) + len(sl) * int(n_xi)
    out = torch.empty((nout, nr), dtype=torch.complex128, device=psi.device)
    out_e = torch.empty(nout, dtype=torch.float64, device=psi.device)
    with torch.cuda.device(psi.device):
        wp, wb = _workspace(workspace)
        _check(lib().gw_pseudobands(psi.data_ptr(), e.data_ptr(), nb, nr, k.ctypes.data, len(k),
                                    idx.ctypes.data, off.ctypes.data, len(sl), int(n_xi),
                                    th.ctypes.data, out.data_ptr(), out_e.data_ptr(), wp, wb,
                                    _stream(psi.device, stream)))
    return out, out_e


@dataclass
class Chi0Problem:
    """One chi0 problem on the device (psi, energies) with host G list and z."""
    n: Sequence[int]
    volume: float
    psi_v: torch.Tensor
    psi_c: torch.Tensor
    e_v: torch.Tensor
    e_c: torch.Tensor
    gvec: np.ndarray
    z: np.ndarray
    chi: Optional[torch.Tensor] = None

    def _fill(self, p: _Problem, keep: list, alloc_chi: bool = True):
        for name, t, dt in (("psi_v", self.psi_v, torch.complex128),
                            ("psi_c", self.psi_c, torch.complex128),
                            ("e_v", self.e_v, torch.float64), ("e_c", self.e_c, torch.float64)):
            _dev(t, name, dt)
        g, z = _host_i32(self.gvec), _host_c128(self.z)
        keep += [g, z]
        ng, nz = g.shape[0], z.shape[0]
        if self.chi is None and alloc_chi:
            self.chi = torch.empty((nz, ng, ng), dtype=torch.complex128, device=self.psi_v.device)
        if self.chi is not None:
            _dev(self.chi, "chi", torch.complex128)
            if tuple(self.chi.shape) != (nz, ng, ng):
                raise ValueError(f"chi must have shape {(nz, ng, ng)}")
        p.grid = _grid(self.n, self.volume)
        p.psi_v, p.nv = self.psi_v.data_ptr(), self.psi_v.shape[0]
        p.psi_c, p.nc = self.psi_c.data_ptr(), self.psi_c.shape[0]
        p.e_v, p.e_c = self.e_v.data_ptr(), self.e_c.data_ptr()
        p.gvec, p.ng = g.ctypes.data, ng
        p.z, p.nz = z.ctypes.data, nz
        p.chi = self.chi.data_ptr() if self.chi is not None else None


def workspace_bytes(problems, *, precision="fp64", n_slices=0, pair_chunk=4096, flags=0,
                    spin=2.0, backward=False) -> int:
    """Device scratch (bytes) gw_chi0 (or, with backward=True, gw_chi0_backward
    on the first problem) needs in a caller workspace for these arguments."""
    probs = [problems] if isinstance(problems, Chi0Problem) else list(problems)
    arr = (_Problem * max(1, len(probs)))()
    keep: list = []
    for i, pr in enumerate(probs):
        pr._fill(arr[i], keep, alloc_chi=not backward)
    o = _opts(precision, n_slices, pair_chunk, flags, spin)
    dev = probs[0].psi_v.device if probs else torch.device("cuda", torch.cuda.current_device())
    with torch.cuda.device(dev):
        n = lib().gw_workspace_bytes(arr, len(probs), ctypes.byref(o), 1 if backward else 0)
    if n == ctypes.c_size_t(-1).value:
        raise GWError(-1, lib().gw_last_error().decode())
    return int(n)


def gw_chi0(problems, *, precision="fp64", n_slices=0, pair_chunk=4096, flags=0, spin=2.0,
            stream=None, workspace=None):
    """Run gw_chi0 on one Chi0Problem or a list of them; returns the chi tensor(s)."""
    single = isinstance(problems, Chi0Problem)
    probs = [problems] if single else list(problems)
    arr = (_Problem * max(1, len(probs)))()
    keep: list = []
    for i, pr in enumerate(probs):
        pr._fill(arr[i], keep)
    o = _opts(precision, n_slices, pair_chunk, flags, spin, workspace)
    dev = probs[0].psi_v.device if probs else torch.device("cuda", torch.cuda.current_device())
    with torch.cuda.device(dev):
        _check(lib().gw_chi0(arr, len(probs), ctypes.byref(o), _stream(dev, stream)))
    return probs[0].chi if single else [p.chi for p in probs]


def gw_chi0_fixed(problem: Chi0Problem, *, precision="fp64", n_slices=0, pair_chunk=4096,
                  flags=0, spin=2.0, stream=None) -> torch.Tensor:
    """gw_chi0 of one problem through the library's fixed device scratch (no
    allocation; the problem's plan must exist, see include/gw.h)."""
    arr = _Problem()
    keep: list = []
    problem._fill(arr, keep)
    o = _opts(precision, n_slices, pair_chunk, flags, spin)
    with torch.cuda.device(problem.psi_v.device):
        _check(lib().gw_chi0_fixed(ctypes.byref(arr), ctypes.byref(o),
                                   _stream(problem.psi_v.device, stream)))
    return problem.chi


def gw_chi0_backward(problem: Chi0Problem, grad_chi: torch.Tensor, *, pair_chunk=4096,
                     spin=2.0, need=(True, True, True, True), stream=None, workspace=None,
                     m_keep: Optional[torch.Tensor] = None):
    """Returns (grad_psi_v, grad_psi_c, grad_e_v, grad_e_c); entries not in `need` are None.
    With m_keep (M from gw_chi0_keep_m with the same problem and pair_chunk) the
    adjoint reads M instead of recomputing it (gw_chi0_backward_from_m)."""
    pr = problem
    if m_keep is not None:
        _dev(m_keep, "m_keep", torch.complex128)
        npairs = pr.psi_v.shape[0] * pr.psi_c.shape[0]
        if tuple(m_keep.shape) != (npairs, int(np.asarray(pr.gvec).shape[0])):
            raise ValueError("m_keep must be [nv*nc, ng] as gw_chi0_keep_m returns it")
    _dev(grad_chi, "grad_chi", torch.complex128)
    p = _Problem()
    keep: list = []
    saved_chi = pr.chi
    pr.chi = grad_chi  # shape check only; the adjoint does not read chi
    try:
        pr._fill(p, keep)
    finally:
        pr.chi = saved_chi
    outs = [torch.empty_like(pr.psi_v) if need[0] else None,
            torch.empty_like(pr.psi_c) if need[1] else None,
            torch.empty_like(pr.e_v) if need[2] else None,
            torch.empty_like(pr.e_c) if need[3] else None]
    ptr = [o.data_ptr() if o is not None else None for o in outs]
    o = _opts("fp64", 0, pair_chunk, 0, spin, workspace)
    with torch.cuda.device(pr.psi_v.device):
        if m_keep is None:
            _check(lib().gw_chi0_backward(ctypes.byref(p), grad_chi.data_ptr(), ptr[0], ptr[1],
                                          ptr[2], ptr[3], ctypes.byref(o),
                                          _stream(pr.psi_v.device, stream)))
        else:
            _check(lib().gw_chi0_backward_from_m(ctypes.byref(p), m_keep.data_ptr(),
                                                 grad_chi.data_ptr(), ptr[0], ptr[1], ptr[2],
                                                 ptr[3], ctypes.byref(o),
                                                 _stream(pr.psi_v.device, stream)))
    return tuple(outs)


def _weight(weight, ng, device):
    if weight is None:
        return None
    _dev(weight, "weight", torch.float64)
    if tuple(weight.shape) != (ng,) or weight.device != device:
        raise ValueError(f"weight must be a float64 vector of {ng} on {device}")
    return weight.data_ptr()


def _diag_opts(tol=0.0, max_iter=0, guard=0, max_degree=0, seed=0, workspace=None, weight=None):
    o = _DiagOpts()
    o.tol, o.max_iter, o.guard, o.max_degree = float(tol), int(max_iter), int(guard), int(max_degree)
    o.seed = int(seed)
    o.weight = weight
    o.workspace, o.workspace_bytes = _workspace(workspace)
    return o


def subspace_basis_workspace_bytes(ng: int, n_eig: int, guard: int = 0,
                                   weighted: bool = False) -> int:
    o = _diag_opts(guard=guard, weight=1 if weighted else None)  # only tested for NULL
    return int(lib().gw_subspace_basis_workspace_bytes(int(ng), int(n_eig), ctypes.byref(o)))


def gw_subspace_basis(chi_static: torch.Tensor, n_eig: int, *, weight=None, tol=0.0, max_iter=0,
                      guard=0, max_degree=0, seed=0, workspace=None, stream=None):
    """Diag: (basis [ng, n_eig], eigenvalues [n_eig], info) of the Hermitian,
    negative semidefinite static polarizability chi_static [ng, ng], or of
    W chi W with W = diag(weight) (weight: float64 device vector [ng])."""
    _dev(chi_static, "chi_static", torch.complex128)
    ng = chi_static.shape[0]
    if tuple(chi_static.shape) != (ng, ng):
        raise ValueError("chi_static must be square")
    basis = torch.empty((ng, int(n_eig)), dtype=torch.complex128, device=chi_static.device)
    ev = torch.empty(int(n_eig), dtype=torch.float64, device=chi_static.device)
    o = _diag_opts(tol, max_iter, guard, max_degree, seed, workspace,
                   _weight(weight, ng, chi_static.device))
    info = _DiagInfo()
    with torch.cuda.device(chi_static.device):
        _check(lib().gw_subspace_basis(chi_static.data_ptr(), ng, int(n_eig), basis.data_ptr(),
                                       ev.data_ptr(), ctypes.byref(o), ctypes.byref(info),
                                       _stream(chi_static.device, stream)))
    return basis, ev, {"iterations": info.iterations, "degree": info.degree,
                       "residual": info.residual, "bound": info.bound, "sweeps": info.sweeps}


def chi0_subspace_workspace_bytes(problem, n_eig: int, *, precision="fp64", n_slices=0,
                                  pair_chunk=4096, flags=0, spin=2.0) -> int:
    arr = _Problem()
    keep: list = []
    problem._fill(arr, keep, alloc_chi=False)
    o = _opts(precision, n_slices, pair_chunk, flags, spin)
    with torch.cuda.device(problem.psi_v.device):
        n = lib().gw_chi0_subspace_workspace_bytes(ctypes.byref(arr), int(n_eig), ctypes.byref(o))
    if n == ctypes.c_size_t(-1).value:
        raise GWError(-1, lib().gw_last_error().decode())
    return int(n)


def gw_chi0_subspace(problem, basis: torch.Tensor, *, weight=None, precision="fp64", n_slices=0,
                     pair_chunk=4096, flags=0, spin=2.0, out=None, workspace=None, stream=None):
    """Transf + CHI-Freq (Eq. (6)): chi_BB'(z) [nz, n_eig, n_eig] of one problem
    in the subspace spanned by the columns of basis [ng, n_eig]; with weight
    [ng], C^H W chi W C."""
    _dev(basis, "basis", torch.complex128)
    ng = int(np.asarray(problem.gvec).shape[0])
    if basis.dim() != 2 or basis.shape[0] != ng or basis.shape[1] < 1:
        raise ValueError(f"basis must be [{ng}, n_eig] with n_eig >= 1")
    wp = _weight(weight, basis.shape[0], basis.device)
    n_eig = basis.shape[1]
    nz = _host_c128(problem.z).shape[0]
    if out is None:
        out = torch.empty((nz, n_eig, n_eig), dtype=torch.complex128, device=basis.device)
    _dev(out, "out", torch.complex128)
    if tuple(out.shape) != (nz, n_eig, n_eig):
        raise ValueError(f"out must have shape {(nz, n_eig, n_eig)}")
    arr = _Problem()
    keep: list = []
    problem._fill(arr, keep, alloc_chi=False)
    arr.chi = out.data_ptr()
    o = _opts(precision, n_slices, pair_chunk, flags, spin, workspace)
    with torch.cuda.device(basis.device):
        _check(lib().gw_chi0_subspace(ctypes.byref(arr), basis.data_ptr(), wp, int(n_eig),
                                      ctypes.byref(o), _stream(basis.device, stream)))
    return out


def gw_chi0_keep_m(problem: Chi0Problem, m_keep: Optional[torch.Tensor] = None, *,
                   precision="fp64", n_slices=0, pair_chunk=4096, flags=0, spin=2.0,
                   workspace=None, stream=None):
    """gw_chi0 of one problem that also keeps M of every pair (device
    [nv*nc, ng], in the order the call streams its chunks); returns
    (chi, m_keep)."""
    npairs = problem.psi_v.shape[0] * problem.psi_c.shape[0]
    ng = int(np.asarray(problem.gvec).shape[0])
    if m_keep is None:
        m_keep = torch.empty((npairs, ng), dtype=torch.complex128, device=problem.psi_v.device)
    _dev(m_keep, "m_keep", torch.complex128)
    if tuple(m_keep.shape) != (npairs, ng):
        raise ValueError(f"m_keep must have shape {(npairs, ng)}")
    arr = _Problem()
    keep: list = []
    problem._fill(arr, keep)
    o = _opts(precision, n_slices, pair_chunk, flags, spin, workspace)
    with torch.cuda.device(problem.psi_v.device):
        _check(lib().gw_chi0_keep_m(ctypes.byref(arr), m_keep.data_ptr(), ctypes.byref(o),
                                    _stream(problem.psi_v.device, stream)))
    return problem.chi, m_keep


def gw_chi0_from_m(problem: Chi0Problem, m_keep: torch.Tensor, basis: Optional[torch.Tensor] = None,
                   *, weight=None, precision="fp64", n_slices=0, pair_chunk=4096, flags=0,
                   spin=2.0, out=None, workspace=None, stream=None) -> torch.Tensor:
    """chi from M kept by gw_chi0_keep_m (same problem shape and pair_chunk):
    Eq. (4) [nz, ng, ng], or with basis [ng, n_eig] (and weight) Eq. (6)
    [nz, n_eig, n_eig]."""
    _dev(m_keep, "m_keep", torch.complex128)
    ng = int(np.asarray(problem.gvec).shape[0])
    nz = _host_c128(problem.z).shape[0]
    n_eig = 0
    wp = None
    if basis is not None:
        _dev(basis, "basis", torch.complex128)
        n_eig = basis.shape[1]
        if basis.dim() != 2 or basis.shape[0] != ng or n_eig < 1:
            raise ValueError(f"basis must be [{ng}, n_eig] with n_eig >= 1")
        wp = _weight(weight, basis.shape[0], basis.device)
    ncol = n_eig or ng
    if out is None:
        out = torch.empty((nz, ncol, ncol), dtype=torch.complex128, device=m_keep.device)
    _dev(out, "out", torch.complex128)
    if tuple(out.shape) != (nz, ncol, ncol):
        raise ValueError(f"out must have shape {(nz, ncol, ncol)}")
    arr = _Problem()
    keep: list = []
    problem._fill(arr, keep, alloc_chi=False)
    arr.chi = out.data_ptr()
    o = _opts(precision, n_slices, pair_chunk, flags, spin, workspace)
    with torch.cuda.device(m_keep.device):
        _check(lib().gw_chi0_from_m(ctypes.byref(arr), m_keep.data_ptr(),
                                    basis.data_ptr() if basis is not None else None, wp,
                                    int(n_eig), ctypes.byref(o), _stream(m_keep.device, stream)))
    return out


def _c128(x) -> _C128:
    x = complex(x)
    return _C128(x.real, x.imag)


def gw_zgemm(opa: str, opb: str, a: torch.Tensor, b: torch.Tensor, *, alpha=1.0, beta=0.0,
             c: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """C = alpha op(A) op(B) + beta C for complex128 device matrices [m, k]
    (or batches [batch, m, k]); op in 'N', 'T', 'C'."""
    _dev(a, "a", torch.complex128)
    _dev(b, "b", torch.complex128)
    batched = a.dim() == 3
    A = a if batched else a[None]
    B = b if batched else b[None]
    if A.shape[0] != B.shape[0]:
        raise ValueError("batch sizes differ")
    m = A.shape[1] if opa.upper() == "N" else A.shape[2]
    k = A.shape[2] if opa.upper() == "N" else A.shape[1]
    kb = B.shape[1] if opb.upper() == "N" else B.shape[2]
    n = B.shape[2] if opb.upper() == "N" else B.shape[1]
    if k != kb:
        raise ValueError("inner dimensions differ")
    batch = A.shape[0]
    if c is None:
        c = torch.zeros((batch, m, n) if batched else (m, n), dtype=torch.complex128,
                        device=a.device)
    _dev(c, "c", torch.complex128)
    with torch.cuda.device(a.device):
        _check(lib().gw_zgemm(opa.encode(), opb.encode(), m, n, k, _c128(alpha), A.data_ptr(),
                              A.shape[2], A.shape[1] * A.shape[2], B.data_ptr(), B.shape[2],
                              B.shape[1] * B.shape[2], _c128(beta), c.data_ptr(), n, m * n,
                              batch, _stream(a.device, stream)))
    return c


def gw_heev(a: torch.Tensor, *, tol=0.0, workspace=None, stream=None):
    """(w, v): eigenvalues (increasing) and eigenvector columns of Hermitian
    a [n, n] or [batch, n, n] (Jacobi rotations on the device)."""
    _dev(a, "a", torch.complex128)
    batched = a.dim() == 3
    A = a if batched else a[None]
    batch, n = A.shape[0], A.shape[1]
    w = torch.empty((batch, n), dtype=torch.float64, device=a.device)
    v = torch.empty((batch, n, n), dtype=torch.complex128, device=a.device)
    wp, wb = _workspace(workspace)
    with torch.cuda.device(a.device):
        _check(lib().gw_heev(A.data_ptr(), n, batch, w.data_ptr(), v.data_ptr(), float(tol), wp,
                             wb, _stream(a.device, stream)))
    return (w, v) if batched else (w[0], v[0])


def gw_epsinv(chi: torch.Tensor, vcoul: torch.Tensor, *, out=None, workspace=None,
              stream=None) -> torch.Tensor:
    """eps^-1(z) = [I - v chi(z)]^-1 (Eq. (3)) for chi [nz, ng, ng] (or
    [ng, ng]) and the Coulomb diagonal vcoul [ng], on the device."""
    _dev(chi, "chi", torch.complex128)
    _dev(vcoul, "vcoul", torch.float64)
    single = chi.dim() == 2
    c = chi[None] if single else chi
    nz, ng = c.shape[0], c.shape[1]
    if c.shape[2] != ng or vcoul.shape != (ng,):
        raise ValueError("chi must be [nz, ng, ng] and vcoul [ng]")
    if out is None:
        out = torch.empty_like(c)
    _dev(out, "out", torch.complex128)
    wp, wb = _workspace(workspace)
    with torch.cuda.device(chi.device):
        _check(lib().gw_epsinv(c.data_ptr(), ng, nz, vcoul.data_ptr(), out.data_ptr(), wp, wb,
                               _stream(chi.device, stream)))
    return out[0] if single else out


def gw_gpp_sigma(m: torch.Tensor, e_n, occupied, energies, omega2: torch.Tensor,
                 wtilde: torch.Tensor, vcoul: torch.Tensor, *, out=None, workspace=None,
                 stream=None) -> torch.Tensor:
    """Full GPP self-energy matrix Sigma[e, l, m] on the energy grid: m
    [nb, ns, ng] device, e_n / occupied [nb] host, energies [ne] host complex,
    omega2 [ng, ng], wtilde [ng, ng], vcoul [ng] device."""
    _dev(m, "m", torch.complex128)
    _dev(omega2, "omega2", torch.complex128)
    _dev(wtilde, "wtilde", torch.float64)
    _dev(vcoul, "vcoul", torch.float64)
    nb, ns, ng = m.shape
    en = np.ascontiguousarray(np.asarray(e_n, dtype=np.float64).reshape(-1))
    oc = np.ascontiguousarray(np.asarray(occupied, dtype=np.int32).reshape(-1))
    ee = _host_c128(energies)
    if en.shape[0] != nb or oc.shape[0] != nb:
        raise ValueError("e_n and occupied must have one entry per band")
    if omega2.shape != (ng, ng) or wtilde.shape != (ng, ng) or vcoul.shape != (ng,):
        raise ValueError("omega2, wtilde must be [ng, ng] and vcoul [ng]")
    if out is None:
        out = torch.empty((ee.shape[0], ns, ns), dtype=torch.complex128, device=m.device)
    _dev(out, "out", torch.complex128)
    wp, wb = _workspace(workspace)
    with torch.cuda.device(m.device):
        _check(lib().gw_gpp_sigma(m.data_ptr(), nb, ns, ng, en.ctypes.data, oc.ctypes.data,
                                  ee.ctypes.data, ee.shape[0], omega2.data_ptr(),
                                  wtilde.data_ptr(), vcoul.data_ptr(), out.data_ptr(), wp, wb,
                                  _stream(m.device, stream)))
    return out


class Chi0(torch.autograd.Function):
    """chi0(psi_v, psi_c, e_v, e_c) with a hand-written adjoint (gw_chi0_backward).

    Gradients follow PyTorch's complex convention.  The G list, frequencies,
    grid and options are non-differentiable constants.  With keep_m the
    forward keeps M of every pair (nv*nc*ng complex values of device memory)
    and the adjoint reads it instead of recomputing it."""

    @staticmethod
    def forward(ctx, psi_v, psi_c, e_v, e_c, gvec, z, n, volume, pair_chunk=4096, spin=2.0,
                precision="fp64", n_slices=0, keep_m=False):
        pr = Chi0Problem(n=n, volume=volume, psi_v=psi_v.contiguous(), psi_c=psi_c.contiguous(),
                         e_v=e_v.contiguous(), e_c=e_c.contiguous(), gvec=_host_i32(gvec),
                         z=_host_c128(z))
        ctx.m_keep = None
        if keep_m:
            chi, ctx.m_keep = gw_chi0_keep_m(pr, precision=precision, n_slices=n_slices,
                                             pair_chunk=pair_chunk, spin=spin)
        else:
            chi = gw_chi0(pr, precision=precision, n_slices=n_slices, pair_chunk=pair_chunk,
                          spin=spin)
        ctx.save_for_backward(pr.psi_v, pr.psi_c, pr.e_v, pr.e_c)
        ctx.meta = (pr.gvec, pr.z, tuple(n), volume, pair_chunk, spin)
        return chi

    @staticmethod
    def backward(ctx, grad_chi):
        psi_v, psi_c, e_v, e_c = ctx.saved_tensors
        gvec, z, n, volume, pair_chunk, spin = ctx.meta
        pr = Chi0Problem(n=n, volume=volume, psi_v=psi_v, psi_c=psi_c, e_v=e_v, e_c=e_c,
                         gvec=gvec, z=z)
        need = tuple(bool(x) for x in ctx.needs_input_grad[:4])
        g = gw_chi0_backward(pr, grad_chi.contiguous(), pair_chunk=pair_chunk, spin=spin,
                             need=need, m_keep=ctx.m_keep)
        ctx.m_keep = None
        return (*g, None, None, None, None, None, None, None, None, None)


def chi0(psi_v, psi_c, e_v, e_c, gvec, z, n, volume, *, pair_chunk=4096, spin=2.0,
         precision="fp64", n_slices=0, keep_m=False):
    return Chi0.apply(psi_v, psi_c, e_v, e_c, gvec, z, n, volume, pair_chunk, spin, precision,
                      n_slices, keep_m)


def release():
    _check(lib().gw_release())


def profile_enable(on: bool = True):
    """Record HIP events around every library launch (see include/gw.h)."""
    _check(lib().gw_profile_enable(1 if on else 0))


def profile_reset():
    _check(lib().gw_profile_reset())


def profile_read(kernel: str):
    """(launches, total_ms) recorded for `kernel` since the last reset."""
    n = ctypes.c_int64(0)
    t = ctypes.c_double(0.0)
    _check(lib().gw_profile_read(kernel.encode(), ctypes.byref(n), ctypes.byref(t)))
    return int(n.value), float(t.value)
