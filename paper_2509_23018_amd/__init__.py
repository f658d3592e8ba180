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
    "GW_FLAG_NO_HERMITIAN", "GW_FLAG_ACCUMULATE", "GW_FLAG_GRAPH", "GW_FLAG_AUTOTUNE",
    "GW_FLAG_FP64_TILE128",
    "Chi0Problem", "gw_mtxel", "gw_chi0",
    "gw_chi0_backward", "gw_pseudobands", "Chi0", "chi0", "release", "profile_enable",
    "profile_reset",
    "profile_read",
]

GW_FP64, GW_FP32, GW_SPLIT_BF16, GW_SPLIT_FP16 = 0, 1, 2, 3
GW_FLAG_NO_HERMITIAN = 1 << 0
GW_FLAG_ACCUMULATE = 1 << 1
GW_FLAG_GRAPH = 1 << 2
GW_FLAG_AUTOTUNE = 1 << 3
GW_FLAG_FP64_TILE128 = 1 << 4
PRECISIONS = {"fp64": GW_FP64, "fp32": GW_FP32, "split_bf16": GW_SPLIT_BF16,
              "split_fp16": GW_SPLIT_FP16}

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
                ("spin", ctypes.c_double)]


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
                                     ctypes.c_void_p, ctypes.c_void_p]
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


def _opts(precision="fp64", n_slices=0, pair_chunk=4096, flags=0, spin=2.0) -> _Opts:
    o = _Opts()
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.n_slices = int(n_slices)
    o.pair_chunk = int(pair_chunk)
    o.flags = int(flags)
    o.spin = float(spin)
    return o


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


def gw_pseudobands(psi: torch.Tensor, e: torch.Tensor, keep, slices, n_xi: int, theta,
                   stream=None):
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
        _check(lib().gw_pseudobands(psi.data_ptr(), e.data_ptr(), nb, nr, k.ctypes.data, len(k),
                                    idx.ctypes.data, off.ctypes.data, len(sl), int(n_xi),
                                    th.ctypes.data, out.data_ptr(), out_e.data_ptr(),
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

    def _fill(self, p: _Problem, keep: list):
        for name, t, dt in (("psi_v", self.psi_v, torch.complex128),
                            ("psi_c", self.psi_c, torch.complex128),
                            ("e_v", self.e_v, torch.float64), ("e_c", self.e_c, torch.float64)):
            _dev(t, name, dt)
        g, z = _host_i32(self.gvec), _host_c128(self.z)
        keep += [g, z]
        ng, nz = g.shape[0], z.shape[0]
        if self.chi is None:
            self.chi = torch.empty((nz, ng, ng), dtype=torch.complex128, device=self.psi_v.device)
        _dev(self.chi, "chi", torch.complex128)
        if tuple(self.chi.shape) != (nz, ng, ng):
            raise ValueError(f"chi must have shape {(nz, ng, ng)}")
        p.grid = _grid(self.n, self.volume)
        p.psi_v, p.nv = self.psi_v.data_ptr(), self.psi_v.shape[0]
        p.psi_c, p.nc = self.psi_c.data_ptr(), self.psi_c.shape[0]
        p.e_v, p.e_c = self.e_v.data_ptr(), self.e_c.data_ptr()
        p.gvec, p.ng = g.ctypes.data, ng
        p.z, p.nz = z.ctypes.data, nz
        p.chi = self.chi.data_ptr()


def gw_chi0(problems, *, precision="fp64", n_slices=0, pair_chunk=4096, flags=0, spin=2.0,
            stream=None):
    """Run gw_chi0 on one Chi0Problem or a list of them; returns the chi tensor(s)."""
    single = isinstance(problems, Chi0Problem)
    probs = [problems] if single else list(problems)
    arr = (_Problem * max(1, len(probs)))()
    keep: list = []
    for i, pr in enumerate(probs):
        pr._fill(arr[i], keep)
    o = _opts(precision, n_slices, pair_chunk, flags, spin)
    dev = probs[0].psi_v.device if probs else torch.device("cuda", torch.cuda.current_device())
    with torch.cuda.device(dev):
        _check(lib().gw_chi0(arr, len(probs), ctypes.byref(o), _stream(dev, stream)))
    return probs[0].chi if single else [p.chi for p in probs]


def gw_chi0_backward(problem: Chi0Problem, grad_chi: torch.Tensor, *, pair_chunk=4096,
                     spin=2.0, need=(True, True, True, True), stream=None):
    """Returns (grad_psi_v, grad_psi_c, grad_e_v, grad_e_c); entries not in `need` are None."""
    pr = problem
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
    o = _opts("fp64", 0, pair_chunk, 0, spin)
    with torch.cuda.device(pr.psi_v.device):
        _check(lib().gw_chi0_backward(ctypes.byref(p), grad_chi.data_ptr(), ptr[0], ptr[1], ptr[2],
                                      ptr[3], ctypes.byref(o), _stream(pr.psi_v.device, stream)))
    return tuple(outs)


class Chi0(torch.autograd.Function):
    """chi0(psi_v, psi_c, e_v, e_c) with a hand-written adjoint (gw_chi0_backward).

    Gradients follow PyTorch's complex convention.  The G list, frequencies,
    grid and options are non-differentiable constants."""

    @staticmethod
    def forward(ctx, psi_v, psi_c, e_v, e_c, gvec, z, n, volume, pair_chunk=4096, spin=2.0,
                precision="fp64", n_slices=0):
        pr = Chi0Problem(n=n, volume=volume, psi_v=psi_v.contiguous(), psi_c=psi_c.contiguous(),
                         e_v=e_v.contiguous(), e_c=e_c.contiguous(), gvec=_host_i32(gvec),
                         z=_host_c128(z))
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
                             need=need)
        return (*g, None, None, None, None, None, None, None, None)


def chi0(psi_v, psi_c, e_v, e_c, gvec, z, n, volume, *, pair_chunk=4096, spin=2.0,
         precision="fp64", n_slices=0):
    return Chi0.apply(psi_v, psi_c, e_v, e_c, gvec, z, n, volume, pair_chunk, spin, precision,
                      n_slices)


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
