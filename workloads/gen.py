"""Seeded input recipes for the chi0 build (input preparation only).

Conventions (the paper's statement of the problem, Overview section and
Eq. (4); the concrete sizes are the five workloads of the benchmark):

* cubic cell of edge ``L = 10`` bohr, volume ``Omega = L**3``;
* FFT grid ``N1 x N2 x N3``; a real-space array is stored row-major with the
  third index fastest, ``r = (j1*N2 + j2)*N3 + j3``;
* wavefunctions are complex128 ``[N_b][N1*N2*N3]``, valence rows first, with
  iid N(0,1) real and imaginary parts, made orthonormal on the grid in band
  order (Gram-Schmidt), i.e. ``dV * sum_r conj(psi_m) psi_n = delta_mn`` with
  ``dV = Omega / (N1*N2*N3)``;
* valence energies uniform in [-0.4, 0] Ha, conduction energies uniform in
  [0.05, 1.1] Ha;
* the G-sphere is the complete set of integer Miller triples with
  ``|g|^2 <= R^2``, ordered by (|g|^2, lexicographic g);
* frequencies are complex numbers ``z``: ``omega + i*eta`` on the real axis,
  ``i*omega`` on the imaginary axis, ``0`` for the static case.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg

CELL_L = 10.0          # bohr
SPIN = 2.0             # spin factor of Eq. (4)

# (grid, N_v, N_c, R^2 of the G-sphere, frequency recipe, pair chunk)
CONFIG_SHAPES = {
    0: dict(n=(16, 16, 16), nv=4, nc=28, r2=10, freq=("static", 1), pair_chunk=4096),
    1: dict(n=(48, 48, 48), nv=64, nc=960, r2=61, freq=("real", 4), pair_chunk=4096),
    2: dict(n=(72, 72, 72), nv=256, nc=3840, r2=126, freq=("imag", 8), pair_chunk=4096),
    3: dict(n=(32, 32, 32), nv=32, nc=480, r2=42, freq=("static", 1), pair_chunk=4096),
}


@dataclass
class Problem:
    """One chi0 problem (one q-point): inputs only."""
    n: tuple
    volume: float
    psi_v: np.ndarray          # complex128 [nv, N_r]
    psi_c: np.ndarray          # complex128 [nc, N_r]
    e_v: np.ndarray            # float64 [nv]
    e_c: np.ndarray            # float64 [nc]
    gvec: np.ndarray           # int32 [ng, 3]
    z: np.ndarray              # complex128 [nz]
    spin: float = SPIN
    pair_chunk: int = 4096
    meta: dict = field(default_factory=dict)

    @property
    def nv(self):
        return self.psi_v.shape[0]

    @property
    def nc(self):
        return self.psi_c.shape[0]

    @property
    def ng(self):
        return self.gvec.shape[0]

    @property
    def npairs(self):
        return self.nv * self.nc

    @property
    def nr(self):
        return int(np.prod(self.n))


def gsphere(r2: int) -> np.ndarray:
    """All integer g with |g|^2 <= r2, ordered by (|g|^2, g lexicographic)."""
    r = int(np.floor(np.sqrt(r2)))
    ax = np.arange(-r, r + 1)
    g = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1).reshape(-1, 3)
    n2 = (g * g).sum(1)
    g, n2 = g[n2 <= r2], n2[n2 <= r2]
    order = np.lexsort((g[:, 2], g[:, 1], g[:, 0], n2))
    return np.ascontiguousarray(g[order], dtype=np.int32)


def gsphere_shifted(q, count: int) -> np.ndarray:
    """The ``count`` integer g with the smallest |q+g|^2 (q in reciprocal-lattice
    units of the cubic cell), ties broken lexicographically in g."""
    q = np.asarray(q, dtype=np.float64)
    r = int(np.ceil((3.0 * count / (4.0 * np.pi)) ** (1.0 / 3.0))) + 3
    ax = np.arange(-r, r + 1)
    g = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1).reshape(-1, 3)
    k2 = ((g + q[None, :]) ** 2).sum(1)
    order = np.lexsort((g[:, 2], g[:, 1], g[:, 0], k2))[:count]
    return np.ascontiguousarray(g[order], dtype=np.int32)


def orthonormal_bands(rng: np.random.Generator, nb: int, n, volume: float,
                      orthonormalize: bool = True) -> np.ndarray:
    """Draw ``nb`` complex Gaussian bands on the grid and orthonormalise them
    in band order (two passes of Cholesky-QR, which equals Gram-Schmidt with a
    positive-diagonal R in exact arithmetic)."""
    nr = int(np.prod(n))
    psi = rng.standard_normal((nb, nr)) + 1j * rng.standard_normal((nb, nr))
    if not orthonormalize or nb == 0:
        return psi
    dv = volume / nr
    for _ in range(2):
        gram = dv * (psi.conj() @ psi.T)            # [nb, nb], Hermitian PD
        lo = np.linalg.cholesky(gram)               # gram = lo lo^H
        psi = scipy.linalg.solve_triangular(lo.conj(), psi, lower=True,
                                            overwrite_b=True, check_finite=False)
    return psi


def band_energies(rng: np.random.Generator, nv: int, nc: int):
    e_v = rng.uniform(-0.4, 0.0, nv)
    e_c = rng.uniform(0.05, 1.1, nc)
    return e_v, e_c


def frequencies(kind: str, count: int, eta: float = 0.005, omega0: float = 1.0):
    """Complex frequencies z for the recipes of the benchmark workloads."""
    if kind == "static":
        return np.zeros(count, dtype=np.complex128)
    if kind == "real":
        return np.linspace(0.0, 1.0, count) + 1j * eta
    if kind == "imag":
        x, _ = np.polynomial.legendre.leggauss(count)
        omega = omega0 * (1.0 + x) / (1.0 - x)
        return 1j * omega
    raise ValueError(kind)


def make_problem(n, nv: int, nc: int, *, r2=None, gvec=None, z=(0.0,), seed: int = 0,
                 cell_l: float = CELL_L, pair_chunk: int = 4096, spin: float = SPIN,
                 orthonormalize: bool = True) -> Problem:
    """Generic seeded problem.  Draw order: psi (real parts, then imaginary
    parts, valence rows first), orthonormalise, then E_v, then E_c."""
    n = tuple(int(x) for x in n)
    volume = cell_l ** 3
    rng = np.random.default_rng(seed)
    psi = orthonormal_bands(rng, nv + nc, n, volume, orthonormalize)
    e_v, e_c = band_energies(rng, nv, nc)
    if gvec is None:
        gvec = gsphere(r2)
    gvec = np.ascontiguousarray(gvec, dtype=np.int32)
    return Problem(n=n, volume=volume,
                   psi_v=np.ascontiguousarray(psi[:nv]), psi_c=np.ascontiguousarray(psi[nv:]),
                   e_v=e_v, e_c=e_c, gvec=gvec,
                   z=np.asarray(z, dtype=np.complex128).reshape(-1),
                   spin=spin, pair_chunk=pair_chunk, meta=dict(seed=seed))


def make_config(index: int, **overrides) -> Problem:
    """Workloads 0-3 at their full sizes (seed = workload index)."""
    s = dict(CONFIG_SHAPES[index])
    s.update(overrides)
    z = frequencies(*s["freq"])
    p = make_problem(s["n"], s["nv"], s["nc"], r2=s["r2"], z=z, seed=index,
                     pair_chunk=s["pair_chunk"])
    p.meta["config"] = index
    return p


def batched_shapes(nq_side: int = 4):
    """q-points of the shifted Monkhorst-Pack grid and the uneven per-q sizes
    of the batched workload: N_G(q) = round(400*10**(j/63)) and
    N_c(q) = round(300 + 600*j'/63), assigned by two seeded permutations."""
    frac = (2.0 * np.arange(nq_side) - nq_side + 1) / (2.0 * nq_side)   # -3/8 .. 3/8
    qs = np.stack(np.meshgrid(frac, frac, frac, indexing="ij"), -1).reshape(-1, 3)
    nq = qs.shape[0]
    rng = np.random.default_rng(4)
    j_ng = rng.permutation(nq)
    j_nc = rng.permutation(nq)
    ng = np.rint(400.0 * 10.0 ** (j_ng / (nq - 1))).astype(int)
    nc = np.rint(300.0 + 600.0 * j_nc / (nq - 1)).astype(int)
    return qs, ng, nc


def make_batched_config(q_indices=None, *, nv: int = 48, n=(40, 40, 40), nfreq: int = 16,
                        orthonormalize: bool = True):
    """The batched multi-q workload: one independent problem per q-point."""
    qs, ng, nc = batched_shapes()
    if q_indices is None:
        q_indices = range(qs.shape[0])
    z = frequencies("imag", nfreq)
    probs = []
    for qi in q_indices:
        g = gsphere_shifted(qs[qi], int(ng[qi]))
        p = make_problem(n, nv, int(nc[qi]), gvec=g, z=z, seed=4000 + int(qi),
                         orthonormalize=orthonormalize)
        p.meta.update(config=4, q_index=int(qi), q=qs[qi].tolist())
        probs.append(p)
    return probs


@dataclass
class DeviceProblem:
    """A seeded problem whose band set lives on the device (torch tensors);
    energies, G list and frequencies stay on the host."""
    n: tuple
    volume: float
    psi: "object"              # torch complex128 [nv + nc, N_r], valence rows first
    nv: int
    e_v: np.ndarray
    e_c: np.ndarray
    gvec: np.ndarray
    z: np.ndarray
    spin: float = SPIN
    pair_chunk: int = 4096

    @property
    def nc(self):
        return self.psi.shape[0] - self.nv

    @property
    def ng(self):
        return self.gvec.shape[0]

    @property
    def psi_v(self):
        return self.psi[:self.nv]

    @property
    def psi_c(self):
        return self.psi[self.nv:]


def orthonormal_bands_device(rng: np.random.Generator, nb: int, n, volume: float,
                             device="cuda", row_block: int = 64):
    """The bands of ``orthonormal_bands`` built for problems too large to
    orthonormalise on the host: the same normals, drawn from ``rng`` in the
    same order (all real parts, then all imaginary parts, row blocks drawn in
    sequence give the same stream as one draw) and copied to the device block
    by block; then two passes of Cholesky-QR there with torch.  Equal to the
    host recipe up to rounding."""
    import torch
    nr = int(np.prod(n))
    psi = torch.empty((nb, nr), dtype=torch.complex128, device=device)
    view = torch.view_as_real(psi)                   # [nb, nr, 2]
    for part in (0, 1):
        for r0 in range(0, nb, row_block):
            r1 = min(nb, r0 + row_block)
            blk = torch.from_numpy(rng.standard_normal((r1 - r0, nr)))
            view[r0:r1, :, part].copy_(blk.to(device))
    if nb == 0:
        return psi
    dv = volume / nr
    for _ in range(2):
        # conj(psi) psi^T = conj(psi psi^H): the conjugate-transposed view maps
        # to the BLAS conjugate-transpose operand, no copy of the bands
        gram = torch.matmul(psi, psi.mH).conj() * dv
        lo = torch.linalg.cholesky(gram)
        # psi <- conj(lo)^-1 psi through the explicit inverse of the small
        # triangular factor (a triangular solve with 10^5-10^6 right-hand
        # sides asks the BLAS for more workspace than it will allocate)
        eye = torch.eye(nb, dtype=psi.dtype, device=psi.device)
        linv = torch.linalg.solve_triangular(lo.conj(), eye, upper=False)
        psi = torch.matmul(linv, psi)
        del gram, lo, eye, linv
    return psi


def make_problem_device(n, nv: int, nc: int, *, r2=None, gvec=None, z=(0.0,), seed: int = 0,
                        device="cuda", pair_chunk: int = 4096) -> DeviceProblem:
    """``make_problem`` with the band set orthonormalised on the device (same
    draw order: psi, then E_v, then E_c)."""
    n = tuple(int(x) for x in n)
    volume = CELL_L ** 3
    rng = np.random.default_rng(seed)
    psi = orthonormal_bands_device(rng, nv + nc, n, volume, device)
    e_v, e_c = band_energies(rng, nv, nc)
    if gvec is None:
        gvec = gsphere(r2)
    return DeviceProblem(n=n, volume=volume, psi=psi, nv=nv, e_v=e_v, e_c=e_c,
                         gvec=np.ascontiguousarray(gvec, dtype=np.int32),
                         z=np.asarray(z, dtype=np.complex128).reshape(-1), pair_chunk=pair_chunk)


def shell_bands_device(rng: np.random.Generator, nb: int, n, volume: float, width: float,
                       device="cuda", row_block: int = 64):
    """Bands with the momentum structure of free-electron-like states, for the
    static-subspace workloads: band j's plane-wave coefficients are the
    recipe's normals (same draw order) damped to a shell around
    |g| = k_j = (3 (j + 1/2) / (4 pi))^(1/3), the radius below which j grid
    wave vectors lie, of Gaussian width ``width`` (g the integer wave vector
    of a grid frequency); brought to the grid and orthonormalised in band order
    as in ``orthonormal_bands_device``.  With free-electron energies
    (``shell_energies``), a large momentum transfer G needs pairs far apart in
    energy, so |chi_GG(0)| falls off with |G| and the spectrum of chi0(0)
    decays, as for the DFT states the paper works with; white bands with the
    recipe's energies give a nearly flat one."""
    import torch
    n = tuple(int(x) for x in n)
    nr = int(np.prod(n))
    ax = [np.fft.fftfreq(k, 1.0 / k) for k in n]            # integer frequencies
    gabs = np.sqrt(ax[0][:, None, None] ** 2 + ax[1][None, :, None] ** 2 +
                   ax[2][None, None, :] ** 2).reshape(-1)
    gabs = torch.from_numpy(gabs).to(device)
    psi = torch.empty((nb, nr), dtype=torch.complex128, device=device)
    view = torch.view_as_real(psi)
    for part in (0, 1):
        for r0 in range(0, nb, row_block):
            r1 = min(nb, r0 + row_block)
            view[r0:r1, :, part].copy_(torch.from_numpy(rng.standard_normal((r1 - r0, nr))).to(device))
    kj = torch.from_numpy((3.0 * (np.arange(nb) + 0.5) / (4.0 * np.pi)) ** (1.0 / 3.0)).to(device)
    for r0 in range(0, nb, row_block):
        r1 = min(nb, r0 + row_block)
        env = torch.exp(-((gabs[None, :] - kj[r0:r1, None]) ** 2) / (2.0 * width * width))
        blk = (psi[r0:r1] * env).reshape(r1 - r0, *n)
        psi[r0:r1] = torch.fft.ifftn(blk, dim=(1, 2, 3)).reshape(r1 - r0, nr)
    if nb == 0:
        return psi
    dv = volume / nr
    for _ in range(2):
        gram = torch.matmul(psi, psi.mH).conj() * dv
        lo = torch.linalg.cholesky(gram)
        eye = torch.eye(nb, dtype=psi.dtype, device=psi.device)
        linv = torch.linalg.solve_triangular(lo.conj(), eye, upper=False)
        psi = torch.matmul(linv, psi)
        del gram, lo, eye, linv
    return psi


def shell_energies(nv: int, nc: int, gap: float = 0.05, cell_l: float = CELL_L):
    """Free-electron energies of the shell bands: band j at
    (2 pi k_j / L)^2 / 2 with k_j as in ``shell_bands_device``, shifted so
    that the valence bands lie below zero and the conduction bands from
    ``gap`` Ha up."""
    nb = nv + nc
    kj = (3.0 * (np.arange(nb) + 0.5) / (4.0 * np.pi)) ** (1.0 / 3.0)
    e = 0.5 * (2.0 * np.pi * kj / cell_l) ** 2
    e_v = e[:nv] - (e[nv - 1] if nv else 0.0)
    e_c = e[nv:] - (e[nv] if nc else 0.0) + gap
    return e_v, e_c


def make_shell_config_device(index: int, width: float = 1.0, device="cuda",
                             **overrides) -> DeviceProblem:
    """Workload ``index``'s shape, seed, G-sphere and frequencies with shell
    bands (``shell_bands_device``) and their free-electron energies
    (``shell_energies``)."""
    s = dict(CONFIG_SHAPES[index])
    s.update(overrides)
    n = tuple(int(x) for x in s["n"])
    volume = CELL_L ** 3
    rng = np.random.default_rng(index)
    psi = shell_bands_device(rng, s["nv"] + s["nc"], n, volume, width, device)
    e_v, e_c = shell_energies(s["nv"], s["nc"])
    return DeviceProblem(n=n, volume=volume, psi=psi, nv=s["nv"], e_v=e_v, e_c=e_c,
                         gvec=gsphere(s["r2"]), z=frequencies(*s["freq"]),
                         pair_chunk=s["pair_chunk"])


def make_config_device(index: int, device="cuda", **overrides) -> DeviceProblem:
    """Workload ``index`` with its band set drawn as in ``make_config`` and
    orthonormalised on the device (for the 72^3 workload: 4,096 bands of
    373,248 points, 24.5 GB)."""
    s = dict(CONFIG_SHAPES[index])
    s.update(overrides)
    return make_problem_device(s["n"], s["nv"], s["nc"], r2=s["r2"], z=frequencies(*s["freq"]),
                               seed=index, device=device, pair_chunk=s["pair_chunk"])


def device_bands(nb: int, nr: int, *, seed: int, volume: float = CELL_L ** 3, device="cuda"):
    """Timing-only band sets generated on the GPU: ``nb`` rows of iid complex
    Gaussians scaled to unit norm on the grid on average (dV sum |psi|^2 ~ 1),
    not orthonormalised.  For throughput runs whose inputs are too large to
    generate on the host; the work done does not depend on the values."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    # complex normal: real and imaginary parts of variance 1/2 each
    psi = torch.randn((nb, nr), generator=g, device=device, dtype=torch.complex128)
    return psi.mul_((1.0 / volume) ** 0.5)


def pseudoband_recipe(e_c, n_protect: int, sizes, n_xi: int, seed: int):
    """Pseudoband inputs for a conduction set: the n_protect lowest bands are
    protected, the rest (in energy order) are cut into consecutive slices of
    the given sizes (growing with energy), and the phases in turns are drawn
    uniform in [0, 1).  Returns (keep, slices, theta)."""
    order = np.argsort(np.asarray(e_c), kind="stable")
    keep = order[:n_protect]
    rest = order[n_protect:]
    if sum(sizes) != len(rest):
        raise ValueError("slice sizes must cover the unprotected bands")
    bounds = np.concatenate([[0], np.cumsum(sizes)])
    slices = [rest[bounds[i]:bounds[i + 1]] for i in range(len(sizes))]
    rng = np.random.default_rng(seed)
    theta = [rng.random((n_xi, len(s))) for s in slices]
    return keep, slices, theta


def gpp_inputs(nb: int, ns: int, ng: int, ne: int, seed: int):
    """Seeded inputs of the GPP off-diagonal self-energy: matrix elements
    M[n][l][G] (complex Gaussian, variance 1/N_G per part, as for normalised
    random states), band energies uniform in [-0.5, 1.5] Ha (sorted; occupied
    below 0), an energy grid of ne points evenly over [-0.5, 1.0] Ha with a
    0.01 Ha imaginary broadening, plasmon-pole parameters Omega2 (Hermitian,
    N(0, 1/2) entries) and wtilde (symmetric, uniform in [0.3, 2.0] Ha), and a
    positive Coulomb-like diagonal v uniform in [0.1, 2.0]."""
    rng = np.random.default_rng(seed)
    sd = (0.5 / max(ng, 1)) ** 0.5
    m = sd * (rng.standard_normal((nb, ns, ng)) + 1j * rng.standard_normal((nb, ns, ng)))
    e_n = np.sort(rng.uniform(-0.5, 1.5, nb))
    occupied = (e_n < 0.0).astype(np.int32)
    energies = np.linspace(-0.5, 1.0, ne) + 0.01j if ne > 1 else np.array([0.25 + 0.01j])
    x = rng.standard_normal((ng, ng)) + 1j * rng.standard_normal((ng, ng))
    omega2 = 0.5 * (x + x.conj().T)
    wt = rng.uniform(0.3, 2.0, (ng, ng))
    wtilde = 0.5 * (wt + wt.T)
    v = rng.uniform(0.1, 2.0, ng)
    return dict(m=m, e_n=e_n, occupied=occupied, energies=np.asarray(energies, np.complex128),
                omega2=omega2, wtilde=wtilde, v=v)
