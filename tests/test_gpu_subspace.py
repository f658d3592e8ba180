"""The static subspace (Diag, Transf, CHI-Freq of Eq. (6)) and the dense
building blocks under it (complex FP64 GEMM on MFMA, Jacobi eigensolver),
against the FP64 oracle and plain NumPy.

Eigenvectors carry a phase, and a degenerate or nearly degenerate eigenspace
any rotation, so the device basis is compared through what is unique: the
eigenvalues, the projector C_s C_s^H where the spectrum has a gap at n_eig,
and C_s chi_B C_s^H; chi_B itself is compared element by element when both
sides use the same basis."""
import numpy as np
import pytest
import torch

import oracle
import paper_2509_23018_amd as gw
from gpu_helpers import FP64_TOL, device, rel_fro, to_dev
from workloads import gen

pytestmark = pytest.mark.gpu


def _crand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _op(x, o):
    return x if o == "N" else (x.swapaxes(-1, -2) if o == "T" else x.conj().swapaxes(-1, -2))


@pytest.mark.parametrize("opa", ["N", "T", "C"])
@pytest.mark.parametrize("opb", ["N", "T", "C"])
def test_zgemm_ops_ragged_batched(opa, opb):
    rng = np.random.default_rng(7)
    m, n, k, batch = 70, 45, 37, 3
    a = _crand(rng, batch, *((m, k) if opa == "N" else (k, m)))
    b = _crand(rng, batch, *((k, n) if opb == "N" else (n, k)))
    c0 = _crand(rng, batch, m, n)
    alpha, beta = 0.7 - 0.2j, -0.3 + 1.1j
    c = torch.from_numpy(c0.copy()).to(device())
    gw.gw_zgemm(opa, opb, torch.from_numpy(a).to(device()), torch.from_numpy(b).to(device()),
                alpha=alpha, beta=beta, c=c)
    want = alpha * (_op(a, opa) @ _op(b, opb)) + beta * c0
    assert rel_fro(c.cpu().numpy(), want) < 1e-14


@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (64, 64, 16), (129, 3, 200), (5, 130, 0)])
def test_zgemm_shapes(m, n, k):
    rng = np.random.default_rng(m + n + k)
    a, b = _crand(rng, m, k), _crand(rng, k, n)
    got = gw.gw_zgemm("N", "N", torch.from_numpy(a).to(device()),
                      torch.from_numpy(b).to(device())).cpu().numpy()
    assert rel_fro(got, a @ b) < 1e-14 if k else np.all(got == 0)


# n < 64: element sweeps; n >= 64: blocks of 16 (129: a ragged last block and
# a phantom block; 300: 19 blocks, ragged, odd count)
@pytest.mark.parametrize("n", [1, 2, 7, 63, 64, 129, 300])
def test_heev_matches_numpy(n):
    rng = np.random.default_rng(n)
    x = _crand(rng, 2, n, n)
    a = 0.5 * (x + x.conj().swapaxes(-1, -2))
    a[1] *= 1e-3                              # a second, differently scaled matrix
    w, v = gw.gw_heev(torch.from_numpy(a).to(device()))
    w, v = w.cpu().numpy(), v.cpu().numpy()
    tol = 1e-13
    for i in range(2):
        scale = np.abs(np.linalg.eigvalsh(a[i])).max()
        assert np.abs(w[i] - np.linalg.eigvalsh(a[i])).max() < tol * scale
        assert np.abs(v[i].conj().T @ v[i] - np.eye(n)).max() < tol
        assert np.abs(a[i] @ v[i] - v[i] * w[i][None, :]).max() < tol * scale


@pytest.mark.parametrize("n", [40, 200])
def test_heev_degenerate_spectrum(n):
    rng = np.random.default_rng(3)
    u, _ = np.linalg.qr(_crand(rng, n, n))
    lam = np.repeat([-2.0, 0.5, 3.0, 3.0 + 1e-9], n // 4)
    a = (u * lam) @ u.conj().T
    w, v = gw.gw_heev(torch.from_numpy(a).to(device()))
    w, v = w.cpu().numpy(), v.cpu().numpy()
    tol = 1e-13
    assert np.abs(w - np.sort(lam)).max() < tol * 3
    assert np.abs(a @ v - v * w[None, :]).max() < tol * 3


def _known_spectrum(ng, lam, seed):
    rng = np.random.default_rng(seed)
    u, _ = np.linalg.qr(_crand(rng, ng, ng))
    return (u * lam[None, :]) @ u.conj().T


def test_subspace_basis_known_spectrum():
    """A negative semidefinite matrix of known spectrum with a gap after the
    40 most negative eigenvalues: eigenvalues to 1e-12 of the norm, the
    projector to the residual over the gap, orthonormal columns."""
    ng, n_eig = 300, 40
    rng = np.random.default_rng(11)
    lam = -np.concatenate([np.sort(rng.uniform(2.0, 10.0, n_eig))[::-1],
                           rng.uniform(0.0, 1.0, ng - n_eig)])
    a = _known_spectrum(ng, lam, 12)
    basis, ev, info = gw.gw_subspace_basis(torch.from_numpy(a).to(device()), n_eig, tol=1e-12)
    basis, ev = basis.cpu().numpy(), ev.cpu().numpy()
    cs, want = oracle.static_subspace_basis(a, n_eig)
    assert info["residual"] <= 1e-12, info
    assert np.abs(ev - want).max() < 1e-12 * 10.0
    assert np.abs(basis.conj().T @ basis - np.eye(n_eig)).max() < 1e-12
    assert np.abs(basis @ basis.conj().T - cs @ cs.conj().T).max() < 1e-10


def _chi_static_problem(seed=41, nv=2, nc=10, r2=10, n=(12, 12, 12)):
    z = (0.0, 0.4j, 1.7j, 0.3 + 0.01j)
    p = gen.make_problem(n, nv, nc, r2=r2, z=z, seed=seed, pair_chunk=7)
    chi = oracle.chi0(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec, p.z, p.n, p.volume,
                      spin=p.spin, pair_chunk=p.pair_chunk)
    return p, chi


@pytest.mark.parametrize("n_eig", [20, 12])
def test_subspace_basis_of_chi0(n_eig):
    """Diag of the oracle's chi0(0) (147 G, 20 pairs: rank 20): the kept
    eigenvalues against numpy's, the static chi in the device basis diagonal;
    at n_eig = rank the gap to zero is complete and the projector must agree."""
    p, chi = _chi_static_problem()
    a = torch.from_numpy(np.ascontiguousarray(chi[0])).to(device())
    basis, ev, info = gw.gw_subspace_basis(a, n_eig, tol=1e-12)
    basis, ev = basis.cpu().numpy(), ev.cpu().numpy()
    cs, want = oracle.static_subspace_basis(chi[0], n_eig)
    scale = np.abs(want).max()
    assert np.abs(ev - want).max() < 1e-11 * scale, (ev, want, info)
    diag = basis.conj().T @ chi[0] @ basis
    assert np.abs(diag - np.diag(ev)).max() < 1e-10 * scale
    if n_eig == 20:
        assert np.abs(basis @ basis.conj().T - cs @ cs.conj().T).max() < 1e-9


@pytest.mark.parametrize("prec,ns,tol", [("fp64", 0, FP64_TOL), ("split_bf16", 5, 1e-10),
                                         ("fp32", 0, 1e-5)])
@pytest.mark.parametrize("chunk", [7, 4096])
def test_chi0_subspace_matches_oracle(prec, ns, tol, chunk):
    """Transf + CHI-Freq with the oracle's basis on both sides: element by
    element against Eq. (6), every frequency kind, several chunks or one."""
    p, chi = _chi_static_problem(seed=42, nv=3, nc=17)
    cs, _ = oracle.static_subspace_basis(chi[0], 24)
    want = oracle.chi0_subspace(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec, p.z, p.n, p.volume, cs,
                                spin=p.spin, pair_chunk=chunk)
    dp = to_dev(p)
    got = gw.gw_chi0_subspace(dp, torch.from_numpy(np.ascontiguousarray(cs)).to(device()),
                              precision=prec, n_slices=ns, pair_chunk=chunk).cpu().numpy()
    assert rel_fro(got, want) < tol, rel_fro(got, want)
    for w in range(len(p.z)):
        assert rel_fro(got[w], want[w]) < tol


def test_subspace_pipeline_on_device():
    """Diag, Transf and CHI-Freq all on the device: C_s chi_B(z) C_s^H equals
    P chi(z) P of the oracle (P the oracle's projector, unique at n_eig = the
    rank of chi0(0)), and chi_B(0) is diagonal with the device eigenvalues."""
    p, chi = _chi_static_problem(seed=43)
    n_eig = 20
    dp = to_dev(p)
    chi_d = gw.gw_chi0(dp, pair_chunk=p.pair_chunk)
    basis, ev, _ = gw.gw_subspace_basis(chi_d[0].contiguous(), n_eig, tol=1e-12)
    chib = gw.gw_chi0_subspace(dp, basis, pair_chunk=p.pair_chunk).cpu().numpy()
    b = basis.cpu().numpy()
    cs, _ = oracle.static_subspace_basis(chi[0], n_eig)
    proj = cs @ cs.conj().T
    for w in range(len(p.z)):
        want = proj @ chi[w] @ proj
        got = b @ chib[w] @ b.conj().T
        assert rel_fro(got, want) < 1e-10, (w, rel_fro(got, want))
    assert np.abs(chib[0] - np.diag(ev.cpu().numpy())).max() < 1e-11 * np.abs(chib[0]).max()


def test_subspace_weighted_against_oracle():
    """The symmetrised form W chi W (w = sqrt of the Coulomb diagonal at a
    shifted q): Diag of the oracle's chi0(0) against the oracle's weighted
    eigenpairs (eigenvalues, diagonal static chi in the device basis), then
    Transf + CHI-Freq with the oracle's weighted basis element by element, and
    the whole weighted pipeline on the device against the oracle's projected
    W chi W."""
    p, chi = _chi_static_problem(seed=44, nv=3, nc=17)
    wt = np.sqrt(oracle.coulomb(p.gvec, q=(0.1, -0.05, 0.2), cell_l=gen.CELL_L))
    wd = torch.from_numpy(wt).to(device())
    n_eig = 24
    cs, want_ev = oracle.static_subspace_basis(chi[0], n_eig, weight=wt)
    a = torch.from_numpy(np.ascontiguousarray(chi[0])).to(device())
    basis, ev, info = gw.gw_subspace_basis(a, n_eig, weight=wd, tol=1e-12)
    b, ev = basis.cpu().numpy(), ev.cpu().numpy()
    scale = np.abs(want_ev).max()
    assert np.abs(ev - want_ev).max() < 1e-11 * scale, (ev, want_ev, info)
    wchiw = wt[None, :, None] * chi * wt[None, None, :]
    assert np.abs(b.conj().T @ wchiw[0] @ b - np.diag(ev)).max() < 1e-10 * scale
    dp = to_dev(p)
    want = oracle.chi0_subspace(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec, p.z, p.n, p.volume, cs,
                                spin=p.spin, pair_chunk=p.pair_chunk, weight=wt)
    got = gw.gw_chi0_subspace(dp, torch.from_numpy(np.ascontiguousarray(cs)).to(device()),
                              weight=wd, pair_chunk=p.pair_chunk).cpu().numpy()
    assert rel_fro(got, want) < FP64_TOL, rel_fro(got, want)
    # whole pipeline at n_eig = rank (20 pairs), where the projector is unique
    p, chi = _chi_static_problem(seed=45)
    wt = np.sqrt(oracle.coulomb(p.gvec, q=(0.1, -0.05, 0.2), cell_l=gen.CELL_L))
    wd = torch.from_numpy(wt).to(device())
    dp = to_dev(p)
    chi_d = gw.gw_chi0(dp, pair_chunk=p.pair_chunk)
    basis, ev, _ = gw.gw_subspace_basis(chi_d[0].contiguous(), 20, weight=wd, tol=1e-12)
    b = basis.cpu().numpy()
    chib = gw.gw_chi0_subspace(dp, basis, weight=wd, pair_chunk=p.pair_chunk).cpu().numpy()
    cs, _ = oracle.static_subspace_basis(chi[0], 20, weight=wt)
    proj = cs @ cs.conj().T
    wchiw = wt[None, :, None] * chi * wt[None, None, :]
    for w in range(len(p.z)):
        ref = proj @ wchiw[w] @ proj
        assert rel_fro(b @ chib[w] @ b.conj().T, ref) < 1e-10, w


def _chunk_order(nv, nc, chunk):
    """Pair indices p = v*nc + c in the order gw_chi0 streams its chunks
    (rectangles of vb valence x cw conduction bands, valence blocks outer)."""
    cw = max(1, min(nc, chunk // max(1, min(nv, 4))))
    vb = max(1, min(nv, chunk // cw))
    order = []
    for v0 in range(0, nv, vb):
        for c0 in range(0, nc, cw):
            for v in range(v0, min(nv, v0 + vb)):
                order.extend(v * nc + c for c in range(c0, min(nc, c0 + cw)))
    return np.array(order)


@pytest.mark.parametrize("chunk", [7, 4096])
def test_keep_m_and_chi_from_kept_m(chunk):
    """gw_chi0_keep_m: chi as gw_chi0 gives it (the same kernels on the same
    data: bit for bit) and M of every pair in chunk order against the oracle's
    MTXEL; gw_chi0_from_m: chi at other frequencies and chi_BB' of Eq. (6)
    (weighted basis) from the kept M, without MTXEL, against the oracle and
    bit for bit against gw_chi0 / gw_chi0_subspace."""
    p, chi = _chi_static_problem(seed=46, nv=3, nc=17)
    dp = to_dev(p)
    want = gw.gw_chi0(dp, pair_chunk=chunk).clone()
    dp2 = to_dev(p)
    got, mk = gw.gw_chi0_keep_m(dp2, pair_chunk=chunk)
    assert torch.equal(got, want)
    m_or = oracle.mtxel(p.psi_v, p.psi_c, p.gvec, p.n, p.volume)
    order = _chunk_order(p.nv, p.nc, chunk)
    assert rel_fro(mk.cpu().numpy(), m_or[order]) < FP64_TOL
    # chi at the same problem's frequencies, from the kept M
    dp3 = to_dev(p)
    from_m = gw.gw_chi0_from_m(dp3, mk, pair_chunk=chunk)
    assert torch.equal(from_m, want)
    assert rel_fro(from_m.cpu().numpy(), chi) < FP64_TOL
    # Eq. (6) from the kept M with the oracle's weighted basis
    wt = np.sqrt(oracle.coulomb(p.gvec, q=(0.1, -0.05, 0.2), cell_l=gen.CELL_L))
    wd = torch.from_numpy(wt).to(device())
    cs, _ = oracle.static_subspace_basis(chi[0], 12, weight=wt)
    csd = torch.from_numpy(np.ascontiguousarray(cs)).to(device())
    sub_m = gw.gw_chi0_from_m(dp3, mk, csd, weight=wd, pair_chunk=chunk)
    sub = gw.gw_chi0_subspace(dp3, csd, weight=wd, pair_chunk=chunk)
    assert torch.equal(sub_m, sub)
    ref = oracle.chi0_subspace(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec, p.z, p.n, p.volume, cs,
                               spin=p.spin, pair_chunk=chunk, weight=wt)
    assert rel_fro(sub_m.cpu().numpy(), ref) < FP64_TOL
    with pytest.raises(ValueError):
        gw.gw_chi0_from_m(dp3, mk, csd[:, :0], pair_chunk=chunk)
    with pytest.raises(ValueError):
        gw.gw_chi0_from_m(dp3, mk, csd[1:], pair_chunk=chunk)
    wide = torch.zeros((p.gvec.shape[0], p.gvec.shape[0] + 1), dtype=torch.complex128,
                       device=device())
    with pytest.raises(gw.GWError):
        gw.gw_chi0_from_m(dp3, mk, wide, pair_chunk=chunk)


@pytest.mark.parametrize("prec,ns", [("fp32", 0), ("split_bf16", 3), ("split_fp16x9", 4)])
def test_chi_from_kept_m_reduced_precision(prec, ns):
    """The kept-M path runs the same contraction kernels in every precision:
    chi from gw_chi0_from_m equals gw_chi0 in that precision bit for bit, on
    several chunks with a ragged last one."""
    p, _ = _chi_static_problem(seed=47, nv=3, nc=17)
    chunk = 11
    want = gw.gw_chi0(to_dev(p), precision=prec, n_slices=ns, pair_chunk=chunk).clone()
    dp = to_dev(p)
    _, mk = gw.gw_chi0_keep_m(dp, pair_chunk=chunk)
    got = gw.gw_chi0_from_m(dp, mk, precision=prec, n_slices=ns, pair_chunk=chunk)
    assert torch.equal(got, want)


def test_subspace_argument_errors():
    a = torch.zeros((8, 8), dtype=torch.complex128, device=device())
    with pytest.raises(gw.GWError):
        gw.gw_subspace_basis(a, 9)
    with pytest.raises(gw.GWError):
        gw.gw_subspace_basis(a, 0)
    with pytest.raises(ValueError):
        gw.gw_subspace_basis(a, 3, weight=torch.ones(7, dtype=torch.float64, device=device()))
    basis, ev, info = gw.gw_subspace_basis(a, 3)      # chi = 0: unit vectors, zero eigenvalues
    assert torch.all(ev == 0)
    b = basis.cpu().numpy()
    assert np.abs(b.conj().T @ b - np.eye(3)).max() == 0
