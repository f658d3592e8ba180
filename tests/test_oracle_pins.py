"""Pins of the FP64 oracle against what the mathematics fixes.

The paper prints no numerical value for the chi0 path, so every pin here is
a closed form, an identity, an invariant or a brute-force evaluation written
independently of the oracle's FFT-based code (explicit Python loops over the
grid, plane waves whose matrix elements are Kronecker deltas, ...).
"""
import cmath
import itertools
import math

import numpy as np
import pytest

import oracle
from workloads import gen

L = 10.0
VOL = L ** 3


def _bands(rng, nb, n, ortho=True):
    return gen.orthonormal_bands(rng, nb, n, VOL, ortho)


def _all_g(n):
    """Every Miller triple with g_i in [-N_i/2, N_i/2): one per grid point."""
    axes = [range(-(k // 2), k - k // 2) for k in n]
    return np.array(list(itertools.product(*axes)), dtype=np.int32)


def _plane_waves(ks, n):
    """psi_k(r) = exp(i k.r)/sqrt(Omega) for integer k (grid wave vectors)."""
    n1, n2, n3 = n
    j1, j2, j3 = np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij")
    out = []
    for k in ks:
        arg = 2 * np.pi * (k[0] * j1 / n1 + k[1] * j2 / n2 + k[2] * j3 / n3)
        out.append(np.exp(1j * arg).reshape(-1) / math.sqrt(VOL))
    return np.array(out)


def _brute_m(psi_v_row, psi_c_row, g, n):
    """Direct triple loop over the grid with cmath (no numpy transforms)."""
    n1, n2, n3 = n
    dv = VOL / (n1 * n2 * n3)
    acc = 0j
    for j1 in range(n1):
        for j2 in range(n2):
            for j3 in range(n3):
                r = (j1 * n2 + j2) * n3 + j3
                ph = cmath.exp(2j * math.pi * (g[0] * j1 / n1 + g[1] * j2 / n2 + g[2] * j3 / n3))
                acc += psi_v_row[r].conjugate() * psi_c_row[r] * ph
    return dv * acc


# ---------------------------------------------------------------- inputs

def test_gsphere_counts_and_order():
    # complete shells |g|^2 <= R^2 of the workloads (~150, ~2000, ~6000, ~1200)
    for r2, count in ((10, 147), (61, 2007), (126, 6031), (42, 1189)):
        g = gen.gsphere(r2)
        assert g.shape == (count, 3)
        n2 = (g.astype(np.int64) ** 2).sum(1)
        assert np.all(np.diff(n2) >= 0)
        assert len({tuple(x) for x in g}) == count
        assert tuple(g[0]) == (0, 0, 0)


def test_gsphere_shifted_sizes():
    qs, ng, nc = gen.batched_shapes()
    assert qs.shape == (64, 3)
    assert ng.min() == 400 and ng.max() == 4000 and len(set(ng.tolist())) == 64
    assert nc.min() == 300 and nc.max() == 900
    g = gen.gsphere_shifted(qs[5], int(ng[5]))
    assert g.shape == (ng[5], 3) and len({tuple(x) for x in g}) == ng[5]
    k2 = ((g + qs[5]) ** 2).sum(1)
    assert np.all(np.diff(k2) >= -1e-12)


def test_generated_bands_orthonormal():
    rng = np.random.default_rng(0)
    n = (6, 5, 4)
    psi = _bands(rng, 20, n)
    dv = VOL / np.prod(n)
    gram = dv * psi.conj() @ psi.T
    assert np.abs(gram - np.eye(20)).max() < 1e-12


# ---------------------------------------------------------------- MTXEL

def test_plane_wave_mtxel_is_kronecker_delta():
    """psi_n = exp(i k_n.r)/sqrt(Omega) gives M_vc(G) = 1 iff G = k_v - k_c mod N."""
    n = (8, 6, 10)
    kv = [(0, 0, 0), (3, -2, 4), (-4, 2, -5)]
    kc = [(1, 0, 0), (3, -2, 3), (-3, 2, 4), (0, 1, -1), (4, 3, 0)]   # includes wraps
    pv, pc = _plane_waves(kv, n), _plane_waves(kc, n)
    gl = _all_g(n)
    m = oracle.mtxel(pv, pc, gl, n, VOL)
    nn = np.array(n)
    for v, c in itertools.product(range(len(kv)), range(len(kc))):
        target = (np.array(kv[v]) - np.array(kc[c])) % nn
        want = np.all((gl % nn) == target, axis=1).astype(float)
        assert want.sum() == 1
        assert np.abs(m[v * len(kc) + c] - want).max() < 1e-12


def test_plane_wave_mtxel_sign_discriminates():
    """The opposite exponent sign would put the 1 at k_c - k_v instead."""
    n = (8, 8, 8)
    pv, pc = _plane_waves([(1, 2, 3)], n), _plane_waves([(0, 0, 0)], n)
    m = oracle.mtxel(pv, pc, np.array([[1, 2, 3], [-1, -2, -3]], np.int32), n, VOL)
    assert abs(m[0, 0] - 1) < 1e-12 and abs(m[0, 1]) < 1e-12


@pytest.mark.parametrize("n", [(4, 4, 4), (6, 6, 6), (8, 8, 8), (10, 10, 10), (12, 12, 12), (4, 6, 5)])
def test_mtxel_brute_force_dft(n):
    rng = np.random.default_rng(sum(n))
    psi = _bands(rng, 5, n, ortho=False)
    pv, pc = psi[:2], psi[2:]
    gl = _all_g(n)
    sel = rng.choice(len(gl), size=min(6, len(gl)), replace=False)
    g = gl[sel]
    m = oracle.mtxel(pv, pc, g, n, VOL)
    for p in range(6):
        v, c = divmod(p, 3)
        for i in range(len(g)):
            ref = _brute_m(pv[v], pc[c], g[i], n)
            assert abs(m[p, i] - ref) < 1e-12 * max(1.0, abs(ref))


def test_mtxel_direct_matches_brute_force():
    n = (4, 6, 5)
    rng = np.random.default_rng(7)
    psi = _bands(rng, 4, n, ortho=False)
    g = (1, -3, 2)
    d = oracle.mtxel_direct(psi[:2], psi[2:], g, n, VOL)
    for v, c in itertools.product(range(2), range(2)):
        assert abs(d[v, c] - _brute_m(psi[v], psi[2 + c], g, n)) < 1e-12


def test_mtxel_parseval_full_grid():
    n = (6, 8, 5)
    rng = np.random.default_rng(3)
    psi = _bands(rng, 4, n)
    gl = _all_g(n)
    m = oracle.mtxel(psi[:2], psi[2:], gl, n, VOL)
    dv = VOL / np.prod(n)
    for p in range(4):
        v, c = divmod(p, 2)
        rhs = VOL * dv * np.sum(np.abs(psi[v]) ** 2 * np.abs(psi[2 + c]) ** 2)
        assert abs(np.sum(np.abs(m[p]) ** 2) - rhs) < 1e-12 * rhs


def test_mtxel_completeness_sum_rule():
    """With N_b = N_r orthonormal states, sum_n |M_vn(G)|^2 = <v|v> = 1."""
    n = (4, 4, 3)
    nr = int(np.prod(n))
    rng = np.random.default_rng(5)
    psi = _bands(rng, nr, n)
    gl = _all_g(n)[::5]
    m = oracle.mtxel(psi[:3], psi, gl, n, VOL).reshape(3, nr, -1)
    s = np.sum(np.abs(m) ** 2, axis=1)
    assert np.abs(s - 1.0).max() < 1e-12


def test_mtxel_orthogonality_at_g0():
    n = (8, 8, 8)
    rng = np.random.default_rng(9)
    psi = _bands(rng, 12, n)
    m = oracle.mtxel(psi[:4], psi[4:], np.zeros((1, 3), np.int32), n, VOL)
    assert np.abs(m).max() < 1e-12


def test_mtxel_translation_phase():
    n = (6, 8, 10)
    rng = np.random.default_rng(11)
    psi = _bands(rng, 4, n, ortho=False)
    a = (2, -3, 4)
    shifted = np.roll(psi.reshape(4, *n), shift=a, axis=(1, 2, 3)).reshape(4, -1)
    gl = _all_g(n)[::7]
    m0 = oracle.mtxel(psi[:2], psi[2:], gl, n, VOL)
    m1 = oracle.mtxel(shifted[:2], shifted[2:], gl, n, VOL)
    ph = np.exp(2j * np.pi * (gl[:, 0] * a[0] / n[0] + gl[:, 1] * a[1] / n[1] + gl[:, 2] * a[2] / n[2]))
    assert np.abs(m1 - m0 * ph[None, :]).max() < 1e-12


def test_mtxel_aliasing_mod_n():
    n = (6, 6, 6)
    rng = np.random.default_rng(13)
    psi = _bands(rng, 3, n, ortho=False)
    g = np.array([[1, -2, 3], [1 + 6, -2 - 6, 3 + 12]], np.int32)
    m = oracle.mtxel(psi[:1], psi[1:], g, n, VOL)
    assert np.abs(m[:, 0] - m[:, 1]).max() < 1e-13


# ---------------------------------------------------------------- energy factor

def test_energy_factor_closed_forms():
    e_v = np.array([-0.3, -0.1])
    e_c = np.array([0.2, 0.7, 1.0])
    de = (e_v[:, None] - e_c[None, :]).reshape(-1)
    d0 = oracle.energy_factor(e_v, e_c, [0.0])[0]
    assert np.allclose(d0, 2.0 / de, rtol=1e-15, atol=0)
    w = 0.37
    di = oracle.energy_factor(e_v, e_c, [1j * w])[0]
    assert np.abs(di.imag).max() < 1e-15
    assert np.allclose(di.real, 2 * de / (de ** 2 + w ** 2), rtol=1e-14, atol=0)
    # real axis with broadening: resonant + anti-resonant, retarded
    z = 0.5 + 0.01j
    dr = oracle.energy_factor(e_v, e_c, [z])[0]
    ecv = -de
    assert np.allclose(dr, 1 / (z - ecv) - 1 / (z + ecv), rtol=1e-14, atol=0)


def test_energy_factor_derivative():
    e_v = np.array([-0.3, -0.05])
    e_c = np.array([0.2, 0.9])
    z = np.array([0.0, 0.4j, 0.3 + 0.02j])
    d = oracle.energy_factor_dE(e_v, e_c, z)
    h = 1e-6
    fd = (oracle.energy_factor(e_v + h, e_c, z) - oracle.energy_factor(e_v - h, e_c, z)) / (2 * h)
    # each E_v shift moves both pairs of that v, so compare per pair
    assert np.allclose(d, fd, rtol=1e-7, atol=1e-7)
    fdc = (oracle.energy_factor(e_v, e_c + h, z) - oracle.energy_factor(e_v, e_c - h, z)) / (2 * h)
    assert np.allclose(-d, fdc, rtol=1e-7, atol=1e-7)


# ---------------------------------------------------------------- chi0

def test_plane_wave_chi_closed_form():
    """chi_GG'(z) = s delta_GG' sum over pairs with k_v - k_c = G of Delta_vc(z)."""
    n = (8, 8, 8)
    kv = [(0, 0, 0), (1, 0, 0)]
    kc = [(1, 0, 0), (2, 0, 0), (0, 1, 0), (0, 0, 3), (-1, 0, 0)]
    pv, pc = _plane_waves(kv, n), _plane_waves(kc, n)
    e_v = np.array([-0.2, -0.35])
    e_c = np.array([0.1, 0.3, 0.45, 0.8, 1.05])
    z = np.array([0.0, 0.6j, 0.25 + 0.005j])
    gl = gen.gsphere(10)
    chi = oracle.chi0(pv, pc, e_v, e_c, gl, z, n, VOL, spin=2.0, pair_chunk=3)
    want = np.zeros_like(chi)
    for w, zz in enumerate(z):
        for v, c in itertools.product(range(2), range(5)):
            gdiff = np.array(kv[v]) - np.array(kc[c])
            hit = np.where(np.all(gl == gdiff, axis=1))[0]
            de = e_v[v] - e_c[c]
            if hit.size:
                want[w, hit[0], hit[0]] += 2.0 * (1 / (de + zz) + 1 / (de - zz))
    assert np.abs(chi - want).max() < 1e-12 * np.abs(want).max()


def test_chi0_brute_force_quadruple_loop():
    n = (4, 4, 6)
    rng = np.random.default_rng(17)
    psi = _bands(rng, 5, n)
    pv, pc = psi[:2], psi[2:]
    e_v, e_c = np.array([-0.3, -0.05]), np.array([0.1, 0.6, 0.9])
    g = np.array([[0, 0, 0], [1, 0, -1], [0, -2, 2], [-1, 1, 1]], np.int32)
    z = np.array([0.3j, 0.4 + 0.01j])
    chi = oracle.chi0(pv, pc, e_v, e_c, g, z, n, VOL, spin=2.0, pair_chunk=4)
    for w, zz in enumerate(z):
        for i, j in itertools.product(range(4), range(4)):
            acc = 0j
            for v, c in itertools.product(range(2), range(3)):
                de = e_v[v] - e_c[c]
                delta = 1 / (de + zz) + 1 / (de - zz)
                acc += _brute_m(pv[v], pc[c], g[i], n).conjugate() * delta * _brute_m(pv[v], pc[c], g[j], n)
            assert abs(chi[w, i, j] - 2 * acc) < 1e-12 * max(1e-3, abs(acc))


def _small_problem(seed=21, n=(6, 6, 6), nv=3, nc=7, r2=3, z=(0.0, 0.5j, 0.3 + 0.005j)):
    return gen.make_problem(n, nv, nc, r2=r2, z=z, seed=seed, pair_chunk=5)


def _chi(p, **kw):
    args = dict(spin=p.spin, pair_chunk=p.pair_chunk)
    args.update(kw)
    return oracle.chi0(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec, p.z, p.n, p.volume, **args)


def test_chi0_trace_identity_full_grid():
    n = (4, 6, 4)
    p = gen.make_problem(n, 2, 5, gvec=_all_g(n), z=(0.0, 0.7j), seed=2)
    chi = _chi(p)
    dv = p.volume / np.prod(n)
    delta = oracle.energy_factor(p.e_v, p.e_c, p.z)
    for w in range(2):
        rhs = 0j
        for v, c in itertools.product(range(2), range(5)):
            rho2 = np.sum(np.abs(p.psi_v[v]) ** 2 * np.abs(p.psi_c[c]) ** 2)
            rhs += 2.0 * delta[w, v * 5 + c] * p.volume * dv * rho2
        assert abs(np.trace(chi[w]) - rhs) < 1e-12 * abs(rhs)


def test_chi0_hermiticity_and_conjugate_frequency():
    p = _small_problem(z=(0.0, 0.8j, 0.4 + 0.01j, 0.4 - 0.01j))
    chi = _chi(p)
    for w in (0, 1):
        assert np.abs(chi[w] - chi[w].conj().T).max() < 1e-13 * np.abs(chi[w]).max()
    # chi(z)^H = chi(conj z)
    assert np.abs(chi[2].conj().T - chi[3]).max() < 1e-13 * np.abs(chi[2]).max()
    # a complex frequency is not Hermitian (catches a dropped conj/transposition)
    assert np.abs(chi[2] - chi[2].conj().T).max() > 1e-6 * np.abs(chi[2]).max()


def test_chi0_negative_semidefinite_and_rank():
    p = _small_problem(nv=2, nc=3, r2=6, z=(0.0, 1.3j))
    chi = _chi(p)
    assert chi.shape[1] > p.npairs          # more G than pairs -> rank deficient
    for w in range(2):
        ev = np.linalg.eigvalsh(chi[w])
        assert ev.max() <= 1e-13 * np.abs(ev).max()
        assert np.sum(np.abs(ev) > 1e-10 * np.abs(ev).max()) <= p.npairs


def test_chi0_head_and_wings_vanish_at_q0():
    p = _small_problem()
    chi = _chi(p)
    assert tuple(p.gvec[0]) == (0, 0, 0)
    scale = np.abs(chi).max()
    assert np.abs(chi[:, 0, :]).max() < 1e-13 * scale
    assert np.abs(chi[:, :, 0]).max() < 1e-13 * scale


def test_chi0_invariances():
    p = _small_problem()
    ref = _chi(p)
    scale = np.abs(ref).max()
    rng = np.random.default_rng(1)
    # band phases
    q = gen.Problem(**{**p.__dict__})
    q.psi_v = p.psi_v * np.exp(1j * rng.uniform(0, 2 * np.pi, p.nv))[:, None]
    q.psi_c = p.psi_c * np.exp(1j * rng.uniform(0, 2 * np.pi, p.nc))[:, None]
    assert np.abs(_chi(q) - ref).max() < 1e-13 * scale
    # common energy shift
    q = gen.Problem(**{**p.__dict__})
    q.e_v, q.e_c = p.e_v + 0.123, p.e_c + 0.123
    assert np.abs(_chi(q) - ref).max() < 1e-12 * scale
    # pair order: permute conduction bands together with their energies
    perm = rng.permutation(p.nc)
    q = gen.Problem(**{**p.__dict__})
    q.psi_c, q.e_c = p.psi_c[perm], p.e_c[perm]
    assert np.abs(_chi(q) - ref).max() < 1e-13 * scale
    # chunk size
    for chunk in (1, 4, 1000):
        assert np.abs(_chi(p, pair_chunk=chunk) - ref).max() < 1e-13 * scale


def test_chi0_single_pair_rank_one():
    p = _small_problem(nv=1, nc=1)
    chi = _chi(p)
    m = oracle.mtxel(p.psi_v, p.psi_c, p.gvec, p.n, p.volume)[0]
    delta = oracle.energy_factor(p.e_v, p.e_c, p.z)[:, 0]
    for w in range(len(p.z)):
        want = 2.0 * delta[w] * np.outer(m.conj(), m)
        assert np.abs(chi[w] - want).max() < 1e-14 * np.abs(want).max()


def test_chi0_entries_match_full():
    p = _small_problem(n=(8, 6, 10), r2=5)
    chi = _chi(p)
    rows, cols = [0, 3, 7], [1, 2, 8, 11]
    e = oracle.chi0_entries(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec[rows], p.gvec[cols], p.z,
                            p.n, p.volume, p.spin)
    assert np.abs(e - chi[:, rows][:, :, cols]).max() < 1e-13 * np.abs(chi).max()


# ---------------------------------------------------------------- adjoint

def _loss(p, a):
    chi = _chi(p)
    return float(np.real(np.sum(a * chi, axis=(1, 2)).sum()))


def _rand_herm(rng, nz, ng):
    x = rng.standard_normal((nz, ng, ng)) + 1j * rng.standard_normal((nz, ng, ng))
    return 0.5 * (x + np.conj(np.transpose(x, (0, 2, 1))))


def test_adjoint_matches_central_differences():
    """L = Re sum_w tr(A_w chi_w) with A Hermitian: dL/dchi = A^T = conj(A), i.e.
    W = conj(A) in the torch convention (dL = Re sum conj(W) dchi)."""
    rng = np.random.default_rng(3)
    p = _small_problem(nv=2, nc=3, r2=3, z=(0.0, 0.7j, 0.2 + 0.01j))
    a = _rand_herm(rng, len(p.z), p.ng)
    # tr(A chi) = sum_ij A_ji chi_ij -> dL/dchi_ij (torch) = conj(A_ji)... = conj(A^T)_ij
    w = np.conj(np.transpose(a, (0, 2, 1)))
    gv, gc, gev, gec = oracle.chi0_backward(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec, p.z, p.n,
                                            p.volume, w, spin=p.spin, pair_chunk=p.pair_chunk)
    tr = lambda q: float(np.real(sum(np.trace(a[k] @ _chi(q)[k]) for k in range(len(p.z)))))
    h = 1e-6
    for trial in range(3):
        for which in ("psi_v", "psi_c", "e"):
            q_plus = gen.Problem(**{**p.__dict__})
            q_minus = gen.Problem(**{**p.__dict__})
            if which == "e":
                dv_, dc_ = rng.standard_normal(p.nv), rng.standard_normal(p.nc)
                q_plus.e_v, q_plus.e_c = p.e_v + h * dv_, p.e_c + h * dc_
                q_minus.e_v, q_minus.e_c = p.e_v - h * dv_, p.e_c - h * dc_
                pred = gev @ dv_ + gec @ dc_
            else:
                x = getattr(p, which)
                d = rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape)
                setattr(q_plus, which, x + h * d)
                setattr(q_minus, which, x - h * d)
                g = gv if which == "psi_v" else gc
                pred = float(np.real(np.sum(np.conj(g) * d)))
            fd = (tr(q_plus) - tr(q_minus)) / (2 * h)
            assert abs(fd - pred) < 1e-6 * max(1.0, abs(fd)), (which, fd, pred)


def test_adjoint_invariances():
    rng = np.random.default_rng(4)
    p = _small_problem(nv=2, nc=4, r2=3, z=(0.0, 0.9j))
    a = _rand_herm(rng, len(p.z), p.ng)
    w = np.conj(np.transpose(a, (0, 2, 1)))
    gv, gc, gev, gec = oracle.chi0_backward(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec, p.z, p.n,
                                            p.volume, w, spin=p.spin, pair_chunk=3)
    scale = np.abs(gev).max() + np.abs(gec).max()
    assert abs(gev.sum() + gec.sum()) < 1e-12 * scale                 # energy shift
    for x, g in ((p.psi_v, gv), (p.psi_c, gc)):                        # band phases
        im = np.imag(np.sum(np.conj(g) * x, axis=1))
        assert np.abs(im).max() < 1e-11 * np.abs(g).max() * np.abs(x).max() * x.shape[1]


def test_adjoint_plane_wave_energy_gradient():
    """For plane waves, L = Re sum_w tr(A chi_w) = s sum_pairs Re[A_GG Delta(z)] for
    the G hit by each pair, so dL/dE_v = s sum Re[A_GG dDelta/dE_v]."""
    n = (6, 6, 6)
    kv = [(0, 0, 0), (1, 1, 0)]
    kc = [(1, 0, 0), (0, 0, 1), (2, 1, 0)]
    pv, pc = _plane_waves(kv, n), _plane_waves(kc, n)
    e_v, e_c = np.array([-0.2, -0.1]), np.array([0.3, 0.5, 0.8])
    gl = gen.gsphere(3)
    z = np.array([0.0, 0.5j])
    rng = np.random.default_rng(8)
    a = _rand_herm(rng, 2, len(gl))
    w = np.conj(np.transpose(a, (0, 2, 1)))
    _, _, gev, gec = oracle.chi0_backward(pv, pc, e_v, e_c, gl, z, n, VOL, w, spin=2.0)
    want_v, want_c = np.zeros(2), np.zeros(3)
    for wi, zz in enumerate(z):
        for v, c in itertools.product(range(2), range(3)):
            gdiff = np.array(kv[v]) - np.array(kc[c])
            hit = np.where(np.all(gl == gdiff, axis=1))[0]
            if not hit.size:
                continue
            de = e_v[v] - e_c[c]
            dd = -1 / (de + zz) ** 2 - 1 / (de - zz) ** 2
            val = 2.0 * np.real(a[wi, hit[0], hit[0]] * dd)
            want_v[v] += val
            want_c[c] -= val
    assert np.abs(gev - want_v).max() < 1e-12 * np.abs(want_v).max()
    assert np.abs(gec - want_c).max() < 1e-12 * np.abs(want_v).max()


# ---------------------------------------------------------------- pseudobands

def _orthonormal_bands(nb, n=(6, 5, 4), seed=3):
    p = gen.make_problem(n, 1, nb, r2=1, z=(0.0,), seed=seed)
    return p.psi_c, p.e_c, p.volume / np.prod(n)


def test_pseudobands_norm_identity():
    """For orthonormal bands, dV ||xi_j^S||^2 = |S| / n_xi for every draw of
    the phases: the cross terms vanish by orthogonality."""
    psi, e, dv = _orthonormal_bands(9)
    rng = np.random.default_rng(11)
    slices = [np.array([0, 3, 4, 8]), np.array([1, 2]), np.array([5, 6, 7])]
    n_xi = 3
    theta = [rng.random((n_xi, len(s))) for s in slices]
    out, eo = oracle.pseudobands(psi, e, [], slices, n_xi, theta)
    norms = dv * np.sum(np.abs(out) ** 2, axis=1)
    expect = np.repeat([len(s) / n_xi for s in slices], n_xi)
    assert np.allclose(norms, expect, rtol=0, atol=1e-12)
    assert np.allclose(eo, np.repeat([e[s].mean() for s in slices], n_xi), rtol=0, atol=0)


def test_pseudobands_phase_average_is_slice_projector():
    """Averaged over every pattern of quarter-turn phases (4^|S| of them), the
    single pseudoband's outer product xi xi^H is exactly the slice projector
    sum_{n in S} psi_n psi_n^H: sum_k exp(2 pi i k a / 4) over k vanishes
    unless a = 0 mod 4."""
    psi, e, dv = _orthonormal_bands(5, n=(3, 2, 2))
    s = np.array([0, 2, 3])
    proj = sum(np.outer(psi[i], np.conj(psi[i])) for i in s)
    acc = np.zeros_like(proj)
    pats = list(itertools.product(range(4), repeat=len(s)))
    for pat in pats:
        th = [np.array([[q / 4.0 for q in pat]])]
        xi, _ = oracle.pseudobands(psi, e, [], [s], 1, th)
        acc += np.outer(xi[0], np.conj(xi[0]))
    assert np.abs(acc / len(pats) - proj).max() < 1e-13 * np.abs(proj).max()


def test_pseudobands_singletons_leave_chi0_unchanged():
    """Slices of one band with one pseudoband each only rephase the bands,
    and chi0 depends on conj(M) M: it is unchanged; protected bands pass
    through."""
    p = gen.make_problem((8, 6, 6), 2, 7, r2=4, z=(0.0, 0.3 + 0.01j), seed=12)
    rng = np.random.default_rng(4)
    slices = [np.array([i]) for i in range(2, 7)]
    theta = [rng.random((1, 1)) for _ in slices]
    pc, ec = oracle.pseudobands(p.psi_c, p.e_c, [0, 1], slices, 1, theta)
    assert np.array_equal(pc[:2], p.psi_c[:2]) and np.array_equal(ec, p.e_c)
    ref = oracle.chi0(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec, p.z, p.n, p.volume)
    got = oracle.chi0(p.psi_v, pc, p.e_v, ec, p.gvec, p.z, p.n, p.volume)
    assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()


# ---------------------------------------------------------------- static subspace (Eq. (6))

def _subspace_problem(seed=31, z=(0.0, 0.9j, 0.35 + 0.01j)):
    return gen.make_problem((6, 6, 6), 3, 14, r2=6, z=z, seed=seed, pair_chunk=7)


def test_subspace_basis_from_known_spectrum():
    """A Hermitian matrix built from a chosen spectrum (mixed magnitudes,
    non-positive, one degenerate pair below the cut): the basis spans the
    eigenvectors of the largest |eigenvalues|, in decreasing |eigenvalue|."""
    rng = np.random.default_rng(5)
    ng = 12
    x = rng.standard_normal((ng, ng)) + 1j * rng.standard_normal((ng, ng))
    u, _ = np.linalg.qr(x)
    lam = -np.array([9.0, 0.1, 4.0, 7.5, 0.0, 2.0, 0.3, 6.0, 1.0, 0.3, 5.0, 0.05])
    a = (u * lam[None, :]) @ u.conj().T
    cs, ev = oracle.static_subspace_basis(a, 5)
    assert np.allclose(ev, [-9.0, -7.5, -6.0, -5.0, -4.0], rtol=0, atol=1e-12)
    keep = [0, 3, 7, 10, 2]
    proj = cs @ cs.conj().T
    want = u[:, keep] @ u[:, keep].conj().T
    assert np.abs(proj - want).max() < 1e-12
    assert np.abs(cs.conj().T @ cs - np.eye(5)).max() < 1e-12
    assert np.abs(a @ cs - cs * ev[None, :]).max() < 1e-12


def test_subspace_full_basis_reproduces_chi():
    """With n_eig = N_G the basis is unitary and C_s chi_B C_s^H is the chi of
    Eq. (4) at every frequency."""
    p = _subspace_problem()
    chi = _chi(p)
    cs, _ = oracle.static_subspace_basis(chi[0], p.ng)
    assert np.abs(cs.conj().T @ cs - np.eye(p.ng)).max() < 1e-12
    chib = oracle.chi0_subspace(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec, p.z, p.n, p.volume, cs,
                                spin=p.spin, pair_chunk=p.pair_chunk)
    back = np.einsum("gb,wbc,hc->wgh", cs, chib, cs.conj())
    assert np.abs(back - chi).max() < 1e-12 * np.abs(chi).max()


def test_subspace_static_chi_is_diagonal():
    """In its own eigenbasis the static chi is diagonal with the eigenvalues,
    and the subspace chi is Hermitian and negative semidefinite on the
    imaginary axis, not Hermitian on the real axis."""
    p = _subspace_problem(seed=32)
    chi0 = _chi(p)[0]
    cs, ev = oracle.static_subspace_basis(chi0, 9)
    chib = oracle.chi0_subspace(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec, p.z, p.n, p.volume, cs,
                                spin=p.spin, pair_chunk=p.pair_chunk)
    scale = np.abs(ev).max()
    assert np.abs(chib[0] - np.diag(ev)).max() < 1e-12 * scale
    for w in (0, 1):
        assert np.abs(chib[w] - chib[w].conj().T).max() < 1e-13 * scale
        assert np.linalg.eigvalsh(chib[w]).max() <= 1e-13 * scale
    assert np.abs(chib[2] - chib[2].conj().T).max() > 1e-6 * scale


def test_subspace_matches_projection_identity():
    """The paper's identity chi_BB' = sum_GG' conj(C_s^GB) chi_GG' C_s^G'B' on a
    partial basis, the two sides computed along different routes (transformed
    matrix elements vs the projected full chi)."""
    p = _subspace_problem(seed=33)
    chi = _chi(p)
    cs, _ = oracle.static_subspace_basis(chi[0], 7)
    chib = oracle.chi0_subspace(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec, p.z, p.n, p.volume, cs,
                                spin=p.spin, pair_chunk=3)
    proj = np.einsum("gb,wgh,hc->wbc", cs.conj(), chi, cs)
    assert np.abs(chib - proj).max() < 1e-12 * np.abs(proj).max()


def test_subspace_plane_waves():
    """Plane waves make chi diagonal: the basis is the unit vectors of the G
    with the largest |chi_GG(0)| (up to phase) and chi_B(z) is diagonal with
    those chi_GG(z), the plane-wave closed form."""
    n = (8, 8, 8)
    kv = [(0, 0, 0), (1, 0, 0)]
    kc = [(1, 0, 0), (2, 0, 0), (0, 1, 0), (0, 0, 2), (-1, 0, 0)]
    pv, pc = _plane_waves(kv, n), _plane_waves(kc, n)
    e_v = np.array([-0.2, -0.35])
    e_c = np.array([0.1, 0.3, 0.45, 0.8, 1.05])
    z = np.array([0.0, 0.6j, 0.25 + 0.005j])
    gl = gen.gsphere(6)
    want = np.zeros((3, gl.shape[0]), dtype=np.complex128)   # closed-form diagonal
    for w, zz in enumerate(z):
        for v, c in itertools.product(range(2), range(5)):
            hit = np.where(np.all(gl == np.array(kv[v]) - np.array(kc[c]), axis=1))[0]
            de = e_v[v] - e_c[c]
            if hit.size:
                want[w, hit[0]] += 2.0 * (1 / (de + zz) + 1 / (de - zz))
    chi_static = np.diag(want[0])
    n_eig = 4
    cs, ev = oracle.static_subspace_basis(chi_static, n_eig)
    top = np.argsort(-np.abs(want[0].real), kind="stable")[:n_eig]
    assert len(set(np.abs(want[0].real[top]).round(12))) == n_eig   # distinct: unique basis
    assert np.allclose(np.abs(cs[top, range(n_eig)]), 1.0, atol=1e-14)
    chib = oracle.chi0_subspace(pv, pc, e_v, e_c, gl, z, n, VOL, cs, spin=2.0, pair_chunk=4)
    for w in range(3):
        assert np.abs(chib[w] - np.diag(want[w, top])).max() < 1e-12 * np.abs(want).max()


def test_subspace_weighted_plane_waves():
    """The symmetrised form W chi W with plane waves: the kept G are those of
    largest w_G^2 |chi_GG(0)| (a different set from the unweighted one here),
    the eigenvalues are w_G^2 chi_GG(0) and chi_B(z) is diag(w_G^2 chi_GG(z)):
    one factor w per matrix element, so a weight applied twice, or to only one
    side, fails."""
    n = (8, 8, 8)
    kv = [(0, 0, 0), (1, 0, 0)]
    kc = [(1, 0, 0), (2, 0, 0), (0, 1, 0), (0, 0, 2), (-1, 0, 0)]
    pv, pc = _plane_waves(kv, n), _plane_waves(kc, n)
    e_v = np.array([-0.2, -0.35])
    e_c = np.array([0.1, 0.3, 0.45, 0.8, 1.05])
    z = np.array([0.0, 0.6j, 0.25 + 0.005j])
    gl = gen.gsphere(6)
    want = np.zeros((3, gl.shape[0]), dtype=np.complex128)
    for w, zz in enumerate(z):
        for v, c in itertools.product(range(2), range(5)):
            hit = np.where(np.all(gl == np.array(kv[v]) - np.array(kc[c]), axis=1))[0]
            de = e_v[v] - e_c[c]
            if hit.size:
                want[w, hit[0]] += 2.0 * (1 / (de + zz) + 1 / (de - zz))
    wt = np.sqrt(oracle.coulomb(gl, q=(0.1, 0.2, -0.3), cell_l=L))
    n_eig = 3
    cs, ev = oracle.static_subspace_basis(np.diag(want[0]), n_eig, weight=wt)
    scaled = wt ** 2 * want[0].real
    top = np.argsort(-np.abs(scaled), kind="stable")[:n_eig]
    plain = np.argsort(-np.abs(want[0].real), kind="stable")[:n_eig]
    assert set(top) != set(plain)
    assert len(set(np.abs(scaled[top]).round(12))) == n_eig
    assert np.allclose(ev, scaled[top], rtol=1e-14, atol=0)
    assert np.allclose(np.abs(cs[top, range(n_eig)]), 1.0, atol=1e-14)
    chib = oracle.chi0_subspace(pv, pc, e_v, e_c, gl, z, n, VOL, cs, spin=2.0, pair_chunk=4,
                                weight=wt)
    for w in range(3):
        d = wt[top] ** 2 * want[w, top]
        assert np.abs(chib[w] - np.diag(d)).max() < 1e-12 * np.abs(d).max()


def test_subspace_weighted_full_basis():
    """With a weight and n_eig = N_G, C_s chi_B C_s^H = W chi W at every
    frequency (chi from Eq. (4) directly), the eigenvalues sum to the trace of
    W chi(0) W, and with unit weights the weighted basis is the plain one."""
    p = _subspace_problem(seed=34)
    chi = _chi(p)
    wt = np.sqrt(oracle.coulomb(p.gvec, q=(0.05, -0.1, 0.15), cell_l=L))
    cs, ev = oracle.static_subspace_basis(chi[0], p.ng, weight=wt)
    wchiw = wt[None, :, None] * chi * wt[None, None, :]
    assert abs(ev.sum() - np.trace(wchiw[0]).real) < 1e-12 * np.abs(ev).sum()
    chib = oracle.chi0_subspace(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec, p.z, p.n, p.volume, cs,
                                spin=p.spin, pair_chunk=p.pair_chunk, weight=wt)
    back = np.einsum("gb,wbc,hc->wgh", cs, chib, cs.conj())
    assert np.abs(back - wchiw).max() < 1e-12 * np.abs(wchiw).max()
    c1, e1 = oracle.static_subspace_basis(chi[0], 6, weight=np.ones(p.ng))
    c0, e0 = oracle.static_subspace_basis(chi[0], 6)
    assert np.array_equal(e1, e0) and np.array_equal(c1, c0)


# ---------------------------------------------------------------- inverse dielectric matrix (Eq. (3))

def test_coulomb_closed_form():
    g = np.array([[0, 0, 0], [1, 0, 0], [0, -2, 0], [1, 1, 1]], np.int32)
    v = oracle.coulomb(g, cell_l=L)
    b = 2 * np.pi / L
    assert v[0] == 0.0                                   # the q = 0 head, read as excluded
    assert np.allclose(v[1:], 4 * np.pi / (b * b * np.array([1.0, 4.0, 3.0])), rtol=1e-15)
    vq = oracle.coulomb(g, q=(0.25, 0.0, 0.0), cell_l=L)
    assert np.isclose(vq[0], 4 * np.pi / (0.25 * b) ** 2, rtol=1e-15)
    assert np.isclose(vq[1], 4 * np.pi / (1.25 * b) ** 2, rtol=1e-15)


def test_epsilon_inverse_identity_and_diagonal():
    rng = np.random.default_rng(8)
    ng = 9
    chi = rng.standard_normal((2, ng, ng)) + 1j * rng.standard_normal((2, ng, ng))
    assert np.abs(oracle.epsilon_inverse(chi, np.zeros(ng)) - np.eye(ng)).max() == 0.0
    d = -rng.uniform(0.1, 2.0, ng)
    v = rng.uniform(0.5, 3.0, ng)
    got = oracle.epsilon_inverse(np.diag(d)[None], v)[0]
    assert np.abs(got - np.diag(1.0 / (1.0 - v * d))).max() < 1e-15


def test_epsilon_inverse_rank_one_sherman_morrison():
    """chi = a u u^H: [I - v a u u^H]^-1 = I + a (v u) u^H / (1 - a u^H v u)."""
    rng = np.random.default_rng(9)
    ng = 11
    u = rng.standard_normal(ng) + 1j * rng.standard_normal(ng)
    v = rng.uniform(0.2, 1.5, ng)
    for a in (-0.7, 0.3 + 0.2j):
        chi = a * np.outer(u, u.conj())
        x = a * v * u
        want = np.eye(ng) + np.outer(x, u.conj()) / (1.0 - u.conj() @ x)
        got = oracle.epsilon_inverse(chi[None], v)[0]
        assert np.abs(got - want).max() < 1e-13 * np.abs(want).max()


def test_epsilon_inverse_symmetrised_form():
    """For a Hermitian negative semidefinite chi (imaginary axis) the
    symmetrised eps~ = I - v^1/2 chi v^1/2 is Hermitian with eigenvalues >= 1,
    and eps^-1 = v^1/2 eps~^-1 v^-1/2: eps^-1 is similar to a Hermitian
    matrix with eigenvalues in (0, 1]."""
    p = _small_problem(z=(0.0, 0.7j))
    chi = _chi(p)
    v = oracle.coulomb(p.gvec, cell_l=p.volume ** (1 / 3))
    einv = oracle.epsilon_inverse(chi, v)
    sq = np.sqrt(v)
    keep = v > 0
    for w in range(2):
        et = np.eye(p.ng) - sq[:, None] * chi[w] * sq[None, :]
        lam = np.linalg.eigvalsh(et)
        assert lam.min() >= 1.0 - 1e-12
        sym = sq[keep, None] * np.linalg.inv(et)[np.ix_(keep, keep)] / sq[None, keep]
        assert np.abs(einv[w][np.ix_(keep, keep)] - sym).max() < 1e-12 * np.abs(sym).max()
        # the excluded head: row and column of G = 0 are those of the identity
        assert np.abs(einv[w][0] - np.eye(p.ng)[0]).max() < 1e-12
        assert np.abs(einv[w][:, 0] - np.eye(p.ng)[:, 0]).max() < 1e-12
        ev = np.linalg.eigvals(einv[w])
        assert np.all(ev.real > 0) and ev.real.max() <= 1.0 + 1e-12


# ---------------------------------------------------------------- GPP off-diagonal self-energy

def _gpp_inputs(seed=5, nb=3, ns=4, ng=6, ne=3):
    rng = np.random.default_rng(seed)
    m = rng.standard_normal((nb, ns, ng)) + 1j * rng.standard_normal((nb, ns, ng))
    e_n = np.sort(rng.uniform(-0.5, 1.0, nb))
    occ = e_n < 0.1
    x = rng.standard_normal((ng, ng)) + 1j * rng.standard_normal((ng, ng))
    omega2 = 0.5 * (x + x.conj().T)
    wt = rng.uniform(0.3, 1.5, (ng, ng))
    wt = 0.5 * (wt + wt.T)
    v = rng.uniform(0.1, 2.0, ng)
    energies = np.linspace(-0.6, 1.2, ne) + 0.05j
    return m, e_n, occ, energies, omega2, wt, v


def test_gpp_offdiag_brute_force():
    """Scalar loops over E, l, m, n, G, G' with the plasmon-pole term written
    out, against the GEMM-pair form."""
    m, e_n, occ, energies, omega2, wt, v = _gpp_inputs()
    got = oracle.gpp_sigma_offdiag(m, e_n, occ, energies, omega2, wt, v)
    nb, ns, ng = m.shape
    for i, e in enumerate(energies):
        for l, mm in itertools.product(range(ns), range(ns)):
            acc = 0j
            for n in range(nb):
                sgn = -1.0 if occ[n] else 1.0
                for g, h in itertools.product(range(ng), range(ng)):
                    pole = e - e_n[n] - sgn * wt[g, h]
                    acc += (m[n, l, g].conjugate() * omega2[g, h] * v[h] * m[n, mm, h]
                            / (2.0 * wt[g, h] * pole))
            assert abs(got[i, l, mm] - acc) < 1e-12 * max(1.0, abs(acc))


def test_gpp_offdiag_band_additivity_and_occupation():
    """The bands add; flipping a band's occupation moves its pole from
    E_n + wt to E_n - wt (a different result)."""
    m, e_n, occ, energies, omega2, wt, v = _gpp_inputs(seed=6, nb=4)
    full = oracle.gpp_sigma_offdiag(m, e_n, occ, energies, omega2, wt, v)
    a = oracle.gpp_sigma_offdiag(m[:2], e_n[:2], occ[:2], energies, omega2, wt, v)
    b = oracle.gpp_sigma_offdiag(m[2:], e_n[2:], occ[2:], energies, omega2, wt, v)
    assert np.abs(full - a - b).max() < 1e-13 * np.abs(full).max()
    flip = oracle.gpp_sigma_offdiag(m, e_n, ~occ, energies, omega2, wt, v)
    assert np.abs(flip - full).max() > 1e-3 * np.abs(full).max()
    # a single G: Sigma = sum_n conj(M_n) M_n^T * Omega2 v / (2 wt (E - E_n - s wt))
    one = oracle.gpp_sigma_offdiag(m[:, :, :1], e_n, occ, energies, omega2[:1, :1], wt[:1, :1],
                                   v[:1])
    for i, e in enumerate(energies):
        want = sum(np.outer(m[n, :, 0].conj(), m[n, :, 0]) * omega2[0, 0] * v[0]
                   / (2 * wt[0, 0] * (e - e_n[n] - (-1.0 if occ[n] else 1.0) * wt[0, 0]))
                   for n in range(m.shape[0]))
        assert np.abs(one[i] - want).max() < 1e-13 * np.abs(want).max()
