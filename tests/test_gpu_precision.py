"""Reduced-precision CHI0 paths (FP32, split BF16/FP16) against the FP64 oracle.

Every result is compared with the exact FP64 chi and with an a-posteriori
bound derived from the slicing definition (fixed-point slices with a common
exponent per block of pairs (64 for FP16, 128 for BF16) and per G):

* each operand element x of block b and column g satisfies
  |Re x|, |Im x| < 2^e, and after S slices the residual of each component is
  at most 2^(e - 8 S - 1), so |x - x~| <= eps = sqrt(2) 2^(e - 8 S - 1);
* slice s carries at most |q_0| 2^(e-8) <= 2^e (s = 0) or 128 2^(e-8-8s)
  (s >= 1) per component; products with sa + sb >= S are dropped;
* FP16: one FP32 accumulator per shift t = sa + sb; those with t <= 2 hold
  integer sums below 2^24 and are exact, those with t >= 3 round;
* BF16: slices are stored scaled (q_s 2^-8s) and t = 0, t = 1 and t >= 2
  share three accumulators; the first two are exact, the third rounds.

Per output, |chi~ - chi| <= s * sum_p [ |a_p| eps_b + eps_a |b~_p| + dropped_p ]
+ FP32 rounding of the small-term accumulator + FP64 rounding.
"""
import numpy as np
import pytest

import oracle
import paper_2509_23018_amd as gw
from gpu_helpers import FP64_TOL, rel_fro, run_chi0
from workloads import gen

pytestmark = pytest.mark.gpu

KB = 64


def _operands(p):
    m = oracle.mtxel(p.psi_v, p.psi_c, p.gvec, p.n, p.volume)          # [K, ng]
    d = oracle.energy_factor(p.e_v, p.e_c, p.z) * p.spin                 # [nz, K]
    return m, d


def _blocks(x, kb):
    """Per (block of kb pairs, column): exponent e with max(|Re|,|Im|) < 2^e."""
    k = x.shape[0]
    nkb = (k + kb - 1) // kb
    e = np.zeros((nkb, x.shape[1]))
    for b in range(nkb):
        blk = x[b * kb:(b + 1) * kb]
        mx = np.maximum(np.abs(blk.real), np.abs(blk.imag)).max(axis=0)
        e[b] = np.where(mx > 0, np.frexp(mx)[1], 0)
    return e


def _chunk_ranges(nv, nc, chunk):
    """The library streams pairs in rectangles of vb valence x cw conduction
    bands; each is a consecutive range of p = v*nc + c."""
    cw = max(1, min(nc, chunk // max(1, min(nv, 4))))
    vb = max(1, min(nv, chunk // cw))
    out = []
    for v0 in range(0, nv, vb):
        for c0 in range(0, nc, cw):
            vs = range(v0, min(nv, v0 + vb))
            out.append(np.array([v * nc + c for v in vs for c in range(c0, min(nc, c0 + cw))]))
    return out


def split_bound(m, d, S, nv, nc, chunk, first_rounded=3, kb=KB, m_cols=None, bits=8):
    """Elementwise bound on |chi_split - chi| for one frequency (d = s*Delta).
    Products with sa + sb >= first_rounded share FP32 accumulators that round
    (BF16 and 9-bit FP16: t >= 2 in one group; FP16: one group per t, t >= 3
    rounding).  bits: slice width (8, or 9 for the 9-bit FP16 slices: the
    residual after S slices is 2^(e - 9 S - 1) per component, slice s >= 1
    at most 2^(e - 1 - 9 s)).
    m holds M at the rows' G; m_cols, if given, M at the columns' G (the
    bound of entry (i, j) depends only on columns i of m and j of m_cols)."""
    m_cols = m if m_cols is None else m_cols
    shape = (m.shape[1], m_cols.shape[1])
    bound = np.zeros(shape)
    amp = lambda e, s: np.where(s == 0, 2.0 ** e, 2.0 ** (e - 1 - bits * s))
    for idx in _chunk_ranges(nv, nc, chunk):
        a = m[idx]
        b = d[idx, None] * m_cols[idx]
        ea, eb = _blocks(a, kb), _blocks(b, kb)
        for blk in range(ea.shape[0]):
            sl = slice(blk * kb, (blk + 1) * kb)
            aa, bb = np.abs(a[sl]), np.abs(b[sl])                         # [kb, ng]
            n = aa.shape[0]
            eps_a = np.sqrt(2) * 2.0 ** (ea[blk] - bits * S - 1)
            eps_b = np.sqrt(2) * 2.0 ** (eb[blk] - bits * S - 1)
            trunc = np.outer(aa.sum(0), eps_b) + np.outer(eps_a, bb.sum(0) + n * eps_b)
            dropped = np.zeros(shape)
            small = np.zeros(shape)
            for sa in range(S):
                for sb in range(S):
                    # complex slice magnitudes <= 2 * amp_a * amp_b (two components each)
                    w = 2.0 * np.outer(amp(ea[blk], sa), amp(eb[blk], sb))
                    if sa + sb >= S:
                        dropped += n * w
                    elif sa + sb >= first_rounded:
                        small += n * w
            # FP32 rounding of the accumulators with sa + sb >= first_rounded: at
            # most 4 n S^2 adds, each off by 2^-24 of a running sum bounded by `small`
            bound += trunc + dropped + 4 * n * S * S * 2.0 ** -24 * small
    return bound


def _problem(z, seed=31):
    return gen.make_problem((20, 18, 24), 5, 41, r2=15, z=z, seed=seed, pair_chunk=150)


@pytest.mark.parametrize("prec", ["split_bf16", "split_fp16"])
def test_split_error_within_bound_and_monotone(prec):
    p = _problem((0.0, 0.4j, 0.35 + 0.005j))
    ref = oracle.chi0(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec, p.z, p.n, p.volume,
                      spin=p.spin, pair_chunk=p.pair_chunk)
    m, d = _operands(p)
    errs = []
    for S in (2, 3, 4, 5, 6):
        got = run_chi0(p, precision=prec, n_slices=S)
        err = rel_fro(got, ref)
        errs.append(err)
        for w in range(len(p.z)):
            bf = prec == "split_bf16"
            bnd = split_bound(m, d[w], S, p.nv, p.nc, p.pair_chunk,
                              first_rounded=2 if bf else 3, kb=128 if bf else 64)
            # Hermitian frequencies mirror the upper tiles: bound their transpose too
            bnd = np.maximum(bnd, bnd.T)
            excess = np.abs(got[w] - ref[w]) - bnd - 1e-15 * np.abs(ref[w]).max()
            assert excess.max() <= 0, (prec, S, w, excess.max())
    assert all(errs[i + 1] < errs[i] for i in range(3)), errs
    assert errs[3] <= 1e-10, errs        # five slices meet 1e-10
    if prec == "split_fp16":
        assert errs[4] < errs[3] and errs[4] <= 1e-12, errs
    else:
        # BF16 rounds the t >= 2 group in FP32 (about 2^-40 per product):
        # a floor near 2e-11 that extra slices do not lower
        assert errs[4] <= 1.05 * errs[3] and errs[4] <= 5e-11, errs


def test_split_fp16x9_within_bound_and_monotone():
    """FP16 slices of 9 bits over blocks of 32 pairs: every element within its
    bound for 2 to 4 slices, the error falling with the slice count, 1e-10
    reached at 4 slices (10 products, as BF16 at 4 slices, which stops near
    1e-9), more than 4 slices refused."""
    p = _problem((0.0, 0.4j, 0.35 + 0.005j))
    ref = oracle.chi0(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec, p.z, p.n, p.volume,
                      spin=p.spin, pair_chunk=p.pair_chunk)
    m, d = _operands(p)
    errs = []
    for S in (2, 3, 4):
        got = run_chi0(p, precision="split_fp16x9", n_slices=S)
        errs.append(rel_fro(got, ref))
        for w in range(len(p.z)):
            bnd = split_bound(m, d[w], S, p.nv, p.nc, p.pair_chunk, first_rounded=2, kb=32, bits=9)
            bnd = np.maximum(bnd, bnd.T)
            excess = np.abs(got[w] - ref[w]) - bnd - 1e-15 * np.abs(ref[w]).max()
            assert excess.max() <= 0, (S, w, excess.max())
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[2] <= 1e-10, errs
    bf4 = rel_fro(run_chi0(p, precision="split_bf16", n_slices=4), ref)
    assert errs[2] < 0.2 * bf4, (errs, bf4)
    with pytest.raises(gw.GWError):
        run_chi0(p, precision="split_fp16x9", n_slices=5)


def test_fp32_path():
    p = _problem((0.0, 0.6j, 0.2 + 0.005j))
    ref = oracle.chi0(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec, p.z, p.n, p.volume,
                      spin=p.spin, pair_chunk=p.pair_chunk)
    got = run_chi0(p, precision="fp32")
    err = rel_fro(got, ref)
    assert 1e-9 < err < 1e-5, err        # FP32 products: clearly not FP64, clearly FP32-accurate
    for w in range(len(p.z)):
        assert rel_fro(got[w], ref[w]) < 1e-5


def fp32_bound(m, d, kblk=64, m_cols=None):
    """Elementwise bound on |chi_fp32 - chi| for one frequency (d = s*Delta).
    Operands are rounded to FP32 (relative 2^-24 per component, the G' side
    after the FP64 product d*m); each FP32 partial sum runs over at most kblk
    pairs, i.e. 4 kblk real products per component, and rounds at most once
    per addition (gamma_n with n = 4 kblk + 2); the FP64 sums of the partials
    are below 1e-15 of the result.  With W = sum_p (|Re a| + |Im a|)
    (|Re b| + |Im b|), which bounds the summed magnitudes of the real products
    in either component: |err| <= sqrt(2) (2u + u^2 + gamma_n) W."""
    u = 2.0 ** -24
    n = 4 * kblk + 2
    gam = n * u / (1 - n * u)
    b = d[:, None] * (m if m_cols is None else m_cols)
    wa = np.abs(m.real) + np.abs(m.imag)
    wb = np.abs(b.real) + np.abs(b.imag)
    wsum = wa.T @ wb
    return np.sqrt(2) * (2 * u + u * u + gam) * wsum


def test_fp32_error_within_bound():
    """FP32 path against an a-posteriori bound from its rounding model, on two
    chunkings (the bound does not depend on them: partial sums restart per
    FP32 block and chunk)."""
    p = _problem((0.0, 0.6j, 0.2 + 0.005j), seed=37)
    ref = oracle.chi0(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec, p.z, p.n, p.volume,
                      spin=p.spin, pair_chunk=p.pair_chunk)
    m, d = _operands(p)
    for chunk in (150, 1000):
        got = run_chi0(p, precision="fp32", pair_chunk=chunk)
        for w in range(len(p.z)):
            bnd = fp32_bound(m, d[w])
            bnd = np.maximum(bnd, bnd.T)   # mirrored Hermitian tiles
            excess = np.abs(got[w] - ref[w]) - bnd - 1e-15 * np.abs(ref[w]).max()
            assert excess.max() <= 0, (chunk, w, excess.max())
            # and the bound is not vacuous: the error uses a real share of it
            assert np.abs(got[w] - ref[w]).max() > 1e-3 * bnd.max()


def test_split_edge_shapes():
    """Chunk smaller than a block, ragged blocks, a single G."""
    p = gen.make_problem((8, 8, 8), 2, 3, gvec=np.array([[0, 1, -1]], np.int32), z=(0.3j,),
                         seed=4, pair_chunk=5)
    ref = oracle.chi0(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec, p.z, p.n, p.volume,
                      spin=p.spin, pair_chunk=5)
    got = run_chi0(p, precision="split_bf16", n_slices=6)
    assert rel_fro(got, ref) < 1e-12
    p = gen.make_problem((12, 12, 12), 3, 70, r2=9, z=(0.0, 0.2 + 0.01j), seed=5, pair_chunk=200)
    ref = oracle.chi0(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec, p.z, p.n, p.volume,
                      spin=p.spin, pair_chunk=200)
    got = run_chi0(p, precision="split_fp16", n_slices=6)
    assert rel_fro(got, ref) < 1e-12
    got = run_chi0(p, precision="split_fp16x9", n_slices=4)
    assert rel_fro(got, ref) < 1e-10


@pytest.mark.parametrize("S", [3, 4, 5])
def test_split_bf16_matches_arithmetic_model(S):
    """The split-BF16 path against a CPU emulation of its arithmetic (block
    exponents, slices rounded to nearest, exact FP32 sums of the shift-0 and
    shift-1 groups, FP32 sums of the rest, FP64 recombination): the method
    error at 3 slices is 1e-7, but device and model differ only by the order
    of the FP32 additions of the shift >= 2 group.
    Every tile is contracted (no Hermitian mirror), so each entry comes from
    the same slices on both sides."""
    from test_precision_bounds_cpu import _split_model, _split_problem
    p = _split_problem()
    m, d = _operands(p)
    model = _split_model(m, d[0], S, p.nv, p.nc, p.pair_chunk)
    got = run_chi0(p, precision="split_bf16", n_slices=S, flags=gw.GW_FLAG_NO_HERMITIAN)[0]
    ref = oracle.chi0(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec, p.z, p.n, p.volume,
                      spin=p.spin)[0]
    # the shift >= 2 group is at most 2^-16 of the result and each FP32
    # addition to it rounds at 2^-24 of its running sum: over a block of 256
    # real products that is about 2^-36 relative, summed in a different order
    # on the two sides
    assert rel_fro(got, model) < 5e-11, (S, rel_fro(got, model), rel_fro(got, ref))
    # far inside the method error where that is large (3 and 4 slices), so a
    # different slicing or grouping would show
    if S < 5:
        assert rel_fro(got, model) < 0.1 * rel_fro(got, ref), (S, rel_fro(got, ref))
