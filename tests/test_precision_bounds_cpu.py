"""The a-posteriori FP32 bound of the GPU precision tests, checked on the CPU
against emulations whose arithmetic is known: a contraction that follows the
FP32 path's rounding model must stay inside the bound, and one that rounds its
operands a bit more coarsely than FP32 must break it somewhere, so the bound
catches a gross loss of precision without being too tight for the model."""
import numpy as np

import oracle
from test_gpu_precision import _operands, fp32_bound
from workloads import gen


def _fp32_model(m, d, kblk=64, order=None):
    """chi by the FP32 path's model: both operands rounded to FP32 (the G' side
    after the FP64 product d*m), real products summed in FP32 over blocks of
    kblk pairs, in the given pair order, block sums added in FP64."""
    a = m.astype(np.complex64)
    b = (d[:, None] * m).astype(np.complex64)
    k = m.shape[0]
    order = np.arange(k) if order is None else order
    chi = np.zeros((m.shape[1], m.shape[1]), np.complex128)
    for k0 in range(0, k, kblk):
        idx = order[k0:k0 + kblk]
        ar, ai = a[idx].real, a[idx].imag
        br, bi = b[idx].real, b[idx].imag
        re = np.zeros(chi.shape, np.float32)
        im = np.zeros(chi.shape, np.float32)
        for p in range(len(idx)):            # one FP32 rounding per addition
            re += np.outer(ar[p], br[p])
            re += np.outer(ai[p], bi[p])
            im += np.outer(ar[p], bi[p])
            im -= np.outer(ai[p], br[p])
        chi += re.astype(np.float64) + 1j * im.astype(np.float64)
    return chi


def _round_bits(x, bits):
    """x with each component rounded to `bits` significant bits."""
    def r(v):
        m, e = np.frexp(v)
        return np.ldexp(np.round(m * 2.0 ** bits) / 2.0 ** bits, e)
    return r(x.real) + 1j * r(x.imag)


def _problem():
    return gen.make_problem((10, 12, 10), 3, 14, r2=6, z=(0.0, 0.5 + 0.01j), seed=77,
                            pair_chunk=1000)


def test_fp32_model_inside_bound():
    p = _problem()
    m, d = _operands(p)
    rng = np.random.default_rng(5)
    for w in range(len(p.z)):
        ref = oracle.chi0(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec, p.z[w:w + 1], p.n, p.volume,
                          spin=p.spin)[0]
        bnd = fp32_bound(m, d[w])
        for order in (None, rng.permutation(m.shape[0])):
            got = _fp32_model(m, d[w], order=order)
            assert np.all(np.abs(got - ref) <= bnd + 1e-15 * np.abs(ref).max())


def test_coarser_operands_break_bound():
    """The bound is a worst case (gamma_n over 4 x 64 sums allows about 2^-16
    of W); operands rounded to 12 significant bits (FP32 keeps 24) put errors
    above it on some entries."""
    p = _problem()
    m, d = _operands(p)
    ref = oracle.chi0(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec, p.z[:1], p.n, p.volume,
                      spin=p.spin)[0]
    mc = _round_bits(m, 12)
    got = np.conj(mc).T @ (d[0][:, None] * mc)
    assert np.any(np.abs(got - ref) > fp32_bound(m, d[0]))


def _split_model(m, d, S, nv, nc, chunk, grouped=True, kb=128, bits=8):
    """chi by the split-BF16 model: per chunk (rectangle of bands, as the
    library streams them) and block of kb pairs, each operand column gets the
    exponent e with max(|Re|, |Im|) < 2^e, and x 2^(8-e) is cut into S
    integer slices by rounding to nearest (q_0 within 256, later ones within
    128); slice s enters as q_s 2^-8s.  Products of slices a, b with
    a + b <= S - 1 are summed in FP32, one real product at a time, in three
    groups a + b = 0, 1 and >= 2 (grouped) or all in one accumulator (not
    grouped); after each block 2^(eA + eB - 16) times the group sum is added
    in FP64."""
    from test_gpu_precision import _chunk_ranges

    def slices(x):
        mx = np.maximum(np.abs(x.real), np.abs(x.imag)).max(axis=0)
        e = np.where(mx > 0, np.frexp(mx)[1], 0).astype(np.float64)
        y = x * 2.0 ** (bits - e)
        out = []
        for s in range(S):
            q = np.round(y.real) + 1j * np.round(y.imag)
            out.append(q * 2.0 ** (-bits * s))
            y = (y - q) * 2.0 ** bits
        return e, out

    ng = m.shape[1]
    chi = np.zeros((ng, ng), np.complex128)
    for idx in _chunk_ranges(nv, nc, chunk):
        a_all, b_all = m[idx], d[idx, None] * m[idx]
        for k0 in range(0, len(idx), kb):
            ea, qa = slices(a_all[k0:k0 + kb])
            eb, qb = slices(b_all[k0:k0 + kb])
            acc_r = [np.zeros((ng, ng), np.float32) for _ in range(3)]
            acc_i = [np.zeros((ng, ng), np.float32) for _ in range(3)]
            for sa in range(S):
                for sb in range(S - sa):
                    g = min(sa + sb, 2) if grouped else 0
                    ar, ai = qa[sa].real.astype(np.float32), qa[sa].imag.astype(np.float32)
                    br, bi = qb[sb].real.astype(np.float32), qb[sb].imag.astype(np.float32)
                    for p in range(ar.shape[0]):   # conj(a) b, one rounding per addition
                        acc_r[g] += np.outer(ar[p], br[p])
                        acc_r[g] += np.outer(ai[p], bi[p])
                        acc_i[g] += np.outer(ar[p], bi[p])
                        acc_i[g] -= np.outer(ai[p], br[p])
            tot = sum(r.astype(np.float64) + 1j * i.astype(np.float64) for r, i in zip(acc_r, acc_i))
            chi += 2.0 ** (ea[:, None] + eb[None, :] - 2 * bits) * tot
    return chi


def _split_problem():
    return gen.make_problem((10, 10, 12), 3, 50, r2=5, z=(0.3j,), seed=81, pair_chunk=100)


def test_split_model_inside_bound():
    """The grouped split-BF16 model stays inside the split bound for 2 to 5
    slices, over chunks of 100 pairs (blocks of 128 cut short by the chunk)."""
    from test_gpu_precision import split_bound
    p = _split_problem()
    m, d = _operands(p)
    ref = oracle.chi0(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec, p.z, p.n, p.volume,
                      spin=p.spin)[0]
    for S in (2, 3, 4, 5):
        got = _split_model(m, d[0], S, p.nv, p.nc, p.pair_chunk)
        bnd = split_bound(m, d[0], S, p.nv, p.nc, p.pair_chunk, first_rounded=2, kb=128)
        assert np.all(np.abs(got - ref) <= bnd + 1e-15 * np.abs(ref).max()), S


def test_split_one_accumulator_breaks_bound():
    """At 5 slices, summing every slice product in one FP32 accumulator (so the
    leading integer sums round) exceeds the bound, which counts FP32 rounding
    only for the group of shifts >= 2."""
    from test_gpu_precision import split_bound
    p = _split_problem()
    m, d = _operands(p)
    ref = oracle.chi0(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec, p.z, p.n, p.volume,
                      spin=p.spin)[0]
    got = _split_model(m, d[0], 5, p.nv, p.nc, p.pair_chunk, grouped=False)
    bnd = split_bound(m, d[0], 5, p.nv, p.nc, p.pair_chunk, first_rounded=2, kb=128)
    assert np.any(np.abs(got - ref) > bnd + 1e-15 * np.abs(ref).max())


def test_split_fp16x9_model_inside_bound():
    """The 9-bit FP16 slicing (blocks of 32 pairs, t = 0 and t = 1 exact, t >= 2
    in one FP32 group) stays inside its bound for 2 to 4 slices, and 4 slices
    reach below 1e-10 where 8-bit slices at 4 do not."""
    from test_gpu_precision import split_bound
    p = _split_problem()
    m, d = _operands(p)
    ref = oracle.chi0(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec, p.z, p.n, p.volume,
                      spin=p.spin)[0]
    errs = {}
    for S in (2, 3, 4):
        got = _split_model(m, d[0], S, p.nv, p.nc, p.pair_chunk, kb=32, bits=9)
        bnd = split_bound(m, d[0], S, p.nv, p.nc, p.pair_chunk, first_rounded=2, kb=32, bits=9)
        assert np.all(np.abs(got - ref) <= bnd + 1e-15 * np.abs(ref).max()), S
        errs[S] = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    bf4 = _split_model(m, d[0], 4, p.nv, p.nc, p.pair_chunk)
    e_bf4 = np.linalg.norm(bf4 - ref) / np.linalg.norm(ref)
    assert errs[2] > errs[3] > errs[4] and errs[4] < 1e-10 < e_bf4, (errs, e_bf4)
