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
