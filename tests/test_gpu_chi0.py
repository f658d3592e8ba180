"""GPU parity of gw_chi0 (FP64) against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2509_23018_amd as gw
from gpu_helpers import FP64_TOL, device, rel_fro, run_chi0, to_dev
from workloads import gen

pytestmark = pytest.mark.gpu


def _oracle_chi(p, **kw):
    args = dict(spin=p.spin, pair_chunk=p.pair_chunk)
    args.update(kw)
    return oracle.chi0(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec, p.z, p.n, p.volume, **args)


def test_chi0_workload0_full():
    """Static chi0 at q=0 on the 16^3 grid, 4 x 28 bands, 147 G."""
    p = gen.make_config(0)
    chi = run_chi0(p)
    ref = _oracle_chi(p)
    assert rel_fro(chi, ref) < FP64_TOL
    assert np.abs(chi[0] - chi[0].conj().T).max() < 1e-13 * np.abs(chi).max()
    assert np.linalg.eigvalsh(chi[0]).max() <= 1e-13 * np.abs(chi).max()


@pytest.mark.parametrize("flags", [0, gw.GW_FLAG_FP64_TILE128], ids=["tile64", "tile128"])
@pytest.mark.parametrize("zs,chunk", [
    ((0.0,), 37),                                  # static, ragged chunks
    ((0.3j, 1.7j, 0.0), 64),                       # imaginary axis: Hermitian shortcut
    ((0.0 + 0.005j, 0.4 + 0.005j, 0.9 + 0.01j), 50),  # real axis: every tile
    ((0.2j, 0.5 + 0.005j), 1000),                  # mixed, one chunk
])
def test_chi0_medium_multichunk(zs, chunk, flags):
    """Several tiles with a ragged edge (N_G = 251: three full 64-wide tiles
    and a ragged one, or one full 128-wide tile and a ragged one) and several
    chunks, on both FP64 tile shapes."""
    p = gen.make_problem((20, 18, 24), 5, 23, r2=15, z=zs, seed=11, pair_chunk=chunk)
    assert p.ng == 251
    chi = run_chi0(p, flags=flags)
    ref = _oracle_chi(p)
    assert rel_fro(chi, ref) < FP64_TOL
    for w, z in enumerate(p.z):
        assert rel_fro(chi[w], ref[w]) < FP64_TOL


def test_chi0_flags_no_hermitian_and_accumulate():
    p = gen.make_problem((12, 12, 12), 3, 9, r2=12, z=(0.0, 0.6j), seed=5, pair_chunk=10)
    ref = _oracle_chi(p)
    full = run_chi0(p, flags=gw.GW_FLAG_NO_HERMITIAN)
    assert rel_fro(full, ref) < FP64_TOL
    dp = to_dev(p)
    dp.chi = torch.full((2, p.ng, p.ng), 1.0 + 2.0j, dtype=torch.complex128, device=device())
    gw.gw_chi0(dp, flags=gw.GW_FLAG_ACCUMULATE, pair_chunk=10)
    acc = dp.chi.cpu().numpy()
    assert rel_fro(acc - (1.0 + 2.0j), ref) < FP64_TOL


@pytest.mark.parametrize("chunk", [1000, 40, 25])
def test_chi0_autotune_and_accumulate(chunk):
    """The tile autotuner times its trials into scratch: an accumulating call
    that tunes first must still add exactly chi to what the output held.
    One chunk (no second contraction stream), two chunks, and three."""
    p = gen.make_problem((14, 12, 12), 5, 13, r2=14, z=(0.0, 0.4 + 0.02j), seed=8,
                         pair_chunk=chunk)
    ref = _oracle_chi(p)
    dp = to_dev(p)
    dp.chi = torch.full((2, p.ng, p.ng), -0.5 + 1.0j, dtype=torch.complex128, device=device())
    gw.gw_chi0(dp, flags=gw.GW_FLAG_ACCUMULATE | gw.GW_FLAG_AUTOTUNE, pair_chunk=chunk)
    torch.cuda.synchronize()
    assert rel_fro(dp.chi.cpu().numpy() - (-0.5 + 1.0j), ref) < FP64_TOL
    got = run_chi0(p, flags=gw.GW_FLAG_AUTOTUNE)
    assert rel_fro(got, ref) < FP64_TOL


def test_chi0_edge_cases():
    # no pairs -> chi = 0
    p = gen.make_problem((8, 8, 8), 2, 3, r2=3, z=(0.0,), seed=1)
    p.psi_c, p.e_c = p.psi_c[:0], p.e_c[:0]
    dp = to_dev(p)
    dp.chi = torch.full((1, p.ng, p.ng), 3.0 + 0j, dtype=torch.complex128, device=device())
    gw.gw_chi0(dp)
    assert torch.all(dp.chi == 0)
    # one G, one pair per chunk, a singleton axis
    p = gen.make_problem((1, 6, 10), 2, 3, gvec=np.array([[0, 2, -3]], np.int32),
                         z=(0.25j,), seed=2, pair_chunk=1)
    assert rel_fro(run_chi0(p), _oracle_chi(p)) < FP64_TOL
    # largest Miller index on a small grid
    p = gen.make_problem((4, 5, 6), 2, 2, gvec=np.array([[-2, -2, -3], [1, 2, 2], [0, 0, 0]], np.int32),
                         z=(0.0, 0.3 + 0.01j), seed=3, pair_chunk=3)
    assert rel_fro(run_chi0(p), _oracle_chi(p)) < FP64_TOL


def test_chi0_invariances_on_device():
    p = gen.make_problem((12, 12, 12), 3, 8, r2=10, z=(0.0, 0.8j), seed=9, pair_chunk=7)
    ref = run_chi0(p)
    rng = np.random.default_rng(0)
    q = gen.Problem(**{**p.__dict__})
    q.psi_v = p.psi_v * np.exp(1j * rng.uniform(0, 6.3, p.nv))[:, None]
    q.e_v, q.e_c = p.e_v + 0.05, p.e_c + 0.05
    assert rel_fro(run_chi0(q), ref) < FP64_TOL
    assert rel_fro(run_chi0(p, pair_chunk=1), ref) < FP64_TOL
    assert np.abs(ref[:, 0, :]).max() < 1e-13 * np.abs(ref).max()   # head/wings at q = 0


def test_chi0_rejects_bad_arguments():
    p = gen.make_problem((8, 8, 8), 2, 3, r2=3, z=(0.0,), seed=1)
    dp = to_dev(p)
    dp.chi = torch.full((1, p.ng, p.ng), 5.0 + 0j, dtype=torch.complex128, device=device())
    with pytest.raises(gw.GWError, match="pair_chunk"):
        gw.gw_chi0(dp, pair_chunk=-3)
    with pytest.raises(gw.GWError, match="n_slices"):
        gw.gw_chi0(dp, precision="split_bf16", n_slices=1)
    dp.z = np.array([np.inf])
    with pytest.raises(gw.GWError, match="finite"):
        gw.gw_chi0(dp)
    torch.cuda.synchronize()
    assert torch.all(dp.chi == 5.0)


_W1 = {}


def _workload1_sample():
    """Workload 1 and the oracle's direct sums on 4 rows x 5 columns (cached:
    the sums over 61,440 pairs are the slow part)."""
    if not _W1:
        p = gen.make_config(1)
        assert (p.ng, p.npairs, len(p.z)) == (2007, 61440, 4)
        rng = np.random.default_rng(101)
        rows = np.sort(rng.choice(p.ng, 4, replace=False))
        cols = np.sort(np.concatenate([[0, p.ng - 1], rng.choice(p.ng, 3, replace=False)]))
        ref = oracle.chi0_entries(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec[rows], p.gvec[cols],
                                  p.z, p.n, p.volume, p.spin)
        _W1.update(p=p, rows=rows, cols=cols, ref=ref)
    return _W1["p"], _W1["rows"], _W1["cols"], _W1["ref"]


@pytest.mark.parametrize("prec,ns,tol", [
    ("fp64", 0, FP64_TOL),
    ("split_bf16", 5, 1e-10),     # the slice count the bench reports at 1e-10
    ("fp32", 0, 1e-5),
])
def test_chi0_workload1_full_size_sampled(prec, ns, tol):
    """48^3 grid, 64 x 960 bands (61,440 pairs in chunks of 4,096), 2,007 G,
    4 real frequencies, in the launch configuration the bench times:
    sampled rows/columns against the oracle's direct sums."""
    p, rows, cols, ref = _workload1_sample()
    chi = run_chi0(p, precision=prec, n_slices=ns)
    got = chi[:, rows][:, :, cols]
    assert rel_fro(got, ref) < tol, rel_fro(got, ref)
    # chi(z)^H = chi(conj z) cannot be checked within one call; check the
    # structure that holds at any size: the G = 0 row vanishes at q = 0
    assert np.abs(chi[:, 0, :]).max() < 1e-12 * np.abs(chi).max()


@pytest.mark.parametrize("prec,ns,tol", [("fp64", 0, FP64_TOL), ("split_bf16", 5, 1e-10)])
def test_chi0_precision_workload_grid_and_sphere(prec, ns, tol):
    """The 72^3 grid and its complete G-sphere (6,031 vectors) with the 8
    imaginary frequencies of the precision study, on 2 x 40 bands: the 32
    rows drawn with seed 1002 (all columns, all frequencies) against the
    oracle's Eq. (4) on those rows."""
    s = gen.CONFIG_SHAPES[2]
    z = gen.frequencies(*s["freq"])
    p = gen.make_problem(s["n"], 2, 40, r2=s["r2"], z=z, seed=2, pair_chunk=48)
    assert p.ng == 6031 and len(p.z) == 8
    rows = np.sort(np.random.default_rng(1002).choice(p.ng, 32, replace=False))
    ref = _oracle_chi(p)[:, rows]
    dp = to_dev(p)
    chi = gw.gw_chi0(dp, precision=prec, n_slices=ns, pair_chunk=48)
    got = chi[:, torch.from_numpy(rows).to(device())].cpu().numpy()
    assert rel_fro(got, ref) < tol, rel_fro(got, ref)


def test_chi0_tile128_tail_round_split():
    """The 128 x 128 FP64 tile (8 waves, one workgroup per CU: 256 resident
    on an MI355X) with a partial last round: N_G = 1,189 (10 tiles a side) and
    three real-axis frequencies give 300 items, the last 44 cut into 5 pair
    ranges; two chunks of 200 pairs.  Parity with the oracle, one tail
    reduction per chunk, and the same bits on a second run."""
    zs = (0.1 + 0.01j, 0.5 + 0.02j, 0.9 + 0.005j)
    p = gen.make_problem((16, 16, 16), 4, 100, r2=42, z=zs, seed=23, pair_chunk=200)
    assert p.ng == 1189, p.ng
    ref = _oracle_chi(p)
    gw.profile_enable(True)
    gw.profile_reset()
    try:
        chi = run_chi0(p, flags=gw.GW_FLAG_FP64_TILE128)
        n_tail, _ = gw.profile_read("chi0_tail")
    finally:
        gw.profile_enable(False)
    assert n_tail == 2
    for w in range(len(zs)):
        assert rel_fro(chi[w], ref[w]) < FP64_TOL
    assert np.array_equal(run_chi0(p, flags=gw.GW_FLAG_FP64_TILE128), chi)


@pytest.mark.parametrize("prec,ns,chunk,tol,kernel,launches", [
    ("fp64", 0, 200, FP64_TOL, "chi0_tail", 2),
    ("split_bf16", 5, 400, 1e-10, "chi0_split_tail", 1),
])
def test_chi0_tail_round_split(prec, ns, chunk, tol, kernel, launches):
    """Launches whose last round of workgroups is partial, N_G = 691 over 1
    Hermitian and 4 other frequencies.  FP64 (tiles of 64, 512 workgroups
    resident on an MI355X): 550 items, the last 38 cut into 13 pair ranges
    each, reduced by a second launch; two chunks of 200 pairs, so the second
    chunk's parts add onto the first's.  Split BF16 (128 x 64 tiles, 256
    resident): 330 items, the last 74 cut into 3 ranges of 128-pair blocks;
    one chunk of 400 pairs.  Accumulating, every frequency takes all tiles
    (FP64: 605 items, 93 cut into 5; split: 360, 104 cut into 2).  Parity with
    the oracle and the same bits on a second run."""
    zs = (0.4j, 0.1 + 0.01j, 0.5 + 0.02j, 0.9 + 0.005j, 1.3 + 0.01j)
    p = gen.make_problem((16, 16, 16), 4, 100, r2=29, z=zs, seed=21, pair_chunk=chunk)
    assert p.ng == 691, p.ng
    ref = _oracle_chi(p)
    kw = dict(precision=prec, n_slices=ns)
    gw.profile_enable(True)
    gw.profile_reset()
    try:
        chi = run_chi0(p, **kw)
        n_tail, _ = gw.profile_read(kernel)
    finally:
        gw.profile_enable(False)
    assert n_tail == launches
    assert rel_fro(chi, ref) < tol, rel_fro(chi, ref)
    for w in range(len(zs)):
        assert rel_fro(chi[w], ref[w]) < tol
    assert np.array_equal(run_chi0(p, **kw), chi)
    dp = to_dev(p)
    dp.chi = torch.full((len(zs), p.ng, p.ng), 0.25 - 1.0j, dtype=torch.complex128, device=device())
    gw.gw_chi0(dp, flags=gw.GW_FLAG_ACCUMULATE, pair_chunk=chunk, **kw)
    torch.cuda.synchronize()
    assert rel_fro(dp.chi.cpu().numpy() - (0.25 - 1.0j), ref) < tol
