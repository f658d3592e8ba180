/*
 * gw.h -- C ABI of libgw, the MI355X (gfx950) chi0 library.
 *
 * The library builds the independent-particle polarizability of Eq. (4) of
 * the paper,
 *
 *     chi_GG'(z) = s * sum_{v,c} conj(M_vc(G)) * Delta_vc(z) * M_vc(G'),
 *
 * from real-space wavefunctions on an FFT grid, band energies, a list of
 * G-vectors (Miller indices) and complex frequencies, in two parts:
 *
 *   MTXEL  the plane-wave matrix elements defined in the Overview section
 *          (after Eq. (2)):  M_vc(G) = dV * sum_r conj(psi_v(r)) psi_c(r)
 *          exp(+i G.r), read on the G-sphere;
 *   CHI0   the dense complex contraction M^H * diag(s*Delta(z)) * M, summed
 *          over chunks of pairs (the paper's NV-Block idea of splitting the
 *          sum over bands so that M never exists whole).
 *
 * The paper specifies the energy factor only as depending on E_v, E_c and
 * the frequency; it is taken here as the resonant plus anti-resonant form
 *     Delta_vc(z) = 1/(E_v - E_c + z) + 1/(E_v - E_c - z),
 * with z = w + i*eta (real axis), z = i*w (imaginary axis) or z = 0 (static).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Complex numbers are interleaved (re, im) doubles, bit-compatible with
 *   C99 double _Complex, std::complex<double> and torch.complex128.
 * - A real-space grid array has N1*N2*N3 elements, row-major with the third
 *   index fastest: r = (j1*N2 + j2)*N3 + j3.  A band set is [nbands][N_r].
 * - A Miller triple g = (g1, g2, g3) stands for G.r_j = 2*pi*(g1*j1/N1 +
 *   g2*j2/N2 + g3*j3/N3); each g_i must lie in [-floor(N_i/2), ceil(N_i/2) - 1]
 *   and the list must hold no duplicate.
 * - Pairs are numbered p = v*nc + c.
 * - dV = volume / (N1*N2*N3); the library applies no 1/Omega or 1/N_k factor.
 * - Device pointers are HIP device memory of the current device; host
 *   pointers are ordinary host memory, read before the call returns.
 * - All work is enqueued on `stream` (a hipStream_t, NULL = legacy default
 *   stream).  The caller owns every pointer it passes and must keep device
 *   buffers alive until the stream reaches the end of the call's work.
 * - Device scratch.  gw_chi0, gw_chi0_backward and gw_pseudobands take their
 *   scratch (streamed M chunks, energy factors, slices, tables) from a
 *   caller-owned `workspace` of at least gw_workspace_bytes() bytes when one
 *   is given; such a call enqueues its work and returns, with no device
 *   allocation and no wait on the device.  A workspace that is too small is
 *   GW_EINVAL, with every output untouched.  Without a workspace the library
 *   uses a scratch buffer of its own per device and stream, which it grows
 *   on demand (growing waits for the stream).  One workspace may serve
 *   consecutive calls on one stream; calls that overlap (other streams) need
 *   workspaces of their own.
 * - Library-owned state, created on first use and kept until gw_release():
 *   one plan (gather and twiddle tables) per device, grid and G list (at most
 *   256 per device; a dropped plan is freed once the work that reads it has
 *   completed), tile-order tables, a companion stream per caller stream,
 *   pinned host buffers that stage host tables without blocking, captured
 *   graphs (GW_FLAG_GRAPH) and autotuning results.  Creating them allocates
 *   and uploads once; a first call with a new grid, G list or tile shape may
 *   therefore wait for its own table upload.  The host side is thread-safe.
 * - Errors: every argument check runs on the host before anything is
 *   enqueued; a non-OK status leaves every output untouched and
 *   gw_last_error() returns a message (thread-local).  No C++ exception
 *   crosses this interface.  A fault inside a kernel surfaces at the
 *   caller's next synchronisation.  A singular energy factor (E_v - E_c = +-z)
 *   is not detected (the energies live on the device) and propagates as
 *   Inf/NaN.
 */
#ifndef GW_H
#define GW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GW_ABI_VERSION 2

typedef struct { double re, im; } gw_c128;

/* FFT grid N1 x N2 x N3 and cell volume Omega (bohr^3). */
typedef struct {
    int32_t n[3];
    double  volume;
} gw_grid_t;

typedef int32_t gw_status_t;
enum {
    GW_OK           = 0,
    GW_EINVAL       = -1,   /* bad argument (message says which) */
    GW_ENOMEM       = -2,   /* device allocation of library scratch failed */
    GW_EHIP         = -3,   /* a HIP runtime call failed */
    GW_EUNSUPPORTED = -4,   /* valid request this library does not implement */
    GW_EINTERNAL    = -5
};

/* Arithmetic of the CHI0 contraction.  MTXEL, the energy factor, the slice
 * recombination and the chi accumulation are FP64 in every mode. */
typedef int32_t gw_precision_t;
enum {
    GW_FP64       = 0,      /* FP64 MFMA */
    GW_FP32       = 1,      /* operands rounded to FP32, FP32 products */
    GW_SPLIT_BF16 = 2,      /* fixed-point slices in BF16, FP32 accumulation */
    GW_SPLIT_FP16 = 3,      /* fixed-point slices in FP16, FP32 accumulation */
    GW_SPLIT_FP16X9 = 4     /* fixed-point 9-bit slices in FP16 (2 to 4 slices), FP32
                               accumulation exact over blocks of 32 pairs */
};

/* gw_opts_t.flags */
#define GW_FLAG_NO_HERMITIAN  (1u << 0)  /* compute every tile even when Delta is real */
#define GW_FLAG_ACCUMULATE    (1u << 1)  /* chi += result instead of chi = result */
#define GW_FLAG_GRAPH         (1u << 2)  /* capture the whole call into a HIP graph on first
                                            use and replay it when called again with the same
                                            problems (same pointers, sizes, G lists, z, opts) */
#define GW_FLAG_AUTOTUNE      (1u << 3)  /* time the CHI0 variants on this data once per
                                            (kernel, N_G, chunk) and keep the fastest (also
                                            GW_AUTOTUNE=1): the FP64 tile shape, or the LDS
                                            ring of the split-BF16 / 9-bit FP16 contraction
                                            (same bits either way).  GW_AUTOTUNE_CACHE names
                                            a file that keeps the choices; GW_CHI0_VARIANT and
                                            GW_SPLIT_VARIANT force one */
#define GW_FLAG_FP64_TILE128  (1u << 4)  /* FP64: contract on 128x128 tiles (8 waves, four
                                            real MFMA products per complex one) instead of the
                                            default 64x64 tiles; takes precedence over the
                                            autotuner and over GW_CHI0_VARIANT; ignored by the
                                            other precisions */
#define GW_FLAG_ACC_HERMITIAN (1u << 5)  /* with GW_FLAG_ACCUMULATE: the caller states that
                                            chi[w] is already Hermitian for every frequency with
                                            Re z = 0 (for instance the sum of earlier calls over
                                            other valence bands, as in the paper's NV-Block
                                            split of the band sum); those frequencies keep the
                                            Hermitian shortcut: only tiles on or above the
                                            diagonal are accumulated and the rest is mirrored
                                            from them (what the lower triangle held is
                                            overwritten).  GW_EINVAL without GW_FLAG_ACCUMULATE */

/* One chi0 problem (one q-point). */
typedef struct {
    gw_grid_t       grid;
    const gw_c128*  psi_v;  /* device [nv][N_r] */
    int32_t         nv;
    const gw_c128*  psi_c;  /* device [nc][N_r] */
    int32_t         nc;
    const double*   e_v;    /* device [nv], Hartree */
    const double*   e_c;    /* device [nc], Hartree */
    const int32_t*  gvec;   /* HOST   [ng][3] Miller indices */
    int32_t         ng;
    const gw_c128*  z;      /* HOST   [nz] complex frequencies, Hartree */
    int32_t         nz;
    gw_c128*        chi;    /* device OUT [nz][ng][ng], row index = G, column = G' */
} gw_problem_t;

typedef struct {
    gw_precision_t precision;   /* GW_FP64 ... */
    int32_t        n_slices;    /* split modes: slices per operand (2..8); ignored otherwise */
    int32_t        pair_chunk;  /* pairs per streamed M chunk; 0 = 4096 */
    uint32_t       flags;       /* GW_FLAG_* */
    double         spin;        /* spin factor s of Eq. (4); 0 = 2 */
    void*          workspace;   /* device scratch owned by the caller, 256-byte aligned, or NULL
                                   for the library's own; read and written by the call's work */
    size_t         workspace_bytes;  /* its size; at least gw_workspace_bytes() for the call */
} gw_opts_t;

/*
 * gw_mtxel -- plane-wave matrix elements (Overview section, after Eq. (2)).
 *
 *   m_out[k][i] = dV * sum_r conj(psi_v[v](r)) * psi_c[c](r) * exp(+i G_i.r)
 *   for k in [0, pair_count), p = pair_begin + k = v*nc + c.
 *
 * grid      host; N_i >= 1, N1*N2*N3 < 2^31.
 * psi_v     device [nv][N_r];  psi_c device [nc][N_r] (may alias psi_v).
 * gvec      HOST [ng][3], ng >= 1.
 * m_out     device [pair_count][ng], overwritten.
 * Returns GW_EINVAL for a NULL pointer with a non-zero size, a Miller index
 * out of range, a duplicate G, or a pair range outside [0, nv*nc).
 */
gw_status_t gw_mtxel(const gw_grid_t* grid,
                     const gw_c128* psi_v, int32_t nv,
                     const gw_c128* psi_c, int32_t nc,
                     const int32_t* gvec, int32_t ng,
                     int64_t pair_begin, int64_t pair_count,
                     gw_c128* m_out, void* stream);

/*
 * gw_chi0 -- polarizability of Eq. (4) for `nprob` independent problems
 * (q-points), each with its own grid, bands, G list and frequencies.
 *
 *   probs[q].chi[w][i][j] (=, or += with GW_FLAG_ACCUMULATE)
 *       s * sum_p Delta_p(z_w) * conj(M_p(G_i)) * M_p(G_j)
 *
 * M is streamed in chunks of opts->pair_chunk pairs through a library
 * scratch buffer and never stored whole.  When a frequency has a zero real
 * part, its Delta is real, its chi is Hermitian, and only the tiles on or
 * above the diagonal are contracted; the rest are mirrored (unless
 * GW_FLAG_NO_HERMITIAN or GW_FLAG_ACCUMULATE).  nv*nc == 0 yields chi = 0.
 * With nprob > 1 in FP64 or split BF16, the chunks of all problems are
 * processed in rounds, each round's contraction as one persistent launch over
 * all (problem, frequency, tile) items, largest first (split BF16: in groups
 * of problems whose slice buffers fit GW_SPLIT_BATCH_BYTES, default 8 GiB);
 * with GW_FLAG_GRAPH the whole call is captured once and replayed (the
 * caller keeps every pointer valid and unchanged between replays; problems
 * must not change size).  FP32 and split FP16 run the problems one by one.
 * A single FP64 or split-BF16 problem cuts the tiles of a contraction's last,
 * partial round of workgroups along the pairs and adds the parts in a fixed
 * order: results are the same on every run on the same device, but not
 * bitwise those of the batched path.
 * opts may be NULL (FP64, chunk 4096, s = 2).  Split precision accepts
 * 2..6 slices; returns GW_EUNSUPPORTED beyond that.
 */
gw_status_t gw_chi0(const gw_problem_t* probs, int32_t nprob,
                    const gw_opts_t* opts, void* stream);

/*
 * gw_chi0_backward -- adjoint of gw_chi0 for one problem (FP64), for a real
 * loss L in PyTorch's complex convention (grad of complex x =
 * dL/dRe x + i dL/dIm x).  grad_chi = dL/dchi, device [nz][ng][ng].
 *
 *   g_M,p  = s * sum_w [conj(Delta_p) W_w^T m_p + Delta_p conj(W_w) m_p]
 *   dL/dE_v = s * sum_w sum_c Re[dDelta/dE_v * m^H conj(W_w) m],
 *   dL/dE_c = -(same summand) summed over v
 *   g_rho(r) = dV * sum_G g_M(G) exp(-i G.r)
 *   dL/dpsi_c = sum_v psi_v * g_rho,  dL/dpsi_v = sum_c psi_c * conj(g_rho)
 *
 * M chunks are recomputed, not stored.  Where Delta is real (zero and
 * imaginary frequencies) the product runs against W + W^H, formed once per
 * call for every frequency when those planes fit GW_SYM_KEEP_BYTES of scratch
 * (default 1 GiB), else once per chunk.  Outputs (device, overwritten):
 * grad_psi_v [nv][N_r], grad_psi_c [nc][N_r], grad_e_v [nv], grad_e_c [nc];
 * any of them may be NULL to skip it.  prob->chi is not read.
 */
gw_status_t gw_chi0_backward(const gw_problem_t* prob, const gw_c128* grad_chi,
                             gw_c128* grad_psi_v, gw_c128* grad_psi_c,
                             double* grad_e_v, double* grad_e_c,
                             const gw_opts_t* opts, void* stream);

/*
 * gw_workspace_bytes -- device scratch, in bytes, that gw_chi0 (backward = 0)
 * or gw_chi0_backward (backward = 1; probs[0] only, every gradient wanted)
 * needs in opts->workspace for these problems and options (opts->workspace
 * itself is ignored).  The same arguments are checked as by those calls; on an
 * invalid argument it returns (size_t)-1 and gw_last_error() says why.  It may
 * build the plans of the problems' G lists (library-owned, kept for the
 * calls).  With GW_FLAG_GRAPH the workspace serves every replay of the
 * captured graph, so the caller keeps it for as long as it replays.
 */
size_t gw_workspace_bytes(const gw_problem_t* probs, int32_t nprob, const gw_opts_t* opts,
                          int32_t backward);

/*
 * gw_pseudobands -- stochastic pseudobands (Reduced Cost and Scaling section
 * of the paper): a band set compressed into
 *   the protected bands keep[0..nkeep), copied as they are, then for each
 *   slice s (bands slice_idx[slice_off[s] .. slice_off[s+1])) n_xi bands
 *     xi_{s,j}(r) = (1/sqrt(n_xi)) sum_{n in s} exp(2 pi i theta_{s,j,n}) psi_n(r)
 *   with the mean energy of the slice's bands.
 *
 * psi       device [nb][nr]; e device [nb] (Hartree).
 * keep      HOST [nkeep] band indices; slice_idx HOST [slice_off[nslices]]
 *           band indices; slice_off HOST [nslices + 1], slice_off[0] = 0,
 *           strictly increasing (no empty slice).  A band may appear in
 *           several places; the caller chooses the partition.
 * theta     HOST, per slice s in order, [n_xi][|s|] phases in turns (the
 *           random numbers are the caller's, so results are reproducible).
 * n_xi      1..8 pseudobands per slice.
 * out_psi   device [nkeep + nslices*n_xi][nr], out_e device [same] (overwritten):
 *           the protected bands first, then slice by slice, j fastest.
 * workspace device scratch owned by the caller (256-byte aligned) of at least
 *           gw_pseudobands_workspace_bytes(nkeep, slice_off[nslices], nslices,
 *           n_xi) bytes, or NULL for the library's own.
 * The host tables are copied into the call's scratch through the library's
 * pinned staging buffers, in stream order, so the call returns without
 * waiting and the host arrays may be reused at once.  Returns GW_EINVAL for an
 * index out of range, an empty slice, n_xi outside 1..8, a non-finite theta,
 * nr of 2^31 or more or a workspace that is too small, and GW_EUNSUPPORTED for
 * more than 65535 protected bands or slices.
 */
gw_status_t gw_pseudobands(const gw_c128* psi, const double* e, int32_t nb, int64_t nr,
                           const int32_t* keep, int32_t nkeep,
                           const int32_t* slice_idx, const int32_t* slice_off, int32_t nslices,
                           int32_t n_xi, const double* theta,
                           gw_c128* out_psi, double* out_e,
                           void* workspace, size_t workspace_bytes, void* stream);

/* Scratch bytes gw_pseudobands needs for nkeep protected bands, nidx slice
 * entries in nslices slices and n_xi pseudobands per slice. */
size_t gw_pseudobands_workspace_bytes(int32_t nkeep, int64_t nidx, int32_t nslices,
                                      int32_t n_xi);

/*
 * gw_chi0_fixed -- gw_chi0 for one problem with no allocation at all, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid it).  Its scratch is a fixed
 * device array of gw_chi0_fixed_scratch_bytes() bytes (128 MiB) that the
 * library holds on every device it runs on until the process ends.
 *
 * Same problem, options and result as gw_chi0 with nprob = 1, except:
 * - the pair chunk is the largest one up to opts->pair_chunk whose buffers fit
 *   the fixed scratch (MTXEL and the contraction alternate on `stream`, every
 *   tile whole), so results agree with gw_chi0 to rounding, not bit for bit;
 * - the plan of the grid and G list and the contraction's tile-order table
 *   must exist on the device: make one ordinary gw_chi0 (or gw_mtxel) call with
 *   the same grid, G list and precision first; otherwise GW_EINVAL before
 *   anything is enqueued;
 * - opts->workspace must be NULL, and GW_FLAG_GRAPH and GW_FLAG_AUTOTUNE are
 *   GW_EINVAL (both allocate);
 * - a problem whose buffers exceed the fixed scratch even at one pair per
 *   chunk is GW_EUNSUPPORTED.
 * Every call on a device shares that device's fixed scratch, which keeps what
 * the last call wrote (every buffer is written before it is read, so nothing
 * needs clearing): calls that overlap on one device (other streams, other
 * threads) race; serialise them.  No allocation, no wait on the device.
 */
gw_status_t gw_chi0_fixed(const gw_problem_t* prob, const gw_opts_t* opts, void* stream);
size_t gw_chi0_fixed_scratch_bytes(void);

/*
 * Static subspace (Fast Full-Frequency GW section of the paper, Eq. (6)).
 * The static polarizability chi(0) of Eq. (4) is diagonalised and its n_eig
 * most significant eigenvectors, the columns of the N_G x n_eig matrix C_s,
 * span the subspace in which the polarizability at the other frequencies is
 * built: M^B_vc = sum_G M^G_vc C_s^{GB} and
 *     chi_BB'(z) = s * sum_vc conj(M^B_vc) Delta_vc(z) M^B'_vc,
 * which equals C_s^H chi(z) C_s.
 * The paper does not say in which metric chi(0) is diagonalised.  Both are
 * offered: chi itself, or, given a weight w (w_G = sqrt(v_G), v the Coulomb
 * diagonal of Eq. (3)), the symmetrised W chi W, W = diag(w), whose spectrum
 * falls off with |q + G| as the Coulomb factor does; then
 * M^B_vc = sum_G M^G_vc w_G C_s^{GB} and chi_BB'(z) = C_s^H W chi(z) W C_s.
 */
typedef struct {
    double   tol;         /* residual |chi x - lambda x| / b of every kept pair, b a bound of
                             |chi| (largest absolute row sum); 0 = 1e-10 */
    int32_t  max_iter;    /* filtered subspace iterations; 0 = 60 */
    int32_t  guard;       /* block columns beyond n_eig; 0 = max(16, n_eig / 8) */
    int32_t  max_degree;  /* Chebyshev filter degree cap; 0 = 16 */
    uint64_t seed;        /* start block (a counter-based hash of seed and index) */
    const double* weight; /* device [ng] or NULL: diagonalise diag(w) chi diag(w) instead of
                             chi (w_G = sqrt(v_G): the symmetrised v^1/2 chi v^1/2) */
    void*    workspace;   /* device scratch owned by the caller (256-byte aligned) or NULL */
    size_t   workspace_bytes;
} gw_diag_opts_t;

typedef struct {
    int32_t iterations;   /* filtered iterations made */
    int32_t degree;       /* filter degree of the last one */
    double  residual;     /* largest relative residual of the kept pairs */
    double  bound;        /* the bound b */
    int32_t sweeps;       /* Jacobi sweeps of the Rayleigh-Ritz steps, in all */
} gw_diag_info_t;

/*
 * gw_subspace_basis -- Diag: the n_eig eigenvectors of the Hermitian static
 * polarizability with the largest |eigenvalue|.  chi0(0) is negative
 * semidefinite (every valence energy below every conduction energy), so those
 * are its most negative eigenvalues; the matrix must be Hermitian and negative
 * semidefinite (positive eigenvalues are treated as insignificant).
 * Chebyshev-filtered subspace iteration with Rayleigh-Ritz steps on FP64
 * MFMA GEMMs, orthonormalisation by Cholesky-QR, Ritz problems by Jacobi
 * rotations, all on the device.
 *
 * chi_static  device [ng][ng], read only.
 * basis       device OUT [ng][n_eig] row-major: column j is the j-th
 *             eigenvector (orthonormal columns); a column's phase, and the
 *             basis of a degenerate eigenspace, are arbitrary.
 * eigenvalues device OUT [n_eig], increasing (most negative first).
 * info        HOST OUT, may be NULL.
 * The iteration reads convergence data back, so the call waits for `stream`.
 * Not converging within max_iter is not an error: info->residual says how far
 * it got.  GW_EINVAL for n_eig outside [1, ng], NULL pointers, bad options or
 * a workspace smaller than gw_subspace_basis_workspace_bytes().
 */
gw_status_t gw_subspace_basis(const gw_c128* chi_static, int32_t ng, int32_t n_eig,
                              gw_c128* basis, double* eigenvalues, const gw_diag_opts_t* opts,
                              gw_diag_info_t* info, void* stream);
size_t gw_subspace_basis_workspace_bytes(int32_t ng, int32_t n_eig, const gw_diag_opts_t* opts);

/*
 * gw_chi0_subspace -- Transf and CHI-Freq: chi_BB'(z) of Eq. (6) for one
 * problem, M streamed in chunks as in gw_chi0, each chunk transformed to the
 * subspace (M^B = M W C_s, FP64 MFMA GEMM) before the contraction over n_eig
 * columns.  prob->chi is device OUT [nz][n_eig][n_eig]; basis is device
 * [ng][n_eig] (for instance from gw_subspace_basis); weight is device [ng]
 * (W = diag(weight), the weight the basis was found with) or NULL (W = I).
 * The options, flags (except GW_FLAG_GRAPH, GW_EUNSUPPORTED), precisions and
 * workspace rules are those of gw_chi0; the workspace size is
 * gw_chi0_subspace_workspace_bytes().
 */
gw_status_t gw_chi0_subspace(const gw_problem_t* prob, const gw_c128* basis,
                             const double* weight, int32_t n_eig, const gw_opts_t* opts,
                             void* stream);
size_t gw_chi0_subspace_workspace_bytes(const gw_problem_t* prob, int32_t n_eig,
                                        const gw_opts_t* opts);

/*
 * Matrix elements kept in device memory.  The static subspace method builds
 * chi(0) in plane waves, diagonalises it, then builds chi_BB'(z) from the
 * same matrix elements; with HBM to hold M of every pair (16 N_G bytes per
 * pair: 95 GB for 983,040 pairs and 6,031 G) the second pass can read M
 * instead of running MTXEL again.
 *
 * gw_chi0_keep_m -- gw_chi0 of one problem (Eq. (4)) that also leaves M of
 * every pair in m_keep: device OUT [nv*nc][ng], in the order the call streams
 * its pair chunks: rectangles of vb valence x cw conduction bands, with
 * cw = min(nc, chunk / min(nv, 4)) and vb = min(nv, chunk / cw) for
 * chunk = opts->pair_chunk (0: 4096), valence blocks outer, conduction blocks
 * inner, each rectangle [vcount][cw] row-major.  Options, precisions, flags
 * (GW_FLAG_GRAPH is GW_EUNSUPPORTED) and workspace as gw_chi0 with nprob = 1
 * (size: gw_workspace_bytes(prob, 1, opts, 0)).  m_keep is owned by the
 * caller; NULL with nv*nc > 0 is GW_EINVAL.
 */
gw_status_t gw_chi0_keep_m(const gw_problem_t* prob, gw_c128* m_keep, const gw_opts_t* opts,
                           void* stream);

/*
 * gw_chi0_from_m -- chi of one problem from M kept by gw_chi0_keep_m with the
 * same problem shape and pair_chunk (no MTXEL; prob->psi_v and psi_c are not
 * read, the energies and frequencies are): with basis NULL Eq. (4) into
 * prob->chi [nz][ng][ng]; with basis (device [ng][n_eig]) and weight (device
 * [ng] or NULL) Transf and CHI-Freq of Eq. (6) as gw_chi0_subspace into
 * prob->chi [nz][n_eig][n_eig].  Workspace size:
 * gw_chi0_from_m_workspace_bytes(prob, basis ? n_eig : 0, opts).  The
 * results are bit-identical to gw_chi0 / gw_chi0_subspace with the same
 * options.  GW_EINVAL: m_keep NULL with nv*nc > 0, n_eig outside [1, ng] with
 * a basis, n_eig != 0 without one; GW_FLAG_GRAPH is GW_EUNSUPPORTED.  An
 * m_keep from another shape or pair_chunk is not detected.
 */
gw_status_t gw_chi0_from_m(const gw_problem_t* prob, const gw_c128* m_keep, const gw_c128* basis,
                           const double* weight, int32_t n_eig, const gw_opts_t* opts,
                           void* stream);
size_t gw_chi0_from_m_workspace_bytes(const gw_problem_t* prob, int32_t n_eig,
                                      const gw_opts_t* opts);

/*
 * gw_chi0_backward_from_m -- gw_chi0_backward reading M kept by
 * gw_chi0_keep_m (same problem shape and pair_chunk) instead of recomputing
 * it: the adjoint's chunks are the forward's rectangles, in the same order,
 * so chunk k is read at its rows of m_keep.  Same gradients, arguments and
 * outputs as gw_chi0_backward (psi_v and psi_c are still read, by the band
 * sums); bit-identical to it.  GW_EINVAL: m_keep NULL with nv*nc > 0, or a
 * pair_chunk whose adjoint chunks would differ from the forward's (chunks of
 * more than 8 valence bands whose per-pair g_rho would exceed 2 GiB).  Scratch:
 * gw_chi0_backward_from_m_workspace_bytes(prob, opts) (no M buffers, no MTXEL
 * intermediate), in opts->workspace or the library's own.
 */
gw_status_t gw_chi0_backward_from_m(const gw_problem_t* prob, const gw_c128* m_keep,
                                    const gw_c128* grad_chi, gw_c128* grad_psi_v,
                                    gw_c128* grad_psi_c, double* grad_e_v, double* grad_e_c,
                                    const gw_opts_t* opts, void* stream);
size_t gw_chi0_backward_from_m_workspace_bytes(const gw_problem_t* prob, const gw_opts_t* opts);

/*
 * gw_epsinv -- the inverse dielectric matrix of Eq. (3),
 *     eps^-1(z) = [I - v chi(z)]^-1,
 * for nz frequencies, with v the diagonal Coulomb matrix.  Block Gauss-Jordan
 * elimination without pivoting (64 columns per step, the updates as FP64
 * MFMA GEMMs), on the device.
 *
 * chi     device [nz][ng][ng] (for instance gw_chi0's output), read only.
 * vcoul   device [ng], v_G = 4 pi / |q + G|^2 in Hartree atomic units, >= 0;
 *         at q = 0 the G = 0 entry is the caller's choice (0 excludes the head:
 *         eps^-1 then has the identity's row and column there).
 * epsinv  device OUT [nz][ng][ng], row index G, column G'; not chi.
 * Without pivoting every leading block must be nonsingular: true for the
 * zero and imaginary frequencies, where eps = v^1/2 eps~ v^-1/2 with eps~
 * Hermitian positive definite (every eigenvalue >= 1); on the real axis the
 * caller relies on it (a singular block propagates Inf/NaN, not an error).
 * Asynchronous; workspace NULL or gw_epsinv_workspace_bytes(ng, nz) bytes.
 */
gw_status_t gw_epsinv(const gw_c128* chi, int32_t ng, int32_t nz, const double* vcoul,
                      gw_c128* epsinv, void* workspace, size_t workspace_bytes, void* stream);
size_t gw_epsinv_workspace_bytes(int32_t ng, int32_t nz);

/*
 * gw_gpp_sigma -- the full GPP self-energy matrix on an energy grid, the
 * paper's off-diagonal kernel (Optimized GPP Kernel for Off-Diagonal
 * Self-Energy Matrix Elements section; flop count of Eq. (8)):
 *     Sigma_lm(E) = sum_n sum_GG' conj(M_ln(G)) P^{nE}_GG' M_mn(G'),
 *     P^{nE}_GG' = Omega2_GG' v_G' / (2 wt_GG' (E - E_n - s_n wt_GG')),
 * s_n = -1 for an occupied band, +1 for an empty one (the plasmon-pole term
 * of the model the paper cites; the paper does not print it).  Per band and
 * energy two complex GEMMs on FP64 MFMA, T = conj(M_n) P (N_Sigma x N_G x
 * N_G, P formed inside the GEMM, never stored) and Sigma(E) += T M_n^T
 * (N_Sigma x N_G x N_Sigma).
 *
 * m         device [nb][ns][ng]: M_ln(G) for the ns states l and the nb bands n.
 * e_n       HOST [nb] band energies (Hartree); occupied HOST [nb] (0 / 1).
 * energies  HOST [ne] complex energies E (the imaginary part broadens).
 * omega2    device [ng][ng] complex; wtilde device [ng][ng] (> 0); vcoul device [ng].
 * sigma     device OUT [ne][ns][ns], overwritten (row l, column m).
 * Asynchronous (the energies are staged in stream order); workspace NULL or
 * gw_gpp_sigma_workspace_bytes(ns, ng, ne) bytes.
 */
gw_status_t gw_gpp_sigma(const gw_c128* m, int32_t nb, int32_t ns, int32_t ng,
                         const double* e_n, const int32_t* occupied, const gw_c128* energies,
                         int32_t ne, const gw_c128* omega2, const double* wtilde,
                         const double* vcoul, gw_c128* sigma, void* workspace,
                         size_t workspace_bytes, void* stream);
size_t gw_gpp_sigma_workspace_bytes(int32_t ns, int32_t ng, int32_t ne);

/*
 * Dense building blocks of the subspace, dielectric and self-energy paths.
 *
 * gw_zgemm -- C = alpha op(A) op(B) + beta C for `batch` products (pointers
 * advanced by the strides, in elements), complex FP64 on MFMA, row-major:
 * op(A) is m x k, op(B) k x n, C m x n; op 'N' (as stored), 'T' (transposed:
 * A stored k x m) or 'C' (conjugate transposed).  All pointers are device
 * memory.  beta = 0 never reads C.  Asynchronous.
 */
gw_status_t gw_zgemm(char opa, char opb, int32_t m, int32_t n, int32_t k, gw_c128 alpha,
                     const gw_c128* a, int64_t lda, int64_t stride_a, const gw_c128* b,
                     int64_t ldb, int64_t stride_b, gw_c128 beta, gw_c128* c, int64_t ldc,
                     int64_t stride_c, int32_t batch, void* stream);

/*
 * gw_heev -- eigenvalues w [batch][n] (increasing) and eigenvectors v
 * [batch][n][n] (columns) of `batch` Hermitian n x n matrices a (device,
 * read only), by cyclic Jacobi rotations in parallel order until the
 * off-diagonal norm is below tol (0 = 1e-15) of the norm.  Waits for
 * `stream`.  workspace: NULL or gw_heev_workspace_bytes(n, batch) bytes.
 */
gw_status_t gw_heev(const gw_c128* a, int32_t n, int32_t batch, double* w, gw_c128* v,
                    double tol, void* workspace, size_t workspace_bytes, void* stream);
size_t gw_heev_workspace_bytes(int32_t n, int32_t batch);

/* Message for the last non-OK status on this thread ("" if none). */
const char* gw_last_error(void);

/* Frees cached plans, graphs, staging buffers and scratch on every device
 * (waits for the work that uses them). */
gw_status_t gw_release(void);

/* GW_ABI_VERSION of the built library. */
int32_t gw_abi_version(void);

/*
 * Launch timing for measurement harnesses.  While enabled, the library
 * records a HIP event on the caller's stream before and after each of its
 * kernel launches and files the pair under the kernel's name ("mtxel_zy",
 * "mtxel_x", "delta", "chi0_f64", "chi0_tail", "chi0_f64_batched",
 * "split_prep", "chi0_split", "chi0_split_tail", "chi0_split_batched",
 * "chi0_f32", "mirror", "bwd_sym", "bwd_gm", "bwd_de", "bwd_de_reduce", "bwd_x", "bwd_yz",
 * "bwd_reduce_cv", "bwd_reduce_c", "bwd_reduce_v", "pseudo_prep", "pseudo_keep",
 * "pseudo_mix").
 * gw_profile_read waits for the recorded events of `kernel` and returns the
 * number of launches and the summed duration in milliseconds (0 and 0.0 for
 * an unknown name).  gw_profile_reset forgets every record.  Timing adds two
 * event records per launch and nothing else.
 */
gw_status_t gw_profile_enable(int32_t on);
gw_status_t gw_profile_read(const char* kernel, int64_t* launches, double* total_ms);
gw_status_t gw_profile_reset(void);

#ifdef __cplusplus
}
#endif
#endif /* GW_H */
