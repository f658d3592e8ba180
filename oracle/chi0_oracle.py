"""FP64 NumPy oracle for the independent-particle polarizability chi0.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the CPU
baseline leg of the benchmark, never by the device library or its binding.

What it computes (Overview of the Problem; Eq. (4) of the paper):

* plane-wave matrix elements (the definition that follows Eq. (2))
  ``M_vc(G) = integral dr conj(psi_v(r)) exp(+i G.r) psi_c(r)``, evaluated on
  the FFT grid as ``dV * sum_r conj(psi_v(r)) psi_c(r) exp(+i G.r)``;
* the polarizability of Eq. (4)
  ``chi_GG'(z) = s * sum_vc conj(M_vc(G)) Delta_vc(z) M_vc(G')`` with the spin
  factor ``s = 2`` and the energy factor read as
  ``Delta_vc(z) = 1/(E_v - E_c + z) + 1/(E_v - E_c - z)`` (the paper only
  says that Delta contains E_v, E_c and the frequency);
* its adjoint with respect to psi_v, psi_c, E_v and E_c (not in the paper;
  derived from the two definitions above by the chain rule);
* the static subspace of the Fast Full-Frequency GW section: the eigenvectors
  of chi(0) with the largest |eigenvalue| as the columns of C_s, and Eq. (6),
  chi0 in that subspace from the transformed matrix elements M^B = M C_s;
* the inverse dielectric matrix of Eq. (3), eps^-1 = [I - v chi]^-1, with the
  Coulomb interaction v_G = 4 pi / |q + G|^2 on the diagonal;
* stochastic pseudobands (Reduced Cost and Scaling section);
* the full self-energy matrix of the GPP off-diagonal kernel: per band n and
  energy E one matrix P^{nE}_{GG'} and the product of Eq. (1)'s matrix
  elements around it, as the two complex GEMMs the paper counts in Eq. (8).

The sum over pairs is taken in chunks of pairs, the way the paper's NV-Block
scheme splits the sum over valence bands (Fast Full-Frequency GW section);
the chunking only changes the order of floating-point additions.

Grid and index conventions: grid point ``r_j = L*(j1/N1, j2/N2, j3/N3)``,
stored row-major with ``j3`` fastest; a Miller triple ``g`` gives
``G.r_j = 2*pi*(g1*j1/N1 + g2*j2/N2 + g3*j3/N3)``, periodic in each ``g_i``
modulo ``N_i``; pair ``p = v*N_c + c``.
"""
from __future__ import annotations

import numpy as np


def grid_phase(g, n) -> np.ndarray:
    """exp(+i G.r) on every grid point, flattened in storage order."""
    n1, n2, n3 = n
    j1, j2, j3 = np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij")
    arg = 2.0 * np.pi * (g[0] * j1 / n1 + g[1] * j2 / n2 + g[2] * j3 / n3)
    return np.exp(1j * arg).reshape(-1)


def pair_density(psi_v_row: np.ndarray, psi_c_row: np.ndarray) -> np.ndarray:
    """rho_vc(r) = conj(psi_v(r)) * psi_c(r) (the integrand of M, Overview)."""
    return np.conj(psi_v_row) * psi_c_row


def mtxel(psi_v, psi_c, gvec, n, volume, pairs=None) -> np.ndarray:
    """M[k, i] = M_{v_k c_k}(G_i) for the pairs ``pairs`` (default: all pairs
    in the order p = v*N_c + c).  Definition after Eq. (2), with the sign
    exp(+i G.r): numpy's inverse FFT carries that sign and a factor 1/N_r, so
    ``Omega * ifftn(rho)`` equals ``dV * sum_r rho(r) exp(+i G.r)``; the value at
    Miller g is read at grid index g mod N.

    Parity: pinned by plane waves (closed form), brute-force DFT, Parseval,
    completeness and translation tests."""
    n = tuple(int(x) for x in n)
    nc = psi_c.shape[0]
    if pairs is None:
        pairs = range(psi_v.shape[0] * nc)
    pairs = np.asarray(list(pairs), dtype=np.int64)
    gvec = np.asarray(gvec)
    idx = (gvec[:, 0] % n[0], gvec[:, 1] % n[1], gvec[:, 2] % n[2])
    out = np.empty((pairs.size, gvec.shape[0]), dtype=np.complex128)
    for k, p in enumerate(pairs):
        v, c = divmod(int(p), nc)
        rho = pair_density(psi_v[v], psi_c[c]).reshape(n)
        full = volume * np.fft.ifftn(rho)
        out[k] = full[idx]
    return out


def mtxel_direct(psi_v, psi_c, g, n, volume) -> np.ndarray:
    """M_vc(G) at a single Miller triple ``g`` for every pair, by the direct
    grid sum of the definition (no FFT).  Returns ``[N_v, N_c]``.

    Parity: pinned against brute force and against ``mtxel`` on small grids."""
    nr = int(np.prod(n))
    dv = volume / nr
    ph = grid_phase(g, n)
    return dv * ((np.conj(psi_v) * ph[None, :]) @ psi_c.T)


def energy_factor(e_v, e_c, z) -> np.ndarray:
    """Delta_vc(z) of Eq. (4), read as the resonant plus anti-resonant terms
    ``1/(E_v - E_c + z) + 1/(E_v - E_c - z)``; returns ``[N_z, N_v*N_c]`` in
    pair order p = v*N_c + c.  Static z = 0 gives 2/(E_v - E_c); z = i*w gives
    the real value 2(E_v - E_c)/((E_v - E_c)^2 + w^2).

    Parity: pinned by those two closed forms."""
    de = (np.asarray(e_v, np.float64)[:, None] - np.asarray(e_c, np.float64)[None, :]).reshape(-1)
    z = np.asarray(z, np.complex128).reshape(-1)
    return 1.0 / (de[None, :] + z[:, None]) + 1.0 / (de[None, :] - z[:, None])


def energy_factor_dE(e_v, e_c, z) -> np.ndarray:
    """d Delta_vc / d E_v  (= - d Delta_vc / d E_c), ``[N_z, N_v*N_c]``.

    Parity: pinned by central differences of ``energy_factor``."""
    de = (np.asarray(e_v, np.float64)[:, None] - np.asarray(e_c, np.float64)[None, :]).reshape(-1)
    z = np.asarray(z, np.complex128).reshape(-1)
    return -1.0 / (de[None, :] + z[:, None]) ** 2 - 1.0 / (de[None, :] - z[:, None]) ** 2


def chi0(psi_v, psi_c, e_v, e_c, gvec, z, n, volume, spin=2.0, pair_chunk=4096) -> np.ndarray:
    """chi[w, i, j] = s * sum_p Delta_p(z_w) conj(M_p(G_i)) M_p(G_j)  (Eq. (4)),
    summed over chunks of ``pair_chunk`` pairs.  Returns ``[N_z, N_G, N_G]``.

    Parity: pinned by the plane-wave closed form, brute force, the trace
    identity, Hermiticity, negative semidefiniteness and invariances."""
    nv, nc = psi_v.shape[0], psi_c.shape[0]
    z = np.asarray(z, np.complex128).reshape(-1)
    ng = np.asarray(gvec).shape[0]
    npairs = nv * nc
    delta = energy_factor(e_v, e_c, z)
    chi = np.zeros((z.size, ng, ng), dtype=np.complex128)
    step = max(1, int(pair_chunk))
    for k0 in range(0, npairs, step):
        k1 = min(npairs, k0 + step)
        m = mtxel(psi_v, psi_c, gvec, n, volume, pairs=range(k0, k1))
        for w in range(z.size):
            chi[w] += spin * ((np.conj(m).T * delta[w, k0:k1][None, :]) @ m)
    return chi


def chi0_entries(psi_v, psi_c, e_v, e_c, g_rows, g_cols, z, n, volume, spin=2.0) -> np.ndarray:
    """A sampled block chi[w][rows, cols] of Eq. (4), with every needed M
    computed at its own G by the direct grid sum (``mtxel_direct``), so that
    single entries of large problems can be checked without a full MTXEL.
    Returns ``[N_z, len(g_rows), len(g_cols)]``.

    Parity: pinned against ``chi0`` on small problems."""
    delta = energy_factor(e_v, e_c, z)                       # [nz, K]
    mr = np.stack([mtxel_direct(psi_v, psi_c, g, n, volume).reshape(-1) for g in g_rows])
    mc = np.stack([mtxel_direct(psi_v, psi_c, g, n, volume).reshape(-1) for g in g_cols])
    out = np.empty((delta.shape[0], len(g_rows), len(g_cols)), dtype=np.complex128)
    for w in range(delta.shape[0]):
        out[w] = spin * ((np.conj(mr) * delta[w][None, :]) @ mc.T)
    return out


def chi0_backward(psi_v, psi_c, e_v, e_c, gvec, z, n, volume, grad_chi, spin=2.0,
                  pair_chunk=4096):
    """Adjoint of ``chi0`` for a real loss L, in PyTorch's complex convention
    (the gradient of a complex x is dL/dRe x + i dL/dIm x).  ``grad_chi`` is
    W = dL/dchi, ``[N_z, N_G, N_G]``.  Derived here (the paper has no adjoint;
    its perturbation-theory section needs the first-order change of M):

    * g_M,p = s * sum_w [conj(Delta_p) W_w^T m_p + Delta_p conj(W_w) m_p]
    * dL/dE_v = s * sum_w sum_c Re[dDelta/dE_v * m^H conj(W_w) m],
      dL/dE_c the same with -dDelta/dE_v, summed over v
    * g_rho(r) = dV * sum_G g_M(G) exp(-i G.r)
    * dL/dpsi_c += psi_v * g_rho,  dL/dpsi_v += psi_c * conj(g_rho).

    M chunks are recomputed from psi, as in the forward.  Returns
    ``(grad_psi_v, grad_psi_c, grad_e_v, grad_e_c)``.

    Parity: pinned by central finite differences of ``chi0`` and by the
    shift and phase invariances of the loss."""
    n = tuple(int(x) for x in n)
    nv, nc = psi_v.shape[0], psi_c.shape[0]
    nr = int(np.prod(n))
    dv = volume / nr
    gvec = np.asarray(gvec)
    z = np.asarray(z, np.complex128).reshape(-1)
    w_all = np.asarray(grad_chi, np.complex128).reshape(z.size, gvec.shape[0], gvec.shape[0])
    delta = energy_factor(e_v, e_c, z)
    ddelta = energy_factor_dE(e_v, e_c, z)
    idx = (gvec[:, 0] % n[0], gvec[:, 1] % n[1], gvec[:, 2] % n[2])
    g_psi_v = np.zeros_like(psi_v, dtype=np.complex128)
    g_psi_c = np.zeros_like(psi_c, dtype=np.complex128)
    g_e_v = np.zeros(nv)
    g_e_c = np.zeros(nc)
    npairs = nv * nc
    step = max(1, int(pair_chunk))
    for k0 in range(0, npairs, step):
        k1 = min(npairs, k0 + step)
        m = mtxel(psi_v, psi_c, gvec, n, volume, pairs=range(k0, k1))    # [kc, ng]
        g_m = np.zeros_like(m)
        for w in range(z.size):
            wt = m @ w_all[w]                      # rows: (W^T m_p)^T
            wc = m @ np.conj(w_all[w]).T           # rows: (conj(W) m_p)^T
            g_m += spin * (np.conj(delta[w, k0:k1])[:, None] * wt + delta[w, k0:k1][:, None] * wc)
            quad = np.sum(np.conj(m) * wc, axis=1)  # m^H conj(W) m per pair
            de = spin * np.real(ddelta[w, k0:k1] * quad)
            for k in range(k1 - k0):
                v, c = divmod(k0 + k, nc)
                g_e_v[v] += de[k]
                g_e_c[c] -= de[k]
        for k in range(k1 - k0):
            v, c = divmod(k0 + k, nc)
            spec = np.zeros(n, dtype=np.complex128)
            np.add.at(spec, idx, g_m[k])
            g_rho = dv * np.fft.fftn(spec).reshape(-1)
            g_psi_c[c] += psi_v[v] * g_rho
            g_psi_v[v] += psi_c[c] * np.conj(g_rho)
    return g_psi_v, g_psi_c, g_e_v, g_e_c


def pseudobands(psi, e, keep, slices, n_xi, theta):
    """Stochastic pseudobands (Reduced Cost and Scaling section): the bands of
    each slice S are replaced by n_xi random-phase combinations
    ``xi_j^S = (1/sqrt(n_xi)) sum_{n in S} exp(2 pi i theta_n^j) psi_n``, each
    given the mean energy of the slice; the protected bands ``keep`` pass
    through unchanged.

    psi [nb][N_r], e [nb]; keep: band indices; slices: list of band-index
    arrays; theta: list (one per slice) of [n_xi][len(S)] arrays in [0, 1)
    (the random numbers are inputs).  Returns (psi_out, e_out) with the kept
    bands first, then the pseudobands slice by slice, j fastest.
    """
    rows = [psi[i] for i in keep]
    ens = [e[i] for i in keep]
    for s, th in zip(slices, theta):
        s = np.asarray(s)
        for j in range(n_xi):
            ph = np.exp(2j * np.pi * np.asarray(th[j], dtype=np.float64))
            rows.append((ph[:, None] * psi[s]).sum(axis=0) / np.sqrt(n_xi))
            ens.append(float(np.mean(e[s])))
    nr = psi.shape[1]
    out = np.array(rows, dtype=np.complex128).reshape(len(rows), nr)
    return out, np.array(ens, dtype=np.float64)


def static_subspace_basis(chi_static, n_eig, weight=None):
    """Diag of the static subspace method (Fast Full-Frequency GW section): the
    static polarizability is diagonalised and its ``n_eig`` most significant
    eigenvectors, read as those of largest |eigenvalue|, become the columns of
    C_s.  Returns ``(C_s [N_G, n_eig], eigenvalues [n_eig])`` in decreasing
    |eigenvalue| (for the negative semidefinite chi0(0): most negative first).
    With ``weight`` w (w_G = sqrt(v_G), v the Coulomb diagonal of Eq. (3)) the
    matrix diagonalised is the symmetrised W chi W, W = diag(w); the paper
    does not name the metric, and both readings are offered.
    A library Hermitian eigensolver is the step.

    Parity: pinned by a matrix built from a known spectrum, by plane waves
    (diagonal chi, unit-vector basis), by the diagonal static chi in the
    subspace, and for the weight by a diagonal chi (eigenvalues w_G^2 chi_GG)
    and the trace of W chi W."""
    chi_static = np.asarray(chi_static, np.complex128)
    if weight is not None:
        w = np.asarray(weight, np.float64)
        chi_static = w[:, None] * chi_static * w[None, :]
    lam, vec = np.linalg.eigh(chi_static)
    order = np.argsort(-np.abs(lam), kind="stable")[:int(n_eig)]
    return vec[:, order], lam[order]


def chi0_subspace(psi_v, psi_c, e_v, e_c, gvec, z, n, volume, basis, spin=2.0,
                  pair_chunk=4096, weight=None) -> np.ndarray:
    """Eq. (6): chi_BB'(z) = s * sum_vc conj(M^B_vc) Delta_vc(z) M^B'_vc, with
    the subspace matrix elements M^B_vc = sum_G M^G_vc C_s^{GB} (the transform
    the paper states after Eq. (6)), summed over chunks of pairs.  ``basis`` is
    C_s, ``[N_G, n_eig]``.  With ``weight`` w the basis is that of W chi W, and
    M^B_vc = sum_G M^G_vc w_G C_s^{GB}.  Returns ``[N_z, n_eig, n_eig]``.

    Parity: pinned by the full basis (C_s chi_B C_s^H = chi of Eq. (4), and
    W chi W with a weight), by the paper's identity chi_BB' = C_s^H chi C_s on a
    partial basis, and by plane waves."""
    nv, nc = psi_v.shape[0], psi_c.shape[0]
    z = np.asarray(z, np.complex128).reshape(-1)
    basis = np.asarray(basis, np.complex128)
    nb = basis.shape[1]
    wcol = np.ones(basis.shape[0]) if weight is None else np.asarray(weight, np.float64)
    delta = energy_factor(e_v, e_c, z)
    chi = np.zeros((z.size, nb, nb), dtype=np.complex128)
    npairs = nv * nc
    step = max(1, int(pair_chunk))
    for k0 in range(0, npairs, step):
        k1 = min(npairs, k0 + step)
        mb = (mtxel(psi_v, psi_c, gvec, n, volume, pairs=range(k0, k1)) * wcol[None, :]) @ basis
        for w in range(z.size):
            chi[w] += spin * ((np.conj(mb).T * delta[w, k0:k1][None, :]) @ mb)
    return chi


def coulomb(gvec, q=(0.0, 0.0, 0.0), cell_l=10.0) -> np.ndarray:
    """Diagonal of the Coulomb matrix of Eq. (3) in the plane-wave basis,
    ``v_G = 4 pi / |q + G|^2`` (Hartree atomic units) with G = 2 pi g / L for
    the cubic cell of edge L and q in units of 2 pi / L.  Where q + G = 0 (the
    G = 0 term at q = 0) the paper is silent; it is read as excluded, v = 0, so
    that the head and wings of eps^-1 reduce to the identity there.

    Parity: pinned by its closed form on axis vectors and the q = 0 head."""
    k = (np.asarray(gvec, np.float64) + np.asarray(q, np.float64)[None, :]) * (2.0 * np.pi / cell_l)
    k2 = np.sum(k * k, axis=1)
    v = np.zeros_like(k2)
    nz = k2 > 0.0
    v[nz] = 4.0 * np.pi / k2[nz]
    return v


def epsilon_inverse(chi, v) -> np.ndarray:
    """Eq. (3): eps^-1(z) = [I - v chi(z)]^-1 for every frequency, v the
    diagonal Coulomb matrix (``v`` its diagonal, ``[N_G]``), chi
    ``[N_z, N_G, N_G]``.  A library matrix inverse is the step.

    Parity: pinned by v = 0 (identity), a diagonal chi, a rank-one chi
    (Sherman-Morrison closed form) and the symmetrised form."""
    chi = np.asarray(chi, np.complex128)
    v = np.asarray(v, np.float64)
    ng = chi.shape[-1]
    eye = np.eye(ng, dtype=np.complex128)
    return np.stack([np.linalg.inv(eye - v[:, None] * c) for c in chi.reshape(-1, ng, ng)])


def gpp_inner(e, e_n, occupied, omega2, wtilde, v) -> np.ndarray:
    """The GPP inner matrix P^{nE}_{GG'} of the off-diagonal kernel (Optimized
    GPP Kernel for Off-Diagonal Self-Energy Matrix Elements section).  The
    paper names the band- and energy-dependent matrices P and the generalized
    plasmon-pole model, but prints no formula; it is read as the plasmon-pole
    correlation term of that model,
        P_GG' = Omega2_GG' v_G' / (2 wt_GG' (E - E_n - s_n wt_GG')),
    s_n = -1 for an occupied band and +1 for an empty one, with E complex (its
    imaginary part a broadening).  ``omega2`` [N_G, N_G] complex, ``wtilde``
    [N_G, N_G] positive, ``v`` [N_G]."""
    s_n = -1.0 if occupied else 1.0
    wt = np.asarray(wtilde, np.float64)
    return (np.asarray(omega2, np.complex128) * np.asarray(v, np.float64)[None, :]
            / (2.0 * wt * (complex(e) - float(e_n) - s_n * wt)))


def gpp_sigma_offdiag(m, e_n, occupied, energies, omega2, wtilde, v) -> np.ndarray:
    """Full GPP self-energy matrix on an energy grid (the off-diagonal kernel):
        Sigma_lm(E) = sum_n sum_GG' conj(M_ln(G)) P^{nE}_GG' M_mn(G'),
    for every E of the grid, taken as the paper describes it: for each (n, E)
    one GEMM N_Sigma x N_G x N_G (conj(M_n) P) and one N_Sigma x N_G x N_Sigma
    (that product times M_n^T).  ``m`` [N_b, N_Sigma, N_G] (M_ln(G) for the
    states l of interest and bands n), ``e_n`` [N_b], ``occupied`` [N_b]
    booleans, ``energies`` [N_E] complex.  Returns [N_E, N_Sigma, N_Sigma].

    Parity: pinned by a brute-force loop over n, G and G' and by linearity in
    the bands."""
    m = np.asarray(m, np.complex128)
    nb, ns, _ = m.shape
    energies = np.asarray(energies, np.complex128).reshape(-1)
    out = np.zeros((energies.size, ns, ns), dtype=np.complex128)
    for i, e in enumerate(energies):
        for n in range(nb):
            p = gpp_inner(e, e_n[n], bool(occupied[n]), omega2, wtilde, v)
            t = np.conj(m[n]) @ p          # N_Sigma x N_G x N_G
            out[i] += t @ m[n].T           # N_Sigma x N_G x N_Sigma
    return out
