// Adjoint of the chi0 build on gfx950 (not in the paper: the chain rule
// through Eq. (4) and through the plane-wave matrix elements, the quantity a
// perturbation-theory variant of GW needs as the first-order change of M).
//
// Per chunk of pairs (M recomputed, never stored):
//   P1 = M W_w, P2 = M W_w^H                    FP64 MFMA, fused epilogue:
//   g_M  = sum_w conj(s Delta_w) P1 + (s Delta_w) P2
//   q_wp = m_p^H conj(W_w) m_p = sum_i conj(M[p][i]) P2[p][i]   (partials per tile)
//   dL/dE_v = s sum_w sum_c Re[dDelta/dE_v q],  dL/dE_c = -(same) over v
//   g_rho = dV sum_G g_M(G) e^{-i G.r}           pruned inverse transform
//   dL/dpsi_c += psi_v g_rho,  dL/dpsi_v += psi_c conj(g_rho)  (ordered sums)
// For chunks of at most 8 valence bands (the default chunk shapes) the last
// two transform stages and both band sums run in one kernel and g_rho stays
// in registers.
// Every reduction runs in a fixed order, so results are bitwise reproducible.
#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <vector>

#include "backward.hpp"
#include "chi0.hpp"
#include "common.hpp"
#include "prof.hpp"

namespace gw {

namespace {

__global__ __launch_bounds__(256) void ddelta_kernel(const double* __restrict__ e_v,
                                                     const double* __restrict__ e_c, PairMap pm,
                                                     int64_t npairs, ZArgs za, int w0,
                                                     double2* __restrict__ dd) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= npairs) return;
    const int64_t lin = pm.k_off + k;
    const double de = e_v[pm.v0 + lin / pm.cw] - e_c[pm.c0 + lin % pm.cw];
    for (int w = 0; w < za.nz; ++w) {
        const double zr = za.re[w], zi = za.im[w];
        // -(de + z)^-2 - (de - z)^-2 with (x)^-1 = conj(x)/|x|^2
        const double ar = de + zr, br = de - zr;
        const double na = ar * ar + zi * zi, nb = br * br + zi * zi;
        const double2 ia = make_double2(ar / na, -zi / na);
        const double2 ib = make_double2(br / nb, zi / nb);
        const double2 a2 = cmul(ia, ia), b2 = cmul(ib, ib);
        dd[static_cast<int64_t>(w0 + w) * npairs + k] = make_double2(-a2.x - b2.x, -a2.y - b2.y);
    }
}

// P1 = M W and P2 = M W^H for one TM (pairs) x 64 (G) tile; fused epilogue.
// 4 waves of (TM/2) x 32.  TM = 32 cuts the last partial round of a launch
// to half of what 64 x 64 tiles leave.
// Each complex product a b is three real MFMA products (Karatsuba,
// p1 = ar br, p2 = ai bi, p3 = (ar + ai)(br + bi); Re = p1 - p2,
// Im = p3 - p1 - p2); the third accumulator set leaves registers for two
// workgroups per CU.
// SYM (Delta real, as on the imaginary and real axes): g_M = s Delta (P1 + P2)
// = s Delta M (W + W^H); w then holds W + W^H (formed by sym_kernel) and one
// product is formed instead of two, with one operand tile per stage; and
// sum_i conj(M_i) (P1 + P2)_i = conj(q) + q = 2 Re q, so half of it is stored
// as q (its real part is all that the energy gradient reads when Delta, and
// so dDelta/dE, is real).
template <int TM, bool SYM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void bwd_gm_kernel(const double2* __restrict__ m, int64_t kc,
                                                     int ng, const double2* __restrict__ w,
                                                     const double2* __restrict__ delta,
                                                     double2* __restrict__ gm,
                                                     double2* __restrict__ qpart, int mode) {
    constexpr int BX = TM / 32, NA = TM * 16 / 256;
    __shared__ double2 s_a[TM][17];
    __shared__ double2 s_b1[16][64];
    __shared__ double2 s_b2[16][64];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63, row = lane & 15, kq = lane >> 4;
    const int wi = wave >> 1, wj = wave & 1;
    const int64_t k0 = static_cast<int64_t>(blockIdx.y) * TM;
    const int i0 = blockIdx.x * 64;

    // p?r = Re a Re b, p?i = Im a Im b, p?s = (Re a + Im a)(Re b + Im b)
    dbl4 p1r[BX][2], p1i[BX][2], p1s[BX][2], p2r[BX][2], p2i[BX][2], p2s[BX][2];
#pragma unroll
    for (int x = 0; x < BX; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
            p1r[x][y] = p1i[x][y] = p1s[x][y] = p2r[x][y] = p2i[x][y] = p2s[x][y] = zero4();

    // Stage j0 (16 G) of the three operands: fetched into registers one stage
    // ahead, so that the global loads of stage j0 + 16 run under the MFMAs of
    // stage j0.  The loads are unconditional (addresses clamped into the
    // arrays) and nothing uses a loaded value before the stage is written to
    // LDS: the bounds masks and the conjugation of the W^H operand are applied
    // there, after the MFMAs, so no wait on a load lands before them.
    double2 ra[NA], rb1[4], rb2[4];
    const int64_t klast = kc - 1;
    const int glast = ng - 1;
    auto fetch = [&](int j0) {
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            const int e = tid + 256 * u;
            const int64_t k = std::min<int64_t>(k0 + (e >> 4), klast);
            const double2* src = m + k * ng + std::min(j0 + (e & 15), glast);
            ra[u].x = src->x;  // component loads (a struct copy into LDS may be
            ra[u].y = src->y;  // fused into one copy issued after the MFMAs)
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = tid + 256 * u;
            const double2* s1 = w + static_cast<int64_t>(std::min(j0 + (e >> 6), glast)) * ng +
                                std::min(i0 + (e & 63), glast);
            const double2* s2 = w + static_cast<int64_t>(std::min(i0 + (e >> 4), glast)) * ng +
                                std::min(j0 + (e & 15), glast);
            rb1[u].x = s1->x;
            rb1[u].y = s1->y;
            if (!SYM) {
                rb2[u].x = s2->x;
                rb2[u].y = s2->y;
            }
        }
    };
    const double2 zero = make_double2(0.0, 0.0);
    fetch(0);
    for (int j0 = 0; j0 < ng; j0 += 16) {
        __syncthreads();  // every wave is done with the previous stage
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            const int e = tid + 256 * u;
            const bool ok = k0 + (e >> 4) < kc && j0 + (e & 15) < ng;
            s_a[e >> 4][e & 15] = ok ? make_double2(ra[u].x, ra[u].y) : zero;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = tid + 256 * u;
            const bool ok1 = j0 + (e >> 6) < ng && i0 + (e & 63) < ng;
            const bool ok2 = i0 + (e >> 4) < ng && j0 + (e & 15) < ng;
            s_b1[e >> 6][e & 63] = ok1 ? make_double2(rb1[u].x, rb1[u].y) : zero;
            if (!SYM) s_b2[e & 15][e >> 4] = ok2 ? make_double2(rb2[u].x, -rb2[u].y) : zero;
        }
        __syncthreads();
        // issue priority 1 for the loads, 2 over the MFMAs, 0 for the stores
        // and barriers: the wave with MFMAs to issue goes first on the SIMD
        __builtin_amdgcn_s_setprio(1);
        if (j0 + 16 < ng) fetch(j0 + 16);
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_setprio(2);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            double2 a[BX], b1[2], b2[2];
#pragma unroll
            for (int x = 0; x < BX; ++x) a[x] = s_a[wi * (TM / 2) + x * 16 + row][s * 4 + kq];
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                b1[y] = s_b1[s * 4 + kq][wj * 32 + y * 16 + row];
                if (!SYM) b2[y] = s_b2[s * 4 + kq][wj * 32 + y * 16 + row];
            }
            double as[BX], bs1[2], bs2[2];
#pragma unroll
            for (int x = 0; x < BX; ++x) as[x] = a[x].x + a[x].y;
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                bs1[y] = b1[y].x + b1[y].y;
                if (!SYM) bs2[y] = b2[y].x + b2[y].y;
            }
#pragma unroll
            for (int x = 0; x < BX; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    p1r[x][y] = mfma_f64(a[x].x, b1[y].x, p1r[x][y]);
                    p1i[x][y] = mfma_f64(a[x].y, b1[y].y, p1i[x][y]);
                    p1s[x][y] = mfma_f64(as[x], bs1[y], p1s[x][y]);
                    if (!SYM) {
                        p2r[x][y] = mfma_f64(a[x].x, b2[y].x, p2r[x][y]);
                        p2i[x][y] = mfma_f64(a[x].y, b2[y].y, p2i[x][y]);
                        p2s[x][y] = mfma_f64(as[x], bs2[y], p2s[x][y]);
                    }
                }
        }
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_setprio(0);
    }

#pragma unroll
    for (int x = 0; x < BX; ++x)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int64_t r = k0 + wi * (TM / 2) + x * 16 + 4 * t + kq;
            const bool rok = r < kc;
            const double2 d = rok ? delta[r] : make_double2(0.0, 0.0);
            double qre = 0.0, qim = 0.0;
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                const int c = i0 + wj * 32 + y * 16 + row;
                if (rok && c < ng) {
                    const double2 a = make_double2(p1r[x][y][t] - p1i[x][y][t],
                                                   p1s[x][y][t] - p1r[x][y][t] - p1i[x][y][t]);
                    double2 g, b;
                    if (SYM) {  // a = M (W + W^H), Delta real
                        g = make_double2(d.x * a.x, d.x * a.y);
                        b = make_double2(0.5 * a.x, 0.5 * a.y);
                    } else {
                        b = make_double2(p2r[x][y][t] - p2i[x][y][t],
                                         p2s[x][y][t] - p2r[x][y][t] - p2i[x][y][t]);
                        g = cmul_conj_a(d, a);
                        const double2 h = cmul(d, b);
                        g.x += h.x;
                        g.y += h.y;
                    }
                    double2* dst = gm + r * ng + c;
                    if (mode) {
                        const double2 o = *dst;
                        g.x += o.x;
                        g.y += o.y;
                    }
                    *dst = g;
                    const double2 q = cmul_conj_a(m[r * ng + c], b);
                    qre += q.x;
                    qim += q.y;
                }
            }
            // sum over the 16 lanes that share this row (same kq)
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) {
                qre += __shfl_xor(qre, off, 64);
                qim += __shfl_xor(qim, off, 64);
            }
            if (row == 0 && rok)
                qpart[static_cast<int64_t>(blockIdx.x * 2 + wj) * kc + r] = make_double2(qre, qim);
        }
}

// out = W + W^H for an [n][n] matrix, 32 x 32 tiles: the transposed tile
// goes through LDS so that both reads are row-contiguous.
__global__ __launch_bounds__(256) void sym_kernel(const double2* __restrict__ w, int n,
                                                  double2* __restrict__ out) {
    __shared__ double2 t[32][33];
    const int i0 = blockIdx.y * 32, j0 = blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8)  // tile (j0.., i0..), transposed into t
        if (j0 + r < n && i0 + tx < n) t[tx][r] = w[static_cast<int64_t>(j0 + r) * n + i0 + tx];
    __syncthreads();
    for (int r = ty; r < 32; r += 8)
        if (i0 + r < n && j0 + tx < n) {
            const int64_t o = static_cast<int64_t>(i0 + r) * n + j0 + tx;
            const double2 a = w[o], b = t[r][tx];
            out[o] = make_double2(a.x + b.x, a.y - b.y);
        }
}

__global__ __launch_bounds__(256) void de_kernel(const double2* __restrict__ qpart, int nparts,
                                                 int nz, int64_t kc, const double2* __restrict__ dd,
                                                 double spin, double* __restrict__ de) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= kc) return;
    double acc = 0.0;
    for (int w = 0; w < nz; ++w) {
        double qr = 0.0, qi = 0.0;
#pragma unroll 8
        for (int p = 0; p < nparts; ++p) {
            const double2 q = qpart[(static_cast<int64_t>(w) * nparts + p) * kc + k];
            qr += q.x;
            qi += q.y;
        }
        const double2 d = dd[static_cast<int64_t>(w) * kc + k];
        acc += d.x * qr - d.y * qi;
    }
    de[k] = spin * acc;
}

// Energy gradients of one chunk from de[vl][cl]: workgroup v < vcount adds
// row v (sum over the chunk's conduction bands, a tree in LDS) into
// g_ev[v0 + v]; workgroups from vcount on take 256 conduction bands each and
// subtract their columns (sums over at most the chunk's valence bands).
__global__ __launch_bounds__(256) void de_reduce_kernel(const double* __restrict__ de, int vcount,
                                                        int cw, int v0, int c0,
                                                        double* __restrict__ g_ev,
                                                        double* __restrict__ g_ec) {
    const int t = threadIdx.x;
    if (static_cast<int>(blockIdx.x) < vcount) {
        if (!g_ev) return;
        const int v = blockIdx.x;
        double acc = 0.0;
        for (int c = t; c < cw; c += 256) acc += de[static_cast<int64_t>(v) * cw + c];
        __shared__ double red[256];
        red[t] = acc;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (t < h) red[t] += red[t + h];
            __syncthreads();
        }
        if (t == 0) g_ev[v0 + v] += red[0];
        return;
    }
    const int i = (blockIdx.x - vcount) * 256 + t;
    if (g_ec && i < cw) {
        double acc = 0.0;
        for (int v = 0; v < vcount; ++v) acc += de[static_cast<int64_t>(v) * cw + i];
        g_ec[c0 + i] -= acc;
    }
}

// The inverse of the pruned transform, g_rho(r) = dV sum_G e^{-i G.r} g_M(G),
// taken as the forward stages transposed, on FP64 MFMA 16x16x4 with twiddle
// operands read in lane order from the plan (A lane l: [row l%16][k l/16];
// B lane l: [k l/16][col l%16]; D element t of lane l: [4t + l/16][l%16]).
// Each axis sums over frequency classes a = min(k, N - k): the two
// frequencies of a class enter as
//   X(+a) e^{-i th} + X(-a) e^{+i th} = P cos th + Q sin th,
//   P = X(+a) + X(-a),  Q = -i (X(+a) - X(-a)),  th = 2 pi a j/N,
// so every stage multiplies by real cos | sin twiddles (two real MFMA
// products per block).  A block's 16 slots are the cos (slots 0-7) and sin
// (8-15) slots of 8 classes; a lane's k index kq meets slot 4 s + kq at
// k-step s, so the P of the classes kq and 4 + kq (k-steps 0, 1) and their
// Q (k-steps 2, 3) come from the same two pairs of values.

// -i x
__device__ __forceinline__ double2 mul_mi(double2 x) { return make_double2(x.y, -x.x); }

// The A or B operand of the 4 k-steps of a class block from the values of
// the lane's two classes: x[0], x[1] at +a, x[2], x[3] at -a.
__device__ __forceinline__ void pq_block(const double2 (&x)[4], double2 (&o)[4]) {
    o[0] = make_double2(x[0].x + x[2].x, x[0].y + x[2].y);
    o[1] = make_double2(x[1].x + x[3].x, x[1].y + x[3].y);
    o[2] = mul_mi(make_double2(x[0].x - x[2].x, x[0].y - x[2].y));
    o[3] = mul_mi(make_double2(x[1].x - x[3].x, x[1].y - x[3].y));
}

// Stage x, one workgroup per pair: U[k][j1][d] = sum over k1 of
// e^{-2 pi i k1 j1/N1} g_M[k][G(k1, d)] (0 where (k1, d) is no G).  The 4 waves
// take (16 j1) x (16 d) output blocks in turn; B[slot][d] is formed from the
// G values at +-a1 (gmapf: (class, sign, d) -> G).
__global__ __launch_bounds__(256) void bwd_x_kernel(const double2* __restrict__ gm, int ng, int n1,
                                                    int n1b, int nbh1, int n23, int n23p,
                                                    const double* __restrict__ w1ir,
                                                    const int* __restrict__ gmapf,
                                                    double2* __restrict__ u) {
    const int64_t k = blockIdx.x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, row = lane & 15, kq = lane >> 4;
    const double2* src = gm + k * ng;
    double2* dst = u + k * n1 * n23;
    const int ndb = n23p >> 4;
    const int ks1 = nbh1 * 4;
    for (int tile = wave; tile < n1b * ndb; tile += 4) {
        const int rb = tile / ndb, db = tile - rb * ndb;
        const int d = db * 16 + row;
        dbl4 ar = zero4(), ai = zero4();
        for (int b = 0; b < nbh1; ++b) {
            double2 x[4], bo[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                // i = 0, 1: classes 8b + kq, 8b + 4 + kq at +a; i = 2, 3 at -a
                const int g = gmapf[((8 * b + 4 * (i & 1) + kq) * 2 + (i >> 1)) * n23p + d];
                x[i] = g >= 0 ? src[g] : make_double2(0.0, 0.0);
            }
            pq_block(x, bo);
#pragma unroll
            for (int sl = 0; sl < 4; ++sl) {
                const double a = w1ir[(rb * ks1 + 4 * b + sl) * 64 + lane];
                ar = mfma_f64(a, bo[sl].x, ar);
                ai = mfma_f64(a, bo[sl].y, ai);
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int j1 = rb * 16 + 4 * t + kq;
            if (j1 < n1 && d < n23) dst[j1 * n23 + d] = make_double2(ar[t], ai[t]);
        }
    }
}

// Stage z of one plane, j3 block nb and k2 block b2: T[k2 row][j3] =
// sum over k3 of U(k2, k3) e^{-2 pi i k3 j3/N3}, the A operand formed from U at
// (k2 of the lane's row, +-a3) (boxi), the B operand the real inverse z
// twiddles.  Rows of T: slot r < 8 is k2 = +a2 of class 8 b2 + r, r >= 8 is
// -a2 of class 8 b2 + r - 8, so a T element t (t = 0, 1) and t + 2 are the
// two frequencies of one k2 class.
template <int NB3>
__device__ __forceinline__ void inv_stage_z(const double2* __restrict__ urow,
                                            const int* __restrict__ boxi, const double* __restrict__ w3ir,
                                            int b2, int nb, int nj3, int lane, int row, int kq,
                                            dbl4& tr, dbl4& ti) {
#pragma unroll
    for (int b3 = 0; b3 < NB3; ++b3) {
        double2 x[4], ao[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int d = boxi[(b2 * 16 + row) * (NB3 * 16) + b3 * 16 + 4 * i + kq];
            x[i] = d >= 0 ? urow[d] : make_double2(0.0, 0.0);
        }
        pq_block(x, ao);
#pragma unroll
        for (int sl = 0; sl < 4; ++sl) {
            const double b = w3ir[((4 * b3 + sl) * nj3 + nb) * 64 + lane];
            tr = mfma_f64(ao[sl].x, b, tr);
            ti = mfma_f64(ao[sl].y, b, ti);
        }
    }
}

// Stage y of one (j2 block rb, j3 block): g_rho[j2][j3] += sum over k2 of
// e^{-2 pi i k2 j2/N2} T[k2][j3]: the B operand of k-step t is P (t = 0, 1) or
// Q (t = 2, 3) of the k2 classes 8 b2 + 4 (t & 1) + kq, formed in the lane from
// T elements t & 1 and (t & 1) + 2.
__device__ __forceinline__ void inv_stage_y(const dbl4& tr, const dbl4& ti, const double* __restrict__ w2ir,
                                            int rb, int ks2, int b2, int lane, dbl4& gr, dbl4& gi) {
    double2 x[4], bo[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) x[t] = make_double2(tr[t], ti[t]);
    pq_block(x, bo);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const double a = w2ir[(rb * ks2 + b2 * 4 + t) * 64 + lane];
        gr = mfma_f64(a, bo[t].x, gr);
        gi = mfma_f64(a, bo[t].y, gi);
    }
}

// Stages z and y, one workgroup per pair, wave w taking the planes j1 = w,
// w + 4, ...: per plane and 16-wide block of j3, T for every k2 block (stage
// z), then each 16-row block of j2 (stage y).
template <int NB2, int NB3>
__global__ __launch_bounds__(256) void bwd_yz_kernel(const double2* __restrict__ u, int n1, int n2,
                                                     int n3, int n23, int nj2, int nj3,
                                                     const double* __restrict__ w2ir,
                                                     const double* __restrict__ w3ir,
                                                     const int* __restrict__ boxi, int64_t nr,
                                                     double dv, double2* __restrict__ grho) {
    const int64_t k = blockIdx.x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, row = lane & 15, kq = lane >> 4;
    constexpr int KS2 = NB2 * 4;
    for (int j1 = wave; j1 < n1; j1 += 4) {
        const double2* urow = u + (k * n1 + j1) * n23;
        double2* out = grho + k * nr + static_cast<int64_t>(j1) * n2 * n3;
        for (int nb = 0; nb < nj3; ++nb) {
            dbl4 tr[NB2], ti[NB2];
#pragma unroll
            for (int b2 = 0; b2 < NB2; ++b2) {
                tr[b2] = ti[b2] = zero4();
                inv_stage_z<NB3>(urow, boxi, w3ir, b2, nb, nj3, lane, row, kq, tr[b2], ti[b2]);
            }
            for (int rb = 0; rb < nj2; ++rb) {
                dbl4 gr = zero4(), gi = zero4();
#pragma unroll
                for (int b2 = 0; b2 < NB2; ++b2) inv_stage_y(tr[b2], ti[b2], w2ir, rb, KS2, b2, lane, gr, gi);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int j2 = rb * 16 + 4 * t + kq, j3 = nb * 16 + row;
                    if (j2 < n2 && j3 < n3) {
                        // g_rho is read back by a later kernel, from HBM: the
                        // stores are non-temporal
                        double* q = reinterpret_cast<double*>(out + j2 * n3 + j3);
                        __builtin_nontemporal_store(dv * gr[t], q);
                        __builtin_nontemporal_store(dv * gi[t], q + 1);
                    }
                }
            }
        }
    }
}

constexpr int kFuseV = 8;   // valence bands of a chunk the fused band reductions take
constexpr int kFuseC = 16;  // conduction bands per block of the fused band reductions
// Valence bands per pass of the fused inverse transform: each pass reads
// psi_c and reads and writes grad_psi_c of the block's conduction bands once,
// so wider passes move fewer bytes; their vpart sums stay in registers, and
// four still leave two waves per SIMD up to two class blocks on the z axis.
constexpr int pass_v(int nb3) { return nb3 <= 2 ? 4 : 2; }

// Stages z and y of the inverse transform fused with both band reductions, so
// that g_rho never leaves registers.  Workgroup (plane j1, block cb of kFuseC
// conduction bands) takes every valence band of the chunk; wave w takes the
// 16 x 16 output blocks (j2 block rb, j3 block nb) w, w + 4, ... of the plane,
// and for each block and pair (vl, cl) forms T (stage z) and the g_rho block
// (stage y) on the MFMAs as bwd_yz_kernel does, each lane then holding 4
// values of the block (rows j2 = 16 rb + 4 t + lane/16, column
// j3 = 16 nb + lane%16).  With those values in hand:
//   grad_psi_c[c0 + cl](r) += sum_vl psi_v[v0 + vl](r) g_rho(r)  (this
//       workgroup alone writes these points of these conduction bands);
//   vpart[cb][vl](r) = sum_{cl in cb} psi_c[c0 + cl](r) conj(g_rho(r)), added
//       over the blocks by vpart_reduce_kernel.
// The valence bands go in passes of pass_v(NB3) (their vpart sums stay in
// registers, psi_v of a pair's band is loaded one pair ahead), and T is formed again for each j2 block it feeds (a third more
// MFMA work on a plane of two j2 blocks), against 2 x 16 bytes per point and
// pair of HBM traffic when g_rho is stored and read back.
// On the smallest box (one class block on the y and z axes) everything that
// does not depend on the pair (the box map, both twiddle operands) is read
// once per block into registers, and the stage-z values of the next pair are
// loaded while the current pair's MFMAs run; larger boxes read them per
// k-step.
template <int NB2, int NB3>
__global__ __launch_bounds__(256) void bwd_yz_reduce_kernel(
    const double2* __restrict__ u, int n1, int n2, int n3, int n23, int nj2, int nj3,
    const double* __restrict__ w2ir, const double* __restrict__ w3ir,
    const int* __restrict__ boxi, int64_t nr, double dv, const double2* __restrict__ psi_v,
    const double2* __restrict__ psi_c, int v0, int c0, int cw, int vcount,
    double2* __restrict__ gpc, double2* __restrict__ vpart) {
    constexpr int KS2 = NB2 * 4;
    constexpr bool HOIST = NB2 * NB3 == 1;
    constexpr int PV = pass_v(NB3);  // valence bands per pass
    const int j1 = blockIdx.x, cb = blockIdx.y;
    const int cl0 = cb * kFuseC, ncl = min(cw, cl0 + kFuseC) - cl0;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, row = lane & 15, kq = lane >> 4;
    const int64_t plane = static_cast<int64_t>(j1) * n2 * n3;
    for (int blk = wave; blk < nj2 * nj3; blk += 4) {
        const int rb = blk / nj3, nb = blk - rb * nj3;
        const int j3 = nb * 16 + row;
        int64_t pos[4];
        bool ok[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int j2 = rb * 16 + 4 * t + kq;
            ok[t] = j2 < n2 && j3 < n3;
            pos[t] = ok[t] ? plane + static_cast<int64_t>(j2) * n3 + j3 : 0;
        }
        // HOIST: the box entries and both twiddle operands of the one class block
        int bm[4];
        double w3[4], w2[4];
        if constexpr (HOIST) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                bm[i] = boxi[row * 16 + 4 * i + kq];
                w3[i] = w3ir[(i * nj3 + nb) * 64 + lane];
                w2[i] = w2ir[(rb * KS2 + i) * 64 + lane];
            }
        }
        // stage-z values of pair (vl, cl) on this plane (HOIST only)
        auto load_x = [&](int vl, int cl, double2 (&x)[4]) {
            const double2* urow =
                u + ((static_cast<int64_t>(vl) * cw + cl0 + cl) * n1 + j1) * n23;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const double2* src = urow + (bm[i] >= 0 ? bm[i] : 0);
                x[i].x = src->x;
                x[i].y = src->y;
            }
        };
        for (int vp = 0; vp < vcount; vp += PV) {
            const int nvp = min(PV, vcount - vp);
            const int nq = ncl * nvp;  // pairs of this pass: q = cl * nvp + i
            double2 av[PV][4];
#pragma unroll
            for (int i = 0; i < PV; ++i)
#pragma unroll
                for (int t = 0; t < 4; ++t) av[i][t] = make_double2(0.0, 0.0);
            // psi_v of a pair's valence band at this lane's points, loaded one
            // pair ahead (the chunk's valence bands stay in the L2): registers
            // for the vpart sums of a wider pass instead of a copy per band
            auto load_pv = [&](int qq, double2 (&dst)[4]) {
                const int c = qq / nvp;
                const double2* pvr = psi_v + static_cast<int64_t>(v0 + vp + (qq - c * nvp)) * nr;
#pragma unroll
                for (int t = 0; t < 4; ++t) dst[t] = pvr[pos[t]];
            };
            double2 pvc[4], pvn[4];
            load_pv(0, pvc);
            // psi_c and the old grad_psi_c of conduction band cl at this lane's
            // points, loaded with its first pair (the MFMAs of that pair, and of
            // the band's other pairs, run before they are used)
            double2 pc[4], ac[4], go[4];
            double2 xcur[4], xnext[4];
            if constexpr (HOIST) load_x(vp, 0, xcur);
            for (int q = 0; q < nq; ++q) {
                const int cl = q / nvp, i = q - cl * nvp;
                if (i == 0) {
                    const int64_t row_c = static_cast<int64_t>(c0 + cl0 + cl) * nr;
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        pc[t] = psi_c[row_c + pos[t]];
                        go[t] = gpc ? gpc[row_c + pos[t]] : make_double2(0.0, 0.0);
                        ac[t] = make_double2(0.0, 0.0);
                    }
                }
                if constexpr (HOIST) {
                    if (q + 1 < nq) {
                        const int cn = (q + 1) / nvp;
                        load_x(vp + (q + 1 - cn * nvp), cn, xnext);
                    }
                }
                if (q + 1 < nq) load_pv(q + 1, pvn);
                double2 pv[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) pv[t] = pvc[t];
                dbl4 gr = zero4(), gi = zero4();
                if constexpr (HOIST) {
                    // stage z on the one class block, then stage y
                    double2 x[4], ao[4];
#pragma unroll
                    for (int ii = 0; ii < 4; ++ii)
                        x[ii] = bm[ii] >= 0 ? xcur[ii] : make_double2(0.0, 0.0);
                    pq_block(x, ao);
                    dbl4 tr = zero4(), ti = zero4();
#pragma unroll
                    for (int sl = 0; sl < 4; ++sl) {
                        tr = mfma_f64(ao[sl].x, w3[sl], tr);
                        ti = mfma_f64(ao[sl].y, w3[sl], ti);
                    }
                    double2 y[4], bo[4];
#pragma unroll
                    for (int t = 0; t < 4; ++t) y[t] = make_double2(tr[t], ti[t]);
                    pq_block(y, bo);
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        gr = mfma_f64(w2[t], bo[t].x, gr);
                        gi = mfma_f64(w2[t], bo[t].y, gi);
                    }
                } else {
                    const double2* urow =
                        u + ((static_cast<int64_t>(vp + i) * cw + cl0 + cl) * n1 + j1) * n23;
#pragma unroll 1
                    for (int b2 = 0; b2 < NB2; ++b2) {
                        dbl4 tr = zero4(), ti = zero4();
                        inv_stage_z<NB3>(urow, boxi, w3ir, b2, nb, nj3, lane, row, kq, tr, ti);
                        inv_stage_y(tr, ti, w2ir, rb, KS2, b2, lane, gr, gi);
                    }
                }
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const double g_r = dv * gr[t], g_i = dv * gi[t];
                    ac[t].x += pv[t].x * g_r - pv[t].y * g_i;  // psi_v g
                    ac[t].y += pv[t].x * g_i + pv[t].y * g_r;
#pragma unroll
                    for (int ii = 0; ii < PV; ++ii)
                        if (ii == i) {
                            av[ii][t].x += pc[t].x * g_r + pc[t].y * g_i;  // psi_c conj(g)
                            av[ii][t].y += pc[t].y * g_r - pc[t].x * g_i;
                        }
                }
                if (i == nvp - 1 && gpc)
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        if (ok[t])
                            gpc[static_cast<int64_t>(c0 + cl0 + cl) * nr + pos[t]] =
                                make_double2(go[t].x + ac[t].x, go[t].y + ac[t].y);
                if constexpr (HOIST) {
#pragma unroll
                    for (int ii = 0; ii < 4; ++ii) xcur[ii] = xnext[ii];
                }
#pragma unroll
                for (int t = 0; t < 4; ++t) pvc[t] = pvn[t];
            }
            if (vpart)
#pragma unroll
                for (int i = 0; i < PV; ++i) {
                    if (i >= nvp) break;
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        if (ok[t])
                            vpart[(static_cast<int64_t>(cb) * vcount + vp + i) * nr + pos[t]] = av[i][t];
                }
        }
    }
}

// grad_psi_c[c0 + cl] += sum_vl psi_v[v0 + vl] * g_rho[vl*cw + cl]
__global__ __launch_bounds__(256) void reduce_c_kernel(const double2* __restrict__ grho,
                                                       const double2* __restrict__ psi_v,
                                                       int64_t nr, int v0, int c0, int cw,
                                                       int vcount, int cl0,
                                                       double2* __restrict__ gpc) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    const int cl = cl0 + blockIdx.y;
    double re = 0.0, im = 0.0;
    for (int vl = 0; vl < vcount; ++vl) {
        const double2 a = psi_v[static_cast<int64_t>(v0 + vl) * nr + r];
        const double2 b = grho[(static_cast<int64_t>(vl) * cw + cl) * nr + r];
        re += a.x * b.x - a.y * b.y;
        im += a.x * b.y + a.y * b.x;
    }
    double2* dst = gpc + static_cast<int64_t>(c0 + cl) * nr + r;
    const double2 o = *dst;
    *dst = make_double2(o.x + re, o.y + im);
}

// grad_psi_v[v0 + vl] += sum_cl psi_c[c0 + cl] * conj(g_rho[vl*cw + cl])
__global__ __launch_bounds__(256) void reduce_v_kernel(const double2* __restrict__ grho,
                                                       const double2* __restrict__ psi_c,
                                                       int64_t nr, int v0, int c0, int cw,
                                                       int vl0, double2* __restrict__ gpv) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    const int vl = vl0 + blockIdx.y;
    double re = 0.0, im = 0.0;
    for (int cl = 0; cl < cw; ++cl) {
        const double2 a = psi_c[static_cast<int64_t>(c0 + cl) * nr + r];
        const double2 b = grho[(static_cast<int64_t>(vl) * cw + cl) * nr + r];
        re += a.x * b.x + a.y * b.y;  // a * conj(b)
        im += a.y * b.x - a.x * b.y;
    }
    double2* dst = gpv + static_cast<int64_t>(v0 + vl) * nr + r;
    const double2 o = *dst;
    *dst = make_double2(o.x + re, o.y + im);
}


// grad_psi_v[v0 + vl][r] += sum_cb vpart[cb][vl][r], in block order.
__global__ __launch_bounds__(256) void vpart_reduce_kernel(const double2* __restrict__ vpart,
                                                           int ncb, int vb, int64_t nr, int v0,
                                                           double2* __restrict__ gpv) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    const int vl = blockIdx.y;
    double re = 0.0, im = 0.0;
    for (int cb = 0; cb < ncb; ++cb) {
        const double2 x = vpart[(static_cast<int64_t>(cb) * vb + vl) * nr + r];
        re += x.x;
        im += x.y;
    }
    double2* dst = gpv + static_cast<int64_t>(v0 + vl) * nr + r;
    const double2 o = *dst;
    *dst = make_double2(o.x + re, o.y + im);
}

__global__ __launch_bounds__(256) void fill_zero_f64_kernel(double* __restrict__ p, int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = 0.0;
}

void fill_zero_f64(double* p, int64_t n, hipStream_t s) {
    if (!p || n <= 0) return;
    const int64_t blocks = std::min<int64_t>(ceil_div64(n, 256), 65536);
    hipLaunchKernelGGL(fill_zero_f64_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                       p, n);
    GW_HIP_TRY(hipGetLastError());
}

struct Carve {
    size_t off = 0;
    size_t take(size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~static_cast<size_t>(255);
        return o;
    }
};

constexpr int kYMax = 65535;  // gridDim.y limit

// Delta of frequency w is real: on the imaginary axis (and at z = 0), where
// delta_kernel sets its imaginary part to zero, and on the real axis.
bool real_delta(const gw_problem_t& p, int w) {
    const double2 z = reinterpret_cast<const double2*>(p.z)[w];
    return z.x == 0.0 || z.y == 0.0;
}

// Chunking and scratch layout of one adjoint call.
// Budget for keeping W + W^H of every frequency (GW_SYM_KEEP_BYTES overrides)
size_t sym_keep_bytes() {
    const char* e = std::getenv("GW_SYM_KEEP_BYTES");
    return e ? static_cast<size_t>(std::strtoull(e, nullptr, 10)) : size_t(1) << 30;
}

struct BwdLayout {
    int vb = 1, cwmax = 1;
    int64_t kmax = 0;
    int nparts = 0;
    bool fuse = false;
    // o_m, o_d, o_dd: two buffers each (MTXEL and Delta of chunk k + 1 on the
    // companion stream while chunk k is worked on); o_t2m: MTXEL's own
    // intermediate; o_t2: the x-stage output of the inverse transform
    size_t o_m[2] = {0, 0}, o_d[2] = {0, 0}, o_dd[2] = {0, 0};
    size_t o_t2m = 0, o_t2 = 0, o_gm = 0, o_q = 0, o_de = 0, o_rho = 0, o_vp = 0;
    // W + W^H (frequencies with a real Delta): of every frequency, formed once
    // per call, when those planes fit in sym_keep_bytes() (sym_all); else of
    // one, formed again per chunk
    size_t o_ws = 0;
    bool sym_all = false;
    size_t total = 0;
};

BwdLayout bwd_layout(const MtxelPlan& plan, const gw_problem_t& p, bool want_psi, bool want_psi_v,
                     int pair_chunk, bool kept) {
    BwdLayout L;
    const int64_t nr = plan.nr;
    const int ng = p.ng, nz = p.nz;
    // chunk rectangle: 4 valence bands per MTXEL tile, conduction width capped
    // at chunk / 4
    auto shape = [&](int chunk) {
        L.cwmax = std::max(1, std::min(p.nc, chunk / std::max(1, std::min(p.nv, 4))));
        L.vb = std::max(1, std::min(p.nv, chunk / L.cwmax));
    };
    shape(pair_chunk);
    // at most kFuseV valence bands: the inverse transform and the band
    // reductions run fused and g_rho is never stored; otherwise the chunk is
    // capped so that the per-pair grids g_rho stay within 2 GiB
    L.fuse = L.vb <= kFuseV;
    if (!L.fuse) {
        const int64_t per_pair = nr * static_cast<int64_t>(sizeof(double2));
        const int64_t cap = std::max<int64_t>(1, (int64_t(1) << 31) / per_pair);
        shape(static_cast<int>(std::min<int64_t>(pair_chunk, cap)));
        L.fuse = L.vb <= kFuseV;
    }
    if (kept) {
        // kept M holds gw_chi0's chunks of the same pair_chunk, in the same order
        const int cwf = std::max(1, std::min(p.nc, pair_chunk / std::max(1, std::min(p.nv, 4))));
        const int vbf = std::max(1, std::min(p.nv, pair_chunk / cwf));
        if (L.vb != vbf || L.cwmax != cwf)
            throw Error{GW_EINVAL,
                        "kept M: the adjoint's chunks (" + std::to_string(L.vb) + " x " +
                            std::to_string(L.cwmax) + ") are not the forward's (" +
                            std::to_string(vbf) + " x " + std::to_string(cwf) +
                            "); use a pair_chunk whose chunks span at most 8 valence bands"};
    }
    L.kmax = static_cast<int64_t>(L.vb) * L.cwmax;
    L.nparts = 2 * ceil_div(ng, 64);
    const int64_t kmax = L.kmax;
    Carve cv;
    for (int b = 0; b < 2; ++b) {
        L.o_m[b] = cv.take(kept ? 0 : kmax * ng * sizeof(double2));
        L.o_d[b] = cv.take(kmax * nz * sizeof(double2));
        L.o_dd[b] = cv.take(kmax * nz * sizeof(double2));
    }
    L.o_t2m = cv.take(kept ? 0 : t2_elems(plan, kmax) * sizeof(double2));
    L.o_t2 = cv.take(t2_elems(plan, kmax) * sizeof(double2));
    L.o_gm = cv.take(kmax * ng * sizeof(double2));
    bool any_sym = false;
    for (int w = 0; w < nz; ++w) any_sym = any_sym || real_delta(p, w);
    const size_t plane = static_cast<size_t>(ng) * ng * sizeof(double2);
    L.sym_all = any_sym && static_cast<size_t>(nz) * plane <= sym_keep_bytes();
    L.o_ws = cv.take(any_sym ? (L.sym_all ? static_cast<size_t>(nz) : 1) * plane : 0);
    L.o_q = cv.take(kmax * nz * L.nparts * sizeof(double2));
    L.o_de = cv.take(kmax * sizeof(double));
    L.o_rho = cv.take(want_psi && !L.fuse ? kmax * nr * sizeof(double2) : 0);
    const int ncb_max = ceil_div(L.cwmax, kFuseC);
    L.o_vp = cv.take(want_psi && L.fuse && want_psi_v
                         ? static_cast<size_t>(ncb_max) * L.vb * nr * sizeof(double2)
                         : 0);
    L.total = cv.off;
    return L;
}

}  // namespace

size_t chi0_backward_bytes(const MtxelPlan& plan, const gw_problem_t& p, bool want_psi_v,
                           bool want_psi_c, bool want_e, int pair_chunk, bool kept) {
    const int64_t npairs = static_cast<int64_t>(p.nv) * p.nc;
    const bool want_psi = want_psi_v || want_psi_c;
    if (npairs == 0 || (!want_psi && !want_e)) return 0;
    return bwd_layout(plan, p, want_psi, want_psi_v, pair_chunk, kept).total;
}

void run_chi0_backward(const MtxelPlan& plan, const gw_problem_t& p, const double2* grad_chi,
                       double2* grad_psi_v, double2* grad_psi_c, double* grad_e_v,
                       double* grad_e_c, double spin, int pair_chunk, hipStream_t s,
                       char* base, hipStream_t aux, hipEvent_t* ev, const double2* m_keep) {
    const int64_t nr = plan.nr;
    const int ng = p.ng, nz = p.nz;
    const int n1 = plan.n[0], n2 = plan.n[1], n3 = plan.n[2];
    const int64_t npairs = static_cast<int64_t>(p.nv) * p.nc;
    const bool want_psi = grad_psi_v || grad_psi_c;
    const bool want_e = grad_e_v || grad_e_c;
    const bool work = npairs > 0 && (want_psi || want_e);
    const BwdLayout L = work ? bwd_layout(plan, p, want_psi, grad_psi_v != nullptr, pair_chunk,
                                          m_keep != nullptr)
                             : BwdLayout{};
    const int vb = L.vb, cwmax = L.cwmax, nparts = L.nparts;
    launch_fill_zero(grad_psi_v, grad_psi_v ? static_cast<int64_t>(p.nv) * nr : 0, s);
    launch_fill_zero(grad_psi_c, grad_psi_c ? static_cast<int64_t>(p.nc) * nr : 0, s);
    fill_zero_f64(grad_e_v, p.nv, s);
    fill_zero_f64(grad_e_c, p.nc, s);
    if (!work) return;
    const bool fuse = L.fuse;
    const size_t o_t2 = L.o_t2, o_gm = L.o_gm, o_q = L.o_q, o_de = L.o_de, o_rho = L.o_rho,
                 o_vp = L.o_vp;
    double2 *mbufs[2], *dbufs[2], *ddbufs[2];
    for (int b = 0; b < 2; ++b) {
        mbufs[b] = reinterpret_cast<double2*>(base + L.o_m[b]);
        dbufs[b] = reinterpret_cast<double2*>(base + L.o_d[b]);
        ddbufs[b] = reinterpret_cast<double2*>(base + L.o_dd[b]);
    }
    double2* t2m = reinterpret_cast<double2*>(base + L.o_t2m);
    double2* t2 = reinterpret_cast<double2*>(base + o_t2);
    double2* gm = reinterpret_cast<double2*>(base + o_gm);
    double2* qpart = reinterpret_cast<double2*>(base + o_q);
    double* de = reinterpret_cast<double*>(base + o_de);
    double2* grho = reinterpret_cast<double2*>(base + o_rho);
    double2* vpart = grad_psi_v && fuse ? reinterpret_cast<double2*>(base + o_vp) : nullptr;
    double2* wsym = reinterpret_cast<double2*>(base + L.o_ws);
    const double2* z = reinterpret_cast<const double2*>(p.z);
    const double2* psi_v = reinterpret_cast<const double2*>(p.psi_v);
    const double2* psi_c = reinterpret_cast<const double2*>(p.psi_c);
    const double dv = p.grid.volume / static_cast<double>(nr);

    // chunks of vb valence x cwmax conduction bands; MTXEL, Delta and dDelta
    // of chunk k + 1 run on the companion stream (buffer (k + 1) & 1) while
    // chunk k is worked on here.  Events: ev[0] start on s; ev[1 + b] buffer
    // b filled; ev[3 + b] buffer b read for the last time.
    struct BChunk {
        int v0, c0, vcount, cw;
    };
    std::vector<BChunk> chunks;
    for (int v0 = 0; v0 < p.nv; v0 += vb)
        for (int c0 = 0; c0 < p.nc; c0 += cwmax)
            chunks.push_back({v0, c0, std::min(vb, p.nv - v0), std::min(cwmax, p.nc - c0)});
    std::vector<int64_t> moff(chunks.size(), 0);  // first row of chunk k in kept M
    for (size_t k = 1; k < chunks.size(); ++k)
        moff[k] = moff[k - 1] + static_cast<int64_t>(chunks[k - 1].vcount) * chunks[k - 1].cw;
    auto produce = [&](size_t k) {
        const int b = static_cast<int>(k & 1);
        const BChunk& c = chunks[k];
        const int64_t kc = static_cast<int64_t>(c.vcount) * c.cw;
        if (k >= 2) GW_HIP_TRY(hipStreamWaitEvent(aux, ev[3 + b], 0));
        PairMap pm{0, c.cw, c.v0, c.c0};
        if (!m_keep)
            launch_mtxel(plan, psi_v, psi_c, Rect{c.v0, c.vcount, c.c0, c.cw}, p.grid.volume, t2m,
                         mbufs[b], aux);
        launch_delta(p.e_v, p.e_c, pm, kc, z, nz, spin, dbufs[b], aux);
        for (int w0 = 0; w0 < nz; w0 += kMaxZ) {
            ZArgs za{};
            za.nz = std::min(kMaxZ, nz - w0);
            for (int w = 0; w < za.nz; ++w) {
                za.re[w] = z[w0 + w].x;
                za.im[w] = z[w0 + w].y;
            }
            hipLaunchKernelGGL(ddelta_kernel, dim3(static_cast<unsigned>(ceil_div64(kc, 256))),
                               dim3(256), 0, aux, p.e_v, p.e_c, pm, kc, za, w0, ddbufs[b]);
            GW_HIP_TRY(hipGetLastError());
        }
        GW_HIP_TRY(hipEventRecord(ev[1 + b], aux));
    };
    if (L.sym_all) {
        ProfScope ps("bwd_sym", s);
        for (int w = 0; w < nz; ++w)
            if (real_delta(p, w))
                hipLaunchKernelGGL(sym_kernel, dim3(ceil_div(ng, 32), ceil_div(ng, 32)), dim3(256),
                                   0, s, grad_chi + static_cast<int64_t>(w) * ng * ng, ng,
                                   wsym + static_cast<int64_t>(w) * ng * ng);
        GW_HIP_TRY(hipGetLastError());
    }
    GW_HIP_TRY(hipEventRecord(ev[0], s));
    GW_HIP_TRY(hipStreamWaitEvent(aux, ev[0], 0));
    produce(0);
    for (size_t ck = 0; ck < chunks.size(); ++ck) {
        {
            const int b = static_cast<int>(ck & 1);
            if (ck + 1 < chunks.size()) produce(ck + 1);
            GW_HIP_TRY(hipStreamWaitEvent(s, ev[1 + b], 0));
            const int v0 = chunks[ck].v0, c0 = chunks[ck].c0;
            const int vcount = chunks[ck].vcount, cw = chunks[ck].cw;
            const int64_t kc = static_cast<int64_t>(vcount) * cw;
            const double2* mbuf = m_keep ? m_keep + moff[ck] * ng : mbufs[b];
            double2* dbuf = dbufs[b];
            double2* ddbuf = ddbufs[b];
            for (int w = 0; w < nz; ++w) {
                ProfScope ps("bwd_gm", s);
                // Delta real: one product against W + W^H
                const bool sym = real_delta(p, w);
                const double2* wop = grad_chi + static_cast<int64_t>(w) * ng * ng;
                if (sym && L.sym_all) {
                    wop = wsym + static_cast<int64_t>(w) * ng * ng;
                } else if (sym) {
                    hipLaunchKernelGGL(sym_kernel, dim3(ceil_div(ng, 32), ceil_div(ng, 32)),
                                       dim3(256), 0, s, wop, ng, wsym);
                    wop = wsym;
                }
                auto gmk = sym ? bwd_gm_kernel<32, true> : bwd_gm_kernel<32, false>;
                hipLaunchKernelGGL(gmk,
                                   dim3(ceil_div(ng, 64), static_cast<unsigned>(ceil_div64(kc, 32))),
                                   dim3(256), 0, s, mbuf, kc, ng, wop, dbuf + w * kc, gm,
                                   qpart + static_cast<int64_t>(w) * nparts * kc, w > 0 ? 1 : 0);
                GW_HIP_TRY(hipGetLastError());
            }
            if (want_e) {
                {
                    ProfScope ps("bwd_de", s);
                    hipLaunchKernelGGL(de_kernel, dim3(static_cast<unsigned>(ceil_div64(kc, 256))),
                                       dim3(256), 0, s, qpart, nparts, nz, kc, ddbuf, spin, de);
                    GW_HIP_TRY(hipGetLastError());
                }
                ProfScope ps("bwd_de_reduce", s);
                hipLaunchKernelGGL(de_reduce_kernel, dim3(vcount + ceil_div(cw, 256)),
                                   dim3(256), 0, s, de, vcount, cw, v0, c0, grad_e_v, grad_e_c);
                GW_HIP_TRY(hipGetLastError());
            }
            // M, Delta and dDelta of buffer b are not read after this point
            GW_HIP_TRY(hipEventRecord(ev[3 + b], s));
            if (!want_psi) continue;
            {
                ProfScope ps("bwd_x", s);
                hipLaunchKernelGGL(bwd_x_kernel, dim3(static_cast<unsigned>(kc)), dim3(256), 0, s,
                                   gm, ng, n1, plan.n1p16 / 16, plan.nbh1, plan.n23, plan.n23p,
                                   plan.w1ir, plan.gmapf, t2);
                GW_HIP_TRY(hipGetLastError());
            }
            const int nj2 = plan.n2p / 16, nj3 = plan.n3p / 16;
            if (fuse) {
                const int ncb = ceil_div(cw, kFuseC);
                {
                    ProfScope ps("bwd_yz_reduce", s);
                    using YzrFn = decltype(&bwd_yz_reduce_kernel<1, 1>);
                    static const YzrFn table[4][4] = {
                        {bwd_yz_reduce_kernel<1, 1>, bwd_yz_reduce_kernel<1, 2>,
                         bwd_yz_reduce_kernel<1, 3>, bwd_yz_reduce_kernel<1, 4>},
                        {bwd_yz_reduce_kernel<2, 1>, bwd_yz_reduce_kernel<2, 2>,
                         bwd_yz_reduce_kernel<2, 3>, bwd_yz_reduce_kernel<2, 4>},
                        {bwd_yz_reduce_kernel<3, 1>, bwd_yz_reduce_kernel<3, 2>,
                         bwd_yz_reduce_kernel<3, 3>, bwd_yz_reduce_kernel<3, 4>},
                        {bwd_yz_reduce_kernel<4, 1>, bwd_yz_reduce_kernel<4, 2>,
                         bwd_yz_reduce_kernel<4, 3>, bwd_yz_reduce_kernel<4, 4>}};
                    hipLaunchKernelGGL(table[plan.nbh2 - 1][plan.nbh3 - 1],
                                       dim3(static_cast<unsigned>(n1), static_cast<unsigned>(ncb)),
                                       dim3(256), 0, s, t2, n1, n2, n3, plan.n23, nj2, nj3,
                                       plan.w2ir, plan.w3ir, plan.boxi, nr, dv, psi_v, psi_c,
                                       v0, c0, cw, vcount, grad_psi_c, vpart);
                    GW_HIP_TRY(hipGetLastError());
                }
                if (vpart) {
                    ProfScope ps("bwd_reduce_v", s);
                    hipLaunchKernelGGL(vpart_reduce_kernel,
                                       dim3(static_cast<unsigned>(ceil_div64(nr, 256)), vcount),
                                       dim3(256), 0, s, vpart, ncb, vcount, nr, v0, grad_psi_v);
                    GW_HIP_TRY(hipGetLastError());
                }
                continue;
            }
            {
                ProfScope ps("bwd_yz", s);
                using YzFn = decltype(&bwd_yz_kernel<1, 1>);
                static const YzFn ytable[4][4] = {
                    {bwd_yz_kernel<1, 1>, bwd_yz_kernel<1, 2>, bwd_yz_kernel<1, 3>, bwd_yz_kernel<1, 4>},
                    {bwd_yz_kernel<2, 1>, bwd_yz_kernel<2, 2>, bwd_yz_kernel<2, 3>, bwd_yz_kernel<2, 4>},
                    {bwd_yz_kernel<3, 1>, bwd_yz_kernel<3, 2>, bwd_yz_kernel<3, 3>, bwd_yz_kernel<3, 4>},
                    {bwd_yz_kernel<4, 1>, bwd_yz_kernel<4, 2>, bwd_yz_kernel<4, 3>, bwd_yz_kernel<4, 4>}};
                hipLaunchKernelGGL(ytable[plan.nbh2 - 1][plan.nbh3 - 1], dim3(static_cast<unsigned>(kc)),
                                   dim3(256), 0, s, t2, n1, n2, n3, plan.n23, nj2, nj3, plan.w2ir,
                                   plan.w3ir, plan.boxi, nr, dv, grho);
                GW_HIP_TRY(hipGetLastError());
            }
            if (grad_psi_c)
                for (int cl0 = 0; cl0 < cw; cl0 += kYMax) {
                    ProfScope ps("bwd_reduce_c", s);
                    hipLaunchKernelGGL(reduce_c_kernel,
                                       dim3(static_cast<unsigned>(ceil_div64(nr, 256)),
                                            std::min(kYMax, cw - cl0)),
                                       dim3(256), 0, s, grho, psi_v, nr, v0, c0, cw, vcount, cl0,
                                       grad_psi_c);
                    GW_HIP_TRY(hipGetLastError());
                }
            if (grad_psi_v)
                for (int vl0 = 0; vl0 < vcount; vl0 += kYMax) {
                    ProfScope ps("bwd_reduce_v", s);
                    hipLaunchKernelGGL(reduce_v_kernel,
                                       dim3(static_cast<unsigned>(ceil_div64(nr, 256)),
                                            std::min(kYMax, vcount - vl0)),
                                       dim3(256), 0, s, grho, psi_c, nr, v0, c0, cw, vl0,
                                       grad_psi_v);
                    GW_HIP_TRY(hipGetLastError());
                }
        }
    }
}

}  // namespace gw
