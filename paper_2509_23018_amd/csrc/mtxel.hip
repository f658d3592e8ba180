// MTXEL on gfx950: plane-wave matrix elements of pair densities (the
// definition after Eq. (2) of the paper), M_vc(G) = dV sum_r conj(psi_v) psi_c
// e^{+i G.r}, taken as a pruned 3D DFT that only produces the frequencies the
// G-sphere needs.
//
// Kernel 1 (fused; one workgroup of 8 waves per tile of 4 valence x 2*PPW
// conduction bands and group of j1 planes): per (plane, 16-row block of j2,
// 16-wide slab of j3) the tile's band rows are staged in LDS once; each wave
// forms rho = conj(psi_v) psi_c for its pairs from them, contracts over j3
// against the z twiddles (FP64 MFMA 16x16x4), feeds the accumulators
// straight back into a second MFMA contraction over j2 against the y
// twiddles, and writes the (k2,k3) values the G list uses.  Twiddle operands
// live in LDS in MFMA lane order.
// Kernel 2 (one workgroup per pair): contracts over j1 with the x twiddles on
// MFMA, reading the stage-y output with coalesced rows, and scatters the
// (k1, disc) box entries that are G vectors to their place in the G list.
#include <algorithm>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <vector>

#include "common.hpp"
#include "plan.hpp"
#include "lifetime.hpp"
#include "prof.hpp"

namespace gw {

namespace {

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int64_t kMaxGrid = int64_t(1) << 30;  // pairs per launch

double2 host_root(int64_t num, int64_t den) {
    // e^{+2 pi i num/den} with the argument reduced to [0, den)
    int64_t r = num % den;
    if (r < 0) r += den;
    const double a = 2.0 * M_PI * static_cast<double>(r) / static_cast<double>(den);
    return make_double2(std::cos(a), std::sin(a));
}

template <typename T>
T* upload(const std::vector<T>& h) {
    T* d = nullptr;
    if (h.empty()) return nullptr;
    GW_HIP_TRY(hipMalloc(&d, h.size() * sizeof(T)));
    GW_HIP_TRY(hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    return d;
}

// ---------------------------------------------------------------- kernel 1

constexpr int kLoadBatch = 8;  // x-stage k-steps whose loads are issued together
constexpr int kZyWaves = 8;
constexpr int kZyThreads = 64 * kZyWaves;
constexpr int kSlab = 16;              // j3 values per LDS slab (4 MFMA k-steps)
constexpr int kRowStride = kSlab + 1;  // padded LDS row: column reads hit distinct banks

// One workgroup = a tile of 4 valence x (2*PPW) conduction bands (4*2*PPW
// pairs); wave w owns valence band w/2 and PPW conduction bands.  For every
// (j1 plane, 16-row block of j2, 16-wide slab of j3) the tile's band rows are
// staged once in LDS and shared by all the pairs that use them; the next
// slab's global loads are in flight while the current one is contracted.
// K3: both stages take each complex product a b as three real MFMA
// products (Karatsuba: a.x b.x, a.y b.y, (a.x + a.y)(b.x + b.y);
// Re = p1 - p2, Im = p3 - p1 - p2), the third accumulator sets paid for by
// one pair fewer per wave.
template <int NB2, int NB3, int PPW, bool K3>
__global__ __launch_bounds__(kZyThreads) void mtxel_zy_kernel(
    const double2* __restrict__ psi_v, const double2* __restrict__ psi_c, int64_t nr, Rect rc,
    int n1, int planes_per_group, int n2, int n3, int n2p, int n3p,
    const double2* __restrict__ w3tab,
    const double2* __restrict__ w2tab, const int* __restrict__ boxmap, int n23,
    double2* __restrict__ t2) {
    constexpr int TV = 4, TC = 2 * PPW, NBANDS = TV + TC;
    constexpr int NFILL = NBANDS * 256 / kZyThreads;  // staged elements per thread
    extern __shared__ double2 lds[];
    const int nslab = n3p / kSlab;
    const int q = n3p >> 2;
    const int nrb1 = n2p >> 4;
    const int w3n = q * NB3 * 64;
    const int w2n = nrb1 * 4 * NB2 * 64;
    constexpr int boxn = NB2 * 16 * NB3 * 16;
    double2* s_w3 = lds;
    double2* s_w2 = lds + w3n;
    int* s_box = reinterpret_cast<int*>(lds + w3n + w2n);
    double2* s_slab = lds + w3n + w2n + boxn / 4;  // [NBANDS][16][kRowStride]
    for (int i = threadIdx.x; i < w3n; i += kZyThreads) s_w3[i] = w3tab[i];
    for (int i = threadIdx.x; i < w2n; i += kZyThreads) s_w2[i] = w2tab[i];
    for (int i = threadIdx.x; i < boxn; i += kZyThreads) s_box[i] = boxmap[i];

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63, row = lane & 15, kq = lane >> 4;
    const int tv0 = blockIdx.y * TV, tc0 = blockIdx.x * TC;

    // staging slots of this thread: band fb[u], row fr[u], column fc[u]
    const double2* fptr[NFILL];
    int fr[NFILL], fc[NFILL], fb[NFILL];
    bool fok[NFILL];
#pragma unroll
    for (int u = 0; u < NFILL; ++u) {
        const int e = tid + kZyThreads * u;
        fb[u] = e >> 8;
        fr[u] = (e >> 4) & 15;
        fc[u] = e & 15;
        if (fb[u] < TV) {
            fok[u] = tv0 + fb[u] < rc.nv;
            fptr[u] = psi_v + (fok[u] ? static_cast<int64_t>(rc.v0 + tv0 + fb[u]) * nr : 0);
        } else {
            fok[u] = tc0 + fb[u] - TV < rc.nc;
            fptr[u] = psi_c + (fok[u] ? static_cast<int64_t>(rc.c0 + tc0 + fb[u] - TV) * nr : 0);
        }
    }
    double2 fv[NFILL];
    auto gload = [&](int j1, int rb1, int sl) {
#pragma unroll
        for (int u = 0; u < NFILL; ++u) {
            const int j2 = rb1 * 16 + fr[u], j3 = sl * kSlab + fc[u];
            fv[u] = (fok[u] && j2 < n2 && j3 < n3)
                        ? fptr[u][(static_cast<int64_t>(j1) * n2 + j2) * n3 + j3]
                        : make_double2(0.0, 0.0);
        }
    };
    auto sstore = [&]() {
#pragma unroll
        for (int u = 0; u < NFILL; ++u) s_slab[(fb[u] * 16 + fr[u]) * kRowStride + fc[u]] = fv[u];
    };

    const int vl = wave >> 1, cl0 = (wave & 1) * PPW;
    bool pok[PPW];
#pragma unroll
    for (int p = 0; p < PPW; ++p) pok[p] = tv0 + vl < rc.nv && tc0 + cl0 + p < rc.nc;

    // accumulators: Re, Im (a?s unused), or with K3 the three products
    dbl4 a1r[PPW][NB3], a1i[PPW][NB3], a1s[PPW][NB3];
    dbl4 a2r[PPW][NB2][NB3], a2i[PPW][NB2][NB3], a2s[PPW][NB2][NB3];
#pragma unroll
    for (int p = 0; p < PPW; ++p)
#pragma unroll
        for (int b3 = 0; b3 < NB3; ++b3) {
            a1r[p][b3] = a1i[p][b3] = a1s[p][b3] = zero4();
#pragma unroll
            for (int b2 = 0; b2 < NB2; ++b2) a2r[p][b2][b3] = a2i[p][b2][b3] = a2s[p][b2][b3] = zero4();
        }

    // this workgroup's planes: j1 in [j1b, j1e)
    const int j1b = blockIdx.z * planes_per_group;
    const int j1e = min(n1, j1b + planes_per_group);
    int j1 = j1b, rb1 = 0, sl = 0;      // position being contracted
    int nj1 = j1b, nrb = 0, nsl = 0;    // position being loaded
    gload(j1b, 0, 0);
    const int total = (j1e - j1b) * nrb1 * nslab;
    for (int it = 0; it < total; ++it) {
        __syncthreads();  // previous slab fully read (and tables visible)
        sstore();
        __syncthreads();
        // advance the load position (clamped at the end: a harmless re-load)
        if (++nsl == nslab) {
            nsl = 0;
            if (++nrb == nrb1) {
                nrb = 0;
                if (++nj1 == j1e) {
                    nj1 = j1e - 1;
                    nrb = nrb1 - 1;
                    nsl = nslab - 1;
                }
            }
        }
        gload(nj1, nrb, nsl);
        __builtin_amdgcn_sched_barrier(0);
        // z stage on this slab: A = rho rows (j2 = rb1*16+row, j3 = 16*sl + 4*kk + kq)
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const int ks = sl * 4 + kk;
            const double2 xv = s_slab[(vl * 16 + row) * kRowStride + 4 * kk + kq];
            double2 w3[NB3];
            double w3s[NB3];
#pragma unroll
            for (int b3 = 0; b3 < NB3; ++b3) {
                w3[b3] = s_w3[(ks * NB3 + b3) * 64 + lane];
                w3s[b3] = w3[b3].x + w3[b3].y;
            }
#pragma unroll
            for (int p = 0; p < PPW; ++p) {
                const double2 xc = s_slab[((TV + cl0 + p) * 16 + row) * kRowStride + 4 * kk + kq];
                const double2 rho = cmul_conj_a(xv, xc);
                if constexpr (K3) {
                    const double rs = rho.x + rho.y;
#pragma unroll
                    for (int b3 = 0; b3 < NB3; ++b3) {
                        a1r[p][b3] = mfma_f64(rho.x, w3[b3].x, a1r[p][b3]);
                        a1i[p][b3] = mfma_f64(rho.y, w3[b3].y, a1i[p][b3]);
                        a1s[p][b3] = mfma_f64(rs, w3s[b3], a1s[p][b3]);
                    }
                } else {
#pragma unroll
                    for (int b3 = 0; b3 < NB3; ++b3)
                        cmfma(a1r[p][b3], a1i[p][b3], rho.x, rho.y, w3[b3].x, w3[b3].y);
                }
            }
        }
        if (sl == nslab - 1) {
            // y stage: a1[p][b3] element t of lane l is T1[j2 = rb1*16 + 4*t + kq][k3 = b3*16 + row],
            // the B operand of k-step t (k index kq)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
#pragma unroll
                for (int b2 = 0; b2 < NB2; ++b2) {
                    const double2 w = s_w2[((rb1 * 4 + t) * NB2 + b2) * 64 + lane];
                    const double ws = w.x + w.y;
#pragma unroll
                    for (int p = 0; p < PPW; ++p)
#pragma unroll
                        for (int b3 = 0; b3 < NB3; ++b3) {
                            if constexpr (K3) {
                                // T1 = (p1 - p2, p3 - p1 - p2); Re T1 + Im T1 = p3 - 2 p2
                                const double p1 = a1r[p][b3][t], p2 = a1i[p][b3][t],
                                             p3 = a1s[p][b3][t];
                                const double tr = p1 - p2, ti = p3 - p1 - p2, ts = p3 - 2.0 * p2;
                                a2r[p][b2][b3] = mfma_f64(w.x, tr, a2r[p][b2][b3]);
                                a2i[p][b2][b3] = mfma_f64(w.y, ti, a2i[p][b2][b3]);
                                a2s[p][b2][b3] = mfma_f64(ws, ts, a2s[p][b2][b3]);
                            } else {
                                cmfma(a2r[p][b2][b3], a2i[p][b2][b3], w.x, w.y, a1r[p][b3][t],
                                      a1i[p][b3][t]);
                            }
                        }
                }
            }
#pragma unroll
            for (int p = 0; p < PPW; ++p)
#pragma unroll
                for (int b3 = 0; b3 < NB3; ++b3) a1r[p][b3] = a1i[p][b3] = a1s[p][b3] = zero4();
            if (rb1 == nrb1 - 1) {
#pragma unroll
                for (int p = 0; p < PPW; ++p) {
                    if (pok[p]) {
                        const int64_t k = static_cast<int64_t>(tv0 + vl) * rc.nc + tc0 + cl0 + p;
                        double2* o = t2 + (k * n1 + j1) * n23;
#pragma unroll
                        for (int b2 = 0; b2 < NB2; ++b2)
#pragma unroll
                            for (int b3 = 0; b3 < NB3; ++b3)
#pragma unroll
                                for (int t = 0; t < 4; ++t) {
                                    const int d = s_box[(b2 * 16 + 4 * t + kq) * (NB3 * 16) +
                                                        b3 * 16 + row];
                                    if (d >= 0) {
                                        const double p1 = a2r[p][b2][b3][t], p2 = a2i[p][b2][b3][t];
                                        o[d] = K3 ? make_double2(p1 - p2, a2s[p][b2][b3][t] - p1 - p2)
                                                  : make_double2(p1, p2);
                                    }
                                }
                    }
#pragma unroll
                    for (int b2 = 0; b2 < NB2; ++b2)
#pragma unroll
                        for (int b3 = 0; b3 < NB3; ++b3)
                            a2r[p][b2][b3] = a2i[p][b2][b3] = a2s[p][b2][b3] = zero4();
                }
            }
        }
        if (++sl == nslab) {
            sl = 0;
            if (++rb1 == nrb1) {
                rb1 = 0;
                ++j1;
            }
        }
    }
}

// ---------------------------------------------------------------- kernel 2

// M_box[k1][d] = sum_j1 W1[k1][j1] T2[j1][d] on MFMA: A = x twiddles (LDS,
// lane order), B = T2 rows (coalesced), output scattered to the G list.
template <int NB1>
__global__ __launch_bounds__(kThreads) void mtxel_x_kernel(
    const double2* __restrict__ t2, int n1, int n1p, int n23, int n23p,
    const double2* __restrict__ w1tab, const int* __restrict__ gmap, int ng, double dv,
    int64_t npairs, double2* __restrict__ m_out) {
    extern __shared__ double2 s_w1[];
    const int q1 = n1p >> 2;
    for (int i = threadIdx.x; i < NB1 * q1 * 64; i += kThreads) s_w1[i] = w1tab[i];
    __syncthreads();
    const int64_t k = blockIdx.x;
    if (k >= npairs) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, row = lane & 15, kq = lane >> 4;
    const double2* src = t2 + k * static_cast<int64_t>(n1) * n23;
    double2* dst = m_out + k * static_cast<int64_t>(ng);
    const int ndb = n23p >> 4;
    for (int db = wave; db < ndb; db += kWaves) {
        dbl4 ar[NB1], ai[NB1];
#pragma unroll
        for (int b = 0; b < NB1; ++b) ar[b] = ai[b] = zero4();
        const int d = db * 16 + row;
        const bool dok = d < n23;
        for (int ks0 = 0; ks0 < q1; ks0 += kLoadBatch) {
            double2 xb[kLoadBatch];
#pragma unroll
            for (int u = 0; u < kLoadBatch; ++u) {
                const int j1 = 4 * (ks0 + u) + kq;
                xb[u] = (dok && j1 < n1) ? src[static_cast<int64_t>(j1) * n23 + d]
                                         : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int u = 0; u < kLoadBatch; ++u) {
                const int ks = ks0 + u;
                if (ks < q1) {
#pragma unroll
                    for (int b = 0; b < NB1; ++b) {
                        const double2 w = s_w1[(b * q1 + ks) * 64 + lane];
                        cmfma(ar[b], ai[b], w.x, w.y, xb[u].x, xb[u].y);
                    }
                }
            }
        }
#pragma unroll
        for (int b = 0; b < NB1; ++b)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int g = gmap[(b * 16 + 4 * t + kq) * n23p + d];
                if (g >= 0) dst[g] = make_double2(dv * ar[b][t], dv * ai[b][t]);
            }
    }
}

using ZyKernel = void (*)(const double2*, const double2*, int64_t, Rect, int, int, int, int, int,
                          int, const double2*, const double2*, const int*, int, double2*);

// Pairs per wave by the widest box axis (in 16-wide blocks), within the
// registers of two waves per SIMD; the single-block case uses K3.
template <int NB2, int NB3>
ZyKernel zy_ptr() {
    constexpr int nb = NB2 > NB3 ? NB2 : NB3;
    constexpr int ppw = nb == 1 ? 3 : (nb == 2 ? 2 : 1);
    return &mtxel_zy_kernel<NB2, NB3, ppw, nb == 1>;
}

int zy_pairs_per_wave(int nb2, int nb3) {
    const int nb = std::max(nb2, nb3);
    return nb == 1 ? 3 : (nb == 2 ? 2 : 1);
}

ZyKernel select_zy(int nb2, int nb3) {
    static const ZyKernel table[4][4] = {
        {zy_ptr<1, 1>(), zy_ptr<1, 2>(), zy_ptr<1, 3>(), zy_ptr<1, 4>()},
        {zy_ptr<2, 1>(), zy_ptr<2, 2>(), zy_ptr<2, 3>(), zy_ptr<2, 4>()},
        {zy_ptr<3, 1>(), zy_ptr<3, 2>(), zy_ptr<3, 3>(), zy_ptr<3, 4>()},
        {zy_ptr<4, 1>(), zy_ptr<4, 2>(), zy_ptr<4, 3>(), zy_ptr<4, 4>()},
    };
    return table[nb2 - 1][nb3 - 1];
}

using XKernel = void (*)(const double2*, int, int, int, int, const double2*, const int*, int,
                         double, int64_t, double2*);

XKernel select_x(int nb1) {
    static const XKernel table[4] = {&mtxel_x_kernel<1>, &mtxel_x_kernel<2>, &mtxel_x_kernel<3>,
                                     &mtxel_x_kernel<4>};
    return table[nb1 - 1];
}

// ---------------------------------------------------------------- plan cache

struct PlanCache {
    std::mutex mu;
    std::map<int, std::vector<PlanRef>> by_device;
};

PlanCache& cache() {
    static PlanCache* c = new PlanCache();  // leaked on purpose: no teardown order issues
    return *c;
}

constexpr size_t kMaxLds = 160 * 1024;

std::unique_ptr<MtxelPlan> build_plan(const int n[3], const int32_t* gvec, int ng) {
    auto p = std::make_unique<MtxelPlan>();
    for (int a = 0; a < 3; ++a) p->n[a] = n[a];
    p->nr = static_cast<int64_t>(n[0]) * n[1] * n[2];
    p->ng = ng;
    p->gvec.assign(gvec, gvec + 3 * static_cast<size_t>(ng));

    std::vector<int> k1(ng), k2(ng), k3(ng);
    std::set<int> s1, s2, s3;
    for (int i = 0; i < ng; ++i) {
        k1[i] = ((gvec[3 * i] % n[0]) + n[0]) % n[0];
        k2[i] = ((gvec[3 * i + 1] % n[1]) + n[1]) % n[1];
        k3[i] = ((gvec[3 * i + 2] % n[2]) + n[2]) % n[2];
        s1.insert(k1[i]);
        s2.insert(k2[i]);
        s3.insert(k3[i]);
    }
    std::vector<int> l1(s1.begin(), s1.end()), l2(s2.begin(), s2.end()), l3(s3.begin(), s3.end());
    p->m1 = static_cast<int>(l1.size());
    p->nb1 = ceil_div(p->m1, 16);
    p->m2 = static_cast<int>(l2.size());
    p->m3 = static_cast<int>(l3.size());
    p->nb2 = ceil_div(p->m2, 16);
    p->nb3 = ceil_div(p->m3, 16);
    if (p->nb1 > 4 || p->nb2 > 4 || p->nb3 > 4)
        throw Error{-4, "G list spans more than 64 distinct values along an axis (unsupported)"};
    p->n2p = ceil_div(n[1], 16) * 16;
    p->n3p = ceil_div(n[2], 16) * 16;
    const int q = p->n3p / 4, nrb1 = p->n2p / 16;
    const int bw2 = p->nb2 * 16, bw3 = p->nb3 * 16;
    {
        const int ppw = zy_pairs_per_wave(p->nb2, p->nb3);
        const size_t nbands = 4 + 2 * static_cast<size_t>(ppw);
        p->lds_yz = (static_cast<size_t>(q) * p->nb3 * 64 + static_cast<size_t>(nrb1) * 4 * p->nb2 * 64 +
                     static_cast<size_t>(bw2) * bw3 / 4 + nbands * 16 * kRowStride) *
                    sizeof(double2);
    }
    if (p->lds_yz > kMaxLds)
        throw Error{-4, "grid too large for the LDS-resident twiddle operands (unsupported)"};
    p->n1p = ceil_div(n[0], 4) * 4;
    p->lds_x = static_cast<size_t>(p->nb1) * (p->n1p / 4) * 64 * sizeof(double2);
    if (p->lds_x > kMaxLds) throw Error{-4, "N1 too large (unsupported)"};

    std::map<int, int> i2, i3;
    for (int i = 0; i < p->m2; ++i) i2[l2[i]] = i;
    for (int i = 0; i < p->m3; ++i) i3[l3[i]] = i;
    std::vector<int> box(static_cast<size_t>(bw2) * bw3, -1);
    std::vector<int> g_disc(ng);
    int nd = 0;
    // disc numbered in (k2 index, k3 index) order
    std::set<std::pair<int, int>> disc;
    for (int i = 0; i < ng; ++i) disc.insert({i2[k2[i]], i3[k3[i]]});
    for (const auto& d : disc) box[d.first * bw3 + d.second] = nd++;
    p->n23 = nd;
    p->n23p = ceil_div(nd, 16) * 16;
    std::map<int, int> i1;
    for (int i = 0; i < p->m1; ++i) i1[l1[i]] = i;
    std::vector<int> gmap(static_cast<size_t>(p->nb1) * 16 * p->n23p, -1);
    for (int i = 0; i < ng; ++i) {
        g_disc[i] = box[i2[k2[i]] * bw3 + i3[k3[i]]];
        gmap[static_cast<size_t>(i1[k1[i]]) * p->n23p + g_disc[i]] = i;
    }
    const int q1 = p->n1p / 4;
    std::vector<double2> w1(static_cast<size_t>(p->nb1) * q1 * 64);
    for (int b = 0; b < p->nb1; ++b)
        for (int ks = 0; ks < q1; ++ks)
            for (int l = 0; l < 64; ++l) {
                const int kk = b * 16 + (l & 15);
                const int j1 = 4 * ks + (l >> 4);
                w1[(static_cast<size_t>(b) * q1 + ks) * 64 + l] =
                    (j1 < n[0] && kk < p->m1) ? host_root(static_cast<int64_t>(l1[kk]) * j1, n[0])
                                             : make_double2(0.0, 0.0);
            }

    std::vector<double2> w3(static_cast<size_t>(q) * p->nb3 * 64);
    for (int ks = 0; ks < q; ++ks)
        for (int b3 = 0; b3 < p->nb3; ++b3)
            for (int l = 0; l < 64; ++l) {
                const int j3 = 4 * ks + (l >> 4);
                const int kk = b3 * 16 + (l & 15);
                w3[(static_cast<size_t>(ks) * p->nb3 + b3) * 64 + l] =
                    (j3 < n[2] && kk < p->m3) ? host_root(static_cast<int64_t>(l3[kk]) * j3, n[2])
                                             : make_double2(0.0, 0.0);
            }
    std::vector<double2> w2(static_cast<size_t>(nrb1) * 4 * p->nb2 * 64);
    for (int rb1 = 0; rb1 < nrb1; ++rb1)
        for (int t = 0; t < 4; ++t)
            for (int b2 = 0; b2 < p->nb2; ++b2)
                for (int l = 0; l < 64; ++l) {
                    const int kk = b2 * 16 + (l & 15);
                    const int j2 = rb1 * 16 + 4 * t + (l >> 4);
                    w2[((static_cast<size_t>(rb1) * 4 + t) * p->nb2 + b2) * 64 + l] =
                        (j2 < n[1] && kk < p->m2)
                            ? host_root(static_cast<int64_t>(l2[kk]) * j2, n[1])
                            : make_double2(0.0, 0.0);
                }
    // adjoint tables, in the lane layouts of the transposed stages:
    //   x: U[j1][d]   = sum_k1 conj(e^{2 pi i k1 j1/N1}) B[k1][d]   (A = W1inv[j1][k1])
    //   z: T[k2][j3]  = sum_k3 Ubox[k2][k3] conj(e^{2 pi i k3 j3/N3}) (B = W3inv[k3][j3])
    //   y: R[j2][j3]  = sum_k2 conj(e^{2 pi i k2 j2/N2}) T[k2][j3]   (A = W2inv[j2][k2])
    p->n1p16 = ceil_div(n[0], 16) * 16;
    auto conj_root = [](int64_t num, int64_t den) {
        const double2 w = host_root(num, den);
        return make_double2(w.x, -w.y);
    };
    const int ks1 = p->nb1 * 4, ks2 = p->nb2 * 4, ks3 = p->nb3 * 4;
    std::vector<double2> w1i(static_cast<size_t>(p->n1p16 / 16) * ks1 * 64);
    for (int rb = 0; rb < p->n1p16 / 16; ++rb)
        for (int s = 0; s < ks1; ++s)
            for (int l = 0; l < 64; ++l) {
                const int j1 = rb * 16 + (l & 15), kk = 4 * s + (l >> 4);
                w1i[(static_cast<size_t>(rb) * ks1 + s) * 64 + l] =
                    (j1 < n[0] && kk < p->m1) ? conj_root(static_cast<int64_t>(l1[kk]) * j1, n[0])
                                             : make_double2(0.0, 0.0);
            }
    std::vector<double2> w2i(static_cast<size_t>(nrb1) * ks2 * 64);
    for (int rb = 0; rb < nrb1; ++rb)
        for (int s = 0; s < ks2; ++s)
            for (int l = 0; l < 64; ++l) {
                const int j2 = rb * 16 + (l & 15), kk = 4 * s + (l >> 4);
                w2i[(static_cast<size_t>(rb) * ks2 + s) * 64 + l] =
                    (j2 < n[1] && kk < p->m2) ? conj_root(static_cast<int64_t>(l2[kk]) * j2, n[1])
                                             : make_double2(0.0, 0.0);
            }
    const int nj3 = p->n3p / 16;
    std::vector<double2> w3i(static_cast<size_t>(ks3) * nj3 * 64);
    for (int s = 0; s < ks3; ++s)
        for (int nb = 0; nb < nj3; ++nb)
            for (int l = 0; l < 64; ++l) {
                const int kk = 4 * s + (l >> 4), j3 = nb * 16 + (l & 15);
                w3i[(static_cast<size_t>(s) * nj3 + nb) * 64 + l] =
                    (j3 < n[2] && kk < p->m3) ? conj_root(static_cast<int64_t>(l3[kk]) * j3, n[2])
                                             : make_double2(0.0, 0.0);
            }

    p->w1tab = upload(w1);
    p->gmap = upload(gmap);
    p->w3tab = upload(w3);
    p->w2tab = upload(w2);
    p->boxmap = upload(box);
    p->w1inv = upload(w1i);
    p->w2inv = upload(w2i);
    p->w3inv = upload(w3i);
    return p;
}

}  // namespace

void MtxelPlan::release() {
    (void)hipFree(w1tab);
    (void)hipFree(gmap);
    (void)hipFree(w3tab);
    (void)hipFree(w2tab);
    (void)hipFree(boxmap);
    (void)hipFree(w1inv);
    (void)hipFree(w2inv);
    (void)hipFree(w3inv);
    w1tab = w3tab = w2tab = w1inv = w2inv = w3inv = nullptr;
    gmap = boxmap = nullptr;
    if (last_use) (void)hipEventDestroy(last_use);
    last_use = nullptr;
}

namespace {

// Deleter of a cached plan: the tables are retired, freed once the last work
// that read them has completed.
void retire_plan(MtxelPlan* p) {
    const hipEvent_t ev = p->last_use;
    retire(p->device, ev, [p] {
        p->release();
        delete p;
    });
}

}  // namespace

PlanRef get_plan(const int n[3], const int32_t* gvec, int ng) {
    int dev = 0;
    GW_HIP_TRY(hipGetDevice(&dev));
    PlanCache& pc = cache();
    PlanRef evicted;  // released after the cache lock
    std::lock_guard<std::mutex> lk(pc.mu);
    auto& plans = pc.by_device[dev];
    for (auto& p : plans) {
        if (p->n[0] == n[0] && p->n[1] == n[1] && p->n[2] == n[2] && p->ng == ng &&
            std::equal(p->gvec.begin(), p->gvec.end(), gvec))
            return p;
    }
    require_alloc("plan (gather and twiddle tables) for this grid and G list");
    if (plans.size() >= 256) {  // bound the cache: drop the oldest plan
        evicted = std::move(plans.front());
        plans.erase(plans.begin());
    }
    std::unique_ptr<MtxelPlan> built = build_plan(n, gvec, ng);
    built->device = dev;
    GW_HIP_TRY(hipEventCreateWithFlags(&built->last_use, hipEventDisableTiming));
    plans.push_back(PlanRef(built.release(), retire_plan));
    return plans.back();
}

void mark_plan_used(MtxelPlan& p, hipStream_t s) {
    if (stream_capturing(s)) return;
    GW_HIP_TRY(hipEventRecord(p.last_use, s));
}

void release_plans() {
    PlanCache& pc = cache();
    std::lock_guard<std::mutex> lk(pc.mu);
    pc.by_device.clear();  // every plan not held elsewhere is retired
}

size_t t2_elems(const MtxelPlan& p, int64_t npairs) {
    return static_cast<size_t>(npairs) * p.n[0] * p.n23;
}

void launch_mtxel(const MtxelPlan& p, const double2* psi_v, const double2* psi_c, Rect rc,
                  double volume, double2* t2, double2* m_out, hipStream_t s) {
    const int64_t npairs = static_cast<int64_t>(rc.nv) * rc.nc;
    if (npairs <= 0) return;
    ZyKernel kz = select_zy(p.nb2, p.nb3);
    const int ppw = zy_pairs_per_wave(p.nb2, p.nb3);
    GW_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(kz),
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   static_cast<int>(p.lds_yz)));
    {
        // pair tiles x groups of j1 planes: enough workgroups to fill the chip
        const int gx = ceil_div(rc.nc, 2 * ppw), gy = ceil_div(rc.nv, 4);
        const int64_t tiles = static_cast<int64_t>(gx) * gy;
        const int want = static_cast<int>(std::min<int64_t>(p.n[0], std::max<int64_t>(1, ceil_div64(2048, tiles))));
        const int pp = ceil_div(p.n[0], want);
        const dim3 grid(gx, gy, ceil_div(p.n[0], pp));
        ProfScope ps("mtxel_zy", s);
        hipLaunchKernelGGL(kz, grid, dim3(kZyThreads), p.lds_yz, s, psi_v, psi_c, p.nr, rc, p.n[0],
                           pp, p.n[1], p.n[2], p.n2p, p.n3p, p.w3tab, p.w2tab, p.boxmap, p.n23, t2);
        GW_HIP_TRY(hipGetLastError());
    }
    XKernel kx = select_x(p.nb1);
    GW_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(kx),
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   static_cast<int>(p.lds_x)));
    const double dv = volume / static_cast<double>(p.nr);
    for (int64_t k0 = 0; k0 < npairs; k0 += kMaxGrid) {
        const int64_t kb = std::min<int64_t>(kMaxGrid, npairs - k0);
        ProfScope ps("mtxel_x", s);
        hipLaunchKernelGGL(kx, dim3(static_cast<unsigned>(kb)), dim3(kThreads), p.lds_x, s,
                           t2 + k0 * static_cast<int64_t>(p.n[0]) * p.n23, p.n[0], p.n1p, p.n23,
                           p.n23p, p.w1tab, p.gmap, p.ng, dv, kb, m_out + k0 * p.ng);
        GW_HIP_TRY(hipGetLastError());
    }
}

}  // namespace gw
