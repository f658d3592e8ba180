// MTXEL on gfx950: plane-wave matrix elements of pair densities (the
// definition after Eq. (2) of the paper), M_vc(G) = dV sum_r conj(psi_v) psi_c
// e^{+i G.r}, taken as a pruned 3D DFT that only produces the frequencies the
// G-sphere needs.
//
// Kernel 1 (fused, one wave per pair, one workgroup per 4 pairs): for each
// j1 plane it forms rho = conj(psi_v) psi_c while loading the MFMA A operand,
// contracts over j3 against the z twiddles (FP64 MFMA 16x16x4), feeds the
// resulting accumulators straight back into a second MFMA contraction over
// j2 against the y twiddles, and writes the (k2,k3) values the G list uses.
// The twiddle operands live in LDS in MFMA lane order.
// Kernel 2 contracts over j1 and gathers onto the G list.
#include <algorithm>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <vector>

#include "common.hpp"
#include "plan.hpp"
#include "prof.hpp"

namespace gw {

namespace {

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;

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

template <int NB2, int NB3>
__global__ __launch_bounds__(kThreads) void mtxel_zy_kernel(
    const double2* __restrict__ psi_v, const double2* __restrict__ psi_c, int64_t nr,
    PairMap pm, int64_t npairs, int n1, int n2, int n3, int n2p, int n3p,
    const double2* __restrict__ w3tab, const double2* __restrict__ w2tab,
    const int* __restrict__ boxmap, int n23, double2* __restrict__ t2) {
    extern __shared__ double2 lds[];
    const int q = n3p >> 2;  // MFMA k-steps of the z stage
    const int nrb1 = n2p >> 4;
    const int w3n = q * NB3 * 64;
    const int w2n = nrb1 * 4 * NB2 * 64;
    double2* s_w3 = lds;
    double2* s_w2 = lds + w3n;
    int* s_box = reinterpret_cast<int*>(lds + w3n + w2n);
    for (int i = threadIdx.x; i < w3n; i += kThreads) s_w3[i] = w3tab[i];
    for (int i = threadIdx.x; i < w2n; i += kThreads) s_w2[i] = w2tab[i];
    for (int i = threadIdx.x; i < NB2 * 16 * NB3 * 16; i += kThreads) s_box[i] = boxmap[i];
    __syncthreads();

    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int row = lane & 15;
    const int kq = lane >> 4;
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kWaves + wave;
    if (k >= npairs) return;
    const int64_t lin = pm.k_off + k;
    const int64_t v = pm.v0 + lin / pm.cw;
    const int64_t c = pm.c0 + lin % pm.cw;
    const double2* pv = psi_v + v * nr;
    const double2* pc = psi_c + c * nr;
    double2* out = t2 + k * static_cast<int64_t>(n1) * n23;

    for (int j1 = 0; j1 < n1; ++j1) {
        dbl4 a2r[NB2][NB3], a2i[NB2][NB3];
#pragma unroll
        for (int b2 = 0; b2 < NB2; ++b2)
#pragma unroll
            for (int b3 = 0; b3 < NB3; ++b3) a2r[b2][b3] = a2i[b2][b3] = zero4();

        for (int rb1 = 0; rb1 < nrb1; ++rb1) {
            dbl4 a1r[NB3], a1i[NB3];
#pragma unroll
            for (int b3 = 0; b3 < NB3; ++b3) a1r[b3] = a1i[b3] = zero4();
            const int j2 = rb1 * 16 + row;
            const bool rowok = j2 < n2;
            const int64_t base = (static_cast<int64_t>(j1) * n2 + j2) * n3 + kq * q;
            // j3 = kq*q + ks: consecutive k-steps of one lane walk consecutive memory
            for (int ks = 0; ks < q; ++ks) {
                double2 rho = make_double2(0.0, 0.0);
                if (rowok && kq * q + ks < n3) rho = cmul_conj_a(pv[base + ks], pc[base + ks]);
#pragma unroll
                for (int b3 = 0; b3 < NB3; ++b3) {
                    const double2 w = s_w3[(ks * NB3 + b3) * 64 + lane];
                    cmfma(a1r[b3], a1i[b3], rho.x, rho.y, w.x, w.y);
                }
            }
            // a1[b3] element t of lane l is T1[j2 = rb1*16 + 4*t + kq][k3 = b3*16 + row]:
            // exactly the B operand of the y stage for k-step t (k index kq).
#pragma unroll
            for (int t = 0; t < 4; ++t) {
#pragma unroll
                for (int b2 = 0; b2 < NB2; ++b2) {
                    const double2 w = s_w2[((rb1 * 4 + t) * NB2 + b2) * 64 + lane];
#pragma unroll
                    for (int b3 = 0; b3 < NB3; ++b3)
                        cmfma(a2r[b2][b3], a2i[b2][b3], w.x, w.y, a1r[b3][t], a1i[b3][t]);
                }
            }
        }
        double2* o = out + static_cast<int64_t>(j1) * n23;
#pragma unroll
        for (int b2 = 0; b2 < NB2; ++b2)
#pragma unroll
            for (int b3 = 0; b3 < NB3; ++b3)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int k2i = b2 * 16 + 4 * t + kq;
                    const int k3i = b3 * 16 + row;
                    const int d = s_box[k2i * (NB3 * 16) + k3i];
                    if (d >= 0) o[d] = make_double2(a2r[b2][b3][t], a2i[b2][b3][t]);
                }
    }
}

// ---------------------------------------------------------------- kernel 2

__global__ __launch_bounds__(256) void mtxel_x_gather_kernel(
    const double2* __restrict__ t2, int n1, int n23, const double2* __restrict__ root1,
    const int* __restrict__ g_k1, const int* __restrict__ g_disc, int ng, double dv,
    int64_t pair0, double2* __restrict__ m_out) {
    extern __shared__ double2 s_root[];
    for (int i = threadIdx.x; i < n1; i += blockDim.x) s_root[i] = root1[i];
    __syncthreads();
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t k = pair0 + blockIdx.y;
    if (g >= ng) return;
    const int k1 = g_k1[g];
    const double2* src = t2 + k * static_cast<int64_t>(n1) * n23 + g_disc[g];
    double re = 0.0, im = 0.0;
    int idx = 0;
    for (int j1 = 0; j1 < n1; ++j1) {
        const double2 w = s_root[idx];
        const double2 x = src[static_cast<int64_t>(j1) * n23];
        re += w.x * x.x - w.y * x.y;
        im += w.x * x.y + w.y * x.x;
        idx += k1;
        if (idx >= n1) idx -= n1;
    }
    m_out[k * ng + g] = make_double2(dv * re, dv * im);
}

using ZyKernel = void (*)(const double2*, const double2*, int64_t, PairMap, int64_t, int, int,
                          int, int, int, const double2*, const double2*, const int*, int,
                          double2*);

template <int NB2, int NB3>
ZyKernel zy_ptr() {
    return &mtxel_zy_kernel<NB2, NB3>;
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

// ---------------------------------------------------------------- plan cache

struct PlanCache {
    std::mutex mu;
    std::map<int, std::vector<std::unique_ptr<MtxelPlan>>> by_device;
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
    std::set<int> s2, s3;
    for (int i = 0; i < ng; ++i) {
        k1[i] = ((gvec[3 * i] % n[0]) + n[0]) % n[0];
        k2[i] = ((gvec[3 * i + 1] % n[1]) + n[1]) % n[1];
        k3[i] = ((gvec[3 * i + 2] % n[2]) + n[2]) % n[2];
        s2.insert(k2[i]);
        s3.insert(k3[i]);
    }
    std::vector<int> l2(s2.begin(), s2.end()), l3(s3.begin(), s3.end());
    p->m2 = static_cast<int>(l2.size());
    p->m3 = static_cast<int>(l3.size());
    p->nb2 = ceil_div(p->m2, 16);
    p->nb3 = ceil_div(p->m3, 16);
    if (p->nb2 > 4 || p->nb3 > 4)
        throw Error{-4, "G list spans more than 64 distinct values along an axis (unsupported)"};
    p->n2p = ceil_div(n[1], 16) * 16;
    p->n3p = ceil_div(n[2], 4) * 4;
    const int q = p->n3p / 4, nrb1 = p->n2p / 16;
    const int bw2 = p->nb2 * 16, bw3 = p->nb3 * 16;
    p->lds_yz = (static_cast<size_t>(q) * p->nb3 * 64 + static_cast<size_t>(nrb1) * 4 * p->nb2 * 64) *
                    sizeof(double2) +
                static_cast<size_t>(bw2) * bw3 * sizeof(int);
    if (p->lds_yz > kMaxLds)
        throw Error{-4, "grid too large for the LDS-resident twiddle operands (unsupported)"};
    if (static_cast<size_t>(n[0]) * sizeof(double2) > kMaxLds)
        throw Error{-4, "N1 too large (unsupported)"};

    std::map<int, int> i2, i3;
    for (int i = 0; i < p->m2; ++i) i2[l2[i]] = i;
    for (int i = 0; i < p->m3; ++i) i3[l3[i]] = i;
    std::vector<int> box(static_cast<size_t>(bw2) * bw3, -1);
    std::vector<int> g_disc(ng), g_k1(ng);
    int nd = 0;
    // disc numbered in (k2 index, k3 index) order
    std::set<std::pair<int, int>> disc;
    for (int i = 0; i < ng; ++i) disc.insert({i2[k2[i]], i3[k3[i]]});
    for (const auto& d : disc) box[d.first * bw3 + d.second] = nd++;
    p->n23 = nd;
    for (int i = 0; i < ng; ++i) {
        g_disc[i] = box[i2[k2[i]] * bw3 + i3[k3[i]]];
        g_k1[i] = k1[i];
    }

    std::vector<double2> w3(static_cast<size_t>(q) * p->nb3 * 64);
    for (int ks = 0; ks < q; ++ks)
        for (int b3 = 0; b3 < p->nb3; ++b3)
            for (int l = 0; l < 64; ++l) {
                const int j3 = (l >> 4) * q + ks;
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
    std::vector<double2> r1(n[0]), r2(n[1]), r3(n[2]);
    for (int t = 0; t < n[0]; ++t) r1[t] = host_root(t, n[0]);
    for (int t = 0; t < n[1]; ++t) r2[t] = host_root(t, n[1]);
    for (int t = 0; t < n[2]; ++t) r3[t] = host_root(t, n[2]);
    std::vector<int> dptr(nd + 1, 0), dg(ng);
    for (int i = 0; i < ng; ++i) dptr[g_disc[i] + 1]++;
    for (int d = 0; d < nd; ++d) dptr[d + 1] += dptr[d];
    {
        std::vector<int> fill(dptr.begin(), dptr.end() - 1);
        for (int i = 0; i < ng; ++i) dg[fill[g_disc[i]]++] = i;
    }

    p->w3tab = upload(w3);
    p->w2tab = upload(w2);
    p->boxmap = upload(box);
    p->g_k1 = upload(g_k1);
    p->g_disc = upload(g_disc);
    p->root1 = upload(r1);
    p->root2 = upload(r2);
    p->root3 = upload(r3);
    p->k2val = upload(l2);
    p->k3val = upload(l3);
    p->disc_ptr = upload(dptr);
    p->disc_g = upload(dg);
    return p;
}

}  // namespace

void MtxelPlan::release() {
    (void)hipFree(w3tab);
    (void)hipFree(w2tab);
    (void)hipFree(boxmap);
    (void)hipFree(g_k1);
    (void)hipFree(g_disc);
    (void)hipFree(root1);
    (void)hipFree(root2);
    (void)hipFree(root3);
    (void)hipFree(k2val);
    (void)hipFree(k3val);
    (void)hipFree(disc_ptr);
    (void)hipFree(disc_g);
    w3tab = w2tab = root1 = root2 = root3 = nullptr;
    boxmap = g_k1 = g_disc = k2val = k3val = disc_ptr = disc_g = nullptr;
}

MtxelPlan* get_plan(const int n[3], const int32_t* gvec, int ng) {
    int dev = 0;
    GW_HIP_TRY(hipGetDevice(&dev));
    PlanCache& pc = cache();
    std::lock_guard<std::mutex> lk(pc.mu);
    auto& plans = pc.by_device[dev];
    for (auto& p : plans) {
        if (p->n[0] == n[0] && p->n[1] == n[1] && p->n[2] == n[2] && p->ng == ng &&
            std::equal(p->gvec.begin(), p->gvec.end(), gvec))
            return p.get();
    }
    if (plans.size() >= 256) {  // bound the cache: drop the oldest plan
        GW_HIP_TRY(hipDeviceSynchronize());
        plans.front()->release();
        plans.erase(plans.begin());
    }
    plans.push_back(build_plan(n, gvec, ng));
    return plans.back().get();
}

void release_plans() {
    PlanCache& pc = cache();
    std::lock_guard<std::mutex> lk(pc.mu);
    for (auto& kv : pc.by_device) {
        (void)hipSetDevice(kv.first);
        (void)hipDeviceSynchronize();
        for (auto& p : kv.second) p->release();
        kv.second.clear();
    }
}

size_t t2_elems(const MtxelPlan& p, int64_t npairs) {
    return static_cast<size_t>(npairs) * p.n[0] * p.n23;
}

void launch_mtxel(const MtxelPlan& p, const double2* psi_v, const double2* psi_c, PairMap pm,
                  int64_t npairs, double volume, double2* t2, double2* m_out, hipStream_t s) {
    if (npairs <= 0) return;
    ZyKernel kz = select_zy(p.nb2, p.nb3);
    GW_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(kz),
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   static_cast<int>(p.lds_yz)));
    const int64_t nblk = ceil_div64(npairs, kWaves);
    {
    ProfScope ps("mtxel_zy", s);
    hipLaunchKernelGGL(kz, dim3(static_cast<unsigned>(nblk)), dim3(kThreads), p.lds_yz, s, psi_v,
                       psi_c, p.nr, pm, npairs, p.n[0], p.n[1], p.n[2], p.n2p, p.n3p, p.w3tab,
                       p.w2tab, p.boxmap, p.n23, t2);
    GW_HIP_TRY(hipGetLastError());
    }
    const double dv = volume / static_cast<double>(p.nr);
    for (int64_t k0 = 0; k0 < npairs; k0 += 65535) {
        const int64_t kb = std::min<int64_t>(65535, npairs - k0);
        ProfScope ps("mtxel_x", s);
        hipLaunchKernelGGL(mtxel_x_gather_kernel, dim3(ceil_div(p.ng, 256), static_cast<unsigned>(kb)),
                           dim3(256), p.n[0] * sizeof(double2), s, t2, p.n[0], p.n23, p.root1,
                           p.g_k1, p.g_disc, p.ng, dv, k0, m_out);
        GW_HIP_TRY(hipGetLastError());
    }
}

}  // namespace gw
