// CHI0 on gfx950: chi_w += M^H diag(s*Delta_w) M over one streamed chunk of
// pairs (Eq. (4) of the paper), FP64 MFMA 16x16x4 tiles, plus the energy
// factor, the Hermitian mirror and the zero fill.
#include <algorithm>
#include <cstdlib>
#include <map>
#include <tuple>
#include <mutex>
#include <vector>

#include "chi0.hpp"
#include "items.hpp"
#include "lifetime.hpp"
#include "common.hpp"
#include "prof.hpp"

namespace gw {

namespace {

// ---------------------------------------------------------------- energy factor

__global__ __launch_bounds__(256) void delta_kernel(const double* __restrict__ e_v,
                                                    const double* __restrict__ e_c, PairMap pm,
                                                    int64_t npairs, ZArgs za, int w0,
                                                    double2* __restrict__ delta) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= npairs) return;
    const int64_t lin = pm.k_off + k;
    const double de = e_v[pm.v0 + lin / pm.cw] - e_c[pm.c0 + lin % pm.cw];
    for (int w = 0; w < za.nz; ++w) {
        const double zr = za.re[w], zi = za.im[w];
        // 1/(de + z) + 1/(de - z), each as conj(d)/|d|^2
        const double ar = de + zr, br = de - zr;
        const double n1 = ar * ar + zi * zi, n2 = br * br + zi * zi;
        double re = ar / n1 + br / n2;
        double im = -zi / n1 + zi / n2;
        if (zr == 0.0) im = 0.0;  // imaginary axis / static: Delta is real
        delta[static_cast<int64_t>(w0 + w) * npairs + k] = make_double2(za.spin * re, za.spin * im);
    }
}

// ---------------------------------------------------------------- FP64 contraction

constexpr int kKt = 16;     // pairs per LDS stage

// One workgroup = one T x T tile of chi_w, WI x WJ waves, each a
// (T/WI) x (T/WJ) sub-tile of 16x16 MFMA blocks.  Per stage of kKt pairs the
// rows of M for the tile's G and G' are staged in LDS (double-buffered; rows
// padded by PAD elements), the G' side already multiplied by s*Delta_w(k);
// the MFMAs accumulate conj(M_i) (Delta M_j), with three real products per
// complex one on the 64x64 tile.  Loads are unconditional: pair
// rows past the chunk end are clamped and carry Delta = 0, columns past N_G
// are clamped and only feed outputs that are not stored.
// mode: 0 overwrite, 1 accumulate.  PART: store the whole T x T tile instead,
// unmasked, row-major at cw (a partial sum over a range of pairs).
template <int T, int WI, int WJ, int PAD, bool PART = false>
__device__ __forceinline__ void f64_tile(double2* lds, const double2* __restrict__ m, int64_t kc,
                                         int ng, const double2* __restrict__ dw,
                                         double2* __restrict__ cw, int mode, int bi, int bj) {
    constexpr int NT = WI * WJ * 64;
    constexpr int BX = T / WI / 16, BY = T / WJ / 16;
    constexpr int LDR = T + PAD;                 // LDS row length (double2)
    constexpr int NLOAD = kKt * T / NT;          // staged elements per thread per side
    static_assert(NLOAD * NT == kKt * T && NT % T == 0, "tile / thread mismatch");
    double2* s_a = lds;                  // [2][kKt][LDR]
    double2* s_b = lds + 2 * kKt * LDR;  // [2][kKt][LDR]
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63, row = lane & 15, kq = lane >> 4;
    const int wi = wave / WJ, wj = wave % WJ;
    const int i0 = bi * T, j0 = bj * T;

    // staging slots: element e = tid + NT*u -> row kk = e / T, column cc = e % T;
    // NT is a multiple of T, so cc is the same for every u and kk steps by NT/T
    constexpr int KSTEP = NT / T;
    const int cc = tid % T, kk0 = tid / T;
    const int64_t ci = min(i0 + cc, ng - 1), cj = min(j0 + cc, ng - 1);

    // conj(a) b with three real products where the registers allow
    // (Karatsuba, K3): p1 = ar br, p2 = ai bi, p3 = (ar - ai)(br + bi);
    // Re = p1 + p2, Im = p3 - p1 + p2.  Otherwise four: p1 = Re, p2 = Im
    // (p3 unused).
    constexpr bool K3 = BX * BY <= 4;
    dbl4 p1[BX][BY], p2[BX][BY], p3[BX][BY];
#pragma unroll
    for (int a = 0; a < BX; ++a)
#pragma unroll
        for (int b = 0; b < BY; ++b) p1[a][b] = p2[a][b] = p3[a][b] = zero4();

    double2 ra[NLOAD], rb[NLOAD];

    // stage 0
#pragma unroll
    for (int u = 0; u < NLOAD; ++u) {
        const int64_t k = kk0 + KSTEP * u;
        const int64_t kr = k < kc ? k : kc - 1;
        const double2 d = k < kc ? dw[kr] : make_double2(0.0, 0.0);
        s_a[(kk0 + KSTEP * u) * LDR + cc] = m[kr * ng + ci];
        s_b[(kk0 + KSTEP * u) * LDR + cc] = cmul(d, m[kr * ng + cj]);
    }
    __syncthreads();
    int buf = 0;
    const int nsteps = static_cast<int>((kc + kKt - 1) / kKt);
    for (int st = 0; st < nsteps; ++st) {
        // unconditional (clamped) prefetch of the next stage keeps the loop
        // free of branches, so the compiler cannot merge the LDS stores into
        // the load block
        // issue priority: 1 while the next stage's loads are issued, 2 over
        // the MFMA block, 0 for the LDS stores and the barrier; of the two
        // waves on a SIMD the one with MFMAs to issue goes first, the other
        // fills the gaps (6.20 -> 5.59 ms per 48^3 chunk)
        __builtin_amdgcn_s_setprio(1);
        const int64_t k1 = static_cast<int64_t>(st + 1) * kKt;
        double2 rd[NLOAD];
#pragma unroll
        for (int u = 0; u < NLOAD; ++u) {
            const int64_t k = k1 + kk0 + KSTEP * u;
            const int64_t kr = k < kc ? k : kc - 1;
            rd[u] = dw[kr];
            rb[u] = m[kr * ng + cj];
            // component loads: a whole-struct copy into LDS would be fused
            // into one global-to-LDS copy placed after the MFMAs, exposing
            // the load latency at every stage
            ra[u].x = m[kr * ng + ci].x;
            ra[u].y = m[kr * ng + ci].y;
        }
        // loads first, then the MFMAs of the current stage (no reordering)
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_setprio(2);
#pragma unroll
        for (int s = 0; s < kKt / 4; ++s) {
            const double2* la = s_a + (buf * kKt + s * 4 + kq) * LDR + wi * (T / WI) + row;
            const double2* lb = s_b + (buf * kKt + s * 4 + kq) * LDR + wj * (T / WJ) + row;
            double2 a[BX], b[BY];
#pragma unroll
            for (int x = 0; x < BX; ++x) a[x] = la[x * 16];
#pragma unroll
            for (int y = 0; y < BY; ++y) b[y] = lb[y * 16];
            if constexpr (K3) {
                double as[BX], bs[BY];
#pragma unroll
                for (int x = 0; x < BX; ++x) as[x] = a[x].x - a[x].y;
#pragma unroll
                for (int y = 0; y < BY; ++y) bs[y] = b[y].x + b[y].y;
#pragma unroll
                for (int x = 0; x < BX; ++x)
#pragma unroll
                    for (int y = 0; y < BY; ++y) {
                        p1[x][y] = mfma_f64(a[x].x, b[y].x, p1[x][y]);
                        p2[x][y] = mfma_f64(a[x].y, b[y].y, p2[x][y]);
                        p3[x][y] = mfma_f64(as[x], bs[y], p3[x][y]);
                    }
            } else {
#pragma unroll
                for (int x = 0; x < BX; ++x)
#pragma unroll
                    for (int y = 0; y < BY; ++y)
                        cmfma_conj_a(p1[x][y], p2[x][y], a[x].x, a[x].y, b[y].x, b[y].y);
            }
        }
        // keep the LDS stores of the next stage after this stage's MFMAs, so
        // the global loads issued above stay in flight during the compute
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_setprio(0);
        const int nb2 = buf ^ 1;
#pragma unroll
        for (int u = 0; u < NLOAD; ++u) {
            const int64_t k = k1 + kk0 + KSTEP * u;
            s_a[(nb2 * kKt + kk0 + KSTEP * u) * LDR + cc] = make_double2(ra[u].x, ra[u].y);
            s_b[(nb2 * kKt + kk0 + KSTEP * u) * LDR + cc] =
                k < kc ? cmul(rd[u], rb[u]) : make_double2(0.0, 0.0);
        }
        __syncthreads();
        buf = nb2;
    }
#pragma unroll
    for (int x = 0; x < BX; ++x)
#pragma unroll
        for (int y = 0; y < BY; ++y)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int li = wi * (T / WI) + x * 16 + 4 * t + kq;
                const int lj = wj * (T / WJ) + y * 16 + row;
                const double re = K3 ? p1[x][y][t] + p2[x][y][t] : p1[x][y][t];
                const double im = K3 ? p3[x][y][t] - p1[x][y][t] + p2[x][y][t] : p2[x][y][t];
                if constexpr (PART) {
                    cw[li * T + lj] = make_double2(re, im);
                    continue;
                }
                const int gi = i0 + li, gj = j0 + lj;
                if (gi < ng && gj < ng) {
                    double2* p = cw + static_cast<int64_t>(gi) * ng + gj;
                    double2 v = make_double2(re, im);
                    if (mode) {
                        const double2 o = *p;
                        v.x += o.x;
                        v.y += o.y;
                    }
                    *p = v;
                }
            }
}


// The first n_main items, one per workgroup, over all pairs of the chunk.
// Each of the remaining items (the last, partial round of workgroups) is cut
// into `parts` ranges of whole stages; workgroup n_main + j*parts + p writes
// item n_main + j's partial sum over range p to ws[j*parts + p] (T x T), and
// tail_reduce_kernel adds the parts into chi.
template <int T, int WI, int WJ, int PAD>
__global__ __launch_bounds__(WI * WJ * 64) void chi0_f64_kernel(
    const double2* __restrict__ m, int64_t kc, int ng, const double2* __restrict__ delta,
    WList wl, double2* __restrict__ chi, int mode, int nb, const int* __restrict__ order,
    int n_main, int parts, double2* __restrict__ ws) {
    extern __shared__ double2 lds[];
    const int b = blockIdx.x;
    int w, bi, bj;
    if (b < n_main) {
        item_tile(xcd_item(b, n_main), wl, nb, order, w, bi, bj);
        f64_tile<T, WI, WJ, PAD>(lds, m, kc, ng, delta + static_cast<int64_t>(w) * kc,
                                 chi + static_cast<int64_t>(w) * ng * ng, mode, bi, bj);
        return;
    }
    const int u = b - n_main, j = u / parts, p = u % parts;
    item_tile(n_main + j, wl, nb, order, w, bi, bj);
    const int64_t nst = (kc + kKt - 1) / kKt;
    const int64_t k0 = p * nst / parts * kKt;
    const int64_t k1 = std::min<int64_t>(kc, (p + 1) * nst / parts * kKt);
    f64_tile<T, WI, WJ, PAD, true>(lds, m + k0 * ng, k1 - k0, ng,
                                   delta + static_cast<int64_t>(w) * kc + k0,
                                   ws + static_cast<int64_t>(u) * T * T, 0, bi, bj);
}

// chi_w[tile] (=|+=) the sum of the parts of tail item n_main + blockIdx.y,
// added in part order.
template <int T>
__global__ __launch_bounds__(256) void tail_reduce_kernel(const double2* __restrict__ ws,
                                                          int parts, int n_main, WList wl, int nb,
                                                          const int* __restrict__ order,
                                                          double2* __restrict__ chi, int ng,
                                                          int mode) {
    const int j = blockIdx.y, e = blockIdx.x * 256 + threadIdx.x;
    int w, bi, bj;
    item_tile(n_main + j, wl, nb, order, w, bi, bj);
    const int gi = bi * T + e / T, gj = bj * T + e % T;
    if (gi >= ng || gj >= ng) return;
    const double2* src = ws + static_cast<int64_t>(j) * parts * T * T + e;
    double2 acc = src[0];
    for (int p = 1; p < parts; ++p) {
        const double2 v = src[static_cast<int64_t>(p) * T * T];
        acc.x += v.x;
        acc.y += v.y;
    }
    double2* dst = chi + static_cast<int64_t>(w) * ng * ng + static_cast<int64_t>(gi) * ng + gj;
    if (mode) {
        const double2 o = *dst;
        acc.x += o.x;
        acc.y += o.y;
    }
    *dst = acc;
}

// Persistent form for batches of problems: every workgroup takes items
// (problem, frequency, tile) from an atomic counter until the list is
// exhausted, so problems of very different N_G share one launch without a
// tail per problem.  Items are sorted by decreasing cost on the host.
template <int T, int WI, int WJ, int PAD>
__global__ __launch_bounds__(WI * WJ * 64) void chi0_f64_batched_kernel(
    const QDesc* __restrict__ qd, const int4* __restrict__ items, int nitems,
    int* __restrict__ counter) {
    extern __shared__ double2 lds[];
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if (it >= nitems) break;
        const int4 itm = items[it];
        const QDesc d = qd[itm.x];
        f64_tile<T, WI, WJ, PAD>(lds, d.m, d.kc, d.ng, d.delta + static_cast<int64_t>(itm.y) * d.kc,
                                 d.chi + static_cast<int64_t>(itm.y) * d.ng * d.ng, d.mode, itm.z,
                                 itm.w);
    }
}

struct Chi0Variant {
    const void* fn;       // per-launch kernel
    const void* fn_batch; // persistent batched kernel
    const void* fn_tail;  // tail_reduce_kernel<T>
    int tile, threads;
    size_t lds;
};

template <int T, int WI, int WJ, int PAD>
Chi0Variant chi0_variant() {
    return {reinterpret_cast<const void*>(&chi0_f64_kernel<T, WI, WJ, PAD>),
            reinterpret_cast<const void*>(&chi0_f64_batched_kernel<T, WI, WJ, PAD>),
            reinterpret_cast<const void*>(&tail_reduce_kernel<T>), T, WI * WJ * 64,
            2 * 2 * kKt * (T + PAD) * sizeof(double2)};
}

// Tile shapes of the FP64 contraction, indexed by variant id (the autotuner
// chooses among them; GW_CHI0_VARIANT forces one).
const Chi0Variant& chi0_variant_by_id(int id) {
    static const Chi0Variant v[2] = {chi0_variant<64, 2, 2, 0>(), chi0_variant<128, 2, 4, 0>()};
    return v[id == 1 ? 1 : 0];
}

// chi[i][j] = conj(chi[j][i]) for every (i, j) in a tile strictly below the
// diagonal of tile x tile blocks (those the Hermitian contraction skipped).
__global__ __launch_bounds__(256) void mirror_kernel(double2* __restrict__ chi, int ng, int tile) {
    const int j = blockIdx.x * 16 + (threadIdx.x & 15);
    const int i = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (i >= ng || j >= ng) return;
    if (i / tile <= j / tile) return;
    const double2 u = chi[static_cast<int64_t>(j) * ng + i];
    chi[static_cast<int64_t>(i) * ng + j] = make_double2(u.x, -u.y);
}

__global__ __launch_bounds__(256) void fill_zero_kernel(double2* __restrict__ p, int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = make_double2(0.0, 0.0);
}

}  // namespace

void launch_delta(const double* e_v, const double* e_c, PairMap pm, int64_t npairs,
                  const double2* z, int nz, double spin, double2* delta, hipStream_t s) {
    if (npairs <= 0) return;
    for (int w0 = 0; w0 < nz; w0 += kMaxZ) {
        ZArgs za{};
        za.nz = std::min(kMaxZ, nz - w0);
        za.spin = spin;
        for (int w = 0; w < za.nz; ++w) {
            za.re[w] = z[w0 + w].x;
            za.im[w] = z[w0 + w].y;
        }
        ProfScope ps("delta", s);
        hipLaunchKernelGGL(delta_kernel, dim3(static_cast<unsigned>(ceil_div64(npairs, 256))),
                           dim3(256), 0, s, e_v, e_c, pm, npairs, za, w0, delta);
        GW_HIP_TRY(hipGetLastError());
    }
}

namespace {
// Workgroups of variant v resident on the current device at once.
int f64_slots(int variant) {
    static std::mutex mu;
    static std::map<std::pair<int, int>, int> cache;  // (device, variant) -> slots
    int dev = 0;
    GW_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    int& n = cache[{dev, variant}];
    if (n > 0) return n;
    const Chi0Variant& v = chi0_variant_by_id(variant);
    GW_HIP_TRY(hipFuncSetAttribute(v.fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   static_cast<int>(v.lds)));
    int per_cu = 0, cus = 0;
    GW_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, v.fn, v.threads, v.lds));
    GW_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    n = std::max(1, per_cu) * std::max(1, cus);
    return n;
}
}  // namespace

size_t chi0_f64_tail_bytes() {
    size_t b = 0;
    for (int v = 0; v < kNumChi0Variants; ++v) {
        const size_t t = static_cast<size_t>(chi0_variant_by_id(v).tile);
        b = std::max(b, static_cast<size_t>(f64_slots(v)) * t * t * sizeof(double2));
    }
    return b;
}

void launch_chi0_f64(const double2* m, int64_t kc, int ng, const double2* delta,
                     const WList& wl, double2* chi, bool accumulate, hipStream_t s, int variant,
                     double2* tail_ws) {
    if (kc <= 0 || wl.nh + wl.nf == 0) return;
    const Chi0Variant& v = chi0_variant_by_id(variant);
    const int nb = ceil_div(ng, v.tile);
    const int64_t nitems = static_cast<int64_t>(wl.nh) * (nb * (nb + 1) / 2) +
                           static_cast<int64_t>(wl.nf) * nb * nb;
    if (nitems >= (int64_t(1) << 30)) throw Error{-4, "too many chi tiles for one launch"};
    GW_HIP_TRY(hipFuncSetAttribute(v.fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   static_cast<int>(v.lds)));
    // A last round of workgroups that fills at most half the chip is cut
    // along the pairs: each of its items becomes `parts` workgroups over
    // ranges of stages, which together fill the round.
    int n_main = static_cast<int>(nitems), parts = 1, n_tail = 0;
    if (tail_ws) {
        const int slots = f64_slots(variant);
        const int rem = static_cast<int>(nitems % slots);
        const int64_t nst = (kc + kKt - 1) / kKt;
        const int pc = static_cast<int>(std::min<int64_t>(rem > 0 ? slots / rem : 0, nst));
        if (rem > 0 && 2 * rem <= slots && pc >= 2) {
            n_tail = rem;
            parts = pc;
            n_main = static_cast<int>(nitems) - rem;
        }
    }
    int mode = accumulate ? 1 : 0;
    const int* order = tile_order(nb);
    {
        ProfScope ps("chi0_f64", s);
        void* args[] = {const_cast<double2**>(&m), &kc, &ng, const_cast<double2**>(&delta),
                        const_cast<WList*>(&wl), &chi, &mode, const_cast<int*>(&nb),
                        const_cast<int**>(&order), &n_main, &parts, &tail_ws};
        const unsigned grid = static_cast<unsigned>(n_main + n_tail * parts);
        GW_HIP_TRY(hipLaunchKernel(v.fn, dim3(grid), dim3(v.threads), args, v.lds, s));
    }
    if (n_tail > 0) {
        ProfScope ps("chi0_tail", s);
        void* args[] = {&tail_ws, &parts, &n_main, const_cast<WList*>(&wl),
                        const_cast<int*>(&nb), const_cast<int**>(&order), &chi, &ng, &mode};
        const unsigned gx = static_cast<unsigned>(v.tile * v.tile / 256);
        GW_HIP_TRY(hipLaunchKernel(v.fn_tail, dim3(gx, static_cast<unsigned>(n_tail)), dim3(256),
                                   args, 0, s));
    }
}

void launch_chi0_f64_batched(const QDesc* qd, const int4* items, int nitems, int* counter,
                             hipStream_t s, int variant, int grid) {
    if (nitems <= 0) return;
    const Chi0Variant& v = chi0_variant_by_id(variant);
    GW_HIP_TRY(hipFuncSetAttribute(v.fn_batch, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   static_cast<int>(v.lds)));
    ProfScope ps("chi0_f64_batched", s);
    void* args[] = {const_cast<QDesc**>(&qd), const_cast<int4**>(&items), &nitems, &counter};
    GW_HIP_TRY(hipLaunchKernel(v.fn_batch, dim3(static_cast<unsigned>(std::min(grid, nitems))),
                               dim3(v.threads), args, v.lds, s));
}

int chi0_variant_tile(int variant) { return chi0_variant_by_id(variant).tile; }

int chi0_f64_batched_blocks_per_cu(int variant) {
    const Chi0Variant& v = chi0_variant_by_id(variant);
    GW_HIP_TRY(hipFuncSetAttribute(v.fn_batch, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   static_cast<int>(v.lds)));
    int n = 0;
    GW_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, v.fn_batch, v.threads, v.lds));
    return std::max(1, n);
}

int chi0_forced_variant() {
    static const int id = [] {
        const char* e = std::getenv("GW_CHI0_VARIANT");
        return e ? std::atoi(e) : -1;
    }();
    return id;
}

void launch_mirror(double2* chi, int ng, int tile, hipStream_t s) {
    ProfScope ps("mirror", s);
    hipLaunchKernelGGL(mirror_kernel, dim3(ceil_div(ng, 16), ceil_div(ng, 16)), dim3(256), 0, s,
                       chi, ng, tile);
    GW_HIP_TRY(hipGetLastError());
}

void launch_fill_zero(double2* p, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    const int64_t blocks = std::min<int64_t>(ceil_div64(n, 256), 65536);
    hipLaunchKernelGGL(fill_zero_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, p, n);
    GW_HIP_TRY(hipGetLastError());
}



namespace {
struct OrderCache {
    std::mutex mu;
    std::map<std::tuple<int, int, int>, int*> tables;  // (device, nb, super) -> device table
};
OrderCache& order_cache() {
    static OrderCache* c = new OrderCache();
    return *c;
}
}  // namespace

const int* tile_order(int nb, int kSuper) {
    int dev = 0;
    GW_HIP_TRY(hipGetDevice(&dev));
    OrderCache& oc = order_cache();
    std::lock_guard<std::mutex> lk(oc.mu);
    int*& t = oc.tables[{dev, nb, kSuper}];
    if (t) return t;
    std::vector<int> h, f;
    for (int si = 0; si < nb; si += kSuper)
        for (int sj = 0; sj < nb; sj += kSuper)
            for (int i = si; i < std::min(nb, si + kSuper); ++i)
                for (int j = sj; j < std::min(nb, sj + kSuper); ++j) {
                    f.push_back((i << 16) | j);
                    if (j >= i) h.push_back((i << 16) | j);
                }
    h.insert(h.end(), f.begin(), f.end());
    require_alloc("tile-order table for this G-list size");
    GW_HIP_TRY(hipMalloc(&t, h.size() * sizeof(int)));
    GW_HIP_TRY(hipMemcpy(t, h.data(), h.size() * sizeof(int), hipMemcpyHostToDevice));
    return t;
}

void release_tile_orders() {
    OrderCache& oc = order_cache();
    std::lock_guard<std::mutex> lk(oc.mu);
    for (auto& kv : oc.tables) {
        (void)hipSetDevice(std::get<0>(kv.first));
        (void)hipDeviceSynchronize();
        (void)hipFree(kv.second);
    }
    oc.tables.clear();
}



}  // namespace gw
