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

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kLoadBatch = 8;  // x-stage k-steps whose loads are issued together
constexpr int kZyWaves = 8;
constexpr int kZyThreads = 64 * kZyWaves;
constexpr int kSlab = 16;  // j3 values per LDS slab (4 MFMA k-steps)

// The value this lane's partner in its 16-lane row (lane ^ 8) holds: a DPP
// row rotation by 8, two 32-bit moves.
__device__ __forceinline__ double row_swap8(double v) {
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b & 0xffffffffull), 0x128, 0xf,
                                               0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), 0x128, 0xf, 0xf, false);
    return __longlong_as_double(static_cast<long long>(
        (static_cast<unsigned long long>(static_cast<unsigned>(hi)) << 32) |
        static_cast<unsigned>(lo)));
}

// The slab ring is written by global_load_lds and read with ds_read, and the
// kernel orders the two itself (vmcnt waits and a barrier per slab).  Both go
// through these helpers' restrict pointers: the alias scopes that inlining
// attaches let the compiler see that a read is not waiting on the loads in
// flight, which it would otherwise drain before every read (with them, the
// ring - 1 slabs in flight keep flying).
template <int NFILL>
__device__ __forceinline__ void ring_fill(double2* __restrict__ ring, int off,
                                          const double2* const (&src)[NFILL]) {
#pragma unroll
    for (int u = 0; u < NFILL; ++u)
        __builtin_amdgcn_global_load_lds(reinterpret_cast<const u32x4*>(src[u]),
                                         reinterpret_cast<u32x4*>(ring + off + u * kZyThreads), 16,
                                         0, 0);
}
__device__ __forceinline__ double2 ring_read(const double2* __restrict__ ring, int off) {
    return ring[off];
}

// vmcnt(n) alone (expcnt and lgkmcnt left at their no-wait maxima).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// One workgroup = a tile of 4 valence x (2*PPW) conduction bands (4*2*PPW
// pairs); wave w owns valence band w/2 and PPW conduction bands.  The planes
// of the workgroup are walked as (j1 plane, 16-row block of j2, 16-wide slab
// of j3); each slab of the tile's band rows is written straight from global
// memory into a ring of `ring` LDS slots (no registers), ring - 1 slabs ahead
// of the one contracted, and shared by all the pairs that use it.  Slab entry
// (band b, row r, position q) holds column q ^ r, so the 16 rows of one
// column sit in 16 distinct bank groups.  Entries past the grid or the tile
// load a clamped in-range value: its products meet zero twiddles, skipped
// k-steps or pairs that are not written.
// Both stages run on real twiddles, two real MFMA products per 16 x 16 block
// (the real and the imaginary part of the complex operand):
//  * stage z: B = the cos | sin columns of 8 k3 classes (NB3 blocks); before
//    stage y each lane swaps with its partner column (c ^ 8) to form T1 at
//    k3 = +a (columns c < 8) and k3 = -a (columns c >= 8);
//  * stage y: A = the cos | sin rows of 8 k2 classes (NB2 blocks).  Output
//    row 4 t + kq sits in element t, so a class's cos row (t = 0, 1) and sin
//    row (t = 2, 3) share a lane and T2 at k2 = +-a is formed in place.
// k-steps of j3 or j2 beyond the grid (the padding to 16) are skipped.
// A launch takes the k2 class blocks [b2_0, b2_0 + NB2) of the plan's NB2T:
// where all NB2T blocks of stage-y accumulators would not fit the registers
// of a wave, two launches split them (each runs stage z again on the same
// slabs and writes its own classes of T2).
template <int NB2, int NB3, int PPW, int NB2T>
__global__ __launch_bounds__(kZyThreads) void mtxel_zy_kernel(
    const double2* __restrict__ psi_v, const double2* __restrict__ psi_c, int64_t nr, Rect rc,
    int n1, int planes_per_group, int n2, int n3, int n2p, int n3p,
    const double* __restrict__ w3re, const double* __restrict__ w2re,
    const int* __restrict__ boxf, int n23, double2* __restrict__ t2, int ring, int b2_first) {
    static_assert(NB2 <= NB2T, "class blocks of one launch");
    const int b2_0 = NB2 == NB2T ? 0 : b2_first;  // a constant where one launch takes all
    constexpr int TV = 4, TC = 2 * PPW, NBANDS = TV + TC;
    constexpr int NSLAB = NBANDS * 256;             // 16-byte entries per slab
    constexpr int NFILL = NSLAB / kZyThreads;       // loads per thread per slab
    static_assert(NSLAB % kZyThreads == 0, "slab fill");
    extern __shared__ double2 lds[];
    const int nslab = n3p / kSlab;
    const int q = n3p >> 2;
    const int nrb1 = n2p >> 4;
    const int w3n = q * NB3 * 64;          // doubles (multiples of 64: whole double2 slots)
    const int w2n = nrb1 * 4 * NB2T * 64;
    constexpr int boxn = NB2T * 16 * NB3 * 16;
    double* s_w3 = reinterpret_cast<double*>(lds);
    double* s_w2 = reinterpret_cast<double*>(lds + w3n / 2);
    int* s_box = reinterpret_cast<int*>(lds + w3n / 2 + w2n / 2);
    double2* s_ring = lds + w3n / 2 + w2n / 2 + boxn / 4;  // [ring][NBANDS][16][16]
    for (int i = threadIdx.x; i < w3n; i += kZyThreads) s_w3[i] = w3re[i];
    for (int i = threadIdx.x; i < w2n; i += kZyThreads) s_w2[i] = w2re[i];
    for (int i = threadIdx.x; i < boxn; i += kZyThreads) s_box[i] = boxf[i];

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63, row = lane & 15, kq = lane >> 4;
    const bool cos_col = row < 8;  // this lane's stage-z column: cosine (else sine) of its class
    const int tv0 = blockIdx.y * TV, tc0 = blockIdx.x * TC;

    // staging entries of this thread: e = u * 512 + tid -> band e / 256, row
    // fr[u], column fc[u] (position e % 16 = fc ^ fr); band rows clamped
    const double2* fptr[NFILL];
    int fr[NFILL], fc[NFILL];
#pragma unroll
    for (int u = 0; u < NFILL; ++u) {
        const int e = tid + kZyThreads * u;
        const int fb = e >> 8;
        fr[u] = (e >> 4) & 15;
        fc[u] = (e & 15) ^ fr[u];
        if (fb < TV)
            fptr[u] = psi_v + static_cast<int64_t>(rc.v0 + min(tv0 + fb, rc.nv - 1)) * nr;
        else
            fptr[u] = psi_c + static_cast<int64_t>(rc.c0 + min(tc0 + fb - TV, rc.nc - 1)) * nr;
    }
    auto issue = [&](int j1, int rb1, int sl, int slot) {
        const double2* src[NFILL];
#pragma unroll
        for (int u = 0; u < NFILL; ++u) {
            const int j2 = min(rb1 * 16 + fr[u], n2 - 1), j3 = min(sl * kSlab + fc[u], n3 - 1);
            src[u] = fptr[u] + (static_cast<int64_t>(j1) * n2 + j2) * n3 + j3;
        }
        ring_fill<NFILL>(s_ring, slot * NSLAB + wave * 64, src);
    };
    // slab entry of (band, row, column)
    auto sent = [&](int band, int r, int c) { return band * 256 + r * 16 + (c ^ r); };

    const int vl = wave >> 1, cl0 = (wave & 1) * PPW;
    bool pok[PPW];
#pragma unroll
    for (int p = 0; p < PPW; ++p) pok[p] = tv0 + vl < rc.nv && tc0 + cl0 + p < rc.nc;

    // accumulators (Re, Im): stage z per class block of k3, stage y per class
    // blocks of k2 and k3
    dbl4 a1r[PPW][NB3], a1i[PPW][NB3];
    dbl4 a2r[PPW][NB2][NB3], a2i[PPW][NB2][NB3];
#pragma unroll
    for (int p = 0; p < PPW; ++p)
#pragma unroll
        for (int b3 = 0; b3 < NB3; ++b3) {
            a1r[p][b3] = a1i[p][b3] = zero4();
#pragma unroll
            for (int b2 = 0; b2 < NB2; ++b2) a2r[p][b2][b3] = a2i[p][b2][b3] = zero4();
        }

    // this workgroup's planes: j1 in [j1b, j1e)
    const int j1b = blockIdx.z * planes_per_group;
    const int j1e = min(n1, j1b + planes_per_group);
    const int total = (j1e - j1b) * nrb1 * nslab;
    int j1 = j1b, rb1 = 0, sl = 0;      // position being contracted
    int nj1 = j1b, nrb = 0, nsl = 0;    // next position to load (clamped at the last slab)
    auto advance = [&](int& a, int& b, int& c) {
        if (++c == nslab) {
            c = 0;
            if (++b == nrb1) {
                b = 0;
                if (++a == j1e) {
                    a = j1e - 1;
                    b = nrb1 - 1;
                    c = nslab - 1;
                }
            }
        }
    };
    __syncthreads();  // tables visible
    for (int i = 0; i < ring - 1; ++i) {
        issue(nj1, nrb, nsl, i);
        advance(nj1, nrb, nsl);
    }
    // T2 of plane pj1: a2[p][b2][b3] elements t = 0, 1 of lane l are the cos
    // sums of k2 class 8*b2 + 4*t + kq, elements t + 2 the sin sums, at
    // stage-y column b3*16 + row.  T2 at k2 = +a is C + i S, at -a C - i S;
    // s_box[(class slot * 2 + sign) * NB3*16 + column] is its disc index.
    auto store_plane = [&](int pj1) {
#pragma unroll
        for (int p = 0; p < PPW; ++p) {
            if (pok[p]) {
                const int64_t k = static_cast<int64_t>(tv0 + vl) * rc.nc + tc0 + cl0 + p;
                double2* o = t2 + (k * n1 + pj1) * n23;
#pragma unroll
                for (int b2 = 0; b2 < NB2; ++b2)
#pragma unroll
                    for (int b3 = 0; b3 < NB3; ++b3)
#pragma unroll
                        for (int t = 0; t < 2; ++t) {
                            const double cr = a2r[p][b2][b3][t], ci = a2i[p][b2][b3][t];
                            const double sr = a2r[p][b2][b3][t + 2], si = a2i[p][b2][b3][t + 2];
                            const int e =
                                (((b2_0 + b2) * 8 + 4 * t + kq) * 2) * (NB3 * 16) + b3 * 16 + row;
                            const int dp = s_box[e], dm = s_box[e + NB3 * 16];
                            if (dp >= 0) o[dp] = make_double2(cr - si, ci + sr);
                            if (dm >= 0) o[dm] = make_double2(cr + si, ci - sr);
                        }
            }
#pragma unroll
            for (int b2 = 0; b2 < NB2; ++b2)
#pragma unroll
                for (int b3 = 0; b3 < NB3; ++b3) a2r[p][b2][b3] = a2i[p][b2][b3] = zero4();
        }
    };
    constexpr bool kPack = PPW % 2 == 0;
    const bool half_last = (n2 & 15) != 0 && (n2 & 15) <= 8;  // last j2 block at most 8 rows
    int pending = -1;  // plane whose T2 is complete and not yet stored
    int cur = 0, fill = ring - 1;  // ring slots: contracted, refilled next
    for (int it = 0; it < total; ++it) {
        // this slab has landed in every wave, and every wave is done with the
        // slot the next load refills.  At most the ring - 2 later slabs' loads
        // of this wave are outstanding: loads complete in order among
        // themselves, so while any load of this slab is in flight so are all
        // NFILL of each later slab, whatever the t2 stores in between do
        if (ring == 3)
            wait_vmcnt<NFILL>();
        else
            wait_vmcnt<0>();
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");  // keep the LDS reads below the barrier
        if (pending >= 0) {  // a slab before the next y stage: a2 is free again in time
            store_plane(pending);
            pending = -1;
        }
        issue(nj1, nrb, nsl, fill);
        advance(nj1, nrb, nsl);
        const int slab = cur * NSLAB;
        // The last 16-row block of j2 may hold at most 8 rows of the grid: then,
        // with an even number of pairs per wave, pairs 2q and 2q + 1 share one
        // row set of the MFMAs (rows r < 8: pair 2q at j2 = rb1*16 + r; rows
        // r >= 8: pair 2q + 1 at j2 = rb1*16 + r - 8) in accumulator set q.
        const bool packed = kPack && rb1 == nrb1 - 1 && half_last;
        // z stage on this slab: A = rho rows (j2 = rb1*16+row, j3 = 16*sl + 4*kk + kq;
        // packed: pair 2p + row/8 at j2 = rb1*16 + row%8 into set p)
        {
            const int zrow = packed ? (row & 7) : row;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int ks = sl * 4 + kk;
                if (4 * ks >= n3) break;  // padding k-steps (uniform)
                const double2 xv = ring_read(s_ring, slab + sent(vl, zrow, 4 * kk + kq));
                double w3[NB3];
#pragma unroll
                for (int b3 = 0; b3 < NB3; ++b3) w3[b3] = s_w3[(ks * 64 + lane) * NB3 + b3];
#pragma unroll
                for (int p = 0; p < PPW; ++p) {
                    if (packed && 2 * p >= PPW) break;  // uniform
                    const int band = packed ? TV + cl0 + 2 * p + (row >> 3) : TV + cl0 + p;
                    const double2 xc = ring_read(s_ring, slab + sent(band, zrow, 4 * kk + kq));
                    const double2 rho = cmul_conj_a(xv, xc);
#pragma unroll
                    for (int b3 = 0; b3 < NB3; ++b3) {
                        a1r[p][b3] = mfma_f64(rho.x, w3[b3], a1r[p][b3]);
                        a1i[p][b3] = mfma_f64(rho.y, w3[b3], a1i[p][b3]);
                    }
                }
            }
        }
        if (sl == nslab - 1) {
            // y stage, k-step t of the block's rows (k index kq): a1[p][b3]
            // element t of lane l is the cos (row < 8) or sin sum of k3 class
            // 8*b3 + (row & 7) at j2 = rb1*16 + 4*t + kq (packed: pair p's sums
            // are set p/2, elements 2 (p % 2) + t, t < 2); with the partner
            // lane's sum, T1 at k3 = +a (cos lanes) is C + i S and at -a (sin
            // lanes) C - i S, the B operand column b3*16 + row
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if ((packed && t >= 2) || rb1 * 16 + 4 * t >= n2) break;  // uniform
                double tre[PPW][NB3], tim[PPW][NB3];
#pragma unroll
                for (int p = 0; p < PPW; ++p)
#pragma unroll
                    for (int b3 = 0; b3 < NB3; ++b3) {
                        const int ps = kPack ? p / 2 : p, es = 2 * (p & 1) + (t & 1);
                        const double r = packed ? a1r[ps][b3][es] : a1r[p][b3][t];
                        const double i = packed ? a1i[ps][b3][es] : a1i[p][b3][t];
                        const double rp = row_swap8(r), ip = row_swap8(i);
                        tre[p][b3] = cos_col ? r - ip : rp + i;
                        tim[p][b3] = cos_col ? i + rp : ip - r;
                    }
#pragma unroll
                for (int b2 = 0; b2 < NB2; ++b2) {
                    const double w = s_w2[((rb1 * 4 + t) * 64 + lane) * NB2T + b2_0 + b2];
#pragma unroll
                    for (int p = 0; p < PPW; ++p)
#pragma unroll
                        for (int b3 = 0; b3 < NB3; ++b3) {
                            a2r[p][b2][b3] = mfma_f64(w, tre[p][b3], a2r[p][b2][b3]);
                            a2i[p][b2][b3] = mfma_f64(w, tim[p][b3], a2i[p][b2][b3]);
                        }
                }
            }
#pragma unroll
            for (int p = 0; p < PPW; ++p)
#pragma unroll
                for (int b3 = 0; b3 < NB3; ++b3) a1r[p][b3] = a1i[p][b3] = zero4();
            if (rb1 == nrb1 - 1) pending = j1;  // stored after the next barrier
        }
        if (++sl == nslab) {
            sl = 0;
            if (++rb1 == nrb1) {
                rb1 = 0;
                ++j1;
            }
        }
        cur = cur + 1 == ring ? 0 : cur + 1;
        fill = fill + 1 == ring ? 0 : fill + 1;
    }
    if (pending >= 0) store_plane(pending);
    wait_vmcnt<0>();  // no load into this workgroup's LDS may outlive it
}

// ---------------------------------------------------------------- kernel 2

// M_box[k1][d] = sum_j1 W1[k1][j1] T2[j1][d] on MFMA: A = the real cos | sin
// rows of 8 k1 classes per block (LDS, lane order), B = the real and the
// imaginary part of T2 rows (coalesced): two real products per block.  Output
// row 4 t + kq is element t, so a class's cos sum (t = 0, 1) and sin sum
// (t = 2, 3) share a lane: M at k1 = +a is C + i S and at -a C - i S,
// scattered to the G list.
// Pair k of the launch (k0 + blockIdx.x in the rectangle's row-major order,
// cw pairs per valence row) is written to output row (k / cw) * ldm + k % cw.
template <int NB1>
__global__ __launch_bounds__(kThreads) void mtxel_x_kernel(
    const double2* __restrict__ t2, int n1, int n1p, int n23, int n23p,
    const double* __restrict__ w1re, const int* __restrict__ gmapf, int ng, double dv,
    int64_t npairs, int64_t k0, int cw, int64_t ldm, double2* __restrict__ m_out) {
    extern __shared__ double2 lds_x[];
    double* s_w1 = reinterpret_cast<double*>(lds_x);
    const int q1 = n1p >> 2;
    for (int i = threadIdx.x; i < NB1 * q1 * 64; i += kThreads) s_w1[i] = w1re[i];
    __syncthreads();
    const int64_t k = blockIdx.x;
    if (k >= npairs) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, row = lane & 15, kq = lane >> 4;
    const double2* src = t2 + k * static_cast<int64_t>(n1) * n23;
    const int64_t kg = k0 + k;
    double2* dst = m_out + ((kg / cw) * ldm + kg % cw) * static_cast<int64_t>(ng);
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
                        const double w = s_w1[(ks * 64 + lane) * NB1 + b];
                        ar[b] = mfma_f64(w, xb[u].x, ar[b]);
                        ai[b] = mfma_f64(w, xb[u].y, ai[b]);
                    }
                }
            }
        }
#pragma unroll
        for (int b = 0; b < NB1; ++b)
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const double cr = ar[b][t], ci = ai[b][t], sr = ar[b][t + 2], si = ai[b][t + 2];
                const int e = ((b * 8 + 4 * t + kq) * 2) * n23p + d;
                const int gp = gmapf[e], gm = gmapf[e + n23p];
                if (gp >= 0) dst[gp] = make_double2(dv * (cr - si), dv * (ci + sr));
                if (gm >= 0) dst[gm] = make_double2(dv * (cr + si), dv * (ci - sr));
            }
    }
}

using ZyKernel = void (*)(const double2*, const double2*, int64_t, Rect, int, int, int, int, int,
                          int, const double*, const double*, const int*, int, double2*, int, int);

// Pairs per wave by the wider class-block count, within the registers of two
// waves per SIMD.
constexpr int zy_ppw(int nb2, int nb3) {
    return (nb2 > nb3 ? nb2 : nb3) == 1 ? 4 : ((nb2 > nb3 ? nb2 : nb3) == 2 ? 2 : 1);
}

// The launches of stage z and y for a box of NB2 x NB3 class blocks: one, or
// where the stage-y accumulators of all NB2 blocks would spill (more than
// three blocks on one axis and three on the other), two over halves of the k2
// blocks.
struct ZyLaunches {
    ZyKernel k[2];
    int b2_0[2];
    int count;
};

template <int NB2, int NB3>
ZyLaunches zy_launches() {
    if constexpr (NB2 * NB3 > 9) {
        constexpr int H = (NB2 + 1) / 2;
        return {{&mtxel_zy_kernel<H, NB3, zy_ppw(H, NB3), NB2>,
                 &mtxel_zy_kernel<NB2 - H, NB3, zy_ppw(NB2 - H, NB3), NB2>},
                {0, H}, 2};
    } else {
        return {{&mtxel_zy_kernel<NB2, NB3, zy_ppw(NB2, NB3), NB2>, nullptr}, {0, 0}, 1};
    }
}

// Pairs per wave of the launches of a box (the same for both halves).
int zy_pairs_per_wave(int nb2, int nb3) {
    return nb2 * nb3 > 9 ? zy_ppw((nb2 + 1) / 2, nb3) : zy_ppw(nb2, nb3);
}

const ZyLaunches& select_zy(int nb2, int nb3) {
    static const ZyLaunches table[4][4] = {
        {zy_launches<1, 1>(), zy_launches<1, 2>(), zy_launches<1, 3>(), zy_launches<1, 4>()},
        {zy_launches<2, 1>(), zy_launches<2, 2>(), zy_launches<2, 3>(), zy_launches<2, 4>()},
        {zy_launches<3, 1>(), zy_launches<3, 2>(), zy_launches<3, 3>(), zy_launches<3, 4>()},
        {zy_launches<4, 1>(), zy_launches<4, 2>(), zy_launches<4, 3>(), zy_launches<4, 4>()},
    };
    return table[nb2 - 1][nb3 - 1];
}

using XKernel = void (*)(const double2*, int, int, int, int, const double*, const int*, int,
                         double, int64_t, int64_t, int, int64_t, double2*);

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
    // frequency classes a = min(k, N - k) along y and z: the forward stages
    // work on these
    auto classes = [](const std::vector<int>& l, int nn) {
        std::set<int> sh;
        for (int k : l) sh.insert(std::min(k, nn - k));
        return std::vector<int>(sh.begin(), sh.end());
    };
    const std::vector<int> lh1 = classes(l1, n[0]), lh2 = classes(l2, n[1]),
                           lh3 = classes(l3, n[2]);
    p->mh1 = static_cast<int>(lh1.size());
    p->mh2 = static_cast<int>(lh2.size());
    p->mh3 = static_cast<int>(lh3.size());
    p->nbh1 = ceil_div(p->mh1, 8);
    p->nbh2 = ceil_div(p->mh2, 8);
    p->nbh3 = ceil_div(p->mh3, 8);
    if (p->nbh1 > 4 || p->nbh2 > 4 || p->nbh3 > 4)
        throw Error{-4, "G list spans more than 32 classes min(k, N - k) along an axis (unsupported)"};
    p->n2p = ceil_div(n[1], 16) * 16;
    p->n3p = ceil_div(n[2], 16) * 16;
    const int q = p->n3p / 4, nrb1 = p->n2p / 16;
    const int bw2 = p->nb2 * 16, bw3 = p->nb3 * 16, bwh3 = p->nbh3 * 16;
    {
        // tables, then a ring of 3 slabs (2 where 3 do not fit)
        const int ppw = zy_pairs_per_wave(p->nbh2, p->nbh3);
        const size_t nbands = 4 + 2 * static_cast<size_t>(ppw);
        const size_t tables = (static_cast<size_t>(q) * p->nbh3 * 32 +
                               static_cast<size_t>(nrb1) * 4 * p->nbh2 * 32 +
                               static_cast<size_t>(p->nbh2) * 16 * bwh3 / 4) * sizeof(double2);
        const size_t slab = nbands * 256 * sizeof(double2);
        p->ring = tables + 3 * slab <= kMaxLds ? 3 : 2;
        p->lds_yz = tables + p->ring * slab;
    }
    if (p->lds_yz > kMaxLds)
        throw Error{-4, "grid too large for the LDS-resident twiddle operands (unsupported)"};
    p->n1p = ceil_div(n[0], 4) * 4;
    p->lds_x = static_cast<size_t>(p->nbh1) * (p->n1p / 4) * 64 * sizeof(double);
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
    // forward stage-y outputs: (k2 class slot h2, sign) x column, the column of
    // block b and slot c giving k3 = +a3 (c < 8) or N3 - a3 (c >= 8) with
    // a3 = lh3[8 b + (c & 7)]; an output whose (k2, k3) is not in the disc, or
    // that repeats +a (a = 0 or N/2), is -1
    auto freq = [](const std::vector<int>& lh, int h, bool minus, int nn) {
        if (h >= static_cast<int>(lh.size())) return -1;
        const int a = lh[h];
        if (minus && (a == 0 || 2 * a == nn)) return -1;
        return minus ? nn - a : a;
    };
    std::vector<int> boxf(static_cast<size_t>(p->nbh2) * 16 * bwh3, -1);
    for (int h2 = 0; h2 < p->nbh2 * 8; ++h2)
        for (int sg = 0; sg < 2; ++sg) {
            const int k2v = freq(lh2, h2, sg == 1, n[1]);
            const auto it2 = i2.find(k2v);
            if (k2v < 0 || it2 == i2.end()) continue;
            for (int col = 0; col < bwh3; ++col) {
                const int k3v = freq(lh3, (col >> 4) * 8 + (col & 7), (col & 15) >= 8, n[2]);
                const auto it3 = i3.find(k3v);
                if (k3v < 0 || it3 == i3.end()) continue;
                boxf[(static_cast<size_t>(h2) * 2 + sg) * bwh3 + col] =
                    box[it2->second * bw3 + it3->second];
            }
        }
    p->n23p = ceil_div(nd, 16) * 16;
    for (int i = 0; i < ng; ++i) g_disc[i] = box[i2[k2[i]] * bw3 + i3[k3[i]]];
    // real twiddle operands of the forward stages, [k-step s][lane l][block b]
    // (a lane reads the blocks of a k-step as one run): for j = 4 s + l/16 and
    // class a = lh[8 b + (l & 7)], cos(2 pi a j/N)
    // (l & 15 < 8) or the sine (exactly 0 for a = 0 and a = N/2); zero past
    // the grid or the classes.  Stage z takes it as B (class = column), stage
    // y as A (class = row): the same lane layout.
    auto real_tab = [](const std::vector<int>& lh, int nbh, int nks, int nn) {
        std::vector<double> w(static_cast<size_t>(nks) * nbh * 64, 0.0);
        for (int s = 0; s < nks; ++s)
            for (int b = 0; b < nbh; ++b)
                for (int l = 0; l < 64; ++l) {
                    const int j = 4 * s + (l >> 4);
                    const int h = b * 8 + (l & 7);
                    if (j >= nn || h >= static_cast<int>(lh.size())) continue;
                    const int a = lh[h];
                    const double2 r = host_root(static_cast<int64_t>(a) * j, nn);
                    const bool sine = (l & 15) >= 8;
                    w[(static_cast<size_t>(s) * 64 + l) * nbh + b] =
                        sine ? ((a == 0 || 2 * a == nn) ? 0.0 : r.y) : r.x;
                }
        return w;
    };
    const std::vector<double> w3 = real_tab(lh3, p->nbh3, q, n[2]);
    const std::vector<double> w2 = real_tab(lh2, p->nbh2, nrb1 * 4, n[1]);
    const std::vector<double> w1 = real_tab(lh1, p->nbh1, p->n1p / 4, n[0]);
    // forward stage-x outputs: (k1 class slot, sign: 0 for k1 = a, 1 for k1 = N1 - a,
    // a != 0, N1/2) x disc index -> G index
    std::vector<int> gmapf(static_cast<size_t>(p->nbh1) * 16 * p->n23p, -1);
    {
        std::map<int, int> ih1;
        for (int h = 0; h < p->mh1; ++h) ih1[lh1[h]] = h;
        for (int i = 0; i < ng; ++i) {
            const int a = std::min(k1[i], n[0] - k1[i]);
            const int sg = k1[i] == a ? 0 : 1;
            gmapf[(static_cast<size_t>(ih1[a]) * 2 + sg) * p->n23p + g_disc[i]] = i;
        }
    }
    // adjoint (inverse) stages, e^{-2 pi i k j/N} summed over classes as
    // P cos + Q sin: the real cos | sin operands in the transposed lane layouts.
    // Slot of lane l at k-step s: 4 (s % 4) + l/16 of class block s/4 (slot < 8:
    // cosine of class 8 (s/4) + slot, else the sine of class 8 (s/4) + slot - 8).
    //   x: A = [j1][slot], [n1p16/16][nbh1*4][64], j1 = 16 rb + l%16
    //   y: A = [j2][slot], [n2p/16][nbh2*4][64],   j2 = 16 rb + l%16
    //   z: B = [slot][j3], [nbh3*4][n3p/16][64],   j3 = 16 nb + l%16
    p->n1p16 = ceil_div(n[0], 16) * 16;
    auto inv_val = [](const std::vector<int>& lh, int s, int l, int j, int nn) {
        const int slot = 4 * (s & 3) + (l >> 4);
        const int h = (s >> 2) * 8 + (slot & 7);
        if (j >= nn || h >= static_cast<int>(lh.size())) return 0.0;
        const int a = lh[h];
        const double2 r = host_root(static_cast<int64_t>(a) * j, nn);
        if (slot < 8) return r.x;
        return (a == 0 || 2 * a == nn) ? 0.0 : r.y;
    };
    auto inv_rows = [&](const std::vector<int>& lh, int nbh, int nrb, int nn) {
        std::vector<double> w(static_cast<size_t>(nrb) * nbh * 4 * 64);
        for (int rb = 0; rb < nrb; ++rb)
            for (int sk = 0; sk < nbh * 4; ++sk)
                for (int l = 0; l < 64; ++l)
                    w[(static_cast<size_t>(rb) * nbh * 4 + sk) * 64 + l] =
                        inv_val(lh, sk, l, rb * 16 + (l & 15), nn);
        return w;
    };
    const std::vector<double> w1i = inv_rows(lh1, p->nbh1, p->n1p16 / 16, n[0]);
    const std::vector<double> w2i = inv_rows(lh2, p->nbh2, nrb1, n[1]);
    const int nj3 = p->n3p / 16;
    std::vector<double> w3i(static_cast<size_t>(p->nbh3) * 4 * nj3 * 64);
    for (int sk = 0; sk < p->nbh3 * 4; ++sk)
        for (int nb = 0; nb < nj3; ++nb)
            for (int l = 0; l < 64; ++l)
                w3i[(static_cast<size_t>(sk) * nj3 + nb) * 64 + l] =
                    inv_val(lh3, sk, l, nb * 16 + (l & 15), n[2]);
    // inverse stage-z gather: row r of k2 block b2 is k2 = +a2 (r < 8) or -a2
    // (r >= 8) of class 8 b2 + r % 8; column 4 i + kq of k3 block b3 is the value
    // i of that lane: k3 = +a3 (i < 2) or -a3 (i >= 2) of class 8 b3 + 4 (i % 2) + kq
    std::vector<int> boxi(static_cast<size_t>(p->nbh2) * 16 * bwh3, -1);
    for (int r2 = 0; r2 < p->nbh2 * 16; ++r2) {
        const int k2v = freq(lh2, (r2 >> 4) * 8 + (r2 & 7), (r2 & 15) >= 8, n[1]);
        const auto it2 = i2.find(k2v);
        if (k2v < 0 || it2 == i2.end()) continue;
        for (int c3 = 0; c3 < bwh3; ++c3) {
            const int i = (c3 & 15) >> 2, kqc = c3 & 3;
            const int k3v = freq(lh3, (c3 >> 4) * 8 + 4 * (i & 1) + kqc, i >= 2, n[2]);
            const auto it3 = i3.find(k3v);
            if (k3v < 0 || it3 == i3.end()) continue;
            boxi[static_cast<size_t>(r2) * bwh3 + c3] = box[it2->second * bw3 + it3->second];
        }
    }

    p->w1re = upload(w1);
    p->gmapf = upload(gmapf);
    p->w3re = upload(w3);
    p->w2re = upload(w2);
    p->boxf = upload(boxf);
    p->w1ir = upload(w1i);
    p->w2ir = upload(w2i);
    p->w3ir = upload(w3i);
    p->boxi = upload(boxi);
    return p;
}

}  // namespace

void MtxelPlan::release() {
    (void)hipFree(w1re);
    (void)hipFree(gmapf);
    (void)hipFree(w3re);
    (void)hipFree(boxf);
    (void)hipFree(w2re);
    (void)hipFree(w1ir);
    (void)hipFree(w2ir);
    (void)hipFree(w3ir);
    (void)hipFree(boxi);
    w1re = w2re = w3re = w1ir = w2ir = w3ir = nullptr;
    gmapf = boxf = boxi = nullptr;
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
                  double volume, double2* t2, double2* m_out, hipStream_t s, int64_t ldm) {
    if (ldm == 0) ldm = rc.nc;
    const int64_t npairs = static_cast<int64_t>(rc.nv) * rc.nc;
    if (npairs <= 0) return;
    const ZyLaunches& zl = select_zy(p.nbh2, p.nbh3);
    const int ppw = zy_pairs_per_wave(p.nbh2, p.nbh3);
    for (int h = 0; h < zl.count; ++h)
        GW_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(zl.k[h]),
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
        for (int h = 0; h < zl.count; ++h)
            hipLaunchKernelGGL(zl.k[h], grid, dim3(kZyThreads), p.lds_yz, s, psi_v, psi_c, p.nr, rc,
                               p.n[0], pp, p.n[1], p.n[2], p.n2p, p.n3p, p.w3re, p.w2re, p.boxf,
                               p.n23, t2, p.ring, zl.b2_0[h]);
        GW_HIP_TRY(hipGetLastError());
    }
    XKernel kx = select_x(p.nbh1);
    GW_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(kx),
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   static_cast<int>(p.lds_x)));
    const double dv = volume / static_cast<double>(p.nr);
    for (int64_t k0 = 0; k0 < npairs; k0 += kMaxGrid) {
        const int64_t kb = std::min<int64_t>(kMaxGrid, npairs - k0);
        ProfScope ps("mtxel_x", s);
        hipLaunchKernelGGL(kx, dim3(static_cast<unsigned>(kb)), dim3(kThreads), p.lds_x, s,
                           t2 + k0 * static_cast<int64_t>(p.n[0]) * p.n23, p.n[0], p.n1p, p.n23,
                           p.n23p, p.w1re, p.gmapf, p.ng, dv, kb, k0, rc.nc, ldm, m_out);
        GW_HIP_TRY(hipGetLastError());
    }
}

}  // namespace gw
