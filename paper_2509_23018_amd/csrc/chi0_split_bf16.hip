// Split-BF16 CHI0 contraction on the 32x32x16 BF16 MFMA of gfx950 (not in the
// paper, which is FP64 only; the energy factor, the slice recombination and
// chi stay FP64).
//
// Slicing.  Per block of 128 pairs and per G, every operand value x (M for the
// G side, Delta_w M for the G' side, both FP64) gets the exponent e with
// max(|Re x|, |Im x|) < 2^e over the block, and is cut into S slices
//     x 2^(8-e) = q_0 + q_1 2^-8 + ... + q_{S-1} 2^(-8(S-1)) (+ residual),
// rounding to nearest each time (|q_0| <= 256, |q_s| <= 128).  Slice s is
// stored as the BF16 value q_s 2^(-8s): exact, since q_s has at most 8
// significant bits.
//
// Products.  Slices a (G side) and b (G' side) with a + b <= S - 1 are
// multiplied on MFMA with FP32 accumulation in three groups: t = a + b = 0,
// t = 1 and t >= 2.  Over a block of 128 pairs (256 real products per complex
// entry and shift) every partial sum of the t = 0 group is an integer of
// magnitude at most 256 * 2^16 = 2^24, and of the t = 1 group an integer
// multiple of 2^-8 of magnitude at most 512 * 2^7 = 2^16: both exact in FP32.
// The t >= 2 group is at most 2^-16 of the result, so its FP32 rounding costs
// about 2^-40 relative.
// After each block, 2^(eA + eB - 16) (acc_0 + acc_1 + acc_2) is added in FP64.
//
// Complex arithmetic uses the real-stacked form: the K axis of one MFMA holds
// 8 pairs with (Re, Im) interleaved, so conj(A) B = sum A'B' (Re) and
// sum A' B'' (Im) with B'' = (Im B, -Re B) formed in registers.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "chi0.hpp"
#include "common.hpp"
#include "items.hpp"
#include "prof.hpp"

namespace gw {

namespace {

constexpr int kStep = 8;                     // pairs per MFMA k-step (K = 16)
constexpr int kTI = 128, kTJ = 64;           // workgroup tile: rows G, columns G'

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Slice formats.
// SlBf16: 8-bit slices, x 2^(8-e) = q_0 + q_1 2^-8 + ... (|q_0| <= 256,
//   |q_s| <= 128), slice s stored as the BF16 value q_s 2^-8s; over blocks of
//   KB = 128 pairs the t = 0 and t = 1 sums stay exact in FP32 (above).
// SlF16x9: 9-bit slices, x 2^(9-e) = q_0 + q_1 2^-9 + ... (|q_0| <= 512,
//   |q_s| <= 256), slice s stored as the FP16 value q_s 2^(6-9s): at most 11
//   significant bits, and for s <= 3 within FP16's range (the fourth slice as
//   an exact subnormal, a multiple of 2^-21), so at most four slices.  A
//   product q_0 q_0' 2^12 reaches 2^30: over KB = 32 pairs (64 real products
//   per component) the t = 0 sum is a multiple of 2^12 below 2^36 and the
//   t = 1 sum (128 products) a multiple of 2^3 below 2^27, both exact in FP32;
//   t >= 2 is below 2^-18 of the result.  sigma = 2^(e - 9 - 6).
// The last slice of four is 2^-35 of the block maximum for FP16 against 2^-32
// for BF16; with the same ten products (t <= 3) the error drops about 20x.
struct SlBf16 {
    static constexpr int KB = 128, BITS = 8, SHIFT = 0, SMAX = 6;
    static __device__ __forceinline__ uint32_t enc(double q, int sl) {
        // q 2^(-8 sl) has at most 8 significant bits: the top half of its FP32
        // bits is its exact BF16 encoding
        return __float_as_uint(ldexpf(static_cast<float>(q), -8 * sl)) >> 16;
    }
    static __device__ __forceinline__ f32x16 mfma(u32x4 a, u32x4 b, f32x16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
    }
};
struct SlF16x9 {
    static constexpr int KB = 32, BITS = 9, SHIFT = 6, SMAX = 4;
    static __device__ __forceinline__ uint32_t enc(double q, int sl) {
        const _Float16 h = static_cast<_Float16>(ldexpf(static_cast<float>(q), SHIFT - 9 * sl));
        return __builtin_bit_cast(uint16_t, h);
    }
    static __device__ __forceinline__ f32x16 mfma(u32x4 a, u32x4 b, f32x16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                      __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
    }
};
template <class F>
constexpr int ksteps() {  // k-steps per exponent block
    return F::KB / kStep;
}

// ---------------------------------------------------------------- slicing

// One workgroup per (block of KB pairs, prep_cols<F>() columns of G); thread
// (k-step ks, column c) keeps the 8 pairs of its k-step in registers: a wave
// holds 4 k-steps of 16 columns, and the KB / 32 waves of a block share one
// set of columns.  Output layout, in 32-bit words (Re in the low half, Im in
// the high half):
//   slices[kb][ks][s][g][p]   p = pair within the k-step (0..7),
// i.e. per (block, k-step, slice) a [ng][8]-word array: a 128-row panel of a
// tile is one contiguous 4 KB run, and a thread writes its 8 pairs as one
// 32-byte run.  sigma[kb][g] = 2^(e - BITS - SHIFT), rows padded to ngp (a
// multiple of 128, which the grid covers) with 1.0 so that a tile's sigma
// panel is whole.
template <class F>
constexpr int prep_cols() {
    return 16 * (4 / (ksteps<F>() / 4));
}

template <class F>
__global__ __launch_bounds__(256) void sbf16_prep_kernel(
    const double2* __restrict__ m, const double2* __restrict__ delta, int64_t kc, int ng, int ngp,
    int S, int nkb, WList wl, uint32_t* __restrict__ slices_a, double* __restrict__ sigma_a,
    uint32_t* __restrict__ slices_b, double* __restrict__ sigma_b) {
    constexpr int WPB = ksteps<F>() / 4;  // waves per block of pairs
    static_assert(WPB >= 1 && 4 % WPB == 0, "prep mapping");
    __shared__ double s_part[4][16];      // per-wave column maxima
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int c = lane & 15, ks = (wave % WPB) * 4 + (lane >> 4);
    const int cg = wave / WPB;  // column group of this wave
    const int g = blockIdx.x * prep_cols<F>() + cg * 16 + c, kb = blockIdx.y;
    const int64_t k0 = static_cast<int64_t>(kb) * F::KB + ks * kStep;
    const int kn = static_cast<int>(std::max<int64_t>(0, std::min<int64_t>(kStep, kc - k0)));
    const bool gv = g < ng;
    // lanes of one k-step read 16 consecutive G: 256-byte runs of a row of M
    double2 x[kStep];
#pragma unroll
    for (int p = 0; p < kStep; ++p)
        x[p] = (gv && p < kn) ? m[(k0 + p) * ng + g] : make_double2(0.0, 0.0);
    const size_t per_op = static_cast<size_t>(nkb) * ksteps<F>() * S * ng * kStep;  // words
    const int nop = 1 + wl.nh + wl.nf;
    for (int op = 0; op < nop; ++op) {
        double2 y[kStep];
        if (op == 0) {
#pragma unroll
            for (int p = 0; p < kStep; ++p) y[p] = x[p];
        } else {
            const double2* dw = delta + static_cast<int64_t>(wl.w[op - 1]) * kc;
#pragma unroll
            for (int p = 0; p < kStep; ++p)
                y[p] = p < kn ? cmul(dw[k0 + p], x[p]) : make_double2(0.0, 0.0);
        }
        double mx = 0.0;
#pragma unroll
        for (int p = 0; p < kStep; ++p) mx = fmax(mx, fmax(fabs(y[p].x), fabs(y[p].y)));
        // over the 4 k-steps of this wave (lanes c, c+16, c+32, c+48), then the
        // WPB waves of the block
        mx = fmax(mx, __shfl_xor(mx, 16));
        mx = fmax(mx, __shfl_xor(mx, 32));
        if (lane < 16) s_part[wave][c] = mx;
        __syncthreads();
#pragma unroll
        for (int w2 = 0; w2 < WPB; ++w2) mx = fmax(mx, s_part[cg * WPB + w2][c]);
        int e = 0;
        if (mx > 0.0) (void)frexp(mx, &e);  // mx = f 2^e, f in [0.5, 1): |x| < 2^e
        if (wave % WPB == 0 && lane < 16 && g < ngp) {
            const double sg = gv ? ldexp(1.0, e - F::BITS - F::SHIFT) : 1.0;
            if (op == 0)
                sigma_a[static_cast<size_t>(kb) * ngp + g] = sg;
            else
                sigma_b[(static_cast<size_t>(wl.w[op - 1]) * nkb + kb) * ngp + g] = sg;
        }
        if (gv) {
            double rr[kStep], ri[kStep];
#pragma unroll
            for (int p = 0; p < kStep; ++p) {
                rr[p] = ldexp(y[p].x, F::BITS - e);
                ri[p] = ldexp(y[p].y, F::BITS - e);
            }
            uint32_t* out = op == 0 ? slices_a : slices_b + static_cast<size_t>(wl.w[op - 1]) * per_op;
            uint32_t* o = out + ((static_cast<size_t>(kb) * ksteps<F>() + ks) * S * ng + g) * kStep;
            for (int sl = 0; sl < S; ++sl) {
                uint32_t word[kStep];
#pragma unroll
                for (int p = 0; p < kStep; ++p) {
                    const double qr = rint(rr[p]), qi = rint(ri[p]);
                    word[p] = (F::enc(qi, sl) << 16) | F::enc(qr, sl);
                    rr[p] = ldexp(rr[p] - qr, F::BITS);
                    ri[p] = ldexp(ri[p] - qi, F::BITS);
                }
                u32x4* dst = reinterpret_cast<u32x4*>(o + static_cast<size_t>(sl) * ng * kStep);
                dst[0] = u32x4{word[0], word[1], word[2], word[3]};
                dst[1] = u32x4{word[4], word[5], word[6], word[7]};
            }
        }
        __syncthreads();  // s_part is rewritten by the next operand
    }
}

// ---------------------------------------------------------------- contraction

// Item t -> frequency w, 128-row block bi, 64-column block bj.  Items come in
// pairs (both 64-column halves of one 128 x 128 block) so that the square
// tile order and the Hermitian rule (blocks on or above the diagonal) of the
// FP64 kernels apply with a 128 tile; workgroups reach items through the XCD
// renumbering (xcd_item), which keeps each XCD on a contiguous run of items,
// and 4 x 4 super-blocks make the 32 workgroups an XCD runs at once share 4
// row panels and 8 column panels.
__device__ __forceinline__ void rect_item_tile(int t, const WList& wl, int nb,
                                               const int* __restrict__ order, int& w, int& bi,
                                               int& bj) {
    const int nh = nb * (nb + 1) / 2, nf = nb * nb;
    const int half = t & 1;
    t >>= 1;
    int code;
    if (t < wl.nh * nh) {
        w = wl.w[t / nh];
        code = order[t % nh];
    } else {
        t -= wl.nh * nh;
        w = wl.w[wl.nh + t / nf];
        code = order[nh + t % nf];
    }
    bi = code >> 16;
    bj = 2 * (code & 0xffff) + half;
}


// (Re, Im) -> (Im, -Re) in every 32-bit word of a fragment.
__device__ __forceinline__ u32x4 swap_neg(u32x4 v) {
    u32x4 r;
#pragma unroll
    for (int d = 0; d < 4; ++d) r[d] = ((v[d] >> 16) | (v[d] << 16)) ^ 0x80000000u;
    return r;
}

// LDS position of 16-byte half h of row r within a panel.  A 128-bit read by
// 32 lanes on consecutive rows is served 8 or 16 lanes at a time; swapping
// the halves of rows with bit 2 xor bit 3 set puts every such group of lanes
// on distinct banks (32 or 64 banks of 4 bytes).
__device__ __forceinline__ int swz(int r) { return ((r >> 2) ^ (r >> 3)) & 1; }
__device__ __forceinline__ int lds_slot(int r, int h) { return 2 * r + (h ^ swz(r)); }

// vmcnt(n) alone (expcnt and lgkmcnt left at their no-wait maxima).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// vmcnt(n) and lgkmcnt(0): also every LDS read of this wave has returned.
template <int N>
__device__ __forceinline__ void wait_vm_lgkm0() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4));
}

// Workgroup tile kTI x kTJ of chi_w, NWI x NWJ waves, each BI x BJ blocks of
// 32 x 32.  Operands are staged per k-step of 8 pairs: both slice panels
// ((kTI + kTJ) rows x S slices x 32 B) and the sigma of the step's 64-pair
// block, written straight from global memory into LDS (no registers) in a
// ring of 3 or 4 stages, 2 or 3 steps ahead of the MFMAs.  Every wave issues
// the same number of 16-byte loads per step (spare lanes fetch a valid
// address into padding), so "this step has landed" is vmcnt(loads per step)
// after the next step's loads are in flight.
// Stage geometry of the contraction for S slices and NW waves; RV picks the
// ring (0: the preferred one below; 1: the other stage height, for the
// autotuner).
template <int S, int NW, int RV = 0>
struct SbGeom {
    static constexpr int NT = NW * 64;
    static constexpr int CA = kTI * 2 * S, CB = kTJ * 2 * S;  // slice chunks (16 B) per k-step
    static constexpr int CSA = kTI / 2, CSB = kTJ / 2;        // sigma chunks (two doubles each)
    static constexpr int NCH = CA + CB + CSA + CSB;
    static constexpr int NLD = (NCH + NT - 1) / NT;  // loads per thread per step
    static constexpr int NCHP = NLD * NT;            // padded k-step slot, in chunks
    // A ring stage holds KSUB k-steps (one barrier per stage); kStages stages.
    // Preference: two k-steps per stage, then depth; all within 159 KB of LDS.
    // At four slices one k-step per stage in a four-stage ring (three steps
    // ahead instead of one stage of two) is about 3 % faster on the 48^3
    // chunk; at five slices, with the same slot size, it is not.
    static constexpr size_t kSlot = static_cast<size_t>(NCHP) * 16;
    static constexpr size_t kMax = 159 * 1024;
    static constexpr int KSUB0 = S == 4 ? 1 : 6 * kSlot <= kMax || 4 * kSlot <= kMax ? 2 : 1;
    // variant 1: one k-step per stage where variant 0 takes two, two where it
    // takes one and four slots fit (else the same ring as variant 0)
    static constexpr int KSUB = RV == 0 ? KSUB0 : KSUB0 == 2 ? 1 : 4 * kSlot <= kMax ? 2 : 1;
    static constexpr int kStages = KSUB == 2 ? (6 * kSlot <= kMax ? 3 : 2) : (4 * kSlot <= kMax ? 4 : 3);
    static constexpr int NSLOT = KSUB * kStages;
    static constexpr size_t lds_bytes = NSLOT * kSlot;
    static_assert(lds_bytes <= kMax, "LDS ring");
};

// One tile (rows bi*kTI.., columns bj*kTJ..) of one frequency plane chi_w:
// sb and sigb are that frequency's B slices and sigma.  The caller has made
// sure every wave of the workgroup calls this with the same arguments and
// that no earlier reader of lds is still running.
template <class F, int S, int NWI, int NWJ, int BI, int BJ, bool PART = false, int RV = 0>
__device__ __forceinline__ void sbf16_tile(const u32x4* __restrict__ sa,
                                           const double* __restrict__ siga,
                                           const u32x4* __restrict__ sb,
                                           const double* __restrict__ sigb, int ng, int ngp,
                                           int nkb, double2* __restrict__ cw, int mode, int bi,
                                           int bj, u32x4* __restrict__ lds) {
    static_assert(NWI * BI * 32 == kTI && NWJ * BJ * 32 == kTJ, "tile shape");
    using Geo = SbGeom<S, NWI * NWJ, RV>;
    constexpr int NW = NWI * NWJ;
    constexpr int G = S < 3 ? S : 3;
    constexpr int CA = Geo::CA, CB = Geo::CB, CSA = Geo::CSA, CSB = Geo::CSB, NCH = Geo::NCH;
    constexpr int NLD = Geo::NLD, NCHP = Geo::NCHP, kStages = Geo::kStages;
    constexpr int KSUB = Geo::KSUB, NSLOT = Geo::NSLOT;
    constexpr int kStepsPerBlk = ksteps<F>();
    static_assert(kStepsPerBlk % KSUB == 0, "stages within a block");
    const int i0 = bi * kTI, j0 = bj * kTJ;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wi = wave / NWJ, wj = wave % NWJ;
    const int rl = lane & 31, hl = lane >> 5;
    const size_t step_stride = static_cast<size_t>(S) * ng * 2;  // slice chunks per k-step
    const u32x4* sga = reinterpret_cast<const u32x4*>(siga);
    const u32x4* sgb = reinterpret_cast<const u32x4*>(sigb);

    // Load u of this wave fills stage slots [(u*NW + wave)*64, +64).  Panel
    // sizes are multiples of 64 chunks, so each load reads one kind of data
    // from one wave-uniform base (advanced per step or per block in scalar
    // registers) plus a fixed per-lane byte offset: A slices, B slices, A
    // sigma, B sigma (32 lanes, the other 32 repeat them into padding) or
    // padding.
    static_assert(CA % 64 == 0 && CB % 64 == 0 && CSA == 64 && CSB == 32, "panel sizes");
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    uint32_t voff[NLD];
#pragma unroll
    for (int u = 0; u < NLD; ++u) {
        const int c = (u * NW + wv) * 64 + lane;
        int off;
        if (c < CA) {
            const int sl = c / (2 * kTI), pp = c % (2 * kTI), rr = pp >> 1;
            const int h = (pp & 1) ^ swz(rr);  // inverse of lds_slot
            off = (sl * ng + min(i0 + rr, ng - 1)) * 2 + h;
        } else if (c < CA + CB) {
            const int cb = c - CA;
            const int sl = cb / (2 * kTJ), pp = cb % (2 * kTJ), rr = pp >> 1;
            const int h = (pp & 1) ^ swz(rr);
            off = (sl * ng + min(j0 + rr, ng - 1)) * 2 + h;
        } else {
            off = lane & (c < CA + CB + CSA ? 63 : 31);
        }
        voff[u] = static_cast<uint32_t>(off) * 16u;
    }
    const int nsteps = nkb * kStepsPerBlk;
    // per load: base at step 0 and which advance applies (all wave-uniform)
    const char* base0[NLD];
    uint64_t step_mask[NLD], blk_mask[NLD];
#pragma unroll
    for (int u = 0; u < NLD; ++u) {
        const int c0 = (u * NW + wv) * 64;
        const bool slices = c0 < CA + CB, sigma = !slices && c0 < NCH;
        base0[u] = c0 < CA               ? reinterpret_cast<const char*>(sa)
                   : c0 < CA + CB        ? reinterpret_cast<const char*>(sb)
                   : c0 < CA + CB + CSA  ? reinterpret_cast<const char*>(sga + (i0 >> 1))
                   : c0 < NCH            ? reinterpret_cast<const char*>(sgb + (j0 >> 1))
                                         : reinterpret_cast<const char*>(sa);
        step_mask[u] = slices ? ~uint64_t(0) : 0;
        blk_mask[u] = sigma ? ~uint64_t(0) : 0;
    }
    auto issue = [&](int st, int stage) {
        const uint64_t so = static_cast<uint64_t>(st) * step_stride * 16;
        const uint64_t bo = static_cast<uint64_t>(st / kStepsPerBlk) * (ngp >> 1) * 16;
#pragma unroll
        for (int u = 0; u < NLD; ++u) {
            const char* base = base0[u] + ((so & step_mask[u]) | (bo & blk_mask[u]));
            __builtin_amdgcn_global_load_lds(reinterpret_cast<const u32x4*>(base + voff[u]),
                                             &lds[stage * NCHP + (u * NW + wv) * 64], 16, 0, 0);
        }
    };

    f32x16 accR[G][BI][BJ], accI[G][BI][BJ];  // set by each block's first step
    double dr[BI][BJ][16], di[BI][BJ][16];
#pragma unroll
    for (int x = 0; x < BI; ++x)
#pragma unroll
        for (int y = 0; y < BJ; ++y)
#pragma unroll
            for (int t = 0; t < 16; ++t) dr[x][y][t] = di[x][y][t] = 0.0;

    const f32x16 zero16 = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f,
                           0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    // Every KSUB k-steps: wait until this stage has landed (at most the
    // kStages - 2 later stages' loads of this wave still outstanding) and this
    // wave's fragment reads have returned; the barrier extends both to the
    // workgroup.  Then refill the stage that the previous KSUB k-steps read.
    auto sync = [&](int st) {
        wait_vm_lgkm0<(kStages - 2) * KSUB * NLD>();
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");  // keep the LDS reads below the barrier
#pragma unroll
        for (int i = 0; i < KSUB; ++i) {
            const int nx = st + (kStages - 1) * KSUB + i;
            issue(min(nx, nsteps - 1), nx % NSLOT);
        }
    };
    // Fragments of one k-step: S slices of this wave's rows of A (FA) and
    // columns of B (FB).
    struct FA {
        u32x4 v[S][BI];
    };
    struct FB {
        u32x4 v[S][BJ];
    };
    auto read_a = [&](int st, FA& f) {
        const u32x4* L = lds + (st % NSLOT) * NCHP;
#pragma unroll
        for (int sl = 0; sl < S; ++sl)
#pragma unroll
            for (int x = 0; x < BI; ++x)
                f.v[sl][x] = L[sl * 2 * kTI + lds_slot(wi * BI * 32 + x * 32 + rl, hl)];
    };
    auto read_b = [&](int st, FB& f) {
        const u32x4* L = lds + (st % NSLOT) * NCHP;
#pragma unroll
        for (int sl = 0; sl < S; ++sl)
#pragma unroll
            for (int y = 0; y < BJ; ++y)
                f.v[sl][y] = L[CA + sl * 2 * kTJ + lds_slot(wj * BJ * 32 + y * 32 + rl, hl)];
    };
    // The MFMAs of one k-step for B slices [B0, B1); on the block's first step
    // (`first`) every group starts from zero.
    auto compute = [&](const FA& fa, const FB& fbs, auto first, auto b0, auto b1) {
#pragma unroll
        for (int b = decltype(b0)::value; b < decltype(b1)::value; ++b)
#pragma unroll
            for (int y = 0; y < BJ; ++y) {
                const u32x4 fb = fbs.v[b][y];
                const u32x4 fbi = swap_neg(fb);
#pragma unroll
                for (int a = 0; a < S - b; ++a) {
                    const int g = a + b < G - 1 ? a + b : G - 1;
                    // the first product of each group in the block (b = 0, a = g)
                    const bool fresh = decltype(first)::value && b == 0 && a == g;
#pragma unroll
                    for (int x = 0; x < BI; ++x) {
                        accR[g][x][y] = F::mfma(fa.v[a][x], fb, fresh ? zero16 : accR[g][x][y]);
                        accI[g][x][y] = F::mfma(fa.v[a][x], fbi, fresh ? zero16 : accI[g][x][y]);
                    }
                }
            }
    };
    using B0 = std::integral_constant<int, 0>;
    using B1 = std::integral_constant<int, 1>;
    using BS = std::integral_constant<int, S>;
    const std::true_type yes{};
    const std::false_type no{};
    // How far ahead the fragments are read, as far as registers allow (two
    // waves of 256 registers per SIMD):
    //   2: both operands of step st + 1 are requested before the MFMAs of step
    //      st, so their LDS reads run under them;
    //   1: the A fragments of step st + 1 are requested after the first B
    //      slice's MFMAs of step st, and step st's own B fragments at its start
    //      (only the first of them is waited for before MFMAs begin);
    //   0: each step reads its fragments just before its MFMAs.
    // A stage sync (which refills the stage of the k-steps just read) comes
    // right before the first read of a step that opens a stage.
    constexpr int kPipe = S <= 3 ? 2 : S <= 5 ? 1 : 0;
    FA a0, a1;
    FB b0, b1;
    // step st with A fragments ca (read earlier) and B fragments cb; with
    // `prefetch`, also reads step st + 1 into na (and nb)
    auto pstep = [&](int st, FA& ca, FB& cb, FA& na, FB& nb, auto first, auto prefetch) {
        constexpr bool pf = decltype(prefetch)::value;
        if constexpr (kPipe == 2) {
            if constexpr (pf) {
                if ((st + 1) % KSUB == 0) sync(st + 1);
                read_a(st + 1, na);
                read_b(st + 1, nb);
            }
            __builtin_amdgcn_sched_barrier(0);
            compute(ca, cb, first, B0{}, BS{});
        } else {
            read_b(st, cb);
            __builtin_amdgcn_sched_barrier(0);
            compute(ca, cb, first, B0{}, B1{});
            if constexpr (pf) {
                if ((st + 1) % KSUB == 0) sync(st + 1);
                read_a(st + 1, na);
            }
            __builtin_amdgcn_sched_barrier(0);
            compute(ca, cb, first, B1{}, BS{});
        }
    };
#pragma unroll
    for (int q = 0; q < (kStages - 1) * KSUB; ++q) issue(min(q, nsteps - 1), q);
    if constexpr (kPipe > 0) {
        sync(0);
        read_a(0, a0);
        if constexpr (kPipe == 2) read_b(0, b0);
    }
    for (int kb = 0; kb < nkb; ++kb) {
        const int st0 = kb * kStepsPerBlk;
        if constexpr (kPipe > 0) {
            // kPipe 1 reads each step's B into its own buffer and never uses nb
            FB& b1x = kPipe == 2 ? b1 : b0;
            pstep(st0, a0, b0, a1, b1x, yes, yes);
            pstep(st0 + 1, a1, b1x, a0, b0, no, yes);
            for (int ks = 2; ks < kStepsPerBlk - 2; ks += 2) {
                pstep(st0 + ks, a0, b0, a1, b1x, no, yes);
                pstep(st0 + ks + 1, a1, b1x, a0, b0, no, yes);
            }
            pstep(st0 + kStepsPerBlk - 2, a0, b0, a1, b1x, no, yes);
            // The block's last step prefetches nothing: the stage sync that the
            // next step needs would refill the stage that holds this block's sigma.
            pstep(st0 + kStepsPerBlk - 1, a1, b1x, a0, b0, no, no);
        } else {
            auto step = [&](int st, auto first) {
                if (st % KSUB == 0) sync(st);
                read_a(st, a0);
                read_b(st, b0);
                __builtin_amdgcn_sched_barrier(0);
                compute(a0, b0, first, B0{}, BS{});
            };
            step(st0, yes);
            for (int ks = 1; ks < kStepsPerBlk; ++ks) step(st0 + ks, no);
        }
        // end of the block: fold the FP32 groups into FP64 with this block's sigma
        const double* sgl = reinterpret_cast<const double*>(
            lds + ((st0 + kStepsPerBlk - 1) % NSLOT) * NCHP + CA + CB);
#pragma unroll
        for (int y = 0; y < BJ; ++y) {
            const double sbj = sgl[kTI + wj * BJ * 32 + y * 32 + rl];
#pragma unroll
            for (int x = 0; x < BI; ++x)
#pragma unroll
                for (int t = 0; t < 16; ++t) {
                    const double sc =
                        sgl[wi * BI * 32 + x * 32 + 8 * (t >> 2) + 4 * hl + (t & 3)] * sbj;
                    double vr = static_cast<double>(accR[0][x][y][t]);
                    double vi = static_cast<double>(accI[0][x][y][t]);
#pragma unroll
                    for (int g = 1; g < G; ++g) {
                        vr += static_cast<double>(accR[g][x][y][t]);
                        vi += static_cast<double>(accI[g][x][y][t]);
                    }
                    dr[x][y][t] = fma(sc, vr, dr[x][y][t]);
                    di[x][y][t] = fma(sc, vi, di[x][y][t]);
                }
        }
        if (kPipe > 0 && kb + 1 < nkb) {
            sync(st0 + kStepsPerBlk);
            read_a(st0 + kStepsPerBlk, a0);
            if constexpr (kPipe == 2) read_b(st0 + kStepsPerBlk, b0);
        }
    }
    wait_vmcnt<0>();  // no load into this workgroup's LDS may outlive the tile
#pragma unroll
    for (int x = 0; x < BI; ++x)
#pragma unroll
        for (int y = 0; y < BJ; ++y)
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const int li = wi * BI * 32 + x * 32 + 8 * (t >> 2) + 4 * hl + (t & 3);
                const int lj = wj * BJ * 32 + y * 32 + rl;
                if constexpr (PART) {
                    // a partial sum: the whole tile, unmasked, row-major
                    cw[li * kTJ + lj] = make_double2(dr[x][y][t], di[x][y][t]);
                    continue;
                }
                const int gi = i0 + li, gj = j0 + lj;
                if (gi < ng && gj < ng) {
                    double2* p = cw + static_cast<int64_t>(gi) * ng + gj;
                    double2 v = make_double2(dr[x][y][t], di[x][y][t]);
                    if (mode) {
                        const double2 o = *p;
                        v.x += o.x;
                        v.y += o.y;
                    }
                    *p = v;
                }
            }
}

// One launch per chunk.  The first n_main items take one workgroup each over
// all blocks of the chunk.  Each remaining item (the last, partial round) is
// cut into `parts` ranges of 128-pair blocks: workgroup n_main + j*parts + p
// writes item n_main + j's partial sum over range p to ws[j*parts + p]
// (kTI x kTJ), and sbf16_tail_reduce_kernel adds the parts into chi.
template <class F, int S, int NWI, int NWJ, int BI, int BJ, int RV>
__global__ __launch_bounds__(NWI* NWJ * 64) void chi0_sbf16_kernel(
    const u32x4* __restrict__ sa, const double* __restrict__ siga, const u32x4* __restrict__ sb_all,
    const double* __restrict__ sigb_all, int ng, int ngp, int nkb, WList wl,
    double2* __restrict__ chi, int mode, int nb, const int* __restrict__ order, int n_main,
    int parts, double2* __restrict__ ws) {
    extern __shared__ u32x4 lds[];
    const int b = blockIdx.x;
    const size_t blk = static_cast<size_t>(ksteps<F>()) * S * ng * 2;  // chunks per block
    const size_t plane = static_cast<size_t>(nkb) * blk;
    int w, bi, bj;
    if (b < n_main) {
        rect_item_tile(xcd_item(b, n_main), wl, nb, order, w, bi, bj);
        if (bj * kTJ >= ng) return;  // right half of the last block column lies past N_G
        sbf16_tile<F, S, NWI, NWJ, BI, BJ, false, RV>(sa, siga, sb_all + w * plane,
                                        sigb_all + static_cast<size_t>(w) * nkb * ngp, ng, ngp,
                                        nkb, chi + static_cast<int64_t>(w) * ng * ng, mode, bi, bj,
                                        lds);
        return;
    }
    const int u = b - n_main, j = u / parts, p = u % parts;
    rect_item_tile(n_main + j, wl, nb, order, w, bi, bj);
    if (bj * kTJ >= ng) return;  // nothing of it is ever read
    const int kb0 = p * nkb / parts, kb1 = (p + 1) * nkb / parts;
    sbf16_tile<F, S, NWI, NWJ, BI, BJ, true, RV>(
        sa + kb0 * blk, siga + static_cast<size_t>(kb0) * ngp, sb_all + w * plane + kb0 * blk,
        sigb_all + (static_cast<size_t>(w) * nkb + kb0) * ngp, ng, ngp, kb1 - kb0,
        ws + static_cast<int64_t>(u) * kTI * kTJ, 0, bi, bj, lds);
}

// chi_w[tile] (=|+=) the sum of the parts of tail item n_main + blockIdx.y,
// added in part order.
__global__ __launch_bounds__(256) void sbf16_tail_reduce_kernel(
    const double2* __restrict__ ws, int parts, int n_main, WList wl, int nb,
    const int* __restrict__ order, double2* __restrict__ chi, int ng, int mode) {
    const int j = blockIdx.y, e = blockIdx.x * 256 + threadIdx.x;
    int w, bi, bj;
    rect_item_tile(n_main + j, wl, nb, order, w, bi, bj);
    const int gi = bi * kTI + e / kTJ, gj = bj * kTJ + e % kTJ;
    if (gi >= ng || gj >= ng) return;
    const double2* src = ws + static_cast<int64_t>(j) * parts * kTI * kTJ + e;
    double2 acc = src[0];
    for (int p = 1; p < parts; ++p) {
        const double2 v = src[static_cast<int64_t>(p) * kTI * kTJ];
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

// Persistent: workgroups pull items (problem, frequency, 128-row block,
// 64-column block) from *counter until none is left.
template <int S, int NWI, int NWJ, int BI, int BJ, int RV>
__global__ __launch_bounds__(NWI* NWJ * 64) void chi0_sbf16_batched_kernel(
    const SbDesc* __restrict__ qd, const int4* __restrict__ items, int nitems,
    int* __restrict__ counter) {
    extern __shared__ u32x4 lds[];
    __shared__ int s_item;
    for (;;) {
        __syncthreads();  // every wave is done with the previous item's LDS
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int it = s_item;
        if (it >= nitems) break;
        const int4 t = items[it];
        const SbDesc d = qd[t.x];
        if (t.w * kTJ >= d.ng) continue;
        const size_t plane = static_cast<size_t>(d.nkb) * ksteps<SlBf16>() * S * d.ng * 2;
        sbf16_tile<SlBf16, S, NWI, NWJ, BI, BJ, false, RV>(
            reinterpret_cast<const u32x4*>(d.sa), d.siga,
            reinterpret_cast<const u32x4*>(d.sb) + t.y * plane,
            d.sigb + static_cast<size_t>(t.y) * d.nkb * d.ngp, d.ng, d.ngp, d.nkb,
            d.chi + static_cast<int64_t>(t.y) * d.ng * d.ng, d.mode, t.z, t.w, lds);
    }
}

template <class F, int S, int NWI, int NWJ, int BI, int BJ, int RV>
void launch_sbf16_t(const uint32_t* sa, const double* siga, const uint32_t* sb,
                    const double* sigb, int ng, int ngp, int nkb, const WList& wl, double2* chi,
                    bool accumulate, int nb, int n_main, int parts, double2* ws, int grid,
                    hipStream_t s) {
    const size_t lds = SbGeom<S, NWI * NWJ, RV>::lds_bytes;
    auto fn = chi0_sbf16_kernel<F, S, NWI, NWJ, BI, BJ, RV>;
    GW_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   static_cast<int>(lds)));
    hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(grid)), dim3(NWI * NWJ * 64), lds, s,
                       reinterpret_cast<const u32x4*>(sa), siga, reinterpret_cast<const u32x4*>(sb),
                       sigb, ng, ngp, nkb, wl, chi, accumulate ? 1 : 0, nb, tile_order(nb, 4),
                       n_main, parts, ws);
}

// Workgroups of the S-slice contraction resident on one CU.
template <int S, int NWI, int NWJ, int BI, int BJ, int RV>
int sbf16_per_cu_t() {
    const size_t lds = SbGeom<S, NWI * NWJ, RV>::lds_bytes;
    const void* fn =
        reinterpret_cast<const void*>(chi0_sbf16_kernel<SlBf16, S, NWI, NWJ, BI, BJ, RV>);
    GW_HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   static_cast<int>(lds)));
    int n = 0;
    GW_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, NWI * NWJ * 64, lds));
    return std::max(1, n);
}

}  // namespace

// Workgroups of the S-slice contraction (ring variant rv) resident on the
// current device.
int sbf16_slots(int S, int rv) {
    static std::mutex mu;
    static std::map<std::tuple<int, int, int>, int> cache;  // (device, S, rv) -> slots
    int dev = 0;
    GW_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    int& n = cache[{dev, S, rv}];
    if (n > 0) return n;
    int per_cu = 1, cus = 0;
    auto pick = [&](auto rvc) {
        constexpr int R = decltype(rvc)::value;
        switch (S) {
            case 2: per_cu = sbf16_per_cu_t<2, 4, 2, 1, 1, R>(); break;
            case 3: per_cu = sbf16_per_cu_t<3, 4, 2, 1, 1, R>(); break;
            case 4: per_cu = sbf16_per_cu_t<4, 4, 2, 1, 1, R>(); break;
            case 5: per_cu = sbf16_per_cu_t<5, 4, 2, 1, 1, R>(); break;
            default: per_cu = sbf16_per_cu_t<6, 4, 2, 1, 1, R>(); break;
        }
    };
    if (rv == 1)
        pick(std::integral_constant<int, 1>{});
    else
        pick(std::integral_constant<int, 0>{});
    GW_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    n = per_cu * std::max(1, cus);
    return n;
}


// Bytes of the layout sbf16_desc describes: A slices, A sigma, nz B slices,
// nz B sigma, each rounded up to 256 B (f16: the FP16 9-bit format).
size_t sbf16_scratch_bytes(int64_t kc, int ng, int nz, int S, bool f16) {
    const int kbp = f16 ? SlF16x9::KB : SlBf16::KB;
    const int64_t nkb = (kc + kbp - 1) / kbp;
    const int ngp = ceil_div(ng, kTI) * kTI;
    const size_t per_b = (static_cast<size_t>(nkb) * (kbp / kStep) * S * ng * kStep * 4 + 255) &
                         ~static_cast<size_t>(255);
    const size_t sig_b =
        (static_cast<size_t>(nkb) * ngp * sizeof(double) + 255) & ~static_cast<size_t>(255);
    return (per_b + sig_b) * static_cast<size_t>(1 + nz);
}

SbDesc sbf16_desc(int S, int64_t kc, int ng, int nz, void* scratch, bool f16) {
    const int kbp = f16 ? SlF16x9::KB : SlBf16::KB;
    const int nkb = static_cast<int>((kc + kbp - 1) / kbp);
    const int ngp = ceil_div(ng, kTI) * kTI;
    const size_t per_b = (static_cast<size_t>(nkb) * (kbp / kStep) * S * ng * kStep * 4 + 255) &
                         ~static_cast<size_t>(255);
    const size_t sig_b =
        (static_cast<size_t>(nkb) * ngp * sizeof(double) + 255) & ~static_cast<size_t>(255);
    char* base = static_cast<char*>(scratch);
    SbDesc d{};
    d.sa = reinterpret_cast<const uint32_t*>(base);
    d.siga = reinterpret_cast<const double*>(base + per_b);
    d.sb = reinterpret_cast<const uint32_t*>(base + per_b + sig_b);
    d.sigb = reinterpret_cast<const double*>(base + per_b + sig_b + static_cast<size_t>(nz) * per_b);
    d.ng = ng;
    d.ngp = ngp;
    d.nkb = nkb;
    return d;
}

SbDesc launch_sbf16_prep(int S, const double2* m, int64_t kc, int ng, const double2* delta,
                         int nz, const WList& wl, void* scratch, hipStream_t s, bool f16) {
    const SbDesc d = sbf16_desc(S, kc, ng, nz, scratch, f16);
    ProfScope ps("split_prep", s);
    auto run = [&](auto fmt) {
        using F = decltype(fmt);
        hipLaunchKernelGGL(sbf16_prep_kernel<F>, dim3(d.ngp / prep_cols<F>(), d.nkb), dim3(256), 0,
                           s, m, delta, kc, ng, d.ngp, S, d.nkb, wl, const_cast<uint32_t*>(d.sa),
                           const_cast<double*>(d.siga), const_cast<uint32_t*>(d.sb),
                           const_cast<double*>(d.sigb));
    };
    if (f16)
        run(SlF16x9{});
    else
        run(SlBf16{});
    GW_HIP_TRY(hipGetLastError());
    return d;
}

size_t sbf16_tail_bytes() {
    int slots = 0;
    for (int S = 2; S <= 6; ++S)
        for (int rv = 0; rv < kNumSplitVariants; ++rv) slots = std::max(slots, sbf16_slots(S, rv));
    return static_cast<size_t>(slots) * kTI * kTJ * sizeof(double2);
}

void launch_chi0_sbf16(int S, const double2* m, int64_t kc, int ng, const double2* delta, int nz,
                       const WList& wl, double2* chi, bool accumulate, void* scratch,
                       hipStream_t s, double2* tail_ws, bool f16, int variant) {
    if (variant < 0 || variant >= kNumSplitVariants) variant = 0;
    if (kc <= 0 || wl.nh + wl.nf == 0) return;
    if (S < 2 || S > (f16 ? SlF16x9::SMAX : SlBf16::SMAX))
        throw Error{-4, f16 ? "split FP16 supports 2..4 slices" : "split BF16 supports 2..6 slices"};
    const SbDesc d = launch_sbf16_prep(S, m, kc, ng, delta, nz, wl, scratch, s, f16);
    const int nb = ceil_div(ng, kTI);
    const int64_t nitems = 2 * (static_cast<int64_t>(wl.nh) * (nb * (nb + 1) / 2) +
                                static_cast<int64_t>(wl.nf) * nb * nb);
    if (nitems >= (int64_t(1) << 30)) throw Error{-4, "too many chi tiles for one launch"};
    // A last round of workgroups that fills at most half the chip is cut
    // along the 128-pair blocks (as in launch_chi0_f64).
    int n_main = static_cast<int>(nitems), parts = 1, n_tail = 0;
    if (tail_ws) {
        const int slots = sbf16_slots(S, variant);
        const int rem = static_cast<int>(nitems % slots);
        const int pc = std::min(rem > 0 ? slots / rem : 0, d.nkb);
        if (rem > 0 && 2 * rem <= slots && pc >= 2) {
            n_tail = rem;
            parts = pc;
            n_main = static_cast<int>(nitems) - rem;
        }
    }
    const int grid = n_main + n_tail * parts;
    {
        ProfScope ps("chi0_split", s);
        auto run = [&](auto fmt, auto sc, auto rvc) {
            using F = decltype(fmt);
            launch_sbf16_t<F, decltype(sc)::value, 4, 2, 1, 1, decltype(rvc)::value>(
                d.sa, d.siga, d.sb, d.sigb, ng, d.ngp, d.nkb, wl, chi, accumulate, nb, n_main,
                parts, tail_ws, grid, s);
        };
        auto by_s = [&](auto fmt, auto rvc) {
            switch (S) {
                case 2: run(fmt, std::integral_constant<int, 2>{}, rvc); break;
                case 3: run(fmt, std::integral_constant<int, 3>{}, rvc); break;
                case 4: run(fmt, std::integral_constant<int, 4>{}, rvc); break;
                case 5:
                    if constexpr (decltype(fmt)::SMAX >= 5) run(fmt, std::integral_constant<int, 5>{}, rvc);
                    break;
                default:
                    if constexpr (decltype(fmt)::SMAX >= 6) run(fmt, std::integral_constant<int, 6>{}, rvc);
                    break;
            }
        };
        auto by_rv = [&](auto fmt) {
            if (variant == 1)
                by_s(fmt, std::integral_constant<int, 1>{});
            else
                by_s(fmt, std::integral_constant<int, 0>{});
        };
        if (f16)
            by_rv(SlF16x9{});
        else
            by_rv(SlBf16{});
        GW_HIP_TRY(hipGetLastError());
    }
    if (n_tail > 0) {
        ProfScope ps("chi0_split_tail", s);
        hipLaunchKernelGGL(sbf16_tail_reduce_kernel, dim3(kTI * kTJ / 256, n_tail), dim3(256), 0,
                           s, tail_ws, parts, n_main, wl, nb, tile_order(nb, 4), chi, ng,
                           accumulate ? 1 : 0);
        GW_HIP_TRY(hipGetLastError());
    }
}

namespace {
template <int S, int RV>
void launch_sbf16_batched_s(const SbDesc* qd, const int4* items, int nitems, int* counter, int grid,
                            hipStream_t s) {
    constexpr int NWI = 4, NWJ = 2;
    const size_t lds = SbGeom<S, NWI * NWJ, RV>::lds_bytes;
    auto fn = chi0_sbf16_batched_kernel<S, NWI, NWJ, 1, 1, RV>;
    GW_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   static_cast<int>(lds)));
    hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(grid)), dim3(NWI * NWJ * 64), lds, s, qd,
                       items, nitems, counter);
}
}  // namespace

void launch_chi0_sbf16_batched(int S, const SbDesc* qd, const int4* items, int nitems,
                               int* counter, int grid, hipStream_t s, int variant) {
    if (nitems <= 0) return;
    if (S < 2 || S > 6) throw Error{-4, "split precision supports 2..6 slices"};
    grid = std::max(1, std::min(grid, nitems));
    ProfScope ps("chi0_split_batched", s);
    auto by_s = [&](auto rvc) {
        constexpr int R = decltype(rvc)::value;
        switch (S) {
            case 2: launch_sbf16_batched_s<2, R>(qd, items, nitems, counter, grid, s); break;
            case 3: launch_sbf16_batched_s<3, R>(qd, items, nitems, counter, grid, s); break;
            case 4: launch_sbf16_batched_s<4, R>(qd, items, nitems, counter, grid, s); break;
            case 5: launch_sbf16_batched_s<5, R>(qd, items, nitems, counter, grid, s); break;
            default: launch_sbf16_batched_s<6, R>(qd, items, nitems, counter, grid, s); break;
        }
    };
    if (variant == 1)
        by_s(std::integral_constant<int, 1>{});
    else
        by_s(std::integral_constant<int, 0>{});
    GW_HIP_TRY(hipGetLastError());
}

}  // namespace gw
