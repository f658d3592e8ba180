// Reduced-precision CHI0 contractions on gfx950 (FP64 everywhere except the
// products of the contraction itself; not in the paper, which is FP64 only).
//
// Split BF16/FP16 ("fixed-point slices"): after the FP64 energy-factor
// scaling, every operand x is cut, per block of kBlk pairs and per G, into
// S integer slices with a common exponent e (|Re x|, |Im x| < 2^e over the
// block):  x = 2^(e-8) * sum_s q_s 2^(-8 s) (+ residual), q_0 in [-256, 256],
// q_s>0 in [-128, 128] (round to nearest each time).  The slices are stored
// as the integers q_s, exact in BF16 and FP16.  Slice products with
// a + b <= S - 1 run on MFMA with FP32 accumulation, one accumulator per
// shift t = a + b: over a block of 64 pairs the integer sums of t = 0, 1, 2
// stay <= 2^24 (exact); for t >= 3 the FP32 rounding is relative to terms
// below 2^-24 of the result.  After each block the accumulators are combined
// as 2^(eA+eB-16) sum_t 2^(-8t) acc_t in FP64; chi is accumulated in FP64.
//
// FP32: operands rounded to FP32 (after the FP64 energy factor), FP32 MFMA
// products and sums over blocks of kBlk32 pairs, FP64 across blocks.
#include <algorithm>
#include <cmath>

#include "chi0.hpp"
#include "items.hpp"
#include "common.hpp"
#include "prof.hpp"

namespace gw {

namespace {

constexpr int kBlk = 64;       // pairs per exponent block / exact accumulation block
constexpr int kKs = 32;        // pairs per MFMA k-step (16x16x32)
constexpr int kSRow = 40;      // LDS row stride (16-bit elements): 80 B, bank-conflict free

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <typename E>
struct MfmaOp;
template <>
struct MfmaOp<__bf16> {
    static __device__ __forceinline__ f32x4 run(u32x4 a, u32x4 b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
    }
};
template <>
struct MfmaOp<_Float16> {
    static __device__ __forceinline__ f32x4 run(u32x4 a, u32x4 b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                      __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
    }
};

__device__ __forceinline__ f32x4 zf4() { return f32x4{0.f, 0.f, 0.f, 0.f}; }

// ---------------------------------------------------------------- slicing

// One workgroup per (block of kBlk pairs, 64 columns of G): the M tile is
// staged in LDS once and sliced for operand A (M itself) and for every
// frequency's operand B (delta_w[k] M[k][g], FP64).  Per operand and column:
// exponent e with max(|Re|, |Im|) < 2^e over the block, then the S integer
// slices.  Outputs (16-bit, pairs past kc are 0):
//   A: slices_a [nkb][S][2 planes][ng][kBlk], sigma_a [nkb][ng] = 2^(e-8)
//   B: slices_b [nz][nkb][S][2][ng][kBlk],    sigma_b [nz][nkb][ng]
// Stores are coalesced: 64 consecutive lanes write one 64-pair row.
template <typename E>
__global__ __launch_bounds__(256) void split_prep_kernel(
    const double2* __restrict__ m, const double2* __restrict__ delta, int64_t kc, int ng, int S,
    int nkb, WList wl, E* __restrict__ slices_a, double* __restrict__ sigma_a,
    E* __restrict__ slices_b, double* __restrict__ sigma_b) {
    static_assert(kBlk == 64, "one lane per pair of the block");
    __shared__ double2 s_m[kBlk][65];
    __shared__ double s_part[4][64];
    __shared__ int s_e[64];
    const int tid = threadIdx.x, lane = tid & 63, quarter = tid >> 6;
    const int g0 = blockIdx.x * 64, kb = blockIdx.y;
    const int64_t k0 = static_cast<int64_t>(kb) * kBlk;
    const int kn = static_cast<int>(std::min<int64_t>(kBlk, kc - k0));
    // stage M[k0 .. k0+64)[g0 .. g0+64): lanes along g (coalesced)
    for (int r = quarter; r < kBlk; r += 4) {
        const int g = g0 + lane;
        s_m[r][lane] = (r < kn && g < ng) ? m[(k0 + r) * ng + g] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const size_t plane = static_cast<size_t>(ng) * kBlk;
    const int nop = 1 + wl.nh + wl.nf;
    for (int op = 0; op < nop; ++op) {
        const double2* dw = op == 0 ? nullptr : delta + static_cast<int64_t>(wl.w[op - 1]) * kc;
        auto value = [&](int p, int c) {
            const double2 x = s_m[p][c];
            return (dw && p < kn) ? cmul(dw[k0 + p], x) : x;
        };
        // per-column maxima: lane = column, quarter = 16 pairs
        double mx = 0.0;
        for (int p = quarter * 16; p < quarter * 16 + 16; ++p) {
            const double2 x = value(p, lane);
            mx = fmax(mx, fmax(fabs(x.x), fabs(x.y)));
        }
        s_part[quarter][lane] = mx;
        __syncthreads();
        if (quarter == 0) {
            mx = fmax(fmax(s_part[0][lane], s_part[1][lane]), fmax(s_part[2][lane], s_part[3][lane]));
            int e = 0;
            if (mx > 0.0) (void)frexp(mx, &e);  // mx = f 2^e, f in [0.5, 1): |x| < 2^e
            s_e[lane] = e;
            if (g0 + lane < ng) {
                const double sg = ldexp(1.0, e - 8);
                if (op == 0)
                    sigma_a[static_cast<size_t>(kb) * ng + g0 + lane] = sg;
                else
                    sigma_b[(static_cast<size_t>(wl.w[op - 1]) * nkb + kb) * ng + g0 + lane] = sg;
            }
        }
        __syncthreads();
        // slices: lane = pair, columns quarter, quarter + 4, ...
        E* out = op == 0 ? slices_a
                         : slices_b + static_cast<size_t>(wl.w[op - 1]) * nkb * S * 2 * plane;
        out += static_cast<size_t>(kb) * S * 2 * plane;
        for (int c = quarter; c < 64; c += 4) {
            const int g = g0 + c;
            if (g >= ng) continue;
            const int e = s_e[c];
            double rr = 0.0, ri = 0.0;
            if (lane < kn) {
                const double2 x = value(lane, c);
                rr = ldexp(x.x, 8 - e);
                ri = ldexp(x.y, 8 - e);
            }
            E* o = out + static_cast<size_t>(g) * kBlk + lane;
            for (int sl = 0; sl < S; ++sl) {
                const double qr = rint(rr), qi = rint(ri);
                // integers |q| <= 256: exact in BF16 and FP16
                o[(static_cast<size_t>(sl) * 2 + 0) * plane] = static_cast<E>(qr);
                o[(static_cast<size_t>(sl) * 2 + 1) * plane] = static_cast<E>(qi);
                rr = (rr - qr) * 256.0;
                ri = (ri - qi) * 256.0;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- split contraction

// Same work items as the FP64 kernel (64x64 tiles of chi_w).  8 waves in a
// 2 x 4 layout, each a 32 x 16 sub-tile (2 MFMA blocks).  Per k-step of 32
// pairs the tile's slices of both operands are staged in LDS.
template <typename E, int S>
__global__ __launch_bounds__(512) void chi0_split_kernel(
    const E* __restrict__ sa_, const double* __restrict__ siga, const E* __restrict__ sb_all,
    const double* __restrict__ sigb_all, int64_t kc, int ng, int nkb, WList wl,
    double2* __restrict__ chi, int mode, int nb, const int* __restrict__ order) {
    constexpr int T = 64;
    int w, bi, bj;
    decode_item(blockIdx.x, wl, nb, order, w, bi, bj);
    // LDS: [2 operands][S][2 planes][64 rows][kSRow]
    __shared__ __attribute__((aligned(16))) E lds[2 * S * 2 * T * kSRow];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63, row = lane & 15, kg = lane >> 4;
    const int wi = wave >> 2, wj = wave & 3;  // rows wi*32 .. +32, cols wj*16 .. +16
    const int i0 = bi * T, j0 = bj * T;
    const size_t plane = static_cast<size_t>(ng) * kBlk;
    const E* sb_ = sb_all + static_cast<size_t>(w) * nkb * S * 2 * plane;
    const double* sigb = sigb_all + static_cast<size_t>(w) * nkb * ng;

    dbl4 acc_r[2], acc_i[2];
    acc_r[0] = acc_r[1] = acc_i[0] = acc_i[1] = zero4();

    // staging: 2 operands x S x 2 planes x 64 rows x 4 chunks of 16 B
    constexpr int NCHUNK = 2 * S * 2 * T * 4;
    for (int kb = 0; kb < nkb; ++kb) {
        f32x4 c_r[S][2], c_i[S][2];  // one accumulator per shift t = a + b
#pragma unroll
        for (int g3 = 0; g3 < S; ++g3)
#pragma unroll
            for (int x = 0; x < 2; ++x) c_r[g3][x] = c_i[g3][x] = zf4();
        for (int ks = 0; ks < kBlk / kKs; ++ks) {
            __syncthreads();
            for (int c = tid; c < NCHUNK; c += 512) {
                const int ch = c & 3, rr = (c >> 2) % T, pl = (c / (4 * T)) & 1;
                const int s = (c / (8 * T)) % S, op = c / (8 * T * S);
                const int gcol = min((op == 0 ? i0 : j0) + rr, ng - 1);
                const E* src = (op == 0 ? sa_ : sb_) + (static_cast<size_t>(kb) * S * 2 + s * 2 + pl) * plane +
                               static_cast<size_t>(gcol) * kBlk + ks * kKs + ch * 8;
                const u32x4 v = *reinterpret_cast<const u32x4*>(src);
                *reinterpret_cast<u32x4*>(&lds[(((op * S + s) * 2 + pl) * T + rr) * kSRow + ch * 8]) = v;
            }
            __syncthreads();
            // B fragments: rows j0 + wj*16 + row, k = 8*kg .. +7
#pragma unroll
            for (int a = 0; a < S; ++a) {
                u32x4 ar[2], ai[2], an[2];
#pragma unroll
                for (int x = 0; x < 2; ++x) {
                    const int rr = wi * 32 + x * 16 + row;
                    ar[x] = *reinterpret_cast<const u32x4*>(&lds[((a * 2 + 0) * T + rr) * kSRow + kg * 8]);
                    ai[x] = *reinterpret_cast<const u32x4*>(&lds[((a * 2 + 1) * T + rr) * kSRow + kg * 8]);
                    an[x] = ai[x] ^ u32x4{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
                }
#pragma unroll
                for (int b = 0; b < S - a; ++b) {
                    const int grp = a + b;
                    const int rr = wj * 16 + row;
                    const u32x4 br = *reinterpret_cast<const u32x4*>(
                        &lds[(((S + b) * 2 + 0) * T + rr) * kSRow + kg * 8]);
                    const u32x4 bim = *reinterpret_cast<const u32x4*>(
                        &lds[(((S + b) * 2 + 1) * T + rr) * kSRow + kg * 8]);
#pragma unroll
                    for (int x = 0; x < 2; ++x) {
                        // conj(A) B: re = Ar Br + Ai Bi, im = Ar Bi - Ai Br
                        c_r[grp][x] = MfmaOp<E>::run(ar[x], br, c_r[grp][x]);
                        c_r[grp][x] = MfmaOp<E>::run(ai[x], bim, c_r[grp][x]);
                        c_i[grp][x] = MfmaOp<E>::run(ar[x], bim, c_i[grp][x]);
                        c_i[grp][x] = MfmaOp<E>::run(an[x], br, c_i[grp][x]);
                    }
                }
            }
        }
        // flush this block into FP64: sigmaA_i sigmaB_j sum_t 2^(-8t) acc_t
        const int gj = min(j0 + wj * 16 + row, ng - 1);
        const double sbj = sigb[static_cast<size_t>(kb) * ng + gj];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int gi = min(i0 + wi * 32 + x * 16 + 4 * kg + t, ng - 1);
                const double sc = siga[static_cast<size_t>(kb) * ng + gi] * sbj;
                double vr = 0.0, vi = 0.0;
#pragma unroll
                for (int g3 = S - 1; g3 >= 0; --g3) {
                    vr = vr * (1.0 / 256.0) + static_cast<double>(c_r[g3][x][t]);
                    vi = vi * (1.0 / 256.0) + static_cast<double>(c_i[g3][x][t]);
                }
                acc_r[x][t] += sc * vr;
                acc_i[x][t] += sc * vi;
            }
    }
    double2* cw = chi + static_cast<int64_t>(w) * ng * ng;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int gi = i0 + wi * 32 + x * 16 + 4 * kg + t;
            const int gj = j0 + wj * 16 + row;
            if (gi < ng && gj < ng) {
                double2* p = cw + static_cast<int64_t>(gi) * ng + gj;
                double2 v = make_double2(acc_r[x][t], acc_i[x][t]);
                if (mode) {
                    const double2 o = *p;
                    v.x += o.x;
                    v.y += o.y;
                }
                *p = v;
            }
        }
}

template <typename E, int S>
void launch_split_t(const E* sa, const double* siga, const E* sb, const double* sigb,
                    int64_t kc, int ng, int nkb, const WList& wl, double2* chi, bool accumulate,
                    int nb, int64_t nitems, hipStream_t s) {
    hipLaunchKernelGGL((chi0_split_kernel<E, S>), dim3(static_cast<unsigned>(nitems)), dim3(512), 0,
                       s, sa, siga, sb, sigb, kc, ng, nkb, wl, chi, accumulate ? 1 : 0, nb,
                       tile_order(nb));
}

template <typename E>
void launch_split_s(int S, const E* sa, const double* siga, const E* sb, const double* sigb,
                    int64_t kc, int ng, int nkb, const WList& wl, double2* chi, bool accumulate,
                    int nb, int64_t nitems, hipStream_t s) {
    switch (S) {
        case 2: launch_split_t<E, 2>(sa, siga, sb, sigb, kc, ng, nkb, wl, chi, accumulate, nb, nitems, s); break;
        case 3: launch_split_t<E, 3>(sa, siga, sb, sigb, kc, ng, nkb, wl, chi, accumulate, nb, nitems, s); break;
        case 4: launch_split_t<E, 4>(sa, siga, sb, sigb, kc, ng, nkb, wl, chi, accumulate, nb, nitems, s); break;
        case 5: launch_split_t<E, 5>(sa, siga, sb, sigb, kc, ng, nkb, wl, chi, accumulate, nb, nitems, s); break;
        case 6: launch_split_t<E, 6>(sa, siga, sb, sigb, kc, ng, nkb, wl, chi, accumulate, nb, nitems, s); break;
        default: throw Error{-4, "split precision supports 2..6 slices"};
    }
}


// ---------------------------------------------------------------- FP32 contraction

constexpr int kBlk32 = 64;  // pairs per FP32 accumulation block

__device__ __forceinline__ f32x4 mfma_f32(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// 64x64 tile per workgroup, 4 waves (2x2) of 32x32.  Operands rounded to
// FP32 when staged (the G' side after the FP64 energy factor); FP32 MFMA
// 16x16x4 (lane l: A[l%16][l/16], B[l/16][l%16], D[4*(l/16)+t][l%16]);
// every kBlk32 pairs the FP32 accumulators are added into FP64.  Stages of
// KT pairs are double-buffered in LDS: the global loads of stage st + 1 are
// issued before the MFMAs of stage st and converted and written to the other
// buffer after them.  Loads are unconditional (pair rows past the chunk end
// clamped, their G' side zeroed at the write; columns past N_G clamped and
// only feeding outputs that are not stored).
__global__ __launch_bounds__(256) void chi0_f32_kernel(const double2* __restrict__ m, int64_t kc,
                                                       int ng, const double2* __restrict__ delta,
                                                       WList wl, double2* __restrict__ chi,
                                                       int mode, int nb,
                                                       const int* __restrict__ order) {
    constexpr int T = 64, KT = 16, NL = KT * T / 256;
    static_assert(kBlk32 % KT == 0, "FP32 blocks must hold whole stages");
    int w, bi, bj;
    decode_item(blockIdx.x, wl, nb, order, w, bi, bj);
    __shared__ float2 s_a[2][KT][T], s_b[2][KT][T];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63, row = lane & 15, kq = lane >> 4;
    const int wi = wave >> 1, wj = wave & 1;
    const int i0 = bi * T, j0 = bj * T;
    const double2* dw = delta + static_cast<int64_t>(w) * kc;
    const int cc = tid & 63, kk0 = tid >> 6;
    const int64_t ci = min(i0 + cc, ng - 1), cj = min(j0 + cc, ng - 1);

    dbl4 accr[2][2], acci[2][2];
    f32x4 fr[2][2], fi[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            accr[a][b] = acci[a][b] = zero4();
            fr[a][b] = fi[a][b] = zf4();
        }

    // stage registers: the G row, the G' row and Delta for NL pair rows
    double ar[NL], ai[NL], br[NL], bim[NL], dr[NL], di[NL];
    auto fetch = [&](int64_t kbase) {
#pragma unroll
        for (int u = 0; u < NL; ++u) {
            const int64_t k = kbase + kk0 + 4 * u;
            const int64_t kr = k < kc ? k : kc - 1;
            const double2* pa = m + kr * ng + ci;
            const double2* pb = m + kr * ng + cj;
            ar[u] = pa->x;  // component loads: no fused global-to-LDS copy
            ai[u] = pa->y;
            br[u] = pb->x;
            bim[u] = pb->y;
            dr[u] = dw[kr].x;
            di[u] = dw[kr].y;
        }
    };
    auto stage = [&](int buf, int64_t kbase) {
#pragma unroll
        for (int u = 0; u < NL; ++u) {
            const bool ok = kbase + kk0 + 4 * u < kc;
            const double bx = ok ? dr[u] * br[u] - di[u] * bim[u] : 0.0;
            const double by = ok ? dr[u] * bim[u] + di[u] * br[u] : 0.0;
            s_a[buf][kk0 + 4 * u][cc] = make_float2(static_cast<float>(ar[u]), static_cast<float>(ai[u]));
            s_b[buf][kk0 + 4 * u][cc] = make_float2(static_cast<float>(bx), static_cast<float>(by));
        }
    };

    fetch(0);
    stage(0, 0);
    __syncthreads();
    const int nsteps = static_cast<int>((kc + KT - 1) / KT);
    int buf = 0;
    for (int st = 0; st < nsteps; ++st) {
        const int64_t knext = static_cast<int64_t>(st + 1) * KT;
        // issue priority 1 for the loads, 2 over the MFMAs, 0 for the stores
        // and the barrier: the wave with MFMAs to issue goes first on the SIMD
        __builtin_amdgcn_s_setprio(1);
        fetch(knext);  // clamped: harmless past the last stage
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_setprio(2);
#pragma unroll
        for (int s = 0; s < KT / 4; ++s) {
            float2 a[2], b[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                a[x] = s_a[buf][s * 4 + kq][wi * 32 + x * 16 + row];
                b[x] = s_b[buf][s * 4 + kq][wj * 32 + x * 16 + row];
            }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    fr[x][y] = mfma_f32(a[x].x, b[y].x, fr[x][y]);
                    fr[x][y] = mfma_f32(a[x].y, b[y].y, fr[x][y]);
                    fi[x][y] = mfma_f32(a[x].x, b[y].y, fi[x][y]);
                    fi[x][y] = mfma_f32(-a[x].y, b[y].x, fi[x][y]);
                }
        }
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_setprio(0);
        if (((st + 1) * KT) % kBlk32 == 0 || st + 1 == nsteps) {
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) {
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        accr[x][y][t] += static_cast<double>(fr[x][y][t]);
                        acci[x][y][t] += static_cast<double>(fi[x][y][t]);
                    }
                    fr[x][y] = fi[x][y] = zf4();
                }
        }
        stage(buf ^ 1, knext);
        __syncthreads();
        buf ^= 1;
    }
    double2* cw = chi + static_cast<int64_t>(w) * ng * ng;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int gi = i0 + wi * 32 + x * 16 + 4 * kq + t;
                const int gj = j0 + wj * 32 + y * 16 + row;
                if (gi < ng && gj < ng) {
                    double2* p = cw + static_cast<int64_t>(gi) * ng + gj;
                    double2 v = make_double2(accr[x][y][t], acci[x][y][t]);
                    if (mode) {
                        const double2 o = *p;
                        v.x += o.x;
                        v.y += o.y;
                    }
                    *p = v;
                }
            }
}

}  // namespace

void launch_chi0_f32(const double2* m, int64_t kc, int ng, const double2* delta, const WList& wl,
                     double2* chi, bool accumulate, hipStream_t s) {
    if (kc <= 0 || wl.nh + wl.nf == 0) return;
    const int nb = ceil_div(ng, 64);
    const int64_t nitems = static_cast<int64_t>(wl.nh) * (nb * (nb + 1) / 2) +
                           static_cast<int64_t>(wl.nf) * nb * nb;
    ProfScope ps("chi0_f32", s);
    hipLaunchKernelGGL(chi0_f32_kernel, dim3(static_cast<unsigned>(nitems)), dim3(256), 0, s, m, kc,
                       ng, delta, wl, chi, accumulate ? 1 : 0, nb, tile_order(nb));
    GW_HIP_TRY(hipGetLastError());
}

size_t split_scratch_bytes(int64_t kmax, int ng, int nz, int S) {
    // the FP16 layout (blocks of kBlk pairs) or the split-BF16 one, whichever is larger
    const int64_t nkb = (kmax + kBlk - 1) / kBlk;
    const size_t per = static_cast<size_t>(nkb) * S * 2 * ng * kBlk * 2 + 256;
    const size_t sig = static_cast<size_t>(nkb) * ng * sizeof(double) + 256;
    return std::max({(per + sig) * static_cast<size_t>(1 + nz), sbf16_scratch_bytes(kmax, ng, nz, S),
                     sbf16_scratch_bytes(kmax, ng, nz, S, true)});
}

void launch_chi0_split(int prec, int S, const double2* m, int64_t kc, int ng,
                       const double2* delta, int nz, const WList& wl, double2* chi,
                       bool accumulate, void* scratch, hipStream_t s, double2* tail_ws,
                       int variant) {
    if (kc <= 0 || wl.nh + wl.nf == 0) return;
    if (S < 2 || S > 6) throw Error{-4, "split precision supports 2..6 slices"};
    if (prec == 2 || prec == 4) {
        launch_chi0_sbf16(S, m, kc, ng, delta, nz, wl, chi, accumulate, scratch, s, tail_ws,
                          prec == 4, variant);
        return;
    }
    const int nkb = static_cast<int>((kc + kBlk - 1) / kBlk);
    const size_t per = static_cast<size_t>(nkb) * S * 2 * ng * kBlk;  // elements
    const size_t per_b = (per * 2 + 255) & ~static_cast<size_t>(255);
    const size_t sig_b = (static_cast<size_t>(nkb) * ng * sizeof(double) + 255) & ~static_cast<size_t>(255);
    char* base = static_cast<char*>(scratch);
    // A slices, A sigma, then per frequency B slices and sigma
    char* pa = base;
    double* siga = reinterpret_cast<double*>(base + per_b);
    char* pb = base + per_b + sig_b;
    double* sigb = reinterpret_cast<double*>(pb + static_cast<size_t>(nz) * per_b);
    const int nbt = ceil_div(ng, 64);
    const int64_t nitems = static_cast<int64_t>(wl.nh) * (nbt * (nbt + 1) / 2) +
                           static_cast<int64_t>(wl.nf) * nbt * nbt;
    auto run = [&](auto tag) {
        using E = decltype(tag);
        {
            ProfScope ps("split_prep", s);
            hipLaunchKernelGGL(split_prep_kernel<E>, dim3(ceil_div(ng, 64), nkb), dim3(256), 0, s, m,
                               delta, kc, ng, S, nkb, wl, reinterpret_cast<E*>(pa), siga,
                               reinterpret_cast<E*>(pb), sigb);
            GW_HIP_TRY(hipGetLastError());
        }
        ProfScope ps("chi0_split", s);
        launch_split_s<E>(S, reinterpret_cast<const E*>(pa), siga,
                          reinterpret_cast<const E*>(pb), sigb, kc, ng, nkb, wl, chi, accumulate,
                          nbt, nitems, s);
        GW_HIP_TRY(hipGetLastError());
    };
    if (prec == 2)
        run(__bf16{});
    else
        run(_Float16{});
}

}  // namespace gw
