// Internal helpers shared by the libgw translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

namespace gw {

typedef double dbl4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- errors

struct Error {
    int status;
    std::string msg;
};

#define GW_HIP_TRY(expr)                                                              \
    do {                                                                              \
        hipError_t e__ = (expr);                                                      \
        if (e__ != hipSuccess) {                                                      \
            (void)hipGetLastError(); /* a reported error must not fail the next call */ \
            throw ::gw::Error{-3, std::string(#expr) + ": " + hipGetErrorString(e__)}; \
        }                                                                             \
    } while (0)

// ---------------------------------------------------------------- complex on double2

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmul_conj_a(double2 a, double2 b) {  // conj(a) * b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// ---------------------------------------------------------------- MFMA FP64 16x16x4
// D[16x16] += A[16x4] * B[4x16].  Lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; it receives D[4*t + l/16][l%16] in element t (t = 0..3)
// (rows interleaved across the four 16-lane groups; measured on gfx950).

__device__ __forceinline__ dbl4 mfma_f64(double a, double b, dbl4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Complex block product acc += A * B on 16x16x4 tiles held as (re, im).
__device__ __forceinline__ void cmfma(dbl4& acc_re, dbl4& acc_im, double ar, double ai, double br,
                                      double bi) {
    acc_re = mfma_f64(ar, br, acc_re);
    acc_re = mfma_f64(-ai, bi, acc_re);
    acc_im = mfma_f64(ar, bi, acc_im);
    acc_im = mfma_f64(ai, br, acc_im);
}

// Complex block product acc += conj(A) * B.
__device__ __forceinline__ void cmfma_conj_a(dbl4& acc_re, dbl4& acc_im, double ar, double ai,
                                             double br, double bi) {
    acc_re = mfma_f64(ar, br, acc_re);
    acc_re = mfma_f64(ai, bi, acc_re);
    acc_im = mfma_f64(ar, bi, acc_im);
    acc_im = mfma_f64(-ai, br, acc_im);
}

__device__ __forceinline__ dbl4 zero4() { return dbl4{0.0, 0.0, 0.0, 0.0}; }

inline int ceil_div(int a, int b) { return (a + b - 1) / b; }
inline int64_t ceil_div64(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace gw
