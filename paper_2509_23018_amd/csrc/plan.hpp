// Per-(grid, G-list) plan of the pruned transform used by MTXEL and its
// adjoint, and the host entry points of the kernels (internal to libgw).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <vector>

namespace gw {

// Pairs handled by one launch: pair k (0-based within the launch) is
// lin = k_off + k, v = v0 + lin / cw, c = c0 + lin % cw.
struct PairMap {
    int64_t k_off;
    int32_t cw;
    int32_t v0;
    int32_t c0;
};

// A rectangle of pairs: v in [v0, v0+nv), c in [c0, c0+nc); pair row
// k = (v - v0)*nc + (c - c0).
struct Rect {
    int32_t v0, nv, c0, nc;
};

// Pruned 3D DFT on the G-sphere.  The transform of a pair density rho(j1,j2,j3)
// is taken axis by axis, keeping on each axis only the frequencies some G
// needs:
//   stage z : T1[j1][j2][k3]  = sum_j3 e^{+2 pi i k3 j3/N3} rho[j1][j2][j3]
//   stage y : T2[j1][k2][k3]  = sum_j2 e^{+2 pi i k2 j2/N2} T1[j1][j2][k3]
//             (kept only on the "disc", the distinct (k2,k3) of the G list)
//   stage x : M(G)            = dV * sum_j1 e^{+2 pi i k1 j1/N1} T2[j1][disc(G)]
// The forward stages z and y run on real twiddles: with a = min(k, N - k) the
// class of a frequency k, C_a = sum_j cos(2 pi a j/N) x_j and S_a = sum_j
// sin(2 pi a j/N) x_j give the transform at k = a as C_a + i S_a and at
// k = N - a as C_a - i S_a, so a pair of conjugate frequencies costs two
// products with real coefficients instead of two complex ones.  Classes are
// packed 8 to a 16-wide block: slot c < 8 holds the cosine of class 8b + c,
// slot c + 8 its sine (stage z: columns of the B operand, stages y and x: rows
// of the A operand).
struct MtxelPlan {
    int n[3] = {0, 0, 0};
    int64_t nr = 0;
    int ng = 0;
    int m1 = 0, m2 = 0, m3 = 0;    // distinct k1, k2, k3 values
    int nb1 = 0, nb2 = 0, nb3 = 0; // 16-wide blocks covering them
    int mh1 = 0, mh2 = 0, mh3 = 0;    // distinct k1, k2, k3 classes min(k, N - k)
    int nbh1 = 0, nbh2 = 0, nbh3 = 0; // 8-class blocks covering them (forward stages x, y, z)
    int n1p = 0;          // N1 rounded up to 4
    int n23p = 0;         // disc size rounded up to 16
    int n2p = 0, n3p = 0; // N2 rounded up to 16, N3 rounded up to 16
    int n23 = 0;          // disc size
    size_t lds_yz = 0;    // dynamic LDS of the fused product + z + y kernel
    int ring = 3;         // slab slots of that kernel's LDS ring (2 where 3 do not fit)
    size_t lds_x = 0;     // dynamic LDS of the x-stage kernel

    std::vector<int32_t> gvec;  // host copy (cache key)

    // device tables (owned)
    double* w1re = nullptr;     // [n1p/4][64][nbh1]     stage-x MFMA A operand (cos | sin), lane layout
    int* gmapf = nullptr;       // [nbh1*8][2][n23p] (k1 class, sign, disc index) -> G index or -1
    double* w3re = nullptr;     // [n3p/4][64][nbh3]     stage-z MFMA B operand (cos | sin), lane layout
    double* w2re = nullptr;     // [n2p/4][64][nbh2]     stage-y MFMA A operand (cos | sin), lane layout
    int* boxf = nullptr;        // [nbh2*8][2][nbh3*16] (k2 class, sign, stage-y column) -> disc or -1
    // used by the adjoint (the transposed stages, e^{-2 pi i k j/N} as P cos + Q sin)
    int n1p16 = 0;              // N1 rounded up to 16
    double* w1ir = nullptr;     // [n1p16/16][nbh1*4][64] adjoint stage-x MFMA A operand (cos | sin)
    double* w2ir = nullptr;     // [n2p/16][nbh2*4][64]   adjoint stage-y MFMA A operand (cos | sin)
    double* w3ir = nullptr;     // [nbh3*4][n3p/16][64]   adjoint stage-z MFMA B operand (cos | sin)
    int* boxi = nullptr;        // [nbh2*16][nbh3*16] adjoint stage-z gather -> disc index or -1

    int device = 0;
    hipEvent_t last_use = nullptr;  // recorded after the last enqueued work that read the tables

    void release();  // frees the tables now (the caller knows no work reads them)
};

using PlanRef = std::shared_ptr<MtxelPlan>;

// Build (or fetch from the per-device cache) the plan for this grid and G list.
// Throws gw::Error on invalid input or unsupported size, and in no-allocation
// mode when the plan does not exist yet.  The cache keeps at most 256 plans
// per device; a plan dropped from it stays alive while a PlanRef holds it and
// its tables are freed once the work recorded in last_use has completed.
PlanRef get_plan(const int n[3], const int32_t* gvec, int ng);
// Record that work just enqueued on s reads the plan's tables (no-op while s
// is capturing a graph: a captured graph holds its own PlanRefs).
void mark_plan_used(MtxelPlan& p, hipStream_t s);
void release_plans();

// MTXEL launches: m_out[k][i] = M_{pair k}(G_i) for the pairs of rc, at output
// row k = (v - v0)*ldm + (c - c0) (ldm = 0: rc.nc, the rectangle's own
// row-major order).  t2 is scratch of t2_elems(plan, pairs).
size_t t2_elems(const MtxelPlan& p, int64_t npairs);
void launch_mtxel(const MtxelPlan& p, const double2* psi_v, const double2* psi_c, Rect rc,
                  double volume, double2* t2, double2* m_out, hipStream_t s, int64_t ldm = 0);

}  // namespace gw
