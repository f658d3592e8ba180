// Host entry points of the CHI0 kernels (internal to libgw).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.hpp"

namespace gw {

constexpr int kMaxZ = 32;  // frequencies per energy-factor launch

struct ZArgs {
    double re[kMaxZ];
    double im[kMaxZ];
    double spin;
    int nz;
};

// delta[w][k] = s * (1/(E_v - E_c + z_w) + 1/(E_v - E_c - z_w)) for the pairs of pm.
void launch_delta(const double* e_v, const double* e_c, PairMap pm, int64_t npairs,
                  const double2* z, int nz, double spin, double2* delta, hipStream_t s);

// Frequencies contracted by one launch: w[0 .. nh) use only the tiles on or
// above the diagonal (Hermitian chi), w[nh .. nh+nf) use every tile.
struct WList {
    int w[kMaxZ];
    int nh;
    int nf;
};

// chi[w] (=|+=) M^H diag(delta[w]) M for every frequency w of wl; M is
// [kc][ng], delta [nz][kc], chi [nz][ng][ng].  variant selects the tile
// shape (0: 64x64, 4 waves; 1: 128x128, 8 waves).  With tail_ws (device,
// chi0_f64_tail_bytes() bytes) a last partial round of tiles is cut along the
// pairs and reduced by a second launch; without it every tile is whole.
void launch_chi0_f64(const double2* m, int64_t kc, int ng, const double2* delta,
                     const WList& wl, double2* chi, bool accumulate, hipStream_t s, int variant,
                     double2* tail_ws = nullptr);
size_t chi0_f64_tail_bytes();  // for the current device
int chi0_variant_tile(int variant);
int chi0_f64_batched_blocks_per_cu(int variant);  // resident workgroups of the persistent kernel
int chi0_forced_variant();  // GW_CHI0_VARIANT, or -1
constexpr int kNumChi0Variants = 2;

// One problem's operands for the batched contraction.
struct QDesc {
    const double2* m;      // [kc][ng]
    const double2* delta;  // [nz][kc]
    double2* chi;          // [nz][ng][ng]
    int64_t kc;
    int ng;
    int mode;              // 0 overwrite, 1 accumulate
};

// Persistent contraction over items (problem, frequency, tile row, tile col);
// counter must be 0 on entry.  grid = number of workgroups to keep resident.
void launch_chi0_f64_batched(const QDesc* qd, const int4* items, int nitems, int* counter,
                             hipStream_t s, int variant, int grid);

// Reduced-precision contractions (same semantics as launch_chi0_f64).
// prec 2 = split BF16, 3 = split FP16, 4 = split FP16 with 9-bit slices, with
// S slices; scratch holds split_scratch_bytes(kc, ng, nz, S) bytes.
size_t split_scratch_bytes(int64_t kmax, int ng, int nz, int S);
void launch_chi0_split(int prec, int S, const double2* m, int64_t kc, int ng,
                       const double2* delta, int nz, const WList& wl, double2* chi,
                       bool accumulate, void* scratch, hipStream_t s,
                       double2* tail_ws = nullptr,  // precisions 2 and 4 (launch_chi0_sbf16)
                       int variant = 0);            // their LDS ring, 0..kNumSplitVariants-1
void launch_chi0_f32(const double2* m, int64_t kc, int ng, const double2* delta, const WList& wl,
                     double2* chi, bool accumulate, hipStream_t s);
constexpr int kSplitTile = 64;  // tile edge of the FP16-split and FP32 kernels
// Split BF16 (f16: split FP16 with 9-bit slices) on the 32x32 MFMA (grouped
// shifts, 128 x 64 workgroup tiles; the Hermitian rule and mirror use
// 128-wide square blocks); same scratch layout size as launch_chi0_split.
// With tail_ws (device, sbf16_tail_bytes() bytes) a last partial round of
// tiles is cut along the exponent blocks and reduced by a second launch.
// variant: the LDS ring (0: the preferred stage height and depth for S; 1:
// the other stage height), the same arithmetic in the same order.
constexpr int kNumSplitVariants = 2;
void launch_chi0_sbf16(int S, const double2* m, int64_t kc, int ng, const double2* delta, int nz,
                       const WList& wl, double2* chi, bool accumulate, void* scratch,
                       hipStream_t s, double2* tail_ws = nullptr, bool f16 = false,
                       int variant = 0);
// Workgroups of the split-BF16 contraction with S slices and ring variant rv
// resident on the current device.
int sbf16_slots(int S, int rv = 0);
size_t sbf16_tail_bytes();  // for the current device
// Operands of one problem's chunk for the split-BF16 contraction (device
// pointers into scratch; frequency w's B slices and sigma follow at fixed
// strides).
struct SbDesc {
    const uint32_t* sa;
    const double* siga;
    const uint32_t* sb;
    const double* sigb;
    double2* chi;  // [nz][ng][ng]
    int ng, ngp, nkb, mode;
};
// Bytes of that layout for a chunk of kc pairs (split_scratch_bytes covers it).
size_t sbf16_scratch_bytes(int64_t kc, int ng, int nz, int S, bool f16 = false);
// Descriptor of the slices of a chunk of kc pairs laid out in scratch (chi and
// mode unset); the layout launch_sbf16_prep writes.
SbDesc sbf16_desc(int S, int64_t kc, int ng, int nz, void* scratch, bool f16 = false);
// Slices of one chunk for the frequencies of wl (scratch as for
// launch_chi0_split); returns the descriptor with chi and mode unset.
SbDesc launch_sbf16_prep(int S, const double2* m, int64_t kc, int ng, const double2* delta,
                         int nz, const WList& wl, void* scratch, hipStream_t s, bool f16 = false);
// Persistent split-BF16 contraction over items (problem, frequency, 128-row
// block, 64-column block); counter must be 0 on entry.  variant: the LDS ring,
// as for launch_chi0_sbf16.
void launch_chi0_sbf16_batched(int S, const SbDesc* qd, const int4* items, int nitems,
                               int* counter, int grid, hipStream_t s, int variant = 0);
constexpr int kSbTileI = 128, kSbTileJ = 64;  // split-BF16 workgroup tile

// Tile edge whose on-or-above-diagonal blocks a reduced-precision mode computes.
inline int split_tile(int prec) { return prec == 2 || prec == 4 ? 128 : kSplitTile; }

// Fill the tiles strictly below the diagonal (tile x tile blocks) from the
// conjugate transpose.
void launch_mirror(double2* chi, int ng, int tile, hipStream_t s);

void launch_fill_zero(double2* p, int64_t n, hipStream_t s);


}  // namespace gw
