// Work items of the CHI0 contraction kernels (internal to libgw).
#pragma once

#include <hip/hip_runtime.h>

#include "chi0.hpp"

namespace gw {

// Device table of tile coordinates (bi << 16 | bj) for nb x nb tiles: first
// the nb(nb+1)/2 tiles on or above the diagonal, then all nb*nb tiles, each
// list in super-tile order (super x super blocks of tiles, row-major inside), so that
// the workgroups one XCD runs at the same time cover a compact block of chi
// and share the M rows of both its sides in that XCD's L2.  Cached per
// device; freed by release_tile_orders().
const int* tile_order(int nb, int super = 8);
void release_tile_orders();

// Item of workgroup b among n items.  The 8 XCDs take workgroups round-robin,
// so blocks are renumbered to give each XCD a contiguous range of items.
__device__ __forceinline__ int xcd_item(int b, int n) {
    const int q = n >> 3, r = n & 7;
    const int x = b & 7, i = b >> 3;
    return x * q + (x < r ? x : r) + i;
}

// Frequency and tile of item t.  Items are frequency-major: every Hermitian
// frequency over the tiles on or above the diagonal, then every other
// frequency over all tiles.
__device__ __forceinline__ void item_tile(int t, const WList& wl, int nb,
                                          const int* __restrict__ order, int& w, int& bi,
                                          int& bj) {
    const int nh = nb * (nb + 1) / 2, nf = nb * nb;
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
    bj = code & 0xffff;
}

// Frequency and tile of workgroup b when one workgroup takes each item.
__device__ __forceinline__ void decode_item(int b, const WList& wl, int nb,
                                            const int* __restrict__ order, int& w, int& bi,
                                            int& bj) {
    const int nitems = wl.nh * (nb * (nb + 1) / 2) + wl.nf * nb * nb;
    item_tile(xcd_item(b, nitems), wl, nb, order, w, bi, bj);
}

}  // namespace gw
