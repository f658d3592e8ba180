// C ABI of libgw: argument checks, scratch management and the chunked
// MTXEL -> energy factor -> CHI0 pipeline (declared in include/gw.h).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <unordered_set>
#include <utility>
#include <vector>

#include "backward.hpp"
#include "chi0.hpp"
#include "common.hpp"
#include "gw.h"
#include "items.hpp"
#include "plan.hpp"
#include "prof.hpp"

namespace gw {
namespace {

thread_local std::string g_last_error;

[[noreturn]] void fail(int status, const std::string& msg) { throw Error{status, msg}; }

// ---------------------------------------------------------------- scratch

struct Scratch {
    void* ptr = nullptr;
    size_t bytes = 0;
};

struct ScratchPool {
    std::mutex mu;
    std::map<std::pair<int, hipStream_t>, Scratch> by_key;
};

ScratchPool& pool() {
    static ScratchPool* p = new ScratchPool();
    return *p;
}

// Scratch of at least `bytes` for (current device, stream).  Growing it waits
// for the stream so that no enqueued kernel still uses the old buffer.
void* scratch(size_t bytes, hipStream_t s) {
    int dev = 0;
    GW_HIP_TRY(hipGetDevice(&dev));
    ScratchPool& p = pool();
    std::lock_guard<std::mutex> lk(p.mu);
    Scratch& sc = p.by_key[{dev, s}];
    if (sc.bytes >= bytes && sc.ptr) return sc.ptr;
    if (sc.ptr) {
        GW_HIP_TRY(hipStreamSynchronize(s));
        GW_HIP_TRY(hipFree(sc.ptr));
        sc.ptr = nullptr;
        sc.bytes = 0;
    }
    const size_t want = std::max<size_t>(bytes, 1 << 20);
    if (hipMalloc(&sc.ptr, want) != hipSuccess) {
        (void)hipGetLastError();
        sc.ptr = nullptr;
        fail(GW_ENOMEM, "hipMalloc of " + std::to_string(want) + " bytes of scratch failed");
    }
    sc.bytes = want;
    return sc.ptr;
}

void release_scratch() {
    ScratchPool& p = pool();
    std::lock_guard<std::mutex> lk(p.mu);
    for (auto& kv : p.by_key) {
        (void)hipSetDevice(kv.first.first);
        (void)hipDeviceSynchronize();
        (void)hipFree(kv.second.ptr);
    }
    p.by_key.clear();
}

// A library-owned companion stream of each caller stream (default priority),
// with events used to fork work onto it and join it back.
struct AuxCtx {
    hipStream_t aux = nullptr;
    hipEvent_t ev[6] = {};
};

struct AuxPool {
    std::mutex mu;
    std::map<std::pair<int, hipStream_t>, AuxCtx> by_key;
};

AuxPool& aux_pool() {
    static AuxPool* p = new AuxPool();
    return *p;
}

AuxCtx& aux_ctx(hipStream_t s) {
    int dev = 0;
    GW_HIP_TRY(hipGetDevice(&dev));
    AuxPool& p = aux_pool();
    std::lock_guard<std::mutex> lk(p.mu);
    AuxCtx& a = p.by_key[{dev, s}];
    if (!a.aux) {
        GW_HIP_TRY(hipStreamCreateWithFlags(&a.aux, hipStreamNonBlocking));
        for (auto& e : a.ev) GW_HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    return a;
}

void release_aux() {
    AuxPool& p = aux_pool();
    std::lock_guard<std::mutex> lk(p.mu);
    for (auto& kv : p.by_key) {
        (void)hipSetDevice(kv.first.first);
        (void)hipStreamSynchronize(kv.second.aux);
        for (auto& e : kv.second.ev) (void)hipEventDestroy(e);
        (void)hipStreamDestroy(kv.second.aux);
    }
    p.by_key.clear();
}

// Carves aligned sub-buffers out of one scratch allocation.
struct Carver {
    size_t off = 0;
    size_t take(size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~static_cast<size_t>(255);
        return o;
    }
};

// ---------------------------------------------------------------- argument checks

void check_grid(const gw_grid_t* g) {
    if (!g) fail(GW_EINVAL, "grid is NULL");
    int64_t nr = 1;
    for (int a = 0; a < 3; ++a) {
        if (g->n[a] < 1) fail(GW_EINVAL, "grid dimension " + std::to_string(a) + " < 1");
        nr *= g->n[a];
    }
    if (nr >= (int64_t(1) << 31)) fail(GW_EINVAL, "grid has 2^31 or more points");
    if (!(g->volume > 0.0) || !std::isfinite(g->volume)) fail(GW_EINVAL, "volume must be > 0");
}

void check_gvec(const int32_t* gvec, int ng, const int n[3]) {
    if (ng < 1) fail(GW_EINVAL, "ng must be >= 1");
    if (!gvec) fail(GW_EINVAL, "gvec is NULL");
    std::unordered_set<int64_t> seen;
    seen.reserve(static_cast<size_t>(ng) * 2);
    for (int i = 0; i < ng; ++i) {
        int64_t key = 0;
        for (int a = 0; a < 3; ++a) {
            const int g = gvec[3 * i + a];
            const int lo = -(n[a] / 2), hi = (n[a] + 1) / 2 - 1;
            if (g < lo || g > hi)
                fail(GW_EINVAL, "gvec[" + std::to_string(i) + "][" + std::to_string(a) + "] = " +
                                    std::to_string(g) + " outside [" + std::to_string(lo) + ", " +
                                    std::to_string(hi) + "]");
            key = key * 4096 + (g - lo);
        }
        if (!seen.insert(key).second) fail(GW_EINVAL, "duplicate G at index " + std::to_string(i));
    }
}

struct Opts {
    int precision = GW_FP64;
    int n_slices = 0;
    int pair_chunk = 4096;
    uint32_t flags = 0;
    double spin = 2.0;
};

Opts read_opts(const gw_opts_t* o) {
    Opts r;
    if (!o) return r;
    r.precision = o->precision;
    r.n_slices = o->n_slices;
    r.pair_chunk = o->pair_chunk == 0 ? 4096 : o->pair_chunk;
    r.flags = o->flags;
    r.spin = o->spin == 0.0 ? 2.0 : o->spin;
    if (r.pair_chunk < 1) fail(GW_EINVAL, "pair_chunk must be >= 1 (or 0 for the default)");
    if (!std::isfinite(r.spin)) fail(GW_EINVAL, "spin must be finite");
    if (r.precision < GW_FP64 || r.precision > GW_SPLIT_FP16)
        fail(GW_EINVAL, "unknown precision " + std::to_string(r.precision));
    if ((r.precision == GW_SPLIT_BF16 || r.precision == GW_SPLIT_FP16) &&
        (r.n_slices < 2 || r.n_slices > 8))
        fail(GW_EINVAL, "n_slices must be in [2, 8] for split precision");
    if (r.flags & ~(GW_FLAG_NO_HERMITIAN | GW_FLAG_ACCUMULATE))
        fail(GW_EINVAL, "unknown flag bits");
    return r;
}

void check_problem(const gw_problem_t& p, int idx) {
    const std::string w = "problem " + std::to_string(idx) + ": ";
    try {
        check_grid(&p.grid);
        if (p.nv < 0 || p.nc < 0) fail(GW_EINVAL, "nv and nc must be >= 0");
        if (p.nv > 0 && (!p.psi_v || !p.e_v)) fail(GW_EINVAL, "psi_v / e_v is NULL");
        if (p.nc > 0 && (!p.psi_c || !p.e_c)) fail(GW_EINVAL, "psi_c / e_c is NULL");
        check_gvec(p.gvec, p.ng, p.grid.n);
        if (p.nz < 1) fail(GW_EINVAL, "nz must be >= 1");
        if (!p.z) fail(GW_EINVAL, "z is NULL");
        for (int i = 0; i < p.nz; ++i)
            if (!std::isfinite(p.z[i].re) || !std::isfinite(p.z[i].im))
                fail(GW_EINVAL, "z[" + std::to_string(i) + "] is not finite");
        if (!p.chi) fail(GW_EINVAL, "chi is NULL");
    } catch (Error& e) {
        e.msg = w + e.msg;
        throw;
    }
}

// Chunks of pairs are rectangles of bands: vb valence x cw conduction bands.
struct ChunkShape {
    int cw, vb;
    int ncv, ncc;  // number of chunks along v and c
};

ChunkShape chunk_shape(int nv, int nc, int pair_chunk) {
    ChunkShape cs;
    cs.cw = std::min(nc, pair_chunk);
    cs.vb = std::max(1, std::min(nv, pair_chunk / std::max(1, cs.cw)));
    cs.ncv = ceil_div(nv, cs.vb);
    cs.ncc = ceil_div(nc, cs.cw);
    return cs;
}

template <typename F>
gw_status_t guarded(F&& f) {
    try {
        f();
        g_last_error.clear();
        return GW_OK;
    } catch (const Error& e) {
        g_last_error = e.msg;
        return e.status;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return GW_ENOMEM;
    } catch (...) {
        g_last_error = "internal error";
        return GW_EINTERNAL;
    }
}

// ---------------------------------------------------------------- forward pipeline

void run_chi0(const gw_problem_t& pr, const Opts& o, hipStream_t s) {
    const MtxelPlan& plan = *get_plan(pr.grid.n, pr.gvec, pr.ng);
    const int64_t ng = pr.ng;
    const int64_t npairs = static_cast<int64_t>(pr.nv) * pr.nc;
    const bool accumulate = (o.flags & GW_FLAG_ACCUMULATE) != 0;
    double2* chi = reinterpret_cast<double2*>(pr.chi);
    if (npairs == 0) {
        if (!accumulate) launch_fill_zero(chi, ng * ng * pr.nz, s);
        return;
    }
    const ChunkShape cs = chunk_shape(pr.nv, pr.nc, o.pair_chunk);
    const int64_t kmax = static_cast<int64_t>(cs.vb) * cs.cw;
    // two M / Delta buffers: MTXEL of chunk k+1 (companion stream) overlaps
    // CHI0 of chunk k (caller stream)
    Carver cv;
    size_t off_m[2], off_d[2];
    for (int b = 0; b < 2; ++b) {
        off_m[b] = cv.take(kmax * ng * sizeof(double2));
        off_d[b] = cv.take(kmax * pr.nz * sizeof(double2));
    }
    const size_t off_t2 = cv.take(t2_elems(plan, kmax) * sizeof(double2));
    const bool split = o.precision == GW_SPLIT_BF16 || o.precision == GW_SPLIT_FP16;
    const size_t off_sp = cv.take(split ? split_scratch_bytes(kmax, pr.ng, pr.nz, o.n_slices) : 0);
    char* base = static_cast<char*>(scratch(cv.off, s));
    double2* mbuf[2] = {reinterpret_cast<double2*>(base + off_m[0]),
                        reinterpret_cast<double2*>(base + off_m[1])};
    double2* dbuf[2] = {reinterpret_cast<double2*>(base + off_d[0]),
                        reinterpret_cast<double2*>(base + off_d[1])};
    double2* t2 = reinterpret_cast<double2*>(base + off_t2);
    const double2* z = reinterpret_cast<const double2*>(pr.z);
    std::vector<bool> herm(pr.nz);
    for (int w = 0; w < pr.nz; ++w)
        herm[w] = pr.z[w].re == 0.0 && !(o.flags & GW_FLAG_NO_HERMITIAN) && !accumulate;
    // launches cover at most kMaxZ frequencies each (Hermitian ones first)
    std::vector<WList> wlists;
    {
        std::vector<int> order;
        for (int w = 0; w < pr.nz; ++w)
            if (herm[w]) order.push_back(w);
        const int nherm = static_cast<int>(order.size());
        for (int w = 0; w < pr.nz; ++w)
            if (!herm[w]) order.push_back(w);
        for (int i0 = 0; i0 < pr.nz; i0 += kMaxZ) {
            WList wl{};
            for (int i = i0; i < std::min(pr.nz, i0 + kMaxZ); ++i) {
                wl.w[i - i0] = order[i];
                if (i < nherm) ++wl.nh; else ++wl.nf;
            }
            wlists.push_back(wl);
        }
    }
    struct Chunk {
        PairMap pm;
        int vcount;
        int64_t kc;
    };
    std::vector<Chunk> chunks;
    for (int iv = 0; iv < cs.ncv; ++iv)
        for (int ic = 0; ic < cs.ncc; ++ic) {
            Chunk c;
            c.pm.v0 = iv * cs.vb;
            c.pm.c0 = ic * cs.cw;
            c.pm.cw = std::min(cs.cw, pr.nc - c.pm.c0);
            c.pm.k_off = 0;
            c.vcount = std::min(cs.vb, pr.nv - c.pm.v0);
            c.kc = static_cast<int64_t>(c.vcount) * c.pm.cw;
            chunks.push_back(c);
        }
    // events: ev[0] caller-stream start, ev[1+b] MTXEL into buffer b done,
    // ev[3+b] CHI0 reading buffer b done
    AuxCtx& ax = aux_ctx(s);
    auto produce = [&](size_t k) {  // MTXEL + Delta of chunk k on the companion stream
        const int b = static_cast<int>(k & 1);
        if (k >= 2) GW_HIP_TRY(hipStreamWaitEvent(ax.aux, ax.ev[3 + b], 0));
        const Chunk& c = chunks[k];
        launch_mtxel(plan, reinterpret_cast<const double2*>(pr.psi_v),
                     reinterpret_cast<const double2*>(pr.psi_c),
                     Rect{c.pm.v0, c.vcount, c.pm.c0, c.pm.cw}, pr.grid.volume, t2, mbuf[b], ax.aux);
        launch_delta(pr.e_v, pr.e_c, c.pm, c.kc, z, pr.nz, o.spin, dbuf[b], ax.aux);
        GW_HIP_TRY(hipEventRecord(ax.ev[1 + b], ax.aux));
    };
    GW_HIP_TRY(hipEventRecord(ax.ev[0], s));
    GW_HIP_TRY(hipStreamWaitEvent(ax.aux, ax.ev[0], 0));
    produce(0);
    for (size_t k = 0; k < chunks.size(); ++k) {
        const int b = static_cast<int>(k & 1);
        if (k + 1 < chunks.size()) produce(k + 1);
        GW_HIP_TRY(hipStreamWaitEvent(s, ax.ev[1 + b], 0));
        for (const WList& wl : wlists) {
            const bool acc = accumulate || k > 0;
            if (o.precision == GW_FP64)
                launch_chi0_f64(mbuf[b], chunks[k].kc, pr.ng, dbuf[b], wl, chi, acc, s);
            else if (o.precision == GW_FP32)
                launch_chi0_f32(mbuf[b], chunks[k].kc, pr.ng, dbuf[b], wl, chi, acc, s);
            else
                launch_chi0_split(o.precision, o.n_slices, mbuf[b], chunks[k].kc, pr.ng, dbuf[b],
                                  pr.nz, wl, chi, acc, base + off_sp, s);
        }
        GW_HIP_TRY(hipEventRecord(ax.ev[3 + b], s));
    }
    for (int w = 0; w < pr.nz; ++w)
        if (herm[w])
            launch_mirror(chi + static_cast<int64_t>(w) * ng * ng, pr.ng,
                          o.precision == GW_FP64 ? chi0_tile() : kSplitTile, s);
}

}  // namespace
}  // namespace gw

using namespace gw;

extern "C" {

gw_status_t gw_mtxel(const gw_grid_t* grid, const gw_c128* psi_v, int32_t nv,
                     const gw_c128* psi_c, int32_t nc, const int32_t* gvec, int32_t ng,
                     int64_t pair_begin, int64_t pair_count, gw_c128* m_out, void* stream) {
    return guarded([&] {
        check_grid(grid);
        if (nv < 0 || nc < 0) fail(GW_EINVAL, "nv and nc must be >= 0");
        check_gvec(gvec, ng, grid->n);
        const int64_t npairs = static_cast<int64_t>(nv) * nc;
        if (pair_begin < 0 || pair_count < 0 || pair_begin + pair_count > npairs)
            fail(GW_EINVAL, "pair range [" + std::to_string(pair_begin) + ", " +
                                std::to_string(pair_begin + pair_count) + ") outside [0, " +
                                std::to_string(npairs) + ")");
        if (pair_count == 0) return;
        if (!psi_v || !psi_c) fail(GW_EINVAL, "psi_v / psi_c is NULL");
        if (!m_out) fail(GW_EINVAL, "m_out is NULL");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const MtxelPlan& plan = *get_plan(grid->n, gvec, ng);
        // the linear pair range as rectangles of at most kBatch pairs
        constexpr int64_t kBatch = 4096;
        std::vector<std::pair<Rect, int64_t>> rects;  // (rectangle, first output row)
        int64_t p0 = pair_begin;
        const int64_t pend = pair_begin + pair_count;
        while (p0 < pend) {
            const int v = static_cast<int>(p0 / nc), c = static_cast<int>(p0 % nc);
            Rect r;
            if (c != 0 || pend - p0 < nc) {  // part of one row
                const int64_t cnt = std::min<int64_t>({nc - c, pend - p0, kBatch});
                r = Rect{v, 1, c, static_cast<int32_t>(cnt)};
            } else if (nc > kBatch) {        // a long row, in pieces
                r = Rect{v, 1, 0, static_cast<int32_t>(kBatch)};
            } else {                          // whole rows
                const int64_t rows = std::min<int64_t>((pend - p0) / nc, kBatch / nc);
                r = Rect{v, static_cast<int32_t>(rows), 0, nc};
            }
            rects.push_back({r, p0 - pair_begin});
            p0 += static_cast<int64_t>(r.nv) * r.nc;
        }
        double2* t2 = static_cast<double2*>(scratch(t2_elems(plan, kBatch) * sizeof(double2), s));
        for (const auto& rr : rects)
            launch_mtxel(plan, reinterpret_cast<const double2*>(psi_v),
                         reinterpret_cast<const double2*>(psi_c), rr.first, grid->volume, t2,
                         reinterpret_cast<double2*>(m_out) + rr.second * ng, s);
    });
}

gw_status_t gw_chi0(const gw_problem_t* probs, int32_t nprob, const gw_opts_t* opts,
                    void* stream) {
    return guarded([&] {
        if (nprob < 0) fail(GW_EINVAL, "nprob must be >= 0");
        if (nprob > 0 && !probs) fail(GW_EINVAL, "probs is NULL");
        const Opts o = read_opts(opts);
        for (int q = 0; q < nprob; ++q) check_problem(probs[q], q);
        if ((o.precision == GW_SPLIT_BF16 || o.precision == GW_SPLIT_FP16) && o.n_slices > 6)
            fail(GW_EUNSUPPORTED, "split precision supports up to 6 slices in this build");
        hipStream_t s = static_cast<hipStream_t>(stream);
        for (int q = 0; q < nprob; ++q) {
            // plan construction may still reject the sizes; do it for all first
            (void)get_plan(probs[q].grid.n, probs[q].gvec, probs[q].ng);
        }
        for (int q = 0; q < nprob; ++q) run_chi0(probs[q], o, s);
    });
}

gw_status_t gw_chi0_backward(const gw_problem_t* prob, const gw_c128* grad_chi,
                             gw_c128* grad_psi_v, gw_c128* grad_psi_c, double* grad_e_v,
                             double* grad_e_c, const gw_opts_t* opts, void* stream) {
    return guarded([&] {
        if (!prob) fail(GW_EINVAL, "prob is NULL");
        const Opts o = read_opts(opts);
        gw_problem_t p = *prob;
        if (!p.chi) p.chi = reinterpret_cast<gw_c128*>(const_cast<gw_c128*>(grad_chi));
        check_problem(p, 0);
        if (!grad_chi) fail(GW_EINVAL, "grad_chi is NULL");
        if (o.precision != GW_FP64) fail(GW_EUNSUPPORTED, "the adjoint is FP64 only");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const MtxelPlan& plan = *get_plan(p.grid.n, p.gvec, p.ng);
        run_chi0_backward(plan, p, reinterpret_cast<const double2*>(grad_chi),
                          reinterpret_cast<double2*>(grad_psi_v),
                          reinterpret_cast<double2*>(grad_psi_c), grad_e_v, grad_e_c, o.spin,
                          o.pair_chunk, s, [&](size_t bytes) { return scratch(bytes, s); });
    });
}

const char* gw_last_error(void) { return g_last_error.c_str(); }

gw_status_t gw_release(void) {
    return guarded([&] {
        release_aux();
        release_scratch();
        release_plans();
        release_tile_orders();
    });
}

int32_t gw_abi_version(void) { return GW_ABI_VERSION; }

gw_status_t gw_profile_enable(int32_t on) {
    return guarded([&] { prof_enable(on != 0); });
}

gw_status_t gw_profile_read(const char* kernel, int64_t* launches, double* total_ms) {
    return guarded([&] {
        if (!kernel) fail(GW_EINVAL, "kernel name is NULL");
        prof_read(kernel, launches, total_ms);
    });
}

gw_status_t gw_profile_reset(void) {
    return guarded([&] { prof_reset(); });
}

}  // extern "C"
