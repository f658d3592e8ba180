// C ABI of libgw: argument checks, scratch management and the chunked
// MTXEL -> energy factor -> CHI0 pipeline (declared in include/gw.h).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cctype>
#include <cstring>
#include <functional>
#include <list>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <unordered_set>
#include <utility>
#include <vector>

#include "backward.hpp"
#include "chi0.hpp"
#include "common.hpp"
#include "epsinv.hpp"
#include "gpp.hpp"
#include "gw.h"
#include "items.hpp"
#include "lifetime.hpp"
#include "linalg.hpp"
#include "plan.hpp"
#include "prof.hpp"
#include "pseudobands.hpp"
#include "subspace.hpp"

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
    require_alloc("scratch buffer");
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
        size_t fr = 0, tot = 0;
        (void)hipMemGetInfo(&fr, &tot);
        fail(GW_ENOMEM, "hipMalloc of " + std::to_string(want) + " bytes of scratch failed (" +
                            std::to_string(fr) + " of " + std::to_string(tot) + " bytes free)");
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
// Events of a companion context: ev[kEvStart] forks from the caller's stream,
// ev[kEvMade + b] marks buffer b written, ev[kEvUsed + b] buffer b read.
constexpr int kEvStart = 0, kEvMade = 1, kEvUsed = 3;

struct AuxCtx {
    hipStream_t aux = nullptr;
    hipEvent_t ev[6] = {};
    hipStream_t cap = nullptr;  // graphs are captured here (the null stream cannot capture)
};

struct AuxPool {
    std::mutex mu;
    std::map<std::pair<int, hipStream_t>, AuxCtx> by_key;
};

AuxPool& aux_pool() {
    static AuxPool* p = new AuxPool();
    return *p;
}

AuxCtx& aux_ctx(hipStream_t s);

hipStream_t capture_stream(hipStream_t s) {
    AuxCtx& a = aux_ctx(s);
    std::lock_guard<std::mutex> lk(aux_pool().mu);
    if (!a.cap) GW_HIP_TRY(hipStreamCreateWithFlags(&a.cap, hipStreamNonBlocking));
    return a.cap;
}

AuxCtx& aux_ctx(hipStream_t s) {
    int dev = 0;
    GW_HIP_TRY(hipGetDevice(&dev));
    AuxPool& p = aux_pool();
    std::lock_guard<std::mutex> lk(p.mu);
    AuxCtx& a = p.by_key[{dev, s}];
    if (!a.aux) {
        require_alloc("companion stream");
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
        if (kv.second.cap) (void)hipStreamDestroy(kv.second.cap);
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
    char* ws = nullptr;      // caller's workspace, or null for the library's scratch
    size_t ws_bytes = 0;
};

// Split precisions: fixed-point slices, FP32 accumulation.
bool is_split(int p) { return p == GW_SPLIT_BF16 || p == GW_SPLIT_FP16 || p == GW_SPLIT_FP16X9; }
// Split precisions contracted by the 32x32 grouped kernel (128 x 64 tiles).
bool sliced_32x32(int p) { return p == GW_SPLIT_BF16 || p == GW_SPLIT_FP16X9; }

Opts read_opts(const gw_opts_t* o) {
    Opts r;
    if (!o) return r;
    r.precision = o->precision;
    r.n_slices = o->n_slices;
    r.pair_chunk = o->pair_chunk == 0 ? 4096 : o->pair_chunk;
    r.flags = o->flags;
    r.spin = o->spin == 0.0 ? 2.0 : o->spin;
    r.ws = static_cast<char*>(o->workspace);
    r.ws_bytes = o->workspace ? o->workspace_bytes : 0;
    if (r.ws && (reinterpret_cast<uintptr_t>(r.ws) & 255))
        fail(GW_EINVAL, "workspace must be 256-byte aligned");
    if (r.pair_chunk < 1) fail(GW_EINVAL, "pair_chunk must be >= 1 (or 0 for the default)");
    if (!std::isfinite(r.spin)) fail(GW_EINVAL, "spin must be finite");
    if (r.precision < GW_FP64 || r.precision > GW_SPLIT_FP16X9)
        fail(GW_EINVAL, "unknown precision " + std::to_string(r.precision));
    if (is_split(r.precision) && (r.n_slices < 2 || r.n_slices > 8))
        fail(GW_EINVAL, "n_slices must be in [2, 8] for split precision");
    if (r.flags & ~(GW_FLAG_NO_HERMITIAN | GW_FLAG_ACCUMULATE | GW_FLAG_GRAPH | GW_FLAG_AUTOTUNE |
                    GW_FLAG_FP64_TILE128 | GW_FLAG_ACC_HERMITIAN))
        fail(GW_EINVAL, "unknown flag bits");
    if ((r.flags & GW_FLAG_ACC_HERMITIAN) && !(r.flags & GW_FLAG_ACCUMULATE))
        fail(GW_EINVAL, "GW_FLAG_ACC_HERMITIAN needs GW_FLAG_ACCUMULATE");
    return r;
}

// Slice counts this library implements (read_opts has checked [2, 8]).
void check_slices(const Opts& o) {
    if (o.precision == GW_SPLIT_FP16X9 && o.n_slices > 4)
        fail(GW_EUNSUPPORTED, "9-bit FP16 slices: at most 4 (a fifth leaves FP16's range)");
    if (is_split(o.precision) && o.n_slices > 6)
        fail(GW_EUNSUPPORTED, "split precision supports up to 6 slices in this library");
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
// The MTXEL tiles take 4 valence bands at a time, so the conduction width is
// capped at pair_chunk / 4 (when there are 4 valence bands), then the valence
// height fills the chunk.
struct ChunkShape {
    int cw, vb;
    int ncv, ncc;  // number of chunks along v and c
};

ChunkShape chunk_shape(int nv, int nc, int pair_chunk) {
    ChunkShape cs;
    cs.cw = std::max(1, std::min(nc, pair_chunk / std::max(1, std::min(nv, 4))));
    cs.vb = std::max(1, std::min(nv, pair_chunk / cs.cw));
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

struct Chunk {
    PairMap pm;
    int vcount;
    int64_t kc;
};

std::vector<Chunk> make_chunks(const gw_problem_t& pr, const ChunkShape& cs) {
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
    return chunks;
}

// Frequencies whose Delta is real (Re z = 0) give Hermitian chi.  Accumulating
// keeps the shortcut only when the caller states that chi is Hermitian already.
std::vector<bool> hermitian_freqs(const gw_problem_t& pr, const Opts& o) {
    std::vector<bool> herm(pr.nz);
    const bool acc = (o.flags & GW_FLAG_ACCUMULATE) && !(o.flags & GW_FLAG_ACC_HERMITIAN);
    for (int w = 0; w < pr.nz; ++w)
        herm[w] = pr.z[w].re == 0.0 && !(o.flags & GW_FLAG_NO_HERMITIAN) && !acc;
    return herm;
}

// ---------------------------------------------------------------- autotuner

bool autotune_enabled(const Opts& o) {
    static const bool env = [] {
        const char* e = std::getenv("GW_AUTOTUNE");
        return e && std::atoi(e) != 0;
    }();
    return env || (o.flags & GW_FLAG_AUTOTUNE);
}

// Best variant per (kernel, N_G, chunk pairs), chosen by timing every
// candidate on real data once: the FP64 tile shape (kernel "f64") or the LDS
// ring of a split contraction ("sbf16-S<n>", "f16x9-S<n>").  Kept for the
// process and, when GW_AUTOTUNE_CACHE names a file, in that file ("kernel ng
// kc variant ms..." per line; a line without the kernel name is an FP64 one).
struct TuneCache {
    std::mutex mu;
    std::map<std::tuple<std::string, int, int64_t>, int> best;
    bool loaded = false;
};

TuneCache& tune_cache() {
    static TuneCache* c = new TuneCache();
    return *c;
}

const char* tune_file() { return std::getenv("GW_AUTOTUNE_CACHE"); }

// Tuning key and number of candidates of a contraction precision.
std::string tune_kind(const Opts& o) {
    if (o.precision == GW_FP64) return "f64";
    return std::string(o.precision == 4 ? "f16x9" : "sbf16") + "-S" + std::to_string(o.n_slices);
}
int tune_count(const std::string& kind) { return kind == "f64" ? kNumChi0Variants : kNumSplitVariants; }

// Forced split ring (GW_SPLIT_VARIANT), or -1.
int split_forced_variant() {
    const char* e = std::getenv("GW_SPLIT_VARIANT");
    if (!e) return -1;
    const int v = std::atoi(e);
    return v >= 0 && v < kNumSplitVariants ? v : 0;
}

int lookup_variant(const std::string& kind, int ng, int64_t kc) {
    const int forced = kind == "f64" ? chi0_forced_variant() : split_forced_variant();
    if (forced >= 0) return forced < tune_count(kind) ? forced : 0;
    TuneCache& tc = tune_cache();
    std::lock_guard<std::mutex> lk(tc.mu);
    if (!tc.loaded) {
        tc.loaded = true;
        if (const char* f = tune_file()) {
            if (FILE* fp = std::fopen(f, "r")) {
                char line[512], name[64];
                while (std::fgets(line, sizeof line, fp)) {
                    int a, v;
                    long long b;
                    if (std::sscanf(line, "%63s %d %lld %d", name, &a, &b, &v) == 4 &&
                        !std::isdigit(static_cast<unsigned char>(name[0]))) {
                        if (v >= 0 && v < tune_count(name)) tc.best[{name, a, b}] = v;
                    } else if (std::sscanf(line, "%d %lld %d", &a, &b, &v) == 3 && v >= 0 &&
                               v < kNumChi0Variants) {
                        tc.best[{"f64", a, b}] = v;
                    }
                }
                std::fclose(fp);
            }
        }
    }
    auto it = tc.best.find({kind, ng, kc});
    return it == tc.best.end() ? -1 : it->second;
}

// trial(v) enqueues variant v's contraction of the same data on s.
int tune_variant(const std::string& kind, int ng, int64_t kc, hipStream_t s,
                 const std::function<void(int)>& trial) {
    const int known = lookup_variant(kind, ng, kc);
    if (known >= 0) return known;
    const int nv = tune_count(kind);
    hipEvent_t e0, e1;
    GW_HIP_TRY(hipEventCreate(&e0));
    GW_HIP_TRY(hipEventCreate(&e1));
    std::vector<float> ms(nv, 0.0f);
    int best = 0;
    for (int v = 0; v < nv; ++v) {
        trial(v);  // warm-up (kernel load, caches)
        GW_HIP_TRY(hipEventRecord(e0, s));
        trial(v);
        GW_HIP_TRY(hipEventRecord(e1, s));
        GW_HIP_TRY(hipEventSynchronize(e1));
        GW_HIP_TRY(hipEventElapsedTime(&ms[v], e0, e1));
        if (ms[v] < ms[best]) best = v;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    TuneCache& tc = tune_cache();
    std::lock_guard<std::mutex> lk(tc.mu);
    tc.best[{kind, ng, kc}] = best;
    if (const char* f = tune_file()) {
        if (FILE* fp = std::fopen(f, "a")) {
            std::fprintf(fp, "%s %d %lld %d", kind.c_str(), ng, static_cast<long long>(kc), best);
            for (int v = 0; v < nv; ++v) std::fprintf(fp, " %.4f", ms[v]);
            std::fprintf(fp, "\n");
            std::fclose(fp);
        }
    }
    return best;
}

// Frequencies grouped into launches of at most kMaxZ, Hermitian ones first.
std::vector<WList> freq_lists(const std::vector<bool>& herm) {
    const int nz = static_cast<int>(herm.size());
    std::vector<int> order;
    for (int w = 0; w < nz; ++w)
        if (herm[w]) order.push_back(w);
    const int nherm = static_cast<int>(order.size());
    for (int w = 0; w < nz; ++w)
        if (!herm[w]) order.push_back(w);
    std::vector<WList> out;
    for (int i0 = 0; i0 < nz; i0 += kMaxZ) {
        WList wl{};
        for (int i = i0; i < std::min(nz, i0 + kMaxZ); ++i) {
            wl.w[i - i0] = order[i];
            if (i < nherm) ++wl.nh; else ++wl.nf;
        }
        out.push_back(wl);
    }
    return out;
}

// Scratch of one call: the caller's workspace, checked against `need` before
// anything is enqueued, or the library's buffer for (device, stream).
char* call_scratch(size_t need, const Opts& o, hipStream_t s) {
    if (o.ws) {
        if (need > o.ws_bytes)
            fail(GW_EINVAL, "workspace of " + std::to_string(o.ws_bytes) +
                                " bytes is too small: this call needs " + std::to_string(need));
        return o.ws;
    }
    if (need == 0) return nullptr;
    return static_cast<char*>(scratch(need, s));
}

// The autotuner may time variants inside this call: FP64 tile shapes (default
// tile) or the LDS ring of the split-BF16 / 9-bit FP16 contractions.
bool tune_candidate(const Opts& o) {
    const bool f64 = o.precision == GW_FP64 && !(o.flags & GW_FLAG_FP64_TILE128);
    const bool split = o.precision == 2 || o.precision == 4;
    return (f64 || split) && autotune_enabled(o);
}

// Scratch layout of one problem's pipeline.  nbuf M/Delta buffers (2: MTXEL
// of chunk k+1 on the companion stream under CHI0 of chunk k; 1: both on the
// caller's stream), room for the autotuner's trial plane, and for the partial
// tiles of a contraction's last round (tail).
// With n_eig > 0 (the static subspace), every chunk's M is transformed to the
// subspace basis, M^B = M C_s, before the contraction, which then runs over
// n_eig columns instead of N_G.
struct Chi0Layout {
    ChunkShape cs{};
    int64_t kmax = 0;
    int nbuf = 2;
    bool tail = true;
    int ncols = 0;  // columns of the contracted operand (N_G, or n_eig)
    size_t off_m[2] = {0, 0}, off_d[2] = {0, 0};
    size_t off_mfull = 0;  // M on the G-sphere before the transform (subspace only)
    size_t off_wbasis = 0; // W C_s, the weighted basis (subspace only)
    size_t off_t2 = 0, off_sp = 0, off_tune = 0, off_tail = 0;
    size_t total = 0;
};

Chi0Layout chi0_layout(const gw_problem_t& pr, const Opts& o, const MtxelPlan& plan, int nbuf,
                       bool tail, int n_eig = 0) {
    Chi0Layout L;
    L.nbuf = nbuf;
    L.tail = tail;
    L.ncols = n_eig > 0 ? n_eig : pr.ng;
    if (static_cast<int64_t>(pr.nv) * pr.nc == 0) return L;
    L.cs = chunk_shape(pr.nv, pr.nc, o.pair_chunk);
    L.kmax = static_cast<int64_t>(L.cs.vb) * L.cs.cw;
    const int64_t nw = L.ncols;
    Carver cv;
    for (int b = 0; b < nbuf; ++b) {
        L.off_m[b] = cv.take(L.kmax * nw * sizeof(double2));
        L.off_d[b] = cv.take(L.kmax * pr.nz * sizeof(double2));
    }
    if (nbuf == 1) {
        L.off_m[1] = L.off_m[0];
        L.off_d[1] = L.off_d[0];
    }
    L.off_mfull = cv.take(n_eig > 0 ? L.kmax * pr.ng * sizeof(double2) : 0);
    L.off_wbasis = cv.take(n_eig > 0 ? static_cast<size_t>(pr.ng) * n_eig * sizeof(double2) : 0);
    L.off_t2 = cv.take(t2_elems(plan, L.kmax) * sizeof(double2));
    const bool split = is_split(o.precision);
    L.off_sp = cv.take(split ? split_scratch_bytes(L.kmax, L.ncols, pr.nz, o.n_slices) : 0);
    L.off_tune = cv.take(tune_candidate(o) ? nw * nw * sizeof(double2) : 0);
    L.off_tail = cv.take(!tail                          ? 0
                         : o.precision == GW_FP64        ? chi0_f64_tail_bytes()
                         : sliced_32x32(o.precision)     ? sbf16_tail_bytes()
                                                        : 0);
    L.total = cv.off;
    return L;
}

// One problem: MTXEL (+ the subspace transform) + Delta + CHI0 per chunk, then
// the Hermitian mirror.  base holds L.total bytes (L from chi0_layout with the
// same arguments); with basis (device [N_G][n_eig], L.ncols = n_eig) chi is
// [nz][n_eig][n_eig], and with weight (device [N_G]) the basis is W C_s.
// M kept in device memory across calls: out (written by MTXEL, chunk by
// chunk) or in (read instead of running MTXEL), both [npairs][N_G] in the
// order the call streams its chunks (the rectangles of chunk_shape for the
// same problem and pair_chunk, each [vcount][cw] row-major).
struct MKeep {
    double2* out = nullptr;
    const double2* in = nullptr;
};

void run_chi0(const gw_problem_t& pr, const Opts& o, hipStream_t s, char* base,
              const Chi0Layout& L, const double2* basis = nullptr,
              const double* weight = nullptr, MKeep mk = {}) {
    const PlanRef plan_ref = get_plan(pr.grid.n, pr.gvec, pr.ng);
    const MtxelPlan& plan = *plan_ref;
    const int64_t ng = L.ncols;  // the contraction's width
    const int64_t npairs = static_cast<int64_t>(pr.nv) * pr.nc;
    const bool accumulate = (o.flags & GW_FLAG_ACCUMULATE) != 0;
    double2* chi = reinterpret_cast<double2*>(pr.chi);
    if (npairs == 0) {
        if (!accumulate) launch_fill_zero(chi, ng * ng * pr.nz, s);
        return;
    }
    const bool two_streams = L.nbuf == 2;
    if (basis && weight) {
        double2* wb = reinterpret_cast<double2*>(base + L.off_wbasis);
        launch_scale_rows(basis, wb, weight, pr.ng, L.ncols, s);
        basis = wb;
    }
    double2* mbuf[2] = {reinterpret_cast<double2*>(base + L.off_m[0]),
                        reinterpret_cast<double2*>(base + L.off_m[1])};
    double2* dbuf[2] = {reinterpret_cast<double2*>(base + L.off_d[0]),
                        reinterpret_cast<double2*>(base + L.off_d[1])};
    double2* t2 = reinterpret_cast<double2*>(base + L.off_t2);
    double2* tail_ws = L.tail && (o.precision == GW_FP64 || sliced_32x32(o.precision))
                           ? reinterpret_cast<double2*>(base + L.off_tail)
                           : nullptr;
    const std::vector<Chunk> chunks = make_chunks(pr, L.cs);
    std::vector<int64_t> moff(chunks.size(), 0);  // first row of chunk k in kept M
    for (size_t k = 1; k < chunks.size(); ++k) moff[k] = moff[k - 1] + chunks[k - 1].kc;
    // the contraction's operand of chunk k: buffer k & 1, or kept M itself
    auto cmat = [&](size_t k) -> const double2* {
        if (basis) return mbuf[k & 1];
        if (mk.in) return mk.in + moff[k] * pr.ng;
        if (mk.out) return mk.out + moff[k] * pr.ng;
        return mbuf[k & 1];
    };
    int variant = 0;
    bool tune = false;
    const bool split_ring = o.precision == 2 || o.precision == 4;
    if (o.precision == GW_FP64 && (o.flags & GW_FLAG_FP64_TILE128)) {
        variant = 1;
    } else if (o.precision == GW_FP64 || split_ring) {
        variant = lookup_variant(tune_kind(o), L.ncols, chunks[0].kc);
        tune = variant < 0 && autotune_enabled(o);
        if (variant < 0) variant = 0;
    }
    const double2* z = reinterpret_cast<const double2*>(pr.z);
    const std::vector<bool> herm = hermitian_freqs(pr, o);
    // launches cover at most kMaxZ frequencies each (Hermitian ones first)
    const std::vector<WList> wlists = freq_lists(herm);
    // events: ev[0] caller-stream start, ev[1+b] MTXEL into buffer b done,
    // ev[3+b] CHI0 reading buffer b done
    AuxCtx* ax = two_streams ? &aux_ctx(s) : nullptr;
    auto produce = [&](size_t k) {  // MTXEL + Delta of chunk k
        const int b = static_cast<int>(k & 1);
        const hipStream_t ps = two_streams ? ax->aux : s;
        if (two_streams && k >= 2) GW_HIP_TRY(hipStreamWaitEvent(ax->aux, ax->ev[3 + b], 0));
        const Chunk& c = chunks[k];
        const double2* mout;
        if (mk.in) {
            mout = mk.in + moff[k] * pr.ng;
        } else {
            double2* dst = mk.out    ? mk.out + moff[k] * pr.ng
                           : basis   ? reinterpret_cast<double2*>(base + L.off_mfull)
                                     : mbuf[b];
            launch_mtxel(plan, reinterpret_cast<const double2*>(pr.psi_v),
                         reinterpret_cast<const double2*>(pr.psi_c),
                         Rect{c.pm.v0, c.vcount, c.pm.c0, c.pm.cw}, pr.grid.volume, t2, dst, ps);
            mout = dst;
        }
        if (basis) {  // Transf: M^B = M C_s
            ZGemm g;
            g.m = static_cast<int>(c.kc);
            g.n = L.ncols;
            g.k = pr.ng;
            g.a = mout;
            g.lda = pr.ng;
            g.b = basis;
            g.ldb = L.ncols;
            g.c = mbuf[b];
            g.ldc = L.ncols;
            launch_zgemm(kOpN, kOpN, g, ps);
        }
        launch_delta(pr.e_v, pr.e_c, c.pm, c.kc, z, pr.nz, o.spin, dbuf[b], ps);
        if (two_streams) GW_HIP_TRY(hipEventRecord(ax->ev[1 + b], ax->aux));
    };
    if (two_streams) {
        GW_HIP_TRY(hipEventRecord(ax->ev[0], s));
        GW_HIP_TRY(hipStreamWaitEvent(ax->aux, ax->ev[0], 0));
    }
    produce(0);
    if (tune) {
        // time the tile shapes on the first chunk and one frequency
        if (two_streams) GW_HIP_TRY(hipStreamWaitEvent(s, ax->ev[1], 0));
        WList one{};
        one.w[0] = 0;
        one.nf = 1;
        double2* trial_chi = reinterpret_cast<double2*>(base + L.off_tune);
        variant = tune_variant(tune_kind(o), L.ncols, chunks[0].kc, s, [&](int v) {
            if (split_ring)
                launch_chi0_split(o.precision, o.n_slices, cmat(0), chunks[0].kc, L.ncols,
                                  dbuf[0], pr.nz, one, trial_chi, false, base + L.off_sp, s,
                                  tail_ws, v);
            else
                launch_chi0_f64(cmat(0), chunks[0].kc, L.ncols, dbuf[0], one, trial_chi, false,
                                s, v, tail_ws);
        });
    }
    for (size_t k = 0; k < chunks.size(); ++k) {
        const int b = static_cast<int>(k & 1);
        if (!two_streams && k > 0) produce(k);
        if (two_streams) {
            if (k + 1 < chunks.size()) produce(k + 1);
            GW_HIP_TRY(hipStreamWaitEvent(s, ax->ev[1 + b], 0));
        }
        for (const WList& wl : wlists) {
            const bool acc = accumulate || k > 0;
            const double2* mk_k = cmat(k);
            if (o.precision == GW_FP64)
                launch_chi0_f64(mk_k, chunks[k].kc, L.ncols, dbuf[b], wl, chi, acc, s, variant,
                                tail_ws);
            else if (o.precision == GW_FP32)
                launch_chi0_f32(mk_k, chunks[k].kc, L.ncols, dbuf[b], wl, chi, acc, s);
            else
                launch_chi0_split(o.precision, o.n_slices, mk_k, chunks[k].kc, L.ncols, dbuf[b],
                                  pr.nz, wl, chi, acc, base + L.off_sp, s, tail_ws, variant);
        }
        if (two_streams) GW_HIP_TRY(hipEventRecord(ax->ev[3 + b], s));
    }
    for (int w = 0; w < pr.nz; ++w)
        if (herm[w])
            launch_mirror(chi + static_cast<int64_t>(w) * ng * ng, L.ncols,
                          o.precision == GW_FP64 ? chi0_variant_tile(variant) : split_tile(o.precision), s);
    mark_plan_used(*plan_ref, s);
}


// ---------------------------------------------------------------- batched problems

// One problem of a batch: its plan, chunks and buffers (offsets into the
// batch's scratch).
struct BatchQ {
    PlanRef plan;
    std::vector<Chunk> chunks;
    std::vector<bool> herm;
    int64_t kmax = 0;
    size_t off_m[2] = {0, 0}, off_d[2] = {0, 0};
    size_t off_sp = 0;  // split-BF16 slices of the current round
};

// A batch advances every problem by one chunk per round; each round's
// contraction is one persistent launch over all (problem, frequency, tile)
// items.  FP64 uses QDesc items on square tiles; split BF16 uses SbDesc
// items on 128 x 64 tiles (Hermitian rule on 128 x 128 blocks).
struct BatchPlan {
    std::vector<BatchQ> q;
    bool split = false;
    int S = 0;
    int rounds = 0;
    int variant = 0;
    int grid = 0;
    // work region (M, Delta, t2, slices: reusable by the next group) and
    // tables region (descriptors, items, counters: one per group)
    size_t off_t2 = 0, work_bytes = 0;
    size_t off_desc = 0, off_items = 0, off_cnt = 0, table_bytes = 0;
    std::vector<int> nitems;       // per round
    std::vector<size_t> item_off;  // per round, in int4 units
};

int resident_cus() {
    int dev = 0, cus = 0;
    GW_HIP_TRY(hipGetDevice(&dev));
    GW_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    return cus;
}

int persistent_grid(const BatchPlan& bp) {
    if (bp.split) return sbf16_slots(bp.S, bp.variant);  // the LDS ring sets the residency
    return resident_cus() * chi0_f64_batched_blocks_per_cu(bp.variant);
}

// Items of round r: (problem, frequency, tile row, tile col), all problems,
// largest chunk first; tiles of one problem and frequency in super-tile order.
std::vector<int4> round_items(const BatchPlan& bp, int r, const gw_problem_t* probs) {
    const int tile = bp.split ? kSbTileI : chi0_variant_tile(bp.variant);
    const int kSuper = bp.split ? 4 : 8;
    std::vector<std::pair<int64_t, int4>> v;
    for (size_t q = 0; q < bp.q.size(); ++q) {
        const BatchQ& b = bp.q[q];
        if (r >= static_cast<int>(b.chunks.size())) continue;
        const int ng = probs[q].ng;
        const int nb = ceil_div(ng, tile);
        for (int w = 0; w < probs[q].nz; ++w) {
            for (int si = 0; si < nb; si += kSuper)
                for (int sj = 0; sj < nb; sj += kSuper)
                    for (int i = si; i < std::min(nb, si + kSuper); ++i)
                        for (int j = sj; j < std::min(nb, sj + kSuper); ++j) {
                            if (b.herm[w] && j < i) continue;
                            if (!bp.split) {
                                v.push_back({b.chunks[r].kc, make_int4(static_cast<int>(q), w, i, j)});
                                continue;
                            }
                            for (int h = 0; h < 2; ++h)  // the two 64-column halves
                                if ((2 * j + h) * kSbTileJ < ng)
                                    v.push_back({b.chunks[r].kc,
                                                 make_int4(static_cast<int>(q), w, i, 2 * j + h)});
                        }
        }
    }
    std::stable_sort(v.begin(), v.end(),
                     [](const auto& a, const auto& b) { return a.first > b.first; });
    std::vector<int4> out(v.size());
    for (size_t i = 0; i < v.size(); ++i) out[i] = v[i].second;
    return out;
}

BatchPlan build_batch(const gw_problem_t* probs, int nprob, const Opts& o, int variant) {
    BatchPlan bp;
    bp.split = o.precision == GW_SPLIT_BF16;
    bp.S = o.n_slices;
    bp.variant = variant;
    bp.grid = persistent_grid(bp);
    bp.q.resize(nprob);
    Carver cv, ct;
    size_t t2max = 0;
    for (int q = 0; q < nprob; ++q) {
        BatchQ& b = bp.q[q];
        const gw_problem_t& pr = probs[q];
        b.plan = get_plan(pr.grid.n, pr.gvec, pr.ng);
        b.herm = hermitian_freqs(pr, o);
        if (static_cast<int64_t>(pr.nv) * pr.nc > 0) {
            const ChunkShape cs = chunk_shape(pr.nv, pr.nc, o.pair_chunk);
            b.chunks = make_chunks(pr, cs);
            b.kmax = static_cast<int64_t>(cs.vb) * cs.cw;
        }
        for (int k = 0; k < 2; ++k) {
            b.off_m[k] = cv.take(b.kmax * pr.ng * sizeof(double2));
            b.off_d[k] = cv.take(b.kmax * pr.nz * sizeof(double2));
        }
        if (bp.split && b.kmax > 0)
            b.off_sp = cv.take(split_scratch_bytes(b.kmax, pr.ng, pr.nz, bp.S));
        t2max = std::max(t2max, t2_elems(*b.plan, b.kmax) * sizeof(double2));
        bp.rounds = std::max(bp.rounds, static_cast<int>(b.chunks.size()));
    }
    bp.off_t2 = cv.take(t2max);
    bp.work_bytes = cv.off;
    const size_t desc_size = bp.split ? sizeof(SbDesc) : sizeof(QDesc);
    bp.off_desc = ct.take(static_cast<size_t>(bp.rounds) * nprob * desc_size);
    size_t ntot = 0;
    for (int r = 0; r < bp.rounds; ++r) {
        bp.item_off.push_back(ntot);
        bp.nitems.push_back(static_cast<int>(round_items(bp, r, probs).size()));
        ntot += bp.nitems.back();
    }
    bp.off_items = ct.take(std::max<size_t>(1, ntot) * sizeof(int4));
    bp.off_cnt = ct.take(std::max(1, bp.rounds) * sizeof(double2));
    bp.table_bytes = ct.off;
    return bp;
}

// Descriptor and item tables into the tables buffer, copied in stream order
// through the pinned staging buffers; descriptors point into the work buffer.
void upload_batch(const BatchPlan& bp, const gw_problem_t* probs, const Opts& o, char* base,
                  char* tab, hipStream_t s) {
    const int nprob = static_cast<int>(bp.q.size());
    std::vector<QDesc> desc;
    std::vector<SbDesc> sdesc;
    std::vector<int4> items;
    for (int r = 0; r < bp.rounds; ++r) {
        for (int q = 0; q < nprob; ++q) {
            const BatchQ& b = bp.q[q];
            const int64_t kc = r < static_cast<int>(b.chunks.size()) ? b.chunks[r].kc : 0;
            const int mode = (r > 0 || (o.flags & GW_FLAG_ACCUMULATE)) ? 1 : 0;
            if (bp.split) {
                SbDesc d = sbf16_desc(bp.S, std::max<int64_t>(kc, 1), probs[q].ng, probs[q].nz,
                                      base + b.off_sp);
                d.chi = reinterpret_cast<double2*>(probs[q].chi);
                d.mode = mode;
                sdesc.push_back(d);
            } else {
                QDesc d;
                d.m = reinterpret_cast<const double2*>(base + b.off_m[r & 1]);
                d.delta = reinterpret_cast<const double2*>(base + b.off_d[r & 1]);
                d.chi = reinterpret_cast<double2*>(probs[q].chi);
                d.kc = kc;
                d.ng = probs[q].ng;
                d.mode = mode;
                desc.push_back(d);
            }
        }
        const std::vector<int4> it = round_items(bp, r, probs);
        items.insert(items.end(), it.begin(), it.end());
    }
    if (bp.split)
        stage_h2d(tab + bp.off_desc, sdesc.data(), sdesc.size() * sizeof(SbDesc), s);
    else
        stage_h2d(tab + bp.off_desc, desc.data(), desc.size() * sizeof(QDesc), s);
    if (!items.empty()) stage_h2d(tab + bp.off_items, items.data(), items.size() * sizeof(int4), s);
}

void enqueue_batch(const BatchPlan& bp, const gw_problem_t* probs, const Opts& o, char* base,
                   char* tab, hipStream_t s) {
    const int nprob = static_cast<int>(bp.q.size());
    double2* t2 = reinterpret_cast<double2*>(base + bp.off_t2);
    // problems without pairs: chi = 0
    for (int q = 0; q < nprob; ++q)
        if (bp.q[q].chunks.empty() && !(o.flags & GW_FLAG_ACCUMULATE))
            launch_fill_zero(reinterpret_cast<double2*>(probs[q].chi),
                             static_cast<int64_t>(probs[q].ng) * probs[q].ng * probs[q].nz, s);
    if (bp.rounds == 0) return;
    launch_fill_zero(reinterpret_cast<double2*>(tab + bp.off_cnt), bp.rounds, s);
    AuxCtx& ax = aux_ctx(s);
    auto produce = [&](int r) {  // MTXEL + Delta of round r, every problem, companion stream
        const int b = r & 1;
        if (r >= 2) GW_HIP_TRY(hipStreamWaitEvent(ax.aux, ax.ev[kEvUsed + b], 0));
        for (int q = 0; q < nprob; ++q) {
            const BatchQ& bq = bp.q[q];
            if (r >= static_cast<int>(bq.chunks.size())) continue;
            const gw_problem_t& pr = probs[q];
            const Chunk& c = bq.chunks[r];
            launch_mtxel(*bq.plan, reinterpret_cast<const double2*>(pr.psi_v),
                         reinterpret_cast<const double2*>(pr.psi_c),
                         Rect{c.pm.v0, c.vcount, c.pm.c0, c.pm.cw}, pr.grid.volume, t2,
                         reinterpret_cast<double2*>(base + bq.off_m[b]), ax.aux);
            launch_delta(pr.e_v, pr.e_c, c.pm, c.kc, reinterpret_cast<const double2*>(pr.z), pr.nz,
                         o.spin, reinterpret_cast<double2*>(base + bq.off_d[b]), ax.aux);
        }
        GW_HIP_TRY(hipEventRecord(ax.ev[kEvMade + b], ax.aux));
    };
    GW_HIP_TRY(hipEventRecord(ax.ev[kEvStart], s));
    GW_HIP_TRY(hipStreamWaitEvent(ax.aux, ax.ev[kEvStart], 0));
    produce(0);
    for (int r = 0; r < bp.rounds; ++r) {
        const int b = r & 1;
        if (r + 1 < bp.rounds) produce(r + 1);
        GW_HIP_TRY(hipStreamWaitEvent(s, ax.ev[kEvMade + b], 0));
        const int4* items = reinterpret_cast<const int4*>(tab + bp.off_items) + bp.item_off[r];
        int* counter = reinterpret_cast<int*>(tab + bp.off_cnt) + r;
        if (bp.split) {
            // slices of every problem's chunk (the previous round's launch, on this
            // stream, has finished reading them), then one persistent contraction
            for (int q = 0; q < nprob; ++q) {
                const BatchQ& bq = bp.q[q];
                if (r >= static_cast<int>(bq.chunks.size())) continue;
                const gw_problem_t& pr = probs[q];
                for (const WList& wl : freq_lists(bq.herm))
                    (void)launch_sbf16_prep(bp.S, reinterpret_cast<const double2*>(base + bq.off_m[b]),
                                            bq.chunks[r].kc, pr.ng,
                                            reinterpret_cast<const double2*>(base + bq.off_d[b]),
                                            pr.nz, wl, base + bq.off_sp, s);
            }
            launch_chi0_sbf16_batched(
                bp.S, reinterpret_cast<const SbDesc*>(tab + bp.off_desc) + static_cast<size_t>(r) * nprob,
                items, bp.nitems[r], counter, bp.grid, s, bp.variant);
        } else {
            launch_chi0_f64_batched(
                reinterpret_cast<const QDesc*>(tab + bp.off_desc) + static_cast<size_t>(r) * nprob,
                items, bp.nitems[r], counter, s, bp.variant, bp.grid);
        }
        GW_HIP_TRY(hipEventRecord(ax.ev[kEvUsed + b], s));
    }
    const int tile = bp.split ? kSbTileI : chi0_variant_tile(bp.variant);
    for (int q = 0; q < nprob; ++q)
        for (int w = 0; w < probs[q].nz; ++w)
            if (bp.q[q].herm[w] && !bp.q[q].chunks.empty())
                launch_mirror(reinterpret_cast<double2*>(probs[q].chi) +
                                  static_cast<int64_t>(w) * probs[q].ng * probs[q].ng,
                              probs[q].ng, tile, s);
    for (int q = 0; q < nprob; ++q) mark_plan_used(*bp.q[q].plan, s);
}

// Scratch the autotuner of a batch needs: the largest problem's first chunk
// (M, Delta, t2) and one trial frequency plane.
struct TuneLayout {
    int qmax = -1;
    size_t om = 0, od = 0, ot = 0, oc = 0, osp = 0, total = 0;
};

TuneLayout batch_tune_layout(const gw_problem_t* probs, int nprob, const Opts& o) {
    TuneLayout t;
    if (!tune_candidate(o)) return t;
    for (int q = 0; q < nprob; ++q)
        if (static_cast<int64_t>(probs[q].nv) * probs[q].nc > 0 &&
            (t.qmax < 0 || probs[q].ng > probs[t.qmax].ng))
            t.qmax = q;
    if (t.qmax < 0) return t;
    const gw_problem_t& pr = probs[t.qmax];
    const ChunkShape cs = chunk_shape(pr.nv, pr.nc, o.pair_chunk);
    const std::vector<Chunk> ch = make_chunks(pr, cs);
    const PlanRef plan = get_plan(pr.grid.n, pr.gvec, pr.ng);
    Carver cv;
    t.om = cv.take(ch[0].kc * pr.ng * sizeof(double2));
    t.od = cv.take(ch[0].kc * pr.nz * sizeof(double2));
    t.ot = cv.take(t2_elems(*plan, ch[0].kc) * sizeof(double2));
    t.oc = cv.take(static_cast<size_t>(pr.ng) * pr.ng * sizeof(double2));
    if (o.precision == GW_SPLIT_BF16)
        t.osp = cv.take(split_scratch_bytes(ch[0].kc, pr.ng, pr.nz, o.n_slices));
    t.total = cv.off;
    return t;
}

// Tile variant (FP64) or LDS ring (split BF16) of a batch: forced, cached, or
// tuned on its largest problem's first chunk (one frequency, into the call's
// scratch so no output is touched; the split ring with the one-launch kernel
// of the same tiles).
int batch_variant(const gw_problem_t* probs, int nprob, const Opts& o, hipStream_t s,
                  char* base) {
    const bool split = o.precision == GW_SPLIT_BF16;
    if (o.precision != GW_FP64 && !split) return 0;
    if (!split && (o.flags & GW_FLAG_FP64_TILE128)) return 1;
    int qmax = -1;
    for (int q = 0; q < nprob; ++q)
        if (static_cast<int64_t>(probs[q].nv) * probs[q].nc > 0 &&
            (qmax < 0 || probs[q].ng > probs[qmax].ng))
            qmax = q;
    if (qmax < 0) return 0;
    const gw_problem_t& pr = probs[qmax];
    const ChunkShape cs = chunk_shape(pr.nv, pr.nc, o.pair_chunk);
    const std::vector<Chunk> ch = make_chunks(pr, cs);
    const std::string kind = tune_kind(o);
    int v = lookup_variant(kind, pr.ng, ch[0].kc);
    if (v >= 0) return v;
    if (!autotune_enabled(o)) return 0;
    const TuneLayout t = batch_tune_layout(probs, nprob, o);
    const PlanRef plan = get_plan(pr.grid.n, pr.gvec, pr.ng);
    launch_mtxel(*plan, reinterpret_cast<const double2*>(pr.psi_v),
                 reinterpret_cast<const double2*>(pr.psi_c),
                 Rect{ch[0].pm.v0, ch[0].vcount, ch[0].pm.c0, ch[0].pm.cw}, pr.grid.volume,
                 reinterpret_cast<double2*>(base + t.ot), reinterpret_cast<double2*>(base + t.om), s);
    launch_delta(pr.e_v, pr.e_c, ch[0].pm, ch[0].kc, reinterpret_cast<const double2*>(pr.z), pr.nz,
                 o.spin, reinterpret_cast<double2*>(base + t.od), s);
    WList wl{};
    wl.w[0] = 0;
    wl.nf = 1;
    v = tune_variant(kind, pr.ng, ch[0].kc, s, [&](int vv) {
        if (split)
            launch_chi0_split(o.precision, o.n_slices, reinterpret_cast<const double2*>(base + t.om),
                              ch[0].kc, pr.ng, reinterpret_cast<const double2*>(base + t.od), pr.nz,
                              wl, reinterpret_cast<double2*>(base + t.oc), false, base + t.osp, s,
                              nullptr, vv);
        else
            launch_chi0_f64(reinterpret_cast<const double2*>(base + t.om), ch[0].kc, pr.ng,
                            reinterpret_cast<const double2*>(base + t.od), wl,
                            reinterpret_cast<double2*>(base + t.oc), false, s, vv);
    });
    mark_plan_used(*plan, s);
    return v;
}

// Captured batches, most recently used first: the graph, the library-owned
// buffers it was captured with (the work buffer unless the caller gave a
// workspace, and the tables), the plans whose tables it reads, and an event
// recorded after its last replay.  The cache holds at most GW_GRAPH_CACHE_MAX
// graphs (default 16) and GW_GRAPH_CACHE_BYTES of buffers (default 64 GiB);
// an evicted graph is destroyed once its last replay has completed.
struct GraphEntry {
    std::string key;
    int device = 0;
    hipGraphExec_t exec = nullptr;
    std::vector<void*> buffers;
    size_t bytes = 0;
    std::vector<PlanRef> plans;
    hipEvent_t last_use = nullptr;
};

struct GraphCache {
    std::mutex mu;
    std::list<GraphEntry> lru;
};

GraphCache& graph_cache() {
    static GraphCache* c = new GraphCache();
    return *c;
}

size_t env_size(const char* name, size_t dflt) {
    const char* e = std::getenv(name);
    const long long v = e ? std::atoll(e) : 0;
    return v > 0 ? static_cast<size_t>(v) : dflt;
}

void retire_graph(GraphEntry& e) {
    hipGraphExec_t exec = e.exec;
    hipEvent_t ev = e.last_use;
    std::vector<void*> bufs = std::move(e.buffers);
    std::vector<PlanRef> plans = std::move(e.plans);
    retire(e.device, ev, [exec, ev, bufs, plans]() mutable {
        (void)hipGraphExecDestroy(exec);
        for (void* b : bufs) (void)hipFree(b);
        if (ev) (void)hipEventDestroy(ev);
        plans.clear();
    });
    e.exec = nullptr;
    e.last_use = nullptr;
}

// Cache key: every field that the captured work depends on, written field by
// field (no struct padding).
std::string batch_key(const gw_problem_t* probs, int nprob, const Opts& o) {
    std::string k;
    auto put = [&](const void* p, size_t n) { k.append(static_cast<const char*>(p), n); };
    auto put_i = [&](int64_t v) { put(&v, sizeof v); };
    auto put_d = [&](double v) { put(&v, sizeof v); };
    auto put_p = [&](const void* p) {
        const uintptr_t v = reinterpret_cast<uintptr_t>(p);
        put(&v, sizeof v);
    };
    int dev = 0;
    (void)hipGetDevice(&dev);
    put_i(dev);
    put_i(nprob);
    put_i(o.precision);
    put_i(o.n_slices);
    put_i(o.pair_chunk);
    put_i(o.flags);
    put_d(o.spin);
    put_p(o.ws);
    put_i(static_cast<int64_t>(o.ws_bytes));
    for (int q = 0; q < nprob; ++q) {
        const gw_problem_t& p = probs[q];
        for (int a = 0; a < 3; ++a) put_i(p.grid.n[a]);
        put_d(p.grid.volume);
        put_p(p.psi_v);
        put_i(p.nv);
        put_p(p.psi_c);
        put_i(p.nc);
        put_p(p.e_v);
        put_p(p.e_c);
        put_i(p.ng);
        put_i(p.nz);
        put_p(p.chi);
        put(p.gvec, static_cast<size_t>(p.ng) * 3 * sizeof(int32_t));
        put(p.z, static_cast<size_t>(p.nz) * sizeof(gw_c128));
    }
    return k;
}

void release_graphs() {
    GraphCache& gc = graph_cache();
    std::lock_guard<std::mutex> lk(gc.mu);
    for (auto& e : gc.lru) retire_graph(e);
    gc.lru.clear();
}

// Problems of one batch call in groups processed one after another: FP64 in a
// single group; split BF16 in groups whose slice buffers (one chunk of every
// problem, all frequencies) fit GW_SPLIT_BATCH_BYTES (default 8 GiB).
std::vector<std::vector<gw_problem_t>> batch_groups(const gw_problem_t* probs, int nprob,
                                                    const Opts& o) {
    std::vector<std::vector<gw_problem_t>> groups(1);
    if (o.precision != GW_SPLIT_BF16) {
        groups[0].assign(probs, probs + nprob);
        return groups;
    }
    const size_t budget = env_size("GW_SPLIT_BATCH_BYTES", size_t(8) << 30);
    size_t used = 0;
    for (int q = 0; q < nprob; ++q) {
        const gw_problem_t& pr = probs[q];
        size_t need = 0;
        if (static_cast<int64_t>(pr.nv) * pr.nc > 0) {
            const ChunkShape cs = chunk_shape(pr.nv, pr.nc, o.pair_chunk);
            need = split_scratch_bytes(static_cast<int64_t>(cs.vb) * cs.cw, pr.ng, pr.nz, o.n_slices);
        }
        if (!groups.back().empty() && used + need > budget) {
            groups.emplace_back();
            used = 0;
        }
        groups.back().push_back(pr);
        used += need;
    }
    return groups;
}

size_t align256(size_t b) { return (b + 255) & ~static_cast<size_t>(255); }

// Tile variants the batch may run with (the layout of its tables depends on it).
std::vector<int> possible_variants(const Opts& o) {
    if (o.precision == GW_SPLIT_BF16) {
        const int forced = split_forced_variant();
        if (forced >= 0) return {forced};
        std::vector<int> v;
        for (int i = 0; i < kNumSplitVariants; ++i) v.push_back(i);
        return v;
    }
    if (o.precision != GW_FP64) return {0};
    if (o.flags & GW_FLAG_FP64_TILE128) return {1};
    const int forced = chi0_forced_variant();
    if (forced >= 0) return {forced < kNumChi0Variants ? forced : 0};
    std::vector<int> v;
    for (int i = 0; i < kNumChi0Variants; ++i) v.push_back(i);
    return v;
}

// Call scratch of a batched call: the autotuner's trial, and per group the
// work buffer and the tables (non-graph), or the work buffer only when a
// captured graph runs in the caller's workspace.
size_t batched_bytes(const gw_problem_t* probs, int nprob, const Opts& o, bool in_workspace) {
    size_t need = batch_tune_layout(probs, nprob, o).total;
    const bool graph = (o.flags & GW_FLAG_GRAPH) != 0;
    if (graph && !in_workspace) return need;
    for (const auto& g : batch_groups(probs, nprob, o))
        for (int v : possible_variants(o)) {
            const BatchPlan bp = build_batch(g.data(), static_cast<int>(g.size()), o, v);
            need = std::max(need, graph ? bp.work_bytes : align256(bp.work_bytes) + bp.table_bytes);
        }
    return need;
}

void run_chi0_batched(const gw_problem_t* probs, int nprob, const Opts& o, hipStream_t s,
                      char* base) {
    const std::vector<std::vector<gw_problem_t>> groups = batch_groups(probs, nprob, o);
    if (!(o.flags & GW_FLAG_GRAPH)) {
        for (const auto& g : groups) {
            const int n = static_cast<int>(g.size());
            const BatchPlan bp = build_batch(g.data(), n, o, batch_variant(g.data(), n, o, s, base));
            const size_t tab_off = align256(bp.work_bytes);
            // in stream order: the previous group's launches have read the tables
            upload_batch(bp, g.data(), o, base, base + tab_off, s);
            enqueue_batch(bp, g.data(), o, base, base + tab_off, s);
        }
        return;
    }
    const std::string key = batch_key(probs, nprob, o);
    GraphCache& gc = graph_cache();
    {
        std::lock_guard<std::mutex> lk(gc.mu);
        for (auto it = gc.lru.begin(); it != gc.lru.end(); ++it)
            if (it->key == key) {
                gc.lru.splice(gc.lru.begin(), gc.lru, it);
                GraphEntry& e = gc.lru.front();
                GW_HIP_TRY(hipGraphLaunch(e.exec, s));
                GW_HIP_TRY(hipEventRecord(e.last_use, s));
                return;
            }
    }
    require_alloc("captured graph");
    // first call: everything that allocates or copies happens before capture
    std::vector<BatchPlan> plans;
    for (const auto& g : groups) {
        const int n = static_cast<int>(g.size());
        plans.push_back(build_batch(g.data(), n, o, batch_variant(g.data(), n, o, s, base)));
        for (const gw_problem_t& pr : g) {
            const int tile = plans.back().split ? kSbTileI : chi0_variant_tile(plans.back().variant);
            (void)tile_order(ceil_div(pr.ng, tile), plans.back().split ? 4 : 8);
        }
    }
    const hipStream_t cs = capture_stream(s);
    (void)aux_ctx(cs);
    GraphEntry e;
    e.key = key;
    GW_HIP_TRY(hipGetDevice(&e.device));
    for (const BatchPlan& bp : plans)
        for (const BatchQ& q : bp.q) e.plans.push_back(q.plan);
    auto free_buffers = [&] {
        for (void* b : e.buffers) (void)hipFree(b);
        if (e.last_use) (void)hipEventDestroy(e.last_use);
    };
    // groups run one after another: one work buffer serves them all (the
    // caller's workspace if given); each group keeps its own tables
    auto alloc = [&](size_t bytes) {
        void* buf = nullptr;
        if (hipMalloc(&buf, std::max<size_t>(bytes, 256)) != hipSuccess) {
            (void)hipGetLastError();
            size_t fr = 0, tot = 0;
            (void)hipMemGetInfo(&fr, &tot);
            fail(GW_ENOMEM, "hipMalloc of " + std::to_string(bytes) +
                                " bytes for a captured batch failed (" + std::to_string(fr) +
                                " of " + std::to_string(tot) + " bytes free)");
        }
        e.buffers.push_back(buf);
        e.bytes += bytes;
        return static_cast<char*>(buf);
    };
    try {
        GW_HIP_TRY(hipEventCreateWithFlags(&e.last_use, hipEventDisableTiming));
        size_t work = 0;
        for (const BatchPlan& bp : plans) work = std::max(work, bp.work_bytes);
        char* wbuf = o.ws ? o.ws : alloc(work);
        std::vector<char*> tabs;
        for (size_t i = 0; i < groups.size(); ++i) {
            tabs.push_back(alloc(plans[i].table_bytes));
            upload_batch(plans[i], groups[i].data(), o, wbuf, tabs.back(), s);
        }
        hipGraph_t g = nullptr;
        GW_HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
        try {
            for (size_t i = 0; i < groups.size(); ++i)
                enqueue_batch(plans[i], groups[i].data(), o, wbuf, tabs[i], cs);
        } catch (...) {
            (void)hipStreamEndCapture(cs, &g);
            if (g) (void)hipGraphDestroy(g);
            (void)hipGetLastError();
            throw;
        }
        GW_HIP_TRY(hipStreamEndCapture(cs, &g));
        const hipError_t ie = hipGraphInstantiate(&e.exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        GW_HIP_TRY(ie);
        // the table uploads are on s; the replay follows them there
        GW_HIP_TRY(hipGraphLaunch(e.exec, s));
        GW_HIP_TRY(hipEventRecord(e.last_use, s));
    } catch (...) {
        if (e.exec) (void)hipGraphExecDestroy(e.exec);
        free_buffers();
        throw;
    }
    std::lock_guard<std::mutex> lk(gc.mu);
    gc.lru.push_front(std::move(e));
    const size_t max_n = env_size("GW_GRAPH_CACHE_MAX", 16);
    const size_t max_b = env_size("GW_GRAPH_CACHE_BYTES", size_t(64) << 30);
    size_t total = 0;
    for (const auto& x : gc.lru) total += x.bytes;
    while (gc.lru.size() > 1 && (gc.lru.size() > max_n || total > max_b)) {
        total -= gc.lru.back().bytes;
        retire_graph(gc.lru.back());
        gc.lru.pop_back();
    }
}

}  // namespace
}  // namespace gw

using namespace gw;

namespace gw {
namespace {

// Checks of gw_chi0's arguments (host only, before anything is enqueued);
// builds the plans, which may still reject a size.
Opts check_chi0_args(const gw_problem_t* probs, int nprob, const gw_opts_t* opts) {
    if (nprob < 0) fail(GW_EINVAL, "nprob must be >= 0");
    if (nprob > 0 && !probs) fail(GW_EINVAL, "probs is NULL");
    const Opts o = read_opts(opts);
    for (int q = 0; q < nprob; ++q) check_problem(probs[q], q);
    check_slices(o);
    for (int q = 0; q < nprob; ++q) (void)get_plan(probs[q].grid.n, probs[q].gvec, probs[q].ng);
    return o;
}

bool batched_call(int nprob, const Opts& o) {
    return nprob > 1 && (o.precision == GW_FP64 || o.precision == GW_SPLIT_BF16);
}

// M/Delta buffers of a per-problem call: 2 (MTXEL of the next chunk on the
// companion stream) unless GW_CHI0_BUFFERS=1 (MTXEL and the contraction in
// turn on the caller's stream).
int chi0_buffers() {
    static const int n = [] {
        const char* e = std::getenv("GW_CHI0_BUFFERS");
        return e && std::atoi(e) == 1 ? 1 : 2;
    }();
    return n;
}

// Scratch of a gw_chi0 call; in_workspace: as the call needs it in a caller
// workspace (a captured graph then keeps its work buffer there).
size_t chi0_call_bytes(const gw_problem_t* probs, int nprob, const Opts& o, bool in_workspace) {
    if (batched_call(nprob, o)) return batched_bytes(probs, nprob, o, in_workspace);
    size_t need = 0;
    for (int q = 0; q < nprob; ++q) {
        const PlanRef plan = get_plan(probs[q].grid.n, probs[q].gvec, probs[q].ng);
        need = std::max(need, chi0_layout(probs[q], o, *plan, chi0_buffers(), true).total);
    }
    return need;
}

void chi0_call(const gw_problem_t* probs, int nprob, const Opts& o, hipStream_t s) {
    char* base = call_scratch(chi0_call_bytes(probs, nprob, o, o.ws != nullptr), o, s);
    if (batched_call(nprob, o)) {
        run_chi0_batched(probs, nprob, o, s, base);
        return;
    }
    for (int q = 0; q < nprob; ++q) {
        const PlanRef plan = get_plan(probs[q].grid.n, probs[q].gvec, probs[q].ng);
        run_chi0(probs[q], o, s, base, chi0_layout(probs[q], o, *plan, chi0_buffers(), true));
    }
}

// The adjoint's problem with chi defaulted (it is not read) and its checks.
gw_problem_t backward_problem(const gw_problem_t* prob, const void* grad_chi) {
    if (!prob) fail(GW_EINVAL, "prob is NULL");
    gw_problem_t p = *prob;
    if (!p.chi) p.chi = reinterpret_cast<gw_c128*>(const_cast<void*>(grad_chi));
    check_problem(p, 0);
    return p;
}

// Scratch layout of gw_pseudobands: the host tables (copied in), then the
// phase table the prep kernel writes.
struct PbLayout {
    size_t o_keep = 0, o_idx = 0, o_off = 0, o_ord = 0, o_toff = 0, o_th = 0, staged = 0, o_ph = 0;
    size_t total = 0;
};

PbLayout pb_layout(int64_t nkeep, int64_t nidx, int64_t nslices, int64_t n_xi) {
    PbLayout L;
    const int64_t ntheta = nidx * (nslices > 0 ? n_xi : 0);
    Carver cv;
    L.o_keep = cv.take(static_cast<size_t>(nkeep) * sizeof(int32_t));
    L.o_idx = cv.take(static_cast<size_t>(nidx) * sizeof(int32_t));
    L.o_off = cv.take(static_cast<size_t>(nslices + 1) * sizeof(int32_t));
    L.o_ord = cv.take(static_cast<size_t>(nslices) * sizeof(int32_t));
    L.o_toff = cv.take(static_cast<size_t>(nslices) * sizeof(int64_t));
    L.o_th = cv.take(static_cast<size_t>(ntheta) * sizeof(double));
    L.staged = cv.off;
    L.o_ph = cv.take(static_cast<size_t>(ntheta) * sizeof(double2));
    L.total = cv.off;
    return L;
}

}  // namespace
}  // namespace gw

extern "C" {

gw_status_t gw_mtxel(const gw_grid_t* grid, const gw_c128* psi_v, int32_t nv,
                     const gw_c128* psi_c, int32_t nc, const int32_t* gvec, int32_t ng,
                     int64_t pair_begin, int64_t pair_count, gw_c128* m_out, void* stream) {
    return guarded([&] {
        sweep_retired();
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
        const PlanRef plan = get_plan(grid->n, gvec, ng);
        // the linear pair range as rectangles of at most kBatch pairs: partial
        // rows alone, whole rows in blocks of up to 4 valence bands (the MTXEL
        // tile height) cut into column ranges, written with row stride nc
        constexpr int64_t kBatch = 4096;
        struct Piece {
            Rect r;
            int64_t row0;  // output row of the rectangle's first pair
        };
        std::vector<Piece> rects;
        int64_t p0 = pair_begin;
        const int64_t pend = pair_begin + pair_count;
        while (p0 < pend) {
            const int v = static_cast<int>(p0 / nc), c = static_cast<int>(p0 % nc);
            if (c != 0 || pend - p0 < nc) {  // part of one row
                const int64_t cnt = std::min<int64_t>({nc - c, pend - p0, kBatch});
                rects.push_back({Rect{v, 1, c, static_cast<int32_t>(cnt)}, p0 - pair_begin});
                p0 += cnt;
                continue;
            }
            const int vb = static_cast<int>(std::min<int64_t>((pend - p0) / nc, 4));
            const int cw = static_cast<int>(std::min<int64_t>(nc, kBatch / vb));
            for (int c0 = 0; c0 < nc; c0 += cw)
                rects.push_back({Rect{v, vb, c0, std::min(cw, nc - c0)}, p0 - pair_begin + c0});
            p0 += static_cast<int64_t>(vb) * nc;
        }
        double2* t2 = static_cast<double2*>(scratch(t2_elems(*plan, kBatch) * sizeof(double2), s));
        for (const auto& rr : rects)
            launch_mtxel(*plan, reinterpret_cast<const double2*>(psi_v),
                         reinterpret_cast<const double2*>(psi_c), rr.r, grid->volume, t2,
                         reinterpret_cast<double2*>(m_out) + rr.row0 * ng, s, nc);
        mark_plan_used(*plan, s);
    });
}

gw_status_t gw_chi0(const gw_problem_t* probs, int32_t nprob, const gw_opts_t* opts,
                    void* stream) {
    return guarded([&] {
        sweep_retired();
        const Opts o = check_chi0_args(probs, nprob, opts);
        chi0_call(probs, nprob, o, static_cast<hipStream_t>(stream));
    });
}

size_t gw_workspace_bytes(const gw_problem_t* probs, int32_t nprob, const gw_opts_t* opts,
                          int32_t backward) {
    size_t out = 0;
    const gw_status_t st = guarded([&] {
        if (!backward) {
            const Opts o = check_chi0_args(probs, nprob, opts);
            out = chi0_call_bytes(probs, nprob, o, true);
            return;
        }
        if (nprob < 1) fail(GW_EINVAL, "the adjoint takes one problem");
        const Opts o = read_opts(opts);
        static const gw_c128 dummy{0.0, 0.0};
        const gw_problem_t p = backward_problem(probs, &dummy);
        const PlanRef plan = get_plan(p.grid.n, p.gvec, p.ng);
        out = chi0_backward_bytes(*plan, p, true, true, true, o.pair_chunk);
    });
    return st == GW_OK ? out : static_cast<size_t>(-1);
}

size_t gw_pseudobands_workspace_bytes(int32_t nkeep, int64_t nidx, int32_t nslices,
                                      int32_t n_xi) {
    if (nkeep < 0 || nidx < 0 || nslices < 0 || n_xi < 0) return static_cast<size_t>(-1);
    return pb_layout(nkeep, nidx, nslices, n_xi).total;
}

gw_status_t gw_pseudobands(const gw_c128* psi, const double* e, int32_t nb, int64_t nr,
                           const int32_t* keep, int32_t nkeep, const int32_t* slice_idx,
                           const int32_t* slice_off, int32_t nslices, int32_t n_xi,
                           const double* theta, gw_c128* out_psi, double* out_e,
                           void* workspace, size_t workspace_bytes, void* stream) {
    return guarded([&] {
        sweep_retired();
        if (nb < 0 || nr < 1) fail(GW_EINVAL, "nb must be >= 0 and nr >= 1");
        if (nr >= (int64_t(1) << 31)) fail(GW_EINVAL, "grid has 2^31 or more points");
        if (nkeep < 0 || nslices < 0) fail(GW_EINVAL, "nkeep and nslices must be >= 0");
        if (nkeep > 65535 || nslices > 65535)
            fail(GW_EUNSUPPORTED, "at most 65535 protected bands and 65535 slices per call");
        if (nkeep > 0 && !keep) fail(GW_EINVAL, "keep is NULL");
        if (nslices > 0) {
            if (!slice_idx || !slice_off || !theta) fail(GW_EINVAL, "slice tables are NULL");
            if (n_xi < 1 || n_xi > kMaxPseudoXi)
                fail(GW_EINVAL, "n_xi must lie in [1, " + std::to_string(kMaxPseudoXi) + "]");
            if (slice_off[0] != 0) fail(GW_EINVAL, "slice_off[0] must be 0");
            for (int sl = 0; sl < nslices; ++sl)
                if (slice_off[sl + 1] <= slice_off[sl])
                    fail(GW_EINVAL, "slice " + std::to_string(sl) + " is empty");
        }
        const int64_t nidx = nslices > 0 ? slice_off[nslices] : 0;
        for (int i = 0; i < nkeep; ++i)
            if (keep[i] < 0 || keep[i] >= nb) fail(GW_EINVAL, "keep index out of range");
        for (int64_t i = 0; i < nidx; ++i)
            if (slice_idx[i] < 0 || slice_idx[i] >= nb) fail(GW_EINVAL, "slice index out of range");
        const int64_t ntheta = nidx * (nslices > 0 ? n_xi : 0);
        for (int64_t i = 0; i < ntheta; ++i)
            if (!std::isfinite(theta[i])) fail(GW_EINVAL, "theta must be finite");
        const int nout = nkeep + nslices * (nslices > 0 ? n_xi : 0);
        if (nout == 0) return;
        if (!psi || !e) fail(GW_EINVAL, "psi / e is NULL");
        if (!out_psi || !out_e) fail(GW_EINVAL, "out_psi / out_e is NULL");
        if (workspace && (reinterpret_cast<uintptr_t>(workspace) & 255))
            fail(GW_EINVAL, "workspace must be 256-byte aligned");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const PbLayout L = pb_layout(nkeep, nidx, nslices, nslices > 0 ? n_xi : 0);
        Opts o;
        o.ws = static_cast<char*>(workspace);
        o.ws_bytes = workspace ? workspace_bytes : 0;
        char* dev = call_scratch(L.total, o, s);
        // the host tables, packed and copied in stream order into scratch
        std::vector<int64_t> toff(nslices);
        for (int sl = 0; sl < nslices; ++sl) toff[sl] = static_cast<int64_t>(slice_off[sl]) * n_xi;
        // largest slices first, so that the longest workgroups start early
        std::vector<int32_t> order(nslices);
        for (int sl = 0; sl < nslices; ++sl) order[sl] = sl;
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
            return slice_off[a + 1] - slice_off[a] > slice_off[b + 1] - slice_off[b];
        });
        std::vector<char> host(L.staged, 0);
        auto put = [&](size_t off, const void* src, size_t n) {
            if (n) std::memcpy(host.data() + off, src, n);
        };
        put(L.o_keep, keep, static_cast<size_t>(nkeep) * sizeof(int32_t));
        put(L.o_idx, slice_idx, static_cast<size_t>(nidx) * sizeof(int32_t));
        if (nslices > 0) put(L.o_off, slice_off, static_cast<size_t>(nslices + 1) * sizeof(int32_t));
        put(L.o_ord, order.data(), order.size() * sizeof(int32_t));
        put(L.o_toff, toff.data(), toff.size() * sizeof(int64_t));
        put(L.o_th, theta, static_cast<size_t>(ntheta) * sizeof(double));
        stage_h2d(dev, host.data(), L.staged, s);
        PseudoTables t{reinterpret_cast<const int*>(dev + L.o_keep),
                       reinterpret_cast<const int*>(dev + L.o_idx),
                       reinterpret_cast<const int*>(dev + L.o_off),
                       reinterpret_cast<const int*>(dev + L.o_ord),
                       reinterpret_cast<const double*>(dev + L.o_th),
                       reinterpret_cast<const int64_t*>(dev + L.o_toff),
                       reinterpret_cast<double2*>(dev + L.o_ph)};
        launch_pseudobands(reinterpret_cast<const double2*>(psi), e, nr, t, nkeep, nslices,
                           nslices > 0 ? n_xi : 1, reinterpret_cast<double2*>(out_psi), out_e, s);
    });
}

gw_status_t gw_chi0_backward(const gw_problem_t* prob, const gw_c128* grad_chi,
                             gw_c128* grad_psi_v, gw_c128* grad_psi_c, double* grad_e_v,
                             double* grad_e_c, const gw_opts_t* opts, void* stream) {
    return guarded([&] {
        sweep_retired();
        const Opts o = read_opts(opts);
        const gw_problem_t p = backward_problem(prob, grad_chi);
        if (!grad_chi) fail(GW_EINVAL, "grad_chi is NULL");
        if (o.precision != GW_FP64) fail(GW_EUNSUPPORTED, "the adjoint is FP64 only");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const PlanRef plan = get_plan(p.grid.n, p.gvec, p.ng);
        const size_t need = chi0_backward_bytes(*plan, p, grad_psi_v != nullptr,
                                                grad_psi_c != nullptr,
                                                grad_e_v != nullptr || grad_e_c != nullptr,
                                                o.pair_chunk);
        char* base = call_scratch(need, o, s);
        AuxCtx& ax = aux_ctx(s);
        run_chi0_backward(*plan, p, reinterpret_cast<const double2*>(grad_chi),
                          reinterpret_cast<double2*>(grad_psi_v),
                          reinterpret_cast<double2*>(grad_psi_c), grad_e_v, grad_e_c, o.spin,
                          o.pair_chunk, s, base, ax.aux, ax.ev);
        mark_plan_used(*plan, s);
    });
}

gw_status_t gw_chi0_backward_from_m(const gw_problem_t* prob, const gw_c128* m_keep,
                                    const gw_c128* grad_chi, gw_c128* grad_psi_v,
                                    gw_c128* grad_psi_c, double* grad_e_v, double* grad_e_c,
                                    const gw_opts_t* opts, void* stream) {
    return guarded([&] {
        sweep_retired();
        const Opts o = read_opts(opts);
        const gw_problem_t p = backward_problem(prob, grad_chi);
        if (!grad_chi) fail(GW_EINVAL, "grad_chi is NULL");
        if (static_cast<int64_t>(p.nv) * p.nc > 0 && !m_keep) fail(GW_EINVAL, "m_keep is NULL");
        if (o.precision != GW_FP64) fail(GW_EUNSUPPORTED, "the adjoint is FP64 only");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const PlanRef plan = get_plan(p.grid.n, p.gvec, p.ng);
        const size_t need = chi0_backward_bytes(*plan, p, grad_psi_v != nullptr,
                                                grad_psi_c != nullptr,
                                                grad_e_v != nullptr || grad_e_c != nullptr,
                                                o.pair_chunk, true);
        char* base = call_scratch(need, o, s);
        AuxCtx& ax = aux_ctx(s);
        run_chi0_backward(*plan, p, reinterpret_cast<const double2*>(grad_chi),
                          reinterpret_cast<double2*>(grad_psi_v),
                          reinterpret_cast<double2*>(grad_psi_c), grad_e_v, grad_e_c, o.spin,
                          o.pair_chunk, s, base, ax.aux, ax.ev,
                          reinterpret_cast<const double2*>(m_keep));
        mark_plan_used(*plan, s);
    });
}

size_t gw_chi0_backward_from_m_workspace_bytes(const gw_problem_t* prob, const gw_opts_t* opts) {
    size_t out = 0;
    const gw_status_t st = guarded([&] {
        const Opts o = read_opts(opts);
        static const gw_c128 dummy{0.0, 0.0};
        const gw_problem_t p = backward_problem(prob, &dummy);
        const PlanRef plan = get_plan(p.grid.n, p.gvec, p.ng);
        out = chi0_backward_bytes(*plan, p, true, true, true, o.pair_chunk, true);
    });
    return st == GW_OK ? out : static_cast<size_t>(-1);
}

// ---------------------------------------------------------------- fixed scratch

}  // extern "C"

namespace gw {
namespace {

// Device scratch of gw_chi0_fixed: a file-scope array that every device the
// library runs on holds from module load until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol): fixed_scratch() looks its device address up once
// per device, with that device current, and every use goes through it.
constexpr size_t kFixedScratchBytes = size_t(128) << 20;
__device__ __align__(256) char g_fixed_scratch[kFixedScratchBytes];

char* fixed_scratch() {
    static std::mutex mu;
    static std::map<int, char*> by_device;
    int dev = 0;
    GW_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    auto it = by_device.find(dev);
    if (it != by_device.end()) return it->second;
    void* ptr = nullptr;
    GW_HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(g_fixed_scratch)));
    if (!ptr) fail(GW_EINTERNAL, "no device address for the fixed scratch");
    by_device[dev] = static_cast<char*>(ptr);
    return static_cast<char*>(ptr);
}

// Throws in no-allocation mode when the tile-order table a contraction of
// `ncols` columns would use does not exist yet.
void require_tile_orders(const Opts& o, int ncols, int variant) {
    if (sliced_32x32(o.precision))
        (void)tile_order(ceil_div(ncols, kSbTileI), 4);
    else if (o.precision == GW_FP64)
        (void)tile_order(ceil_div(ncols, chi0_variant_tile(variant)));
    else
        (void)tile_order(ceil_div(ncols, kSplitTile));
}

}  // namespace
}  // namespace gw

extern "C" {

size_t gw_chi0_fixed_scratch_bytes(void) { return kFixedScratchBytes; }

gw_status_t gw_chi0_fixed(const gw_problem_t* prob, const gw_opts_t* opts, void* stream) {
    return guarded([&] {
        if (!prob) fail(GW_EINVAL, "prob is NULL");
        Opts o = read_opts(opts);
        check_problem(*prob, 0);
        if (o.ws) fail(GW_EINVAL, "gw_chi0_fixed uses its fixed scratch: workspace must be NULL");
        if (o.flags & (GW_FLAG_GRAPH | GW_FLAG_AUTOTUNE))
            fail(GW_EINVAL, "GW_FLAG_GRAPH and GW_FLAG_AUTOTUNE allocate: not with gw_chi0_fixed");
        check_slices(o);
        hipStream_t s = static_cast<hipStream_t>(stream);
        char* base = fixed_scratch();  // once per device; no allocation
        NoAllocScope no_alloc;
        const PlanRef plan = get_plan(prob->grid.n, prob->gvec, prob->ng);  // must exist
        // the largest chunk up to the requested one whose buffers (one M/Delta
        // buffer, everything on the caller's stream, whole tiles) fit
        auto need = [&](int chunk) {
            Opts oc = o;
            oc.pair_chunk = chunk;
            return chi0_layout(*prob, oc, *plan, 1, false).total;
        };
        if (need(1) > kFixedScratchBytes)
            fail(GW_EUNSUPPORTED, "this problem needs " + std::to_string(need(1)) +
                                      " bytes of scratch at one pair per chunk; the fixed scratch "
                                      "holds " + std::to_string(kFixedScratchBytes));
        int lo = 1, hi = o.pair_chunk;
        while (lo < hi) {
            const int mid = lo + (hi - lo + 1) / 2;
            if (need(mid) <= kFixedScratchBytes) lo = mid; else hi = mid - 1;
        }
        o.pair_chunk = lo;
        const Chi0Layout L = chi0_layout(*prob, o, *plan, 1, false);
        if (static_cast<int64_t>(prob->nv) * prob->nc > 0) {
            int variant = 0;
            if (o.precision == GW_FP64) {
                const std::vector<Chunk> ch = make_chunks(*prob, L.cs);
                variant = (o.flags & GW_FLAG_FP64_TILE128)
                              ? 1
                              : std::max(0, lookup_variant("f64", prob->ng, ch[0].kc));
            }
            require_tile_orders(o, prob->ng, variant);
        }
        run_chi0(*prob, o, s, base, L);
    });
}

// ---------------------------------------------------------------- static subspace

size_t gw_subspace_basis_workspace_bytes(int32_t ng, int32_t n_eig, const gw_diag_opts_t* opts) {
    if (ng < 1 || n_eig < 1 || n_eig > ng) return static_cast<size_t>(-1);
    return subspace_basis_bytes(ng, n_eig, opts ? opts->guard : 0, opts && opts->weight);
}

gw_status_t gw_subspace_basis(const gw_c128* chi_static, int32_t ng, int32_t n_eig,
                              gw_c128* basis, double* eigenvalues, const gw_diag_opts_t* opts,
                              gw_diag_info_t* info, void* stream) {
    return guarded([&] {
        sweep_retired();
        if (ng < 1) fail(GW_EINVAL, "ng must be >= 1");
        if (n_eig < 1 || n_eig > ng) fail(GW_EINVAL, "n_eig must lie in [1, ng]");
        if (!chi_static || !basis || !eigenvalues) fail(GW_EINVAL, "a device pointer is NULL");
        DiagParams prm;
        Opts o;
        if (opts) {
            if (opts->tol < 0.0 || !std::isfinite(opts->tol)) fail(GW_EINVAL, "tol must be >= 0");
            if (opts->max_iter < 0 || opts->guard < 0 || opts->max_degree < 0)
                fail(GW_EINVAL, "max_iter, guard and max_degree must be >= 0");
            if (opts->tol > 0.0) prm.tol = opts->tol;
            if (opts->max_iter > 0) prm.max_iter = opts->max_iter;
            if (opts->max_degree > 0) prm.max_degree = opts->max_degree;
            prm.guard = opts->guard;
            prm.seed = opts->seed;
            prm.weight = opts->weight;
            o.ws = static_cast<char*>(opts->workspace);
            o.ws_bytes = opts->workspace ? opts->workspace_bytes : 0;
            if (o.ws && (reinterpret_cast<uintptr_t>(o.ws) & 255))
                fail(GW_EINVAL, "workspace must be 256-byte aligned");
        }
        hipStream_t s = static_cast<hipStream_t>(stream);
        char* base = call_scratch(subspace_basis_bytes(ng, n_eig, prm.guard, prm.weight), o, s);
        const DiagResult r = run_subspace_basis(reinterpret_cast<const double2*>(chi_static), ng,
                                                n_eig, reinterpret_cast<double2*>(basis),
                                                eigenvalues, prm, base, s);
        if (info) {
            info->iterations = r.iterations;
            info->degree = r.degree;
            info->residual = r.residual;
            info->bound = r.bound;
            info->sweeps = r.sweeps;
        }
    });
}

size_t gw_chi0_subspace_workspace_bytes(const gw_problem_t* prob, int32_t n_eig,
                                        const gw_opts_t* opts) {
    size_t out = 0;
    const gw_status_t st = guarded([&] {
        if (!prob) fail(GW_EINVAL, "prob is NULL");
        if (n_eig < 1) fail(GW_EINVAL, "n_eig must be >= 1");
        const Opts o = read_opts(opts);
        gw_problem_t p = *prob;
        static gw_c128 dummy{0.0, 0.0};
        if (!p.chi) p.chi = &dummy;
        check_problem(p, 0);
        const PlanRef plan = get_plan(p.grid.n, p.gvec, p.ng);
        out = chi0_layout(p, o, *plan, 2, true, n_eig).total;
    });
    return st == GW_OK ? out : static_cast<size_t>(-1);
}

gw_status_t gw_chi0_subspace(const gw_problem_t* prob, const gw_c128* basis,
                             const double* weight, int32_t n_eig, const gw_opts_t* opts,
                             void* stream) {
    return guarded([&] {
        sweep_retired();
        if (!prob) fail(GW_EINVAL, "prob is NULL");
        const Opts o = read_opts(opts);
        check_problem(*prob, 0);
        if (n_eig < 1 || n_eig > prob->ng) fail(GW_EINVAL, "n_eig must lie in [1, ng]");
        if (!basis) fail(GW_EINVAL, "basis is NULL");
        if (o.flags & GW_FLAG_GRAPH) fail(GW_EUNSUPPORTED, "GW_FLAG_GRAPH is for batched gw_chi0");
        check_slices(o);
        hipStream_t s = static_cast<hipStream_t>(stream);
        const PlanRef plan = get_plan(prob->grid.n, prob->gvec, prob->ng);
        const Chi0Layout L = chi0_layout(*prob, o, *plan, 2, true, n_eig);
        char* base = call_scratch(L.total, o, s);
        run_chi0(*prob, o, s, base, L, reinterpret_cast<const double2*>(basis), weight);
    });
}

// ---------------------------------------------------------------- kept matrix elements

gw_status_t gw_chi0_keep_m(const gw_problem_t* prob, gw_c128* m_keep, const gw_opts_t* opts,
                           void* stream) {
    return guarded([&] {
        sweep_retired();
        if (!prob) fail(GW_EINVAL, "prob is NULL");
        const Opts o = read_opts(opts);
        check_problem(*prob, 0);
        check_slices(o);
        if (static_cast<int64_t>(prob->nv) * prob->nc > 0 && !m_keep)
            fail(GW_EINVAL, "m_keep is NULL");
        if (o.flags & GW_FLAG_GRAPH) fail(GW_EUNSUPPORTED, "GW_FLAG_GRAPH is for batched gw_chi0");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const PlanRef plan = get_plan(prob->grid.n, prob->gvec, prob->ng);
        const Chi0Layout L = chi0_layout(*prob, o, *plan, chi0_buffers(), true);
        char* base = call_scratch(L.total, o, s);
        MKeep mk;
        mk.out = reinterpret_cast<double2*>(m_keep);
        run_chi0(*prob, o, s, base, L, nullptr, nullptr, mk);
    });
}

size_t gw_chi0_from_m_workspace_bytes(const gw_problem_t* prob, int32_t n_eig,
                                      const gw_opts_t* opts) {
    size_t out = 0;
    const gw_status_t st = guarded([&] {
        if (!prob) fail(GW_EINVAL, "prob is NULL");
        const Opts o = read_opts(opts);
        gw_problem_t p = *prob;
        static gw_c128 dummy{0.0, 0.0};
        if (!p.chi) p.chi = &dummy;
        check_problem(p, 0);
        const PlanRef plan = get_plan(p.grid.n, p.gvec, p.ng);
        out = chi0_layout(p, o, *plan, 2, true, n_eig > 0 ? n_eig : 0).total;
    });
    return st == GW_OK ? out : static_cast<size_t>(-1);
}

gw_status_t gw_chi0_from_m(const gw_problem_t* prob, const gw_c128* m_keep, const gw_c128* basis,
                           const double* weight, int32_t n_eig, const gw_opts_t* opts,
                           void* stream) {
    return guarded([&] {
        sweep_retired();
        if (!prob) fail(GW_EINVAL, "prob is NULL");
        const Opts o = read_opts(opts);
        check_problem(*prob, 0);
        check_slices(o);
        if (static_cast<int64_t>(prob->nv) * prob->nc > 0 && !m_keep)
            fail(GW_EINVAL, "m_keep is NULL");
        if (basis && (n_eig < 1 || n_eig > prob->ng)) fail(GW_EINVAL, "n_eig must lie in [1, ng]");
        if (!basis && n_eig != 0) fail(GW_EINVAL, "n_eig must be 0 when basis is NULL");
        if (o.flags & GW_FLAG_GRAPH) fail(GW_EUNSUPPORTED, "GW_FLAG_GRAPH is for batched gw_chi0");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const PlanRef plan = get_plan(prob->grid.n, prob->gvec, prob->ng);
        const Chi0Layout L = chi0_layout(*prob, o, *plan, 2, true, basis ? n_eig : 0);
        char* base = call_scratch(L.total, o, s);
        MKeep mk;
        mk.in = reinterpret_cast<const double2*>(m_keep);
        run_chi0(*prob, o, s, base, L, reinterpret_cast<const double2*>(basis),
                 basis ? weight : nullptr, mk);
    });
}

// ---------------------------------------------------------------- inverse dielectric matrix

size_t gw_epsinv_workspace_bytes(int32_t ng, int32_t nz) {
    if (ng < 1 || nz < 1) return static_cast<size_t>(-1);
    return epsinv_bytes(ng, nz);
}

gw_status_t gw_epsinv(const gw_c128* chi, int32_t ng, int32_t nz, const double* vcoul,
                      gw_c128* epsinv, void* workspace, size_t workspace_bytes, void* stream) {
    return guarded([&] {
        sweep_retired();
        if (ng < 1 || nz < 1) fail(GW_EINVAL, "ng and nz must be >= 1");
        if (nz > 65535) fail(GW_EUNSUPPORTED, "at most 65535 frequencies per call");
        if (!chi || !vcoul || !epsinv) fail(GW_EINVAL, "a device pointer is NULL");
        if (static_cast<const void*>(chi) == static_cast<const void*>(epsinv))
            fail(GW_EINVAL, "chi and epsinv must not be the same buffer");
        Opts o;
        o.ws = static_cast<char*>(workspace);
        o.ws_bytes = workspace ? workspace_bytes : 0;
        if (o.ws && (reinterpret_cast<uintptr_t>(o.ws) & 255))
            fail(GW_EINVAL, "workspace must be 256-byte aligned");
        hipStream_t s = static_cast<hipStream_t>(stream);
        char* base = call_scratch(epsinv_bytes(ng, nz), o, s);
        run_epsinv(reinterpret_cast<const double2*>(chi), ng, nz, vcoul,
                   reinterpret_cast<double2*>(epsinv), base, s);
    });
}

// ---------------------------------------------------------------- GPP off-diagonal self-energy

size_t gw_gpp_sigma_workspace_bytes(int32_t ns, int32_t ng, int32_t ne) {
    if (ns < 0 || ng < 0 || ne < 1) return static_cast<size_t>(-1);
    return gpp_bytes(ns, ng, ne);
}

gw_status_t gw_gpp_sigma(const gw_c128* m, int32_t nb, int32_t ns, int32_t ng,
                         const double* e_n, const int32_t* occupied, const gw_c128* energies,
                         int32_t ne, const gw_c128* omega2, const double* wtilde,
                         const double* vcoul, gw_c128* sigma, void* workspace,
                         size_t workspace_bytes, void* stream) {
    return guarded([&] {
        sweep_retired();
        if (nb < 0 || ns < 1 || ng < 1 || ne < 1) fail(GW_EINVAL, "need nb >= 0, ns, ng, ne >= 1");
        if (ne > 65535) fail(GW_EUNSUPPORTED, "at most 65535 energies per call");
        if (!sigma || !energies) fail(GW_EINVAL, "sigma / energies is NULL");
        if (nb > 0 && (!m || !e_n || !occupied || !omega2 || !wtilde || !vcoul))
            fail(GW_EINVAL, "an input pointer is NULL");
        for (int32_t i = 0; i < ne; ++i)
            if (!std::isfinite(energies[i].re) || !std::isfinite(energies[i].im))
                fail(GW_EINVAL, "energies must be finite");
        for (int32_t n = 0; n < nb; ++n)
            if (!std::isfinite(e_n[n])) fail(GW_EINVAL, "e_n must be finite");
        Opts o;
        o.ws = static_cast<char*>(workspace);
        o.ws_bytes = workspace ? workspace_bytes : 0;
        if (o.ws && (reinterpret_cast<uintptr_t>(o.ws) & 255))
            fail(GW_EINVAL, "workspace must be 256-byte aligned");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const size_t need = gpp_bytes(ns, ng, ne);
        char* base = call_scratch(need, o, s);
        // the energies follow the first-GEMM buffer, staged in stream order
        const size_t e_off = need - ((static_cast<size_t>(ne) * sizeof(double2) + 255) & ~size_t(255));
        stage_h2d(base + e_off, energies, static_cast<size_t>(ne) * sizeof(double2), s);
        run_gpp_sigma(reinterpret_cast<const double2*>(m), nb, ns, ng, e_n, occupied,
                      reinterpret_cast<const double2*>(base + e_off), ne,
                      reinterpret_cast<const double2*>(omega2), wtilde, vcoul,
                      reinterpret_cast<double2*>(sigma), base, s);
    });
}

// ---------------------------------------------------------------- dense building blocks

gw_status_t gw_zgemm(char opa, char opb, int32_t m, int32_t n, int32_t k, gw_c128 alpha,
                     const gw_c128* a, int64_t lda, int64_t stride_a, const gw_c128* b,
                     int64_t ldb, int64_t stride_b, gw_c128 beta, gw_c128* c, int64_t ldc,
                     int64_t stride_c, int32_t batch, void* stream) {
    return guarded([&] {
        auto op = [](char x) {
            switch (x) {
                case 'N': case 'n': return kOpN;
                case 'T': case 't': return kOpT;
                case 'C': case 'c': return kOpC;
                default: fail(GW_EINVAL, std::string("op must be N, T or C, got ") + x);
            }
        };
        const ZOp oa = op(opa), ob = op(opb);
        if (m < 0 || n < 0 || k < 0 || batch < 0) fail(GW_EINVAL, "sizes must be >= 0");
        if (m == 0 || n == 0 || batch == 0) return;
        const int64_t acols = oa == kOpN ? k : m, bcols = ob == kOpN ? n : k;
        const int64_t arows = oa == kOpN ? m : k, brows = ob == kOpN ? k : n;
        if (!c) fail(GW_EINVAL, "c is NULL");
        if (ldc < n) fail(GW_EINVAL, "ldc < n");
        if (k > 0) {
            if (!a || !b) fail(GW_EINVAL, "a / b is NULL");
            if (lda < acols || ldb < bcols) fail(GW_EINVAL, "lda / ldb below the row length");
        }
        (void)arows;
        (void)brows;
        if (batch > 1 && stride_c < static_cast<int64_t>(m - 1) * ldc + n)
            fail(GW_EINVAL, "stride_c must hold a whole C (products must not overlap)");
        if (batch > 65535) fail(GW_EUNSUPPORTED, "at most 65535 products per call");
        ZGemm g;
        g.m = m;
        g.n = n;
        g.k = k;
        g.a = reinterpret_cast<const double2*>(a);
        g.lda = lda;
        g.stride_a = stride_a;
        g.b = reinterpret_cast<const double2*>(b);
        g.ldb = ldb;
        g.stride_b = stride_b;
        g.c = reinterpret_cast<double2*>(c);
        g.ldc = ldc;
        g.stride_c = stride_c;
        g.alpha = make_double2(alpha.re, alpha.im);
        g.beta = make_double2(beta.re, beta.im);
        g.batch = batch;
        launch_zgemm(oa, ob, g, static_cast<hipStream_t>(stream));
    });
}

size_t gw_heev_workspace_bytes(int32_t n, int32_t batch) {
    if (n < 1 || batch < 1) return static_cast<size_t>(-1);
    const size_t nn = static_cast<size_t>(n) * n * batch * sizeof(double2);
    return ((nn + 255) & ~size_t(255)) + jacobi_work_bytes(n, batch) +
           ((static_cast<size_t>(n) * batch * sizeof(int) + 255) & ~size_t(255));
}

gw_status_t gw_heev(const gw_c128* a, int32_t n, int32_t batch, double* w, gw_c128* v,
                    double tol, void* workspace, size_t workspace_bytes, void* stream) {
    return guarded([&] {
        sweep_retired();
        if (n < 1 || batch < 1) fail(GW_EINVAL, "n and batch must be >= 1");
        if (batch > 65535) fail(GW_EUNSUPPORTED, "at most 65535 matrices per call");
        if (!a || !w || !v) fail(GW_EINVAL, "a device pointer is NULL");
        if (!(tol >= 0.0) || !std::isfinite(tol)) fail(GW_EINVAL, "tol must be >= 0");
        Opts o;
        o.ws = static_cast<char*>(workspace);
        o.ws_bytes = workspace ? workspace_bytes : 0;
        if (o.ws && (reinterpret_cast<uintptr_t>(o.ws) & 255))
            fail(GW_EINVAL, "workspace must be 256-byte aligned");
        hipStream_t s = static_cast<hipStream_t>(stream);
        char* base = call_scratch(gw_heev_workspace_bytes(n, batch), o, s);
        const size_t nn = static_cast<size_t>(n) * n;
        const size_t abytes = (nn * batch * sizeof(double2) + 255) & ~size_t(255);
        double2* ac = reinterpret_cast<double2*>(base);
        void* jw = base + abytes;
        int* perm_d = reinterpret_cast<int*>(base + abytes + jacobi_work_bytes(n, batch));
        GW_HIP_TRY(hipMemcpyAsync(ac, a, nn * batch * sizeof(double2), hipMemcpyDeviceToDevice, s));
        double2* vtmp = reinterpret_cast<double2*>(v);
        (void)jacobi_eigh(ac, vtmp, n, batch, tol > 0.0 ? tol : 1e-15, 100, jw, s);
        // eigenvalues in increasing order, eigenvectors to match
        // (the diagonals gathered into w on the device, then one plain copy)
        std::vector<double> dg(static_cast<size_t>(n) * batch);
        launch_diag_re(ac, n, batch, w, s);
        GW_HIP_TRY(hipMemcpyAsync(dg.data(), w, dg.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        GW_HIP_TRY(hipStreamSynchronize(s));
        std::vector<int> perm(static_cast<size_t>(n) * batch);
        std::vector<double> wv(static_cast<size_t>(n) * batch);
        for (int b = 0; b < batch; ++b) {
            int* pb = perm.data() + static_cast<size_t>(b) * n;
            const double* db = dg.data() + static_cast<size_t>(b) * n;
            for (int i = 0; i < n; ++i) pb[i] = i;
            std::stable_sort(pb, pb + n, [&](int x, int y) { return db[x] < db[y]; });
            for (int i = 0; i < n; ++i) wv[static_cast<size_t>(b) * n + i] = db[pb[i]];
        }
        GW_HIP_TRY(hipMemcpyAsync(perm_d, perm.data(), perm.size() * sizeof(int),
                                  hipMemcpyHostToDevice, s));
        GW_HIP_TRY(hipMemcpyAsync(w, wv.data(), wv.size() * sizeof(double), hipMemcpyHostToDevice, s));
        // v <- v[:, perm] through the matrix buffer
        GW_HIP_TRY(hipMemcpyAsync(ac, vtmp, nn * batch * sizeof(double2), hipMemcpyDeviceToDevice, s));
        launch_gather_cols(ac, vtmp, n, n, n, perm_d, batch, s);
        GW_HIP_TRY(hipStreamSynchronize(s));  // the host vectors above are read by now
    });
}

const char* gw_last_error(void) { return g_last_error.c_str(); }

gw_status_t gw_release(void) {
    return guarded([&] {
        release_graphs();
        release_plans();
        drain_retired();
        release_aux();
        release_scratch();
        release_tile_orders();
        release_staging();
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
