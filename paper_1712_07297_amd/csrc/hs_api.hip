// Host orchestration and C ABI of the hierarchical solver (include/hs.h).
//
// hs_factor runs Alg. 1 level by level: the host plans one level from the
// symbolic analysis and the level's cluster sizes (the ranks of the level
// below decide them, so the stream is synchronised once per level), the
// device assembles the level's dense blocks (Sec. 5.3 keeps every non-zero
// block dense) and processes the colours of Sec. 3.4 one after the other.
// hs_solve runs Alg. 2; hs_pcg / hs_gmres use it as the preconditioner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "hs.h"
#include "kernels.h"
#include "symbolic.h"

namespace hs {

// ------------------------------------------------------------------ errors

static thread_local std::string g_err;

static int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

// For the serving runtime (same library): record the calling thread's message.
int fail_with(int code, const char* msg) { return fail(code, msg); }

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t _e = (expr);                                                              \
        if (_e != hipSuccess)                                                                \
            return fail(HS_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e));    \
    } while (0)

// --------------------------------------------------------------- allocator

// An installed allocator is stream-ordered: alloc(bytes, stream, ctx) gives
// memory for use on `stream`, free(ptr, stream, ctx) takes it back for reuse
// by later work on that stream.
static void* (*g_alloc_fn)(size_t, void*, void*) = nullptr;
static void (*g_free_fn)(void*, void*, void*) = nullptr;
static void* g_alloc_ctx = nullptr;
static std::atomic<int> g_live_factors{0};  // the allocator may change only while this is 0

static void* dev_alloc(size_t bytes, hipStream_t st) {
    if (bytes == 0) bytes = 256;
    if (g_alloc_fn) return g_alloc_fn(bytes, (void*)st, g_alloc_ctx);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

// Stream-ordered allocation: inside an entry point (StreamScope) library
// buffers come from the device's default memory pool on the caller's stream,
// whose release threshold is raised so freed memory stays reserved for the
// next allocation instead of being unmapped (large level stores come and go
// every level).  A buffer is freed on the stream it was allocated on; freed
// from elsewhere, the device is synchronised first.
// A device-wide synchronisation from one thread would invalidate a graph
// capture running in another (serving workers): both take this lock.
static std::mutex g_capture_mu;
static void device_sync() {
    std::lock_guard<std::mutex> lk(g_capture_mu);
    (void)hipDeviceSynchronize();
}

static thread_local hipStream_t t_stream = nullptr;
static thread_local bool t_stream_set = false;
static thread_local bool t_device_synced = false;
struct StreamScope {
    hipStream_t prev;
    bool prev_set, prev_synced;
    StreamScope(hipStream_t s, bool device_synced = false)
        : prev(t_stream), prev_set(t_stream_set), prev_synced(t_device_synced) {
        t_stream = s;
        t_stream_set = true;
        t_device_synced = device_synced;
    }
    ~StreamScope() {
        t_stream = prev;
        t_stream_set = prev_set;
        t_device_synced = prev_synced;
    }
};
static void pool_init() {
    static std::once_flag once;
    std::call_once(once, [] {
        int dev = 0;
        hipMemPool_t pool;
        if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
            uint64_t keep = UINT64_MAX;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
        }
        (void)hipGetLastError();
    });
}

// Device bytes held by one factorization (current and largest so far).
// Buffers allocated while a call works on a factorization are charged to it
// (t_acct is set for the duration of the call).
struct ByteAccount {
    int64_t held = 0, peak = 0;
};
static thread_local ByteAccount* t_acct = nullptr;
struct AcctScope {
    ByteAccount* prev;
    explicit AcctScope(ByteAccount* a) : prev(t_acct) { t_acct = a; }
    ~AcctScope() { t_acct = prev; }
};

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    ByteAccount* acct = nullptr;
    bool pooled = false;
    hipStream_t stream = nullptr;
    void (*free_fn)(void*, void*, void*) = nullptr;  // the installed allocator that gave p, if any
    void* free_ctx = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept
        : p(o.p), bytes(o.bytes), acct(o.acct), pooled(o.pooled), stream(o.stream), free_fn(o.free_fn),
          free_ctx(o.free_ctx) {
        o.p = nullptr;
        o.bytes = 0;
        o.acct = nullptr;
    }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) {
            release();
            p = o.p;
            bytes = o.bytes;
            acct = o.acct;
            pooled = o.pooled;
            stream = o.stream;
            free_fn = o.free_fn;
            free_ctx = o.free_ctx;
            o.p = nullptr;
            o.bytes = 0;
            o.acct = nullptr;
        }
        return *this;
    }
    ~DevBuf() { release(); }
    void release() {
        if (p && pooled) {
            if (t_stream_set && t_stream == stream) {
                (void)hipFreeAsync(p, stream);
            } else {
                if (!t_device_synced) device_sync();
                (void)hipFreeAsync(p, nullptr);
            }
        } else if (p && free_fn) {
            // an installed allocator may hand the block to the next request on
            // its stream at once: every use must be ordered on that stream
            if (!(t_stream_set && t_stream == stream) && !t_device_synced) device_sync();
            free_fn(p, (void*)stream, free_ctx);
        } else if (p) {
            (void)hipFree(p);
        }
        if (acct) acct->held -= (int64_t)bytes;
        p = nullptr;
        bytes = 0;
        acct = nullptr;
        pooled = false;
        free_fn = nullptr;
    }
    bool alloc(size_t n) {
        release();
        if (!g_alloc_fn && t_stream_set) {
            pool_init();
            if (hipMallocAsync(&p, n ? n : 256, t_stream) != hipSuccess) {
                (void)hipGetLastError();
                p = nullptr;
            }
            pooled = p != nullptr;
            stream = t_stream;
        } else {
            stream = t_stream_set ? t_stream : nullptr;
            p = dev_alloc(n, stream);
            free_fn = g_alloc_fn ? g_free_fn : nullptr;
            free_ctx = g_alloc_ctx;
        }
        bytes = p ? n : 0;
        if (p && t_acct) {
            acct = t_acct;
            acct->held += (int64_t)n;
            acct->peak = std::max(acct->peak, acct->held);
        }
        return p != nullptr;
    }
    bool ensure(size_t n) { return bytes >= n ? true : alloc(n); }
    template <class T>
    T* as() const {
        return static_cast<T*>(p);
    }
};

// Host blob of aligned arrays uploaded in one copy.  Its storage is not
// zero-filled on growth: every byte is written once (arrays copied in,
// alignment gaps and reserved or zero runs cleared).
using cvec = std::vector<char, NoInitAlloc<char>>;
struct Blob {
    cvec data;
    size_t grow(size_t bytes) {  // aligned run of `bytes`, the gap before it cleared
        const size_t end = data.size(), off = (end + 255) & ~size_t(255);
        data.resize(off + bytes);
        if (off > end) std::memset(data.data() + end, 0, off - end);
        return off;
    }
    template <class T, class A>
    size_t add(const std::vector<T, A>& v) {
        const size_t off = grow(v.size() * sizeof(T));
        if (!v.empty()) std::memcpy(data.data() + off, v.data(), v.size() * sizeof(T));
        return off;
    }
    size_t reserve(size_t bytes) {  // a zeroed run
        const size_t off = grow(bytes);
        if (bytes) std::memset(data.data() + off, 0, bytes);
        return off;
    }
    template <class T>
    size_t zeros(size_t count) {  // count zero-initialised elements
        return reserve(count * sizeof(T));
    }
};

// The level metadata blob of the calling thread, reused from level to level
// and call to call: its capacity stays, so the host does not fault in fresh
// pages for tens of megabytes every level (its contents are on the device
// before the level's synchronisation, which precedes the next reuse).
static thread_local cvec t_blob_store;
struct BlobLease {
    Blob& b;
    explicit BlobLease(Blob& blob) : b(blob) { b.data.swap(t_blob_store); }
    ~BlobLease() {
        b.data.clear();
        b.data.swap(t_blob_store);
    }
};

// Run fn(0) .. fn(count - 1) on up to `threads` host threads.
template <class Fn>
static void parallel_for(int count, int threads, Fn fn) {
    threads = std::max(1, std::min(threads, count));
    if (threads == 1) {
        for (int i = 0; i < count; ++i) fn(i);
        return;
    }
    std::atomic<int> next(0);
    std::vector<std::thread> pool;
    for (int t = 0; t < threads; ++t)
        pool.emplace_back([&] {
            for (int i = next++; i < count; i = next++) fn(i);
        });
    for (auto& th : pool) th.join();
}
static int host_threads() { return (int)std::min(16u, std::max(1u, std::thread::hardware_concurrency())); }

// ---------------------------------------------------------------- tracing

struct ProfFamily {
    const char* name;
    int64_t launches = 0;
    double seconds = 0.0, bytes = 0.0, flops = 0.0;
};
enum ProfId {
    PF_GRAM = 0, PF_PIVOT, PF_FILL, PF_NBR, PF_SCHUR, PF_SCHUR_F32, PF_MERGE, PF_APPLY, PF_SPMV, PF_DENSE,
    PF_PIVOT_F32,
    // host wall time of the factorization: symbolic analysis, level planning,
    // metadata uploads, device allocations, per-level rank read-back
    PF_H_SYMBOLIC, PF_H_PLAN, PF_H_UPLOAD, PF_H_ALLOC, PF_H_SYNC, PF_H_SOLVE_PLAN, PF_COUNT
};
static ProfFamily g_prof[PF_COUNT] = {{"gram"}, {"pivot"}, {"fill"}, {"nbr"},   {"schur"}, {"schur_f32"},
                                      {"merge"}, {"apply"}, {"spmv"}, {"dense"}, {"pivot_f32"},
                                      {"host_symbolic"}, {"host_plan"}, {"host_upload"}, {"host_alloc"}, {"host_sync"},
                                      {"host_solve_plan"}};
static bool g_prof_on = false;
static uint32_t g_prof_mask = 0xffffffffu;  // families timed while on (hs_profile_select)
static bool prof_timed(int fam) { return fam >= 0 && g_prof_on && ((g_prof_mask >> fam) & 1u); }
struct ProfPending {
    int fam;
    hipEvent_t a, b;
};
static std::vector<ProfPending> g_prof_pending;
static std::vector<hipEvent_t> g_prof_pool;
static std::mutex g_prof_mu;  // calls on several threads (serving workers, concurrent factorizations)

static hipEvent_t prof_event() {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_pool.empty()) {
        hipEvent_t e = g_prof_pool.back();
        g_prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

// Bracket one launch: call with begin=true before, begin=false after.
struct ProfScope {
    int fam;
    hipStream_t st;
    hipEvent_t a = nullptr;
    ProfScope(int f, hipStream_t s) : fam(f), st(s) {
        if (prof_timed(fam)) {
            a = prof_event();
            (void)hipEventRecord(a, st);
        }
    }
    ~ProfScope() {
        if (g_prof_on && a) {
            hipEvent_t b = prof_event();
            (void)hipEventRecord(b, st);
            std::lock_guard<std::mutex> lk(g_prof_mu);
            g_prof_pending.push_back({fam, a, b});
        }
    }
};

// Host wall time of a scope, added to a host family.
struct HostScope {
    int fam;
    std::chrono::steady_clock::time_point t0;
    explicit HostScope(int f) : fam(f), t0(std::chrono::steady_clock::now()) {}
    ~HostScope() {
        if (prof_timed(fam)) {
            std::lock_guard<std::mutex> lk(g_prof_mu);
            g_prof[fam].seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            g_prof[fam].launches += 1;
        }
    }
};

// Read back finished intervals; those still running (another thread's
// stream) stay pending.
static void prof_flush() {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    std::vector<ProfPending> left;
    for (auto& p : g_prof_pending) {
        if (hipEventQuery(p.b) != hipSuccess) {
            (void)hipGetLastError();
            left.push_back(p);
            continue;
        }
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            g_prof[p.fam].seconds += ms * 1e-3;
            g_prof[p.fam].launches += 1;
        } else {
            (void)hipGetLastError();
        }
        g_prof_pool.push_back(p.a);
        g_prof_pool.push_back(p.b);
    }
    g_prof_pending.swap(left);
}

// ------------------------------------------------------------- level state

// Work lists of one colour by storage type: [0] the float32 clusters, [1] the
// float64 clusters with those factored densely on this level last.  The
// factor lists (fac) leave the dense clusters out; the solve lists (sol) hold
// every cluster of the colour.
// Factor lists are cut into chunks whose per-cluster workspace stays within
// WS_CHUNK_BYTES (launched one after the other, reusing the workspace).
struct ListPlan {
    int start = 0;                                 // first cluster within the type's list
    size_t off_pre[3] = {0, 0, 0};                 // blob offsets: neighbour, fill, tile prefixes
};
struct ColourHost {
    int first = 0, n = 0;                          // slice of the processing order
    int n_t[2] = {0, 0};                           // clusters per type
    int nfac_t[2] = {0, 0};                        // of which factored by the colour kernels
    ListPlan sol_plan[2];
    std::vector<ListPlan> fac_plan[2];
    std::vector<ColourDev> fac[2];                 // factor lists (chunks)
    ColourDev sol[2];
    const int64_t* part_off[2] = {nullptr, nullptr};  // [neighbour groups + 1] in units of f
    int64_t part_total[2] = {0, 0};                // sum of f over the groups
};

struct LevelData {
    int ncl = 0;
    int nblk = 0;
    int any_f32 = 0;                               // some cluster's blocks and records are float32
    std::vector<int> f32;                          // per cluster: float32 storage (mixed form)
    std::vector<char> dense;                       // per cluster: factored densely on this level
    int64_t npairs = 0;                            // sum over clusters of |n(s)|^2
    DevBuf pairs;                                  // block id of every neighbour pair (a_i, a_j) of s
    std::vector<int> m, k;                         // sizes at the start, ranks after
    i64vec blk_off;                                // in units of the block's element type (set in parallel)
    std::vector<int64_t> rec_off;                  // in units of the record's element type
    int64_t block_bytes = 0;
    int64_t rec_bytes = 0;
    int64_t ws_elems = 0;
    int gram_splits = 1;
    int max_m = 0;
    DevBuf meta;
    DevBuf blocks;
    DevBuf rec;
    LevelDev dev{};
    SolveLevelDev sdev{};
    const int* dev_pat_ptr = nullptr;  // final pattern on the device
    const int* dev_pat = nullptr;
    const int* dev_f32 = nullptr;      // per-cluster storage type on the device
    const int* dev_pos = nullptr;      // processing positions on the device
    DevBuf ids;                        // block ids / flags of the entries (launch_level_ids)
    int64_t nadj = 0, nfill = 0;
    std::vector<ColourHost> colours;
    std::vector<int> order_host;                   // the colour slices by type (host copy of the work lists)
    std::vector<int64_t> seg;                      // [ncl+1] segment offsets
    std::vector<int> ntot_host;                    // per cluster: neighbour unknowns (from the device)
    Knobs kn{};                                    // the level's kernel-variant thresholds
    int64_t nseg = 0;
    int64_t part_max = 0;                          // largest colour part buffer (units of f)
    std::vector<double> kept;                      // dense starting matrix (keep_levels)
    size_t esz(int s) const { return f32[s] ? sizeof(float) : sizeof(double); }
};

// Process-wide kernel-variant thresholds (hs_config_set), copied into a
// factorization when it starts; the variants compute the same numbers.
struct Config {
    Knobs kn{LDS_M, TRI_MFMA_MAX, TRI_MFMA_MAX12, 64, 128, TRI_MFMA_MAX, GRAM_SPLITS_MAX, 256, 1024, 1, 0};
    // Crowded levels (at least crowded_min clusters per colour on average) are
    // bound by throughput, sparse ones by the latency of each cluster's chain.
    // On a crowded level the pivot kernel takes gram_splits_crowded Gram
    // partials per cluster, forms the complement's columns wave by wave from
    // the reflectors (wy_max_crowded 0) and U by Householder QR
    // (cholqr_crowded 0): fewer, shorter device-function chains, measured 4 %
    // and 13 % faster on the batched convection-diffusion workload.  A sparse
    // level keeps one fill partner per Gram workgroup, the compact WY form and
    // Cholesky QR: on the 3D Poisson factorization (few clusters per colour,
    // larger ranks) the crowded settings took 1624 instead of 675 ms.
    int crowded_min = 512;
    int gram_splits_crowded = 4;
    int wy_max_crowded = 0;
    int cholqr_crowded = 0;
    int dense_panel = 128;
    int apply_fwd = 0;              // forward solve step: 0 by cost, 1 one launch, 2 two launches
    // one right-hand side: own products one wave per cluster in colours of at
    // least this many clusters (0: never); 1024 keeps the sparse levels of a
    // single 3D system on the workgroup form (its PCG took 5.6 s with every
    // colour by waves, 2.7 s so)
    int apply_wave = 1024;
    // apply_fwd 0 splits a colour's forward step (where the one-launch form
    // would re-read T_L' more than twice) only for at most this many
    // right-hand sides: with 8 the one-launch form took the 64^3 Poisson PCG
    // from 346 to 262 ms, with one the split form is the faster
    int apply_split_nrhs_max = 1;
    int compression = 0;            // rank revelation: 0 by eps and cap, 1 pivoted QR, 2 Gram
    double qrcp_below_eps = 1e-5;   // 0: pivoted QR of F^T below this eps (or under a rank cap)
};

}  // namespace hs

struct hs_factor_s {
    struct Live {  // counts existing factorizations; first member, so destroyed after every buffer
        Live() { ++hs::g_live_factors; }
        ~Live() { --hs::g_live_factors; }
    } live;
    hs::ByteAccount acct;                 // first member: outlives every buffer below
    int64_t n = 0;
    hs_opts opts{};
    hs::Config cfg;                       // kernel-variant thresholds of this factorization
    int qrcp = 0;                         // rank revelation by the pivoted QR of F^T (else the Gram route)
    int symmetric = 1;
    hs::Symbolic sym;
    hs::Forest forest;                    // the systems (one for hs_factor)
    hs::DevBuf seg_buf;                   // per-system Krylov segment and chunk tables
    hs::SegDev segs;
    std::vector<hs::LevelData> levels;
    hs::DevBuf A_row, A_col, A_val;
    hs::DevBuf cluster_of, local_of;
    hs::DevBuf ws;
    // solve buffers
    int solve_nrhs = 0;
    hs::DevBuf vecs;                      // y, z, out of every level
    std::vector<int64_t> vec_off;         // per level base (units of doubles / nrhs), set by hs_factor
    int64_t vec_total = 0;
    int64_t part_max = 0;                 // largest backward-partial buffer of a colour (units of nrhs)
    hs::DevBuf part;
    // Krylov buffers
    hs::DevBuf kry;
    int kry_nrhs = 0;
    int kry_restart = 0;
    hs_info info{};
    // The level sweeps of a solve (Alg. 2 between scattering the right-hand
    // sides and gathering the solution) captured as one HIP graph per
    // right-hand-side count: they touch only the solve buffers above, so a
    // graph stays valid until those are reallocated or released.
    std::vector<std::pair<int, hipGraphExec_t>> sweeps;
    hipStream_t cap_stream = nullptr;
    hipStream_t sweep_stream = nullptr;  // stream of the latest graph launch
    void drop_sweeps() {
        if (sweeps.empty()) return;
        (void)hipStreamSynchronize(sweep_stream);  // no launch of them may still be pending
        for (auto& g : sweeps) (void)hipGraphExecDestroy(g.second);
        sweeps.clear();
    }
    ~hs_factor_s() {
        drop_sweeps();
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }
};

struct hs_symbolic_s {
    hs::Symbolic sym;
};

namespace hs {

static const char* kVersion = "hs 0.1 (gfx950)";
// Mixed form: levels with at most this many unknowns keep float64 storage
// (default of hs_opts.coarse_fp64_dofs).
constexpr int64_t MIXED_FP64_DOFS = 16384;
// Per-cluster workspace of one factor launch at most (colours beyond it are
// launched in chunks that reuse the workspace).
constexpr int64_t WS_CHUNK_BYTES = int64_t(4) << 30;

// ============================================================ configuration

static std::mutex g_config_mu;
static Config g_config;
static Config config_snapshot() {
    std::lock_guard<std::mutex> lk(g_config_mu);
    return g_config;
}
struct ConfigEntry {
    const char* name;
    double lo, hi;
    int* ival;        // integer parameter, or
    double* dval;     // real parameter
};
static std::vector<ConfigEntry> config_table(Config& c) {
    return {
        {"pivot_lds_max", 0, LDS_M, &c.kn.pivot_lds_max, nullptr},
        {"trinv8_max", 0, TRI_MFMA_MAX, &c.kn.trinv8_max, nullptr},
        {"trinv12_max", 0, TRI_MFMA_MAX12, &c.kn.trinv12_max, nullptr},
        {"qr_reg1_max", 0, 64, &c.kn.qr_reg1_max, nullptr},
        {"qr_reg2_max", 0, 128, &c.kn.qr_reg2_max, nullptr},
        {"wy_max", 0, TRI_MFMA_MAX, &c.kn.wy_max, nullptr},
        {"gram_splits_max", 1, GRAM_SPLITS_MAX, &c.kn.gram_splits_max, nullptr},
        {"schur_ptab_max", 0, 256, &c.kn.schur_ptab_max, nullptr},
        {"schur_noff_max", 0, 1024, &c.kn.schur_noff_max, nullptr},
        {"cholqr", 0, 1, &c.kn.cholqr, nullptr},
        {"crowded_min", 0, 1 << 30, &c.crowded_min, nullptr},
        {"gram_splits_crowded", 1, GRAM_SPLITS_MAX, &c.gram_splits_crowded, nullptr},
        {"wy_max_crowded", 0, TRI_MFMA_MAX, &c.wy_max_crowded, nullptr},
        {"cholqr_crowded", 0, 1, &c.cholqr_crowded, nullptr},
        {"dense_panel", 16, 128, &c.dense_panel, nullptr},
        {"apply_fwd", 0, 2, &c.apply_fwd, nullptr},
        {"apply_wave", 0, 1 << 30, &c.apply_wave, nullptr},
        {"apply_split_nrhs_max", 0, 1 << 20, &c.apply_split_nrhs_max, nullptr},
        {"compression", 0, 2, &c.compression, nullptr},
        {"qrcp_below_eps", 0, 1, nullptr, &c.qrcp_below_eps},
    };
}

// =============================================================== validation

// The first defect of a host CSR pattern: 0 = none, 1 = bad ends, 2 = row_ptr
// decreasing, 3 = column out of range, 4 = columns not sorted / unique.
static int csr_defect(int64_t n, int64_t nnz, const int64_t* rp, const int32_t* ci) {
    if (rp[0] != 0 || rp[n] != nnz) return 1;
    for (int64_t i = 0; i < n; ++i) {
        if (rp[i + 1] < rp[i]) return 2;
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            if (ci[e] < 0 || ci[e] >= n) return 3;
            if (e > rp[i] && ci[e] <= ci[e - 1]) return 4;
        }
    }
    return 0;
}
static int csr_defect_error(int d) {
    static const char* msg[] = {"", "row_ptr[0] must be 0 and row_ptr[n] = nnz", "row_ptr not non-decreasing",
                                "column index out of range", "column indices not sorted / unique"};
    return d ? fail(HS_ERR_PATTERN, msg[d]) : HS_OK;
}
static int validate_csr_host(int64_t n, int64_t nnz, const int64_t* rp, const int32_t* ci) {
    return csr_defect_error(csr_defect(n, nnz, rp, ci));
}

// ================================================================ planning

// Plan one level: block offsets, per-cluster lists, colours, records and
// workspace.  LD.m, LD.f32 and LD.dense are set by the caller.  Builds the
// metadata blob (uploaded by the caller).
static int plan_level(hs_factor_s* F, int lvl, Blob& blob, std::vector<size_t>& offs) {
    LevelData& LD = F->levels[lvl];
    const LevelSymbolic& S = F->sym.levels[lvl];
    const int ncl = S.ncl;
    const std::vector<int>& m = LD.m;
    LD.ncl = ncl;
    LD.nblk = (int)S.pat.size();
    LD.nadj = (int64_t)S.adj.size();
    LD.nfill = (int64_t)S.fill.size();
    LD.max_m = 0;
    for (int c = 0; c < ncl; ++c)
        if (!LD.dense[c]) LD.max_m = std::max(LD.max_m, m[c]);
    if (LD.max_m > MAX_M)
        return fail(HS_ERR_UNSUPPORTED, "cluster of size " + std::to_string(LD.max_m) + " at level " +
                                            std::to_string(lvl) + " exceeds the supported " + std::to_string(MAX_M));
    // blocks (capacity m_a x m_b, column major, ld m_a), each in its cluster's
    // element type; offsets count elements of that type
    auto place = [](int64_t& cursor, int64_t elems, size_t es) {
        cursor = (cursor + 15) & ~int64_t(15);
        const int64_t o = cursor / (int64_t)es;
        cursor += elems * (int64_t)es;
        return o;
    };
    // every block starts 16-byte aligned, so a cluster's blocks take the sum of
    // their sizes rounded up to 16 bytes: per-cluster totals in parallel, a
    // prefix sum, then each cluster's offsets (the same layout as one cursor)
    LD.blk_off.resize(LD.nblk);
    const int nth = host_threads();
    std::vector<int64_t> ctot(ncl + 1, 0);
    parallel_for(nth, nth, [&](int t) {
        for (int a = (int)((int64_t)ncl * t / nth); a < (int)((int64_t)ncl * (t + 1) / nth); ++a) {
            int64_t b = 0;
            for (int e = S.pat_ptr[a]; e < S.pat_ptr[a + 1]; ++e)
                b += ((int64_t)m[a] * m[S.pat[e]] * (int64_t)LD.esz(a) + 15) & ~int64_t(15);
            ctot[a + 1] = b;
        }
    });
    for (int a = 0; a < ncl; ++a) ctot[a + 1] += ctot[a];
    parallel_for(nth, nth, [&](int t) {
        for (int a = (int)((int64_t)ncl * t / nth); a < (int)((int64_t)ncl * (t + 1) / nth); ++a) {
            int64_t c = ctot[a];
            for (int e = S.pat_ptr[a]; e < S.pat_ptr[a + 1]; ++e)
                LD.blk_off[e] = place(c, (int64_t)m[a] * m[S.pat[e]], LD.esz(a));
        }
    });
    LD.block_bytes = ctot[ncl];

    // per-cluster lists (the block ids of every neighbour / fill entry and of
    // all neighbour pairs are found on the device: launch_level_ids,
    // launch_pair_blocks)
    std::vector<int> ncap(ncl);
    std::vector<int64_t> pair_base(ncl), ws_off(ncl, 0);
    LD.rec_off.assign(ncl, 0);
    int64_t pp = 0, roff = 0;
    int max_nf = 0;
    for (int s = 0; s < ncl; ++s) {
        int cap = 0;
        for (int e = S.adj_ptr[s]; e < S.adj_ptr[s + 1]; ++e) cap += m[S.adj[e]];
        ncap[s] = cap;
        max_nf = std::max(max_nf, S.fill_ptr[s + 1] - S.fill_ptr[s]);
        pair_base[s] = pp;
        const int64_t nb = S.adj_ptr[s + 1] - S.adj_ptr[s];
        pp += nb * nb;
        LD.rec_off[s] = place(roff, 2 * (int64_t)m[s] * m[s] + 2 * (int64_t)m[s] * cap, LD.esz(s));
    }
    LD.rec_bytes = roff;
    LD.npairs = pp;
    // workspace slots; each cluster uses gram_splits_of(its nf); the pivoted-QR
    // route keeps F (m x its fill columns) behind the slots instead
    // the level's kernel-variant thresholds: the crowded settings when its
    // colours hold at least crowded_min clusters on average
    LD.kn = F->cfg.kn;
    if ((int64_t)ncl >= (int64_t)F->cfg.crowded_min * std::max(1, S.ncolors)) {
        LD.kn.gram_splits_max = F->cfg.gram_splits_crowded;
        LD.kn.wy_max = F->cfg.wy_max_crowded;
        LD.kn.cholqr = F->cfg.cholqr_crowded;
    }
    LD.gram_splits = F->qrcp ? 1 : gram_splits_of(max_nf, LD.kn.gram_splits_max);
    const int64_t slots = ws_slots(LD.gram_splits);
    std::vector<int64_t> fcap(ncl, 0);
    if (F->qrcp)
        for (int s = 0; s < ncl; ++s) {
            int64_t c = 0;
            for (int e = S.fill_ptr[s]; e < S.fill_ptr[s + 1]; ++e) c += m[S.fill[e]];
            fcap[s] = (F->symmetric ? 1 : 2) * c;
        }

    // colours: every colour's slice of the processing order is reordered into
    // [float32 clusters | float64 clusters | dense clusters] (stable, so each
    // system keeps its own order; clusters of one colour never interact)
    std::vector<int> order(ncl);
    LD.colours.assign(S.ncolors, ColourHost());
    int64_t ws_max = 0;
    struct Pre {
        std::vector<int> np, fp;
        std::vector<int64_t> tp;
    };
    struct ListPre {
        int start;
        Pre pre;
    };
    std::vector<std::array<ListPre, 2>> spres(S.ncolors);
    std::vector<std::array<std::vector<ListPre>, 2>> fpres(S.ncolors);
    std::vector<int64_t> ws_max_c(S.ncolors, 0);
    // colours touch disjoint slices of order and disjoint clusters: in parallel
    parallel_for(S.ncolors, nth, [&](int c) {
        int64_t& ws_max = ws_max_c[c];
        ColourHost& CH = LD.colours[c];
        CH.first = S.color_ptr[c];
        CH.n = S.color_ptr[c + 1] - S.color_ptr[c];
        int w = CH.first;
        for (int pass = 0; pass < 3; ++pass)
            for (int i = 0; i < CH.n; ++i) {
                const int s = S.order[CH.first + i];
                const int cls = LD.f32[s] ? 0 : (LD.dense[s] ? 2 : 1);
                if (cls == pass) order[w++] = s;
            }
        for (int i = 0; i < CH.n; ++i) {
            const int s = order[CH.first + i];
            const int t = LD.f32[s] ? 0 : 1;
            CH.n_t[t]++;
            if (!LD.dense[s]) CH.nfac_t[t]++;
        }
        int base = CH.first;
        for (int t = 0; t < 2; ++t) {
            const int nt = CH.n_t[t], nf = CH.nfac_t[t];
            // prefix arrays and maxima of the list entries [i0, i1)
            auto make = [&](int i0, int i1, ColourDev& D, Pre& P) {
                const int n = i1 - i0;
                P.np.assign(n + 1, 0);
                P.fp.assign(n + 1, 0);
                P.tp.assign(n + 1, 0);
                int mm = 0, mn = 0;
                for (int i = 0; i < n; ++i) {
                    const int s = order[base + i0 + i];
                    P.np[i + 1] = P.np[i] + (S.adj_ptr[s + 1] - S.adj_ptr[s]);
                    P.fp[i + 1] = P.fp[i] + (S.fill_ptr[s + 1] - S.fill_ptr[s]);
                    const int64_t tpr = (ncap[s] + SCHUR_T - 1) / SCHUR_T;
                    P.tp[i + 1] = P.tp[i] + (m[s] > 0 ? tpr * tpr : 0);
                    int nm = 0;
                    for (int e = S.adj_ptr[s]; e < S.adj_ptr[s + 1]; ++e) nm = std::max(nm, m[S.adj[e]]);
                    for (int e = S.fill_ptr[s]; e < S.fill_ptr[s + 1]; ++e) nm = std::max(nm, m[S.fill[e]]);
                    mm = std::max(mm, m[s]);
                    mn = std::max(mn, nm);
                }
                D = ColourDev();
                D.n = n;
                D.nbr_total = P.np[n];
                D.fill_total = P.fp[n];
                D.tile_total = P.tp[n];
                D.max_m = mm;
                D.max_nbr_m = mn;
                const int pw = panel_width(mm);
                D.panels = (mn + pw - 1) / pw;
                D.f32 = t == 0;
            };
            spres[c][t].start = 0;
            make(0, nt, CH.sol[t], spres[c][t].pre);
            // factor chunks: workspace offsets restart in every chunk
            CH.fac[t].clear();
            int i0 = 0;
            while (i0 < nf) {
                int64_t wso = 0;
                int i1 = i0;
                while (i1 < nf) {
                    const int s = order[base + i1];
                    const int64_t need = slots * (int64_t)m[s] * m[s] + (int64_t)m[s] * fcap[s];
                    if (i1 > i0 && (wso + need) * (int64_t)sizeof(double) > WS_CHUNK_BYTES) break;
                    ws_off[s] = wso;
                    wso += need;
                    ++i1;
                }
                ws_max = std::max(ws_max, wso);
                fpres[c][t].push_back(ListPre{i0, Pre()});
                CH.fac[t].emplace_back();
                make(i0, i1, CH.fac[t].back(), fpres[c][t].back().pre);
                i0 = i1;
            }
            base += nt;
        }
    });
    for (int c = 0; c < S.ncolors; ++c) ws_max = std::max(ws_max, ws_max_c[c]);
    LD.ws_elems = ws_max;

    // blob layout
    offs.clear();
    offs.push_back(blob.add(m));                 // 0 m
    offs.push_back(blob.add(m));                 // 1 k (initialised to m)
    offs.push_back(blob.zeros<int>(ncl));       // 2 flag
    offs.push_back(blob.add(LD.blk_off));        // 3
    offs.push_back(blob.add(S.pos));             // 4 processing position
    offs.push_back(blob.add(S.adj_ptr));         // 5
    offs.push_back(blob.add(S.adj));             // 6
    offs.push_back(0);                           // 7-9 (LD.ids)
    offs.push_back(0);
    offs.push_back(0);
    offs.push_back(blob.zeros<int>(S.adj.size()));  // 10 nbr_noff
    offs.push_back(blob.zeros<int>(ncl));           // 11 ntot
    offs.push_back(blob.add(ncap));              // 12
    offs.push_back(blob.add(S.fill_ptr));        // 13
    offs.push_back(blob.add(S.fill));            // 14
    offs.push_back(0);                           // 15-17 (LD.ids)
    offs.push_back(0);
    offs.push_back(0);
    offs.push_back(blob.add(pair_base));         // 18
    offs.push_back(blob.add(std::vector<int>()));  // 19 (pair block ids: LD.pairs)
    offs.push_back(blob.add(LD.rec_off));        // 20
    offs.push_back(blob.add(ws_off));            // 21
    offs.push_back(blob.add(S.pat_ptr));         // 22
    offs.push_back(blob.add(S.pat));             // 23
    offs.push_back(blob.add(order));             // 24 colour slices by type (the work lists)
    LD.order_host = order;
    offs.push_back(blob.add(LD.f32));            // 25 per-cluster storage type
    offs.push_back(blob.zeros<int>(ncl));       // 26 fill columns (written by k_offsets)
    auto add_pre = [&](ListPlan& L, const ListPre& lp) {
        L.start = lp.start;
        L.off_pre[0] = blob.add(lp.pre.np);
        L.off_pre[1] = blob.add(lp.pre.fp);
        L.off_pre[2] = blob.add(lp.pre.tp);
    };
    for (int c = 0; c < S.ncolors; ++c) {
        ColourHost& CH = LD.colours[c];
        for (int t = 0; t < 2; ++t) {
            add_pre(CH.sol_plan[t], spres[c][t]);
            CH.fac_plan[t].assign(fpres[c][t].size(), ListPlan());
            for (size_t q = 0; q < fpres[c][t].size(); ++q) add_pre(CH.fac_plan[t][q], fpres[c][t][q]);
        }
    }
    return HS_OK;
}

static void bind_level(LevelData& LD, const std::vector<size_t>& offs, const hs_factor_s* F) {
    char* base = LD.meta.as<char>();
    auto P = [&](int i) { return (void*)(base + offs[i]); };
    LevelDev& D = LD.dev;
    D.ncl = LD.ncl;
    D.symmetric = F->symmetric;
    D.eps = F->opts.eps;
    D.fixed_rank = F->opts.fixed_rank;
    D.pivoting = F->opts.pivoting;
    D.gram_splits = LD.gram_splits;
    D.kn = LD.kn;
    D.kn.qrcp = F->qrcp;
    D.m = (const int*)P(0);
    D.k = (int*)P(1);
    D.flag = (int*)P(2);
    D.blk_off = (const int64_t*)P(3);
    D.blocks = LD.blocks.as<double>();
    // block ids and processed-before flags: [diag | nbr_before, bsa, bas | fill_before, bst, bts]
    int* ids = LD.ids.as<int>();
    const int64_t na = LD.nadj, nf = LD.nfill;
    D.diag_blk = ids;
    D.nbr_ptr = (const int*)P(5);
    D.nbr_id = (const int*)P(6);
    D.nbr_before = ids + LD.ncl;
    D.nbr_bsa = ids + LD.ncl + na;
    D.nbr_bas = ids + LD.ncl + 2 * na;
    D.nbr_noff = (int*)P(10);
    D.ntot = (int*)P(11);
    D.ncap = (const int*)P(12);
    D.fill_ptr = (const int*)P(13);
    D.fill_id = (const int*)P(14);
    D.fill_before = ids + LD.ncl + 3 * na;
    D.fill_bst = ids + LD.ncl + 3 * na + nf;
    D.fill_bts = ids + LD.ncl + 3 * na + 2 * nf;
    LD.dev_pos = (const int*)P(4);
    D.pair_base = (const int64_t*)P(18);
    D.pair_blk = LD.pairs.as<int>();
    D.rec_off = (const int64_t*)P(20);
    D.rec = LD.rec.as<double>();
    D.ws_off = (const int64_t*)P(21);
    D.ws = F->ws.as<double>();
    LD.dev_pat_ptr = (const int*)P(22);
    LD.dev_pat = (const int*)P(23);
    LD.dev_f32 = (const int*)P(25);
    D.fcols = (int*)P(26);
    const int* order = (const int*)P(24);
    auto bind = [&](ColourDev& Cd, const ListPlan& L, int first) {
        Cd.clist = order + first + L.start;
        Cd.nbr_pre = (const int*)(base + L.off_pre[0]);
        Cd.fill_pre = (const int*)(base + L.off_pre[1]);
        Cd.tile_pre = (const int64_t*)(base + L.off_pre[2]);
    };
    for (auto& CH : LD.colours) {
        int first = CH.first;
        for (int t = 0; t < 2; ++t) {
            bind(CH.sol[t], CH.sol_plan[t], first);
            for (size_t q = 0; q < CH.fac[t].size(); ++q) bind(CH.fac[t][q], CH.fac_plan[t][q], first);
            first += CH.n_t[t];
        }
    }
    SolveLevelDev& SD = LD.sdev;
    SD.ncl = LD.ncl;
    SD.m = D.m;
    SD.k = D.k;
    SD.nbr_ptr = D.nbr_ptr;
    SD.nbr_id = D.nbr_id;
    SD.nbr_before = D.nbr_before;
    SD.nbr_noff = D.nbr_noff;
    SD.ntot = D.ntot;
    SD.ncap = D.ncap;
    SD.rec_off = D.rec_off;
    SD.rec = D.rec;
}

// =============================================================== flop model

// Algorithmic flops of one cluster (same formulas as the oracle's count).
static double cluster_flops(int m, int k, int nt, int wt, bool symmetric) {
    if (m == 0 || k == m) return 0.0;
    const double f = m - k;
    double fl = 2.0 * m * (double)m * m / 3.0;
    if (k == 0) return fl + 2.0 * m * (double)m * nt + 2.0 * m * (double)nt * nt;
    const double ncol = symmetric ? wt : 2.0 * wt;
    const double sy = symmetric ? 1.0 : 2.0;
    fl += 4.0 * m * ncol * k - 2.0 * k * (double)k * (m + ncol) + 4.0 * k * (double)k * k / 3.0;
    fl += 2.0 * m * k * ncol;
    fl += 2.0 * m * (double)m * k * sy;
    fl += 4.0 * m * k * f * sy;
    fl += 2.0 * m * (double)m * f;
    fl += 2.0 * m * f * f + 2.0 * f * f * f / 3.0;
    fl += 2.0 * m * (double)m * nt;
    fl += 2.0 * m * nt * (k + f) * 2.0;
    fl += 2.0 * f * f * nt;
    fl += 2.0 * m * (double)k * k + 2.0 * k * (double)k * wt * sy;
    fl += 2.0 * f * (double)nt * nt;
    return fl;
}

// ================================================================ factor

static int keep_level_matrix(hs_factor_s* F, LevelData& LD, hipStream_t st) {
    const LevelSymbolic& S = F->sym.levels[&LD - F->levels.data()];
    std::vector<char> raw(LD.block_bytes);
    if (LD.block_bytes)
        HIP_TRY(hipMemcpyAsync(raw.data(), LD.blocks.p, LD.block_bytes, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    std::vector<int64_t> off(LD.ncl + 1, 0);
    for (int c = 0; c < LD.ncl; ++c) off[c + 1] = off[c] + LD.m[c];
    const int64_t dim = off[LD.ncl];
    LD.kept.assign((size_t)(dim * dim), 0.0);
    for (int a = 0; a < LD.ncl; ++a)
        for (int e = S.pat_ptr[a]; e < S.pat_ptr[a + 1]; ++e) {
            const int b = S.pat[e];
            const float* bf = reinterpret_cast<const float*>(raw.data()) + LD.blk_off[e];
            const double* bd = reinterpret_cast<const double*>(raw.data()) + LD.blk_off[e];
            for (int j = 0; j < LD.m[b]; ++j)
                for (int i = 0; i < LD.m[a]; ++i) {
                    const int64_t x = i + (int64_t)j * LD.m[a];
                    LD.kept[(off[a] + i) + (off[b] + j) * dim] = LD.f32[a] ? (double)bf[x] : bd[x];
                }
        }
    return HS_OK;
}

// Dense factorization of the systems that are complete on this level (one
// cluster range each): ranks become 0 and the solve metadata (packed
// neighbour offsets, n_tot) is written for every cluster of the ranges.  A
// zero or non-finite pivot sets the range's entry of dflag (read back with
// the level's ranks).  aux / dense are workspaces kept until that read-back.
static int factor_dense_ranges(hs_factor_s* F, int lvl, const std::vector<std::array<int, 2>>& ranges, DevBuf& aux,
                               DevBuf& dense, int*& dflag, hipStream_t st) {
    LevelData& LD = F->levels[lvl];
    const LevelSymbolic& S = F->sym.levels[lvl];
    const int nr = (int)ranges.size();
    // packed offsets: neighbours before s are eliminated (size 0)
    std::vector<int> noff(S.adj.size(), 0), ntot(LD.ncl, 0), zeros(LD.ncl, 0);
    std::vector<std::vector<int64_t>> offs(nr);
    int64_t maxN = 0;
    for (int r = 0; r < nr; ++r) {
        const int c0 = ranges[r][0], c1 = ranges[r][1];
        for (int s = c0; s < c1; ++s) {
            int acc = 0;
            for (int e = S.adj_ptr[s]; e < S.adj_ptr[s + 1]; ++e) {
                noff[e] = acc;
                const int a = S.adj[e];
                acc += a < s ? 0 : LD.m[a];
            }
            ntot[s] = acc;
        }
        offs[r].assign(c1 - c0 + 1, 0);
        for (int c = c0; c < c1; ++c) offs[r][c - c0 + 1] = offs[r][c - c0] + LD.m[c];
        maxN = std::max(maxN, offs[r].back());
    }
    Blob b;
    const size_t o_noff = b.add(noff), o_ntot = b.add(ntot), o_zero = b.add(zeros);
    std::vector<size_t> o_off(nr);
    for (int r = 0; r < nr; ++r) o_off[r] = b.add(offs[r]);
    const size_t o_flag = b.add(std::vector<int>(nr, 0));
    const size_t o_inv = b.reserve((2 * 128 * 128) * sizeof(double));
    if (!aux.alloc(b.data.size())) return fail(HS_ERR_NOMEM, "dense level");
    if (maxN > 0 && !dense.alloc((size_t)maxN * maxN * sizeof(double)))
        return fail(HS_ERR_NOMEM, "dense level matrix");
    // the blob stays alive in aux; copies out of it are device to device.
    // Copies are stream-ordered: a legacy-stream copy would synchronise with
    // a graph capture that another thread may be running.
    HIP_TRY(hipMemcpyAsync(aux.p, b.data.data(), b.data.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    char* base = aux.as<char>();
    dflag = (int*)(base + o_flag);
    double* inv = (double*)(base + o_inv);
    for (int r = 0; r < nr; ++r) {
        const int c0 = ranges[r][0], c1 = ranges[r][1];
        const int e0 = S.adj_ptr[c0], e1 = S.adj_ptr[c1];
        if (e1 > e0)
            HIP_TRY(hipMemcpyAsync(LD.dev.nbr_noff + e0, base + o_noff + e0 * sizeof(int), (e1 - e0) * sizeof(int),
                                   hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipMemcpyAsync(LD.dev.ntot + c0, base + o_ntot + c0 * sizeof(int), (c1 - c0) * sizeof(int),
                               hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipMemcpyAsync(LD.dev.k + c0, base + o_zero, (c1 - c0) * sizeof(int), hipMemcpyDeviceToDevice, st));
        const int64_t N = offs[r].back();
        if (N == 0) continue;
        std::vector<int> m_host(LD.m.begin() + c0, LD.m.begin() + c1);
        ProfScope ps(PF_DENSE, st);
        const int b0 = S.pat_ptr[c0];
        const int rc = dense_level_factor(dense.as<double>(), N, LD.dev_pat_ptr, LD.dev_pat, c0, b0, LD.dev.m + c0,
                                          (const int64_t*)(base + o_off[r]), LD.dev.blk_off, LD.dev.blocks, c1 - c0,
                                          S.pat_ptr[c1] - b0, inv, dflag + r, LD.dev.ncap + c0, LD.dev.rec_off + c0,
                                          LD.dev.rec, m_host, offs[r], F->cfg.dense_panel, st);
        if (rc) return fail(HS_ERR_HIP, "dense level launch failed");
    }
    return HS_OK;
}

// ---- solve plan of one level (Alg. 2 metadata; needs the level's ranks).
// The host part runs while the next level's kernels are on the device; the
// metadata is uploaded once every level is planned.
struct SolveGroupOffsets {
    size_t part = 0, pre = 0, e0 = 0, e1 = 0;  // blob offsets: part offsets, group prefix, entry ranges
};
struct SolvePlan {
    Blob blob;
    size_t seg = 0;
    std::vector<std::array<SolveGroupOffsets, 2>> grp;  // per colour and type
    double rec_bytes = 0.0, apply_flops = 0.0;
    double factor_flops = 0.0;  // the level's share of info.factor_flops
};

static void plan_solve_level(hs_factor_s* F, int lvl, SolvePlan& P) {
    LevelData& LD = F->levels[lvl];
    const LevelSymbolic& S = F->sym.levels[lvl];
    Blob& sb = P.blob;
    P.seg = sb.add(LD.seg);
    P.grp.assign(LD.colours.size(), {});
    // neighbour groups of the backward sweep: consecutive entries of a
    // cluster's list up to SOLVE_GROUP_COLS columns of E_R and
    // SOLVE_GROUP_ENTRIES entries; one f x nrhs partial per group
    LD.part_max = 0;
    for (size_t c = 0; c < LD.colours.size(); ++c) {
        ColourHost& CH = LD.colours[c];
        for (int t = 0; t < 2; ++t) {
            std::vector<int64_t> po;
            std::vector<int> pre(1, 0), ge0, ge1;
            int64_t acc = 0;
            // forward step in one launch: every neighbour-row workgroup
            // forms z_s[:f] = T_L'[:f] y_s again (f m reads each); in two,
            // z_s is formed once and read back
            double own_elems = 0.0, reformed_elems = 0.0;
            int max_nt = 0;
            for (int i = 0; i < CH.n_t[t]; ++i) {
                const int s = LD.order_host[CH.first + (t ? CH.n_t[0] : 0) + i];
                const int f = LD.m[s] - LD.k[s];
                own_elems += (double)LD.m[s] * LD.m[s];
                int nt_s = 0;
                for (int e = S.adj_ptr[s]; e < S.adj_ptr[s + 1]; ++e) {
                    const int a = S.adj[e];
                    nt_s += S.pos[a] < S.pos[s] ? LD.k[a] : LD.m[a];
                }
                max_nt = std::max(max_nt, nt_s);
                int ng = 0;
                if (LD.m[s] > 0 && f > 0) {
                    int cols = 0;
                    for (int e = S.adj_ptr[s]; e < S.adj_ptr[s + 1]; ++e) {
                        const int a = S.adj[e];
                        const int ca = S.pos[a] < S.pos[s] ? LD.k[a] : LD.m[a];
                        reformed_elems += (double)((ca + 63) / 64) * f * LD.m[s];
                        const bool open = ng > 0 && ge1.back() == e;
                        if (open && cols + ca <= SOLVE_GROUP_COLS && e - ge0.back() < SOLVE_GROUP_ENTRIES) {
                            ge1.back() = e + 1;
                            cols += ca;
                        } else {
                            ge0.push_back(e);
                            ge1.push_back(e + 1);
                            po.push_back(acc);
                            acc += f;
                            cols = ca;
                            ++ng;
                        }
                    }
                }
                pre.push_back(pre.back() + ng);
            }
            po.push_back(acc);
            CH.part_total[t] = acc;
            CH.sol[t].grp_total = pre.back();
            CH.sol[t].fwd_split =
                F->cfg.apply_fwd == 2 ? 1 : (F->cfg.apply_fwd == 0 && reformed_elems > 2.0 * own_elems ? 2 : 0);
            CH.sol[t].split_nrhs_max = F->cfg.apply_split_nrhs_max;
            CH.sol[t].max_nt = max_nt;
            CH.sol[t].apply_wave = F->cfg.apply_wave;
            LD.part_max = std::max(LD.part_max, acc);
            P.grp[c][t] = {sb.add(po), sb.add(pre), sb.add(ge0), sb.add(ge1)};
        }
    }
    P.rec_bytes = P.apply_flops = 0.0;
    for (int c = 0; c < LD.ncl; ++c) {
        const double m = LD.m[c], k = LD.k[c], f = m - k;
        if (LD.m[c] == 0 || LD.k[c] == LD.m[c]) continue;
        int nt = 0;
        for (int e = S.adj_ptr[c]; e < S.adj_ptr[c + 1]; ++e) {
            const int a = S.adj[e];
            nt += S.pos[a] < S.pos[c] ? LD.k[a] : LD.m[a];
        }
        P.rec_bytes += (double)LD.esz(c) * (2.0 * m * m + 2.0 * f * nt);
        P.apply_flops += 4.0 * m * m + 4.0 * f * nt;
    }
}

// Per-level work model: the factorization flops (info.factor_flops) and, while
// the profiler times them, the pivot and Schur families' algorithmic flops and
// bytes.  Host only; runs while the next level is on the device.
static void account_level(hs_factor_s* F, int lvl, SolvePlan& P) {
    LevelData& LD = F->levels[lvl];
    const LevelSymbolic& S = F->sym.levels[lvl];
    P.factor_flops = 0.0;
    if (g_prof_on) {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        for (int c = 0; c < LD.ncl; ++c) {
            const double m = LD.m[c], kk = LD.k[c], f = m - kk, nt = LD.ntot_host[c];
            if (LD.m[c] == 0 || LD.dense[c]) continue;
            const int pid = LD.f32[c] ? PF_PIVOT_F32 : PF_PIVOT;
            if (prof_timed(pid) && f > 0) {
                // the pivot kernel's share of the algorithmic work (counted as in the
                // flop model below): LU of A_ss; with fill X = A^{-1} U, the
                // complement(s), A^{-1} V, F_ff and its LU, C = U^T A^{-1} U; bytes:
                // A_ss and the Gram matrix read, T_L', T_R' and C written
                const double sides = F->symmetric ? 1.0 : 2.0;
                double fl = 2.0 * m * m * m / 3.0, by = (double)LD.esz(c) * (3.0 * m * m);
                if (kk > 0)
                    fl += sides * (2.0 * m * m * kk + 4.0 * m * kk * f) + 2.0 * m * m * f + 2.0 * m * f * f +
                          2.0 * f * f * f / 3.0 + 2.0 * m * kk * kk;
                if (S.fill_ptr[c + 1] > S.fill_ptr[c] && F->opts.eps > 0.0)
                    by += 8.0 * m * m + (double)LD.esz(c) * kk * kk;
                g_prof[pid].flops += fl;
                g_prof[pid].bytes += by;
            }
            if (f == 0 || nt == 0) continue;
            const int fid = LD.f32[c] ? PF_SCHUR_F32 : PF_SCHUR;
            if (!prof_timed(fid)) continue;
            ProfFamily& fam = g_prof[fid];
            fam.flops += 2.0 * f * nt * nt;
            fam.bytes += (double)LD.esz(c) * (2.0 * f * nt + 2.0 * nt * nt);
        }
    }
    for (int c = 0; c < LD.ncl; ++c) {
        int wt = 0;
        for (int e = S.fill_ptr[c]; e < S.fill_ptr[c + 1]; ++e) {
            const int t = S.fill[e];
            wt += S.pos[t] < S.pos[c] ? LD.k[t] : LD.m[t];
        }
        P.factor_flops += cluster_flops(LD.m[c], LD.k[c], LD.ntot_host[c], wt, F->symmetric != 0);
    }
}

// Upload a level's solve metadata (after its block store is no longer needed:
// the buffer takes the block store's slot) and point the colours at it.
static int bind_solve_level(hs_factor_s* F, int lvl, SolvePlan& P, hipStream_t st) {
    LevelData& LD = F->levels[lvl];
    const Blob& sb = P.blob;
    DevBuf buf;
    if (!buf.alloc(sb.data.size())) return fail(HS_ERR_NOMEM, "solve metadata");
    HIP_TRY(hipMemcpyAsync(buf.p, sb.data.data(), sb.data.size(), hipMemcpyHostToDevice, st));
    LD.sdev.seg = (const int64_t*)(buf.as<char>() + P.seg);
    for (size_t c = 0; c < LD.colours.size(); ++c)
        for (int t = 0; t < 2; ++t) {
            ColourHost& CH = LD.colours[c];
            const char* b = buf.as<char>();
            CH.part_off[t] = (const int64_t*)(b + P.grp[c][t].part);
            CH.sol[t].grp_pre = (const int*)(b + P.grp[c][t].pre);
            CH.sol[t].grp_e0 = (const int*)(b + P.grp[c][t].e0);
            CH.sol[t].grp_e1 = (const int*)(b + P.grp[c][t].e1);
        }
    LD.blocks = std::move(buf);  // the block store slot now owns the solve metadata
    return HS_OK;
}

// Pinned host staging of device-resident patterns (the symbolic analysis
// reads them on the host; pageable copies run at a fraction of the link's
// rate).  One buffer, grown on demand and kept until the process ends; a
// factorization that finds it in use (another thread) copies through
// pageable memory instead.
static std::mutex g_pin_mu;
static char* g_pin = nullptr;
static size_t g_pin_bytes = 0;

// Factor nsys independent systems as one block-diagonal system (Alg. 1 on
// the forest of their cluster trees): every kernel launch of a level and
// colour covers the clusters of all systems.
static int factor_impl(hs_factor_s* F, int nsys, const hs_csr* A, const hs_geometry* G, hipStream_t st) {
    using clock = std::chrono::steady_clock;
    int rc;
    int64_t n = 0, nnz = 0;
    std::vector<int64_t> nnz_off(nsys + 1, 0), row_off(nsys + 1, 0);
    for (int i = 0; i < nsys; ++i) {
        row_off[i + 1] = row_off[i] + A[i].n;
        nnz_off[i + 1] = nnz_off[i] + A[i].nnz;
    }
    n = row_off[nsys];
    nnz = nnz_off[nsys];
    if (n > INT32_MAX) return fail(HS_ERR_ARG, "more than 2^31 - 1 unknowns in total");
    F->n = n;
    // ---- host copies of the patterns (the symbolic analysis needs them):
    // into the pinned staging buffer when it is free and can hold them all
    std::vector<i64vec> rp_h(nsys);  // pageable fallback, filled by the copies (no zeroing first)
    std::vector<ivec> ci_h(nsys);
    std::vector<const int64_t*> rp(nsys);
    std::vector<const int32_t*> ci(nsys);
    bool dev_copy = false;
    auto align256 = [](size_t b) { return (b + 255) & ~size_t(255); };
    size_t pin_need = 0;
    for (int i = 0; i < nsys; ++i)
        if (A[i].on_device) pin_need += align256((A[i].n + 1) * sizeof(int64_t)) + align256(A[i].nnz * sizeof(int32_t));
    std::unique_lock<std::mutex> pin_lock(g_pin_mu, std::defer_lock);
    char* pin = nullptr;
    if (pin_need > 0 && pin_lock.try_lock()) {
        if (g_pin_bytes < pin_need) {
            if (g_pin) (void)hipHostFree(g_pin);
            g_pin = nullptr;
            g_pin_bytes = 0;
            const size_t want = pin_need + pin_need / 4;
            if (hipHostMalloc((void**)&g_pin, want, hipHostMallocDefault) == hipSuccess)
                g_pin_bytes = want;
            else
                g_pin = nullptr;
            (void)hipGetLastError();
        }
        if (g_pin_bytes >= pin_need)
            pin = g_pin;
        else
            pin_lock.unlock();
    }
    // an early return drains the copies into the staging buffer before the
    // lock is released (declared after the lock, so destroyed first)
    struct PinDrain {
        hipStream_t st;
        bool on = false;
        ~PinDrain() {
            if (on) (void)hipStreamSynchronize(st);
        }
    } pin_drain{st, pin != nullptr};
    size_t pin_off = 0;
    for (int i = 0; i < nsys; ++i) {
        if (A[i].on_device) {
            int64_t* rdst;
            int32_t* cdst;
            if (pin) {
                rdst = (int64_t*)(pin + pin_off);
                pin_off += align256((A[i].n + 1) * sizeof(int64_t));
                cdst = (int32_t*)(pin + pin_off);
                pin_off += align256(A[i].nnz * sizeof(int32_t));
            } else {
                rp_h[i].resize(A[i].n + 1);
                ci_h[i].resize(A[i].nnz);
                rdst = rp_h[i].data();
                cdst = ci_h[i].data();
            }
            HIP_TRY(hipMemcpyAsync(rdst, A[i].row_ptr, (A[i].n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, st));
            if (A[i].nnz)
                HIP_TRY(hipMemcpyAsync(cdst, A[i].col_idx, A[i].nnz * sizeof(int32_t), hipMemcpyDeviceToHost, st));
            rp[i] = rdst;
            ci[i] = cdst;
            dev_copy = true;
        } else {
            rp[i] = A[i].row_ptr;
            ci[i] = A[i].col_idx;
        }
    }
    if (dev_copy) HIP_TRY(hipStreamSynchronize(st));
    pin_drain.on = false;
    {  // the systems' patterns checked on host threads, the first defect reported
        std::vector<int> defect(nsys, 0);
        parallel_for(nsys, std::min(host_threads(), 16),
                     [&](int i) { defect[i] = csr_defect(A[i].n, A[i].nnz, rp[i], ci[i]); });
        for (int i = 0; i < nsys; ++i)
            if (defect[i]) {
                rc = csr_defect_error(defect[i]);
                return nsys > 1 ? fail(rc, "system " + std::to_string(i) + ": " + g_err) : rc;
            }
    }
    // ---- device copy of A: block diagonal, systems in the caller's order
    if (!F->A_row.alloc((n + 1) * sizeof(int64_t)) || !F->A_col.alloc(nnz * sizeof(int32_t) + 4) ||
        !F->A_val.alloc(nnz * sizeof(double) + 8))
        return fail(HS_ERR_NOMEM, "device copy of A");
    for (int i = 0; i < nsys; ++i) {
        const hipMemcpyKind kind = A[i].on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        HIP_TRY(hipMemcpyAsync(F->A_row.as<int64_t>() + row_off[i], A[i].row_ptr, (A[i].n + 1) * sizeof(int64_t),
                               kind, st));
        if (A[i].nnz) {
            HIP_TRY(hipMemcpyAsync(F->A_col.as<int32_t>() + nnz_off[i], A[i].col_idx, A[i].nnz * sizeof(int32_t),
                                   kind, st));
            HIP_TRY(hipMemcpyAsync(F->A_val.as<double>() + nnz_off[i], A[i].val, A[i].nnz * sizeof(double), kind,
                                   st));
        }
        launch_shift_csr(A[i].n, A[i].nnz, row_off[i], nnz_off[i], F->A_row.as<int64_t>() + row_off[i],
                         F->A_col.as<int32_t>() + nnz_off[i], st);
    }
    // ---- symmetry (the batch is factored in the general form unless every system is symmetric)
    if (F->opts.symmetric < 0) {
        int sym = 1;
        for (int i = 0; i < nsys && sym; ++i) {
            std::vector<double> v_h(A[i].nnz);
            if (A[i].nnz)
                HIP_TRY(hipMemcpyAsync(v_h.data(), A[i].val, A[i].nnz * sizeof(double),
                                       A[i].on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            for (int64_t r = 0; r < A[i].n && sym; ++r)
                for (int64_t e = rp[i][r]; e < rp[i][r + 1] && sym; ++e) {
                    const int64_t j = ci[i][e];
                    const int32_t* lo = ci[i] + rp[i][j];
                    const int32_t* hi = ci[i] + rp[i][j + 1];
                    const int32_t* it = std::lower_bound(lo, hi, (int32_t)r);
                    if (it == hi || *it != r || v_h[it - ci[i]] != v_h[e]) sym = 0;
                }
        }
        F->symmetric = sym;
    } else {
        F->symmetric = F->opts.symmetric ? 1 : 0;
    }

    // ---- symbolic analysis (integer work only), one host thread per system
    auto t0 = clock::now();
    {
        HostScope hs_(PF_H_SYMBOLIC);
        std::vector<Symbolic> parts(nsys);
        std::vector<int> rcs(nsys, 0);
        const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
        parallel_for(nsys, std::min(hw, 16), [&](int i) {
            const bool grid = G[i].dim > 0;  // dim 0: partition the graph of A
            rcs[i] = build_symbolic(A[i].n, rp[i], ci[i], grid ? G[i].nx : 0, grid ? G[i].ny : 0, grid ? G[i].nz : 0,
                                    F->opts.leaf_size, parts[i]);
        });
        for (int i = 0; i < nsys; ++i)
            if (rcs[i])
                return fail(rcs[i], (nsys > 1 ? "system " + std::to_string(i) + ": " : std::string()) +
                                        (rcs[i] == HS_ERR_GEOMETRY ? "n != nx*ny*nz" : "bad symbolic arguments"));
        combine_symbolic(parts, nsys == 1, F->sym, F->forest);
    }
    // the host patterns are no longer read: the staging buffer is free again
    if (pin_lock.owns_lock()) pin_lock.unlock();
    auto t1 = clock::now();
    F->info.symbolic_seconds = std::chrono::duration<double>(t1 - t0).count();
    const int nlev = F->sym.nlevels;
    if (nlev > 64) return fail(HS_ERR_UNSUPPORTED, "more than 64 levels");
    F->levels.clear();
    F->levels.resize(nlev);
    std::vector<SolvePlan> splans(nlev);
    if (!F->cluster_of.alloc(n * sizeof(int)) || !F->local_of.alloc(n * sizeof(int)))
        return fail(HS_ERR_NOMEM, "dof maps");
    HIP_TRY(hipMemcpyAsync(F->cluster_of.p, F->sym.cluster_of.data(), n * sizeof(int), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(F->local_of.p, F->sym.local_of.data(), n * sizeof(int), hipMemcpyHostToDevice, st));
    // ---- per-system Krylov segments: chunks of KRY_CHUNK rows from each system's first row
    {
        std::vector<int> chunk_sys, sys_chunk0(nsys + 1, 0);
        std::vector<int64_t> chunk_r0;
        for (int i = 0; i < nsys; ++i) {
            for (int64_t r = row_off[i]; r < row_off[i + 1]; r += KRY_CHUNK) {
                chunk_sys.push_back(i);
                chunk_r0.push_back(r);
            }
            sys_chunk0[i + 1] = (int)chunk_sys.size();
        }
        Blob sb;
        const size_t o_ro = sb.add(row_off), o_cs = sb.add(chunk_sys), o_cr = sb.add(chunk_r0),
                     o_sc = sb.add(sys_chunk0);
        if (!F->seg_buf.alloc(sb.data.size())) return fail(HS_ERR_NOMEM, "segment tables");
        HIP_TRY(hipMemcpyAsync(F->seg_buf.p, sb.data.data(), sb.data.size(), hipMemcpyHostToDevice, st));
        HIP_TRY(hipStreamSynchronize(st));
        char* b = F->seg_buf.as<char>();
        F->segs.nsys = nsys;
        F->segs.nchunks = (int)chunk_sys.size();
        F->segs.row_off = (const int64_t*)(b + o_ro);
        F->segs.chunk_sys = (const int*)(b + o_cs);
        F->segs.chunk_r0 = (const int64_t*)(b + o_cr);
        F->segs.sys_chunk0 = (const int*)(b + o_sc);
    }

    // ---- numeric factorization, level by level (Alg. 1)
    LevelData* prev = nullptr;
    std::vector<size_t> offs;
    double flops = 0.0;
    const bool mixed = F->opts.precision == HS_MIXED;
    const int64_t fp64_dofs = F->opts.coarse_fp64_dofs > 0 ? F->opts.coarse_fp64_dofs : MIXED_FP64_DOFS;
    for (int lvl = 0; lvl < nlev; ++lvl) {
        LevelData& LD = F->levels[lvl];
        const LevelSymbolic& S = F->sym.levels[lvl];
        if (lvl == 0) {
            LD.m.resize(S.ncl);
            for (int c = 0; c < S.ncl; ++c) LD.m[c] = F->sym.leaf_ptr[c + 1] - F->sym.leaf_ptr[c];
        } else {
            LD.m.assign(S.ncl, 0);
            for (int p = 0; p < S.ncl; ++p)
                for (int c = 2 * p; c < std::min(2 * p + 2, prev->ncl); ++c) LD.m[p] += prev->k[c];
        }
        // per system: a level whose clusters all neighbour each other has no
        // fill and is factored densely (Alg. 1, conventional factorization);
        // the mixed form stores a system's level in float32 when it is not
        // that level and has more than fp64_dofs unknowns
        const std::vector<int>& coff = F->forest.cl_off[lvl];
        const int alive = (int)coff.size() - 1;
        LD.f32.assign(S.ncl, 0);
        LD.dense.assign(S.ncl, 0);
        LD.any_f32 = 0;
        std::vector<std::array<int, 2>> dense_ranges;
        for (int j = 0; j < alive; ++j) {
            const int c0 = coff[j], c1 = coff[j + 1];
            int64_t dofs = 0;
            for (int c = c0; c < c1; ++c) dofs += LD.m[c];
            // with pivoting a complete level runs through the per-cluster kernels
            const bool dn = F->forest.dense[j] == lvl && !F->opts.pivoting;
            const int single = (mixed && lvl < F->forest.dense[j] && dofs > fp64_dofs) ? 1 : 0;
            for (int c = c0; c < c1; ++c) {
                LD.f32[c] = single;
                LD.dense[c] = dn;
            }
            LD.any_f32 |= single;
            if (dn) dense_ranges.push_back({c0, c1});
        }
        Blob blob;
        BlobLease lease(blob);
        {
            HostScope hs_(PF_H_PLAN);
            rc = plan_level(F, lvl, blob, offs);
        }
        if (rc) return rc;
        {
            HostScope hs_(PF_H_ALLOC);
            if (!LD.meta.alloc(blob.data.size())) return fail(HS_ERR_NOMEM, "level metadata");
            if (!LD.blocks.alloc(LD.block_bytes)) return fail(HS_ERR_NOMEM, "block store");
            if (!LD.rec.alloc(LD.rec_bytes)) return fail(HS_ERR_NOMEM, "factor records");
            if (!F->ws.ensure(LD.ws_elems * sizeof(double))) return fail(HS_ERR_NOMEM, "workspace");
            if (!LD.pairs.alloc((LD.npairs + 1) * sizeof(int))) return fail(HS_ERR_NOMEM, "neighbour pairs");
            if (!LD.ids.alloc((LD.ncl + 3 * (LD.nadj + LD.nfill) + 1) * sizeof(int)))
                return fail(HS_ERR_NOMEM, "level block ids");
        }
        {
            HostScope hs_(PF_H_UPLOAD);
            HIP_TRY(hipMemcpyAsync(LD.meta.p, blob.data.data(), blob.data.size(), hipMemcpyHostToDevice, st));
        }
        bind_level(LD, offs, F);
        launch_level_ids(S.ncl, LD.dev.nbr_ptr, LD.dev.nbr_id, LD.dev.fill_ptr, LD.dev.fill_id, LD.dev_pos,
                         LD.dev_pat_ptr, LD.dev_pat, LD.ids.as<int>(), LD.ids.as<int>() + LD.ncl,
                         LD.ids.as<int>() + LD.ncl + LD.nadj, LD.ids.as<int>() + LD.ncl + 2 * LD.nadj,
                         LD.ids.as<int>() + LD.ncl + 3 * LD.nadj, LD.ids.as<int>() + LD.ncl + 3 * LD.nadj + LD.nfill,
                         LD.ids.as<int>() + LD.ncl + 3 * LD.nadj + 2 * LD.nfill, st);
        launch_pair_blocks(S.ncl, LD.dev.nbr_ptr, LD.dev.nbr_id, LD.dev_pat_ptr, LD.dev_pat, LD.dev.pair_base,
                           LD.pairs.as<int>(), st);
        launch_fill_zero(LD.blocks.p, LD.block_bytes, st);
        if (lvl == 0) {
            launch_assemble0(n, F->A_row.as<int64_t>(), F->A_col.as<int32_t>(), F->A_val.as<double>(),
                             F->cluster_of.as<int>(), F->local_of.as<int>(), LD.dev.m, LD.dev_pat_ptr, LD.dev_pat,
                             LD.dev.blk_off, LD.blocks.p, LD.dev_f32, st);
        } else {
            // parent blocks from the children's coarse blocks
            {
                ProfScope ps(PF_MERGE, st);
                launch_merge(LD.nblk, LD.dev_pat_ptr, LD.dev_pat, LD.ncl, prev->dev_pat_ptr, prev->dev_pat, prev->ncl,
                             prev->dev.k, prev->dev.m, prev->dev.blk_off, prev->blocks.p, prev->dev_f32, LD.dev.m,
                             LD.dev.blk_off, LD.blocks.p, LD.dev_f32, st);
            }
            // the children's blocks are freed once the merge has read them, as
            // observed by the host: a pool trim on another thread (the serving
            // loop's, after an eviction) may return memory whose asynchronous
            // free is still pending, and the merge would then read freed memory
            {
                HostScope hs_(PF_H_SYNC);
                HIP_TRY(hipStreamSynchronize(st));
            }
            prev->blocks.release();
            prev->dev.blocks = nullptr;
        }
        if (F->opts.keep_levels) {
            rc = keep_level_matrix(F, LD, st);
            if (rc) return rc;
        }
        DevBuf dense_aux, dense_mat;
        int* dflag = nullptr;
        if (!dense_ranges.empty()) {
            rc = factor_dense_ranges(F, lvl, dense_ranges, dense_aux, dense_mat, dflag, st);
            if (rc) return rc;
        }
        for (auto& CH : LD.colours)
            for (int t = 0; t < 2; ++t)
                for (const ColourDev& C : CH.fac[t]) {
                if (C.n == 0) continue;
                const bool rank = F->opts.eps > 0.0 && C.fill_total > 0;  // rank revelation needed
                const bool gram = rank && !F->qrcp;
                // the offsets ride in the Gram launch unless either family is timed
                const int pivot_fam = t == 0 ? PF_PIVOT_F32 : PF_PIVOT;
                const bool fused_offsets = gram && !prof_timed(PF_GRAM) && !prof_timed(pivot_fam);
                if (gram) {
                    ProfScope ps(PF_GRAM, st);
                    launch_gram(LD.dev, C, st, fused_offsets);
                }
                if (!fused_offsets) launch_offsets(LD.dev, C, st);
                if (rank && F->qrcp) {
                    ProfScope ps(PF_GRAM, st);
                    launch_qrcp(LD.dev, C, st);
                }
                {
                    ProfScope ps(pivot_fam, st);
                    launch_pivot(LD.dev, C, st);
                }
                if (prof_timed(PF_FILL) || prof_timed(PF_NBR)) {  // one family per launch
                    if (C.fill_total > 0) {
                        ProfScope ps(PF_FILL, st);
                        launch_fill_update(LD.dev, C, st);
                    }
                    if (C.nbr_total > 0) {
                        ProfScope ps(PF_NBR, st);
                        launch_nbr_update(LD.dev, C, st);
                    }
                } else {
                    launch_fill_nbr_update(LD.dev, C, st);
                }
                if (C.tile_total > 0) {
                    ProfScope ps(t == 0 ? PF_SCHUR_F32 : PF_SCHUR, st);
                    launch_schur(LD.dev, C, st);
                }
            }
        HIP_TRY(hipGetLastError());
        // the previous level's solve plan on the host while this level runs
        if (lvl > 0) {
            HostScope hs_(PF_H_SOLVE_PLAN);
            plan_solve_level(F, lvl - 1, splans[lvl - 1]);
            account_level(F, lvl - 1, splans[lvl - 1]);
        }
        // ranks decide the next level's sizes: one synchronisation per level
        LD.k.resize(LD.ncl);
        std::vector<int> flag(LD.ncl), ntot(LD.ncl), hdflag(dense_ranges.size(), 0);
        {
            HostScope hs_(PF_H_SYNC);
            HIP_TRY(hipMemcpyAsync(LD.k.data(), LD.dev.k, LD.ncl * sizeof(int), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipMemcpyAsync(flag.data(), LD.dev.flag, LD.ncl * sizeof(int), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipMemcpyAsync(ntot.data(), LD.dev.ntot, LD.ncl * sizeof(int), hipMemcpyDeviceToHost, st));
            if (dflag)
                HIP_TRY(hipMemcpyAsync(hdflag.data(), dflag, hdflag.size() * sizeof(int), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
        }
        LD.pairs.release();  // used by this level's Schur updates only
        LD.dev.pair_blk = nullptr;
        for (size_t r = 0; r < dense_ranges.size(); ++r)
            if (hdflag[r]) {
                F->info.breakdown_level = lvl;
                F->info.breakdown_cluster = -1;
                return fail(HS_ERR_BREAKDOWN, "zero or non-finite pivot at level " + std::to_string(lvl) +
                                                  " (dense level, clusters " + std::to_string(dense_ranges[r][0]) +
                                                  ".." + std::to_string(dense_ranges[r][1] - 1) + ")");
            }
        for (int c = 0; c < LD.ncl; ++c)
            if (flag[c]) {
                F->info.breakdown_level = lvl;
                F->info.breakdown_cluster = c;
                return fail(HS_ERR_BREAKDOWN, "zero or non-finite pivot at level " + std::to_string(lvl) +
                                                  ", cluster " + std::to_string(c) +
                                                  (flag[c] == 2 ? " (fine block)" : " (pivot block)"));
            }
        if (g_prof_on) prof_flush();
        LD.ntot_host = std::move(ntot);  // read by account_level
        // solve plan of the level: segments and part offsets
        LD.seg.assign(LD.ncl + 1, 0);
        for (int c = 0; c < LD.ncl; ++c) LD.seg[c + 1] = LD.seg[c] + LD.m[c];
        LD.nseg = LD.seg[LD.ncl];
        int64_t coarse = 0;
        int max_all = 0;
        for (int c = 0; c < LD.ncl; ++c) {
            coarse += LD.k[c];
            max_all = std::max(max_all, LD.m[c]);
        }
        F->info.coarse_dofs[lvl] = coarse;
        F->info.level_clusters[lvl] = LD.ncl;
        F->info.level_colors[lvl] = S.ncolors;
        F->info.ncolors_total += S.ncolors;
        F->info.max_cluster = std::max(F->info.max_cluster, max_all);
        LD.max_m = max_all;  // from here on: the solve's largest cluster
        prev = &LD;
    }
    // the last level's blocks are no longer needed
    if (prev) {
        prev->blocks.release();
        prev->dev.blocks = nullptr;
    }
    F->ws.release();

    // ---- solve plan: the last level's host part, then every level's metadata uploaded
    {
        HostScope hs_solve(PF_H_SOLVE_PLAN);
        plan_solve_level(F, nlev - 1, splans[nlev - 1]);
        account_level(F, nlev - 1, splans[nlev - 1]);
        for (int lvl = 0; lvl < nlev; ++lvl) {
            rc = bind_solve_level(F, lvl, splans[lvl], st);
            if (rc) return rc;
        }
    }
    double rec_bytes = 0.0, apply_flops = 0.0;
    for (const SolvePlan& sp : splans) {
        rec_bytes += sp.rec_bytes;
        apply_flops += sp.apply_flops;
        flops += sp.factor_flops;
    }
    // solve vector layout: y, z and out of every level, level after level
    F->vec_off.assign(nlev + 1, 0);
    F->part_max = 0;
    for (int l = 0; l < nlev; ++l) {
        F->vec_off[l + 1] = F->vec_off[l] + 3 * F->levels[l].nseg;
        F->part_max = std::max(F->part_max, F->levels[l].part_max);
    }
    F->vec_total = F->vec_off[nlev];
    HIP_TRY(hipStreamSynchronize(st));
    if (g_prof_on) prof_flush();
    F->info.factor_flops = flops;
    F->info.apply_flops_per_rhs = apply_flops;
    F->info.factor_bytes = rec_bytes;
    F->info.numeric_seconds = std::chrono::duration<double>(clock::now() - t1).count();
    F->info.nlevels = nlev;
    F->info.n = n;
    return HS_OK;
}

// ================================================================= solve

static int ensure_solve_buffers(hs_factor_s* F, int nrhs) {
    if (F->solve_nrhs >= nrhs && F->vecs.p) return HS_OK;
    F->drop_sweeps();  // captured sweeps refer to the buffers reallocated below
    if (!F->vecs.alloc((F->vec_total * nrhs + 1) * sizeof(double))) return fail(HS_ERR_NOMEM, "solve vectors");
    if (!F->part.alloc((F->part_max * nrhs + 1) * sizeof(double))) return fail(HS_ERR_NOMEM, "solve partials");
    F->solve_nrhs = nrhs;
    return HS_OK;
}

static int solve_chunk(hs_factor_s* F, int nrhs, const double* B, int64_t ldb, double* X, int64_t ldx, hipStream_t st);

// Right-hand sides per pass so that an m x nrhs tile of the largest cluster
// stays within 64 KB of LDS in the apply kernels.
static int solve_impl(hs_factor_s* F, int nrhs, const double* B, int64_t ldb, double* X, int64_t ldx, hipStream_t st) {
    int maxm = 1;
    for (auto& LD : F->levels) maxm = std::max(maxm, LD.max_m);
    const int per = std::max(1, std::min(nrhs, 8192 / maxm));
    for (int r0 = 0; r0 < nrhs; r0 += per) {
        const int nr = std::min(per, nrhs - r0);
        int rc = solve_chunk(F, nr, B + r0 * ldb, ldb, X + r0 * ldx, ldx, st);
        if (rc) return rc;
    }
    return HS_OK;
}

// Alg. 2: forward sweep colour by colour up the levels, backward sweep down
// (level vectors only).  A colour's float32 and float64 lists are independent
// launches.  base: the level vectors (vec_total x nrhs doubles), part: the
// backward partials (part_max x nrhs); prof: bracket the launches for the
// per-family profiler.
static void solve_sweeps(hs_factor_s* F, int nrhs, hipStream_t st, double* base, double* part, bool prof = true) {
    const int nlev = (int)F->levels.size();
    auto Y = [&](int l) { return base + F->vec_off[l] * nrhs; };
    auto Z = [&](int l) { return base + (F->vec_off[l] + F->levels[l].nseg) * nrhs; };
    auto O = [&](int l) { return base + (F->vec_off[l] + 2 * F->levels[l].nseg) * nrhs; };
    const int fam = prof ? PF_APPLY : -1;
    for (int l = 0; l < nlev; ++l) {
        LevelData& LD = F->levels[l];
        for (auto& CH : LD.colours)
            for (int t = 0; t < 2; ++t) {
                const ColourDev& C = CH.sol[t];
                if (C.n == 0) continue;
                ProfScope ps(fam, st);
                launch_apply_fwd(LD.sdev, C, Y(l), Z(l), nrhs, st);
            }
        if (l + 1 < nlev)
            launch_to_coarse(LD.sdev, F->levels[l + 1].sdev.seg, F->levels[l + 1].ncl, Z(l), Y(l + 1), nrhs, st);
    }
    for (int l = nlev - 1; l >= 0; --l) {
        LevelData& LD = F->levels[l];
        if (l + 1 < nlev)
            launch_from_coarse(LD.sdev, F->levels[l + 1].sdev.seg, F->levels[l + 1].ncl, O(l + 1), Z(l), nrhs, st);
        for (int c = (int)LD.colours.size() - 1; c >= 0; --c) {
            auto& CH = LD.colours[c];
            for (int t = 0; t < 2; ++t) {
                const ColourDev& C = CH.sol[t];
                if (C.n == 0) continue;
                ProfScope ps(fam, st);
                launch_apply_bwd_acc(LD.sdev, C, Z(l), O(l), part, CH.part_off[t], nrhs, st);
                launch_apply_bwd_t(LD.sdev, C, Z(l), O(l), part, CH.part_off[t], nrhs, st);
            }
        }
    }
}

// The sweeps run from a graph captured at the first solve with this
// right-hand-side count (thousands of small launches become one), or launch
// by launch while the per-family profiler is on.
static int solve_chunk(hs_factor_s* F, int nrhs, const double* B, int64_t ldb, double* X, int64_t ldx, hipStream_t st) {
    int rc = ensure_solve_buffers(F, nrhs);
    if (rc) return rc;
    const int nlev = (int)F->levels.size();
    LevelData& L0 = F->levels[0];
    double* Y0 = F->vecs.as<double>();
    double* O0 = Y0 + 2 * L0.nseg * nrhs;
    launch_scatter_rhs(F->n, F->cluster_of.as<int>(), F->local_of.as<int>(), L0.sdev.seg, L0.dev.m, B, ldb, Y0, nrhs,
                       st);
    if (prof_timed(PF_APPLY) || nlev == 0) {
        solve_sweeps(F, nrhs, st, F->vecs.as<double>(), F->part.as<double>());
    } else {
        hipGraphExec_t ex = nullptr;
        for (auto& g : F->sweeps)
            if (g.first == nrhs) ex = g.second;
        if (!ex) {
            if (!F->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&F->cap_stream, hipStreamNonBlocking));
            hipGraph_t g = nullptr;
            bool ok;
            {
                std::lock_guard<std::mutex> lk(g_capture_mu);
                ok = hipStreamBeginCapture(F->cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
                if (ok) {
                    solve_sweeps(F, nrhs, F->cap_stream, F->vecs.as<double>(), F->part.as<double>());
                    ok = hipStreamEndCapture(F->cap_stream, &g) == hipSuccess && g;
                }
            }
            if (ok) ok = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess;
            if (g) (void)hipGraphDestroy(g);
            if (ok) {
                F->sweeps.push_back({nrhs, ex});
            } else {
                // a capture can be invalidated from outside (for instance by
                // work another thread puts on the legacy default stream):
                // nothing it recorded ran, so the sweeps run launch by launch
                (void)hipGetLastError();
                ex = nullptr;
            }
        }
        if (ex) {
            HIP_TRY(hipGraphLaunch(ex, st));
            F->sweep_stream = st;
        } else {
            solve_sweeps(F, nrhs, st, F->vecs.as<double>(), F->part.as<double>());
        }
    }
    launch_gather_sol(F->n, F->cluster_of.as<int>(), F->local_of.as<int>(), L0.sdev.seg, L0.dev.m, O0, X, ldx, nrhs,
                      st);
    HIP_TRY(hipGetLastError());
    return HS_OK;
}

// ------------------------------------------------- allocation-free solve
// hs_solve_noalloc keeps the level vectors and backward partials of the
// sweeps in this file-scope device array instead of buffers of its own.  Each
// GPU holds its own copy, from when the library's code is loaded on it until
// the process ends.  In host code the name `scratch` stands for a host-side
// shadow, not for device memory: the array's device address is taken once per
// device with hipGetSymbolAddress (scratch_ptr) and only that address is
// handed to kernels.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_BYTES / sizeof(double)];
constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};
static size_t g_noalloc_limit = NOALLOC_SCRATCH_BYTES;  // test hook: bytes of the array a call may use

// Device address of the current device's array (looked up on the first call
// with that device current).
static int scratch_ptr(double** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(HS_ERR_ARG, "device index beyond the supported 64");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(HS_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return HS_OK;
}

// The sweeps of Alg. 2 on buffers cut from the array at base (launch by
// launch, no graph, no profiler events): columns in passes of as many as the
// array and the apply kernels' LDS tiles allow.
static int solve_noalloc_impl(hs_factor_s* F, int nrhs, const double* B, int64_t ldb, double* X, int64_t ldx,
                              hipStream_t st, double* base) {
    const int64_t per_col = F->vec_total + F->part_max + 1;  // doubles per right-hand side
    size_t limit_bytes;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        limit_bytes = g_noalloc_limit;
    }
    const int64_t cap = (int64_t)(limit_bytes / sizeof(double));
    if (per_col > cap)
        return fail(HS_ERR_NOMEM, "the allocation-free solve needs " + std::to_string(per_col * sizeof(double)) +
                                      " bytes of scratch per right-hand side; its device array has " +
                                      std::to_string(limit_bytes) + " (use hs_solve)");
    int maxm = 1;
    for (auto& LD : F->levels) maxm = std::max(maxm, LD.max_m);
    const int per = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)nrhs, 8192 / maxm, cap / per_col}));
    LevelData& L0 = F->levels[0];
    for (int r0 = 0; r0 < nrhs; r0 += per) {
        const int nr = std::min(per, nrhs - r0);
        double* Y0 = base;
        double* O0 = Y0 + 2 * L0.nseg * nr;
        double* part = base + F->vec_total * nr;
        launch_scatter_rhs(F->n, F->cluster_of.as<int>(), F->local_of.as<int>(), L0.sdev.seg, L0.dev.m,
                           B + r0 * ldb, ldb, Y0, nr, st);
        solve_sweeps(F, nr, st, base, part, false);
        launch_gather_sol(F->n, F->cluster_of.as<int>(), F->local_of.as<int>(), L0.sdev.seg, L0.dev.m, O0,
                          X + r0 * ldx, ldx, nr, st);
    }
    HIP_TRY(hipGetLastError());
    return HS_OK;
}

// ================================================================ Krylov
//
// CG and GMRES(restart) of Sec. 5 in float64 with the factorization as the
// preconditioner.  Every system of the factor and every right-hand side is
// its own lane l = s + nsys * c with its own scalars and stopping test
// (||b - A x||_2 <= tol ||b||_2); lanes advance together, a finished lane is
// frozen (its coefficients are zero), so its numbers are those of a solve of
// that system alone.

// Work vectors (n x nrhs each): 4 for CG, 3 + restart + 1 for GMRES; lane
// scalars and chunk partials behind them.
static int ensure_krylov(hs_factor_s* F, int nrhs, int restart) {
    const int64_t n = F->n;
    const int64_t L = (int64_t)F->forest.nsys * nrhs;
    const int64_t r1 = restart > 0 ? restart + 1 : 1;
    const int64_t vecs = restart > 0 ? 3 + r1 : 4;
    const size_t bytes =
        (size_t)(vecs * n * nrhs + (2 * r1 + 8) * L + r1 * (int64_t)nrhs * F->segs.nchunks + 64) * sizeof(double);
    if (F->kry.bytes >= bytes) return HS_OK;
    if (!F->kry.alloc(bytes)) return fail(HS_ERR_NOMEM, "Krylov workspace");
    return HS_OK;
}

// hout[v * L + l] = per-lane dot products of a_v and b (one synchronisation).
static int sdots_host(hs_factor_s* F, int nvec, const double* a, int64_t vstride, int64_t lda, const double* b,
                      int64_t ldb, int nrhs, double* part, double* dout, double* hout, hipStream_t st) {
    launch_sdots(F->segs, nvec, a, vstride, lda, b, ldb, nrhs, part, dout, st);
    const int64_t L = (int64_t)F->forest.nsys * nrhs;
    HIP_TRY(hipMemcpyAsync(hout, dout, nvec * L * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (g_prof_on) prof_flush();
    return HS_OK;
}

static int upload(double* d, const std::vector<double>& h, hipStream_t st) {
    HIP_TRY(hipMemcpyAsync(d, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, st));
    return HS_OK;
}

static int pcg_impl(hs_factor_s* F, int nrhs, const double* B, int64_t ldb, double* X, int64_t ldx, double tol,
                    int maxit, int* iters, double* relres, hipStream_t st) {
    int rc = ensure_krylov(F, nrhs, 0);
    if (rc) return rc;
    const int64_t n = F->n;
    const int L = F->forest.nsys * nrhs;
    const SegDev& G = F->segs;
    double* w = F->kry.as<double>();
    double* R = w;
    double* Zv = R + n * nrhs;
    double* P = Zv + n * nrhs;
    double* Q = P + n * nrhs;
    double* d_alpha = Q + n * nrhs;  // lane scalars
    double* d_beta = d_alpha + L;
    double* d_one = d_beta + L;
    double* d_zero = d_one + L;
    double* d_dot = d_zero + L;
    double* part = d_dot + 2 * L;
    std::vector<double> one(L, 1.0), zero(L, 0.0);
    if ((rc = upload(d_one, one, st)) || (rc = upload(d_zero, zero, st))) return rc;
    std::vector<double> bn(L), rz(L), rzn(L), rzo(L, 0.0), pq(L), rr(L), alpha(L), beta(L);
    // A float32 factor is a slightly nonlinear preconditioner: the flexible
    // (Polak-Ribiere) beta = r_new^T (z_new - z_old) / r_old^T z_old keeps CG
    // converging; with a float64 factor the classical beta is used.
    const bool flexible = F->opts.precision == HS_MIXED;
    auto dots = [&](const double* a, int64_t lda, const double* b, int64_t ldb_, double* out) {
        return sdots_host(F, 1, a, 0, lda, b, ldb_, nrhs, part, d_dot, out, st);
    };
    if ((rc = dots(B, ldb, B, ldb, bn.data()))) return rc;
    for (auto& v : bn) v = v > 0 ? std::sqrt(v) : 1.0;
    // x0 = 0, r0 = b
    launch_saxpby(G, d_zero, B, ldb, d_zero, X, ldx, nrhs, st);
    launch_copy(n, B, ldb, R, n, nrhs, st);
    std::vector<char> active(L, 1);
    int nact = L;
    if ((rc = solve_impl(F, nrhs, R, n, Zv, n, st))) return rc;
    launch_copy(n, Zv, n, P, n, nrhs, st);
    if ((rc = dots(R, n, Zv, n, rz.data()))) return rc;
    int it = 0;
    while (nact > 0 && it < maxit) {
        ++it;
        launch_spmv(n, F->A_row.as<int64_t>(), F->A_col.as<int32_t>(), F->A_val.as<double>(), P, n, Q, n, nrhs, st);
        if ((rc = dots(P, n, Q, n, pq.data()))) return rc;
        for (int l = 0; l < L; ++l) alpha[l] = (active[l] && pq[l] != 0.0) ? rz[l] / pq[l] : 0.0;
        if ((rc = upload(d_alpha, alpha, st))) return rc;
        launch_saxpby(G, d_alpha, P, n, d_one, X, ldx, nrhs, st);  // x += alpha p
        for (int l = 0; l < L; ++l) alpha[l] = -alpha[l];
        if ((rc = upload(d_beta, alpha, st))) return rc;
        launch_saxpby(G, d_beta, Q, n, d_one, R, n, nrhs, st);  // r -= alpha q
        if ((rc = dots(R, n, R, n, rr.data()))) return rc;
        nact = 0;
        for (int l = 0; l < L; ++l) {
            if (active[l] && std::sqrt(std::max(rr[l], 0.0)) <= tol * bn[l]) active[l] = 0;
            nact += active[l];
        }
        if (nact == 0) break;
        if (flexible && (rc = dots(R, n, Zv, n, rzo.data()))) return rc;
        if ((rc = solve_impl(F, nrhs, R, n, Zv, n, st))) return rc;
        if ((rc = dots(R, n, Zv, n, rzn.data()))) return rc;
        for (int l = 0; l < L; ++l) {
            beta[l] = (active[l] && rz[l] != 0.0) ? (rzn[l] - rzo[l]) / rz[l] : 0.0;
            rz[l] = rzn[l];
        }
        if ((rc = upload(d_beta, beta, st))) return rc;
        launch_saxpby(G, d_one, Zv, n, d_beta, P, n, nrhs, st);  // p = z + beta p
    }
    // true residual
    launch_spmv(n, F->A_row.as<int64_t>(), F->A_col.as<int32_t>(), F->A_val.as<double>(), X, ldx, Q, n, nrhs, st);
    launch_xmy(n, B, ldb, Q, n, nrhs, st);
    if ((rc = dots(Q, n, Q, n, rr.data()))) return rc;
    bool ok = true;
    for (int l = 0; l < L; ++l) {
        const double r = std::sqrt(std::max(rr[l], 0.0)) / bn[l];
        if (relres) relres[l] = r;
        if (!(r <= tol)) ok = false;
    }
    if (iters) *iters = it;
    return ok ? HS_OK : HS_WARN_NOT_CONVERGED;
}

// Right-preconditioned GMRES(restart): x = M^{-1} V y, the basis V
// orthonormalised by classical Gram-Schmidt applied twice (each pass one
// batched product V^T w), Givens rotations on the host per lane.
static int gmres_impl(hs_factor_s* F, int nrhs, const double* B, int64_t ldb, double* X, int64_t ldx, double tol,
                      int maxit, int restart, int* iters, double* relres, hipStream_t st) {
    if (restart < 1) restart = 30;
    int rc = ensure_krylov(F, nrhs, restart);
    if (rc) return rc;
    const int64_t n = F->n;
    const int L = F->forest.nsys * nrhs;
    const int R1 = restart + 1;
    const SegDev& G = F->segs;
    const int64_t vs = n * nrhs;  // stride between basis vectors
    double* w = F->kry.as<double>();
    double* Rv = w;
    double* T = Rv + vs;
    double* Wv = T + vs;
    double* V = Wv + vs;
    double* d_coef = V + (int64_t)R1 * vs;  // R1 x L
    double* d_a = d_coef + (int64_t)R1 * L;
    double* d_b = d_a + L;
    double* d_one = d_b + L;
    double* d_zero = d_one + L;
    double* d_dot = d_zero + L;  // R1 x L
    double* part = d_dot + (int64_t)R1 * L;
    std::vector<double> one(L, 1.0), zero(L, 0.0);
    if ((rc = upload(d_one, one, st)) || (rc = upload(d_zero, zero, st))) return rc;
    auto hidx = [&](int i, int j) { return (size_t)i + (size_t)j * R1; };
    std::vector<double> bn(L), rnorm(L), h1((size_t)R1 * L), h2((size_t)R1 * L), hn2(L), a(L), coef((size_t)R1 * L);
    std::vector<std::vector<double>> H(L), g(L), cs(L), sn(L);
    std::vector<int> it_l(L, 0), jused(L, 0);
    std::vector<char> active(L, 0), inc(L, 0), live(L, 0);
    if ((rc = sdots_host(F, 1, B, 0, ldb, B, ldb, nrhs, part, d_dot, bn.data(), st))) return rc;
    for (int l = 0; l < L; ++l) {
        bn[l] = std::sqrt(std::max(bn[l], 0.0));
        rnorm[l] = bn[l];
        active[l] = bn[l] > 0.0;  // b = 0: x = 0 is exact
        if (bn[l] == 0.0) bn[l] = 1.0;
    }
    launch_saxpby(G, d_zero, B, ldb, d_zero, X, ldx, nrhs, st);  // x = 0
    launch_copy(n, B, ldb, Rv, n, nrhs, st);
    for (;;) {
        int ninc = 0;
        for (int l = 0; l < L; ++l) {
            inc[l] = active[l] && it_l[l] < maxit;
            live[l] = inc[l];
            ninc += inc[l];
            jused[l] = 0;
        }
        if (ninc == 0) break;
        // V_0 = r / ||r||
        for (int l = 0; l < L; ++l) {
            a[l] = inc[l] ? 1.0 / rnorm[l] : 0.0;
            if (inc[l]) {
                H[l].assign((size_t)R1 * restart, 0.0);
                g[l].assign(R1, 0.0);
                cs[l].assign(restart, 0.0);
                sn[l].assign(restart, 0.0);
                g[l][0] = rnorm[l];
            }
        }
        if ((rc = upload(d_a, a, st))) return rc;
        launch_saxpby(G, d_a, Rv, n, d_zero, V, n, nrhs, st);
        int jmax = 0;
        for (int j = 0; j < restart; ++j) {
            int nlive = 0;
            for (int l = 0; l < L; ++l) nlive += live[l];
            if (nlive == 0) break;
            double* Vj = V + (int64_t)j * vs;
            if ((rc = solve_impl(F, nrhs, Vj, n, T, n, st))) return rc;
            launch_spmv(n, F->A_row.as<int64_t>(), F->A_col.as<int32_t>(), F->A_val.as<double>(), T, n, Wv, n, nrhs,
                        st);
            // two passes of classical Gram-Schmidt against V_0 .. V_j
            for (int pass = 0; pass < 2; ++pass) {
                std::vector<double>& h = pass ? h2 : h1;
                if ((rc = sdots_host(F, j + 1, V, vs, n, Wv, n, nrhs, part, d_dot, h.data(), st))) return rc;
                for (int v = 0; v <= j; ++v)
                    for (int l = 0; l < L; ++l) coef[(size_t)v * L + l] = live[l] ? -h[(size_t)v * L + l] : 0.0;
                HIP_TRY(hipMemcpyAsync(d_coef, coef.data(), (size_t)(j + 1) * L * sizeof(double),
                                       hipMemcpyHostToDevice, st));
                launch_scomb(G, j + 1, d_coef, V, vs, n, d_one, Wv, n, nrhs, st);
            }
            if ((rc = sdots_host(F, 1, Wv, 0, n, Wv, n, nrhs, part, d_dot, hn2.data(), st))) return rc;
            for (int l = 0; l < L; ++l) {
                a[l] = 0.0;
                if (!live[l]) continue;
                std::vector<double>& Hl = H[l];
                for (int v = 0; v <= j; ++v) Hl[hidx(v, j)] = h1[(size_t)v * L + l] + h2[(size_t)v * L + l];
                const double hn = std::sqrt(std::max(hn2[l], 0.0));
                Hl[hidx(j + 1, j)] = hn;
                for (int i = 0; i < j; ++i) {
                    const double a0 = Hl[hidx(i, j)], a1 = Hl[hidx(i + 1, j)];
                    Hl[hidx(i, j)] = cs[l][i] * a0 + sn[l][i] * a1;
                    Hl[hidx(i + 1, j)] = -sn[l][i] * a0 + cs[l][i] * a1;
                }
                const double a0 = Hl[hidx(j, j)], a1 = Hl[hidx(j + 1, j)];
                const double den = std::hypot(a0, a1);
                cs[l][j] = den > 0 ? a0 / den : 1.0;
                sn[l][j] = den > 0 ? a1 / den : 0.0;
                Hl[hidx(j, j)] = cs[l][j] * a0 + sn[l][j] * a1;
                Hl[hidx(j + 1, j)] = 0.0;
                g[l][j + 1] = -sn[l][j] * g[l][j];
                g[l][j] = cs[l][j] * g[l][j];
                jused[l] = j + 1;
                ++it_l[l];
                if (std::fabs(g[l][j + 1]) <= tol * bn[l] || hn == 0.0 || it_l[l] >= maxit)
                    live[l] = 0;
                else
                    a[l] = 1.0 / hn;
            }
            jmax = j + 1;
            if ((rc = upload(d_a, a, st))) return rc;
            launch_saxpby(G, d_a, Wv, n, d_zero, V + (int64_t)(j + 1) * vs, n, nrhs, st);
        }
        // y = H^{-1} g per lane; x += M^{-1} V y
        std::fill(coef.begin(), coef.end(), 0.0);
        for (int l = 0; l < L; ++l) {
            a[l] = jused[l] > 0 ? 1.0 : 0.0;
            const int ju = jused[l];
            std::vector<double> y(ju);
            for (int i = ju - 1; i >= 0; --i) {
                double s = g[l][i];
                for (int c = i + 1; c < ju; ++c) s -= H[l][hidx(i, c)] * y[c];
                y[i] = s / H[l][hidx(i, i)];
            }
            for (int i = 0; i < ju; ++i) coef[(size_t)i * L + l] = y[i];
        }
        HIP_TRY(hipMemcpyAsync(d_coef, coef.data(), (size_t)std::max(jmax, 1) * L * sizeof(double),
                               hipMemcpyHostToDevice, st));
        launch_scomb(G, jmax, d_coef, V, vs, n, d_zero, Wv, n, nrhs, st);
        if ((rc = solve_impl(F, nrhs, Wv, n, T, n, st))) return rc;
        if ((rc = upload(d_a, a, st))) return rc;
        launch_saxpby(G, d_a, T, n, d_one, X, ldx, nrhs, st);
        // true residual
        launch_spmv(n, F->A_row.as<int64_t>(), F->A_col.as<int32_t>(), F->A_val.as<double>(), X, ldx, Rv, n, nrhs, st);
        launch_xmy(n, B, ldb, Rv, n, nrhs, st);
        std::vector<double> rn2(L);
        if ((rc = sdots_host(F, 1, Rv, 0, n, Rv, n, nrhs, part, d_dot, rn2.data(), st))) return rc;
        for (int l = 0; l < L; ++l) {
            if (!inc[l]) continue;
            rnorm[l] = std::sqrt(std::max(rn2[l], 0.0));
            if (rnorm[l] <= tol * bn[l]) active[l] = 0;
        }
    }
    bool ok = true;
    int itmax = 0;
    for (int l = 0; l < L; ++l) {
        const double r = rnorm[l] / bn[l];
        if (relres) relres[l] = r;
        if (!(r <= tol)) ok = false;
        itmax = std::max(itmax, it_l[l]);
    }
    if (iters) *iters = itmax;
    return ok ? HS_OK : HS_WARN_NOT_CONVERGED;
}

static int check_device() {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
        (void)hipGetLastError();
        return fail(HS_ERR_NODEVICE, "no HIP device visible");
    }
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(HS_ERR_NODEVICE, std::string("device is ") + prop.gcnArchName + ", the kernels are built for gfx950");
    static bool attr_done = false;
    if (!attr_done) {
        // the pivot kernel keeps clusters up to LDS_M in LDS (dynamic)
        attr_done = true;
    }
    return HS_OK;
}

}  // namespace hs

// =================================================================== C ABI

using namespace hs;

extern "C" {

static int check_opts(const hs_opts* opts) {
    if (!(opts->eps >= 0.0) || opts->leaf_size <= 0 || opts->fixed_rank < 0 || opts->coarse_fp64_dofs < 0 ||
        (opts->precision != HS_FP64 && opts->precision != HS_MIXED) || (opts->pivoting != 0 && opts->pivoting != 1))
        return fail(HS_ERR_ARG, "bad options");
    return HS_OK;
}

static int check_system(const hs_csr* A, const hs_geometry* geom) {
    if (!A->row_ptr || (A->nnz > 0 && (!A->col_idx || !A->val))) return fail(HS_ERR_ARG, "null argument");
    if (A->n <= 0 || A->nnz < 0 || A->n > INT32_MAX) return fail(HS_ERR_ARG, "bad matrix size");
    if (geom->dim < 0 || geom->dim > 3 || (geom->dim > 0 && (int64_t)geom->nx * geom->ny * geom->nz != A->n))
        return fail(HS_ERR_GEOMETRY, "n != nx*ny*nz");
    return HS_OK;
}

static int factor_entry(int32_t nsys, const hs_csr* A, const hs_geometry* geom, const hs_opts* opts, void* hip_stream,
                        hs_factor_t* F_out) {
    g_err.clear();
    if (!F_out) return fail(HS_ERR_ARG, "F_out is NULL");
    *F_out = nullptr;
    if (!A || !geom || !opts || nsys < 1) return fail(HS_ERR_ARG, "null argument or no system");
    int rc = check_opts(opts);
    if (rc) return rc;
    for (int i = 0; i < nsys; ++i) {
        rc = check_system(&A[i], &geom[i]);
        if (rc) return nsys > 1 ? fail(rc, "system " + std::to_string(i) + ": " + g_err) : rc;
    }
    rc = check_device();
    if (rc) return rc;
    std::unique_ptr<hs_factor_s> F(new hs_factor_s());
    F->opts = *opts;
    F->cfg = config_snapshot();
    // rank revelation (Eq. lra): the pivoted Householder QR of F^T under a rank
    // cap or below qrcp_below_eps, else the pivoted Cholesky of F F^T
    F->qrcp = opts->eps > 0.0 &&
              (F->cfg.compression == 1 ||
               (F->cfg.compression == 0 && (opts->fixed_rank > 0 || opts->eps < F->cfg.qrcp_below_eps)));
    F->info.breakdown_level = -1;
    F->info.breakdown_cluster = -1;
    AcctScope scope(&F->acct);
    StreamScope sscope((hipStream_t)hip_stream);
    rc = factor_impl(F.get(), nsys, A, geom, (hipStream_t)hip_stream);
    if (rc < 0) return rc;
    *F_out = F.release();
    return HS_OK;
}

int hs_factor(const hs_csr* A, const hs_geometry* geom, const hs_opts* opts, void* hip_stream, hs_factor_t* F_out) {
    return factor_entry(1, A, geom, opts, hip_stream, F_out);
}

int hs_factor_batch(int32_t nsys, const hs_csr* A, const hs_geometry* geom, const hs_opts* opts, void* hip_stream,
                    hs_factor_t* F_out) {
    return factor_entry(nsys, A, geom, opts, hip_stream, F_out);
}

int hs_factor_systems(hs_factor_t F, int32_t* nsys, int64_t* row_off) {
    if (!F) return fail(HS_ERR_ARG, "null factor");
    if (nsys) *nsys = F->forest.nsys;
    if (row_off) std::copy(F->forest.row_off.begin(), F->forest.row_off.end(), row_off);
    return HS_OK;
}

int hs_solve(hs_factor_t F, int64_t nrhs, const double* B, int64_t ldb, double* X, int64_t ldx, void* hip_stream) {
    g_err.clear();
    if (!F || !B || !X || nrhs < 1 || nrhs > 64 || ldb < F->n || ldx < F->n) return fail(HS_ERR_ARG, "bad argument");
    if (B == X && ldb != ldx) return fail(HS_ERR_ARG, "aliased B and X need equal leading dimensions");
    AcctScope scope(&F->acct);
    StreamScope sscope((hipStream_t)hip_stream);
    return solve_impl(F, (int)nrhs, B, ldb, X, ldx, (hipStream_t)hip_stream);
}

int hs_solve_noalloc(hs_factor_t F, int64_t nrhs, const double* B, int64_t ldb, double* X, int64_t ldx,
                     void* hip_stream) {
    g_err.clear();
    if (!F || !B || !X || nrhs < 1 || nrhs > 64 || ldb < F->n || ldx < F->n) return fail(HS_ERR_ARG, "bad argument");
    if (B == X && ldb != ldx) return fail(HS_ERR_ARG, "aliased B and X need equal leading dimensions");
    double* base = nullptr;
    const int rc = scratch_ptr(&base);
    if (rc) return rc;
    return solve_noalloc_impl(F, (int)nrhs, B, ldb, X, ldx, (hipStream_t)hip_stream, base);
}

int hs_pcg(hs_factor_t F, int64_t nrhs, const double* B, int64_t ldb, double* X, int64_t ldx, double tol, int32_t maxit,
           int32_t* iters_out, double* relres_out, void* hip_stream) {
    g_err.clear();
    if (!F || !B || !X || nrhs < 1 || nrhs > 64 || ldb < F->n || ldx < F->n || !(tol >= 0) || maxit < 0 || B == X)
        return fail(HS_ERR_ARG, "bad argument");
    AcctScope scope(&F->acct);
    StreamScope sscope((hipStream_t)hip_stream);
    return pcg_impl(F, (int)nrhs, B, ldb, X, ldx, tol, maxit, iters_out, relres_out, (hipStream_t)hip_stream);
}

int hs_gmres(hs_factor_t F, int64_t nrhs, const double* B, int64_t ldb, double* X, int64_t ldx, double tol,
             int32_t maxit, int32_t restart, int32_t* iters_out, double* relres_out, void* hip_stream) {
    g_err.clear();
    if (!F || !B || !X || nrhs < 1 || ldb < F->n || ldx < F->n || !(tol >= 0) || maxit < 0 || restart < 1 ||
        restart > 1000 || B == X)
        return fail(HS_ERR_ARG, "bad argument");
    AcctScope scope(&F->acct);
    StreamScope sscope((hipStream_t)hip_stream);
    return gmres_impl(F, (int)nrhs, B, ldb, X, ldx, tol, maxit, restart, iters_out, relres_out,
                      (hipStream_t)hip_stream);
}

int hs_factor_info(hs_factor_t F, hs_info* out) {
    if (!F || !out) return fail(HS_ERR_ARG, "null argument");
    F->info.device_bytes = (double)F->acct.held;
    F->info.peak_device_bytes = (double)F->acct.peak;
    *out = F->info;
    return HS_OK;
}

int hs_factor_ranks(hs_factor_t F, int32_t level, int32_t* ranks) {
    if (!F || !ranks || level < 0 || level >= (int)F->levels.size()) return fail(HS_ERR_ARG, "bad argument");
    const auto& k = F->levels[level].k;
    std::copy(k.begin(), k.end(), ranks);
    return HS_OK;
}

int hs_factor_sizes(hs_factor_t F, int32_t level, int32_t* sizes) {
    if (!F || !sizes || level < 0 || level >= (int)F->levels.size()) return fail(HS_ERR_ARG, "bad argument");
    const auto& m = F->levels[level].m;
    std::copy(m.begin(), m.end(), sizes);
    return HS_OK;
}

int hs_factor_level_matrix(hs_factor_t F, int32_t level, double* out, int64_t dim) {
    if (!F || !out || level < 0 || level >= (int)F->levels.size()) return fail(HS_ERR_ARG, "bad argument");
    const auto& LD = F->levels[level];
    if (LD.kept.empty() && LD.nseg > 0) return fail(HS_ERR_ARG, "level matrices were not kept (opts.keep_levels = 0)");
    if (dim != LD.nseg) return fail(HS_ERR_ARG, "dim must be the level's size");
    std::copy(LD.kept.begin(), LD.kept.end(), out);
    return HS_OK;
}

int hs_factor_record(hs_factor_t F, int32_t level, int32_t cluster, int32_t which, double* out, int64_t cap,
                     int64_t* rows, int64_t* cols) {
    if (!F || !rows || !cols || level < 0 || level >= (int)F->levels.size() || which < 0 || which > 3)
        return fail(HS_ERR_ARG, "bad argument");
    const auto& LD = F->levels[level];
    if (cluster < 0 || cluster >= LD.ncl) return fail(HS_ERR_ARG, "bad cluster");
    const int m = LD.m[cluster], k = LD.k[cluster], f = m - k;
    if (m == 0 || f == 0) {
        *rows = *cols = 0;
        return HS_OK;
    }
    std::vector<int> ntot(1), ncap(1);
    HIP_TRY(hipMemcpy(ntot.data(), LD.dev.ntot + cluster, sizeof(int), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(ncap.data(), LD.dev.ncap + cluster, sizeof(int), hipMemcpyDeviceToHost));
    const int64_t MM = (int64_t)m * m;
    int64_t r, c, ld, e0;
    switch (which) {
        case 0: r = m; c = m; ld = m; e0 = 0; break;
        case 1: r = m; c = m; ld = m; e0 = MM; break;
        case 2: r = f; c = ntot[0]; ld = m; e0 = 2 * MM; break;
        default: r = ntot[0]; c = f; ld = ncap[0]; e0 = 2 * MM + (int64_t)m * ncap[0]; break;
    }
    *rows = r;
    *cols = c;
    if (!out) return HS_OK;  // shape query
    if (r * c > cap) return fail(HS_ERR_ARG, "output too small");
    if (r * c == 0) return HS_OK;
    const size_t es = LD.esz(cluster);
    const char* src = LD.rec.as<char>() + (LD.rec_off[cluster] + e0) * es;
    if (!LD.f32[cluster]) {
        HIP_TRY(hipMemcpy2D(out, r * sizeof(double), src, ld * es, r * es, c, hipMemcpyDeviceToHost));
    } else {
        std::vector<float> tmp((size_t)(r * c));
        HIP_TRY(hipMemcpy2D(tmp.data(), r * es, src, ld * es, r * es, c, hipMemcpyDeviceToHost));
        for (size_t i = 0; i < tmp.size(); ++i) out[i] = tmp[i];
    }
    return HS_OK;
}

int hs_factor_trim(hs_factor_t F, void* hip_stream) {
    if (!F) return fail(HS_ERR_ARG, "null factor");
    StreamScope sscope((hipStream_t)hip_stream);
    F->drop_sweeps();
    F->vecs.release();
    F->part.release();
    F->kry.release();
    F->solve_nrhs = 0;
    return HS_OK;
}

void hs_free(hs_factor_t F) {
    if (!F) return;
    device_sync();  // nothing may still use the buffers or the graphs
    for (auto& g : F->sweeps) (void)hipGraphExecDestroy(g.second);
    F->sweeps.clear();
    StreamScope sscope(nullptr, true);
    delete F;
}

int hs_symbolic_create(const hs_csr* A, const hs_geometry* geom, int32_t leaf_size, hs_symbolic_t* S_out) {
    g_err.clear();
    if (!S_out || !A || !geom || !A->row_ptr || A->on_device) return fail(HS_ERR_ARG, "host CSR required");
    *S_out = nullptr;
    if (A->n <= 0 || leaf_size <= 0) return fail(HS_ERR_ARG, "bad size");
    int rc = validate_csr_host(A->n, A->nnz, A->row_ptr, A->col_idx);
    if (rc) return rc;
    std::unique_ptr<hs_symbolic_s> S(new hs_symbolic_s());
    if (geom->dim < 0 || geom->dim > 3) return fail(HS_ERR_GEOMETRY, "dim must be 0..3");
    const bool grid = geom->dim > 0;  // dim 0: partition the graph of A
    rc = build_symbolic(A->n, A->row_ptr, A->col_idx, grid ? geom->nx : 0, grid ? geom->ny : 0, grid ? geom->nz : 0,
                        leaf_size, S->sym);
    if (rc) return fail(rc, "symbolic analysis failed");
    *S_out = S.release();
    return HS_OK;
}

int hs_symbolic_levels(hs_symbolic_t S, int32_t* nlevels) {
    if (!S || !nlevels) return fail(HS_ERR_ARG, "null argument");
    *nlevels = S->sym.nlevels;
    return HS_OK;
}

int hs_symbolic_level(hs_symbolic_t S, int32_t level, int32_t* nclusters, int32_t* ncolors, int64_t* nadj,
                      int64_t* nfill, int64_t* npattern) {
    if (!S || level < 0 || level >= S->sym.nlevels) return fail(HS_ERR_ARG, "bad level");
    const auto& L = S->sym.levels[level];
    if (nclusters) *nclusters = L.ncl;
    if (ncolors) *ncolors = L.ncolors;
    if (nadj) *nadj = (int64_t)L.adj.size();
    if (nfill) *nfill = (int64_t)L.fill.size();
    if (npattern) *npattern = (int64_t)L.pat.size();
    return HS_OK;
}

int hs_symbolic_leaves(hs_symbolic_t S, int32_t* leaf_of_dof, int32_t* local_of_dof) {
    if (!S) return fail(HS_ERR_ARG, "null argument");
    if (leaf_of_dof) std::copy(S->sym.cluster_of.begin(), S->sym.cluster_of.end(), leaf_of_dof);
    if (local_of_dof) std::copy(S->sym.local_of.begin(), S->sym.local_of.end(), local_of_dof);
    return HS_OK;
}

int hs_symbolic_arrays(hs_symbolic_t S, int32_t level, int32_t* colors, int32_t* order, int32_t* adj_ptr, int32_t* adj,
                       int32_t* fill_ptr, int32_t* fill, int32_t* pat_ptr, int32_t* pat) {
    if (!S || level < 0 || level >= S->sym.nlevels) return fail(HS_ERR_ARG, "bad level");
    const auto& L = S->sym.levels[level];
    auto cp = [](const ivec& v, int32_t* o) {
        if (o) std::copy(v.begin(), v.end(), o);
    };
    cp(L.color, colors);
    cp(L.order, order);
    cp(L.adj_ptr, adj_ptr);
    cp(L.adj, adj);
    cp(L.fill_ptr, fill_ptr);
    cp(L.fill, fill);
    cp(L.pat_ptr, pat_ptr);
    cp(L.pat, pat);
    return HS_OK;
}

void hs_symbolic_free(hs_symbolic_t S) { delete S; }

int hs_set_allocator(void* (*alloc_fn)(size_t, void*, void*), void (*free_fn)(void*, void*, void*), void* ctx) {
    if ((alloc_fn == nullptr) != (free_fn == nullptr)) return fail(HS_ERR_ARG, "give both functions or neither");
    if (g_live_factors.load() != 0) return fail(HS_ERR_ARG, "factorizations still exist");
    g_alloc_fn = alloc_fn;
    g_free_fn = free_fn;
    g_alloc_ctx = ctx;
    return HS_OK;
}

int hs_profile_enable(int32_t enable) {
    g_prof_on = enable != 0;
    return HS_OK;
}

int hs_profile_select(const char* families) {
    if (!families || !*families) {
        g_prof_mask = 0xffffffffu;
        return HS_OK;
    }
    uint32_t mask = 0;
    std::string list(families);
    size_t p0 = 0;
    while (p0 <= list.size()) {
        size_t p1 = list.find(',', p0);
        if (p1 == std::string::npos) p1 = list.size();
        const std::string name = list.substr(p0, p1 - p0);
        int id = -1;
        for (int f = 0; f < PF_COUNT; ++f)
            if (name == g_prof[f].name) id = f;
        if (id < 0) return fail(HS_ERR_ARG, "unknown family " + name);
        mask |= 1u << id;
        p0 = p1 + 1;
    }
    g_prof_mask = mask;
    return HS_OK;
}

int hs_profile_reset(void) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto& f : g_prof) {
        f.launches = 0;
        f.seconds = f.bytes = f.flops = 0.0;
    }
    g_prof_pending.clear();
    return HS_OK;
}

int hs_profile_read(const char* family, int64_t* launches, double* seconds, double* bytes, double* flops) {
    if (!family) return fail(HS_ERR_ARG, "null family");
    prof_flush();  // intervals finished since the last synchronisation of the library
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto& f : g_prof)
        if (std::strcmp(f.name, family) == 0) {
            if (launches) *launches = f.launches;
            if (seconds) *seconds = f.seconds;
            if (bytes) *bytes = f.bytes;
            if (flops) *flops = f.flops;
            return HS_OK;
        }
    return fail(HS_ERR_ARG, std::string("unknown family ") + family);
}

const char* hs_last_error(void) { return g_err.c_str(); }

const char* hs_strerror(int code) {
    switch (code) {
        case HS_OK: return "ok";
        case HS_ERR_ARG: return "invalid argument";
        case HS_ERR_PATTERN: return "invalid CSR pattern";
        case HS_ERR_GEOMETRY: return "geometry does not match the matrix";
        case HS_ERR_BREAKDOWN: return "zero or non-finite pivot";
        case HS_ERR_NOMEM: return "out of device memory";
        case HS_ERR_HIP: return "HIP runtime error";
        case HS_ERR_UNSUPPORTED: return "unsupported size";
        case HS_ERR_NODEVICE: return "no gfx950 device";
        case HS_WARN_NOT_CONVERGED: return "not converged";
        default: return "unknown status";
    }
}

const char* hs_version(void) { return kVersion; }

int hs_config_set(const char* name, double value) {
    if (!name) return fail(HS_ERR_ARG, "null name");
    if (std::strcmp(name, "noalloc_scratch_max") == 0) {
        if (!(value >= 0 && value <= (double)NOALLOC_SCRATCH_BYTES) || value != std::floor(value))
            return fail(HS_ERR_ARG, "noalloc_scratch_max outside [0, " + std::to_string(NOALLOC_SCRATCH_BYTES) + "]");
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        g_noalloc_limit = (size_t)value;
        return HS_OK;
    }
    std::lock_guard<std::mutex> lk(g_config_mu);
    for (const ConfigEntry& e : config_table(g_config)) {
        if (std::strcmp(e.name, name) != 0) continue;
        if (!(value >= e.lo && value <= e.hi))
            return fail(HS_ERR_ARG, std::string(name) + " outside [" + std::to_string(e.lo) + ", " +
                                        std::to_string(e.hi) + "]");
        if (e.ival) {
            if (value != std::floor(value)) return fail(HS_ERR_ARG, std::string(name) + " takes an integer");
            *e.ival = (int)value;
        } else {
            *e.dval = value;
        }
        return HS_OK;
    }
    return fail(HS_ERR_ARG, std::string("unknown configuration parameter ") + name);
}

int hs_config_get(const char* name, double* value) {
    if (!name || !value) return fail(HS_ERR_ARG, "null argument");
    if (std::strcmp(name, "noalloc_scratch_max") == 0) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        *value = (double)g_noalloc_limit;
        return HS_OK;
    }
    std::lock_guard<std::mutex> lk(g_config_mu);
    for (const ConfigEntry& e : config_table(g_config))
        if (std::strcmp(e.name, name) == 0) {
            *value = e.ival ? (double)*e.ival : *e.dval;
            return HS_OK;
        }
    return fail(HS_ERR_ARG, std::string("unknown configuration parameter ") + name);
}

int hs_config_reset(void) {
    {
        std::lock_guard<std::mutex> lk(g_config_mu);
        g_config = Config();
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    g_noalloc_limit = NOALLOC_SCRATCH_BYTES;
    return HS_OK;
}

}  // extern "C"
