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
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
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

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t _e = (expr);                                                              \
        if (_e != hipSuccess)                                                                \
            return fail(HS_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e));    \
    } while (0)

// --------------------------------------------------------------- allocator

static void* (*g_alloc_fn)(size_t, void*) = nullptr;
static void (*g_free_fn)(void*, void*) = nullptr;
static void* g_alloc_ctx = nullptr;

static void* dev_alloc(size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (g_alloc_fn) return g_alloc_fn(bytes, g_alloc_ctx);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}
static void dev_free(void* p) {
    if (!p) return;
    if (g_free_fn)
        g_free_fn(p, g_alloc_ctx);
    else
        (void)hipFree(p);
}

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) {
        o.p = nullptr;
        o.bytes = 0;
    }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) {
            release();
            p = o.p;
            bytes = o.bytes;
            o.p = nullptr;
            o.bytes = 0;
        }
        return *this;
    }
    ~DevBuf() { release(); }
    void release() {
        dev_free(p);
        p = nullptr;
        bytes = 0;
    }
    bool alloc(size_t n) {
        release();
        p = dev_alloc(n);
        bytes = p ? n : 0;
        return p != nullptr;
    }
    bool ensure(size_t n) { return bytes >= n ? true : alloc(n); }
    template <class T>
    T* as() const {
        return static_cast<T*>(p);
    }
};

// Host blob of aligned arrays uploaded in one copy.
struct Blob {
    std::vector<char> data;
    template <class T>
    size_t add(const std::vector<T>& v) {
        size_t off = (data.size() + 255) & ~size_t(255);
        data.resize(off + v.size() * sizeof(T));
        if (!v.empty()) std::memcpy(data.data() + off, v.data(), v.size() * sizeof(T));
        return off;
    }
    size_t reserve(size_t bytes) {
        size_t off = (data.size() + 255) & ~size_t(255);
        data.resize(off + bytes);
        return off;
    }
};

// ---------------------------------------------------------------- tracing

struct ProfFamily {
    const char* name;
    int64_t launches = 0;
    double seconds = 0.0, bytes = 0.0, flops = 0.0;
};
enum ProfId {
    PF_GRAM = 0, PF_PIVOT, PF_FILL, PF_NBR, PF_SCHUR, PF_MERGE, PF_APPLY, PF_SPMV, PF_DENSE,
    // host wall time of the factorization: symbolic analysis, level planning,
    // metadata uploads, device allocations, per-level rank read-back
    PF_H_SYMBOLIC, PF_H_PLAN, PF_H_UPLOAD, PF_H_ALLOC, PF_H_SYNC, PF_COUNT
};
static ProfFamily g_prof[PF_COUNT] = {{"gram"}, {"pivot"}, {"fill"}, {"nbr"},   {"schur"},
                                      {"merge"}, {"apply"}, {"spmv"}, {"dense"},
                                      {"host_symbolic"}, {"host_plan"}, {"host_upload"}, {"host_alloc"}, {"host_sync"}};
static bool g_prof_on = false;
struct ProfPending {
    int fam;
    hipEvent_t a, b;
};
static std::vector<ProfPending> g_prof_pending;
static std::vector<hipEvent_t> g_prof_pool;

static hipEvent_t prof_event() {
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
        if (g_prof_on) {
            a = prof_event();
            (void)hipEventRecord(a, st);
        }
    }
    ~ProfScope() {
        if (g_prof_on && a) {
            hipEvent_t b = prof_event();
            (void)hipEventRecord(b, st);
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
        if (g_prof_on) {
            g_prof[fam].seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            g_prof[fam].launches += 1;
        }
    }
};

// Read back finished intervals (the caller has synchronised the stream).
static void prof_flush() {
    for (auto& p : g_prof_pending) {
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
    g_prof_pending.clear();
}

// ------------------------------------------------------------- level state

struct ColourHost {
    int first = 0, n = 0;                          // slice of the processing order
    size_t off_clist, off_nbr_pre, off_fill_pre, off_tile_pre, off_part_off;
    ColourDev dev;
    const int64_t* part_off = nullptr;             // [nbr_total] in units of f
    int64_t part_total = 0;                        // sum of f over the entries
};

struct LevelData {
    int ncl = 0;
    int nblk = 0;
    int f32 = 0;                                   // blocks and records stored in float (mixed form)
    int64_t npairs = 0;                            // sum over clusters of |n(s)|^2
    DevBuf pairs;                                  // block id of every neighbour pair (a_i, a_j) of s
    size_t esz() const { return f32 ? sizeof(float) : sizeof(double); }
    std::vector<int> m, k;                         // sizes at the start, ranks after
    std::vector<int64_t> blk_off;
    int64_t block_elems = 0;
    int64_t rec_elems = 0;
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
    std::vector<ColourHost> colours;
    std::vector<int64_t> seg;                      // [ncl+1] segment offsets
    int64_t nseg = 0;
    int64_t part_max = 0;                          // largest colour part buffer (units of f)
    std::vector<double> kept;                      // dense starting matrix (keep_levels)
};

}  // namespace hs

struct hs_factor_s {
    int64_t n = 0;
    hs_opts opts{};
    int symmetric = 1;
    hs::Symbolic sym;
    std::vector<hs::LevelData> levels;
    hs::DevBuf A_row, A_col, A_val;
    hs::DevBuf cluster_of, local_of;
    hs::DevBuf ws;
    // solve buffers
    int solve_nrhs = 0;
    hs::DevBuf vecs;                      // y, z, out of every level
    std::vector<int64_t> vec_off;         // per level base (units of doubles / nrhs)
    int64_t vec_total = 0;
    hs::DevBuf part;
    // Krylov buffers
    hs::DevBuf kry;
    int kry_nrhs = 0;
    int kry_restart = 0;
    hs_info info{};
};

struct hs_symbolic_s {
    hs::Symbolic sym;
};

namespace hs {

static const char* kVersion = "hs 0.1 (gfx950)";
// Mixed form: levels with at most this many unknowns keep float64 storage
// (default of hs_opts.coarse_fp64_dofs).
constexpr int64_t MIXED_FP64_DOFS = 16384;

// =============================================================== validation

static int validate_csr_host(int64_t n, int64_t nnz, const int64_t* rp, const int32_t* ci) {
    if (rp[0] != 0 || rp[n] != nnz) return fail(HS_ERR_PATTERN, "row_ptr[0] must be 0 and row_ptr[n] = nnz");
    for (int64_t i = 0; i < n; ++i) {
        if (rp[i + 1] < rp[i]) return fail(HS_ERR_PATTERN, "row_ptr not non-decreasing");
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            if (ci[e] < 0 || ci[e] >= n) return fail(HS_ERR_PATTERN, "column index out of range");
            if (e > rp[i] && ci[e] <= ci[e - 1]) return fail(HS_ERR_PATTERN, "column indices not sorted / unique");
        }
    }
    return HS_OK;
}

// ================================================================ planning

// Plan one level: block offsets, per-cluster lists, colours, records and
// workspace.  Builds the metadata blob (uploaded by the caller).
static int plan_level(hs_factor_s* F, int lvl, Blob& blob, std::vector<size_t>& offs) {
    LevelData& LD = F->levels[lvl];
    const LevelSymbolic& S = F->sym.levels[lvl];
    const int ncl = S.ncl;
    const std::vector<int>& m = LD.m;
    LD.ncl = ncl;
    LD.nblk = (int)S.pat.size();
    LD.max_m = 0;
    for (int c = 0; c < ncl; ++c) LD.max_m = std::max(LD.max_m, m[c]);
    if (LD.max_m > MAX_M)
        return fail(HS_ERR_UNSUPPORTED, "cluster of size " + std::to_string(LD.max_m) + " at level " +
                                            std::to_string(lvl) + " exceeds the supported " + std::to_string(MAX_M));
    // blocks (capacity m_a x m_b, column major, ld m_a)
    LD.blk_off.resize(LD.nblk);
    int64_t off = 0;
    for (int a = 0; a < ncl; ++a)
        for (int e = S.pat_ptr[a]; e < S.pat_ptr[a + 1]; ++e) {
            LD.blk_off[e] = off;
            off += (int64_t)m[a] * m[S.pat[e]];
        }
    LD.block_elems = off;

    // per-cluster lists
    std::vector<int> diag_blk(ncl), nbr_before, nbr_bsa, nbr_bas, ncap(ncl), fill_before, fill_bst, fill_bts;
    std::vector<int64_t> pair_base(ncl), rec_off(ncl), ws_off(ncl, 0);
    nbr_before.resize(S.adj.size());
    nbr_bsa.resize(S.adj.size());
    nbr_bas.resize(S.adj.size());
    fill_before.resize(S.fill.size());
    fill_bst.resize(S.fill.size());
    fill_bts.resize(S.fill.size());
    // (the block ids of all neighbour pairs, sum of |n(s)|^2 entries, are
    // found on the device: launch_pair_blocks)
    auto bid = [&](int a, int b) { return S.block_id(a, b); };
    int64_t pp = 0, roff = 0;
    int max_nf = 0;
    for (int s = 0; s < ncl; ++s) {
        diag_blk[s] = bid(s, s);
        int cap = 0;
        for (int e = S.adj_ptr[s]; e < S.adj_ptr[s + 1]; ++e) {
            int a = S.adj[e];
            nbr_before[e] = S.pos[a] < S.pos[s];
            nbr_bsa[e] = bid(s, a);
            nbr_bas[e] = bid(a, s);
            cap += m[a];
        }
        ncap[s] = cap;
        for (int e = S.fill_ptr[s]; e < S.fill_ptr[s + 1]; ++e) {
            int t = S.fill[e];
            fill_before[e] = S.pos[t] < S.pos[s];
            fill_bst[e] = bid(s, t);
            fill_bts[e] = bid(t, s);
        }
        max_nf = std::max(max_nf, S.fill_ptr[s + 1] - S.fill_ptr[s]);
        pair_base[s] = pp;
        const int64_t nb = S.adj_ptr[s + 1] - S.adj_ptr[s];
        pp += nb * nb;
        rec_off[s] = roff;
        roff += 2 * (int64_t)m[s] * m[s] + 2 * (int64_t)m[s] * cap;
    }
    LD.rec_elems = roff;
    LD.npairs = pp;
    // about four fill partners per Gram workgroup
    LD.gram_splits = std::min(64, std::max(1, (max_nf + 3) / 4));
    const int64_t slots = ws_slots(LD.gram_splits);

    // colours
    LD.colours.assign(S.ncolors, ColourHost());
    std::vector<std::vector<int>> c_nbr_pre(S.ncolors), c_fill_pre(S.ncolors);
    std::vector<std::vector<int64_t>> c_tile_pre(S.ncolors);
    int64_t ws_max = 0;
    for (int c = 0; c < S.ncolors; ++c) {
        ColourHost& CH = LD.colours[c];
        CH.first = S.color_ptr[c];
        CH.n = S.color_ptr[c + 1] - S.color_ptr[c];
        auto& np = c_nbr_pre[c];
        auto& fp = c_fill_pre[c];
        auto& tp = c_tile_pre[c];
        np.assign(CH.n + 1, 0);
        fp.assign(CH.n + 1, 0);
        tp.assign(CH.n + 1, 0);
        int max_m = 0, max_nm = 0;
        int64_t wso = 0;
        for (int i = 0; i < CH.n; ++i) {
            int s = S.order[CH.first + i];
            np[i + 1] = np[i] + (S.adj_ptr[s + 1] - S.adj_ptr[s]);
            fp[i + 1] = fp[i] + (S.fill_ptr[s + 1] - S.fill_ptr[s]);
            int64_t tpr = (ncap[s] + SCHUR_T - 1) / SCHUR_T;
            tp[i + 1] = tp[i] + (m[s] > 0 ? tpr * tpr : 0);
            max_m = std::max(max_m, m[s]);
            for (int e = S.adj_ptr[s]; e < S.adj_ptr[s + 1]; ++e) max_nm = std::max(max_nm, m[S.adj[e]]);
            for (int e = S.fill_ptr[s]; e < S.fill_ptr[s + 1]; ++e) max_nm = std::max(max_nm, m[S.fill[e]]);
            ws_off[s] = wso;
            wso += slots * (int64_t)m[s] * m[s];
        }
        ws_max = std::max(ws_max, wso);
        CH.dev.n = CH.n;
        CH.dev.nbr_total = np[CH.n];
        CH.dev.fill_total = fp[CH.n];
        CH.dev.tile_total = tp[CH.n];
        CH.dev.max_m = max_m;
        CH.dev.max_nbr_m = max_nm;
        const int pw = panel_width(max_m);
        CH.dev.panels = (max_nm + pw - 1) / pw;
    }
    LD.ws_elems = ws_max;

    // blob layout
    std::vector<int> order(S.order);
    offs.clear();
    offs.push_back(blob.add(m));                 // 0 m
    offs.push_back(blob.add(m));                 // 1 k (initialised to m)
    offs.push_back(blob.add(std::vector<int>(ncl, 0)));  // 2 flag
    offs.push_back(blob.add(LD.blk_off));        // 3
    offs.push_back(blob.add(diag_blk));          // 4
    offs.push_back(blob.add(S.adj_ptr));         // 5
    offs.push_back(blob.add(S.adj));             // 6
    offs.push_back(blob.add(nbr_before));        // 7
    offs.push_back(blob.add(nbr_bsa));           // 8
    offs.push_back(blob.add(nbr_bas));           // 9
    offs.push_back(blob.add(std::vector<int>(S.adj.size(), 0)));  // 10 nbr_noff
    offs.push_back(blob.add(std::vector<int>(ncl, 0)));           // 11 ntot
    offs.push_back(blob.add(ncap));              // 12
    offs.push_back(blob.add(S.fill_ptr));        // 13
    offs.push_back(blob.add(S.fill));            // 14
    offs.push_back(blob.add(fill_before));       // 15
    offs.push_back(blob.add(fill_bst));          // 16
    offs.push_back(blob.add(fill_bts));          // 17
    offs.push_back(blob.add(pair_base));         // 18
    offs.push_back(blob.add(std::vector<int>()));  // 19 (pair block ids: LD.pairs)
    offs.push_back(blob.add(rec_off));           // 20
    offs.push_back(blob.add(ws_off));            // 21
    offs.push_back(blob.add(S.pat_ptr));         // 22
    offs.push_back(blob.add(S.pat));             // 23
    offs.push_back(blob.add(order));             // 24 processing order (colour lists are slices)
    for (int c = 0; c < S.ncolors; ++c) {
        ColourHost& CH = LD.colours[c];
        CH.off_nbr_pre = blob.add(c_nbr_pre[c]);
        CH.off_fill_pre = blob.add(c_fill_pre[c]);
        CH.off_tile_pre = blob.add(c_tile_pre[c]);
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
    D.gram_splits = LD.gram_splits;
    D.m = (const int*)P(0);
    D.k = (int*)P(1);
    D.flag = (int*)P(2);
    D.blk_off = (const int64_t*)P(3);
    D.blocks = LD.blocks.as<double>();
    D.f32 = LD.f32;
    D.diag_blk = (const int*)P(4);
    D.nbr_ptr = (const int*)P(5);
    D.nbr_id = (const int*)P(6);
    D.nbr_before = (const int*)P(7);
    D.nbr_bsa = (const int*)P(8);
    D.nbr_bas = (const int*)P(9);
    D.nbr_noff = (int*)P(10);
    D.ntot = (int*)P(11);
    D.ncap = (const int*)P(12);
    D.fill_ptr = (const int*)P(13);
    D.fill_id = (const int*)P(14);
    D.fill_before = (const int*)P(15);
    D.fill_bst = (const int*)P(16);
    D.fill_bts = (const int*)P(17);
    D.pair_base = (const int64_t*)P(18);
    D.pair_blk = LD.pairs.as<int>();
    D.rec_off = (const int64_t*)P(20);
    D.rec = LD.rec.as<double>();
    D.ws_off = (const int64_t*)P(21);
    D.ws = F->ws.as<double>();
    LD.dev_pat_ptr = (const int*)P(22);
    LD.dev_pat = (const int*)P(23);
    const int* order = (const int*)P(24);
    for (auto& CH : LD.colours) {
        CH.dev.clist = order + CH.first;
        CH.dev.nbr_pre = (const int*)(base + CH.off_nbr_pre);
        CH.dev.fill_pre = (const int*)(base + CH.off_fill_pre);
        CH.dev.tile_pre = (const int64_t*)(base + CH.off_tile_pre);
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
    SD.f32 = LD.f32;
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
    std::vector<double> blk(LD.block_elems);
    if (LD.block_elems) {
        if (LD.f32) {
            std::vector<float> bf(LD.block_elems);
            HIP_TRY(hipMemcpyAsync(bf.data(), LD.blocks.p, LD.block_elems * sizeof(float), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            for (int64_t i = 0; i < LD.block_elems; ++i) blk[i] = bf[i];
        } else {
            HIP_TRY(hipMemcpyAsync(blk.data(), LD.blocks.p, LD.block_elems * sizeof(double), hipMemcpyDeviceToHost,
                                   st));
        }
    }
    HIP_TRY(hipStreamSynchronize(st));
    std::vector<int64_t> off(LD.ncl + 1, 0);
    for (int c = 0; c < LD.ncl; ++c) off[c + 1] = off[c] + LD.m[c];
    const int64_t dim = off[LD.ncl];
    LD.kept.assign((size_t)(dim * dim), 0.0);
    for (int a = 0; a < LD.ncl; ++a)
        for (int e = S.pat_ptr[a]; e < S.pat_ptr[a + 1]; ++e) {
            const int b = S.pat[e];
            for (int j = 0; j < LD.m[b]; ++j)
                for (int i = 0; i < LD.m[a]; ++i)
                    LD.kept[(off[a] + i) + (off[b] + j) * dim] = blk[LD.blk_off[e] + i + (int64_t)j * LD.m[a]];
        }
    return HS_OK;
}

// Dense factorization of a complete level; ranks become 0 and the solve
// metadata (packed neighbour offsets, n_tot) is written for every cluster.
static int factor_dense_level(hs_factor_s* F, int lvl, hipStream_t st) {
    LevelData& LD = F->levels[lvl];
    const LevelSymbolic& S = F->sym.levels[lvl];
    std::vector<int64_t> off(LD.ncl + 1, 0);
    for (int c = 0; c < LD.ncl; ++c) off[c + 1] = off[c] + LD.m[c];
    const int64_t N = off[LD.ncl];
    // packed offsets: neighbours before s are eliminated (size 0)
    std::vector<int> noff(S.adj.size()), ntot(LD.ncl), zeros(LD.ncl, 0);
    for (int s = 0; s < LD.ncl; ++s) {
        int acc = 0;
        for (int e = S.adj_ptr[s]; e < S.adj_ptr[s + 1]; ++e) {
            noff[e] = acc;
            const int a = S.adj[e];
            acc += a < s ? 0 : LD.m[a];
        }
        ntot[s] = acc;
    }
    HIP_TRY(hipMemcpyAsync(LD.dev.nbr_noff, noff.data(), noff.size() * sizeof(int), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(LD.dev.ntot, ntot.data(), ntot.size() * sizeof(int), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(LD.dev.k, zeros.data(), zeros.size() * sizeof(int), hipMemcpyHostToDevice, st));
    if (N == 0) return HS_OK;
    Blob b;
    const size_t o_off = b.add(off);
    DevBuf aux, dense;
    if (!aux.alloc(b.data.size() + (2 * 128 * 128 + 64) * sizeof(double))) return fail(HS_ERR_NOMEM, "dense level");
    if (!dense.alloc((size_t)N * N * sizeof(double))) return fail(HS_ERR_NOMEM, "dense level matrix");
    HIP_TRY(hipMemcpyAsync(aux.p, b.data.data(), b.data.size(), hipMemcpyHostToDevice, st));
    char* base = aux.as<char>();
    const size_t o_inv = (b.data.size() + 255) & ~size_t(255);
    double* inv = (double*)(base + o_inv);
    int* flag = (int*)(inv + 2 * 128 * 128);
    HIP_TRY(hipMemsetAsync(flag, 0, sizeof(int), st));
    int rc;
    {
        ProfScope ps(PF_DENSE, st);
        rc = dense_level_factor(dense.as<double>(), N, LD.dev_pat_ptr, LD.dev_pat, LD.dev.m,
                                (const int64_t*)(base + o_off), LD.dev.blk_off, LD.dev.blocks, LD.ncl, LD.nblk, inv,
                                flag, LD.dev.ncap, LD.dev.rec_off, LD.dev.rec, LD.m, off, st);
    }
    if (rc) return fail(HS_ERR_HIP, "dense level launch failed");
    int hflag = 0;
    HIP_TRY(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (hflag) {
        F->info.breakdown_level = lvl;
        F->info.breakdown_cluster = -1;
        return fail(HS_ERR_BREAKDOWN, "zero or non-finite pivot at level " + std::to_string(lvl) + " (dense level)");
    }
    return HS_OK;
}

static int factor_impl(hs_factor_s* F, const hs_csr* A, const hs_geometry* G, hipStream_t st) {
    using clock = std::chrono::steady_clock;
    const int64_t n = A->n, nnz = A->nnz;
    // ---- host copy of the pattern (the symbolic analysis needs it), device copy of A
    std::vector<int64_t> rp_h;
    std::vector<int32_t> ci_h;
    std::vector<double> v_h;
    const int64_t* rp;
    const int32_t* ci;
    if (A->on_device) {
        rp_h.resize(n + 1);
        ci_h.resize(nnz);
        HIP_TRY(hipMemcpyAsync(rp_h.data(), A->row_ptr, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, st));
        if (nnz) HIP_TRY(hipMemcpyAsync(ci_h.data(), A->col_idx, nnz * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        rp = rp_h.data();
        ci = ci_h.data();
    } else {
        rp = A->row_ptr;
        ci = A->col_idx;
    }
    int rc = validate_csr_host(n, nnz, rp, ci);
    if (rc) return rc;
    if (!F->A_row.alloc((n + 1) * sizeof(int64_t)) || !F->A_col.alloc(nnz * sizeof(int32_t) + 4) ||
        !F->A_val.alloc(nnz * sizeof(double) + 8))
        return fail(HS_ERR_NOMEM, "device copy of A");
    const hipMemcpyKind kind = A->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIP_TRY(hipMemcpyAsync(F->A_row.p, A->row_ptr, (n + 1) * sizeof(int64_t), kind, st));
    if (nnz) {
        HIP_TRY(hipMemcpyAsync(F->A_col.p, A->col_idx, nnz * sizeof(int32_t), kind, st));
        HIP_TRY(hipMemcpyAsync(F->A_val.p, A->val, nnz * sizeof(double), kind, st));
    }
    if (F->opts.symmetric < 0) {
        v_h.resize(nnz);
        if (nnz) HIP_TRY(hipMemcpyAsync(v_h.data(), A->val, nnz * sizeof(double),
                                        A->on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        int sym = 1;
        for (int64_t i = 0; i < n && sym; ++i)
            for (int64_t e = rp[i]; e < rp[i + 1] && sym; ++e) {
                const int64_t j = ci[e];
                const int32_t* lo = ci + rp[j];
                const int32_t* hi = ci + rp[j + 1];
                const int32_t* it = std::lower_bound(lo, hi, (int32_t)i);
                if (it == hi || *it != i || v_h[it - ci] != v_h[e]) sym = 0;
            }
        F->symmetric = sym;
    } else {
        F->symmetric = F->opts.symmetric ? 1 : 0;
    }

    // ---- symbolic analysis (integer work only)
    auto t0 = clock::now();
    {
        HostScope hs_(PF_H_SYMBOLIC);
        rc = build_symbolic(n, rp, ci, G->nx, G->ny, G->nz, F->opts.leaf_size, F->sym);
    }
    if (rc) return fail(rc, rc == HS_ERR_GEOMETRY ? "n != nx*ny*nz" : "bad symbolic arguments");
    auto t1 = clock::now();
    F->info.symbolic_seconds = std::chrono::duration<double>(t1 - t0).count();
    const int nlev = F->sym.nlevels;
    if (nlev > 64) return fail(HS_ERR_UNSUPPORTED, "more than 64 levels");
    F->levels.clear();
    F->levels.resize(nlev);
    if (!F->cluster_of.alloc(n * sizeof(int)) || !F->local_of.alloc(n * sizeof(int)))
        return fail(HS_ERR_NOMEM, "dof maps");
    HIP_TRY(hipMemcpyAsync(F->cluster_of.p, F->sym.cluster_of.data(), n * sizeof(int), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(F->local_of.p, F->sym.local_of.data(), n * sizeof(int), hipMemcpyHostToDevice, st));

    // ---- numeric factorization, level by level (Alg. 1)
    LevelData* prev = nullptr;
    std::vector<size_t> offs;
    double flops = 0.0;
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
        Blob blob;
        {
            HostScope hs_(PF_H_PLAN);
            rc = plan_level(F, lvl, blob, offs);
        }
        if (rc) return rc;
        // A level whose clusters all neighbour each other has no fill: it is
        // factored densely (Alg. 1, conventional factorization).
        bool complete = true;
        for (int c = 0; c < S.ncl && complete; ++c)
            if (S.adj_ptr[c + 1] - S.adj_ptr[c] != S.ncl - 1 || S.order[c] != c) complete = false;
        // mixed form: float storage except on the coarse levels
        int64_t level_dofs = 0;
        for (int c = 0; c < S.ncl; ++c) level_dofs += LD.m[c];
        const int64_t fp64_dofs = F->opts.coarse_fp64_dofs > 0 ? F->opts.coarse_fp64_dofs : MIXED_FP64_DOFS;
        LD.f32 = (F->opts.precision == HS_MIXED && !complete && level_dofs > fp64_dofs) ? 1 : 0;
        {
            HostScope hs_(PF_H_ALLOC);
            if (!LD.meta.alloc(blob.data.size())) return fail(HS_ERR_NOMEM, "level metadata");
            if (!LD.blocks.alloc(LD.block_elems * LD.esz())) return fail(HS_ERR_NOMEM, "block store");
            if (!LD.rec.alloc(LD.rec_elems * LD.esz())) return fail(HS_ERR_NOMEM, "factor records");
            if (!F->ws.ensure(LD.ws_elems * sizeof(double))) return fail(HS_ERR_NOMEM, "workspace");
            if (!LD.pairs.alloc((LD.npairs + 1) * sizeof(int))) return fail(HS_ERR_NOMEM, "neighbour pairs");
        }
        {
            HostScope hs_(PF_H_UPLOAD);
            HIP_TRY(hipMemcpyAsync(LD.meta.p, blob.data.data(), blob.data.size(), hipMemcpyHostToDevice, st));
        }
        bind_level(LD, offs, F);
        launch_pair_blocks(S.ncl, LD.dev.nbr_ptr, LD.dev.nbr_id, LD.dev_pat_ptr, LD.dev_pat, LD.dev.pair_base,
                           LD.pairs.as<int>(), st);
        launch_fill_zero(LD.blocks.p, LD.block_elems, LD.f32, st);
        if (lvl == 0) {
            launch_assemble0(n, F->A_row.as<int64_t>(), F->A_col.as<int32_t>(), F->A_val.as<double>(),
                             F->cluster_of.as<int>(), F->local_of.as<int>(), LD.dev.m, (const int*)(LD.meta.as<char>() + offs[22]),
                             (const int*)(LD.meta.as<char>() + offs[23]), LD.dev.blk_off, LD.dev.blocks, LD.f32, st);
        } else {
            // parent blocks from the children's coarse blocks
            const LevelSymbolic& PS = F->sym.levels[lvl - 1];
            HostScope hs_(PF_H_PLAN);
            std::vector<int> nb_row(LD.nblk), nb_col(LD.nblk), src4(4 * (size_t)LD.nblk);
            for (int P = 0; P < S.ncl; ++P)
                for (int e = S.pat_ptr[P]; e < S.pat_ptr[P + 1]; ++e) {
                    const int Q = S.pat[e];
                    nb_row[e] = P;
                    nb_col[e] = Q;
                    for (int h = 0; h < 4; ++h) {
                        const int a = 2 * P + (h >> 1), c = 2 * Q + (h & 1);
                        src4[4 * (size_t)e + h] = (a < PS.ncl && c < PS.ncl) ? PS.block_id(a, c) : -1;
                    }
                }
            Blob mb;
            size_t o_r = mb.add(nb_row), o_c = mb.add(nb_col), o_s = mb.add(src4);
            DevBuf mbuf;
            if (!mbuf.alloc(mb.data.size())) return fail(HS_ERR_NOMEM, "merge metadata");
            HIP_TRY(hipMemcpyAsync(mbuf.p, mb.data.data(), mb.data.size(), hipMemcpyHostToDevice, st));
            {
                ProfScope ps(PF_MERGE, st);
                launch_merge(LD.nblk, (const int*)(mbuf.as<char>() + o_r), (const int*)(mbuf.as<char>() + o_c),
                             (const int*)(mbuf.as<char>() + o_s), prev->dev.k, prev->dev.m, prev->dev.blk_off,
                             prev->dev.blocks, prev->f32, LD.dev.m, LD.dev.blk_off, LD.dev.blocks, LD.f32, prev->ncl,
                             st);
            }
            HIP_TRY(hipStreamSynchronize(st));  // merge metadata and the children's blocks are freed below
            prev->blocks.release();
            prev->dev.blocks = nullptr;
        }
        if (F->opts.keep_levels) {
            rc = keep_level_matrix(F, LD, st);
            if (rc) return rc;
        }
        if (complete) {
            rc = factor_dense_level(F, lvl, st);
            if (rc) return rc;
        }
        for (auto& CH : LD.colours) {
            if (complete) break;
            if (F->opts.eps > 0.0 && CH.dev.fill_total > 0) {
                ProfScope ps(PF_GRAM, st);
                launch_gram(LD.dev, CH.dev, st);
            }
            {
                ProfScope ps(PF_PIVOT, st);
                launch_pivot(LD.dev, CH.dev, st);
            }
            if (CH.dev.fill_total > 0) {
                ProfScope ps(PF_FILL, st);
                launch_fill_update(LD.dev, CH.dev, st);
            }
            if (CH.dev.nbr_total > 0) {
                ProfScope ps(PF_NBR, st);
                launch_nbr_update(LD.dev, CH.dev, st);
            }
            if (CH.dev.tile_total > 0) {
                ProfScope ps(PF_SCHUR, st);
                launch_schur(LD.dev, CH.dev, st);
            }
        }
        HIP_TRY(hipGetLastError());
        // ranks decide the next level's sizes: one synchronisation per level
        LD.k.resize(LD.ncl);
        std::vector<int> flag(LD.ncl), ntot(LD.ncl);
        {
            HostScope hs_(PF_H_SYNC);
            HIP_TRY(hipMemcpyAsync(LD.k.data(), LD.dev.k, LD.ncl * sizeof(int), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipMemcpyAsync(flag.data(), LD.dev.flag, LD.ncl * sizeof(int), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipMemcpyAsync(ntot.data(), LD.dev.ntot, LD.ncl * sizeof(int), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
        }
        LD.pairs.release();  // used by this level's Schur updates only
        LD.dev.pair_blk = nullptr;
        for (int c = 0; c < LD.ncl; ++c)
            if (flag[c]) {
                F->info.breakdown_level = lvl;
                F->info.breakdown_cluster = c;
                return fail(HS_ERR_BREAKDOWN, "zero or non-finite pivot at level " + std::to_string(lvl) +
                                                  ", cluster " + std::to_string(c) +
                                                  (flag[c] == 2 ? " (fine block)" : " (pivot block)"));
            }
        if (g_prof_on) {
            prof_flush();
            for (int c = 0; c < LD.ncl; ++c) {
                const double f = LD.m[c] - LD.k[c], nt = ntot[c];
                if (LD.m[c] == 0 || f == 0 || nt == 0) continue;
                g_prof[PF_SCHUR].flops += 2.0 * f * nt * nt;
                g_prof[PF_SCHUR].bytes += (double)LD.esz() * (2.0 * f * nt + 2.0 * nt * nt);
            }
        }
        for (int c = 0; c < LD.ncl; ++c) {
            int wt = 0;
            for (int e = S.fill_ptr[c]; e < S.fill_ptr[c + 1]; ++e) {
                const int t = S.fill[e];
                wt += S.pos[t] < S.pos[c] ? LD.k[t] : LD.m[t];
            }
            flops += cluster_flops(LD.m[c], LD.k[c], ntot[c], wt, F->symmetric != 0);
        }
        // solve plan of the level: segments and part offsets
        LD.seg.assign(LD.ncl + 1, 0);
        for (int c = 0; c < LD.ncl; ++c) LD.seg[c + 1] = LD.seg[c] + LD.m[c];
        LD.nseg = LD.seg[LD.ncl];
        int64_t coarse = 0;
        for (int c = 0; c < LD.ncl; ++c) coarse += LD.k[c];
        F->info.coarse_dofs[lvl] = coarse;
        F->info.level_clusters[lvl] = LD.ncl;
        F->info.level_colors[lvl] = S.ncolors;
        F->info.ncolors_total += S.ncolors;
        F->info.max_cluster = std::max(F->info.max_cluster, LD.max_m);
        prev = &LD;
    }
    // the last level's blocks are no longer needed
    if (prev) {
        prev->blocks.release();
        prev->dev.blocks = nullptr;
    }
    F->ws.release();

    // ---- solve plan (needs every rank): segments, part offsets per colour
    double rec_bytes = 0.0, apply_flops = 0.0;
    for (int lvl = 0; lvl < nlev; ++lvl) {
        LevelData& LD = F->levels[lvl];
        const LevelSymbolic& S = F->sym.levels[lvl];
        Blob sb;
        size_t o_seg = sb.add(LD.seg);
        std::vector<size_t> o_part(LD.colours.size());
        LD.part_max = 0;
        for (size_t c = 0; c < LD.colours.size(); ++c) {
            ColourHost& CH = LD.colours[c];
            std::vector<int64_t> po;
            int64_t acc = 0;
            for (int i = 0; i < CH.n; ++i) {
                const int s = S.order[CH.first + i];
                const int f = LD.m[s] - LD.k[s];
                for (int e = S.adj_ptr[s]; e < S.adj_ptr[s + 1]; ++e) {
                    po.push_back(acc);
                    acc += f;
                }
            }
            po.push_back(acc);
            CH.part_total = acc;
            LD.part_max = std::max(LD.part_max, acc);
            o_part[c] = sb.add(po);
        }
        // keep the solve metadata next to the level metadata
        DevBuf buf;
        if (!buf.alloc(sb.data.size())) return fail(HS_ERR_NOMEM, "solve metadata");
        HIP_TRY(hipMemcpyAsync(buf.p, sb.data.data(), sb.data.size(), hipMemcpyHostToDevice, st));
        LD.sdev.seg = (const int64_t*)(buf.as<char>() + o_seg);
        for (size_t c = 0; c < LD.colours.size(); ++c)
            LD.colours[c].part_off = (const int64_t*)(buf.as<char>() + o_part[c]);
        LD.blocks = std::move(buf);  // the block store slot now owns the solve metadata
        for (int c = 0; c < LD.ncl; ++c) {
            const double m = LD.m[c], k = LD.k[c], f = m - k;
            if (LD.m[c] == 0 || LD.k[c] == LD.m[c]) continue;
            int nt = 0;
            for (int e = S.adj_ptr[c]; e < S.adj_ptr[c + 1]; ++e) {
                const int a = S.adj[e];
                nt += S.pos[a] < S.pos[c] ? LD.k[a] : LD.m[a];
            }
            rec_bytes += (double)LD.esz() * (2.0 * m * m + 2.0 * f * nt);
            apply_flops += 4.0 * m * m + 4.0 * f * nt;
        }
    }
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
    const int nlev = (int)F->levels.size();
    F->vec_off.assign(nlev + 1, 0);
    for (int l = 0; l < nlev; ++l) F->vec_off[l + 1] = F->vec_off[l] + 3 * F->levels[l].nseg;
    F->vec_total = F->vec_off[nlev];
    int64_t pm = 0;
    for (auto& LD : F->levels) pm = std::max(pm, LD.part_max);
    if (!F->vecs.alloc((F->vec_total * nrhs + 1) * sizeof(double))) return fail(HS_ERR_NOMEM, "solve vectors");
    if (!F->part.alloc((pm * nrhs + 1) * sizeof(double))) return fail(HS_ERR_NOMEM, "solve partials");
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

static int solve_chunk(hs_factor_s* F, int nrhs, const double* B, int64_t ldb, double* X, int64_t ldx, hipStream_t st) {
    int rc = ensure_solve_buffers(F, nrhs);
    if (rc) return rc;
    const int nlev = (int)F->levels.size();
    double* base = F->vecs.as<double>();
    auto Y = [&](int l) { return base + F->vec_off[l] * nrhs; };
    auto Z = [&](int l) { return base + (F->vec_off[l] + F->levels[l].nseg) * nrhs; };
    auto O = [&](int l) { return base + (F->vec_off[l] + 2 * F->levels[l].nseg) * nrhs; };
    double* part = F->part.as<double>();
    LevelData& L0 = F->levels[0];
    launch_scatter_rhs(F->n, F->cluster_of.as<int>(), F->local_of.as<int>(), L0.sdev.seg, L0.dev.m, B, ldb, Y(0), nrhs,
                       st);
    for (int l = 0; l < nlev; ++l) {
        LevelData& LD = F->levels[l];
        for (auto& CH : LD.colours) {
            ProfScope ps(PF_APPLY, st);
            launch_apply_fwd_t(LD.sdev, CH.dev, Y(l), Z(l), nrhs, st);
            launch_apply_fwd_u(LD.sdev, CH.dev, Y(l), Z(l), nrhs, CH.dev.max_nbr_m, st);
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
            ProfScope ps(PF_APPLY, st);
            launch_apply_bwd_acc(LD.sdev, CH.dev, Z(l), O(l), part, CH.part_off, nrhs, st);
            launch_apply_bwd_t(LD.sdev, CH.dev, Z(l), O(l), part, CH.part_off, nrhs, st);
        }
    }
    launch_gather_sol(F->n, F->cluster_of.as<int>(), F->local_of.as<int>(), L0.sdev.seg, L0.dev.m, O(0), X, ldx, nrhs,
                      st);
    HIP_TRY(hipGetLastError());
    return HS_OK;
}

// ================================================================ Krylov

// Work vectors: R, Zv, P, Q (n x nrhs each), scalars.
static int ensure_krylov(hs_factor_s* F, int nrhs, int restart) {
    const int64_t n = F->n;
    const int64_t vecs = 4 + (restart > 0 ? restart + 1 : 0);
    const size_t bytes = (size_t)(vecs * n * nrhs + 8 * nrhs + nrhs * KRYLOV_BLOCKS + 64 * (restart + 2)) * sizeof(double);
    if (F->kry.bytes >= bytes) return HS_OK;
    if (!F->kry.alloc(bytes)) return fail(HS_ERR_NOMEM, "Krylov workspace");
    return HS_OK;
}

static int dots_host(hs_factor_s* F, int64_t n, const double* a, int64_t lda, const double* b, int64_t ldb, int nrhs,
                     double* part, double* dout, double* hout, hipStream_t st) {
    launch_dots(n, a, lda, b, ldb, nrhs, part, dout, st);
    HIP_TRY(hipMemcpyAsync(hout, dout, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (g_prof_on) prof_flush();
    (void)F;
    return HS_OK;
}

static int pcg_impl(hs_factor_s* F, int nrhs, const double* B, int64_t ldb, double* X, int64_t ldx, double tol,
                    int maxit, int* iters, double* relres, hipStream_t st) {
    int rc = ensure_krylov(F, nrhs, 0);
    if (rc) return rc;
    const int64_t n = F->n;
    double* w = F->kry.as<double>();
    double* R = w;
    double* Zv = R + n * nrhs;
    double* P = Zv + n * nrhs;
    double* Q = P + n * nrhs;
    double* sc = Q + n * nrhs;             // 8 * nrhs scalars
    double* part = sc + 8 * nrhs;
    double* d_alpha = sc;
    double* d_beta = sc + nrhs;
    double* d_one = sc + 2 * nrhs;
    double* d_mone = sc + 3 * nrhs;
    double* d_zero = sc + 4 * nrhs;
    double* d_dot = sc + 5 * nrhs;
    std::vector<double> one(nrhs, 1.0), mone(nrhs, -1.0), zero(nrhs, 0.0);
    HIP_TRY(hipMemcpyAsync(d_one, one.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(d_mone, mone.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(d_zero, zero.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, st));
    std::vector<double> bn(nrhs), rz(nrhs), rzn(nrhs), rzo(nrhs, 0.0), pq(nrhs), rr(nrhs), alpha(nrhs), beta(nrhs);
    // A float32 factor is a slightly nonlinear preconditioner: the flexible
    // (Polak-Ribiere) beta = r_new^T (z_new - z_old) / r_old^T z_old keeps CG
    // converging; with a float64 factor the classical beta is used.
    const bool flexible = F->opts.precision == HS_MIXED;
    rc = dots_host(F, n, B, ldb, B, ldb, nrhs, part, d_dot, bn.data(), st);
    if (rc) return rc;
    for (auto& v : bn) v = v > 0 ? std::sqrt(v) : 1.0;
    // x0 = 0, r0 = b
    launch_axpby(n, d_zero, B, ldb, d_zero, X, ldx, nrhs, st);
    launch_copy(n, B, ldb, R, n, nrhs, st);
    std::vector<char> active(nrhs, 1);
    int nact = nrhs;
    rc = solve_impl(F, nrhs, R, n, Zv, n, st);
    if (rc) return rc;
    launch_copy(n, Zv, n, P, n, nrhs, st);
    rc = dots_host(F, n, R, n, Zv, n, nrhs, part, d_dot, rz.data(), st);
    if (rc) return rc;
    int it = 0;
    while (nact > 0 && it < maxit) {
        ++it;
        launch_spmv(n, F->A_row.as<int64_t>(), F->A_col.as<int32_t>(), F->A_val.as<double>(), P, n, Q, n, nrhs, st);
        rc = dots_host(F, n, P, n, Q, n, nrhs, part, d_dot, pq.data(), st);
        if (rc) return rc;
        for (int j = 0; j < nrhs; ++j) alpha[j] = (active[j] && pq[j] != 0.0) ? rz[j] / pq[j] : 0.0;
        HIP_TRY(hipMemcpyAsync(d_alpha, alpha.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, st));
        launch_axpby(n, d_alpha, P, n, d_one, X, ldx, nrhs, st);      // x += alpha p
        for (int j = 0; j < nrhs; ++j) alpha[j] = -alpha[j];
        HIP_TRY(hipMemcpyAsync(d_beta, alpha.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, st));
        launch_axpby(n, d_beta, Q, n, d_one, R, n, nrhs, st);          // r -= alpha q
        rc = dots_host(F, n, R, n, R, n, nrhs, part, d_dot, rr.data(), st);
        if (rc) return rc;
        nact = 0;
        for (int j = 0; j < nrhs; ++j) {
            if (active[j] && std::sqrt(std::max(rr[j], 0.0)) <= tol * bn[j]) active[j] = 0;
            nact += active[j];
        }
        if (nact == 0) break;
        if (flexible) {
            rc = dots_host(F, n, R, n, Zv, n, nrhs, part, d_dot, rzo.data(), st);
            if (rc) return rc;
        }
        rc = solve_impl(F, nrhs, R, n, Zv, n, st);
        if (rc) return rc;
        rc = dots_host(F, n, R, n, Zv, n, nrhs, part, d_dot, rzn.data(), st);
        if (rc) return rc;
        for (int j = 0; j < nrhs; ++j) {
            beta[j] = (active[j] && rz[j] != 0.0) ? (rzn[j] - rzo[j]) / rz[j] : 0.0;
            rz[j] = rzn[j];
        }
        HIP_TRY(hipMemcpyAsync(d_beta, beta.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, st));
        launch_axpby(n, d_one, Zv, n, d_beta, P, n, nrhs, st);         // p = z + beta p
    }
    // true residual
    launch_spmv(n, F->A_row.as<int64_t>(), F->A_col.as<int32_t>(), F->A_val.as<double>(), X, ldx, Q, n, nrhs, st);
    launch_xmy(n, B, ldb, Q, n, nrhs, st);
    rc = dots_host(F, n, Q, n, Q, n, nrhs, part, d_dot, rr.data(), st);
    if (rc) return rc;
    bool ok = true;
    for (int j = 0; j < nrhs; ++j) {
        const double r = std::sqrt(std::max(rr[j], 0.0)) / bn[j];
        if (relres) relres[j] = r;
        if (!(r <= tol)) ok = false;
    }
    if (iters) *iters = it;
    return ok ? HS_OK : HS_WARN_NOT_CONVERGED;
}

static int gmres_impl(hs_factor_s* F, int nrhs, const double* B, int64_t ldb, double* X, int64_t ldx, double tol,
                      int maxit, int restart, int* iters, double* relres, hipStream_t st) {
    if (restart < 1) restart = 30;
    int rc = ensure_krylov(F, 1, restart);
    if (rc) return rc;
    const int64_t n = F->n;
    double* w = F->kry.as<double>();
    double* R = w;
    double* T = R + n;      // preconditioned vector
    double* Wv = T + n;
    double* Q = Wv + n;
    double* V = Q + n;      // restart + 1 basis vectors
    double* sc = V + (int64_t)(restart + 1) * n;
    double* part = sc + 8;
    double* d_a = sc;
    double* d_b = sc + 1;
    double* d_dot = sc + 2;
    int total_it = 0;
    bool ok = true;
    for (int col = 0; col < nrhs; ++col) {
        const double* b = B + col * ldb;
        double* x = X + col * ldx;
        auto setc = [&](double* d, double v) { return hipMemcpyAsync(d, &v, sizeof(double), hipMemcpyHostToDevice, st); };
        double bn2;
        rc = dots_host(F, n, b, n, b, n, 1, part, d_dot, &bn2, st);
        if (rc) return rc;
        const double bn = bn2 > 0 ? std::sqrt(bn2) : 1.0;
        HIP_TRY(setc(d_a, 0.0));
        launch_axpby(n, d_a, b, n, d_a, x, n, 1, st);  // x = 0
        int it = 0;
        double rnorm = bn;
        launch_copy(n, b, n, R, n, 1, st);
        while (it < maxit && rnorm > tol * bn) {
            std::vector<double> H((size_t)(restart + 1) * restart, 0.0), g(restart + 1, 0.0), cs(restart), sn(restart);
            HIP_TRY(setc(d_a, 1.0 / rnorm));
            HIP_TRY(setc(d_b, 0.0));
            launch_axpby(n, d_a, R, n, d_b, V, n, 1, st);
            g[0] = rnorm;
            int j_used = 0;
            for (int j = 0; j < restart && it < maxit; ++j) {
                ++it;
                rc = solve_impl(F, 1, V + j * n, n, T, n, st);
                if (rc) return rc;
                launch_spmv(n, F->A_row.as<int64_t>(), F->A_col.as<int32_t>(), F->A_val.as<double>(), T, n, Wv, n, 1, st);
                for (int i = 0; i <= j; ++i) {
                    double h;
                    rc = dots_host(F, n, Wv, n, V + i * n, n, 1, part, d_dot, &h, st);
                    if (rc) return rc;
                    H[i + j * (restart + 1)] = h;
                    HIP_TRY(setc(d_a, -h));
                    HIP_TRY(setc(d_b, 1.0));
                    launch_axpby(n, d_a, V + i * n, n, d_b, Wv, n, 1, st);
                }
                double hn2;
                rc = dots_host(F, n, Wv, n, Wv, n, 1, part, d_dot, &hn2, st);
                if (rc) return rc;
                const double hn = std::sqrt(std::max(hn2, 0.0));
                H[(j + 1) + j * (restart + 1)] = hn;
                if (hn > 0) {
                    HIP_TRY(setc(d_a, 1.0 / hn));
                    HIP_TRY(setc(d_b, 0.0));
                    launch_axpby(n, d_a, Wv, n, d_b, V + (j + 1) * n, n, 1, st);
                }
                for (int i = 0; i < j; ++i) {
                    const double a0 = H[i + j * (restart + 1)], a1 = H[(i + 1) + j * (restart + 1)];
                    H[i + j * (restart + 1)] = cs[i] * a0 + sn[i] * a1;
                    H[(i + 1) + j * (restart + 1)] = -sn[i] * a0 + cs[i] * a1;
                }
                const double a0 = H[j + j * (restart + 1)], a1 = H[(j + 1) + j * (restart + 1)];
                const double den = std::hypot(a0, a1);
                cs[j] = den > 0 ? a0 / den : 1.0;
                sn[j] = den > 0 ? a1 / den : 0.0;
                H[j + j * (restart + 1)] = cs[j] * a0 + sn[j] * a1;
                H[(j + 1) + j * (restart + 1)] = 0.0;
                g[j + 1] = -sn[j] * g[j];
                g[j] = cs[j] * g[j];
                j_used = j + 1;
                if (std::fabs(g[j + 1]) <= tol * bn) break;
            }
            // y = H^{-1} g, x += M^{-1} V y
            std::vector<double> y(j_used);
            for (int i = j_used - 1; i >= 0; --i) {
                double s = g[i];
                for (int c = i + 1; c < j_used; ++c) s -= H[i + c * (restart + 1)] * y[c];
                y[i] = s / H[i + i * (restart + 1)];
            }
            HIP_TRY(setc(d_b, 0.0));
            HIP_TRY(setc(d_a, 0.0));
            launch_axpby(n, d_a, Wv, n, d_b, Wv, n, 1, st);  // Wv = 0
            for (int i = 0; i < j_used; ++i) {
                HIP_TRY(setc(d_a, y[i]));
                HIP_TRY(setc(d_b, 1.0));
                launch_axpby(n, d_a, V + i * n, n, d_b, Wv, n, 1, st);
            }
            rc = solve_impl(F, 1, Wv, n, T, n, st);
            if (rc) return rc;
            HIP_TRY(setc(d_a, 1.0));
            HIP_TRY(setc(d_b, 1.0));
            launch_axpby(n, d_a, T, n, d_b, x, ldx, 1, st);
            // true residual
            launch_spmv(n, F->A_row.as<int64_t>(), F->A_col.as<int32_t>(), F->A_val.as<double>(), x, ldx, R, n, 1, st);
            launch_xmy(n, b, n, R, n, 1, st);
            double rn2;
            rc = dots_host(F, n, R, n, R, n, 1, part, d_dot, &rn2, st);
            if (rc) return rc;
            rnorm = std::sqrt(std::max(rn2, 0.0));
        }
        if (relres) relres[col] = rnorm / bn;
        if (!(rnorm <= tol * bn)) ok = false;
        total_it = std::max(total_it, it);
    }
    if (iters) *iters = total_it;
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

int hs_factor(const hs_csr* A, const hs_geometry* geom, const hs_opts* opts, void* hip_stream, hs_factor_t* F_out) {
    g_err.clear();
    if (!F_out) return fail(HS_ERR_ARG, "F_out is NULL");
    *F_out = nullptr;
    if (!A || !geom || !opts || !A->row_ptr || (A->nnz > 0 && (!A->col_idx || !A->val)))
        return fail(HS_ERR_ARG, "null argument");
    if (A->n <= 0 || A->nnz < 0 || A->n > INT32_MAX) return fail(HS_ERR_ARG, "bad matrix size");
    if (!(opts->eps >= 0.0) || opts->leaf_size <= 0 || opts->fixed_rank < 0 || opts->coarse_fp64_dofs < 0 ||
        (opts->precision != HS_FP64 && opts->precision != HS_MIXED))
        return fail(HS_ERR_ARG, "bad options");
    if (geom->dim < 1 || geom->dim > 3 || (int64_t)geom->nx * geom->ny * geom->nz != A->n)
        return fail(HS_ERR_GEOMETRY, "n != nx*ny*nz");
    int rc = check_device();
    if (rc) return rc;
    std::unique_ptr<hs_factor_s> F(new hs_factor_s());
    F->n = A->n;
    F->opts = *opts;
    F->info.breakdown_level = -1;
    F->info.breakdown_cluster = -1;
    rc = factor_impl(F.get(), A, geom, (hipStream_t)hip_stream);
    if (rc < 0) return rc;
    *F_out = F.release();
    return HS_OK;
}

int hs_solve(hs_factor_t F, int64_t nrhs, const double* B, int64_t ldb, double* X, int64_t ldx, void* hip_stream) {
    g_err.clear();
    if (!F || !B || !X || nrhs < 1 || nrhs > 64 || ldb < F->n || ldx < F->n) return fail(HS_ERR_ARG, "bad argument");
    if (B == X && ldb != ldx) return fail(HS_ERR_ARG, "aliased B and X need equal leading dimensions");
    return solve_impl(F, (int)nrhs, B, ldb, X, ldx, (hipStream_t)hip_stream);
}

int hs_pcg(hs_factor_t F, int64_t nrhs, const double* B, int64_t ldb, double* X, int64_t ldx, double tol, int32_t maxit,
           int32_t* iters_out, double* relres_out, void* hip_stream) {
    g_err.clear();
    if (!F || !B || !X || nrhs < 1 || nrhs > 64 || ldb < F->n || ldx < F->n || !(tol >= 0) || maxit < 0 || B == X)
        return fail(HS_ERR_ARG, "bad argument");
    return pcg_impl(F, (int)nrhs, B, ldb, X, ldx, tol, maxit, iters_out, relres_out, (hipStream_t)hip_stream);
}

int hs_gmres(hs_factor_t F, int64_t nrhs, const double* B, int64_t ldb, double* X, int64_t ldx, double tol,
             int32_t maxit, int32_t restart, int32_t* iters_out, double* relres_out, void* hip_stream) {
    g_err.clear();
    if (!F || !B || !X || nrhs < 1 || ldb < F->n || ldx < F->n || !(tol >= 0) || maxit < 0 || restart < 1 ||
        restart > 1000 || B == X)
        return fail(HS_ERR_ARG, "bad argument");
    return gmres_impl(F, (int)nrhs, B, ldb, X, ldx, tol, maxit, restart, iters_out, relres_out,
                      (hipStream_t)hip_stream);
}

int hs_factor_info(hs_factor_t F, hs_info* out) {
    if (!F || !out) return fail(HS_ERR_ARG, "null argument");
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
    std::vector<int64_t> roff(1);
    HIP_TRY(hipMemcpy(ntot.data(), LD.dev.ntot + cluster, sizeof(int), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(ncap.data(), LD.dev.ncap + cluster, sizeof(int), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(roff.data(), LD.dev.rec_off + cluster, sizeof(int64_t), hipMemcpyDeviceToHost));
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
    const size_t es = LD.esz();
    const char* src = LD.rec.as<char>() + (roff[0] + e0) * es;
    if (!LD.f32) {
        HIP_TRY(hipMemcpy2D(out, r * sizeof(double), src, ld * es, r * es, c, hipMemcpyDeviceToHost));
    } else {
        std::vector<float> tmp((size_t)(r * c));
        HIP_TRY(hipMemcpy2D(tmp.data(), r * es, src, ld * es, r * es, c, hipMemcpyDeviceToHost));
        for (size_t i = 0; i < tmp.size(); ++i) out[i] = tmp[i];
    }
    return HS_OK;
}

void hs_free(hs_factor_t F) { delete F; }

int hs_symbolic_create(const hs_csr* A, const hs_geometry* geom, int32_t leaf_size, hs_symbolic_t* S_out) {
    g_err.clear();
    if (!S_out || !A || !geom || !A->row_ptr || A->on_device) return fail(HS_ERR_ARG, "host CSR required");
    *S_out = nullptr;
    if (A->n <= 0 || leaf_size <= 0) return fail(HS_ERR_ARG, "bad size");
    int rc = validate_csr_host(A->n, A->nnz, A->row_ptr, A->col_idx);
    if (rc) return rc;
    std::unique_ptr<hs_symbolic_s> S(new hs_symbolic_s());
    rc = build_symbolic(A->n, A->row_ptr, A->col_idx, geom->nx, geom->ny, geom->nz, leaf_size, S->sym);
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
    auto cp = [](const std::vector<int>& v, int32_t* o) {
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

int hs_set_allocator(void* (*alloc_fn)(size_t, void*), void (*free_fn)(void*, void*), void* ctx) {
    if ((alloc_fn == nullptr) != (free_fn == nullptr)) return fail(HS_ERR_ARG, "give both functions or neither");
    g_alloc_fn = alloc_fn;
    g_free_fn = free_fn;
    g_alloc_ctx = ctx;
    return HS_OK;
}

int hs_profile_enable(int32_t enable) {
    g_prof_on = enable != 0;
    return HS_OK;
}

int hs_profile_reset(void) {
    for (auto& f : g_prof) {
        f.launches = 0;
        f.seconds = f.bytes = f.flops = 0.0;
    }
    g_prof_pending.clear();
    return HS_OK;
}

int hs_profile_read(const char* family, int64_t* launches, double* seconds, double* bytes, double* flops) {
    if (!family) return fail(HS_ERR_ARG, "null family");
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

}  // extern "C"
