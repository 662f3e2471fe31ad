// C ABI of the RAS-PML GMRES hot path (declared in include/ras_pml.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "devpool.h"
#include "device.h"
#include "internal.h"
#include "warm.h"

namespace raspml {

// kernels (k_*.hip)
void launch_global_stencil(const DevProb *, int, long long, double2 *, long long, hipStream_t);
void launch_local_stencil(const DevProb *, const DevSub *, int, int, double2 *, hipStream_t);
void launch_rhs(const DevProb *, int, long long, const double2 *, double2 *, hipStream_t);
void launch_band_ldlt(bool, int, const DevSub *, const int *, int, const double2 *, void *, int *,
                      hipStream_t);
int ldlt_mfma_tiles(int W);
bool ldlt_mfma_default_occ(bool, int NT);
void launch_band_ldlt_mfma(bool, int, bool, const DevSub *, const int *, int, const double2 *, void *,
                           int *, hipStream_t);
void launch_band_solve(bool, bool, int, const DevProb *, const DevSub *, const int *, int,
                       const int *, const SolveSrc &, const void *, void *, void *,
                       const SolveDispatch &, hipStream_t);
long long ldlt_wide_scratch(int K);
void launch_band_ldlt_wide(bool, int, const DevSub *, const int *, int, const double2 *, void *,
                           void *, int *, hipStream_t);
void launch_band_solve_wide(bool, const DevProb *, const DevSub *, const int *, int, const int *,
                            const SolveSrc &, const void *, void *, void *, hipStream_t);
void launch_pou_sum(bool, const DevProb *, int, long long, const DevSub *, const int *,
                    const int *, const int *, const double *, const void *, const SumDst &, bool,
                    hipStream_t);
void launch_export_local(bool, const DevSub *, int, int, const void *, double2 *, hipStream_t);
void launch_spmv(const DevProb *, int, long long, const int *, const double2 *, long long,
                 const double2 *, const double2 *, double2 *, hipStream_t);
void launch_mgs(const DevProb *, int, const KState *, double2 *, const double2 *, long long, int,
                int, int, int, double2 *, double2 *, unsigned int *, hipStream_t);
void launch_reduce(const DevProb *, int, const int *, const double2 *, const double2 *, int,
                   double2 *, double2 *, unsigned int *, hipStream_t);
void launch_normalize(const DevProb *, int, long long, const KState *, double2 *, int, int,
                      const double2 *, hipStream_t);
void launch_start_cycle(const DevProb *, int, long long, const KState *, const double2 *,
                        double2 *, hipStream_t);
void launch_rich_update(RState *, int *, const double2 *, double *, int, int, double, hipStream_t);
void launch_givens(KState *, int, int, double2 *, double *, double2 *, double2 *, double *, int *,
                   hipStream_t);
void launch_solve_y(const KState *, int, int, const double2 *, const double2 *, double2 *,
                    hipStream_t);
void launch_update_x(const DevProb *, int, long long, const KState *, const int *, int,
                     const double2 *, long long, const double2 *, double2 *, hipStream_t);
int arnoldi_variants();
int arnoldi_variant_e(int variant);
int arnoldi_block_capacity(int variant, int *blocks_per_cu);
hipError_t launch_arnoldi(int variant, int nblocks, const DevProb *, const KState *,
                          const ArnoldiBlock *, const double2 *, long long, const double2 *,
                          double2 *, int, double2 *, double2 *, unsigned long long *,
                          unsigned long long *, int *, int, hipStream_t);

constexpr int kRedBlocksHost = 512;

enum Cat { C_SOLVE = 0, C_SUM, C_SPMV, C_MGS, C_GIVENS, C_NCAT };

struct Status {
    int code = RAS_OK;
    std::string msg;
};

}  // namespace raspml

using namespace raspml;

struct ras_pml_handle {
    std::vector<PlanProblem> plans;
    std::vector<DevProb> hprobs;
    std::vector<DevSub> hsubs;
    std::vector<int> order;
    // factorisation: subdomains grouped by window size (tiles per side),
    // largest first within a group; {tiles, first, count, kernel variant
    // (LU_*), largest W} per group
    std::vector<int> lu_order;
    std::vector<std::array<int, 5>> lu_groups;
    // wide subdomains (W > kMaxW): {K = W / 64, first in lu_order, count},
    // factorised one group after another through the scratch d_wscratch
    std::vector<std::array<int, 3>> wide_groups;
    void *d_wscratch = nullptr;
    // order: the nsub_reg subdomains with W <= kMaxW (largest first, widest
    // maxW_reg), then the nsub_wide wide ones
    int nsub_reg = 0, nsub_wide = 0, maxW_reg = 0;
    bool solve_deep = true;    // band-solve prefetch depth variant
    bool solve_queue = false;  // band-solve dispatch: persistent waves and a work queue
    int solve_waves = 0;       // waves of the persistent band solve (one per SIMD)
    bool graph_steps = false;  // GMRES steps replayed from a graph (RAS_FLAG_GRAPH_STEPS)
    std::vector<double> tune_ms;   // the last autotune's timings (ras_pml_tune_report)
    std::string arch;          // gfx name of the device (tuning cache keys)
    std::string tune_cache;    // opts.tune_cache (empty: none)
    long long skipped_steps = 0;   // GMRES steps enqueued after every problem had stopped
    int nprob = 0, nsub = 0, maxW = 0, max_n = 0;
    long long ntot = 0, nloc = 0, nvec = 0, max_ndof = 0;
    bool fp64 = false;
    int flags = 0;
    int device = 0;            // the device current at setup
    size_t csize = 8;          // bytes of one local complex value
    size_t fac_elems = 0;

    DevProb *d_probs = nullptr;
    DevSub *d_subs = nullptr;
    int *d_order = nullptr, *d_lu_order = nullptr;
    int *d_pcnt = nullptr, *d_pchunk = nullptr;
    double *d_pw = nullptr;
    double2 *d_coef = nullptr;
    double2 *d_lst = nullptr;
    void *d_F = nullptr, *d_ybuf = nullptr, *d_xout = nullptr;
    int *d_status = nullptr;
    unsigned int *d_queue = nullptr;   // work counter of the persistent band solve (2 words)

    // Krylov workspace
    int m_alloc = 0;
    double2 *d_V = nullptr, *d_Z = nullptr, *d_r = nullptr;
    double2 *d_H = nullptr, *d_g = nullptr, *d_sn = nullptr, *d_y = nullptr;
    double *d_cs = nullptr, *d_hist = nullptr;
    KState *d_ks = nullptr;
    int *d_active = nullptr;
    // fixed-point iteration: per-problem state and residual histories
    RState *d_rs = nullptr, *h_rs = nullptr;      // h_rs pinned
    double *d_rhist = nullptr;
    int rhist_cap = -1;                            // maxit the history holds
    double2 *d_partials = nullptr, *d_redout = nullptr;
    unsigned int *d_counters = nullptr;
    // fused Arnoldi step (cooperative launch); E = 0 selects the
    // one-launch-per-projection path
    int arn_E = -1, arn_nblocks = 0, arn_var = 0;   // fused Arnoldi: unknowns per thread, variant
    int arn_pref = -1;         // preferred fused-Arnoldi variant (-1: the first that fits)
    ArnoldiBlock *d_ablocks = nullptr;
    double2 *d_part2 = nullptr;
    unsigned long long *d_bar = nullptr;
    size_t bar_words = 0;
    unsigned long long *d_epoch = nullptr;   // barrier epoch reached (device)
    bool bar_reset = false;    // a barrier wait ran out: clear the counters first
    int *d_err = nullptr;
    // one graph of kGraphSteps FGMRES steps (recorded on cap_stream)
    hipStream_t cap_stream = nullptr;
    hipGraph_t step_graph = nullptr;
    hipGraphExec_t step_exec = nullptr;
    int graph_m = 0;
    const void *graph_V = nullptr;
    KState *h_ks = nullptr;        // pinned
    int *h_err = nullptr;          // pinned
    double2 *h_red = nullptr;      // pinned
    std::vector<int> res_iters;
    std::vector<double> res_relres;
    std::vector<int> res_conv;

    std::string last_error;

    struct EvPair {
        hipEvent_t a, b;
    };
    std::vector<EvPair> ev[C_NCAT];
    std::vector<EvPair> pool;
    ras_pml_stats stats{};

    ~ras_pml_handle();
};

namespace {

thread_local std::string g_plan_error;

// Device buffers come from the process-wide cache (devpool.cpp), which may
// hand a released block to the next request at once: release only what no
// queued work uses (idle_device first).
void dfree(void *p) {
    if (p) pool_free(p);
}

// One auxiliary stream per device (default priority, created on first use,
// kept until ras_pml_shutdown): the smaller factorisation classes run on it
// beside the largest, so their workgroups take the slots the largest class
// leaves free in its last round.
std::mutex g_aux_mu;
std::vector<hipStream_t> g_aux;

hipStream_t aux_stream(int device) {
    std::lock_guard<std::mutex> g(g_aux_mu);
    if (device < 0) return nullptr;
    if (g_aux.size() <= static_cast<size_t>(device)) g_aux.resize(device + 1, nullptr);
    if (!g_aux[device] && hipStreamCreateWithFlags(&g_aux[device], hipStreamNonBlocking) != hipSuccess)
        g_aux[device] = nullptr;
    return g_aux[device];
}

// Destroys the auxiliary streams (each on its own device, after its work).
void destroy_aux_streams() {
    std::lock_guard<std::mutex> g(g_aux_mu);
    int cur = -1;
    const bool have_cur = hipGetDevice(&cur) == hipSuccess;
    for (size_t d = 0; d < g_aux.size(); ++d) {
        if (!g_aux[d]) continue;
        if (hipSetDevice(static_cast<int>(d)) == hipSuccess) {
            (void)hipStreamSynchronize(g_aux[d]);
            (void)hipStreamDestroy(g_aux[d]);
        }
        g_aux[d] = nullptr;
    }
    if (have_cur) (void)hipSetDevice(cur);
}

// Waits for the handle's device, as hipFree would.
void idle_device(int device) {
    int cur = -1;
    const bool other = hipGetDevice(&cur) == hipSuccess && cur != device;
    if (other) (void)hipSetDevice(device);
    (void)hipDeviceSynchronize();
    if (other) (void)hipSetDevice(cur);
}

#define HCHK(H, call)                                                                 \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) {                                                       \
            (H)->last_error = std::string(#call) + ": " + hipGetErrorString(e_);      \
            return (e_ == hipErrorOutOfMemory) ? RAS_ENOMEM : RAS_EHIP;               \
        }                                                                             \
    } while (0)

template <typename P>
int dalloc(ras_pml_handle *H, P **p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 16;
    const auto t0 = std::chrono::steady_clock::now();
    hipError_t e = pool_alloc(reinterpret_cast<void **>(p), bytes);
    H->stats.alloc_ms +=
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (e != hipSuccess) {
        char buf[128];
        std::snprintf(buf, sizeof buf, "device allocation of %zu bytes failed: ", bytes);
        H->last_error = std::string(buf) + hipGetErrorString(e);
        *p = nullptr;
        return e == hipErrorOutOfMemory ? RAS_ENOMEM : RAS_EHIP;
    }
    return RAS_OK;
}

#define RCHK(x)                   \
    do {                          \
        int r_ = (x);             \
        if (r_ != RAS_OK) return r_; \
    } while (0)

hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

ras_pml_handle::EvPair take_pair(ras_pml_handle *H) {
    if (!H->pool.empty()) {
        auto p = H->pool.back();
        H->pool.pop_back();
        return p;
    }
    // timing only: no system-scope fence at the record (a default event
    // writes back and invalidates the caches there, which slows the kernel
    // it brackets); the stats are read after a stream synchronisation
    ras_pml_handle::EvPair p{};
    (void)hipEventCreateWithFlags(&p.a, hipEventDisableSystemFence);
    (void)hipEventCreateWithFlags(&p.b, hipEventDisableSystemFence);
    return p;
}

struct Timer {
    ras_pml_handle *H;
    int cat;
    hipStream_t s;
    bool on;
    ras_pml_handle::EvPair p{};
    Timer(ras_pml_handle *H_, int cat_, hipStream_t s_, bool timed = true)
        : H(H_), cat(cat_), s(s_), on(timed && (H_->flags & RAS_FLAG_TIMING) != 0) {
        if (on) {
            p = take_pair(H);
            (void)hipEventRecord(p.a, s);
        }
    }
    ~Timer() {
        if (on) {
            (void)hipEventRecord(p.b, s);
            H->ev[cat].push_back(p);
        }
    }
};

void collect_events(ras_pml_handle *H) {
    long long *cnt[C_NCAT] = {&H->stats.n_solve, &H->stats.n_sum, &H->stats.n_spmv, &H->stats.n_mgs,
                              &H->stats.n_givens};
    double *ms[C_NCAT] = {&H->stats.solve_ms, &H->stats.sum_ms, &H->stats.spmv_ms, &H->stats.mgs_ms,
                          &H->stats.givens_ms};
    for (int c = 0; c < C_NCAT; ++c) {
        for (auto &p : H->ev[c]) {
            (void)hipEventSynchronize(p.b);
            float t = 0.0f;
            if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
                *ms[c] += t;
                *cnt[c] += 1;
            }
            H->pool.push_back(p);
        }
        H->ev[c].clear();
    }
}

}  // namespace

ras_pml_handle::~ras_pml_handle() {
    void *ptrs[] = {d_probs, d_subs,  d_order, d_lu_order, d_pcnt, d_pchunk, d_pw,     d_coef,     d_lst,
                    d_F,     d_ybuf,  d_xout,  d_status, d_V,    d_Z,      d_r,        d_H,
                    d_g,     d_sn,    d_y,     d_cs,   d_hist,   d_ks,     d_active,   d_partials,
                    d_redout, d_counters, d_ablocks, d_part2, d_bar, d_err, d_rs, d_rhist,
                    d_queue, d_epoch, d_wscratch};
    bool any = false;
    for (void *p : ptrs) any = any || p != nullptr;
    if (any) idle_device(device);
    if (step_exec) (void)hipGraphExecDestroy(step_exec);
    if (step_graph) (void)hipGraphDestroy(step_graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (void *p : ptrs) dfree(p);
    if (h_ks) (void)hipHostFree(h_ks);
    if (h_rs) (void)hipHostFree(h_rs);
    if (h_red) (void)hipHostFree(h_red);
    if (h_err) (void)hipHostFree(h_err);
    for (int c = 0; c < C_NCAT; ++c)
        for (auto &p : ev[c]) pool.push_back(p);
    for (auto &p : pool) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
}

namespace {

void apply_cache(ras_pml_handle *H, const char *path);

// Factorisation kernel of a window class: the blocked one with the
// matrix-core trailing update, unconstrained or held to the register budget
// that lets four (complex64) or two (complex128) workgroups share a CU, or
// the one-column kernel on the vector ALUs (rank-1 update per column).
enum { LU_MFMA = 0, LU_MFMA_CAPPED = 1, LU_VALU = 2, LU_NVARIANTS = 3 };

// The factorisation of every window class with its kernel variant
// (lu_groups[i][3]): the largest class on the caller's stream, the others
// beside it on the auxiliary stream (fork and join through events), so that
// their workgroups take the slots the largest class leaves free in its last
// round.
int factorise(ras_pml_handle *H, hipStream_t st) {
    hipStream_t aux = H->lu_groups.size() > 1 ? aux_stream(H->device) : nullptr;
    hipEvent_t fork{}, join{};
    if (aux) {
        HCHK(H, hipEventCreateWithFlags(&fork, hipEventDisableTiming));
        if (hipEventCreateWithFlags(&join, hipEventDisableTiming) != hipSuccess) {
            (void)hipEventDestroy(fork);
            H->last_error = "factorisation: cannot create an event";
            return RAS_EHIP;
        }
        if (hipEventRecord(fork, st) != hipSuccess || hipStreamWaitEvent(aux, fork, 0) != hipSuccess)
            aux = nullptr;          // everything on the caller's stream instead
    }
    for (size_t i = 0; i < H->lu_groups.size(); ++i) {
        const auto &g = H->lu_groups[i];
        const hipStream_t s = i == 0 || !aux ? st : aux;
        if (g[3] == LU_VALU)
            launch_band_ldlt(H->fp64, g[4], H->d_subs, H->d_lu_order + g[1], g[2], H->d_lst,
                             H->d_F, H->d_status, s);
        else
            launch_band_ldlt_mfma(H->fp64, g[0], g[3] == LU_MFMA_CAPPED, H->d_subs,
                                  H->d_lu_order + g[1], g[2], H->d_lst, H->d_F, H->d_status, s);
    }
    for (const auto &g : H->wide_groups)
        launch_band_ldlt_wide(H->fp64, g[0], H->d_subs, H->d_lu_order + g[1], g[2], H->d_lst,
                              H->d_F, H->d_wscratch, H->d_status, st);
    hipError_t e = hipGetLastError();
    if (aux && e == hipSuccess) {
        e = hipEventRecord(join, aux);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, join, 0);
    }
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
    if (e != hipSuccess) {
        H->last_error = std::string("factorisation launch: ") + hipGetErrorString(e);
        return RAS_EHIP;
    }
    return RAS_OK;
}

int build(ras_pml_handle *H, hipStream_t st) {
    // ---- concatenate problems
    H->nprob = static_cast<int>(H->plans.size());
    long long dof = 0, vec = 0, loc = 0;
    size_t fac = 0;
    int pou_off = 0;
    H->hprobs.clear();
    H->hsubs.clear();
    std::vector<int> pcnt, pchunk;
    std::vector<double> pw;
    H->maxW = 0;
    H->max_n = 0;
    H->max_ndof = 0;
    for (int p = 0; p < H->nprob; ++p) {
        PlanProblem &pl = H->plans[p];
        DevProb P{};
        P.k = pl.k;
        P.h = pl.h;
        P.sigma = pl.sigma;
        P.G = pl.G;
        P.Nc = pl.Nc;
        P.n1 = pl.Nc - 1;
        P.Px = pl.Px;
        P.Py = pl.Py;
        P.sub_first = static_cast<int>(H->hsubs.size());
        P.dof_off = dof;
        P.ndof = pl.ndof;
        for (int axis = 0; axis < 2; ++axis) {
            (axis == 0 ? P.pou_x : P.pou_y) = pou_off;
            pcnt.insert(pcnt.end(), pl.pou_cnt[axis].begin(), pl.pou_cnt[axis].end());
            pchunk.insert(pchunk.end(), pl.pou_chunk[axis].begin(), pl.pou_chunk[axis].end());
            pw.insert(pw.end(), pl.pou_w[axis].begin(), pl.pou_w[axis].end());
            pou_off += pl.Nc + 1;
        }
        for (DevSub s : pl.subs) {
            s.prob = p;
            s.fac_off = static_cast<long long>(fac);
            s.vec_off = vec;
            s.loc_off = loc;
            // local index of node (i, j): (j - jy0) nx + (i - ix0) along x, else
            // (i - ix0) ny + (j - jy0)
            s.pou_sx = s.xfast ? 1 : s.ny;
            s.pou_sy = s.xfast ? s.nx : 1;
            s.pou_off = static_cast<int>(vec) - (s.xfast ? s.jy0 * s.nx + s.ix0 : s.ix0 * s.ny + s.jy0);
            s.pou_pad_ = 0;
            if (vec + s.npad >= (1LL << 30)) {
                H->last_error = "too many local unknowns (2^30)";
                return RAS_EINVAL;
            }
            if (s.W & 1) {            // the pair-layout solve relies on even W
                H->last_error = "internal: odd factor column length";
                return RAS_EINVAL;
            }
            fac += static_cast<size_t>(s.npad) * (2 * s.W + 1);   // L, rows of L, D^{-1}
            vec += s.npad;
            loc += s.n;
            H->maxW = std::max(H->maxW, s.W);
            H->max_n = std::max(H->max_n, s.n);
            H->hsubs.push_back(s);
        }
        dof += pl.ndof;
        H->max_ndof = std::max(H->max_ndof, pl.ndof);
        H->hprobs.push_back(P);
    }
    if (dof > (1LL << 31) - 1 || vec > (1LL << 31) - 1) {
        H->last_error = "problem too large for 32-bit unknown indices";
        return RAS_ENOTSUP;
    }
    H->nsub = static_cast<int>(H->hsubs.size());
    H->ntot = dof;
    H->nvec = vec;
    H->nloc = loc;
    H->fac_elems = fac;
    H->csize = H->fp64 ? 16 : 8;
    // largest subdomains first (longest processing time first), those of
    // the register-ring kernels (W <= kMaxW) ahead of the wide ones
    auto wide = [&](int j) { return H->hsubs[j].W > kMaxW; };
    H->order.resize(H->nsub);
    std::iota(H->order.begin(), H->order.end(), 0);
    std::stable_sort(H->order.begin(), H->order.end(),
                     [&](int a, int b) { return H->hsubs[a].n > H->hsubs[b].n; });
    std::stable_partition(H->order.begin(), H->order.end(), [&](int j) { return !wide(j); });
    H->nsub_wide = static_cast<int>(std::count_if(H->order.begin(), H->order.end(), wide));
    H->nsub_reg = H->nsub - H->nsub_wide;
    H->maxW_reg = 0;
    for (int i = 0; i < H->nsub_reg; ++i)
        H->maxW_reg = std::max(H->maxW_reg, H->hsubs[H->order[i]].W);
    H->lu_groups.clear();
    H->wide_groups.clear();
    {
        H->lu_order = H->order;
        // window classes of the register kernel, widest first; then the wide
        // subdomains by W
        auto tiles = [&](int j) { return ldlt_mfma_tiles(H->hsubs[j].W); };
        std::stable_sort(H->lu_order.begin(), H->lu_order.begin() + H->nsub_reg,
                         [&](int a, int b) { return tiles(a) > tiles(b); });
        std::stable_sort(H->lu_order.begin() + H->nsub_reg, H->lu_order.end(),
                         [&](int a, int b) { return H->hsubs[a].W > H->hsubs[b].W; });
        for (int i = H->nsub_reg; i < H->nsub;) {
            int e = i;
            while (e < H->nsub && H->hsubs[H->lu_order[e]].W == H->hsubs[H->lu_order[i]].W) ++e;
            H->wide_groups.push_back({H->hsubs[H->lu_order[i]].W / 64, i, e - i});
            i = e;
        }
        for (int i = 0; i < H->nsub_reg;) {
            int e = i, wmax = 0;
            while (e < H->nsub_reg && tiles(H->lu_order[e]) == tiles(H->lu_order[i]))
                wmax = std::max(wmax, H->hsubs[H->lu_order[e++]].W);
            const int nt = tiles(H->lu_order[i]);
            H->lu_groups.push_back(
                {nt, i, e - i, ldlt_mfma_default_occ(H->fp64, nt) ? LU_MFMA_CAPPED : LU_MFMA, wmax});
            i = e;
        }
    }
    if (!H->tune_cache.empty()) apply_cache(H, H->tune_cache.c_str());

    // algorithmic bytes of one band-solve launch: the nf + 1 band entries of
    // every column of L, read by both sweeps, D^{-1}, the gathered
    // right-hand side (complex128), the forward result written and read
    // back, the local solution written -- over the n rows of the matrix
    // (the stored zeros of the padding rows, the diagonal slot and the slot
    // that makes W even are not counted).
    double sb = 0.0, fb = 0.0;
    for (const DevSub &s : H->hsubs) {
        sb += (2.0 * s.n * (s.nf + 1) + s.n + 3.0 * s.n) * H->csize + 16.0 * s.n;
        fb += static_cast<double>(s.npad) * (2 * s.W + 1) * H->csize;
    }
    H->stats.solve_bytes = sb;
    H->stats.factor_bytes = fb;

    // ---- device memory
    RCHK(dalloc(H, &H->d_probs, sizeof(DevProb) * H->nprob));
    RCHK(dalloc(H, &H->d_subs, sizeof(DevSub) * H->nsub));
    RCHK(dalloc(H, &H->d_order, sizeof(int) * H->nsub));
    RCHK(dalloc(H, &H->d_lu_order, sizeof(int) * H->nsub));
    RCHK(dalloc(H, &H->d_pcnt, sizeof(int) * pcnt.size()));
    RCHK(dalloc(H, &H->d_pchunk, sizeof(int) * pchunk.size()));
    RCHK(dalloc(H, &H->d_pw, sizeof(double) * pw.size()));
    RCHK(dalloc(H, &H->d_coef, sizeof(double2) * 4 * H->ntot));
    RCHK(dalloc(H, &H->d_lst, sizeof(double2) * 4 * H->nloc));
    RCHK(dalloc(H, &H->d_F, H->csize * fac + kFactorSlack));
    RCHK(dalloc(H, &H->d_ybuf, H->csize * H->nvec));
    RCHK(dalloc(H, &H->d_xout, H->csize * H->nvec));
    RCHK(dalloc(H, &H->d_status, sizeof(int) * H->nsub));
    RCHK(dalloc(H, &H->d_queue, sizeof(unsigned int) * 2));
    {
        long long wsc = 0;
        for (const auto &g : H->wide_groups)
            wsc = std::max(wsc, static_cast<long long>(g[2]) * ldlt_wide_scratch(g[0]));
        if (wsc > 0) RCHK(dalloc(H, &H->d_wscratch, H->csize * static_cast<size_t>(wsc)));
    }
    HCHK(H, hipMemsetAsync(H->d_queue, 0, sizeof(unsigned int) * 2, st));
    {
        int cus = 0;
        HCHK(H, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, H->device));
        H->solve_waves = 4 * cus;          // one wave per SIMD
    }
    HCHK(H, hipMemcpyAsync(H->d_probs, H->hprobs.data(), sizeof(DevProb) * H->nprob,
                           hipMemcpyHostToDevice, st));
    HCHK(H, hipMemcpyAsync(H->d_subs, H->hsubs.data(), sizeof(DevSub) * H->nsub,
                           hipMemcpyHostToDevice, st));
    HCHK(H, hipMemcpyAsync(H->d_order, H->order.data(), sizeof(int) * H->nsub,
                           hipMemcpyHostToDevice, st));
    HCHK(H, hipMemcpyAsync(H->d_lu_order, H->lu_order.data(), sizeof(int) * H->nsub,
                           hipMemcpyHostToDevice, st));
    HCHK(H, hipMemcpyAsync(H->d_pcnt, pcnt.data(), sizeof(int) * pcnt.size(),
                           hipMemcpyHostToDevice, st));
    HCHK(H, hipMemcpyAsync(H->d_pchunk, pchunk.data(), sizeof(int) * pchunk.size(),
                           hipMemcpyHostToDevice, st));
    HCHK(H, hipMemcpyAsync(H->d_pw, pw.data(), sizeof(double) * pw.size(),
                           hipMemcpyHostToDevice, st));

    hipEvent_t e0{}, e1{}, e2{};
    const bool timing = (H->flags & RAS_FLAG_TIMING) != 0;
    if (timing) {
        HCHK(H, hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
        HCHK(H, hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
        HCHK(H, hipEventCreateWithFlags(&e2, hipEventDisableSystemFence));
        HCHK(H, hipEventRecord(e0, st));
    }
    launch_global_stencil(H->d_probs, H->nprob, H->max_ndof, H->d_coef, H->ntot, st);
    HCHK(H, hipGetLastError());
    launch_local_stencil(H->d_probs, H->d_subs, H->nsub, H->max_n, H->d_lst, st);
    HCHK(H, hipGetLastError());
    if (timing) HCHK(H, hipEventRecord(e1, st));
    RCHK(factorise(H, st));
    if (timing) HCHK(H, hipEventRecord(e2, st));
    std::vector<int> status(H->nsub);
    HCHK(H, hipMemcpyAsync(status.data(), H->d_status, sizeof(int) * H->nsub,
                           hipMemcpyDeviceToHost, st));
    HCHK(H, hipStreamSynchronize(st));
    if (timing) {
        float a = 0, b = 0;
        (void)hipEventElapsedTime(&a, e0, e1);
        (void)hipEventElapsedTime(&b, e1, e2);
        H->stats.setup_assemble_ms = a;
        H->stats.setup_factor_ms = b;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        (void)hipEventDestroy(e2);
    }
    for (int s = 0; s < H->nsub; ++s) {
        if (status[s] >= 0) {
            char buf[160];
            std::snprintf(buf, sizeof buf, "zero pivot in subdomain %d (problem %d) at column %d",
                          s, H->hsubs[s].prob, status[s]);
            H->last_error = buf;
            return RAS_EZEROPIVOT;
        }
    }
    return RAS_OK;
}

void destroy_step_graph(ras_pml_handle *H);

// Whether fused-Arnoldi variant `var` keeps every block of this handle's
// grid co-resident; *blocks: the grid.
bool arnoldi_fits(const ras_pml_handle *H, int var, int cus, int *blocks) {
    int per_cu = 0;
    if (arnoldi_block_capacity(var, &per_cu) != 0 || per_cu < 1) return false;
    const long long slice = 256LL * arnoldi_variant_e(var);
    long long need = 0;
    for (const DevProb &P : H->hprobs) need += (P.ndof + slice - 1) / slice;
    *blocks = static_cast<int>(need);
    return need <= static_cast<long long>(per_cu) * cus;
}

// Choose the register slice per thread (E unknowns) so that every block of
// the fused Arnoldi step is co-resident, and build the block table: the
// variant H->arn_pref when it fits (RAS_KNOB_ARNOLDI, the tuning cache),
// else the first that fits.  Releases an earlier plan's buffers (the device
// is idle first) and the step graph, which records the launch.
int plan_arnoldi(ras_pml_handle *H) {
    if (H->d_ablocks) {
        idle_device(H->device);
        void *old[] = {H->d_ablocks, H->d_part2, H->d_bar, H->d_epoch, H->d_err};
        for (void *q : old) dfree(q);
        H->d_ablocks = nullptr;
        H->d_part2 = nullptr;
        H->d_bar = nullptr;
        H->d_epoch = nullptr;
        H->d_err = nullptr;
    }
    destroy_step_graph(H);
    H->arn_E = 0;
    if (H->flags & RAS_FLAG_UNFUSED_ARNOLDI) return RAS_OK;
    int dev = 0, cus = 0;
    HCHK(H, hipGetDevice(&dev));
    HCHK(H, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    int coop = 0;
    HCHK(H, hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    if (!coop) return RAS_OK;
    for (int k = -1; k < arnoldi_variants(); ++k) {
        const int var = k < 0 ? H->arn_pref : k;
        int need = 0;
        if (var < 0 || !arnoldi_fits(H, var, cus, &need)) continue;
        const int E = arnoldi_variant_e(var);
        const long long slice = 256LL * E;
        std::vector<ArnoldiBlock> tab;
        for (int p = 0; p < H->nprob; ++p) {
            const DevProb &P = H->hprobs[p];
            const int nb = static_cast<int>((P.ndof + slice - 1) / slice);
            const int first = static_cast<int>(tab.size());
            for (int b = 0; b < nb; ++b) {
                ArnoldiBlock B{};
                B.prob = p;
                B.first_blk = first;
                B.nblk = nb;
                B.first = P.dof_off + b * slice;
                B.n = static_cast<int>(std::min<long long>(slice, P.ndof - b * slice));
                tab.push_back(B);
            }
        }
        H->arn_nblocks = static_cast<int>(tab.size());
        RCHK(dalloc(H, &H->d_ablocks, sizeof(ArnoldiBlock) * tab.size()));
        RCHK(dalloc(H, &H->d_part2, sizeof(double2) * 2 * tab.size()));
        const size_t bar_words = 32 * (tab.size() / 16 + 2);   // covers groups of 16 or more
        H->bar_words = bar_words;
        RCHK(dalloc(H, &H->d_bar, sizeof(unsigned long long) * bar_words));
        RCHK(dalloc(H, &H->d_epoch, sizeof(unsigned long long)));
        RCHK(dalloc(H, &H->d_err, sizeof(int)));
        HCHK(H, hipMemcpy(H->d_ablocks, tab.data(), sizeof(ArnoldiBlock) * tab.size(),
                          hipMemcpyHostToDevice));
        HCHK(H, hipMemset(H->d_bar, 0, sizeof(unsigned long long) * bar_words));
        HCHK(H, hipMemset(H->d_epoch, 0, sizeof(unsigned long long)));
        HCHK(H, hipMemset(H->d_err, 0, sizeof(int)));
        H->arn_E = E;
        H->arn_var = var;
        return RAS_OK;
    }
    return RAS_OK;
}

int ensure_krylov(ras_pml_handle *H, int m) {
    if (H->m_alloc >= m) return RAS_OK;
    void *ptrs[] = {H->d_V, H->d_Z, H->d_r, H->d_H, H->d_g, H->d_sn, H->d_y, H->d_cs, H->d_hist};
    if (H->m_alloc > 0) idle_device(H->device);
    for (void *p : ptrs) dfree(p);
    H->d_V = H->d_Z = H->d_r = H->d_H = H->d_g = H->d_sn = H->d_y = nullptr;
    H->d_cs = H->d_hist = nullptr;
    H->m_alloc = 0;
    const long long n = H->ntot;
    const int P = H->nprob;
    RCHK(dalloc(H, &H->d_V, sizeof(double2) * n * (m + 1)));
    RCHK(dalloc(H, &H->d_Z, sizeof(double2) * n * m));
    RCHK(dalloc(H, &H->d_r, sizeof(double2) * n));
    RCHK(dalloc(H, &H->d_H, sizeof(double2) * static_cast<size_t>(P) * (m + 1) * m));
    RCHK(dalloc(H, &H->d_g, sizeof(double2) * static_cast<size_t>(P) * (m + 1)));
    RCHK(dalloc(H, &H->d_sn, sizeof(double2) * static_cast<size_t>(P) * m));
    RCHK(dalloc(H, &H->d_y, sizeof(double2) * static_cast<size_t>(P) * m));
    RCHK(dalloc(H, &H->d_cs, sizeof(double) * static_cast<size_t>(P) * m));
    RCHK(dalloc(H, &H->d_hist, sizeof(double) * static_cast<size_t>(P) * (m + 1)));
    if (!H->d_ks) {
        RCHK(dalloc(H, &H->d_ks, sizeof(KState) * P));
        RCHK(dalloc(H, &H->d_active, sizeof(int) * P));
        RCHK(dalloc(H, &H->d_partials, sizeof(double2) * static_cast<size_t>(P) * kRedBlocksHost));
        RCHK(dalloc(H, &H->d_redout, sizeof(double2) * P));
        RCHK(dalloc(H, &H->d_counters, sizeof(unsigned int) * P));
        HCHK(H, hipMemset(H->d_counters, 0, sizeof(unsigned int) * P));
        HCHK(H, hipHostMalloc(reinterpret_cast<void **>(&H->h_ks), sizeof(KState) * P));
        HCHK(H, hipHostMalloc(reinterpret_cast<void **>(&H->h_err), sizeof(int)));
        *H->h_err = 0;
        HCHK(H, hipHostMalloc(reinterpret_cast<void **>(&H->h_red), sizeof(double2) * P));
    }
    H->m_alloc = m;
    if (H->arn_E < 0) RCHK(plan_arnoldi(H));
    return RAS_OK;
}

int check_handle(ras_pml_handle *H) { return H ? RAS_OK : RAS_EINVAL; }

SolveDispatch solve_dispatch(const ras_pml_handle *H) {
    return SolveDispatch{H->solve_queue ? H->d_queue : nullptr, H->solve_waves};
}

// Band solves of every subdomain: the register-ring kernel for those with
// W <= kMaxW, then the wide kernel for the others.
void launch_solves(const ras_pml_handle *H, bool deep, const int *active, const SolveSrc &src,
                   const SolveDispatch &dsp, hipStream_t st) {
    if (H->nsub_reg > 0)
        launch_band_solve(H->fp64, deep, H->maxW_reg, H->d_probs, H->d_subs, H->d_order,
                          H->nsub_reg, active, src, H->d_F, H->d_ybuf, H->d_xout, dsp, st);
    if (H->nsub_wide > 0)
        launch_band_solve_wide(H->fp64, H->d_probs, H->d_subs, H->d_order + H->nsub_reg,
                               H->nsub_wide, active, src, H->d_F, H->d_ybuf, H->d_xout, st);
}

int do_apply(ras_pml_handle *H, const double2 *v, double2 *z, const int *active, hipStream_t st,
             bool acc = false, bool timed = true) {
    {
        Timer t(H, C_SOLVE, st, timed);
        launch_solves(H, H->solve_deep, active, SolveSrc{v, nullptr, 0}, solve_dispatch(H), st);
    }
    HCHK(H, hipGetLastError());
    {
        Timer t(H, C_SUM, st, timed);
        launch_pou_sum(H->fp64, H->d_probs, H->nprob, H->max_ndof, H->d_subs, active, H->d_pcnt,
                       H->d_pchunk, H->d_pw, H->d_xout, SumDst{z, nullptr, 0}, acc, st);
    }
    HCHK(H, hipGetLastError());
    return RAS_OK;
}

// Deterministic per-problem reduction into H->h_red (synchronises).
int reduce_sync(ras_pml_handle *H, const double2 *a, const double2 *b, int mode, hipStream_t st) {
    launch_reduce(H->d_probs, H->nprob, nullptr, a, b, mode, H->d_redout, H->d_partials,
                  H->d_counters, st);
    HCHK(H, hipGetLastError());
    HCHK(H, hipMemcpyAsync(H->h_red, H->d_redout, sizeof(double2) * H->nprob,
                           hipMemcpyDeviceToHost, st));
    HCHK(H, hipStreamSynchronize(st));
    return RAS_OK;
}

// Steps between the host's looks at the convergence flags, and the steps
// one replay of the step graph runs.
constexpr int kSyncSteps = 8;

// The kernels of one FGMRES step (Section 4.1: one application of B^{-1},
// then the Arnoldi process with modified Gram-Schmidt, then the Givens
// update) for every problem still in its cycle.  The band solve, the PoU sum,
// the fused Arnoldi step and the Givens update read the step index on the
// device (each problem's step count kp; the Arnoldi barrier epoch from its
// device word), so the same launches, with the same arguments, serve every
// step: enqueued one by one, or recorded once into a graph and replayed.
// The one-launch-per-projection path (arn_E == 0) needs the host's step
// index j and is enqueued only.  timed: per-launch events (RAS_FLAG_TIMING).
int enqueue_step(ras_pml_handle *H, int j, int m, hipStream_t st, bool timed) {
    const long long n = H->ntot;
    const int P = H->nprob;
    {
        Timer t(H, C_SOLVE, st, timed);
        launch_solves(H, H->solve_deep, H->d_active, SolveSrc{H->d_V, H->d_ks, n},
                      solve_dispatch(H), st);
    }
    HCHK(H, hipGetLastError());
    {
        Timer t(H, C_SUM, st, timed);
        launch_pou_sum(H->fp64, H->d_probs, P, H->max_ndof, H->d_subs, H->d_active, H->d_pcnt,
                       H->d_pchunk, H->d_pw, H->d_xout, SumDst{H->d_Z, H->d_ks, n}, false, st);
    }
    HCHK(H, hipGetLastError());
    if (H->arn_E > 0) {
        Timer t(H, C_MGS, st, timed);
        const hipError_t e = launch_arnoldi(H->arn_var, H->arn_nblocks, H->d_probs, H->d_ks,
                                            H->d_ablocks, H->d_coef, n, H->d_Z, H->d_V, m, H->d_H,
                                            H->d_part2, H->d_bar, H->d_epoch, H->d_err, P, st);
        if (e != hipSuccess) {
            H->last_error = std::string("cooperative Arnoldi launch: ") + hipGetErrorString(e);
            return RAS_EHIP;
        }
    } else {
        double2 *Vj1 = H->d_V + static_cast<long long>(j + 1) * n;
        const double2 *Zj = H->d_Z + static_cast<long long>(j) * n;
        {
            Timer t(H, C_SPMV, st, timed);
            launch_spmv(H->d_probs, P, H->max_ndof, H->d_active, H->d_coef, n, Zj, nullptr, Vj1,
                        st);
        }
        HCHK(H, hipGetLastError());
        Timer t(H, C_MGS, st, timed);
        for (int i = 0; i <= j; ++i)
            launch_mgs(H->d_probs, P, H->d_ks, Vj1, H->d_V, n, j, i, i == 0 ? 0 : 1, m, H->d_H,
                       H->d_partials, H->d_counters, st);
        launch_mgs(H->d_probs, P, H->d_ks, Vj1, H->d_V, n, j, j + 1, 2, m, H->d_H, H->d_partials,
                   H->d_counters, st);
        launch_normalize(H->d_probs, P, H->max_ndof, H->d_ks, Vj1, j, m, H->d_H, st);
    }
    HCHK(H, hipGetLastError());
    {
        Timer t(H, C_GIVENS, st, timed);
        launch_givens(H->d_ks, P, m, H->d_H, H->d_cs, H->d_sn, H->d_g, H->d_hist, H->d_active, st);
    }
    HCHK(H, hipGetLastError());
    return RAS_OK;
}

void destroy_step_graph(ras_pml_handle *H) {
    if (H->step_exec) (void)hipGraphExecDestroy(H->step_exec);
    if (H->step_graph) (void)hipGraphDestroy(H->step_graph);
    H->step_exec = nullptr;
    H->step_graph = nullptr;
    H->graph_m = 0;
    H->graph_V = nullptr;
}

// The graph of kSyncSteps FGMRES steps (fused Arnoldi path): recorded by
// stream capture on the handle's own stream (a caller's stream may be the
// legacy default stream, which cannot capture) the first time a solve needs
// it, and again when the restart length or the Krylov workspace changes
// (their buffers are part of the recorded launches).  No allocation, copy or
// memset is recorded: only the kernels of enqueue_step.
int ensure_step_graph(ras_pml_handle *H, int m) {
    if (H->step_exec && H->graph_m == m && H->graph_V == H->d_V) return RAS_OK;
    destroy_step_graph(H);
    if (!H->cap_stream) HCHK(H, hipStreamCreateWithFlags(&H->cap_stream, hipStreamNonBlocking));
    HCHK(H, hipStreamBeginCapture(H->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = RAS_OK;
    for (int s = 0; s < kSyncSteps && rc == RAS_OK; ++s) rc = enqueue_step(H, -1, m, H->cap_stream, false);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(H->cap_stream, &g);
    if (rc != RAS_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        if (rc == RAS_OK) {
            H->last_error = std::string("capture of the GMRES step graph: ") + hipGetErrorString(e);
            rc = RAS_EHIP;
        }
        return rc;
    }
    hipGraphExec_t x = nullptr;
    const hipError_t e2 = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e2 != hipSuccess) {
        (void)hipGraphDestroy(g);
        H->last_error = std::string("instantiation of the GMRES step graph: ") +
                        hipGetErrorString(e2);
        return RAS_EHIP;
    }
    H->step_graph = g;
    H->step_exec = x;
    H->graph_m = m;
    H->graph_V = H->d_V;
    return RAS_OK;
}

// rtol: one tolerance per problem.
int gmres_impl(ras_pml_handle *H, const double2 *b, double2 *x, const double *rtol, int m, int maxit,
               int *iters, double *relres, double *hist, hipStream_t st) {
    const int P = H->nprob;
    RCHK(ensure_krylov(H, m));
    // the barrier-timeout flag of the fused Arnoldi step reports this call
    // only; after a timeout the counters and the epoch start again from zero
    if (H->arn_E > 0) {
        if (H->bar_reset) {
            HCHK(H, hipMemsetAsync(H->d_bar, 0, sizeof(unsigned long long) * H->bar_words, st));
            HCHK(H, hipMemsetAsync(H->d_epoch, 0, sizeof(unsigned long long), st));
            H->bar_reset = false;
        }
        HCHK(H, hipMemsetAsync(H->d_err, 0, sizeof(int), st));
    }
    const bool graph = H->graph_steps && H->arn_E > 0 && !(H->flags & RAS_FLAG_TIMING);
    if (graph) RCHK(ensure_step_graph(H, m));
    H->res_iters.assign(P, 0);
    H->res_relres.assign(P, 0.0);
    H->res_conv.assign(P, 0);
    std::vector<double> bnorm(P), beta(P);
    std::vector<int> need(P, 0);
    RCHK(reduce_sync(H, b, nullptr, 0, st));
    for (int p = 0; p < P; ++p) {
        bnorm[p] = std::sqrt(H->h_red[p].x);
        if (!std::isfinite(bnorm[p])) {
            H->last_error = "right-hand side is not finite";
            return RAS_ENONFINITE;
        }
        if (bnorm[p] == 0.0) {
            const DevProb &D = H->hprobs[p];
            HCHK(H, hipMemsetAsync(x + D.dof_off, 0, sizeof(double2) * D.ndof, st));
        }
    }
    launch_spmv(H->d_probs, P, H->max_ndof, nullptr, H->d_coef, H->ntot, x, b, H->d_r, st);
    HCHK(H, hipGetLastError());
    RCHK(reduce_sync(H, H->d_r, nullptr, 0, st));
    int nneed = 0;
    for (int p = 0; p < P; ++p) {
        beta[p] = std::sqrt(H->h_red[p].x);
        if (!std::isfinite(beta[p])) {
            H->last_error = "initial residual is not finite";
            return RAS_ENONFINITE;
        }
        need[p] = (bnorm[p] > 0.0 && beta[p] > rtol[p] * bnorm[p]) ? 1 : 0;
        H->res_relres[p] = bnorm[p] > 0.0 ? beta[p] / bnorm[p] : 0.0;
        H->res_conv[p] = need[p] ? 0 : 1;
        nneed += need[p];
    }
    int total = 0;
    int hist_n = 0;
    if (hist) hist[hist_n++] = *std::max_element(H->res_relres.begin(), H->res_relres.end());
    std::vector<double2> g0(static_cast<size_t>(P) * (m + 1));
    bool broke = false;
    while (nneed > 0 && total < maxit) {
        const int mc = std::min(m, maxit - total);
        for (int p = 0; p < P; ++p) {
            KState &K = H->h_ks[p];
            K.bnorm = bnorm[p];
            K.beta = beta[p];
            K.est = beta[p];
            K.rtol = rtol[p];
            K.kp = 0;
            K.in_cycle = need[p];
            K.breakdown = 0;
            K.mc = mc;
            for (int i = 0; i <= m; ++i) g0[static_cast<size_t>(p) * (m + 1) + i] = make_double2(0, 0);
            g0[static_cast<size_t>(p) * (m + 1)] = make_double2(beta[p], 0.0);
        }
        HCHK(H, hipMemcpyAsync(H->d_ks, H->h_ks, sizeof(KState) * P, hipMemcpyHostToDevice, st));
        HCHK(H, hipMemcpyAsync(H->d_active, need.data(), sizeof(int) * P, hipMemcpyHostToDevice, st));
        HCHK(H, hipMemcpyAsync(H->d_g, g0.data(), sizeof(double2) * g0.size(), hipMemcpyHostToDevice,
                               st));
        launch_start_cycle(H->d_probs, P, H->max_ndof, H->d_ks, H->d_r, H->d_V, st);
        HCHK(H, hipGetLastError());
        // Steps are enqueued without waiting: the Givens kernel clears a
        // problem's in-cycle flag (and its active flag, read by the next
        // step's launches) on convergence, breakdown or the cycle's end (mc
        // steps), and every later launch of the cycle skips that problem (the
        // Arnoldi launch as a whole once no problem is left).  The host looks
        // at the flags every kSyncSteps steps -- enqueued one by one, or one
        // replay of the step graph -- and stops when none is set.
        int enqueued = 0;
        for (int j0 = 0; j0 < mc; j0 += kSyncSteps) {
            if (graph) {
                HCHK(H, hipGraphLaunch(H->step_exec, st));
                enqueued += kSyncSteps;
            } else {
                const int j1 = std::min(mc, j0 + kSyncSteps);
                for (int j = j0; j < j1; ++j) {
                    RCHK(enqueue_step(H, j, m, st, true));
                    ++enqueued;
                }
            }
            HCHK(H, hipMemcpyAsync(H->h_ks, H->d_ks, sizeof(KState) * P, hipMemcpyDeviceToHost, st));
            if (H->arn_E > 0)
                HCHK(H, hipMemcpyAsync(H->h_err, H->d_err, sizeof(int), hipMemcpyDeviceToHost, st));
            HCHK(H, hipStreamSynchronize(st));
            if (H->arn_E > 0 && *H->h_err != 0) {
                H->bar_reset = true;
                H->last_error = "grid barrier of the fused Arnoldi step timed out";
                return RAS_EHIP;
            }
            int still = 0;
            for (int p = 0; p < P; ++p) still += H->h_ks[p].in_cycle;
            if (still == 0) break;
        }
        // steps taken in this cycle (per problem: kp) and the estimate history
        {
            std::vector<double> eh(static_cast<size_t>(P) * (m + 1));
            HCHK(H, hipMemcpyAsync(eh.data(), H->d_hist, sizeof(double) * eh.size(),
                                   hipMemcpyDeviceToHost, st));
            HCHK(H, hipStreamSynchronize(st));
            int steps = 0;
            for (int p = 0; p < P; ++p)
                if (need[p]) {
                    H->res_iters[p] += H->h_ks[p].kp;
                    steps = std::max(steps, H->h_ks[p].kp);
                }
            for (int t = 0; t < steps; ++t) {
                double worst = 0.0;
                for (int p = 0; p < P; ++p)
                    if (need[p] && t < H->h_ks[p].kp)
                        worst = std::max(worst, eh[static_cast<size_t>(p) * (m + 1) + t]);
                if (hist) hist[hist_n++] = worst;
            }
            total += steps;
            H->skipped_steps += enqueued - steps;
        }
        // x += Z y for every problem that took steps
        launch_solve_y(H->d_ks, P, m, H->d_H, H->d_g, H->d_y, st);
        HCHK(H, hipMemcpyAsync(H->d_active, need.data(), sizeof(int) * P, hipMemcpyHostToDevice, st));
        launch_update_x(H->d_probs, P, H->max_ndof, H->d_ks, H->d_active, m, H->d_Z, H->ntot,
                        H->d_y, x, st);
        HCHK(H, hipGetLastError());
        launch_spmv(H->d_probs, P, H->max_ndof, nullptr, H->d_coef, H->ntot, x, b, H->d_r, st);
        HCHK(H, hipGetLastError());
        RCHK(reduce_sync(H, H->d_r, nullptr, 0, st));
        nneed = 0;
        for (int p = 0; p < P; ++p) {
            if (!need[p]) continue;
            beta[p] = std::sqrt(H->h_red[p].x);
            if (!std::isfinite(beta[p])) {
                H->last_error = "iterate is not finite";
                return RAS_ENONFINITE;
            }
            H->res_relres[p] = beta[p] / bnorm[p];
            if (beta[p] <= rtol[p] * bnorm[p]) {
                need[p] = 0;
                H->res_conv[p] = 1;
            } else if (H->h_ks[p].breakdown) {
                need[p] = 0;
                broke = true;
            }
            nneed += need[p];
        }
    }
    if (iters) *iters = total;
    if (relres) *relres = *std::max_element(H->res_relres.begin(), H->res_relres.end());
    for (int p = 0; p < P; ++p)
        if (!H->res_conv[p]) {
            if (broke) {
                H->last_error = "Arnoldi breakdown before the tolerance was reached";
                return RAS_EBREAKDOWN;
            }
            H->last_error = "maximum number of iterations reached";
            return RAS_ENOTCONV;
        }
    return RAS_OK;
}

// Buffers of one fixed-point solve.  ras_pml_richardson takes them from
// the handle (allocated on first use), ras_pml_richardson_noalloc from the
// library's static scratch array; the host arrays hold nprob values.
struct RichWork {
    double2 *r;               // residual b - A x (all unknowns)
    int *active;              // per problem: 1 while it iterates
    RState *rs;               // per problem: state of the iteration
    double *rhist;            // per problem: maxit + 1 relative residuals
    double2 *redout;          // per problem: reduction result
    double2 *partials;        // per problem: kRedBlocksHost partial sums
    unsigned int *counters;   // per problem: arrivals (0 between reductions)
    RState *h_rs;             // host: rs
    double2 *h_red;           // host: redout
    int *h_need;              // host: active
    double *h_bnorm, *h_rel0; // host: ||b||, relative residual of x0
    bool timed;               // record timing events (RAS_FLAG_TIMING)
};

// Deterministic per-problem reduction into W.h_red (synchronises).
int reduce_sync_w(ras_pml_handle *H, const RichWork &W, const double2 *a, hipStream_t st) {
    launch_reduce(H->d_probs, H->nprob, nullptr, a, nullptr, 0, W.redout, W.partials, W.counters,
                  st);
    HCHK(H, hipGetLastError());
    HCHK(H, hipMemcpyAsync(W.h_red, W.redout, sizeof(double2) * H->nprob, hipMemcpyDeviceToHost,
                           st));
    HCHK(H, hipStreamSynchronize(st));
    return RAS_OK;
}

// Algorithm 1 as an iteration: x <- x + B^{-1} (b - A x) for every problem
// not yet converged.  The correction is summed straight into x (the PoU sum
// in accumulate mode), so a step is one batched solve, one sum, one
// residual and one reduction.  The stopping test runs on the device
// (k_rich_update clears a finished problem's active flag, which every later
// launch reads); the host enqueues steps ahead and looks at the flags every
// kSyncSteps steps.  Allocates nothing (W holds every buffer).
int richardson_impl(ras_pml_handle *H, const RichWork &W, const double2 *b, double2 *x,
                    double rtol, int maxit, int *iters, double *relres, double *hist,
                    hipStream_t st) {
    const int P = H->nprob;
    H->res_iters.assign(P, 0);
    H->res_relres.assign(P, 0.0);
    H->res_conv.assign(P, 0);
    double *bnorm = W.h_bnorm, *rel0 = W.h_rel0;
    int *need = W.h_need;
    RCHK(reduce_sync_w(H, W, b, st));
    for (int p = 0; p < P; ++p) {
        bnorm[p] = std::sqrt(W.h_red[p].x);
        if (!std::isfinite(bnorm[p])) {
            H->last_error = "right-hand side is not finite";
            return RAS_ENONFINITE;
        }
        if (bnorm[p] == 0.0) {
            const DevProb &D = H->hprobs[p];
            HCHK(H, hipMemsetAsync(x + D.dof_off, 0, sizeof(double2) * D.ndof, st));
        }
    }
    launch_spmv(H->d_probs, P, H->max_ndof, nullptr, H->d_coef, H->ntot, x, b, W.r, st);
    HCHK(H, hipGetLastError());
    RCHK(reduce_sync_w(H, W, W.r, st));
    int nneed = 0;
    for (int p = 0; p < P; ++p) {
        const double beta = std::sqrt(W.h_red[p].x);
        if (!std::isfinite(beta)) {
            H->last_error = "initial residual is not finite";
            return RAS_ENONFINITE;
        }
        rel0[p] = bnorm[p] > 0.0 ? beta / bnorm[p] : 0.0;
        need[p] = (bnorm[p] > 0.0 && beta > rtol * bnorm[p] && maxit > 0) ? 1 : 0;
        nneed += need[p];
        W.h_rs[p] = RState{bnorm[p] > 0.0 ? bnorm[p] : 1.0, rel0[p], 0, 0};
    }
    HCHK(H, hipMemcpyAsync(W.rs, W.h_rs, sizeof(RState) * P, hipMemcpyHostToDevice, st));
    HCHK(H, hipMemcpyAsync(W.active, need, sizeof(int) * P, hipMemcpyHostToDevice, st));
    for (int it = 1; nneed > 0 && it <= maxit; ++it) {
        RCHK(do_apply(H, W.r, x, W.active, st, true, W.timed));
        launch_spmv(H->d_probs, P, H->max_ndof, W.active, H->d_coef, H->ntot, x, b, W.r, st);
        launch_reduce(H->d_probs, P, nullptr, W.r, nullptr, 0, W.redout, W.partials, W.counters,
                      st);
        launch_rich_update(W.rs, W.active, W.redout, W.rhist, P, maxit, rtol, st);
        HCHK(H, hipGetLastError());
        if (it % kSyncSteps != 0 && it != maxit) continue;
        HCHK(H, hipMemcpyAsync(need, W.active, sizeof(int) * P, hipMemcpyDeviceToHost, st));
        HCHK(H, hipStreamSynchronize(st));
        nneed = 0;
        for (int p = 0; p < P; ++p) nneed += need[p];
    }
    // per-problem outcome and histories
    HCHK(H, hipMemcpyAsync(W.h_rs, W.rs, sizeof(RState) * P, hipMemcpyDeviceToHost, st));
    int steps = 0;
    HCHK(H, hipStreamSynchronize(st));
    bool nonfinite = false;
    for (int p = 0; p < P; ++p) {
        const RState &R = W.h_rs[p];
        H->res_iters[p] = R.iters;
        H->res_relres[p] = R.nonfinite ? HUGE_VAL : R.relres;
        H->res_conv[p] = (!R.nonfinite && R.relres <= rtol) || bnorm[p] == 0.0 ? 1 : 0;
        nonfinite = nonfinite || R.nonfinite;
        steps = std::max(steps, R.iters);
    }
    if (hist) {
        // the worst problem after every step (a problem that stopped keeps
        // its last value), read back one problem and one chunk at a time
        for (int t = 0; t <= steps; ++t) hist[t] = 0.0;
        constexpr int kChunk = 512;
        double buf[kChunk];
        for (int p = 0; p < P; ++p) {
            const int ip = H->res_iters[p];
            hist[0] = std::max(hist[0], rel0[p]);
            for (int t0 = 1; t0 <= ip; t0 += kChunk) {
                const int cnt = std::min(kChunk, ip - t0 + 1);
                HCHK(H, hipMemcpy(buf, W.rhist + static_cast<size_t>(p) * (maxit + 1) + t0,
                                  sizeof(double) * cnt, hipMemcpyDeviceToHost));
                for (int u = 0; u < cnt; ++u) hist[t0 + u] = std::max(hist[t0 + u], buf[u]);
            }
            if (ip < steps) {
                double lastv = rel0[p];
                if (ip > 0)
                    HCHK(H, hipMemcpy(&lastv, W.rhist + static_cast<size_t>(p) * (maxit + 1) + ip,
                                      sizeof(double), hipMemcpyDeviceToHost));
                for (int t = ip + 1; t <= steps; ++t) hist[t] = std::max(hist[t], lastv);
            }
        }
    }
    if (iters) *iters = steps;
    if (relres) *relres = *std::max_element(H->res_relres.begin(), H->res_relres.end());
    if (nonfinite) {                   // a diverging iteration overflows
        H->last_error = "iterate is not finite";
        return RAS_ENONFINITE;
    }
    for (int p = 0; p < P; ++p)
        if (!H->res_conv[p]) {
            H->last_error = "maximum number of iterations reached";
            return RAS_ENOTCONV;
        }
    return RAS_OK;
}

// ras_pml_richardson's buffers: the handle's own, allocated on first use
// (the history grows with maxit).
int rich_work_handle(ras_pml_handle *H, int maxit, RichWork &W) {
    const int P = H->nprob;
    RCHK(ensure_krylov(H, 1));
    if (!H->d_rs) {
        RCHK(dalloc(H, &H->d_rs, sizeof(RState) * P));
        HCHK(H, hipHostMalloc(reinterpret_cast<void **>(&H->h_rs), sizeof(RState) * P));
    }
    if (H->rhist_cap < maxit) {
        if (H->d_rhist) idle_device(H->device);
        dfree(H->d_rhist);
        H->d_rhist = nullptr;
        H->rhist_cap = -1;
        RCHK(dalloc(H, &H->d_rhist, sizeof(double) * static_cast<size_t>(P) * (maxit + 1)));
        H->rhist_cap = maxit;
    }
    W.r = H->d_r;
    W.active = H->d_active;
    W.rs = H->d_rs;
    W.rhist = H->d_rhist;
    W.redout = H->d_redout;
    W.partials = H->d_partials;
    W.counters = H->d_counters;
    W.h_rs = H->h_rs;
    W.h_red = H->h_red;
    W.timed = true;
    return RAS_OK;
}

// ---- ras_pml_richardson_noalloc: every buffer of the solve in one static
// device array (each device that runs it holds its own copy until the
// process ends).  Host code never uses the array's name as an address: its
// device address comes from hipGetSymbolAddress, once per device, with that
// device current.
constexpr size_t kScratchBytes = static_cast<size_t>(64) << 20;
constexpr int kNoAllocMaxProb = 64;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
unsigned char *g_scratch_dev[kMaxDevices] = {};

int scratch_address(ras_pml_handle *H, unsigned char **out) {
    *out = nullptr;
    if (H->device < 0 || H->device >= kMaxDevices) {
        H->last_error = "device index beyond the scratch table";
        return RAS_EINVAL;
    }
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_dev[H->device]) {
        int cur = -1;
        HCHK(H, hipGetDevice(&cur));
        if (cur != H->device) HCHK(H, hipSetDevice(H->device));
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != H->device) (void)hipSetDevice(cur);
        if (e != hipSuccess || ptr == nullptr) {
            H->last_error = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return RAS_EHIP;
        }
        g_scratch_dev[H->device] = static_cast<unsigned char *>(ptr);
    }
    *out = g_scratch_dev[H->device];
    return RAS_OK;
}

// Lays the buffers of one solve out in the scratch array (256-byte aligned
// pieces); RAS_EINVAL when they do not fit.
int rich_work_scratch(ras_pml_handle *H, unsigned char *base, int maxit, RichWork &W) {
    const size_t P = static_cast<size_t>(H->nprob);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~static_cast<size_t>(255);
        return base + o;
    };
    W.r = reinterpret_cast<double2 *>(take(sizeof(double2) * static_cast<size_t>(H->ntot)));
    W.partials = reinterpret_cast<double2 *>(take(sizeof(double2) * P * kRedBlocksHost));
    W.redout = reinterpret_cast<double2 *>(take(sizeof(double2) * P));
    W.counters = reinterpret_cast<unsigned int *>(take(sizeof(unsigned int) * P));
    W.rs = reinterpret_cast<RState *>(take(sizeof(RState) * P));
    W.active = reinterpret_cast<int *>(take(sizeof(int) * P));
    W.rhist = reinterpret_cast<double *>(take(sizeof(double) * P * (static_cast<size_t>(maxit) + 1)));
    if (off > kScratchBytes) {
        char buf[200];
        std::snprintf(buf, sizeof buf,
                      "the fixed-point solve needs %zu bytes of scratch (%lld unknowns, %d "
                      "problems, maxit %d); the static scratch holds %zu",
                      off, H->ntot, H->nprob, maxit, kScratchBytes);
        H->last_error = buf;
        return RAS_EINVAL;
    }
    return RAS_OK;
}

int setup_common(int nprob, const double *k, const double *h, const int *grid, const int *subs,
                 const int *overlap, const int *pml, const ras_pml_opts *opts, void *stream,
                 ras_pml_t *out) {
    if (out == nullptr) {
        g_plan_error = "out is NULL";
        return RAS_EINVAL;
    }
    *out = nullptr;
    if (nprob < 1 || !k || !h || !grid || !subs || !overlap || !pml) {
        g_plan_error = "invalid problem arrays";
        return RAS_EINVAL;
    }
    ras_pml_opts o;
    ras_pml_default_opts(&o);
    if (opts) o = *opts;
    std::unique_ptr<ras_pml_handle> H(new (std::nothrow) ras_pml_handle());
    if (!H) return RAS_ENOMEM;
    H->plans.resize(nprob);
    // per-problem results: sized here so that no solve allocates host memory
    H->res_iters.reserve(nprob);
    H->res_relres.reserve(nprob);
    H->res_conv.reserve(nprob);
    for (int p = 0; p < nprob; ++p) {
        std::string err;
        int rc = plan_problem(k[p], h[p], grid + 2 * p, subs + 2 * p, overlap[p], pml[p], o,
                              H->plans[p], err);
        if (rc != RAS_OK) {
            g_plan_error = nprob > 1 ? "problem " + std::to_string(p) + ": " + err : err;
            return rc;
        }
    }
    H->fp64 = o.precision == RAS_FP64;
    H->flags = o.flags;
    H->graph_steps = (o.flags & RAS_FLAG_GRAPH_STEPS) != 0;
    if (o.tune_cache) H->tune_cache = o.tune_cache;
    if (hipGetDevice(&H->device) != hipSuccess) {
        g_plan_error = "no HIP device";
        return RAS_EHIP;
    }
    int rc = build(H.get(), as_stream(stream));
    if (rc != RAS_OK) {
        g_plan_error = H->last_error;
        return rc;
    }
    *out = H.release();
    return RAS_OK;
}

// ---- tuning cache: a flat JSON object {"key": 0 | 1, ...}
std::string device_arch() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return "unknown";
    std::string a(prop.gcnArchName);
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

int pow2_bucket(int n) {
    int b = 1;
    while (b < n) b <<= 1;
    return b;
}

std::string lu_key(const ras_pml_handle *H, const std::array<int, 5> &g) {
    return H->arch + (H->fp64 ? "/c128" : "/c64") + "/ldlt/tiles=" + std::to_string(g[0]) +
           "/count=" + std::to_string(pow2_bucket(g[2]));
}

std::string arnoldi_key(const ras_pml_handle *H) {
    return H->arch + "/c128/arnoldi/nprob=" + std::to_string(H->nprob) + "/ndof=" +
           std::to_string(pow2_bucket(static_cast<int>(std::min<long long>(H->ntot, 1LL << 30))));
}

std::string queue_key(const ras_pml_handle *H) {
    return H->arch + (H->fp64 ? "/c128" : "/c64") + "/solve_queue/maxW=" +
           std::to_string(H->maxW) + "/nsub=" + std::to_string(pow2_bucket(H->nsub));
}

std::string solve_key(const ras_pml_handle *H) {
    return H->arch + (H->fp64 ? "/c128" : "/c64") + "/solve/maxW=" + std::to_string(H->maxW) +
           "/nsub=" + std::to_string(pow2_bucket(H->nsub));
}

// Reads "key": integer pairs; a missing or unreadable file is an empty cache.
std::vector<std::pair<std::string, int>> read_cache(const char *path) {
    std::vector<std::pair<std::string, int>> out;
    FILE *f = path ? std::fopen(path, "rb") : nullptr;
    if (!f) return out;
    std::string txt;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, got);
    std::fclose(f);
    size_t i = 0;
    while ((i = txt.find('"', i)) != std::string::npos) {
        const size_t j = txt.find('"', i + 1);
        if (j == std::string::npos) break;
        std::string key = txt.substr(i + 1, j - i - 1);
        size_t k = txt.find(':', j);
        if (k == std::string::npos) break;
        char *end = nullptr;
        const long v = std::strtol(txt.c_str() + k + 1, &end, 10);
        if (end != txt.c_str() + k + 1) out.emplace_back(key, static_cast<int>(v));
        i = end ? static_cast<size_t>(end - txt.c_str()) : k + 1;
    }
    return out;
}

int cache_lookup(const std::vector<std::pair<std::string, int>> &c, const std::string &key,
                 int fallback) {
    for (const auto &kv : c)
        if (kv.first == key) return kv.second;
    return fallback;
}

bool write_cache(const char *path, std::vector<std::pair<std::string, int>> c) {
    std::sort(c.begin(), c.end());
    std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return false;
    std::fprintf(f, "{\n");
    for (size_t i = 0; i < c.size(); ++i)
        std::fprintf(f, "  \"%s\": %d%s\n", c[i].first.c_str(), c[i].second,
                     i + 1 < c.size() ? "," : "");
    std::fprintf(f, "}\n");
    const bool ok = std::fclose(f) == 0;
    return ok && std::rename(tmp.c_str(), path) == 0;
}

void cache_set(std::vector<std::pair<std::string, int>> &c, const std::string &key, int v) {
    for (auto &kv : c)
        if (kv.first == key) {
            kv.second = v;
            return;
        }
    c.emplace_back(key, v);
}

// Choices from the cache (setup): classes and configurations it does not
// know keep their defaults.
void apply_cache(ras_pml_handle *H, const char *path) {
    if (!path) return;
    const auto c = read_cache(path);
    if (c.empty()) return;
    if (H->arch.empty()) H->arch = device_arch();
    for (auto &g : H->lu_groups) {
        const int v = cache_lookup(c, lu_key(H, g), g[3]);
        if (v >= 0 && v < LU_NVARIANTS) g[3] = v;
    }
    H->solve_deep = cache_lookup(c, solve_key(H), H->solve_deep) != 0;
    H->solve_queue = cache_lookup(c, queue_key(H), H->solve_queue) != 0;
    const int av = cache_lookup(c, arnoldi_key(H), H->arn_pref);
    if (av >= -1 && av < arnoldi_variants()) H->arn_pref = av;
}

}  // namespace

// ====================================================================== ABI
extern "C" {

void ras_pml_default_opts(ras_pml_opts *o) {
    if (!o) return;
    o->sigma = 0.0;
    o->global_pml = -1;
    o->bc = RAS_BC_IMP;
    o->pou = RAS_POU_LINEAR;
    o->precision = RAS_MIXED;
    o->flags = 0;
    o->tune_cache = nullptr;
    o->width_c_delta = 1.0 / 6.0;
    o->width_c_kappa = 0.5;
    o->width_k0 = 150.0;
}

const char *ras_pml_plan_error(void) { return g_plan_error.c_str(); }

int ras_pml_width_rule(double k, double h, double C, double k0, int *cells) {
    if (cells == nullptr) {
        g_plan_error = "cells is NULL";
        return RAS_EINVAL;
    }
    return width_rule_cells(k, h, C, k0, *cells, g_plan_error);
}

int ras_pml_plan(double k, double h, const int grid[2], const int subdomains[2], int overlap,
                 int pml_width, const ras_pml_opts *opts, int *nsub, int *desc, int desc_cap) {
    try {
        ras_pml_opts o;
        ras_pml_default_opts(&o);
        if (opts) o = *opts;
        PlanProblem pl;
        std::string err;
        int rc = plan_problem(k, h, grid, subdomains, overlap, pml_width, o, pl, err);
        if (rc != RAS_OK) {
            g_plan_error = err;
            return rc;
        }
        const int ns = static_cast<int>(pl.subs.size());
        if (nsub) *nsub = ns;
        if (desc) {
            if (desc_cap < ns) {
                g_plan_error = "desc_cap too small";
                return RAS_EINVAL;
            }
            for (int s = 0; s < ns; ++s) desc_ints(pl.subs[s], pl, desc + s * RAS_DESC_INTS);
        }
        return RAS_OK;
    } catch (const std::exception &e) {
        g_plan_error = e.what();
        return RAS_ENOMEM;
    }
}

int ras_pml_setup(double k, double h, const int grid[2], const int subdomains[2], int overlap,
                  int pml_width, const ras_pml_opts *opts, void *stream, ras_pml_t *out) {
    try {
        return setup_common(1, &k, &h, grid, subdomains, &overlap, &pml_width, opts, stream, out);
    } catch (const std::exception &e) {
        g_plan_error = e.what();
        return RAS_ENOMEM;
    }
}

int ras_pml_setup_batch(int nprob, const double *k, const double *h, const int *grid,
                        const int *subdomains, const int *overlap, const int *pml_width,
                        const ras_pml_opts *opts, void *stream, ras_pml_t *out) {
    try {
        return setup_common(nprob, k, h, grid, subdomains, overlap, pml_width, opts, stream, out);
    } catch (const std::exception &e) {
        g_plan_error = e.what();
        return RAS_ENOMEM;
    }
}

void ras_pml_destroy(ras_pml_t H) { delete H; }

int ras_pml_num_dofs(ras_pml_t H, long long *n) {
    if (!H || !n) return RAS_EINVAL;
    *n = H->ntot;
    return RAS_OK;
}

int ras_pml_num_problems(ras_pml_t H, int *nprob) {
    if (!H || !nprob) return RAS_EINVAL;
    *nprob = H->nprob;
    return RAS_OK;
}

int ras_pml_problem_offset(ras_pml_t H, int p, long long *off, long long *n) {
    if (!H || p < 0 || p >= H->nprob) return RAS_EINVAL;
    if (off) *off = H->hprobs[p].dof_off;
    if (n) *n = H->hprobs[p].ndof;
    return RAS_OK;
}

int ras_pml_num_subdomains(ras_pml_t H, int *nsub) {
    if (!H || !nsub) return RAS_EINVAL;
    *nsub = H->nsub;
    return RAS_OK;
}

int ras_pml_num_local(ras_pml_t H, long long *nloc) {
    if (!H || !nloc) return RAS_EINVAL;
    *nloc = H->nloc;
    return RAS_OK;
}

int ras_pml_subdomain_desc(ras_pml_t H, int *desc, int desc_cap) {
    if (!H || !desc || desc_cap < H->nsub) return RAS_EINVAL;
    for (int s = 0; s < H->nsub; ++s)
        desc_ints(H->hsubs[s], H->plans[H->hsubs[s].prob], desc + s * RAS_DESC_INTS);
    return RAS_OK;
}

int ras_pml_rhs(ras_pml_t H, const void *f, void *b, void *stream) {
    if (!H || !f || !b) return RAS_EINVAL;
    launch_rhs(H->d_probs, H->nprob, H->max_ndof, static_cast<const double2 *>(f),
               static_cast<double2 *>(b), as_stream(stream));
    HCHK(H, hipGetLastError());
    return RAS_OK;
}

int ras_pml_spmv(ras_pml_t H, const void *x, void *y, void *stream) {
    if (!H || !x || !y || x == y) {
        if (H) H->last_error = "invalid vectors (x and y must be distinct, non-NULL)";
        return RAS_EINVAL;
    }
    hipStream_t st = as_stream(stream);
    {
        Timer t(H, C_SPMV, st);
        launch_spmv(H->d_probs, H->nprob, H->max_ndof, nullptr, H->d_coef, H->ntot,
                    static_cast<const double2 *>(x), nullptr, static_cast<double2 *>(y), st);
    }
    HCHK(H, hipGetLastError());
    return RAS_OK;
}

int ras_pml_apply(ras_pml_t H, const void *v, void *z, void *stream) {
    if (!H || !v || !z || v == z) {
        if (H) H->last_error = "invalid vectors (v and z must be distinct, non-NULL)";
        return RAS_EINVAL;
    }
    return do_apply(H, static_cast<const double2 *>(v), static_cast<double2 *>(z), nullptr,
                    as_stream(stream));
}

int ras_pml_local_solve(ras_pml_t H, const void *v, void *xloc, void *stream) {
    if (!H || !v) return RAS_EINVAL;
    hipStream_t st = as_stream(stream);
    {
        Timer t(H, C_SOLVE, st);
        launch_solves(H, H->solve_deep, nullptr,
                      SolveSrc{static_cast<const double2 *>(v), nullptr, 0}, solve_dispatch(H), st);
    }
    HCHK(H, hipGetLastError());
    if (xloc == nullptr) return RAS_OK;        // the solves alone (timing)
    launch_export_local(H->fp64, H->d_subs, H->nsub, H->max_n, H->d_xout,
                        static_cast<double2 *>(xloc), st);
    HCHK(H, hipGetLastError());
    return RAS_OK;
}

int gmres_solve(ras_pml_t H, const void *b, void *x, double rtol, int restart, int maxit,
                int *iters, double *relres, double *hist, void *stream) {
    if (!H) return RAS_EINVAL;
    if (!b || !x || b == x || !(rtol > 0.0) || restart < 1 || maxit < 0) {
        H->last_error = "invalid gmres arguments";
        return RAS_EINVAL;
    }
    try {
        const std::vector<double> r(H->nprob, rtol);
        return gmres_impl(H, static_cast<const double2 *>(b), static_cast<double2 *>(x), r.data(),
                          restart, maxit, iters, relres, hist, as_stream(stream));
    } catch (const std::exception &e) {
        H->last_error = e.what();
        return RAS_ENOMEM;
    }
}

int gmres_solve_batch(ras_pml_t H, const void *b, void *x, const double *rtol, int restart,
                      int maxit, int *iters, double *relres, double *hist, void *stream) {
    if (!H) return RAS_EINVAL;
    if (!b || !x || b == x || !rtol || restart < 1 || maxit < 0) {
        H->last_error = "invalid gmres arguments";
        return RAS_EINVAL;
    }
    for (int p = 0; p < H->nprob; ++p)
        if (!(rtol[p] > 0.0)) {
            H->last_error = "every tolerance must be positive";
            return RAS_EINVAL;
        }
    try {
        int it = 0;
        double rr = 0.0;
        const int rc = gmres_impl(H, static_cast<const double2 *>(b), static_cast<double2 *>(x), rtol,
                                  restart, maxit, &it, &rr, hist, as_stream(stream));
        if (!H->res_iters.empty())
            for (int p = 0; p < H->nprob; ++p) {
                if (iters) iters[p] = H->res_iters[p];
                if (relres) relres[p] = H->res_relres[p];
            }
        return rc;
    } catch (const std::exception &e) {
        H->last_error = e.what();
        return RAS_ENOMEM;
    }
}

int ras_pml_richardson(ras_pml_t H, const void *b, void *x, double rtol, int maxit, int *iters,
                       double *relres, double *hist, void *stream) {
    if (!H) return RAS_EINVAL;
    if (!b || !x || b == x || !(rtol > 0.0) || maxit < 0) {
        H->last_error = "invalid richardson arguments";
        return RAS_EINVAL;
    }
    try {
        RichWork W{};
        RCHK(rich_work_handle(H, maxit, W));
        std::vector<int> need(H->nprob, 0);
        std::vector<double> bnorm(H->nprob), rel0(H->nprob);
        W.h_need = need.data();
        W.h_bnorm = bnorm.data();
        W.h_rel0 = rel0.data();
        return richardson_impl(H, W, static_cast<const double2 *>(b), static_cast<double2 *>(x),
                               rtol, maxit, iters, relres, hist, as_stream(stream));
    } catch (const std::exception &e) {
        H->last_error = e.what();
        return RAS_ENOMEM;
    }
}

int ras_pml_richardson_noalloc(ras_pml_t H, const void *b, void *x, double rtol, int maxit,
                               int *iters, double *relres, double *hist, void *stream) {
    if (!H) return RAS_EINVAL;
    if (!b || !x || b == x || !(rtol > 0.0) || maxit < 0) {
        H->last_error = "invalid richardson arguments";
        return RAS_EINVAL;
    }
    if (H->nprob > kNoAllocMaxProb) {
        H->last_error = "ras_pml_richardson_noalloc takes at most 64 problems per handle";
        return RAS_EINVAL;
    }
    unsigned char *base = nullptr;
    RCHK(scratch_address(H, &base));
    RichWork W{};
    RCHK(rich_work_scratch(H, base, maxit, W));
    const hipStream_t st = as_stream(stream);
    // the reduction counters must start at zero; the rest is written before
    // it is read (the array keeps the previous call's contents)
    HCHK(H, hipMemsetAsync(W.counters, 0, sizeof(unsigned int) * H->nprob, st));
    RState h_rs[kNoAllocMaxProb];
    double2 h_red[kNoAllocMaxProb];
    int need[kNoAllocMaxProb];
    double bnorm[kNoAllocMaxProb], rel0[kNoAllocMaxProb];
    W.h_rs = h_rs;
    W.h_red = h_red;
    W.h_need = need;
    W.h_bnorm = bnorm;
    W.h_rel0 = rel0;
    W.timed = false;
    return richardson_impl(H, W, static_cast<const double2 *>(b), static_cast<double2 *>(x), rtol,
                           maxit, iters, relres, hist, st);
}

static int single_grid(ras_pml_t H, int *grid) {
    if (H->nprob != 1) {
        H->last_error = "the interior grid is defined for single-problem handles";
        return RAS_EINVAL;
    }
    const DevProb &D = H->hprobs[0];
    if (D.G < 1) {
        H->last_error = "the interior grid needs a global PML of at least one cell";
        return RAS_EINVAL;
    }
    *grid = D.Nc - 2 * D.G;
    return RAS_OK;
}

int ras_pml_grid_sample(ras_pml_t H, const void *vec, double scale, float *grid_out, void *stream) {
    if (!H || !vec || !grid_out) return RAS_EINVAL;
    int grid = 0;
    RCHK(single_grid(H, &grid));
    const DevProb &D = H->hprobs[0];
    warm_grid_sample(static_cast<const double2 *>(vec), D.n1, D.G, grid, scale, grid_out,
                     as_stream(stream));
    HCHK(H, hipGetLastError());
    return RAS_OK;
}

int ras_pml_warm_start(ras_pml_t H, ras_pml_wsnet_t N, const void *f, const void *b, void *x0,
                       double fscale, int *used, void *stream) {
    if (!H || !N || !f || !b || !x0 || b == x0 || f == x0) return RAS_EINVAL;
    if (!(fscale > 0.0) || !std::isfinite(fscale)) {
        H->last_error = "fscale must be a positive finite number";
        return RAS_EINVAL;
    }
    int grid = 0;
    RCHK(single_grid(H, &grid));
    if (grid != wsnet_grid(N)) {
        H->last_error = "the network's grid differs from the problem's interior grid";
        return RAS_EINVAL;
    }
    hipStream_t st = as_stream(stream);
    const DevProb &D = H->hprobs[0];
    double2 *x = static_cast<double2 *>(x0);
    const double2 *bb = static_cast<const double2 *>(b);
    RCHK(ensure_krylov(H, 1));
    warm_grid_sample(static_cast<const double2 *>(f), D.n1, D.G, grid, 1.0 / fscale, wsnet_stage(N),
                     st);
    HCHK(H, hipGetLastError());
    RCHK(wsnet_forward(N, wsnet_stage(N), 1, wsnet_out(N), st));
    warm_grid_scatter(wsnet_out(N), D.n1, D.G, grid, fscale / (D.k * D.k), x, D.ndof, st);
    HCHK(H, hipGetLastError());
    // keep the guess only if its residual is below that of x0 = 0
    RCHK(reduce_sync(H, bb, nullptr, 0, st));
    const double bn = H->h_red[0].x;
    launch_spmv(H->d_probs, 1, H->max_ndof, nullptr, H->d_coef, H->ntot, x, bb, H->d_r, st);
    HCHK(H, hipGetLastError());
    RCHK(reduce_sync(H, H->d_r, nullptr, 0, st));
    const double rn = H->h_red[0].x;
    const bool keep = std::isfinite(rn) && rn <= bn;
    if (!keep) {
        HCHK(H, hipMemsetAsync(x, 0, sizeof(double2) * D.ndof, st));
        HCHK(H, hipStreamSynchronize(st));
    }
    if (used) *used = keep ? 1 : 0;
    return RAS_OK;
}

int ras_pml_batch_result(ras_pml_t H, int p, int *iters, double *relres, int *converged) {
    if (!H || p < 0 || p >= H->nprob || H->res_iters.empty()) return RAS_EINVAL;
    if (iters) *iters = H->res_iters[p];
    if (relres) *relres = H->res_relres[p];
    if (converged) *converged = H->res_conv[p];
    return RAS_OK;
}

int ras_pml_export_stencil(ras_pml_t H, void *host_out) {
    if (!H || !host_out) return RAS_EINVAL;
    HCHK(H, hipDeviceSynchronize());
    HCHK(H, hipMemcpy(host_out, H->d_coef, sizeof(double2) * 4 * H->ntot, hipMemcpyDeviceToHost));
    return RAS_OK;
}

int ras_pml_export_local(ras_pml_t H, int j, void *host_out) {
    if (!H || !host_out || j < 0 || j >= H->nsub) return RAS_EINVAL;
    const DevSub &s = H->hsubs[j];
    HCHK(H, hipDeviceSynchronize());
    HCHK(H, hipMemcpy(host_out, H->d_lst + 4 * s.loc_off, sizeof(double2) * 4 * s.n,
                      hipMemcpyDeviceToHost));
    return RAS_OK;
}

int ras_pml_export_factor(ras_pml_t H, int j, void *host_out, long long cap_values) {
    if (!H || !host_out || j < 0 || j >= H->nsub) return RAS_EINVAL;
    const DevSub &s = H->hsubs[j];
    const long long cnt = static_cast<long long>(s.npad) * (2 * s.W + 1);
    if (cap_values < cnt) {
        H->last_error = "export_factor: capacity too small";
        return RAS_EINVAL;
    }
    HCHK(H, hipDeviceSynchronize());
    const char *src = static_cast<const char *>(H->d_F) + H->csize * s.fac_off;
    double *out = static_cast<double *>(host_out);
    if (H->fp64) {
        HCHK(H, hipMemcpy(out, src, 16 * cnt, hipMemcpyDeviceToHost));
    } else {
        std::vector<float> tmp(2 * cnt);
        HCHK(H, hipMemcpy(tmp.data(), src, 8 * cnt, hipMemcpyDeviceToHost));
        for (long long i = 0; i < 2 * cnt; ++i) out[i] = tmp[i];
    }
    // the device keeps the rows of L last row first; export them in row order
    const long long rw = 2LL * s.W;                       // doubles per row
    double *rows = out + 2LL * s.npad * s.W;
    for (int i = 0, k = s.npad - 1; i < k; ++i, --k)
        for (long long e = 0; e < rw; ++e) std::swap(rows[i * rw + e], rows[k * rw + e]);
    return RAS_OK;
}

int ras_pml_autotune(ras_pml_t H, const char *cache_path, void *stream) {
    if (!H) return RAS_EINVAL;
    hipStream_t st = as_stream(stream);
    if (H->arch.empty()) H->arch = device_arch();
    hipEvent_t e0{}, e1{};
    HCHK(H, hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
    HCHK(H, hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
    // best of `reps` timed runs of fn (ms)
    auto timeit = [&](auto fn, int reps) -> float {
        float best = 1e30f;
        for (int r = 0; r < reps; ++r) {
            if (hipEventRecord(e0, st) != hipSuccess) return best;
            fn();
            if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
                return best;
            float ms = 0;
            if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess) best = std::min(best, ms);
        }
        return best;
    };
    int rc = RAS_OK;
    H->tune_ms.clear();
    // factorisation classes: the three kernel variants, one class at a time
    // with the others at their current choice, each timed as the whole
    // factorisation (the classes run side by side there); then the factor is
    // formed again with the chosen variants (the matrix-core and the
    // one-column kernels round differently), as a setup with these choices
    // forms it
    for (auto &g : H->lu_groups) {
        float t[LU_NVARIANTS];
        for (int v = 0; v < LU_NVARIANTS; ++v) {
            g[3] = v;
            t[v] = timeit([&] { (void)factorise(H, st); }, 2);
        }
        g[3] = static_cast<int>(std::min_element(t, t + LU_NVARIANTS) - t);
        H->tune_ms.insert(H->tune_ms.end(), t, t + LU_NVARIANTS);
    }
    {
        RCHK(factorise(H, st));
        std::vector<int> status(H->nsub);
        HCHK(H, hipMemcpyAsync(status.data(), H->d_status, sizeof(int) * H->nsub,
                               hipMemcpyDeviceToHost, st));
        HCHK(H, hipStreamSynchronize(st));
        for (int s = 0; s < H->nsub; ++s)
            if (status[s] >= 0) {
                H->last_error = "autotune: a chosen factorisation variant met a zero pivot";
                return RAS_EZEROPIVOT;
            }
    }
    // band solve: both prefetch depths on a zero right-hand side (the kernel
    // has no data-dependent control flow)
    double2 *v = nullptr;
    if (hipMalloc(reinterpret_cast<void **>(&v), sizeof(double2) * H->ntot) != hipSuccess) {
        H->last_error = "autotune: no memory for the test vector";
        rc = RAS_ENOMEM;
    } else {
        // prefetch depth x dispatch (the persistent queue only matters with
        // more subdomains than SIMDs)
        float t[2][2] = {{1e30f, 1e30f}, {1e30f, 1e30f}};
        const int nq = H->nsub_reg > H->solve_waves ? 2 : 1;
        if (hipMemsetAsync(v, 0, sizeof(double2) * H->ntot, st) == hipSuccess) {
            for (int q = 0; q < nq; ++q)
                for (int deep = 0; deep < 2; ++deep)
                    t[q][deep] = timeit([&] {
                        launch_solves(H, deep != 0, nullptr, SolveSrc{v, nullptr, 0},
                                      SolveDispatch{q ? H->d_queue : nullptr, H->solve_waves},
                                      st);
                    }, 3);
            int bq = 0, bd = 1;
            for (int q = 0; q < nq; ++q)
                for (int deep = 0; deep < 2; ++deep)
                    if (t[q][deep] < t[bq][bd]) {
                        bq = q;
                        bd = deep;
                    }
            H->solve_deep = bd != 0;
            H->solve_queue = bq != 0;
        }
        for (int q = 0; q < 2; ++q)
            for (int deep = 0; deep < 2; ++deep) H->tune_ms.push_back(t[q][deep]);
    }
    // fused Arnoldi variants: each whose grid stays co-resident, timed as
    // one step at step index 20 on zero vectors of the handle's own Krylov
    // workspace (best of three; the work does not depend on the values);
    // the device state it leaves is reset by the next solve's cycle start
    double arn_t[3] = {1e30, 1e30, 1e30};
    if (rc == RAS_OK && !(H->flags & RAS_FLAG_UNFUSED_ARNOLDI)) {
        constexpr int jt = 20;
        rc = ensure_krylov(H, std::max(H->m_alloc, jt + 2));
        int cus = 0;
        if (rc == RAS_OK && H->arn_E > 0 &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, H->device) ==
                hipSuccess) {
            std::vector<KState> ks(H->nprob);
            for (KState &K : ks) K = KState{1.0, 1.0, 1.0, 0.0, jt, 1, 0, jt + 2};
            const long long n = H->ntot;
            HCHK(H, hipMemcpyAsync(H->d_ks, ks.data(), sizeof(KState) * ks.size(),
                                   hipMemcpyHostToDevice, st));
            HCHK(H, hipMemsetAsync(H->d_V, 0, sizeof(double2) * n * (jt + 2), st));
            HCHK(H, hipMemsetAsync(H->d_Z, 0, sizeof(double2) * n * (jt + 1), st));
            const int m = H->m_alloc;
            for (int v = 0; v < arnoldi_variants() && rc == RAS_OK; ++v) {
                int blocks = 0;
                if (!arnoldi_fits(H, v, cus, &blocks)) continue;
                H->arn_pref = v;
                rc = plan_arnoldi(H);
                if (rc != RAS_OK || H->arn_var != v) continue;
                arn_t[v] = timeit([&] {
                    (void)launch_arnoldi(H->arn_var, H->arn_nblocks, H->d_probs, H->d_ks,
                                         H->d_ablocks, H->d_coef, n, H->d_Z, H->d_V, m, H->d_H,
                                         H->d_part2, H->d_bar, H->d_epoch, H->d_err, H->nprob, st);
                }, 3);
            }
            if (rc == RAS_OK) {
                H->arn_pref = static_cast<int>(std::min_element(arn_t, arn_t + 3) - arn_t);
                rc = plan_arnoldi(H);
            }
        }
    }
    {
        for (double a : arn_t) H->tune_ms.push_back(a);
        (void)hipStreamSynchronize(st);
        (void)hipFree(v);
    }
    const hipError_t e = hipGetLastError();
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) {
        H->last_error = std::string("autotune: ") + hipGetErrorString(e);
        return RAS_EHIP;
    }
    if (rc != RAS_OK) return rc;
    if (cache_path) {
        auto c = read_cache(cache_path);
        for (const auto &g : H->lu_groups) cache_set(c, lu_key(H, g), g[3]);
        cache_set(c, solve_key(H), H->solve_deep ? 1 : 0);
        cache_set(c, queue_key(H), H->solve_queue ? 1 : 0);
        if (H->arn_E > 0) cache_set(c, arnoldi_key(H), H->arn_pref);
        if (!write_cache(cache_path, c)) {
            H->last_error = std::string("autotune: cannot write ") + cache_path;
            return RAS_EINVAL;
        }
    }
    return RAS_OK;
}

int ras_pml_tune_report(ras_pml_t H, double *ms, int cap, int *n) {
    if (!H || !n || (cap > 0 && !ms)) return RAS_EINVAL;
    *n = static_cast<int>(H->tune_ms.size());
    for (int i = 0; i < std::min(cap, *n); ++i) ms[i] = H->tune_ms[i];
    return RAS_OK;
}

int ras_pml_tuning(ras_pml_t H, int *solve_deep, int *groups, int cap_groups, int *n_groups) {
    if (!H || !solve_deep || !n_groups || (cap_groups > 0 && !groups)) return RAS_EINVAL;
    *solve_deep = H->solve_deep ? 1 : 0;
    *n_groups = static_cast<int>(H->lu_groups.size());
    for (int i = 0; i < std::min(cap_groups, *n_groups); ++i) {
        groups[3 * i + 0] = H->lu_groups[i][0];
        groups[3 * i + 1] = H->lu_groups[i][2];
        groups[3 * i + 2] = H->lu_groups[i][3];
    }
    return RAS_OK;
}

int ras_pml_get_stats(ras_pml_t H, ras_pml_stats *out) {
    if (!H || !out) return RAS_EINVAL;
    collect_events(H);
    *out = H->stats;
    // launches of steps enqueued after convergence returned at once: count
    // only the steps that ran (their few microseconds stay in the times)
    const long long sk = H->skipped_steps;
    out->n_solve = std::max(0LL, out->n_solve - sk);
    out->n_sum = std::max(0LL, out->n_sum - sk);
    out->n_givens = std::max(0LL, out->n_givens - sk);
    out->n_mgs = std::max(0LL, out->n_mgs - sk);
    if (H->arn_E <= 0) out->n_spmv = std::max(0LL, out->n_spmv - sk);
    return RAS_OK;
}

int ras_pml_reset_stats(ras_pml_t H) {
    if (!H) return RAS_EINVAL;
    collect_events(H);
    const double sb = H->stats.solve_bytes, fb = H->stats.factor_bytes;
    const double a = H->stats.setup_assemble_ms, f = H->stats.setup_factor_ms;
    const double al = H->stats.alloc_ms;
    std::memset(&H->stats, 0, sizeof(H->stats));
    H->stats.alloc_ms = al;
    H->skipped_steps = 0;
    H->stats.solve_bytes = sb;
    H->stats.factor_bytes = fb;
    H->stats.setup_assemble_ms = a;
    H->stats.setup_factor_ms = f;
    return RAS_OK;
}

int ras_pml_set_knob(ras_pml_t H, int knob, int value) {
    if (!H) return RAS_EINVAL;
    if (knob == RAS_KNOB_ARNOLDI) {
        if (value < -1 || value >= arnoldi_variants()) {
            H->last_error = "fused Arnoldi variant out of range";
            return RAS_EINVAL;
        }
        H->arn_pref = value;
        // planned already (Krylov workspace allocated): plan again now
        return H->arn_E >= 0 ? plan_arnoldi(H) : RAS_OK;
    }
    if (value != 0 && value != 1) return RAS_EINVAL;
    switch (knob) {
        case RAS_KNOB_SOLVE_DEEP: H->solve_deep = value != 0; return RAS_OK;
        case RAS_KNOB_SOLVE_QUEUE: H->solve_queue = value != 0; return RAS_OK;
        default: H->last_error = "unknown knob"; return RAS_EINVAL;
    }
}

int ras_pml_get_knob(ras_pml_t H, int knob, int *value) {
    if (!H || !value) return RAS_EINVAL;
    switch (knob) {
        case RAS_KNOB_SOLVE_DEEP: *value = H->solve_deep ? 1 : 0; return RAS_OK;
        case RAS_KNOB_SOLVE_QUEUE: *value = H->solve_queue ? 1 : 0; return RAS_OK;
        case RAS_KNOB_ARNOLDI:    // the variant in use once planned, else the preference
            *value = H->arn_E > 0 ? H->arn_var : H->arn_E == 0 ? -2 : H->arn_pref;
            return RAS_OK;
        default: H->last_error = "unknown knob"; return RAS_EINVAL;
    }
}

const char *ras_pml_strerror(int status) {
    switch (status) {
        case RAS_OK: return "success";
        case RAS_EINVAL: return "invalid argument";
        case RAS_ENOMEM: return "out of device memory";
        case RAS_EHIP: return "HIP runtime error";
        case RAS_EZEROPIVOT: return "zero pivot in a local factorisation";
        case RAS_ENONFINITE: return "non-finite value";
        case RAS_ENOTCONV: return "GMRES did not converge within maxit";
        case RAS_EBREAKDOWN: return "GMRES breakdown";
        case RAS_ENOTSUP: return "size not supported";
        default: return "unknown status";
    }
}

const char *ras_pml_last_error(ras_pml_t H) { return H ? H->last_error.c_str() : ""; }

int ras_pml_shutdown(void) {
    destroy_aux_streams();
    (void)ras_pml_empty_cache(nullptr);
    return RAS_OK;
}

}  // extern "C"
