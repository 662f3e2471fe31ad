// Krylov-side kernels, all complex128 (Section 4.1: GMRES accelerated by
// RAS-PML).  Every kernel runs over all problems of a handle at once: grid
// row blockIdx.y is the problem, and a problem whose `active` flag is 0 is
// skipped.
//
//   k_spmv       y = A x or y = b - A x with the 7-point stencil
//   k_mgs        one modified Gram-Schmidt projection, fused with the
//                previous one's update:  w -= h_{i-1} v_{i-1};  h_i = <v_i, w>
//                (or the final update and ||w||); deterministic two-level
//                reduction finished by the last block of each problem
//   k_normalize  v_{j+1} = w / h_{j+1,j}
//   k_givens     complex Givens rotations on the Hessenberg column, residual
//                estimate |g_{j+1}|, cycle bookkeeping
//   k_cycle_end  back substitution R y = g and x += Z y
#include "device.h"

namespace raspml {

constexpr int kRedBlocks = 512;   // blocks per problem of a reduction
constexpr int kRedThreads = 256;

namespace {

__device__ __forceinline__ cplx<double> ld(const double2 *p, long long i) {
    double2 v = p[i];
    return {v.x, v.y};
}
__device__ __forceinline__ void st(double2 *p, long long i, cplx<double> v) {
    p[i] = make_double2(v.re, v.im);
}

__global__ void k_spmv(const DevProb *__restrict__ probs, const int *__restrict__ active,
                       const double2 *__restrict__ coef, long long ntot,
                       const double2 *__restrict__ x, const double2 *__restrict__ b,
                       double2 *__restrict__ y) {
    const DevProb P = probs[blockIdx.y];
    if (active != nullptr && active[blockIdx.y] == 0) return;
    const long long idx = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= P.ndof) return;
    const int n1 = P.n1;
    const int i = static_cast<int>(idx % n1) + 1;
    const int j = static_cast<int>(idx / n1) + 1;
    const long long g = P.dof_off + idx;
    const double2 *C = coef, *E = coef + ntot, *N = coef + 2 * ntot, *NE = coef + 3 * ntot;
    cplx<double> acc = cmul(ld(C, g), ld(x, g));
    if (i < n1) acc = cfma(acc, ld(E, g), ld(x, g + 1));
    if (i > 1) acc = cfma(acc, ld(E, g - 1), ld(x, g - 1));
    if (j < n1) acc = cfma(acc, ld(N, g), ld(x, g + n1));
    if (j > 1) acc = cfma(acc, ld(N, g - n1), ld(x, g - n1));
    if (i < n1 && j < n1) acc = cfma(acc, ld(NE, g), ld(x, g + n1 + 1));
    if (i > 1 && j > 1) acc = cfma(acc, ld(NE, g - n1 - 1), ld(x, g - n1 - 1));
    if (b != nullptr) acc = csub(ld(b, g), acc);
    st(y, g, acc);
}

__device__ __forceinline__ int red_blocks(long long n) {
    long long nb = (n + kRedThreads - 1) / kRedThreads;
    return static_cast<int>(nb < kRedBlocks ? (nb < 1 ? 1 : nb) : kRedBlocks);
}

// Block sum of a complex value held by every thread (fixed order).
__device__ cplx<double> block_sum(cplx<double> v, cplx<double> *sh) {
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int o = kRedThreads / 2; o > 0; o >>= 1) {
        if (tid < o) sh[tid] = cadd(sh[tid], sh[tid + o]);
        __syncthreads();
    }
    cplx<double> r = sh[0];
    __syncthreads();
    return r;
}

// Values exchanged between blocks inside one launch (partial sums) are
// written and read with device-scope atomic accesses, which are coherent
// across the XCDs without L2 write-back/invalidate fences; the store is
// complete (s_waitcnt) before the arrival is counted.
__device__ __forceinline__ void put_agent(double2 *p, cplx<double> v) {
    __hip_atomic_store(&p->x, v.re, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&p->y, v.im, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ cplx<double> get_agent(const double2 *p) {
    double2 *q = const_cast<double2 *>(p);
    return {__hip_atomic_load(&q->x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
            __hip_atomic_load(&q->y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)};
}
__device__ __forceinline__ unsigned long long peek(unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Write this block's partial; the last block of the problem to arrive sums
// all partials in index order and returns true with the total in *out.
// The partials travel through agent-scope atomic accesses (the store is
// complete before the ticket is drawn): no fence, which on this part would
// write back and invalidate the L2 of the block's XCD.
__device__ bool finish_reduction(cplx<double> part, int p, int nb, double2 *partials,
                                 unsigned int *counters, cplx<double> *sh, cplx<double> *out) {
    __shared__ int last;
    const int tid = threadIdx.x;
    if (tid == 0) {
        put_agent(partials + static_cast<long long>(p) * kRedBlocks + blockIdx.x, part);
        __builtin_amdgcn_s_waitcnt(0);
        const unsigned int ticket = atomicAdd(&counters[p], 1u);
        last = (ticket == static_cast<unsigned int>(nb - 1)) ? 1 : 0;
    }
    __syncthreads();
    if (!last) return false;
    cplx<double> acc{0, 0};
    for (int e = tid; e < nb; e += kRedThreads)
        acc = cadd(acc, get_agent(partials + static_cast<long long>(p) * kRedBlocks + e));
    *out = block_sum(acc, sh);
    if (tid == 0) __hip_atomic_store(&counters[p], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

// mode 0: h_{0,j} = <v_0, w>
// mode 1: w -= h_{i-1,j} v_{i-1};  h_{i,j} = <v_i, w>
// mode 2: w -= h_{j,j} v_j;        h_{j+1,j} = ||w||
// H is column-major with leading dimension m+1, one matrix per problem.
__global__ __launch_bounds__(kRedThreads) void k_mgs(
    const DevProb *__restrict__ probs, const KState *__restrict__ ks, double2 *__restrict__ w,
    const double2 *__restrict__ V, long long ntot, int j, int i, int mode, int m,
    double2 *__restrict__ H, double2 *__restrict__ partials, unsigned int *__restrict__ counters) {
    __shared__ cplx<double> sh[kRedThreads];
    const int p = blockIdx.y;
    if (ks[p].in_cycle == 0) return;
    const DevProb P = probs[p];
    const int nb = red_blocks(P.ndof);
    if (static_cast<int>(blockIdx.x) >= nb) return;
    double2 *Hp = H + static_cast<long long>(p) * (m + 1) * m;
    const long long col = static_cast<long long>(j) * (m + 1);
    cplx<double> hprev{0, 0};
    const double2 *vprev = nullptr;
    if (mode == 1) {
        hprev = ld(Hp, col + i - 1);
        vprev = V + static_cast<long long>(i - 1) * ntot;
    } else if (mode == 2) {
        hprev = ld(Hp, col + j);
        vprev = V + static_cast<long long>(j) * ntot;
    }
    const double2 *vi = (mode == 2) ? nullptr : V + static_cast<long long>(i) * ntot;
    cplx<double> acc{0, 0};
    const long long stride = static_cast<long long>(nb) * kRedThreads;
    for (long long e = static_cast<long long>(blockIdx.x) * kRedThreads + threadIdx.x; e < P.ndof;
         e += stride) {
        const long long g = P.dof_off + e;
        cplx<double> x = ld(w, g);
        if (mode != 0) {
            x = cfms(x, hprev, ld(vprev, g));
            st(w, g, x);
        }
        if (mode == 2)
            acc.re = fma(x.re, x.re, fma(x.im, x.im, acc.re));
        else
            acc = cdotacc(acc, ld(vi, g), x);
    }
    cplx<double> part = block_sum(acc, sh);
    cplx<double> tot;
    if (finish_reduction(part, p, nb, partials, counters, sh, &tot) && threadIdx.x == 0) {
        if (mode == 2)
            st(Hp, col + j + 1, cplx<double>{sqrt(tot.re), 0.0});
        else
            st(Hp, col + i, tot);
    }
}

// Plain deterministic reductions used outside the Arnoldi step:
// mode 0: out[p] = ||a_p||^2 (real part), mode 1: out[p] = <a_p, b_p>.
__global__ __launch_bounds__(kRedThreads) void k_reduce(
    const DevProb *__restrict__ probs, const int *__restrict__ active, const double2 *__restrict__ a,
    const double2 *__restrict__ b, int mode, double2 *__restrict__ out,
    double2 *__restrict__ partials, unsigned int *__restrict__ counters) {
    __shared__ cplx<double> sh[kRedThreads];
    const int p = blockIdx.y;
    if (active != nullptr && active[p] == 0) return;
    const DevProb P = probs[p];
    const int nb = red_blocks(P.ndof);
    if (static_cast<int>(blockIdx.x) >= nb) return;
    cplx<double> acc{0, 0};
    const long long stride = static_cast<long long>(nb) * kRedThreads;
    for (long long e = static_cast<long long>(blockIdx.x) * kRedThreads + threadIdx.x; e < P.ndof;
         e += stride) {
        const long long g = P.dof_off + e;
        cplx<double> x = ld(a, g);
        if (mode == 0)
            acc.re = fma(x.re, x.re, fma(x.im, x.im, acc.re));
        else
            acc = cdotacc(acc, x, ld(b, g));
    }
    cplx<double> part = block_sum(acc, sh);
    cplx<double> tot;
    if (finish_reduction(part, p, nb, partials, counters, sh, &tot) && threadIdx.x == 0)
        out[p] = make_double2(tot.re, tot.im);
}

__global__ void k_normalize(const DevProb *__restrict__ probs, const KState *__restrict__ ks,
                            double2 *__restrict__ w, int j, int m, const double2 *__restrict__ H) {
    const int p = blockIdx.y;
    if (ks[p].in_cycle == 0) return;
    const DevProb P = probs[p];
    const long long idx = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= P.ndof) return;
    const double hn = H[static_cast<long long>(p) * (m + 1) * m + static_cast<long long>(j) * (m + 1) + j + 1].x;
    const double s = hn > 0.0 ? 1.0 / hn : 0.0;
    const long long g = P.dof_off + idx;
    st(w, g, cscale(ld(w, g), s));
}

// v0 = r / beta for problems that start a cycle (beta from ks).
__global__ void k_start_cycle(const DevProb *__restrict__ probs, const KState *__restrict__ ks,
                              const double2 *__restrict__ r, double2 *__restrict__ v0) {
    const int p = blockIdx.y;
    if (ks[p].in_cycle == 0) return;
    const DevProb P = probs[p];
    const long long idx = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= P.ndof) return;
    const long long g = P.dof_off + idx;
    st(v0, g, cscale(ld(r, g), 1.0 / ks[p].beta));
}

// One thread per problem.  Rotation [[c, s], [-conj(s), c]] with c real
// zeroes h_{j+1,j}; g_{j+1} = -conj(s) g_j, g_j = c g_j.
// hist (optional): est / ||b|| of step j at hist[p (m + 1) + j]; active
// (optional): the problem's in-cycle flag after this step, for the next
// step's launches.
// The step index j is the problem's step count kp (read on the device).
__global__ void k_givens(KState *__restrict__ ks, int nprob, int m, double2 *__restrict__ H,
                         double *__restrict__ cs, double2 *__restrict__ sn,
                         double2 *__restrict__ gv, double *__restrict__ hist,
                         int *__restrict__ active) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nprob || ks[p].in_cycle == 0) return;
    const int j = ks[p].kp;
    double2 *Hc = H + static_cast<long long>(p) * (m + 1) * m + static_cast<long long>(j) * (m + 1);
    double *c_ = cs + static_cast<long long>(p) * m;
    double2 *s_ = sn + static_cast<long long>(p) * m;
    double2 *g = gv + static_cast<long long>(p) * (m + 1);
    double colnorm2 = 0.0;
    for (int i = 0; i <= j + 1; ++i) colnorm2 += Hc[i].x * Hc[i].x + Hc[i].y * Hc[i].y;
    const double hn = Hc[j + 1].x;
    for (int i = 0; i < j; ++i) {
        cplx<double> a{Hc[i].x, Hc[i].y}, b{Hc[i + 1].x, Hc[i + 1].y};
        cplx<double> s{s_[i].x, s_[i].y};
        const double c = c_[i];
        cplx<double> t = cadd(cscale(a, c), cmul(s, b));
        cplx<double> nb = cadd(cscale(cmul(cplx<double>{-s.re, s.im}, a), 1.0), cscale(b, c));
        Hc[i] = make_double2(t.re, t.im);
        Hc[i + 1] = make_double2(nb.re, nb.im);
    }
    cplx<double> a{Hc[j].x, Hc[j].y};
    const double aa = sqrt(a.re * a.re + a.im * a.im);
    double c;
    cplx<double> s;
    if (hn == 0.0) {
        c = 1.0;
        s = {0.0, 0.0};
    } else if (aa == 0.0) {
        c = 0.0;
        s = {1.0, 0.0};
    } else {
        const double rho = hypot(aa, hn);
        c = aa / rho;
        s = cscale(a, hn / (aa * rho));
    }
    c_[j] = c;
    s_[j] = make_double2(s.re, s.im);
    cplx<double> r = cadd(cscale(a, c), cscale(s, hn));
    Hc[j] = make_double2(r.re, r.im);
    Hc[j + 1] = make_double2(0.0, 0.0);
    cplx<double> gj{g[j].x, g[j].y};
    cplx<double> g1 = cmul(cplx<double>{-s.re, s.im}, gj);
    g[j + 1] = make_double2(g1.re, g1.im);
    g[j] = make_double2(c * gj.re, c * gj.im);
    const double est = sqrt(g1.re * g1.re + g1.im * g1.im);
    KState &K = ks[p];
    K.est = est;
    K.kp = j + 1;
    if (hist != nullptr) hist[static_cast<long long>(p) * (m + 1) + j] = est / K.bnorm;
    const bool brk = hn <= 1e-14 * sqrt(colnorm2);
    if (brk) K.breakdown = 1;
    if (est <= K.rtol * K.bnorm || brk || j + 1 >= K.mc) K.in_cycle = 0;
    if (active != nullptr) active[p] = K.in_cycle;
}

// Back substitution R y = g (one thread per problem, kp <= m).
__global__ void k_solve_y(const KState *__restrict__ ks, int nprob, int m,
                          const double2 *__restrict__ H, const double2 *__restrict__ gv,
                          double2 *__restrict__ y) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nprob) return;
    const int kp = ks[p].kp;
    const double2 *Hp = H + static_cast<long long>(p) * (m + 1) * m;
    const double2 *g = gv + static_cast<long long>(p) * (m + 1);
    double2 *yp = y + static_cast<long long>(p) * m;
    for (int i = kp - 1; i >= 0; --i) {
        cplx<double> acc{g[i].x, g[i].y};
        for (int l = i + 1; l < kp; ++l) {
            double2 h = Hp[static_cast<long long>(l) * (m + 1) + i];
            acc = cfms(acc, cplx<double>{h.x, h.y}, cplx<double>{yp[l].x, yp[l].y});
        }
        double2 d = Hp[static_cast<long long>(i) * (m + 1) + i];
        cplx<double> yi = cmul(acc, crecip(cplx<double>{d.x, d.y}));
        yp[i] = make_double2(yi.re, yi.im);
    }
}

// x += Z y for problems that took steps in this cycle (kp > 0).
__global__ void k_update_x(const DevProb *__restrict__ probs, const KState *__restrict__ ks,
                           const int *__restrict__ active, int m, const double2 *__restrict__ Z,
                           long long ntot, const double2 *__restrict__ y, double2 *__restrict__ x) {
    const int p = blockIdx.y;
    if (active[p] == 0) return;
    const int kp = ks[p].kp;
    const DevProb P = probs[p];
    const long long idx = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= P.ndof || kp == 0) return;
    const long long g = P.dof_off + idx;
    const double2 *yp = y + static_cast<long long>(p) * m;
    cplx<double> acc = ld(x, g);
    for (int i = 0; i < kp; ++i)
        acc = cfma(acc, cplx<double>{yp[i].x, yp[i].y}, ld(Z, static_cast<long long>(i) * ntot + g));
    st(x, g, acc);
}

// ---------------------------------------------------------------- fixed point
// After one step of the fixed-point iteration: for every problem that took
// it, the residual norm (from the reduction) becomes its relative residual,
// history entry `iters` and stopping test; a stopped problem's active flag
// is cleared, so later steps enqueued ahead of the host's check skip it.
__global__ void k_rich_update(RState *__restrict__ rs, int *__restrict__ active,
                              const double2 *__restrict__ red, double *__restrict__ hist,
                              int nprob, int maxit, double rtol) {
    for (int p = threadIdx.x; p < nprob; p += blockDim.x) {
        if (!active[p]) continue;
        RState R = rs[p];
        const double beta = sqrt(red[p].x);
        R.iters += 1;
        R.relres = beta / R.bnorm;
        hist[static_cast<long long>(p) * (maxit + 1) + R.iters] = R.relres;
        if (!isfinite(beta)) R.nonfinite = 1;
        if (R.nonfinite || R.relres <= rtol || R.iters >= maxit) active[p] = 0;
        rs[p] = R;
    }
}

// ---------------------------------------------------------------- fused step

// Barrier words, each on its own 256-byte line: [0] top arrivals,
// [32 (g+1)] arrivals of group g, [32 (g+1) + 16] release epoch of group g.
constexpr int kBarGroup = 32;           // blocks per group (13 groups of the 416 at k = 640)
constexpr int kBarStride = 32;          // unsigned long long per line

// Grid-wide barrier for a cooperative launch (every block co-resident).
// Counters only grow: barrier `epoch` (absolute, counted since the handle
// was created) is complete when every block has arrived at it.  A block
// arrives by incrementing its group's counter; the block whose increment
// completes the group (epoch * size(g)) increments the top counter, and the
// block whose increment completes the top (epoch * ngroups) writes the
// epoch to every group's release word, which the group's blocks poll.  No
// block waits to forward an arrival, so the release follows the last
// arrival by two atomic round trips and a store.  Polls are bounded: running
// out sets *err, and the block stops waiting at this launch's later
// barriers (`failed`), so the launch ends quickly with wrong numbers that
// the host reports, never a hang.
__device__ __forceinline__ bool spin_until(unsigned long long *p, unsigned long long target) {
    unsigned int polls = 0;
    while (peek(p) < target) {
        __builtin_amdgcn_s_sleep(1);
        if (++polls > (1u << 22)) return false;
    }
    return true;
}

// Counts this block's arrival and releases the epoch `target` when it
// completes it.
__device__ __forceinline__ void barrier_arrive(unsigned long long *bar, unsigned long long target) {
    const int nb = gridDim.x;
    const int ngroups = (nb + kBarGroup - 1) / kBarGroup;
    const int g = blockIdx.x / kBarGroup;
    const unsigned long long gsize = min(kBarGroup, nb - g * kBarGroup);
    const unsigned long long old = atomicAdd(bar + kBarStride * (g + 1), 1ull);
    if (old + 1 != target * gsize) return;                  // not the group's last arrival
    const unsigned long long t = atomicAdd(bar, 1ull);
    if (t + 1 != target * static_cast<unsigned long long>(ngroups)) return;
    for (int q = 0; q < ngroups; ++q)
        __hip_atomic_store(bar + kBarStride * (q + 1) + 16, target, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// The barrier in two halves, so that a block can issue loads that do not
// depend on it between its arrival and its wait.
__device__ __forceinline__ void grid_arrive(unsigned long long *bar, unsigned long long epoch) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_s_waitcnt(0);          // this block's published values are complete
        barrier_arrive(bar, epoch);
    }
}

__device__ __forceinline__ void grid_wait(unsigned long long *bar, unsigned long long epoch,
                                          int *err, bool &failed) {
    if (threadIdx.x == 0) {
        unsigned long long *grel = bar + kBarStride * (blockIdx.x / kBarGroup + 1) + 16;
        if (!failed && !spin_until(grel, epoch)) {
            failed = true;
            atomicOr(err, 1);
        }
    }
    __syncthreads();
}

__device__ __forceinline__ void grid_barrier(unsigned long long *bar, unsigned long long epoch,
                                             int *err, bool &failed) {
    grid_arrive(bar, epoch);
    grid_wait(bar, epoch, err, failed);
}

// Block sum for the fused step: each wave reduces its lanes with DPP moves
// (no LDS round trip), the four wave sums meet in LDS and every thread adds
// them in wave order (fixed order: deterministic).  sh4 alternates between
// two buffers of four values from call to call (`par`), so one barrier per
// call suffices: a buffer is written again only two calls later, after
// every thread has passed the barrier of the call in between.
__device__ __forceinline__ cplx<double> block_sum_dpp(cplx<double> v, cplx<double> (*sh4)[4],
                                                      int &par) {
    const cplx<double> w = wave_sum(v);
    cplx<double> *b = sh4[par];
    par ^= 1;
    if ((threadIdx.x & 63) == 0) b[threadIdx.x >> 6] = w;
    __syncthreads();
    return cadd(cadd(b[0], b[1]), cadd(b[2], b[3]));
}

// Sum the problem's per-block partials in index order within each thread,
// then over the block (every block of the problem obtains the same value).
__device__ cplx<double> problem_sum(const double2 *__restrict__ part, const ArnoldiBlock &B,
                                    cplx<double> (*sh4)[4], int &par) {
    cplx<double> acc{0, 0};
    for (int e = threadIdx.x; e < B.nblk; e += kRedThreads)
        acc = cadd(acc, get_agent(part + B.first_blk + e));
    return block_sum_dpp(acc, sh4, par);
}

// One Arnoldi step for every problem in one launch:
//   w = A z_j (7-point stencil);
//   for i = 0..j: h_ij = <v_i, w>; w -= h_ij v_i   (modified Gram-Schmidt)
//   h_{j+1,j} = ||w||; v_{j+1} = w / h_{j+1,j}.
// Each block keeps its slice of w (and the current v_i) in registers, so w is
// never re-read; j + 2 grid barriers separate the reductions.  With v_i kept
// (KEEPV), the block loads v_{i+1} between its arrival at barrier i and its
// wait there, so the load overlaps the wait for the other blocks.  Problems
// not in the cycle skip the arithmetic but take part in every barrier.
//
// The step index j is the step count kp of the problems still in the cycle
// (they all take their steps together), and the barrier epoch reached so far
// is kept on the device (*epoch): the launch's arguments are the same at
// every step, so that steps can be replayed from a graph.  Every block reads
// both at its start; block 0 advances the epoch by j + 2 after the last
// barrier, when every block has read it.
template <int E, bool KEEPV>
__device__ __forceinline__ void arnoldi_step(
    const DevProb *__restrict__ probs, const KState *__restrict__ ks,
    const ArnoldiBlock *__restrict__ blocks, const double2 *__restrict__ coef, long long ntot,
    const double2 *__restrict__ Z, double2 *__restrict__ V, int m, double2 *__restrict__ H,
    double2 *__restrict__ part2, unsigned long long *bar, unsigned long long *epoch, int *err,
    int nprob) {
    static_assert(kRedThreads == 256, "four waves per block");
    __shared__ cplx<double> sh4[2][4];
    int par = 0;
    // No problem left in the cycle (the host enqueues steps ahead of the
    // convergence test): every block sees the same flags, so the whole grid
    // skips the step, barriers and epoch included.
    int j = -1;
    for (int q = 0; q < nprob; ++q)
        if (ks[q].in_cycle != 0) j = max(j, ks[q].kp);
    if (j < 0) return;
    const unsigned long long epoch0 = peek(epoch);
    const double2 *__restrict__ zj = Z + static_cast<long long>(j) * ntot;
    const ArnoldiBlock B = blocks[blockIdx.x];
    const int nblocks = gridDim.x;
    const int p = B.prob;
    const bool on = ks[p].in_cycle != 0;
    const DevProb P = probs[p];
    const int n1 = P.n1;
    double2 *Hp = H + static_cast<long long>(p) * (m + 1) * m;
    const long long col = static_cast<long long>(j) * (m + 1);
    cplx<double> w[E];
#pragma unroll
    for (int q = 0; q < E; ++q) {
        const int o = threadIdx.x + q * kRedThreads;
        w[q] = cplx<double>{0, 0};
        if (on && o < B.n) {
            const long long g = B.first + o;
            int i, jj;
            if constexpr (KEEPV) {
                const long long idx = g - P.dof_off;
                i = static_cast<int>(idx % n1) + 1;
                jj = static_cast<int>(idx / n1) + 1;
            } else {   // (a problem's unknowns are int-indexed)
                const int idx = static_cast<int>(g - P.dof_off);
                i = idx % n1 + 1;
                jj = idx / n1 + 1;
            }
            const double2 *C = coef, *Ec = coef + ntot, *N = coef + 2 * ntot, *NE = coef + 3 * ntot;
            cplx<double> acc = cmul(ld(C, g), ld(zj, g));
            if (i < n1) acc = cfma(acc, ld(Ec, g), ld(zj, g + 1));
            if (i > 1) acc = cfma(acc, ld(Ec, g - 1), ld(zj, g - 1));
            if (jj < n1) acc = cfma(acc, ld(N, g), ld(zj, g + n1));
            if (jj > 1) acc = cfma(acc, ld(N, g - n1), ld(zj, g - n1));
            if (i < n1 && jj < n1) acc = cfma(acc, ld(NE, g), ld(zj, g + n1 + 1));
            if (i > 1 && jj > 1) acc = cfma(acc, ld(NE, g - n1 - 1), ld(zj, g - n1 - 1));
            w[q] = acc;
        }
        // lean variant: at most two unknowns' stencil loads in flight
        if constexpr (!KEEPV)
            if ((q & 1) == 1) __builtin_amdgcn_sched_barrier(0);
    }
    unsigned long long ep = 0;            // barriers passed in this launch
    bool failed = false;                  // (thread 0) a poll of this launch ran out
    // KEEPV: v holds v_i at the top of projection i, vnext receives v_{i+1}
    cplx<double> v[KEEPV ? E : 1], vnext[KEEPV ? E : 1];
    auto load_v = [&](const double2 *vi, cplx<double> *dst) {
#pragma unroll
        for (int q = 0; q < E; ++q) {
            const int o = threadIdx.x + q * kRedThreads;
            dst[q] = (on && o < B.n) ? ld(vi, B.first + o) : cplx<double>{0, 0};
        }
    };
    if constexpr (KEEPV) load_v(V, v);
    for (int i = 0; i <= j; ++i) {
        const double2 *vi = V + static_cast<long long>(i) * ntot;
        cplx<double> acc{0, 0};
#pragma unroll
        for (int q = 0; q < E; ++q) {
            const int o = threadIdx.x + q * kRedThreads;
            const cplx<double> vq =
                KEEPV ? v[q] : ((on && o < B.n) ? ld(vi, B.first + o) : cplx<double>{0, 0});
            acc = cdotacc(acc, vq, w[q]);
        }
        double2 *part = part2 + static_cast<long long>(i & 1) * nblocks;
        const cplx<double> bs = block_sum_dpp(acc, sh4, par);
        if (threadIdx.x == 0) put_agent(part + blockIdx.x, bs);
        ++ep;
        grid_arrive(bar, epoch0 + ep);
        if constexpr (KEEPV)
            if (i < j) load_v(vi + ntot, vnext);
        grid_wait(bar, epoch0 + ep, err, failed);
        const cplx<double> h = problem_sum(part, B, sh4, par);
#pragma unroll
        for (int q = 0; q < E; ++q) {
            const int o = threadIdx.x + q * kRedThreads;
            // KEEPV: v_i stayed in registers; else it is read again (the
            // register budget then leaves room for more blocks per CU)
            const cplx<double> vq =
                KEEPV ? v[q] : ((on && o < B.n) ? ld(vi, B.first + o) : cplx<double>{0, 0});
            w[q] = cfms(w[q], h, vq);
            if (KEEPV) v[q] = vnext[q];
        }
        if (on && blockIdx.x == B.first_blk && threadIdx.x == 0) st(Hp, col + i, h);
    }
    double nrm = 0.0;
#pragma unroll
    for (int q = 0; q < E; ++q) nrm = fma(w[q].re, w[q].re, fma(w[q].im, w[q].im, nrm));
    double2 *part = part2 + static_cast<long long>((j + 1) & 1) * nblocks;
    const cplx<double> bs = block_sum_dpp(cplx<double>{nrm, 0.0}, sh4, par);
    if (threadIdx.x == 0) put_agent(part + blockIdx.x, cplx<double>{bs.re, 0.0});
    ++ep;
    grid_barrier(bar, epoch0 + ep, err, failed);
    if (blockIdx.x == 0 && threadIdx.x == 0)
        __hip_atomic_store(epoch, epoch0 + ep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const double hn = sqrt(problem_sum(part, B, sh4, par).re);
    if (!on) return;
    const double s = hn > 0.0 ? 1.0 / hn : 0.0;
    double2 *vn = V + static_cast<long long>(j + 1) * ntot;
#pragma unroll
    for (int q = 0; q < E; ++q) {
        const int o = threadIdx.x + q * kRedThreads;
        if (o < B.n) st(vn, B.first + o, cscale(w[q], s));
    }
    if (blockIdx.x == B.first_blk && threadIdx.x == 0) st(Hp, col + j + 1, cplx<double>{hn, 0.0});
}

#define ARNOLDI_PARAMS                                                                          \
    const DevProb *__restrict__ probs, const KState *__restrict__ ks,                           \
        const ArnoldiBlock *__restrict__ blocks, const double2 *__restrict__ coef,              \
        long long ntot, const double2 *__restrict__ Z, double2 *__restrict__ V, int m,          \
        double2 *__restrict__ H, double2 *__restrict__ part2, unsigned long long *bar,          \
        unsigned long long *epoch, int *err, int nprob
#define ARNOLDI_ARGS probs, ks, blocks, coef, ntot, Z, V, m, H, part2, bar, epoch, err, nprob

template <int E>
__global__ __launch_bounds__(kRedThreads) void k_arnoldi(ARNOLDI_PARAMS) {
    arnoldi_step<E, true>(ARNOLDI_ARGS);
}

// v_i read again after each barrier instead of kept, and the register
// budget held to three workgroups per CU: for grids the kernel above cannot
// keep co-resident.
template <int E>
__global__ __launch_bounds__(kRedThreads) __attribute__((amdgpu_waves_per_eu(3))) void
k_arnoldi_lean(ARNOLDI_PARAMS) {
    arnoldi_step<E, false>(ARNOLDI_ARGS);
}
#undef ARNOLDI_PARAMS
#undef ARNOLDI_ARGS

}  // namespace

void launch_spmv(const DevProb *probs, int nprob, long long max_ndof, const int *active,
                 const double2 *coef, long long ntot, const double2 *x, const double2 *b,
                 double2 *y, hipStream_t s) {
    dim3 grid(static_cast<unsigned>((max_ndof + 255) / 256), nprob);
    hipLaunchKernelGGL(k_spmv, grid, dim3(256), 0, s, probs, active, coef, ntot, x, b, y);
}

void launch_mgs(const DevProb *probs, int nprob, const KState *ks, double2 *w, const double2 *V,
                long long ntot, int j, int i, int mode, int m, double2 *H, double2 *partials,
                unsigned int *counters, hipStream_t s) {
    dim3 grid(kRedBlocks, nprob);
    hipLaunchKernelGGL(k_mgs, grid, dim3(kRedThreads), 0, s, probs, ks, w, V, ntot, j, i, mode, m,
                       H, partials, counters);
}

void launch_reduce(const DevProb *probs, int nprob, const int *active, const double2 *a,
                   const double2 *b, int mode, double2 *out, double2 *partials,
                   unsigned int *counters, hipStream_t s) {
    dim3 grid(kRedBlocks, nprob);
    hipLaunchKernelGGL(k_reduce, grid, dim3(kRedThreads), 0, s, probs, active, a, b, mode, out,
                       partials, counters);
}

void launch_normalize(const DevProb *probs, int nprob, long long max_ndof, const KState *ks,
                      double2 *w, int j, int m, const double2 *H, hipStream_t s) {
    dim3 grid(static_cast<unsigned>((max_ndof + 255) / 256), nprob);
    hipLaunchKernelGGL(k_normalize, grid, dim3(256), 0, s, probs, ks, w, j, m, H);
}

void launch_start_cycle(const DevProb *probs, int nprob, long long max_ndof, const KState *ks,
                        const double2 *r, double2 *v0, hipStream_t s) {
    dim3 grid(static_cast<unsigned>((max_ndof + 255) / 256), nprob);
    hipLaunchKernelGGL(k_start_cycle, grid, dim3(256), 0, s, probs, ks, r, v0);
}

void launch_rich_update(RState *rs, int *active, const double2 *red, double *hist, int nprob,
                        int maxit, double rtol, hipStream_t s) {
    hipLaunchKernelGGL(k_rich_update, dim3(1), dim3(64), 0, s, rs, active, red, hist, nprob, maxit,
                       rtol);
}

void launch_givens(KState *ks, int nprob, int m, double2 *H, double *cs, double2 *sn,
                   double2 *g, double *hist, int *active, hipStream_t s) {
    hipLaunchKernelGGL(k_givens, dim3((nprob + 63) / 64), dim3(64), 0, s, ks, nprob, m, H, cs, sn,
                       g, hist, active);
}

void launch_solve_y(const KState *ks, int nprob, int m, const double2 *H, const double2 *g,
                    double2 *y, hipStream_t s) {
    hipLaunchKernelGGL(k_solve_y, dim3((nprob + 63) / 64), dim3(64), 0, s, ks, nprob, m, H, g, y);
}

void launch_update_x(const DevProb *probs, int nprob, long long max_ndof, const KState *ks,
                     const int *active, int m, const double2 *Z, long long ntot,
                     const double2 *y, double2 *x, hipStream_t s) {
    dim3 grid(static_cast<unsigned>((max_ndof + 255) / 256), nprob);
    hipLaunchKernelGGL(k_update_x, grid, dim3(256), 0, s, probs, ks, active, m, Z, ntot, y, x);
}

}  // namespace raspml

namespace raspml {

// Fused Arnoldi variants in the order the planner tries them: 8 or 16
// unknowns per thread with v_i kept in registers across the barrier, then 12
// with v_i read again (168 registers, three workgroups per CU instead of two;
// the few values it spills live outside the projection loop): for batches
// whose grid would not fit otherwise.
namespace {
const void *arnoldi_fn(int variant) {
    switch (variant) {
        case 0: return reinterpret_cast<const void *>(k_arnoldi<8>);
        case 1: return reinterpret_cast<const void *>(k_arnoldi<16>);
        default: return reinterpret_cast<const void *>(k_arnoldi_lean<12>);
    }
}
}  // namespace

int arnoldi_variants() { return 3; }
int arnoldi_variant_e(int variant) { return variant == 0 ? 8 : variant == 1 ? 16 : 12; }

int arnoldi_block_capacity(int variant, int *blocks_per_cu) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, arnoldi_fn(variant), kRedThreads, 0) !=
        hipSuccess)
        return -1;
    *blocks_per_cu = nb;
    return 0;
}

hipError_t launch_arnoldi(int variant, int nblocks, const DevProb *probs, const KState *ks,
                          const ArnoldiBlock *blocks, const double2 *coef, long long ntot,
                          const double2 *Z, double2 *V, int m, double2 *H, double2 *part2,
                          unsigned long long *bar, unsigned long long *epoch, int *err, int nprob,
                          hipStream_t s) {
    void *args[] = {(void *)&probs, (void *)&ks, (void *)&blocks, (void *)&coef, (void *)&ntot,
                    (void *)&Z, (void *)&V, (void *)&m, (void *)&H, (void *)&part2,
                    (void *)&bar, (void *)&epoch, (void *)&err, (void *)&nprob};
    return hipLaunchCooperativeKernel(arnoldi_fn(variant), dim3(nblocks), dim3(kRedThreads), args, 0,
                                      s);
}

}  // namespace raspml
