// RAS-PML preconditioner application (Section 2, discrete RAS):
//     z = B^{-1} v = sum_j R~_j^T A_j^{-1} R_j v.
//
// k_band_solve: one wave64 per subdomain (largest first).  With
// A_j = L D L^T it runs
//   forward   L y = R_j v   and   backward   L^T x = D^{-1} y,
// both in column form: once the pivot value of row c is final, every other
// row of the band window takes -(factor entry) * pivot.  The forward reads
// column c of L, the backward row c of L; the factorisation stores the
// columns, then the rows last row first, so the two sweeps read one
// contiguous stream of W complex values per step, which a single pointer
// walks PD vectors ahead of the arithmetic (prefetch into registers).  Each
// step is one v_readlane broadcast of the pivot, one complex FMA per ring
// slot and a v_writelane of the pivot into the block's output register.
// The window rows live in registers as a ring spread over the lanes: row r
// in slot r mod W.  Three layouts of the slots over the lanes:
//   ONE   (W <= 64): slot s in lane s;
//   SPLIT (W > 64, complex128): slot s in lane s mod 64, a second register
//         for slots 64..127;
//   PAIR  (W > 64, complex64): slots 2l and 2l+1 in lane l, so that a lane
//         takes its two entries of a factor vector with one 16-byte load.
//         W is even (the planner rounds it up), so slot sl of step c has the
//         parity of c and the register holding the pivot is known at
//         compile time in the unrolled 64-step blocks.
// A slot whose row is finished is not reset: it keeps accumulating for the
// row W further on, and when that row's block of 64 steps starts the slot
// is corrected by (right-hand side - finished value), read from an LDS
// history of the last 128 outputs (ONE: the right-hand side enters the slot
// at retirement instead).
//
// The factor stream is read once per application: its loads are
// non-temporal, so they do not displace the gathered vectors in the caches.
//
// The stream pointer is not clamped at the ends: the prefetch runs up to PD
// vectors past the last backward row (into D^{-1}, the next subdomain, or
// the allocation's slack); those vectors are loaded and never used.  Lanes
// past the vector end re-read its last entry (their ring registers hold no
// slot).
//
// k_pou_sum: deterministic partition-of-unity weighted sum of the local
// solutions into z (fixed summation order, complex128).
#include "device.h"

namespace raspml {

namespace {


// Branch-free (the load is always issued, in bounds) so that the compiler's
// memory-counter waits stay exact across the unrolled loop.  Returns the raw
// complex128 value; rows past the end give 0 after `to_T`.
__device__ __forceinline__ double2 gather_raw(const DevSub &S, int dof_off, int n1,
                                              const double2 *__restrict__ v, int r0) {
    const int r = min(r0, S.n - 1);
    int i, j;
    if (S.xfast) {
        i = S.ix0 + r % S.nf;
        j = S.jy0 + r / S.nf;
    } else {
        j = S.jy0 + r % S.nf;
        i = S.ix0 + r / S.nf;
    }
    return v[static_cast<long long>(dof_off) + static_cast<long long>(j - 1) * n1 + (i - 1)];
}
template <typename T>
__device__ __forceinline__ cplx<T> to_T(double2 x, bool in) {
    return cplx<T>{in ? static_cast<T>(x.x) : T(0), in ? static_cast<T>(x.y) : T(0)};
}

template <typename T>
__device__ __forceinline__ cplx<T> gather_rhs(const DevSub &S, int dof_off, int n1,
                                              const double2 *__restrict__ v, int r0) {
    return to_T<T>(gather_raw(S, dof_off, n1, v, r0), r0 < S.n);
}

// Non-temporal loads of one complex value / of two adjacent complex64 values.
template <typename T>
__device__ __forceinline__ cplx<T> nt_load(const cplx<T> *p) {
    using v2 = T __attribute__((ext_vector_type(2)));
    const v2 q = __builtin_nontemporal_load(reinterpret_cast<const v2 *>(p));
    return cplx<T>{q.x, q.y};
}
__device__ __forceinline__ void nt_load_pair(const cplx<float> *p, cplx<float> &a,
                                             cplx<float> &b) {
    using v4 = float __attribute__((ext_vector_type(4)));
    const v4 q = __builtin_nontemporal_load(reinterpret_cast<const v4 *>(p));
    a = cplx<float>{q.x, q.y};
    b = cplx<float>{q.z, q.w};
}

enum RingLayout { RING_ONE = 0, RING_SPLIT = 1, RING_PAIR = 2 };

// Offset of slot s (held by this lane) from slot `sl` in the ring, in the
// direction of the sweep: the slot holds row (pivot row) +/- that offset.
__device__ __forceinline__ int ring_offset(int s, int sl, int W, bool down) {
    int t = down ? sl - s : s - sl;
    return t < 0 ? t + W : t;
}

// Both sweeps for one subdomain.  RING: slot layout (above); SPLIT and PAIR
// have a second register and the block correction, ONE takes incoming rows
// at retirement.  PD: prefetch depth in vectors (divides 64).
template <typename T, int RING, int PD>
__device__ __forceinline__ void solve_subdomain(const DevProb *__restrict__ probs, const DevSub &S,
                                                const double2 *__restrict__ v,
                                                const cplx<T> *__restrict__ F,
                                                cplx<T> *__restrict__ ybuf,
                                                cplx<T> *__restrict__ xout, cplx<T> *hist,
                                                cplx<T> *inc) {
    const int dof_off = static_cast<int>(probs[S.prob].dof_off);
    const int n1 = probs[S.prob].n1;
    const int lane = threadIdx.x;
    const int W = S.W, npad = S.npad;
    const long long NW = static_cast<long long>(npad) * W;
    const cplx<T> *L = F + S.fac_off;          // [columns of L | rows of L, last first]
    const cplx<T> *Dv = L + 2 * NW;             // D^{-1}
    cplx<T> *yb = ybuf + S.vec_off;
    cplx<T> *xo = xout + S.vec_off;
    constexpr bool TWO = RING != RING_ONE;
    constexpr bool PAIR = RING == RING_PAIR;
    static_assert(!PAIR || sizeof(T) == 4, "the pair layout is for complex64");
    const cplx<T> zero{0, 0};
    // slots of this lane's two registers, and whether they exist
    const int slo = PAIR ? 2 * lane : lane, shi = PAIR ? 2 * lane + 1 : lane + 64;
    const bool lo_ok = slo < W, hi_ok = shi < W;
    // stream offsets: lanes past the vector end re-read its last entries
    const int olo = PAIR ? 2 * min(lane, W / 2 - 1) : min(lane, W - 1);
    const int ohi = min(lane + 64, W - 1);

    // pivot of step t (row c0 + t) in slot q; PAIR: the parity of q is that
    // of t (W and c0 even), a compile-time constant in the unrolled loops
    auto pivot = [&](const cplx<T> &lo, const cplx<T> &hi, int q, int t) {
        if constexpr (PAIR) return readlane((t & 1) ? hi : lo, q >> 1);
        else return readlane(csel(!TWO || q < 64, lo, hi), q & 63);
    };
    auto load = [&](const cplx<T> *p, cplx<T> &a, cplx<T> &b) {
        if constexpr (PAIR) {
            nt_load_pair(p + olo, a, b);
        } else {
            a = nt_load(p + olo);
            if (TWO) b = nt_load(p + ohi);
        }
    };
    // block correction (W > 64): the slot of every row r of the block gets
    // rhs_r - (finished value of the row W before it)
    auto correct = [&](cplx<T> &lo, cplx<T> &hi, int sl, int rfirst, bool down) {
        __builtin_amdgcn_wave_barrier();
        const int tlo = ring_offset(slo, sl, W, down);
        const int thi = ring_offset(shi, sl, W, down);
        const int qlo = down ? 63 - tlo : tlo, qhi = down ? 63 - thi : thi;   // index into inc
        const int rlo = rfirst + qlo, rhi = rfirst + qhi;                     // rows
        const int plo = down ? rlo + W : rlo - W, phi = down ? rhi + W : rhi - W;
        const cplx<T> dlo = csub(inc[min(max(qlo, 0), 63)], hist[plo & 127]);
        const cplx<T> dhi = csub(inc[min(max(qhi, 0), 63)], hist[phi & 127]);
        lo = cadd(lo, csel(lo_ok && tlo < 64, dlo, zero));
        hi = cadd(hi, csel(hi_ok && thi < 64, dhi, zero));
        __builtin_amdgcn_wave_barrier();
    };

    // one pointer runs through the whole stream: PD vectors ahead of the step
    const cplx<T> *pf = L;
    cplx<T> flo[PD], fhi[PD];
#pragma unroll
    for (int u = 0; u < PD; ++u) {
        load(pf, flo[u], fhi[u]);
        pf += W;
    }
    if (TWO) {
        hist[lane] = zero;
        hist[lane + 64] = zero;
    }

    // ------------------------------------------------------------ forward
    cplx<T> ylo = zero, yhi = zero;
    if (!TWO) ylo = csel(lane < W, gather_rhs<T>(S, dof_off, n1, v, lane), zero);
    // rows of the next block: TWO -> rows whose pivot step is in it,
    // one register -> rows entering the window during it
    const int ahead = TWO ? 0 : W;
    cplx<T> rnext = gather_rhs<T>(S, dof_off, n1, v, ahead + lane);
    int sl = 0;
    for (int c0 = 0; c0 < npad; c0 += 64) {
        const cplx<T> rblk = rnext;
        const double2 rraw = gather_raw(S, dof_off, n1, v, c0 + 64 + ahead + lane);
        if (TWO) {
            inc[lane] = rblk;
            correct(ylo, yhi, sl, c0, false);
        }
        cplx<T> yout = zero;
#pragma unroll
        for (int t = 0; t < 64; ++t) {
            const int u = t % PD;
            const cplx<T> piv = pivot(ylo, yhi, sl, t);              // y_(c0+t)
            ylo = cfms(ylo, flo[u], piv);
            if (TWO) yhi = cfms(yhi, fhi[u], piv);
            if (!TWO) ylo = writelane(ylo, readlane(rblk, t), sl);   // row c + W enters
            yout = writelane(yout, piv, t);
            load(pf, flo[u], fhi[u]);
            pf += W;
            sl = (sl + 1 == W) ? 0 : sl + 1;
            __builtin_amdgcn_sched_barrier(0);   // keep each step's loads in place
        }
        rnext = to_T<T>(rraw, c0 + 64 + ahead + lane < S.n);
        yb[c0 + lane] = yout;
        if (TWO) hist[(c0 + lane) & 127] = yout;
    }

    // ------------------------------------------------------------ backward
    // L^T x = z with z = D^{-1} y: after x_c is final, rows r < c in the
    // window take -L[c, r] x_c, i.e. row c of L (next in the stream).
    if (TWO) {
        __builtin_amdgcn_wave_barrier();
        hist[lane] = zero;
        hist[lane + 64] = zero;
    }
    cplx<T> xlo = zero, xhi = zero;
    // z of the rows of the next block: TWO -> rows whose pivot step is in it
    // (c0 .. c0+63), one register -> rows entering the window (c0-W .. c0+63-W)
    const int behind = TWO ? 0 : W;
    auto zrow = [&](int r) {           // z_r, 0 for r < 0
        const int rr = max(r, 0);
        return csel(r >= 0, cmul(yb[rr], Dv[rr]), zero);
    };
    if (!TWO) {
        const int r0 = npad - 1 - ((npad - 1 - lane) % W + W) % W;   // row of slot `lane`
        xlo = csel(lane < W && r0 >= npad - W, zrow(r0), zero);
    }
    sl = (npad - 1) % W;
    cplx<T> znext = zrow(npad - 64 - behind + lane);
    for (int c0 = npad - 64; c0 >= 0; c0 -= 64) {
        const cplx<T> zblk = znext;
        const int rn = c0 - 64 - behind + lane;
        const cplx<T> ynx = yb[max(rn, 0)];
        const cplx<T> dnx = Dv[max(rn, 0)];
        if (TWO) {
            inc[lane] = zblk;
            correct(xlo, xhi, sl, c0, true);
        }
        cplx<T> xr = zero;
#pragma unroll
        for (int q = 0; q < 64; ++q) {
            const int t = 63 - q;
            const int u = q % PD;
            const cplx<T> piv = pivot(xlo, xhi, sl, t);              // x_(c0+t)
            xlo = cfms(xlo, flo[u], piv);
            if (TWO) xhi = cfms(xhi, fhi[u], piv);
            if (!TWO) xlo = writelane(xlo, readlane(zblk, t), sl);   // row c - W enters
            xr = writelane(xr, piv, t);
            load(pf, flo[u], fhi[u]);
            pf += W;
            sl = (sl == 0) ? W - 1 : sl - 1;
            __builtin_amdgcn_sched_barrier(0);
        }
        znext = csel(rn >= 0, cmul(ynx, dnx), zero);
        xo[c0 + lane] = xr;
        if (TWO) hist[(c0 + lane) & 127] = xr;
    }
}

// One wave per SIMD by design (1024 subdomains on 1024 SIMDs at k = 640):
// the whole register file is available to the prefetch ring.  A launch built
// for W up to 128 still solves its subdomains with W <= 64 in the
// one-register form (uniform branch per subdomain).  W > 64 takes the pair
// layout in complex64 (W is even) and the split layout in complex128.
//
// Right-hand side: v, or (ks non-null) v + ks[problem].kp * vstride, the
// Krylov vector of the problem's current GMRES step, so that the launch's
// arguments stay the same from step to step (replay from a graph).
//
// Dispatch: QUEUE = false, one wave per subdomain, launched in the order of
// `order` (largest first), the hardware dispatcher handing each wave to the
// next free SIMD; QUEUE = true, a persistent grid of at most one wave per
// SIMD, each wave taking the next subdomain of `order` from an atomic
// counter until none is left (largest first: a list schedule).  The last
// wave to finish resets the two counter words to zero for the next launch.
template <typename T, bool TWO, int PD, bool QUEUE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_band_solve(
    const DevProb *__restrict__ probs, const DevSub *__restrict__ subs,
    const int *__restrict__ order, int nsub, const int *__restrict__ active,
    const double2 *__restrict__ v, const KState *__restrict__ ks, long long vstride,
    const cplx<T> *__restrict__ F, cplx<T> *__restrict__ ybuf, cplx<T> *__restrict__ xout,
    unsigned int *__restrict__ queue) {
    __shared__ cplx<T> hist[128];               // outputs, by row mod 128
    __shared__ cplx<T> inc[64];                 // right-hand side of the current block
    auto one = [&](int item) {
        const DevSub S = subs[order[item]];
        if (active != nullptr && active[S.prob] == 0) return;
        const double2 *vs = ks != nullptr ? v + static_cast<long long>(ks[S.prob].kp) * vstride : v;
        constexpr int WIDE = sizeof(T) == 4 ? RING_PAIR : RING_SPLIT;
        if (TWO && S.W > 64)
            solve_subdomain<T, WIDE, PD>(probs, S, vs, F, ybuf, xout, hist, inc);
        else
            solve_subdomain<T, RING_ONE, PD>(probs, S, vs, F, ybuf, xout, hist, inc);
    };
    if constexpr (!QUEUE) {
        one(blockIdx.x);
    } else {
        for (;;) {
            int item = 0;
            if (threadIdx.x == 0) item = static_cast<int>(atomicAdd(queue, 1u));
            item = __shfl(item, 0);
            if (item >= nsub) break;
            one(item);
            __builtin_amdgcn_wave_barrier();
        }
        if (threadIdx.x == 0) {
            const unsigned int done = atomicAdd(queue + 1, 1u);
            if (done == gridDim.x - 1) {       // every wave has taken its last item
                __hip_atomic_store(queue, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(queue + 1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

// z = sum over subdomains covering the node of chi_x * chi_y * x_local
// (acc != 0: z += that sum, the fixed-point update of Algorithm 1).
// (ks non-null: into z + ks[problem].kp * zstride, the Krylov vector of the
// problem's current step.)
template <typename T>
__global__ void k_pou_sum(const DevProb *__restrict__ probs, const DevSub *__restrict__ subs,
                          const int *__restrict__ active, const int *__restrict__ pcnt,
                          const int *__restrict__ pchunk, const double *__restrict__ pw,
                          const cplx<T> *__restrict__ xout, double2 *__restrict__ z,
                          const KState *__restrict__ ks, long long zstride, int acc) {
    const DevProb P = probs[blockIdx.y];
    if (active != nullptr && active[blockIdx.y] == 0) return;
    if (ks != nullptr) z += static_cast<long long>(ks[blockIdx.y].kp) * zstride;
    const long long idx = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= P.ndof) return;
    const int i = static_cast<int>(idx % P.n1) + 1;
    const int j = static_cast<int>(idx / P.n1) + 1;
    const int ex = P.pou_x + i, ey = P.pou_y + j;
    const int nxc = pcnt[ex], nyc = pcnt[ey];
    double zr = 0.0, zi = 0.0;
    if (nxc <= 2 && nyc <= 2) {
        // at most two subdomains along each axis (every node when the chunks
        // are wider than the overlap): the four descriptors and values are
        // loaded before the first FMA (a missing second subdomain repeats the
        // first, whose value is then not added), the sum in the loop's order
        const int p0 = pchunk[ex * kMaxPou], q0 = pchunk[ey * kMaxPou];
        const int p1 = nxc > 1 ? pchunk[ex * kMaxPou + 1] : p0;
        const int q1 = nyc > 1 ? pchunk[ey * kMaxPou + 1] : q0;
        const double wx0 = pw[ex * kMaxPou], wx1 = pw[ex * kMaxPou + 1];
        const double wy0 = pw[ey * kMaxPou], wy1 = pw[ey * kMaxPou + 1];
        const DevSub *sb = subs + P.sub_first;
        const int4 s00 = *reinterpret_cast<const int4 *>(&sb[q0 * P.Px + p0].pou_off);
        const int4 s01 = *reinterpret_cast<const int4 *>(&sb[q0 * P.Px + p1].pou_off);
        const int4 s10 = *reinterpret_cast<const int4 *>(&sb[q1 * P.Px + p0].pou_off);
        const int4 s11 = *reinterpret_cast<const int4 *>(&sb[q1 * P.Px + p1].pou_off);
        const cplx<T> x00 = xout[s00.x + i * s00.y + j * s00.z];
        const cplx<T> x01 = xout[s01.x + i * s01.y + j * s01.z];
        const cplx<T> x10 = xout[s10.x + i * s10.y + j * s10.z];
        const cplx<T> x11 = xout[s11.x + i * s11.y + j * s11.z];
        zr = fma(wx0 * wy0, static_cast<double>(x00.re), zr);
        zi = fma(wx0 * wy0, static_cast<double>(x00.im), zi);
        if (nxc > 1) {
            zr = fma(wx1 * wy0, static_cast<double>(x01.re), zr);
            zi = fma(wx1 * wy0, static_cast<double>(x01.im), zi);
        }
        if (nyc > 1) {
            zr = fma(wx0 * wy1, static_cast<double>(x10.re), zr);
            zi = fma(wx0 * wy1, static_cast<double>(x10.im), zi);
            if (nxc > 1) {
                zr = fma(wx1 * wy1, static_cast<double>(x11.re), zr);
                zi = fma(wx1 * wy1, static_cast<double>(x11.im), zi);
            }
        }
    } else
    for (int b = 0; b < nyc; ++b) {
        const int q = pchunk[ey * kMaxPou + b];
        const double wy = pw[ey * kMaxPou + b];
        for (int a = 0; a < nxc; ++a) {
            const int p = pchunk[ex * kMaxPou + a];
            const double w = pw[ex * kMaxPou + a] * wy;
            const DevSub &S = subs[P.sub_first + q * P.Px + p];
            const int r = S.xfast ? (j - S.jy0) * S.nx + (i - S.ix0) : (i - S.ix0) * S.ny + (j - S.jy0);
            const cplx<T> x = xout[S.vec_off + r];
            zr = fma(w, static_cast<double>(x.re), zr);
            zi = fma(w, static_cast<double>(x.im), zi);
        }
    }
    if (acc) {
        const double2 z0 = z[P.dof_off + idx];
        zr += z0.x;
        zi += z0.y;
    }
    z[P.dof_off + idx] = make_double2(zr, zi);
}

template <typename T>
__global__ void k_export_local(const DevSub *__restrict__ subs, const cplx<T> *__restrict__ xout,
                               double2 *__restrict__ xl) {
    const DevSub S = subs[blockIdx.y];
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= S.n) return;
    const cplx<T> x = xout[S.vec_off + r];
    xl[S.loc_off + r] = make_double2(static_cast<double>(x.re), static_cast<double>(x.im));
}

// Wide bands (W = 64 K, K = 3..7), two waves per subdomain.  Ring register
// k of lane l holds slot 64 k + l, the slot of the rows congruent to it mod
// W; W is a multiple of 64, so the pivots of a block of 64 steps all sit in
// register (block index) mod K.  Wave 0 holds registers 0 .. KA-1, wave 1
// the rest (KA = ceil(K / 2)).  Every pivot updates every register, but the
// pivots of a block come from one wave, its owner, which runs the block's
// serial steps on its own registers and publishes the 64 pivots in LDS; the
// other wave applies them to its registers one block later (no serial
// dependence there).  In the lock-step iteration of block b the owner of b
// first applies block b - 1 if the other wave owned it, then runs block b;
// the other wave applies block b - 1 if it did not own it.  Both waves pass
// one workgroup barrier per block.  Ownership changes every KA or K - KA
// blocks, so per K blocks about K / 2 + 1 of the half-width block times are
// on the critical path instead of K full ones.  A finished slot keeps
// accumulating for the row W further on; at the start of that row's block
// its owner adds (right-hand side - finished value), the finished values
// being its block outputs K blocks before (hk).  Each wave reads its part of
// every factor vector it applies, PD steps ahead; the stream layout is that
// of the other kernels.
template <typename T, int K, int PD>
__device__ __forceinline__ void solve_wide(const DevProb *__restrict__ probs, const DevSub &S,
                                           const double2 *__restrict__ v,
                                           const cplx<T> *__restrict__ F,
                                           cplx<T> *__restrict__ ybuf,
                                           cplx<T> *__restrict__ xout, cplx<T> (*pbuf)[64]) {
    constexpr int W = 64 * K;
    constexpr int KA = (K + 1) / 2;            // registers per wave (wave 1: K - KA)
    const int dof_off = static_cast<int>(probs[S.prob].dof_off);
    const int n1 = probs[S.prob].n1;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int g0 = wv ? KA : 0;                // first ring register of this wave
    const int npad = S.npad, nb = npad / 64;
    const long long NW = static_cast<long long>(npad) * W;
    const cplx<T> *L = F + S.fac_off;
    const cplx<T> *Dv = L + 2 * NW;
    cplx<T> *yb = ybuf + S.vec_off;
    cplx<T> *xo = xout + S.vec_off;
    const cplx<T> zero{0, 0};
    // this wave's lane offsets in a factor vector (wave 1 of an odd K has
    // one register fewer: its last one re-reads a valid entry and is never
    // a pivot)
    int off[KA];
#pragma unroll
    for (int j = 0; j < KA; ++j) off[j] = 64 * min(g0 + j, K - 1) + lane;
    auto owner = [&](int kb) { return kb < KA ? 0 : 1; };
    auto pick = [&](const cplx<T> *a, int j) {
        cplx<T> r = a[0];
#pragma unroll
        for (int i = 1; i < KA; ++i) r = csel(j == i, a[i], r);
        return r;
    };
    const cplx<T> *pf;
    cplx<T> f[PD][KA];
    auto start = [&](const cplx<T> *p) {
        pf = p;
#pragma unroll
        for (int u = 0; u < PD; ++u) {
#pragma unroll
            for (int j = 0; j < KA; ++j) f[u][j] = nt_load(pf + off[j]);
            pf += W;
        }
    };
    cplx<T> y[KA], hk[KA];
    // 64 steps applying the pivots of register vector pv (lane t: step t;
    // down: steps in decreasing t)
    auto apply = [&](const cplx<T> pv, bool down) {
#pragma unroll
        for (int q = 0; q < 64; ++q) {
            const int t = down ? 63 - q : q;
            const int u = q % PD;
            const cplx<T> piv = readlane(pv, t);
#pragma unroll
            for (int j = 0; j < KA; ++j) y[j] = cfms(y[j], f[u][j], piv);
#pragma unroll
            for (int j = 0; j < KA; ++j) f[u][j] = nt_load(pf + off[j]);
            pf += W;
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    // 64 serial steps with the pivots in local register jl; returns them
    auto chain = [&](int jl, bool down) {
        cplx<T> out = zero;
#pragma unroll
        for (int q = 0; q < 64; ++q) {
            const int t = down ? 63 - q : q;
            const int u = q % PD;
            const cplx<T> piv = readlane(pick(y, jl), t);
#pragma unroll
            for (int j = 0; j < KA; ++j) y[j] = cfms(y[j], f[u][j], piv);
            out = writelane(out, piv, t);
#pragma unroll
            for (int j = 0; j < KA; ++j) f[u][j] = nt_load(pf + off[j]);
            pf += W;
            __builtin_amdgcn_sched_barrier(0);
        }
        return out;
    };
    // one sweep: blocks b0, b0 + db, ... (nb of them), right-hand side of
    // block b from rhs(b), outputs to dst
    auto sweep = [&](int b0, int db, bool down, auto rhs, cplx<T> *dst) {
#pragma unroll
        for (int j = 0; j < KA; ++j) y[j] = hk[j] = zero;
        cplx<T> rnext = rhs(b0);
        for (int i = 0; i < nb; ++i) {
            const int b = b0 + i * db;
            const int kb = b % K, kbp = (b - db) % K;
            const cplx<T> rblk = rnext;
            if (i + 1 < nb) rnext = rhs(b + db);
            if (i > 0 && owner(kbp) != wv) apply(pbuf[(i - 1) & 1][lane], down);
            if (owner(kb) == wv) {
                const int jl = kb - g0;
#pragma unroll
                for (int j = 0; j < KA; ++j) y[j] = csel(j == jl, cadd(y[j], csub(rblk, hk[j])), y[j]);
                const cplx<T> out = chain(jl, down);
#pragma unroll
                for (int j = 0; j < KA; ++j) hk[j] = csel(j == jl, out, hk[j]);
                dst[64 * b + lane] = out;
                pbuf[i & 1][lane] = out;
            }
            __syncthreads();
        }
    };

    // forward L y = R_j v (columns of L, blocks in increasing order)
    start(L);
    sweep(0, 1, false, [&](int b) { return gather_rhs<T>(S, dof_off, n1, v, 64 * b + lane); }, yb);
    // backward L^T x = D^{-1} y (rows of L, last first; the forward results
    // of the other wave are visible after the sweep's last barrier)
    start(L + NW);
    sweep(nb - 1, -1, true, [&](int b) { return cmul(yb[64 * b + lane], Dv[64 * b + lane]); }, xo);
}

// Two waves per wide subdomain (order[0 .. nsub)), the right-hand side as
// for k_band_solve.
template <typename T, int PD>
__global__ __launch_bounds__(128) void k_band_solve_wide(
    const DevProb *__restrict__ probs, const DevSub *__restrict__ subs,
    const int *__restrict__ order, const int *__restrict__ active,
    const double2 *__restrict__ v, const KState *__restrict__ ks, long long vstride,
    const cplx<T> *__restrict__ F, cplx<T> *__restrict__ ybuf, cplx<T> *__restrict__ xout) {
    __shared__ cplx<T> pbuf[2][64];            // the last two blocks' pivots
    const DevSub S = subs[order[blockIdx.x]];
    if (active != nullptr && active[S.prob] == 0) return;
    const double2 *vs = ks != nullptr ? v + static_cast<long long>(ks[S.prob].kp) * vstride : v;
    switch (S.W >> 6) {
        case 3: solve_wide<T, 3, PD>(probs, S, vs, F, ybuf, xout, pbuf); break;
        case 4: solve_wide<T, 4, PD>(probs, S, vs, F, ybuf, xout, pbuf); break;
        case 5: solve_wide<T, 5, PD>(probs, S, vs, F, ybuf, xout, pbuf); break;
        case 6: solve_wide<T, 6, PD>(probs, S, vs, F, ybuf, xout, pbuf); break;
        default: solve_wide<T, 7, PD>(probs, S, vs, F, ybuf, xout, pbuf); break;
    }
}

template <typename T, bool TWO, int PD>
void launch_solve_cfg(const DevProb *probs, const DevSub *subs, const int *order, int nsub,
                      const int *active, const SolveSrc &src, const void *F, void *ybuf,
                      void *xout, const SolveDispatch &dsp, hipStream_t st) {
    const cplx<T> *Fc = static_cast<const cplx<T> *>(F);
    cplx<T> *yb = static_cast<cplx<T> *>(ybuf);
    cplx<T> *xo = static_cast<cplx<T> *>(xout);
    if (dsp.queue != nullptr && dsp.waves > 0 && dsp.waves < nsub)
        hipLaunchKernelGGL((k_band_solve<T, TWO, PD, true>), dim3(dsp.waves), dim3(64), 0, st,
                           probs, subs, order, nsub, active, src.v, src.ks, src.stride, Fc, yb,
                           xo, dsp.queue);
    else
        hipLaunchKernelGGL((k_band_solve<T, TWO, PD, false>), dim3(nsub), dim3(64), 0, st, probs,
                           subs, order, nsub, active, src.v, src.ks, src.stride, Fc, yb, xo,
                           dsp.queue);
}

}  // namespace

// One wave per subdomain.  deep: prefetch depth 16 vectors (32 for a
// complex64 batch with W <= 64, whose lanes hold one slot each), else half
// of that; the default is deep, the autotuner measures both.  (In the pair
// layout a vector takes four registers per lane: 32 would not fit.)  F must carry 64 KB of slack past the last
// factor (the prefetch runs past each stream's end).  dsp: hardware
// dispatch of one wave per subdomain, or a persistent grid of dsp.waves
// waves taking subdomains from the counter dsp.queue (two words, zero
// between launches) when fewer waves than subdomains are asked for.
// The wide subdomains order[0 .. nsub) (W = 192, 256, 320, 384 or 448), two
// waves each; prefetch 16 vectors in complex64, 8 in complex128.
void launch_band_solve_wide(bool fp64, const DevProb *probs, const DevSub *subs, const int *order,
                            int nsub, const int *active, const SolveSrc &src, const void *F,
                            void *ybuf, void *xout, hipStream_t st) {
    if (fp64)
        hipLaunchKernelGGL((k_band_solve_wide<double, 8>), dim3(nsub), dim3(128), 0, st, probs, subs,
                           order, active, src.v, src.ks, src.stride,
                           static_cast<const cplx<double> *>(F), static_cast<cplx<double> *>(ybuf),
                           static_cast<cplx<double> *>(xout));
    else
        hipLaunchKernelGGL((k_band_solve_wide<float, 16>), dim3(nsub), dim3(128), 0, st, probs, subs,
                           order, active, src.v, src.ks, src.stride,
                           static_cast<const cplx<float> *>(F), static_cast<cplx<float> *>(ybuf),
                           static_cast<cplx<float> *>(xout));
}

void launch_band_solve(bool fp64, bool deep, int maxW, const DevProb *probs, const DevSub *subs,
                       const int *order, int nsub, const int *active, const SolveSrc &src,
                       const void *F, void *ybuf, void *xout, const SolveDispatch &dsp,
                       hipStream_t st) {
    const bool two = maxW > 64;
#define RAS_SOLVE(T, TWO, PD) \
    launch_solve_cfg<T, TWO, PD>(probs, subs, order, nsub, active, src, F, ybuf, xout, dsp, st)
    if (fp64) {
        if (two) {
            if (deep) RAS_SOLVE(double, true, 16); else RAS_SOLVE(double, true, 8);
        } else {
            if (deep) RAS_SOLVE(double, false, 16); else RAS_SOLVE(double, false, 8);
        }
    } else {
        if (two) {
            if (deep) RAS_SOLVE(float, true, 16); else RAS_SOLVE(float, true, 8);
        } else {
            if (deep) RAS_SOLVE(float, false, 32); else RAS_SOLVE(float, false, 16);
        }
    }
#undef RAS_SOLVE
}

void launch_pou_sum(bool fp64, const DevProb *probs, int nprob, long long max_ndof,
                    const DevSub *subs, const int *active, const int *pcnt, const int *pchunk,
                    const double *pw, const void *xout, const SumDst &dst, bool acc,
                    hipStream_t st) {
    dim3 grid(static_cast<unsigned>((max_ndof + 255) / 256), nprob);
    if (fp64)
        hipLaunchKernelGGL(k_pou_sum<double>, grid, dim3(256), 0, st, probs, subs, active, pcnt,
                           pchunk, pw, static_cast<const cplx<double> *>(xout), dst.z, dst.ks,
                           dst.stride, acc ? 1 : 0);
    else
        hipLaunchKernelGGL(k_pou_sum<float>, grid, dim3(256), 0, st, probs, subs, active, pcnt,
                           pchunk, pw, static_cast<const cplx<float> *>(xout), dst.z, dst.ks,
                           dst.stride, acc ? 1 : 0);
}

void launch_export_local(bool fp64, const DevSub *subs, int nsub, int max_n, const void *xout,
                         double2 *xl, hipStream_t st) {
    dim3 grid(static_cast<unsigned>((max_n + 255) / 256), nsub);
    if (fp64)
        hipLaunchKernelGGL(k_export_local<double>, grid, dim3(256), 0, st, subs,
                           static_cast<const cplx<double> *>(xout), xl);
    else
        hipLaunchKernelGGL(k_export_local<float>, grid, dim3(256), 0, st, subs,
                           static_cast<const cplx<float> *>(xout), xl);
}

}  // namespace raspml
