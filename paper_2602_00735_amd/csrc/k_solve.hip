// RAS-PML preconditioner application (Section 2, discrete RAS):
//     z = B^{-1} v = sum_j R~_j^T A_j^{-1} R_j v.
//
// k_band_solve: one wave64 per subdomain (largest first).  With
// A_j = L D L^T it runs
//   forward   L y = R_j v  (column form: y_c is final, then every row below
//             it in the band takes -L[r,c] y_c),
//   diagonal  z = D^{-1} y,
//   backward  L^T x = z    (dot form: x_c = z_c - sum_r L[r,c] x_r over the
//             band rows below c).
// Both sweeps keep the band rows of the current window in registers as a
// ring spread over the lanes: row r lives in slot r mod W, slot s in lane
// s mod 64 (second register for slots 64..127).  Factor column c is stored in
// the same slot order, so each step reads one contiguous column, fully
// coalesced, prefetched PD steps ahead into registers.  The pivot value is
// broadcast with v_readlane, incoming right-hand-side values and the
// outputs move with v_writelane; the backward dot product is a DPP wave sum.
// The restricted right-hand side R_j v is gathered from the global complex128
// vector one block of 64 rows ahead and converted to the factor precision.
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
    const int r = min(r0, S.n - 1);
    int i, j;
    if (S.xfast) {
        i = S.ix0 + r % S.nf;
        j = S.jy0 + r / S.nf;
    } else {
        j = S.jy0 + r % S.nf;
        i = S.ix0 + r / S.nf;
    }
    const double2 x = v[static_cast<long long>(dof_off) + static_cast<long long>(j - 1) * n1 + (i - 1)];
    const bool in = r0 < S.n;
    return cplx<T>{in ? static_cast<T>(x.x) : T(0), in ? static_cast<T>(x.y) : T(0)};
}

// Column `col` of L in slot order.  Lanes past the column end re-read its
// last entry (always in bounds, no branch): their ring registers are never
// read in the forward sweep and stay exactly zero in the backward sweep, so
// those values never reach a result.
template <typename T, bool TWO>
__device__ __forceinline__ void load_col(const cplx<T> *__restrict__ L, int W, int col, int lane,
                                         cplx<T> &lo, cplx<T> &hi) {
    const cplx<T> *p = L + static_cast<long long>(col) * W;
    lo = p[min(lane, W - 1)];
    if (TWO) hi = p[min(lane + 64, W - 1)];
}

// PD: factor prefetch depth in columns (divides 64).
template <typename T, bool TWO, int PD>
__global__ __launch_bounds__(64) void k_band_solve(const DevProb *__restrict__ probs,
                                                   const DevSub *__restrict__ subs,
                                                   const int *__restrict__ order,
                                                   const int *__restrict__ active,
                                                   const double2 *__restrict__ v,
                                                   const cplx<T> *__restrict__ F,
                                                   cplx<T> *__restrict__ ybuf,
                                                   cplx<T> *__restrict__ xout) {
    const int s = order[blockIdx.x];
    const DevSub S = subs[s];
    if (active != nullptr && active[S.prob] == 0) return;
    const int dof_off = static_cast<int>(probs[S.prob].dof_off);
    const int n1 = probs[S.prob].n1;
    const int lane = threadIdx.x;
    const int W = S.W, npad = S.npad;
    const cplx<T> *L = F + S.fac_off;
    const cplx<T> *Dv = L + static_cast<long long>(npad) * W;
    cplx<T> *yb = ybuf + S.vec_off;
    cplx<T> *xo = xout + S.vec_off;

    __shared__ cplx<T> stage[64];     // per-step outputs of one block of 64 rows

    // ------------------------------------------------------------ forward
    cplx<T> ylo = gather_rhs<T>(S, dof_off, n1, v, lane);
    cplx<T> yhi{0, 0};
    if (TWO) yhi = gather_rhs<T>(S, dof_off, n1, v, lane + 64);
    if (lane >= W) ylo = cplx<T>{0, 0};
    if (lane + 64 >= W) yhi = cplx<T>{0, 0};
    cplx<T> rnext = gather_rhs<T>(S, dof_off, n1, v, W + lane);
    cplx<T> flo[PD], fhi[PD];
#pragma unroll
    for (int u = 0; u < PD; ++u) load_col<T, TWO>(L, W, min(u, npad - 1), lane, flo[u], fhi[u]);
    int sl = 0;
    for (int c0 = 0; c0 < npad; c0 += 64) {
        // rows entering the window during this block: c0 + W + t
        // rows entering during this block were gathered one block ago; the
        // next block's rows are gathered now and converted after the steps
        const cplx<T> rblk = rnext;
        const double2 rraw = gather_raw(S, dof_off, n1, v, c0 + 64 + W + lane);
#pragma unroll
        for (int t = 0; t < 64; ++t) {
            const int u = t % PD;
            const int c = c0 + t;
            const cplx<T> yc = readlane((!TWO || sl < 64) ? ylo : yhi, sl & 63);
            ylo = cfms(ylo, flo[u], yc);
            if (TWO) yhi = cfms(yhi, fhi[u], yc);
            const cplx<T> rin = readlane(rblk, t);
            ylo = writelane(ylo, rin, sl);
            if (TWO) yhi = writelane(yhi, rin, sl - 64);
            stage[t] = yc;                              // same value from every lane
            load_col<T, TWO>(L, W, min(c + PD, npad - 1), lane, flo[u], fhi[u]);
            sl = (sl + 1 == W) ? 0 : sl + 1;
            __builtin_amdgcn_sched_barrier(0);   // keep each step's loads in place
        }
        rnext = to_T<T>(rraw, c0 + 64 + W + lane < S.n);
        __builtin_amdgcn_wave_barrier();
        yb[c0 + lane] = stage[lane];
        __builtin_amdgcn_wave_barrier();
    }

    // ------------------------------------------------------------ backward
    cplx<T> xlo{0, 0}, xhi{0, 0};
    cplx<T> znext = cmul(yb[npad - 64 + lane], Dv[npad - 64 + lane]);
#pragma unroll
    for (int u = 0; u < PD; ++u) load_col<T, TWO>(L, W, max(npad - 1 - u, 0), lane, flo[u], fhi[u]);
    sl = (npad - 1) % W;
    for (int c0 = npad - 64; c0 >= 0; c0 -= 64) {
        const cplx<T> zblk = znext;
        const cplx<T> ynx = yb[max(c0 - 64, 0) + lane];
        const cplx<T> dnx = Dv[max(c0 - 64, 0) + lane];
#pragma unroll
        for (int q = 0; q < 64; ++q) {
            const int t = 63 - q;
            const int u = q % PD;
            const int c = c0 + t;
            cplx<T> p = cmul(flo[u], xlo);
            if (TWO) p = cfma(p, fhi[u], xhi);
            const cplx<T> sum = wave_sum(p);
            const cplx<T> xc = csub(readlane(zblk, t), sum);
            xlo = writelane(xlo, xc, sl);
            if (TWO) xhi = writelane(xhi, xc, sl - 64);
            stage[t] = xc;
            load_col<T, TWO>(L, W, max(c - PD, 0), lane, flo[u], fhi[u]);
            sl = (sl == 0) ? W - 1 : sl - 1;
            __builtin_amdgcn_sched_barrier(0);
        }
        znext = cmul(ynx, dnx);
        __builtin_amdgcn_wave_barrier();
        xo[c0 + lane] = stage[lane];
        __builtin_amdgcn_wave_barrier();
    }
}

// z = sum over subdomains covering the node of chi_x * chi_y * x_local.
template <typename T>
__global__ void k_pou_sum(const DevProb *__restrict__ probs, const DevSub *__restrict__ subs,
                          const int *__restrict__ active, const int *__restrict__ pcnt,
                          const int *__restrict__ pchunk, const double *__restrict__ pw,
                          const cplx<T> *__restrict__ xout, double2 *__restrict__ z) {
    const DevProb P = probs[blockIdx.y];
    if (active != nullptr && active[blockIdx.y] == 0) return;
    const long long idx = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= P.ndof) return;
    const int i = static_cast<int>(idx % P.n1) + 1;
    const int j = static_cast<int>(idx / P.n1) + 1;
    const int ex = P.pou_x + i, ey = P.pou_y + j;
    const int nxc = pcnt[ex], nyc = pcnt[ey];
    double zr = 0.0, zi = 0.0;
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

template <typename T, bool TWO, int PD>
void launch_solve_cfg(const DevProb *probs, const DevSub *subs, const int *order, int nsub,
                      const int *active, const double2 *v, const void *F, void *ybuf, void *xout,
                      hipStream_t st) {
    hipLaunchKernelGGL((k_band_solve<T, TWO, PD>), dim3(nsub), dim3(64), 0, st, probs, subs, order,
                       active, v, static_cast<const cplx<T> *>(F), static_cast<cplx<T> *>(ybuf),
                       static_cast<cplx<T> *>(xout));
}

}  // namespace

// One wave per subdomain; the prefetch depth keeps ~32 (complex64) or ~16
// (complex128) factor columns in flight per wave.
void launch_band_solve(bool fp64, int maxW, const DevProb *probs, const DevSub *subs,
                       const int *order, int nsub, const int *active, const double2 *v,
                       const void *F, void *ybuf, void *xout, hipStream_t st) {
    if (fp64) {
        if (maxW <= 64)
            launch_solve_cfg<double, false, 16>(probs, subs, order, nsub, active, v, F, ybuf, xout, st);
        else
            launch_solve_cfg<double, true, 16>(probs, subs, order, nsub, active, v, F, ybuf, xout, st);
    } else {
        if (maxW <= 64)
            launch_solve_cfg<float, false, 32>(probs, subs, order, nsub, active, v, F, ybuf, xout, st);
        else
            launch_solve_cfg<float, true, 32>(probs, subs, order, nsub, active, v, F, ybuf, xout, st);
    }
}

void launch_pou_sum(bool fp64, const DevProb *probs, int nprob, long long max_ndof,
                    const DevSub *subs, const int *active, const int *pcnt, const int *pchunk,
                    const double *pw, const void *xout, double2 *z, hipStream_t st) {
    dim3 grid(static_cast<unsigned>((max_ndof + 255) / 256), nprob);
    if (fp64)
        hipLaunchKernelGGL(k_pou_sum<double>, grid, dim3(256), 0, st, probs, subs, active, pcnt,
                           pchunk, pw, static_cast<const cplx<double> *>(xout), z);
    else
        hipLaunchKernelGGL(k_pou_sum<float>, grid, dim3(256), 0, st, probs, subs, active, pcnt,
                           pchunk, pw, static_cast<const cplx<float> *>(xout), z);
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
